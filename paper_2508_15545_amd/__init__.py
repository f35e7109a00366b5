"""MI355X state-vector gate engine (Python binding of libqvec.so).

Every operation runs in the HIP library behind ``include/sv.h``; this module
only marshals arguments. PyTorch provides the device memory (the state is a
``torch.complex64``/``complex128`` tensor of 2^n amplitudes, qubit k = bit k
of the index) and the stream the library enqueues on.

Gates are described by objects with ``op``, ``qubits``, ``params`` and
``param_index`` attributes (and optionally ``controls``); observables are
lists of ``(coeff, x_mask, z_mask)`` Pauli strings.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _binding as B
from ._binding import SvError, check, gate_array, lib, pauli_array

__all__ = ["State", "SvError", "plan_stats", "expectation", "Expectation", "copy", "expect_noalloc"]

_DTYPES = {torch.complex128: B.SV_C128, torch.complex64: B.SV_C64}


def _stream_handle(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class State:
    """An n-qubit state vector in HBM bound to a libqvec handle.

    The tensor (``.tensor``) owns the memory; the handle enqueues on the
    current torch stream of the tensor's device at creation time.
    """

    def __init__(self, n: int, dtype: torch.dtype = torch.complex128, device=None,
                 tensor: Optional[torch.Tensor] = None):
        if dtype not in _DTYPES:
            raise ValueError("dtype must be torch.complex64 or torch.complex128")
        if tensor is None:
            device = torch.device(device if device is not None else "cuda")
            tensor = torch.empty(1 << n, dtype=dtype, device=device)
        if tensor.dtype != dtype or tensor.numel() != (1 << n) or not tensor.is_contiguous():
            raise ValueError("tensor must be a contiguous vector of 2^n amplitudes of the given dtype")
        if tensor.device.type != "cuda":
            raise ValueError("the state must live on a GPU")
        self.n = n
        self.dtype = dtype
        self.tensor = tensor
        self._h = ctypes.c_void_p()
        with torch.cuda.device(tensor.device):
            check(lib().sv_alloc(ctypes.byref(self._h), n, _DTYPES[dtype], ctypes.c_void_p(tensor.data_ptr()),
                                 tensor.numel() * tensor.element_size(), _stream_handle(tensor.device)))

    # -- lifetime -------------------------------------------------------------
    def close(self) -> None:
        if self._h:
            check(lib().sv_free(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._h:
                lib().sv_free(self._h)
        except Exception:
            pass

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    # -- gates ----------------------------------------------------------------
    def set_basis(self, x: int = 0) -> "State":
        check(lib().sv_set_basis(self._h, x))
        return self

    def apply_matrix(self, targets: Sequence[int], matrix, controls: Sequence[int] = ()) -> "State":
        m = np.asarray(matrix, dtype=np.complex128).reshape(-1)
        flat = np.empty(2 * m.size, dtype=np.float64)
        flat[0::2], flat[1::2] = m.real, m.imag
        t = (ctypes.c_int * 2)(*targets)
        c = (ctypes.c_int * 2)(*controls) if controls else None
        check(lib().sv_apply_gate(self._h, len(targets), t, len(controls), c,
                                  flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return self

    def apply(self, circuit, fused: bool = True) -> "State":
        arr = gate_array(circuit)
        fn = lib().sv_apply_fused if fused else lib().sv_apply_unfused
        check(fn(self._h, arr, len(circuit)))
        return self

    # -- reductions (these wait for the stream) -------------------------------
    def norm2(self) -> float:
        out = ctypes.c_double()
        check(lib().sv_norm2(self._h, ctypes.byref(out)))
        return out.value

    def expect(self, terms) -> float:
        terms = list(terms)
        out = ctypes.c_double()
        check(lib().sv_expect(self._h, pauli_array(terms), len(terms), ctypes.byref(out)))
        return out.value

    def apply_pauli_sum(self, terms, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        terms = list(terms)
        if out is None:
            out = torch.empty_like(self.tensor)
        if out.dtype != self.dtype or out.numel() != self.tensor.numel() or not out.is_contiguous():
            raise ValueError("out must match the state")
        check(lib().sv_apply_pauli_sum(self._h, pauli_array(terms), len(terms), ctypes.c_void_p(out.data_ptr()),
                                       out.numel() * out.element_size()))
        return out

    def adjoint_grad(self, circuit, terms, n_params: int, work: Optional[torch.Tensor] = None):
        """(f, grad) for f = <psi|H|psi>; the state must hold the circuit's
        output on entry and holds the recomputed input state afterwards."""
        terms = list(terms)
        if work is None:
            work = torch.empty_like(self.tensor)
        grad = np.zeros(max(1, n_params), dtype=np.float64)
        f = ctypes.c_double()
        check(lib().sv_adjoint_grad(self._h, gate_array(circuit), len(circuit), pauli_array(terms), len(terms),
                                    ctypes.c_void_p(work.data_ptr()), work.numel() * work.element_size(),
                                    grad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n_params,
                                    ctypes.byref(f)))
        return f.value, grad[:n_params]

    def compare(self, other: "State") -> dict:
        d = B.SvDiff()
        check(lib().sv_compare(self._h, other._h, ctypes.byref(d)))
        return {k: getattr(d, k) for k, _ in B.SvDiff._fields_}

    def sync(self) -> None:
        check(lib().sv_sync(self._h))

    # -- timing ---------------------------------------------------------------
    def timing(self, on: bool) -> None:
        check(lib().sv_timing_enable(self._h, int(on)))

    def timing_reset(self) -> None:
        check(lib().sv_timing_reset(self._h))

    def timing_read(self, family: int):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        check(lib().sv_timing_read(self._h, family, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value


def copy(state: State, dst: torch.Tensor, src: torch.Tensor) -> None:
    """Device copy with the library's streaming kernel (bandwidth reference)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst too small")
    check(lib().sv_copy(state.handle, ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes))


def expect_noalloc(state: torch.Tensor, terms, out: torch.Tensor) -> torch.Tensor:
    """<psi|H|psi> of a state tensor into out (a one-element float64 tensor
    on the state's device) through sv_expect_noalloc: enqueued on the current
    stream, no allocation by the library, no wait."""
    if state.dtype not in _DTYPES or state.device.type != "cuda" or not state.is_contiguous():
        raise ValueError("state must be a contiguous complex64/complex128 GPU tensor")
    n = state.numel().bit_length() - 1
    if state.numel() != 1 << n:
        raise ValueError("state must have 2^n entries")
    if out.dtype != torch.float64 or out.device != state.device or out.numel() < 1:
        raise ValueError("out must be a float64 tensor on the state's device")
    terms = list(terms)
    with torch.cuda.device(state.device):
        check(lib().sv_expect_noalloc(ctypes.c_void_p(state.data_ptr()), n, _DTYPES[state.dtype],
                                      pauli_array(terms), len(terms), ctypes.c_void_p(out.data_ptr()),
                                      _stream_handle(state.device)))
    return out


def host_apply(state: torch.Tensor, circuit, chunk_qubits: int) -> dict:
    """Apply a circuit to a state held in pinned host memory (a 1-D complex
    CPU tensor made with pin_memory=True, 2^n entries), chunk by chunk through
    the GPU (sv_host_apply). Returns the call's statistics."""
    if state.device.type != "cpu" or not state.is_pinned():
        raise ValueError("the host state must be a pinned CPU tensor")
    if state.dtype not in _DTYPES or not state.is_contiguous():
        raise ValueError("the host state must be a contiguous complex64/complex128 tensor")
    n = state.numel().bit_length() - 1
    if state.numel() != 1 << n:
        raise ValueError("the host state must have 2^n entries")
    st = B.SvHostStats()
    check(lib().sv_host_apply(ctypes.c_void_p(state.data_ptr()), n, _DTYPES[state.dtype], gate_array(circuit),
                              len(circuit), chunk_qubits, ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in B.SvHostStats._fields_}


def plan_stats(n: int, dtype: torch.dtype, circuit) -> dict:
    st = B.SvPlanStats()
    check(lib().sv_plan(n, _DTYPES[dtype], gate_array(circuit), len(circuit), ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in B.SvPlanStats._fields_}


def _with_angles(circuit, thetas: np.ndarray):
    out = []
    for g in circuit:
        if g.param_index >= 0:
            out.append(type(g)(g.op, g.qubits, (float(thetas[g.param_index]),), g.param_index))
        else:
            out.append(g)
    return out


class Expectation(torch.autograd.Function):
    """f(theta) = <psi(theta)|H|psi(theta)>, psi(theta) = U(theta) e_{x0}.

    Forward runs the fused circuit and the FP64 expectation on the GPU;
    backward runs the adjoint sweep (inverse gates, no checkpoints)."""

    @staticmethod
    def forward(ctx, thetas: torch.Tensor, circuit, terms, n: int, dtype: torch.dtype, x0: int = 0,
                device=None):
        th = thetas.detach().to("cpu", torch.float64).numpy()
        circ = _with_angles(circuit, th)
        dev = torch.device(device) if device is not None else (
            thetas.device if thetas.device.type == "cuda" else torch.device("cuda"))
        st = State(n, dtype, device=dev)
        st.set_basis(x0).apply(circ, fused=True)
        f = st.expect(terms)
        ctx.state, ctx.circ, ctx.terms, ctx.n_params = st, circ, list(terms), thetas.numel()
        return torch.tensor(f, dtype=torch.float64, device=thetas.device)

    @staticmethod
    def backward(ctx, grad_out):
        _, g = ctx.state.adjoint_grad(ctx.circ, ctx.terms, ctx.n_params)
        ctx.state = None
        gt = torch.from_numpy(g).to(grad_out.device) * grad_out
        return gt, None, None, None, None, None, None


def expectation(thetas: torch.Tensor, circuit, terms, n: int, dtype: torch.dtype = torch.complex128,
                x0: int = 0) -> torch.Tensor:
    return Expectation.apply(thetas, circuit, terms, n, dtype, x0)
