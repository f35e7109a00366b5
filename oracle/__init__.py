"""FP64 CPU oracle (test infrastructure only).

Only the test-suite, the package's smoke check and the benchmark's CPU-baseline
leg may import this package. The product path (the HIP library and its Python
binding) never imports, loads or calls it, and the two share no code: this
wrapper loads ``liboracle.so`` built from ``sv_oracle.c`` with gcc.

Functions take circuits as sequences of gate descriptions with attributes
``op``, ``qubits``, ``params`` and ``param_index`` (see the ``circuits`` input
module) and observables as ``(coeff, x_mask, z_mask)`` triples.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_OPS = {
    "h": 0, "x": 1, "y": 2, "z": 3, "s": 4, "sdg": 5, "t": 6, "tdg": 7,
    "rx": 8, "ry": 9, "rz": 10, "p": 11, "u3": 12, "mat1": 13,
    "cx": 14, "cz": 15, "cp": 16, "swap": 17, "mat2": 18,
}


class OrGate(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_int32),
        ("q0", ctypes.c_int32),
        ("q1", ctypes.c_int32),
        ("param_index", ctypes.c_int32),
        ("p", ctypes.c_double * 32),
    ]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-fcx-limited-range", _SRC, "-o", tmp, "-lm"],
            check=True,
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        gp = ctypes.POINTER(OrGate)
        cp = ctypes.c_void_p
        L.or_gate_matrix.argtypes = [gp, dp]
        L.or_gate_matrix.restype = ctypes.c_int
        L.or_apply_1q.argtypes = [cp, ctypes.c_int, ctypes.c_int, cp, ctypes.c_uint64]
        L.or_apply_1q.restype = None
        L.or_apply_2q.argtypes = [cp, ctypes.c_int, ctypes.c_int, ctypes.c_int, cp]
        L.or_apply_2q.restype = None
        L.or_apply_gate.argtypes = [cp, ctypes.c_int, gp, ctypes.c_int]
        L.or_apply_gate.restype = ctypes.c_int
        L.or_run.argtypes = [cp, ctypes.c_int, gp, ctypes.c_int]
        L.or_run.restype = ctypes.c_int
        L.or_run_inverse.argtypes = [cp, ctypes.c_int, gp, ctypes.c_int]
        L.or_run_inverse.restype = ctypes.c_int
        L.or_set_basis.argtypes = [cp, ctypes.c_int, ctypes.c_uint64]
        L.or_set_basis.restype = None
        L.or_pairwise_sum.argtypes = [dp, ctypes.c_int64]
        L.or_pairwise_sum.restype = ctypes.c_double
        L.or_expect.argtypes = [cp, ctypes.c_int, ctypes.c_int, dp, u64p, u64p]
        L.or_expect.restype = ctypes.c_double
        L.or_apply_pauli_sum.argtypes = [cp, cp, ctypes.c_int, ctypes.c_int, dp, u64p, u64p]
        L.or_apply_pauli_sum.restype = ctypes.c_int
        L.or_adjoint_grad.argtypes = [ctypes.c_int, ctypes.c_uint64, gp, ctypes.c_int,
                                      ctypes.c_int, dp, u64p, u64p, dp, ctypes.c_int]
        L.or_adjoint_grad.restype = ctypes.c_double
        L.or_param_shift_grad.argtypes = [ctypes.c_int, ctypes.c_uint64, gp, ctypes.c_int,
                                          ctypes.c_int, dp, u64p, u64p, dp, ctypes.c_int, i32p, ctypes.c_int]
        L.or_param_shift_grad.restype = ctypes.c_int
        L.or_finite_diff_grad.argtypes = [ctypes.c_int, ctypes.c_uint64, gp, ctypes.c_int,
                                          ctypes.c_int, dp, u64p, u64p, dp, ctypes.c_int,
                                          ctypes.c_double, i32p, ctypes.c_int]
        L.or_finite_diff_grad.restype = ctypes.c_int
        L.or_pair_updates.argtypes = []
        L.or_pair_updates.restype = ctypes.c_uint64
        L.or_reset_pair_updates.argtypes = []
        L.or_reset_pair_updates.restype = None
        L.or_num_threads.argtypes = []
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_set_threads.restype = None
        _lib = L
    return _lib


# ------------------------------------------------------------- marshalling ---

def _gate_struct(g) -> OrGate:
    s = OrGate()
    if g.op not in _OPS:
        raise ValueError(f"unknown op {g.op!r}")
    s.op = _OPS[g.op]
    s.q0 = g.qubits[0]
    s.q1 = g.qubits[1] if len(g.qubits) > 1 else -1
    s.param_index = g.param_index
    for i, v in enumerate(g.params):
        s.p[i] = v
    return s


def _gates(circuit: Sequence) -> "ctypes.Array[OrGate]":
    arr = (OrGate * max(1, len(circuit)))()
    for i, g in enumerate(circuit):
        arr[i] = _gate_struct(g)
    return arr


def _terms(terms: Iterable):
    terms = list(terms)
    c = np.array([t[0] for t in terms] or [0.0], dtype=np.float64)
    x = np.array([t[1] for t in terms] or [0], dtype=np.uint64)
    z = np.array([t[2] for t in terms] or [0], dtype=np.uint64)
    dp = ctypes.POINTER(ctypes.c_double)
    up = ctypes.POINTER(ctypes.c_uint64)
    return len(terms), c, x, z, c.ctypes.data_as(dp), x.ctypes.data_as(up), z.ctypes.data_as(up)


def _check_state(state: np.ndarray, n: int):
    if state.dtype != np.complex128 or state.shape != (1 << n,) or not state.flags.c_contiguous:
        raise ValueError("state must be a contiguous complex128 vector of length 2^n")


# ---------------------------------------------------------------- public ---

def gate_matrix(g) -> np.ndarray:
    out = (ctypes.c_double * 32)()
    s = _gate_struct(g)
    dim = lib().or_gate_matrix(ctypes.byref(s), out)
    if dim < 0:
        raise ValueError(f"no matrix for {g.op}")
    a = np.frombuffer(out, dtype=np.float64)[: 2 * dim * dim]
    return (a[0::2] + 1j * a[1::2]).reshape(dim, dim)


def basis_state(n: int, x: int = 0) -> np.ndarray:
    s = np.empty(1 << n, dtype=np.complex128)
    lib().or_set_basis(s.ctypes.data, n, x)
    return s


def apply_gate(state: np.ndarray, n: int, g, dagger: bool = False) -> np.ndarray:
    _check_state(state, n)
    s = _gate_struct(g)
    if lib().or_apply_gate(state.ctypes.data, n, ctypes.byref(s), int(dagger)):
        raise ValueError(f"bad gate {g}")
    return state


def apply_1q(state: np.ndarray, n: int, k: int, u: np.ndarray, ctrl_mask: int = 0) -> np.ndarray:
    _check_state(state, n)
    uu = np.ascontiguousarray(u, dtype=np.complex128).reshape(4)
    lib().or_apply_1q(state.ctypes.data, n, k, uu.ctypes.data, ctrl_mask)
    return state


def apply_2q(state: np.ndarray, n: int, qa: int, qb: int, u: np.ndarray) -> np.ndarray:
    _check_state(state, n)
    uu = np.ascontiguousarray(u, dtype=np.complex128).reshape(16)
    lib().or_apply_2q(state.ctypes.data, n, qa, qb, uu.ctypes.data)
    return state


def run(circuit: Sequence, n: int, x0: int = 0, state: Optional[np.ndarray] = None) -> np.ndarray:
    """Apply ``circuit`` to e_{x0} (or to a copy of ``state``) gate by gate."""
    if state is None:
        s = basis_state(n, x0)
    else:
        s = np.array(state, dtype=np.complex128, copy=True)
        _check_state(s, n)
    if circuit and lib().or_run(s.ctypes.data, n, _gates(circuit), len(circuit)):
        raise ValueError("bad circuit")
    return s


def run_inplace(state: np.ndarray, n: int, circuit: Sequence) -> np.ndarray:
    """Apply ``circuit`` gate by gate to ``state`` itself (no copy)."""
    _check_state(state, n)
    if circuit and lib().or_run(state.ctypes.data, n, _gates(circuit), len(circuit)):
        raise ValueError("bad circuit")
    return state


def run_inverse(circuit: Sequence, n: int, state: np.ndarray) -> np.ndarray:
    s = np.array(state, dtype=np.complex128, copy=True)
    _check_state(s, n)
    if circuit and lib().or_run_inverse(s.ctypes.data, n, _gates(circuit), len(circuit)):
        raise ValueError("bad circuit")
    return s


def pairwise_sum(v: np.ndarray) -> float:
    v = np.ascontiguousarray(v, dtype=np.float64)
    return lib().or_pairwise_sum(v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), v.size)


def expect(state: np.ndarray, n: int, terms) -> float:
    _check_state(state, n)
    k, c, x, z, cp, xp, zp = _terms(terms)
    return lib().or_expect(state.ctypes.data, n, k, cp, xp, zp)


def apply_pauli_sum(state: np.ndarray, n: int, terms) -> np.ndarray:
    _check_state(state, n)
    out = np.empty_like(state)
    k, c, x, z, cp, xp, zp = _terms(terms)
    lib().or_apply_pauli_sum(state.ctypes.data, out.ctypes.data, n, k, cp, xp, zp)
    return out


def adjoint_grad(circuit: Sequence, n: int, terms, n_params: int, x0: int = 0):
    """(f, grad) by the adjoint method on the CPU."""
    k, c, x, z, cp, xp, zp = _terms(terms)
    grad = np.zeros(max(1, n_params), dtype=np.float64)
    f = lib().or_adjoint_grad(n, x0, _gates(circuit), len(circuit), k, cp, xp, zp,
                              grad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n_params)
    if np.isnan(f):
        raise ValueError("adjoint failed (bad parameter slot or non-trainable op)")
    return f, grad[:n_params]


def _which(which):
    if which is None:
        return None, 0, None
    w = np.ascontiguousarray(which, dtype=np.int32)
    return w.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), w.size, w


def param_shift_grad(circuit: Sequence, n: int, terms, n_params: int, x0: int = 0, which=None) -> np.ndarray:
    k, c, x, z, cp, xp, zp = _terms(terms)
    grad = np.zeros(max(1, n_params), dtype=np.float64)
    wp, nw, _keep = _which(which)
    rc = lib().or_param_shift_grad(n, x0, _gates(circuit), len(circuit), k, cp, xp, zp,
                                   grad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n_params, wp, nw)
    if rc:
        raise ValueError("parameter shift failed")
    return grad[:n_params]


def finite_diff_grad(circuit: Sequence, n: int, terms, n_params: int, h: float = 1e-6, x0: int = 0,
                     which=None) -> np.ndarray:
    k, c, x, z, cp, xp, zp = _terms(terms)
    grad = np.zeros(max(1, n_params), dtype=np.float64)
    wp, nw, _keep = _which(which)
    rc = lib().or_finite_diff_grad(n, x0, _gates(circuit), len(circuit), k, cp, xp, zp,
                                   grad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n_params, h, wp, nw)
    if rc:
        raise ValueError("finite differences failed")
    return grad[:n_params]


def pair_updates() -> int:
    return int(lib().or_pair_updates())


def reset_pair_updates() -> None:
    lib().or_reset_pair_updates()


def num_threads() -> int:
    """OpenMP threads the oracle's loops run on."""
    return int(lib().or_num_threads())


def set_threads(k: int) -> None:
    """Run the oracle's OpenMP loops on k threads from now on."""
    lib().or_set_threads(int(k))


def qft_basis_amplitudes(n: int, x: int, lo: int, hi: int) -> np.ndarray:
    """Amplitudes lo .. hi-1 of the quantum Fourier transform of the basis
    state e_x (the definition of the transform that the textbook circuit of
    H and controlled phases realises, qubit n-1 most significant):
    alpha_y = 2^(-n/2) exp(2 pi i ((x y) mod 2^n) / 2^n). The phase numerator
    is formed in exact integer arithmetic, so each amplitude carries one
    rounding of the angle and one complex exponential."""
    if not (0 <= x < (1 << n) and 0 <= lo <= hi <= (1 << n)) or n > 31:
        raise ValueError("need 0 <= x < 2^n, 0 <= lo <= hi <= 2^n, n <= 31")
    y = np.arange(lo, hi, dtype=np.uint64)
    num = (np.uint64(x) * y) & np.uint64((1 << n) - 1)  # x y < 2^62: exact
    return np.exp(2j * np.pi * (num.astype(np.float64) / float(1 << n))) / math.sqrt(1 << n)
