"""ctypes declarations for libqvec.so (include/sv.h). Marshalling only."""
from __future__ import annotations

import ctypes
import struct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqvec.so")

SV_OK, SV_EINVAL, SV_ENOMEM, SV_EDEVICE, SV_EUNSUPPORTED = 0, 1, 2, 3, 4
SV_C64, SV_C128 = 1, 2

OPS = {
    "mat1": 0, "mat2": 1, "h": 2, "x": 3, "y": 4, "z": 5, "s": 6, "sdg": 7, "t": 8, "tdg": 9,
    "rx": 10, "ry": 11, "rz": 12, "p": 13, "u3": 14, "cx": 15, "cz": 16, "cp": 17, "swap": 18,
}

# Kernel families of sv_timing_read.
KF_BLOCK, KF_SWEEP1, KF_SWEEP2, KF_DIAG, KF_REDUCE, KF_INIT, KF_COPY, KF_ADJ_BLOCK = range(8)


class SvGate(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_int32),
        ("qubits", ctypes.c_int32 * 2),
        ("n_controls", ctypes.c_int32),
        ("controls", ctypes.c_int32 * 2),
        ("param_index", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("angles", ctypes.c_double * 3),
        ("matrix", ctypes.c_double * 32),
    ]


class SvPauli(ctypes.Structure):
    _fields_ = [("coeff", ctypes.c_double), ("x_mask", ctypes.c_uint64), ("z_mask", ctypes.c_uint64)]


class SvDiff(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("max_abs", "l2", "inner_re", "inner_im", "norm2_a", "norm2_b")]


class SvPlanStats(ctypes.Structure):
    _fields_ = [
        ("n_gates", ctypes.c_int64),
        ("n_passes", ctypes.c_int64),
        ("n_block_passes", ctypes.c_int64),
        ("block_qubits", ctypes.c_int64),
        ("bytes_moved", ctypes.c_double),
        ("n_stages", ctypes.c_int64),
        ("n_ops", ctypes.c_int64),
        ("n_phase_ops", ctypes.c_int64),
    ]


class SvHostStats(ctypes.Structure):
    _fields_ = [
        ("n_passes", ctypes.c_int64),
        ("n_chunks", ctypes.c_int64),
        ("chunk_qubits", ctypes.c_int64),
        ("high_qubits", ctypes.c_int64),
        ("bytes_h2d", ctypes.c_double),
        ("bytes_d2h", ctypes.c_double),
        ("seconds", ctypes.c_double),
    ]


class SvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"sv status {status}: {msg}")
        self.status = status


# Every symbol include/sv.h declares, with its ctypes signature.
_vp = ctypes.c_void_p
_i = ctypes.c_int
_st = ctypes.c_int
SIGNATURES = {
    "sv_alloc": (_st, [ctypes.POINTER(_vp), _i, _i, _vp, ctypes.c_size_t, _vp]),
    "sv_free": (_st, [_vp]),
    "sv_data": (_vp, [_vp]),
    "sv_num_qubits": (_i, [_vp]),
    "sv_get_dtype": (_i, [_vp]),
    "sv_set_basis": (_st, [_vp, ctypes.c_uint64]),
    "sv_apply_gate": (_st, [_vp, _i, ctypes.POINTER(_i), _i, ctypes.POINTER(_i), ctypes.POINTER(ctypes.c_double)]),
    "sv_apply_unfused": (_st, [_vp, ctypes.POINTER(SvGate), _i]),
    "sv_apply_fused": (_st, [_vp, ctypes.POINTER(SvGate), _i]),
    "sv_plan": (_st, [_i, _i, ctypes.POINTER(SvGate), _i, ctypes.POINTER(SvPlanStats)]),
    "sv_host_apply": (_st, [_vp, _i, _i, ctypes.POINTER(SvGate), _i, _i, ctypes.POINTER(SvHostStats)]),
    "sv_norm2": (_st, [_vp, ctypes.POINTER(ctypes.c_double)]),
    "sv_expect": (_st, [_vp, ctypes.POINTER(SvPauli), _i, ctypes.POINTER(ctypes.c_double)]),
    "sv_expect_noalloc": (_st, [_vp, _i, _i, ctypes.POINTER(SvPauli), _i, _vp, _vp]),
    "sv_apply_pauli_sum": (_st, [_vp, ctypes.POINTER(SvPauli), _i, _vp, ctypes.c_size_t]),
    "sv_adjoint_grad": (_st, [_vp, ctypes.POINTER(SvGate), _i, ctypes.POINTER(SvPauli), _i, _vp, ctypes.c_size_t,
                              ctypes.POINTER(ctypes.c_double), _i, ctypes.POINTER(ctypes.c_double)]),
    "sv_compare": (_st, [_vp, _vp, ctypes.POINTER(SvDiff)]),
    "sv_copy": (_st, [_vp, _vp, _vp, ctypes.c_size_t]),
    "sv_sync": (_st, [_vp]),
    "sv_timing_enable": (_st, [_vp, _i]),
    "sv_timing_reset": (_st, [_vp]),
    "sv_timing_read": (_st, [_vp, _i, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    "sv_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libqvec.so. There is no fallback: a missing library is an error."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2508_15545_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != SV_OK:
        msg = lib().sv_last_error()
        raise SvError(status, msg.decode() if msg else "")


def gate_struct(g) -> SvGate:
    """Gate description (op, qubits, params, param_index) -> sv_gate."""
    s = SvGate()
    if g.op not in OPS:
        raise ValueError(f"unknown op {g.op!r}")
    s.op = OPS[g.op]
    for i, q in enumerate(g.qubits[:2]):
        s.qubits[i] = q
    ctrls = getattr(g, "controls", ()) or ()
    s.n_controls = len(ctrls)
    for i, q in enumerate(ctrls[:2]):
        s.controls[i] = q
    s.param_index = g.param_index
    if g.op in ("mat1", "mat2"):
        for i, v in enumerate(g.params):
            s.matrix[i] = v
    else:
        for i, v in enumerate(g.params[:3]):
            s.angles[i] = v
    return s


# op, qubits[2], n_controls, controls[2], param_index, reserved, angles[3]
_GATE_HEAD = struct.Struct("<8i3d")


def gate_array(circuit) -> "ctypes.Array[SvGate]":
    """Gate list -> contiguous sv_gate array (packed with struct; the ctypes
    array keeps its byte buffer alive)."""
    circuit = list(circuit)
    n = len(circuit)
    size = ctypes.sizeof(SvGate)
    mat_off = SvGate.matrix.offset
    buf = bytearray(size * max(1, n))
    pack = _GATE_HEAD.pack_into
    for i, g in enumerate(circuit):
        op = OPS.get(g.op)
        if op is None:
            raise ValueError(f"unknown op {g.op!r}")
        q = g.qubits
        ctrls = getattr(g, "controls", None) or ()
        c0 = ctrls[0] if len(ctrls) > 0 else 0
        c1 = ctrls[1] if len(ctrls) > 1 else 0
        p = g.params
        base = i * size
        if g.op in ("mat1", "mat2"):
            pack(buf, base, op, q[0], q[1] if len(q) > 1 else 0, len(ctrls), c0, c1, g.param_index, 0, 0.0, 0.0, 0.0)
            struct.pack_into(f"<{len(p)}d", buf, base + mat_off, *p)
        else:
            a = (tuple(p[:3]) + (0.0, 0.0, 0.0)) if len(p) < 3 else p
            pack(buf, base, op, q[0], q[1] if len(q) > 1 else 0, len(ctrls), c0, c1, g.param_index, 0,
                 a[0], a[1], a[2])
    return (SvGate * max(1, n)).from_buffer(buf)


def pauli_array(terms) -> "ctypes.Array[SvPauli]":
    terms = list(terms)
    arr = (SvPauli * max(1, len(terms)))()
    for i, (c, x, z) in enumerate(terms):
        arr[i].coeff = c
        arr[i].x_mask = x
        arr[i].z_mask = z
    return arr
