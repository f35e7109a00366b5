"""CPU checks of the C ABI: the library loads, exports every function that
include/sv.h declares, rejects bad arguments before touching a device, and
plans circuits (sv_plan is host-only)."""
import collections
import ctypes
import os
import re

import numpy as np
import pytest

import circuits as C
from paper_2508_15545_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sv.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    L = B.lib()
    names = header_functions()
    assert "sv_apply_fused" in names and "sv_adjoint_grad" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(B.SIGNATURES), "binding and header disagree"


def test_struct_layouts_match_header():
    # sizes follow the field lists in include/sv.h (natural alignment)
    assert ctypes.sizeof(B.SvGate) == 4 * 8 + 8 * 3 + 8 * 32
    assert ctypes.sizeof(B.SvPauli) == 24
    assert ctypes.sizeof(B.SvDiff) == 48
    assert ctypes.sizeof(B.SvHostStats) == 4 * 8 + 3 * 8


def status(fn, *args):
    return fn(*args)


def test_alloc_argument_errors_return_before_any_device_call():
    L = B.lib()
    h = ctypes.c_void_p()
    assert L.sv_alloc(None, 4, B.SV_C128, None, 0, None) == B.SV_EINVAL
    assert L.sv_alloc(ctypes.byref(h), 0, B.SV_C128, None, 0, None) == B.SV_EINVAL
    assert L.sv_alloc(ctypes.byref(h), 35, B.SV_C128, None, 0, None) == B.SV_EINVAL
    assert L.sv_alloc(ctypes.byref(h), 4, 7, None, 0, None) == B.SV_EINVAL
    # a fake non-null buffer that is too small / misaligned is rejected first
    assert L.sv_alloc(ctypes.byref(h), 4, B.SV_C128, ctypes.c_void_p(4096), 255, None) == B.SV_EINVAL
    assert b"2^n" in L.sv_last_error()
    assert L.sv_alloc(ctypes.byref(h), 4, B.SV_C128, ctypes.c_void_p(4104), 256, None) == B.SV_EINVAL
    assert b"aligned" in L.sv_last_error()
    assert not h.value


def test_host_apply_argument_errors_return_before_any_copy():
    """sv_host_apply validates everything before it touches the host state or
    the GPU (the pointer below is never dereferenced)."""
    L = B.lib()
    fake = ctypes.c_void_p(1 << 20)
    one = B.gate_array([C.gate("h", 3)])
    st = B.SvHostStats()
    assert L.sv_host_apply(None, 10, B.SV_C128, one, 1, 6, ctypes.byref(st)) == B.SV_EINVAL
    assert L.sv_host_apply(ctypes.c_void_p((1 << 20) + 8), 10, B.SV_C128, one, 1, 6, None) == B.SV_EINVAL
    assert b"aligned" in L.sv_last_error()
    assert L.sv_host_apply(fake, 0, B.SV_C128, one, 1, 6, None) == B.SV_EINVAL
    assert L.sv_host_apply(fake, 10, B.SV_C128, one, 1, 0, None) == B.SV_EINVAL
    assert L.sv_host_apply(fake, 10, 5, one, 1, 6, None) == B.SV_EINVAL
    assert L.sv_host_apply(fake, 3, B.SV_C128, one, 1, 2, None) == B.SV_EINVAL  # qubit 3 >= n
    # a chunk of 4 of 20 qubits has 2 free high qubits: a gate on 3 high qubits cannot fit
    CtrlGate = collections.namedtuple("CtrlGate", "op qubits params param_index controls")
    big = B.gate_array([CtrlGate("x", (17,), (), -1, (18, 19))])
    assert L.sv_host_apply(fake, 20, B.SV_C128, big, 1, 4, ctypes.byref(st)) == B.SV_EUNSUPPORTED
    assert L.sv_host_apply(fake, 20, B.SV_C128, one, 0, 8, ctypes.byref(st)) == B.SV_OK  # nothing to do
    assert st.n_passes == 0 and st.chunk_qubits == 8 and st.n_chunks == 1 << 12


def test_null_handle_errors():
    L = B.lib()
    g = B.gate_array([C.gate("h", 0)])
    out = ctypes.c_double()
    assert L.sv_set_basis(None, 0) == B.SV_EINVAL
    assert L.sv_apply_fused(None, g, 1) == B.SV_EINVAL
    assert L.sv_apply_unfused(None, g, 1) == B.SV_EINVAL
    assert L.sv_norm2(None, ctypes.byref(out)) == B.SV_EINVAL
    assert L.sv_expect(None, None, 0, ctypes.byref(out)) == B.SV_EINVAL
    assert L.sv_sync(None) == B.SV_EINVAL
    assert L.sv_free(None) == B.SV_OK
    assert L.sv_data(None) is None and L.sv_num_qubits(None) == 0


def plan(n, circuit, dtype=B.SV_C128):
    st = B.SvPlanStats()
    rc = B.lib().sv_plan(n, dtype, B.gate_array(circuit), len(circuit), ctypes.byref(st))
    return rc, st


@pytest.mark.parametrize("bad,why", [
    (C.Gate("h", (5,), (), -1), "out of range"),
    (C.Gate("cx", (1, 1), (), -1), "repeated"),
    (C.Gate("h", (0,), (), 3), "param_index"),
    (C.Gate("rx", (0,), (float("nan"),), -1), "non-finite"),
])
def test_gate_validation(bad, why):
    rc, _ = plan(4, [C.gate("h", 0), bad])
    assert rc == B.SV_EINVAL
    assert why in B.lib().sv_last_error().decode()
    assert "gate 1" in B.lib().sv_last_error().decode()


def test_unsupported_controls_on_two_qubit_op():
    g = B.gate_array([C.gate("swap", 0, 1)])
    g[0].n_controls = 1
    g[0].controls[0] = 2
    st = B.SvPlanStats()
    assert B.lib().sv_plan(4, B.SV_C128, g, 1, ctypes.byref(st)) == B.SV_EUNSUPPORTED


def test_reserved_field_must_be_zero():
    g = B.gate_array([C.gate("h", 0)])
    g[0].reserved = 1
    st = B.SvPlanStats()
    assert B.lib().sv_plan(4, B.SV_C128, g, 1, ctypes.byref(st)) == B.SV_EINVAL


def test_plan_small_state_is_one_pass():
    # n <= b: the whole state is one block, the whole circuit one pass
    rc, st = plan(10, C.random_u3_layers(10, 5, 0))
    assert rc == B.SV_OK
    assert st.n_passes == 1 and st.n_block_passes == 1 and st.block_qubits == 10
    assert st.bytes_moved == 2 * 16 * 2 ** 10


def test_plan_single_gate_bytes_follow_touched_subspace():
    n = 20
    for circ, touched in [([C.gate("h", 17)], 2 ** n), ([C.gate("cz", 15, 18)], 2 ** (n - 2)),
                          ([C.gate("cx", 13, 19)], 2 ** (n - 1)), ([C.gate("rz", 16, params=(0.3,))], 2 ** n),
                          ([C.gate("z", 16)], 2 ** (n - 1))]:
        rc, st = plan(n, circ)
        assert rc == B.SV_OK and st.n_passes == 1 and st.n_block_passes == 0
        assert st.bytes_moved == 2 * 16 * touched


def test_plan_fuses_bench_circuits():
    n = 29
    rc, st = plan(n, C.random_u3_layers(n, 40, 0))
    assert rc == B.SV_OK
    # far fewer passes than gates; every pass is one read + write of 8 GiB
    assert st.n_passes < 1720 / 4
    rc, st = plan(n, C.qft(n))
    assert rc == B.SV_OK and st.n_passes < 40
    rc, st = plan(n, C.qft(n), B.SV_C64)
    assert rc == B.SV_OK and st.n_passes < 40


@pytest.mark.parametrize("park", ["0", "1"])
@pytest.mark.parametrize("dtype", [B.SV_C128, B.SV_C64])
def test_planner_handles_benchmark_and_random_circuits(dtype, park, monkeypatch):
    """The planner raises on an internal inconsistency (an op outside its
    stage's window, a phase term on an unmapped position, no progress).
    Plans for the benchmark circuits, their inverses, the 33-qubit circuit,
    the ansatz and random circuits over every op must all succeed, also when
    passes move qubits between state bits (it then also checks that every
    store writes a permutation of its block's qubits)."""
    monkeypatch.setenv("QVEC_PARK", park)
    def inverse(circ):
        out = []
        for g in reversed(circ):
            if g.op == "u3":
                th, ph, la = g.params
                out.append(C.gate("u3", *g.qubits, params=(-th, -la, -ph)))
            elif g.op in ("rx", "ry", "rz", "p", "cp"):
                out.append(C.gate(g.op, *g.qubits, params=(-g.params[0],)))
            else:
                out.append(g)
        return out
    cases = [(29, C.random_u3_layers(29, 40, 0)), (29, inverse(C.random_u3_layers(29, 40, 0))),
             (29, inverse(C.qft(29))), (33, C.random_u3_layers(33, 30, 0, "cz")),
             (24, C.hea(24, 20, C.hea_params(24, 20, 0)))]
    cases += [(18, C.random_mixed_circuit(18, 500, seed)) for seed in range(8)]
    for n, circ in cases:
        rc, st = plan(n, circ, dtype)
        assert rc == B.SV_OK, (n, B.lib().sv_last_error())


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        B.lib()
