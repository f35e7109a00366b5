"""The planner's block passes executed on the host (tests/plan_emulator.cpp):
the load and store mappings, op positions, controls and phase-op encodings as
the register kernel reads them give the same state as applying the gates one
by one, and the structural rules the kernel relies on hold (within-wave
exchanges keep each wave's indices; with no workgroup-wide exchange a wave
stores only where it loaded; a pass stores from the mapping it is in). Runs
on the CPU; plans with and without qubit moves between passes."""
import os
import subprocess

import pytest

import circuits as C
from paper_2508_15545_amd import _binding as B

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2508_15545_amd", "csrc")


@pytest.fixture(scope="module")
def emulator(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("emu") / "plan_emulator")
    cmd = ["g++", "-O2", "-std=c++17", "-w", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{CSRC}",
           "-o", exe, os.path.join(HERE, "plan_emulator.cpp"), os.path.join(CSRC, "planner.cpp"),
           os.path.join(CSRC, "gates.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail("emulator build failed:\n" + r.stderr[-2000:])
    return exe


def gate_lines(circ):
    out = []
    for g in circ:
        q = list(g.qubits) + [0]
        a = list(g.params) + [0.0, 0.0, 0.0]
        out.append(f"{B.OPS[g.op]} {q[0]} {q[1]} {a[0]!r} {a[1]!r} {a[2]!r}")
    return "\n".join(out) + "\n"


CASES = [
    ("cx", 17, 8, 0), ("cx", 18, 10, 1), ("cx", 20, 10, 0), ("cx", 20, 10, 1), ("cx", 20, 10, 2),
    ("cz", 19, 8, 3), ("qft", 16, 0, 0), ("qft", 19, 0, 0), ("hea", 15, 4, 0), ("mixed", 16, 400, 5),
]
# every op the gate-line format carries (no matrix gates): Z, CZ and the
# other diagonals among dense gates on random qubits
MIXED_OPS = tuple(op for op in C.ONE_QUBIT + C.TWO_QUBIT if op not in ("mat1", "mat2"))


@pytest.mark.parametrize("park", [0, 1])
@pytest.mark.parametrize("elem", [16, 8])
@pytest.mark.parametrize("kind,n,depth,seed", CASES)
def test_planned_passes_equal_gate_by_gate(emulator, kind, n, depth, seed, elem, park):
    if kind == "qft":
        circ = C.qft(n)
    elif kind == "hea":
        circ = C.hea(n, depth, C.hea_params(n, depth, seed))
    elif kind == "mixed":
        circ = C.random_mixed_circuit(n, depth, seed, ops=MIXED_OPS)
    else:
        circ = C.random_u3_layers(n, depth, seed, entangler=kind)
    r = subprocess.run([emulator, str(n), str(elem), str(park)], input=gate_lines(circ), capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "structure_errors=0" in r.stdout


@pytest.mark.parametrize("elem", [16, 8])
@pytest.mark.parametrize("coalesce", [2, 4, 5, 6])
@pytest.mark.parametrize("kind,n,depth,seed", [("cx", 18, 8, 4), ("qft", 17, 0, 0), ("mixed", 16, 300, 6)])
def test_coalescing_knob_plans(emulator, kind, n, depth, seed, elem, coalesce):
    """Plans with 2 to 6 low qubits kept in every block (QVEC_COALESCE) give
    the gate-by-gate state."""
    if kind == "qft":
        circ = C.qft(n)
    elif kind == "mixed":
        circ = C.random_mixed_circuit(n, depth, seed, ops=MIXED_OPS)
    else:
        circ = C.random_u3_layers(n, depth, seed, entangler=kind)
    r = subprocess.run([emulator, str(n), str(elem), "0", str(coalesce)], input=gate_lines(circ),
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "structure_errors=0" in r.stdout



@pytest.mark.parametrize("park", [0, 1])
@pytest.mark.parametrize("elem", [16, 8])
@pytest.mark.parametrize("kind,n,depth,seed", [("cx", 20, 10, 0), ("cx", 18, 12, 1), ("cz", 19, 8, 3),
                                               ("qft", 17, 0, 0), ("mixed", 16, 400, 5)])
def test_lookahead_plans(emulator, kind, n, depth, seed, elem, park):
    """Plans whose local sets are chosen with lookahead (8 extra candidates,
    each scored with the pass after it; on by default for states of 4 GiB
    and more) give the gate-by-gate state."""
    if kind == "qft":
        circ = C.qft(n)
    elif kind == "mixed":
        circ = C.random_mixed_circuit(n, depth, seed, ops=MIXED_OPS)
    else:
        circ = C.random_u3_layers(n, depth, seed, entangler=kind)
    coalesce = 3 if elem == 16 else 4
    r = subprocess.run([emulator, str(n), str(elem), str(park), str(coalesce), "8"], input=gate_lines(circ),
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "structure_errors=0" in r.stdout


@pytest.mark.parametrize("elem", [16, 8])
@pytest.mark.parametrize("lookahead", [0, 8, 16])
def test_benchmark_plan_structure(emulator, elem, lookahead):
    """The 29-qubit random U3 + CNOT circuit of depth 40 as planned for the
    benchmark (structure only: the state is too large to emulate here):
    every exchange, exit permutation and store satisfies the kernel's rules,
    among them that no exit permutation moves values between waves (after
    a within-wave exchange other waves may still read those slots)."""
    circ = C.random_u3_layers(29, 40, 0)
    coalesce = 3 if elem == 16 else 4
    r = subprocess.run([emulator, "29", str(elem), "0", str(coalesce), str(lookahead), "1", "1"],
                       input=gate_lines(circ), capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "structure_errors=0" in r.stdout
