"""Parity of the out-of-core tier (sv_host_apply) with the FP64 oracle: the
state stays in pinned host memory and moves through the GPU in chunks.
Sizes force many chunks, many passes, high local qubits chosen per pass,
controlled and two-qubit gates across chunk boundaries, and the one-chunk
case (chunk at least as large as the state)."""
import numpy as np
import pytest
import torch

import circuits as C
import oracle

pytestmark = pytest.mark.gpu

TOL = {torch.complex128: 1e-12, torch.complex64: 1e-5}


@pytest.fixture(scope="module")
def qv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_15545_amd as qv
    return qv


def pinned(psi, dtype):
    t = torch.empty(psi.size, dtype=dtype, pin_memory=True)
    t.copy_(torch.from_numpy(psi).to(dtype))
    return t


def circuit(kind, n, seed):
    if kind == "qft":
        return C.qft(n)
    if kind == "mixed":
        return C.random_mixed_circuit(n, 300, seed)
    return C.random_u3_layers(n, 6, seed, entangler=kind)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("kind,n,c", [("cx", 16, 10), ("cz", 18, 12), ("qft", 17, 11), ("mixed", 15, 8),
                                      ("cx", 12, 14)])
def test_host_tier_matches_oracle(qv, kind, n, c, dtype):
    print(f"host tier {kind} n={n} c={c} dtype={dtype}", flush=True)
    seed = n + c
    circ = circuit(kind, n, seed)
    psi = C.random_state(n, seed)
    want = oracle.run(circ, n, state=psi.copy())
    t = pinned(psi, dtype)
    stats = qv.host_apply(t, circ, c)
    got = t.to(torch.complex128).numpy()
    assert np.max(np.abs(got - want)) <= TOL[dtype]
    cc = min(c, n)
    assert stats["chunk_qubits"] == cc and stats["n_chunks"] == 2 ** (n - cc)
    assert stats["n_passes"] >= 1
    assert stats["bytes_h2d"] == stats["n_passes"] * 2 ** n * t.element_size()


def test_host_tier_round_trip(qv):
    """A circuit and its inverse through the tier bring a basis state back."""
    n, c = 18, 12
    circ = C.random_u3_layers(n, 4, 3)
    inv = []
    for g in reversed(circ):
        if g.op == "u3":
            th, ph, la = g.params
            inv.append(C.gate("u3", *g.qubits, params=(-th, -la, -ph)))
        else:
            inv.append(g)
    t = torch.zeros(1 << n, dtype=torch.complex128, pin_memory=True)
    t[5] = 1
    qv.host_apply(t, circ + inv, c)
    want = np.zeros(1 << n)
    want[5] = 1
    assert np.max(np.abs(t.numpy() - want)) <= 1e-12
