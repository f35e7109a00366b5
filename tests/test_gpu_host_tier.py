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


def test_host_tier_29q_matches_device_path(qv):
    """At the benchmark's size: a 29-qubit complex128 random circuit (depth 3)
    through the host tier equals the in-HBM fused path, compared on the
    device (the oracle checks the device path at this size elsewhere)."""
    n, c = 29, 26
    print("host tier 29q vs device path", flush=True)
    circ = C.random_u3_layers(n, 3, 0)
    host = torch.zeros(1 << n, dtype=torch.complex128, pin_memory=True)
    host[0] = 1
    stats = qv.host_apply(host, circ, c)
    assert stats["n_chunks"] == 8 and stats["n_passes"] >= 1
    a = qv.State(n, torch.complex128).set_basis(0).apply(circ)
    b = qv.State(n, torch.complex128)
    b.tensor.copy_(host, non_blocking=False)
    del host
    d = a.compare(b)
    assert d["max_abs"] <= 1e-12
    assert abs(d["norm2_b"] - 1) <= 1e-12
    del a, b
    torch.cuda.empty_cache()
