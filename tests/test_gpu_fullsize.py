"""Full-size checks on the GPU at the benchmark's sizes and launch
configuration (29 qubits complex128 = 8 GiB; 33 qubits complex128 = 128 GiB
with its complex64 twin = 64 GiB).

At 29 qubits the oracle can still run a few dozen gates over the whole
state, and the QFT of a basis state has a closed form for every amplitude
(checked on a seeded sample of indices plus the ends). Deeper circuits and
33 qubits are checked through properties that hold at any size: the norm, the
inverse round trip back to the start state, and complex64 against
complex128 on the device."""
import math

import numpy as np
import pytest
import torch

import circuits as C
import oracle

pytestmark = pytest.mark.gpu


def mem_gib():
    return torch.cuda.get_device_properties(0).total_memory / 2 ** 30


@pytest.fixture(scope="module")
def qv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_15545_amd as qv
    return qv


def qft_amplitudes(n, x, ys):
    N = 1 << n
    ph = np.array([(x * int(y)) % N for y in ys], dtype=np.float64) / N
    return np.exp(2j * np.pi * ph) / math.sqrt(N)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_qft_29q_closed_form_sampled(qv, dtype):
    n = 29
    print(f"qft 29q {dtype}", flush=True)
    x = C.random_basis_index(n, seed=0)
    st = qv.State(n, dtype).set_basis(x).apply(C.qft(n))
    idx = np.unique(np.concatenate([C.rng_for(5).integers(0, 1 << n, size=8192), [0, 1, (1 << n) - 1]]))
    got = st.tensor[torch.from_numpy(idx).cuda()].to(torch.complex128).cpu().numpy()
    tol = 1e-12 if dtype == torch.complex128 else 1e-5
    assert np.max(np.abs(got - qft_amplitudes(n, x, idx))) <= tol
    assert abs(st.norm2() - 1) <= (1e-12 if dtype == torch.complex128 else 1e-5)


def test_random_29q_first_layer_against_oracle(qv):
    """The benchmark's random circuit, first layer (U3 on all 29 qubits and
    14 CNOTs): every amplitude against the oracle."""
    n = 29
    print("random 29q layer 1", flush=True)
    circ = C.random_u3_layers(n, 40, seed=0)[: n + n // 2]
    st = qv.State(n, torch.complex128).set_basis(0).apply(circ)
    want = oracle.run(circ, n)
    torch.cuda.synchronize()
    got = st.tensor.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-12
    del got, want


def test_random_29q_two_layers_sampled_against_oracle(qv):
    """Two layers through the fused path: a seeded sample of amplitudes."""
    n = 29
    circ = C.random_u3_layers(n, 40, seed=0)[: 2 * (n + n // 2)]
    st = qv.State(n, torch.complex128).set_basis(0).apply(circ)
    want = oracle.run(circ, n)
    idx = np.unique(C.rng_for(9).integers(0, 1 << n, size=65536))
    got = st.tensor[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert np.max(np.abs(got - want[idx])) <= 1e-12
    del want


def test_random_29q_depth40_norm_and_round_trip(qv):
    n = 29
    circ = C.random_u3_layers(n, 40, seed=0)
    st = qv.State(n, torch.complex128).set_basis(0).apply(circ)
    assert abs(st.norm2() - 1) <= 1e-12
    inv = inverse(circ)
    st.apply(inv)
    v0 = st.tensor[0].item()
    assert abs(v0 - 1) <= 1e-11
    assert abs(st.norm2() - 1) <= 1e-12


def inverse(circ):
    """The inverse circuit as gate descriptions: reversed order, each gate
    replaced by its inverse (angles negated / reordered, Hermitian gates kept)."""
    out = []
    for g in reversed(circ):
        if g.op == "u3":
            th, ph, la = g.params
            out.append(C.gate("u3", *g.qubits, params=(-th, -la, -ph)))
        elif g.op in ("rx", "ry", "rz", "p", "cp"):
            out.append(C.gate(g.op, *g.qubits, params=(-g.params[0],)))
        elif g.op in ("h", "x", "y", "z", "cx", "cz", "swap"):
            out.append(g)
        else:
            raise ValueError(g.op)
    return out


def test_inverse_helper_is_an_inverse():
    n = 5
    circ = C.random_u3_layers(n, 3, 1) + C.qft(n) + C.random_u3_layers(n, 2, 2, "cz")
    s = oracle.run(inverse(circ), n, state=oracle.run(circ, n))
    assert abs(s[0] - 1) <= 1e-13


@pytest.mark.skipif(not torch.cuda.is_available() or mem_gib() < 200, reason="needs >= 200 GiB of HBM")
def test_33q_c64_vs_c128_and_round_trip(qv):
    """33 qubits, random U3 + CZ matching (3 layers here; the benchmark runs
    30): complex128 (128 GiB) and complex64 (64 GiB) on the same circuit,
    compared on the device, then the complex128 state is run back to e_0."""
    n = 33
    print("33q c128 + c64", flush=True)
    circ = C.random_u3_layers(n, 3, seed=0, entangler="cz")
    a = qv.State(n, torch.complex128).set_basis(0).apply(circ)
    b = qv.State(n, torch.complex64).set_basis(0).apply(circ)
    d = a.compare(b)
    assert d["max_abs"] <= 1e-5
    assert abs(d["norm2_a"] - 1) <= 1e-12 and abs(d["norm2_b"] - 1) <= 1e-5
    fidelity = (d["inner_re"] ** 2 + d["inner_im"] ** 2) / (d["norm2_a"] * d["norm2_b"])
    assert fidelity >= 1 - 1e-9
    del b
    torch.cuda.empty_cache()
    a.apply(inverse(circ))
    assert abs(a.tensor[0].item() - 1) <= 1e-11
    assert abs(a.norm2() - 1) <= 1e-12


def test_24q_instance_of_33q_generator_against_oracle(qv):
    """The error instance: same generator at 24 qubits, depth 30, both dtypes
    against the oracle."""
    n = 24
    circ = C.random_u3_layers(n, 30, seed=0, entangler="cz")
    want = oracle.run(circ, n)
    for dtype, tol in ((torch.complex128, 1e-12), (torch.complex64, 1e-5)):
        st = qv.State(n, dtype).set_basis(0).apply(circ)
        torch.cuda.synchronize()
        got = st.tensor.to(torch.complex128).cpu().numpy()
        assert np.max(np.abs(got - want)) <= tol, dtype


def test_34q_c64_streaming_launches(qv):
    """34 qubits complex64 (128 GiB, 2^34 amplitudes: more than one dispatch
    can hold one per work-item): basis init, unfused X sweeps on low, middle
    and high targets (the lane, one-pair and four-pair forms), and fused
    Hadamards on every qubit."""
    n = 34
    if mem_gib() < 160:
        pytest.skip("needs 128 GiB of device memory")
    print("34q c64", flush=True)
    x = C.random_basis_index(n, 3)
    st = qv.State(n, torch.complex64).set_basis(x)
    targets = [0, 2, 15, 25, 33]
    st.apply([C.gate("x", q) for q in targets], fused=False)
    y = x
    for q in targets:
        y ^= 1 << q
    idx = torch.from_numpy(np.unique(np.concatenate([[0, y, (1 << n) - 1],
                                                     C.rng_for(5).integers(0, 1 << n, size=4096)])))
    got = st.tensor[idx.cuda()].cpu().numpy()
    want = np.where(idx.numpy() == y, 1.0, 0.0)
    assert np.max(np.abs(got - want)) == 0.0
    assert abs(st.norm2() - 1) <= 1e-6
    st.set_basis(0).apply([C.gate("h", q) for q in range(n)])
    got = st.tensor[idx.cuda()].cpu().numpy()
    assert np.max(np.abs(got - 2.0 ** (-n / 2))) <= 1e-5 * 2.0 ** (-n / 2) * 10
    assert abs(st.norm2() - 1) <= 1e-5
    del st
    torch.cuda.empty_cache()
