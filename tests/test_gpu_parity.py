"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: max-abs amplitude 1e-12 for complex128 and 1e-5 for complex64
(the precision targets of the engine); expectations and gradients as stated
per test. Sizes span n <= b (one block), n = b + 1 (two blocks), several
blocks, and every target qubit including 0, b - 1, b and n - 1."""
import math

import numpy as np
import pytest
import torch

import circuits as C
import oracle

pytestmark = pytest.mark.gpu

TOL = {torch.complex128: 1e-12, torch.complex64: 1e-5}
DTYPES = [torch.complex128, torch.complex64]


@pytest.fixture(scope="module")
def qv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_15545_amd as qv
    return qv


def load(qv, n, psi, dtype):
    st = qv.State(n, dtype)
    st.tensor.copy_(torch.from_numpy(psi).to(dtype))
    return st


def host(st):
    torch.cuda.synchronize()
    return st.tensor.to(torch.complex128).cpu().numpy()


def maxabs(a, b):
    return float(np.max(np.abs(a - b)))


# ------------------------------------------------------------ single gates ---

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 2, 5, 12, 13, 15])
def test_every_op_every_qubit_unfused_and_fused(qv, n, dtype):
    print(f"single gates n={n} dtype={dtype}", flush=True)
    rng = C.rng_for(100 + n)
    psi = C.random_state(n, n)
    qs = sorted({0, n - 1, min(11, n - 1), min(12, n - 1), n // 2})
    gates = []
    for q in qs:
        for op in ("h", "x", "y", "z", "s", "t", "sdg", "tdg"):
            gates.append(C.gate(op, q))
        gates.append(C.gate("rx", q, params=(0.3,)))
        gates.append(C.gate("ry", q, params=(1.3,)))
        gates.append(C.gate("rz", q, params=(2.3,)))
        gates.append(C.gate("p", q, params=(0.9,)))
        gates.append(C.gate("u3", q, params=tuple(rng.uniform(0, 2 * math.pi, 3))))
        gates.append(C.gate("mat1", q, params=C.matrix_params(C.random_unitary(2, rng))))
    if n >= 2:
        for a in qs:
            for b in qs:
                if a == b:
                    continue
                gates.append(C.gate("cx", a, b))
                gates.append(C.gate("cz", a, b))
                gates.append(C.gate("cp", a, b, params=(0.77,)))
                gates.append(C.gate("swap", a, b))
                gates.append(C.gate("mat2", a, b, params=C.matrix_params(C.random_unitary(4, rng))))
    want = psi.copy()
    for g in gates:
        want = oracle.apply_gate(want, n, g)
    for fused in (False, True):
        st = load(qv, n, psi, dtype)
        st.apply(gates, fused=fused)
        err = maxabs(host(st), want)
        assert err <= TOL[dtype], (fused, err)


@pytest.mark.parametrize("dtype", DTYPES)
def test_apply_matrix_with_controls(qv, dtype):
    n = 14
    rng = C.rng_for(5)
    psi = C.random_state(n, 5)
    st = load(qv, n, psi, dtype)
    want = psi.copy()
    for (t, ctrls) in [(0, (13,)), (13, (0, 7)), (12, (3,)), (5, (12, 13))]:
        u = C.random_unitary(2, rng)
        st.apply_matrix([t], u, controls=ctrls)
        mask = sum(1 << c for c in ctrls)
        want = oracle.apply_1q(want, n, t, u, ctrl_mask=mask)
    for (a, b) in [(0, 13), (12, 2)]:
        u4 = C.random_unitary(4, rng)
        st.apply_matrix([a, b], u4)
        want = oracle.apply_2q(want, n, a, b, u4)
    assert maxabs(host(st), want) <= TOL[dtype]


# ------------------------------------------------------------ circuits ---

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,n_gates,seed", [(3, 60, 0), (6, 100, 6), (8, 150, 7), (9, 150, 8), (10, 150, 9),
                                            (11, 200, 1), (12, 200, 2), (13, 300, 3), (16, 400, 4), (19, 300, 5)])
def test_random_mixed_circuits(qv, n, n_gates, seed, dtype):
    print(f"mixed n={n} gates={n_gates} seed={seed} dtype={dtype}", flush=True)
    circ = C.random_mixed_circuit(n, n_gates, seed)
    want = oracle.run(circ, n)
    for fused in (True, False):
        st = qv.State(n, dtype).set_basis(0).apply(circ, fused=fused)
        err = maxabs(host(st), want)
        assert err <= TOL[dtype], (fused, err)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_config_16q_random_u3_cnot_depth20(qv, seed):
    """16 qubits, complex128, depth 20 of U3 on every qubit + CNOT matching."""
    n = 16
    circ = C.random_u3_layers(n, 20, seed)
    want = oracle.run(circ, n)
    st = qv.State(n, torch.complex128).set_basis(0).apply(circ)
    assert maxabs(host(st), want) <= 1e-12


@pytest.mark.parametrize("dtype", DTYPES)
def test_random_circuit_22q_against_oracle(qv, dtype):
    n = 22
    circ = C.random_u3_layers(n, 6, 7, entangler="cz")
    want = oracle.run(circ, n)
    st = qv.State(n, dtype).set_basis(0).apply(circ)
    assert maxabs(host(st), want) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("kind,n,seed", [("cx", 16, 0), ("cx", 18, 5), ("cz", 20, 2), ("qft", 18, 1),
                                         ("mixed", 17, 9)])
def test_qubit_moves_between_passes(qv, monkeypatch, kind, n, seed, dtype):
    """Plans whose passes permute their local qubits at the store (and end
    with every qubit back on its own bit, by an extra pass when needed) give
    the oracle's state, as do plans that keep every qubit in place."""
    print(f"qubit moves {kind} n={n} seed={seed} dtype={dtype}", flush=True)
    if kind == "qft":
        circ = C.qft(n)
    elif kind == "mixed":
        circ = C.random_mixed_circuit(n, 400, seed)
    else:
        circ = C.random_u3_layers(n, 20, seed, entangler=kind)
    x = C.random_basis_index(n, seed)
    want = oracle.run(circ, n, x0=x)
    passes = {}
    for park in ("1", "0"):
        monkeypatch.setenv("QVEC_PARK", park)
        passes[park] = qv.plan_stats(n, dtype, circ)["n_passes"]
        st = qv.State(n, dtype).set_basis(x).apply(circ)
        err = maxabs(host(st), want)
        assert err <= TOL[dtype], (park, err)
    assert passes["1"] <= passes["0"] + 1, passes


KNOBS = [("QVEC_COALESCE", "2"), ("QVEC_COALESCE", "4"), ("QVEC_COALESCE", "5"), ("QVEC_COALESCE", "6"),
         ("QVEC_REG_BITS", "3"), ("QVEC_FUSE", "0"), ("QVEC_WAVE_MODE", "0"), ("QVEC_WAVE_MODE", "1"),
         ("QVEC_BLOCK_QUBITS", "10"), ("QVEC_BLOCK_QUBITS", "11"), ("QVEC_PREFETCH", "1"),
         ("QVEC_BLOCK_KERNEL", "lds"), ("QVEC_PASS_SELECT", "greedy"), ("QVEC_LOOKAHEAD", "8"), ("QVEC_LOOKAHEAD", "16"),
         ("QVEC_STREAM_PLAN", "1"), ("QVEC_FOLD_PERMS", "0")]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("knob,value", KNOBS)
def test_scheduling_knobs_keep_the_state(qv, monkeypatch, knob, value, dtype):
    """Every scheduling knob changes how the passes are formed or run, never
    the result: a mixed circuit and a QFT against the oracle under each."""
    print(f"knob {knob}={value} dtype={dtype}", flush=True)
    monkeypatch.setenv(knob, value)
    n = 17
    for circ, x in ((C.random_mixed_circuit(n, 300, 4), C.random_basis_index(n, 4)), (C.qft(n), 12345)):
        want = oracle.run(circ, n, x0=x)
        st = qv.State(n, dtype).set_basis(x).apply(circ)
        assert maxabs(host(st), want) <= TOL[dtype], (knob, value)


@pytest.mark.parametrize("dtype", DTYPES)
def test_streamed_planning(qv, monkeypatch, dtype):
    """Passes launched as soon as they are planned (on by default for states
    of 1 GiB and more; forced here), with lookahead: calls in a row with no
    wait between them, a call planned whole in between, and a call of about
    115 passes, whose tables outgrow the staging buffer once (the run waits
    for the stream and reuses it from the start), against the oracle."""
    n = 17
    print(f"streamed planning dtype={dtype}", flush=True)
    monkeypatch.setenv("QVEC_LOOKAHEAD", "8")
    psi = C.random_state(n, 17)
    st = load(qv, n, psi, dtype)
    want = psi.copy()
    circs = [("1", C.random_u3_layers(n, 12, 7)), ("1", C.qft(n)), ("0", C.random_mixed_circuit(n, 300, 8)),
             ("1", C.random_u3_layers(n, 8, 9, entangler="cz")), ("1", C.random_u3_layers(n, 300, 10)),
             ("lds", C.random_mixed_circuit(n, 200, 11))]
    for stream, circ in circs:
        # "lds": streamed passes of the LDS-resident block kernel
        monkeypatch.setenv("QVEC_STREAM_PLAN", "1" if stream == "lds" else stream)
        if stream == "lds":
            monkeypatch.setenv("QVEC_BLOCK_KERNEL", "lds")
        st.apply(circ)
        monkeypatch.delenv("QVEC_BLOCK_KERNEL", raising=False)
        want = oracle.run(circ, n, state=want)
    assert maxabs(host(st), want) <= 10 * TOL[dtype]


# ------------------------------------------------------------ closed forms ---

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 13, 20])
def test_uniform_state(qv, n, dtype):
    st = qv.State(n, dtype).set_basis(0).apply([C.gate("h", q) for q in range(n)])
    got = host(st)
    assert np.max(np.abs(got - 2 ** (-n / 2))) <= TOL[dtype] * 2 ** (-n / 2) * 10


def qft_closed_form(n, x, ys):
    N = 1 << n
    ph = np.array([(x * int(y)) % N for y in ys], dtype=np.float64) / N
    return np.exp(2j * np.pi * ph) / math.sqrt(N)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,seed", [(4, 0), (12, 1), (17, 2), (21, 3)])
def test_qft_closed_form(qv, n, seed, dtype):
    x = C.random_basis_index(n, seed)
    st = qv.State(n, dtype).set_basis(x).apply(C.qft(n))
    got = host(st)
    assert maxabs(got, qft_closed_form(n, x, range(1 << n))) <= TOL[dtype]


@pytest.mark.parametrize("n", [3, 16, 24])
def test_ghz(qv, n):
    circ = [C.gate("h", 0)] + [C.gate("cx", 0, q) for q in range(1, n)]
    st = qv.State(n, torch.complex128).set_basis(0).apply(circ)
    got = host(st)
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = want[-1] = 2 ** -0.5
    assert maxabs(got, want) <= 1e-15


def test_set_basis_and_norm(qv):
    for n, x in [(1, 1), (9, 300), (20, 12345)]:
        st = qv.State(n, torch.complex128).set_basis(x)
        got = host(st)
        want = np.zeros(1 << n)
        want[x] = 1
        assert np.array_equal(got, want)
        assert st.norm2() == 1.0


# ------------------------------------------------------------ expectations ---

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,seed", [(1, 0), (6, 1), (14, 2)])
def test_expectation_random_pauli_sums(qv, n, seed, dtype):
    psi = C.random_state(n, seed)
    terms = C.random_pauli_sum(n, 40, seed) + [(0.25, 0, 0), (-0.5, 1, 1), (0.7, 0, 1 << (n - 1))]
    st = load(qv, n, psi, dtype)
    psi_in = host(st)  # the stored (possibly rounded) state
    want = oracle.expect(psi_in, n, terms)
    got = st.expect(terms)
    assert abs(got - want) <= (1e-12 if dtype == torch.complex128 else 1e-12 * len(terms))
    assert abs(st.norm2() - oracle.expect(psi_in, n, [(1.0, 0, 0)])) <= 1e-12


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [5, 14])
def test_apply_pauli_sum(qv, n, dtype):
    psi = C.random_state(n, 3)
    terms = C.random_pauli_sum(n, 25, 3)
    st = load(qv, n, psi, dtype)
    psi_in = host(st)
    out = st.apply_pauli_sum(terms)
    torch.cuda.synchronize()
    got = out.to(torch.complex128).cpu().numpy()
    assert maxabs(got, oracle.apply_pauli_sum(psi_in, n, terms)) <= (1e-12 if dtype == torch.complex128 else 1e-5)


def test_expectation_hea_observable_closed_forms(qv):
    n = 20
    H = C.zz_x_chain(n)
    st = qv.State(n, torch.complex128).set_basis(0)
    assert abs(st.expect(H) - (n - 1)) <= 1e-12
    st.apply([C.gate("h", q) for q in range(n)])
    assert abs(st.expect(H) - 0.5 * n) <= 1e-12


# ------------------------------------------------------------ gradients ---

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,layers", [(3, 2), (8, 3), (13, 2)])
def test_adjoint_matches_oracle(qv, n, layers, dtype):
    print(f"adjoint n={n} layers={layers} dtype={dtype}", flush=True)
    th = C.hea_params(n, layers, seed=n)
    circ = C.hea(n, layers, th)
    H = C.zz_x_chain(n)
    P = 2 * n * layers
    f_o, g_o = oracle.adjoint_grad(circ, n, H, P)
    st = qv.State(n, dtype).set_basis(0).apply(circ)
    f, g = st.adjoint_grad(circ, H, P)
    tol = 1e-10 if dtype == torch.complex128 else 1e-4
    assert abs(f - f_o) <= tol
    assert np.max(np.abs(g - g_o)) <= tol
    # the state was walked back to e_0 by the inverse gates
    back = host(st)
    e0 = np.zeros(1 << n)
    e0[0] = 1
    assert maxabs(back, e0) <= (1e-12 if dtype == torch.complex128 else 1e-5)


@pytest.mark.parametrize("dtype", DTYPES)
def test_adjoint_grouped_z_reads_match_single_reads(qv, monkeypatch, dtype):
    """Z reads sharing one register pass (window, thread and outer-qubit
    reads, 20 qubits, several blocks) give the gradients of reads taken one
    by one, and both match the oracle. A read that waits is taken after ops
    on other qubits, so the two agree to the rounding of those ops (complex64:
    FP32 state updates)."""
    n, layers = 20, 3
    th = C.hea_params(n, layers, seed=11)
    circ = C.hea(n, layers, th)
    H = C.zz_x_chain(n)
    P = 2 * n * layers
    f_o, g_o = oracle.adjoint_grad(circ, n, H, P)
    grads = {}
    for group in ("1", "0"):
        monkeypatch.setenv("QVEC_GROUP_READS", group)
        st = qv.State(n, dtype).set_basis(0).apply(circ)
        f, g = st.adjoint_grad(circ, H, P)
        tol = 1e-10 if dtype == torch.complex128 else 1e-4
        assert abs(f - f_o) <= tol and np.max(np.abs(g - g_o)) <= tol, group
        grads[group] = g
    assert np.max(np.abs(grads["1"] - grads["0"])) <= (1e-12 if dtype == torch.complex128 else 1e-5)


def test_adjoint_rx_and_shared_parameters(qv):
    n = 6
    circ = [C.gate("h", q) for q in range(n)]
    circ += [C.gate("rx", 1, params=(0.4,), param_index=0), C.gate("cx", 0, 2),
             C.gate("rx", 2, params=(0.4,), param_index=0), C.gate("ry", 5, params=(1.1,), param_index=1),
             C.gate("rz", 0, params=(-0.6,), param_index=2), C.gate("cx", 5, 1),
             C.gate("rz", 4, params=(0.2,), param_index=1)]
    terms = C.random_pauli_sum(n, 10, 9)
    f_o, g_o = oracle.adjoint_grad(circ, n, terms, 3)
    st = qv.State(n, torch.complex128).set_basis(0).apply(circ)
    f, g = st.adjoint_grad(circ, terms, 3)
    assert abs(f - f_o) <= 1e-12
    np.testing.assert_allclose(g, g_o, atol=1e-12)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [7, 13])  # 7: LDS block kernel; 13: register kernel
def test_adjoint_diagonal_before_rotation_reads(qv, n, dtype):
    """Rotations directly followed by one-qubit diagonal gates on the same
    qubit (RX then T, RY then RZ, RX then P then S, ...): in the reverse sweep
    the diagonal gate is folded into the rotation and the X/Y read is
    rotated. Checked against the oracle's plain adjoint."""
    print(f"adjoint folds n={n} dtype={dtype}", flush=True)
    rng = C.rng_for(21)
    circ = [C.gate("u3", q, params=tuple(float(x) for x in rng.uniform(0, 6, 3))) for q in range(n)]
    k = 0
    for layer in range(3):
        for q in range(n):
            rot = ("rx", "ry")[int(rng.integers(0, 2))]
            circ.append(C.gate(rot, q, params=(float(rng.uniform(-3, 3)),), param_index=k))
            k += 1
            for _ in range(int(rng.integers(0, 3))):
                d = ("t", "s", "z", "p", "rz", "sdg")[int(rng.integers(0, 6))]
                if d in ("p", "rz"):
                    pi = k if d == "rz" else -1
                    circ.append(C.gate(d, q, params=(float(rng.uniform(-3, 3)),), param_index=pi))
                    k += 1 if d == "rz" else 0
                else:
                    circ.append(C.gate(d, q))
        for q in range(layer % 2, n - 1, 2):
            circ.append(C.gate("cz" if layer % 2 else "cx", q, q + 1))
    terms = C.random_pauli_sum(n, 12, 5)
    f_o, g_o = oracle.adjoint_grad(circ, n, terms, k)
    st = qv.State(n, dtype).set_basis(0).apply(circ)
    f, g = st.adjoint_grad(circ, terms, k)
    tol = 1e-11 if dtype == torch.complex128 else 1e-4
    assert abs(f - f_o) <= tol
    assert np.max(np.abs(g - g_o)) <= tol


def test_config_20q_hea_adjoint_vs_oracle_fd_and_shift(qv):
    """20 qubits, 10 layers, 400 parameters; complex128."""
    n, layers = 20, 10
    P = 2 * n * layers
    th = C.hea_params(n, layers, seed=0)
    circ = C.hea(n, layers, th)
    H = C.zz_x_chain(n)
    st = qv.State(n, torch.complex128).set_basis(0).apply(circ)
    f, g = st.adjoint_grad(circ, H, P)
    f_o, g_o = oracle.adjoint_grad(circ, n, H, P)
    assert abs(f - f_o) <= 1e-10
    assert np.max(np.abs(g - g_o)) <= 1e-10

    def value(thetas):
        s = qv.State(n, torch.complex128).set_basis(0).apply(C.with_params(circ, thetas))
        return s.expect(H)

    sub = C.rng_for(1).choice(P, size=32, replace=False)
    for p in sub:
        e = np.zeros(P)
        e[p] = 1.0
        fd = (value(th + 1e-6 * e) - value(th - 1e-6 * e)) / 2e-6
        ps = 0.5 * (value(th + 0.5 * math.pi * e) - value(th - 0.5 * math.pi * e))
        assert abs(fd - g[p]) <= 1e-7, (p, fd, g[p])
        assert abs(ps - g[p]) <= 1e-10, (p, ps, g[p])


def test_autograd_function(qv):
    n, layers = 6, 2
    th = torch.tensor(C.hea_params(n, layers, seed=4), dtype=torch.float64, requires_grad=True)
    circ = C.hea(n, layers, th.detach().numpy())
    H = C.zz_x_chain(n)
    f = qv.expectation(th, circ, H, n, torch.complex128)
    f.backward()
    f_o, g_o = oracle.adjoint_grad(circ, n, H, th.numel())
    assert abs(f.item() - f_o) <= 1e-12
    np.testing.assert_allclose(th.grad.numpy(), g_o, atol=1e-12)


# ------------------------------------------------------------ device utils ---

def test_compare_c64_against_c128(qv):
    n = 18
    circ = C.random_u3_layers(n, 8, 3, entangler="cz")
    a = qv.State(n, torch.complex128).set_basis(0).apply(circ)
    b = qv.State(n, torch.complex64).set_basis(0).apply(circ)
    d = a.compare(b)
    ha, hb = host(a), host(b)
    assert abs(d["max_abs"] - np.max(np.abs(ha - hb))) <= 1e-15
    assert abs(d["l2"] - np.linalg.norm(ha - hb)) <= 1e-12
    inner = np.vdot(ha, hb)
    assert abs(d["inner_re"] - inner.real) <= 1e-12 and abs(d["inner_im"] - inner.imag) <= 1e-12
    assert abs(d["norm2_a"] - 1) <= 1e-12 and abs(d["norm2_b"] - 1) <= 1e-5
    assert d["max_abs"] <= 1e-5


def test_copy_kernel(qv):
    n = 20
    st = qv.State(n, torch.complex128)
    src = torch.randn(1 << n, dtype=torch.complex128, device="cuda")
    dst = torch.empty_like(src)
    qv.copy(st, dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


@pytest.mark.parametrize("dtype", DTYPES)
def test_degenerate_inputs(qv, dtype):
    """An empty circuit leaves the state bit for bit (both paths); an empty
    Pauli sum is 0; an adjoint call with no parameters returns the
    expectation, an empty gradient and the circuit's input state."""
    n = 13
    psi0 = C.random_state(n, 3)
    st = load(qv, n, psi0, dtype)
    before = host(st)
    st.apply([])
    st.apply([], fused=False)
    assert np.array_equal(host(st), before)
    assert st.expect([]) == 0.0
    circ = C.random_mixed_circuit(n, 60, 3)
    H = C.zz_x_chain(n)
    st.apply(circ)
    f_want = st.expect(H)
    f, g = st.adjoint_grad(circ, H, 0)
    assert g.shape == (0,)
    assert abs(f - f_want) <= (1e-12 if dtype == torch.complex128 else 1e-5)
    assert maxabs(host(st), before) <= TOL[dtype] * 10


def test_bad_arguments_leave_state_untouched(qv):
    n = 8
    st = qv.State(n, torch.complex128).set_basis(3)
    before = host(st)
    with pytest.raises(qv.SvError):
        st.apply([C.gate("h", 0), C.gate("h", 9)])
    with pytest.raises(qv.SvError):
        st.set_basis(1 << n)
    with pytest.raises(qv.SvError):
        st.expect([(1.0, 1 << n, 0)])
    assert np.array_equal(host(st), before)


def test_timing_counts_launches(qv):
    n = 16
    st = qv.State(n, torch.complex128)
    st.timing(True)
    st.timing_reset()
    st.set_basis(0).apply(C.random_u3_layers(n, 3, 0))
    from paper_2508_15545_amd import _binding as B
    launches, ms = st.timing_read(B.KF_BLOCK)
    assert launches >= 1 and ms > 0
    assert st.timing_read(B.KF_INIT)[0] == 1


# ------------------------------------------------------------ matrix layout ---

PERM4 = (1, 3, 0, 2)
PH4 = (1.0, 1j, -1.0, -1j)


def phased_cycle_4x4():
    """|m> -> PH4[m] |PERM4[m]> on the basis m = bit(t0) + 2 bit(t1): neither
    symmetric nor invariant under exchanging t0 and t1."""
    m = np.zeros((4, 4), dtype=np.complex128)
    for c in range(4):
        m[PERM4[c], c] = PH4[c]
    return m


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("fused", [False, True])
def test_matrix_layout_closed_form(qv, dtype, fused):
    """MATRIX1 / MATRIX2 read row-major (re, im) pairs with the two-qubit
    index bit(t0) + 2 bit(t1): [[0, 1], [i, 0]] sends |0> to i|1> and |1> to
    |0> on its qubit, and the phased 4-cycle sends each basis state to one
    known basis state with a known phase. Exact for both dtypes (every entry
    is 0, +-1 or +-i), on qubits inside and outside one block."""
    n = 14
    u1 = np.array([[0, 1], [1j, 0]], dtype=np.complex128)
    u4 = phased_cycle_4x4()
    xs = [0, 1, (1 << n) - 1, 0x2A5C, C.random_basis_index(n, 4)]
    for q in (0, 5, 13):
        g = C.gate("mat1", q, params=C.matrix_params(u1))
        for x in xs:
            st = qv.State(n, dtype).set_basis(x).apply([g], fused=fused)
            want = np.zeros(1 << n, dtype=np.complex128)
            want[x ^ (1 << q)] = 1.0 if (x >> q) & 1 else 1j
            assert np.array_equal(host(st), want), (q, x)
    for t0, t1 in ((3, 1), (0, 13), (13, 0), (12, 6)):
        g = C.gate("mat2", t0, t1, params=C.matrix_params(u4))
        for x in xs:
            m = ((x >> t0) & 1) + 2 * ((x >> t1) & 1)
            r = PERM4[m]
            y = (x & ~((1 << t0) | (1 << t1))) | ((r & 1) << t0) | ((r >> 1) << t1)
            want = np.zeros(1 << n, dtype=np.complex128)
            want[y] = PH4[m]
            st = qv.State(n, dtype).set_basis(x).apply([g], fused=fused)
            assert np.array_equal(host(st), want), (t0, t1, x)


def test_autograd_function_complex64(qv):
    """The autograd path in complex64: FP32 state, FP64 expectation and
    gradient accumulation, against the oracle's FP64 adjoint."""
    n, layers = 10, 3
    th = torch.tensor(C.hea_params(n, layers, seed=6), dtype=torch.float64, requires_grad=True)
    circ = C.hea(n, layers, th.detach().numpy())
    H = C.zz_x_chain(n)
    f = qv.expectation(th, circ, H, n, torch.complex64)
    (2.0 * f).backward()
    f_o, g_o = oracle.adjoint_grad(circ, n, H, th.numel())
    assert abs(f.item() - f_o) <= 1e-5
    assert np.max(np.abs(th.grad.numpy() - 2.0 * g_o)) <= 1e-4


# ------------------------------------------------------------ matrix cores ---

@pytest.mark.parametrize("kind,n,seed", [("mixed", 13, 0), ("mixed", 16, 1), ("cx", 19, 2), ("cz", 22, 3),
                                         ("qft", 17, 4)])
def test_complex64_matrix_core_4x4(qv, monkeypatch, kind, n, seed):
    """complex64 with the 4x4 updates on the matrix cores (QVEC_MFMA=1)
    against the oracle, and against the default path."""
    print(f"mfma {kind} n={n} seed={seed}", flush=True)
    if kind == "qft":
        circ = C.qft(n)
    elif kind == "mixed":
        circ = C.random_mixed_circuit(n, 300, seed)
    else:
        circ = C.random_u3_layers(n, 12, seed, entangler=kind)
    x = C.random_basis_index(n, seed)
    want = oracle.run(circ, n, x0=x)
    got = {}
    for knob in ("1", "0"):
        monkeypatch.setenv("QVEC_MFMA", knob)
        st = qv.State(n, torch.complex64).set_basis(x).apply(circ)
        got[knob] = host(st)
        assert maxabs(got[knob], want) <= 1e-5, knob
    assert maxabs(got["1"], got["0"]) <= 1e-5


@pytest.mark.parametrize("dtype", DTYPES)
def test_sweeps_with_xcd_split(qv, dtype):
    """Unfused one-qubit gates on every target of a 22-qubit state: from 19
    qubits up the sweep places each XCD's workgroups by a split bit that
    depends on the target and the amplitude size, so every target (near
    and far partners, both split rules) is checked against the oracle."""
    n = 22
    print(f"xcd-split sweeps n={n} dtype={dtype}", flush=True)
    rng = C.rng_for(22)
    psi = C.random_state(n, 22)
    gates = [C.gate("mat1", t, params=C.matrix_params(C.random_unitary(2, rng))) for t in range(n)]
    # controlled sweeps: controls below, on and above the split bit
    for a, b in [(11, 20), (20, 11), (13, 21), (13, 20), (14, 20), (3, 19), (21, 0), (17, 16)]:
        gates.append(C.gate("cx", a, b))
    # SWAP, CZ and CP sweeps, which place the XCDs' workgroups the same way
    for a, b in [(3, 19), (20, 11), (21, 17), (7, 12), (0, 21)]:
        gates.append(C.gate("swap", a, b))
        gates.append(C.gate("cz", a, b))
        gates.append(C.gate("cp", b, a, params=(0.7 + a,)))
    want = psi.copy()
    for g in gates:
        want = oracle.apply_gate(want, n, g)
    st = load(qv, n, psi, dtype)
    st.apply(gates, fused=False)
    for (t, ctrls) in [(21, (13, 14)), (20, (0, 16)), (16, (15, 21))]:
        u = C.random_unitary(2, rng)
        st.apply_matrix([t], u, controls=ctrls)
        want = oracle.apply_1q(want, n, t, u, ctrl_mask=sum(1 << c for c in ctrls))
    assert maxabs(host(st), want) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_low_qubit_sweeps(qv, dtype):
    """Unfused gates whose qubits all lie among the lowest five (one
    coalesced lane pass): every two-qubit op on every ordered pair of
    qubits 0..4, one-qubit matrices with one and two low controls, and a
    controlled one-qubit gate mixing low and high qubits; one-qubit gates on
    targets 0..5 and 4x4 gates on a low and a high qubit (lane shuffles)."""
    n = 10
    rng = C.rng_for(77)
    psi = C.random_state(n, 12)
    gates = []
    for a in range(5):
        for b in range(5):
            if a == b:
                continue
            gates.append(C.gate("cx", a, b))
            gates.append(C.gate("cz", a, b))
            gates.append(C.gate("cp", a, b, params=(1.1,)))
            gates.append(C.gate("swap", a, b))
            gates.append(C.gate("mat2", a, b, params=C.matrix_params(C.random_unitary(4, rng))))
    # one-qubit gates on targets 0..5 (lane shuffles within a wave), and 4x4
    # gates on one qubit below 6 and one above (lanes plus a strided half)
    for t in range(6):
        gates.append(C.gate("u3", t, params=tuple(rng.uniform(0, 2 * math.pi, 3))))
        gates.append(C.gate("mat1", t, params=C.matrix_params(C.random_unitary(2, rng))))
    for a, b in [(3, 7), (8, 5), (0, 9), (9, 2), (5, 6)]:
        gates.append(C.gate("mat2", a, b, params=C.matrix_params(C.random_unitary(4, rng))))
    want = psi.copy()
    for g in gates:
        want = oracle.apply_gate(want, n, g)
    st = load(qv, n, psi, dtype)
    st.apply(gates, fused=False)
    for (t, ctrls) in [(0, (3,)), (4, (0, 2)), (2, (1,)), (1, (4, 9)), (7, (0,))]:
        u = C.random_unitary(2, rng)
        st.apply_matrix([t], u, controls=ctrls)
        want = oracle.apply_1q(want, n, t, u, ctrl_mask=sum(1 << c for c in ctrls))
    assert maxabs(host(st), want) <= TOL[dtype]
