"""Pins for the FP64 oracle: each check compares it with something other than
itself (the dense Kronecker product of Sec. II Eq. 3-4 through numpy, matrix
exponentials through scipy, closed forms, brute force on tiny inputs, numbers
printed in the paper), so that a dropped term, a wrong sign, a wrong index or a
transposed operand anywhere in the oracle fails at least one of them."""
import math
import os

import numpy as np
import pytest
import scipy.linalg
from hypothesis import given, settings, strategies as st

import circuits as C
import oracle

I2 = np.eye(2, dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)


# ------------------------------------------------------- dense references ---

def kron_1q(u, k, n):
    """Eq. 3: I x ... x u x ... x I with qubit n-1 as the leftmost factor."""
    out = np.eye(1, dtype=np.complex128)
    for q in range(n - 1, -1, -1):
        out = np.kron(out, u if q == k else I2)
    return out


def tensordot_2q(state, u4, t0, t1, n):
    """Apply a 4x4 matrix (index bit(t0) + 2 bit(t1)) by contracting the state
    tensor's axes; axis a of the (2,)*n tensor is qubit n-1-a."""
    psi = state.reshape((2,) * n)
    g = u4.reshape(2, 2, 2, 2)  # (out t1, out t0, in t1, in t0)
    a1, a0 = n - 1 - t1, n - 1 - t0
    out = np.tensordot(g, psi, axes=([2, 3], [a1, a0]))
    # tensordot puts (t1, t0) first; move them back
    out = np.moveaxis(out, [0, 1], [a1, a0])
    return out.reshape(-1)


def dense_apply(state, g, n):
    m = oracle.gate_matrix(g)
    if m.shape == (2, 2):
        return kron_1q(m, g.qubits[0], n) @ state
    return tensordot_2q(state, m, g.qubits[0], g.qubits[1], n)


def pauli_dense(n, xm, zm):
    out = np.eye(1, dtype=np.complex128)
    for q in range(n - 1, -1, -1):
        x, z = (xm >> q) & 1, (zm >> q) & 1
        p = PY if (x and z) else PX if x else PZ if z else I2
        out = np.kron(out, p)
    return out


# ---------------------------------------------------------- gate matrices ---

@pytest.mark.parametrize("theta", [0.0, 0.3, -1.7, 2 * math.pi, 5.1])
def test_rotations_are_pauli_exponentials(theta):
    for op, p in (("rx", PX), ("ry", PY), ("rz", PZ)):
        m = oracle.gate_matrix(C.gate(op, 0, params=(theta,)))
        np.testing.assert_allclose(m, scipy.linalg.expm(-0.5j * theta * p), atol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_u3_is_zyz_decomposition(seed):
    th, ph, la = C.rng_for(seed).uniform(0, 2 * math.pi, 3)
    u3 = oracle.gate_matrix(C.gate("u3", 0, params=(th, ph, la)))
    rz = lambda a: scipy.linalg.expm(-0.5j * a * PZ)
    ry = lambda a: scipy.linalg.expm(-0.5j * a * PY)
    np.testing.assert_allclose(u3, np.exp(0.5j * (ph + la)) * rz(ph) @ ry(th) @ rz(la), atol=1e-14)


def test_fixed_gates_algebra():
    m = {op: oracle.gate_matrix(C.gate(op, 0)) for op in ("h", "x", "y", "z", "s", "sdg", "t", "tdg")}
    np.testing.assert_allclose(m["x"] @ m["y"], 1j * m["z"], atol=1e-15)  # XY = iZ
    np.testing.assert_allclose(m["y"] @ m["z"], 1j * m["x"], atol=1e-15)  # YZ = iX
    np.testing.assert_allclose(m["z"] @ m["x"], 1j * m["y"], atol=1e-15)  # ZX = iY
    np.testing.assert_allclose(m["z"] @ np.array([1, 0]), [1, 0], atol=0)  # Z|0> = |0>
    np.testing.assert_allclose(m["x"] @ np.array([1, 0]), [0, 1], atol=0)  # X|0> = |1>
    np.testing.assert_allclose(m["h"] @ m["x"] @ m["h"], m["z"], atol=1e-15)
    np.testing.assert_allclose(m["h"] @ np.array([1, 0]), [2 ** -0.5, 2 ** -0.5], atol=1e-16)
    np.testing.assert_allclose(m["s"] @ m["s"], m["z"], atol=1e-15)
    np.testing.assert_allclose(m["t"] @ m["t"], m["s"], atol=1e-15)
    np.testing.assert_allclose(m["sdg"], m["s"].conj().T, atol=0)
    np.testing.assert_allclose(m["tdg"], m["t"].conj().T, atol=0)
    u3 = lambda *a: oracle.gate_matrix(C.gate("u3", 0, params=a))
    np.testing.assert_allclose(u3(math.pi / 2, 0, math.pi), m["h"], atol=1e-15)
    np.testing.assert_allclose(u3(math.pi, 0, math.pi), m["x"], atol=1e-15)
    p = lambda a: oracle.gate_matrix(C.gate("p", 0, params=(a,)))
    np.testing.assert_allclose(p(math.pi), m["z"], atol=1e-15)
    np.testing.assert_allclose(p(math.pi / 2), m["s"], atol=1e-15)
    np.testing.assert_allclose(p(math.pi / 4), m["t"], atol=1e-15)


def test_two_qubit_truth_tables():
    """Brute force on the four basis states of two qubits (qubit 0 = bit 0)."""
    n = 2
    for x in range(4):
        b0, b1 = x & 1, (x >> 1) & 1
        cx = oracle.run([C.gate("cx", 0, 1)], n, x0=x)  # control 0, target 1
        assert abs(cx[b0 | ((b1 ^ b0) << 1)] - 1) < 1e-15
        cx10 = oracle.run([C.gate("cx", 1, 0)], n, x0=x)  # control 1, target 0
        assert abs(cx10[(b0 ^ b1) | (b1 << 1)] - 1) < 1e-15
        sw = oracle.run([C.gate("swap", 0, 1)], n, x0=x)
        assert abs(sw[b1 | (b0 << 1)] - 1) < 1e-15
        cz = oracle.run([C.gate("cz", 0, 1)], n, x0=x)
        assert abs(cz[x] - (-1 if x == 3 else 1)) < 1e-15
        cp = oracle.run([C.gate("cp", 0, 1, params=(0.7,))], n, x0=x)
        assert abs(cp[x] - (np.exp(0.7j) if x == 3 else 1)) < 1e-15
    np.testing.assert_allclose(oracle.gate_matrix(C.gate("cp", 0, 1, params=(math.pi,))),
                               oracle.gate_matrix(C.gate("cz", 0, 1)), atol=1e-15)


def test_mat1_decode_is_row_major_closed_form():
    """A MATRIX1 gate reads its 2x2 matrix row-major as (re, im) pairs: the
    non-symmetric [[0, 1], [i, 0]] sends |0> to i|1> and |1> to |0> on its
    qubit (its transpose would send |0> to |1>)."""
    u = np.array([[0, 1], [1j, 0]], dtype=np.complex128)
    g = C.gate("mat1", 2, params=C.matrix_params(u))
    np.testing.assert_array_equal(oracle.gate_matrix(g), u)
    n = 4
    for x in range(1 << n):
        want = np.zeros(1 << n, dtype=np.complex128)
        want[x ^ 4] = 1.0 if (x >> 2) & 1 else 1j
        np.testing.assert_array_equal(oracle.run([g], n, x0=x), want)


# A phased 4-cycle on the two-qubit basis m = bit(t0) + 2 bit(t1):
# |m> -> PH[m] |PERM[m]>. It is neither symmetric nor invariant under
# exchanging t0 and t1, so a transposed decode or a swapped index order
# sends some basis state elsewhere.
PERM4 = (1, 3, 0, 2)
PH4 = (1.0, 1j, -1.0, -1j)


def phased_cycle_4x4():
    m = np.zeros((4, 4), dtype=np.complex128)
    for c in range(4):
        m[PERM4[c], c] = PH4[c]
    return m


@pytest.mark.parametrize("t0,t1", [(3, 1), (0, 4), (4, 0)])
def test_mat2_decode_closed_form(t0, t1):
    u = phased_cycle_4x4()
    g = C.gate("mat2", t0, t1, params=C.matrix_params(u))
    np.testing.assert_array_equal(oracle.gate_matrix(g), u)
    n = 5
    for x in range(1 << n):
        m = ((x >> t0) & 1) + 2 * ((x >> t1) & 1)
        r = PERM4[m]
        y = (x & ~((1 << t0) | (1 << t1))) | ((r & 1) << t0) | ((r >> 1) << t1)
        want = np.zeros(1 << n, dtype=np.complex128)
        want[y] = PH4[m]
        np.testing.assert_array_equal(oracle.run([g], n, x0=x), want)


@pytest.mark.parametrize("seed", range(3))
def test_matrix_gates_against_dense_products_of_their_matrices(seed):
    """MATRIX1 / MATRIX2 gates against Eq. 3-4 built from the unitary itself
    (not from the oracle's decode of it)."""
    n = 6
    rng = C.rng_for(40 + seed)
    s0 = C.random_state(n, seed)
    for k in range(n):
        u = C.random_unitary(2, rng)
        got = oracle.run([C.gate("mat1", k, params=C.matrix_params(u))], n, state=s0)
        np.testing.assert_allclose(got, kron_1q(u, k, n) @ s0, atol=1e-13)
    for a, b in [(0, 5), (5, 0), (2, 3), (4, 1)]:
        u4 = C.random_unitary(4, rng)
        got = oracle.run([C.gate("mat2", a, b, params=C.matrix_params(u4))], n, state=s0)
        np.testing.assert_allclose(got, tensordot_2q(s0, u4, a, b, n), atol=1e-13)


def test_tensordot_reference_orientation():
    """The dense two-qubit reference itself: CNOT as a 4x4 in the basis
    bit(t0) + 2 bit(t1) (control t0) flips t1 exactly where t0 is set."""
    n = 4
    cx = np.zeros((4, 4))
    for m in range(4):
        cx[m ^ (2 if m & 1 else 0), m] = 1
    for x in range(1 << n):
        e = np.zeros(1 << n, dtype=np.complex128)
        e[x] = 1
        got = tensordot_2q(e, cx, 1, 3, n)
        assert got[x ^ (8 if (x >> 1) & 1 else 0)] == 1 and abs(got).sum() == 1


@pytest.mark.parametrize("seed", range(3))
def test_all_matrices_unitary(seed):
    for g in C.random_mixed_circuit(3, 40, seed):
        m = oracle.gate_matrix(g)
        np.testing.assert_allclose(m @ m.conj().T, np.eye(m.shape[0]), atol=1e-14)


# ------------------------------------------- pair loop vs Eq. 3-4 products ---

@settings(max_examples=60, deadline=None)
@given(n=st.integers(1, 7), seed=st.integers(0, 2 ** 31 - 1), n_gates=st.integers(1, 12))
def test_pair_loop_matches_dense_product(n, seed, n_gates):
    circ = C.random_mixed_circuit(n, n_gates, seed)
    s0 = C.random_state(n, seed + 1)
    want = s0.copy()
    for g in circ:
        want = dense_apply(want, g, n)
    got = oracle.run(circ, n, state=s0)
    np.testing.assert_allclose(got, want, atol=1e-12)


@pytest.mark.parametrize("n", [9, 10])
def test_pair_loop_matches_dense_product_every_qubit(n):
    rng = C.rng_for(n)
    s = C.random_state(n, 7)
    for k in range(n):
        u = C.random_unitary(2, rng)
        want = kron_1q(u, k, n) @ s
        got = oracle.apply_1q(s.copy(), n, k, u)
        np.testing.assert_allclose(got, want, atol=1e-12)
    for (a, b) in [(0, n - 1), (n - 1, 0), (3, 5), (5, 4)]:
        u4 = C.random_unitary(4, rng)
        want = tensordot_2q(s, u4, a, b, n)
        got = oracle.apply_2q(s.copy(), n, a, b, u4)
        np.testing.assert_allclose(got, want, atol=1e-12)


def test_controlled_pair_loop_matches_projector_sum():
    """Controlled-u = |0><0|_c x I + |1><1|_c x u (dense, through kron)."""
    n = 5
    rng = C.rng_for(3)
    s = C.random_state(n, 11)
    p0 = np.diag([1, 0]).astype(np.complex128)
    p1 = np.diag([0, 1]).astype(np.complex128)
    for c, t in [(0, 4), (4, 0), (2, 3)]:
        u = C.random_unitary(2, rng)
        full = kron_1q(p0, c, n) + kron_1q(p1, c, n) @ kron_1q(u, t, n)
        got = oracle.apply_1q(s.copy(), n, t, u, ctrl_mask=1 << c)
        np.testing.assert_allclose(got, full @ s, atol=1e-12)


def test_table1_one_pass_half_the_pairs():
    """Sec. III.A / Table I: a one-qubit gate touches 2^(n-1) pairs, each once."""
    n = 12
    s = oracle.basis_state(n, 0)
    for k in (0, 5, 11):
        oracle.reset_pair_updates()
        oracle.apply_1q(s, n, k, np.eye(2))
        assert oracle.pair_updates() == 2 ** (n - 1)


def test_table2_data_size_is_16_bytes_per_amplitude():
    path = os.path.join(os.path.dirname(__file__), "golden", "table2_data_size.txt")
    unit = {"M": 2 ** 20, "G": 2 ** 30}
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 8
    for q, size in rows:
        n = int(q)
        assert int(size[:-1]) * unit[size[-1]] == (1 << n) * 16
        if n <= 20:
            assert oracle.basis_state(n, 0).nbytes == int(size[:-1]) * unit[size[-1]]


# ------------------------------------------------------------ closed forms ---

@pytest.mark.parametrize("n", [1, 2, 7, 16])
def test_hadamard_on_every_qubit_gives_uniform_state(n):
    s = oracle.run([C.gate("h", q) for q in range(n)], n)
    np.testing.assert_allclose(s, np.full(1 << n, 2 ** (-n / 2)), atol=1e-15)


@pytest.mark.parametrize("n", [2, 5, 14])
def test_ghz(n):
    circ = [C.gate("h", 0)] + [C.gate("cx", 0, q) for q in range(1, n)]
    s = oracle.run(circ, n)
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = want[-1] = 2 ** -0.5
    np.testing.assert_allclose(s, want, atol=1e-15)


def qft_closed_form(n, x, ys):
    """alpha_y = 2^(-n/2) exp(2 pi i ((x y) mod 2^n) / 2^n), exact integer phase
    (Python integers, one term at a time)."""
    N = 1 << n
    ph = np.array([(x * int(y)) % N for y in ys], dtype=np.float64) / N
    return np.exp(2j * np.pi * ph) / math.sqrt(N)


@pytest.mark.parametrize("n,seed", [(1, 0), (3, 1), (6, 2), (10, 3), (13, 4)])
def test_qft_of_basis_state(n, seed):
    x = C.random_basis_index(n, seed)
    s = oracle.run(C.qft(n), n, x0=x)
    np.testing.assert_allclose(s, qft_closed_form(n, x, range(1 << n)), atol=1e-12)
    if n <= 10:
        e = np.zeros(1 << n)
        e[x] = 1
        np.testing.assert_allclose(s, np.fft.ifft(e) * math.sqrt(1 << n), atol=1e-12)


@pytest.mark.parametrize("n,seed", [(1, 0), (5, 1), (10, 2), (13, 3)])
def test_oracle_qft_amplitudes_against_circuit_and_fft(n, seed):
    """The oracle's QFT amplitudes (used for every amplitude of the 29-qubit
    check) against the gate-by-gate QFT circuit, numpy's FFT and the
    per-term closed form, also over sub-ranges."""
    x = C.random_basis_index(n, seed)
    N = 1 << n
    amp = oracle.qft_basis_amplitudes(n, x, 0, N)
    np.testing.assert_allclose(amp, oracle.run(C.qft(n), n, x0=x), atol=1e-12)
    e = np.zeros(N)
    e[x] = 1
    np.testing.assert_allclose(amp, np.fft.ifft(e) * math.sqrt(N), atol=1e-12)
    lo, hi = N // 3, N // 3 + max(1, N // 4)
    np.testing.assert_allclose(oracle.qft_basis_amplitudes(n, x, lo, hi), qft_closed_form(n, x, range(lo, hi)),
                               atol=1e-15)


def test_oracle_qft_amplitudes_large_n_exact_phase():
    """At 29 qubits x y reaches 2^58: the integer phase must stay exact
    (Python integers as the reference)."""
    n = 29
    x = C.random_basis_index(n, 0)
    ys = [0, 1, 2, (1 << n) - 1, (1 << n) - 2, 123456789, (1 << 28) + 17]
    for y in ys:
        got = oracle.qft_basis_amplitudes(n, x, y, y + 1)[0]
        assert abs(got - qft_closed_form(n, x, [y])[0]) <= 1e-18


def test_qft_gate_count():
    n = 29
    assert len(C.qft(n)) == n + n * (n - 1) // 2 + n // 2 == 449


@pytest.mark.parametrize("seed", range(3))
def test_norm_and_inverse_round_trip(seed):
    n = 11
    circ = C.random_mixed_circuit(n, 80, seed)
    s = oracle.run(circ, n)
    assert abs(np.vdot(s, s).real - 1) < 1e-13
    back = oracle.run_inverse(circ, n, s)
    want = np.zeros(1 << n, dtype=np.complex128)
    want[0] = 1
    np.testing.assert_allclose(back, want, atol=1e-13)


def test_random_u3_layers_shape():
    circ = C.random_u3_layers(29, 40, seed=0)
    assert len(circ) == 40 * (29 + 14) == 1720
    circ = C.random_u3_layers(33, 30, seed=0, entangler="cz")
    assert len(circ) == 30 * (33 + 16) == 1470
    assert C.random_u3_layers(16, 20, 0) == C.random_u3_layers(16, 20, 0)


# ------------------------------------------------------------- expectation ---

def test_pairwise_sum_matches_fsum():
    v = C.rng_for(1).standard_normal(100003) * 1e3
    assert abs(oracle.pairwise_sum(v) - math.fsum(v)) < 1e-8


def _pairwise_tree(v, lo, n):
    if n <= 8:
        t = 0.0
        for i in range(lo, lo + n):
            t += float(v[i])
        return t
    h = n // 2
    return _pairwise_tree(v, lo, h) + _pairwise_tree(v, lo + h, n - h)


@pytest.mark.parametrize("n", [7, 1000, 65535, 65536, 100003])
def test_pairwise_sum_is_the_halving_tree(n):
    """The oracle sums long ranges on threads; the result must be the plain
    halving tree's, bit for bit (values over ten decades, so that a changed
    order would show)."""
    rng = C.rng_for(n)
    v = rng.standard_normal(n) * 10.0 ** rng.integers(-5, 6, n)
    assert oracle.pairwise_sum(v) == _pairwise_tree(v, 0, n)


@pytest.mark.parametrize("n", [3, 8])
def test_expectation_closed_forms(n):
    H = C.zz_x_chain(n)
    assert len(H) == 2 * n - 1
    assert abs(oracle.expect(oracle.basis_state(n, 0), n, H) - (n - 1)) < 1e-13
    plus = oracle.run([C.gate("h", q) for q in range(n)], n)
    assert abs(oracle.expect(plus, n, H) - 0.5 * n) < 1e-13
    th = C.rng_for(n).uniform(-math.pi, math.pi, n)
    prod = oracle.run([C.gate("ry", q, params=(th[q],)) for q in range(n)], n)
    want = sum(math.cos(th[i]) * math.cos(th[i + 1]) for i in range(n - 1)) + 0.5 * sum(map(math.sin, th))
    assert abs(oracle.expect(prod, n, H) - want) < 1e-13


@pytest.mark.parametrize("seed", range(3))
def test_expectation_matches_dense_pauli_matrices(seed):
    n = 6
    s = C.random_state(n, seed)
    terms = C.random_pauli_sum(n, 12, seed)
    Hd = sum(c * pauli_dense(n, x, z) for c, x, z in terms)
    assert abs(oracle.expect(s, n, terms) - np.vdot(s, Hd @ s).real) < 1e-12
    np.testing.assert_allclose(oracle.apply_pauli_sum(s, n, terms), Hd @ s, atol=1e-12)


# --------------------------------------------------------------- gradients ---

def test_gradient_of_product_state_closed_form():
    n = 6
    th = C.rng_for(5).uniform(-math.pi, math.pi, n)
    circ = [C.gate("ry", q, params=(th[q],), param_index=q) for q in range(n)]
    H = C.zz_x_chain(n)
    want = np.array([
        -math.sin(th[i]) * ((math.cos(th[i - 1]) if i > 0 else 0) + (math.cos(th[i + 1]) if i < n - 1 else 0))
        + 0.5 * math.cos(th[i]) for i in range(n)])
    f, g_adj = oracle.adjoint_grad(circ, n, H, n)
    np.testing.assert_allclose(g_adj, want, atol=1e-13)
    np.testing.assert_allclose(oracle.param_shift_grad(circ, n, H, n), want, atol=1e-13)
    np.testing.assert_allclose(oracle.finite_diff_grad(circ, n, H, n, h=1e-6), want, atol=1e-8)


@pytest.mark.parametrize("n,layers", [(4, 2), (5, 3)])
def test_adjoint_matches_shift_and_differences_on_hea(n, layers):
    th = C.hea_params(n, layers, seed=n)
    circ = C.hea(n, layers, th)
    H = C.zz_x_chain(n)
    P = 2 * n * layers
    f, g_adj = oracle.adjoint_grad(circ, n, H, P)
    assert abs(f - oracle.expect(oracle.run(circ, n), n, H)) < 1e-13
    g_ps = oracle.param_shift_grad(circ, n, H, P)
    g_fd = oracle.finite_diff_grad(circ, n, H, P, h=1e-6)
    np.testing.assert_allclose(g_adj, g_ps, atol=1e-12)
    np.testing.assert_allclose(g_adj, g_fd, atol=1e-7)


def test_rx_gradient_and_shared_parameter():
    """RX and a parameter used by two gates: shift rule sums per occurrence."""
    n = 3
    circ = [C.gate("h", 0), C.gate("rx", 1, params=(0.4,), param_index=0),
            C.gate("cx", 0, 2), C.gate("rx", 2, params=(0.4,), param_index=0),
            C.gate("rz", 0, params=(1.1,), param_index=1)]
    terms = C.random_pauli_sum(n, 6, 3)
    f, ga = oracle.adjoint_grad(circ, n, terms, 2)
    np.testing.assert_allclose(ga, oracle.param_shift_grad(circ, n, terms, 2), atol=1e-13)
    np.testing.assert_allclose(ga, oracle.finite_diff_grad(circ, n, terms, 2), atol=1e-8)
