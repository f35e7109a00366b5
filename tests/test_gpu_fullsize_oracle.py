"""Every amplitude and every gradient of the full-size workloads against the
FP64 oracle (the method is exact: the fused passes must reach the result of
Eq. 3-4, Sec. II, up to rounding).

* 29 qubits, the random U3 + CNOT-matching circuit of depth 40 (1720 gates):
  the oracle runs the whole circuit gate by gate on the host (8 GiB,
  multithreaded), then complex128 (default plan and the qubit-move plan) and
  complex64 are compared with it amplitude by amplitude, in slices.
* 29 qubits, the textbook QFT of a seeded basis state: every amplitude
  against the transform's definition (exact integer phase per index).
* The 24-qubit, 20-layer hardware-efficient ansatz (960 parameters): the
  complex64 and complex128 adjoint gradients against the oracle's adjoint.
* The 20-qubit, 10-layer ansatz (400 parameters): central differences and
  parameter shift on every parameter, through the GPU path.

Progress lines go to stdout (run with -s to see them while a test runs)."""
import math
import time

import numpy as np
import pytest
import torch

import circuits as C
import oracle

pytestmark = pytest.mark.gpu

N29 = 29
SLICE = 1 << 24


@pytest.fixture(scope="module")
def qv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_15545_amd as qv
    return qv


def say(msg):
    print(f"[fullsize-oracle] {msg}", flush=True)


def errors_vs(st, want_slice):
    """(max |st - want|, ||st - want|| / ||want||) over the whole state, one
    slice of 2^24 amplitudes at a time (want_slice(lo, hi) gives the expected
    complex128 values). At 29 qubits a typical amplitude is about 2^-14.5,
    so the relative l2 error is the sharper of the two."""
    N = st.tensor.numel()
    err, d2, w2 = 0.0, 0.0, 0.0
    for lo in range(0, N, SLICE):
        hi = min(N, lo + SLICE)
        got = st.tensor[lo:hi].to(torch.complex128).cpu().numpy()
        want = want_slice(lo, hi)
        diff = np.abs(got - want)
        err = max(err, float(np.max(diff)))
        d2 += float(np.sum(diff * diff))
        w2 += float(np.sum(np.abs(want) ** 2))
    return err, math.sqrt(d2 / w2)


# max-abs (the stated tolerance) and relative l2 bounds per dtype
TOLS = {torch.complex128: (1e-12, 1e-12), torch.complex64: (1e-5, 1e-5)}


@pytest.fixture(scope="module")
def random29_oracle():
    """The oracle's state after the whole 29-qubit depth-40 circuit."""
    n = N29
    circ = C.random_u3_layers(n, 40, seed=0)
    per_layer = n + n // 2
    s = oracle.basis_state(n, 0)
    t0 = time.perf_counter()
    for l in range(40):
        oracle.run_inplace(s, n, circ[l * per_layer:(l + 1) * per_layer])
        say(f"oracle 29q layer {l + 1}/40 ({time.perf_counter() - t0:.0f} s, {oracle.num_threads()} threads)")
    return circ, s


@pytest.mark.timeout(1500)
@pytest.mark.parametrize("dtype,park", [(torch.complex128, "0"), (torch.complex64, "0"), (torch.complex128, "1")])
def test_random_29q_depth40_every_amplitude(qv, random29_oracle, monkeypatch, dtype, park):
    """Config: 29 qubits, random U3 + CNOT matching, depth 40 (the benchmark's
    circuit). park=1 plans passes that move qubits between state bits."""
    circ, want = random29_oracle
    monkeypatch.setenv("QVEC_PARK", park)
    say(f"GPU 29q depth 40 {dtype} park={park}")
    st = qv.State(N29, dtype).set_basis(0).apply(circ)
    err, rel = errors_vs(st, lambda lo, hi: want[lo:hi])
    say(f"max abs error {err:.3e}, relative l2 error {rel:.3e}")
    assert err <= TOLS[dtype][0] and rel <= TOLS[dtype][1], (err, rel)
    assert abs(st.norm2() - 1) <= (1e-12 if dtype == torch.complex128 else 1e-5)
    del st
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_qft_29q_every_amplitude(qv, dtype):
    """Config: the textbook QFT (449 gates) of a seeded basis state at 29
    qubits, every amplitude against alpha_y = 2^(-n/2) e^(2 pi i x y / 2^n)."""
    n = N29
    x = C.random_basis_index(n, seed=0)
    say(f"GPU 29q QFT {dtype}")
    st = qv.State(n, dtype).set_basis(x).apply(C.qft(n))
    err, rel = errors_vs(st, lambda lo, hi: oracle.qft_basis_amplitudes(n, x, lo, hi))
    say(f"max abs error {err:.3e}, relative l2 error {rel:.3e}")
    assert err <= TOLS[dtype][0] and rel <= TOLS[dtype][1], (err, rel)
    del st
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def hea24_oracle():
    n, layers = 24, 20
    th = C.hea_params(n, layers, seed=0)
    circ = C.hea(n, layers, th)
    H = C.zz_x_chain(n)
    P = 2 * n * layers
    t0 = time.perf_counter()
    f, g = oracle.adjoint_grad(circ, n, H, P)
    say(f"oracle adjoint 24q ansatz: {time.perf_counter() - t0:.0f} s")
    return n, circ, H, P, f, g


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype,tol", [(torch.complex64, 1e-4), (torch.complex128, 1e-10)])
def test_hea_24q_960_gradients_against_oracle(qv, hea24_oracle, dtype, tol):
    """Config: 24-qubit ansatz, 20 layers, 960 parameters; every gradient of
    the complex64 (FP64 accumulation) and complex128 adjoint against the
    oracle's adjoint."""
    n, circ, H, P, f_o, g_o = hea24_oracle
    st = qv.State(n, dtype).set_basis(0).apply(circ)
    f, g = st.adjoint_grad(circ, H, P)
    err = float(np.max(np.abs(g - g_o)))
    say(f"24q ansatz {dtype}: f error {abs(f - f_o):.2e}, gradient max abs error {err:.2e}")
    assert abs(f - f_o) <= tol
    assert err <= tol


@pytest.mark.timeout(900)
def test_hea_20q_400_gradients_fd_and_shift(qv):
    """Config: 20-qubit ansatz, 10 layers, 400 parameters, complex128: the
    adjoint gradient against central differences (h = 1e-6) and parameter
    shift on every parameter, both through the GPU path."""
    n, layers = 20, 10
    P = 2 * n * layers
    th = C.hea_params(n, layers, seed=0)
    circ = C.hea(n, layers, th)
    H = C.zz_x_chain(n)
    st = qv.State(n, torch.complex128).set_basis(0).apply(circ)
    f, g = st.adjoint_grad(circ, H, P)
    ev = qv.State(n, torch.complex128)

    def value(thetas):
        return ev.set_basis(0).apply(C.with_params(circ, thetas)).expect(H)

    fd = np.empty(P)
    ps = np.empty(P)
    t0 = time.perf_counter()
    for p in range(P):
        e = np.zeros(P)
        e[p] = 1.0
        fd[p] = (value(th + 1e-6 * e) - value(th - 1e-6 * e)) / 2e-6
        ps[p] = 0.5 * (value(th + 0.5 * math.pi * e) - value(th - 0.5 * math.pi * e))
        if p % 100 == 99:
            say(f"20q ansatz: {p + 1}/{P} parameters ({time.perf_counter() - t0:.0f} s)")
    e_fd = float(np.max(np.abs(fd - g)))
    e_ps = float(np.max(np.abs(ps - g)))
    say(f"20q ansatz: adjoint vs central differences {e_fd:.2e}, vs parameter shift {e_ps:.2e}")
    assert e_fd <= 1e-7
    assert e_ps <= 1e-10
