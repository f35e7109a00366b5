"""sv_expect_noalloc (the non-allocating variant of sv_expect, for callers
that cannot allocate device memory) through the C ABI, against sv_expect on
the same state and terms: two calls in a row, the second on a smaller state
with fewer terms, then the capacity limit and the empty sum."""
import numpy as np
import pytest
import torch

import circuits as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_15545_amd as qv
    return qv


def load(qv, n, dtype, seed):
    st = qv.State(n, dtype)
    st.tensor.copy_(torch.from_numpy(C.random_state(n, seed)).to(dtype))
    return st


def test_expect_noalloc_matches_expect(qv):
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    cases = [(20, torch.complex128, C.random_pauli_sum(20, 30, 1) + C.zz_x_chain(20)),
             (11, torch.complex64, C.random_pauli_sum(11, 9, 2) + [(0.5, 0, 0), (0.25, 3, 3)])]
    for n, dtype, terms in cases:
        print(f"expect_noalloc n={n} dtype={dtype} terms={len(terms)}", flush=True)
        st = load(qv, n, dtype, n)
        want = st.expect(terms)
        qv.expect_noalloc(st.tensor, terms, out)
        torch.cuda.synchronize()
        assert out.item() == want, (out.item(), want)
        del st


def test_expect_noalloc_limits(qv):
    n = 9
    st = load(qv, n, torch.complex128, 3)
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    # 64 batches: 62 distinct x masks, plus 17 terms on x = 0 (two batches)
    terms = [(0.1 * (x + 1), x, x ^ 5) for x in range(1, 63)] + [(0.01 * k, 0, k) for k in range(17)]
    want = st.expect(terms)
    qv.expect_noalloc(st.tensor, terms, out)
    torch.cuda.synchronize()
    assert out.item() == want
    with pytest.raises(qv.SvError) as e:
        qv.expect_noalloc(st.tensor, terms + [(1.0, 64, 0)], out)
    assert "64 term batches" in str(e.value)
    qv.expect_noalloc(st.tensor, [], out)
    torch.cuda.synchronize()
    assert out.item() == 0.0 == st.expect([])
    assert np.isfinite(st.norm2())
