"""The allocation-free solve (stc_solve_noalloc) against stc_solve, through the
C ABI: same factor, same right-hand sides, two calls in a row on one device
(the second on a smaller system with fewer right-hand sides, so it runs on
what the first left in the shared device scratch), each compared bit for bit
with stc_solve and within the solve tolerance with the oracle."""
import ctypes as C

import numpy as np
import pytest

from tests._build_once import ensure_built

ensure_built()

from oracle import oracle as O  # noqa: E402
from paper_2609_29765_amd import stc as S  # noqa: E402
from paper_2609_29765_amd import workloads as W  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SCRATCH_DOUBLES = 1 << 22


def _solve_both(a, B):
    """(stc_solve, stc_solve_noalloc) of the column-major copy of B."""
    L = S.lib()
    st = S._stream_ptr()
    X1 = B.t().contiguous()
    X2 = B.t().contiguous()
    S._check(L.stc_solve(a._h, S._dptr(X1), int(B.shape[1]), st))
    S._check(L.stc_solve_noalloc(a._h, S._dptr(X2), int(B.shape[1]), st))
    torch.cuda.synchronize()
    return X1.t().cpu().numpy(), X2.t().cpu().numpy()


def _case(w, nb, ordering, nrhs, seed):
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=nb, ordering=ordering).bind()
    a.factorize(torch.from_numpy(w.values).cuda())
    assert a.info() == 0
    B = torch.from_numpy(np.random.default_rng(seed).standard_normal((w.n, nrhs))).cuda()
    X1, X2 = _solve_both(a, B)
    o = O.Analysis(w.n, w.colptr, w.rowind, ordering, nb=nb)
    Lo, info = o.factor(w.values)
    assert info == 0
    Xo = o.solve(Lo, B.cpu().numpy())
    return a, X1, X2, Xo


def test_noalloc_matches_solve_two_calls():
    print("noalloc: spatio-temporal arrowhead 10x20x20+8, nb 64, nrhs 12; then GMRF 24x24, nb 32, nrhs 3",
          flush=True)
    big = W.spatiotemporal_arrowhead(T=10, m=20)
    a1, X1, X2, Xo = _case(big, 64, "nd", 12, 1)
    assert np.array_equal(X1, X2)
    assert np.max(np.abs(X2 - Xo)) <= 1e-10 * np.max(np.abs(Xo))
    small = W.gmrf_grid2d(24, 24, 0.1, 0)
    a2, Y1, Y2, Yo = _case(small, 32, "nd", 3, 2)
    assert np.array_equal(Y1, Y2)
    assert np.max(np.abs(Y2 - Yo)) <= 1e-10 * np.max(np.abs(Yo))
    # and the first system again, after the second overwrote the scratch
    B = torch.from_numpy(np.random.default_rng(1).standard_normal((big.n, 12))).cuda()
    Z1, Z2 = _solve_both(a1, B)
    assert np.array_equal(Z2, X2)


def test_noalloc_rejects_sizes_beyond_its_scratch():
    w = W.gmrf_grid2d(32, 32, 0.1, 0)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd").bind()
    a.factorize(torch.from_numpy(w.values).cuda())
    np_ = a.NT * a.nb
    assert np_ * 64 <= SCRATCH_DOUBLES  # this pattern fits with every nrhs
    B = torch.zeros((64, w.n), dtype=torch.float64, device="cuda")
    assert S.lib().stc_solve_noalloc(a._h, S._dptr(B), 65, S._stream_ptr()) == -1  # nrhs > 64
    # a pattern whose padded order times 64 right-hand sides exceeds the scratch
    big = W.gmrf_grid2d(300, 300, 0.1, 0)
    ab = S.Analysis(big.n, big.colptr, big.rowind, nb=64, ordering="nd").bind()
    ab.factorize(torch.from_numpy(big.values).cuda())
    assert ab.NT * ab.nb * 64 > SCRATCH_DOUBLES
    X = torch.zeros((64, big.n), dtype=torch.float64, device="cuda")
    rc = S.lib().stc_solve_noalloc(ab._h, S._dptr(X), 64, S._stream_ptr())
    assert rc == -1 and b"scratch" in S.lib().stc_last_error()
    torch.cuda.synchronize()
    assert float(X.abs().max()) == 0.0  # rejected before any launch


def test_solve_after_failed_factorization_is_nan():
    A = np.diag([4.0, 5.0, -1.0, 3.0])
    A[1, 0] = A[0, 1] = 1.0
    import scipy.sparse as sp
    cp, ri, v = W.lower_csc(sp.csr_matrix(A))
    a = S.Analysis(4, cp, ri, nb=32, ordering="natural").bind()
    a.factorize(torch.from_numpy(v).cuda())
    assert a.info() == 3
    X1, X2 = _solve_both(a, torch.ones((4, 2), dtype=torch.float64, device="cuda"))
    assert np.all(np.isnan(X1)) and np.all(np.isnan(X2))
