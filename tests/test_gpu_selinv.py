"""GPU parity of the selected inversion (stc_selinv, stc_get_selinv) against
the oracle's Takahashi recurrence (orc_selinv): every entry of Z = (P A P^T)^-1
on the pattern of L, fill included, and diag(A^-1) in original numbering.

Tolerance: per column of the pattern ||dZ_:j||_inf <= 1e-10 ||Z_:j||_inf
(both sides FP64, sums in different orders; the recurrence amplifies
rounding like a solve, so the factor's per-column bound is used), and the
same for the diagonal relative to max |diag|.  Small cases are also checked
against LAPACK's dense inverse."""
import numpy as np
import pytest
import scipy.sparse as sp

from tests._build_once import ensure_built

ensure_built()

from oracle import oracle as O  # noqa: E402
from paper_2609_29765_amd import stc as S  # noqa: E402
from paper_2609_29765_amd import workloads as W  # noqa: E402
from tests.test_gpu_parity import factor_close  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run(w, ordering, nb, mode="auto", dense_check=False):
    print(f"[gpu] selinv n={w.n} nb={nb} mode={mode} ordering={ordering}", flush=True)
    o = O.Analysis(w.n, w.colptr, w.rowind, ordering, nb=nb, mode=mode)
    Lo, info = o.factor(w.values)
    assert info == 0
    Zo = o.selinv(Lo)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=nb, mode=mode, ordering=ordering).bind()
    a.factorize(dev(w.values))
    diag = a.selinv().cpu().numpy()
    Z = a.selinv_pattern()
    lp, li = o.L_pattern()
    factor_close(Z, Zo, lp)
    p = o.perm()
    dref = np.empty(w.n)
    dref[p] = Zo[lp[:-1]]
    assert np.max(np.abs(diag - dref)) <= 1e-10 * np.max(np.abs(dref))
    if dense_check:
        A = W.dense_from_csc(w.n, w.colptr, w.rowind, w.values)
        Ai = np.linalg.inv(A)
        assert np.max(np.abs(diag - np.diag(Ai))) <= 1e-10 * np.max(np.abs(np.diag(Ai)))
        col = np.repeat(np.arange(w.n), np.diff(lp))
        Ap = Ai[np.ix_(p, p)]
        assert np.max(np.abs(Z - Ap[li, col])) <= 1e-10 * np.max(np.abs(Ai))
    return a


@pytest.mark.parametrize("seed", range(6))
def test_selinv_random(seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(20, 400))
    w = W.random_spd(n, float(rng.choice([0.01, 0.05, 0.2])), seed, dense_rows=int(rng.integers(0, 3)))
    nb = int(rng.choice([32, 64, 128]))
    mode = ["dense", "semisparse"][seed % 2]
    run(w, ["natural", "rcm", "nd"][seed % 3], nb, mode, dense_check=True)


def test_selinv_gmrf_full():
    w = W.gmrf_grid2d(32, 32, 0.1, 0)
    run(w, "nd", 64, dense_check=True)


@pytest.mark.parametrize("nb", [64, 128])
def test_selinv_differentiable_arrowhead_full(nb):
    w = W.differentiable_arrowhead(20, 25, 8, 0)
    run(w, "nd", nb)


def test_selinv_states_and_failure():
    w = W.random_spd(120, 0.05, 4)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=32, ordering="nd").bind()
    a.factorize(dev(w.values))
    with pytest.raises(S.STCError):
        a.selinv_pattern()  # no selected inverse of this factorization yet
    a.selinv()
    a.selinv_pattern()
    a.factorize(dev(w.values))
    with pytest.raises(S.STCError):
        a.selinv_pattern()  # a new factorization invalidates it
    vals = w.values.copy()
    diag = np.nonzero(w.rowind == np.repeat(np.arange(w.n), np.diff(w.colptr)))[0]
    vals[diag[50]] = -3.0
    a.factorize(dev(vals))
    assert a.info() > 0
    assert np.all(np.isnan(a.selinv().cpu().numpy()))
    assert np.all(np.isnan(a.selinv_pattern()))
