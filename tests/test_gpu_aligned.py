"""GPU parity on tile grids aligned to the elimination tree (stc_opts.align):
every subtree of at least `align` columns with consecutive columns starts on a
tile boundary, the tile before it padded with identity rows.  The factor's
values do not depend on the grid, so each case is checked against the
oracle's factor of the same permuted matrix, as on the uniform grid: factor
entries on the pattern of L, logdet, solve, selected inverse, gradient
values, the failing pivot's column, batched members.

Tolerances as in test_gpu_parity (factor per column 1e-10 relative, logdet
1e-12, solve 1e-10) and test_gpu_selinv / test_gpu_backward (1e-10).  Every
case asserts that the grid really is padded, so that padding rows sit inside
the tiles the kernels touch.
"""
import numpy as np
import pytest

from tests._build_once import ensure_built

ensure_built()

from oracle import oracle as O  # noqa: E402
from paper_2609_29765_amd import stc as S  # noqa: E402
from paper_2609_29765_amd import workloads as W  # noqa: E402
from tests.test_gpu_parity import factor_close, logdet_close  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def padded(a):
    pos = a.grid_positions()
    return int(pos[-1]) + 1 - a.n


def aligned_case(w, ordering, nb, align, mode="auto", solve=True, selinv=False, grad=False, wg_slots=0):
    o = O.Analysis(w.n, w.colptr, w.rowind, ordering, nb=nb, mode=mode)
    Lo, info_o = o.factor(w.values)
    assert info_o == 0
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=nb, mode=mode, ordering=ordering, align=align,
                   wg_slots=wg_slots).bind()
    pad = padded(a)
    print(f"[gpu] aligned n={w.n} nb={nb} align={align} mode={a.mode} ordering={ordering} padding={pad} "
          f"NT={a.NT} levels={a.nlevels}", flush=True)
    assert pad > 0
    assert np.array_equal(a.perm(), o.perm())
    a.factorize(dev(w.values))
    assert a.info() == 0
    lp, li = o.L_pattern()
    factor_close(a.factor(), Lo, lp)
    logdet_close(float(a.logdet().item()), o.logdet(Lo), Lo[lp[:-1]])
    if solve:
        b = np.random.default_rng(11).standard_normal((w.n, 3))
        x = a.solve(dev(b)).cpu().numpy()
        xo = o.solve(Lo, b)
        assert np.max(np.abs(x - xo)) <= 1e-10 * np.max(np.abs(xo))
        x1 = a.solve(dev(b[:, 0].copy())).cpu().numpy()
        assert np.max(np.abs(x1 - xo[:, 0])) <= 1e-10 * np.max(np.abs(xo[:, 0]))
    if selinv:
        Zo = o.selinv(Lo)
        diag = a.selinv().cpu().numpy()
        factor_close(a.selinv_pattern(), Zo, lp)
        dref = np.empty(w.n)
        dref[o.perm()] = Zo[lp[:-1]]
        assert np.max(np.abs(diag - dref)) <= 1e-10 * np.max(np.abs(dref))
    if grad:
        go = o.logdet_grad_values(Lo)
        g = a.logdet_backward(torch.ones(1, dtype=torch.float64, device="cuda")).cpu().numpy()
        assert np.max(np.abs(g - go)) <= 1e-10 * np.max(np.abs(go))
    return a, o, Lo


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 6, 7, 8])  # patterns whose aligned grid is padded
def test_aligned_random(seed):
    rng = np.random.default_rng(1300 + seed)
    n = int(rng.integers(150, 700)) + 250 * (seed % 2)
    nb = [32, 64][seed % 2]
    w = W.random_spd(n, float(rng.choice([0.004, 0.01, 0.02])), 60 + seed, dense_rows=int(rng.integers(0, 3)))
    mode = ["semisparse", "dense"][seed // 2 % 2]
    align = nb if nb == 64 else nb * int(rng.choice([1, 2]))
    aligned_case(w, "nd", nb, align, mode=mode, selinv=seed < 4, grad=seed >= 4)


def test_aligned_gmrf_closed_form():
    w = W.gmrf_grid2d(32, 32, 0.1, 0)
    a, *_ = aligned_case(w, "nd", 64, 128, selinv=True, grad=True)
    lam = 2 - 2 * np.cos(np.pi * np.arange(32) / 32)
    closed = np.log(lam[:, None] + lam[None, :] + 0.1).sum()
    assert abs(float(a.logdet().item()) - closed) <= 1e-12 * abs(closed)


@pytest.mark.parametrize("nb,align", [(64, 256), (128, 512)])
def test_aligned_differentiable_arrowhead(nb, align):
    w = W.differentiable_arrowhead(20, 25, 8, 0)
    aligned_case(w, "nd", nb, align, selinv=nb == 128, grad=True)


@pytest.mark.parametrize("wg_slots", [2, 16])
def test_aligned_forced_schedules(wg_slots):
    w = W.differentiable_arrowhead(10, 20, 8, 1)
    a, *_ = aligned_case(w, "nd", 64, 128, wg_slots=wg_slots)
    st = a.plan_stats()
    assert st["split_tasks"] > 0


def test_aligned_not_spd_reports_the_column():
    """A negative pivot at a column placed after padding: the reported column
    is that column of P A P^T plus one, as in the oracle."""
    w = W.gmrf_grid2d(24, 24, 0.1, 1)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=32, ordering="nd", align=64).bind()
    pos = a.grid_positions()
    assert padded(a) > 0
    shifted = np.nonzero(pos != np.arange(w.n))[0]  # columns placed after some padding
    j = int(shifted[len(shifted) // 2])
    perm = a.perm()
    diag = np.nonzero(w.rowind == np.repeat(np.arange(w.n), np.diff(w.colptr)))[0]
    vals = w.values.copy()
    vals[diag[perm[j]]] = -4.0
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=32)
    _, info_o = o.factor(vals)
    assert 0 < info_o <= j + 1
    a.factorize(dev(vals))
    assert a.info() == info_o
    assert np.isnan(float(a.logdet().item()))
    x = a.solve(dev(np.ones(w.n))).cpu().numpy()
    assert np.all(np.isnan(x))
    a.factorize(dev(w.values))
    assert a.info() == 0


@pytest.mark.parametrize("hint", [0, 4])
def test_aligned_batched_members_and_solves(hint):
    """hint: stc_opts.batch, the schedule balanced for B value sets at once."""
    B = 4
    w = W.batched_laplacian3d(m=16, B=B, seed=2)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd", align=256, batch=hint).bind(batch=B)
    assert padded(a) > 0
    print(f"[gpu] aligned batched n={w.n} B={B} padding={padded(a)}", flush=True)
    ld, info = a.factorize_batched(dev(w.values))
    assert np.all(info.cpu().numpy() == 0)
    ld = ld.cpu().numpy()
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=64)
    lp, _ = o.L_pattern()
    rng = np.random.default_rng(3)
    b = rng.standard_normal((B, w.n, 2))
    x = a.solve_batched(dev(b)).cpu().numpy()
    for m in range(B):
        Lo, _ = o.factor(w.values[m])
        factor_close(a.factor(member=m), Lo, lp)
        logdet_close(ld[m], o.logdet(Lo), Lo[lp[:-1]])
        xo = o.solve(Lo, b[m])
        assert np.max(np.abs(x[m] - xo)) <= 1e-10 * np.max(np.abs(xo))
    # one value set alone, on the same plan, gives the batched member's logdet bit for bit
    a1 = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd", align=256, batch=hint).bind()
    a1.factorize(dev(w.values[2]))
    assert float(a1.logdet().item()) == ld[2]


def test_aligned_solve_noalloc_matches_solve():
    w = W.differentiable_arrowhead(8, 12, 8, 0)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=32, ordering="nd", align=64).bind()
    assert padded(a) > 0
    a.factorize(dev(w.values))
    b = dev(np.random.default_rng(4).standard_normal((w.n, 2)))
    x = a.solve(b)
    X = b.t().clone(memory_format=torch.contiguous_format)
    S._check(S.lib().stc_solve_noalloc(a._h, S._dptr(X), 2, S._stream_ptr()))
    assert torch.equal(X.t(), x)


def test_supernodal_route_gmrf_closed_form():
    """The 100 x 100 2-D GMRF routes supernodal at tile 128 and is factorized
    on the grid aligned at n_b: factor, logdet (also against its closed form),
    solve, selected inverse and gradient against the oracle, which applies
    the same route rule."""
    w = W.gmrf_grid2d(100, 100, 0.1, 0)
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=128)
    Lo, info_o = o.factor(w.values)
    assert info_o == 0 and o.route == "supernodal"
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=128, ordering="nd").bind()
    print(f"[gpu] supernodal route gmrf100 nb=128 align={a.align} padding={padded(a)} levels={a.nlevels}", flush=True)
    assert a.route == "supernodal" and a.align == 128 and padded(a) > 0
    assert np.array_equal(a.grid_positions(), o.positions())
    a.factorize(dev(w.values))
    assert a.info() == 0
    lp, _ = o.L_pattern()
    factor_close(a.factor(), Lo, lp)
    ld = float(a.logdet().item())
    logdet_close(ld, o.logdet(Lo), Lo[lp[:-1]])
    lam = 2 - 2 * np.cos(np.pi * np.arange(100) / 100)
    closed = np.log(lam[:, None] + lam[None, :] + 0.1).sum()
    assert abs(ld - closed) <= 1e-12 * abs(closed)
    b = np.random.default_rng(12).standard_normal((w.n, 2))
    x = a.solve(dev(b)).cpu().numpy()
    xo = o.solve(Lo, b)
    assert np.max(np.abs(x - xo)) <= 1e-10 * np.max(np.abs(xo))
    Zo = o.selinv(Lo)
    diag = a.selinv().cpu().numpy()
    factor_close(a.selinv_pattern(), Zo, lp)
    dref = np.empty(w.n)
    dref[o.perm()] = Zo[lp[:-1]]
    assert np.max(np.abs(diag - dref)) <= 1e-10 * np.max(np.abs(dref))
    go = o.logdet_grad_values(Lo)
    g = a.logdet_backward(torch.ones(1, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert np.max(np.abs(g - go)) <= 1e-10 * np.max(np.abs(go))
