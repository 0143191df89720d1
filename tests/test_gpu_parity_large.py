"""GPU parity against the oracle, entry by entry, on the schedules and sizes
the small cases do not reach:

  * forced schedule shapes: few concurrent update work-groups (wg_slots 2,
    4, 16, 32) make the plan split update K streams over several
    work-groups (partial sums folded by the tile's next update) and give
    last-group updates kernels of their own -- on the dense route (n 2048,
    n_b 256) and on the active-column route (the differentiable arrowhead,
    n 12,508, n_b 128);
  * the dense route at n 4096, n_b 256, with the default plan (91 split
    tasks);
  * the spatio-temporal arrowhead at full size (n 101,258, n_b 128);
  * four members of the 24^3 batch (n 13,824, B 128), and a batch where one
    member's values hold a NaN.

Tolerances as in test_gpu_parity: factor per column ||dL_:j||_inf <= 1e-10
||L_:j||_inf on the identical pattern, logdet 1e-12 relative to
max(|ld|, sum |2 log L_ii|), solve 1e-10 relative to the oracle's solution.
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

_ORACLE = {}


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def oracle_factor(key, w, ordering, nb, values=None):
    """Oracle analysis and factor, computed once per key in this process."""
    if key not in _ORACLE:
        print(f"[oracle] {key}: n={w.n} nb={nb} {ordering}", flush=True)
        o = O.Analysis(w.n, w.colptr, w.rowind, ordering, nb=nb)
        Lo, info = o.factor(w.values if values is None else values)
        assert info == 0
        _ORACLE[key] = (o, Lo)
    return _ORACLE[key]


def gpu_vs_oracle(w, ordering, nb, key, wg_slots=0, solve=False, align=0):
    o, Lo = oracle_factor(key, w, ordering, nb)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=nb, ordering=ordering, wg_slots=wg_slots, align=align).bind()
    print(f"[gpu] {key} wg_slots={wg_slots} align={align} {a.plan_stats()}", flush=True)
    a.factorize(dev(w.values))
    assert a.info() == 0
    lp, _ = o.L_pattern()
    factor_close(a.factor(), Lo, lp)
    logdet_close(float(a.logdet().item()), o.logdet(Lo), Lo[lp[:-1]])
    if solve:
        b = np.random.default_rng(5).standard_normal((w.n, 3))
        x = a.solve(dev(b)).cpu().numpy()
        xo = o.solve(Lo, b)
        assert np.max(np.abs(x - xo)) <= 1e-10 * np.max(np.abs(xo))
    return a


@pytest.mark.parametrize("wg_slots", [2, 4, 16, 32])
def test_forced_schedules_dense(wg_slots):
    w = W.dense_spd(2048, 0.2, 0)
    a = gpu_vs_oracle(w, "natural", 256, "dense2048", wg_slots=wg_slots, solve=wg_slots == 16)
    st = a.plan_stats()
    assert a.mode == "dense" and st["separate_last_levels"] > 0
    if wg_slots >= 16:
        assert st["split_tasks"] > 0


@pytest.mark.parametrize("wg_slots", [2, 4, 16])
def test_forced_schedules_semisparse(wg_slots):
    w = W.differentiable_arrowhead(20, 25, 8, 0)
    a = gpu_vs_oracle(w, "nd", 128, "c5nb128", wg_slots=wg_slots, solve=wg_slots == 4)
    st = a.plan_stats()
    assert a.mode == "semisparse" and st["split_tasks"] > 0 and st["separate_last_levels"] > 0


def test_dense_4096_default_plan():
    w = W.dense_spd(4096, 0.2, 0)
    a = gpu_vs_oracle(w, "natural", 256, "dense4096", solve=True)
    assert a.mode == "dense" and a.plan_stats()["split_tasks"] > 0


@pytest.mark.timeout(900)
def test_c3_full_entrywise():
    """The spatio-temporal arrowhead at full size, n_b 128: the configuration
    the bench times (the oracle takes one to two minutes here)."""
    w = W.spatiotemporal_arrowhead()
    gpu_vs_oracle(w, "nd", 128, "c3nb128", solve=True)


@pytest.mark.timeout(900)
def test_c3_full_entrywise_aligned_grid():
    """The same matrix on the grid aligned to subtrees of 512 columns (the
    factor's values do not depend on the grid: same oracle factor)."""
    w = W.spatiotemporal_arrowhead()
    a = gpu_vs_oracle(w, "nd", 128, "c3nb128", solve=True, align=512)
    assert a.align == 512 and a.NT > (w.n + 127) // 128


def test_c4_members_entrywise():
    """Members 0, 1, 63 and 127 of the 24^3 batch, each against the oracle's
    factor of its own values."""
    B = 128
    w = W.batched_laplacian3d(m=24, B=B, seed=0)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd").bind(batch=B)
    ld, info = a.factorize_batched(dev(w.values))
    assert np.all(info.cpu().numpy() == 0)
    ld = ld.cpu().numpy()
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=64)
    lp, _ = o.L_pattern()
    for b in (0, 1, 63, 127):
        Lo, io = o.factor(w.values[b])
        assert io == 0
        factor_close(a.factor(member=b), Lo, lp)
        logdet_close(ld[b], o.logdet(Lo), Lo[lp[:-1]])


def test_batched_nan_in_one_member():
    """A NaN on one diagonal entry of member 5 fails that member alone, at the
    permuted column of that entry, as in the oracle; every other member's
    logdet and factor are bit-identical to the run without the NaN."""
    B = 8
    w = W.batched_laplacian3d(m=10, B=B, seed=3)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd").bind(batch=B)
    ld0, info0 = a.factorize_batched(dev(w.values))
    ld0 = ld0.cpu().numpy()
    assert np.all(info0.cpu().numpy() == 0)
    F0 = [a.factor(member=b) for b in range(B)]
    diag = np.nonzero(w.rowind == np.repeat(np.arange(w.n), np.diff(w.colptr)))[0]
    v = w.values.copy()
    v[5, diag[417]] = np.nan
    ld1, info1 = a.factorize_batched(dev(v))
    ld1, info1 = ld1.cpu().numpy(), info1.cpu().numpy()
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=64)
    _, io = o.factor(v[5])
    col = int(np.nonzero(o.perm() == 417)[0][0]) + 1
    assert io == col and info1[5] == col
    assert np.isnan(ld1[5])
    for b in range(B):
        if b == 5:
            continue
        assert info1[b] == 0 and ld1[b] == ld0[b]
        assert np.array_equal(a.factor(member=b), F0[b])


def test_solve_batched_members():
    """stc_solve_batched: each value set of the 24^3 batch (B = 16 of them,
    1 and 3 right-hand sides) against the oracle's solve with that value
    set's factor; a failed member gives NaN and leaves the others exact."""
    B = 16
    w = W.batched_laplacian3d(m=24, B=B, seed=1)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd").bind(batch=B)
    ld, info = a.factorize_batched(dev(w.values))
    assert np.all(info.cpu().numpy() == 0)
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=64)
    rng = np.random.default_rng(7)
    for nrhs in (1, 3):
        b = rng.standard_normal((B, w.n)) if nrhs == 1 else rng.standard_normal((B, w.n, nrhs))
        x = a.solve_batched(dev(b)).cpu().numpy()
        for m in (0, 5, 15):
            Lo, _ = o.factor(w.values[m])
            xo = o.solve(Lo, b[m])
            assert np.max(np.abs(x[m] - xo)) <= 1e-10 * np.max(np.abs(xo)), (nrhs, m)
        # one value set's solve alone equals the batched one bit for bit
        a1 = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd").bind()
        a1.factorize(dev(w.values[5]))
        assert np.array_equal(a1.solve(dev(b[5])).cpu().numpy(), x[5])
    v = w.values.copy()
    diag = np.nonzero(w.rowind == np.repeat(np.arange(w.n), np.diff(w.colptr)))[0]
    v[3, diag[100]] = -1.0
    a.factorize_batched(dev(v))
    b = rng.standard_normal((B, w.n))
    x = a.solve_batched(dev(b)).cpu().numpy()
    assert np.all(np.isnan(x[3])) and np.all(np.isfinite(np.delete(x, 3, axis=0)))
    with pytest.raises(S.STCError):
        a.solve_batched(dev(np.zeros((B, w.n, 9))))  # nrhs > 8


def test_loaded_analysis_factorizes_identically(tmp_path):
    """A handle read back by stc_load binds and factorizes to the same bits as
    the handle that was saved."""
    w = W.differentiable_arrowhead(20, 25, 8, 0)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=128, ordering="auto").bind()
    a.save(tmp_path / "c5.stc")
    b = S.Analysis.load(tmp_path / "c5.stc").bind()
    v = dev(w.values)
    a.factorize(v)
    b.factorize(v)
    assert np.array_equal(a.factor(), b.factor())
    assert float(a.logdet().item()) == float(b.logdet().item())
    x = dev(np.random.default_rng(2).standard_normal(w.n))
    assert np.array_equal(a.solve(x).cpu().numpy(), b.solve(x).cpu().numpy())
