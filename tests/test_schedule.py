"""Host checks of the factorization schedule (no device work).

The factorization replays a graph with one node per POTRF, update and TRSM
kernel of a level, whose edges stand for the waits Algorithm 2 performs on
its progress matrix (Sec. 5.3).  stc_check_schedule re-derives from the plan
what every kernel reads and writes and verifies that each two kernels that
touch one object, one of them writing it, are ordered by the graph.  Small
work-group slot counts force split K streams (partial slots folded by a later
task) and separate last-group update nodes, so every kind of edge occurs.

The same patterns go through stc_check_solve_schedule, which replays the
solve sweeps' launches (Sec. 6.7) and verifies that each block is solved once,
after all tiles feeding it, and each tile applied once, after its source
block, with no two items of a launch writing the same rows.  Tile sizes 32
to 256 cover fused levels (step items that apply their tiles) and split
ones (n_b 256 dense: a launch of chunks, then one of diagonal solves).
"""
import numpy as np
import pytest

from tests._build_once import ensure_built

ensure_built()

from paper_2609_29765_amd import stc as S  # noqa: E402
from paper_2609_29765_amd import workloads as W  # noqa: E402


def _check(w, nb, ordering, mode="auto", wg_slots=0, **kw):
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=nb, mode=mode, ordering=ordering, wg_slots=wg_slots, **kw)
    st = a.check_schedule()
    assert st["nodes"] >= 1 and st["objects"] >= 1
    assert st["edges"] >= st["nodes"] - 1 - st["unordered_pairs"] or st["nodes"] == 1
    sv = a.check_solve_schedule()
    assert sv["step_items"] == 2 * a.NT
    assert sv["launches"] == a.solve_launches >= 2
    if a.nb <= 64:  # a step item reads no more than a chunk: every level is one launch
        assert sv["launches"] <= 2 * a.NT
    if a.nb == 256 and a.mode == "dense" and a.NT > 2:  # full 256-row tiles: those levels split
        assert sv["launches"] > 2 * a.NT
    ps = a.plan_stats()
    assert ps["partial_doubles"] <= ps["partial_doubles_unshared"]
    assert (ps["partial_doubles"] == 0) == (ps["split_tasks"] == 0)
    return st


@pytest.mark.parametrize("nb", [32, 64, 128, 256])
@pytest.mark.parametrize("slots", [0, 4, 32])
def test_dense(nb, slots):
    _check(W.dense_spd(3 * nb + 37, 0.3, 1), nb, "natural", mode="dense", wg_slots=slots)


@pytest.mark.parametrize("nb", [32, 64, 128])
@pytest.mark.parametrize("slots", [0, 8])
def test_gmrf_nd(nb, slots):
    _check(W.gmrf_grid2d(40, 40), nb, "nd", wg_slots=slots)


@pytest.mark.parametrize("seed", range(12))
def test_random(seed):
    rng = np.random.default_rng(77 + seed)
    n = int(rng.integers(100, 700))
    w = W.random_spd(n, float(rng.choice([0.005, 0.02, 0.1])), seed, dense_rows=int(rng.integers(0, 3)))
    nb = int(rng.choice([32, 64, 128]))
    ordering = ["natural", "rcm", "nd", "auto"][seed % 4]
    _check(w, nb, ordering, wg_slots=int(rng.choice([0, 2, 16])))


def test_bordered_and_batched_patterns():
    _check(W.spatiotemporal_arrowhead(T=10, m=20, nborder=8), 64, "nd", wg_slots=8)
    _check(W.differentiable_arrowhead(6, 10, 8, 0), 32, "nd")
    _check(W.batched_laplacian3d(m=10, B=2), 64, "nd", wg_slots=4)


@pytest.mark.parametrize("max_split,fold_pct", [(1, 0), (4, 50), (16, 300), (64, 50), (64, 0)])
def test_split_cap_and_fold_weight(max_split, fold_pct):
    """The split-K schedule options on aligned and uniform grids: every plan
    passes both checks; a cap of 1 splits nothing; no split exceeds the cap
    (partial slots per split task <= cap - 1)."""
    w = W.spatiotemporal_arrowhead(T=12, m=20, nborder=8)
    for align in (0, 128):
        st = _check(w, 64, "nd", wg_slots=16, align=align, max_split=max_split, fold_pct=fold_pct)
        a = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd", wg_slots=16, align=align,
                       max_split=max_split, fold_pct=fold_pct)
        ps = a.plan_stats()
        if max_split == 1:
            assert ps["split_tasks"] == 0 and ps["partial_doubles"] == 0
        else:
            assert ps["split_tasks"] > 0
        cap = max_split or 64  # each split task holds (parts - 1) slots of at most 64 x 64 doubles
        assert ps["partial_doubles"] <= ps["split_tasks"] * (cap - 1) * 64 * 64
        assert st["nodes"] == ps["graph_kernels"]


@pytest.mark.parametrize("case", ["dense", "arrowhead_aligned", "laplacian"])
def test_slot_memory_shared(case):
    """Split-K partial slots share memory where the kernel graph orders the
    fold of one slot before the write of the next.  The checker verifies every
    pair of kernels whose slot ranges overlap (slot_pairs of them here, each
    ordered), and the shared memory is a fraction of one slot per split task."""
    if case == "dense":
        w, kw = W.dense_spd(2100, 0.3, 2), dict(nb=128, ordering="natural", mode="dense")
    elif case == "arrowhead_aligned":
        w, kw = W.spatiotemporal_arrowhead(T=12, m=20, nborder=8), dict(nb=64, ordering="nd", align=128)
    else:
        w, kw = W.batched_laplacian3d(m=12, B=2), dict(nb=32, ordering="nd")
    st = _check(w, wg_slots=16, **kw)
    a = S.Analysis(w.n, w.colptr, w.rowind, wg_slots=16, **kw)
    ps = a.plan_stats()
    print(case, ps, st)
    assert ps["split_tasks"] > 4
    assert st["slot_pairs"] > 0
    assert 2 * ps["partial_doubles"] <= ps["partial_doubles_unshared"]


def test_schedule_options_rejected():
    w = W.gmrf_grid2d(8, 8, 0.1, 0)
    for kw in (dict(max_split=-1), dict(max_split=65), dict(fold_pct=-5), dict(batch=-1)):
        with pytest.raises(S.STCError):
            S.Analysis(w.n, w.colptr, w.rowind, nb=32, ordering="nd", **kw)


def test_automatic_tile_size():
    """nb = 0: tile 64, or 256 (n >= 2048) / 128 (n >= 512) when the pattern
    takes the dense route at 64; the result equals an explicit analysis at
    that tile size."""
    cases = [(W.dense_spd(2100, 0.3, 2), "natural", 256), (W.dense_spd(700, 0.3, 2), "natural", 128),
             (W.dense_spd(300, 0.3, 2), "natural", 64), (W.gmrf_grid2d(32, 32), "nd", 64),
             (W.spatiotemporal_arrowhead(T=6, m=20, nborder=8), "nd", 64)]
    for w, ordering, want in cases:
        a = S.Analysis(w.n, w.colptr, w.rowind, nb=0, ordering=ordering)
        assert a.nb == want, (w.n, a.mode, a.nb)
        b = S.Analysis(w.n, w.colptr, w.rowind, nb=want, ordering=ordering)
        assert a.mode == b.mode and a.NT == b.NT and np.array_equal(a.perm(), b.perm())
        assert a.plan_stats() == b.plan_stats()


def test_batch_hint_balances_each_set_for_its_share():
    """stc_opts.batch = B > 1: each value set's split is balanced for
    max(16, wg_slots / B) work-groups, so a 128-member batch splits far less
    than one value set; the plan equals the one for that budget and passes
    the schedule checks."""
    w = W.batched_laplacian3d(m=12, B=2)
    one = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd", align=128)
    big = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd", align=128, batch=128)
    ref = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd", align=128, wg_slots=16)
    assert big.plan_stats() == ref.plan_stats()
    assert big.plan_stats()["split_tasks"] < one.plan_stats()["split_tasks"]
    half = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd", align=128, batch=2)
    assert half.plan_stats() == S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd", align=128,
                                           wg_slots=448).plan_stats()
    _check(w, 64, "nd", align=128, batch=128)


@pytest.mark.parametrize("case", ["random", "dense", "gmrf_nd", "arrowhead_aligned", "differentiable_full", "batched_lap"])
def test_backward_plan(case):
    """stc_check_backward on the reverse-mode plan: every term in exactly one
    task, every tile read written at an earlier level, every tile written
    once, partial slots in bounds and disjoint per level, folds matching the
    parts of their level.  Long tasks are split (folds > 0) where the levels
    hold tasks with many terms."""
    if case == "random":
        w, kw = W.random_spd(500, 0.02, 3), dict(nb=32, ordering="nd")
    elif case == "dense":
        w, kw = W.dense_spd(700, 0.3, 1), dict(nb=128, ordering="natural")
    elif case == "gmrf_nd":
        w, kw = W.gmrf_grid2d(40, 40), dict(nb=64, ordering="nd")
    elif case == "arrowhead_aligned":
        w, kw = W.spatiotemporal_arrowhead(T=12, m=20, nborder=8), dict(nb=64, ordering="nd", align=128)
    elif case == "differentiable_full":
        w, kw = W.differentiable_arrowhead(20, 25, 8, 0), dict(nb=128, ordering="nd", align=512)
    else:
        w, kw = W.batched_laplacian3d(m=12, B=2), dict(nb=32, ordering="nd")
    a = S.Analysis(w.n, w.colptr, w.rowind, **kw)
    st = a.check_backward()
    print(case, st)
    assert st["levels"] >= 3 and st["reads"] > 0
    assert st["levels"] == a.work()["levels_backward"]
    if case in ("differentiable_full", "arrowhead_aligned", "random"):
        assert st["folds"] > 0 and st["slots"] > 0
