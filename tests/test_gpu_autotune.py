"""The autotuner (tile size, storage mode and schedule slots chosen by timing
captured replays on the caller's values): every candidate is timed and
reported, candidates share one ordering, the winner is bound and is the
fastest row of the table, and its factorization matches the oracle."""
import numpy as np
import pytest

from tests._build_once import ensure_built

ensure_built()

from oracle import oracle as O  # noqa: E402
from paper_2609_29765_amd import workloads as W  # noqa: E402
from paper_2609_29765_amd.autotune import autotune  # noqa: E402
from tests.test_gpu_parity import factor_close  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_autotune_tiles_modes_and_slots():
    w = W.spatiotemporal_arrowhead(T=10, m=20, nborder=8)
    v = torch.from_numpy(w.values).cuda()
    a, table = autotune(w.n, w.colptr, w.rowind, v, nbs=(32, 64, 128), modes=("semisparse", "dense"),
                        ordering="nd", trials=2, slots=(0, 16))
    assert len(table) == 3 * 2 * 2
    assert {(r["nb"], r["mode"], r["wg_slots"]) for r in table} == \
        {(nb, m, s) for nb in (32, 64, 128) for m in ("semisparse", "dense") for s in (0, 16)}
    best = min(table, key=lambda r: r["ms"])
    assert (a.nb, a.mode) == (best["nb"], best["mode"])
    a.factorize(v)
    assert a.info() == 0
    o = O.Analysis(w.n, w.colptr, w.rowind, "given", nb=a.nb, mode=a.mode, perm=a.perm())
    Lo, info = o.factor(w.values)
    assert info == 0
    lp, _ = o.L_pattern()
    factor_close(a.factor(), Lo, lp)


def test_autotune_tile_grids():
    """The grid axis: uniform and two aligned grids per tile size; every
    candidate is reported with its alignment in columns, the winner is the
    fastest row, and its factorization matches the oracle."""
    w = W.differentiable_arrowhead(12, 20, 8, 0)
    v = torch.from_numpy(w.values).cuda()
    a, table = autotune(w.n, w.colptr, w.rowind, v, nbs=(32, 64), ordering="nd", trials=2, aligns=(0, 2, 4))
    assert {(r["nb"], r["align"]) for r in table} == {(nb, f * nb) for nb in (32, 64) for f in (0, 2, 4)}
    best = min(table, key=lambda r: r["ms"])
    assert (a.nb, a.align, a.nlevels) == (best["nb"], best["align"], best["levels"])
    a.factorize(v)
    assert a.info() == 0
    o = O.Analysis(w.n, w.colptr, w.rowind, "given", nb=a.nb, mode=a.mode, perm=a.perm())
    Lo, info = o.factor(w.values)
    assert info == 0
    factor_close(a.factor(), Lo, o.L_pattern()[0])


def test_autotune_fold_weight_round():
    """The second round tries each fold weight on the first round's winner
    only; the returned analysis is the fastest row."""
    w = W.differentiable_arrowhead(12, 20, 8, 0)
    v = torch.from_numpy(w.values).cuda()
    a, table = autotune(w.n, w.colptr, w.rowind, v, nbs=(32, 64), ordering="nd", trials=2, aligns=(0, 2),
                        folds=(0, 50, 300))
    assert len(table) == 2 * 2 + 2
    first = min(table[:4], key=lambda r: r["ms"])
    assert all((r["nb"], r["align"]) == (first["nb"], first["align"]) for r in table[4:])
    assert [r["fold_pct"] for r in table[4:]] == [50, 300]
    best = min(table, key=lambda r: r["ms"])
    assert (a.nb, a.align, a.nlevels) == (best["nb"], best["align"], best["levels"])
    a.factorize(v)
    assert a.info() == 0


def test_autotune_batched_objective():
    w = W.batched_laplacian3d(m=10, B=4, seed=0)
    V = torch.from_numpy(w.values).cuda()
    a, table = autotune(w.n, w.colptr, w.rowind, V, nbs=(32, 64), ordering="nd", batched=True, trials=2)
    assert len(table) == 2 and a.batch == 4
    ld, info = a.factorize_batched(V)
    assert np.all(info.cpu().numpy() == 0)
