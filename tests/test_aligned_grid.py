"""The tile grid aligned to the elimination tree (stc_opts.align), on the CPU.

Rule: every subtree T(r) of the elimination tree of P A P^T (r and its
descendants) with at least `align` columns whose columns are consecutive
starts on a tile boundary; the columns before it are padded up to the next
multiple of n_b.  Tiles, kd and Algorithm 1's task list are then those of
the padded grid; features, route and storage mode stay those of the uniform
grid.

Pinned here by hand-worked trees (expected positions, tiles and task lists
derived in the docstrings, not by calling either implementation), then the
analyser against the oracle's independent implementation bit for bit on
random patterns and on every workload at full size.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from tests._build_once import ensure_built

ensure_built()

from oracle import oracle as O  # noqa: E402
from paper_2609_29765_amd import stc as S  # noqa: E402
from paper_2609_29765_amd import workloads as W  # noqa: E402
from tests.test_analyser_vs_oracle import _compare  # noqa: E402

POTRF, SYRK, TRSM, GEMM = 1, 2, 3, 4


def _pattern(n, edges):
    """Lower CSC of an SPD pattern with the given edges (plus the diagonal)."""
    r = [max(a, b) for a, b in edges] + list(range(n))
    c = [min(a, b) for a, b in edges] + list(range(n))
    A = sp.csc_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    A.sort_indices()
    return np.asarray(A.indptr, np.int64), np.asarray(A.indices, np.int32)


def _both(n, edges, nb, align, ordering="natural"):
    cp, ri = _pattern(n, edges)
    a = S.Analysis(n, cp, ri, nb=nb, ordering=ordering, mode="semisparse", align=align)
    o = O.Analysis(n, cp, ri, ordering, nb=nb, mode="semisparse", align=align)
    return a, o


def _path(lo, hi):
    return [(j, j + 1) for j in range(lo, hi)]


def test_two_paths_and_a_separator():
    """Path A on columns 0..39, path B on 40..79, column 80 joined to 39 and
    79; natural order, n_b 32, align 40.  The elimination tree is A's chain
    and B's chain, both hanging from 80, with no fill.  T(39) = {0..39} and
    T(79) = {40..79} have 40 consecutive columns each (T(80) starts at 0 as
    well), so the aligned starts are 0 and 40: column 40 moves from position
    40 to the next boundary, 64, and every later column follows it
    (positions 64..104, 105 positions, 4 tiles).  Blocks: 0 = columns 0..31,
    1 = columns 32..39 and padding, 2 = columns 40..71, 3 = columns 72..80 and
    padding.  Off-diagonal entries crossing blocks: L(32,31) -> tile (1,0)
    local row 0; L(80,39) -> tile (3,1) local row 104 - 96 = 8; L(72,71) ->
    tile (3,2) local row 0.  Algorithm 1 on these tiles: k=0 POTRF, TRSM(1,0);
    k=1 SYRK from 0, POTRF, TRSM(3,1); k=2 POTRF, TRSM(3,2); k=3 SYRK from 1
    and from 2, POTRF.  On the uniform grid the same pattern gives the tiles
    (1,0) rows {0} and (2,1) rows {0, 16}: block 2 couples B to A."""
    edges = _path(0, 39) + _path(40, 79) + [(39, 80), (79, 80)]
    a, o = _both(81, edges, 32, 40)
    expect_pos = np.r_[np.arange(40), np.arange(64, 105)]
    for x in (a, o):
        assert np.array_equal(x.grid_positions() if x is a else x.positions(), expect_pos)
        assert x.NT == 4
    ta = a.tiles()
    assert list(zip(ta["m"], ta["k"])) == [(1, 0), (3, 1), (3, 2)]
    assert [list(ta["rows"][ta["roff"][t]:ta["roff"][t + 1]]) for t in range(3)] == [[0], [8], [0]]
    assert list(ta["kd"]) == [1, 1, 1, 1]
    expect_tasks = [(POTRF, -1, 0, -1), (TRSM, 1, 0, -1), (SYRK, -1, 1, 0), (POTRF, -1, 1, -1),
                    (TRSM, 3, 1, -1), (POTRF, -1, 2, -1), (TRSM, 3, 2, -1), (SYRK, -1, 3, 1),
                    (SYRK, -1, 3, 2), (POTRF, -1, 3, -1)]
    assert [tuple(t) for t in a.tasks()] == expect_tasks
    assert [tuple(t) for t in o.tasks()] == expect_tasks
    # uniform grid of the same pattern
    u, uo = _both(81, edges, 32, 0)
    tu = u.tiles()
    assert list(zip(tu["m"], tu["k"])) == [(1, 0), (2, 1)]
    assert list(tu["rows"][tu["roff"][1]:tu["roff"][2]]) == [0, 16]
    assert np.array_equal(u.grid_positions(), np.arange(81))
    # features, route and mode are those of the uniform grid
    assert (a.phi, a.rho, a.sigma, a.route, a.mode, a.tact) == (u.phi, u.rho, u.sigma, u.route, u.mode, u.tact)


def test_subtree_with_a_gap_is_not_aligned():
    """Columns 0..4 form a path of their own; 5..14 a path, 15 an isolated
    column, 16..25 a path, and 26 joins 14 and 25.  T(26) = {5..14, 16..26}
    has 21 columns but its smallest is 5 while 26 - 21 + 1 = 6: column 15
    sits inside its range, so with align 15 no subtree qualifies (the paths
    have 5, 10 and 10 columns) and the grid is the uniform one.  When 15
    joins path B instead (15..25 a path), T(26) = {5..26} is consecutive with
    22 columns: column 5 starts tile 1 (position 32) and every later column
    shifts by 27."""
    edges = _path(0, 4) + _path(5, 14) + _path(16, 25) + [(14, 26), (25, 26)]
    a, o = _both(27, edges, 32, 15)
    assert np.array_equal(a.grid_positions(), np.arange(27))
    assert np.array_equal(o.positions(), np.arange(27))
    edges2 = _path(0, 4) + _path(5, 14) + _path(15, 25) + [(14, 26), (25, 26)]
    a2, o2 = _both(27, edges2, 32, 15)
    expect = np.r_[np.arange(5), np.arange(5, 27) + 27]
    assert np.array_equal(a2.grid_positions(), expect)
    assert np.array_equal(o2.positions(), expect)
    assert a2.NT == 2


def test_threshold_is_inclusive_and_boundaries_are_kept():
    """Two paths of 32 columns (0..31, 32..63) under a separator 64, n_b 32:
    the second subtree already starts on a boundary, so no padding for any
    align; with align 33 neither path qualifies (32 < 33).  Paths of 30
    (0..29, 30..59) and separator 60: align 30 pads column 30 to position 32
    (size 30 >= 30); align 31 leaves it."""
    e1 = _path(0, 31) + _path(32, 63) + [(31, 64), (63, 64)]
    for al in (1, 32, 33):
        a, o = _both(65, e1, 32, al)
        assert np.array_equal(a.grid_positions(), np.arange(65))
        assert np.array_equal(o.positions(), np.arange(65))
    e2 = _path(0, 29) + _path(30, 59) + [(29, 60), (59, 60)]
    a, o = _both(61, e2, 32, 30)
    expect = np.r_[np.arange(30), np.arange(30, 61) + 2]
    assert np.array_equal(a.grid_positions(), expect) and np.array_equal(o.positions(), expect)
    a, o = _both(61, e2, 32, 31)
    assert np.array_equal(a.grid_positions(), np.arange(61)) and np.array_equal(o.positions(), np.arange(61))


@pytest.mark.parametrize("seed", range(24))
def test_random_patterns_aligned(seed):
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(40, 900))
    w = W.random_spd(n, float(rng.choice([0.003, 0.01, 0.03])), seed, dense_rows=int(rng.integers(0, 3)))
    ordering = ["nd", "auto", "rcm", "nd"][seed % 4]
    nb = int(rng.choice([32, 64]))
    mode = ["auto", "dense", "semisparse"][seed % 3]
    align = int(rng.choice([1, 16, nb, 2 * nb]))
    _compare(w, ordering, nb, mode, align=align)


@pytest.mark.parametrize("name,nb,align", [("c1", 64, 128), ("c5", 128, 512), ("c5", 64, 256),
                                           ("c4", 64, 256), ("c3", 128, 512), ("c3", 256, 1024)])
def test_workloads_full_size_aligned(name, nb, align):
    w = {"c1": lambda: W.gmrf_grid2d(32, 32, 0.1, 0),
         "c5": lambda: W.differentiable_arrowhead(20, 25, 8, 0),
         "c4": lambda: W.batched_laplacian3d(m=24, B=1),
         "c3": lambda: W.spatiotemporal_arrowhead()}[name]()
    a, o = _compare(w, "nd", nb, align=align)
    u = S.Analysis(w.n, w.colptr, w.rowind, nb=nb, ordering="nd")
    assert a.NT > u.NT and a.align == align and u.align == 0  # padded
    assert (a.phi, a.rho, a.sigma, a.route, a.mode, a.tact) == (u.phi, u.rho, u.sigma, u.route, u.mode, u.tact)
    # the tile DAG is far shallower than on the uniform grid
    assert a.nlevels < u.nlevels / 2


def test_rejects_negative_align():
    w = W.gmrf_grid2d(8, 8, 0.1, 0)
    with pytest.raises(S.STCError):
        S.Analysis(w.n, w.colptr, w.rowind, nb=32, ordering="nd", align=-1)


def test_supernodal_route_takes_the_tree_aligned_grid():
    """Patterns the selector routes supernodal (mode AUTO) are factorized on
    fixed-width tiles aligned to the elimination tree at n_b (their tiles
    follow the fill, Sec. 5.4); a fixed mode or an explicit grid overrides
    it.  The 100 x 100 2-D GMRF routes supernodal at tile 128 (rho < 0.15,
    phi > 2); analyser and oracle apply the rule independently and agree bit
    for bit."""
    w = W.gmrf_grid2d(100, 100, 0.1, 0)
    a, o = _compare(w, "nd", 128)
    assert a.route == o.route == "supernodal" and a.mode == "semisparse"
    assert a.align == 128
    assert not np.array_equal(a.grid_positions(), np.arange(w.n))
    u = S.Analysis(w.n, w.colptr, w.rowind, nb=128, ordering="nd", mode="semisparse")
    assert u.route == "supernodal" and u.align == 0
    assert np.array_equal(u.grid_positions(), np.arange(w.n))
    e = S.Analysis(w.n, w.colptr, w.rowind, nb=128, ordering="nd", align=512)
    assert e.align == 512
    # a semisparse-routed pattern keeps the uniform grid by default
    s64 = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd")
    assert s64.route == "semisparse" and s64.align == 0
