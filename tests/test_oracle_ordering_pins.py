"""Hand-worked pins of the oracle's ordering choice (Sec. 3), pseudo-peripheral
root, tile features (Sec. 5.1) and multi-column solve.

Every expected value below is derived by hand in the docstring of its test and
re-derived in the test body by small independent code (breadth-first search,
the elimination game, tile counting written here); nothing is computed by
calling the oracle.  The oracle's answer is then compared with it, and the
same patterns go through the product's host analyser, which must agree bit
for bit.

The AUTO rule being pinned (the reading of Sec. 3's candidate scoring this
build takes, since the paper gives no constants): candidates NATURAL, RCM, ND
are scored by (nnz(L), active tiles, mean occupancy rho).  If NATURAL's rho <
0.15, the candidate of least nnz(L) wins.  Otherwise the candidate of fewest
active tiles wins, unless some candidate's nnz(L) is at most half of that
winner's, in which case the least such nnz(L) wins.  Finally, when n >= 50,000
and ND's nnz(L) is within 1.25x of the least, ND wins.  Ties go to the earlier
candidate.  Orderings are numbered NATURAL 0, RCM 1, ND 2.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from tests._build_once import ensure_built

ensure_built()

from oracle import oracle as O  # noqa: E402
from paper_2609_29765_amd import stc as S  # noqa: E402
from paper_2609_29765_amd import workloads as W  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NAT, RCM, ND = 0, 1, 2


# ---------------------------------------------------------------------------
# independent helpers (no oracle code)
# ---------------------------------------------------------------------------

def _spd_from_edges(n, edges):
    """Lower CSC of diag(degree + 1) - adjacency: SPD, with the given graph."""
    r = np.array([e[0] for e in edges] + [e[1] for e in edges], np.int64)
    c = np.array([e[1] for e in edges] + [e[0] for e in edges], np.int64)
    A = sp.csr_matrix((-np.ones(r.size), (r, c)), shape=(n, n))
    deg = np.asarray((A != 0).sum(axis=1)).ravel()
    A = A + sp.diags(deg + 1.0)
    return W.lower_csc(A)


def _path_edges(seq):
    return [(int(a), int(b)) for a, b in zip(seq[:-1], seq[1:])]


def _eliminate(n, edges, perm):
    """Elimination game on the graph under `perm` (perm[new] = old): for each
    new column j, the set of rows i > j of L (new numbering)."""
    inv = np.empty(n, np.int64)
    inv[np.asarray(perm)] = np.arange(n)
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[inv[a]].add(int(inv[b]))
        adj[inv[b]].add(int(inv[a]))
    cols = []
    for j in range(n):
        hi = sorted(x for x in adj[j] if x > j)
        cols.append(hi)
        for a in hi:
            for b in hi:
                if a != b:
                    adj[a].add(b)
    return cols


def _scores(n, edges, perm, nb):
    """(nnz(L), active tiles, rho, phi, sigma, tiles) from the elimination
    game: tiles maps (m, k) to the sorted local active rows of block m."""
    cols = _eliminate(n, edges, perm)
    lnz = n + sum(len(c) for c in cols)
    tiles = {}
    rowcount = np.ones(n, np.int64)
    for j, c in enumerate(cols):
        for i in c:
            rowcount[i] += 1
            m, k = i // nb, j // nb
            if m != k:
                tiles.setdefault((m, k), set()).add(i - m * nb)
    NT = (n + nb - 1) // nb
    rho = (sum(len(v) for v in tiles.values()) / (nb * len(tiles))) if tiles else 1.0
    qnz = n + len(edges)
    return {"lnz": lnz, "tact": len(tiles) + NT, "rho": rho, "phi": lnz / qnz,
            "sigma": rowcount.max() * n / lnz, "tiles": {k: sorted(v) for k, v in tiles.items()}}


def _bfs_levels(adj, r, members=None):
    lev = {r: 0}
    q = [r]
    for u in q:
        for w in sorted(adj[u]):
            if (members is None or w in members) and w not in lev:
                lev[w] = lev[u] + 1
                q.append(w)
    return lev


def _auto_both(n, cp, ri, nb):
    """The oracle's and the analyser's AUTO choice: (method, perm) of each,
    plus a bit-exact check of every symbolic export between the two."""
    o = O.Analysis(n, cp, ri, "auto", nb=nb)
    a = S.Analysis(n, cp, ri, nb=nb, ordering="auto")
    assert a.method == o.method
    assert np.array_equal(a.perm(), o.perm())
    assert (a.lnz, a.ntiles, a.tact) == (o.lnz, o.ntiles, o.tact)
    assert (a.phi, a.rho, a.sigma) == (o.phi, o.rho, o.sigma)
    assert np.array_equal(a.tasks(), o.tasks())
    return o


def _check_candidates(n, edges, cp, ri, nb, expect_perm, expect_scores):
    """The oracle's fixed orderings give the hand-derived permutations, and
    the elimination game on those permutations gives the hand-derived scores."""
    for meth, name in ((NAT, "natural"), (RCM, "rcm"), (ND, "nd")):
        o = O.Analysis(n, cp, ri, name, nb=nb)
        if expect_perm.get(meth) is not None:
            assert o.perm().tolist() == list(expect_perm[meth]), name
        sc = _scores(n, edges, o.perm(), nb)
        lnz, tact = expect_scores[meth][:2]
        assert (sc["lnz"], sc["tact"]) == (lnz, tact), (name, sc["lnz"], sc["tact"])
        assert (o.lnz, o.tact) == (lnz, tact), name
        if len(expect_scores[meth]) > 2:
            assert sc["rho"] == expect_scores[meth][2] and o.rho == expect_scores[meth][2], name


# ---------------------------------------------------------------------------
# pseudo-peripheral root: degree beats index, then index breaks ties
# ---------------------------------------------------------------------------

ROOT_EDGES = [(0, 1), (1, 6), (6, 3), (1, 7), (2, 6), (2, 7), (1, 8), (8, 4), (8, 5)]


def test_pseudo_peripheral_tie_breaks_decide_rcm():
    """Nine vertices: W=0 hangs off the hub C=1; C reaches y=3 through a1=6,
    x=2 through a1=6 and b1=7 (so x has degree 2), and the leaves p=4, q=5
    through d1=8.  Degrees: 0:1, 1:4, 2:2, 3:1, 4:1, 5:1, 6:3, 7:2, 8:3.

    1. Start: the least degree (1) at the lowest index: vertex 0.
    2. Levels from 0: {0} {1} {6,7,8} {2,3,4,5}; eccentricity 3.  In the last
       level x=2 has the lowest index but degree 2, so the least degree wins:
       among 3, 4, 5 (degree 1) the lowest index, 3.  (Taking the lowest index
       alone would pick 2.)
    3. Levels from 3: {3} {6} {1,2} {0,7,8} {4,5}; eccentricity 4 > 3, so 3 is
       adopted.  Last level {4,5}, both degree 1: the lowest index, 4.
    4. Levels from 4: {4} {8} {1,5} {0,6,7} {2,3}; eccentricity 4, not larger:
       stop.  Root 3.
    Cuthill-McKee from 3, unvisited neighbours by (degree, index): 3; 6; then
    6's neighbours 2 (degree 2) before 1 (degree 4, lower index); 2's
    neighbour 7; 1's neighbours 0 (degree 1), 8 (degree 3); 8's 4, 5:
    3 6 2 1 7 0 8 4 5.  Reversed: 5 4 8 0 7 1 2 6 3."""
    n = 9
    adj = [set() for _ in range(n)]
    for a, b in ROOT_EDGES:
        adj[a].add(b)
        adj[b].add(a)
    deg = [len(s) for s in adj]
    assert deg == [1, 4, 2, 1, 1, 1, 3, 2, 3]
    # the hand steps, re-derived
    l0 = _bfs_levels(adj, 0)
    assert max(l0.values()) == 3 and sorted(v for v in l0 if l0[v] == 3) == [2, 3, 4, 5]
    l3 = _bfs_levels(adj, 3)
    assert max(l3.values()) == 4 and sorted(v for v in l3 if l3[v] == 4) == [4, 5]
    assert max(_bfs_levels(adj, 4).values()) == 4
    expect = [5, 4, 8, 0, 7, 1, 2, 6, 3]
    cp, ri, _ = _spd_from_edges(n, ROOT_EDGES)
    o = O.Analysis(n, cp, ri, "rcm", nb=32)
    assert o.perm().tolist() == expect
    a = S.Analysis(n, cp, ri, nb=32, ordering="rcm")
    assert a.perm().tolist() == expect


# ---------------------------------------------------------------------------
# AUTO, one pattern per branch (n = 64, tile 32: two diagonal blocks)
# ---------------------------------------------------------------------------

CASE1_SEQ = list(range(1, 32)) + [0] + list(range(32, 64))
CASE2_SEQ = [v for k in range(32) for v in (k, 32 + k)]


def test_auto_low_occupancy_takes_least_fill():
    """Path 1-2-...-31-0-32-33-...-63 (64 vertices), tile 32.

    NATURAL (identity): eliminating 0 first joins its neighbours 31 and 32
    (one fill entry); every later vertex has at most one later neighbour.
    nnz(L) = 64 + 63 + 1 = 128.  Block 1 meets block 0 only in row 32
    (L_32,0 and the fill L_32,31): one active row of 32, rho = 1/32 < 0.15.
    Active tiles: 2 diagonal + 1 = 3.
    ND: 64 vertices is a leaf, ordered by index: the identity, same scores.
    RCM: the path's end points 1 and 63 have degree 1, the root is 1 and the
    far end 63 is no farther; Cuthill-McKee walks the path 1..31, 0, 32..63,
    reversed: 63..32, 0, 31..1.  A path ordered along itself fills nothing:
    nnz(L) = 127; one entry crosses the block boundary: 3 active tiles.
    Rule: rho(NATURAL) < 0.15, so the least nnz(L) wins: RCM (127 < 128).
    With the occupancy test reversed, the fewest active tiles (a three-way
    tie at 3, so NATURAL) would win instead; with the fill comparison
    reversed NATURAL would stay the fill winner; with the size allowance
    applied below n = 50,000, ND (128 <= 1.25 x 127) would win."""
    n, nb = 64, 32
    edges = _path_edges(CASE1_SEQ)
    cp, ri, _ = _spd_from_edges(n, edges)
    rcm = list(range(63, 31, -1)) + [0] + list(range(31, 0, -1))
    _check_candidates(n, edges, cp, ri, nb, {NAT: range(n), RCM: rcm, ND: range(n)},
                      {NAT: (128, 3, 1 / 32), RCM: (127, 3), ND: (128, 3)})
    o = _auto_both(n, cp, ri, nb)
    assert o.method == RCM and o.perm().tolist() == rcm


def test_auto_ties_go_to_the_earlier_candidate():
    """Path 0-1-2-...-63 (64 vertices), tile 32.  NATURAL walks the path: no
    fill, nnz(L) = 127, one active row in tile (1,0) (rho = 1/32), 3 active
    tiles.  RCM: root 0 (the lower end point), reversed: 63..0, the same
    scores.  ND: leaf, the identity, the same.  rho < 0.15: least fill, a
    three-way tie: the earliest, NATURAL, wins (a later one on ties would
    give ND)."""
    n, nb = 64, 32
    edges = _path_edges(list(range(n)))
    cp, ri, _ = _spd_from_edges(n, edges)
    _check_candidates(n, edges, cp, ri, nb, {NAT: range(n), RCM: range(n - 1, -1, -1), ND: range(n)},
                      {NAT: (127, 3, 1 / 32), RCM: (127, 3), ND: (127, 3)})
    o = _auto_both(n, cp, ri, nb)
    assert o.method == NAT and o.perm().tolist() == list(range(n))


def test_auto_high_occupancy_takes_fewest_active_tiles():
    """Path 0-32-1-33-2-34-...-31-63 (64 vertices), tile 32.

    NATURAL: vertex 0 has one later neighbour (32); each k = 1..31 sits
    between 31+k and 32+k, which the elimination of k joins: 31 fill entries,
    after which 32..63 form a path.  nnz(L) = 127 + 31 = 158.  Column k of
    block 0 has rows 31+k and 32+k in block 1, so all 32 rows of tile (1,0)
    are active: rho = 1 and 3 active tiles.
    ND: leaf of 64, the identity: (158, 3).
    RCM: end points 0 and 63 (degree 1), root 0, the path order reversed:
    63, 31, 62, 30, ..., 32, 0; no fill, nnz(L) = 127, 3 active tiles.
    Rule: rho(NATURAL) >= 0.15, so the fewest active tiles win: all three
    have 3, the earliest is NATURAL.  No override: 2 x 127 = 254 > 158.
    NATURAL wins.  With the occupancy test reversed the least fill (RCM)
    would win; without the factor 2 of the override RCM (127 <= 158) would
    win; with the size allowance applied below n = 50,000, ND (4 x 158 =
    632 <= 5 x 127 = 635) would win."""
    n, nb = 64, 32
    edges = _path_edges(CASE2_SEQ)
    cp, ri, _ = _spd_from_edges(n, edges)
    rcm = CASE2_SEQ[::-1]
    _check_candidates(n, edges, cp, ri, nb, {NAT: range(n), RCM: rcm, ND: range(n)},
                      {NAT: (158, 3, 1.0), RCM: (127, 3), ND: (158, 3)})
    o = _auto_both(n, cp, ri, nb)
    assert o.method == NAT and o.perm().tolist() == list(range(n))


def test_auto_fewest_active_tiles_strictly():
    """Eight interleaved paths: path c (c = 0..7) runs c, c+8, c+16, ..., c+56,
    so vertex i is joined to i + 8 (64 vertices, tile 32).

    Every path is monotone in its labels, so no ordering below fills:
    nnz(L) = 64 + 56 = 120 for all three candidates.
    NATURAL (identity): bandwidth 8; columns 24..31 reach rows 32..39, so tile
    (1,0) has 8 active rows, rho = 8/32 = 0.25; 3 active tiles.
    ND: each path is a component of 8 vertices (a leaf), components in order
    of their least vertex, each by index: 0, 8, ..., 56, 1, 9, ..., 57, ...,
    7, ..., 63.  Paths 0..3 fill positions 0..31 and paths 4..7 positions
    32..63, and no edge joins two paths: tile (1,0) is empty, 2 active tiles.
    RCM: the same components in the same order, each walked from its lower
    end point and reversed: 56, 48, ..., 0, 57, ..., 1, ..., 63, ..., 7;
    likewise 2 active tiles.
    Rule: rho >= 0.15, fewest active tiles: RCM and ND have 2, the earlier is
    RCM; no override (equal fill).  RCM wins.  With the tile comparison
    reversed the most active tiles (NATURAL) would win; with the occupancy
    test reversed the least fill (a three-way tie: NATURAL) would win."""
    n, nb = 64, 32
    edges = [(i, i + 8) for i in range(n - 8)]
    cp, ri, _ = _spd_from_edges(n, edges)
    nd = [c + 8 * s for c in range(8) for s in range(8)]
    rcm = [c + 8 * s for c in range(8) for s in range(7, -1, -1)]
    _check_candidates(n, edges, cp, ri, nb, {NAT: range(n), RCM: rcm, ND: nd},
                      {NAT: (120, 3, 0.25), RCM: (120, 2), ND: (120, 2)})
    o = _auto_both(n, cp, ri, nb)
    assert o.method == RCM and o.perm().tolist() == rcm


def test_auto_half_fill_overrides_fewest_tiles():
    """Star: centre 0 joined to leaves 1..63 (64 vertices), tile 32.  The
    centre's degree 63 is below the dense-row cut max(16, floor(sqrt(6400)))
    = 80, so nothing is set aside.

    NATURAL: the centre goes first and makes its 63 neighbours a clique:
    L is full, nnz(L) = 64 x 65 / 2 = 2080, tile (1,0) full, rho = 1,
    3 active tiles.  ND: leaf, identity, the same.
    RCM: the root starts at leaf 1 (degree 1, lowest index); its levels are
    {1} {0} {2..63}, the last level's least degree at the lowest index is 2,
    whose eccentricity (2) is no larger: root 1.  Cuthill-McKee: 1, 0, then
    the leaves 2..63 by index; reversed: 63..2, 0, 1.  Every leaf goes before
    the centre: no fill, nnz(L) = 127.  The centre sits at position 62, in
    block 1, joined to positions 0..61: tile (1,0) active, 3 active tiles.
    Rule: rho >= 0.15; fewest active tiles: tie, NATURAL; but RCM's 127 is at
    most half of 2080, so RCM overrides.  With the override's comparison
    reversed the earliest candidate with more than half (NATURAL) would win."""
    n, nb = 64, 32
    edges = [(0, v) for v in range(1, n)]
    cp, ri, _ = _spd_from_edges(n, edges)
    rcm = list(range(63, 1, -1)) + [0, 1]
    _check_candidates(n, edges, cp, ri, nb, {NAT: range(n), RCM: rcm, ND: range(n)},
                      {NAT: (2080, 3, 1.0), RCM: (127, 3), ND: (2080, 3)})
    o = _auto_both(n, cp, ri, nb)
    assert o.method == RCM and o.perm().tolist() == rcm


def _copies(C, with_star=False):
    """C disjoint copies of the path of test_auto_high_occupancy_takes_fewest_
    active_tiles, copy c on vertices 64c..64c+63; with_star replaces the last
    copy by the star of test_auto_half_fill_overrides_fewest_tiles."""
    edges = []
    for c in range(C):
        base = 64 * c
        if with_star and c == C - 1:
            edges += [(base, base + v) for v in range(1, 64)]
        else:
            edges += [(base + a, base + b) for a, b in _path_edges(CASE2_SEQ)]
    return 64 * C, edges


@pytest.mark.parametrize("C,with_star,expect", [(782, False, ND), (781, False, NAT), (782, True, NAT)])
def test_auto_nested_dissection_allowance_on_large_orders(C, with_star, expect):
    """C disjoint copies of the 64-vertex path of the high-occupancy case,
    copy c on the consecutive vertices 64c..64c+63, tile 32.  Components are
    independent, so each score is a sum over copies, and each copy fills
    exactly two diagonal blocks.

    Every component has 64 vertices, an ND leaf: ND orders the components by
    their least vertex, each by index -- the identity, like NATURAL.  Per copy:
    NATURAL and ND nnz(L) 158, RCM 127, one active off-diagonal tile each, rho
    of NATURAL 1.  Without the allowance NATURAL wins (previous test).
      * C = 782, n = 50,048 >= 50,000: ND's 158 C is within 1.25 x the least
        (4 x 158 = 632 <= 5 x 127 = 635): ND wins (same permutation as
        NATURAL, reported as ND).
      * C = 781, n = 49,984 < 50,000: no allowance, NATURAL wins.
      * C = 782 with the last copy a 64-vertex star (its centre's degree 63 is
        far below the dense cut of 2,237): NATURAL and ND nnz(L) 158 x 781 +
        2080 = 125,478, RCM 127 x 782 = 99,314; 4 x 125,478 = 501,912 >
        5 x 99,314 = 496,570, so ND is more than 1.25 x the least: no
        allowance; no override either (2 x 99,314 > 125,478): NATURAL wins."""
    n, edges = _copies(C, with_star)
    nb = 32
    cp, ri, _ = _spd_from_edges(n, edges)
    per = _scores(64, _path_edges(CASE2_SEQ), list(range(64)), nb)["lnz"]
    per_rcm = _scores(64, _path_edges(CASE2_SEQ), CASE2_SEQ[::-1], nb)["lnz"]
    star = _scores(64, [(0, v) for v in range(1, 64)], list(range(64)), nb)["lnz"]
    assert (per, per_rcm, star) == (158, 127, 2080)
    nat_lnz = per * C if not with_star else per * (C - 1) + star
    rcm_lnz = per_rcm * C
    for name, lnz in (("natural", nat_lnz), ("rcm", rcm_lnz), ("nd", nat_lnz)):
        o = O.Analysis(n, cp, ri, name, nb=nb)
        assert o.lnz == lnz and o.tact == 3 * C, name
    o = _auto_both(n, cp, ri, nb)
    assert o.method == expect
    assert o.perm().tolist() == list(range(n))


# ---------------------------------------------------------------------------
# features phi, rho, sigma and the route on a hand-worked tile pattern
# ---------------------------------------------------------------------------

def test_features_cycle_worked_example():
    """tests/golden/features_cycle10.json: the 10-cycle 0-1-...-9-0, natural
    order, tile 4 (blocks {0..3}, {4..7}, {8,9}).  Worked out in the file."""
    g = json.load(open(os.path.join(GOLD, "features_cycle10.json")))
    n, nb = g["n"], g["nb"]
    edges = [tuple(e) for e in g["edges"]]
    cp, ri, _ = _spd_from_edges(n, edges)
    sc = _scores(n, edges, list(range(n)), nb)
    e = g["expect"]
    phi = e["phi"][0] / e["phi"][1]
    rho = e["rho"][0] / e["rho"][1]
    sigma = e["sigma"][0] / e["sigma"][1]
    assert sc["lnz"] == e["lnz"] and sc["tact"] == e["tact"]
    assert {f"{m},{k}": v for (m, k), v in sc["tiles"].items()} == e["tiles"]
    assert (sc["phi"], sc["rho"], sc["sigma"]) == (phi, rho, sigma)
    o = O.Analysis(n, cp, ri, "natural", nb=nb)
    assert (o.lnz, o.tact, o.ntiles) == (e["lnz"], e["tact"], len(e["tiles"]))
    assert (o.phi, o.rho, o.sigma) == (phi, rho, sigma)
    assert o.route == e["route"]
    t = o.tiles()
    got = {f"{t.m[i]},{t.k[i]}": t.rows_of(i).tolist() for i in range(o.ntiles)}
    assert got == e["tiles"]
    assert t.kd.tolist() == e["kd"]
    assert t.contig.tolist() == [1] * len(e["tiles"])


# ---------------------------------------------------------------------------
# multi-column solve
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nrhs", [2, 5, 17])
def test_solve_many_right_hand_sides_vs_lapack(nrhs):
    """Each column of the oracle's solve with nrhs right-hand sides equals
    LAPACK's dense solve, and the columns do not interact (a permuted copy of
    B gives the permuted columns)."""
    w = W.random_spd(150, 0.05, 21, dense_rows=2)
    a = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=16)
    Lx, info = a.factor(w.values)
    assert info == 0
    A = W.dense_from_csc(w.n, w.colptr, w.rowind, w.values)
    B = np.random.default_rng(nrhs).standard_normal((w.n, nrhs))
    X = a.solve(Lx, B)
    Xr = np.linalg.solve(A, B)
    assert np.max(np.abs(X - Xr)) <= 1e-12 * np.max(np.abs(Xr))
    p = np.random.default_rng(1).permutation(nrhs)
    assert np.array_equal(a.solve(Lx, B[:, p]), X[:, p])
