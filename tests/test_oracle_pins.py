"""Pins of the oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expectation comes from
dense LAPACK, a closed form, a spectral identity, brute-force elimination, a
hand-worked example, or a value printed in the paper (the worked examples of
Sec. 4.1 / Sec. 4.3 and the cut-offs of Table 5, kept under tests/golden/).
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import oracle as O
from paper_2609_29765_amd import workloads as W
from tests import closed_forms as CF

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _csc(A):
    return W.lower_csc(sp.csr_matrix(A))


# ---------------------------------------------------------------------------
# pattern checks
# ---------------------------------------------------------------------------

def test_pattern_errors():
    cp = np.array([0, 2, 3], np.int64)
    assert O.check_pattern(2, cp, np.array([0, 1, 1], np.int32)) == 0
    assert O.check_pattern(2, cp, np.array([1, 0, 1], np.int32)) != 0  # diagonal not first
    assert O.check_pattern(2, np.array([0, 2, 2], np.int64), np.array([0, 1], np.int32)) != 0
    assert O.check_pattern(3, np.array([0, 3, 4, 5], np.int64),
                           np.array([0, 2, 2, 1, 2], np.int32)) != 0  # duplicate
    assert O.check_pattern(2, np.array([0, 2, 3], np.int64), np.array([0, 5, 1], np.int32)) != 0


# ---------------------------------------------------------------------------
# factor against dense LAPACK, symbolic against brute-force elimination
# ---------------------------------------------------------------------------

def _elimination_game(A):
    """Boolean elimination of a symmetric pattern: returns the lower pattern
    of L as a dense boolean matrix."""
    n = A.shape[0]
    G = (A != 0)
    Lp = np.zeros((n, n), bool)
    for j in range(n):
        nb = [i for i in range(j + 1, n) if G[i, j]]
        Lp[j, j] = True
        for i in nb:
            Lp[i, j] = True
        for a in nb:
            for b in nb:
                G[a, b] = True
    return Lp


@pytest.mark.parametrize("n,density,seed,dense_rows", [(7, 0.3, 1, 0), (23, 0.12, 2, 1),
                                                      (40, 0.08, 3, 2), (40, 0.25, 4, 0)])
@pytest.mark.parametrize("ordering", ["natural", "rcm", "nd", "auto"])
def test_symbolic_and_factor_vs_dense(n, density, seed, dense_rows, ordering):
    w = W.random_spd(n, density, seed, dense_rows)
    a = O.Analysis(n, w.colptr, w.rowind, ordering, nb=4)
    p = a.perm()
    assert sorted(p.tolist()) == list(range(n))
    A = W.dense_from_csc(n, w.colptr, w.rowind, w.values)
    PA = A[np.ix_(p, p)]
    # symbolic: exact pattern of L equals the elimination game
    lp, li = a.L_pattern()
    Lpat = np.zeros((n, n), bool)
    for j in range(n):
        Lpat[li[lp[j]:lp[j + 1]], j] = True
    assert np.array_equal(Lpat, _elimination_game(PA))
    # elimination tree by its definition: parent(j) = min{i > j : L_ij != 0}
    par = a.etree()
    for j in range(n):
        below = np.nonzero(Lpat[j + 1:, j])[0]
        assert par[j] == (below[0] + j + 1 if below.size else -1)
    # numeric: dense Cholesky of P A P^T
    Lx, info = a.factor(w.values)
    assert info == 0
    Lref = np.linalg.cholesky(PA)
    Ld = a.dense_L(Lx)
    assert np.max(np.abs(Ld - Lref)) <= 1e-12 * np.max(np.abs(Lref))
    # no value outside the symbolic pattern
    assert np.all(np.abs(Lref[~Lpat]) <= 1e-12 * np.max(np.abs(Lref)))
    # logdet against LAPACK's slogdet
    sign, ld = np.linalg.slogdet(A)
    assert sign > 0 and abs(a.logdet(Lx) - ld) <= 1e-12 * max(1.0, abs(ld))


def test_residual_medium():
    w = W.random_spd(300, 0.02, 7, dense_rows=3)
    a = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=32)
    Lx, info = a.factor(w.values)
    assert info == 0
    A = W.dense_from_csc(w.n, w.colptr, w.rowind, w.values)
    p = a.perm()
    L = a.dense_L(Lx)
    res = np.linalg.norm(A[np.ix_(p, p)] - L @ L.T) / np.linalg.norm(A)
    assert res <= 1e-13


def test_not_spd_reports_first_pivot():
    A = np.diag([4.0, 5.0, -1.0, 3.0])
    A[1, 0] = A[0, 1] = 1.0
    cp, ri, v = _csc(A)
    a = O.Analysis(4, cp, ri, "natural", nb=2)
    _, info = a.factor(v)
    assert info == 3


# ---------------------------------------------------------------------------
# closed forms (natural ordering)
# ---------------------------------------------------------------------------

def test_tridiag_closed_form():
    n = 50
    A = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    cp, ri, v = _csc(A)
    a = O.Analysis(n, cp, ri, "natural", nb=8)
    Lx, info = a.factor(v)
    L = a.dense_L(Lx)
    j = np.arange(n)
    assert np.allclose(np.diag(L), np.sqrt((j + 2) / (j + 1)), rtol=1e-14, atol=0)
    assert np.allclose(np.diag(L, -1), -np.sqrt((j[:-1] + 1) / (j[:-1] + 2)), rtol=1e-14, atol=0)
    assert abs(a.logdet(Lx) - np.log(n + 1)) <= 1e-13


def test_anchored_rw1_closed_form():
    n = 40
    A = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    A[0, 0] = 1.0
    cp, ri, v = _csc(A)
    a = O.Analysis(n, cp, ri, "natural", nb=8)
    Lx, _ = a.factor(v)
    L = a.dense_L(Lx)
    assert np.array_equal(L, np.eye(n) - np.eye(n, k=-1))
    assert a.logdet(Lx) == 0.0


@pytest.mark.parametrize("rho", [0.3, 0.9, -0.7])
def test_ar1_closed_form(rho):
    T = 30
    # unit innovation: tridiag(-rho; 1, 1+rho^2, ..., 1+rho^2, 1)
    A = (W.ar1_precision(T, rho) * (1 - rho * rho)).toarray()
    cp, ri, v = _csc(A)
    a = O.Analysis(T, cp, ri, "natural", nb=8)
    Lx, _ = a.factor(v)
    L = a.dense_L(Lx)
    d = np.ones(T)
    d[-1] = np.sqrt(1 - rho * rho)
    assert np.allclose(np.diag(L), d, rtol=1e-14, atol=1e-15)
    assert np.allclose(np.diag(L, -1), -rho, rtol=1e-14, atol=1e-15)
    assert abs(a.logdet(Lx) - np.log(1 - rho * rho)) <= 1e-13
    # unit marginal variance version: divided by (1 - rho^2)
    cp, ri, v = _csc(W.ar1_precision(T, rho).toarray())
    a = O.Analysis(T, cp, ri, "natural", nb=8)
    Lx, _ = a.factor(v)
    assert abs(a.logdet(Lx) + (T - 1) * np.log(1 - rho * rho)) <= 1e-12


# ---------------------------------------------------------------------------
# spectral identities
# ---------------------------------------------------------------------------

def test_gmrf32_spectral_logdet_and_solve():
    w = W.gmrf_grid2d(32, 32, 0.1, 0)
    a = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=64)
    Lx, info = a.factor(w.values)
    assert info == 0
    lam = CF.lam(32)
    ld = np.log(lam[:, None] + lam[None, :] + 0.1).sum()
    assert abs(a.logdet(Lx) - ld) <= 1e-12 * abs(ld)
    # exact solve in the DCT eigenbasis of the path Laplacian
    ev, V1 = np.linalg.eigh(W.path_laplacian(32).toarray())
    B = w.b.reshape(32, 32)
    Y = V1.T @ B @ V1
    X = V1 @ (Y / (ev[:, None] + ev[None, :] + 0.1)) @ V1.T
    x = a.solve(Lx, w.b)
    assert np.max(np.abs(x - X.reshape(-1))) <= 1e-12 * np.max(np.abs(X))


@pytest.mark.parametrize("member", [0, 3, 7])
def test_lap3d_member_spectral_logdet(member):
    w = W.batched_laplacian3d(m=6, B=8, seed=0)
    a = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=16)
    Lx, info = a.factor(w.values[member])
    assert info == 0
    wb, sb = w.meta["hyper"][member]
    lam = CF.lam(6)
    ld = np.log(wb * (lam[:, None, None] + lam[None, :, None] + lam[None, None, :]) + 0.05 * sb).sum()
    assert abs(a.logdet(Lx) - ld) <= 1e-12 * abs(ld)


def test_small_spatiotemporal_closed_form():
    w = W.spatiotemporal_arrowhead(T=6, m=8, kappa=0.5, rho=0.9, nborder=8, seed=0)
    a = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=32)
    Lx, info = a.factor(w.values)
    assert info == 0
    ld = CF.bordered_logdet(6, 8, 1.0, 0.5, 0.9, w.meta["Bc"], w.meta["D"])
    assert abs(a.logdet(Lx) - ld) <= 1e-12 * abs(ld)


def test_differentiable_arrowhead_closed_form_full_size():
    w = W.differentiable_arrowhead(20, 25, 8, 0)
    a = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=64)
    Lx, info = a.factor(w.values)
    assert info == 0
    mt = w.meta
    ld = CF.bordered_logdet(20, 25, mt["tau"], mt["kappa"], mt["rho"], mt["Bc"], mt["D"])
    assert abs(a.logdet(Lx) - ld) <= 1e-12 * abs(ld)


# ---------------------------------------------------------------------------
# selected inverse and gradient
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,seed", [(30, 1), (120, 2)])
def test_selinv_vs_inverse(n, seed):
    w = W.random_spd(n, 0.05, seed, dense_rows=2)
    a = O.Analysis(n, w.colptr, w.rowind, "nd", nb=16)
    Lx, _ = a.factor(w.values)
    Z = a.selinv(Lx)
    A = W.dense_from_csc(n, w.colptr, w.rowind, w.values)
    p = a.perm()
    Zref = np.linalg.inv(A[np.ix_(p, p)])
    lp, li = a.L_pattern()
    cols = np.repeat(np.arange(n), np.diff(lp))
    assert np.max(np.abs(Z - Zref[li, cols])) <= 1e-12 * np.max(np.abs(Zref))


def test_gradient_trace_vs_closed_form_fd():
    T, m = 5, 6
    w = W.differentiable_arrowhead(T, m, 8, seed=3)
    a = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=16)
    Lx, _ = a.factor(w.values)
    gv = a.logdet_grad_values(Lx)
    g = w.dvalues @ gv
    th = w.meta["theta"]
    h = 1e-5
    fd = np.zeros(3)
    for i in range(3):
        vals = []
        for s in (+1, -1):
            t2 = th.copy()
            t2[i] += s * h
            w2 = W.differentiable_arrowhead(T, m, 8, seed=3, theta=t2)
            mt = w2.meta
            vals.append(CF.bordered_logdet(T, m, mt["tau"], mt["kappa"], mt["rho"], mt["Bc"], mt["D"]))
        fd[i] = (vals[0] - vals[1]) / (2 * h)
    assert np.all(np.abs(g - fd) <= 1e-7 * np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max()))


# ---------------------------------------------------------------------------
# tiles: the worked examples of Sec. 4.1 and Sec. 4.3
# ---------------------------------------------------------------------------

def test_active_column_worked_example():
    g = json.load(open(os.path.join(GOLD, "active_column_example.json")))
    nb = g["nb"]
    n = 2 * nb
    A = np.eye(n) * 10.0
    # transpose entry (r, c): L^T tile row r is column r of block 0, column c is
    # row c of block 1, i.e. L entry (nb + c, r)
    for r, c in g["transpose_entries"]:
        A[nb + c, r] = A[r, nb + c] = 1.0
    cp, ri, v = _csc(A)
    a = O.Analysis(n, cp, ri, "natural", nb=nb, mode="semisparse")
    t = a.tiles()
    assert a.ntiles == 1 and (t.m[0], t.k[0]) == (1, 0)
    assert t.rows_of(0).tolist() == g["aind"]
    assert [int(t.cnt[0]), nb] == g["stored_shape"][::-1]
    assert bool(t.contig[0]) == g["contiguous"]
    assert (int(t.cnt[0]) == nb) == g["full_width"]
    # the dense route stores the same tile at full height
    a2 = O.Analysis(n, cp, ri, "natural", nb=nb, mode="dense")
    assert a2.tiles().rows_of(0).tolist() == list(range(nb))


def test_band_kd_worked_example():
    g = json.load(open(os.path.join(GOLD, "band_example.json")))
    n, kd = g["n"], g["kd"]
    A = np.eye(n) * 10.0
    for i in range(n):
        for j in range(n):
            if 0 < abs(i - j) <= kd:
                A[i, j] = 1.0
    cp, ri, v = _csc(A)
    a = O.Analysis(n, cp, ri, "natural", nb=n)
    assert a.tiles().kd.tolist() == [kd]
    # the packed map (kd + i - j, j) of the example: the main diagonal lands on
    # the bottom row and exactly kd(kd+1)/2 corner slots stay unused
    used = {(kd + i - j, j) for j in range(n) for i in range(j + 1) if j - i <= kd}
    labels = {(kd + i - j, j): f"a{i}{j}" for j in range(n) for i in range(j + 1) if j - i <= kd}
    for r, row in enumerate(g["packed"]):
        for c, lab in enumerate(row):
            assert (lab == "*") == ((r, c) not in used)
            if lab != "*":
                assert labels[(r, c)] == lab


def test_kd_grows_with_fill():
    # arrow pointing up: column 0 couples to every later row -> fill makes the
    # whole tile dense, kd = n - 1
    n = 6
    A = np.eye(n) * 10.0
    A[1:, 0] = A[0, 1:] = 1.0
    cp, ri, v = _csc(A)
    a = O.Analysis(n, cp, ri, "natural", nb=n)
    assert a.tiles().kd.tolist() == [n - 1]
    assert a.lnz == n * (n + 1) // 2


def test_ragged_last_tile_rows_stay_inside():
    w = W.random_spd(45, 0.1, 5)
    a = O.Analysis(45, w.colptr, w.rowind, "nd", nb=16, mode="dense")
    t = a.tiles()
    for q in range(a.ntiles):
        h = 45 - 32 if t.m[q] == 2 else 16
        assert t.rows_of(q).tolist() == list(range(h))


# ---------------------------------------------------------------------------
# Algorithm 1 on hand-built tile patterns
# ---------------------------------------------------------------------------

def test_algorithm1_dense_three_tiles():
    n, nb = 6, 2
    A = np.ones((n, n)) + n * np.eye(n)
    cp, ri, v = _csc(A)
    a = O.Analysis(n, cp, ri, "natural", nb=nb)
    P, S, T_, G = O.OP_POTRF, O.OP_SYRK, O.OP_TRSM, O.OP_GEMM
    expect = [
        (P, -1, 0, -1), (T_, 1, 0, -1), (T_, 2, 0, -1),
        (S, -1, 1, 0), (P, -1, 1, -1), (G, 2, 1, 0), (T_, 2, 1, -1),
        (S, -1, 2, 0), (S, -1, 2, 1), (P, -1, 2, -1),
    ]
    assert [tuple(x) for x in a.tasks().tolist()] == expect


def test_algorithm1_skips_empty_tiles():
    # block pattern: tiles (2,0) and (3,1) and (3,2) present; (1,0), (2,1) empty
    nb = 2
    n = 8
    A = 10 * np.eye(n)
    def link(i, j):
        A[i, j] = A[j, i] = 1.0
    link(4, 0)   # tile (2,0)
    link(6, 3)   # tile (3,1)
    link(7, 5)   # tile (3,2)
    cp, ri, v = _csc(A)
    a = O.Analysis(n, cp, ri, "natural", nb=nb)
    t = a.tiles()
    assert sorted(zip(t.m.tolist(), t.k.tolist())) == [(2, 0), (3, 1), (3, 2)]
    P, S, T_, G = O.OP_POTRF, O.OP_SYRK, O.OP_TRSM, O.OP_GEMM
    expect = [
        (P, -1, 0, -1), (T_, 2, 0, -1),
        (P, -1, 1, -1), (T_, 3, 1, -1),
        (S, -1, 2, 0), (P, -1, 2, -1), (T_, 3, 2, -1),
        (S, -1, 3, 1), (S, -1, 3, 2), (P, -1, 3, -1),
    ]
    assert [tuple(x) for x in a.tasks().tolist()] == expect


def test_algorithm1_gemm_needs_both_neighbours():
    nb, n = 2, 6
    A = 10 * np.eye(n)
    A[2, 0] = A[0, 2] = 1.0   # tile (1,0)
    A[4, 1] = A[1, 4] = 1.0   # tile (2,0)
    # L_20 L_10^T: rows 4 and 2 share no column of block 0, so no fill: (2,1) empty
    cp, ri, v = _csc(A)
    a = O.Analysis(n, cp, ri, "natural", nb=nb)
    t = a.tiles()
    assert sorted(zip(t.m.tolist(), t.k.tolist())) == [(1, 0), (2, 0)]
    ops = [tuple(x) for x in a.tasks().tolist()]
    assert not any(op == O.OP_GEMM for op, *_ in ops)
    # now couple them through a shared column: fill activates (2,1) and the GEMM
    A[4, 0] = A[0, 4] = 1.0
    cp, ri, v = _csc(A)
    a = O.Analysis(n, cp, ri, "natural", nb=nb)
    ops = [tuple(x) for x in a.tasks().tolist()]
    assert (O.OP_GEMM, 2, 1, 0) in ops


# ---------------------------------------------------------------------------
# selector (Sec. 5.1, Table 5) and features
# ---------------------------------------------------------------------------

def test_selector_table5_boundaries():
    g = json.load(open(os.path.join(GOLD, "selector_table5.json")))
    for c in g["cases"]:
        assert O.route(c["phi"], c["rho"], c["sigma"]) == c["route"], c


def test_features_definitions():
    w = W.random_spd(60, 0.06, 11, dense_rows=2)
    a = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=8)
    lp, li = a.L_pattern()
    assert a.phi == a.lnz / w.nnz
    rc = np.bincount(li, minlength=w.n)
    assert a.sigma == rc.max() * w.n / a.lnz
    t = a.tiles()
    assert a.rho == t.true_cnt.sum() / (8 * a.ntiles)
    assert a.route == O.route(a.phi, a.rho, a.sigma)


# ---------------------------------------------------------------------------
# orderings on hand-worked graphs
# ---------------------------------------------------------------------------

def _path(n):
    A = 3 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return _csc(A)


def test_rcm_path_reverses():
    cp, ri, v = _path(30)
    a = O.Analysis(30, cp, ri, "rcm", nb=8)
    assert a.perm().tolist() == list(range(29, -1, -1))


def test_nd_path_by_hand():
    cp, ri, v = _path(200)
    a = O.Analysis(200, cp, ri, "nd", nb=8)
    expect = (list(range(0, 50)) + list(range(51, 100)) + [50] + list(range(101, 150))
              + list(range(151, 200)) + [150] + [100])
    assert a.perm().tolist() == expect


def test_dense_vertex_set_aside():
    n = 400  # threshold max(16, floor(sqrt(100 n))) = 200; the hub has degree 399
    A = 500 * np.eye(n)
    A[1:, 0] = A[0, 1:] = 1.0
    cp, ri, v = _csc(A)
    for ordering in ("natural", "rcm", "nd"):
        a = O.Analysis(n, cp, ri, ordering, nb=64)
        assert a.perm().tolist() == list(range(1, n)) + [0]
        assert a.ndense == 1
        assert a.lnz == n + (n - 1)  # no fill: the hub is eliminated last


def test_ordering_components_in_min_index_order():
    # two paths interleaved: even vertices form one path, odd vertices another
    n = 20
    A = 3 * np.eye(n)
    for i in range(0, n - 2, 1):
        A[i, i + 2] = A[i + 2, i] = -1.0
    cp, ri, v = _csc(A)
    a = O.Analysis(n, cp, ri, "rcm", nb=4)
    evens = list(range(0, n, 2))
    odds = list(range(1, n, 2))
    assert a.perm().tolist() == evens[::-1] + odds[::-1]


def test_orderings_deterministic_and_valid():
    w = W.gmrf_grid2d(20, 20)
    for ordering in ("rcm", "nd", "auto"):
        p1 = O.Analysis(w.n, w.colptr, w.rowind, ordering, nb=32).perm()
        p2 = O.Analysis(w.n, w.colptr, w.rowind, ordering, nb=32).perm()
        assert np.array_equal(p1, p2)
        assert np.array_equal(np.sort(p1), np.arange(w.n))
    # nested dissection beats the band ordering on a 2-D grid
    nd = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=32).lnz
    nat = O.Analysis(w.n, w.colptr, w.rowind, "natural", nb=32).lnz
    assert nd < nat
