"""Seeded synthetic inputs for the five workloads and for small test patterns.

This module only builds matrices (graph Laplacians, Kronecker products, random
SPD patterns); it holds none of the factorization's arithmetic.  Both the
product path and the oracle read what it returns.  Every generator takes a
seed and draws from numpy's PCG64 (``numpy.random.default_rng``) in a fixed,
documented order, so a workload is the same on every machine.

All matrices are returned as the lower triangle (diagonal included) in CSC
form: int64 column pointers, int32 row indices ascending within each column
(so the diagonal comes first), float64 values.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class Workload:
    name: str
    n: int
    colptr: np.ndarray
    rowind: np.ndarray
    values: np.ndarray              # (nnz,) or (B, nnz) for batched workloads
    b: np.ndarray | None = None     # right-hand side
    meta: dict = field(default_factory=dict)
    dvalues: np.ndarray | None = None  # (ntheta, nnz): d values / d theta

    @property
    def nnz(self) -> int:
        return int(self.colptr[-1])


def lower_csc(A: sp.spmatrix):
    """Lower triangle of a symmetric sparse matrix as sorted CSC arrays.
    Every diagonal entry must be structurally present."""
    L = sp.tril(sp.csc_matrix(A), format="csc")
    L.sum_duplicates()
    L.sort_indices()
    n = L.shape[0]
    if not (np.all(np.diff(L.indptr) > 0) and np.all(L.indices[L.indptr[:-1]] == np.arange(n))):
        raise ValueError("matrix has a structurally missing diagonal entry")
    return (np.ascontiguousarray(L.indptr, np.int64),
            np.ascontiguousarray(L.indices, np.int32),
            np.ascontiguousarray(L.data, np.float64))


def path_laplacian(m: int) -> sp.csr_matrix:
    """Graph Laplacian of a path with m vertices (free boundary)."""
    main = np.full(m, 2.0)
    main[0] = main[-1] = 1.0
    if m == 1:
        main[:] = 0.0
    off = -np.ones(m - 1)
    return sp.diags([off, main, off], [-1, 0, 1], format="csr")


def grid_laplacian(*dims: int) -> sp.csr_matrix:
    """Graph Laplacian of a 2-D or 3-D grid (5- or 7-point stencil),
    free boundary: diagonal = degree, off-diagonal = -1.  Vertex (i0, i1, ...)
    has index i0 * prod(dims[1:]) + ...; the last axis runs fastest."""
    L = None
    for ax, m in enumerate(dims):
        parts = [sp.identity(d, format="csr") for d in dims]
        parts[ax] = path_laplacian(m)
        term = parts[0]
        for p in parts[1:]:
            term = sp.kron(term, p, format="csr")
        L = term if L is None else L + term
    return L.tocsr()


def ar1_precision(T: int, rho: float) -> sp.csr_matrix:
    """Precision of a stationary AR(1) with unit marginal variance:
    tridiag(-rho; 1, 1+rho^2, ..., 1+rho^2, 1) / (1 - rho^2)."""
    main = np.full(T, 1.0 + rho * rho)
    main[0] = main[-1] = 1.0
    off = np.full(T - 1, -rho)
    return (sp.diags([off, main, off], [-1, 0, 1], format="csr") / (1.0 - rho * rho)).tocsr()


def dar1_drho(T: int, rho: float) -> sp.csr_matrix:
    """Element-wise derivative of ar1_precision with respect to rho."""
    s = 1.0 - rho * rho
    main = np.full(T, (2 * rho * s + (1 + rho * rho) * 2 * rho) / (s * s))
    main[0] = main[-1] = 2 * rho / (s * s)
    off = np.full(T - 1, (-s - rho * 2 * rho) / (s * s))
    return sp.diags([off, main, off], [-1, 0, 1], format="csr")


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------

def gmrf_grid2d(nx: int = 32, ny: int = 32, shift: float = 0.1, seed: int = 0) -> Workload:
    """2-D GMRF precision: 5-point graph Laplacian + shift*I; b ~ N(0, 1)."""
    Q = grid_laplacian(nx, ny) + shift * sp.identity(nx * ny)
    cp, ri, v = lower_csc(Q)
    rng = np.random.default_rng(seed)
    b = rng.standard_normal(nx * ny)
    return Workload(f"gmrf{nx}x{ny}", nx * ny, cp, ri, v, b,
                    meta=dict(nx=nx, ny=ny, shift=shift, seed=seed))


def dense_spd(n: int = 12288, density: float = 0.2, seed: int = 0) -> Workload:
    """Random SPD with a uniform off-diagonal pattern of the given density.

    Draw order: for every column c = 0..n-2 of the lower triangle, a uniform
    vector of length n-c-1 (entry r > c present when < density), then one
    standard normal per present entry.  The diagonal is the row's absolute
    sum plus one (strictly diagonally dominant, hence SPD).  b ~ N(0, 1) last.
    """
    rng = np.random.default_rng(seed)
    colptr = np.zeros(n + 1, np.int64)
    rows_l, vals_l = [], []
    rowabs = np.zeros(n)
    for c in range(n):
        if c < n - 1:
            mask = rng.random(n - c - 1) < density
            r = np.nonzero(mask)[0].astype(np.int32) + (c + 1)
            v = rng.standard_normal(r.size)
        else:
            r = np.zeros(0, np.int32)
            v = np.zeros(0)
        rows_l.append(r)
        vals_l.append(v)
        a = np.abs(v)
        rowabs[c] += a.sum()
        np.add.at(rowabs, r, a)
        colptr[c + 1] = colptr[c] + r.size + 1
    rowind = np.empty(colptr[-1], np.int32)
    values = np.empty(colptr[-1])
    for c in range(n):
        p = colptr[c]
        rowind[p] = c
        values[p] = rowabs[c] + 1.0
        rowind[p + 1:colptr[c + 1]] = rows_l[c]
        values[p + 1:colptr[c + 1]] = vals_l[c]
    b = rng.standard_normal(n)
    return Workload(f"dense{n}", n, colptr, rowind, values, b,
                    meta=dict(density=density, seed=seed))


def _bordered_st(T, m, tau, kappa, rho, nborder, rng, coupling_sd=0.1, border_diag=1e3):
    """tau * kron(AR1(rho), kappa^2 I + L_{m x m}) plus a dense border of
    nborder rows/columns placed last: couplings N(0, coupling_sd^2) to every
    field vertex, border block with diagonal border_diag and symmetric
    N(0, coupling_sd^2) off-diagonal entries.  Draw order: couplings
    (nfield x nborder, row-major), then the border block's strictly lower
    triangle (nborder x nborder normals, lower part used)."""
    G = m * m
    Lg = grid_laplacian(m, m)
    M = kappa * kappa * sp.identity(G) + Lg
    A = ar1_precision(T, rho)
    field = tau * sp.kron(A, M, format="csr")
    nf = T * G
    Bc = rng.normal(0.0, coupling_sd, size=(nf, nborder))
    Dr = rng.normal(0.0, coupling_sd, size=(nborder, nborder))
    D = np.tril(Dr, -1)
    D = D + D.T + border_diag * np.eye(nborder)
    Q = sp.bmat([[field, sp.csr_matrix(Bc)], [sp.csr_matrix(Bc.T), sp.csr_matrix(D)]], format="csr")
    parts = dict(A=A, M=M, Lg=Lg, Bc=Bc, D=D)
    return Q, parts


def spatiotemporal_arrowhead(T: int = 50, m: int = 45, kappa: float = 0.5, rho: float = 0.9,
                             nborder: int = 8, seed: int = 0) -> Workload:
    """Block-tridiagonal space-time precision kron(AR1(rho), kappa^2 I + L)
    on T steps of an m x m grid, plus nborder dense fixed-effect rows/cols."""
    rng = np.random.default_rng(seed)
    Q, parts = _bordered_st(T, m, 1.0, kappa, rho, nborder, rng)
    cp, ri, v = lower_csc(Q)
    n = Q.shape[0]
    b = rng.standard_normal(n)
    return Workload(f"st{T}x{m}x{m}+{nborder}", n, cp, ri, v, b,
                    meta=dict(T=T, m=m, kappa=kappa, rho=rho, tau=1.0, nborder=nborder,
                              seed=seed, Bc=parts["Bc"], D=parts["D"]))


def batched_laplacian3d(m: int = 24, B: int = 128, shift: float = 0.05, seed: int = 0) -> Workload:
    """3-D 7-point Laplacian + shift*I on an m^3 grid, B value sets: member b
    is w_b * L + shift * s_b * I with (w_b, s_b) = exp(U(ln 1e-2, ln 1e2)),
    drawn as one (B, 2) array."""
    rng = np.random.default_rng(seed)
    hp = np.exp(rng.uniform(np.log(1e-2), np.log(1e2), size=(B, 2)))
    L = grid_laplacian(m, m, m)
    n = m ** 3
    cpL, riL, vL = lower_csc(L + 0.0 * sp.identity(n))
    diag = riL == np.repeat(np.arange(n), np.diff(cpL))
    vals = np.empty((B, vL.size))
    for b in range(B):
        vals[b] = hp[b, 0] * vL + np.where(diag, shift * hp[b, 1], 0.0)
    rhs = rng.standard_normal(n)
    return Workload(f"lap3d{m}^3xB{B}", n, cpL, riL, vals, rhs,
                    meta=dict(m=m, B=B, shift=shift, seed=seed, hyper=hp))


def differentiable_arrowhead(T: int = 20, m: int = 25, nborder: int = 8, seed: int = 0,
                             theta=None) -> Workload:
    """Q(theta) = tau kron(AR1(rho), kappa^2 I + L) + border, with
    theta = (log tau, log kappa, atanh rho) ~ N(0, 0.3^2) drawn first unless
    given.  dvalues holds dQ/dtheta on the same CSC pattern."""
    rng = np.random.default_rng(seed)
    th = rng.normal(0.0, 0.3, size=3)
    if theta is not None:
        th = np.asarray(theta, dtype=np.float64)
    tau, kappa, rho = np.exp(th[0]), np.exp(th[1]), np.tanh(th[2])
    Q, parts = _bordered_st(T, m, tau, kappa, rho, nborder, rng)
    cp, ri, v = lower_csc(Q)
    n = Q.shape[0]
    G = m * m
    A, M = parts["A"], parts["M"]
    nf = T * G
    zb = sp.csr_matrix((n - nf, n - nf))

    def padded(F):
        return sp.bmat([[F, None], [None, zb]], format="csr")

    dQ = [
        padded(tau * sp.kron(A, M, format="csr")),                                   # d/d log tau
        padded(tau * sp.kron(A, 2 * kappa * kappa * sp.identity(G), format="csr")),  # d/d log kappa
        padded(tau * sp.kron(dar1_drho(T, rho) * (1 - rho * rho), M, format="csr")),  # d/d atanh rho
    ]
    # align each derivative to Q's lower pattern
    dv = np.zeros((3, v.size))
    for t, D in enumerate(dQ):
        Dl = sp.tril(sp.csc_matrix(D), format="csc")
        Dl.sort_indices()
        Dl.sum_duplicates()
        # Q's pattern contains D's; scatter by (row, col)
        key_q = np.repeat(np.arange(n, dtype=np.int64), np.diff(cp)) * n + ri
        Dc = Dl.tocoo()
        key_d = Dc.col.astype(np.int64) * n + Dc.row
        pos = np.searchsorted(key_q, key_d)
        assert np.all(key_q[pos] == key_d)
        dv[t, pos] = Dc.data
    b = rng.standard_normal(n)
    return Workload(f"dst{T}x{m}x{m}+{nborder}", n, cp, ri, v, b,
                    meta=dict(T=T, m=m, nborder=nborder, seed=seed, theta=th, tau=tau,
                              kappa=kappa, rho=rho, Bc=parts["Bc"], D=parts["D"]),
                    dvalues=dv)


def random_spd(n: int, density: float = 0.1, seed: int = 0, dense_rows: int = 0) -> Workload:
    """Small random sparse SPD: symmetric Bernoulli(density) pattern with
    N(0,1) entries, a few optional dense rows, diagonal = row |sum| + 1."""
    rng = np.random.default_rng(seed)
    U = np.triu((rng.random((n, n)) < density) * rng.standard_normal((n, n)), 1)
    for r in range(min(dense_rows, n)):
        i = n - 1 - r
        U[:i, i] = rng.standard_normal(i)
    S = U + U.T
    S += np.diag(np.abs(S).sum(axis=1) + 1.0)
    cp, ri, v = lower_csc(sp.csr_matrix(S))
    b = rng.standard_normal(n)
    return Workload(f"rand{n}", n, cp, ri, v, b, meta=dict(density=density, seed=seed))


def dense_from_csc(n, colptr, rowind, values) -> np.ndarray:
    """Full symmetric dense matrix from a lower CSC (small n only)."""
    A = np.zeros((n, n))
    for j in range(n):
        r = rowind[colptr[j]:colptr[j + 1]]
        A[r, j] = values[colptr[j]:colptr[j + 1]]
    return A + np.tril(A, -1).T


CONFIGS = {
    "gmrf32": lambda: gmrf_grid2d(32, 32, 0.1, 0),
    "dense12288": lambda: dense_spd(12288, 0.2, 0),
    "st50x45": lambda: spatiotemporal_arrowhead(50, 45, 0.5, 0.9, 8, 0),
    "lap3d24": lambda: batched_laplacian3d(24, 128, 0.05, 0),
    "dst20x25": lambda: differentiable_arrowhead(20, 25, 8, 0),
}
