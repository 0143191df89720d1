"""ctypes wrapper of the plain serial oracle (oracle.c).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg use it to check and to time the product path; the product
library never loads it.  Every function here is a thin marshalling layer over
oracle.c; the arithmetic lives there and follows the paper's definitions (see
the header of oracle.c for the passage each part follows).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

ORDERINGS = {"natural": 0, "rcm": 1, "nd": 2, "auto": 3, "given": 4}
MODES = {"auto": 0, "dense": 1, "semisparse": 2}
ROUTES = {0: "dense", 1: "semisparse", 2: "supernodal"}
OP_POTRF, OP_SYRK, OP_TRSM, OP_GEMM = 1, 2, 3, 4

_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # type: ignore

            _b.build()
        L = C.CDLL(path)
        L.orc_check_pattern.argtypes = [C.c_int64, _i64p, _i32p]
        L.orc_check_pattern.restype = C.c_int
        L.orc_analyse.argtypes = [C.c_int64, _i64p, _i32p, C.c_int, C.c_int, C.c_int, C.c_void_p,
                                  C.POINTER(C.c_int)]
        L.orc_analyse.restype = C.c_void_p
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_sizes.argtypes = [C.c_void_p, _i64p]
        L.orc_features.argtypes = [C.c_void_p, _f64p]
        L.orc_get_perm.argtypes = [C.c_void_p, _i32p]
        L.orc_get_etree.argtypes = [C.c_void_p, _i32p]
        L.orc_get_L_pattern.argtypes = [C.c_void_p, _i64p, _i32p]
        L.orc_get_value_map.argtypes = [C.c_void_p, _i64p]
        L.orc_get_tiles.argtypes = [C.c_void_p, _i32p, _i32p, _i32p, _i32p, _i8p, _i64p, _i32p, _i32p]
        L.orc_get_tasks.argtypes = [C.c_void_p, _i32p]
        L.orc_align.argtypes = [C.c_void_p, C.c_int64]
        L.orc_align.restype = C.c_int
        L.orc_get_positions.argtypes = [C.c_void_p, _i64p]
        L.orc_factor.argtypes = [C.c_void_p, _f64p, _f64p]
        L.orc_factor.restype = C.c_int64
        L.orc_logdet.argtypes = [C.c_void_p, _f64p]
        L.orc_logdet.restype = C.c_double
        L.orc_solve.argtypes = [C.c_void_p, _f64p, _f64p, C.c_int64]
        L.orc_selinv.argtypes = [C.c_void_p, _f64p, _f64p]
        L.orc_route.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_route.restype = C.c_int
        _LIB = L
    return _LIB


def check_pattern(n, colptr, rowind) -> int:
    return lib().orc_check_pattern(int(n), np.ascontiguousarray(colptr, np.int64),
                                   np.ascontiguousarray(rowind, np.int32))


def route(phi: float, rho: float, sigma: float) -> str:
    return ROUTES[lib().orc_route(float(phi), float(rho), float(sigma))]


@dataclass
class Tiles:
    m: np.ndarray
    k: np.ndarray
    cnt: np.ndarray       # stored active rows (full height on the dense route)
    true_cnt: np.ndarray  # active rows of the pattern
    contig: np.ndarray
    roff: np.ndarray
    rows: np.ndarray
    kd: np.ndarray

    def rows_of(self, t: int) -> np.ndarray:
        return self.rows[self.roff[t]:self.roff[t + 1]]


class Analysis:
    """Symbolic state for one pattern: ordering, L pattern, tiles, tasks."""

    def __init__(self, n, colptr, rowind, ordering="nd", nb=64, mode="auto", perm=None, align=0):
        self.colptr = np.ascontiguousarray(colptr, np.int64)
        self.rowind = np.ascontiguousarray(rowind, np.int32)
        err = C.c_int(0)
        pperm = None
        if ordering == "given":
            self._perm_in = np.ascontiguousarray(perm, np.int32)
            pperm = self._perm_in.ctypes.data_as(C.c_void_p)
        h = lib().orc_analyse(int(n), self.colptr, self.rowind, ORDERINGS[ordering], int(nb),
                              MODES[mode], pperm, C.byref(err))
        if not h:
            raise ValueError(f"oracle analyse failed with code {err.value}")
        self._h = h
        if not align and mode == "auto" and self._route_now() == "supernodal":
            # the supernodal route's tiles follow the fill (Sec. 5.4): on the
            # fixed-width tiles, a grid aligned to the elimination tree at n_b
            align = int(nb)
        if align:
            rc = lib().orc_align(h, int(align))
            if rc:
                raise ValueError(f"oracle alignment failed with code {rc}")
        sz = np.zeros(16, np.int64)
        lib().orc_sizes(h, sz)
        (self.n, self.qnz, self.lnz, self.nb, self.NT, self.ntiles, self.nrows, self.ntasks,
         mode_i, route_i, self.ndense, self.method, self.tact) = (int(x) for x in sz[:13])
        self.mode = {1: "dense", 2: "semisparse"}[mode_i]
        self.route = ROUTES[route_i]
        f = np.zeros(3)
        lib().orc_features(h, f)
        self.phi, self.rho, self.sigma = (float(x) for x in f)

    def _route_now(self):
        sz = np.zeros(16, np.int64)
        lib().orc_sizes(self._h, sz)
        return ROUTES[int(sz[9])]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    # symbolic exports ------------------------------------------------------
    def perm(self) -> np.ndarray:
        p = np.zeros(self.n, np.int32)
        lib().orc_get_perm(self._h, p)
        return p

    def etree(self) -> np.ndarray:
        p = np.zeros(self.n, np.int32)
        lib().orc_get_etree(self._h, p)
        return p

    def L_pattern(self):
        lp = np.zeros(self.n + 1, np.int64)
        li = np.zeros(self.lnz, np.int32)
        lib().orc_get_L_pattern(self._h, lp, li)
        return lp, li

    def value_map(self) -> np.ndarray:
        """Position in L's CSC of every input entry."""
        v = np.zeros(self.qnz, np.int64)
        lib().orc_get_value_map(self._h, v)
        return v

    def tiles(self) -> Tiles:
        nt = self.ntiles
        m = np.zeros(nt, np.int32)
        k = np.zeros(nt, np.int32)
        cnt = np.zeros(nt, np.int32)
        tc = np.zeros(nt, np.int32)
        cg = np.zeros(nt, np.int8)
        ro = np.zeros(nt + 1, np.int64)
        rows = np.zeros(max(self.nrows, 1), np.int32)
        kd = np.zeros(self.NT, np.int32)
        lib().orc_get_tiles(self._h, m, k, cnt, tc, cg, ro, rows, kd)
        return Tiles(m, k, cnt, tc, cg, ro, rows[:self.nrows], kd)

    def positions(self) -> np.ndarray:
        """Grid position of every column of P A P^T (the identity on the uniform grid)."""
        p = np.zeros(self.n, np.int64)
        lib().orc_get_positions(self._h, p)
        return p

    def tasks(self) -> np.ndarray:
        t = np.zeros((max(self.ntasks, 1), 4), np.int32)
        lib().orc_get_tasks(self._h, t)
        return t[:self.ntasks]

    # numeric ----------------------------------------------------------------
    def factor(self, values):
        """Return (Lx, info); info = 0 or the 1-based failing permuted column."""
        v = np.ascontiguousarray(values, np.float64)
        assert v.shape == (self.qnz,)
        Lx = np.zeros(self.lnz)
        info = lib().orc_factor(self._h, v, Lx)
        return Lx, int(info)

    def logdet(self, Lx) -> float:
        return float(lib().orc_logdet(self._h, np.ascontiguousarray(Lx, np.float64)))

    def solve(self, Lx, b):
        b = np.array(b, dtype=np.float64, order="F", copy=True)
        nrhs = 1 if b.ndim == 1 else b.shape[1]
        flat = np.ascontiguousarray(b.reshape(-1, order="F"))
        lib().orc_solve(self._h, np.ascontiguousarray(Lx, np.float64), flat, nrhs)
        return flat.reshape(b.shape, order="F")

    def selinv(self, Lx) -> np.ndarray:
        Z = np.zeros(self.lnz)
        lib().orc_selinv(self._h, np.ascontiguousarray(Lx, np.float64), Z)
        return Z

    def dense_L(self, Lx) -> np.ndarray:
        """Dense n x n copy of L (small n only)."""
        lp, li = self.L_pattern()
        L = np.zeros((self.n, self.n))
        for j in range(self.n):
            L[li[lp[j]:lp[j + 1]], j] = Lx[lp[j]:lp[j + 1]]
        return L

    def logdet_grad_values(self, Lx) -> np.ndarray:
        """d logdet / d value for every input entry, the symmetric matrix being
        parameterised by its lower triangle: 2 (A^-1)_ij off the diagonal and
        (A^-1)_ii on it."""
        Z = self.selinv(Lx)
        z = Z[self.value_map()]
        rows = self.rowind
        cols = np.repeat(np.arange(self.n), np.diff(self.colptr))
        return np.where(rows == cols, z, 2.0 * z)


def logdet_of(n, colptr, rowind, values, ordering="nd", nb=64):
    a = Analysis(n, colptr, rowind, ordering=ordering, nb=nb)
    Lx, info = a.factor(values)
    if info:
        raise ValueError(f"not SPD at permuted column {info}")
    return a.logdet(Lx)
