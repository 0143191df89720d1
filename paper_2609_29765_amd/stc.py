"""Python binding of libstc.so (include/stc.h): argument marshalling only.

Every step of the factorization, log-determinant, solve and adjoint runs in
the library's HIP kernels; PyTorch only provides device memory (the
workspace, value and right-hand-side tensors) and the current HIP stream.
There is no CPU fallback: without the built library, or without a GPU, the
numerical entry points raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstc.so")

ORDERINGS = {"natural": 0, "rcm": 1, "nd": 2, "auto": 3, "given": 4}
MODES = {"auto": 0, "dense": 1, "semisparse": 2}
ROUTES = {0: "dense", 1: "semisparse", 2: "supernodal"}
NOT_SPD = 1

_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")

# every entry point of include/stc.h
EXPORTS = [
    "stc_analyse", "stc_workspace_bytes", "stc_bind", "stc_factorize", "stc_factorize_batched",
    "stc_logdet", "stc_solve", "stc_solve_noalloc", "stc_solve_batched", "stc_logdet_backward", "stc_selinv", "stc_get_selinv", "stc_info", "stc_get_sizes",
    "stc_get_features", "stc_get_perm", "stc_get_etree", "stc_get_L_pattern", "stc_get_tiles",
    "stc_get_tasks", "stc_get_grid_positions", "stc_get_factor", "stc_get_batch_factor", "stc_get_work", "stc_get_plan_stats", "stc_check_schedule", "stc_check_solve_schedule", "stc_check_backward", "stc_profile_factorize",
    "stc_fp64_mfma_peak", "stc_save", "stc_load", "stc_destroy",
    "stc_last_error",
]

_LIB = None


class STCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libstc error {code}: {msg}")
        self.code = code


class _opts(C.Structure):
    _fields_ = [("nb", C.c_int32), ("mode", C.c_int32), ("ordering", C.c_int32),
                ("perm", C.c_void_p), ("wg_slots", C.c_int32), ("align", C.c_int32),
                ("max_split", C.c_int32), ("fold_pct", C.c_int32), ("batch", C.c_int32)]


def lib():
    """Load libstc.so (built in-tree by paper_2609_29765_amd/build.py)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2609_29765_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.stc_analyse.argtypes = [C.c_int64, _i64p, _i32p, C.POINTER(_opts), C.POINTER(vp)]
    L.stc_workspace_bytes.argtypes = [vp, C.c_int32, C.POINTER(C.c_size_t)]
    L.stc_bind.argtypes = [vp, vp, C.c_size_t, C.c_int32, vp]
    L.stc_factorize.argtypes = [vp, vp, vp]
    L.stc_factorize_batched.argtypes = [vp, vp, C.c_int32, vp, vp, vp]
    L.stc_logdet.argtypes = [vp, vp, vp]
    L.stc_solve.argtypes = [vp, vp, C.c_int32, vp]
    L.stc_solve_noalloc.argtypes = [vp, vp, C.c_int32, vp]
    L.stc_solve_batched.argtypes = [vp, vp, C.c_int32, C.c_int32, vp]
    L.stc_logdet_backward.argtypes = [vp, vp, vp, vp]
    L.stc_selinv.argtypes = [vp, vp, vp]
    L.stc_get_selinv.argtypes = [vp, _f64p, vp]
    L.stc_info.argtypes = [vp, C.POINTER(C.c_int32)]
    L.stc_get_sizes.argtypes = [vp, _i64p]
    L.stc_get_features.argtypes = [vp, _f64p]
    L.stc_get_perm.argtypes = [vp, _i32p]
    L.stc_get_etree.argtypes = [vp, _i32p]
    L.stc_get_L_pattern.argtypes = [vp, _i64p, _i32p]
    L.stc_get_tiles.argtypes = [vp, _i32p, _i32p, _i32p, _i32p, _i8p, _i64p, _i32p, _i32p]
    L.stc_get_tasks.argtypes = [vp, _i32p]
    L.stc_get_grid_positions.argtypes = [vp, _i64p, C.POINTER(C.c_int64)]
    L.stc_get_factor.argtypes = [vp, _f64p, vp]
    L.stc_get_batch_factor.argtypes = [vp, C.c_int32, _f64p, vp]
    L.stc_get_work.argtypes = [vp, _f64p]
    L.stc_get_plan_stats.argtypes = [vp, _i64p]
    L.stc_check_schedule.argtypes = [vp, _i64p]
    L.stc_check_solve_schedule.argtypes = [vp, _i64p]
    L.stc_check_backward.argtypes = [vp, _i64p]
    L.stc_profile_factorize.argtypes = [vp, vp, vp, _f64p, _i64p, _f64p]
    L.stc_fp64_mfma_peak.argtypes = [vp, _f64p]
    L.stc_save.argtypes = [vp, C.c_char_p]
    L.stc_load.argtypes = [C.c_char_p, C.POINTER(vp)]
    L.stc_destroy.argtypes = [vp]
    L.stc_destroy.restype = None
    L.stc_last_error.restype = C.c_char_p
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("stc_destroy", "stc_last_error"):
            f.restype = C.c_int
    _LIB = L
    return L


def _check(rc):
    if rc != 0:
        raise STCError(rc, lib().stc_last_error().decode())
    return rc


def _stream_ptr():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def _need_cuda(t, dtype_name="float64"):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("expected a device tensor")
    if str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"expected dtype {dtype_name}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")


class Analysis:
    """Once-per-pattern analysis; factorize / logdet / solve many times.

    nb: tile size 32, 64, 128 or 256, or 0 for the library's automatic
    choice (64, larger tiles for patterns on the dense route; see stc_opts).
    """

    def __init__(self, n, colptr, rowind, nb=64, mode="auto", ordering="auto", perm=None,
                 wg_slots=0, align=0, max_split=0, fold_pct=0, batch=0, _handle=None):
        L = lib()
        if _handle is None:
            self.colptr = np.ascontiguousarray(colptr, np.int64)
            self.rowind = np.ascontiguousarray(rowind, np.int32)
            self._perm_in = None if perm is None else np.ascontiguousarray(perm, np.int32)
            o = _opts(int(nb), MODES[mode], ORDERINGS[ordering],
                      None if self._perm_in is None else self._perm_in.ctypes.data, int(wg_slots),
                      int(align), int(max_split), int(fold_pct), int(batch))
            h = C.c_void_p()
            _check(L.stc_analyse(int(n), self.colptr, self.rowind, C.byref(o), C.byref(h)))
        else:
            h = _handle
        self._h = h
        sz = np.zeros(16, np.int64)
        _check(L.stc_get_sizes(h, sz))
        (self.n, self.qnz, self.lnz, self.nb, self.NT, self.ntiles, self.nrows, self.ntasks,
         mode_i, route_i, self.ndense, self.method, self.tact, self.store, self.nlevels,
         self.solve_launches) = (int(x) for x in sz)
        self.mode = {1: "dense", 2: "semisparse"}[mode_i]
        self.route = ROUTES[route_i]
        f = np.zeros(3)
        _check(L.stc_get_features(h, f))
        self.phi, self.rho, self.sigma = (float(x) for x in f)
        self._ws = None
        self.batch = 0

    def save(self, path):
        """Write the analysis to a file (see stc_save)."""
        _check(lib().stc_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path):
        """A new, unbound Analysis read from a file written by save()."""
        h = C.c_void_p()
        _check(lib().stc_load(os.fsencode(path), C.byref(h)))
        return cls(None, None, None, _handle=h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _LIB is not None:  # _LIB is None at interpreter exit
            _LIB.stc_destroy(h)
            self._h = None

    # ---------------------------------------------------------------- symbolic
    def perm(self):
        p = np.zeros(self.n, np.int32)
        _check(lib().stc_get_perm(self._h, p))
        return p

    def etree(self):
        p = np.zeros(self.n, np.int32)
        _check(lib().stc_get_etree(self._h, p))
        return p

    def L_pattern(self):
        lp = np.zeros(self.n + 1, np.int64)
        li = np.zeros(self.lnz, np.int32)
        _check(lib().stc_get_L_pattern(self._h, lp, li))
        return lp, li

    def tiles(self):
        nt = self.ntiles
        out = dict(m=np.zeros(nt, np.int32), k=np.zeros(nt, np.int32), cnt=np.zeros(nt, np.int32),
                   true_cnt=np.zeros(nt, np.int32), contig=np.zeros(nt, np.int8),
                   roff=np.zeros(nt + 1, np.int64), rows=np.zeros(max(self.nrows, 1), np.int32),
                   kd=np.zeros(self.NT, np.int32))
        _check(lib().stc_get_tiles(self._h, out["m"], out["k"], out["cnt"], out["true_cnt"],
                                   out["contig"], out["roff"], out["rows"], out["kd"]))
        out["rows"] = out["rows"][:self.nrows]
        return out

    def grid_positions(self):
        """Tile-grid position of every column of P A P^T (stc_get_grid_positions)."""
        p = np.zeros(self.n, np.int64)
        _check(lib().stc_get_grid_positions(self._h, p, None))
        return p

    @property
    def align(self):
        """stc_opts.align of the analysis (0: the uniform grid)."""
        p = np.zeros(self.n, np.int64)
        al = C.c_int64(0)
        _check(lib().stc_get_grid_positions(self._h, p, C.byref(al)))
        return int(al.value)

    def tasks(self):
        t = np.zeros((max(self.ntasks, 1), 4), np.int32)
        _check(lib().stc_get_tasks(self._h, t))
        return t[:self.ntasks]

    # ---------------------------------------------------------------- binding
    def workspace_bytes(self, batch=1):
        b = C.c_size_t()
        _check(lib().stc_workspace_bytes(self._h, int(batch), C.byref(b)))
        return int(b.value)

    def bind(self, batch=1, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libstc needs a HIP device; none is visible")
        nbytes = self.workspace_bytes(batch)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
        base = ws.data_ptr()
        off = (-base) % 256
        _check(lib().stc_bind(self._h, C.c_void_p(base + off), nbytes, int(batch), _stream_ptr()))
        self._ws = ws
        self.batch = int(batch)
        return self

    def _bound(self):
        if self._ws is None:
            self.bind()

    def release(self):
        """Drop the workspace; the next factorize binds a new one."""
        self._ws = None
        self.batch = 0

    def _ws_device(self):
        if self._ws is None:
            raise RuntimeError("the analysis is not bound to a workspace (factorize first)")
        return self._ws.device

    # ---------------------------------------------------------------- numeric
    def factorize(self, values):
        """values: device float64 tensor [nnz] in the analysed CSC entry order."""
        self._bound()
        _need_cuda(values)
        assert values.numel() == self.qnz
        self._values = values  # keep alive until the stream has consumed it
        _check(lib().stc_factorize(self._h, _dptr(values), _stream_ptr()))
        self._fact_id = getattr(self, "_fact_id", 0) + 1
        return self

    def factorize_batched(self, values):
        """values: device float64 [B, nnz]; returns (logdet[B], info[B]) on device."""
        import torch
        self._bound()
        _need_cuda(values)
        B = values.shape[0]
        if B > self.batch:
            self.bind(batch=B)
        ld = torch.empty(B, dtype=torch.float64, device=values.device)
        info = torch.empty(B, dtype=torch.int32, device=values.device)
        self._values = values
        _check(lib().stc_factorize_batched(self._h, _dptr(values), int(B), _dptr(ld), _dptr(info),
                                           _stream_ptr()))
        self._fact_id = getattr(self, "_fact_id", 0) + 1
        return ld, info

    def logdet(self):
        import torch
        out = torch.empty(1, dtype=torch.float64, device=self._ws_device())
        _check(lib().stc_logdet(self._h, _dptr(out), _stream_ptr()))
        return out[0]

    def solve(self, b):
        """Solve A x = b; b device float64 [n] or [n, nrhs] (column-major copy made)."""
        import torch
        _need_cuda(b)
        self._ws_device()
        one = b.dim() == 1
        if not (b.shape[0] == self.n and b.dim() in (1, 2)):
            raise ValueError(f"b must have shape [{self.n}] or [{self.n}, nrhs], got {tuple(b.shape)}")
        B = b.reshape(self.n, 1) if one else b
        nrhs = B.shape[1]
        X = B.t().clone(memory_format=torch.contiguous_format)  # column-major n x nrhs, never b itself
        _check(lib().stc_solve(self._h, _dptr(X), int(nrhs), _stream_ptr()))
        X = X.t()
        return X.reshape(-1) if one else X.contiguous()

    def solve_batched(self, b):
        """Solve A_b x_b = b_b for every value set b of the last batched
        factorization: b device float64 [B, n] or [B, n, nrhs] (nrhs <= 8)."""
        import torch
        _need_cuda(b)
        self._ws_device()
        one = b.dim() == 2
        if not (b.dim() in (2, 3) and b.shape[1] == self.n):
            raise ValueError(f"b must have shape [B, {self.n}] or [B, {self.n}, nrhs], got {tuple(b.shape)}")
        Bv = b.reshape(b.shape[0], self.n, 1) if one else b
        X = Bv.transpose(1, 2).clone(memory_format=torch.contiguous_format)  # per value set column-major
        _check(lib().stc_solve_batched(self._h, _dptr(X), int(Bv.shape[0]), int(Bv.shape[2]), _stream_ptr()))
        X = X.transpose(1, 2)
        return X.reshape(b.shape[0], self.n) if one else X.contiguous()

    def logdet_backward(self, gbar):
        import torch
        g = gbar.reshape(1).to(torch.float64).contiguous()
        out = torch.empty(self.qnz, dtype=torch.float64, device=self._ws_device())
        _check(lib().stc_logdet_backward(self._h, _dptr(g), _dptr(out), _stream_ptr()))
        return out

    def selinv(self):
        """Selected inversion of the last factorization: returns diag(A^-1) in
        original numbering (device float64 [n]); Z on the pattern of L stays
        in the workspace (selinv_pattern copies it to the host)."""
        import torch
        out = torch.empty(self.n, dtype=torch.float64, device=self._ws_device())
        _check(lib().stc_selinv(self._h, _dptr(out), _stream_ptr()))
        return out

    def selinv_pattern(self):
        """Host copy of Z = (P A P^T)^-1 on the pattern of L (L_pattern order)."""
        self._ws_device()
        Zx = np.zeros(self.lnz)
        _check(lib().stc_get_selinv(self._h, Zx, _stream_ptr()))
        return Zx

    def work(self):
        """Static flop and byte counts of one factorization (see stc_get_work)."""
        w = np.zeros(10)
        _check(lib().stc_get_work(self._h, w))
        keys = ["flops_update", "flops_potrf", "flops_trsm", "flops_tile", "flops_exact",
                "bytes_update", "bytes_load", "levels", "flops_backward", "levels_backward"]
        return dict(zip(keys, (float(x) for x in w)))

    def plan_stats(self):
        """{split_tasks, partial_doubles, separate_last_levels, graph_kernels,
        partial_doubles_unshared} of the factorization plan (see
        stc_get_plan_stats)."""
        st = np.zeros(5, dtype=np.int64)
        _check(lib().stc_get_plan_stats(self._h, st))
        return dict(zip(["split_tasks", "partial_doubles", "separate_last_levels", "graph_kernels",
                         "partial_doubles_unshared"], (int(x) for x in st)))

    def check_schedule(self):
        """Host check of the kernel dependency graph the factorization replays
        (see stc_check_schedule); raises on a conflicting pair of kernels.
        Returns {nodes, edges, unordered_pairs, objects, slot_pairs}."""
        st = np.zeros(5, dtype=np.int64)
        _check(lib().stc_check_schedule(self._h, st))
        return dict(zip(["nodes", "edges", "unordered_pairs", "objects", "slot_pairs"], (int(x) for x in st)))

    def check_solve_schedule(self):
        """Host check of the solve sweeps' work items against the tile
        dependencies (see stc_check_solve_schedule); raises on a violation.
        Returns {launches, step_items, panel_items, fused_launches}."""
        st = np.zeros(4, dtype=np.int64)
        _check(lib().stc_check_solve_schedule(self._h, st))
        return dict(zip(["launches", "step_items", "panel_items", "fused_launches"], (int(x) for x in st)))

    def check_backward(self):
        """Host check of the reverse-mode plan (see stc_check_backward);
        raises on a violation.  Returns {levels, tasks, reads, folds, slots}."""
        st = np.zeros(5, dtype=np.int64)
        _check(lib().stc_check_backward(self._h, st))
        return dict(zip(["levels", "tasks", "reads", "folds", "slots"], (int(x) for x in st)))

    KERNEL_KINDS = ["load", "k_potrf", "k_upd<G>", "k_upd", "k_trsm"]

    def profile_factorize(self, values):
        """Event timing of one eager factorization, per kernel form:
        {kind: (ms, launches, flops)} (see stc_profile_factorize)."""
        self._bound()
        _need_cuda(values)
        ms = np.zeros(5)
        cnt = np.zeros(5, np.int64)
        fl = np.zeros(5)
        _check(lib().stc_profile_factorize(self._h, _dptr(values), _stream_ptr(), ms, cnt, fl))
        self._fact_id = getattr(self, "_fact_id", 0) + 1
        return {k: (float(ms[i]), int(cnt[i]), float(fl[i])) for i, k in enumerate(self.KERNEL_KINDS)}

    def info(self):
        self._ws_device()
        v = C.c_int32()
        _check(lib().stc_info(self._h, C.byref(v)))
        return int(v.value)

    def factor(self, member=None):
        """Host copy of L in L_pattern() order: the last single factorization,
        or value set `member` of the last batched one."""
        self._ws_device()
        Lx = np.zeros(self.lnz)
        if member is None:
            _check(lib().stc_get_factor(self._h, Lx, _stream_ptr()))
        else:
            _check(lib().stc_get_batch_factor(self._h, int(member), Lx, _stream_ptr()))
        return Lx


def fp64_mfma_peak():
    """Measured FP64 MFMA issue rate of the current device, TFLOP/s."""
    out = np.zeros(1)
    _check(lib().stc_fp64_mfma_peak(_stream_ptr(), out))
    return float(out[0])


def _make_logdet_function():
    import torch

    class LogDet(torch.autograd.Function):
        """logdet A(values) with the library's adjoint as the backward."""

        @staticmethod
        def forward(ctx, values, analysis):
            analysis.factorize(values)
            ctx.analysis = analysis
            ctx.fact_id = analysis._fact_id
            ctx.save_for_backward(values)
            return analysis.logdet().clone()

        @staticmethod
        def backward(ctx, g):
            a = ctx.analysis
            if a._fact_id != ctx.fact_id:  # another factorization ran since: redo this one
                (values,) = ctx.saved_tensors
                a.factorize(values.detach())
            return a.logdet_backward(g), None

    return LogDet


def logdet(values, analysis):
    """Differentiable log-determinant of the matrix with the given values."""
    global _LOGDET
    try:
        fn = _LOGDET
    except NameError:
        fn = _LOGDET = _make_logdet_function()
    return fn.apply(values, analysis)
