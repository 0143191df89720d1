"""Benchmark: FP64 tile-Cholesky factorizations per second on one MI355X.

Headline workload: the dense-route matrix -- random SPD of order 12288 with
~20% off-diagonal density (uniform pattern, N(0,1) entries, diagonal = row
absolute sum + 1), tile 256, every tile dense.  One step = value load + the
whole POTRF/SYRK/GEMM/TRSM tile schedule (one HIP-graph replay), values
already resident in HBM.

Prints one JSON line.  Besides the headline value it carries:
  roofline      the level kernel (POTRF, updates with or without 128-blocks,
                TRSM) that takes most of the factorization time:
                tile-algorithmic flops of the tasks it runs per launch /
                its event-timed average launch duration, against the FP64
                matrix peak of 78.6 TFLOP/s; HBM traffic per launch from the
                committed counter summary when it matches the current kernels;
  cpu_baseline  the oracle (plain serial C, one core) timed on the leading
                principal blocks of order n/4 and n/2 of this matrix, the
                larger scaled to the full order by the exact flop ratio
                (a model, stated as such); cpu_baseline_configs times the
                oracle on the other workloads beside their GPU figures;
  extras        the other forms of the metric, measured in a child process
                (so the headline process's kernel statistics cover the
                headline only): batched factorization of 128 value sets
                against the plain path, logdet backward against the forward
                and against central differences, the semisparse
                spatio-temporal matrix, and the small 2-D GMRF.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 matrix peak (published)
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E (published)
# tile grids the extras' autotuner tries, as multiples of the tile size: the
# uniform grid and grids aligned to elimination subtrees of 1, 2, 4 and 8 tiles
GRID_ALIGNS = (0, 1, 2, 4, 8)
# weights of a partial-slot fold in the split-K cost model (percent of the
# measured one) tried on the best grid
FOLD_PCTS = (0, 50, 200, 300)
KERNEL_SOURCES = ["paper_2609_29765_amd/csrc/kernels.hpp", "paper_2609_29765_amd/csrc/device_types.hpp",
                  "paper_2609_29765_amd/csrc/runtime.hip", "paper_2609_29765_amd/csrc/analyse.cpp"]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_lib():
    import torch
    from paper_2609_29765_amd import stc
    if not os.path.exists(stc.LIB_PATH):
        from paper_2609_29765_amd import build as pb
        pb.build()
    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)
    return stc


def events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def timed(fn, reps):
    """Milliseconds per call of fn over reps calls, bracketed by syncs."""
    import torch
    torch.cuda.synchronize()
    e0, e1 = events()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# headline: dense route, n = 12288, tile 256
# ---------------------------------------------------------------------------

def semisparse_pass(align, nb=128):
    """Counter runs over the active-column route: the spatio-temporal
    arrowhead (n = 101,258, tile nb, ND, grid aligned to subtrees of `align`
    columns, 0 = uniform) factorized once through the graph and
    once kernel by kernel (one launch per level and kernel kind, the launches
    the per-kind figures charge), then a plain 1 GiB device copy whose counter
    readings calibrate the byte counters.  Prints one JSON line: the per-kind
    eager times and flops and the plan's byte terms."""
    import torch
    stc = load_lib()
    from paper_2609_29765_amd import workloads
    w = workloads.spatiotemporal_arrowhead()
    v = torch.from_numpy(w.values).cuda()
    a = stc.Analysis(w.n, w.colptr, w.rowind, nb=nb, ordering="nd", align=align).bind()
    a.factorize(v)
    torch.cuda.synchronize()
    assert a.info() == 0
    prof = a.profile_factorize(v)
    x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"workload": f"spatio-temporal arrowhead n=101258, tile {nb}, ND, grid align {align}", "work": a.work(),
                      "kinds": {k: {"ms": ms, "launches": c, "flops": f} for k, (ms, c, f) in prof.items()}}),
          flush=True)


def backward_pass(align, nb=128):
    """Counter runs over the reverse mode: the spatio-temporal arrowhead
    (n = 101,258, tile nb, ND, grid aligned to subtrees of `align` columns)
    factorized and differentiated (selected inverse on the factor's pattern,
    then the logdet gradient) twice, each through its graph; segment 2 of a
    trace is the second pass.  Prints one JSON line: the plan's reverse-mode
    flops and levels and the reverse-mode plan checker's counts."""
    import torch
    stc = load_lib()
    from paper_2609_29765_amd import workloads
    w = workloads.spatiotemporal_arrowhead()
    v = torch.from_numpy(w.values).cuda()
    a = stc.Analysis(w.n, w.colptr, w.rowind, nb=nb, ordering="nd", align=align).bind()
    one = torch.ones(1, dtype=torch.float64, device="cuda")
    for _ in range(2):
        a.factorize(v)
        a.logdet_backward(one)
    torch.cuda.synchronize()
    assert a.info() == 0
    wk = a.work()
    print(json.dumps({"workload": f"spatio-temporal arrowhead n=101258, tile {nb}, ND, grid align {align}",
                      "flops_backward": wk["flops_backward"], "levels_backward": wk["levels_backward"],
                      "check_backward": a.check_backward()}), flush=True)


def batched_pass(batch_hint):
    """Counter runs over the batched form: the 3-D Laplacian 24^3 with 128
    value sets (tile 64, ND, grid aligned at 128 columns, split-K schedule for
    a batch of `batch_hint` value sets, 0 = for one), factorized twice in one
    batched call each, then a plain 1 GiB device copy whose counter readings
    calibrate the byte counters.  Prints one JSON line: the plan's work terms
    and the batch's time."""
    import torch
    stc = load_lib()
    from paper_2609_29765_amd import workloads
    w = workloads.batched_laplacian3d(m=24, B=128, seed=0)
    V = torch.from_numpy(w.values).cuda()
    a = stc.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd", align=128, batch=batch_hint).bind(batch=128)
    for _ in range(2):
        _, info = a.factorize_batched(V)
    torch.cuda.synchronize()
    assert int(info.abs().sum().item()) == 0
    ms = timed(lambda: a.factorize_batched(V), 1)
    x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"workload": f"3-D Laplacian 24^3, B=128, tile 64, ND, grid align 128, batch hint {batch_hint}",
                      "work": a.work(), "plan": a.plan_stats(), "ms_batched": ms}), flush=True)


def solve_pass(align, nb=128):
    """Kernel-trace runs over the solve: the spatio-temporal arrowhead
    (n = 101,258, tile nb, ND, grid alignment `align`) factorized once, then three solves with one
    right-hand side and three with eight, each group's sweeps replayed from
    its graph (the first call of a group captures it).  Prints one JSON line
    with the event-timed solves and the sweeps' launch count."""
    import torch
    stc = load_lib()
    from paper_2609_29765_amd import workloads
    w = workloads.spatiotemporal_arrowhead()
    v = torch.from_numpy(w.values).cuda()
    a = stc.Analysis(w.n, w.colptr, w.rowind, nb=nb, ordering="nd", align=align).bind()
    a.factorize(v)
    torch.cuda.synchronize()
    assert a.info() == 0
    g = torch.Generator(device="cuda").manual_seed(0)
    out = {}
    for nrhs in (1, 8):
        b = torch.randn((w.n,) if nrhs == 1 else (w.n, nrhs), dtype=torch.float64, device="cuda", generator=g)
        ms = []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            a.solve(b)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        out[f"solve_{nrhs}rhs_ms"] = [round(x, 3) for x in ms]
    print(json.dumps({"workload": f"spatio-temporal arrowhead n=101258, tile {nb}, ND, grid align {align}",
                      "sweep_launches": a.solve_launches, **out}), flush=True)


def kind_table(prof, work):
    """Per kernel kind of one eager factorization: time, launches, FP64
    TFLOP/s of the tile-algorithmic flops (update, POTRF, TRSM kinds) and, for
    the value load (zero fill plus scatter), GB/s of its algorithmic bytes."""
    out = {}
    for k, (ms, cnt, fl) in prof.items():
        e = {"ms_per_factorization": round(ms, 4), "launches": cnt,
             "avg_launch_ms": round(ms / max(cnt, 1), 5),
             "tflops": round(fl / (ms * 1e-3) / 1e12, 3) if ms > 0 and fl > 0 else None}
        if k == "load" and ms > 0:
            e["hbm_gbs"] = round(work["bytes_load"] / (ms * 1e-3) / 1e9, 1)
        out[k] = e
    return out


def headline(args):
    import torch
    stc = load_lib()
    from paper_2609_29765_amd import workloads

    t0 = time.time()
    w = workloads.dense_spd(args.n, 0.2, 0)
    t_gen = time.time() - t0
    t0 = time.time()
    a = stc.Analysis(w.n, w.colptr, w.rowind, nb=args.nb, mode="auto", ordering="natural")
    t_analyse = time.time() - t0
    vals = torch.from_numpy(w.values).cuda()
    # the schedule axis of the autotuner: concurrent update work-groups the
    # split-K plan balances for, timed on this matrix at the headline tile
    tune_table = None
    if args.tune_slots:
        from paper_2609_29765_amd.autotune import autotune
        del a
        a, tune_table = autotune(w.n, w.colptr, w.rowind, vals, nbs=(args.nb,), ordering="natural", trials=3,
                                 slots=tuple(int(x) for x in args.tune_slots.split(",")),
                                 folds=tuple(int(x) for x in args.tune_folds.split(",")) if args.tune_folds else (0,))
        log(f"schedule tuning: {tune_table}")
    else:
        a.bind()
    work = a.work()
    log(f"n={w.n} nnz={w.nnz} nb={a.nb} mode={a.mode} route={a.route} levels={a.nlevels} "
        f"analyse={t_analyse:.2f}s gen={t_gen:.2f}s")

    for _ in range(args.warmup):
        a.factorize(vals)
    torch.cuda.synchronize()
    assert a.info() == 0, "warm-up factorization failed"
    torch.cuda.synchronize()
    e0, e1 = events()
    e0.record()
    for _ in range(args.steps):
        a.factorize(vals)
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    ld = float(a.logdet().item())
    assert a.info() == 0
    log(f"{args.steps} steps {ms_step:.3f} ms/step logdet={ld:.6f}")
    # the same replays timed one by one, after the timed region: median and min
    per = []
    for _ in range(args.steps):
        s0, s1 = events()
        s0.record()
        a.factorize(vals)
        s1.record()
        torch.cuda.synchronize()
        per.append(s0.elapsed_time(s1))
    per.sort()
    step_stats = {"median_ms": round(per[len(per) // 2], 4), "min_ms": round(per[0], 4)}

    # per-launch event timing of eager factorizations (same kernels, one
    # stream), charged to the kernel each launch uses
    agg = {}
    for _ in range(args.prof_reps):
        for k, (ms, cnt, fl) in a.profile_factorize(vals).items():
            m0, c0, f0 = agg.get(k, (0.0, 0, 0.0))
            agg[k] = (m0 + ms, c0 + cnt, f0 + fl)
    level_kinds = [k for k in agg if k != "load" and agg[k][1] > 0]
    dom = max(level_kinds, key=lambda k: agg[k][0])
    ms_d, cnt_d, fl_d = agg[dom]
    avg_ms = ms_d / cnt_d
    flops_per_launch = fl_d / cnt_d
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    cull = "false" if a.mode == "dense" else "true"  # active-column plans run the group-skipping update kernels
    symbol = {"k_potrf": f"k_potrf<{a.nb}>", "k_upd<G>": f"k_upd<{a.nb}, true, {cull}>",
              "k_upd": f"k_upd<{a.nb}, false, {cull}>", "k_trsm": f"k_trsm<{a.nb}>"}[dom]
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic_dense12288_nb256.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            tr = json.load(fh)
        if tr.get("source_hash") == kernel_source_hash() and symbol in tr.get("kernels", {}):
            traffic = tr["kernels"][symbol]["bytes_per_launch"]
    roofline = {
        "bound": "mfma",
        "achieved": round(achieved, 3),
        "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
        "traffic": traffic,
        "kernel": symbol,
        "launches": cnt_d // args.prof_reps,
        "avg_launch_ms": round(avg_ms, 5),
        "flops_per_launch": flops_per_launch,
    }
    if dom in ("k_upd<G>", "k_upd") and work["flops_update"] > 0:
        # operand rows read + output tiles read and written, the plan's
        # update bytes shared out in proportion to the launch's flops
        roofline["algorithmic_bytes_per_launch"] = work["bytes_update"] * flops_per_launch / work["flops_update"]
    fam_ms = sum(agg[k][0] for k in level_kinds)
    fam_fl = sum(agg[k][2] for k in level_kinds)
    kinds = kind_table({k: (v[0] / args.prof_reps, v[1] // args.prof_reps, v[2] / args.prof_reps)
                        for k, v in agg.items()}, work)
    log(f"roofline {symbol}: {achieved:.2f} TFLOP/s over {cnt_d // args.prof_reps} launches; "
        f"all level kernels {fam_fl / (fam_ms * 1e-3) / 1e12:.2f} TFLOP/s")

    # measured ceilings: MFMA issue microkernel, library DGEMM (rocBLAS via torch)
    mfma_peak = stc.fp64_mfma_peak()
    nd = 8192
    xa = torch.randn(nd, nd, dtype=torch.float64, device="cuda")
    xb = torch.randn(nd, nd, dtype=torch.float64, device="cuda")
    torch.matmul(xa, xb)
    dgemm_ms = timed(lambda: torch.matmul(xa, xb), 3)
    dgemm_tf = 2.0 * nd ** 3 / (dgemm_ms * 1e-3) / 1e12
    del xa, xb
    log(f"measured FP64 MFMA issue {mfma_peak:.1f} TFLOP/s, library DGEMM n={nd} {dgemm_tf:.1f} TFLOP/s")

    # the consumers of the resident factor on the same workload (Sec. 6.7):
    # logdet, and the solve for 1 and 8 right-hand sides
    a.factorize(vals)
    b1 = torch.randn(w.n, dtype=torch.float64, device="cuda")
    b8 = torch.randn(w.n, 8, dtype=torch.float64, device="cuda")
    a.logdet(), a.solve(b1.clone()), a.solve(b8.clone())  # graphs captured on first use
    uses = {"logdet_ms": round(timed(lambda: a.logdet(), 10), 4),
            "solve_1rhs_ms": round(timed(lambda: a.solve(b1), 5), 4),
            "solve_8rhs_ms": round(timed(lambda: a.solve(b8), 5), 4)}
    log(f"resident factor: {uses}")

    return dict(
        ms_step=ms_step, step_stats=step_stats, logdet=ld, analyse_s=t_analyse, a=a, w=w, work=work,
        tune_table=tune_table, wg_slots=(min(tune_table, key=lambda r: r["ms"])["wg_slots"] if tune_table else 0),
        roofline=roofline, uses=uses,
        kinds=kinds, level_family_tflops=round(fam_fl / (fam_ms * 1e-3) / 1e12, 3),
        peaks={"mfma_issue": round(mfma_peak, 2), "dgemm_library_8192": round(dgemm_tf, 2)})


# ---------------------------------------------------------------------------
# extras (child process)
# ---------------------------------------------------------------------------

def extra_gmrf():
    """Small 2-D GMRF (n = 1024, ND): factorize + logdet + solve, tile size
    and grid tuned."""
    import torch
    from paper_2609_29765_amd import workloads
    from paper_2609_29765_amd.autotune import autotune
    w = workloads.gmrf_grid2d(32, 32, 0.1, 0)
    v = torch.from_numpy(w.values).cuda()
    a, table = autotune(w.n, w.colptr, w.rowind, v, nbs=(32, 64), ordering="nd", trials=20, aligns=GRID_ALIGNS)
    b = torch.from_numpy(w.b).cuda()
    out = torch.empty(1, dtype=torch.float64, device="cuda")

    def step():
        a.factorize(v)
        a.logdet()
        a.solve(b)

    step()
    us_f = timed(lambda: a.factorize(v), 200) * 1e3
    us = timed(step, 200) * 1e3
    del out
    return {"workload": "2-D GMRF 32x32 grid, Laplacian + 0.1 I, n=1024, ND",
            "nb": a.nb, "align": a.align,
            "us_per_factorization": round(us_f, 2), "us_per_factorize_logdet_solve": round(us, 2),
            "levels": a.nlevels, "mode": a.mode, "autotune": table}


def extra_supernodal():
    """2-D GMRF on a 200 x 200 grid (n = 40,000, ND), which the selector
    routes supernodal at tile 128: the route's tree-aligned grid against the
    uniform grid (the same tiles forced semisparse), and logdet against its
    closed form."""
    import numpy as np
    import torch
    from paper_2609_29765_amd import stc, workloads
    w = workloads.gmrf_grid2d(200, 200, 0.1, 0)
    v = torch.from_numpy(w.values).cuda()
    out = {"workload": "2-D GMRF 200x200 grid, Laplacian + 0.1 I, n=40000, ND, tile 128"}
    for key, mode in (("route", "auto"), ("uniform_grid", "semisparse")):
        a = stc.Analysis(w.n, w.colptr, w.rowind, nb=128, ordering="nd", mode=mode).bind()
        ms = timed(lambda: a.factorize(v), 50)
        ld = float(a.logdet().item())
        assert a.info() == 0
        out[key] = {"route": a.route, "align": a.align, "levels": a.nlevels, "ms_per_factorization": round(ms, 4),
                    "logdet": ld}
        a.release()
        del a
    lam = 2 - 2 * np.cos(np.pi * np.arange(200) / 200)
    closed = float(np.log(lam[:, None] + lam[None, :] + 0.1).sum())
    out["rel_logdet_vs_closed_form"] = max(abs(out[k]["logdet"] - closed) / abs(closed) for k in ("route", "uniform_grid"))
    out["speedup_vs_uniform_grid"] = round(out["uniform_grid"]["ms_per_factorization"] /
                                          out["route"]["ms_per_factorization"], 2)
    return out


def extra_semisparse():
    """Spatio-temporal arrowhead, n = 101,258: tile size (64, 128, 256) and grid tuned."""
    import torch
    from paper_2609_29765_amd import workloads
    from paper_2609_29765_amd.autotune import autotune
    w = workloads.spatiotemporal_arrowhead()
    v = torch.from_numpy(w.values).cuda()
    t0 = time.time()
    a, table = autotune(w.n, w.colptr, w.rowind, v, nbs=(64, 128, 256), ordering="nd", trials=3, aligns=GRID_ALIGNS,
                        folds=FOLD_PCTS)
    t_tune = time.time() - t0
    ms = timed(lambda: a.factorize(v), 10)
    assert a.info() == 0
    wk = a.work()
    prof = a.profile_factorize(v)
    return {"workload": "spatio-temporal arrowhead n=101258 (50 steps x 45x45 grid, AR1 0.9, kappa 0.5, "
                        "8 dense border rows), ND ordering",
            "nb": a.nb, "align": a.align, "mode": a.mode, "route": a.route, "levels": a.nlevels,
            "factorizations_per_s": round(1000.0 / ms, 3), "ms_per_factorization": round(ms, 3),
            "gflops_tile": round(wk["flops_tile"] / (ms * 1e-3) / 1e9, 1),
            "gflops_exact": round(wk["flops_exact"] / (ms * 1e-3) / 1e9, 1),
            "tile_gflop": round(wk["flops_tile"] / 1e9, 2), "exact_gflop": round(wk["flops_exact"] / 1e9, 2),
            "autotune": table, "autotune_s": round(t_tune, 1),
            "kernels": kind_table(prof, wk),
            "logdet": float(a.logdet().item())}


def extra_batched(B):
    """3-D Laplacian 24^3 + 0.05 I, B value sets: one batched call vs B plain calls."""
    import torch
    from paper_2609_29765_amd import workloads
    from paper_2609_29765_amd.autotune import autotune
    w = workloads.batched_laplacian3d(m=24, B=B, seed=0)
    V = torch.from_numpy(w.values).cuda()
    a, table = autotune(w.n, w.colptr, w.rowind, V, nbs=(64, 128), ordering="nd", batched=True, trials=2,
                        aligns=GRID_ALIGNS, folds=FOLD_PCTS)
    ms_batched = timed(lambda: a.factorize_batched(V), 3)
    ld_b, info = a.factorize_batched(V)
    assert int(info.abs().sum().item()) == 0
    ld_s = torch.empty(B, dtype=torch.float64, device="cuda")
    # the plain path on its own schedule: same tiles and grid, split balanced
    # for one value set
    from paper_2609_29765_amd import stc
    p1 = stc.Analysis(w.n, w.colptr, w.rowind, nb=a.nb, ordering="nd", align=a.align).bind()

    def plain():
        for i in range(B):
            p1.factorize(V[i])
            ld_s[i:i + 1].copy_(p1.logdet().reshape(1))

    plain()
    ms_plain = timed(plain, 2)
    dev = float(((ld_s - ld_b).abs() / ld_b.abs()).max().item())
    return {"workload": f"3-D Laplacian 24^3 + 0.05 I, n=13824, B={B} hyperparameter value sets, ND",
            "nb": a.nb, "align": a.align, "mode": a.mode, "levels": a.nlevels, "B": B,
            "ms_batched": round(ms_batched, 3), "ms_plain_loop": round(ms_plain, 3),
            "batched_speedup": round(ms_plain / ms_batched, 3),
            "factorizations_per_s_batched": round(B * 1000.0 / ms_batched, 1),
            "factorizations_per_s_plain": round(B * 1000.0 / ms_plain, 1),
            "max_rel_logdet_batched_vs_plain": dev, "autotune": table}


def extra_backward():
    """Differentiable arrowhead n = 12,508: logdet + gradient vs forward and FD."""
    import numpy as np
    import torch
    from paper_2609_29765_amd import workloads
    from paper_2609_29765_amd.autotune import autotune
    w = workloads.differentiable_arrowhead(20, 25, 8, 0)
    v = torch.from_numpy(w.values).cuda()
    a, table = autotune(w.n, w.colptr, w.rowind, v, nbs=(32, 64, 128), ordering="nd", trials=3,
                        objective="logdet_grad", aligns=GRID_ALIGNS, folds=FOLD_PCTS)
    one = torch.ones(1, dtype=torch.float64, device="cuda")
    dv = torch.from_numpy(w.dvalues).cuda()

    def fwd():
        a.factorize(v)
        return a.logdet()

    def fwd_bwd():
        a.factorize(v)
        a.logdet()
        return dv @ a.logdet_backward(one)

    fwd_bwd()
    ms_f = timed(fwd, 20)
    ms_fb = timed(fwd_bwd, 20)
    g = fwd_bwd().cpu().numpy()
    th = w.meta["theta"]
    h = 1e-5
    plus_minus = []
    for i in range(3):
        for s in (+1, -1):
            t2 = th.copy()
            t2[i] += s * h
            plus_minus.append(torch.from_numpy(workloads.differentiable_arrowhead(20, 25, 8, 0, theta=t2).values).cuda())
    lds = torch.empty(6, dtype=torch.float64, device="cuda")

    def fd():
        for j, vv in enumerate(plus_minus):
            a.factorize(vv)
            lds[j:j + 1].copy_(a.logdet().reshape(1))

    fd()
    ms_fd = timed(fd, 5)
    l6 = lds.cpu().numpy()
    gfd = (l6[0::2] - l6[1::2]) / (2 * h)
    wk = a.work()
    return {"workload": "differentiable arrowhead n=12508 (20 steps x 25x25 grid + 8 border rows), "
                        "theta=(log tau, log kappa, atanh rho) seed 0, ND",
            "nb": a.nb, "align": a.align, "levels_forward": a.nlevels, "levels_backward": int(wk["levels_backward"]),
            "ms_forward": round(ms_f, 4), "ms_forward_backward": round(ms_fb, 4),
            "backward_ratio": round(ms_fb / ms_f, 3),
            "ms_fd_gradient": round(ms_fd, 4), "speedup_vs_fd": round(ms_fd / ms_fb, 3),
            "grad": [float(x) for x in g], "grad_fd": [float(x) for x in gfd],
            "max_rel_grad_vs_fd": float(np.max(np.abs(g - gfd) / np.abs(gfd))),
            "backward_gflop": round(wk["flops_backward"] / 1e9, 3), "autotune": table}


def extra_backward_semisparse():
    """Spatio-temporal arrowhead n = 101,258 (tile 128, ND, grid aligned at
    512 columns): logdet and its gradient with respect to the input values
    against the factorization alone, and the gradient's trace identity
    (gradient . values = tr(Q^-1 Q) = n)."""
    import torch
    stc = load_lib()
    from paper_2609_29765_amd import workloads
    w = workloads.spatiotemporal_arrowhead()
    v = torch.from_numpy(w.values).cuda()
    a = stc.Analysis(w.n, w.colptr, w.rowind, nb=128, ordering="nd", align=512).bind()
    one = torch.ones(1, dtype=torch.float64, device="cuda")

    def fwd():
        a.factorize(v)
        return a.logdet()

    def fwd_bwd():
        a.factorize(v)
        a.logdet()
        return a.logdet_backward(one)

    g = fwd_bwd()
    ms_f = timed(fwd, 10)
    ms_fb = timed(fwd_bwd, 10)
    wk = a.work()
    return {"workload": "spatio-temporal arrowhead n=101258, tile 128, ND, grid aligned at 512 columns",
            "levels_forward": a.nlevels, "levels_backward": int(wk["levels_backward"]),
            "ms_forward": round(ms_f, 3), "ms_forward_backward": round(ms_fb, 3),
            "backward_ratio": round(ms_fb / ms_f, 3), "backward_gflop": round(wk["flops_backward"] / 1e9, 1),
            "rel_trace_identity": abs(float(g @ v) - w.n) / w.n}


def run_extras(path, batch):
    load_lib()
    out = {}
    for name, fn in [("gmrf_2d", extra_gmrf), ("backward", extra_backward),
                     ("batched", lambda: extra_batched(batch)), ("supernodal", extra_supernodal),
                     ("semisparse", extra_semisparse), ("backward_semisparse", extra_backward_semisparse)]:
        t0 = time.time()
        log(f"extra {name} ...")
        out[name] = fn()
        out[name]["wall_s"] = round(time.time() - t0, 1)
        log(f"extra {name}: {json.dumps(out[name])[:300]}")
        import torch
        torch.cuda.empty_cache()
    with open(path, "w") as fh:
        json.dump(out, fh)


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample
# ---------------------------------------------------------------------------

def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "the host"


def _best_of(fn, reps):
    """Minimum wall time of reps calls of fn after one warm-up call (the
    paper's timing convention, Sec. 6.1)."""
    fn()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return min(ts)


def _leading_block(w, m):
    """Lower CSC of the leading m x m principal block of a workload: an SPD
    matrix whose Cholesky factor is the leading block of the full factor."""
    import numpy as np
    cp, ri, v = w.colptr, w.rowind, w.values
    keep = ri < m
    col = np.repeat(np.arange(w.n), np.diff(cp))
    keep &= col < m
    cnt = np.bincount(col[keep], minlength=m)[:m]
    cp2 = np.zeros(m + 1, np.int64)
    np.cumsum(cnt, out=cp2[1:])
    return cp2, np.ascontiguousarray(ri[keep], np.int32), np.ascontiguousarray(v[keep])


def cpu_baseline(args):
    """The oracle (plain serial C, one thread) on bounded samples of the
    headline matrix itself: its leading principal blocks of order n/4 and
    n/2, whose factors are the leading blocks of the full factor.  Dense
    Cholesky work grows as the cube of the order, so the full factorization's
    time is modelled as the larger sample's time times the exact flop ratio;
    the two samples' rates show how far that rate holds."""
    from oracle import oracle
    from paper_2609_29765_amd import workloads
    w = workloads.dense_spd(args.n, 0.2, 0)
    flops = lambda m: m * (m + 1) * (2 * m + 1) / 6.0  # sum_j c_j^2 of a dense factor of order m
    rates = {}
    t_big, m_big = None, None
    for m in (args.n // 4, args.n // 2):
        cp, ri, v = _leading_block(w, m)
        o = oracle.Analysis(m, cp, ri, "natural", nb=args.nb)
        t0 = time.perf_counter()
        _, info = o.factor(v)
        t = time.perf_counter() - t0
        assert info == 0
        rates[m] = (t, flops(m) / t / 1e9)
        t_big, m_big = t, m
        log(f"cpu baseline: oracle on the leading {m} x {m} block: {t:.2f} s, {rates[m][1]:.2f} GFLOP/s")
    scale = flops(args.n) / flops(m_big)
    return {
        "value": round(1.0 / (t_big * scale), 6),
        "unit": "factorizations/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"oracle factorization (serial C, one thread) of the leading principal {m_big} x {m_big} block of "
                  f"the headline matrix took {t_big:.2f} s on {_cpu_model()} ({os.cpu_count()} logical CPUs visible); "
                  f"model: times the exact flop ratio {scale:.2f} to n={args.n}.  Rates: "
                  + ", ".join(f"n={m}: {r[1]:.2f} GFLOP/s ({r[0]:.2f} s)" for m, r in rates.items()),
    }


def cpu_baseline_configs(extras):
    """The oracle on the other workloads, beside the GPU figures of the same
    run: analysis (symbolic) and factorization (numeric) timed apart; the
    cheap ones as the minimum of 3 after a warm-up, the spatio-temporal
    arrowhead once (one factorization is tens of seconds), the batch on four
    of its 128 members."""
    from oracle import oracle
    from paper_2609_29765_amd import workloads
    ex = extras or {}
    out = {"cpu": _cpu_model(), "cores": 1, "logical_cpus_visible": os.cpu_count()}

    def gpu(name, key):
        return ex.get(name, {}).get(key)

    def row(name, w, nb, gpu_ms, reps=3):
        if reps:
            t_sym = _best_of(lambda: oracle.Analysis(w.n, w.colptr, w.rowind, "nd", nb=nb), reps)
            o = oracle.Analysis(w.n, w.colptr, w.rowind, "nd", nb=nb)
            t_num = _best_of(lambda: o.factor(w.values), reps)
        else:
            t0 = time.perf_counter()
            o = oracle.Analysis(w.n, w.colptr, w.rowind, "nd", nb=nb)
            t_sym = time.perf_counter() - t0
            t0 = time.perf_counter()
            o.factor(w.values)
            t_num = time.perf_counter() - t0
        r = {"oracle_symbolic_s": round(t_sym, 4), "oracle_numeric_s": round(t_num, 5),
             "timing": "min of 3 after a warm-up" if reps else "one run", "gpu_ms": gpu_ms}
        if gpu_ms:
            r["gpu_speedup_vs_oracle"] = round(t_num * 1e3 / gpu_ms, 2)
        log(f"oracle {name}: {r}")
        return o, r

    w = workloads.gmrf_grid2d(32, 32, 0.1, 0)
    us = gpu("gmrf_2d", "us_per_factorization")
    out["gmrf_2d"] = row("gmrf_2d", w, 64, us * 1e-3 if us else None)[1]
    w = workloads.differentiable_arrowhead(20, 25, 8, 0)
    o, r = row("backward", w, gpu("backward", "nb") or 128, gpu("backward", "ms_forward"))
    Lx, _ = o.factor(w.values)
    r["oracle_selected_inverse_gradient_s"] = round(_best_of(lambda: o.logdet_grad_values(Lx), 3), 4)
    r["gpu_forward_backward_ms"] = gpu("backward", "ms_forward_backward")
    out["backward"] = r
    wb = workloads.batched_laplacian3d(m=24, B=128, seed=0)
    o = oracle.Analysis(wb.n, wb.colptr, wb.rowind, "nd", nb=gpu("batched", "nb") or 64)
    o.factor(wb.values[0])
    ts = []
    for b in (0, 1, 63, 127):
        t0 = time.perf_counter()
        o.factor(wb.values[b])
        ts.append(time.perf_counter() - t0)
    per = sum(ts) / len(ts)
    ms_b = gpu("batched", "ms_batched")
    out["batched"] = {"oracle_numeric_s_per_member": round(per, 4), "members_timed": [0, 1, 63, 127],
                      "oracle_numeric_s_batch_model": round(per * 128, 2),
                      "timing": "one run per member after a warm-up; the batch as 128 x the mean",
                      "gpu_ms_batched": ms_b,
                      "gpu_speedup_vs_oracle": round(per * 128 * 1e3 / ms_b, 1) if ms_b else None}
    log(f"oracle batched: {out['batched']}")
    w = workloads.gmrf_grid2d(200, 200, 0.1, 0)
    out["supernodal"] = row("supernodal", w, 128, (ex.get("supernodal", {}).get("route") or {}).get(
        "ms_per_factorization"))[1]
    w = workloads.spatiotemporal_arrowhead()
    out["semisparse"] = row("semisparse", w, gpu("semisparse", "nb") or 128,
                            gpu("semisparse", "ms_per_factorization"), reps=0)[1]
    return out


# ---------------------------------------------------------------------------
# reduction of rocprofv3 CSV output into the tables under profiles/
# ---------------------------------------------------------------------------

def _short_kernel(name):
    """'void stc::k_upd<128, true, true>(stc::LevelArgs)' -> 'k_upd<128, true, true>'."""
    n = name.strip()
    if n.startswith("void "):
        n = n[5:]
    depth, cut = 0, len(n)
    for i, ch in enumerate(n):  # drop the argument list: the first '(' outside template brackets
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    n = n[:cut]
    return n[5:] if n.startswith("stc::") else n


def _csv_rows(root, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True)):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _segments(disp, marker):
    """Split dispatches (sorted by start) at each dispatch of the marker
    kernel; a factorization begins with one."""
    segs, cur = [], []
    for d in disp:
        if d["kernel"].startswith(marker) and cur:
            segs.append(cur)
            cur = []
        cur.append(d)
    if cur:
        segs.append(cur)
    return segs


def summarize_trace(args):
    """Markdown summary of a rocprofv3 --kernel-trace CSV directory, and of
    --pmc counter directories if given: per kernel launches, time, and
    (with counters) copy-calibrated HBM bytes and MFMA flops."""
    import statistics
    disp = []
    for r in _csv_rows(args.summarize_trace, "kernel_trace.csv"):
        disp.append({"kernel": _short_kernel(r["Kernel_Name"]), "start": int(r["Start_Timestamp"]),
                     "end": int(r["End_Timestamp"]), "id": int(r.get("Dispatch_Id", 0) or 0)})
    disp.sort(key=lambda d: d["start"])
    if not disp:
        print("no kernel_trace.csv under " + args.summarize_trace, file=sys.stderr)
        sys.exit(1)
    segs = _segments(disp, args.segment_marker)
    if args.segment is not None:
        disp = segs[args.segment]
    if args.kernel_filter:
        disp = [d for d in disp if any(d["kernel"].startswith(k) for k in args.kernel_filter.split(","))]
    t0 = min(d["start"] for d in disp)
    t1 = max(d["end"] for d in disp)
    busy, last = 0, t0  # union of kernel intervals
    for d in sorted(disp, key=lambda d: d["start"]):
        s, e = max(d["start"], last), d["end"]
        if e > s:
            busy += e - s
            last = e
    print(f"Segments delimited by {args.segment_marker}: {len(segs)}"
          + (f"; this table: segment {args.segment}" if args.segment is not None else "; this table: all"))
    print(f"Span {(t1 - t0) / 1e6:.2f} ms, of which {busy / 1e6:.2f} ms has at least one kernel running.\n")
    per = {}
    for d in disp:
        per.setdefault(d["kernel"], []).append((d["end"] - d["start"]) / 1e3)
    ids = {d["id"] for d in disp}
    cnt = {}
    for suffix in ("counter_collection.csv",):
        for cdir in args.counters or []:
            for r in _csv_rows(cdir, suffix):
                k = _short_kernel(r["Kernel_Name"])
                cnt.setdefault(r["Counter_Name"], []).append((k, int(r.get("Dispatch_Id", 0) or 0),
                                                             float(r["Counter_Value"])))
    scale = {}
    for c, vals in cnt.items():
        cal = [v for k, _, v in vals if "copy" in k.lower()]
        if c in ("FETCH_SIZE", "WRITE_SIZE") and cal:
            scale[c] = 1048576.0 / max(cal)  # KiB the counter reads for the plain 1 GiB copy
        if args.segment is not None:  # the same run of dispatches as the trace table
            vals.sort(key=lambda x: x[1])
            sg = _segments([{"kernel": k, "id": i, "v": v} for k, i, v in vals], args.segment_marker)
            cnt[c] = [(d["kernel"], d["id"], d["v"]) for d in sg[args.segment]] if args.segment < len(sg) else []
    cols = ["kernel", "launches", "total ms", "average us", "median us"]
    extra = [c for c in ("FETCH_SIZE", "WRITE_SIZE") if c in scale]
    if extra:
        cols += ["HBM MB", "HBM GB/s"]
    if "SQ_INSTS_VALU_MFMA_MOPS_F64" in cnt:
        cols += ["MFMA GFLOP executed"]
    print("| " + " | ".join(cols) + " |")
    print("|" + "---|" * len(cols))
    for k, ts in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        tot = sum(ts)
        row = [k, str(len(ts)), f"{tot / 1e3:.2f}", f"{tot / len(ts):.1f}", f"{statistics.median(ts):.1f}"]
        if extra:
            by = 0.0
            for c in extra:
                by += sum(v for kk, _, v in cnt[c] if kk == k) * 1024.0 * scale[c] / args.counter_runs
            row += [f"{by / 1e6:.1f}", f"{by / (tot * 1e-6) / 1e9:.0f}" if tot > 0 else "-"]  # tot: us
        if "SQ_INSTS_VALU_MFMA_MOPS_F64" in cnt:
            mops = sum(v for kk, _, v in cnt["SQ_INSTS_VALU_MFMA_MOPS_F64"] if kk == k) / args.counter_runs
            row += [f"{mops * 512 / 1e9:.2f}"]
        print("| " + " | ".join(row) + " |")
    if scale:
        print("\nCounter scale from the plain 1 GiB copy: " +
              ", ".join(f"{c} x {v:.3f}" for c, v in scale.items()))
    if args.traffic_json and extra:
        # HBM bytes per launch of each kernel in the selected dispatches, for
        # the bench's roofline entry (read only while the sources match)
        out = {"source_hash": kernel_source_hash(), "segment": args.segment,
               "scale": {c: round(v, 6) for c, v in scale.items()}, "kernels": {}}
        for k, ts in per.items():
            by = {c: sum(v for kk, _, v in cnt[c] if kk == k) * 1024.0 * scale[c] / args.counter_runs for c in extra}
            out["kernels"][k] = {"launches": len(ts), "fetch_bytes": by.get("FETCH_SIZE", 0.0),
                                 "write_bytes": by.get("WRITE_SIZE", 0.0),
                                 "bytes_per_launch": sum(by.values()) / len(ts)}
        with open(args.traffic_json, "w") as fh:
            json.dump(out, fh, indent=1)
    if args.chain:
        ch = [d for d in disp if d["kernel"].startswith(args.chain)]
        gaps = [(b["start"] - a["end"]) / 1e3 for a, b in zip(ch[:-1], ch[1:])]
        tot = sum((d["end"] - d["start"]) for d in ch) / 1e6
        if gaps:
            print(f"\nChain of {args.chain}: {len(ch)} launches, {tot:.2f} ms inside them; from the end of one to the "
                  f"start of the next: median {statistics.median(gaps):.1f} us, mean {statistics.mean(gaps):.1f} us; "
                  f"launch time plus these intervals: {tot + sum(gaps) / 1e3:.2f} ms of the span.")
    _ = ids


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=12288)
    ap.add_argument("--nb", type=int, default=256)
    ap.add_argument("--prof-reps", type=int, default=3)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--tune-slots", default="0,320,640",
                    help="wg_slots candidates the headline's schedule is tuned over (empty: no tuning)")
    ap.add_argument("--tune-folds", default="0,50",
                    help="fold weights (percent) of the second tuning round on the winning schedule (empty: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras-out", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--solve-pass", action="store_true",
                    help="factorize the semisparse config, then solve it 3 times with 1 and with 8 "
                         "right-hand sides (for a kernel trace), print one JSON line and exit")
    ap.add_argument("--batched-pass", type=int, default=None, metavar="HINT",
                    help="factorize the batched config (B=128) three times with the split-K schedule for a batch of "
                         "HINT value sets (0: for one), then a 1 GiB copy, for the counter runs; print one JSON line")
    ap.add_argument("--semisparse-pass", action="store_true",
                    help="only: one eager C3 factorization (kernel by kernel) and a 1 GiB copy, "
                         "for counter runs over the active-column route")
    ap.add_argument("--backward-pass", action="store_true",
                    help="only: the C3 factorization and its logdet reverse mode, twice through the graphs, "
                         "for kernel traces and counter runs over the reverse mode")
    ap.add_argument("--pass-align", type=int, default=512,
                    help="tile-grid alignment (columns, 0 = uniform grid) of --solve-pass, --semisparse-pass "
                         "and --backward-pass")
    ap.add_argument("--pass-nb", type=int, default=128,
                    help="tile size of --solve-pass, --semisparse-pass and --backward-pass")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration runs)")
    ap.add_argument("--summarize-trace", default=None, metavar="DIR",
                    help="print a markdown summary of the rocprofv3 kernel-trace CSVs under DIR and exit")
    ap.add_argument("--counters", action="append", metavar="DIR",
                    help="with --summarize-trace: rocprofv3 --pmc CSV directories (FETCH_SIZE, WRITE_SIZE, "
                         "SQ_INSTS_VALU_MFMA_MOPS_F64), calibrated by the plain copy's reading")
    ap.add_argument("--counter-runs", type=int, default=1,
                    help="with --counters: factorizations each counter run covers per traced one")
    ap.add_argument("--segment", type=int, default=None,
                    help="with --summarize-trace: only the i-th run of dispatches between two marker kernels")
    ap.add_argument("--segment-marker", default="k_value_gather")
    ap.add_argument("--kernel-filter", default=None, help="comma-separated kernel name prefixes to keep")
    ap.add_argument("--chain", default=None, help="kernel name prefix whose successive launches form a chain")
    ap.add_argument("--traffic-json", default=None, metavar="FILE",
                    help="with --counters: write the calibrated HBM bytes per launch of each kernel to FILE")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    if args.extras_out:
        run_extras(args.extras_out, args.batch)
        return
    if args.solve_pass:
        solve_pass(args.pass_align, args.pass_nb)
        return
    if args.batched_pass is not None:
        batched_pass(args.batched_pass)
        return
    if args.semisparse_pass:
        semisparse_pass(args.pass_align, args.pass_nb)
        return
    if args.backward_pass:
        backward_pass(args.pass_align, args.pass_nb)
        return

    import torch
    hl = headline(args)
    if args.copy_calibration:
        x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1.0)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    a, w, work = hl["a"], hl["w"], hl["work"]
    a.release()
    torch.cuda.empty_cache()

    extras = None
    if not args.no_extras:
        fd, path = tempfile.mkstemp(suffix=".json")
        os.close(fd)
        cmd = [sys.executable, os.path.abspath(__file__), "--extras-out", path, "--batch", str(args.batch)]
        rc = subprocess.run(cmd).returncode
        if rc != 0:
            print(f"extras child failed with status {rc}", file=sys.stderr)
            sys.exit(rc)
        with open(path) as fh:
            extras = json.load(fh)
        os.unlink(path)

    cpu = None if args.no_cpu_baseline else cpu_baseline(args)
    cpu_cfg = None if (args.no_cpu_baseline or args.no_extras) else cpu_baseline_configs(extras)

    ms_step = hl["ms_step"]
    line = {
        "metric": "FP64 factorizations/s + % FP64 MFMA peak; batched & backward vs plain path",
        "value": round(1000.0 / ms_step, 4),
        "unit": "factorizations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"dense-route random SPD n={args.n}, 20% off-diagonal density, "
                               f"tile {a.nb}, natural order (every tile dense)",
                   "n": args.n, "nb": a.nb, "nnz_lower": w.nnz, "route": a.route, "levels": a.nlevels,
                   "wg_slots": hl["wg_slots"]},
        "gflops_tile": round(work["flops_tile"] / (ms_step * 1e-3) / 1e9, 2),
        "frac_peak_whole_factorization": round(work["flops_tile"] / (ms_step * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4),
        "roofline": hl["roofline"],
        "level_kernels_tflops": hl["level_family_tflops"],
        "kernels": hl["kinds"],
        "measured_peaks_tflops": hl["peaks"],
        "cpu_baseline": cpu,
        "cpu_baseline_configs": cpu_cfg,
        "extras": extras,
        "logdet": hl["logdet"],
        "factor_uses": hl["uses"],
        "analyse_s": round(hl["analyse_s"], 3),
        "single_replays": hl["step_stats"],
        "autotune": hl["tune_table"],
    }
    if cpu:
        # factorizations after which the one-off analysis has paid for itself
        # against the oracle's factorization time
        saved = 1.0 / cpu["value"] - ms_step * 1e-3
        line["analyse_breakeven_factorizations"] = round(hl["analyse_s"] / saved, 4) if saved > 0 else None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
