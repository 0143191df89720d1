"""Benchmark: FP64 tile-Cholesky factorizations per second on one MI355X.

Workload: the dense-route matrix -- random SPD of order 12288 with ~20%
off-diagonal density (uniform pattern, N(0,1) entries, diagonal = row
absolute sum + 1), tile 256, every tile dense.  One step = value load +
the whole POTRF/SYRK/GEMM/TRSM tile schedule (one HIP-graph replay), values
already resident in HBM.

Prints one JSON line.  Besides the headline value it carries:
  roofline      the update kernel (SYRK+GEMM contributions on FP64 MFMA),
                algorithmic flops / event-timed kernel time against the FP64
                matrix peak of 78.6 TFLOP/s;
  cpu_baseline  the oracle (plain serial C, one core) timed on a smaller
                instance of the same generator, scaled to this order by the
                flop ratio.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=12288)
    ap.add_argument("--nb", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=4096)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2609_29765_amd import stc, workloads

    if not os.path.exists(stc.LIB_PATH):
        from paper_2609_29765_amd import build as pb
        pb.build()
    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)

    t0 = time.time()
    w = workloads.dense_spd(args.n, 0.2, 0)
    t_gen = time.time() - t0
    t0 = time.time()
    a = stc.Analysis(w.n, w.colptr, w.rowind, nb=args.nb, mode="auto", ordering="natural")
    t_analyse = time.time() - t0
    a.bind()
    work = a.work()
    vals = torch.from_numpy(w.values).cuda()
    print(f"[bench] n={w.n} nnz={w.nnz} nb={a.nb} mode={a.mode} route={a.route} "
          f"levels={a.nlevels} analyse={t_analyse:.2f}s gen={t_gen:.2f}s", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        a.factorize(vals)
    torch.cuda.synchronize()
    assert a.info() == 0, "warm-up factorization failed"
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        a.factorize(vals)
    stop.record()
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(stop)
    ms_step = ms_total / args.steps
    ld = float(a.logdet().item())
    info = a.info()
    print(f"[bench] {args.steps} steps {ms_step:.3f} ms/step logdet={ld:.6f} info={info}",
          file=sys.stderr, flush=True)

    # per-kernel-kind event timing of one eager factorization (same kernels)
    prof = a.profile_factorize(vals)
    upd_ms, upd_launches = prof["update"]
    achieved = work["flops_update"] / (upd_ms * 1e-3) / 1e12
    roofline = {
        "bound": "mfma",
        "achieved": round(achieved, 3),
        "peak": PEAK_FP64_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
        "traffic": None,
        "kernel": f"k_update<{a.nb}>",
        "launches": upd_launches,
        "avg_launch_ms": round(upd_ms / max(upd_launches, 1), 4),
        "flops_per_launch": work["flops_update"] / max(upd_launches, 1),
    }
    kinds = {k: {"ms": round(v[0], 3), "launches": v[1]} for k, v in prof.items()}

    # measured ceilings: MFMA issue microkernel, library DGEMM (rocBLAS via torch)
    mfma_peak = stc.fp64_mfma_peak()
    nd = 8192
    xa = torch.randn(nd, nd, dtype=torch.float64, device="cuda")
    xb = torch.randn(nd, nd, dtype=torch.float64, device="cuda")
    torch.matmul(xa, xb)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        torch.matmul(xa, xb)
    e1.record()
    torch.cuda.synchronize()
    dgemm_tf = 3 * 2.0 * nd ** 3 / (e0.elapsed_time(e1) * 1e-3) / 1e12
    del xa, xb
    print(f"[bench] measured FP64 MFMA issue {mfma_peak:.1f} TFLOP/s, library DGEMM n={nd} "
          f"{dgemm_tf:.1f} TFLOP/s", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle
        ns = args.cpu_sample_n
        ws = workloads.dense_spd(ns, 0.2, 0)
        o = oracle.Analysis(ws.n, ws.colptr, ws.rowind, "natural", nb=args.nb)
        t0 = time.time()
        Lx, oinfo = o.factor(ws.values)
        t_cpu = time.time() - t0
        assert oinfo == 0
        scale = (args.n / ns) ** 3
        cpu = {
            "value": round(1.0 / (t_cpu * scale), 6),
            "unit": "factorizations/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"oracle factor of the same generator at n={ns} (seed 0) took {t_cpu:.2f} s; "
                      f"scaled by (n/{ns})^3 = {scale:.1f} to n={args.n}",
        }

    gflops = work["flops_tile"] / (ms_step * 1e-3) / 1e9
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
                               f"tile {a.nb}, natural order (every row dense)",
                   "n": args.n, "nb": a.nb, "nnz_lower": w.nnz, "route": a.route},
        "gflops_tile": round(gflops, 2),
        "frac_peak_whole_factorization": round(gflops / 1e3 / PEAK_FP64_TFLOPS, 4),
        "kernels": kinds,
        "measured_peaks_tflops": {"mfma_issue": round(mfma_peak, 2), "dgemm_library_8192": round(dgemm_tf, 2)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "logdet": ld,
        "analyse_s": round(t_analyse, 3),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
