"""Tile-size / storage-mode / tile-grid autotuner.

The paper fixes n_b per regime by hand (80 by default, 120 for structured
sparse problems on its CPU nodes; 512 and beyond on its GPU, Sec. 6.1 and
Sec. 6.7) and leaves the choice open.  Here the choice is measured: the
pattern is analysed at every candidate (n_b, storage mode), each candidate's
captured schedule is replayed on the caller's own values (one value set, or
the whole batch), and the fastest is kept.  The ordering is computed once, at
the first candidate, and handed to the others as a given permutation, so the
candidates differ only in their tiling and schedule.  Besides n_b the grid
itself is a candidate axis: uniform, or aligned to the elimination tree with
subtrees of at least a given multiple of n_b starting on tile boundaries.
"""
from . import stc


def autotune(n, colptr, rowind, values, nbs=(64, 128, 256), modes=("auto",), ordering="auto",
             batched=False, trials=3, warmup=1, objective="factorize", slots=(0,), aligns=(0,), folds=(0,)):
    """Return (best Analysis, bound; table of every candidate).

    values: device float64 [nnz] (batched=False) or [B, nnz] (batched=True).
    objective: "factorize" times one factorization call; "logdet_grad" times
    a factorization followed by the logdet reverse mode (the unit of work of
    a gradient-based fit).
    slots: candidate wg_slots of the schedule (0 = the library default).
    aligns: candidate tile grids as multiples of n_b (0 = the uniform grid;
    a > 0 aligns every subtree of at least a * n_b consecutive columns).
    folds: fold_pct values (the split-K cost model's weight of a fold, 0 =
    the library default) tried in a second round on the best candidate of
    the first.
    Each table row: nb, mode, wg_slots, align (columns), fold_pct, ms per
    call, levels, tile flops.
    Candidates that lose release their workspace.
    """
    import torch

    perm = None
    best = None
    table = []

    def trial(nb, mode, ws, al, fp):
        nonlocal perm, best
        kw = dict(nb=nb, mode=mode, wg_slots=ws, align=al * nb, fold_pct=fp,
                  batch=values.shape[0] if batched else 0)
        if perm is None:
            a = stc.Analysis(n, colptr, rowind, ordering=ordering, **kw)
            perm = a.perm()
        else:
            a = stc.Analysis(n, colptr, rowind, ordering="given", perm=perm, **kw)
        a.bind(batch=values.shape[0] if batched else 1)

        one = torch.ones(1, dtype=torch.float64, device=values.device)

        def run():
            if batched:
                a.factorize_batched(values)
            else:
                a.factorize(values)
                if objective == "logdet_grad":
                    a.logdet_backward(one)

        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(trials):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / trials
        table.append(dict(nb=a.nb, mode=a.mode, wg_slots=ws, align=al * nb, fold_pct=fp, ms=round(ms, 4),
                          levels=a.nlevels, tile_gflop=round(a.work()["flops_tile"] / 1e9, 3)))
        if best is None or ms < best[0]:
            if best is not None:
                best[1].release()
            best = (ms, a, (nb, mode, ws, al))
        else:
            a.release()

    for nb, mode, ws, al in ((nb, mode, ws, al) for nb in nbs for mode in modes for ws in slots for al in aligns):
        trial(nb, mode, ws, al, folds[0])
    nb, mode, ws, al = best[2]
    for fp in folds[1:]:
        trial(nb, mode, ws, al, fp)
    return best[1], table
