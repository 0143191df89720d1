"""Persistence of the analysis (stc_save / stc_load, Sec. 6.6: the analysis
is the one-off cost that repeated factorizations amortize).  A loaded handle
must match the saved one bit for bit in every host export -- permutation,
elimination tree, pattern of L, tiles, Algorithm 1's tasks, features, work
terms, schedule shape and both schedule checks -- and a damaged file must be
refused.  CPU only: nothing here touches a device."""
import os

import numpy as np
import pytest

from tests._build_once import ensure_built

ensure_built()

from paper_2609_29765_amd import stc as S  # noqa: E402
from paper_2609_29765_amd import workloads as W  # noqa: E402


def exports(a):
    t = a.tiles()
    lp, li = a.L_pattern()
    return {"sizes": (a.n, a.qnz, a.lnz, a.nb, a.NT, a.ntiles, a.nrows, a.ntasks, a.mode, a.route, a.ndense,
                      a.method, a.tact, a.store, a.nlevels, a.solve_launches),
            "features": (a.phi, a.rho, a.sigma), "perm": a.perm(), "etree": a.etree(), "lp": lp, "li": li,
            "positions": a.grid_positions(),
            **{f"tile_{k}": v for k, v in t.items()}, "tasks": a.tasks(), "work": a.work(),
            "plan": a.plan_stats(), "schedule": a.check_schedule(), "solve": a.check_solve_schedule(),
            "backward": a.check_backward()}


def same(x, y):
    assert x.keys() == y.keys()
    for k in x:
        if isinstance(x[k], np.ndarray):
            assert np.array_equal(x[k], y[k]), k
        else:
            assert x[k] == y[k], k


CASES = [
    ("random", lambda: W.random_spd(300, 0.03, 5, dense_rows=2), dict(nb=32, ordering="auto")),
    ("gmrf", lambda: W.gmrf_grid2d(32, 32, 0.1, 0), dict(nb=64, ordering="nd")),
    ("arrowhead", lambda: W.differentiable_arrowhead(20, 25, 8, 0), dict(nb=128, ordering="nd", wg_slots=4)),
    ("dense", lambda: W.dense_spd(700, 0.2, 0), dict(nb=256, ordering="natural", mode="dense")),
    ("aligned", lambda: W.differentiable_arrowhead(20, 25, 8, 0), dict(nb=128, ordering="nd", align=512)),
]


@pytest.mark.parametrize("name,make,opts", CASES, ids=[c[0] for c in CASES])
def test_save_load_round_trip(tmp_path, name, make, opts):
    w = make()
    a = S.Analysis(w.n, w.colptr, w.rowind, **opts)
    path = tmp_path / f"{name}.stc"
    a.save(path)
    b = S.Analysis.load(path)
    same(exports(a), exports(b))
    # saving the loaded handle writes the same bytes
    b.save(tmp_path / "again.stc")
    assert (tmp_path / "again.stc").read_bytes() == path.read_bytes()


def test_damaged_files_are_refused(tmp_path):
    w = W.random_spd(120, 0.05, 3)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=32, ordering="nd")
    good = tmp_path / "good.stc"
    a.save(good)
    data = good.read_bytes()
    cases = {"truncated": data[:-100], "empty": b"", "magic": b"X" + data[1:],
             "flipped": data[:len(data) // 2] + bytes([data[len(data) // 2] ^ 1]) + data[len(data) // 2 + 1:],
             "extended": data + b"\0"}
    for what, blob in cases.items():
        p = tmp_path / f"{what}.stc"
        p.write_bytes(blob)
        with pytest.raises(S.STCError) as e:
            S.Analysis.load(p)
        assert e.value.code == -1, what
    with pytest.raises(S.STCError):
        S.Analysis.load(tmp_path / "missing.stc")
    with pytest.raises(S.STCError):
        a.save(tmp_path / "no_such_dir" / "x.stc")
    assert os.path.exists(good)
