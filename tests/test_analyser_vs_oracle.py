"""The product's host analyser (libstc.so) against the oracle: every symbolic
output -- permutation, elimination tree, pattern of L, tiles and their active
rows, kd, features, route, Algorithm 1's task list -- must agree bit for bit.
CPU only: these entry points make no HIP call."""
import re
import os

import numpy as np
import pytest

from tests._build_once import ensure_built, ROOT

ensure_built()

from oracle import oracle as O  # noqa: E402
from paper_2609_29765_amd import stc as S  # noqa: E402
from paper_2609_29765_amd import workloads as W  # noqa: E402


def _compare(w, ordering, nb, mode="auto", align=0):
    o = O.Analysis(w.n, w.colptr, w.rowind, ordering, nb=nb, mode=mode, align=align)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=nb, mode=mode, ordering=ordering, align=align)
    assert np.array_equal(a.grid_positions(), o.positions())
    assert (a.lnz, a.NT, a.ntiles, a.nrows, a.ntasks, a.ndense, a.method, a.tact) == \
           (o.lnz, o.NT, o.ntiles, o.nrows, o.ntasks, o.ndense, o.method, o.tact)
    assert (a.mode, a.route) == (o.mode, o.route)
    assert (a.phi, a.rho, a.sigma) == (o.phi, o.rho, o.sigma)
    assert np.array_equal(a.perm(), o.perm())
    assert np.array_equal(a.etree(), o.etree())
    lpa, lia = a.L_pattern()
    lpo, lio = o.L_pattern()
    assert np.array_equal(lpa, lpo) and np.array_equal(lia, lio)
    ta, to = a.tiles(), o.tiles()
    for key in ("m", "k", "cnt", "true_cnt", "contig", "roff", "rows", "kd"):
        assert np.array_equal(ta[key], getattr(to, key)), key
    assert np.array_equal(a.tasks(), o.tasks())
    return a, o


@pytest.mark.parametrize("seed", range(40))
def test_random_patterns(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 90))
    dens = float(rng.choice([0.02, 0.05, 0.1, 0.3]))
    w = W.random_spd(n, dens, seed, dense_rows=int(rng.integers(0, 3)))
    ordering = ["natural", "rcm", "nd", "auto"][seed % 4]
    nb = int(rng.choice([32, 64]))
    mode = ["auto", "dense", "semisparse"][seed % 3]
    _compare(w, ordering, nb, mode)


@pytest.mark.parametrize("ordering", ["natural", "rcm", "nd", "auto"])
def test_gmrf32(ordering):
    w = W.gmrf_grid2d(32, 32)
    _compare(w, ordering, 64)


def test_lap3d_small_and_bordered():
    _compare(W.batched_laplacian3d(m=10, B=2), "nd", 64)
    _compare(W.spatiotemporal_arrowhead(T=6, m=12, nborder=8), "nd", 32)
    _compare(W.spatiotemporal_arrowhead(T=6, m=12, nborder=8), "auto", 64)


def test_differentiable_arrowhead_full_size():
    a, o = _compare(W.differentiable_arrowhead(20, 25, 8, 0), "nd", 64)
    assert a.route == "semisparse"


@pytest.mark.parametrize("nb", [128, 256])
def test_spatiotemporal_full_size(nb):
    """The spatio-temporal arrowhead at its full size (n 101,258) with the
    ND ordering the bench uses, at both tile sizes the autotuner tries."""
    a, o = _compare(W.spatiotemporal_arrowhead(), "nd", nb)
    assert a.route == "semisparse" and a.ndense == 8


@pytest.mark.parametrize("nb", [64, 128])
def test_lap3d_full_size(nb):
    """The 24^3 Laplacian of the batched workload (one value set: the
    pattern is shared by every member)."""
    a, o = _compare(W.batched_laplacian3d(m=24, B=1), "nd", nb)
    assert a.route == "semisparse"


def test_dense_route_small():
    w = W.dense_spd(512, 0.2, 0)
    a, o = _compare(w, "natural", 64)
    assert a.route == "dense" and a.mode == "dense"
    assert np.array_equal(a.perm(), np.arange(512))  # every row is set aside as dense


def test_pattern_errors_match():
    bad = [(2, [0, 2, 3], [1, 0, 1]), (2, [0, 2, 2], [0, 1]), (3, [0, 3, 4, 5], [0, 2, 2, 1, 2])]
    for n, cp, ri in bad:
        cp = np.array(cp, np.int64)
        ri = np.array(ri, np.int32)
        assert O.check_pattern(n, cp, ri) != 0
        with pytest.raises(S.STCError) as e:
            S.Analysis(n, cp, ri)
        assert e.value.code == -2


def test_bad_options():
    w = W.random_spd(10, 0.2, 0)
    with pytest.raises(S.STCError):
        S.Analysis(w.n, w.colptr, w.rowind, nb=48)
    with pytest.raises(S.STCError):
        S.Analysis(w.n, w.colptr, w.rowind, ordering="given", perm=np.zeros(10, np.int32))


def test_abi_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "stc.h")).read()
    declared = set(re.findall(r"\b(stc_[A-Za-z0-9_]+)\s*\(", hdr))
    lib = S.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(S.EXPORTS)


def test_empty_and_malformed_inputs_rejected():
    # n = 0 and n < 0 are argument errors; a column with no entry (no
    # diagonal) and an upper-triangle entry are pattern errors
    for n, cp, ri, code in [(0, [0], [], -1), (-1, [0], [], -1), (1, [0, 0], [], -2),
                            (2, [0, 1, 3], [0, 1, 0], -2)]:
        with pytest.raises(S.STCError) as e:
            S.Analysis(n, np.array(cp, np.int64), np.array(ri, np.int32))
        assert e.value.code == code


def test_no_device_fails_loudly():
    # the product path has no CPU fallback: without a HIP device binding and
    # factorizing raise instead of computing anything on the host
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a HIP device is visible")
    w = W.random_spd(50, 0.1, 0)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=32)
    with pytest.raises(RuntimeError, match="HIP device"):
        a.bind()
    with pytest.raises(RuntimeError, match="HIP device"):
        a.factorize(torch.from_numpy(w.values))
