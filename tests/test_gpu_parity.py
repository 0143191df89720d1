"""GPU parity: the HIP path (libstc.so through its C ABI) against the oracle on
the same seeded inputs.

Tolerances (both sides in FP64, summing in different orders, so they agree to
rounding amplified by each column's conditioning): factor entries per column
||dL_:j||_inf <= 1e-10 ||L_:j||_inf on the identical pattern; logdet
|d| <= 1e-12 * max(|ld|, sum |2 log L_ii|); solve relative 1e-10 of the
oracle's solution; pivot failures bit-exact (same first failing column).
"""
import numpy as np
import pytest

from tests._build_once import ensure_built

ensure_built()

from oracle import oracle as O  # noqa: E402
from paper_2609_29765_amd import stc as S  # noqa: E402
from paper_2609_29765_amd import workloads as W  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def factor_close(L, Lref, lp, tol=1e-10):
    n = len(lp) - 1
    col = np.repeat(np.arange(n), np.diff(lp))
    scale = np.zeros(n)
    np.maximum.at(scale, col, np.abs(Lref))
    err = np.zeros(n)
    np.maximum.at(err, col, np.abs(L - Lref))
    bad = err > tol * scale
    assert not bad.any(), f"{bad.sum()} columns off, worst {np.max(err / np.maximum(scale, 1e-300))}"


def logdet_close(ld, ld_ref, Lref_diag=None, tol=1e-12):
    scale = abs(ld_ref)
    if Lref_diag is not None:
        scale = max(scale, np.sum(np.abs(2 * np.log(Lref_diag))))
    assert abs(ld - ld_ref) <= tol * scale, (ld, ld_ref)


def run_case(w, ordering, nb, mode, values=None, check_solve=True):
    values = w.values if values is None else values
    o = O.Analysis(w.n, w.colptr, w.rowind, ordering, nb=nb, mode=mode)
    Lo, info_o = o.factor(values)
    assert info_o == 0
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=nb, mode=mode, ordering=ordering).bind()
    print(f"[gpu] factorize n={w.n} nb={nb} mode={a.mode} ordering={ordering}", flush=True)
    a.factorize(dev(values))
    assert a.info() == 0
    L = a.factor()
    lp, _ = o.L_pattern()
    factor_close(L, Lo, lp)
    ld = float(a.logdet().item())
    logdet_close(ld, o.logdet(Lo), Lo[lp[:-1]])
    if check_solve and w.b is not None:
        x = a.solve(dev(w.b)).cpu().numpy()
        xo = o.solve(Lo, w.b)
        assert np.max(np.abs(x - xo)) <= 1e-10 * np.max(np.abs(xo))
    return a, o, L, Lo


@pytest.mark.parametrize("seed", range(12))
def test_random_small(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(3, 300))
    w = W.random_spd(n, float(rng.choice([0.01, 0.05, 0.2])), seed, dense_rows=int(rng.integers(0, 4)))
    nb = int(rng.choice([32, 64]))
    mode = ["dense", "semisparse"][seed % 2]
    ordering = ["natural", "rcm", "nd", "auto"][seed % 4]
    run_case(w, ordering, nb, mode)


def test_gmrf32_config():
    w = W.gmrf_grid2d(32, 32, 0.1, 0)
    a, o, L, Lo = run_case(w, "nd", 64, "auto")
    assert a.mode == "semisparse"
    lam = 2 - 2 * np.cos(np.pi * np.arange(32) / 32)
    closed = np.log(lam[:, None] + lam[None, :] + 0.1).sum()
    assert abs(float(a.logdet().item()) - closed) <= 1e-12 * abs(closed)


@pytest.mark.parametrize("nb", [32, 64, 128, 256])
def test_tile_sizes_ragged(nb):
    # n is not a multiple of nb: the last diagonal tile is padded
    w = W.random_spd(700, 0.03, 3, dense_rows=2)
    run_case(w, "nd", nb, "semisparse")
    run_case(w, "nd", nb, "dense", check_solve=False)


def test_route_equivalence():
    """With the ordering held fixed the dense and active-column routes produce
    the same factor entry by entry (Sec. 6.1)."""
    w = W.spatiotemporal_arrowhead(T=5, m=10, nborder=8)
    _, _, Ld, Lo = run_case(w, "nd", 64, "dense")
    _, _, Ls, _ = run_case(w, "nd", 64, "semisparse")
    assert np.max(np.abs(Ld - Ls)) <= 1e-12 * np.max(np.abs(Lo))


def test_dense_route_medium():
    w = W.dense_spd(1536, 0.2, 0)
    a, *_ = run_case(w, "natural", 256, "auto")
    assert a.mode == "dense"


def test_not_spd_reports_first_pivot():
    w = W.random_spd(200, 0.05, 9)
    vals = w.values.copy()
    diag = w.rowind == np.repeat(np.arange(w.n), np.diff(w.colptr))
    idx = np.nonzero(diag)[0][137]
    vals[idx] = -5.0
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=32, mode="semisparse")
    _, info_o = o.factor(vals)
    assert info_o > 0
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=32, mode="semisparse", ordering="nd").bind()
    a.factorize(dev(vals))
    assert a.info() == info_o
    assert np.isnan(float(a.logdet().item()))
    # the next good factorization clears the status
    a.factorize(dev(w.values))
    assert a.info() == 0


def test_batched_members_match_single_and_oracle():
    w = W.batched_laplacian3d(m=8, B=6, seed=0)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd").bind(batch=6)
    print(f"[gpu] batched n={w.n} B=6", flush=True)
    ld, info = a.factorize_batched(dev(w.values))
    ld = ld.cpu().numpy()
    assert np.all(info.cpu().numpy() == 0)
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=64)
    lam = 2 - 2 * np.cos(np.pi * np.arange(8) / 8)
    s3 = lam[:, None, None] + lam[None, :, None] + lam[None, None, :]
    for b in range(6):
        Lo, _ = o.factor(w.values[b])
        logdet_close(ld[b], o.logdet(Lo), Lo[o.L_pattern()[0][:-1]])
        wb, sb = w.meta["hyper"][b]
        closed = np.log(wb * s3 + 0.05 * sb).sum()
        assert abs(ld[b] - closed) <= 1e-12 * abs(closed)
        a.factorize(dev(w.values[b]))
        assert float(a.logdet().item()) == ld[b]


def test_batched_member_failure_is_isolated():
    w = W.batched_laplacian3d(m=6, B=4, seed=1)
    vals = w.values.copy()
    vals[2, 0] = -1.0  # first diagonal entry of member 2
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=32, ordering="nd").bind(batch=4)
    ld, info = a.factorize_batched(dev(vals))
    info = info.cpu().numpy()
    ld = ld.cpu().numpy()
    assert info[2] > 0 and np.isnan(ld[2])
    assert np.all(info[[0, 1, 3]] == 0) and np.all(np.isfinite(ld[[0, 1, 3]]))


def test_graph_replays_agree():
    w = W.differentiable_arrowhead(8, 10, 8, 0)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd").bind()
    v = dev(w.values)
    lds = []
    for _ in range(4):
        a.factorize(v)
        lds.append(float(a.logdet().item()))
        torch.cuda.synchronize()
    assert len(set(lds)) == 1


def test_differentiable_arrowhead_full_size():
    w = W.differentiable_arrowhead(20, 25, 8, 0)
    run_case(w, "nd", 64, "auto")


@pytest.mark.parametrize("nb,mode,nrhs", [(32, "semisparse", 2), (64, "semisparse", 8), (64, "dense", 11),
                                          (128, "semisparse", 17), (256, "dense", 64)])
def test_solve_many_right_hand_sides(nb, mode, nrhs):
    # groups of 8 columns with a ragged last group, the 64-column maximum,
    # ragged last tile; every column against the oracle's solve
    rng = np.random.default_rng(700 + nrhs)
    w = W.random_spd(nb * 3 + 19, 0.05, nrhs, dense_rows=2)
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=nb, mode=mode)
    Lo, info_o = o.factor(w.values)
    assert info_o == 0
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=nb, mode=mode, ordering="nd").bind()
    print(f"[gpu] solve n={w.n} nb={nb} mode={a.mode} nrhs={nrhs}", flush=True)
    a.factorize(dev(w.values))
    assert a.info() == 0
    B = rng.standard_normal((w.n, nrhs))
    X = a.solve(dev(B)).cpu().numpy()
    Xo = o.solve(Lo, B)
    for c in range(nrhs):
        assert np.max(np.abs(X[:, c] - Xo[:, c])) <= 1e-10 * np.max(np.abs(Xo[:, c])), c
    # a second call with fewer columns reuses the handle's graphs and scratch
    x1 = a.solve(dev(B[:, 0].copy())).cpu().numpy()
    assert np.array_equal(x1, X[:, 0])


def test_solve_mixed_fused_and_split_levels():
    # n_b 256 on a sparse grid: levels whose step items read few stored rows
    # apply their tiles inside the step item (in 64-row chunks), the others
    # get a launch of chunks and then one of diagonal solves
    w = W.gmrf_grid2d(60, 60)
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=256, mode="semisparse")
    Lo, info_o = o.factor(w.values)
    assert info_o == 0
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=256, mode="semisparse", ordering="nd").bind()
    sv = a.check_solve_schedule()
    assert sv["fused_launches"] > 0 and sv["launches"] > 2 * a.NT
    print(f"[gpu] solve n={w.n} nb=256 semisparse, {sv['launches']} launches", flush=True)
    a.factorize(dev(w.values))
    assert a.info() == 0
    B = np.random.default_rng(5).standard_normal((w.n, 8))
    X = a.solve(dev(B)).cpu().numpy()
    Xo = o.solve(Lo, B)
    for c in range(8):
        assert np.max(np.abs(X[:, c] - Xo[:, c])) <= 1e-10 * np.max(np.abs(Xo[:, c])), c
    x1 = a.solve(dev(B[:, 3].copy())).cpu().numpy()
    assert np.array_equal(x1, X[:, 3])


def test_solve_rejects_bad_column_counts():
    w = W.random_spd(100, 0.05, 3)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=32, ordering="nd").bind()
    a.factorize(dev(w.values))
    for nrhs in (65, 0):
        with pytest.raises(S.STCError):
            a.solve(torch.zeros(w.n, nrhs, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("n,nb,mode", [(1, 32, "auto"), (2, 32, "dense"), (20, 64, "semisparse"),
                                       (128, 128, "dense"), (129, 128, "semisparse"), (256, 256, "dense")])
def test_degenerate_sizes(n, nb, mode):
    # one scalar, fewer rows than a tile, exactly one tile, one row past a tile
    w = W.random_spd(n, 0.3, n)
    run_case(w, "natural" if n < 3 else "nd", nb, mode)


def test_diagonal_solve_and_batch_of_one():
    # no off-diagonal tile: the sweeps hold diagonal kernels only
    n = 300
    d = np.random.default_rng(4).uniform(0.5, 2.0, n)
    colptr = np.arange(n + 1, dtype=np.int64)
    rowind = np.arange(n, dtype=np.int32)
    a = S.Analysis(n, colptr, rowind, nb=64, ordering="natural").bind(batch=2)
    a.factorize(dev(d))
    b = np.random.default_rng(5).standard_normal((n, 3))
    x = a.solve(dev(b)).cpu().numpy()
    assert np.max(np.abs(x - b / d[:, None])) <= 1e-14 * np.max(np.abs(b / d[:, None]))
    ld, info = a.factorize_batched(dev(d[None, :].copy()))
    assert int(info.cpu()[0]) == 0
    assert abs(float(ld.cpu()[0]) - np.log(d).sum()) <= 1e-12 * abs(np.log(d).sum())


@pytest.mark.parametrize("seed", range(8))
def test_random_large_tiles_semisparse(seed):
    # tiles of 128 and 256 on random sparse patterns: the update kernels skip
    # 16-row groups a contribution leaves empty, so partly filled groups in
    # many shapes must still give the oracle's factor
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(300, 900))
    w = W.random_spd(n, float(rng.choice([0.005, 0.02, 0.06])), 40 + seed, dense_rows=int(rng.integers(0, 5)))
    nb = [128, 256][seed % 2]
    run_case(w, ["nd", "rcm"][seed // 2 % 2], nb, "semisparse")


def test_solve_leaves_its_input_alone():
    """The binding solves a column-major copy: b keeps its values for 1-D b,
    one-column and many-column b, and for batched right-hand sides."""
    w = W.gmrf_grid2d(16, 16, 0.1, 0)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd").bind()
    a.factorize(dev(w.values))
    for shape in ((w.n,), (w.n, 1), (w.n, 3)):
        b = torch.randn(*shape, dtype=torch.float64, device="cuda")
        keep = b.clone()
        x = a.solve(b)
        assert torch.equal(b, keep) and not torch.equal(x, b)
    ab = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd").bind(batch=2)
    ab.factorize_batched(dev(np.stack([w.values, 2 * w.values])))
    for shape in ((2, w.n), (2, w.n, 1)):
        b = torch.randn(*shape, dtype=torch.float64, device="cuda")
        keep = b.clone()
        ab.solve_batched(b)
        assert torch.equal(b, keep)
