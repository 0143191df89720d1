"""GPU parity of the logdet reverse mode.  Its gradient is the selected
inverse on the pattern of L, one of the consumers of the resident factor the
paper lists (Sec. 6.7).  Checked here: library gradient values against the
oracle's selected inverse; the parameter gradient of the differentiable
arrowhead against the oracle's trace tr(Q^-1 dQ/dtheta) and against central
finite differences of the library's own logdet; the autograd wiring.

Tolerances: gradient values ||g - g_o||_inf <= 1e-10 ||g_o||_inf (the
selected inverse reuses the factor, whose entries agree to 1e-10 relative);
theta gradient rel 1e-8 against the oracle trace; central differences with
h = 1e-5 carry truncation error h^2 |f'''|/6 and rounding eps |logdet| / h,
both below 1e-8 relative here, so the same 1e-8 bound is used.
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


def grad_case(w, ordering, nb, mode, tol=1e-10):
    o = O.Analysis(w.n, w.colptr, w.rowind, ordering, nb=nb, mode=mode)
    Lo, info = o.factor(w.values)
    assert info == 0
    go = o.logdet_grad_values(Lo)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=nb, mode=mode, ordering=ordering).bind()
    print(f"[gpu] backward n={w.n} nb={nb} mode={a.mode} ordering={ordering}", flush=True)
    a.factorize(dev(w.values))
    g = a.logdet_backward(torch.ones(1, dtype=torch.float64, device="cuda")).cpu().numpy()
    err = np.max(np.abs(g - go))
    assert err <= tol * np.max(np.abs(go)), (err, np.max(np.abs(go)))
    return a, g, go


@pytest.mark.parametrize("seed", range(10))
def test_grad_values_random(seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(2, 400))
    w = W.random_spd(n, float(rng.choice([0.01, 0.05, 0.2])), seed, dense_rows=int(rng.integers(0, 4)))
    nb = int(rng.choice([32, 64, 128]))
    mode = ["dense", "semisparse"][seed % 2]
    ordering = ["natural", "rcm", "nd", "auto"][seed % 4]
    grad_case(w, ordering, nb, mode)


@pytest.mark.parametrize("nb", [32, 64, 128, 256])
def test_grad_values_tile_sizes_ragged(nb):
    w = W.random_spd(700, 0.03, 3, dense_rows=2)
    grad_case(w, "nd", nb, "semisparse")
    grad_case(w, "nd", nb, "dense")


def test_grad_values_one_by_one():
    w = W.random_spd(1, 0.0, 0)
    a, g, go = grad_case(w, "natural", 32, "auto")
    assert abs(g[0] - 1.0 / w.values[0]) <= 1e-15 / w.values[0]


def test_grad_gmrf_spectral():
    """Sum over the diagonal of the gradient is tr(Q^-1), known in closed form
    from the DCT spectrum of the 2-D Laplacian."""
    w = W.gmrf_grid2d(32, 32, 0.1, 0)
    a, g, go = grad_case(w, "nd", 64, "auto")
    diag = w.rowind == np.repeat(np.arange(w.n), np.diff(w.colptr))
    lam = 2 - 2 * np.cos(np.pi * np.arange(32) / 32)
    tr = (1.0 / (lam[:, None] + lam[None, :] + 0.1)).sum()
    assert abs(g[diag].sum() - tr) <= 1e-11 * tr


def _theta_grad(a, w):
    a.factorize(dev(w.values))
    gv = a.logdet_backward(torch.ones(1, dtype=torch.float64, device="cuda")).cpu().numpy()
    return w.dvalues @ gv


@pytest.mark.parametrize("T,m,nb", [(4, 6, 64), (20, 25, 64), (20, 25, 128)])
def test_theta_gradient_vs_trace_and_fd(T, m, nb):
    w = W.differentiable_arrowhead(T, m, 8, 0)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=nb, ordering="nd").bind()
    print(f"[gpu] theta gradient n={w.n}", flush=True)
    g = _theta_grad(a, w)
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=nb)
    Lo, _ = o.factor(w.values)
    gt = w.dvalues @ o.logdet_grad_values(Lo)
    assert np.all(np.abs(g - gt) <= 1e-8 * np.abs(gt)), (g, gt)
    th = w.meta["theta"]
    h = 1e-5
    fd = np.zeros(3)
    for i in range(3):
        ld = []
        for s in (+1, -1):
            t2 = th.copy()
            t2[i] += s * h
            w2 = W.differentiable_arrowhead(T, m, 8, 0, theta=t2)
            a.factorize(dev(w2.values))
            ld.append(float(a.logdet().item()))
        fd[i] = (ld[0] - ld[1]) / (2 * h)
    print(f"[gpu] theta grad {g} fd {fd} rel {np.abs(g - fd) / np.abs(fd)}", flush=True)
    assert np.all(np.abs(g - fd) <= 1e-8 * np.abs(fd)), (g, fd)


def test_autograd_logdet():
    w = W.differentiable_arrowhead(4, 6, 8, 1)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=32, ordering="nd").bind()
    v = dev(w.values).requires_grad_(True)
    ld = S.logdet(v, a)
    (2.5 * ld).backward()
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=32)
    Lo, _ = o.factor(w.values)
    go = 2.5 * o.logdet_grad_values(Lo)
    assert np.max(np.abs(v.grad.cpu().numpy() - go)) <= 1e-10 * np.max(np.abs(go))
    # theta chain rule through torch: dvalues as a dense Jacobian
    th = torch.tensor(w.meta["theta"], dtype=torch.float64, device="cuda", requires_grad=True)
    J = dev(w.dvalues)
    vals = dev(w.values) + (th - th.detach()) @ J  # values(theta) to first order
    S.logdet(vals, a).backward()
    gt = w.dvalues @ o.logdet_grad_values(Lo)
    assert np.all(np.abs(th.grad.cpu().numpy() - gt) <= 1e-8 * np.abs(gt))


def test_autograd_refactorizes_when_interleaved():
    """A factorization of other values between forward and backward does not
    change the gradient of the first."""
    w = W.random_spd(150, 0.05, 4)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=32, ordering="nd").bind()
    v = dev(w.values).requires_grad_(True)
    ld = S.logdet(v, a)
    a.factorize(dev(w.values * 3.0))
    ld.backward()
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=32)
    Lo, _ = o.factor(w.values)
    go = o.logdet_grad_values(Lo)
    assert np.max(np.abs(v.grad.cpu().numpy() - go)) <= 1e-10 * np.max(np.abs(go))


def test_gradcheck_tiny():
    w = W.random_spd(12, 0.3, 5)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=32, ordering="natural").bind()
    v = dev(w.values).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: S.logdet(x, a), (v,), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_backward_leaves_factor_and_repeats():
    w = W.random_spd(300, 0.02, 6)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=64, ordering="nd").bind()
    a.factorize(dev(w.values))
    L0 = a.factor()
    one = torch.ones(1, dtype=torch.float64, device="cuda")
    g1 = a.logdet_backward(one).cpu().numpy()
    g2 = a.logdet_backward(one).cpu().numpy()
    assert np.array_equal(g1, g2)
    assert np.array_equal(a.factor(), L0)


@pytest.mark.parametrize("nb,align", [(128, 512), (64, 256)])
def test_split_reverse_levels_reproducible_and_match_oracle(nb, align):
    """The differentiable arrowhead's reverse-mode levels hold tasks with many
    terms, which the plan splits over several work-groups and folds after the
    level in a fixed order: gradients equal the oracle's to 1e-10 and are bit
    for bit the same on every call, with refactorizations between calls."""
    w = W.differentiable_arrowhead(20, 25, 8, 0)
    o = O.Analysis(w.n, w.colptr, w.rowind, "nd", nb=nb)
    Lo, info = o.factor(w.values)
    assert info == 0
    go = o.logdet_grad_values(Lo)
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=nb, ordering="nd", align=align).bind()
    v = dev(w.values)
    one = torch.ones(1, dtype=torch.float64, device="cuda")
    print(f"[gpu] split reverse nb={nb} align={align} levels={a.work()['levels_backward']}", flush=True)
    gs = []
    for _ in range(3):
        a.factorize(v)
        gs.append(a.logdet_backward(one).cpu().numpy())
    assert np.max(np.abs(gs[0] - go)) <= 1e-10 * np.max(np.abs(go))
    assert np.array_equal(gs[0], gs[1]) and np.array_equal(gs[0], gs[2])


def test_full_size_arrowhead_reverse_mode_trace_identity_and_solve_columns():
    """The spatio-temporal arrowhead at full size (n = 101,258, tile 128, grid
    aligned at 512 columns), whose reverse-mode levels are split most: (1) the
    derivative of logdet along Q itself is tr(Q^-1 Q) = n, so the gradient
    dotted with the values is n at any size; (2) on sampled columns j (the
    border rows among them) the gradient entries of column j equal, up to the
    factor 2 off the diagonal, the entries of Q^-1 e_j from the library's
    solve, a separate path (triangular sweeps) checked against the oracle
    elsewhere.  Tolerances: both sides carry rounding of order cond(Q) eps
    (cond about 1e4 here); 1e-9 relative leaves a wide margin."""
    w = W.spatiotemporal_arrowhead()
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=128, ordering="nd", align=512).bind()
    print(f"[gpu] full-size reverse n={w.n} levels={a.work()['levels_backward']}", flush=True)
    a.factorize(dev(w.values))
    assert a.info() == 0
    g = a.logdet_backward(torch.ones(1, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert abs(float(g @ w.values) - w.n) <= 1e-9 * w.n
    rng = np.random.default_rng(3)
    cols = [0, w.n // 2, w.n - 9, w.n - 8, w.n - 1] + [int(c) for c in rng.integers(0, w.n, 5)]
    E = torch.zeros(w.n, len(cols), dtype=torch.float64, device="cuda")
    for k, j in enumerate(cols):
        E[j, k] = 1.0
    X = a.solve(E).cpu().numpy()
    for k, j in enumerate(cols):
        lo, hi = w.colptr[j], w.colptr[j + 1]
        rows = w.rowind[lo:hi]
        want = np.where(rows == j, 1.0, 2.0) * X[rows, k]
        err = np.max(np.abs(g[lo:hi] - want))
        assert err <= 1e-9 * np.max(np.abs(want)), (j, err)


def test_backward_after_failed_factorization_is_nan():
    w = W.random_spd(100, 0.05, 7)
    vals = w.values.copy()
    vals[w.colptr[10]] = -3.0
    a = S.Analysis(w.n, w.colptr, w.rowind, nb=32, ordering="nd").bind()
    a.factorize(dev(vals))
    assert a.info() > 0
    g = a.logdet_backward(torch.ones(1, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert np.all(np.isnan(g))
