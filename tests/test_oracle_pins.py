"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formulas: each compares the oracle's
time stepping, filter or outer iteration with an independent statement of the
same thing (a closed form, a defining relation, a printed value, a direct
sparse solve, brute force), so that a dropped term, a wrong sign or index or a
transposed operand in the oracle fails at least one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import core as oc
import workloads as wl


def _mode(grid, ks):
    xs = oc.coords(grid)
    m = np.ones(grid.shape)
    for x, k in zip(xs, ks):
        m = m * np.sin(k * math.pi * x)
    return m


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------------------
# printed values (golden fixtures)
# ---------------------------------------------------------------------------
def test_b_mu_matches_listed_values(golden):
    for mu, num, den in golden("b_mu_listed.txt"):
        assert oc.b_mu(int(mu)) == pytest.approx(float(Fraction(int(num), int(den))), rel=1e-15)
        assert cf.B_MU_LISTED[int(mu)] == Fraction(int(num), int(den))


def test_pi_b_roots_match_quoted_values(golden):
    for p, val in golden("pi_b_roots.txt"):
        p = int(p)
        got = (math.pi * oc.b_mu(p // 2)) ** (1.0 / p)
        assert abs(got - float(val)) <= 0.005 + 1e-12


def test_ppw_table(golden):
    for row in golden("ppw_table.txt"):
        eps, nl = float(row[0]), float(row[1])
        for p, printed in zip((2, 4, 6, 8), row[2:]):
            val = 2 * math.pi * (math.pi * oc.b_mu(p // 2)) ** (1.0 / p) * (nl / eps) ** (1.0 / p)
            assert abs(val - float(printed)) <= 0.5 + 1e-9, (eps, nl, p, val, printed)


def test_stability_constants_bound_the_oracle_leapfrog(golden):
    """Run the oracle's leapfrog with dt at 0.98 and 1.02 times the stated limit:
    the first stays bounded, the second blows up (von Neumann limit)."""
    for p, cval in golden("stability_constants.txt"):
        p, cval = int(p), float(cval)
        grid = oc.Grid(2, (40, 40), p)
        v = wl.random_field(grid.shape, seed=11)
        root = math.sqrt(sum(1.0 / h ** 2 for h in grid.h))
        growth = {}
        for frac in (0.98, 1.02):
            dt = frac * cval / root
            tp = dict(nt=200, periods=1, dt=dt, omega_e=2 * math.pi / (200 * dt), alpha=0.5)
            _, wfin = oc.apply(grid, 1.0, None, v, tp, with_forcing=False, return_final=True)
            growth[frac] = np.abs(wfin).max() / np.abs(v).max()
        assert growth[0.98] < 10.0
        assert growth[1.02] > 1e6


# ---------------------------------------------------------------------------
# operator: sine modes, polynomials
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("dim,n", [(2, (20, 13)), (3, (9, 12, 7))])
def test_laplacian_on_sine_modes(order, dim, n):
    grid = oc.Grid(dim, n, order)
    ks = [1, 3, 5][:dim]
    mode = _mode(grid, ks)
    lap = oc.laplacian(grid, 1.0, mode)
    lam2 = sum(cf.lambda_h_sq_1d(k * math.pi, 1.0 / nn, order) for k, nn in zip(ks, n))
    inner = oc.interior_mask(grid)
    np.testing.assert_allclose(lap[inner], -lam2 * mode[inner], rtol=0, atol=1e-10 * lam2)


@pytest.mark.parametrize("order", [2, 4])
def test_laplacian_exact_on_polynomials(order):
    """Away from the walls the order-p operator differentiates polynomials of
    degree <= p+1 exactly."""
    grid = oc.Grid(2, (30, 30), order)
    x, y = oc.coords(grid)
    r = order // 2
    d2 = lambda k, t: k * (k - 1) * t ** (k - 2) if k >= 2 else np.zeros_like(t)
    for deg in range(order + 2):
        b = max(deg - 1, 0)
        u = x ** deg + 0.5 * y ** b
        exact = d2(deg, x) + 0.5 * d2(b, y)
        lap = oc.laplacian(grid, 1.0, u)
        sl = (slice(r, -r), slice(r, -r))
        np.testing.assert_allclose(lap[sl], exact[sl], atol=1e-7)


def test_laplacian_variable_c2_is_nondivergence_form():
    grid = oc.Grid(2, (17, 23), 4)
    c2 = 1.0 + wl.random_field(grid.shape, seed=3, zero_walls=False) ** 2
    u = wl.random_field(grid.shape, seed=4)
    lap1 = oc.laplacian(grid, 1.0, u)
    lapc = oc.laplacian(grid, c2, u)
    inner = oc.interior_mask(grid)
    np.testing.assert_allclose(lapc[inner], c2[inner] * lap1[inner], rtol=1e-14)


# ---------------------------------------------------------------------------
# time parameters: defining relations (Appendix A.1, eq. alphad, Sec. 3.2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim,n,order,omega,c2", [
    (2, 128, 2, 10.3, 1.0), (2, 2048, 4, 200.0, 2.0), (3, 512, 2, 80.0, 2.25),
    (3, 512, 4, 80.0, 2.25), (2, 64, 4, 3.7, 0.5), (2, 4, 2, 1.0, 1.0)])
def test_time_params_defining_relations(dim, n, order, omega, c2):
    grid = oc.Grid(dim, (n,) * dim, order)
    tp = oc.time_params(grid, c2, omega)
    dt, we, nt = tp["dt"], tp["omega_e"], tp["nt"]
    # the corrected frequency reproduces omega through the leapfrog symbol
    assert math.sin(we * dt / 2) / (dt / 2) == pytest.approx(omega, rel=1e-13)
    # Nt steps of dt cover one corrected period exactly
    assert we * nt * dt == pytest.approx(2 * math.pi, rel=1e-14)
    # stable at the requested fraction of the limit, and Nt is minimal unless floored at 5
    limit = 0.9 * oc.stability_constant(order)
    root = math.sqrt(sum(1 / h ** 2 for h in grid.h))
    assert math.sqrt(c2) * dt * root <= limit * (1 + 1e-14)
    if nt > 5:
        dt_less = (2 / omega) * math.sin(math.pi / (nt - 1))
        assert math.sqrt(c2) * dt_less * root > limit
    # alpha_d: beta_d(omega_e) = 1 and beta_d has zero slope at omega_e
    Tbar = nt * dt
    b = lambda lam: float(cf.beta_d(lam, we, Tbar, dt, tp["alpha"]))
    assert b(we) == pytest.approx(1.0, abs=1e-13)
    eps = 1e-4 * we
    slope = (b(we + eps) - b(we - eps)) / (2 * eps)
    assert abs(slope) * we < 1e-6
    # with alpha = 1/2 instead the slope does not vanish (so the check has teeth)
    b_half = lambda lam: float(cf.beta_d(lam, we, Tbar, dt, 0.5))
    assert abs((b_half(we + eps) - b_half(we - eps)) / (2 * eps)) * we > 10 * abs(slope) * we


def test_alpha_d_tends_to_one_half():
    grid = oc.Grid(2, (4096, 4096), 2)
    tp = oc.time_params(grid, 1.0, 5.0)
    assert tp["alpha_d"] == pytest.approx(0.5, abs=1e-5)


# ---------------------------------------------------------------------------
# filter: the oracle's trapezoid weights vs the three-sinc closed form
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("periods", [1, 2, 3])
@pytest.mark.parametrize("nt", [5, 17, 123])
def test_filter_weights_sum_to_three_sinc_form(periods, nt):
    omega = 7.0
    dt = (2 / omega) * math.sin(math.pi / nt)
    we = 2 * math.pi / (nt * dt)
    alpha = math.tan(we * dt / 2) / math.tan(we * dt)
    tp = dict(nt=nt, periods=periods, dt=dt, omega_e=we, alpha=alpha)
    N = nt * periods
    w = np.array([oc.filter_weight(k, tp) for k in range(N + 1)])
    t = np.arange(N + 1) * dt
    lams = np.concatenate([[0.0, we, 0.5 * we, 2 * we], np.linspace(0.01, 3 * we, 37)])
    for lam in lams:
        trap = float(np.sum(w * np.cos(lam * t)))
        closed = float(cf.beta_d(lam, we, N * dt, dt, alpha))
        assert trap == pytest.approx(closed, abs=2e-14), (lam, trap, closed)


# ---------------------------------------------------------------------------
# one WaveHoltz application on a sine mode: W_h(mode, 0) = beta_d(lambda~) mode
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("periods", [1, 2])
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("dim,n,ks", [(2, (16, 21), (1, 3)), (2, (16, 16), (15, 2)),
                                      (3, (10, 8, 11), (1, 2, 3))])
def test_apply_on_eigenmode(periods, order, dim, n, ks):
    grid = oc.Grid(dim, n, order)
    tp = oc.time_params(grid, 1.0, 9.1, periods=periods)
    mode = _mode(grid, ks)
    out = oc.apply(grid, 1.0, None, mode, tp, with_forcing=False)
    lam2 = sum(cf.lambda_h_sq_1d(k * math.pi, 1.0 / nn, order) for k, nn in zip(ks, n))
    beta = float(cf.beta_d_tp(cf.lambda_tilde(math.sqrt(lam2), tp["dt"]), tp))
    assert np.abs(out - beta * mode).max() < 1e-13


# ---------------------------------------------------------------------------
# fixed-point iterates against the sine-basis closed form (Sec. 4.2.1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("periods", [1, 2])
def test_fpi_iterates_closed_form_small(order, periods):
    w = wl.single_gaussian_source(dim=2, n=32, omega=10.3)
    grid = oc.Grid(2, (32, 32), order)
    tp = oc.time_params(grid, 1.0, w["omega"], periods=periods)
    v0 = wl.random_field(grid.shape, seed=7)
    iters = []
    oc.fpi(grid, 1.0, w["f"], tp, 4, v0=v0, callback=lambda k, v: iters.append(v.copy()))
    for k, v in enumerate(iters, start=1):
        ref = cf.fpi_iterate_closed_form(grid, 1.0, w["f"], w["omega"], tp, k, v0=v0)
        assert _rel(v, ref) < 1e-12


def test_fpi_iterates_closed_form_3d():
    grid = oc.Grid(3, (12, 10, 9), 4)
    x, y, z = oc.coords(grid)
    f = np.exp(-60 * ((x - 0.4) ** 2 + (y - 0.5) ** 2 + (z - 0.6) ** 2))
    f[~oc.interior_mask(grid)] = 0
    tp = oc.time_params(grid, 1.0, 6.3)
    v, _ = oc.fpi(grid, 1.0, f, tp, 3)
    ref = cf.fpi_iterate_closed_form(grid, 1.0, f, 6.3, tp, 3)
    assert _rel(v, ref) < 1e-12


def test_single_gaussian_square_30_iterations():
    """The 128^2 second-order single-source case, 30 iterations, against the
    sine-basis closed form; also the predicted rate mu of Theorem 2."""
    w = wl.single_gaussian_source()
    grid = oc.Grid(2, (128, 128), 2)
    tp = oc.time_params(grid, 1.0, w["omega"])
    assert tp["nt"] == 123
    v, hist = oc.fpi(grid, 1.0, w["f"], tp, 30)
    ref = cf.fpi_iterate_closed_form(grid, 1.0, w["f"], w["omega"], tp, 30)
    assert _rel(v, ref) < 1e-12
    U = cf.helmholtz_closed_form(grid, 1.0, w["f"], w["omega"])
    assert _rel(v, U) == pytest.approx(0.739, abs=2e-3)  # 30 iterations are far from converged
    mu, lam = cf.predicted_rate(grid, 1.0, tp)
    assert mu == pytest.approx(0.99198, abs=1e-4)
    # the residual ratio of the last steps approaches mu from below
    ratios = hist[1:] / hist[:-1]
    assert ratios[-1] <= mu + 1e-6


# ---------------------------------------------------------------------------
# convergence rate (Theorem 2): measured FPI rate tends to mu
# ---------------------------------------------------------------------------
def test_measured_rate_matches_theorem():
    grid = oc.Grid(2, (16, 16), 2)
    omega = 9.0
    tp = oc.time_params(grid, 1.0, omega)
    mu, _ = cf.predicted_rate(grid, 1.0, tp)
    f = wl.random_field(grid.shape, seed=5)
    _, hist = oc.fpi(grid, 1.0, f, tp, 400)
    rate = hist[-1] / hist[-2]
    assert rate == pytest.approx(mu, rel=2e-3)


# ---------------------------------------------------------------------------
# converged GMRES against a sparse direct solve of the discrete Helmholtz problem
# ---------------------------------------------------------------------------
def _best_omega(grid, c2, candidates):
    """Pick the candidate frequency farthest from resonance (largest min |1 - beta_d|)."""
    import scipy.sparse as sp
    inner = (slice(1, -1),) * grid.dim
    L = cf.laplacian_matrix(grid)
    c2i = (np.full(grid.shape, c2) if np.isscalar(c2) else c2)[inner].ravel()
    ev = np.linalg.eigvals((sp.diags(c2i) @ L).toarray())
    lam = np.sqrt(np.maximum(-ev.real, 0))
    best = None
    for om in candidates:
        tp = oc.time_params(grid, c2, om)
        gap = float(np.min(np.abs(1 - cf.beta_d_tp(cf.lambda_tilde(lam, tp["dt"]), tp))))
        if best is None or gap > best[1]:
            best = (om, gap)
    return best[0]


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("dim,n", [(2, (18, 14)), (3, (8, 9, 7))])
def test_gmres_converges_to_direct_solve(order, dim, n):
    grid = oc.Grid(dim, n, order)
    rng_c2 = wl.random_field(grid.shape, seed=21, zero_walls=False)
    c2 = 0.5 + 1.5 / (1 + np.exp(-rng_c2))  # smooth-ish, in (0.5, 2)
    x = oc.coords(grid)
    f = np.exp(-40 * sum((xi - 0.45) ** 2 for xi in x))
    f[~oc.interior_mask(grid)] = 0
    omega = _best_omega(grid, c2, np.linspace(6.0, 14.0, 17))
    tp = oc.time_params(grid, c2, omega)
    sol, info = oc.gmres(grid, c2, f, tp, restart=30, rtol=1e-13, maxit=600)
    assert info["rel_res"] <= 1e-13
    U = cf.dhs_direct(grid, c2, f, omega)
    assert _rel(sol, U) < 1e-10
    res = oc.helmholtz_residual(grid, c2, f, sol, omega)
    assert np.linalg.norm(res) / np.linalg.norm(f) < 1e-10


@pytest.mark.parametrize("order", [2, 4])
def test_cg_converges_to_direct_solve(order):
    """CG in the 1/c^2-weighted inner product reaches the discrete Helmholtz
    solution (variable c^2, non-square grid)."""
    grid = oc.Grid(2, (20, 15), order)
    g = wl.random_field(grid.shape, seed=23, zero_walls=False)
    c2 = 0.5 + 1.5 / (1 + np.exp(-g))
    x = oc.coords(grid)
    f = np.exp(-50 * ((x[0] - 0.3) ** 2 + (x[1] - 0.6) ** 2))
    f[~oc.interior_mask(grid)] = 0
    omega = _best_omega(grid, c2, np.linspace(6.0, 14.0, 17))
    tp = oc.time_params(grid, c2, omega)
    sol, info = oc.cg(grid, c2, f, tp, rtol=1e-13, maxit=3000)
    assert info["rel_res"] <= 1e-12
    U = cf.dhs_direct(grid, c2, f, omega)
    assert _rel(sol, U) < 1e-10


def test_filter_function_bounded_by_one():
    """beta_d <= 1 on the whole range of lambda~ an explicit step can produce,
    with equality only at omega_e: A = I - S_h is positive semi-definite."""
    for (n, order, c2max, om, Np) in [(2048, 4, 2.0, 200.0, 1), (128, 2, 1.0, 10.3, 1), (64, 4, 1.0, 3.7, 2)]:
        grid = oc.Grid(2, (n, n), order)
        tp = oc.time_params(grid, c2max, om, periods=Np)
        lt = np.linspace(0.0, math.pi / tp["dt"] * (1 - 1e-9), 400001)
        b = cf.beta_d_tp(lt, tp)
        assert b.max() <= 1.0 + 1e-12
        assert b.min() >= -0.5 - 1e-12
        far = np.abs(lt - tp["omega_e"]) > 0.05 * tp["omega_e"]
        assert b[far].max() < 0.999


def test_fpi_converges_to_closed_form_dhs():
    """Far from resonance the plain fixed-point iteration itself reaches the DHS."""
    grid = oc.Grid(2, (12, 12), 4)
    f = wl.random_field(grid.shape, seed=8)
    tp = oc.time_params(grid, 1.0, 5.0)
    mu, _ = cf.predicted_rate(grid, 1.0, tp)
    assert mu < 0.95
    iters = int(math.log(1e-15) / math.log(mu)) + 20
    v, _ = oc.fpi(grid, 1.0, f, tp, iters)
    U = cf.helmholtz_closed_form(grid, 1.0, f, 5.0)
    assert _rel(v, U) < 1e-12


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------
def test_invariants_linear_affine_symmetric():
    grid = oc.Grid(2, (15, 19), 4)
    tp = oc.time_params(grid, 1.0, 8.2)
    f = wl.random_field(grid.shape, seed=1)
    u = wl.random_field(grid.shape, seed=2)
    v = wl.random_field(grid.shape, seed=3)
    S = lambda a: oc.apply(grid, 1.0, None, a, tp, with_forcing=False)
    assert np.abs(oc.apply_A(grid, 1.0, np.zeros(grid.shape), tp)).max() == 0.0
    np.testing.assert_allclose(S(2.0 * u - 3.0 * v), 2.0 * S(u) - 3.0 * S(v), atol=1e-12)
    b = oc.apply(grid, 1.0, f, np.zeros(grid.shape), tp)
    np.testing.assert_allclose(oc.apply(grid, 1.0, f, u, tp), S(u) + b, atol=1e-12)
    # S is self-adjoint for constant c (Sec. 5.3)
    assert float(np.sum(u * S(v))) == pytest.approx(float(np.sum(S(u) * v)), rel=1e-12)


def test_leapfrog_is_time_reversible():
    """Stepping W^{n-1} = 2W^n - W^{n+1} + dt^2 L W^n back from the last two
    levels recovers the initial data (no forcing)."""
    grid = oc.Grid(2, (20, 20), 4)
    c2 = 1.0 + 0.3 * np.abs(wl.random_field(grid.shape, seed=9, zero_walls=False))
    tp = oc.time_params(grid, c2, 7.0)
    v = wl.random_field(grid.shape, seed=10)
    tp1 = dict(tp, nt=tp["nt"] - 1)
    _, w_last = oc.apply(grid, c2, None, v, tp, with_forcing=False, return_final=True)
    _, w_prev = oc.apply(grid, c2, None, v, tp1, with_forcing=False, return_final=True)
    a, b = w_last, w_prev
    for _ in range(tp["nt"] - 1):
        a, b = b, 2 * b - a + tp["dt"] ** 2 * oc.laplacian(grid, c2, b)
    # b is now W^0 reconstructed from the end
    assert np.abs(b - v).max() < 1e-9


def test_apply_at_points_matches_full_apply():
    grid = oc.Grid(2, (60, 45), 4)
    c2 = 0.7 + 0.5 * np.abs(wl.random_field(grid.shape, seed=12, zero_walls=False))
    f = wl.random_field(grid.shape, seed=13)
    v = wl.random_field(grid.shape, seed=14)
    tp = oc.time_params(grid, c2, 30.0)
    full = oc.apply(grid, c2, f, v, tp)
    pts = [(1, 1), (30, 22), (59, 44), (0, 10), (45, 3), (2, 43)]
    got = oc.apply_at_points(grid, c2, f, v, tp, pts)
    want = np.array([full[p[1], p[0]] for p in pts])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(full).max())
