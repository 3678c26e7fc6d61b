"""Pins of the implicit-stepping oracle (Sec. 4.2.2, Appendix A.2) against
what the paper and the mathematics fix: the two conditions that define the
corrected time step (eq. cosOmegaTilde, eq. impOmegaTildeEquation), the sine
eigenmodes mapped by beta_d(lambda~_i) (theorem on the implicit FPI rate),
the discrete Helmholtz solution as the fixed point of W_h(., f) (variable
c^2: sparse direct solve), every FPI iterate against its DST-I closed form,
and the measured rate; planted mistakes in a copy of the oracle must fail one
of these pins."""
import importlib.util
import math
import os

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import core as oc
from oracle import implicit as oi
import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "implicit.py")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("nits", [5, 7, 10, 16, 40])
def test_time_step_conditions(nits):
    omega = 23.5
    tp = oi.time_params_implicit(omega, nits)
    dt, wi = tp["dt"], tp["omega_e"]
    # cos(omega_i dt) = 1 / (1 + (omega dt)^2 / 2) and N_t dt = 2 pi / omega_i
    assert math.cos(wi * dt) == pytest.approx(1.0 / (1.0 + (omega * dt) ** 2 / 2.0), rel=1e-14)
    assert nits * dt == pytest.approx(2.0 * math.pi / wi, rel=1e-15)
    # the time-periodic solution of the scheme solves the Helmholtz equation
    # with the true omega: (2 - 2 cos(omega_i dt)) / (dt^2 cos(omega_i dt)) = omega^2
    assert (2.0 - 2.0 * math.cos(wi * dt)) / (dt * dt * math.cos(wi * dt)) == pytest.approx(omega ** 2, rel=1e-12)
    # beta_d(omega_i) = 1: the filter passes the corrected frequency
    assert float(cf.beta_d_tp(wi, tp)) == pytest.approx(1.0, abs=1e-13)


def test_fewer_than_five_steps_rejected():
    with pytest.raises(ValueError):
        oi.time_params_implicit(10.0, 4)


def _sine(grid, k):
    axes = [np.sin(km * math.pi * np.arange(nm + 1) / nm) for km, nm in zip(k, grid.n)]
    out = axes[0]
    for a in axes[1:]:
        out = np.multiply.outer(a, out)
    return out


def _check_modes(mod, grid, c2, omega, nits, modes):
    tp = mod.time_params_implicit(omega, nits)
    worst = 0.0
    for k in modes:
        phi = _sine(grid, k)
        lam = math.sqrt(c2 * sum(float(cf.lambda_h_sq_1d(km * math.pi, 1.0 / nm, grid.order))
                                 for km, nm in zip(k, grid.n)))
        beta = float(cf.beta_d_tp(oi.lambda_tilde_implicit(lam, tp["dt"]), tp))
        got = mod.apply_implicit(grid, c2, None, phi, tp, with_forcing=False)
        worst = max(worst, float(np.abs(got - beta * phi).max()))
    return worst


@pytest.mark.parametrize("dim,n,order,c2,omega,nits", [(2, (24, 20), 2, 1.0, 9.0, 10), (2, (18, 22), 4, 1.7, 13.0, 7),
                                                      (3, (8, 7, 9), 2, 1.2, 6.0, 5)])
def test_sine_modes_filtered_by_beta(dim, n, order, c2, omega, nits):
    grid = oc.Grid(dim, n, order)
    modes = [(1,) * dim, tuple(min(3, k - 1) for k in n), tuple(k - 1 for k in n), (2,) + (1,) * (dim - 1)]
    assert _check_modes(oi, grid, c2, omega, nits, modes) <= 1e-12


def _check_fixed_point(mod, grid, c2, omega, nits, periods=1):
    f = wl.random_field(grid.shape, seed=721)
    tp = mod.time_params_implicit(omega, nits, periods)
    U = cf.dhs_direct(grid, c2, f, omega)
    return _rel(mod.apply_implicit(grid, c2, f, U, tp), U)


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("periods", [1, 2])
def test_dhs_is_the_fixed_point(order, periods):
    """Variable c^2: the DHS with the true omega is reproduced by one
    application (the cos(omega_i dt) factor of the forcing and its phase)."""
    grid = oc.Grid(2, (21, 26), order)
    g = wl.random_field(grid.shape, seed=722, zero_walls=False)
    c2 = 0.7 + 0.6 / (1.0 + np.exp(-g))
    assert _check_fixed_point(oi, grid, c2, 11.3, 8, periods) <= 1e-11


@pytest.mark.parametrize("order,nits", [(2, 10), (4, 6)])
def test_fpi_iterates_closed_form_and_rate(order, nits):
    grid = oc.Grid(2, (26, 22), order)
    c2, omega = 1.1, 10.7
    f = wl.random_field(grid.shape, seed=731)
    tp = oi.time_params_implicit(omega, nits)
    _, hist = oi.fpi_implicit(grid, c2, f, tp, 40)
    inner = (slice(1, -1),) * grid.dim
    fh = cf._dst(f[inner])
    lam2 = cf.mode_eigenvalues(grid, c2)
    U = fh / (omega ** 2 - lam2)
    beta = cf.beta_d_tp(oi.lambda_tilde_implicit(np.sqrt(lam2), tp["dt"]), tp)
    for k in (1, 2, 7, 40):
        want = np.zeros(grid.shape)
        want[inner] = cf._idst((1.0 - beta ** k) * U)
        assert _rel(hist[k - 1], want) <= 1e-11, k
    # the contraction of the iterate differences tends to the predicted rate
    mu, _ = oi.predicted_rate_implicit(grid, c2, tp)
    _, hist = oi.fpi_implicit(grid, c2, f, tp, 1500)
    d = [np.linalg.norm(hist[k + 1] - hist[k]) for k in range(len(hist) - 3, len(hist) - 1)]
    assert d[-1] / d[-2] == pytest.approx(mu, rel=2e-3)


MUTATIONS = [
    ("forcing without the cos(omega_i dt) factor",
     "g = -dt * dt * math.cos(2.0 * math.pi * (n % tp[\"nt\"]) / tp[\"nt\"]) * cw",
     "g = -dt * dt * math.cos(2.0 * math.pi * (n % tp[\"nt\"]) / tp[\"nt\"])"),
    ("explicit first step", "cur = st.solve(prev - 0.5 * dt * dt * cw * fi)",
     "cur = prev - 0.5 * dt * dt * cw * fi"),
    ("wrong sign in M", "sp.identity(L.shape[0]) - 0.5 * dt * dt * self.CL",
     "sp.identity(L.shape[0]) + 0.5 * dt * dt * self.CL"),
    ("previous level not multiplied by M", "nxt = st.solve(2.0 * cur - st.mul(prev) + g * fi)",
     "nxt = st.solve(2.0 * cur - prev + g * fi)"),
    ("time step of the explicit recipe", "dt = math.sqrt(2.0 / math.cos(2.0 * math.pi / nits) - 2.0) / omega",
     "dt = 2.0 * math.sin(math.pi / nits) / omega"),
]


@pytest.mark.parametrize("desc,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_implicit_mistake_is_caught(tmp_path, desc, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / "implicit_mutant.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("oracle.implicit_mutant", str(path))
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    spec.loader.exec_module(mod)
    grid = oc.Grid(2, (14, 12), 2)
    try:
        bad_modes = _check_modes(mod, grid, 1.3, 8.0, 7, [(1, 1), (3, 2), (13, 11)]) > 1e-12
        bad_fixed = _check_fixed_point(mod, grid, 1.3, 8.0, 7) > 1e-11
    except Exception:
        return
    assert bad_modes or bad_fixed, desc


@pytest.mark.parametrize("nits", [5, 10, 20])
def test_mode_map_limit(nits):
    """The implicit mode map saturates: lambda~_i tends to omega_i N_t / 4 as
    lambda grows (stated with the figure of the adjusted lambda, Sec. 4.2.2),
    and it is increasing, with lambda~_i ~ lambda for lambda dt -> 0."""
    tp = oi.time_params_implicit(3.0, nits)
    dt, wi = tp["dt"], tp["omega_e"]
    big = oi.lambda_tilde_implicit(1e9 / dt, dt)
    assert big == pytest.approx(wi * nits / 4.0, rel=1e-9)
    lam = np.linspace(1e-3, 50.0, 200) / dt
    lt = oi.lambda_tilde_implicit(lam, dt)
    assert np.all(np.diff(lt) > 0)
    small = 1e-4 / dt
    assert oi.lambda_tilde_implicit(small, dt) == pytest.approx(small, rel=1e-8)
