"""Pins of the oracle's discrete adjoint against what fixes it independently
of its own code: the forward C oracle (dot-product identity, finite
differences of the forward map, which is affine in f and v and polynomial in
c^2), the closed-form eigenmodes (S^T of a sine mode is beta_d times the mode
for constant c^2), the weighted-symmetry reformulation, and finite
differences of a receiver misfit through converged solves.  Planted
mistakes in a copy of the adjoint source must each fail one of these pins.
"""
import importlib.util
import os

import numpy as np
import pytest

from oracle import adjoint as oa
from oracle import closed_forms as cf
from oracle import core as oc
import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
ADJ_SRC = os.path.join(os.path.dirname(HERE), "oracle", "adjoint.py")

CASES = [
    # dim, n, order, c2 kind, periods, omega
    (2, (13, 11), 4, "var", 1, 7.0),
    (2, (12, 9), 2, "var", 2, 6.0),
    (2, (10, 10), 4, "const", 1, 5.5),
    (3, (6, 5, 7), 2, "var", 1, 4.0),
    (3, (6, 6, 5), 4, "var", 1, 4.5),
]


def _problem(dim, n, order, kind, seed):
    grid = oc.Grid(dim, n, order)
    if kind == "const":
        c2 = 1.3
    else:
        g = wl.random_field(grid.shape, seed=seed, zero_walls=False)
        c2 = 0.6 + 1.2 / (1.0 + np.exp(-g))
    f = wl.random_field(grid.shape, seed=seed + 1)
    v = wl.random_field(grid.shape, seed=seed + 2)
    lam = wl.random_field(grid.shape, seed=seed + 3)
    d = wl.random_field(grid.shape, seed=seed + 4)
    return grid, c2, f, v, lam, d


def _dot(grid, a, b):
    m = oc.interior_mask(grid)
    return float(np.sum(np.asarray(a)[m] * np.asarray(b)[m]))


def _check_all(mod, case, seed=300):
    """Every pin for one case with the adjoint module `mod`; returns a dict
    of relative errors."""
    dim, n, order, kind, periods, omega = case
    grid, c2, f, v, lam, d = _problem(dim, n, order, kind, seed)
    tp = oc.time_params(grid, c2, omega, periods=periods)
    err = {}
    # trajectory and weights reproduce the forward oracle
    W = mod.trajectory(grid, c2, f, v, tp)
    Y = sum(w * Wn for w, Wn in zip(mod.weights(tp), W))
    Yc = oc.apply(grid, c2, f, v, tp)
    err["trajectory"] = float(np.linalg.norm(Y - Yc) / np.linalg.norm(Yc))
    # dot-product identity <lam, S v> = <S^T lam, v>
    Sv = oc.apply(grid, c2, None, v, tp, with_forcing=False)
    STl = mod.apply_transpose(grid, c2, lam, tp)
    a, b = _dot(grid, lam, Sv), _dot(grid, STl, v)
    err["dot"] = abs(a - b) / abs(a)
    # sensitivities against finite differences of the forward oracle
    d_c2, d_f, d_v = mod.parameter_gradient(grid, c2, f, v, lam, tp)
    c2a = np.full(grid.shape, float(c2)) if np.isscalar(c2) else c2

    def phi(c=c2a, ff=f, vv=v):
        return _dot(grid, lam, oc.apply(grid, c, ff, vv, tp))

    e = 2e-3
    fd1 = (phi(c=c2a + e * d) - phi(c=c2a - e * d)) / (2 * e)
    fd2 = (phi(c=c2a + 0.5 * e * d) - phi(c=c2a - 0.5 * e * d)) / e
    fd = (4.0 * fd2 - fd1) / 3.0  # Richardson: O(e^4)
    err["c2"] = abs(_dot(grid, d_c2, d) - fd) / abs(fd)
    fdf = (phi(ff=f + d) - phi(ff=f - d)) / 2.0  # affine in f
    err["f"] = abs(_dot(grid, d_f, d) - fdf) / abs(fdf)
    fdv = (phi(vv=v + d) - phi(vv=v - d)) / 2.0  # affine in v
    err["v"] = abs(_dot(grid, d_v, d) - fdv) / abs(fdv)
    return err


@pytest.mark.parametrize("case", CASES)
def test_adjoint_pins(case):
    err = _check_all(oa, case)
    assert err["trajectory"] <= 1e-13, err
    assert err["dot"] <= 1e-12, err
    assert err["c2"] <= 1e-7, err
    assert err["f"] <= 1e-10, err
    assert err["v"] <= 1e-10, err


@pytest.mark.parametrize("order", [2, 4])
def test_transpose_of_sine_mode_is_beta_d(order):
    """Constant c^2: S is symmetric and the sine modes are its eigenvectors
    with eigenvalue beta_d(lambda_tilde) (Sec. 4.2.1, three-sinc form)."""
    grid = oc.Grid(2, (16, 12), order)
    c2 = 1.7
    tp = oc.time_params(grid, c2, 9.0)
    x, y = oc.coords(grid)
    lam2 = cf.mode_eigenvalues(grid, c2)  # [ky - 1, kx - 1]
    for kx, ky in [(1, 1), (3, 2), (7, 5), (15, 11)]:
        mode = np.sin(kx * np.pi * x) * np.sin(ky * np.pi * y)
        beta = cf.beta_d_tp(cf.lambda_tilde(np.sqrt(lam2[ky - 1, kx - 1]), tp["dt"]), tp)
        got = oa.apply_transpose(grid, c2, mode, tp)
        assert np.linalg.norm(got - beta * mode) <= 1e-12 * np.linalg.norm(mode), (kx, ky)


def test_adjoint_solve_matches_weighted_symmetry():
    """(I - S)^T = C^{-1} (I - S) C with C = diag(c^2): the adjoint solution
    equals C^{-1} times the forward CG solution for the right-hand side C g."""
    grid, c2, _, _, _, _ = _problem(2, (12, 10), 4, "var", 71)
    tp = oc.time_params(grid, c2, 6.5)
    g = wl.random_field(grid.shape, seed=72)
    lam = oa.solve_adjoint(grid, c2, g, tp)
    m = oc.interior_mask(grid)
    res = (lam - oa.apply_transpose(grid, c2, lam, tp) - g)[m]
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(g[m])
    mu, info = oc.cg(grid, c2, None, tp, rtol=1e-14, maxit=5000, b=oa._interior(grid, c2 * g))
    assert np.linalg.norm((mu / c2 - lam)[m]) <= 1e-10 * np.linalg.norm(lam[m])


def test_misfit_gradient_matches_finite_differences():
    """d/dc^2 and d/df of J = 1/2 ||R v*(c^2, f) - d||^2 through converged
    fixed-point solves, against central differences of J."""
    grid = oc.Grid(2, (12, 10), 2)
    rng = np.random.Generator(np.random.PCG64(81))
    c2 = 1.0 + 0.3 * wl.random_field(grid.shape, seed=82, zero_walls=False) ** 2
    f = wl.random_field(grid.shape, seed=83)
    omega = 6.3
    tp = oc.time_params(grid, c2, omega)
    tp_fixed = dict(tp)
    idx = np.array(sorted(set(int(i) for i in rng.integers(0, grid.nodes, 25))))
    idx = idx[oc.interior_mask(grid).ravel()[idx]]
    data = rng.uniform(-0.1, 0.1, idx.size)

    def solve(c, ff):
        x, info = oc.cg(grid, c, ff, tp_fixed, rtol=1e-14, maxit=5000)
        return x

    def J(c, ff):
        return oa.receiver_misfit(solve(c, ff), idx, data)[0]

    v = solve(c2, f)
    _, gv = oa.receiver_misfit(v, idx, data)
    lam = oa.solve_adjoint(grid, c2, gv, tp_fixed)
    d_c2, d_f, _ = oa.parameter_gradient(grid, c2, f, v, lam, tp_fixed)
    d = wl.random_field(grid.shape, seed=84)
    e = 1e-4
    fd_c = (J(c2 + e * d, f) - J(c2 - e * d, f)) / (2 * e)
    assert abs(_dot(grid, d_c2, d) - fd_c) <= 1e-5 * abs(fd_c)
    fd_f = (J(c2, f + e * d) - J(c2, f - e * d)) / (2 * e)
    assert abs(_dot(grid, d_f, d) - fd_f) <= 1e-6 * abs(fd_f)


def test_receiver_misfit_brute_force():
    u = np.arange(20.0).reshape(4, 5)
    idx = np.array([3, 7, 7, 12])
    data = np.array([1.0, 2.0, 3.0, 4.0])
    J, g = oa.receiver_misfit(u, idx, data)
    r = np.array([3 - 1, 7 - 2, 7 - 3, 12 - 4], dtype=float)
    assert J == 0.5 * float(np.sum(r * r))
    want = np.zeros(20)
    want[3], want[7], want[12] = 2.0, 5.0 + 4.0, 8.0
    assert np.array_equal(g.ravel(), want)


# planted mistakes: (description, text replaced, replacement)
MUTATIONS = [
    ("first-step sensitivity weight 1 instead of 1/2", "kappa = 0.5 if n == 0 else 1.0", "kappa = 1.0"),
    ("c^2 applied after the Laplacian in the transpose",
     "return oc.laplacian(grid, 1.0, _interior(grid, _c2_array(grid, c2) * Z))",
     "return oc.laplacian(grid, c2, _interior(grid, Z))"),
    ("first forcing coefficient without the 1/2", "return [-0.5 * dt * dt] +", "return [-dt * dt] +"),
    ("second-previous adjoint level dropped", "2.0 * Z[n + 1] - Z[n + 2] +", "2.0 * Z[n + 1] +"),
    ("weights shifted by one level", "Z[n] = w[n] * lam", "Z[n] = w[n - 1] * lam"),
    ("cosine time shifted by one step", "math.cos(tp[\"omega_e\"] * n * dt)", "math.cos(tp[\"omega_e\"] * (n + 1) * dt)"),
    ("first adjoint level without the 1/2 on L^T", "Z[1] + 0.5 * dt2 * _LT(grid, c2, Z[1])",
     "Z[1] + dt2 * _LT(grid, c2, Z[1])"),
]


def _load_mutant(tmp_path, old, new):
    src = open(ADJ_SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / "adjoint_mutant.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("oracle.adjoint_mutant", str(path))
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("desc,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_adjoint_mistake_is_caught(tmp_path, desc, old, new):
    mod = _load_mutant(tmp_path, old, new)
    bars = {"trajectory": 1e-13, "dot": 1e-12, "c2": 1e-7, "f": 1e-10, "v": 1e-10}
    caught = False
    for case in CASES[:2]:
        err = _check_all(mod, case)
        if any(err[k] > bars[k] for k in bars):
            caught = True
            break
    assert caught, desc
