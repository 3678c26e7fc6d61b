"""Pins of the oracle's outer iterations at fixed step counts, and of its
Helmholtz residual, by the properties that define them.

* GMRES (Sec. 5.3, Krylov form (I - S_h) v = b): after j Arnoldi steps of a
  cycle that starts from x, the iterate is x + z with z minimising
  ||r - A z||_2 over the Krylov space K_j(A, r), r = b - A x; every `restart`
  steps a new cycle starts from the current iterate.  The reference below
  obtains the Krylov basis from LAPACK's Householder QR and the minimiser
  from a dense least-squares solve, so it shares neither the oracle's
  modified Gram-Schmidt nor its Givens rotations.
* CG in the inner product <u, w> = sum u w / c^2: after k steps from 0 the
  iterate minimises the energy norm (x - x*)^T W A (x - x*), W = diag(1/c^2),
  over K_k(A, b) (W A is symmetric positive definite: Sec. 5.3 states that S
  is self-adjoint, here in the 1/c^2 inner product).  The reference solves
  the projected normal equations with the dense exact solution x*.
* Helmholtz residual (eq. HelmholtzBVP with L = c^2 Delta_{h,p}): equal to
  (diag(c^2) L_p + omega^2 I) u - f with L_p the sparse Kronecker-sum
  Dirichlet Laplacian assembled from the 1-D second-difference matrix.

A is assembled column by column from the oracle's own apply_A: these pins are
on the iterations, the operator itself is pinned by the sine-mode, closed-form
and direct-solve tests.  Planted mistakes in copies of the iteration code
(restart off by one, a Givens sign, the inner-product weight, the direction
update) must each fail a pin.
"""
import importlib.util
import math
import os
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import closed_forms as cf
from oracle import core as oc
import workloads as wl

ORACLE_CORE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "core.py")


def _problem(order, n=(9, 8), seed=31):
    grid = oc.Grid(2, n, order)
    g = wl.random_field(grid.shape, seed=seed, zero_walls=False)
    c2 = 0.5 + 1.5 / (1 + np.exp(-g))
    x = oc.coords(grid)
    f = np.exp(-30 * ((x[0] - 0.4) ** 2 + (x[1] - 0.55) ** 2))
    f[~oc.interior_mask(grid)] = 0
    tp = oc.time_params(grid, c2, 7.3)
    return grid, c2, f, tp


def _dense_A(grid, c2, tp, core=oc):
    """A = I - S_h on the interior unknowns, one column per unit vector."""
    inner = oc.interior_mask(grid)
    idx = np.flatnonzero(inner.ravel())
    A = np.zeros((idx.size, idx.size))
    for j, node in enumerate(idx):
        e = np.zeros(grid.nodes)
        e[node] = 1.0
        A[:, j] = core.apply_A(grid, c2, e.reshape(grid.shape), tp).ravel()[idx]
    return A, idx


def _krylov_basis(A, r, k):
    """Orthonormal basis of span{r, A r, ..., A^{k-1} r} by Householder QR."""
    Q = (r / np.linalg.norm(r))[:, None]
    for _ in range(1, k):
        Q, _ = np.linalg.qr(np.column_stack([Q, A @ Q[:, -1]]))
    return Q


def _gmres_by_definition(A, b, restart, steps):
    x = np.zeros_like(b)
    done = 0
    while done < steps:
        j = min(restart, steps - done)
        r = b - A @ x
        Q = _krylov_basis(A, r, j)
        z, *_ = np.linalg.lstsq(A @ Q, r, rcond=None)
        x = x + Q @ z
        done += j
    return x


def _cg_by_definition(A, W, b, k):
    xs = np.linalg.solve(A, b)
    M = W @ A
    Q = _krylov_basis(A, b, k)
    y = np.linalg.solve(Q.T @ M @ Q, Q.T @ M @ xs)
    return Q @ y


def _load_core(tmp_path, name, old, new):
    """A copy of oracle/core.py with one textual substitution, loaded as its
    own module that reuses the already built C oracle."""
    src = open(ORACLE_CORE).read()
    assert src.count(old) == 1, f"mutation {name} does not match the oracle source exactly once"
    path = tmp_path / f"core_{name}.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"oracle_core_{name}", path)
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod
    spec.loader.exec_module(mod)
    mod._lib = oc._load()
    return mod


def _gmres_pin_error(core, order=4, restart=3, steps=7):
    grid, c2, f, tp = _problem(order)
    A, idx = _dense_A(grid, c2, tp)
    b = oc.apply(grid, c2, f, np.zeros(grid.shape), tp).ravel()[idx]
    want = _gmres_by_definition(A, b, restart, steps)
    got, info = core.gmres(grid, c2, f, tp, restart=restart, fixed_iters=steps)
    assert info["iters"] == steps
    return float(np.linalg.norm(got.ravel()[idx] - want) / np.linalg.norm(want))


def _cg_pin_error(core, order=4, steps=6):
    grid, c2, f, tp = _problem(order)
    A, idx = _dense_A(grid, c2, tp)
    W = np.diag(1.0 / c2.ravel()[idx])
    b = oc.apply(grid, c2, f, np.zeros(grid.shape), tp).ravel()[idx]
    want = _cg_by_definition(A, W, b, steps)
    got, info = core.cg(grid, c2, f, tp, fixed_iters=steps)
    assert info["iters"] == steps
    return float(np.linalg.norm(got.ravel()[idx] - want) / np.linalg.norm(want))


# ---------------------------------------------------------------------------
# GMRES
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("restart,steps", [(10, 1), (10, 5), (3, 7), (2, 6), (4, 4)])
def test_gmres_iterate_minimises_residual_over_krylov_space(order, restart, steps):
    assert _gmres_pin_error(oc, order, restart, steps) <= 1e-9


def test_gmres_iterate_beats_every_other_point_of_the_space():
    """The iterate's residual is no larger than that of random points of the
    same affine Krylov space (a check of the minimising property that needs
    no least-squares solve)."""
    grid, c2, f, tp = _problem(2)
    A, idx = _dense_A(grid, c2, tp)
    b = oc.apply(grid, c2, f, np.zeros(grid.shape), tp).ravel()[idx]
    k = 4
    got, _ = oc.gmres(grid, c2, f, tp, restart=10, fixed_iters=k)
    x = got.ravel()[idx]
    rmin = np.linalg.norm(b - A @ x)
    Q = _krylov_basis(A, b, k)
    rng = np.random.default_rng(5)
    for _ in range(200):
        z = x + Q @ (rng.standard_normal(k) * 1e-3 * np.linalg.norm(x))
        assert np.linalg.norm(b - A @ z) >= rmin * (1 - 1e-12)


# ---------------------------------------------------------------------------
# CG in the 1/c^2 inner product
# ---------------------------------------------------------------------------
def test_weighted_operator_is_symmetric_positive_definite():
    grid, c2, f, tp = _problem(4)
    A, idx = _dense_A(grid, c2, tp)
    M = np.diag(1.0 / c2.ravel()[idx]) @ A
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    # and A alone is not symmetric with variable c^2 (the weight matters)
    assert np.abs(A - A.T).max() > 1e-6 * np.abs(A).max()


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("steps", [1, 2, 4, 6])
def test_cg_iterate_minimises_energy_norm_over_krylov_space(order, steps):
    assert _cg_pin_error(oc, order, steps) <= 1e-9


# ---------------------------------------------------------------------------
# Helmholtz residual
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("dim,n", [(2, (13, 10)), (3, (7, 6, 8))])
def test_helmholtz_residual_equals_assembled_operator(order, dim, n):
    grid = oc.Grid(dim, n, order)
    c2 = 0.6 + np.abs(wl.random_field(grid.shape, seed=41, zero_walls=False))
    u = wl.random_field(grid.shape, seed=42)
    f = wl.random_field(grid.shape, seed=43)
    omega = 6.7
    inner = (slice(1, -1),) * dim
    L = cf.laplacian_matrix(grid)
    want = (sp.diags(c2[inner].ravel()) @ L + omega ** 2 * sp.identity(L.shape[0])) @ u[inner].ravel() \
        - f[inner].ravel()
    got = oc.helmholtz_residual(grid, c2, f, u, omega)
    assert np.abs(got[inner].ravel() - want).max() <= 1e-10 * np.abs(want).max()
    wall = ~oc.interior_mask(grid)
    assert np.all(got[wall] == 0.0)


def test_helmholtz_residual_of_direct_solution_vanishes_and_of_zero_is_minus_f():
    grid = oc.Grid(2, (11, 9), 4)
    c2 = 0.8 + 0.4 * np.abs(wl.random_field(grid.shape, seed=44, zero_walls=False))
    f = wl.random_field(grid.shape, seed=45)
    U = cf.dhs_direct(grid, c2, f, 5.5)
    r = oc.helmholtz_residual(grid, c2, f, U, 5.5)
    assert np.linalg.norm(r) <= 1e-11 * np.linalg.norm(f)
    r0 = oc.helmholtz_residual(grid, c2, f, np.zeros(grid.shape), 5.5)
    inner = oc.interior_mask(grid)
    np.testing.assert_array_equal(r0[inner], -f[inner])


# ---------------------------------------------------------------------------
# planted mistakes in copies of the iteration code
# ---------------------------------------------------------------------------
GMRES_MUTATIONS = {
    "restart_off_by_one": ("m = min(restart, limit - total)", "m = min(restart + 1, limit - total)"),
    "givens_rhs_sign": ("g[j + 1] = -sn[j] * g[j]", "g[j + 1] = sn[j] * g[j]"),
    "givens_rotation_sign": ("H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]",
                             "H[i + 1, j] = sn[i] * H[i, j] + cs[i] * H[i + 1, j]"),
    "gram_schmidt_one_short": ("for i in range(j + 1):  # modified Gram-Schmidt",
                               "for i in range(j):  # modified Gram-Schmidt"),
}

CG_MUTATIONS = {
    "unweighted_inner_product": ("ip = lambda a, b: float(np.sum(a * b * wgt))",
                                 "ip = lambda a, b: float(np.sum(a * b))"),
    "direction_ratio_inverted": ("p = r + (rr_new / rr) * p", "p = r + (rr / rr_new) * p"),
    "residual_update_sign": ("r = r - alpha * q", "r = r + alpha * q"),
}


@pytest.mark.parametrize("name", sorted(GMRES_MUTATIONS))
def test_planted_gmres_mistake_is_caught(tmp_path, name):
    core = _load_core(tmp_path, name, *GMRES_MUTATIONS[name])
    errs = [_gmres_pin_error(core, 4, restart, steps) for restart, steps in [(3, 7), (10, 5)]]
    assert max(errs) > 1e-6, f"planted mistake '{name}' slipped through: {errs}"


@pytest.mark.parametrize("name", sorted(CG_MUTATIONS))
def test_planted_cg_mistake_is_caught(tmp_path, name):
    core = _load_core(tmp_path, name, *CG_MUTATIONS[name])
    errs = [_cg_pin_error(core, 4, steps) for steps in (2, 4)]
    assert max(errs) > 1e-6, f"planted mistake '{name}' slipped through: {errs}"
