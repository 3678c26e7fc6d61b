"""The oracle's pins have teeth: plant a plausible mistake in a copy of the C
oracle, build it on the CPU, and check that a pin fails.

Each mutation is a textual substitution in a temporary copy of
``oracle/wh_oracle.c``; the committed oracle is never modified.
"""
import math
import os
import subprocess

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import core as oc
import workloads as wl

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "wh_oracle.c")

MUTATIONS = {
    "forcing_sign": ("(LW[idx] - forcing * fint[idx])", "(LW[idx] + forcing * fint[idx])"),
    "first_step_half": ("Wcur[idx] + 0.5 * dt * dt * (LW[idx]", "Wcur[idx] + dt * dt * (LW[idx]"),
    "first_step_forcing": ("(LW[idx] - s * fint[idx])", "(LW[idx])"),
    "trapezoid_end": ("(n == 0 || n == nsteps) ? 0.5", "(n == 0) ? 0.5"),
    "alpha_half": ("- 0.5 * alpha)", "- alpha)"),
    "ghost_sign": ("      ix[m] = -ix[m];\n      sign = -sign;", "      ix[m] = -ix[m];"),
    "stencil_index": ("seg[s + 2] - 2.0 * seg[s + 1] + seg[s]", "seg[s + 2] - 2.0 * seg[s] + seg[s]"),
    "c2_dropped": ("out[idx] = c2[idx] * lap;", "out[idx] = lap;"),
    "axes_transposed": ("for (int m = g->dim - 1; m >= 0; --m) idx = idx * (g->n[m] + 1) + ix[m];",
                        "for (int m = 0; m < g->dim; ++m) idx = idx * (g->n[m] + 1) + ix[m];"),
    "leapfrog_sign": ("2.0 * Wcur[idx] - Wprev[idx]", "2.0 * Wcur[idx] + Wprev[idx]"),
    "residual_zero": ("res[idx] = orc_is_boundary(&g, ix) ? 0.0 : res[idx] + omega * omega * u[idx] - f[idx];",
                      "res[idx] = 0.0;"),
    "residual_omega_sign": ("res[idx] + omega * omega * u[idx] - f[idx]", "res[idx] - omega * omega * u[idx] - f[idx]"),
    "residual_f_dropped": ("res[idx] + omega * omega * u[idx] - f[idx]", "res[idx] + omega * omega * u[idx]"),
}


def _build_mutant(tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation {name} does not match the oracle source exactly once"
    mpath = tmp_path / f"{name}.c"
    mpath.write_text(src.replace(old, new))
    lib = tmp_path / f"lib_{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(lib), str(mpath), "-lm"],
                   check=True)
    return str(lib)


def _pins_pass():
    """A fast subset of the pins: eigenmodes (p = 2, 4, non-square grid, Np = 2),
    the closed-form fixed-point iterates with a source, a variable-c^2
    operator check against the assembled sparse matrix, and the Helmholtz
    residual against the same assembled operator."""
    ok = True
    for order in (2, 4):
        grid = oc.Grid(2, (14, 11), order)
        tp = oc.time_params(grid, 1.0, 9.1, periods=2)
        x, y = oc.coords(grid)
        mode = np.sin(math.pi * x) * np.sin(3 * math.pi * y)
        out = oc.apply(grid, 1.0, None, mode, tp, with_forcing=False)
        lam2 = cf.lambda_h_sq_1d(math.pi, 1 / 14, order) + cf.lambda_h_sq_1d(3 * math.pi, 1 / 11, order)
        beta = float(cf.beta_d_tp(cf.lambda_tilde(math.sqrt(lam2), tp["dt"]), tp))
        ok &= bool(np.abs(out - beta * mode).max() < 1e-13)
    grid = oc.Grid(2, (16, 16), 2)
    w = wl.single_gaussian_source(dim=2, n=16, omega=10.3)
    tp = oc.time_params(grid, 1.0, w["omega"])
    v, _ = oc.fpi(grid, 1.0, w["f"], tp, 2)
    ref = cf.fpi_iterate_closed_form(grid, 1.0, w["f"], w["omega"], tp, 2)
    ok &= bool(np.linalg.norm(v - ref) <= 1e-12 * np.linalg.norm(ref))
    grid = oc.Grid(2, (9, 7), 4)
    c2 = 1.0 + np.abs(wl.random_field(grid.shape, seed=3, zero_walls=False))
    u = wl.random_field(grid.shape, seed=4)
    inner = (slice(1, -1),) * 2
    import scipy.sparse as sp
    want = (sp.diags(c2[inner].ravel()) @ cf.laplacian_matrix(grid)) @ u[inner].ravel()
    got = oc.laplacian(grid, c2, u)[inner].ravel()
    ok &= bool(np.abs(got - want).max() <= 1e-9 * np.abs(want).max())
    f = wl.random_field(grid.shape, seed=5)
    omega = 4.5
    L = cf.laplacian_matrix(grid)
    want = (sp.diags(c2[inner].ravel()) @ L + omega ** 2 * sp.identity(L.shape[0])) @ u[inner].ravel() \
        - f[inner].ravel()
    got = oc.helmholtz_residual(grid, c2, f, u, omega)[inner].ravel()
    ok &= bool(np.abs(got - want).max() <= 1e-9 * np.abs(want).max())
    return ok


def test_unmutated_oracle_passes_the_subset():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    prev = oc.use_library(_build_mutant(tmp_path, name))
    try:
        caught = not _pins_pass()
    finally:
        oc.restore_library(prev)
    assert caught, f"planted mistake '{name}' slipped through the pins"
