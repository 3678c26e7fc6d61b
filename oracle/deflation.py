"""Double-precision CPU oracle of WaveHoltz with deflation (Alg. 3,
Sec. 5.2) on the unit box with constant c^2.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and never by the GPU
library.

On the unit box with Dirichlet walls and constant c^2 the discrete
eigenfunctions are the sine modes phi_k(x_i) = prod_a sqrt(2/n_a)
sin(k_a pi i_a / n_a) (orthonormal in the plain nodal sum) with eigenvalues
lambda_k^2 = c^2 sum_a lambda_{h,1d}^2(k_a) of the order-p operator (App. B).
Alg. 3 removes the components along the deflated modes after every filter
step and, once the iteration has converged, adds back the Helmholtz
components (f, phi_k) / (omega^2 - lambda_k^2) of those modes.  The deflated
modes are chosen as the slowest to converge, i.e. the largest |beta_d|, so
that the rate of the theorem on deflated convergence, the largest |beta_d|
over the modes kept, is as small as possible.

Reading: the eigenvalues used in the inflation are the discrete ones of the
spatial operator, so that the inflated fixed point is the discrete Helmholtz
solution itself.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import closed_forms as cf
from . import core as oc


def sine_mode(grid, k):
    """Normalized sine mode with wave numbers k = (k_x, k_y[, k_z])."""
    axes = []
    for m, (km, nm) in enumerate(zip(k, grid.n)):
        i = np.arange(nm + 1)
        axes.append(math.sqrt(2.0 / nm) * np.sin(km * math.pi * i / nm))
    out = axes[0]
    for a in axes[1:]:
        out = np.multiply.outer(a, out)  # slower axis first
    return out


def mode_eigenvalue(grid, c2, k):
    """lambda_k^2 of -c^2 Delta_h for the sine mode k."""
    return float(c2) * sum(float(cf.lambda_h_sq_1d(km * math.pi, 1.0 / nm, grid.order))
                           for km, nm in zip(k, grid.n))


def select_modes(grid, c2, tp, count):
    """The `count` modes with the largest |beta_d| (slowest to converge) and
    the predicted deflated rate max |beta_d| over the remaining modes."""
    modes = list(itertools.product(*[range(1, nm) for nm in grid.n]))
    lam2 = np.array([mode_eigenvalue(grid, c2, k) for k in modes])
    beta = np.abs(cf.beta_d_tp(cf.lambda_tilde(np.sqrt(lam2), tp["dt"]), tp))
    order = np.argsort(-beta, kind="stable")
    chosen = [modes[i] for i in order[:count]]
    rest = beta[order[count:]]
    return chosen, (float(rest.max()) if rest.size else 0.0)


def project_out(grid, v, modes):
    """v - sum over the modes of (v, phi) phi."""
    out = np.array(v, dtype=np.float64, copy=True)
    for k in modes:
        phi = sine_mode(grid, k)
        out -= float(np.sum(out * phi)) * phi
    return out


def inflate(grid, c2, f, omega, modes, v):
    """v + sum over the modes of (f, phi) / (omega^2 - lambda^2) phi."""
    out = np.array(v, dtype=np.float64, copy=True)
    fi = np.array(f, dtype=np.float64, copy=True)
    fi[~oc.interior_mask(grid)] = 0.0
    for k in modes:
        phi = sine_mode(grid, k)
        out += float(np.sum(fi * phi)) / (omega ** 2 - mode_eigenvalue(grid, c2, k)) * phi
    return out


def fpi_deflated(grid, c2, f, tp, modes, iters, inflate_result=True, callback=None):
    """Alg. 3: v^0 = 0; v^{k+1} = W_h(v^k, f) with the deflated components
    removed; the converged iterate is inflated.  Returns the final iterate
    (inflated unless asked otherwise) and the list of deflated iterates."""
    v = np.zeros(grid.shape)
    hist = []
    for _ in range(iters):
        v = oc.apply(grid, c2, f, v, tp, with_forcing=True)
        v = project_out(grid, v, modes)
        hist.append(v)
        if callback is not None:
            callback(v)
    out = inflate(grid, c2, f, tp["omega"], modes, v) if inflate_result else v
    return out, hist
