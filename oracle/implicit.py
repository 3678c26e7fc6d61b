"""Double-precision CPU oracle of WaveHoltz with implicit time stepping
(Sec. 4.2.2, eq. WaveSchemeImplicit; time correction of Appendix A.2).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and never by the GPU
library.

The scheme is the trapezoidal-in-time leapfrog
    (W^{n+1} - 2 W^n + W^{n-1}) / dt^2 = (1/2) L_ph (W^{n+1} + W^{n-1})
                                         - f cos(omega_i t^n) cos(omega_i dt),
so every step solves M W^{n+1} = 2 W^n - M W^{n-1} - dt^2 f cos(omega_i t^n)
cos(omega_i dt) with M = I - (dt^2/2) L_ph, here by a sparse LU factorisation
of M on the interior unknowns (the walls stay 0).  The time step and the
corrected frequency follow the implicit correction recipe: for N_t >= 5
steps per period, dt = sqrt(2/cos(2 pi/N_t) - 2) / omega and
omega_i = 2 pi / (N_t dt), which makes cos(omega_i dt) = 1 / (1 + (omega dt)^2/2)
(eq. cosOmegaTilde).  The filter is the explicit scheme's trapezoid filter
over N_t N_p steps with omega_i in place of the explicit corrected frequency.

Readings (also listed in the design notes):
  * The first step eliminates W^{-1} with the initial condition D0t W^0 = 0,
    i.e. W^{-1} = W^1, in the scheme at n = 0:
    M W^1 = W^0 - (dt^2/2) f cos(omega_i dt).
  * alpha_d is tan(pi/N_t) / tan(2 pi/N_t), as for the explicit scheme.
  * With N_p > 1 periods the forcing phase is omega_i t^n = 2 pi n / N_t.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import closed_forms as cf
from . import core as oc


def time_params_implicit(omega: float, nits: int = 10, periods: int = 1) -> dict:
    """Implicit time-stepping correction recipe (Appendix A.2)."""
    if not omega > 0:
        raise ValueError("omega must be positive")
    if nits < 5:
        raise ValueError("the implicit correction needs at least 5 steps per period")
    dt = math.sqrt(2.0 / math.cos(2.0 * math.pi / nits) - 2.0) / omega
    omega_i = 2.0 * math.pi / (nits * dt)
    alpha_d = math.tan(math.pi / nits) / math.tan(2.0 * math.pi / nits)
    return dict(nt=int(nits), dt=dt, omega_e=omega_i, alpha=alpha_d, alpha_d=alpha_d, periods=int(periods),
                omega=float(omega), scheme="implicit")


def lambda_tilde_implicit(lam_h, dt: float):
    """Mode map of eq. (lambdaTildeImplicit): acos(1 / (1 + (lambda dt)^2/2)) / dt."""
    return np.arccos(1.0 / (1.0 + (np.asarray(lam_h) * dt) ** 2 / 2.0)) / dt


def predicted_rate_implicit(grid, c2: float, tp: dict):
    """Theorem on the implicit FPI rate: max |beta_d(lambda~_i)| (constant c^2)."""
    lam = np.sqrt(cf.mode_eigenvalues(grid, c2))
    beta = np.abs(cf.beta_d_tp(lambda_tilde_implicit(lam, tp["dt"]), tp))
    i = int(np.argmax(beta))
    return float(beta.ravel()[i]), float(lam.ravel()[i])


def _interior(grid, a):
    inner = (slice(1, -1),) * grid.dim
    return np.asarray(a, dtype=np.float64)[inner].ravel()


def _c2_interior(grid, c2):
    return np.full(grid.unknowns, float(c2)) if np.isscalar(c2) else _interior(grid, c2)


class ImplicitStepper:
    """M = I - (dt^2/2) C L on the interior unknowns, factorised once."""

    def __init__(self, grid, c2, dt: float):
        self.grid = grid
        L = cf.laplacian_matrix(grid)
        self.CL = sp.diags(_c2_interior(grid, c2)) @ L
        self.M = (sp.identity(L.shape[0]) - 0.5 * dt * dt * self.CL).tocsc()
        self.lu = spla.splu(self.M)

    def solve(self, rhs):
        return self.lu.solve(rhs)

    def mul(self, x):
        return self.M @ x


def apply_implicit(grid, c2, f, v, tp: dict, with_forcing: bool = True, return_final: bool = False,
                   stepper: ImplicitStepper | None = None):
    """One WaveHoltz application W_h(v, s f) with implicit time stepping."""
    dt = tp["dt"]
    N = tp["nt"] * tp["periods"]
    st = stepper or ImplicitStepper(grid, c2, dt)
    fi = _interior(grid, f) if (with_forcing and f is not None) else np.zeros(grid.unknowns)
    cw = math.cos(tp["omega_e"] * dt)
    prev = _interior(grid, v)
    cur = st.solve(prev - 0.5 * dt * dt * cw * fi)
    acc = oc.filter_weight(0, tp) * prev + oc.filter_weight(1, tp) * cur
    for n in range(1, N):
        g = -dt * dt * math.cos(2.0 * math.pi * (n % tp["nt"]) / tp["nt"]) * cw
        nxt = st.solve(2.0 * cur - st.mul(prev) + g * fi)
        acc += oc.filter_weight(n + 1, tp) * nxt
        prev, cur = cur, nxt
    shape = tuple(k - 1 for k in reversed(grid.n))
    out = np.zeros(grid.shape)
    out[(slice(1, -1),) * grid.dim] = acc.reshape(shape)
    if not return_final:
        return out
    fin = np.zeros(grid.shape)
    fin[(slice(1, -1),) * grid.dim] = cur.reshape(shape)
    return out, fin


def apply_A_implicit(grid, c2, v, tp: dict, stepper=None):
    va = np.array(v, dtype=np.float64, copy=True)
    va[~oc.interior_mask(grid)] = 0.0
    return va - apply_implicit(grid, c2, None, va, tp, with_forcing=False, stepper=stepper)


def fpi_implicit(grid, c2, f, tp: dict, iters: int, v0=None):
    """Alg. 1 with implicit steps: v^{k+1} = W_h(v^k, f); returns the iterate
    and the list of iterates."""
    st = ImplicitStepper(grid, c2, tp["dt"])
    v = np.zeros(grid.shape) if v0 is None else np.array(v0, dtype=np.float64)
    hist = []
    for _ in range(iters):
        v = apply_implicit(grid, c2, f, v, tp, stepper=st)
        hist.append(v)
    return v, hist
