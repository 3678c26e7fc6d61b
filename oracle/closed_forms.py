"""Closed-form results that pin the oracle (test infrastructure only).

Nothing here runs the time stepping.  These are the paper's analytic results
for a single Cartesian grid with constant wave speed, plus a direct sparse
solve of the discrete Helmholtz problem:

  * the discrete filter function beta_d as three approximate sincs
    (Appendix A.3, eqs. discreteBetaThreeSincs and sincd);
  * the Dirichlet sine-mode eigenvalues of the order-p operator, from the
    discrete dispersion relation of Appendix B (eq. disperionRelationOrderp)
    with the b_mu the paper lists after the b_mu theorem of Sec. 6.1;
  * the mode map lambda~ = (2/dt) asin(lambda_h dt / 2) (eq.
    discreteExplicitLambdaTilde) and the closed-form fixed-point iterates
    V^(k) = beta^k V^(0) + (1 - beta^k) U in the sine basis (Sec. 4.2.1,
    eq. waveHoltzFourierFPIexplicit), evaluated with scipy's DST-I;
  * the discrete Helmholtz solution (DHS) of c^2 Delta_{h,p} U + omega^2 U = f
    by scipy.sparse.linalg.spsolve on a matrix assembled from Kronecker sums
    of powers of the 1-D Dirichlet second-difference matrix.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# b_0..b_4 as listed after the b_mu theorem (Sec. 6.1, eq. uxxCoeff).
B_MU_LISTED = (Fraction(1), Fraction(1, 12), Fraction(1, 90), Fraction(1, 560), Fraction(1, 3150))


def sinc_d(z, T: float, dt: float):
    """Approximate sinc of eq. (sincd): sin(zT) / (T tan(z dt/2) / (dt/2)).

    Where tan(z dt/2) vanishes (z dt a multiple of 2 pi, including z = 0) the
    removable singularity takes its limit value 1.
    """
    z = np.asarray(z, dtype=np.float64)
    t = np.tan(z * dt / 2.0)
    small = np.abs(t) < 1e-300
    with np.errstate(divide="ignore", invalid="ignore"):
        val = np.sin(z * T) / (T * t / (dt / 2.0))
    return np.where(small, 1.0, val)


def beta_d(lam, omega_e: float, Tbar: float, dt: float, alpha: float):
    """Discrete filter function, eq. (discreteBetaThreeSincs), over Tbar."""
    return (sinc_d(omega_e + np.asarray(lam), Tbar, dt) + sinc_d(omega_e - np.asarray(lam), Tbar, dt)
            - alpha * sinc_d(lam, Tbar, dt))


def beta_d_tp(lam, tp: dict):
    """beta_d for the time parameters dict returned by oracle.core.time_params."""
    Tbar = tp["periods"] * tp["nt"] * tp["dt"]
    return beta_d(lam, tp["omega_e"], Tbar, tp["dt"], tp["alpha"])


def lambda_h_sq_1d(kappa, h: float, order: int):
    """Eigenvalue of -d^2/dx^2 (order p, Dirichlet) for sine mode sin(kappa x):
    (1/h^2) sum_{mu < p/2} b_mu (4 sin^2(kappa h/2))^{mu+1}."""
    s4 = 4.0 * np.sin(np.asarray(kappa) * h / 2.0) ** 2
    out = np.zeros_like(s4)
    for mu in range(order // 2):
        out = out + float(B_MU_LISTED[mu]) * s4 ** (mu + 1)
    return out / h ** 2


def mode_eigenvalues(grid, c2: float):
    """lambda_h^2 for every sine mode (k_x, k_y, k_z), array of the interior shape
    (slowest axis first)."""
    per_axis = [c2 * lambda_h_sq_1d(np.arange(1, k) * math.pi, 1.0 / k, grid.order) for k in grid.n]
    total = np.zeros(tuple(k - 1 for k in reversed(grid.n)))
    for m, lam in enumerate(per_axis):
        shp = [1] * grid.dim
        shp[grid.dim - 1 - m] = lam.size
        total = total + lam.reshape(shp)
    return total


def lambda_tilde(lam_h, dt: float):
    """Mode map of eq. (discreteExplicitLambdaTilde)."""
    return (2.0 / dt) * np.arcsin(np.asarray(lam_h) * dt / 2.0)


def _dst(a):
    return scipy.fft.dstn(a, type=1)


def _idst(a):
    return scipy.fft.idstn(a, type=1)


def fpi_iterate_closed_form(grid, c2: float, f, omega: float, tp: dict, k: int, v0=None):
    """k-th fixed-point iterate in closed form (constant c^2 only).

    Interior values are expanded in the sine basis (DST-I); each coefficient
    evolves as V <- beta V + (1 - beta) U with U = f^/(omega^2 - lambda_h^2).
    """
    inner = (slice(1, -1),) * grid.dim
    fh = _dst(np.asarray(f, dtype=np.float64)[inner])
    lam2 = mode_eigenvalues(grid, c2)
    U = fh / (omega ** 2 - lam2)
    beta = beta_d_tp(lambda_tilde(np.sqrt(lam2), tp["dt"]), tp)
    V0 = np.zeros_like(U) if v0 is None else _dst(np.asarray(v0, dtype=np.float64)[inner])
    Vk = beta ** k * V0 + (1.0 - beta ** k) * U
    out = np.zeros(grid.shape)
    out[inner] = _idst(Vk)
    return out


def helmholtz_closed_form(grid, c2: float, f, omega: float):
    """DHS for constant c^2 by DST-I diagonalisation."""
    inner = (slice(1, -1),) * grid.dim
    fh = _dst(np.asarray(f, dtype=np.float64)[inner])
    lam2 = mode_eigenvalues(grid, c2)
    out = np.zeros(grid.shape)
    out[inner] = _idst(fh / (omega ** 2 - lam2))
    return out


def predicted_rate(grid, c2: float, tp: dict):
    """Theorem 2 (Sec. 4.2.1): mu = max over modes of |beta_d(lambda~)| (constant c^2).
    Returns (mu, lambda_h at the maximiser)."""
    lam2 = mode_eigenvalues(grid, c2)
    lam = np.sqrt(lam2)
    beta = np.abs(beta_d_tp(lambda_tilde(lam, tp["dt"]), tp))
    i = int(np.argmax(beta))
    return float(beta.ravel()[i]), float(lam.ravel()[i])


def second_difference_1d(n: int, h: float):
    """(n-1)x(n-1) Dirichlet matrix of D+D- on interior nodes."""
    m = n - 1
    return sp.diags([np.ones(m - 1), -2.0 * np.ones(m), np.ones(m - 1)], [-1, 0, 1]) / h ** 2


def laplacian_matrix(grid):
    """Order-p Dirichlet Laplacian on interior unknowns (x fastest ordering):
    per axis sum_{mu<p/2} b_mu (-h^2)^mu T^{mu+1} with T the D+D- matrix, then
    a Kronecker sum over the axes."""
    mats = []
    for k in grid.n:
        h = 1.0 / k
        T = second_difference_1d(k, h).tocsr()
        acc = sp.csr_matrix((k - 1, k - 1))
        P = T
        for mu in range(grid.order // 2):
            acc = acc + float(B_MU_LISTED[mu]) * (-h * h) ** mu * P
            P = P @ T
        mats.append(acc)
    sizes = [k - 1 for k in grid.n]
    total = None
    for m in range(grid.dim):
        left = sp.identity(int(np.prod(sizes[m + 1:])) if m + 1 < grid.dim else 1)
        right = sp.identity(int(np.prod(sizes[:m])) if m > 0 else 1)
        term = sp.kron(sp.kron(left, mats[m]), right)
        total = term if total is None else total + term
    return total.tocsr()


def dhs_direct(grid, c2, f, omega: float):
    """Solve c^2 Delta_{h,p} U + omega^2 U = f (U = 0 on the walls) directly."""
    inner = (slice(1, -1),) * grid.dim
    L = laplacian_matrix(grid)
    c2i = (np.full(grid.shape, float(c2)) if np.isscalar(c2) else np.asarray(c2))[inner].ravel()
    A = sp.diags(c2i) @ L + omega ** 2 * sp.identity(L.shape[0])
    u = spla.spsolve(A.tocsc(), np.asarray(f, dtype=np.float64)[inner].ravel())
    out = np.zeros(grid.shape)
    out[inner] = u.reshape(tuple(k - 1 for k in reversed(grid.n)))
    return out


def ppw(p: int, n_lambda: float, eps: float) -> float:
    """Points-per-wavelength rule (Sec. 6.2, eq. ppwPollution): PPW_p = 2 pi (pi b_{p/2})^{1/p} (N_Lambda/eps)^{1/p}."""
    return 2.0 * math.pi * (math.pi * float(B_MU_LISTED[p // 2])) ** (1.0 / p) * (n_lambda / eps) ** (1.0 / p)
