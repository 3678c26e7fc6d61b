"""Double-precision CPU oracle of the discrete adjoint of one WaveHoltz
application and of the fixed-point problem.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and never by the GPU
library.

What is differentiated.  One application Y = W_h(v, f) of Sec. 4.2.1 is the
explicit leapfrog (eq. WaveSchemeexplicit) started from W^0 = v with zero
velocity,

    W^1     = W^0 + (dt^2/2) (L W^0 - f),
    W^{n+1} = 2 W^n - W^{n-1} + dt^2 (L W^n - f cos(omega_e t^n)),

with L W = c^2 Delta_h W (interior nodes; walls held at 0), followed by the
trapezoid filter Y = sum_n w_n W^n (eq. updateDiscreteExplicit).  The
solution of the fixed-point problem of Alg. 1 is v* = W_h(v*, f), i.e.
(I - S) v* = b with S v = W_h(v, 0).  For a misfit J(v*):

    (I - S)^T lam = dJ/dv,      dJ/dtheta = lam . (d/dtheta) W_h(v*, f; theta)

with the time parameters (dt, N_t, omega_e, alpha) held fixed.

How it is computed here: the plain reverse-mode recursion of the scheme,
written with explicit transposes.  With Z^n = d(lam . Y)/dW^n,

    Z^n = w_n lam + 2 Z^{n+1} - Z^{n+2} + dt^2 L^T Z^{n+1},   n = N .. 1,
    Z^0 = w_0 lam + Z^1 + (dt^2/2) L^T Z^1 - Z^2,

where L^T Z = Delta_h (c^2 Z) (Delta_h with the odd wall reflection is
symmetric on interior nodes), and the parameter sensitivities collect

    dJ/dc^2 = sum_{n=0}^{N-1} kappa_n Z^{n+1} * (dt^2 Delta_h W^n),
    dJ/df   = sum_{n=0}^{N-1} gamma_n Z^{n+1},

kappa_0 = 1/2, kappa_n = 1; gamma_0 = -dt^2/2, gamma_n = -dt^2 cos(omega_e t^n).
The forward levels W^n are stored whole (no checkpointing): the oracle only
runs on small grids.
"""
from __future__ import annotations

import math

import numpy as np

from . import core as oc


def _interior(grid, a):
    a = np.array(a, dtype=np.float64, copy=True)
    a[~oc.interior_mask(grid)] = 0.0
    return a


def _c2_array(grid, c2):
    return np.full(grid.shape, float(c2)) if np.isscalar(c2) else np.asarray(c2, dtype=np.float64)


def weights(tp):
    """w_n, n = 0..N, as the forward oracle applies them."""
    N = tp["nt"] * tp["periods"]
    return [oc.filter_weight(n, tp) for n in range(N + 1)]


def forcing_coefficients(tp):
    """gamma_n, n = 0..N-1: the coefficient of f in the update producing W^{n+1}."""
    N = tp["nt"] * tp["periods"]
    dt = tp["dt"]
    return [-0.5 * dt * dt] + [-dt * dt * math.cos(tp["omega_e"] * n * dt) for n in range(1, N)]


def trajectory(grid, c2, f, v, tp, with_forcing=True):
    """Every level W^0..W^N of one application (list of node arrays)."""
    N = tp["nt"] * tp["periods"]
    dt2 = tp["dt"] ** 2
    fi = _interior(grid, 0.0 if f is None or not with_forcing else f)
    gam = forcing_coefficients(tp)
    W = [_interior(grid, v)]
    W.append(W[0] + 0.5 * dt2 * oc.laplacian(grid, c2, W[0]) + gam[0] * fi)
    for n in range(1, N):
        W.append(2.0 * W[n] - W[n - 1] + dt2 * oc.laplacian(grid, c2, W[n]) + gam[n] * fi)
    return W


def _LT(grid, c2, Z):
    """L^T Z = Delta_h (c^2 Z) on interior nodes (walls 0)."""
    return oc.laplacian(grid, 1.0, _interior(grid, _c2_array(grid, c2) * Z))


def reverse_sweep(grid, c2, lam, tp):
    """Z^0..Z^N of the recursion above for the cotangent lam on Y."""
    N = tp["nt"] * tp["periods"]
    dt2 = tp["dt"] ** 2
    w = weights(tp)
    lam = _interior(grid, lam)
    Z = [None] * (N + 3)
    Z[N + 1] = np.zeros(grid.shape)
    Z[N + 2] = np.zeros(grid.shape)
    for n in range(N, 0, -1):
        Z[n] = w[n] * lam + 2.0 * Z[n + 1] - Z[n + 2] + dt2 * _LT(grid, c2, Z[n + 1])
    Z[0] = _interior(grid, w[0] * lam + Z[1] + 0.5 * dt2 * _LT(grid, c2, Z[1]) - Z[2])
    return Z[: N + 1]


def apply_transpose(grid, c2, lam, tp):
    """S^T lam, the transpose of v -> W_h(v, 0) (walls 0)."""
    return reverse_sweep(grid, c2, lam, tp)[0]


def parameter_gradient(grid, c2, f, v, lam, tp):
    """Sensitivities of lam . W_h(v, f) with respect to c^2 and f at fixed time
    parameters, and with respect to v.  Returns (d_c2, d_f, d_v), walls 0."""
    N = tp["nt"] * tp["periods"]
    dt2 = tp["dt"] ** 2
    W = trajectory(grid, c2, f, v, tp)
    Z = reverse_sweep(grid, c2, lam, tp)
    gam = forcing_coefficients(tp)
    d_c2 = np.zeros(grid.shape)
    d_f = np.zeros(grid.shape)
    for n in range(N):
        kappa = 0.5 if n == 0 else 1.0
        d_c2 += kappa * Z[n + 1] * (dt2 * oc.laplacian(grid, 1.0, W[n]))
        d_f += gam[n] * Z[n + 1]
    return _interior(grid, d_c2), _interior(grid, d_f), Z[0]


def solve_adjoint(grid, c2, g, tp, rtol=1e-12, maxit=200, dense_limit=2500):
    """lam with (I - S)^T lam = g (walls of g ignored).  Up to `dense_limit`
    unknowns the matrix I - S^T is assembled column by column from
    apply_transpose and solved directly (LAPACK); beyond that, GMRES on the
    operator (library Krylov routine, relative tolerance rtol)."""
    mask = oc.interior_mask(grid)
    m = int(mask.sum())

    def mv(x):
        full = np.zeros(grid.shape)
        full[mask] = x
        return (full - apply_transpose(grid, c2, full, tp))[mask]

    rhs = np.asarray(g, dtype=np.float64)[mask]
    if m <= dense_limit:
        M = np.empty((m, m))
        e = np.zeros(m)
        for i in range(m):
            e[i] = 1.0
            M[:, i] = mv(e)
            e[i] = 0.0
        x = np.linalg.solve(M, rhs)
    else:
        import scipy.sparse.linalg as sla
        op = sla.LinearOperator((m, m), matvec=mv, dtype=np.float64)
        x, info = sla.gmres(op, rhs, rtol=rtol, atol=0.0, restart=200, maxiter=maxit)
        if info != 0:
            raise RuntimeError(f"adjoint GMRES did not converge (info={info})")
    lam = np.zeros(grid.shape)
    lam[mask] = x
    return lam


def receiver_misfit(u, idx, data):
    """J = 1/2 sum_r (u[idx_r] - d_r)^2 and dJ/du (flat receiver indices)."""
    uf = np.asarray(u, dtype=np.float64).ravel()
    r = uf[np.asarray(idx)] - np.asarray(data, dtype=np.float64)
    g = np.zeros_like(uf)
    np.add.at(g, np.asarray(idx), r)
    return 0.5 * float(np.dot(r, r)), g.reshape(np.shape(u))
