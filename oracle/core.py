"""Double-precision CPU oracle for the explicit WaveHoltz hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the package smoke check and
the CPU-baseline leg of ``bench.py``; never by the GPU library.

The heavy per-node loops (the operator L_ph and the time stepping of one
WaveHoltz application) live in ``wh_oracle.c``; the outer iterations (the
fixed-point iteration of Alg. 1 and restarted GMRES on the Krylov form of
Sec. 5.3) are written here in numpy.  The time parameters follow the explicit
time-correction recipe (Appendix A.1), the stability limit of
eq. (dtForCartesian) and the adjusted filter parameter of eq. (alphad).

Readings of points where the paper is silent (each is listed in the design
notes as well):
  * n is the number of cells per axis, h = 1/n, nodes 0..n.
  * The explicit stability limit is c_max * dt * sqrt(sum_m h_m^-2) <= C_{2,p}
    with C_{2,2} = 1 and C_{2,4} = sqrt(3)/2 (the non-squared form, which is
    the one these constants belong to); "CFL 0.9" scales C_{2,p} by 0.9.
  * c_max is taken over interior nodes.
  * The recipe's first estimate is Nt = ceil(T / dt_max); Nt is then raised
    until dt = (2/omega) sin(pi/Nt) meets the limit, and is never below 5 so
    that the adjusted filter parameter stays positive.
  * For Np > 1 periods the filter runs over Tbar = Np * 2pi/omega_e with the
    same alpha_d.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

C22 = 1.0                  # stability constant C_{2,2} (Sec. 3.2)
C24 = math.sqrt(3.0) / 2.0  # stability constant C_{2,4} (Sec. 3.2)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    default = os.path.join(_HERE, "liboracle.so")
    if _LIB_PATH == default and (not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "wh_oracle.c")))):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.orc_b_mu.restype = ctypes.c_double
    lib.orc_b_mu.argtypes = [ctypes.c_int]
    lib.orc_filter_weight.restype = ctypes.c_double
    lib.orc_filter_weight.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double]
    lib.orc_laplacian.restype = ctypes.c_int
    lib.orc_laplacian.argtypes = [ctypes.c_int, i64p, dp, ctypes.c_int, dp, dp, dp]
    lib.orc_apply.restype = ctypes.c_int
    lib.orc_apply.argtypes = [ctypes.c_int, i64p, dp, ctypes.c_int, dp, dp, dp,
                              ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_int, dp, dp]
    lib.orc_helmholtz_residual.restype = ctypes.c_int
    lib.orc_helmholtz_residual.argtypes = [ctypes.c_int, i64p, dp, ctypes.c_int, dp, dp, dp,
                                           ctypes.c_double, dp]
    lib.orc_max_threads.restype = ctypes.c_int
    lib.orc_max_threads.argtypes = []
    lib.orc_set_threads.restype = None
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def use_library(path: str):
    """Load the oracle's routines from another build of ``wh_oracle.c``.

    Used only by the tests that plant a mistake in a copy of the C source to
    show that the pins catch it; returns the previously loaded library so the
    caller can restore it with ``restore_library``."""
    global _lib, _LIB_PATH
    prev = (_lib, _LIB_PATH)
    _lib, _LIB_PATH = None, path
    _load()
    return prev


def restore_library(prev):
    global _lib, _LIB_PATH
    _lib, _LIB_PATH = prev


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c_grid(grid: "Grid", h=None):
    n = (ctypes.c_int64 * 3)(*(list(grid.n) + [0] * (3 - grid.dim)))
    hh = grid.h if h is None else tuple(h)
    hv = (ctypes.c_double * 3)(*(list(hh) + [1.0] * (3 - grid.dim)))
    return n, hv


@dataclass(frozen=True)
class Grid:
    """Cartesian grid on the unit box [0,1]^dim with n[m] cells per axis."""
    dim: int
    n: tuple
    order: int

    @property
    def h(self):
        return tuple(1.0 / k for k in self.n)

    @property
    def shape(self):
        """numpy shape of a node array (slowest axis first, x fastest)."""
        return tuple(k + 1 for k in reversed(self.n))

    @property
    def unknowns(self):
        return int(np.prod([k - 1 for k in self.n]))

    @property
    def nodes(self):
        return int(np.prod([k + 1 for k in self.n]))


def b_mu(mu: int) -> float:
    """b_mu of eq. (uxxCoeff), Sec. 6.1, as the C oracle computes it."""
    return float(_load().orc_b_mu(int(mu)))


def interior_mask(grid: Grid) -> np.ndarray:
    m = np.zeros(grid.shape, dtype=bool)
    m[(slice(1, -1),) * grid.dim] = True
    return m


def coords(grid: Grid):
    """Node coordinates as arrays of the node shape, in x, y, z order."""
    axes = [np.arange(k + 1) / k for k in grid.n]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")
    return list(reversed(mesh))


# ---------------------------------------------------------------------------
# time parameters: stability limit (eq. dtForCartesian), explicit correction
# recipe (Appendix A.1), eq. alphad
# ---------------------------------------------------------------------------
def stability_constant(order: int) -> float:
    if order == 2:
        return C22
    if order == 4:
        return C24
    raise ValueError("stability constant known for p = 2 and p = 4 only")


def time_params(grid: Grid, c2, omega: float, periods: int = 1, cfl_frac: float = 0.9,
                nt: int | None = None, alpha: float | None = None) -> dict:
    """Explicit time-stepping correction recipe (Appendix A.1) for frequency omega.

    c2 is a node array (or a scalar for constant speed).  Returns a dict with
    nt, dt, omega_e (the adjusted frequency), alpha (alpha_d unless given),
    periods, nu (the CFL number c_max dt sqrt(sum h^-2)) and c_max.
    """
    if not omega > 0:
        raise ValueError("omega must be positive")
    if np.isscalar(c2):
        c2max = float(c2)
    else:
        c2max = float(np.max(np.asarray(c2)[interior_mask(grid)]))
    cmax = math.sqrt(c2max)
    root = math.sqrt(sum(1.0 / hm ** 2 for hm in grid.h))
    nu_max = cfl_frac * stability_constant(grid.order)
    dt_max = nu_max / (cmax * root)
    period = 2.0 * math.pi / omega
    if nt is None:
        nt = max(5, math.ceil(period / dt_max))
        while (2.0 / omega) * math.sin(math.pi / nt) > dt_max:
            nt += 1
    dt = (2.0 / omega) * math.sin(math.pi / nt)
    omega_e = 2.0 * math.pi / (nt * dt)
    alpha_d = math.tan(omega_e * dt / 2.0) / math.tan(omega_e * dt)
    nu = cmax * dt * root
    return dict(nt=int(nt), dt=dt, omega_e=omega_e, alpha=alpha_d if alpha is None else float(alpha),
                alpha_d=alpha_d, periods=int(periods), nu=nu, c_max=cmax, omega=float(omega),
                stable=nu <= stability_constant(grid.order))


def filter_weight(n: int, tp: dict) -> float:
    """Trapezoid weight of time level n, as the C oracle applies it."""
    return float(_load().orc_filter_weight(int(n), int(tp["nt"] * tp["periods"]), tp["dt"],
                                           tp["omega_e"], tp["alpha"]))


# ---------------------------------------------------------------------------
# operators
# ---------------------------------------------------------------------------
def _prep(grid: Grid, a, name: str) -> np.ndarray:
    if a is None:
        return None
    if np.isscalar(a):
        return np.full(grid.shape, float(a))
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != grid.shape:
        raise ValueError(f"{name}: expected shape {grid.shape}, got {a.shape}")
    return a


def laplacian(grid: Grid, c2, W, h=None) -> np.ndarray:
    """L_ph W = c^2 Delta_{h,p} W on interior nodes, 0 on the walls."""
    lib = _load()
    c2a, Wa = _prep(grid, c2, "c2"), _prep(grid, W, "W")
    out = np.empty(grid.shape)
    n, hv = _c_grid(grid, h)
    if lib.orc_laplacian(grid.dim, n, hv, grid.order, _dptr(c2a), _dptr(Wa), _dptr(out)):
        raise ValueError("orc_laplacian rejected its arguments")
    return out


def apply(grid: Grid, c2, f, v, tp: dict, with_forcing: bool = True, return_final: bool = False,
          h=None):
    """One WaveHoltz application W_h(v, s f) (Alg. 1 loop body, Sec. 4.2.1)."""
    lib = _load()
    c2a = _prep(grid, c2, "c2")
    fa = _prep(grid, 0.0 if f is None else f, "f")
    va = _prep(grid, v, "v")
    out = np.empty(grid.shape)
    fin = np.empty(grid.shape) if return_final else None
    n, hv = _c_grid(grid, h)
    rc = lib.orc_apply(grid.dim, n, hv, grid.order, _dptr(c2a), _dptr(fa), _dptr(va),
                       tp["nt"], tp["periods"], tp["dt"], tp["omega_e"], tp["alpha"],
                       1 if with_forcing else 0, _dptr(out),
                       _dptr(fin) if fin is not None else None)
    if rc:
        raise ValueError(f"orc_apply failed with {rc}")
    return (out, fin) if return_final else out


def apply_A(grid: Grid, c2, v, tp: dict) -> np.ndarray:
    """Matrix-free A v = v - W_h(v, 0) (Sec. 5.3, eq. MevalII); 0 on the walls."""
    va = _prep(grid, v, "v").copy()
    va[~interior_mask(grid)] = 0.0
    return va - apply(grid, c2, None, va, tp, with_forcing=False)


def helmholtz_residual(grid: Grid, c2, f, u, omega: float) -> np.ndarray:
    lib = _load()
    c2a, fa, ua = _prep(grid, c2, "c2"), _prep(grid, f, "f"), _prep(grid, u, "u")
    out = np.empty(grid.shape)
    n, hv = _c_grid(grid)
    if lib.orc_helmholtz_residual(grid.dim, n, hv, grid.order, _dptr(c2a), _dptr(fa), _dptr(ua),
                                  float(omega), _dptr(out)):
        raise ValueError("orc_helmholtz_residual rejected its arguments")
    return out


def apply_at_points(grid: Grid, c2, f, v, tp: dict, points, with_forcing: bool = True):
    """W_h(v, s f) at selected nodes only, each computed on the sub-box that
    holds its domain of dependence.

    After N explicit steps a node depends only on data within N*r cells
    (r = p/2 per step), so the apply is run on the box of half-width
    (N+1)*r around the node, clipped to the grid.  Sides clipped by a wall
    keep the true wall condition; the other sides carry a zero condition whose
    influence travels r cells per step and never reaches the centre.
    """
    c2a = _prep(grid, c2, "c2")
    fa = _prep(grid, 0.0 if f is None else f, "f")
    va = _prep(grid, v, "v")
    r = grid.order // 2
    half = (tp["nt"] * tp["periods"] + 1) * r
    out = []
    for p in points:
        p = tuple(int(x) for x in p)  # x, y, z order
        lo = [max(0, p[m] - half) for m in range(grid.dim)]
        hi = [min(grid.n[m], p[m] + half) for m in range(grid.dim)]
        sub = Grid(grid.dim, tuple(hi[m] - lo[m] for m in range(grid.dim)), grid.order)
        sl = tuple(slice(lo[m], hi[m] + 1) for m in reversed(range(grid.dim)))
        res = apply(sub, c2a[sl], fa[sl], va[sl], tp, with_forcing=with_forcing, h=grid.h)
        loc = tuple(p[m] - lo[m] for m in reversed(range(grid.dim)))
        out.append(res[loc])
    return np.array(out)


# ---------------------------------------------------------------------------
# outer iterations
# ---------------------------------------------------------------------------
def fpi(grid: Grid, c2, f, tp: dict, iters: int, v0=None, callback=None):
    """WaveHoltz fixed-point iteration (Alg. 1) for a fixed iteration count.

    Returns (v, hist) where hist[k] = ||v^{k+1} - v^k||_2 for k = 0..iters-1.
    """
    v = np.zeros(grid.shape) if v0 is None else _prep(grid, v0, "v0").copy()
    hist = []
    for k in range(iters):
        vn = apply(grid, c2, f, v, tp, with_forcing=True)
        hist.append(float(np.linalg.norm(vn - v)))
        v = vn
        if callback:
            callback(k, v)
    return v, np.array(hist)


def gmres(grid: Grid, c2, f, tp: dict, restart: int = 50, rtol: float = 1e-8, maxit: int = 1000,
          x0=None, fixed_iters: int | None = None, b=None):
    """Restarted GMRES(m) on (I - S_h) v = b with b = W_h(0, f) (Sec. 5.3).

    Textbook Arnoldi with modified Gram-Schmidt and Givens rotations; x0 = 0
    unless given.  Stops when ||b - A x||_2 <= rtol ||b||_2 (true residual at
    each restart) or after maxit Arnoldi steps; with fixed_iters it performs
    exactly that many Arnoldi steps (restarting every `restart`) and returns
    the iterate.  Returns (x, info) with info = dict(iters, rel_res, hist).
    """
    mask = interior_mask(grid)
    if b is None:
        b = apply(grid, c2, f, np.zeros(grid.shape), tp, with_forcing=True)
    b = np.asarray(b, dtype=np.float64).ravel()
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(b.size) if x0 is None else _prep(grid, x0, "x0").ravel().copy()
    x[~mask.ravel()] = 0.0

    def A(vec):
        return apply_A(grid, c2, vec.reshape(grid.shape), tp).ravel()

    hist = []
    total = 0
    limit = fixed_iters if fixed_iters is not None else maxit
    while True:
        r = b - A(x)
        beta = float(np.linalg.norm(r))
        rel = beta / bnorm if bnorm > 0 else 0.0
        hist.append(rel)
        if fixed_iters is None and (rel <= rtol or total >= limit):
            break
        if fixed_iters is not None and total >= limit:
            break
        if beta == 0.0:
            break
        m = min(restart, limit - total)
        V = np.zeros((m + 1, b.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        for j in range(m):
            w = A(V[j])
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            hnext = float(np.linalg.norm(w))
            H[j + 1, j] = hnext
            if hnext != 0.0:
                V[j + 1] = w / hnext
            for i in range(j):  # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            denom = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / denom
            sn[j] = H[j + 1, j] / denom
            H[j, j] = denom
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k_used = j + 1
            total += 1
            if fixed_iters is None and abs(g[j + 1]) <= rtol * bnorm:
                break
            if hnext == 0.0:  # lucky breakdown: the Krylov space is invariant
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
        x = x + V[:k_used].T @ y
    return x.reshape(grid.shape), dict(iters=total, rel_res=hist[-1], hist=hist, bnorm=bnorm)


def cg(grid: Grid, c2, f, tp: dict, rtol: float = 1e-8, maxit: int = 1000, x0=None,
       fixed_iters: int | None = None, b=None):
    """Conjugate gradients on (I - S_h) v = b, b = W_h(0, f), in the inner
    product <u, w> = sum_i u_i w_i / c^2_i.

    S_h is a polynomial in c^2 Delta_h, which is self-adjoint in that inner
    product, and its eigenvalues are beta_d in [-1/2, 1] (Sec. 4.2.1 and
    Sec. 5.3), so I - S_h is positive semi-definite there.  Textbook
    Hestenes-Stiefel recurrences; stops when the recursively updated residual
    satisfies ||r||_2 <= rtol ||b||_2, or after exactly fixed_iters iterations.
    Returns (x, info) with info = dict(iters, rel_res (true residual), hist).
    """
    mask = interior_mask(grid)
    wgt = 1.0 / (np.full(grid.shape, float(c2)) if np.isscalar(c2) else np.asarray(c2, dtype=np.float64))
    ip = lambda a, b: float(np.sum(a * b * wgt))
    A = lambda vec: apply_A(grid, c2, vec, tp)
    if b is None:
        b = apply(grid, c2, f, np.zeros(grid.shape), tp, with_forcing=True)
    b = np.asarray(b, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(grid.shape) if x0 is None else _prep(grid, x0, "x0").copy()
    x[~mask] = 0.0
    r = b - A(x)
    p = r.copy()
    rr = ip(r, r)
    hist = [float(np.linalg.norm(r)) / bnorm]
    limit = fixed_iters if fixed_iters is not None else maxit
    k = 0
    while k < limit:
        if fixed_iters is None and hist[-1] <= rtol:
            break
        q = A(p)
        alpha = rr / ip(p, q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = ip(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        k += 1
        hist.append(float(np.linalg.norm(r)) / bnorm)
    true_rel = float(np.linalg.norm(b - A(x))) / bnorm
    return x, dict(iters=k, rel_res=true_rel, hist=hist, bnorm=bnorm)


def max_threads() -> int:
    return int(_load().orc_max_threads())


def set_threads(n: int) -> None:
    """Thread count of the C oracle's parallel loops (for timing)."""
    _load().orc_set_threads(int(n))
