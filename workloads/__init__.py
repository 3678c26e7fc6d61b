"""Seeded synthetic inputs for the WaveHoltz solver.

This module only draws numbers: wave-speed fields, Gaussian sources
(eq. gaussianSource of the numerical-results section) and random initial
iterates.  It holds none of the method's arithmetic, so both the GPU tests and
the CPU oracle can be fed from it without sharing any solver code.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` and draws in the
order written in its docstring.  Sizes are parameters, so the tests can use
smaller grids built by the same recipe as the benchmark workloads.  Node arrays
have numpy shape (n_z+1, n_y+1, n_x+1) (or (n_y+1, n_x+1)), x fastest, on the
unit box with n cells per axis; values on wall nodes are set to 0 for sources.
"""
from __future__ import annotations

import numpy as np


def node_coords(dim: int, n: int):
    """Coordinates x, y[, z] of the nodes, each of the node-array shape."""
    ax = np.arange(n + 1, dtype=np.float64) / n
    mesh = np.meshgrid(*([ax] * dim), indexing="ij")  # slowest axis first
    return list(reversed(mesh))  # x, y, z


def _zero_walls(a: np.ndarray) -> np.ndarray:
    for axis in range(a.ndim):
        idx = [slice(None)] * a.ndim
        idx[axis] = 0
        a[tuple(idx)] = 0.0
        idx[axis] = -1
        a[tuple(idx)] = 0.0
    return a


def gaussian(dim: int, n: int, center, amplitude: float, width: float) -> np.ndarray:
    """amplitude * exp(-width * |x - center|^2) on the nodes."""
    xs = node_coords(dim, n)
    r2 = sum((x - c) ** 2 for x, c in zip(xs, center))
    return amplitude * np.exp(-width * r2)


def random_field(shape, seed: int, zero_walls: bool = True) -> np.ndarray:
    """Standard-normal node array (a random initial iterate)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.standard_normal(shape)
    return _zero_walls(a) if zero_walls else a


def single_gaussian_source(dim: int = 2, n: int = 128, omega: float = 10.3):
    """Square with one Gaussian source exp(-200 |x - (0.4, 0.6)|^2), c = 1,
    2nd order, one period, 30 fixed-point iterations, FP64.  No random draws."""
    center = (0.4, 0.6, 0.5)[:dim]
    f = _zero_walls(gaussian(dim, n, center, 1.0, 200.0))
    return dict(name=f"square{dim}d_n{n}_single_gaussian", dim=dim, n=n, order=2, omega=omega,
                periods=1, cfl=0.9, c2=1.0, f=f, fpi_iters=30)


def smooth_random_speed_sources(n: int = 2048, order: int = 4, omega: float = 200.0, seed: int = 2,
                                n_bumps: int = 16, n_sources: int = 4):
    """Square, smooth random c^2 in [0.5, 2], several random Gaussian sources.

    Draw order (one PCG64 stream):
      1. n_bumps amplitudes a_i ~ U[-1, 1]
      2. n_bumps centres x_i ~ U[0, 1]^2 (x then y per bump)
      3. n_bumps widths s_i ~ U[0.05, 0.25]
      4. n_sources amplitude magnitudes ~ U[0.5, 1.5]
      5. n_sources signs (+1 or -1, fair)
      6. n_sources centres ~ U[0.15, 0.85]^2
      7. n_sources exponents b_g ~ U[500, 2000]
    c^2 = 0.5 + 1.5 (g - min g)/(max g - min g) with
    g = sum_i a_i exp(-|x - x_i|^2 / (2 s_i^2)).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(-1.0, 1.0, n_bumps)
    xc = rng.uniform(0.0, 1.0, (n_bumps, 2))
    s = rng.uniform(0.05, 0.25, n_bumps)
    amp = rng.uniform(0.5, 1.5, n_sources)
    sign = np.where(rng.integers(0, 2, n_sources) == 1, 1.0, -1.0)
    sc = rng.uniform(0.15, 0.85, (n_sources, 2))
    bg = rng.uniform(500.0, 2000.0, n_sources)
    x, y = node_coords(2, n)
    g = np.zeros_like(x)
    for i in range(n_bumps):
        g += a[i] * np.exp(-((x - xc[i, 0]) ** 2 + (y - xc[i, 1]) ** 2) / (2.0 * s[i] ** 2))
    c2 = 0.5 + 1.5 * (g - g.min()) / (g.max() - g.min())
    f = np.zeros_like(x)
    for i in range(n_sources):
        f += sign[i] * amp[i] * np.exp(-bg[i] * ((x - sc[i, 0]) ** 2 + (y - sc[i, 1]) ** 2))
    return dict(name=f"square2d_n{n}_p{order}_random_c2", dim=2, n=n, order=order, omega=omega,
                periods=1, cfl=0.9, c2=c2, f=_zero_walls(f), gmres_restart=50, rtol=1e-8)


def cube_inclusion(n: int = 512, order: int = 2, omega: float = 80.0, seed: int = 3):
    """Unit cube, c = 1 with one ball of c = 1.5, point-like Gaussian source.

    Draw order: ball centre ~ U[0.4, 0.7]^3 (x, y, z), then radius ~ U[0.1, 0.2].
    Source: amplitude 1, exponent 5000, centre (0.5, 0.5, 0.15), which lies
    outside every ball the draw can produce.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    center = rng.uniform(0.4, 0.7, 3)
    radius = rng.uniform(0.1, 0.2)
    x, y, z = node_coords(3, n)
    inside = (x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2 <= radius ** 2
    c2 = np.where(inside, 1.5 ** 2, 1.0)
    del inside
    f = _zero_walls(gaussian(3, n, (0.5, 0.5, 0.15), 1.0, 5000.0))
    return dict(name=f"cube_n{n}_p{order}_inclusion", dim=3, n=n, order=order, omega=omega,
                periods=1, cfl=0.9, c2=c2, f=f, ball=(tuple(center), float(radius)))


def batched_problems(count: int = 64, sizes=(256, 512, 1024), omega_range=(20.0, 150.0), seed: int = 4):
    """Many independent 2-D problems: size drawn from `sizes`, omega ~ U[range],
    one random Gaussian source each (c = 1, 2nd order).

    Draw order per problem: size index, omega, source centre (x, y) ~ U[0.2, 0.8]^2,
    exponent ~ U[100, 1000], amplitude ~ U[0.5, 1.5].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(sizes[rng.integers(0, len(sizes))])
        om = float(rng.uniform(*omega_range))
        c = rng.uniform(0.2, 0.8, 2)
        bg = float(rng.uniform(100.0, 1000.0))
        amp = float(rng.uniform(0.5, 1.5))
        out.append(dict(dim=2, n=n, order=2, omega=om, periods=1, cfl=0.9, c2=1.0,
                        source=(tuple(c), bg, amp)))
    return out


def materialise_source(dim: int, n: int, source) -> np.ndarray:
    center, bg, amp = source
    return _zero_walls(gaussian(dim, n, center, amp, bg))


def ring_receivers(n: int, count: int = 128, inset: float = 0.05) -> np.ndarray:
    """Flat node indices (2-D, x fastest) of `count` receivers evenly spaced
    around the square ring `inset` inside the walls, starting at the corner
    (inset, inset) and going counter-clockwise; positions snap to the nearest
    node.  No random draws."""
    per_side = count // 4
    if per_side * 4 != count:
        raise ValueError("count must be a multiple of 4")
    a, b = inset, 1.0 - inset
    t = a + (b - a) * np.arange(per_side) / per_side
    xs = np.concatenate([t, np.full(per_side, b), b + a - t, np.full(per_side, a)])
    ys = np.concatenate([np.full(per_side, a), t, np.full(per_side, b), b + a - t])
    ix = np.rint(xs * n).astype(np.int64)
    iy = np.rint(ys * n).astype(np.int64)
    return iy * (n + 1) + ix


def adjoint_problem(n: int = 1024, omega: float = 60.0, n_sources: int = 8, n_receivers: int = 128,
                    seed: int = 5):
    """Receiver-misfit gradient problem on the unit square, 2nd order:
    background c^2 = 1; the 'true' model lowers c^2 by 0.2 in a Gaussian
    bump 0.2 * exp(-|x - x_b|^2 / (2 * 0.1^2)) (so c_max stays 1 and both
    models share the time step); n_sources Gaussian sources of amplitude 1
    and width b_g = 400; receivers on the ring 0.05 inside the walls.

    Draw order: bump centre x_b ~ U[0.35, 0.65]^2, then per source its
    centre ~ U[0.2, 0.8]^2.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    xb = rng.uniform(0.35, 0.65, 2)
    centres = [tuple(rng.uniform(0.2, 0.8, 2)) for _ in range(n_sources)]
    x, y = node_coords(2, n)
    bump = 0.2 * np.exp(-((x - xb[0]) ** 2 + (y - xb[1]) ** 2) / (2.0 * 0.1 ** 2))
    c2_bg = np.ones((n + 1, n + 1))
    c2_true = c2_bg - bump
    sources = [_zero_walls(gaussian(2, n, c, 1.0, 400.0)) for c in centres]
    return dict(n=n, order=2, omega=omega, periods=1, cfl=0.9, c2_background=c2_bg, c2_true=c2_true,
                sources=sources, receivers=ring_receivers(n, n_receivers), bump_centre=tuple(xb))
