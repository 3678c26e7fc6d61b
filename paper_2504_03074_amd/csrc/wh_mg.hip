// Implicit time stepping (Sec. 4.2.2, eq. WaveSchemeImplicit) on 2-D grids:
// the right-hand side of each step, the filter update, and the geometric
// multigrid V-cycle that preconditions conjugate gradients on the step's
// linear system.
//
// Each implicit step solves M W^{n+1} = R with M = I - theta c^2 Delta_{h,p},
// theta = dt^2 / 2.  M is self-adjoint in the 1/c^2-weighted inner product,
// so the library solves the symmetric form
//     S X = D R,   S = D + theta A_p,   D = diag(1/c^2),  A_p = -Delta_{h,p},
// which is symmetric positive definite.  With the stencil sums of the
// explicit kernels (S_m the symmetric neighbour sum along axis m),
//     S x = (d + ac) x - ax S_x(x) - ay S_y(x)
// with ax = theta n_x^2 (/12 for p = 4), ac = 2 (ax + ay) (30 (ax + ay) for
// p = 4).  Order-4 stencils use the odd reflection across the walls.  Coarse
// levels (every second node) use the 2nd-order operator with 1/c^2 injected;
// the smoother is damped Jacobi, restriction full weighting, prolongation
// bilinear interpolation (4 x the transpose of the restriction), so the
// V-cycle with equal pre- and post-smoothing is a symmetric preconditioner.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wh_internal.h"

namespace wh {
namespace {

constexpr int kMgBlock = 256;

__device__ __forceinline__ bool mg_node(const MgGeom &g, int64_t id, int &i, int &j) {
  i = (int)(id % g.sy);
  j = (int)(id / g.sy);
  return i > 0 && i < g.nx && j > 0 && j < g.ny;
}

// (S x)(i, j) at an interior node; x is 0 on the walls.
__device__ __forceinline__ double mg_S(const MgGeom &g, const double *__restrict__ x, int64_t id, int i, int j,
                                       double d) {
  const double c = x[id];
  double sx, sy;
  if (g.order == 2) {
    sx = x[id - 1] + x[id + 1];
    sy = x[id - g.sy] + x[id + g.sy];
  } else {
    const double xm2 = i >= 2 ? x[id - 2] : -x[id];  // odd reflection across x = 0
    const double xp2 = i <= g.nx - 2 ? x[id + 2] : -x[id];
    const double ym2 = j >= 2 ? x[id - 2 * g.sy] : -x[id];
    const double yp2 = j <= g.ny - 2 ? x[id + 2 * g.sy] : -x[id];
    sx = 16.0 * (x[id - 1] + x[id + 1]) - (xm2 + xp2);
    sy = 16.0 * (x[id - g.sy] + x[id + g.sy]) - (ym2 + yp2);
  }
  return (d + g.ac) * c - g.ax * sx - g.ay * sy;
}

__device__ __forceinline__ double mg_d(const double *__restrict__ dinv, double dconst, int64_t id) {
  return dinv ? dinv[id] : dconst;
}

// x_out = x_in + w (b - S x_in) / diag(S); x_in == nullptr means x_in = 0.
__global__ void mg_smooth_kernel(MgGeom g, const double *__restrict__ dinv, double dconst,
                                 const double *__restrict__ x_in, const double *__restrict__ b,
                                 double *__restrict__ x_out, double w) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= g.nodes) return;
  int i, j;
  if (!mg_node(g, id, i, j)) {
    x_out[id] = 0.0;
    return;
  }
  const double d = mg_d(dinv, dconst, id);
  const double diag = d + g.ac;
  if (x_in) x_out[id] = x_in[id] + w * (b[id] - mg_S(g, x_in, id, i, j, d)) / diag;
  else x_out[id] = w * b[id] / diag;
}

// r = b - S x (b == nullptr: r = S x); walls 0.
__global__ void mg_residual_kernel(MgGeom g, const double *__restrict__ dinv, double dconst,
                                   const double *__restrict__ x, const double *__restrict__ b,
                                   double *__restrict__ r) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= g.nodes) return;
  int i, j;
  if (!mg_node(g, id, i, j)) {
    r[id] = 0.0;
    return;
  }
  const double s = mg_S(g, x, id, i, j, mg_d(dinv, dconst, id));
  r[id] = b ? b[id] - s : s;
}

// Full weighting onto the coarse grid (coarse node (I, J) = fine (2I, 2J)).
__global__ void mg_restrict_kernel(MgGeom gf, const double *__restrict__ rf, MgGeom gc, double *__restrict__ bc) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= gc.nodes) return;
  int I, J;
  if (!mg_node(gc, id, I, J)) {
    bc[id] = 0.0;
    return;
  }
  const int64_t f = (int64_t)(2 * I) + (int64_t)(2 * J) * gf.sy;
  const double edge = rf[f - 1] + rf[f + 1] + rf[f - gf.sy] + rf[f + gf.sy];
  const double corner = rf[f - gf.sy - 1] + rf[f - gf.sy + 1] + rf[f + gf.sy - 1] + rf[f + gf.sy + 1];
  bc[id] = 0.25 * rf[f] + 0.125 * edge + 0.0625 * corner;
}

// x_f += bilinear interpolation of x_c (coarse walls are 0).
__global__ void mg_prolong_kernel(MgGeom gc, const double *__restrict__ xc, MgGeom gf, double *__restrict__ xf) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= gf.nodes) return;
  int i, j;
  if (!mg_node(gf, id, i, j)) return;
  const int I0 = i >> 1, J0 = j >> 1;
  const int I1 = I0 + (i & 1), J1 = J0 + (j & 1);
  const double v = 0.25 * (xc[I0 + (int64_t)J0 * gc.sy] + xc[I1 + (int64_t)J0 * gc.sy] +
                           xc[I0 + (int64_t)J1 * gc.sy] + xc[I1 + (int64_t)J1 * gc.sy]);
  xf[id] += v;
}

// coarse 1/c^2 by injection
__global__ void mg_inject_kernel(MgGeom gf, const double *__restrict__ df, MgGeom gc, double *__restrict__ dc) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= gc.nodes) return;
  const int I = (int)(id % gc.sy), J = (int)(id / gc.sy);
  dc[id] = df[(int64_t)(2 * I) + (int64_t)(2 * J) * gf.sy];
}

// d = 1 / c^2 on every node (walls: 1, never used)
__global__ void mg_inverse_kernel(MgGeom g, const double *__restrict__ c2, double *__restrict__ d) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= g.nodes) return;
  int i, j;
  d[id] = mg_node(g, id, i, j) ? 1.0 / c2[id] : 1.0;
}

// Right-hand side of an implicit step in the symmetric form and the initial
// guess of the solve:
//   first step (prev == nullptr):  B = d (W^0 + gn f),               X0 = W^0
//   later steps:                   B = d (2 W^n + gn f) - S W^{n-1},  X0 = 2 W^n - W^{n-1}
// (S W^{n-1} = d M W^{n-1}); walls 0.
__global__ void imp_rhs_kernel(MgGeom g, const double *__restrict__ dinv, double dconst,
                               const double *__restrict__ cur, const double *__restrict__ prev,
                               const double *__restrict__ f, double gn, double *__restrict__ B,
                               double *__restrict__ X0) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= g.nodes) return;
  int i, j;
  if (!mg_node(g, id, i, j)) {
    B[id] = 0.0;
    X0[id] = 0.0;
    return;
  }
  const double d = mg_d(dinv, dconst, id);
  const double fv = f ? gn * f[id] : 0.0;
  if (!prev) {
    B[id] = d * (cur[id] + fv);
    X0[id] = cur[id];
  } else {
    B[id] = d * (2.0 * cur[id] + fv) - mg_S(g, prev, id, i, j, d);
    X0[id] = 2.0 * cur[id] - prev[id];
  }
}

// Filter update with the new level x: ACCUMULATE acc (+)= w x (init: =),
// FINAL_FILTER out = acc + w x, FINAL_A out = v - (acc + w x); walls 0.
__global__ void imp_filter_kernel(int64_t n, const double *__restrict__ x, double w, double *__restrict__ acc,
                                  int init, int mode, const double *__restrict__ v, double *__restrict__ out,
                                  MgGeom g) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  int i, j;
  const bool inner = mg_node(g, id, i, j);
  const double a = (init ? 0.0 : acc[id]) + w * x[id];
  if (mode == ACCUMULATE) acc[id] = a;
  else if (mode == FINAL_FILTER) out[id] = inner ? a : 0.0;
  else out[id] = inner ? v[id] - a : 0.0;
}

// x += alpha p, r -= alpha q (alpha = num / den, device scalars)
__global__ void pcg_update_kernel(int64_t n, double *__restrict__ x, double *__restrict__ r,
                                  const double *__restrict__ p, const double *__restrict__ q,
                                  const double *__restrict__ num, const double *__restrict__ den) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const double alpha = *num / *den;
  x[id] += alpha * p[id];
  r[id] -= alpha * q[id];
}

// p = z + beta p (beta = num / den, device scalars; den == nullptr: beta = 0)
__global__ void pcg_xpay_kernel(int64_t n, const double *__restrict__ z, double *__restrict__ p,
                                const double *__restrict__ num, const double *__restrict__ den) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n) return;
  const double beta = den ? *num / *den : 0.0;
  p[id] = z[id] + beta * p[id];
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kMgBlock - 1) / kMgBlock); }

}  // namespace

hipError_t launch_mg_smooth(const MgGeom &g, const double *dinv, double dconst, const double *x_in,
                            const double *b, double *x_out, double w, hipStream_t s) {
  mg_smooth_kernel<<<blocks_for(g.nodes), kMgBlock, 0, s>>>(g, dinv, dconst, x_in, b, x_out, w);
  return hipGetLastError();
}

hipError_t launch_mg_residual(const MgGeom &g, const double *dinv, double dconst, const double *x, const double *b,
                              double *r, hipStream_t s) {
  mg_residual_kernel<<<blocks_for(g.nodes), kMgBlock, 0, s>>>(g, dinv, dconst, x, b, r);
  return hipGetLastError();
}

hipError_t launch_mg_restrict(const MgGeom &gf, const double *rf, const MgGeom &gc, double *bc, hipStream_t s) {
  mg_restrict_kernel<<<blocks_for(gc.nodes), kMgBlock, 0, s>>>(gf, rf, gc, bc);
  return hipGetLastError();
}

hipError_t launch_mg_prolong(const MgGeom &gc, const double *xc, const MgGeom &gf, double *xf, hipStream_t s) {
  mg_prolong_kernel<<<blocks_for(gf.nodes), kMgBlock, 0, s>>>(gc, xc, gf, xf);
  return hipGetLastError();
}

hipError_t launch_mg_inject(const MgGeom &gf, const double *df, const MgGeom &gc, double *dc, hipStream_t s) {
  mg_inject_kernel<<<blocks_for(gc.nodes), kMgBlock, 0, s>>>(gf, df, gc, dc);
  return hipGetLastError();
}

hipError_t launch_mg_inverse(const MgGeom &g, const double *c2, double *d, hipStream_t s) {
  mg_inverse_kernel<<<blocks_for(g.nodes), kMgBlock, 0, s>>>(g, c2, d);
  return hipGetLastError();
}

hipError_t launch_imp_rhs(const MgGeom &g, const double *dinv, double dconst, const double *cur, const double *prev,
                          const double *f, double gn, double *B, double *X0, hipStream_t s) {
  imp_rhs_kernel<<<blocks_for(g.nodes), kMgBlock, 0, s>>>(g, dinv, dconst, cur, prev, f, gn, B, X0);
  return hipGetLastError();
}

hipError_t launch_imp_filter(const MgGeom &g, const double *x, double w, double *acc, bool init, int mode,
                             const double *v, double *out, hipStream_t s) {
  imp_filter_kernel<<<blocks_for(g.nodes), kMgBlock, 0, s>>>(g.nodes, x, w, acc, init ? 1 : 0, mode, v, out, g);
  return hipGetLastError();
}

hipError_t launch_pcg_update(int64_t n, double *x, double *r, const double *p, const double *q, const double *num,
                             const double *den, hipStream_t s) {
  pcg_update_kernel<<<blocks_for(n), kMgBlock, 0, s>>>(n, x, r, p, q, num, den);
  return hipGetLastError();
}

hipError_t launch_pcg_xpay(int64_t n, const double *z, double *p, const double *num, const double *den,
                           hipStream_t s) {
  pcg_xpay_kernel<<<blocks_for(n), kMgBlock, 0, s>>>(n, z, p, num, den);
  return hipGetLastError();
}

}  // namespace wh
