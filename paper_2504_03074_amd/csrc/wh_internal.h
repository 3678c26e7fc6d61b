// Internal interface between the C-ABI layer (wh_api.cpp) and the HIP kernels
// (wh_kernels.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <cstdint>

namespace wh {

// Geometry and per-step coefficients of one leapfrog launch.
//   next = 2 cur - prev + c2 * (sum_m k_m * S_m(cur) - kc * cur) + gn * f
// where S_m is the symmetric neighbour sum along axis m:
//   p = 2: W[i-1] + W[i+1],             k_m = dt^2 n_m^2
//   p = 4: 16 (W[i-1] + W[i+1]) - (W[i-2] + W[i+2]),  k_m = dt^2 n_m^2 / 12
// and kc = 2 sum k_m (p = 2) or 30 sum k_m (p = 4).
struct StepGeom {
  int dim;
  int order;
  int nx, ny, nz;      // cells per axis (nz = 0 in 2-D)
  int64_t sy, sz;      // strides of the node arrays (x stride is 1)
  int64_t nodes;       // (nx+1)(ny+1)(nz+1)
  double kx, ky, kz, kc;
  double c2const;      // used when the c2 pointer is null
};

enum FinalMode { ACCUMULATE = 0, FINAL_FILTER = 1, FINAL_A = 2 };

// First step: W0 = v (walls 0), W1 = W0 + (1/2)(L W0 dt^2) + g0 f,
// acc = w0 W0 + w1 W1.  c2/f may be null (constant c2 / no forcing).
// `half` geometry has k_m and kc already halved.
hipError_t launch_first_step(bool fp32, const StepGeom &half, const double *v, void *W0, void *W1,
                             double *acc, const void *c2, const void *f, double g0, double w0,
                             double w1, hipStream_t s);

// One leapfrog step in place: prev_next holds W^{n-1} on entry, W^{n+1} on exit.
// mode ACCUMULATE: acc += wn W^{n+1}; FINAL_FILTER: out = acc + wn W^{n+1};
// FINAL_A: out = v - (acc + wn W^{n+1}).  Final modes also zero `out` on walls.
hipError_t launch_step(bool fp32, const StepGeom &g, const void *cur, void *prev_next, double *acc,
                       const void *c2, const void *f, double gn, double wn, int mode,
                       const double *v, double *out, hipStream_t s);

// Fixed device scratch of the allocation-free entry point (wh_noalloc.hip):
// kStaticScratchBytes per device; static_scratch returns its address on the
// current device (looked up once per device).
constexpr size_t kStaticScratchBytes = (size_t)192 << 20;
hipError_t static_scratch(int device, void **ptr);

// Streaming-bandwidth reference kernel: kind 0 copy, 1 read, 2 write of
// `bytes` (a multiple of 16), kind 3 the FP32 blocked pass's per-node mix
// (`bytes` = 36 x nodes, a multiple of 144), with `groups` work-groups of
// 256 lanes.
hipError_t launch_stream(int kind, const void *src, void *dst, int64_t bytes, int groups, float *sink,
                         hipStream_t s);

// Temporally blocked steps for 2-D grids: ksteps <= K leapfrog steps per pass
// over the grid (K fixes the halo K*p/2 and the tile shape).  in_prev/in_cur
// hold W^{n-1}, W^n; out_prev/out_cur receive W^{n+ks-1}, W^{n+ks}.  gn[s],
// wn[s] belong to the step producing W^{n+1+s}.  The last pass of an
// application uses mode != ACCUMULATE.
constexpr int kMaxBlockSteps = 8;
struct BlockCoef {
  double gn[kMaxBlockSteps];
  double wn[kMaxBlockSteps];
};
hipError_t launch_block_steps_2d(bool fp32, const StepGeom &g, int K, int rows, int ksteps, const void *in_prev,
                                 const void *in_cur, void *out_prev, void *out_cur, double *acc, const void *c2,
                                 const void *f, const BlockCoef &coef, int mode, const double *v, double *out,
                                 hipStream_t s);
// rows = tile height of the loaded region (waves per group x rows per lane):
// FP64 p = 4: 40, 80, 100; FP64 p = 2: 32, 64, 80; FP32 96 or 192.
bool block_config_supported(bool fp32, int order, int K, int rows);
int block_default_rows(bool fp32, int order);
// rows of a tile held by one lane (tile rows are multiples of it)
int block_rows_per_lane(bool fp32, int order);
// Owned tile (nodes) of one work-group of the blocked kernel.
void block_tile_shape(bool fp32, int order, int K, int rows, int *owned_x, int *owned_y);

// Temporally blocked steps for 3-D grids: K (1..4) leapfrog steps per pass,
// pipelined along z over (x, y) tiles of 64 columns x `rows` rows (16 or 32)
// and segments of z planes.  Same buffers, modes and
// coefficients as launch_block_steps_2d; every pass takes exactly K steps.
hipError_t launch_block_steps_3d(bool fp32, const StepGeom &g, int K, int rows, const void *in_prev,
                                 const void *in_cur, void *out_prev, void *out_cur, double *acc, const void *c2,
                                 const void *f, const BlockCoef &coef, int mode, const double *v, double *out,
                                 hipStream_t s);
bool block3d_config_supported(bool fp32, int order, int K, int rows);
int block3d_default_rows(bool fp32, int order, int K);
int block3d_rows_per_lane(bool fp32);
constexpr int kMaxBlockSteps3d = 4;

// One leapfrog step for a 3-D grid with zb consecutive z nodes per thread
// (zb in {4, 8, 16}); same arguments and modes as launch_step.
hipError_t launch_step3d_zcol(bool fp32, const StepGeom &g, int zb, const void *cur, void *prev_next, double *acc,
                              const void *c2, const void *f, double gn, double wn, int mode, const double *v,
                              double *out, hipStream_t s);
bool zcol_supported(int zb);

// ---------------------------------------------------------------------------
// Implicit time stepping on 2-D grids (FP64): one multigrid level of the
// symmetric step operator S x = (d + ac) x - ax S_x(x) - ay S_y(x), d = 1/c^2.
// ---------------------------------------------------------------------------
struct MgGeom {
  int nx, ny;       // cells per axis
  int64_t sy;       // row stride (nx + 1)
  int64_t nodes;    // (nx + 1)(ny + 1)
  int order;        // 2 or 4 (coarse levels: 2)
  double ax, ay, ac;
};
hipError_t launch_mg_smooth(const MgGeom &g, const double *dinv, double dconst, const double *x_in,
                            const double *b, double *x_out, double w, hipStream_t s);
hipError_t launch_mg_residual(const MgGeom &g, const double *dinv, double dconst, const double *x, const double *b,
                              double *r, hipStream_t s);
hipError_t launch_mg_restrict(const MgGeom &gf, const double *rf, const MgGeom &gc, double *bc, hipStream_t s);
hipError_t launch_mg_prolong(const MgGeom &gc, const double *xc, const MgGeom &gf, double *xf, hipStream_t s);
hipError_t launch_mg_inject(const MgGeom &gf, const double *df, const MgGeom &gc, double *dc, hipStream_t s);
hipError_t launch_mg_inverse(const MgGeom &g, const double *c2, double *d, hipStream_t s);
hipError_t launch_imp_rhs(const MgGeom &g, const double *dinv, double dconst, const double *cur, const double *prev,
                          const double *f, double gn, double *B, double *X0, hipStream_t s);
hipError_t launch_imp_filter(const MgGeom &g, const double *x, double w, double *acc, bool init, int mode,
                             const double *v, double *out, hipStream_t s);
hipError_t launch_pcg_update(int64_t n, double *x, double *r, const double *p, const double *q, const double *num,
                             const double *den, hipStream_t s);
hipError_t launch_pcg_xpay(int64_t n, const double *z, double *p, const double *num, const double *den,
                           hipStream_t s);

// ---------------------------------------------------------------------------
// Batches of independent 2-D problems (same order and precision).
// ---------------------------------------------------------------------------
// One problem of a batched blocked pass (device-resident table).
struct BatchDesc {
  StepGeom g;           // stencil scaled by dt^2
  const void *c2;       // null: constant g.c2const
  const void *f;        // null: no forcing
  void *W[4];           // state buffers: pass j reads pair j%2, writes the other
  double *acc;          // FP64 filter accumulator
  const double *v;      // input of the application (read by FINAL_A)
  double *out;          // output of the application
  int tiles_x, tiles;   // tile grid of this problem for the batch's (K, rows)
  int steps;            // leapfrog steps after the first (N - 1)
  int passes;           // ceil(steps / K)
  int coef_offset;      // index of this problem's first BlockCoef
};
// Pass `pass` of every active problem (the first nactive of the table, sorted
// by pass count) in one launch; tile_prefix[i] = first tile of problem i.
hipError_t launch_batch_block_steps(bool fp32, int order, int K, int rows, bool force, const BatchDesc *descs,
                                    const int *tile_prefix, int nactive, int total_tiles, int pass,
                                    const BlockCoef *coefs, int final_mode, hipStream_t s);

// First step of every problem of a batch in one launch.
struct BatchFirst {
  StepGeom half;        // stencil scaled by dt^2 / 2
  const double *v;
  void *W0, *W1;
  double *acc;
  const void *c2;       // null: constant
  const void *f;        // null: no forcing
  double g0, w0, w1;
  int block_offset;     // first thread block of this problem
};
hipError_t launch_batch_first_step(bool fp32, int order, const BatchFirst *firsts, int nprob, int total_blocks,
                                   hipStream_t s);
int batch_node_blocks(int64_t nodes);

// Per-(precision, order) launchers of the blocked kernels (one translation
// unit each; the routing above picks one).
using BlockDispatch = hipError_t (*)(const StepGeom &, int, int, int, const void *, const void *, void *, void *,
                                     double *, const void *, const void *, const BlockCoef &, int, const double *,
                                     double *, hipStream_t);
using Block3dDispatch = hipError_t (*)(const StepGeom &, int, int, const void *, const void *, void *, void *,
                                       double *, const void *, const void *, const BlockCoef &, int, const double *,
                                       double *, hipStream_t);
using BatchDispatch = hipError_t (*)(int, int, bool, const BatchDesc *, const int *, int, int, int, const BlockCoef *,
                                     int, hipStream_t);
#define WH_BLOCK_DISPATCH_DECL(name)                                                                            \
  hipError_t block_dispatch_##name(const StepGeom &g, int K, int nw, int ksteps, const void *in_prev,           \
                                   const void *in_cur, void *out_prev, void *out_cur, double *acc, const void *c2, \
                                   const void *f, const BlockCoef &coef, int mode, const double *v, double *out, \
                                   hipStream_t s);                                                              \
  hipError_t batch_dispatch_##name(int K, int nw, bool force, const BatchDesc *descs, const int *tile_prefix,   \
                                   int nactive, int total_tiles, int pass, const BlockCoef *coefs,               \
                                   int final_mode, hipStream_t s);
#define WH_BLOCK3D_DISPATCH_DECL(name)                                                                          \
  hipError_t block3d_dispatch_##name(const StepGeom &g, int K, int nw, const void *in_prev, const void *in_cur, \
                                     void *out_prev, void *out_cur, double *acc, const void *c2, const void *f,  \
                                     const BlockCoef &coef, int mode, const double *v, double *out, hipStream_t s);
WH_BLOCK3D_DISPATCH_DECL(f64_p2)
WH_BLOCK3D_DISPATCH_DECL(f64_p4)
WH_BLOCK3D_DISPATCH_DECL(f32_p2)
WH_BLOCK3D_DISPATCH_DECL(f32_p4)
#undef WH_BLOCK3D_DISPATCH_DECL
WH_BLOCK_DISPATCH_DECL(f64_p2)
WH_BLOCK_DISPATCH_DECL(f64_p4)
WH_BLOCK_DISPATCH_DECL(f32_p2)
WH_BLOCK_DISPATCH_DECL(f32_p4)
#undef WH_BLOCK_DISPATCH_DECL

// Vectors of one problem for the batched Krylov kernels.
struct BatchVec {
  double *x, *r, *p, *q;
  const double *b;
  const void *c2;       // weights 1/c2 of the inner product (null: 1)
  int64_t n;
  int block_offset;     // first reduction block of this problem
  int nblocks;
  int active;           // 0: frozen (converged)
};
int batch_red_blocks(int64_t n);
// out[2*i] = <a_i, b_i>_w (which = 0: a = p, b = q; which = 1: a = b = r)
hipError_t launch_batch_dot(bool fp32_c2, const BatchVec *vecs, int nprob, int total_blocks, int which,
                            double *partials, double *out, int out_stride, hipStream_t s);
// x += a p, r -= a q with a = num[i*stride]/den[i*stride]; then
// out[2*i] = <r,r>_w, out[2*i+1] = <r,r>.  Frozen problems are untouched.
hipError_t launch_batch_cg_update(bool fp32_c2, const BatchVec *vecs, int nprob, int total_blocks, const double *num,
                                  const double *den, int stride, double *partials, double *out, hipStream_t s);
// p = r + (num/den) p for active problems
hipError_t launch_batch_xpay(const BatchVec *vecs, int nprob, int total_blocks, const double *num, const double *den,
                             int stride, hipStream_t s);
// r = b - q, p = r for every problem (start or restart of CG)
hipError_t launch_batch_residual(const BatchVec *vecs, int nprob, int total_blocks, hipStream_t s);

// Convert/copy helpers.
hipError_t launch_to_state(bool fp32, const double *src, void *dst, int64_t n, hipStream_t s);
hipError_t launch_from_state(bool fp32, const void *src, double *dst, int64_t n, hipStream_t s);

// Reductions (deterministic: fixed block count and fixed combine order).
int reduction_blocks(int64_t n);
// partials[i * nb + b] = block b's share of sum_e V_i[e] * w[e], i < k.
hipError_t launch_mdot(const double *V, int64_t ldv, int k, const double *w, int64_t n, double *partials,
                       int nb, hipStream_t s);
// out[i] = sum_b partials[i * nb + b] (block-tree order).
hipError_t launch_reduce_rows(const double *partials, int nb, int k, double *out, hipStream_t s);
// partials of sum_e x_e y_e / c2_e (c2 null: plain dot), one row of nb
hipError_t launch_wdot(const double *x, const double *y, const void *c2, bool fp32_c2, int64_t n, double *partials,
                       int nb, hipStream_t s);
// CG step: a = *num / *den; x += a p; r -= a q; partials of <r,r>_{1/c2}
// (row 0) and <r,r> (row 1).  c2 null: unweighted.
hipError_t launch_cg_update(double *x, double *r, const double *p, const double *q, const void *c2, bool fp32_c2,
                            const double *num, const double *den, int64_t n, double *partials, int nb,
                            hipStream_t s);
// p = r + (*num / *den) p
hipError_t launch_xpay(const double *r, double *p, const double *num, const double *den, int64_t n, hipStream_t s);
// w[e] -= sum_i coef[i] * V_i[e]  (coef on device)
hipError_t launch_block_axpy(const double *V, int64_t ldv, int k, const double *coef, double *w, int64_t n,
                             hipStream_t s);
// x[e] += sum_i coef[i] * V_i[e]  (coef on device)
hipError_t launch_block_gemv_add(const double *V, int64_t ldv, int k, const double *coef, double *x,
                                 int64_t n, hipStream_t s);
// dst[e] = src[e] / sqrt(*norm2)
hipError_t launch_scale_by_rnorm(const double *src, double *dst, const double *norm2, int64_t n,
                                 hipStream_t s);
// partials of sum (a - b)^2, then b = a
hipError_t launch_diff_norm_copy(const double *a, double *b, int64_t n, double *partials, int nb,
                                 hipStream_t s);
// dst = a + b
hipError_t launch_add(const double *a, const double *b, double *dst, int64_t n, hipStream_t s);
// dst = a - b
hipError_t launch_sub(const double *a, const double *b, double *dst, int64_t n, hipStream_t s);
// partial min/max/non-finite count of src over interior nodes (3 * nb values)
hipError_t launch_interior_stats(const StepGeom &g, const double *src, double *partials, int nb,
                                 hipStream_t s);
// res = c2 Delta u + omega^2 u - f (interior), 0 on walls; state precision FP64
hipError_t launch_helmholtz_residual(const StepGeom &g_unscaled, const double *u, const void *c2, bool fp32_c2,
                                     const void *f, bool fp32_f, double omega2, double *res, hipStream_t s);
hipError_t launch_fill(double *dst, double value, int64_t n, hipStream_t s);

// Discrete adjoint (FP64 state).  One reverse-time step: zprev_next <-
// 2 zcur - zprev_next + c2 (g-scaled Delta_h zcur) + wn clam; then
// gf += gam * new (gf nullable), gc += kap * new * (g-scaled Delta_h wprev)
// (gc nullable).  c2 null = constant g.c2const.
hipError_t launch_adjoint_step(const StepGeom &g, const double *zcur, double *zprev_next, const double *c2,
                               const double *clam, double wn, const double *wprev, double gam, double kap, double *gf,
                               double *gc, hipStream_t s);
// out = (w0 clam + z1 + c2 (half-scaled Delta_h z1) - z2) / c2, walls 0
hipError_t launch_adjoint_first(const StepGeom &half, const double *z1, const double *z2, const double *c2,
                                const double *clam, double w0, double *out, hipStream_t s);
// out = in * c2 or in / c2 (divide) on interior nodes, 0 on walls
hipError_t launch_scale_c2(const StepGeom &g, const double *c2, const double *in, double *out, bool divide,
                           hipStream_t s);
// Deflation with sine modes: mode_blocks = work-groups (and partials per
// mode) of the mode kernels; coef[m] = sum_interior v phi_m (v in state
// precision when fp32); out += alpha coef[m] scale[m] phi_m (scale nullable).
int mode_blocks(const StepGeom &g);
hipError_t launch_mode_dot(const StepGeom &g, bool fp32, const void *v, int nmodes, const double *sx, const double *sy,
                           const double *sz, double *partials, double *coef, hipStream_t s);
hipError_t launch_mode_combine(const StepGeom &g, double *out, int nmodes, const double *sx, const double *sy,
                               const double *sz, const double *coef, const double *scale, double alpha,
                               hipStream_t s);
// receiver misfit: out[0] = J, out[1] = count of out-of-range indices;
// grad (nullable, pre-zeroed) += residuals at the receiver nodes
hipError_t launch_misfit(const double *u, const int64_t *idx, const double *data, int nrec, int64_t nodes,
                         double *grad, double *out, hipStream_t s);
// Overwrite the wall nodes of a state-precision node array with `value`.
hipError_t launch_set_walls(bool fp32, const StepGeom &g, void *a, double value, hipStream_t s);

}  // namespace wh
