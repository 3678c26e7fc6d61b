// HIP kernels of the WaveHoltz hot path for CDNA4 (gfx950): the first step,
// the fused leapfrog + filter step, and the FP64 reductions of the outer
// solvers.  One node per thread; node arrays are dense, x fastest.
//
// The scheme is the explicit leapfrog of Sec. 4.2.1 (eq. WaveSchemeexplicit)
// with the trapezoid filter of eq. (updateDiscreteExplicit) accumulated in FP64
// as the steps are taken, so the time history is never stored.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "wh_internal.h"
#include "wh_xcd.h"

namespace wh {
namespace {

constexpr int kBlockX = 64;
constexpr int kBlockY = 4;
constexpr int kRedThreads = 256;

template <typename T>
struct Coef {
  T kx, ky, kz, kc;
};

// Read by the first steps in place of a neighbour that lies on a wall (its
// value is 0 there); never written.
__device__ double kZeroNode = 0.0;

// Value at a node index that may lie up to 2 nodes beyond a wall: odd
// reflection u(-j) = -u(j), u(n+j) = -u(n-j).  Wall nodes themselves hold 0 in
// every state array.
template <typename T, int DIM>
__device__ __forceinline__ T load_reflect(const T *__restrict__ W, int i, int j, int k,
                                          const StepGeom &g) {
  T s = T(1);
  if (i < 0) { i = -i; s = -s; } else if (i > g.nx) { i = 2 * g.nx - i; s = -s; }
  if (j < 0) { j = -j; s = -s; } else if (j > g.ny) { j = 2 * g.ny - j; s = -s; }
  if (DIM == 3) {
    if (k < 0) { k = -k; s = -s; } else if (k > g.nz) { k = 2 * g.nz - k; s = -s; }
  }
  return s * W[(int64_t)i + (int64_t)j * g.sy + (int64_t)k * g.sz];
}

// sum_m k_m S_m(W) - kc W at an interior node (see StepGeom).
template <typename T, int DIM, int P>
__device__ __forceinline__ T stencil(const T *__restrict__ W, int i, int j, int k, int64_t idx,
                                     const StepGeom &g, const Coef<T> &c) {
  const T w0 = W[idx];
  if (P == 2) {
    // neighbours of an interior node are interior or wall nodes: no ghosts
    T r = c.kx * (W[idx - 1] + W[idx + 1]) + c.ky * (W[idx - g.sy] + W[idx + g.sy]);
    if (DIM == 3) r += c.kz * (W[idx - g.sz] + W[idx + g.sz]);
    return r - c.kc * w0;
  } else {
    const bool near = (i < 2) || (i > g.nx - 2) || (j < 2) || (j > g.ny - 2) ||
                      (DIM == 3 && ((k < 2) || (k > g.nz - 2)));
    T ax1, ax2, ay1, ay2, az1 = T(0), az2 = T(0);
    if (!near) {
      ax1 = W[idx - 1] + W[idx + 1];
      ax2 = W[idx - 2] + W[idx + 2];
      ay1 = W[idx - g.sy] + W[idx + g.sy];
      ay2 = W[idx - 2 * g.sy] + W[idx + 2 * g.sy];
      if (DIM == 3) {
        az1 = W[idx - g.sz] + W[idx + g.sz];
        az2 = W[idx - 2 * g.sz] + W[idx + 2 * g.sz];
      }
    } else {
      ax1 = load_reflect<T, DIM>(W, i - 1, j, k, g) + load_reflect<T, DIM>(W, i + 1, j, k, g);
      ax2 = load_reflect<T, DIM>(W, i - 2, j, k, g) + load_reflect<T, DIM>(W, i + 2, j, k, g);
      ay1 = load_reflect<T, DIM>(W, i, j - 1, k, g) + load_reflect<T, DIM>(W, i, j + 1, k, g);
      ay2 = load_reflect<T, DIM>(W, i, j - 2, k, g) + load_reflect<T, DIM>(W, i, j + 2, k, g);
      if (DIM == 3) {
        az1 = load_reflect<T, DIM>(W, i, j, k - 1, g) + load_reflect<T, DIM>(W, i, j, k + 1, g);
        az2 = load_reflect<T, DIM>(W, i, j, k - 2, g) + load_reflect<T, DIM>(W, i, j, k + 2, g);
      }
    }
    T r = c.kx * (T(16) * ax1 - ax2) + c.ky * (T(16) * ay1 - ay2);
    if (DIM == 3) r += c.kz * (T(16) * az1 - az2);
    return r - c.kc * w0;
  }
}

// Same stencil applied to a caller array whose wall values must be ignored
// (treated as 0): used by the first step, which reads the iterate v directly.
// The load address is selected per lane (the reflected node, or kZeroNode
// for a wall node), so that no load sits behind a branch: a load behind a
// per-lane test makes the compiler drain all loads in flight at its wait.
template <typename T, int DIM, int P>
__device__ __forceinline__ T stencil_from_v(const double *__restrict__ v, int i, int j, int k,
                                            const StepGeom &g, const Coef<T> &c) {
  auto val = [&](int a, int b, int d) -> T {
    T s = T(1);
    if (a < 0) { a = -a; s = -s; } else if (a > g.nx) { a = 2 * g.nx - a; s = -s; }
    if (b < 0) { b = -b; s = -s; } else if (b > g.ny) { b = 2 * g.ny - b; s = -s; }
    if (DIM == 3) {
      if (d < 0) { d = -d; s = -s; } else if (d > g.nz) { d = 2 * g.nz - d; s = -s; }
    }
    const bool wall = a <= 0 || a >= g.nx || b <= 0 || b >= g.ny || (DIM == 3 && (d <= 0 || d >= g.nz));
    const double *p = wall ? &kZeroNode : v + ((int64_t)a + (int64_t)b * g.sy + (int64_t)d * g.sz);
    return (wall ? T(1) : s) * static_cast<T>(*p);
  };
  const T w0 = val(i, j, k);
  if (P == 2) {
    T r = c.kx * (val(i - 1, j, k) + val(i + 1, j, k)) + c.ky * (val(i, j - 1, k) + val(i, j + 1, k));
    if (DIM == 3) r += c.kz * (val(i, j, k - 1) + val(i, j, k + 1));
    return r - c.kc * w0;
  } else {
    T r = c.kx * (T(16) * (val(i - 1, j, k) + val(i + 1, j, k)) - (val(i - 2, j, k) + val(i + 2, j, k))) +
          c.ky * (T(16) * (val(i, j - 1, k) + val(i, j + 1, k)) - (val(i, j - 2, k) + val(i, j + 2, k)));
    if (DIM == 3)
      r += c.kz * (T(16) * (val(i, j, k - 1) + val(i, j, k + 1)) - (val(i, j, k - 2) + val(i, j, k + 2)));
    return r - c.kc * w0;
  }
}

template <typename T>
__device__ __forceinline__ Coef<T> coef_of(const StepGeom &g) {
  return Coef<T>{static_cast<T>(g.kx), static_cast<T>(g.ky), static_cast<T>(g.kz), static_cast<T>(g.kc)};
}

// First step at node (i, j, k): W0 = v (0 on walls), W1 = W0 + c2 (half-scaled
// stencil of v) + g0 f, acc = w0 W0 + w1 W1.
template <typename T, int DIM, int P>
__device__ __forceinline__ void first_step_node(const StepGeom &g, int i, int j, int k, const double *__restrict__ v,
                                                T *__restrict__ W0, T *__restrict__ W1, double *__restrict__ acc,
                                                const T *__restrict__ c2, const T *__restrict__ f, double g0,
                                                double w0, double w1) {
  const int64_t idx = (int64_t)i + (int64_t)j * g.sy + (int64_t)k * g.sz;
  const bool wall = i == 0 || i == g.nx || j == 0 || j == g.ny || (DIM == 3 && (k == 0 || k == g.nz));
  if (wall) {
    W0[idx] = T(0);
    W1[idx] = T(0);
    acc[idx] = 0.0;
    return;
  }
  const Coef<T> c = coef_of<T>(g);
  const T u0 = static_cast<T>(v[idx]);
  const T c2v = c2 ? c2[idx] : static_cast<T>(g.c2const);
  T u1 = u0 + c2v * stencil_from_v<T, DIM, P>(v, i, j, k, g, c);
  if (f) u1 += static_cast<T>(g0) * f[idx];
  W0[idx] = u0;
  W1[idx] = u1;
  acc[idx] = w0 * static_cast<double>(u0) + w1 * static_cast<double>(u1);
}

template <typename T, int DIM, int P>
__global__ __launch_bounds__(kBlockX *kBlockY) void first_step_kernel(
    StepGeom g, const double *__restrict__ v, T *__restrict__ W0, T *__restrict__ W1,
    double *__restrict__ acc, const T *__restrict__ c2, const T *__restrict__ f, double g0, double w0,
    double w1) {
  const int i = blockIdx.x * kBlockX + threadIdx.x;
  const int j = blockIdx.y * kBlockY + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  if (i > g.nx || j > g.ny) return;
  first_step_node<T, DIM, P>(g, i, j, k, v, W0, W1, acc, c2, f, g0, w0, w1);
}

// 3-D first step with z coarsening: thread (i, j) takes planes k0..k0+ZB-1
// of its column and keeps v along the column in registers (as T, zero on the
// walls, odd reflection beyond them), so each z-neighbour is loaded once per
// column segment.  The load addresses are selected per lane, without
// branches: the reflected index of each x-, y- and z-neighbour (clamped into
// the grid) or, for a wall neighbour, kZeroNode.  Every load is then
// unconditional, so a wave waits on its loads by count; with a load behind a
// branch each wait drains the whole memory pipeline (1.46 ms against 1.09 ms
// for an FP32 512^3 first step).  Work-groups are numbered so that each XCD
// takes a contiguous range of (x, y, z) blocks, whose shared halo rows meet in
// its L2.  The same arithmetic per node as first_step_node.
template <typename T, int P, int ZB, bool CVAR, bool FORCE>
__global__ __launch_bounds__(kBlockX *kBlockY) void first_step3d_zcol_kernel(
    StepGeom g, int gx, int gy, int nblk, const double *__restrict__ v, T *__restrict__ W0, T *__restrict__ W1,
    double *__restrict__ acc, const T *__restrict__ c2, const T *__restrict__ f, double g0, double w0,
    double w1) {
  constexpr int R = P / 2;
  const int64_t lb64 = xcd_block((int64_t)blockIdx.y * gridDim.x + blockIdx.x, (int64_t)gridDim.x * gridDim.y);
  if (lb64 >= nblk) return;
  const int lb = (int)lb64;
  const int bx = lb % gx, rest = lb / gx, by = rest % gy, bz = rest / gy;
  const int i = bx * kBlockX + threadIdx.x;
  const int j = by * kBlockY + threadIdx.y;
  const int k0 = bz * ZB;
  if (i > g.nx || j > g.ny) return;
  const bool col_wall = i == 0 || i == g.nx || j == 0 || j == g.ny;
  const int64_t base = (int64_t)i + (int64_t)j * g.sy;
  // neighbour p + d along an axis of n cells: odd reflection at the walls
  // (index q, clamped into 0..n, and sign); `zero` marks a wall node
  auto reflect = [](int p, int d, int n, int &q, T &sign, bool &zero) {
    int a = p + d;
    sign = T(1);
    if (a < 0) { a = -a; sign = -sign; }
    if (a > n) { a = 2 * n - a; sign = -sign; }
    zero = a <= 0 || a >= n;
    if (zero) sign = T(1);
    q = a < 0 ? 0 : (a > n ? n : a);
  };
  const double *zero_node = &kZeroNode;
  int64_t xoff[2 * R], yoff[2 * R];  // neighbours -R..-1, 1..R
  T xsign[2 * R], ysign[2 * R];
  bool xzero[2 * R], yzero[2 * R];
#pragma unroll
  for (int e = 0; e < 2 * R; ++e) {
    const int d = e < R ? e - R : e - R + 1;
    int q;
    reflect(i, d, g.nx, q, xsign[e], xzero[e]);
    xoff[e] = (int64_t)(q - i);
    reflect(j, d, g.ny, q, ysign[e], yzero[e]);
    yoff[e] = (int64_t)(q - j) * g.sy;
  }
  T col[ZB + 2 * R];
#pragma unroll
  for (int t = 0; t < ZB + 2 * R; ++t) {
    int q;
    T sign;
    bool zero;
    reflect(k0, t - R, g.nz, q, sign, zero);
    zero = zero || col_wall;
    const double *p = zero ? zero_node : v + base + (int64_t)q * g.sz;
    col[t] = (zero ? T(1) : sign) * static_cast<T>(*p);
  }
  const Coef<T> c = coef_of<T>(g);
  T u1[ZB];
#pragma unroll
  for (int t = 0; t < ZB; ++t) {
    const int k = k0 + t;
    const int64_t idx = base + (int64_t)(k > g.nz ? g.nz : k) * g.sz;
    const bool wall = col_wall || k <= 0 || k >= g.nz;
    T xn[2 * R], yn[2 * R];
#pragma unroll
    for (int e = 0; e < 2 * R; ++e) {
      const double *px = (wall || xzero[e]) ? zero_node : v + idx + xoff[e];
      const double *py = (wall || yzero[e]) ? zero_node : v + idx + yoff[e];
      xn[e] = xsign[e] * static_cast<T>(*px);
      yn[e] = ysign[e] * static_cast<T>(*py);
    }
    const T u0 = col[t + R];
    T r;
    if constexpr (P == 2) {
      r = c.kx * (xn[0] + xn[1]) + c.ky * (yn[0] + yn[1]);
      r += c.kz * (col[t + R - 1] + col[t + R + 1]);
    } else {
      r = c.kx * (T(16) * (xn[1] + xn[2]) - (xn[0] + xn[3])) + c.ky * (T(16) * (yn[1] + yn[2]) - (yn[0] + yn[3]));
      r += c.kz * (T(16) * (col[t + R - 1] + col[t + R + 1]) - (col[t + R - 2] + col[t + R + 2]));
    }
    const T lap = r - c.kc * u0;
    const T c2v = CVAR ? c2[idx] : static_cast<T>(g.c2const);
    T u = u0 + c2v * lap;
    if constexpr (FORCE) u += static_cast<T>(g0) * f[idx];
    u1[t] = wall ? T(0) : u;
  }
#pragma unroll
  for (int t = 0; t < ZB; ++t) {
    const int k = k0 + t;
    if (k > g.nz) break;
    const int64_t idx = base + (int64_t)k * g.sz;
    const bool wall = col_wall || k <= 0 || k >= g.nz;
    W0[idx] = col[t + R];
    W1[idx] = u1[t];
    acc[idx] = wall ? 0.0 : w0 * static_cast<double>(col[t + R]) + w1 * static_cast<double>(u1[t]);
  }
}

// Batched first step of 2-D problems: flat node blocks, problem found from
// the block offsets (ascending).
template <typename T, int P>
__global__ __launch_bounds__(256) void batch_first_step_kernel(const BatchFirst *__restrict__ firsts, int nprob) {
  const int b = blockIdx.x;
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (firsts[mid].block_offset <= b) lo = mid;
    else hi = mid - 1;
  }
  const BatchFirst &d = firsts[lo];
  const int64_t e = (int64_t)(b - d.block_offset) * 256 + threadIdx.x;
  if (e >= d.half.nodes) return;
  const int i = (int)(e % d.half.sy), j = (int)(e / d.half.sy);
  first_step_node<T, 2, P>(d.half, i, j, 0, d.v, static_cast<T *>(d.W0), static_cast<T *>(d.W1), d.acc,
                           static_cast<const T *>(d.c2), static_cast<const T *>(d.f), d.g0, d.w0, d.w1);
}

template <typename T, int DIM, int P>
__global__ __launch_bounds__(kBlockX *kBlockY) void step_kernel(
    StepGeom g, const T *__restrict__ cur, T *__restrict__ prev_next, double *__restrict__ acc,
    const T *__restrict__ c2, const T *__restrict__ f, double gn, double wn, int mode,
    const double *__restrict__ v, double *__restrict__ out) {
  const int i = blockIdx.x * kBlockX + threadIdx.x;
  const int j = blockIdx.y * kBlockY + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  if (i > g.nx || j > g.ny) return;
  const int64_t idx = (int64_t)i + (int64_t)j * g.sy + (int64_t)k * g.sz;
  const bool wall = i == 0 || i == g.nx || j == 0 || j == g.ny || (DIM == 3 && (k == 0 || k == g.nz));
  if (wall) {
    if (mode != ACCUMULATE) out[idx] = 0.0;
    return;
  }
  const Coef<T> c = coef_of<T>(g);
  const T c2v = c2 ? c2[idx] : static_cast<T>(g.c2const);
  const T lap = stencil<T, DIM, P>(cur, i, j, k, idx, g, c);
  T nxt = T(2) * cur[idx] - prev_next[idx] + c2v * lap;
  if (f) nxt += static_cast<T>(gn) * f[idx];
  prev_next[idx] = nxt;
  const double a = acc[idx] + wn * static_cast<double>(nxt);
  if (mode == ACCUMULATE) {
    acc[idx] = a;
  } else if (mode == FINAL_FILTER) {
    out[idx] = a;
  } else {
    out[idx] = v[idx] - a;
  }
}

// 3-D step with z coarsening: thread (i, j) updates nodes k0..k0+ZB-1 of its
// column, keeping W^n along the column in registers so each z-neighbour is
// loaded once per column segment instead of once per node; x- and
// y-neighbours are loaded as in step_kernel.  Same arithmetic per node.
template <typename T, int P, int ZB>
__global__ __launch_bounds__(kBlockX *kBlockY) void step3d_zcol_kernel(
    StepGeom g, const T *__restrict__ cur, T *__restrict__ prev_next, double *__restrict__ acc,
    const T *__restrict__ c2, const T *__restrict__ f, double gn, double wn, int mode,
    const double *__restrict__ v, double *__restrict__ out) {
  constexpr int R = P / 2;
  const int i = blockIdx.x * kBlockX + threadIdx.x;
  const int j = blockIdx.y * kBlockY + threadIdx.y;
  const int k0 = blockIdx.z * ZB;
  if (i > g.nx || j > g.ny) return;
  const bool col_wall = i == 0 || i == g.nx || j == 0 || j == g.ny;
  const int64_t base = (int64_t)i + (int64_t)j * g.sy;
  // column of W^n for planes k0-R .. k0+ZB-1+R (odd reflection beyond the z walls)
  T col[ZB + 2 * R];
#pragma unroll
  for (int t = 0; t < ZB + 2 * R; ++t) {
    int k = k0 - R + t;
    T sgn = T(1);
    if (k < 0) { k = -k; sgn = -sgn; } else if (k > g.nz) { k = 2 * g.nz - k; sgn = -sgn; }
    col[t] = (col_wall || k > g.nz) ? T(0) : sgn * cur[base + (int64_t)k * g.sz];
  }
  const Coef<T> c = coef_of<T>(g);
#pragma unroll
  for (int t = 0; t < ZB; ++t) {
    const int k = k0 + t;
    if (k > g.nz) break;
    const int64_t idx = base + (int64_t)k * g.sz;
    const bool wall = col_wall || k == 0 || k == g.nz;
    if (wall) {
      if (mode != ACCUMULATE) out[idx] = 0.0;
      continue;
    }
    const T w0 = col[t + R];
    T r;
    if (P == 2) {
      r = c.kx * (cur[idx - 1] + cur[idx + 1]) + c.ky * (cur[idx - g.sy] + cur[idx + g.sy]) +
          c.kz * (col[t + R - 1] + col[t + R + 1]);
    } else {
      const bool near = (i < 2) || (i > g.nx - 2) || (j < 2) || (j > g.ny - 2);
      T ax1, ax2, ay1, ay2;
      if (!near) {
        ax1 = cur[idx - 1] + cur[idx + 1];
        ax2 = cur[idx - 2] + cur[idx + 2];
        ay1 = cur[idx - g.sy] + cur[idx + g.sy];
        ay2 = cur[idx - 2 * g.sy] + cur[idx + 2 * g.sy];
      } else {
        ax1 = load_reflect<T, 3>(cur, i - 1, j, k, g) + load_reflect<T, 3>(cur, i + 1, j, k, g);
        ax2 = load_reflect<T, 3>(cur, i - 2, j, k, g) + load_reflect<T, 3>(cur, i + 2, j, k, g);
        ay1 = load_reflect<T, 3>(cur, i, j - 1, k, g) + load_reflect<T, 3>(cur, i, j + 1, k, g);
        ay2 = load_reflect<T, 3>(cur, i, j - 2, k, g) + load_reflect<T, 3>(cur, i, j + 2, k, g);
      }
      r = c.kx * (T(16) * ax1 - ax2) + c.ky * (T(16) * ay1 - ay2) +
          c.kz * (T(16) * (col[t + R - 1] + col[t + R + 1]) - (col[t + R - 2] + col[t + R + 2]));
    }
    const T lap = r - c.kc * w0;
    const T c2v = c2 ? c2[idx] : static_cast<T>(g.c2const);
    T nxt = T(2) * w0 - prev_next[idx] + c2v * lap;
    if (f) nxt += static_cast<T>(gn) * f[idx];
    prev_next[idx] = nxt;
    const double a = acc[idx] + wn * static_cast<double>(nxt);
    if (mode == ACCUMULATE) acc[idx] = a;
    else if (mode == FINAL_FILTER) out[idx] = a;
    else out[idx] = v[idx] - a;
  }
}

// ---------------------------------------------------------------------------
// conversions
// ---------------------------------------------------------------------------
template <typename T>
__global__ void to_state_kernel(const double *__restrict__ src, T *__restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = static_cast<T>(src[e]);
}

template <typename T>
__global__ void from_state_kernel(const T *__restrict__ src, double *__restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = static_cast<double>(src[e]);
}

// Overwrite the wall nodes of a node array with `value`.
template <typename T>
__global__ void set_walls_kernel(StepGeom g, T *__restrict__ a, T value) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < g.nodes; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % g.sy;
    const int64_t j = (e / g.sy) % (g.ny + 1);
    const int64_t k = (g.dim == 3) ? e / g.sz : 0;
    if (i == 0 || i == g.nx || j == 0 || j == g.ny || (g.dim == 3 && (k == 0 || k == g.nz))) a[e] = value;
  }
}

__global__ void fill_kernel(double *__restrict__ dst, double value, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = value;
}

// ---------------------------------------------------------------------------
// reductions: wavefront shuffle tree, then the 4 wave results in fixed order
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  return x;
}

__device__ __forceinline__ double block_sum(double x, double *sm) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sm[wave] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sm[0] + sm[1]) + (sm[2] + sm[3]);
  return r;  // valid in thread 0
}

__global__ __launch_bounds__(kRedThreads) void mdot_kernel(const double *__restrict__ V, int64_t ldv,
                                                           const double *__restrict__ w, int64_t n,
                                                           double *__restrict__ partials, int nb) {
  __shared__ double sm[4];
  const int vec = blockIdx.y;
  const double *x = V + (int64_t)vec * ldv;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; e < n; e += (int64_t)nb * kRedThreads)
    s += x[e] * w[e];
  s = block_sum(s, sm);
  if (threadIdx.x == 0) partials[(int64_t)vec * nb + blockIdx.x] = s;
}

// Dots of w with up to kMdotGroup basis vectors per block row: w is read
// once per group instead of once per vector (Arnoldi's Gram-Schmidt pass).
constexpr int kMdotGroup = 8;
template <int G>
__global__ __launch_bounds__(kRedThreads) void mdot_group_kernel(const double *__restrict__ V, int64_t ldv, int k,
                                                                 const double *__restrict__ w, int64_t n,
                                                                 double *__restrict__ partials, int nb) {
  __shared__ double sm[4];
  const int v0 = blockIdx.y * G;
  double s[G];
#pragma unroll
  for (int g = 0; g < G; ++g) s[g] = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; e < n; e += (int64_t)nb * kRedThreads) {
    const double we = w[e];
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (v0 + g < k) s[g] += V[(int64_t)(v0 + g) * ldv + e] * we;
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (v0 + g >= k) break;  // uniform over the block
    const double t = block_sum(s[g], sm);
    if (threadIdx.x == 0) partials[(int64_t)(v0 + g) * nb + blockIdx.x] = t;
  }
}

// partials of sum_e x_e y_e / c2_e (the inner product in which c^2 Delta_h,
// and hence the WaveHoltz operator, is self-adjoint)
template <typename TC>
__global__ __launch_bounds__(kRedThreads) void wdot_kernel(const double *__restrict__ x, const double *__restrict__ y,
                                                           const TC *__restrict__ c2, int64_t n,
                                                           double *__restrict__ partials, int nb) {
  __shared__ double sm[4];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; e < n; e += (int64_t)nb * kRedThreads)
    s += x[e] * y[e] / static_cast<double>(c2[e]);
  s = block_sum(s, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// x += a p, r -= a q with a = num/den read from device memory; partials of
// <r, r>_w (row 0) and <r, r> (row 1) of the updated residual.
template <typename TC>
__global__ __launch_bounds__(kRedThreads) void cg_update_kernel(double *__restrict__ x, double *__restrict__ r,
                                                                const double *__restrict__ p,
                                                                const double *__restrict__ q,
                                                                const TC *__restrict__ c2, const double *__restrict__ num,
                                                                const double *__restrict__ den, int64_t n,
                                                                double *__restrict__ partials, int nb) {
  __shared__ double sm[4];
  const double a = *num / *den;
  double sw = 0.0, se = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; e < n; e += (int64_t)nb * kRedThreads) {
    x[e] += a * p[e];
    const double re = r[e] - a * q[e];
    r[e] = re;
    se += re * re;
    sw += re * re / (c2 ? static_cast<double>(c2[e]) : 1.0);
  }
  sw = block_sum(sw, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = sw;
  se = block_sum(se, sm);
  if (threadIdx.x == 0) partials[nb + blockIdx.x] = se;
}

// p = r + (num/den) p
__global__ void xpay_kernel(const double *__restrict__ r, double *__restrict__ p, const double *__restrict__ num,
                            const double *__restrict__ den, int64_t n) {
  const double b = *num / *den;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = r[e] + b * p[e];
}

__global__ __launch_bounds__(kRedThreads) void reduce_rows_kernel(const double *__restrict__ partials, int nb,
                                                                  double *__restrict__ out) {
  __shared__ double sm[4];
  const double *row = partials + (int64_t)blockIdx.x * nb;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedThreads) s += row[b];
  s = block_sum(s, sm);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void block_axpy_kernel(const double *__restrict__ V, int64_t ldv, int k, const double *__restrict__ coef,
                                  double *__restrict__ w, int64_t n, double sign) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += coef[i] * V[(int64_t)i * ldv + e];
    w[e] += sign * s;
  }
}

__global__ void scale_kernel(const double *__restrict__ src, double *__restrict__ dst,
                             const double *__restrict__ norm2, int64_t n) {
  const double r = 1.0 / sqrt(*norm2);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = src[e] * r;
}

__global__ __launch_bounds__(kRedThreads) void diff_norm_copy_kernel(const double *__restrict__ a,
                                                                     double *__restrict__ b, int64_t n,
                                                                     double *__restrict__ partials, int nb) {
  __shared__ double sm[4];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; e < n; e += (int64_t)nb * kRedThreads) {
    const double d = a[e] - b[e];
    s += d * d;
    b[e] = a[e];
  }
  s = block_sum(s, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void add_kernel(const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ dst,
                           int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = a[e] + b[e];
}

__global__ void sub_kernel(const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ dst,
                           int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = a[e] - b[e];
}

__global__ __launch_bounds__(kRedThreads) void interior_stats_kernel(StepGeom g, const double *__restrict__ src,
                                                                     double *__restrict__ partials, int nb) {
  __shared__ double smx[kRedThreads], smn[kRedThreads], sbad[kRedThreads];
  double mx = -__builtin_huge_val(), mn = __builtin_huge_val(), bad = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; e < g.nodes; e += (int64_t)nb * kRedThreads) {
    const int64_t i = e % g.sy;
    const int64_t j = (e / g.sy) % (g.ny + 1);
    const int64_t k = (g.dim == 3) ? e / g.sz : 0;
    const bool wall = i == 0 || i == g.nx || j == 0 || j == g.ny || (g.dim == 3 && (k == 0 || k == g.nz));
    if (wall) continue;
    const double x = src[e];
    if (!(x == x) || x == __builtin_huge_val() || x == -__builtin_huge_val()) bad += 1.0;
    else {
      mx = x > mx ? x : mx;
      mn = x < mn ? x : mn;
    }
  }
  smx[threadIdx.x] = mx;
  smn[threadIdx.x] = mn;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smx[threadIdx.x] = smx[threadIdx.x] > smx[threadIdx.x + w] ? smx[threadIdx.x] : smx[threadIdx.x + w];
      smn[threadIdx.x] = smn[threadIdx.x] < smn[threadIdx.x + w] ? smn[threadIdx.x] : smn[threadIdx.x + w];
      sbad[threadIdx.x] += sbad[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[3 * blockIdx.x + 0] = smx[0];
    partials[3 * blockIdx.x + 1] = smn[0];
    partials[3 * blockIdx.x + 2] = sbad[0];
  }
}

template <typename TC, typename TF, int DIM, int P>
__global__ __launch_bounds__(kBlockX *kBlockY) void helmholtz_residual_kernel(
    StepGeom g, const double *__restrict__ u, const TC *__restrict__ c2, const TF *__restrict__ f, double omega2,
    double *__restrict__ res) {
  const int i = blockIdx.x * kBlockX + threadIdx.x;
  const int j = blockIdx.y * kBlockY + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  if (i > g.nx || j > g.ny) return;
  const int64_t idx = (int64_t)i + (int64_t)j * g.sy + (int64_t)k * g.sz;
  const bool wall = i == 0 || i == g.nx || j == 0 || j == g.ny || (DIM == 3 && (k == 0 || k == g.nz));
  if (wall) {
    res[idx] = 0.0;
    return;
  }
  const Coef<double> c = coef_of<double>(g);
  const double c2v = c2 ? static_cast<double>(c2[idx]) : g.c2const;
  const double lap = stencil_from_v<double, DIM, P>(u, i, j, k, g, c);
  const double fv = f ? static_cast<double>(f[idx]) : 0.0;
  res[idx] = c2v * lap + omega2 * u[idx] - fv;
}

// ---------------------------------------------------------------------------
// batched Krylov vector kernels (problem found from the block offsets)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int batch_problem(const BatchVec *__restrict__ vecs, int nprob, int b) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (vecs[mid].block_offset <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename TC>
__device__ __forceinline__ double inv_weight(const void *c2, int64_t e) {
  return c2 ? 1.0 / static_cast<double>(static_cast<const TC *>(c2)[e]) : 1.0;
}

template <typename TC>
__global__ __launch_bounds__(kRedThreads) void batch_dot_kernel(const BatchVec *__restrict__ vecs, int nprob,
                                                                int which, double *__restrict__ partials) {
  __shared__ double sm[4];
  const int i = batch_problem(vecs, nprob, blockIdx.x);
  const BatchVec &d = vecs[i];
  const int lb = blockIdx.x - d.block_offset;
  const double *a = which == 0 ? d.p : d.r;
  const double *c = which == 0 ? d.q : d.r;
  double s = 0.0;
  for (int64_t e = (int64_t)lb * kRedThreads + threadIdx.x; e < d.n; e += (int64_t)d.nblocks * kRedThreads)
    s += a[e] * c[e] * inv_weight<TC>(d.c2, e);
  s = block_sum(s, sm);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// out[i * stride + row] = sum of the problem's partials of that row
__global__ __launch_bounds__(kRedThreads) void batch_reduce_kernel(const BatchVec *__restrict__ vecs,
                                                                   const double *__restrict__ partials, int rows,
                                                                   double *__restrict__ out, int stride) {
  __shared__ double sm[4];
  const BatchVec &d = vecs[blockIdx.x];
  for (int row = 0; row < rows; ++row) {
    double s = 0.0;
    for (int b = threadIdx.x; b < d.nblocks; b += kRedThreads) s += partials[(int64_t)(d.block_offset + b) * rows + row];
    s = block_sum(s, sm);
    if (threadIdx.x == 0) out[(int64_t)blockIdx.x * stride + row] = s;
  }
}

template <typename TC>
__global__ __launch_bounds__(kRedThreads) void batch_cg_update_kernel(const BatchVec *__restrict__ vecs, int nprob,
                                                                      const double *__restrict__ num,
                                                                      const double *__restrict__ den, int stride,
                                                                      double *__restrict__ partials) {
  __shared__ double sm[4];
  const int i = batch_problem(vecs, nprob, blockIdx.x);
  const BatchVec &d = vecs[i];
  const int lb = blockIdx.x - d.block_offset;
  double sw = 0.0, se = 0.0;
  if (d.active) {
    const double a = num[(int64_t)i * stride] / den[(int64_t)i * stride];
    for (int64_t e = (int64_t)lb * kRedThreads + threadIdx.x; e < d.n; e += (int64_t)d.nblocks * kRedThreads) {
      d.x[e] += a * d.p[e];
      const double re = d.r[e] - a * d.q[e];
      d.r[e] = re;
      se += re * re;
      sw += re * re * inv_weight<TC>(d.c2, e);
    }
  }
  sw = block_sum(sw, sm);
  if (threadIdx.x == 0) partials[2 * (int64_t)blockIdx.x] = sw;
  se = block_sum(se, sm);
  if (threadIdx.x == 0) partials[2 * (int64_t)blockIdx.x + 1] = se;
}

__global__ __launch_bounds__(kRedThreads) void batch_xpay_kernel(const BatchVec *__restrict__ vecs, int nprob,
                                                                 const double *__restrict__ num,
                                                                 const double *__restrict__ den, int stride) {
  const int i = batch_problem(vecs, nprob, blockIdx.x);
  const BatchVec &d = vecs[i];
  if (!d.active) return;
  const int lb = blockIdx.x - d.block_offset;
  const double bt = num[(int64_t)i * stride] / den[(int64_t)i * stride];
  for (int64_t e = (int64_t)lb * kRedThreads + threadIdx.x; e < d.n; e += (int64_t)d.nblocks * kRedThreads)
    d.p[e] = d.r[e] + bt * d.p[e];
}

__global__ __launch_bounds__(kRedThreads) void batch_residual_kernel(const BatchVec *__restrict__ vecs, int nprob) {
  const int i = batch_problem(vecs, nprob, blockIdx.x);
  const BatchVec &d = vecs[i];
  const int lb = blockIdx.x - d.block_offset;
  for (int64_t e = (int64_t)lb * kRedThreads + threadIdx.x; e < d.n; e += (int64_t)d.nblocks * kRedThreads) {
    const double re = d.b[e] - d.q[e];
    d.r[e] = re;
    d.p[e] = re;
  }
}

dim3 node_grid(const StepGeom &g) {
  return dim3((unsigned)((g.nx + 1 + kBlockX - 1) / kBlockX), (unsigned)((g.ny + 1 + kBlockY - 1) / kBlockY),
              (unsigned)(g.dim == 3 ? g.nz + 1 : 1));
}

unsigned flat_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

template <typename T, int DIM, int P>
void first_step_typed(const StepGeom &g, const double *v, void *W0, void *W1, double *acc, const void *c2,
                      const void *f, double g0, double w0, double w1, hipStream_t s) {
  if constexpr (DIM == 3) {
    constexpr int ZB = 4;
    const int gx = (g.nx + kBlockX) / kBlockX, gy = (g.ny + kBlockY) / kBlockY, gz = (g.nz + ZB) / ZB;
    const int nblk = gx * gy * gz;  // at most about nodes / 12 < 2^30 (nodes <= 2^33)
    const dim3 grid = xcd_grid(nblk);
    const dim3 block(kBlockX, kBlockY);
    const T *c2t = static_cast<const T *>(c2), *ft = static_cast<const T *>(f);
    T *W0t = static_cast<T *>(W0), *W1t = static_cast<T *>(W1);
    if (c2 && f)
      first_step3d_zcol_kernel<T, P, ZB, true, true><<<grid, block, 0, s>>>(g, gx, gy, nblk, v, W0t, W1t, acc, c2t,
                                                                            ft, g0, w0, w1);
    else if (c2)
      first_step3d_zcol_kernel<T, P, ZB, true, false><<<grid, block, 0, s>>>(g, gx, gy, nblk, v, W0t, W1t, acc, c2t,
                                                                             ft, g0, w0, w1);
    else if (f)
      first_step3d_zcol_kernel<T, P, ZB, false, true><<<grid, block, 0, s>>>(g, gx, gy, nblk, v, W0t, W1t, acc, c2t,
                                                                             ft, g0, w0, w1);
    else
      first_step3d_zcol_kernel<T, P, ZB, false, false><<<grid, block, 0, s>>>(g, gx, gy, nblk, v, W0t, W1t, acc,
                                                                              c2t, ft, g0, w0, w1);
  } else {
    first_step_kernel<T, DIM, P><<<node_grid(g), dim3(kBlockX, kBlockY), 0, s>>>(
        g, v, static_cast<T *>(W0), static_cast<T *>(W1), acc, static_cast<const T *>(c2),
        static_cast<const T *>(f), g0, w0, w1);
  }
}

template <typename T, int DIM, int P>
void step_typed(const StepGeom &g, const void *cur, void *prev_next, double *acc, const void *c2, const void *f,
                double gn, double wn, int mode, const double *v, double *out, hipStream_t s) {
  step_kernel<T, DIM, P><<<node_grid(g), dim3(kBlockX, kBlockY), 0, s>>>(
      g, static_cast<const T *>(cur), static_cast<T *>(prev_next), acc, static_cast<const T *>(c2),
      static_cast<const T *>(f), gn, wn, mode, v, out);
}

template <typename T>
void dispatch_first(const StepGeom &g, const double *v, void *W0, void *W1, double *acc, const void *c2,
                    const void *f, double g0, double w0, double w1, hipStream_t s) {
  if (g.dim == 2 && g.order == 2) first_step_typed<T, 2, 2>(g, v, W0, W1, acc, c2, f, g0, w0, w1, s);
  else if (g.dim == 2) first_step_typed<T, 2, 4>(g, v, W0, W1, acc, c2, f, g0, w0, w1, s);
  else if (g.order == 2) first_step_typed<T, 3, 2>(g, v, W0, W1, acc, c2, f, g0, w0, w1, s);
  else first_step_typed<T, 3, 4>(g, v, W0, W1, acc, c2, f, g0, w0, w1, s);
}

template <typename T>
void dispatch_step(const StepGeom &g, const void *cur, void *prev_next, double *acc, const void *c2, const void *f,
                   double gn, double wn, int mode, const double *v, double *out, hipStream_t s) {
  if (g.dim == 2 && g.order == 2) step_typed<T, 2, 2>(g, cur, prev_next, acc, c2, f, gn, wn, mode, v, out, s);
  else if (g.dim == 2) step_typed<T, 2, 4>(g, cur, prev_next, acc, c2, f, gn, wn, mode, v, out, s);
  else if (g.order == 2) step_typed<T, 3, 2>(g, cur, prev_next, acc, c2, f, gn, wn, mode, v, out, s);
  else step_typed<T, 3, 4>(g, cur, prev_next, acc, c2, f, gn, wn, mode, v, out, s);
}

// Streaming-bandwidth reference: 16-byte accesses per lane over a buffer,
// grid-stride.  kind 0 copies src to dst, 1 reads src (the sum is kept live by
// a store taken only for NaN data), 2 writes dst.
typedef float stream_vec __attribute__((ext_vector_type(4)));
template <int KIND>
__global__ __launch_bounds__(256) void stream_kernel(const stream_vec *__restrict__ src, stream_vec *__restrict__ dst,
                                                     int64_t n, float *__restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  float acc = 0.0f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    if constexpr (KIND == 0) {
      dst[i] = src[i];
    } else if constexpr (KIND == 1) {
      const stream_vec v = src[i];
      acc += (v.x + v.y) + (v.z + v.w);
    } else {
      dst[i] = stream_vec{1.0f, 2.0f, 3.0f, 4.0f};
    }
  }
  if constexpr (KIND == 1) {
    if (acc != acc && sink) sink[0] = acc;
  }
}

typedef double stream_d2 __attribute__((ext_vector_type(2)));

// The per-node traffic of a blocked pass of FP32 state without its stencil:
// W^{n-1}, W^n and c^2 (FP32) and the FP64 accumulator read, two FP32 levels
// and the accumulator written (36 B per node), four nodes per lane with
// 16-byte accesses, grid-stride.  The values written are a cheap function of
// the values read, so nothing can be elided.
__global__ __launch_bounds__(256) void stream_mix_kernel(const stream_vec *__restrict__ ip,
                                                         const stream_vec *__restrict__ ic,
                                                         const stream_vec *__restrict__ c2,
                                                         stream_d2 *__restrict__ acc, stream_vec *__restrict__ op,
                                                         stream_vec *__restrict__ oc, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += stride) {
    const stream_vec a = ic[i], b = ip[i], c = c2[i];
    const stream_vec nx = (a + a - b) + c * a;
    stream_d2 lo = acc[2 * i], hi = acc[2 * i + 1];
    lo.x += 0.5 * (double)nx.x;
    lo.y += 0.5 * (double)nx.y;
    hi.x += 0.5 * (double)nx.z;
    hi.y += 0.5 * (double)nx.w;
    op[i] = a;
    oc[i] = nx;
    acc[2 * i] = lo;
    acc[2 * i + 1] = hi;
  }
}

}  // namespace

hipError_t launch_first_step(bool fp32, const StepGeom &half, const double *v, void *W0, void *W1, double *acc,
                             const void *c2, const void *f, double g0, double w0, double w1, hipStream_t s) {
  if (fp32) dispatch_first<float>(half, v, W0, W1, acc, c2, f, g0, w0, w1, s);
  else dispatch_first<double>(half, v, W0, W1, acc, c2, f, g0, w0, w1, s);
  return hipGetLastError();
}

hipError_t launch_step(bool fp32, const StepGeom &g, const void *cur, void *prev_next, double *acc, const void *c2,
                       const void *f, double gn, double wn, int mode, const double *v, double *out,
                       hipStream_t s) {
  if (fp32) dispatch_step<float>(g, cur, prev_next, acc, c2, f, gn, wn, mode, v, out, s);
  else dispatch_step<double>(g, cur, prev_next, acc, c2, f, gn, wn, mode, v, out, s);
  return hipGetLastError();
}

template <typename T, int P, int ZB>
static void zcol_typed(const StepGeom &g, const void *cur, void *prev_next, double *acc, const void *c2,
                       const void *f, double gn, double wn, int mode, const double *v, double *out, hipStream_t s) {
  dim3 grid((unsigned)((g.nx + 1 + kBlockX - 1) / kBlockX), (unsigned)((g.ny + 1 + kBlockY - 1) / kBlockY),
            (unsigned)((g.nz + 1 + ZB - 1) / ZB));
  step3d_zcol_kernel<T, P, ZB><<<grid, dim3(kBlockX, kBlockY), 0, s>>>(
      g, static_cast<const T *>(cur), static_cast<T *>(prev_next), acc, static_cast<const T *>(c2),
      static_cast<const T *>(f), gn, wn, mode, v, out);
}

template <typename T, int P>
static hipError_t zcol_zb(const StepGeom &g, int zb, const void *cur, void *prev_next, double *acc, const void *c2,
                          const void *f, double gn, double wn, int mode, const double *v, double *out, hipStream_t s) {
  switch (zb) {
    case 4: zcol_typed<T, P, 4>(g, cur, prev_next, acc, c2, f, gn, wn, mode, v, out, s); break;
    case 8: zcol_typed<T, P, 8>(g, cur, prev_next, acc, c2, f, gn, wn, mode, v, out, s); break;
    case 16: zcol_typed<T, P, 16>(g, cur, prev_next, acc, c2, f, gn, wn, mode, v, out, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool zcol_supported(int zb) { return zb == 4 || zb == 8 || zb == 16; }

hipError_t launch_step3d_zcol(bool fp32, const StepGeom &g, int zb, const void *cur, void *prev_next, double *acc,
                              const void *c2, const void *f, double gn, double wn, int mode, const double *v,
                              double *out, hipStream_t s) {
  if (g.dim != 3 || !zcol_supported(zb)) return hipErrorInvalidValue;
  if (fp32) {
    if (g.order == 2) return zcol_zb<float, 2>(g, zb, cur, prev_next, acc, c2, f, gn, wn, mode, v, out, s);
    return zcol_zb<float, 4>(g, zb, cur, prev_next, acc, c2, f, gn, wn, mode, v, out, s);
  }
  if (g.order == 2) return zcol_zb<double, 2>(g, zb, cur, prev_next, acc, c2, f, gn, wn, mode, v, out, s);
  return zcol_zb<double, 4>(g, zb, cur, prev_next, acc, c2, f, gn, wn, mode, v, out, s);
}

hipError_t launch_to_state(bool fp32, const double *src, void *dst, int64_t n, hipStream_t s) {
  if (fp32) to_state_kernel<float><<<flat_blocks(n), 256, 0, s>>>(src, static_cast<float *>(dst), n);
  else to_state_kernel<double><<<flat_blocks(n), 256, 0, s>>>(src, static_cast<double *>(dst), n);
  return hipGetLastError();
}

hipError_t launch_from_state(bool fp32, const void *src, double *dst, int64_t n, hipStream_t s) {
  if (fp32) from_state_kernel<float><<<flat_blocks(n), 256, 0, s>>>(static_cast<const float *>(src), dst, n);
  else from_state_kernel<double><<<flat_blocks(n), 256, 0, s>>>(static_cast<const double *>(src), dst, n);
  return hipGetLastError();
}

hipError_t launch_set_walls(bool fp32, const StepGeom &g, void *a, double value, hipStream_t s) {
  if (fp32) set_walls_kernel<float><<<flat_blocks(g.nodes), 256, 0, s>>>(g, static_cast<float *>(a), (float)value);
  else set_walls_kernel<double><<<flat_blocks(g.nodes), 256, 0, s>>>(g, static_cast<double *>(a), value);
  return hipGetLastError();
}

hipError_t launch_stream(int kind, const void *src, void *dst, int64_t bytes, int groups, float *sink,
                         hipStream_t s) {
  const stream_vec *a = static_cast<const stream_vec *>(src);
  stream_vec *b = static_cast<stream_vec *>(dst);
  if (kind == 3) {
    // four nodes per 16-byte FP32 vector: src = W^{n-1}, W^n, c^2; dst =
    // the two FP32 outputs, then the FP64 accumulator
    const int64_t n4 = bytes / 144;
    stream_mix_kernel<<<groups, 256, 0, s>>>(a, a + n4, a + 2 * n4, reinterpret_cast<stream_d2 *>(b + 2 * n4), b,
                                             b + n4, n4);
    return hipGetLastError();
  }
  const int64_t n = bytes / 16;
  if (kind == 0) stream_kernel<0><<<groups, 256, 0, s>>>(a, b, n, sink);
  else if (kind == 1) stream_kernel<1><<<groups, 256, 0, s>>>(a, b, n, sink);
  else stream_kernel<2><<<groups, 256, 0, s>>>(a, b, n, sink);
  return hipGetLastError();
}

hipError_t launch_fill(double *dst, double value, int64_t n, hipStream_t s) {
  fill_kernel<<<flat_blocks(n), 256, 0, s>>>(dst, value, n);
  return hipGetLastError();
}

int reduction_blocks(int64_t n) {
  int64_t b = (n + 4 * kRedThreads - 1) / (4 * kRedThreads);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_mdot(const double *V, int64_t ldv, int k, const double *w, int64_t n, double *partials, int nb,
                       hipStream_t s) {
  if (k == 1) mdot_kernel<<<dim3((unsigned)nb, 1u), kRedThreads, 0, s>>>(V, ldv, w, n, partials, nb);
  else
    mdot_group_kernel<kMdotGroup><<<dim3((unsigned)nb, (unsigned)((k + kMdotGroup - 1) / kMdotGroup)), kRedThreads, 0,
                                    s>>>(V, ldv, k, w, n, partials, nb);
  return hipGetLastError();
}

hipError_t launch_reduce_rows(const double *partials, int nb, int k, double *out, hipStream_t s) {
  reduce_rows_kernel<<<(unsigned)k, kRedThreads, 0, s>>>(partials, nb, out);
  return hipGetLastError();
}

hipError_t launch_wdot(const double *x, const double *y, const void *c2, bool fp32_c2, int64_t n, double *partials,
                       int nb, hipStream_t s) {
  if (!c2) {
    mdot_kernel<<<dim3((unsigned)nb, 1u), kRedThreads, 0, s>>>(x, 0, y, n, partials, nb);
  } else if (fp32_c2) {
    wdot_kernel<float><<<(unsigned)nb, kRedThreads, 0, s>>>(x, y, static_cast<const float *>(c2), n, partials, nb);
  } else {
    wdot_kernel<double><<<(unsigned)nb, kRedThreads, 0, s>>>(x, y, static_cast<const double *>(c2), n, partials, nb);
  }
  return hipGetLastError();
}

hipError_t launch_cg_update(double *x, double *r, const double *p, const double *q, const void *c2, bool fp32_c2,
                            const double *num, const double *den, int64_t n, double *partials, int nb,
                            hipStream_t s) {
  if (fp32_c2)
    cg_update_kernel<float><<<(unsigned)nb, kRedThreads, 0, s>>>(x, r, p, q, static_cast<const float *>(c2), num, den,
                                                                n, partials, nb);
  else
    cg_update_kernel<double><<<(unsigned)nb, kRedThreads, 0, s>>>(x, r, p, q, static_cast<const double *>(c2), num,
                                                                 den, n, partials, nb);
  return hipGetLastError();
}

hipError_t launch_xpay(const double *r, double *p, const double *num, const double *den, int64_t n, hipStream_t s) {
  xpay_kernel<<<flat_blocks(n), 256, 0, s>>>(r, p, num, den, n);
  return hipGetLastError();
}

hipError_t launch_block_axpy(const double *V, int64_t ldv, int k, const double *coef, double *w, int64_t n,
                             hipStream_t s) {
  block_axpy_kernel<<<flat_blocks(n), 256, 0, s>>>(V, ldv, k, coef, w, n, -1.0);
  return hipGetLastError();
}

hipError_t launch_block_gemv_add(const double *V, int64_t ldv, int k, const double *coef, double *x, int64_t n,
                                 hipStream_t s) {
  block_axpy_kernel<<<flat_blocks(n), 256, 0, s>>>(V, ldv, k, coef, x, n, 1.0);
  return hipGetLastError();
}

hipError_t launch_scale_by_rnorm(const double *src, double *dst, const double *norm2, int64_t n, hipStream_t s) {
  scale_kernel<<<flat_blocks(n), 256, 0, s>>>(src, dst, norm2, n);
  return hipGetLastError();
}

hipError_t launch_diff_norm_copy(const double *a, double *b, int64_t n, double *partials, int nb, hipStream_t s) {
  diff_norm_copy_kernel<<<(unsigned)nb, kRedThreads, 0, s>>>(a, b, n, partials, nb);
  return hipGetLastError();
}

hipError_t launch_add(const double *a, const double *b, double *dst, int64_t n, hipStream_t s) {
  add_kernel<<<flat_blocks(n), 256, 0, s>>>(a, b, dst, n);
  return hipGetLastError();
}

hipError_t launch_sub(const double *a, const double *b, double *dst, int64_t n, hipStream_t s) {
  sub_kernel<<<flat_blocks(n), 256, 0, s>>>(a, b, dst, n);
  return hipGetLastError();
}

hipError_t launch_interior_stats(const StepGeom &g, const double *src, double *partials, int nb, hipStream_t s) {
  interior_stats_kernel<<<(unsigned)nb, kRedThreads, 0, s>>>(g, src, partials, nb);
  return hipGetLastError();
}

template <typename TC, typename TF>
static void residual_typed(const StepGeom &g, const double *u, const void *c2, const void *f, double omega2,
                           double *res, hipStream_t s) {
  const TC *c = static_cast<const TC *>(c2);
  const TF *ff = static_cast<const TF *>(f);
  if (g.dim == 2 && g.order == 2)
    helmholtz_residual_kernel<TC, TF, 2, 2><<<node_grid(g), dim3(kBlockX, kBlockY), 0, s>>>(g, u, c, ff, omega2, res);
  else if (g.dim == 2)
    helmholtz_residual_kernel<TC, TF, 2, 4><<<node_grid(g), dim3(kBlockX, kBlockY), 0, s>>>(g, u, c, ff, omega2, res);
  else if (g.order == 2)
    helmholtz_residual_kernel<TC, TF, 3, 2><<<node_grid(g), dim3(kBlockX, kBlockY), 0, s>>>(g, u, c, ff, omega2, res);
  else
    helmholtz_residual_kernel<TC, TF, 3, 4><<<node_grid(g), dim3(kBlockX, kBlockY), 0, s>>>(g, u, c, ff, omega2, res);
}

hipError_t launch_helmholtz_residual(const StepGeom &g, const double *u, const void *c2, bool fp32_c2, const void *f,
                                     bool fp32_f, double omega2, double *res, hipStream_t s) {
  if (fp32_c2 && fp32_f) residual_typed<float, float>(g, u, c2, f, omega2, res, s);
  else if (fp32_c2) residual_typed<float, double>(g, u, c2, f, omega2, res, s);
  else if (fp32_f) residual_typed<double, float>(g, u, c2, f, omega2, res, s);
  else residual_typed<double, double>(g, u, c2, f, omega2, res, s);
  return hipGetLastError();
}

int batch_node_blocks(int64_t nodes) { return (int)((nodes + 255) / 256); }

hipError_t launch_batch_first_step(bool fp32, int order, const BatchFirst *firsts, int nprob, int total_blocks,
                                   hipStream_t s) {
  if (total_blocks <= 0) return hipSuccess;
  if (fp32) {
    if (order == 2) batch_first_step_kernel<float, 2><<<total_blocks, 256, 0, s>>>(firsts, nprob);
    else batch_first_step_kernel<float, 4><<<total_blocks, 256, 0, s>>>(firsts, nprob);
  } else {
    if (order == 2) batch_first_step_kernel<double, 2><<<total_blocks, 256, 0, s>>>(firsts, nprob);
    else batch_first_step_kernel<double, 4><<<total_blocks, 256, 0, s>>>(firsts, nprob);
  }
  return hipGetLastError();
}

int batch_red_blocks(int64_t n) {
  int64_t b = (n + 8 * kRedThreads - 1) / (8 * kRedThreads);
  if (b > 512) b = 512;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_batch_dot(bool fp32_c2, const BatchVec *vecs, int nprob, int total_blocks, int which,
                            double *partials, double *out, int out_stride, hipStream_t s) {
  if (fp32_c2) batch_dot_kernel<float><<<total_blocks, kRedThreads, 0, s>>>(vecs, nprob, which, partials);
  else batch_dot_kernel<double><<<total_blocks, kRedThreads, 0, s>>>(vecs, nprob, which, partials);
  batch_reduce_kernel<<<nprob, kRedThreads, 0, s>>>(vecs, partials, 1, out, out_stride);
  return hipGetLastError();
}

hipError_t launch_batch_cg_update(bool fp32_c2, const BatchVec *vecs, int nprob, int total_blocks, const double *num,
                                  const double *den, int stride, double *partials, double *out, hipStream_t s) {
  if (fp32_c2)
    batch_cg_update_kernel<float><<<total_blocks, kRedThreads, 0, s>>>(vecs, nprob, num, den, stride, partials);
  else
    batch_cg_update_kernel<double><<<total_blocks, kRedThreads, 0, s>>>(vecs, nprob, num, den, stride, partials);
  batch_reduce_kernel<<<nprob, kRedThreads, 0, s>>>(vecs, partials, 2, out, stride);
  return hipGetLastError();
}

hipError_t launch_batch_xpay(const BatchVec *vecs, int nprob, int total_blocks, const double *num, const double *den,
                             int stride, hipStream_t s) {
  batch_xpay_kernel<<<total_blocks, kRedThreads, 0, s>>>(vecs, nprob, num, den, stride);
  return hipGetLastError();
}

hipError_t launch_batch_residual(const BatchVec *vecs, int nprob, int total_blocks, hipStream_t s) {
  batch_residual_kernel<<<total_blocks, kRedThreads, 0, s>>>(vecs, nprob);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// discrete adjoint (FP64)
//
// With Z^n the adjoint of level W^n of one application and Zh^n = c^2 Z^n,
// the transpose of the leapfrog is the same leapfrog run backwards in time:
//   Zh^n = 2 Zh^{n+1} - Zh^{n+2} + c^2 (dt^2 Delta_h Zh^{n+1}) + w_n (c^2 lam),
// because Delta_h (with the odd wall reflection) is symmetric.  The
// sensitivities are collected as the sweep passes each level:
//   gf += gamma_{n-1} Zh^n,   gc += kappa_{n-1} Zh^n (dt^2 Delta_h W^{n-1}),
// and divided by c^2 at the end.
// ---------------------------------------------------------------------------
namespace {

template <int DIM, int P>
__global__ __launch_bounds__(kBlockX *kBlockY) void adjoint_step_kernel(
    StepGeom g, const double *__restrict__ zcur, double *__restrict__ zprev_next, const double *__restrict__ c2,
    const double *__restrict__ clam, double wn, const double *__restrict__ wprev, double gam, double kap,
    double *__restrict__ gf, double *__restrict__ gc) {
  const int i = blockIdx.x * kBlockX + threadIdx.x;
  const int j = blockIdx.y * kBlockY + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  if (i > g.nx || j > g.ny) return;
  const int64_t idx = (int64_t)i + (int64_t)j * g.sy + (int64_t)k * g.sz;
  const bool wall = i == 0 || i == g.nx || j == 0 || j == g.ny || (DIM == 3 && (k == 0 || k == g.nz));
  if (wall) {
    zprev_next[idx] = 0.0;
    return;
  }
  const Coef<double> c = coef_of<double>(g);
  const double c2v = c2 ? c2[idx] : g.c2const;
  const double zn =
      2.0 * zcur[idx] - zprev_next[idx] + c2v * stencil<double, DIM, P>(zcur, i, j, k, idx, g, c) + wn * clam[idx];
  zprev_next[idx] = zn;
  if (gf) gf[idx] += gam * zn;
  if (gc) gc[idx] += kap * zn * stencil<double, DIM, P>(wprev, i, j, k, idx, g, c);
}

// Adjoint of the initial level: out = (w_0 c^2 lam + Zh^1 + c^2 (dt^2/2)
// Delta_h Zh^1 - Zh^2) / c^2, the sensitivity to v (half-scaled geometry).
template <int DIM, int P>
__global__ __launch_bounds__(kBlockX *kBlockY) void adjoint_first_kernel(
    StepGeom half, const double *__restrict__ z1, const double *__restrict__ z2, const double *__restrict__ c2,
    const double *__restrict__ clam, double w0, double *__restrict__ out) {
  const int i = blockIdx.x * kBlockX + threadIdx.x;
  const int j = blockIdx.y * kBlockY + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  if (i > half.nx || j > half.ny) return;
  const int64_t idx = (int64_t)i + (int64_t)j * half.sy + (int64_t)k * half.sz;
  const bool wall = i == 0 || i == half.nx || j == 0 || j == half.ny || (DIM == 3 && (k == 0 || k == half.nz));
  if (wall) {
    out[idx] = 0.0;
    return;
  }
  const Coef<double> c = coef_of<double>(half);
  const double c2v = c2 ? c2[idx] : half.c2const;
  const double zh = w0 * clam[idx] + z1[idx] + c2v * stencil<double, DIM, P>(z1, i, j, k, idx, half, c) - z2[idx];
  out[idx] = zh / c2v;
}

// out = in * c^2 (divide = false) or in / c^2 on interior nodes, 0 on walls
template <int DIM>
__global__ __launch_bounds__(kBlockX *kBlockY) void scale_c2_kernel(StepGeom g, const double *__restrict__ c2,
                                                                   const double *__restrict__ in,
                                                                   double *__restrict__ out, int divide) {
  const int i = blockIdx.x * kBlockX + threadIdx.x;
  const int j = blockIdx.y * kBlockY + threadIdx.y;
  const int k = (DIM == 3) ? (int)blockIdx.z : 0;
  if (i > g.nx || j > g.ny) return;
  const int64_t idx = (int64_t)i + (int64_t)j * g.sy + (int64_t)k * g.sz;
  const bool wall = i == 0 || i == g.nx || j == 0 || j == g.ny || (DIM == 3 && (k == 0 || k == g.nz));
  if (wall) {
    out[idx] = 0.0;
    return;
  }
  const double c2v = c2 ? c2[idx] : g.c2const;
  out[idx] = divide ? in[idx] / c2v : in[idx] * c2v;
}

// Receiver misfit: one work-group.  res_r = u[idx_r] - d_r; out[0] = 1/2
// sum res_r^2, out[1] = number of indices outside [0, nodes); grad (nullable,
// zeroed by the caller) receives res_r at idx_r.
__global__ __launch_bounds__(kRedThreads) void misfit_kernel(const double *__restrict__ u,
                                                             const int64_t *__restrict__ idx,
                                                             const double *__restrict__ data, int nrec,
                                                             int64_t nodes, double *__restrict__ grad,
                                                             double *__restrict__ out) {
  __shared__ double sm[4];
  double s = 0.0, bad = 0.0;
  for (int r = threadIdx.x; r < nrec; r += kRedThreads) {
    const int64_t e = idx[r];
    if (e < 0 || e >= nodes) {
      bad += 1.0;
      continue;
    }
    const double res = u[e] - data[r];
    s += res * res;
    if (grad) atomicAdd(grad + e, res);
  }
  s = block_sum(s, sm);
  bad = block_sum(bad, sm);
  if (threadIdx.x == 0) {
    out[0] = 0.5 * s;
    out[1] = bad;
  }
}

}  // namespace

hipError_t launch_adjoint_step(const StepGeom &g, const double *zcur, double *zprev_next, const double *c2,
                               const double *clam, double wn, const double *wprev, double gam, double kap, double *gf,
                               double *gc, hipStream_t s) {
  const dim3 grid = node_grid(g), block(kBlockX, kBlockY);
  if (g.dim == 2 && g.order == 2)
    adjoint_step_kernel<2, 2><<<grid, block, 0, s>>>(g, zcur, zprev_next, c2, clam, wn, wprev, gam, kap, gf, gc);
  else if (g.dim == 2)
    adjoint_step_kernel<2, 4><<<grid, block, 0, s>>>(g, zcur, zprev_next, c2, clam, wn, wprev, gam, kap, gf, gc);
  else if (g.order == 2)
    adjoint_step_kernel<3, 2><<<grid, block, 0, s>>>(g, zcur, zprev_next, c2, clam, wn, wprev, gam, kap, gf, gc);
  else
    adjoint_step_kernel<3, 4><<<grid, block, 0, s>>>(g, zcur, zprev_next, c2, clam, wn, wprev, gam, kap, gf, gc);
  return hipGetLastError();
}

hipError_t launch_adjoint_first(const StepGeom &half, const double *z1, const double *z2, const double *c2,
                                const double *clam, double w0, double *out, hipStream_t s) {
  const dim3 grid = node_grid(half), block(kBlockX, kBlockY);
  if (half.dim == 2 && half.order == 2)
    adjoint_first_kernel<2, 2><<<grid, block, 0, s>>>(half, z1, z2, c2, clam, w0, out);
  else if (half.dim == 2)
    adjoint_first_kernel<2, 4><<<grid, block, 0, s>>>(half, z1, z2, c2, clam, w0, out);
  else if (half.order == 2)
    adjoint_first_kernel<3, 2><<<grid, block, 0, s>>>(half, z1, z2, c2, clam, w0, out);
  else
    adjoint_first_kernel<3, 4><<<grid, block, 0, s>>>(half, z1, z2, c2, clam, w0, out);
  return hipGetLastError();
}

hipError_t launch_scale_c2(const StepGeom &g, const double *c2, const double *in, double *out, bool divide,
                           hipStream_t s) {
  const dim3 grid = node_grid(g), block(kBlockX, kBlockY);
  if (g.dim == 2) scale_c2_kernel<2><<<grid, block, 0, s>>>(g, c2, in, out, divide ? 1 : 0);
  else scale_c2_kernel<3><<<grid, block, 0, s>>>(g, c2, in, out, divide ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_misfit(const double *u, const int64_t *idx, const double *data, int nrec, int64_t nodes,
                         double *grad, double *out, hipStream_t s) {
  misfit_kernel<<<1, kRedThreads, 0, s>>>(u, idx, data, nrec, nodes, grad, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// deflation with the sine modes of the unit box (Alg. 3)
//
// A mode is phi_m(i, j, k) = sx[m][i] sy[m][j] sz[m][k] (tables of the
// normalized 1-D sine factors, exactly 0 on the walls).  A work-group covers
// a 64 x kDefRows tile of (x, y) and every z plane; modes are taken kDefChunk
// at a time with their factors for the tile staged in LDS.
// ---------------------------------------------------------------------------
namespace {

constexpr int kDefChunk = 32;
constexpr int kDefRows = 8;

template <typename T, int DIM>
__global__ __launch_bounds__(256) void mode_dot_kernel(StepGeom g, const T *__restrict__ v, int nmodes,
                                                       const double *__restrict__ sx, const double *__restrict__ sy,
                                                       const double *__restrict__ sz, double *__restrict__ partials,
                                                       int nblocks) {
  __shared__ double tx[kDefChunk][64];
  __shared__ double ty[kDefChunk][kDefRows];
  __shared__ double red[4][kDefChunk];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int j0 = blockIdx.y * kDefRows;
  const int b = blockIdx.x + blockIdx.y * gridDim.x;
  const int nzp = DIM == 3 ? g.nz + 1 : 1;
  for (int m0 = 0; m0 < nmodes; m0 += kDefChunk) {
    const int mc = min(kDefChunk, nmodes - m0);
    for (int t = threadIdx.x; t < kDefChunk * 64; t += 256) {
      const int q = t / 64, l = t % 64, ii = blockIdx.x * 64 + l;
      tx[q][l] = (q < mc && ii <= g.nx) ? sx[(int64_t)(m0 + q) * (g.nx + 1) + ii] : 0.0;
    }
    for (int t = threadIdx.x; t < kDefChunk * kDefRows; t += 256) {
      const int q = t / kDefRows, r = t % kDefRows, jj = j0 + r;
      ty[q][r] = (q < mc && jj <= g.ny) ? sy[(int64_t)(m0 + q) * (g.ny + 1) + jj] : 0.0;
    }
    __syncthreads();
    double acc[kDefChunk];
#pragma unroll
    for (int q = 0; q < kDefChunk; ++q) acc[q] = 0.0;
    const bool col = i > 0 && i < g.nx;
    for (int k = (DIM == 3 ? 1 : 0); k < (DIM == 3 ? g.nz : 1); ++k) {
      for (int r = wave; r < kDefRows; r += 4) {
        const int j = j0 + r;
        if (!col || j <= 0 || j >= g.ny) continue;
        const double val = static_cast<double>(v[(int64_t)i + (int64_t)j * g.sy + (int64_t)k * g.sz]);
#pragma unroll
        for (int q = 0; q < kDefChunk; ++q) {
          double w = tx[q][lane] * ty[q][r];
          if (DIM == 3) w *= (q < mc) ? sz[(int64_t)(m0 + q) * (g.nz + 1) + k] : 0.0;
          acc[q] += val * w;
        }
      }
    }
    (void)nzp;
#pragma unroll
    for (int q = 0; q < kDefChunk; ++q) {
      const double sum = wave_sum(acc[q]);
      if (lane == 0) red[wave][q] = sum;
    }
    __syncthreads();
    if ((int)threadIdx.x < mc) {
      const int q = threadIdx.x;
      partials[(int64_t)(m0 + q) * nblocks + b] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    }
    __syncthreads();
  }
}

// coef[m] = sum of the mode's partials (one work-group per mode)
__global__ __launch_bounds__(kRedThreads) void mode_reduce_kernel(const double *__restrict__ partials, int nblocks,
                                                                  double *__restrict__ coef) {
  __shared__ double sm[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kRedThreads) s += partials[(int64_t)blockIdx.x * nblocks + b];
  s = block_sum(s, sm);
  if (threadIdx.x == 0) coef[blockIdx.x] = s;
}

// out += sum_m alpha coef[m] (scale[m]) phi_m on interior nodes
template <int DIM>
__global__ __launch_bounds__(256) void mode_combine_kernel(StepGeom g, double *__restrict__ out, int nmodes,
                                                           const double *__restrict__ sx,
                                                           const double *__restrict__ sy,
                                                           const double *__restrict__ sz,
                                                           const double *__restrict__ coef,
                                                           const double *__restrict__ scale, double alpha) {
  __shared__ double tx[kDefChunk][64];
  __shared__ double ty[kDefChunk][kDefRows];
  __shared__ double am[kDefChunk];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int j0 = blockIdx.y * kDefRows;
  const bool col = i > 0 && i < g.nx;
  for (int m0 = 0; m0 < nmodes; m0 += kDefChunk) {
    const int mc = min(kDefChunk, nmodes - m0);
    for (int t = threadIdx.x; t < kDefChunk * 64; t += 256) {
      const int q = t / 64, l = t % 64, ii = blockIdx.x * 64 + l;
      tx[q][l] = (q < mc && ii <= g.nx) ? sx[(int64_t)(m0 + q) * (g.nx + 1) + ii] : 0.0;
    }
    for (int t = threadIdx.x; t < kDefChunk * kDefRows; t += 256) {
      const int q = t / kDefRows, r = t % kDefRows, jj = j0 + r;
      ty[q][r] = (q < mc && jj <= g.ny) ? sy[(int64_t)(m0 + q) * (g.ny + 1) + jj] : 0.0;
    }
    if ((int)threadIdx.x < kDefChunk) {
      const int q = threadIdx.x;
      am[q] = q < mc ? alpha * coef[m0 + q] * (scale ? scale[m0 + q] : 1.0) : 0.0;
    }
    __syncthreads();
    for (int k = (DIM == 3 ? 1 : 0); k < (DIM == 3 ? g.nz : 1); ++k) {
      for (int r = wave; r < kDefRows; r += 4) {
        const int j = j0 + r;
        if (!col || j <= 0 || j >= g.ny) continue;
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < kDefChunk; ++q) {
          double w = am[q] * tx[q][lane] * ty[q][r];
          if (DIM == 3) w *= (q < mc) ? sz[(int64_t)(m0 + q) * (g.nz + 1) + k] : 0.0;
          s += w;
        }
        out[(int64_t)i + (int64_t)j * g.sy + (int64_t)k * g.sz] += s;
      }
    }
    __syncthreads();
  }
}

dim3 mode_grid(const StepGeom &g) {
  return dim3((unsigned)((g.nx + 1 + 63) / 64), (unsigned)((g.ny + 1 + kDefRows - 1) / kDefRows), 1);
}

}  // namespace

int mode_blocks(const StepGeom &g) {
  const dim3 d = mode_grid(g);
  return (int)(d.x * d.y);
}

hipError_t launch_mode_dot(const StepGeom &g, bool fp32, const void *v, int nmodes, const double *sx, const double *sy,
                           const double *sz, double *partials, double *coef, hipStream_t s) {
  if (nmodes <= 0) return hipSuccess;
  const dim3 grid = mode_grid(g);
  const int nb = (int)(grid.x * grid.y);
  if (g.dim == 2) {
    if (fp32)
      mode_dot_kernel<float, 2><<<grid, 256, 0, s>>>(g, static_cast<const float *>(v), nmodes, sx, sy, sz, partials,
                                                     nb);
    else
      mode_dot_kernel<double, 2><<<grid, 256, 0, s>>>(g, static_cast<const double *>(v), nmodes, sx, sy, sz, partials,
                                                      nb);
  } else {
    if (fp32)
      mode_dot_kernel<float, 3><<<grid, 256, 0, s>>>(g, static_cast<const float *>(v), nmodes, sx, sy, sz, partials,
                                                     nb);
    else
      mode_dot_kernel<double, 3><<<grid, 256, 0, s>>>(g, static_cast<const double *>(v), nmodes, sx, sy, sz, partials,
                                                      nb);
  }
  mode_reduce_kernel<<<nmodes, kRedThreads, 0, s>>>(partials, nb, coef);
  return hipGetLastError();
}

hipError_t launch_mode_combine(const StepGeom &g, double *out, int nmodes, const double *sx, const double *sy,
                               const double *sz, const double *coef, const double *scale, double alpha,
                               hipStream_t s) {
  if (nmodes <= 0) return hipSuccess;
  const dim3 grid = mode_grid(g);
  if (g.dim == 2)
    mode_combine_kernel<2><<<grid, 256, 0, s>>>(g, out, nmodes, sx, sy, sz, coef, scale, alpha);
  else
    mode_combine_kernel<3><<<grid, 256, 0, s>>>(g, out, nmodes, sx, sy, sz, coef, scale, alpha);
  return hipGetLastError();
}

}  // namespace wh
