// Temporally blocked leapfrog + filter kernel for 2-D grids (gfx950):
// templates shared by the per-(precision, order) translation units.
//
// One work-group advances a tile of the grid by K leapfrog steps per pass
// over HBM, instead of one:  W^{n-1}, W^n, c^2 (and f) are read once, K steps
// of the explicit scheme (Sec. 4.2.1, eq. WaveSchemeexplicit) are taken on
// chip, the filter terms w_{n+s} W^{n+s} (eq. updateDiscreteExplicit) are
// added to the FP64 accumulator in registers, and W^{n+K-1}, W^{n+K} and the
// accumulator are written once.
//
// Layout on chip.  A work-group is NW wavefronts of 64 lanes.  Lane l of
// every wave holds grid column x0 - H + l; wave w holds rows
// y0 - H + w*RS .. + RS - 1 of that column in registers (W^n, W^{n-1}, c^2,
// f, accumulator).  Neighbours along x come from the adjacent lanes through
// DPP wave shifts (no LDS traffic); neighbours along y are in the lane's own
// registers except across a wave boundary, where the r = p/2 edge rows are
// exchanged through a small double-buffered LDS array (one barrier per step).
// Values at the edges of the region are wrong after each step; the error
// front moves r nodes per step, so with halo H = K*r the owned tile
// (64 - 2H) x (NW*RS - 2H) is exact after K steps.
//
// Walls.  Nodes beyond a wall are loaded as the odd reflection of interior
// nodes (c^2 as the even reflection).  The update is evaluated as the same
// expression on symmetric neighbour-pair sums at every node, so mirrored
// nodes stay exact negatives of their originals and wall nodes stay exactly
// zero through all K steps; no per-step boundary fix-up is needed.  Wall
// nodes are written as 0 explicitly.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "wh_internal.h"

namespace wh {
namespace {

// lane l receives the value of lane l-1 (x - 1); lane 0 receives 0.  The
// bound-control form writes 0 for the lane without a source, so no register
// has to be zeroed first.
__device__ __forceinline__ int dpp_from_left(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
// lane l receives the value of lane l+1 (x + 1); lane 63 receives 0
__device__ __forceinline__ int dpp_from_right(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ float from_left(float v) { return __int_as_float(dpp_from_left(__float_as_int(v))); }
__device__ __forceinline__ float from_right(float v) { return __int_as_float(dpp_from_right(__float_as_int(v))); }
__device__ __forceinline__ double from_left(double v) {
  return __hiloint2double(dpp_from_left(__double2hiint(v)), dpp_from_left(__double2loint(v)));
}
__device__ __forceinline__ double from_right(double v) {
  return __hiloint2double(dpp_from_right(__double2hiint(v)), dpp_from_right(__double2loint(v)));
}

// Odd periodic extension of a node index i of an axis with n cells:
// returns the interior/wall index and the sign of the reflection.
__device__ __forceinline__ int reflect(int i, int n, float &sign) {
  const int two_n = 2 * n;
  int m = i % two_n;
  if (m < 0) m += two_n;
  if (m <= n) return m;
  sign = -sign;
  return two_n - m;
}

// Element e of an array addressed as uniform base + 32-bit byte offset
// (callers guarantee e * sizeof(U) < 2^32).
template <typename U>
__device__ __forceinline__ U ld_at(const U *__restrict__ p, uint32_t e) {
  return *reinterpret_cast<const U *>(reinterpret_cast<const char *>(p) + e * (uint32_t)sizeof(U));
}
template <typename U>
__device__ __forceinline__ void st_at(U *__restrict__ p, uint32_t e, U x) {
  *reinterpret_cast<U *>(reinterpret_cast<char *>(p) + e * (uint32_t)sizeof(U)) = x;
}

// A wave whose rows the error front from the tile's top or bottom edge has
// reached skips the rest of the pass's steps: such rows are never stored and
// feed only rows that are not stored either.  2048^2, 4th order, FP64, K = 6,
// 8 waves of 10 rows: 4 of 48 wave-steps skipped, 1.3% per launch.  (Skipping
// single rows instead makes the compiler keep every row live across the
// branches and spill; skipping rows in the 3-D kernel made it 6% slower.)
#ifndef WH_BLOCK_SKIP_HALO_WAVES
#define WH_BLOCK_SKIP_HALO_WAVES 1
#endif
constexpr bool kSkipHaloWaves = WH_BLOCK_SKIP_HALO_WAVES != 0;

// The FP64 4th-order kernel with variable c^2 keeps the forcing values of its
// tile in LDS (NW*RS x 64 values) instead of registers: with them in
// registers it needs 143 VGPRs, which leaves room for three waves per SIMD
// and so one 8-wave group per CU instead of two.  Each lane reads back only
// what it wrote, so no barrier is needed.
template <typename T, int P, bool FORCE, bool CVAR>
constexpr bool forcing_in_lds() {
  return FORCE && CVAR && sizeof(T) == 8 && P == 4;
}

// XCD-aware tile order: consecutive work-groups are dispatched round-robin
// over the 8 XCDs; give each XCD a contiguous run of tiles so that the halo
// re-reads of neighbouring tiles hit the same L2.
__device__ __forceinline__ int xcd_tile_order(int b, int nblk) {
  const int per_xcd = (nblk + 7) / 8;
  return (b % 8) * per_xcd + (b / 8);
}

// K (ksteps <= K) leapfrog steps of one tile (tx, ty) of one grid: the body
// shared by the single-grid and the batched kernels.
template <typename T, int P, int K, int RS, int NW, bool FORCE, bool CVAR, bool INNER>
__device__ __forceinline__ void advance_tile_impl(
    const StepGeom &g, int ksteps, int tx, int ty, const T *__restrict__ in_prev, const T *__restrict__ in_cur,
    T *__restrict__ out_prev, T *__restrict__ out_cur, double *__restrict__ acc, const T *__restrict__ c2g,
    const T *__restrict__ fg, const BlockCoef &coef, int mode, const double *__restrict__ v,
    double *__restrict__ out, T (*__restrict__ halo)[NW][2][P / 2][64], T (*__restrict__ fsh)[64]) {
  constexpr bool FL = forcing_in_lds<T, P, FORCE, CVAR>();
  constexpr int R = P / 2;
  constexpr int H = K * R;
  constexpr int OX = 64 - 2 * H;
  constexpr int OY = NW * RS - 2 * H;
  static_assert(OX > 0 && OY > 0, "tile too small for the halo");
  static_assert(RS >= R, "each wave must hold at least r rows");

  const int lane = threadIdx.x & 63;
  // the wave index is uniform: keep it (and everything derived from it) in
  // scalar registers so per-row ownership tests are scalar branches
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x0 = tx * OX, y0 = ty * OY;
  const int gx = x0 - H + lane;
  const int gy0 = y0 - H + wave * RS;

  T A[RS], B[RS], C2[RS], F[FL ? 1 : RS];
  double ACC[RS];
  uint32_t own = 0;  // bit q: row q of this lane is an owned interior node
  [[maybe_unused]] uint32_t own_wall = 0;  // bit q: an owned wall node (outputs 0)

  // Inner tiles (tile and halo strictly inside the walls, the usual case)
  // need no reflection and hold no wall node: every row is addressed by one
  // 32-bit byte offset shared by all arrays (uniform base + offset).
  const bool col_in = lane >= H && lane < H + OX;
  const uint32_t base = INNER ? (uint32_t)gx + (uint32_t)gy0 * (uint32_t)g.sy : 0u;
  if constexpr (INNER) {
#pragma unroll
    for (int q = 0; q < RS; ++q) {
      const uint32_t e = base + (uint32_t)q * (uint32_t)g.sy;
      B[q] = ld_at(in_prev, e);
      A[q] = ld_at(in_cur, e);
      C2[q] = CVAR ? ld_at(c2g, e) : static_cast<T>(g.c2const);
      if constexpr (FL) fsh[wave * RS + q][lane] = ld_at(fg, e);
      else F[q] = FORCE ? ld_at(fg, e) : T(0);
      const int r = wave * RS + q;
      ACC[q] = 0.0;
      if (r >= H && r < H + OY) {
        if (col_in) {
          own |= 1u << q;
          ACC[q] = ld_at(acc, e);
        }
      }
    }
  } else {
    float sx = 1.0f;
    const int ix = reflect(gx, g.nx, sx);
    const bool col_owned = col_in && gx <= g.nx;
    const bool col_wall = ix == 0 || ix == g.nx;
    // Every load here is unconditional (a load behind a per-lane test makes
    // the compiler drain all loads in flight at the next wait): the
    // accumulator is read at the nearest node owned by the tile (the node
    // itself if it is owned; never a node another tile writes) and used only
    // at owned interior nodes; owned wall nodes get their zeros at the end.
    const int64_t ax = min(max(gx, x0), min(x0 + OX - 1, g.nx));
    const int ay_lo = y0, ay_hi = min(y0 + OY - 1, g.ny);
#pragma unroll
    for (int q = 0; q < RS; ++q) {
      float s = sx;
      const int gy = gy0 + q;
      const int iy = reflect(gy, g.ny, s);
      const int64_t id = (int64_t)ix + (int64_t)iy * g.sy;
      const T sg = static_cast<T>(s);
      B[q] = sg * in_prev[id];
      A[q] = sg * in_cur[id];
      C2[q] = CVAR ? c2g[id] : static_cast<T>(g.c2const);
      if constexpr (FL) fsh[wave * RS + q][lane] = sg * fg[id];
      else F[q] = FORCE ? sg * fg[id] : T(0);
      ACC[q] = acc[ax + (int64_t)min(max(gy, ay_lo), ay_hi) * g.sy];
      const int r = wave * RS + q;
      const bool in_tile = col_owned && r >= H && r < H + OY && gy <= g.ny;
      const bool wall = col_wall || iy == 0 || iy == g.ny;
      if (in_tile && !wall) own |= 1u << q;
      else if (in_tile) own_wall |= 1u << q;
    }
  }

  // c^2 folded into two per-node coefficients: with X, Y the x and y
  // stencil sums, W^{n+1} = (2 - c^2 kc) W^n + c^2 kx (X + (ky/kx) Y) - W^{n-1}
  // (2 - c^2 kc) is rebuilt from c^2 kx with one FMA per use, which keeps
  // one register pair per row free for a taller tile
  T CB[RS];
  {
    const T kx = static_cast<T>(g.kx);
#pragma unroll
    for (int q = 0; q < RS; ++q) CB[q] = C2[q] * kx;
  }
  const T rc = static_cast<T>(g.kc / g.kx);
  const T ry = static_cast<T>(g.ky / g.kx);

#pragma unroll
  for (int s = 0; s < K; ++s) {
    if (s < ksteps) {
      T *cur = (s & 1) ? B : A;
      T *prv = (s & 1) ? A : B;
      // y-halo: publish this wave's edge rows, fetch the neighbours'
      const int hb = s & 1;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        halo[hb][wave][0][k][lane] = cur[k];           // top rows
        halo[hb][wave][1][k][lane] = cur[RS - R + k];  // bottom rows
      }
      __syncthreads();
      T up[R], dn[R];
#pragma unroll
      for (int k = 0; k < R; ++k) {
        up[k] = wave > 0 ? halo[hb][wave - 1][1][k][lane] : T(0);      // rows above: q = k - R
        dn[k] = wave < NW - 1 ? halo[hb][wave + 1][0][k][lane] : T(0);  // rows below: q = RS + k
      }
      const T gn = static_cast<T>(coef.gn[s]);
      const double wn = coef.wn[s];
      // rows within r (s + 1) of the tile's top or bottom edge are wrong
      // after this step and feed only rows that are wrong too: a wave whose
      // rows all lie there skips the step (a scalar branch; it still takes
      // part in the halo exchange and its barrier)
      if (kSkipHaloWaves && ((wave + 1) * RS <= R * (s + 1) || wave * RS >= NW * RS - R * (s + 1))) continue;
#pragma unroll
      for (int q = 0; q < RS; ++q) {
        auto row = [&](int qq) -> T {
          if (qq < 0) return up[qq + R];
          if (qq >= RS) return dn[qq - RS];
          return cur[qq];
        };
        const T c = cur[q];
        const T xl1 = from_left(c), xr1 = from_right(c);
        T S;
        if (P == 2) {
          S = (xl1 + xr1) + ry * (row(q - 1) + row(q + 1));
        } else {
          const T xl2 = from_left(xl1), xr2 = from_right(xr1);
          const T X = T(16) * (xl1 + xr1) - (xl2 + xr2);
          const T Y = T(16) * (row(q - 1) + row(q + 1)) - (row(q - 2) + row(q + 2));
          S = X + ry * Y;
        }
        T nxt = (T(2) - rc * CB[q]) * c - prv[q] + CB[q] * S;
        if constexpr (FL) nxt += gn * fsh[wave * RS + q][lane];
        else if (FORCE) nxt += gn * F[q];
        prv[q] = nxt;
        ACC[q] += wn * static_cast<double>(nxt);
      }
    }
  }

  // after ksteps steps the newest level is in B if ksteps is odd, else in A
  const bool odd = ksteps & 1;
  if constexpr (INNER) {
    if (col_in) {
#pragma unroll
      for (int q = 0; q < RS; ++q) {
        const int r = wave * RS + q;
        if (r < H || r >= H + OY) continue;
        const uint32_t e = base + (uint32_t)q * (uint32_t)g.sy;
        st_at(out_cur, e, odd ? B[q] : A[q]);
        st_at(out_prev, e, odd ? A[q] : B[q]);
        if (mode == ACCUMULATE) st_at(acc, e, ACC[q]);
        else if (mode == FINAL_FILTER) st_at(out, e, ACC[q]);
        else st_at(out, e, ld_at(v, e) - ACC[q]);
      }
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < RS; ++q) {
    const int64_t id = (int64_t)gx + (int64_t)(gy0 + q) * g.sy;  // owned nodes need no reflection
    if ((own_wall >> q) & 1u) {
      // wall node owned by this tile: its outputs are exactly 0
      out_prev[id] = T(0);
      out_cur[id] = T(0);
      if (mode != ACCUMULATE) out[id] = 0.0;
      continue;
    }
    if (!((own >> q) & 1u)) continue;
    out_cur[id] = odd ? B[q] : A[q];
    out_prev[id] = odd ? A[q] : B[q];
    if (mode == ACCUMULATE) acc[id] = ACC[q];
    else if (mode == FINAL_FILTER) out[id] = ACC[q];
    else out[id] = v[id] - ACC[q];
  }
}

template <typename T, int P, int K, int RS, int NW, bool FORCE, bool CVAR>
__device__ __forceinline__ void advance_tile(const StepGeom &g, int ksteps, int tx, int ty,
                                             const T *__restrict__ in_prev, const T *__restrict__ in_cur,
                                             T *__restrict__ out_prev, T *__restrict__ out_cur,
                                             double *__restrict__ acc, const T *__restrict__ c2g,
                                             const T *__restrict__ fg, const BlockCoef &coef, int mode,
                                             const double *__restrict__ v, double *__restrict__ out,
                                             T (*__restrict__ halo)[NW][2][P / 2][64], T (*__restrict__ fsh)[64]) {
  constexpr int H = K * (P / 2);
  constexpr int OX = 64 - 2 * H;
  constexpr int OY = NW * RS - 2 * H;
  const int x0 = tx * OX - H, y0 = ty * OY - H;
  // uniform over the work-group: one of the two bodies runs
  const bool inner = x0 >= 1 && x0 + 63 <= g.nx - 1 && y0 >= 1 && y0 + NW * RS - 1 <= g.ny - 1 &&
                     g.nodes <= (int64_t(1) << 28);
  if (inner)
    advance_tile_impl<T, P, K, RS, NW, FORCE, CVAR, true>(g, ksteps, tx, ty, in_prev, in_cur, out_prev, out_cur, acc,
                                                          c2g, fg, coef, mode, v, out, halo, fsh);
  else
    advance_tile_impl<T, P, K, RS, NW, FORCE, CVAR, false>(g, ksteps, tx, ty, in_prev, in_cur, out_prev, out_cur,
                                                           acc, c2g, fg, coef, mode, v, out, halo, fsh);
}

template <typename T, int P, int K, int RS, int NW, bool FORCE, bool CVAR>
__global__ __launch_bounds__(64 * NW) void block_steps_kernel(
    StepGeom g, int ksteps, int tiles_x, int tiles_total, const T *__restrict__ in_prev,
    const T *__restrict__ in_cur, T *__restrict__ out_prev, T *__restrict__ out_cur, double *__restrict__ acc,
    const T *__restrict__ c2g, const T *__restrict__ fg, BlockCoef coef, int mode, const double *__restrict__ v,
    double *__restrict__ out) {
  __shared__ T halo[2][NW][2][P / 2][64];  // y-halo rows, double-buffered over steps
  __shared__ T fsh[forcing_in_lds<T, P, FORCE, CVAR>() ? NW * RS : 1][64];
  const int tile = xcd_tile_order(blockIdx.x, gridDim.x);
  if (tile >= tiles_total) return;
  advance_tile<T, P, K, RS, NW, FORCE, CVAR>(g, ksteps, tile % tiles_x, tile / tiles_x, in_prev, in_cur, out_prev,
                                             out_cur, acc, c2g, fg, coef, mode, v, out, halo, fsh);
}

// Batched pass: work-group -> (problem, tile) through the prefix sums of the
// active problems' tile counts (problems are sorted by pass count, so the
// problems still stepping in pass `pass` are a prefix of the table).
template <typename T, int P, int K, int RS, int NW, bool FORCE>
__global__ __launch_bounds__(64 * NW) void batch_block_steps_kernel(const BatchDesc *__restrict__ descs,
                                                                    const int *__restrict__ tile_prefix, int nactive,
                                                                    int pass, const BlockCoef *__restrict__ coefs,
                                                                    int final_mode) {
  __shared__ T halo[2][NW][2][P / 2][64];
  __shared__ T fsh[forcing_in_lds<T, P, FORCE, true>() ? NW * RS : 1][64];
  const int total = tile_prefix[nactive];
  const int tile = xcd_tile_order(blockIdx.x, gridDim.x);
  if (tile >= total) return;
  int lo = 0, hi = nactive - 1;  // last problem whose first tile is <= tile
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_prefix[mid] <= tile) lo = mid;
    else hi = mid - 1;
  }
  const BatchDesc &d = descs[lo];
  const int local = tile - tile_prefix[lo];
  const int ks = min(K, d.steps - pass * K);
  const int mode = (pass == d.passes - 1) ? final_mode : ACCUMULATE;
  const bool even = (pass & 1) == 0;
  const T *ip = static_cast<const T *>(even ? d.W[0] : d.W[2]);
  const T *ic = static_cast<const T *>(even ? d.W[1] : d.W[3]);
  T *op = static_cast<T *>(even ? d.W[2] : d.W[0]);
  T *oc = static_cast<T *>(even ? d.W[3] : d.W[1]);
  const BlockCoef coef = coefs[d.coef_offset + pass];
  const int tx = local % d.tiles_x, ty = local / d.tiles_x;
  if (d.c2)
    advance_tile<T, P, K, RS, NW, FORCE, true>(d.g, ks, tx, ty, ip, ic, op, oc, d.acc, static_cast<const T *>(d.c2),
                                               static_cast<const T *>(d.f), coef, mode, d.v, d.out, halo, fsh);
  else
    advance_tile<T, P, K, RS, NW, FORCE, false>(d.g, ks, tx, ty, ip, ic, op, oc, d.acc, nullptr,
                                                static_cast<const T *>(d.f), coef, mode, d.v, d.out, halo, fsh);
}

template <typename T, int P, int K, int RS, int NW>
hipError_t launch_typed(const StepGeom &g, int ksteps, const void *in_prev, const void *in_cur, void *out_prev,
                        void *out_cur, double *acc, const void *c2, const void *f, const BlockCoef &coef, int mode,
                        const double *v, double *out, hipStream_t s) {
  constexpr int H = K * (P / 2);
  constexpr int OX = 64 - 2 * H;
  constexpr int OY = NW * RS - 2 * H;
  const int tiles_x = (g.nx + 1 + OX - 1) / OX;
  const int tiles_y = (g.ny + 1 + OY - 1) / OY;
  const int tiles = tiles_x * tiles_y;
  const int blocks = ((tiles + 7) / 8) * 8;
  const T *ip = static_cast<const T *>(in_prev);
  const T *ic = static_cast<const T *>(in_cur);
  T *op = static_cast<T *>(out_prev);
  T *oc = static_cast<T *>(out_cur);
  const T *cc = static_cast<const T *>(c2);
  const T *ff = static_cast<const T *>(f);
  dim3 grid(blocks), block(64 * NW);
  if (f && c2)
    block_steps_kernel<T, P, K, RS, NW, true, true><<<grid, block, 0, s>>>(g, ksteps, tiles_x, tiles, ip, ic, op, oc,
                                                                          acc, cc, ff, coef, mode, v, out);
  else if (f)
    block_steps_kernel<T, P, K, RS, NW, true, false><<<grid, block, 0, s>>>(g, ksteps, tiles_x, tiles, ip, ic, op, oc,
                                                                           acc, cc, ff, coef, mode, v, out);
  else if (c2)
    block_steps_kernel<T, P, K, RS, NW, false, true><<<grid, block, 0, s>>>(g, ksteps, tiles_x, tiles, ip, ic, op,
                                                                           oc, acc, cc, ff, coef, mode, v, out);
  else
    block_steps_kernel<T, P, K, RS, NW, false, false><<<grid, block, 0, s>>>(g, ksteps, tiles_x, tiles, ip, ic, op,
                                                                            oc, acc, cc, ff, coef, mode, v, out);
  return hipGetLastError();
}

// Rows per lane: FP32 keeps 24 rows per lane, FP64 10 for p = 4 and 8 for
// p = 2 (the fastest measured; larger register arrays are not promoted to
// VGPRs, or cost occupancy).  Waves per work-group (NW) set the tile height
// NW * RS; smaller groups let two groups share a CU so that one group's loads
// overlap the other's arithmetic.
template <typename T, int P>
struct RowsPerLane {
  static constexpr int RS = sizeof(T) == 8 ? (P == 4 ? 10 : 8) : 24;
};

template <typename T, int P, int K, int NW>
hipError_t launch_if_fits(const StepGeom &g, int ksteps, const void *ip, const void *ic, void *op, void *oc,
                          double *acc, const void *c2, const void *f, const BlockCoef &coef, int mode,
                          const double *v, double *out, hipStream_t s) {
  constexpr int RS = RowsPerLane<T, P>::RS;
  if constexpr (NW * RS - 2 * K * (P / 2) > 0)
    return launch_typed<T, P, K, RS, NW>(g, ksteps, ip, ic, op, oc, acc, c2, f, coef, mode, v, out, s);
  return hipErrorInvalidValue;
}

template <typename T, int P, int K>
hipError_t dispatch_nw(const StepGeom &g, int nw, int ksteps, const void *ip, const void *ic, void *op, void *oc,
                       double *acc, const void *c2, const void *f, const BlockCoef &coef, int mode, const double *v,
                       double *out, hipStream_t s) {
  switch (nw) {
    case 4: return launch_if_fits<T, P, K, 4>(g, ksteps, ip, ic, op, oc, acc, c2, f, coef, mode, v, out, s);
    case 8: return launch_if_fits<T, P, K, 8>(g, ksteps, ip, ic, op, oc, acc, c2, f, coef, mode, v, out, s);
    // FP32's 24-row arrays do not fit groups of more than 8 waves; FP64
    // groups of 16 waves would spill
    case 10:
      if constexpr (sizeof(T) == 8)
        return launch_if_fits<T, P, K, 10>(g, ksteps, ip, ic, op, oc, acc, c2, f, coef, mode, v, out, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// Steps per launch: 2..6 for p = 4 (halo 2K); 2, 3, 4, 6, 8 for p = 2 (halo K).
constexpr bool k_instantiated(int P, int K) {
  return P == 4 ? (K >= 2 && K <= 6) : (K == 2 || K == 3 || K == 4 || K == 6 || K == 8);
}

template <typename T, int P>
hipError_t dispatch_k(const StepGeom &g, int K, int nw, int ksteps, const void *ip, const void *ic, void *op,
                      void *oc, double *acc, const void *c2, const void *f, const BlockCoef &coef, int mode,
                      const double *v, double *out, hipStream_t s) {
  switch (K) {
    case 2: return dispatch_nw<T, P, 2>(g, nw, ksteps, ip, ic, op, oc, acc, c2, f, coef, mode, v, out, s);
    case 3: return dispatch_nw<T, P, 3>(g, nw, ksteps, ip, ic, op, oc, acc, c2, f, coef, mode, v, out, s);
    case 4: return dispatch_nw<T, P, 4>(g, nw, ksteps, ip, ic, op, oc, acc, c2, f, coef, mode, v, out, s);
    case 5:
      if constexpr (k_instantiated(P, 5))
        return dispatch_nw<T, P, 5>(g, nw, ksteps, ip, ic, op, oc, acc, c2, f, coef, mode, v, out, s);
      return hipErrorInvalidValue;
    case 6: return dispatch_nw<T, P, 6>(g, nw, ksteps, ip, ic, op, oc, acc, c2, f, coef, mode, v, out, s);
    case 8:
      if constexpr (k_instantiated(P, 8))
        return dispatch_nw<T, P, 8>(g, nw, ksteps, ip, ic, op, oc, acc, c2, f, coef, mode, v, out, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int P, int K, int NW>
hipError_t batch_launch_fits(bool force, const BatchDesc *descs, const int *tile_prefix, int nactive, int total,
                             int pass, const BlockCoef *coefs, int final_mode, hipStream_t s) {
  constexpr int RS = RowsPerLane<T, P>::RS;
  if constexpr (NW * RS - 2 * K * (P / 2) > 0) {
    const int blocks = ((total + 7) / 8) * 8;
    if (force)
      batch_block_steps_kernel<T, P, K, RS, NW, true><<<blocks, 64 * NW, 0, s>>>(descs, tile_prefix, nactive, pass,
                                                                                 coefs, final_mode);
    else
      batch_block_steps_kernel<T, P, K, RS, NW, false><<<blocks, 64 * NW, 0, s>>>(descs, tile_prefix, nactive, pass,
                                                                                  coefs, final_mode);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <typename T, int P, int K>
hipError_t batch_nw(int nw, bool force, const BatchDesc *descs, const int *tp, int nactive, int total, int pass,
                    const BlockCoef *coefs, int final_mode, hipStream_t s) {
  switch (nw) {
    case 4: return batch_launch_fits<T, P, K, 4>(force, descs, tp, nactive, total, pass, coefs, final_mode, s);
    case 8: return batch_launch_fits<T, P, K, 8>(force, descs, tp, nactive, total, pass, coefs, final_mode, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int P>
hipError_t batch_k(int K, int nw, bool force, const BatchDesc *descs, const int *tp, int nactive, int total, int pass,
                   const BlockCoef *coefs, int final_mode, hipStream_t s) {
  switch (K) {
    case 2: return batch_nw<T, P, 2>(nw, force, descs, tp, nactive, total, pass, coefs, final_mode, s);
    case 3: return batch_nw<T, P, 3>(nw, force, descs, tp, nactive, total, pass, coefs, final_mode, s);
    case 4: return batch_nw<T, P, 4>(nw, force, descs, tp, nactive, total, pass, coefs, final_mode, s);
    case 5:
      if constexpr (k_instantiated(P, 5))
        return batch_nw<T, P, 5>(nw, force, descs, tp, nactive, total, pass, coefs, final_mode, s);
      return hipErrorInvalidValue;
    case 6: return batch_nw<T, P, 6>(nw, force, descs, tp, nactive, total, pass, coefs, final_mode, s);
    case 8:
      if constexpr (k_instantiated(P, 8))
        return batch_nw<T, P, 8>(nw, force, descs, tp, nactive, total, pass, coefs, final_mode, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}
}  // namespace
}  // namespace wh
