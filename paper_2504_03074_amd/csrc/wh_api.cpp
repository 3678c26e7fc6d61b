// C ABI of the WaveHoltz library: context, validation, time parameters,
// workspace layout, one WaveHoltz application, and the outer solvers
// (fixed-point iteration of Alg. 1 and restarted GMRES on (I - S_h) v = b,
// Sec. 5.3).  All grid-sized work runs in the HIP kernels; this file only
// sequences launches and does O(restart^2) host arithmetic (Hessenberg,
// Givens rotations).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "wh.h"
#include "wh_internal.h"

struct wh_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  bool grid_set = false;
  int dim = 0, order = 0, prec = WH_FP64;
  int64_t n[3] = {0, 0, 0};
  int64_t nodes = 0;

  char *ws = nullptr;
  size_t ws_bytes = 0;
  int ws_restart = 0;
  void *c2 = nullptr;
  void *f = nullptr;
  void *W[4] = {nullptr, nullptr, nullptr, nullptr};
  double *acc = nullptr, *tmp = nullptr, *b = nullptr, *V = nullptr, *partials = nullptr, *scal = nullptr;
  int64_t ldv = 0;

  bool c2_set = false, c2_is_const = false;
  double c2_value = 1.0, c2max = 1.0;
  bool f_set = false;
  bool freq_set = false;
  wh_time_params tp{};
  std::vector<double> wts;   // filter weight of level n, n = 0..N
  std::vector<double> frc;   // -dt^2 cos(omega_e t^n), n = 0..N-1

  int kernel = WH_KERNEL_AUTO, kblock = 0, tile = 0;
  char *adj = nullptr;  // adjoint workspace (checkpoints, reverse sweep)
  size_t adj_bytes = 0;
  // deflation with sine modes (count 0 = off)
  int defl_count = 0;
  std::vector<int32_t> defl_modes;  // count x dim wave numbers
  std::vector<double> defl_lam2;    // eigenvalue of -L_h per mode
  double *d_sx = nullptr, *d_sy = nullptr, *d_sz = nullptr;
  double *d_coef = nullptr, *d_coef_f = nullptr, *d_scale = nullptr, *d_dpart = nullptr;
  double *pinned = nullptr;  // host staging for reduction results
  size_t pinned_count = 0;

  // implicit time stepping (2-D, FP64 state): steps per period, tolerance of
  // the inner solves, and the multigrid hierarchy held in the caller's
  // implicit workspace
  bool implicit = false;
  int nits = 10;
  double imp_rtol = 1e-12;
  char *imp = nullptr;
  size_t imp_bytes = 0;
  struct MgLevel {
    wh::MgGeom g;
    double *d, *x, *b, *t;  // 1/c^2, solution, right-hand side, smoother buffer
  };
  std::vector<MgLevel> mg;
  double dconst = 1.0;  // 1/c^2 when c^2 is constant (d == nullptr)
  bool mg_ready = false;
  hipStream_t mg_cap = nullptr;  // capture stream of the V-cycle graph
  hipGraph_t mg_graph = nullptr;
  hipGraphExec_t mg_exec = nullptr;
  double *imp_r = nullptr, *imp_z = nullptr, *imp_p = nullptr, *imp_q = nullptr;
  double *imp_part = nullptr, *imp_scal = nullptr;
  int64_t imp_steps = 0, imp_iters = 0;
  int imp_max = 0;

  struct Timed {
    hipEvent_t a, b;
    int64_t launches;
    double bytes, point_steps;
  };
  bool profiling = false;
  std::vector<Timed> pending;
  std::vector<hipEvent_t> event_pool;
  wh_profile prof{};
};

namespace {

constexpr int kMaxScalars = 4 * (WH_MAX_RESTART + 2);

wh_status fail(wh_ctx *ctx, wh_status st, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

#define WH_HIP(ctx, call)                                                                          \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      return fail((ctx), WH_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));               \
  } while (0)

#define WH_TRY(expr)                 \
  do {                               \
    wh_status s_ = (expr);           \
    if (s_ != WH_OK) return s_;      \
  } while (0)

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t state_bytes(const wh_ctx *c) { return c->prec == WH_FP32_STATE ? 4 : 8; }

struct Layout {
  size_t c2, f, W[4], acc, tmp, b, V, partials, scal, total;
  int64_t ldv;
};

Layout layout(const wh_ctx *c, int restart) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t nb = (size_t)c->nodes;
  const size_t T = state_bytes(c);
  L.c2 = take(nb * T);
  L.f = take(nb * T);
  for (int i = 0; i < 4; ++i) L.W[i] = take(nb * T);
  L.acc = take(nb * 8);
  L.tmp = take(nb * 8);
  L.b = take(nb * 8);
  L.ldv = (int64_t)(align256(nb * 8) / 8);
  L.V = take(restart > 0 ? (size_t)(restart + 1) * (size_t)L.ldv * 8 : 0);
  const int rows = std::max(restart + 1, 3);
  L.partials = take((size_t)rows * (size_t)wh::reduction_blocks(c->nodes) * 8);
  L.scal = take((size_t)kMaxScalars * 8);
  L.total = off;
  return L;
}

// Geometry with the stencil scaled by `scale` (dt^2 for the steps, dt^2/2
// for the first step, 1 for the Helmholtz residual).
wh::StepGeom geometry(const wh_ctx *c, double scale) {
  wh::StepGeom g{};
  g.dim = c->dim;
  g.order = c->order;
  g.nx = (int)c->n[0];
  g.ny = (int)c->n[1];
  g.nz = c->dim == 3 ? (int)c->n[2] : 0;
  g.sy = c->n[0] + 1;
  g.sz = (c->n[0] + 1) * (c->n[1] + 1);
  g.nodes = c->nodes;
  const double div = c->order == 4 ? 12.0 : 1.0;
  const double centre = c->order == 4 ? 30.0 : 2.0;
  g.kx = scale * (double)c->n[0] * (double)c->n[0] / div;
  g.ky = scale * (double)c->n[1] * (double)c->n[1] / div;
  g.kz = c->dim == 3 ? scale * (double)c->n[2] * (double)c->n[2] / div : 0.0;
  g.kc = centre * (g.kx + g.ky + g.kz);
  g.c2const = c->c2_value;
  return g;
}

wh_status need(wh_ctx *c, bool grid, bool ws, bool c2, bool f, bool freq) {
  if (!c) return WH_EINVAL;
  if (grid && !c->grid_set) return fail(c, WH_ESTATE, "grid not set (call wh_set_grid first)");
  if (ws && !c->ws) return fail(c, WH_ENOMEM, "no workspace bound (call wh_bind_workspace)");
  if (c2 && !c->c2_set) return fail(c, WH_ESTATE, "c^2 not set (call wh_set_c2 or wh_set_c2_constant)");
  if (f && !c->f_set) return fail(c, WH_ESTATE, "source not set (call wh_set_source)");
  if (freq && !c->freq_set) return fail(c, WH_ESTATE, "frequency not set (call wh_set_frequency)");
  return WH_OK;
}

wh_status set_device(wh_ctx *c) {
  WH_HIP(c, hipSetDevice(c->device));
  return WH_OK;
}

// Reduce `k` rows of partials into scal[dst..dst+k) on the device.
wh_status reduce_to(wh_ctx *c, int k, int dst) {
  const int nb = wh::reduction_blocks(c->nodes);
  WH_HIP(c, wh::launch_reduce_rows(c->partials, nb, k, c->scal + dst, c->stream));
  return WH_OK;
}

wh_status fetch_scalars(wh_ctx *c, int first, int count, double *out) {
  WH_HIP(c, hipMemcpyAsync(c->pinned, c->scal + first, (size_t)count * 8, hipMemcpyDeviceToHost, c->stream));
  WH_HIP(c, hipStreamSynchronize(c->stream));
  std::memcpy(out, c->pinned, (size_t)count * 8);
  return WH_OK;
}

// sum_e x_e y_e -> scal[dst] (device), deterministic.
wh_status dot_dev(wh_ctx *c, const double *x, const double *y, int dst) {
  const int nb = wh::reduction_blocks(c->nodes);
  WH_HIP(c, wh::launch_mdot(x, 0, 1, y, c->nodes, c->partials, nb, c->stream));
  return reduce_to(c, 1, dst);
}

// Is ptr device memory usable on ctx->device?
bool is_device_ptr(const void *p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

wh_status check_dev(wh_ctx *c, const void *p, const char *name) {
  if (!p) return fail(c, WH_EINVAL, "%s is NULL", name);
  if (!is_device_ptr(p)) return fail(c, WH_EINVAL, "%s is not device memory", name);
  return WH_OK;
}

// Copy a caller node array (host or device, FP64) into a workspace array in
// state precision.
wh_status upload_field(wh_ctx *c, const double *src, int on_device, void *dst) {
  const bool fp32 = c->prec == WH_FP32_STATE;
  const size_t bytes = (size_t)c->nodes * 8;
  if (on_device) {
    if (fp32) {
      WH_HIP(c, wh::launch_to_state(true, src, dst, c->nodes, c->stream));
    } else {
      WH_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
    }
  } else {
    if (fp32) {
      // stage in the FP64 accumulator, then convert
      WH_HIP(c, hipMemcpyAsync(c->acc, src, bytes, hipMemcpyHostToDevice, c->stream));
      WH_HIP(c, wh::launch_to_state(true, c->acc, dst, c->nodes, c->stream));
    } else {
      WH_HIP(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
    }
    WH_HIP(c, hipStreamSynchronize(c->stream));  // the host buffer may be freed on return
  }
  return WH_OK;
}

void build_tables(wh_ctx *c) {
  const int64_t nt = c->tp.nt, N = (int64_t)c->tp.nt * c->tp.periods;
  const double two_pi = 2.0 * M_PI;
  c->wts.assign((size_t)N + 1, 0.0);
  c->frc.assign((size_t)N, 0.0);
  const double norm = 2.0 / (double)N;
  for (int64_t m = 0; m <= N; ++m) {
    const double phase = std::cos(two_pi * (double)(m % nt) / (double)nt);
    const double sigma = (m == 0 || m == N) ? 0.5 : 1.0;
    c->wts[(size_t)m] = norm * sigma * (phase - 0.5 * c->tp.alpha);
    if (m < N) c->frc[(size_t)m] = -c->tp.dt * c->tp.dt * phase;
  }
}

double interior_nodes(const wh_ctx *c) {
  double u = 1.0;
  for (int m = 0; m < c->dim; ++m) u *= (double)(c->n[m] - 1);
  return u;
}

wh_status take_events(wh_ctx *c, hipEvent_t *a, hipEvent_t *b) {
  for (hipEvent_t *e : {a, b}) {
    if (!c->event_pool.empty()) {
      *e = c->event_pool.back();
      c->event_pool.pop_back();
    } else {
      WH_HIP(c, hipEventCreate(e));
    }
  }
  return WH_OK;
}

// Wait for the recorded applications and fold their times into the counters.
wh_status drain_profile(wh_ctx *c) {
  WH_HIP(c, hipStreamSynchronize(c->stream));
  for (auto &t : c->pending) {
    float ms = 0.0f;
    WH_HIP(c, hipEventElapsedTime(&ms, t.a, t.b));
    c->prof.applies += 1;
    c->prof.launches += t.launches;
    c->prof.ms += ms;
    c->prof.bytes += t.bytes;
    c->prof.point_steps += t.point_steps;
    c->event_pool.push_back(t.a);
    c->event_pool.push_back(t.b);
  }
  c->pending.clear();
  return WH_OK;
}

// Leapfrog steps per blocked launch when the caller does not choose: the
// fastest measured on MI355X at the default tile heights (2048^2: K = 6 for
// p = 4, K = 8 for p = 2 — more steps per HBM pass outweigh the larger halo
// until the arithmetic dominates).
int default_kblock(int order, bool fp32) {
  (void)fp32;
  return order == 2 ? 8 : 6;
}

struct Tuning {
  int kernel, kblock, tile;
};

bool tuning_supported(const wh_ctx *c, int kernel, int kblock, int tile);

// The kernel family, steps per launch and tile parameter actually used.
Tuning resolve_tuning(const wh_ctx *c) {
  const bool fp32 = c->prec == WH_FP32_STATE;
  if (c->kernel == WH_KERNEL_AUTO) {
    if (c->dim == 2)
      return {WH_KERNEL_BLOCKED_2D, default_kblock(c->order, fp32), wh::block_default_rows(fp32, c->order)};
    // the fastest measured per state type and order; FP64 p = 2 at K = 4 and
    // FP64 p = 4 at K >= 3 run out of registers and spill; FP32 p = 4 at K = 2
    // stages two planes ahead, which makes it faster per step than K = 3
    const int k3 = c->order == 2 ? (fp32 ? 4 : 3) : 2;
    if (tuning_supported(c, WH_KERNEL_BLOCKED_3D, k3, 0))
      return {WH_KERNEL_BLOCKED_3D, k3, wh::block3d_default_rows(fp32, c->order, k3)};
    return {WH_KERNEL_NODE, 1, 0};
  }
  if (c->kernel == WH_KERNEL_BLOCKED_2D)
    return {c->kernel, c->kblock, c->tile > 0 ? c->tile : wh::block_default_rows(fp32, c->order)};
  if (c->kernel == WH_KERNEL_ZCOL_3D) return {c->kernel, 1, c->tile > 0 ? c->tile : 8};
  if (c->kernel == WH_KERNEL_BLOCKED_3D)
    return {c->kernel, c->kblock, c->tile > 0 ? c->tile : wh::block3d_default_rows(fp32, c->order, c->kblock)};
  return {WH_KERNEL_NODE, 1, 0};
}

bool tuning_supported(const wh_ctx *c, int kernel, int kblock, int tile) {
  const bool fp32 = c->prec == WH_FP32_STATE;
  switch (kernel) {
    case WH_KERNEL_AUTO: return kblock == 0 && tile == 0;
    case WH_KERNEL_NODE: return kblock <= 1 && tile == 0;
    case WH_KERNEL_BLOCKED_2D:
      return c->dim == 2 && kblock >= 2 && kblock <= wh::kMaxBlockSteps &&
             (tile == 0 || wh::block_config_supported(fp32, c->order, kblock, tile));
    case WH_KERNEL_ZCOL_3D: return c->dim == 3 && kblock <= 1 && (tile == 0 || wh::zcol_supported(tile));
    case WH_KERNEL_BLOCKED_3D:
      if (c->dim != 3 || kblock < 1 || kblock > wh::kMaxBlockSteps3d) return false;
      if ((double)(c->n[0] + 1) * (double)(c->n[1] + 1) * 8.0 >= 4294967296.0) return false;
      // the last pass of an application may take fewer steps: every smaller
      // K must be supported with the same rows
      for (int k = 1; k <= kblock; ++k)
        if (!wh::block3d_config_supported(fp32, c->order, k,
                                          tile == 0 ? wh::block3d_default_rows(fp32, c->order, kblock) : tile))
          return false;
      return true;
    default: return false;
  }
}

// ---------------------------------------------------------------------------
// implicit time stepping (Sec. 4.2.2): multigrid-preconditioned CG per step
// ---------------------------------------------------------------------------
constexpr int kMgPreSweeps = 2;     // = post-sweeps (symmetric V-cycle)
constexpr int kMgCoarseSweeps = 20;  // even: the result ends in x
constexpr int kImpMaxInner = 500;

// Grid sizes of the multigrid levels: halve while both axes are even and the
// coarse grid keeps at least two cells per axis.
std::vector<std::pair<int, int>> mg_shapes(const wh_ctx *c) {
  std::vector<std::pair<int, int>> out;
  int nx = (int)c->n[0], ny = (int)c->n[1];
  out.push_back({nx, ny});
  while (nx % 2 == 0 && ny % 2 == 0 && nx >= 4 && ny >= 4) {
    nx /= 2;
    ny /= 2;
    out.push_back({nx, ny});
  }
  return out;
}

struct ImpLayout {
  size_t total = 0;
  std::vector<size_t> off;  // level 0: d, t, r, z, p, q; level l >= 1: d, x, b, t; then partials, scalars
};

ImpLayout imp_layout(const wh_ctx *c) {
  ImpLayout L;
  auto seg = [&](size_t bytes) {
    L.off.push_back(L.total);
    L.total += (bytes + 255) / 256 * 256;
  };
  const auto shapes = mg_shapes(c);
  for (size_t l = 0; l < shapes.size(); ++l) {
    const size_t nodes = (size_t)(shapes[l].first + 1) * (size_t)(shapes[l].second + 1);
    for (int a = 0; a < (l == 0 ? 6 : 4); ++a) seg(nodes * 8);
  }
  seg((size_t)wh::reduction_blocks(c->nodes) * 8);
  seg(16 * 8);
  return L;
}

// Level geometry for theta = dt^2 / 2 (fine level: order p; coarse: order 2).
wh::MgGeom mg_geom(int nx, int ny, int order, double theta) {
  wh::MgGeom g{};
  g.nx = nx;
  g.ny = ny;
  g.sy = nx + 1;
  g.nodes = (int64_t)(nx + 1) * (ny + 1);
  g.order = order;
  const double div = order == 4 ? 12.0 : 1.0;
  g.ax = theta * (double)nx * nx / div;
  g.ay = theta * (double)ny * ny / div;
  g.ac = (order == 4 ? 30.0 : 2.0) * (g.ax + g.ay);
  return g;
}

wh_status mg_vcycle(wh_ctx *c, size_t l, hipStream_t s);

wh_status mg_drop_graph(wh_ctx *c) {
  if (c->mg_exec || c->mg_graph) WH_HIP(c, hipStreamSynchronize(c->stream));  // no replay in flight
  if (c->mg_exec) (void)hipGraphExecDestroy(c->mg_exec);
  if (c->mg_graph) (void)hipGraphDestroy(c->mg_graph);
  c->mg_exec = nullptr;
  c->mg_graph = nullptr;
  return WH_OK;
}

wh_status mg_setup(wh_ctx *c) {
  if (!c->imp) return fail(c, WH_ESTATE, "implicit stepping needs its workspace (wh_bind_implicit_workspace)");
  const ImpLayout L = imp_layout(c);
  const auto shapes = mg_shapes(c);
  const double theta = 0.5 * c->tp.dt * c->tp.dt;
  auto at = [&](size_t k) { return reinterpret_cast<double *>(c->imp + L.off[k]); };
  c->mg.clear();
  size_t k = 0;
  const bool cvar = !c->c2_is_const;
  c->dconst = 1.0 / c->c2_value;
  for (size_t l = 0; l < shapes.size(); ++l) {
    wh_ctx::MgLevel lev{};
    lev.g = mg_geom(shapes[l].first, shapes[l].second, l == 0 ? c->order : 2, theta);
    if (l == 0) {
      lev.d = at(k);
      lev.t = at(k + 1);
      c->imp_r = at(k + 2);
      c->imp_z = at(k + 3);
      c->imp_p = at(k + 4);
      c->imp_q = at(k + 5);
      lev.b = c->imp_r;
      lev.x = c->imp_z;
      k += 6;
    } else {
      lev.d = at(k);
      lev.x = at(k + 1);
      lev.b = at(k + 2);
      lev.t = at(k + 3);
      k += 4;
    }
    if (!cvar) lev.d = nullptr;
    c->mg.push_back(lev);
  }
  c->imp_part = at(k);
  c->imp_scal = at(k + 1);
  // coarsen only while the level's operator is far from its diagonal: once
  // theta n^2 <= 1/2 damped Jacobi alone solves it well
  size_t used = 1;
  while (used < c->mg.size()) {
    const wh::MgGeom &gl = c->mg[used - 1].g;
    const double nmax = (double)std::max(gl.nx, gl.ny);
    if (theta * nmax * nmax <= 0.5) break;
    ++used;
  }
  c->mg.resize(used);
  if (cvar) {
    WH_HIP(c, wh::launch_mg_inverse(c->mg[0].g, static_cast<const double *>(c->c2), c->mg[0].d, c->stream));
    for (size_t l = 1; l < c->mg.size(); ++l)
      WH_HIP(c, wh::launch_mg_inject(c->mg[l - 1].g, c->mg[l - 1].d, c->mg[l].g, c->mg[l].d, c->stream));
  }
  // the V-cycle is a fixed sequence of launches on fixed buffers: capture it
  // once (on the context's own capture stream) and replay it per iteration
  WH_TRY(mg_drop_graph(c));
  if (!c->mg_cap) WH_HIP(c, hipStreamCreateWithFlags(&c->mg_cap, hipStreamNonBlocking));
  WH_HIP(c, hipStreamBeginCapture(c->mg_cap, hipStreamCaptureModeThreadLocal));
  const wh_status st = mg_vcycle(c, 0, c->mg_cap);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(c->mg_cap, &graph);
  if (st != WH_OK || ec != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    if (st != WH_OK) return st;
    return fail(c, WH_EDEVICE, "V-cycle graph capture failed: %s", hipGetErrorString(ec));
  }
  c->mg_graph = graph;
  WH_HIP(c, hipGraphInstantiate(&c->mg_exec, graph, nullptr, nullptr, 0));
  c->mg_ready = true;
  return WH_OK;
}

// x_l = V-cycle approximation of S_l^{-1} b_l (x_l starts from 0).
wh_status mg_vcycle(wh_ctx *c, size_t l, hipStream_t s) {
  wh_ctx::MgLevel &L = c->mg[l];
  const double w = L.g.order == 4 ? 0.75 : 0.8;
  const int sweeps = l + 1 == c->mg.size() ? kMgCoarseSweeps : kMgPreSweeps;
  // damped Jacobi from x = 0, ping-ponging between t and x (even count: ends in x)
  WH_HIP(c, wh::launch_mg_smooth(L.g, L.d, c->dconst, nullptr, L.b, L.t, w, s));
  for (int sw = 1; sw < sweeps; ++sw) {
    const bool to_x = (sw & 1) != 0;
    WH_HIP(c, wh::launch_mg_smooth(L.g, L.d, c->dconst, to_x ? L.t : L.x, L.b, to_x ? L.x : L.t, w, s));
  }
  if (l + 1 == c->mg.size()) return WH_OK;
  wh_ctx::MgLevel &C = c->mg[l + 1];
  WH_HIP(c, wh::launch_mg_residual(L.g, L.d, c->dconst, L.x, L.b, L.t, s));
  WH_HIP(c, wh::launch_mg_restrict(L.g, L.t, C.g, C.b, s));
  WH_TRY(mg_vcycle(c, l + 1, s));
  WH_HIP(c, wh::launch_mg_prolong(C.g, C.x, L.g, L.x, s));
  for (int sw = 0; sw < kMgPreSweeps; ++sw) {
    const bool to_t = (sw & 1) == 0;
    WH_HIP(c, wh::launch_mg_smooth(L.g, L.d, c->dconst, to_t ? L.x : L.t, L.b, to_t ? L.t : L.x, w, s));
  }
  return WH_OK;
}

wh_status imp_dot(wh_ctx *c, const double *x, const double *y, int slot) {
  const int nb = wh::reduction_blocks(c->nodes);
  WH_HIP(c, wh::launch_mdot(x, 0, 1, y, c->nodes, c->imp_part, nb, c->stream));
  WH_HIP(c, wh::launch_reduce_rows(c->imp_part, nb, 1, c->imp_scal + slot, c->stream));
  return WH_OK;
}

// Copy count scalars from slot on to the host (one synchronisation).
wh_status imp_fetch(wh_ctx *c, int slot, double *out, int count = 1) {
  WH_HIP(c, hipMemcpyAsync(c->pinned, c->imp_scal + slot, (size_t)count * 8, hipMemcpyDeviceToHost, c->stream));
  WH_HIP(c, hipStreamSynchronize(c->stream));
  std::memcpy(out, c->pinned, (size_t)count * 8);
  return WH_OK;
}

// Solve S x = B (B in imp_q, x holds the initial guess) by CG preconditioned
// with one V-cycle, to ||B - S x|| <= imp_rtol ||B||.
wh_status pcg_solve(wh_ctx *c, double *x) {
  const wh::MgGeom &g = c->mg[0].g;
  const double *d = c->mg[0].d;
  const int64_t N = c->nodes;
  double *r = c->imp_r, *z = c->imp_z, *p = c->imp_p, *q = c->imp_q;
  double bb = 0.0, rr = 0.0;
  WH_TRY(imp_dot(c, q, q, 4));
  WH_TRY(imp_fetch(c, 4, &bb));
  if (!std::isfinite(bb)) return fail(c, WH_ENONFINITE, "implicit step: right-hand side is not finite");
  if (bb == 0.0) {
    WH_HIP(c, wh::launch_fill(x, 0.0, N, c->stream));
    return WH_OK;
  }
  const double tol2 = c->imp_rtol * c->imp_rtol * bb;
  WH_HIP(c, wh::launch_mg_residual(g, d, c->dconst, x, q, r, c->stream));
  WH_TRY(imp_dot(c, r, r, 2));
  WH_TRY(imp_fetch(c, 2, &rr));
  int it = 0;
  if (rr > tol2) {
    WH_HIP(c, hipGraphLaunch(c->mg_exec, c->stream));  // z = V-cycle(r)
    WH_TRY(imp_dot(c, r, z, 0));
    WH_HIP(c, wh::launch_pcg_xpay(N, z, p, nullptr, nullptr, c->stream));
    while (true) {
      WH_HIP(c, wh::launch_mg_residual(g, d, c->dconst, p, nullptr, q, c->stream));  // q = S p
      WH_TRY(imp_dot(c, p, q, 1));
      WH_HIP(c, wh::launch_pcg_update(N, x, r, p, q, c->imp_scal + 0, c->imp_scal + 1, c->stream));
      WH_TRY(imp_dot(c, r, r, 2));
      double sc[3];  // r.z, p.Sp of this iteration, then the new r.r
      WH_TRY(imp_fetch(c, 0, sc, 3));
      rr = sc[2];
      ++it;
      if (!std::isfinite(rr)) return fail(c, WH_ENONFINITE, "implicit step: inner CG became non-finite");
      if (rr <= tol2) break;
      // S and the V-cycle are both symmetric positive definite in exact
      // arithmetic; a non-positive r.z or p.Sp means one of them is not
      if (!(sc[0] > 0.0 && sc[1] > 0.0))
        return fail(c, WH_ENOTCONV, "implicit step: inner CG lost positive definiteness (r.z = %g, p.Sp = %g) "
                    "after %d iterations", sc[0], sc[1], it);
      if (it >= kImpMaxInner)
        return fail(c, WH_ENOTCONV, "implicit step: inner CG did not reach %g in %d iterations (at %g)",
                    c->imp_rtol, it, std::sqrt(rr / bb));
      WH_HIP(c, hipGraphLaunch(c->mg_exec, c->stream));
      WH_TRY(imp_dot(c, r, z, 3));
      WH_HIP(c, wh::launch_pcg_xpay(N, z, p, c->imp_scal + 3, c->imp_scal + 0, c->stream));
      WH_HIP(c, hipMemcpyAsync(c->imp_scal + 0, c->imp_scal + 3, 8, hipMemcpyDeviceToDevice, c->stream));
    }
  }
  c->imp_steps += 1;
  c->imp_iters += it;
  c->imp_max = std::max(c->imp_max, it);
  return WH_OK;
}

// One WaveHoltz application with implicit steps (eq. WaveSchemeImplicit):
// M W^1 = W^0 - (dt^2/2) cos(omega_i dt) f (the initial condition eliminates
// W^{-1}), then M W^{n+1} = 2 W^n - M W^{n-1} - dt^2 cos(omega_i t^n)
// cos(omega_i dt) f, each solved in the symmetric form by pcg_solve.
wh_status apply_implicit(wh_ctx *c, const double *v, bool forcing, int mode, double *out, double *w_final) {
  if (!c->mg_ready) WH_TRY(mg_setup(c));
  const int64_t nt = c->tp.nt, N = nt * (int64_t)c->tp.periods;
  const double dt = c->tp.dt, cw = std::cos(c->tp.omega_e * dt);
  const wh::MgGeom &g = c->mg[0].g;
  const double *d = c->mg[0].d;
  const double *f = forcing ? static_cast<const double *>(c->f) : nullptr;
  double *lv[3] = {static_cast<double *>(c->W[0]), static_cast<double *>(c->W[1]), static_cast<double *>(c->W[2])};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (c->profiling) {
    WH_TRY(take_events(c, &ev0, &ev1));
    WH_HIP(c, hipEventRecord(ev0, c->stream));
  }
  // W^0 = v with the walls set to 0
  WH_HIP(c, hipMemcpyAsync(lv[0], v, (size_t)c->nodes * 8, hipMemcpyDeviceToDevice, c->stream));
  WH_HIP(c, wh::launch_set_walls(false, geometry(c, 1.0), lv[0], 0.0, c->stream));
  WH_HIP(c, wh::launch_imp_rhs(g, d, c->dconst, lv[0], nullptr, f, -0.5 * dt * dt * cw, c->imp_q, lv[1], c->stream));
  WH_TRY(pcg_solve(c, lv[1]));
  WH_HIP(c, wh::launch_imp_filter(g, lv[0], c->wts[0], c->acc, true, wh::ACCUMULATE, v, out, c->stream));
  WH_HIP(c, wh::launch_imp_filter(g, lv[1], c->wts[1], c->acc, false, N == 1 ? mode : wh::ACCUMULATE, v, out,
                                  c->stream));
  int prev = 0, cur = 1, nxt = 2;
  for (int64_t n = 1; n < N; ++n) {
    const double gn = -dt * dt * std::cos(2.0 * M_PI * (double)(n % nt) / (double)nt) * cw;
    WH_HIP(c, wh::launch_imp_rhs(g, d, c->dconst, lv[cur], lv[prev], f, gn, c->imp_q, lv[nxt], c->stream));
    WH_TRY(pcg_solve(c, lv[nxt]));
    WH_HIP(c, wh::launch_imp_filter(g, lv[nxt], c->wts[(size_t)n + 1], c->acc, false,
                                    n == N - 1 ? mode : wh::ACCUMULATE, v, out, c->stream));
    const int t = prev;
    prev = cur;
    cur = nxt;
    nxt = t;
  }
  if (c->profiling) {
    WH_HIP(c, hipEventRecord(ev1, c->stream));
    c->pending.push_back({ev0, ev1, N, 0.0, interior_nodes(c) * (double)N});
    if (c->pending.size() >= 256) WH_TRY(drain_profile(c));
  }
  if (w_final) WH_HIP(c, hipMemcpyAsync(w_final, lv[cur], (size_t)c->nodes * 8, hipMemcpyDeviceToDevice, c->stream));
  return WH_OK;
}

// One WaveHoltz application.  mode: ACCUMULATE (acc keeps the filter),
// FINAL_FILTER (out = filtered) or FINAL_A (out = v - filtered).
wh_status apply_impl(wh_ctx *c, const double *v, bool forcing, int mode, double *out, double *w_final) {
  if (c->implicit) return apply_implicit(c, v, forcing, mode, out, w_final);
  const bool fp32 = c->prec == WH_FP32_STATE;
  const int64_t N = (int64_t)c->tp.nt * c->tp.periods;
  const double dt2 = c->tp.dt * c->tp.dt;
  const wh::StepGeom g = geometry(c, dt2);
  const wh::StepGeom half = geometry(c, 0.5 * dt2);
  const void *c2 = c->c2_is_const ? nullptr : c->c2;
  const void *f = forcing ? c->f : nullptr;
  WH_HIP(c, wh::launch_first_step(fp32, half, v, c->W[0], c->W[1], c->acc, c2, f, forcing ? -0.5 * dt2 : 0.0,
                                  c->wts[0], c->wts[1], c->stream));
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (c->profiling) {
    WH_TRY(take_events(c, &ev0, &ev1));
    WH_HIP(c, hipEventRecord(ev0, c->stream));
  }
  const Tuning tu = resolve_tuning(c);
  const bool blocked = tu.kernel == WH_KERNEL_BLOCKED_2D || tu.kernel == WH_KERNEL_BLOCKED_3D;
  const int K = blocked ? tu.kblock : 1;
  const double T = (double)state_bytes(c);
  const double aux = (c2 ? T : 0.0) + (f ? T : 0.0);  // c^2 and f reads per node and launch
  int64_t launches = 0;
  double bytes_per_node = 0.0;
  void *cur;
  if (!blocked) {
    void *prev = c->W[0];
    cur = c->W[1];
    for (int64_t n = 1; n < N; ++n) {
      const int m = (n == N - 1) ? mode : wh::ACCUMULATE;
      if (tu.kernel == WH_KERNEL_ZCOL_3D)
        WH_HIP(c, wh::launch_step3d_zcol(fp32, g, tu.tile, cur, prev, c->acc, c2, f,
                                         forcing ? c->frc[(size_t)n] : 0.0, c->wts[(size_t)n + 1], m, v, out,
                                         c->stream));
      else
        WH_HIP(c, wh::launch_step(fp32, g, cur, prev, c->acc, c2, f, forcing ? c->frc[(size_t)n] : 0.0,
                                  c->wts[(size_t)n + 1], m, v, out, c->stream));
      std::swap(prev, cur);
      ++launches;
      // W^n, W^{n-1} read, W^{n+1} written, accumulator read and written
      bytes_per_node += 3.0 * T + aux + 16.0;
    }
  } else {
    void *ip = c->W[0], *ic = c->W[1], *op = c->W[2], *oc = c->W[3];
    const int64_t total = N - 1;  // steps after the first
    int64_t done = 0;
    while (done < total) {
      const int ks = (int)std::min<int64_t>(K, total - done);
      wh::BlockCoef coef{};
      for (int s = 0; s < ks; ++s) {
        const int64_t n = 1 + done + s;  // step from level n to n + 1
        coef.gn[s] = forcing ? c->frc[(size_t)n] : 0.0;
        coef.wn[s] = c->wts[(size_t)n + 1];
      }
      const int m = (done + ks == total) ? mode : wh::ACCUMULATE;
      if (tu.kernel == WH_KERNEL_BLOCKED_3D)
        WH_HIP(c, wh::launch_block_steps_3d(fp32, g, ks, tu.tile, ip, ic, op, oc, c->acc, c2, f, coef, m, v, out,
                                            c->stream));
      else
        WH_HIP(c, wh::launch_block_steps_2d(fp32, g, K, tu.tile, ks, ip, ic, op, oc, c->acc, c2, f, coef, m, v, out,
                                            c->stream));
      std::swap(ip, op);
      std::swap(ic, oc);
      done += ks;
      ++launches;
      // two levels read and two written, accumulator read and written
      bytes_per_node += 4.0 * T + aux + 16.0;
    }
    cur = ic;
  }
  if (c->profiling) {
    WH_HIP(c, hipEventRecord(ev1, c->stream));
    const double interior = interior_nodes(c);
    const double extra = (mode == wh::FINAL_A) ? 8.0 : 0.0;  // v read on the last launch
    c->pending.push_back({ev0, ev1, launches, interior * (bytes_per_node + extra), interior * (double)(N - 1)});
    if (c->pending.size() >= 256) WH_TRY(drain_profile(c));
  }
  if (w_final) WH_HIP(c, wh::launch_from_state(fp32, cur, w_final, c->nodes, c->stream));
  return WH_OK;
}

double point_steps_per_apply(const wh_ctx *c) {
  double u = 1.0;
  for (int m = 0; m < c->dim; ++m) u *= (double)(c->n[m] - 1);
  return u * (double)c->tp.nt * (double)c->tp.periods;
}

// Library's own evaluation of the discrete filter function (three-sinc
// form, Appendix A.3) for the predicted rate of Theorem 2.
double sincd(double z, double T, double dt) {
  const double t = std::tan(0.5 * z * dt);
  if (std::fabs(t) < 1e-300) return 1.0;
  return std::sin(z * T) / (T * t / (0.5 * dt));
}

// Eigenvalue of -d^2/dx^2 (order p, Dirichlet) on sin(k pi x) with n cells:
// n^2 sum_{mu < p/2} b_mu (4 sin^2(k pi / (2n)))^{mu+1}, b_0 = 1, b_1 = 1/12
// (App. B).
double axis_eigenvalue(int order, int64_t n, int64_t k) {
  const double nn = (double)n;
  const double s = std::sin(0.5 * M_PI * (double)k / nn);
  const double s2 = s * s;
  double lam = 4.0 * nn * nn * s2;
  if (order == 4) lam += (4.0 / 3.0) * nn * nn * s2 * s2;
  return lam;
}

// beta_d of the discrete filter (three-sinc form, App. A.3) for a mode whose
// eigenvalue of -L_h is lam2; NaN if the mode is beyond the stability limit.
double mode_beta(const wh_ctx *c, double lam2) {
  const double dt = c->tp.dt, we = c->tp.omega_e, al = c->tp.alpha;
  const double Tbar = (double)c->tp.nt * c->tp.periods * dt;
  double lt;
  if (c->implicit) {
    // mode map of the implicit scheme, eq. (lambdaTildeImplicit)
    lt = std::acos(1.0 / (1.0 + 0.5 * lam2 * dt * dt)) / dt;
  } else {
    const double arg = 0.5 * std::sqrt(lam2) * dt;
    if (arg >= 1.0) return NAN;
    lt = (2.0 / dt) * std::asin(arg);  // eq. (discreteExplicitLambdaTilde)
  }
  return sincd(we + lt, Tbar, dt) + sincd(we - lt, Tbar, dt) - al * sincd(lt, Tbar, dt);
}

int64_t mode_index(const wh_ctx *c, const int32_t *k) {
  int64_t idx = 0, stride = 1;
  for (int m = 0; m < c->dim; ++m) {
    idx += (int64_t)(k[m] - 1) * stride;
    stride *= c->n[m] - 1;
  }
  return idx;
}

// Theorem 2 (and, with deflation, the theorem on deflated convergence):
// max |beta_d| over the sine modes that are not deflated (constant c^2).
double predicted_rate(const wh_ctx *c) {
  if (!c->c2_is_const) return NAN;
  double modes = 1.0;
  for (int m = 0; m < c->dim; ++m) modes *= (double)(c->n[m] - 1);
  if (modes > (double)(1 << 22)) return NAN;
  std::vector<double> ax[3];
  for (int m = 0; m < c->dim; ++m)
    for (int64_t k = 1; k < c->n[m]; ++k) ax[m].push_back(axis_eigenvalue(c->order, c->n[m], k));
  std::vector<char> skip;
  if (c->defl_count > 0) {
    skip.assign((size_t)modes, 0);
    for (int q = 0; q < c->defl_count; ++q) skip[(size_t)mode_index(c, &c->defl_modes[(size_t)q * c->dim])] = 1;
  }
  double mu = 0.0;
  const size_t nz = c->dim == 3 ? ax[2].size() : 1;
  size_t idx = 0;
  for (size_t kz = 0; kz < nz; ++kz)
    for (double ly : ax[1])
      for (double lx : ax[0]) {
        const size_t here = idx++;
        if (!skip.empty() && skip[here]) continue;
        const double b = mode_beta(c, c->c2_value * (lx + ly + (c->dim == 3 ? ax[2][kz] : 0.0)));
        if (std::isfinite(b)) mu = std::max(mu, std::fabs(b));
      }
  return mu;
}

}  // namespace

extern "C" {

int32_t wh_version(void) { return 10000; }

const char *wh_status_string(int32_t s) {
  switch (s) {
    case WH_OK: return "WH_OK";
    case WH_EINVAL: return "WH_EINVAL";
    case WH_ENOMEM: return "WH_ENOMEM";
    case WH_EDEVICE: return "WH_EDEVICE";
    case WH_EUNSTABLE: return "WH_EUNSTABLE";
    case WH_ENOTCONV: return "WH_ENOTCONV";
    case WH_ENONFINITE: return "WH_ENONFINITE";
    case WH_ESTATE: return "WH_ESTATE";
    default: return "unknown wh_status";
  }
}

wh_status wh_compute_time_params(int32_t dim, const int64_t n[3], int32_t order, double c2max, double omega,
                                 int32_t periods, double cfl_frac, int32_t nt_override, double alpha,
                                 wh_time_params *out) {
  if (!n || !out) return WH_EINVAL;
  if (dim != 2 && dim != 3) return WH_EINVAL;
  if (order != 2 && order != 4) return WH_EINVAL;
  for (int m = 0; m < dim; ++m)
    if (n[m] < 2 || n[m] > (int64_t)1 << 20) return WH_EINVAL;
  if (!(c2max > 0.0) || !std::isfinite(c2max)) return WH_EINVAL;
  if (!(omega > 0.0) || !std::isfinite(omega)) return WH_EINVAL;
  if (periods < 1 || periods > 1000) return WH_EINVAL;
  if (!(cfl_frac > 0.0) || cfl_frac > 1.0) return WH_EINVAL;
  if (nt_override < 0 || (nt_override > 0 && nt_override < 5)) return WH_EINVAL;
  if (!std::isfinite(alpha)) return WH_EINVAL;
  const double limit = order == 2 ? 1.0 : std::sqrt(3.0) / 2.0;  // C_{2,p}
  double root = 0.0;
  for (int m = 0; m < dim; ++m) root += (double)n[m] * (double)n[m];
  root = std::sqrt(root);
  const double cmax = std::sqrt(c2max);
  const double dt_max = cfl_frac * limit / (cmax * root);
  int64_t nt;
  if (nt_override > 0) {
    nt = nt_override;
    const double dt = (2.0 / omega) * std::sin(M_PI / (double)nt);
    if (cmax * dt * root > limit * (1.0 + 1e-12)) return WH_EUNSTABLE;
  } else {
    const double est = std::ceil((2.0 * M_PI / omega) / dt_max);
    if (!(est < 1e8)) return WH_EINVAL;
    nt = std::max<int64_t>(5, (int64_t)est);
    while ((2.0 / omega) * std::sin(M_PI / (double)nt) > dt_max) ++nt;
  }
  if (nt * (int64_t)periods > (int64_t)1 << 26) return WH_EINVAL;
  const double dt = (2.0 / omega) * std::sin(M_PI / (double)nt);
  out->nt = (int32_t)nt;
  out->periods = periods;
  out->dt = dt;
  out->omega = omega;
  out->omega_e = 2.0 * M_PI / ((double)nt * dt);
  out->alpha = alpha < 0.0 ? std::tan(M_PI / (double)nt) / std::tan(2.0 * M_PI / (double)nt) : alpha;
  out->cfl = cmax * dt * root;
  out->c2max = c2max;
  return WH_OK;
}

wh_status wh_create(wh_ctx **out, int32_t device, void *stream) {
  if (!out) return WH_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return WH_EDEVICE;
  }
  wh_ctx *c = new (std::nothrow) wh_ctx();
  if (!c) return WH_ENOMEM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  if (hipSetDevice(device) != hipSuccess ||
      hipHostMalloc((void **)&c->pinned, (size_t)kMaxScalars * 8, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return WH_EDEVICE;
  }
  c->pinned_count = kMaxScalars;
  *out = c;
  return WH_OK;
}

void wh_destroy(wh_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (!c->pending.empty()) (void)hipStreamSynchronize(c->stream);
  for (auto &t : c->pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  if (c->mg_exec || c->mg_graph) {
    (void)hipStreamSynchronize(c->stream);
    if (c->mg_exec) (void)hipGraphExecDestroy(c->mg_exec);
    if (c->mg_graph) (void)hipGraphDestroy(c->mg_graph);
  }
  if (c->mg_cap) (void)hipStreamDestroy(c->mg_cap);
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
}

wh_status wh_profile_enable(wh_ctx *c, int32_t enable) {
  if (!c) return WH_EINVAL;
  WH_TRY(set_device(c));
  if (!c->pending.empty()) WH_TRY(drain_profile(c));
  if (enable) c->prof = wh_profile{};
  c->profiling = enable != 0;
  return WH_OK;
}

wh_status wh_profile_read(wh_ctx *c, wh_profile *out) {
  if (!c || !out) return WH_EINVAL;
  WH_TRY(set_device(c));
  if (!c->pending.empty()) WH_TRY(drain_profile(c));
  *out = c->prof;
  return WH_OK;
}

const char *wh_last_error(const wh_ctx *c) {
  if (!c) return "no context";
  return c->err.c_str();
}

wh_status wh_set_grid(wh_ctx *c, int32_t dim, const int64_t n[3], int32_t order, int32_t precision) {
  if (!c) return WH_EINVAL;
  if (dim != 2 && dim != 3) return fail(c, WH_EINVAL, "dim must be 2 or 3 (got %d)", dim);
  if (!n) return fail(c, WH_EINVAL, "n is NULL");
  if (order != 2 && order != 4) return fail(c, WH_EINVAL, "order must be 2 or 4 (got %d)", order);
  if (precision != WH_FP64 && precision != WH_FP32_STATE)
    return fail(c, WH_EINVAL, "precision must be WH_FP64 or WH_FP32_STATE");
  int64_t nodes = 1;
  for (int m = 0; m < dim; ++m) {
    if (n[m] < 2 || n[m] > 65535) return fail(c, WH_EINVAL, "n[%d] = %lld out of range [2, 65535]", m, (long long)n[m]);
    nodes *= n[m] + 1;
  }
  if (nodes > ((int64_t)1 << 33)) return fail(c, WH_EINVAL, "grid too large (%lld nodes)", (long long)nodes);
  c->grid_set = true;
  c->dim = dim;
  c->order = order;
  c->prec = precision;
  c->n[0] = n[0];
  c->n[1] = n[1];
  c->n[2] = dim == 3 ? n[2] : 0;
  c->nodes = nodes;
  c->ws = nullptr;
  c->ws_bytes = 0;
  c->c2_set = c->f_set = c->freq_set = false;
  c->c2_is_const = false;
  c->kernel = WH_KERNEL_AUTO;
  c->kblock = c->tile = 0;
  c->adj = nullptr;
  c->adj_bytes = 0;
  c->defl_count = 0;
  c->implicit = false;
  c->imp = nullptr;
  c->imp_bytes = 0;
  c->mg_ready = false;
  c->imp_steps = c->imp_iters = 0;
  c->imp_max = 0;
  c->err.clear();
  return WH_OK;
}

wh_status wh_workspace_size(const wh_ctx *c, int32_t restart, size_t *bytes) {
  if (!c || !bytes) return WH_EINVAL;
  if (!c->grid_set) return WH_ESTATE;
  if (restart < 0 || restart > WH_MAX_RESTART) return WH_EINVAL;
  *bytes = layout(c, restart).total;
  return WH_OK;
}

wh_status wh_bind_workspace(wh_ctx *c, void *ptr, size_t bytes, int32_t restart) {
  WH_TRY(need(c, true, false, false, false, false));
  if (restart < 0 || restart > WH_MAX_RESTART) return fail(c, WH_EINVAL, "restart out of range");
  if (!ptr) return fail(c, WH_EINVAL, "workspace pointer is NULL");
  if (reinterpret_cast<uintptr_t>(ptr) % 256 != 0) return fail(c, WH_EINVAL, "workspace must be 256-byte aligned");
  const Layout L = layout(c, restart);
  if (bytes < L.total)
    return fail(c, WH_ENOMEM, "workspace too small: %zu bytes given, %zu needed", bytes, L.total);
  WH_TRY(set_device(c));
  if (!is_device_ptr(ptr)) return fail(c, WH_EINVAL, "workspace is not device memory");
  char *base = static_cast<char *>(ptr);
  c->ws = base;
  c->ws_bytes = bytes;
  c->ws_restart = restart;
  c->c2 = base + L.c2;
  c->f = base + L.f;
  for (int i = 0; i < 4; ++i) c->W[i] = base + L.W[i];
  c->acc = reinterpret_cast<double *>(base + L.acc);
  c->tmp = reinterpret_cast<double *>(base + L.tmp);
  c->b = reinterpret_cast<double *>(base + L.b);
  c->V = restart > 0 ? reinterpret_cast<double *>(base + L.V) : nullptr;
  c->ldv = L.ldv;
  c->partials = reinterpret_cast<double *>(base + L.partials);
  c->scal = reinterpret_cast<double *>(base + L.scal);
  c->c2_set = c->f_set = c->freq_set = false;
  return WH_OK;
}

static wh_status finish_c2(wh_ctx *c) {
  // Any change of c^2 invalidates the time parameters and the deflation
  // eigenvalues.
  c->freq_set = false;
  c->defl_count = 0;
  c->c2_set = true;
  return WH_OK;
}

wh_status wh_set_c2_constant(wh_ctx *c, double c2) {
  WH_TRY(need(c, true, true, false, false, false));
  if (!(c2 > 0.0) || !std::isfinite(c2)) return fail(c, WH_EINVAL, "c2 must be finite and > 0");
  c->c2_is_const = true;
  c->c2_value = c2;
  c->c2max = c2;
  return finish_c2(c);
}

wh_status wh_set_c2(wh_ctx *c, const double *c2, int32_t on_device) {
  WH_TRY(need(c, true, true, false, false, false));
  if (!c2) return wh_set_c2_constant(c, 1.0);
  WH_TRY(set_device(c));
  if (on_device) WH_TRY(check_dev(c, c2, "c2"));
  // stats on the FP64 values: stage through the accumulator when on host
  const double *src = c2;
  if (!on_device) {
    WH_HIP(c, hipMemcpyAsync(c->acc, c2, (size_t)c->nodes * 8, hipMemcpyHostToDevice, c->stream));
    src = c->acc;
  }
  const int nb = wh::reduction_blocks(c->nodes);
  const wh::StepGeom g = geometry(c, 1.0);
  WH_HIP(c, wh::launch_interior_stats(g, src, c->partials, nb, c->stream));
  std::vector<double> part((size_t)3 * nb);
  WH_HIP(c, hipMemcpyAsync(part.data(), c->partials, part.size() * 8, hipMemcpyDeviceToHost, c->stream));
  WH_HIP(c, hipStreamSynchronize(c->stream));
  double mx = -INFINITY, mn = INFINITY, bad = 0.0;
  for (int b = 0; b < nb; ++b) {
    mx = std::max(mx, part[3 * b]);
    mn = std::min(mn, part[3 * b + 1]);
    bad += part[3 * b + 2];
  }
  if (bad > 0.0) return fail(c, WH_EINVAL, "c2 has %.0f non-finite interior values", bad);
  if (!(mn > 0.0)) return fail(c, WH_EINVAL, "c2 must be > 0 on interior nodes (min %g)", mn);
  if (c->prec == WH_FP32_STATE) {
    WH_HIP(c, wh::launch_to_state(true, src, c->c2, c->nodes, c->stream));
  } else {
    WH_HIP(c, hipMemcpyAsync(c->c2, src, (size_t)c->nodes * 8, hipMemcpyDeviceToDevice, c->stream));
  }
  // wall values are ignored by contract; the blocked kernels evaluate wall
  // nodes (where the Laplacian is exactly 0), so give them a finite value
  WH_HIP(c, wh::launch_set_walls(c->prec == WH_FP32_STATE, geometry(c, 1.0), c->c2, 1.0, c->stream));
  WH_HIP(c, hipStreamSynchronize(c->stream));
  c->c2_is_const = false;
  c->c2_value = 1.0;
  c->c2max = mx;
  return finish_c2(c);
}

wh_status wh_set_source(wh_ctx *c, const double *f, int32_t on_device) {
  WH_TRY(need(c, true, true, false, false, false));
  if (!f) return fail(c, WH_EINVAL, "f is NULL");
  WH_TRY(set_device(c));
  if (on_device) WH_TRY(check_dev(c, f, "f"));
  WH_TRY(upload_field(c, f, on_device, c->f));
  // wall values are ignored by contract: the source is 0 there
  WH_HIP(c, wh::launch_set_walls(c->prec == WH_FP32_STATE, geometry(c, 1.0), c->f, 0.0, c->stream));
  c->f_set = true;
  return WH_OK;
}

wh_status wh_set_frequency(wh_ctx *c, double omega, int32_t periods, double cfl_frac, int32_t nt_override,
                           double alpha) {
  WH_TRY(need(c, true, true, true, false, false));
  if (c->implicit) {
    // implicit time-stepping correction recipe (Appendix A.2): N_t steps per
    // period, dt = sqrt(2 / cos(2 pi / N_t) - 2) / omega, omega_i = 2 pi / (N_t dt)
    if (!(omega > 0.0) || !std::isfinite(omega) || periods < 1 || periods > 10000)
      return fail(c, WH_EINVAL, "invalid frequency parameters (omega %g, periods %d)", omega, periods);
    if (nt_override != 0 && nt_override != c->nits)
      return fail(c, WH_EINVAL, "with implicit stepping the steps per period are set by wh_set_implicit");
    const int nt = c->nits;
    wh_time_params tp{};
    tp.nt = nt;
    tp.periods = periods;
    tp.omega = omega;
    tp.dt = std::sqrt(2.0 / std::cos(2.0 * M_PI / nt) - 2.0) / omega;
    tp.omega_e = 2.0 * M_PI / (nt * tp.dt);
    const double alpha_d = std::tan(M_PI / nt) / std::tan(2.0 * M_PI / nt);
    tp.alpha = alpha < 0.0 ? alpha_d : alpha;
    double s2 = 0.0;
    for (int m = 0; m < c->dim; ++m) s2 += (double)c->n[m] * (double)c->n[m];
    tp.cfl = std::sqrt(c->c2max) * tp.dt * std::sqrt(s2);
    tp.c2max = c->c2max;
    c->tp = tp;
    build_tables(c);
    c->freq_set = true;
    c->mg_ready = false;
    return c->imp ? mg_setup(c) : WH_OK;
  }
  wh_time_params tp{};
  const wh_status st =
      wh_compute_time_params(c->dim, c->n, c->order, c->c2max, omega, periods, cfl_frac, nt_override, alpha, &tp);
  if (st == WH_EUNSTABLE)
    return fail(c, st, "nt = %d violates the explicit stability limit for this grid and c^2", nt_override);
  if (st != WH_OK) return fail(c, st, "invalid frequency parameters (omega %g, periods %d, cfl %g, nt %d)", omega,
                                periods, cfl_frac, nt_override);
  c->tp = tp;
  build_tables(c);
  c->freq_set = true;
  return WH_OK;
}

wh_status wh_get_time_params(const wh_ctx *c, wh_time_params *out) {
  if (!c || !out) return WH_EINVAL;
  if (!c->freq_set) return WH_ESTATE;
  *out = c->tp;
  return WH_OK;
}

wh_status wh_run_periods(wh_ctx *c, const double *w0, int32_t with_forcing, double *w_final, double *filtered) {
  WH_TRY(need(c, true, true, true, with_forcing != 0, true));
  WH_TRY(set_device(c));
  WH_TRY(check_dev(c, w0, "w0"));
  if (w_final) WH_TRY(check_dev(c, w_final, "w_final"));
  if (filtered) WH_TRY(check_dev(c, filtered, "filtered"));
  if (w_final == w0 || filtered == w0) return fail(c, WH_EINVAL, "outputs may not alias w0");
  return apply_impl(c, w0, with_forcing != 0, filtered ? wh::FINAL_FILTER : wh::ACCUMULATE, filtered, w_final);
}

wh_status wh_apply(wh_ctx *c, const double *v, double *out, int32_t with_forcing) {
  WH_TRY(need(c, true, true, true, with_forcing != 0, true));
  WH_TRY(set_device(c));
  WH_TRY(check_dev(c, v, "v"));
  WH_TRY(check_dev(c, out, "out"));
  if (out == v) return fail(c, WH_EINVAL, "out may not alias v");
  return apply_impl(c, v, with_forcing != 0, wh::FINAL_FILTER, out, nullptr);
}

wh_status wh_apply_A(wh_ctx *c, const double *v, double *Av) {
  WH_TRY(need(c, true, true, true, false, true));
  WH_TRY(set_device(c));
  WH_TRY(check_dev(c, v, "v"));
  WH_TRY(check_dev(c, Av, "Av"));
  if (Av == v) return fail(c, WH_EINVAL, "Av may not alias v");
  return apply_impl(c, v, false, wh::FINAL_A, Av, nullptr);
}

wh_status wh_apply_A_noalloc(wh_ctx *c, const double *v, double *Av) {
  WH_TRY(need(c, true, true, true, false, true));
  if (c->implicit)
    return fail(c, WH_EINVAL, "implicit stepping keeps its levels in the implicit workspace: use wh_apply_A");
  WH_TRY(set_device(c));
  WH_TRY(check_dev(c, v, "v"));
  WH_TRY(check_dev(c, Av, "Av"));
  if (Av == v) return fail(c, WH_EINVAL, "Av may not alias v");
  // four state levels and the FP64 accumulator, 256-byte aligned
  const size_t level = align256((size_t)c->nodes * state_bytes(c));
  const size_t accb = align256((size_t)c->nodes * 8);
  const size_t need_bytes = 4 * level + accb;
  if (need_bytes > wh::kStaticScratchBytes)
    return fail(c, WH_EINVAL,
                "this grid needs %zu bytes of scratch (four state levels and the FP64 accumulator); the static "
                "scratch holds %zu bytes",
                need_bytes, wh::kStaticScratchBytes);
  void *base = nullptr;
  WH_HIP(c, wh::static_scratch(c->device, &base));
  char *p = static_cast<char *>(base);
  void *W[4] = {c->W[0], c->W[1], c->W[2], c->W[3]};
  double *acc = c->acc;
  const bool profiling = c->profiling;
  for (int i = 0; i < 4; ++i) c->W[i] = p + (size_t)i * level;
  c->acc = reinterpret_cast<double *>(p + 4 * level);
  c->profiling = false;  // no event creation on this path
  const wh_status st = apply_impl(c, v, false, wh::FINAL_A, Av, nullptr);
  for (int i = 0; i < 4; ++i) c->W[i] = W[i];
  c->acc = acc;
  c->profiling = profiling;
  return st;
}

wh_status wh_filter_spectrum(wh_ctx *c, double c2, double *a_min, double *a_max, int32_t *k_min) {
  WH_TRY(need(c, true, false, false, false, true));
  if (!a_min || !a_max) return fail(c, WH_EINVAL, "a_min and a_max must not be NULL");
  if (!(c2 > 0.0) || !std::isfinite(c2)) return fail(c, WH_EINVAL, "c2 must be finite and > 0");
  double modes = 1.0;
  for (int m = 0; m < c->dim; ++m) modes *= (double)(c->n[m] - 1);
  if (modes > (double)((int64_t)1 << 31)) return fail(c, WH_EINVAL, "more than 2^31 modes");
  std::vector<double> ax[3];
  for (int m = 0; m < c->dim; ++m)
    for (int64_t k = 1; k < c->n[m]; ++k) ax[m].push_back(axis_eigenvalue(c->order, c->n[m], k));
  const size_t nz = c->dim == 3 ? ax[2].size() : 1;
  unsigned nthreads = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
  struct Part {
    double lo = INFINITY, hi = -INFINITY;
    int32_t k[3] = {0, 0, 0};
    bool unstable = false;
  };
  std::vector<Part> parts(nthreads);
  auto work = [&](unsigned t) {
    Part &pt = parts[t];
    for (size_t kz = t; kz < nz; kz += nthreads)
      for (size_t ky = 0; ky < ax[1].size(); ++ky)
        for (size_t kx = 0; kx < ax[0].size(); ++kx) {
          const double lam2 = c2 * (ax[0][kx] + ax[1][ky] + (c->dim == 3 ? ax[2][kz] : 0.0));
          const double a = 1.0 - mode_beta(c, lam2);
          if (!std::isfinite(a)) {
            pt.unstable = true;
            continue;
          }
          if (a < pt.lo) {
            pt.lo = a;
            pt.k[0] = (int32_t)kx + 1;
            pt.k[1] = (int32_t)ky + 1;
            pt.k[2] = c->dim == 3 ? (int32_t)kz + 1 : 0;
          }
          pt.hi = std::max(pt.hi, a);
        }
  };
  try {
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nthreads; ++t) pool.emplace_back(work, t);
    work(0);
    for (auto &th : pool) th.join();
  } catch (const std::exception &) {
    return fail(c, WH_ENOMEM, "could not start host threads");
  }
  Part all;
  for (const Part &pt : parts) {
    all.unstable |= pt.unstable;
    all.hi = std::max(all.hi, pt.hi);
    if (pt.lo < all.lo) {
      all.lo = pt.lo;
      std::memcpy(all.k, pt.k, sizeof all.k);
    }
  }
  if (all.unstable) return fail(c, WH_EUNSTABLE, "c2 = %g puts modes beyond the stability limit of dt", c2);
  *a_min = all.lo;
  *a_max = all.hi;
  if (k_min) std::memcpy(k_min, all.k, sizeof all.k);
  return WH_OK;
}

wh_status wh_stream_bandwidth(int32_t kind, const void *src, void *dst, size_t bytes, int32_t groups, int32_t reps,
                              void *stream, double *ms_per_launch) {
  if (kind < 0 || kind > 3 || !ms_per_launch || reps < 1 || reps > 10000) return WH_EINVAL;
  if (bytes < 16 || bytes % (kind == 3 ? 144 : 16) != 0 || bytes > ((size_t)1 << 40)) return WH_EINVAL;
  if (groups < 0 || groups > 65535) return WH_EINVAL;
  if (kind != 2 && (!src || !is_device_ptr(src) || reinterpret_cast<uintptr_t>(src) % 16 != 0)) return WH_EINVAL;
  if (kind != 1 && (!dst || !is_device_ptr(dst) || reinterpret_cast<uintptr_t>(dst) % 16 != 0)) return WH_EINVAL;
  // kind 3: src holds 12 B and dst 16 B per node (bytes / 36 nodes)
  const size_t src_len = kind == 3 ? bytes / 3 : bytes, dst_len = kind == 3 ? bytes / 36 * 16 : bytes;
  if ((kind == 0 || kind == 3) && static_cast<const char *>(src) < static_cast<const char *>(dst) + dst_len &&
      static_cast<const char *>(dst) < static_cast<const char *>(src) + src_len)
    return WH_EINVAL;
  const int g = groups > 0 ? groups : 1024;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return WH_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return WH_EDEVICE;
  }
  wh_status st = WH_OK;
  float ms = 0.0f;
  if (wh::launch_stream(kind, src, dst, (int64_t)bytes, g, nullptr, s) != hipSuccess ||
      hipEventRecord(e0, s) != hipSuccess) {
    st = WH_EDEVICE;
  } else {
    for (int r = 0; r < reps && st == WH_OK; ++r)
      if (wh::launch_stream(kind, src, dst, (int64_t)bytes, g, nullptr, s) != hipSuccess) st = WH_EDEVICE;
    if (st == WH_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = WH_EDEVICE;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == WH_OK) *ms_per_launch = (double)ms / reps;
  return st;
}

wh_status wh_dot(wh_ctx *c, const double *x, const double *y, double *out) {
  WH_TRY(need(c, true, true, false, false, false));
  if (!out) return fail(c, WH_EINVAL, "out is NULL");
  WH_TRY(set_device(c));
  WH_TRY(check_dev(c, x, "x"));
  WH_TRY(check_dev(c, y, "y"));
  WH_TRY(dot_dev(c, x, y, 0));
  return fetch_scalars(c, 0, 1, out);
}

wh_status wh_helmholtz_residual(wh_ctx *c, const double *u, double *res, double *rel) {
  WH_TRY(need(c, true, true, true, true, true));
  WH_TRY(set_device(c));
  WH_TRY(check_dev(c, u, "u"));
  if (res) WH_TRY(check_dev(c, res, "res"));
  double *r = res ? res : c->tmp;
  if (r == u) return fail(c, WH_EINVAL, "res may not alias u");
  const wh::StepGeom g = geometry(c, 1.0);
  const bool fp32 = c->prec == WH_FP32_STATE;
  const double om = c->tp.omega;
  WH_HIP(c, wh::launch_helmholtz_residual(g, u, c->c2_is_const ? nullptr : c->c2, fp32, c->f, fp32, om * om, r,
                                          c->stream));
  if (rel) {
    // ||f||: f lives in state precision; convert into acc for the dot
    WH_HIP(c, wh::launch_from_state(fp32, c->f, c->acc, c->nodes, c->stream));
    WH_TRY(dot_dev(c, r, r, 0));
    WH_TRY(dot_dev(c, c->acc, c->acc, 1));
    double s[2];
    WH_TRY(fetch_scalars(c, 0, 2, s));
    *rel = s[1] > 0.0 ? std::sqrt(s[0] / s[1]) : std::sqrt(s[0]);
  }
  return WH_OK;
}

wh_status wh_set_tuning(wh_ctx *c, int32_t kernel, int32_t kblock, int32_t tile) {
  WH_TRY(need(c, true, false, false, false, false));
  if (!tuning_supported(c, kernel, kblock, tile))
    return fail(c, WH_EINVAL, "kernel %d with kblock %d and tile %d is not supported for this grid, order and precision",
                kernel, kblock, tile);
  c->kernel = kernel;
  c->kblock = kblock;
  c->tile = tile;
  return WH_OK;
}

wh_status wh_get_tuning(const wh_ctx *c, int32_t *kernel, int32_t *kblock, int32_t *tile, int32_t *owned_x,
                        int32_t *owned_y) {
  if (!c) return WH_EINVAL;
  if (!c->grid_set) return WH_ESTATE;
  const Tuning tu = resolve_tuning(c);
  int ox = 64, oy = 4;
  const int r = c->order / 2;
  if (tu.kernel == WH_KERNEL_BLOCKED_2D) {
    wh::block_tile_shape(c->prec == WH_FP32_STATE, c->order, tu.kblock, tu.tile, &ox, &oy);
  } else if (tu.kernel == WH_KERNEL_ZCOL_3D) {
    oy = 4;
  } else if (tu.kernel == WH_KERNEL_BLOCKED_3D) {
    ox = 64 - 2 * tu.kblock * r;
    oy = tu.tile - 2 * tu.kblock * r;
  }
  (void)r;
  if (kernel) *kernel = tu.kernel;
  if (kblock) *kblock = tu.kblock;
  if (tile) *tile = tu.tile;
  if (owned_x) *owned_x = ox;
  if (owned_y) *owned_y = oy;
  return WH_OK;
}

wh_status wh_autotune(wh_ctx *c, int32_t applies, int32_t *kernel, int32_t *kblock, int32_t *tile,
                      double *ms_per_apply) {
  WH_TRY(need(c, true, true, true, false, true));
  if (c->implicit) return fail(c, WH_EINVAL, "the autotuner chooses among explicit stepping kernels");
  if (applies < 1 || applies > 100) return fail(c, WH_EINVAL, "applies must be in 1..100");
  WH_TRY(set_device(c));
  std::vector<Tuning> cands{{WH_KERNEL_NODE, 1, 0}};
  if (c->dim == 3) {
    for (int zb : {4, 8, 16}) cands.push_back({WH_KERNEL_ZCOL_3D, 1, zb});
    const int rs = wh::block3d_rows_per_lane(c->prec == WH_FP32_STATE);
    for (int k = 2; k <= wh::kMaxBlockSteps3d; ++k)
      for (int rows : {16, 32})
        if (rows % rs == 0) cands.push_back({WH_KERNEL_BLOCKED_3D, k, rows});
  } else {
    for (int k = 2; k <= wh::kMaxBlockSteps; ++k)
      for (int nw : {4, 8, 10})
        cands.push_back({WH_KERNEL_BLOCKED_2D, k, nw * wh::block_rows_per_lane(c->prec == WH_FP32_STATE, c->order)});
  }
  const Tuning saved{c->kernel, c->kblock, c->tile};
  const bool saved_prof = c->profiling;
  c->profiling = false;
  hipEvent_t e0, e1;
  WH_HIP(c, hipEventCreate(&e0));
  WH_HIP(c, hipEventCreate(&e1));
  double best_ms = INFINITY;
  Tuning best = cands[0];
  wh_status st = WH_OK;
  // v = 0 (values do not change the timing of the stencil arithmetic)
  WH_HIP(c, wh::launch_fill(c->tmp, 0.0, c->nodes, c->stream));
  for (const Tuning &cd : cands) {
    if (!tuning_supported(c, cd.kernel, cd.kblock, cd.tile)) continue;
    c->kernel = cd.kernel;
    c->kblock = cd.kblock;
    c->tile = cd.tile;
    st = apply_impl(c, c->tmp, false, wh::FINAL_A, c->b, nullptr);  // warm-up
    if (st != WH_OK) break;
    if (hipEventRecord(e0, c->stream) != hipSuccess) {
      st = fail(c, WH_EDEVICE, "hipEventRecord failed");
      break;
    }
    for (int a = 0; a < applies && st == WH_OK; ++a) st = apply_impl(c, c->tmp, false, wh::FINAL_A, c->b, nullptr);
    if (st != WH_OK) break;
    float ms = 0.0f;
    if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(c, WH_EDEVICE, "event timing failed");
      break;
    }
    const double per = ms / applies;
    if (per < best_ms) {
      best_ms = per;
      best = cd;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->profiling = saved_prof;
  if (st != WH_OK) {
    c->kernel = saved.kernel;
    c->kblock = saved.kblock;
    c->tile = saved.tile;
    return st;
  }
  c->kernel = best.kernel;
  c->kblock = best.kblock;
  c->tile = best.tile;
  if (kernel) *kernel = best.kernel;
  if (kblock) *kblock = best.kblock;
  if (tile) *tile = best.tile;
  if (ms_per_apply) *ms_per_apply = best_ms;
  return WH_OK;
}

// ---------------------------------------------------------------------------
// solvers
// ---------------------------------------------------------------------------
// c->b <- the right-hand side: the given device vector, or b = W_h(0, f).
// Deflation (Alg. 3): remove the components along the deflated sine modes,
// or add back their Helmholtz components (f, phi) / (omega^2 - lambda^2).
static wh_status defl_project(wh_ctx *c, double *x) {
  if (c->defl_count == 0) return WH_OK;
  const wh::StepGeom g = geometry(c, 1.0);
  WH_HIP(c, wh::launch_mode_dot(g, false, x, c->defl_count, c->d_sx, c->d_sy, c->d_sz, c->d_dpart, c->d_coef,
                                c->stream));
  WH_HIP(c, wh::launch_mode_combine(g, x, c->defl_count, c->d_sx, c->d_sy, c->d_sz, c->d_coef, nullptr, -1.0,
                                    c->stream));
  return WH_OK;
}

static wh_status defl_inflate(wh_ctx *c, double *x) {
  if (c->defl_count == 0) return WH_OK;
  const double w2 = c->tp.omega * c->tp.omega;
  std::vector<double> scale((size_t)c->defl_count);
  for (int q = 0; q < c->defl_count; ++q) {
    const double d = w2 - c->defl_lam2[(size_t)q];
    if (d == 0.0) return fail(c, WH_EINVAL, "deflated mode %d is resonant (lambda = omega)", q);
    scale[(size_t)q] = 1.0 / d;
  }
  WH_HIP(c, hipMemcpyAsync(c->d_scale, scale.data(), scale.size() * 8, hipMemcpyHostToDevice, c->stream));
  const wh::StepGeom g = geometry(c, 1.0);
  WH_HIP(c, wh::launch_mode_dot(g, c->prec == WH_FP32_STATE, c->f, c->defl_count, c->d_sx, c->d_sy, c->d_sz,
                                c->d_dpart, c->d_coef_f, c->stream));
  WH_HIP(c, wh::launch_mode_combine(g, x, c->defl_count, c->d_sx, c->d_sy, c->d_sz, c->d_coef_f, c->d_scale, 1.0,
                                    c->stream));
  WH_HIP(c, hipStreamSynchronize(c->stream));  // scale is a host temporary
  return WH_OK;
}

static wh_status make_rhs(wh_ctx *c, const double *rhs, int *applies) {
  if (rhs) {
    if (rhs != c->b)
      WH_HIP(c, hipMemcpyAsync(c->b, rhs, (size_t)c->nodes * 8, hipMemcpyDeviceToDevice, c->stream));
    return WH_OK;
  }
  WH_HIP(c, wh::launch_fill(c->tmp, 0.0, c->nodes, c->stream));
  WH_TRY(apply_impl(c, c->tmp, true, wh::FINAL_FILTER, c->b, nullptr));
  ++*applies;
  return defl_project(c, c->b);
}

static wh_status solve_fpi(wh_ctx *c, const wh_solve_opts *o, double *v, wh_solve_info *info, const double *rhs) {
  const int nb = wh::reduction_blocks(c->nodes);
  WH_TRY(defl_project(c, v));
  // ||b||: b = W_h(0, f); when the initial guess is zero the first iterate is b
  double vv;
  WH_TRY(dot_dev(c, v, v, 0));
  WH_TRY(fetch_scalars(c, 0, 1, &vv));
  if (!std::isfinite(vv)) return fail(c, WH_ENONFINITE, "initial guess is not finite");
  double bnorm = -1.0;
  int applies = 0;
  if (vv != 0.0 || rhs) {
    WH_TRY(make_rhs(c, rhs, &applies));
    double bb;
    WH_TRY(dot_dev(c, c->b, c->b, 0));
    WH_TRY(fetch_scalars(c, 0, 1, &bb));
    bnorm = std::sqrt(bb);
  }
  double r_first = 0.0, r_prev = 0.0, r_last = 0.0;
  int k = 0;
  wh_status st = WH_OK;
  for (k = 1; k <= o->maxit; ++k) {
    if (rhs) {  // v <- S v + b
      WH_TRY(apply_impl(c, v, false, wh::FINAL_FILTER, c->tmp, nullptr));
      WH_HIP(c, wh::launch_add(c->tmp, c->b, c->tmp, c->nodes, c->stream));
    } else {  // v <- W_h(v, f), deflated
      WH_TRY(apply_impl(c, v, true, wh::FINAL_FILTER, c->tmp, nullptr));
      WH_TRY(defl_project(c, c->tmp));
    }
    ++applies;
    WH_HIP(c, wh::launch_diff_norm_copy(c->tmp, v, c->nodes, c->partials, nb, c->stream));
    WH_TRY(reduce_to(c, 1, 0));
    double rr;
    WH_TRY(fetch_scalars(c, 0, 1, &rr));
    const double r = std::sqrt(rr);
    if (!std::isfinite(r)) {
      st = fail(c, WH_ENONFINITE, "FPI residual became non-finite at iteration %d", k);
      break;
    }
    if (bnorm < 0.0) bnorm = r;  // zero initial guess: v^1 - v^0 = b
    if (k == 1) r_first = r;
    r_prev = r_last;
    r_last = r;
    const double rel = bnorm > 0.0 ? r / bnorm : 0.0;
    if (o->on_iter) o->on_iter(k, rel, o->user);
    if (o->rtol > 0.0 && rel <= o->rtol) break;
  }
  if (k > o->maxit) k = o->maxit;
  if (st == WH_OK) WH_TRY(defl_inflate(c, v));
  if (info) {
    info->iters = k;
    info->applies = applies;
    info->bnorm = bnorm;
    info->rel_res = bnorm > 0.0 ? r_last / bnorm : 0.0;
    info->scaled_res = r_last / std::sqrt((double)c->nodes);
    info->cr_last = (k >= 2 && r_prev > 0.0) ? r_last / r_prev : NAN;
    info->cr_avg = (k >= 2 && r_first > 0.0) ? std::pow(r_last / r_first, 1.0 / (k - 1)) : NAN;
    info->ecr = std::pow(info->cr_avg, 1.0 / c->tp.periods);
    info->point_steps = applies * point_steps_per_apply(c);
  }
  if (st == WH_OK && o->rtol > 0.0 && !(bnorm > 0.0 ? r_last / bnorm <= o->rtol : true))
    st = fail(c, WH_ENOTCONV, "FPI reached maxit = %d at relative residual %g", o->maxit,
              bnorm > 0.0 ? r_last / bnorm : 0.0);
  return st;
}

static wh_status solve_gmres(wh_ctx *c, const wh_solve_opts *o, double *x, wh_solve_info *info, const double *rhs) {
  const int m = o->restart;
  if (m < 1 || m > c->ws_restart)
    return fail(c, WH_EINVAL, "restart %d must be in 1..%d (the workspace's restart length)", m, c->ws_restart);
  const int64_t N = c->nodes;
  const int nb = wh::reduction_blocks(N);
  auto Vj = [&](int j) { return c->V + (int64_t)j * c->ldv; };
  // scalar slots on the device
  const int S_H1 = 0, S_H2 = m + 2, S_NRM = 2 * (m + 2);

  int applies = 0;
  WH_TRY(make_rhs(c, rhs, &applies));
  double bb;
  WH_TRY(dot_dev(c, c->b, c->b, S_NRM));
  WH_TRY(fetch_scalars(c, S_NRM, 1, &bb));
  const double bnorm = std::sqrt(bb);
  if (!std::isfinite(bnorm)) return fail(c, WH_ENONFINITE, "||b|| is not finite");

  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), h(2 * (m + 2) + 1);
  auto Hat = [&](int i, int j) -> double & { return H[(size_t)i * m + j]; };

  int total = 0;
  double rel = 0.0, r0_first = -1.0;
  wh_status st = WH_OK;
  bool done = false;
  // r = b - A x into V_0
  WH_TRY(defl_project(c, x));
  WH_TRY(apply_impl(c, x, false, wh::FINAL_A, c->tmp, nullptr));
  ++applies;
  WH_HIP(c, wh::launch_sub(c->b, c->tmp, Vj(0), N, c->stream));
  WH_TRY(defl_project(c, Vj(0)));
  while (!done) {
    double rr;
    WH_TRY(dot_dev(c, Vj(0), Vj(0), S_NRM));
    WH_TRY(fetch_scalars(c, S_NRM, 1, &rr));
    const double beta = std::sqrt(rr);
    if (!std::isfinite(beta)) {
      st = fail(c, WH_ENONFINITE, "GMRES residual became non-finite");
      break;
    }
    rel = bnorm > 0.0 ? beta / bnorm : 0.0;
    if (r0_first < 0.0) r0_first = rel;
    if (bnorm == 0.0 || rel <= o->rtol || total >= o->maxit) break;
    WH_HIP(c, wh::launch_scale_by_rnorm(Vj(0), Vj(0), c->scal + S_NRM, N, c->stream));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int kused = 0;
    for (int j = 0; j < m && total < o->maxit; ++j) {
      double *w = Vj(j + 1);
      WH_TRY(apply_impl(c, Vj(j), false, wh::FINAL_A, w, nullptr));
      WH_TRY(defl_project(c, w));
      ++applies;
      // classical Gram-Schmidt, twice (coefficients stay on the device between passes)
      WH_HIP(c, wh::launch_mdot(c->V, c->ldv, j + 1, w, N, c->partials, nb, c->stream));
      WH_TRY(reduce_to(c, j + 1, S_H1));
      WH_HIP(c, wh::launch_block_axpy(c->V, c->ldv, j + 1, c->scal + S_H1, w, N, c->stream));
      WH_HIP(c, wh::launch_mdot(c->V, c->ldv, j + 1, w, N, c->partials, nb, c->stream));
      WH_TRY(reduce_to(c, j + 1, S_H2));
      WH_HIP(c, wh::launch_block_axpy(c->V, c->ldv, j + 1, c->scal + S_H2, w, N, c->stream));
      WH_TRY(dot_dev(c, w, w, S_NRM));
      WH_TRY(fetch_scalars(c, 0, S_NRM + 1, h.data()));
      const double hn = std::sqrt(h[S_NRM]);
      for (int i = 0; i <= j; ++i) Hat(i, j) = h[S_H1 + i] + h[S_H2 + i];
      Hat(j + 1, j) = hn;
      if (!std::isfinite(hn)) {
        st = fail(c, WH_ENONFINITE, "GMRES Arnoldi vector became non-finite");
        done = true;
        break;
      }
      if (hn > 0.0) WH_HIP(c, wh::launch_scale_by_rnorm(w, w, c->scal + S_NRM, N, c->stream));
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * Hat(i, j) + sn[i] * Hat(i + 1, j);
        Hat(i + 1, j) = -sn[i] * Hat(i, j) + cs[i] * Hat(i + 1, j);
        Hat(i, j) = t;
      }
      const double den = std::hypot(Hat(j, j), Hat(j + 1, j));
      cs[j] = den > 0.0 ? Hat(j, j) / den : 1.0;
      sn[j] = den > 0.0 ? Hat(j + 1, j) / den : 0.0;
      Hat(j, j) = den;
      Hat(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      kused = j + 1;
      const double est = bnorm > 0.0 ? std::fabs(g[j + 1]) / bnorm : 0.0;
      if (o->on_iter) o->on_iter(total, est, o->user);
      if (est <= o->rtol || hn == 0.0) break;
    }
    if (st != WH_OK) break;
    if (kused == 0) break;
    // y = R^{-1} g, x += V y
    for (int i = kused - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < kused; ++l) s -= Hat(i, l) * y[l];
      y[i] = s / Hat(i, i);
    }
    std::memcpy(c->pinned, y.data(), (size_t)kused * 8);
    WH_HIP(c, hipMemcpyAsync(c->scal + S_H1, c->pinned, (size_t)kused * 8, hipMemcpyHostToDevice, c->stream));
    WH_HIP(c, wh::launch_block_gemv_add(c->V, c->ldv, kused, c->scal + S_H1, x, N, c->stream));
    // true residual, also the next cycle's starting vector
    WH_TRY(apply_impl(c, x, false, wh::FINAL_A, c->tmp, nullptr));
    ++applies;
    WH_HIP(c, wh::launch_sub(c->b, c->tmp, Vj(0), N, c->stream));
    WH_TRY(defl_project(c, Vj(0)));
  }
  if (st == WH_OK) WH_TRY(defl_inflate(c, x));
  WH_HIP(c, hipStreamSynchronize(c->stream));
  if (info) {
    info->iters = total;
    info->applies = applies;
    info->bnorm = bnorm;
    info->rel_res = rel;
    info->scaled_res = rel * bnorm / std::sqrt((double)N);
    info->cr_last = (total > 0 && r0_first > 0.0) ? std::pow(rel / r0_first, 1.0 / total) : NAN;
    info->cr_avg = info->cr_last;
    info->ecr = std::pow(info->cr_avg, 1.0 / c->tp.periods);
    info->point_steps = applies * point_steps_per_apply(c);
  }
  if (st == WH_OK && rel > o->rtol)
    st = fail(c, WH_ENOTCONV, "GMRES reached maxit = %d at relative residual %g", o->maxit, rel);
  return st;
}

// Extreme eigenvalues of the symmetric tridiagonal matrix that CG's step
// lengths alpha_j and residual ratios beta_j define (the Lanczos matrix of
// the Krylov space CG has built): T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
// T_j,j+1 = sqrt(beta_j)/alpha_j.  Bisection on Sturm counts.
static void lanczos_extremes(const std::vector<double> &alpha, const std::vector<double> &beta, double *lo,
                             double *hi) {
  const size_t m = alpha.size();
  *lo = *hi = NAN;
  if (m == 0) return;
  std::vector<double> d(m), e(m > 1 ? m - 1 : 0);
  for (size_t j = 0; j < m; ++j) d[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
  for (size_t j = 0; j + 1 < m; ++j) e[j] = std::sqrt(beta[j]) / alpha[j];
  double glo = INFINITY, ghi = -INFINITY;
  for (size_t j = 0; j < m; ++j) {
    const double r = (j > 0 ? std::fabs(e[j - 1]) : 0.0) + (j + 1 < m ? std::fabs(e[j]) : 0.0);
    glo = std::min(glo, d[j] - r);
    ghi = std::max(ghi, d[j] + r);
  }
  if (!std::isfinite(glo) || !std::isfinite(ghi)) return;
  // number of eigenvalues below x
  auto below = [&](double x) {
    size_t cnt = 0;
    double q = d[0] - x;
    if (q < 0.0) ++cnt;
    for (size_t j = 1; j < m; ++j) {
      if (q == 0.0) q = 1e-300;
      q = d[j] - x - e[j - 1] * e[j - 1] / q;
      if (q < 0.0) ++cnt;
    }
    return cnt;
  };
  double a = glo, b = ghi;
  for (int it = 0; it < 200 && b - a > 1e-15 * std::max(std::fabs(a), std::fabs(b)); ++it) {
    const double mid = 0.5 * (a + b);
    if (below(mid) >= 1) b = mid;
    else a = mid;
  }
  *lo = 0.5 * (a + b);
  a = glo;
  b = ghi;
  for (int it = 0; it < 200 && b - a > 1e-15 * std::max(std::fabs(a), std::fabs(b)); ++it) {
    const double mid = 0.5 * (a + b);
    if (below(mid) >= m) b = mid;
    else a = mid;
  }
  *hi = 0.5 * (a + b);
}

// Conjugate gradients on A v = b in the inner product <u, w> = sum u w / c^2.
// Iteration k keeps <r, r>_w and ||r||^2 in device slot (k & 1); the update
// kernels read their coefficients from device memory, so each iteration
// synchronises with the host once (for the convergence test).
static wh_status solve_cg(wh_ctx *c, const wh_solve_opts *o, double *x, wh_solve_info *info, const double *rhs) {
  if (c->ws_restart < 2) return fail(c, WH_ENOMEM, "CG needs a workspace sized for restart >= 2");
  const int64_t N = c->nodes;
  const int nb = wh::reduction_blocks(N);
  const bool fp32 = c->prec == WH_FP32_STATE;
  const void *c2w = c->c2_is_const ? nullptr : c->c2;
  double *r = c->V, *p = c->V + c->ldv, *q = c->V + 2 * c->ldv;
  const int S_PQ = 2;
  auto slot = [](int64_t k) { return 4 + 2 * (int)(k & 1); };  // [<r,r>_w, <r,r>]

  int applies = 0;
  WH_TRY(make_rhs(c, rhs, &applies));
  double bb;
  WH_TRY(dot_dev(c, c->b, c->b, 0));
  WH_TRY(fetch_scalars(c, 0, 1, &bb));
  const double bnorm = std::sqrt(bb);
  if (!std::isfinite(bnorm)) return fail(c, WH_ENONFINITE, "||b|| is not finite");

  // r = b - A x, p = r, slot(k) = [<r,r>_w, <r,r>]
  WH_TRY(defl_project(c, x));
  auto restart = [&](int64_t k, double *rel) -> wh_status {
    WH_TRY(apply_impl(c, x, false, wh::FINAL_A, c->tmp, nullptr));
    ++applies;
    WH_HIP(c, wh::launch_sub(c->b, c->tmp, r, N, c->stream));
    WH_TRY(defl_project(c, r));
    WH_HIP(c, wh::launch_wdot(r, r, c2w, fp32, N, c->partials, nb, c->stream));
    WH_TRY(reduce_to(c, 1, slot(k)));
    WH_TRY(dot_dev(c, r, r, slot(k) + 1));
    WH_HIP(c, hipMemcpyAsync(p, r, (size_t)N * 8, hipMemcpyDeviceToDevice, c->stream));
    double ee;
    WH_TRY(fetch_scalars(c, slot(k) + 1, 1, &ee));
    *rel = bnorm > 0.0 ? std::sqrt(ee) / bnorm : 0.0;
    return WH_OK;
  };

  double rel = 0.0, rel0 = -1.0, rel_rec = NAN;
  int64_t k = 0;
  wh_status st = WH_OK;
  // CG's coefficients since the last restart (the Lanczos matrix)
  std::vector<double> alphas, betas, best_a, best_b;
  WH_TRY(restart(k, &rel));
  rel0 = rel;
  while (bnorm > 0.0 && rel > o->rtol && k < o->maxit) {
    WH_TRY(apply_impl(c, p, false, wh::FINAL_A, q, nullptr));  // q = A p
    WH_TRY(defl_project(c, q));
    ++applies;
    WH_HIP(c, wh::launch_wdot(p, q, c2w, fp32, N, c->partials, nb, c->stream));
    WH_TRY(reduce_to(c, 1, S_PQ));
    const int cur = slot(k), nxt = slot(k + 1);
    WH_HIP(c, wh::launch_cg_update(x, r, p, q, c2w, fp32, c->scal + cur, c->scal + S_PQ, N, c->partials, nb,
                                   c->stream));
    WH_TRY(reduce_to(c, 2, nxt));
    ++k;
    double sc[8];
    WH_TRY(fetch_scalars(c, 0, 8, sc));
    const double pq = sc[S_PQ];
    const double ee = sc[nxt + 1];
    if (!std::isfinite(pq) || !std::isfinite(ee)) {
      st = fail(c, WH_ENONFINITE, "CG became non-finite at iteration %lld", (long long)k);
      break;
    }
    if (!(pq > 0.0)) {
      st = fail(c, WH_ENOTCONV, "CG breakdown: <p, A p> = %g <= 0 at iteration %lld", pq, (long long)k);
      break;
    }
    rel = bnorm > 0.0 ? std::sqrt(ee) / bnorm : 0.0;
    rel_rec = rel;
    alphas.push_back(sc[cur] / pq);
    betas.push_back(sc[nxt] / sc[cur]);
    if (o->on_iter) o->on_iter((int32_t)k, rel, o->user);
    if (rel <= o->rtol) {
      // confirm with the true residual; continue from it if rounding drifted
      WH_TRY(restart(k, &rel));
      if (rel <= o->rtol) break;
      // a restart begins a new Lanczos sequence; keep the longest one
      if (alphas.size() > best_a.size()) {
        best_a.swap(alphas);
        best_b.swap(betas);
      }
      alphas.clear();
      betas.clear();
      continue;
    }
    WH_HIP(c, wh::launch_xpay(r, p, c->scal + nxt, c->scal + cur, N, c->stream));
  }
  // stopped by maxit: report the true residual beside the recursive one
  if (st == WH_OK && bnorm > 0.0 && rel > o->rtol && k > 0) WH_TRY(restart(k, &rel));
  if (st == WH_OK) WH_TRY(defl_inflate(c, x));
  WH_HIP(c, hipStreamSynchronize(c->stream));
  if (info) {
    info->iters = (int32_t)k;
    info->applies = applies;
    info->bnorm = bnorm;
    info->rel_res = rel;
    info->scaled_res = rel * bnorm / std::sqrt((double)N);
    info->cr_last = (k > 0 && rel0 > 0.0) ? std::pow(rel / rel0, 1.0 / (double)k) : NAN;
    info->cr_avg = info->cr_last;
    info->ecr = std::pow(info->cr_avg, 1.0 / c->tp.periods);
    info->point_steps = applies * point_steps_per_apply(c);
    info->rel_res_recursive = rel_rec;
    if (best_a.size() > alphas.size()) {
      alphas.swap(best_a);
      betas.swap(best_b);
    }
    if (!betas.empty()) betas.pop_back();  // beta_k only couples to a step not taken
    lanczos_extremes(alphas, betas, &info->ritz_min, &info->ritz_max);
  }
  if (st == WH_OK && rel > o->rtol)
    st = fail(c, WH_ENOTCONV, "CG reached maxit = %d at relative residual %g", o->maxit, rel);
  return st;
}

static wh_status check_opts(wh_ctx *c, const wh_solve_opts *o) {
  if (!o) return fail(c, WH_EINVAL, "opts is NULL");
  if (o->flags != 0) return fail(c, WH_EINVAL, "opts.flags must be 0");
  if (o->maxit < 1) return fail(c, WH_EINVAL, "maxit must be >= 1");
  if (!(o->rtol >= 0.0) || !std::isfinite(o->rtol)) return fail(c, WH_EINVAL, "rtol must be finite and >= 0");
  if (o->method != WH_SOLVER_FPI && o->method != WH_SOLVER_GMRES && o->method != WH_SOLVER_CG)
    return fail(c, WH_EINVAL, "unknown method");
  return WH_OK;
}

static wh_status solve_dispatch(wh_ctx *c, const wh_solve_opts *o, const double *rhs, double *v,
                                wh_solve_info *info) {
  WH_TRY(set_device(c));
  WH_TRY(check_dev(c, v, "v"));
  if (rhs) {
    WH_TRY(check_dev(c, rhs, "b"));
    if (rhs == v) return fail(c, WH_EINVAL, "b may not alias v");
    if (c->defl_count > 0)
      return fail(c, WH_EINVAL, "deflation applies to wh_solve (right-hand side from the source); "
                                "call wh_set_deflation with count 0 first");
  }
  if (info) std::memset(info, 0, sizeof *info);
  const auto t0 = std::chrono::steady_clock::now();
  wh_status st;
  try {
    if (o->method == WH_SOLVER_FPI) st = solve_fpi(c, o, v, info, rhs);
    else if (o->method == WH_SOLVER_GMRES) st = solve_gmres(c, o, v, info, rhs);
    else st = solve_cg(c, o, v, info, rhs);
  } catch (const std::bad_alloc &) {
    st = fail(c, WH_ENOMEM, "host allocation failed");
  } catch (...) {
    st = fail(c, WH_EDEVICE, "unexpected exception");
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess && st == WH_OK)
    st = fail(c, WH_EDEVICE, "stream synchronisation failed");
  if (info) {
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->mu_pred = predicted_rate(c);
    if (o->method != WH_SOLVER_CG) info->rel_res_recursive = info->ritz_min = info->ritz_max = NAN;
  }
  return st;
}

wh_status wh_solve(wh_ctx *c, const wh_solve_opts *o, double *v, wh_solve_info *info) {
  WH_TRY(need(c, true, true, true, true, true));
  WH_TRY(check_opts(c, o));
  return solve_dispatch(c, o, nullptr, v, info);
}

wh_status wh_solve_rhs(wh_ctx *c, const wh_solve_opts *o, const double *b, double *v, wh_solve_info *info) {
  WH_TRY(need(c, true, true, true, false, true));
  WH_TRY(check_opts(c, o));
  if (!b) return fail(c, WH_EINVAL, "b is NULL");
  return solve_dispatch(c, o, b, v, info);
}

wh_status wh_solve_mixed(wh_ctx *hi, wh_ctx *lo, const wh_solve_opts *outer, const wh_solve_opts *inner, double *v,
                         wh_solve_info *info) {
  WH_TRY(need(hi, true, true, true, true, true));
  WH_TRY(need(lo, true, true, true, false, true));
  if (!outer || !inner) return fail(hi, WH_EINVAL, "opts is NULL");
  if (outer->maxit < 1 || !(outer->rtol > 0.0) || !std::isfinite(outer->rtol))
    return fail(hi, WH_EINVAL, "outer maxit must be >= 1 and outer rtol finite and > 0");
  WH_TRY(check_opts(lo, inner));
  if (hi->prec != WH_FP64) return fail(hi, WH_EINVAL, "the outer context must use WH_FP64");
  if (hi->device != lo->device) return fail(hi, WH_EINVAL, "contexts on different devices");
  if (hi->dim != lo->dim || hi->order != lo->order || hi->n[0] != lo->n[0] || hi->n[1] != lo->n[1] ||
      hi->n[2] != lo->n[2])
    return fail(hi, WH_EINVAL, "the two contexts must describe the same grid and order");
  if (hi->tp.nt != lo->tp.nt || hi->tp.periods != lo->tp.periods || hi->tp.dt != lo->tp.dt ||
      hi->tp.alpha != lo->tp.alpha)
    return fail(hi, WH_EINVAL, "the two contexts must use the same time parameters");
  if (hi->ws_restart < 2) return fail(hi, WH_ENOMEM, "the outer context needs a workspace sized for restart >= 2");
  if (hi->defl_count > 0 || lo->defl_count > 0)
    return fail(hi, WH_EINVAL, "residual correction does not deflate: call wh_set_deflation with count 0 on both "
                               "contexts first");
  WH_TRY(set_device(hi));
  WH_TRY(check_dev(hi, v, "v"));
  if (info) std::memset(info, 0, sizeof *info);
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t N = hi->nodes;
  double *r = hi->V, *d = hi->V + hi->ldv;
  int applies_hi = 0, applies_lo = 0, inner_iters = 0;
  WH_TRY(make_rhs(hi, nullptr, &applies_hi));
  double bb;
  WH_TRY(dot_dev(hi, hi->b, hi->b, 0));
  WH_TRY(fetch_scalars(hi, 0, 1, &bb));
  const double bnorm = std::sqrt(bb);
  if (!std::isfinite(bnorm)) return fail(hi, WH_ENONFINITE, "||b|| is not finite");
  double rel = 0.0, rel0 = -1.0;
  int k = 0;
  wh_status st = WH_OK;
  for (;;) {
    // FP64 residual of the current iterate
    WH_TRY(apply_impl(hi, v, false, wh::FINAL_A, hi->tmp, nullptr));
    ++applies_hi;
    WH_HIP(hi, wh::launch_sub(hi->b, hi->tmp, r, N, hi->stream));
    double rr;
    WH_TRY(dot_dev(hi, r, r, 0));
    WH_TRY(fetch_scalars(hi, 0, 1, &rr));
    rel = bnorm > 0.0 ? std::sqrt(rr) / bnorm : 0.0;
    if (!std::isfinite(rel)) {
      st = fail(hi, WH_ENONFINITE, "mixed-precision residual became non-finite");
      break;
    }
    if (rel0 < 0.0) rel0 = rel;
    if (outer->on_iter) outer->on_iter(k, rel, outer->user);
    if (rel <= outer->rtol || k >= outer->maxit) break;
    // correction from the state-precision operator: A_lo d = r
    WH_HIP(hi, wh::launch_fill(d, 0.0, N, hi->stream));
    WH_HIP(hi, hipStreamSynchronize(hi->stream));
    wh_solve_info in{};
    const wh_status sl = solve_dispatch(lo, inner, r, d, &in);
    applies_lo += in.applies;
    inner_iters += in.iters;
    if (sl != WH_OK && sl != WH_ENOTCONV) {
      st = fail(hi, sl, "inner solve failed: %s", lo->err.c_str());
      break;
    }
    WH_HIP(hi, wh::launch_add(v, d, v, N, hi->stream));
    ++k;
  }
  WH_HIP(hi, hipStreamSynchronize(hi->stream));
  if (info) {
    info->iters = k;
    info->applies = applies_hi + applies_lo;
    info->bnorm = bnorm;
    info->rel_res = rel;
    info->scaled_res = rel * bnorm / std::sqrt((double)N);
    info->cr_last = (k > 0 && rel0 > 0.0) ? std::pow(rel / rel0, 1.0 / k) : NAN;
    info->cr_avg = info->cr_last;
    info->ecr = std::pow(info->cr_avg, 1.0 / hi->tp.periods);
    info->point_steps = applies_hi * point_steps_per_apply(hi) + applies_lo * point_steps_per_apply(lo);
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->mu_pred = predicted_rate(hi);
    info->rel_res_recursive = info->ritz_min = info->ritz_max = NAN;
  }
  (void)inner_iters;
  if (st == WH_OK && rel > outer->rtol)
    st = fail(hi, WH_ENOTCONV, "mixed-precision refinement reached maxit = %d at relative residual %g",
              outer->maxit, rel);
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// deflation with the sine modes of the unit box (Alg. 3)
// ---------------------------------------------------------------------------
namespace {

struct DeflLayout {
  size_t sx, sy, sz, coef, coef_f, scale, part, total;
  int nblocks;
};

DeflLayout defl_layout(const wh_ctx *c, int count) {
  DeflLayout L{};
  L.nblocks = wh::mode_blocks(geometry(c, 1.0));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t M = (size_t)count;
  L.sx = take(M * (size_t)(c->n[0] + 1) * 8);
  L.sy = take(M * (size_t)(c->n[1] + 1) * 8);
  L.sz = take(c->dim == 3 ? M * (size_t)(c->n[2] + 1) * 8 : 8);
  L.coef = take(M * 8);
  L.coef_f = take(M * 8);
  L.scale = take(M * 8);
  L.part = take(M * (size_t)L.nblocks * 8);
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

wh_status wh_deflation_workspace_size(wh_ctx *c, int32_t count, size_t *bytes) {
  WH_TRY(need(c, true, false, false, false, false));
  if (!bytes) return fail(c, WH_EINVAL, "bytes is NULL");
  if (count < 0 || count > WH_MAX_DEFLATION) return fail(c, WH_EINVAL, "count must be in 0..%d", WH_MAX_DEFLATION);
  *bytes = defl_layout(c, count).total;
  return WH_OK;
}

wh_status wh_set_deflation(wh_ctx *c, const int32_t *modes, int32_t count, void *workspace, size_t bytes) {
  WH_TRY(need(c, true, true, true, false, false));
  if (count == 0) {
    c->defl_count = 0;
    return WH_OK;
  }
  if (!c->c2_is_const) return fail(c, WH_EINVAL, "deflation with sine modes needs a constant c^2");
  if (count < 0 || count > WH_MAX_DEFLATION) return fail(c, WH_EINVAL, "count must be in 0..%d", WH_MAX_DEFLATION);
  if (!modes) return fail(c, WH_EINVAL, "modes is NULL");
  const DeflLayout L = defl_layout(c, count);
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(c, WH_EINVAL, "deflation workspace must be a 256-byte aligned device pointer");
  if (bytes < L.total) return fail(c, WH_ENOMEM, "deflation workspace of %zu bytes needed", L.total);
  WH_TRY(set_device(c));
  WH_TRY(check_dev(c, workspace, "deflation workspace"));
  std::vector<int64_t> seen;
  seen.reserve((size_t)count);
  for (int q = 0; q < count; ++q) {
    for (int m = 0; m < c->dim; ++m) {
      const int32_t k = modes[(size_t)q * c->dim + m];
      if (k < 1 || k >= c->n[m]) return fail(c, WH_EINVAL, "mode %d: wave number %d outside 1..%lld", q, k,
                                              (long long)(c->n[m] - 1));
    }
    seen.push_back(mode_index(c, modes + (size_t)q * c->dim));
  }
  std::sort(seen.begin(), seen.end());
  if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) return fail(c, WH_EINVAL, "modes repeat");
  char *base = static_cast<char *>(workspace);
  c->d_sx = reinterpret_cast<double *>(base + L.sx);
  c->d_sy = reinterpret_cast<double *>(base + L.sy);
  c->d_sz = reinterpret_cast<double *>(base + L.sz);
  c->d_coef = reinterpret_cast<double *>(base + L.coef);
  c->d_coef_f = reinterpret_cast<double *>(base + L.coef_f);
  c->d_scale = reinterpret_cast<double *>(base + L.scale);
  c->d_dpart = reinterpret_cast<double *>(base + L.part);
  // normalized 1-D factors sqrt(2/n) sin(k pi i / n), exactly 0 on the walls
  double *tables[3] = {c->d_sx, c->d_sy, c->d_sz};
  c->defl_lam2.assign((size_t)count, 0.0);
  for (int m = 0; m < c->dim; ++m) {
    const int64_t n = c->n[m];
    std::vector<double> t((size_t)count * (n + 1), 0.0);
    const double nrm = std::sqrt(2.0 / (double)n);
    for (int q = 0; q < count; ++q) {
      const int32_t k = modes[(size_t)q * c->dim + m];
      for (int64_t i = 1; i < n; ++i) t[(size_t)q * (n + 1) + i] = nrm * std::sin(M_PI * (double)k * (double)i / (double)n);
      c->defl_lam2[(size_t)q] += c->c2_value * axis_eigenvalue(c->order, n, k);
    }
    WH_HIP(c, hipMemcpyAsync(tables[m], t.data(), t.size() * 8, hipMemcpyHostToDevice, c->stream));
    WH_HIP(c, hipStreamSynchronize(c->stream));
  }
  c->defl_modes.assign(modes, modes + (size_t)count * c->dim);
  c->defl_count = count;
  return WH_OK;
}

wh_status wh_select_deflation(wh_ctx *c, int32_t count, int32_t *modes, double *mu_after) {
  WH_TRY(need(c, true, false, true, false, true));
  if (!c->c2_is_const) return fail(c, WH_EINVAL, "deflation with sine modes needs a constant c^2");
  if (count < 0 || count > WH_MAX_DEFLATION) return fail(c, WH_EINVAL, "count must be in 0..%d", WH_MAX_DEFLATION);
  if (count > 0 && !modes) return fail(c, WH_EINVAL, "modes is NULL");
  double total = 1.0;
  for (int m = 0; m < c->dim; ++m) total *= (double)(c->n[m] - 1);
  if (total > (double)(1 << 24)) return fail(c, WH_EINVAL, "too many modes to rank (%.0f)", total);
  if ((double)count > total) return fail(c, WH_EINVAL, "count %d exceeds the %.0f modes", count, total);
  std::vector<double> ax[3];
  for (int m = 0; m < c->dim; ++m)
    for (int64_t k = 1; k < c->n[m]; ++k) ax[m].push_back(axis_eigenvalue(c->order, c->n[m], k));
  const size_t M = (size_t)total;
  std::vector<double> absb(M);
  const size_t nx = ax[0].size(), ny = ax[1].size();
  for (size_t idx = 0; idx < M; ++idx) {
    const size_t i = idx % nx, j = (idx / nx) % ny, k = idx / (nx * ny);
    const double lam2 = c->c2_value * (ax[0][i] + ax[1][j] + (c->dim == 3 ? ax[2][k] : 0.0));
    const double b = mode_beta(c, lam2);
    absb[idx] = std::isfinite(b) ? std::fabs(b) : 0.0;
  }
  // the count slowest-converging modes (largest |beta_d|; ties by index)
  std::vector<int64_t> order(M);
  for (size_t i = 0; i < M; ++i) order[i] = (int64_t)i;
  auto slower = [&](int64_t a, int64_t b) { return absb[a] > absb[b] || (absb[a] == absb[b] && a < b); };
  std::partial_sort(order.begin(), order.begin() + count, order.end(), slower);
  for (int q = 0; q < count; ++q) {
    const size_t idx = (size_t)order[(size_t)q];
    modes[(size_t)q * c->dim + 0] = (int32_t)(idx % nx) + 1;
    modes[(size_t)q * c->dim + 1] = (int32_t)((idx / nx) % ny) + 1;
    if (c->dim == 3) modes[(size_t)q * c->dim + 2] = (int32_t)(idx / (nx * ny)) + 1;
  }
  if (mu_after) {
    std::vector<char> taken(M, 0);
    for (int q = 0; q < count; ++q) taken[(size_t)order[(size_t)q]] = 1;
    double mu = 0.0;
    for (size_t idx = 0; idx < M; ++idx)
      if (!taken[idx]) mu = std::max(mu, absb[idx]);
    *mu_after = mu;
  }
  return WH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// discrete adjoint: gradient of lam . W_h(v, f) and the adjoint fixed-point
// solve
// ---------------------------------------------------------------------------
namespace {

// Checkpointing of the forward levels W^0..W^{N-1} of one application: pairs
// (W^k, W^{k+1}) at k = j s (s = ceil(sqrt(N)), j < ncp = ceil(N/s)); the
// reverse sweep recomputes one segment of s levels at a time.
struct AdjLayout {
  int64_t N;
  int seg, ncp;
  size_t stride, total;
  size_t buffers;
};

AdjLayout adjoint_layout(const wh_ctx *c) {
  AdjLayout L{};
  L.N = (int64_t)c->tp.nt * c->tp.periods;
  L.seg = (int)std::ceil(std::sqrt((double)L.N));
  if ((int64_t)L.seg * L.seg < L.N) ++L.seg;
  L.ncp = (int)((L.N + L.seg - 1) / L.seg);
  L.stride = align256((size_t)c->nodes * 8);
  // checkpoint pairs, segment levels beyond the pair, two adjoint levels,
  // c^2 lam and the two sensitivity accumulators
  L.buffers = (size_t)2 * L.ncp + (size_t)std::max(L.seg - 2, 0) + 2 + 3;
  L.total = L.buffers * L.stride;
  return L;
}

wh_status need_fp64(wh_ctx *c, const char *what) {
  if (c->prec != WH_FP64) return fail(c, WH_EINVAL, "%s needs an FP64-state context", what);
  if (c->implicit) return fail(c, WH_EINVAL, "%s is built for explicit time stepping", what);
  return WH_OK;
}

}  // namespace

extern "C" {

wh_status wh_set_implicit(wh_ctx *c, int32_t nits, double inner_rtol) {
  WH_TRY(need(c, true, false, false, false, false));
  if (nits == 0) {
    c->implicit = false;
    c->freq_set = false;
    c->mg_ready = false;
    return WH_OK;
  }
  if (c->dim != 2) return fail(c, WH_EINVAL, "implicit time stepping is built for 2-D grids");
  if (c->prec != WH_FP64) return fail(c, WH_EINVAL, "implicit time stepping needs an FP64-state context");
  if (nits < 5 || nits > 100000)
    return fail(c, WH_EINVAL, "implicit stepping needs 5 <= steps per period <= 100000 (got %d)", nits);
  if (!(inner_rtol > 0.0) || inner_rtol > 1e-2)
    return fail(c, WH_EINVAL, "inner tolerance must be in (0, 1e-2] (got %g)", inner_rtol);
  c->implicit = true;
  c->nits = nits;
  c->imp_rtol = inner_rtol;
  c->freq_set = false;
  c->mg_ready = false;
  c->defl_count = 0;
  return WH_OK;
}

wh_status wh_implicit_workspace_size(const wh_ctx *c, size_t *bytes) {
  if (!c || !bytes) return WH_EINVAL;
  if (!c->grid_set) return WH_ESTATE;
  *bytes = imp_layout(c).total;
  return WH_OK;
}

wh_status wh_bind_implicit_workspace(wh_ctx *c, void *ptr, size_t bytes) {
  WH_TRY(need(c, true, false, false, false, false));
  c->mg_ready = false;
  if (!ptr) {
    c->imp = nullptr;
    c->imp_bytes = 0;
    return WH_OK;
  }
  if (reinterpret_cast<uintptr_t>(ptr) % 256 != 0)
    return fail(c, WH_EINVAL, "implicit workspace must be 256-byte aligned");
  const size_t need_bytes = imp_layout(c).total;
  if (bytes < need_bytes)
    return fail(c, WH_ENOMEM, "implicit workspace too small: %zu bytes given, %zu needed", bytes, need_bytes);
  WH_TRY(set_device(c));
  WH_TRY(check_dev(c, ptr, "implicit workspace"));
  c->imp = static_cast<char *>(ptr);
  c->imp_bytes = bytes;
  if (c->implicit && c->freq_set) return mg_setup(c);
  return WH_OK;
}

wh_status wh_implicit_stats(const wh_ctx *c, int64_t *steps, int64_t *inner_iters, int32_t *max_inner,
                            int32_t *levels) {
  if (!c) return WH_EINVAL;
  if (steps) *steps = c->imp_steps;
  if (inner_iters) *inner_iters = c->imp_iters;
  if (max_inner) *max_inner = c->imp_max;
  if (levels) *levels = c->mg_ready ? (int32_t)c->mg.size() : 0;
  return WH_OK;
}

wh_status wh_adjoint_workspace_size(wh_ctx *c, size_t *bytes) {
  WH_TRY(need(c, true, false, false, false, true));
  if (!bytes) return fail(c, WH_EINVAL, "bytes is NULL");
  *bytes = adjoint_layout(c).total;
  return WH_OK;
}

wh_status wh_bind_adjoint_workspace(wh_ctx *c, void *ptr, size_t bytes) {
  WH_TRY(need(c, true, false, false, false, false));
  if (!ptr) {
    c->adj = nullptr;
    c->adj_bytes = 0;
    return WH_OK;
  }
  if (reinterpret_cast<uintptr_t>(ptr) % 256 != 0) return fail(c, WH_EINVAL, "adjoint workspace must be 256-byte aligned");
  WH_TRY(set_device(c));
  WH_TRY(check_dev(c, ptr, "adjoint workspace"));
  c->adj = static_cast<char *>(ptr);
  c->adj_bytes = bytes;
  return WH_OK;
}

wh_status wh_gradient(wh_ctx *c, const double *v, const double *lam, double *grad_c2, double *grad_f,
                      double *grad_v) {
  WH_TRY(need(c, true, true, true, true, true));
  WH_TRY(need_fp64(c, "wh_gradient"));
  WH_TRY(set_device(c));
  WH_TRY(check_dev(c, v, "v"));
  WH_TRY(check_dev(c, lam, "lam"));
  double *outs[3] = {grad_c2, grad_f, grad_v};
  for (int i = 0; i < 3; ++i) {
    if (!outs[i]) continue;
    WH_TRY(check_dev(c, outs[i], "gradient output"));
    if (outs[i] == v || outs[i] == lam) return fail(c, WH_EINVAL, "gradient outputs may not alias v or lam");
    for (int k = 0; k < i; ++k)
      if (outs[k] == outs[i]) return fail(c, WH_EINVAL, "gradient outputs must be distinct");
  }
  const AdjLayout L = adjoint_layout(c);
  if (!c->adj || c->adj_bytes < L.total)
    return fail(c, WH_ENOMEM, "adjoint workspace of %zu bytes needed (wh_adjoint_workspace_size)", L.total);
  auto buf = [&](size_t i) { return reinterpret_cast<double *>(c->adj + i * L.stride); };
  auto cpA = [&](int j) { return buf((size_t)2 * j); };
  auto cpB = [&](int j) { return buf((size_t)2 * j + 1); };
  const size_t seg0 = (size_t)2 * L.ncp, zbase = seg0 + (size_t)std::max(L.seg - 2, 0);
  double *zc = buf(zbase), *zp = buf(zbase + 1), *clam = buf(zbase + 2), *gf = buf(zbase + 3),
         *gc = buf(zbase + 4);
  const double dt2 = c->tp.dt * c->tp.dt;
  const wh::StepGeom g = geometry(c, dt2), half = geometry(c, 0.5 * dt2);
  const double *c2p = c->c2_is_const ? nullptr : static_cast<const double *>(c->c2);
  const double *f = static_cast<const double *>(c->f);
  const size_t nb = (size_t)c->nodes * 8;
  hipStream_t s = c->stream;
  auto step = [&](const double *cur, double *prev_next, int64_t from) -> wh_status {
    // W^{from+1} = 2 W^from - W^{from-1} + c^2 dt^2 Delta_h W^from + frc[from] f
    WH_HIP(c, wh::launch_step(false, g, cur, prev_next, c->acc, c2p, f, c->frc[(size_t)from], 0.0, wh::ACCUMULATE,
                              nullptr, nullptr, s));
    return WH_OK;
  };

  // forward sweep: first step into checkpoint 0, then roll two levels and
  // copy the pairs at the checkpoints (the accumulator is scratch here)
  WH_HIP(c, wh::launch_first_step(false, half, v, cpA(0), cpB(0), c->acc, c2p, f, -0.5 * dt2, 0.0, 0.0, s));
  if (L.ncp > 1) {
    double *prev = static_cast<double *>(c->W[0]), *cur = static_cast<double *>(c->W[1]);
    WH_HIP(c, hipMemcpyAsync(prev, cpA(0), nb, hipMemcpyDeviceToDevice, s));
    WH_HIP(c, hipMemcpyAsync(cur, cpB(0), nb, hipMemcpyDeviceToDevice, s));
    const int64_t last = (int64_t)(L.ncp - 1) * L.seg + 1;
    for (int64_t m = 2; m <= last; ++m) {
      WH_TRY(step(cur, prev, m - 1));
      std::swap(prev, cur);  // cur = W^m
      if (m % L.seg == 0) WH_HIP(c, hipMemcpyAsync(cpA((int)(m / L.seg)), cur, nb, hipMemcpyDeviceToDevice, s));
      if (m % L.seg == 1 && m > L.seg)
        WH_HIP(c, hipMemcpyAsync(cpB((int)((m - 1) / L.seg)), cur, nb, hipMemcpyDeviceToDevice, s));
    }
  }

  // reverse sweep, one segment at a time from the last
  WH_HIP(c, wh::launch_fill(zc, 0.0, c->nodes, s));
  WH_HIP(c, wh::launch_fill(zp, 0.0, c->nodes, s));
  WH_HIP(c, wh::launch_fill(gf, 0.0, c->nodes, s));
  WH_HIP(c, wh::launch_fill(gc, 0.0, c->nodes, s));
  WH_HIP(c, wh::launch_scale_c2(g, c2p, lam, clam, false, s));
  std::vector<double *> lev((size_t)L.seg);
  for (int j = L.ncp - 1; j >= 0; --j) {
    const int64_t k = (int64_t)j * L.seg;
    const int64_t top = std::min<int64_t>(k + L.seg, L.N);
    lev[0] = cpA(j);
    if (top - k > 1) lev[1] = cpB(j);
    for (int64_t i = 2; i < top - k; ++i) {
      double *dst = buf(seg0 + (size_t)(i - 2));
      WH_HIP(c, hipMemcpyAsync(dst, lev[(size_t)i - 2], nb, hipMemcpyDeviceToDevice, s));
      WH_TRY(step(lev[(size_t)i - 1], dst, k + i - 1));
      lev[(size_t)i] = dst;
    }
    for (int64_t n = top; n > k; --n) {
      const bool first = n == 1;
      const double gam = first ? -0.5 * dt2 : c->frc[(size_t)(n - 1)];
      WH_HIP(c, wh::launch_adjoint_step(g, zc, zp, c2p, clam, c->wts[(size_t)n], lev[(size_t)(n - 1 - k)], gam,
                                        first ? 0.5 : 1.0, gf, gc, s));
      std::swap(zc, zp);  // zc = Zh^n, zp = Zh^{n+1}
    }
  }
  if (grad_v) WH_HIP(c, wh::launch_adjoint_first(half, zc, zp, c2p, clam, c->wts[0], grad_v, s));
  if (grad_c2) WH_HIP(c, wh::launch_scale_c2(g, c2p, gc, grad_c2, true, s));
  if (grad_f) WH_HIP(c, wh::launch_scale_c2(g, c2p, gf, grad_f, true, s));
  return WH_OK;
}

wh_status wh_solve_adjoint(wh_ctx *c, const wh_solve_opts *o, const double *g, double *lam, wh_solve_info *info) {
  WH_TRY(need(c, true, true, true, false, true));
  WH_TRY(need_fp64(c, "wh_solve_adjoint"));
  WH_TRY(check_opts(c, o));
  WH_TRY(set_device(c));
  WH_TRY(check_dev(c, g, "g"));
  WH_TRY(check_dev(c, lam, "lam"));
  if (g == lam) return fail(c, WH_EINVAL, "lam may not alias g");
  // (I - S)^T = C^{-1} (I - S) C, C = diag(c^2): solve (I - S) mu = C g,
  // starting from C lam, then lam = mu / c^2
  const wh::StepGeom g1 = geometry(c, 1.0);
  const double *c2p = c->c2_is_const ? nullptr : static_cast<const double *>(c->c2);
  WH_HIP(c, wh::launch_scale_c2(g1, c2p, g, c->b, false, c->stream));
  WH_HIP(c, wh::launch_scale_c2(g1, c2p, lam, lam, false, c->stream));
  const wh_status st = solve_dispatch(c, o, c->b, lam, info);
  WH_HIP(c, wh::launch_scale_c2(g1, c2p, lam, lam, true, c->stream));
  WH_HIP(c, hipStreamSynchronize(c->stream));
  return st;
}

wh_status wh_receiver_misfit(wh_ctx *c, const double *u, const int64_t *idx, const double *data, int32_t nrec,
                             double *J, double *grad) {
  WH_TRY(need(c, true, true, false, false, false));
  if (!J) return fail(c, WH_EINVAL, "J is NULL");
  if (nrec < 0) return fail(c, WH_EINVAL, "nrec must be >= 0");
  WH_TRY(set_device(c));
  WH_TRY(check_dev(c, u, "u"));
  if (nrec > 0) {
    WH_TRY(check_dev(c, idx, "idx"));
    WH_TRY(check_dev(c, data, "data"));
  }
  if (grad) {
    WH_TRY(check_dev(c, grad, "grad"));
    if (grad == u) return fail(c, WH_EINVAL, "grad may not alias u");
    WH_HIP(c, wh::launch_fill(grad, 0.0, c->nodes, c->stream));
  }
  double out[2] = {0.0, 0.0};
  if (nrec > 0) {
    WH_HIP(c, wh::launch_misfit(u, idx, data, nrec, c->nodes, grad, c->scal, c->stream));
    WH_TRY(fetch_scalars(c, 0, 2, out));
    if (out[1] > 0.0) return fail(c, WH_EINVAL, "%.0f receiver indices lie outside the grid", out[1]);
  }
  *J = out[0];
  return WH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches of independent 2-D problems
// ---------------------------------------------------------------------------
namespace {
constexpr int kBatchStride = 8;  // device scalars per table row
// scalar slots of a row: 0 <p,q>_w; 2,3 / 4,5 <r,r>_w, <r,r> of even / odd
// iterations
inline int cg_slot(int64_t k) { return 2 + 2 * (int)(k & 1); }
}  // namespace

struct wh_batch {
  int device = 0;
  hipStream_t stream = nullptr;  // caller's stream (apply)
  hipStream_t own = nullptr;     // private stream: solve, graph capture
  hipEvent_t ev = nullptr;
  std::string err;
  std::vector<wh_ctx *> probs;  // insertion order
  bool finalized = false;
  int prec = WH_FP64, order = 2, K = 0, rows = 0;  // 0 = default
  std::vector<int> coef_off;  // per problem
  std::vector<int> passes;    // per problem
  // tables of the current selection (host mirror)
  std::vector<int> ids;
  std::vector<wh::BatchDesc> desc;
  std::vector<wh::BatchFirst> first;
  std::vector<wh::BatchVec> vecs;
  std::vector<int> prefix, active_at;
  int maxpasses = 0, first_blocks = 0, red_blocks = 0;
  // device tables, carved from the bound workspace
  wh::BatchDesc *d_desc = nullptr;
  wh::BatchFirst *d_first = nullptr;
  wh::BlockCoef *d_coef = nullptr;
  int *d_prefix = nullptr;
  wh::BatchVec *d_vecs = nullptr, *d_vecs_e = nullptr;
  double *d_part = nullptr, *d_sc = nullptr;
  double *pinned = nullptr;  // WH_MAX_BATCH rows of scalars
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipGraph_t graph[2] = {nullptr, nullptr};
};

namespace {

wh_status bfail(wh_batch *b, wh_status st, const char *fmt, ...) {
  if (b) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    b->err = buf;
  }
  return st;
}

#define WH_BHIP(b, call)                                                                                 \
  do {                                                                                                   \
    hipError_t e_ = (call);                                                                              \
    if (e_ != hipSuccess) return bfail((b), WH_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

void batch_resolve_tuning(wh_batch *b) {
  const bool fp32 = b->prec == WH_FP32_STATE;
  if (b->K == 0) b->K = default_kblock(b->order, fp32);
  if (b->rows == 0) b->rows = wh::block_default_rows(fp32, b->order);
}

int batch_passes(const wh_ctx *c, int K) {
  const int64_t steps = (int64_t)c->tp.nt * c->tp.periods - 1;
  return (int)((steps + K - 1) / K);
}

struct BatchLayout {
  size_t desc, first, coef, prefix, vecs, vecs_e, part, sc, total;
};

BatchLayout batch_layout(size_t P, size_t ncoef, int red_blocks) {
  BatchLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  L.desc = take(P * sizeof(wh::BatchDesc));
  L.first = take(P * sizeof(wh::BatchFirst));
  L.coef = take(ncoef * sizeof(wh::BlockCoef));
  L.prefix = take((P + 1) * sizeof(int));
  L.vecs = take(P * sizeof(wh::BatchVec));
  L.vecs_e = take(P * sizeof(wh::BatchVec));
  L.part = take((size_t)2 * red_blocks * 8);
  L.sc = take(P * kBatchStride * 8);
  L.total = off;
  return L;
}

// Build and upload the tables of the problems `ids` (any order; stored by
// decreasing pass count).  The apply of problem i reads in[i] and writes
// out[i]; its Krylov vectors are x[i] (nullable) and the r, p, q columns of
// its workspace.  Row scalars are uploaded from `rowsc` (P x kBatchStride,
// by problem) when given.
wh_status batch_select(wh_batch *b, std::vector<int> ids, const double *const *in, double *const *out, bool forcing,
                       double *const *x, const double *rowsc, hipStream_t s) {
  const bool fp32 = b->prec == WH_FP32_STATE;
  std::stable_sort(ids.begin(), ids.end(), [&](int a, int c) { return b->passes[a] > b->passes[c]; });
  int ox, oy;
  wh::block_tile_shape(fp32, b->order, b->K, b->rows, &ox, &oy);
  const size_t n = ids.size();
  b->ids = ids;
  b->desc.assign(n, wh::BatchDesc{});
  b->first.assign(n, wh::BatchFirst{});
  b->vecs.assign(n, wh::BatchVec{});
  b->prefix.assign(n + 1, 0);
  b->first_blocks = 0;
  b->red_blocks = 0;
  for (size_t t = 0; t < n; ++t) {
    const int i = ids[t];
    wh_ctx *c = b->probs[(size_t)i];
    const double dt2 = c->tp.dt * c->tp.dt;
    const void *c2 = c->c2_is_const ? nullptr : c->c2;
    wh::BatchDesc &d = b->desc[t];
    d.g = geometry(c, dt2);
    d.c2 = c2;
    d.f = forcing ? c->f : nullptr;
    for (int q = 0; q < 4; ++q) d.W[q] = c->W[q];
    d.acc = c->acc;
    d.v = in[i];
    d.out = out[i];
    d.tiles_x = (int)((c->n[0] + 1 + ox - 1) / ox);
    d.tiles = d.tiles_x * (int)((c->n[1] + 1 + oy - 1) / oy);
    d.steps = (int)((int64_t)c->tp.nt * c->tp.periods - 1);
    d.passes = b->passes[(size_t)i];
    d.coef_offset = b->coef_off[(size_t)i];
    b->prefix[t + 1] = b->prefix[t] + d.tiles;
    wh::BatchFirst &f = b->first[t];
    f.half = geometry(c, 0.5 * dt2);
    f.v = in[i];
    f.W0 = c->W[0];
    f.W1 = c->W[1];
    f.acc = c->acc;
    f.c2 = c2;
    f.f = forcing ? c->f : nullptr;
    f.g0 = forcing ? -0.5 * dt2 : 0.0;
    f.w0 = c->wts[0];
    f.w1 = c->wts[1];
    f.block_offset = b->first_blocks;
    b->first_blocks += wh::batch_node_blocks(c->nodes);
    wh::BatchVec &v = b->vecs[t];
    v.x = x ? x[i] : nullptr;
    v.r = c->V;
    v.p = c->V + c->ldv;
    v.q = c->V + 2 * c->ldv;
    v.b = c->b;
    v.c2 = c2;
    v.n = c->nodes;
    v.block_offset = b->red_blocks;
    v.nblocks = wh::batch_red_blocks(c->nodes);
    v.active = 1;
    b->red_blocks += v.nblocks;
  }
  b->maxpasses = n ? b->desc[0].passes : 0;
  b->active_at.assign((size_t)b->maxpasses, 0);
  for (int j = 0; j < b->maxpasses; ++j)
    for (size_t t = 0; t < n; ++t)
      if (b->desc[t].passes > j) b->active_at[(size_t)j] = (int)t + 1;
  std::vector<wh::BatchVec> ve = b->vecs;
  for (auto &v : ve) v.c2 = nullptr;  // Euclidean products
  WH_BHIP(b, hipStreamSynchronize(s));  // host staging below is reused
  WH_BHIP(b, hipMemcpyAsync(b->d_desc, b->desc.data(), n * sizeof(wh::BatchDesc), hipMemcpyHostToDevice, s));
  WH_BHIP(b, hipMemcpyAsync(b->d_first, b->first.data(), n * sizeof(wh::BatchFirst), hipMemcpyHostToDevice, s));
  WH_BHIP(b, hipMemcpyAsync(b->d_prefix, b->prefix.data(), (n + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  WH_BHIP(b, hipMemcpyAsync(b->d_vecs, b->vecs.data(), n * sizeof(wh::BatchVec), hipMemcpyHostToDevice, s));
  WH_BHIP(b, hipMemcpyAsync(b->d_vecs_e, ve.data(), n * sizeof(wh::BatchVec), hipMemcpyHostToDevice, s));
  if (rowsc) {
    for (size_t t = 0; t < n; ++t)
      std::memcpy(b->pinned + t * kBatchStride, rowsc + (size_t)ids[t] * kBatchStride, kBatchStride * 8);
    WH_BHIP(b, hipMemcpyAsync(b->d_sc, b->pinned, n * kBatchStride * 8, hipMemcpyHostToDevice, s));
  }
  WH_BHIP(b, hipStreamSynchronize(s));
  return WH_OK;
}

// Launches of one batched application over the selected problems.
wh_status batch_enqueue_apply(wh_batch *b, bool forcing, int final_mode, hipStream_t s) {
  const bool fp32 = b->prec == WH_FP32_STATE;
  const int n = (int)b->ids.size();
  if (n == 0) return WH_OK;
  WH_BHIP(b, wh::launch_batch_first_step(fp32, b->order, b->d_first, n, b->first_blocks, s));
  for (int j = 0; j < b->maxpasses; ++j) {
    const int na = b->active_at[(size_t)j];
    WH_BHIP(b, wh::launch_batch_block_steps(fp32, b->order, b->K, b->rows, forcing, b->d_desc, b->d_prefix, na,
                                            b->prefix[(size_t)na], j, b->d_coef, final_mode, s));
  }
  return WH_OK;
}

// Copy the selected rows' scalars to rowsc (by problem).
wh_status batch_fetch(wh_batch *b, double *rowsc, hipStream_t s) {
  const size_t n = b->ids.size();
  WH_BHIP(b, hipMemcpyAsync(b->pinned, b->d_sc, n * kBatchStride * 8, hipMemcpyDeviceToHost, s));
  WH_BHIP(b, hipStreamSynchronize(s));
  for (size_t t = 0; t < n; ++t)
    std::memcpy(rowsc + (size_t)b->ids[t] * kBatchStride, b->pinned + t * kBatchStride, kBatchStride * 8);
  return WH_OK;
}

void batch_drop_graphs(wh_batch *b) {
  for (int i = 0; i < 2; ++i) {
    if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
    if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
    b->exec[i] = nullptr;
    b->graph[i] = nullptr;
  }
}

// Capture one CG iteration over the selected problems for each slot parity:
// q = A p, <p,q>_w, x += a p, r -= a q (with the new <r,r>_w, <r,r>), and
// p = r + beta p.
wh_status batch_capture(wh_batch *b) {
  batch_drop_graphs(b);
  const bool fp32 = b->prec == WH_FP32_STATE;
  const int n = (int)b->ids.size();
  for (int par = 0; par < 2; ++par) {
    const int cur = cg_slot(par), nxt = cg_slot(par + 1);
    WH_BHIP(b, hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal));
    wh_status st = batch_enqueue_apply(b, false, wh::FINAL_A, b->own);
    if (st == WH_OK) {
      hipError_t e = wh::launch_batch_dot(fp32, b->d_vecs, n, b->red_blocks, 0, b->d_part, b->d_sc, kBatchStride,
                                          b->own);
      if (e == hipSuccess)
        e = wh::launch_batch_cg_update(fp32, b->d_vecs, n, b->red_blocks, b->d_sc + cur, b->d_sc, kBatchStride,
                                       b->d_part, b->d_sc + nxt, b->own);
      if (e == hipSuccess)
        e = wh::launch_batch_xpay(b->d_vecs, n, b->red_blocks, b->d_sc + nxt, b->d_sc + cur, kBatchStride, b->own);
      if (e != hipSuccess) st = bfail(b, WH_EDEVICE, "batched CG launch failed: %s", hipGetErrorString(e));
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->own, &g);
    if (st != WH_OK || ec != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      if (st != WH_OK) return st;
      return bfail(b, WH_EDEVICE, "graph capture failed: %s", hipGetErrorString(ec));
    }
    b->graph[par] = g;
    WH_BHIP(b, hipGraphInstantiate(&b->exec[par], g, nullptr, nullptr, 0));
  }
  return WH_OK;
}

// Steps per launch and tile rows: pass counts and the per (problem, pass)
// step coefficients (steps 1 + j K + q and the weights of the levels they
// produce), uploaded to the coefficient table.
wh_status batch_set_k(wh_batch *b, int K, int rows) {
  const size_t P = b->probs.size();
  std::vector<wh::BlockCoef> coefs;
  b->coef_off.assign(P, 0);
  b->passes.assign(P, 0);
  for (size_t i = 0; i < P; ++i) {
    wh_ctx *c = b->probs[i];
    b->passes[i] = batch_passes(c, K);
    b->coef_off[i] = (int)coefs.size();
    for (int j = 0; j < b->passes[i]; ++j) {
      wh::BlockCoef cf{};
      for (int q = 0; q < K; ++q) {
        const int64_t n = 1 + (int64_t)j * K + q;
        if (n + 1 >= (int64_t)c->wts.size()) break;
        cf.gn[q] = c->frc[(size_t)n];
        cf.wn[q] = c->wts[(size_t)n + 1];
      }
      coefs.push_back(cf);
    }
  }
  b->K = K;
  b->rows = rows;
  WH_BHIP(b, hipStreamSynchronize(b->own));
  WH_BHIP(b, hipMemcpyAsync(b->d_coef, coefs.data(), coefs.size() * sizeof(wh::BlockCoef), hipMemcpyHostToDevice,
                            b->own));
  WH_BHIP(b, hipStreamSynchronize(b->own));
  return WH_OK;
}

wh_status batch_need(wh_batch *b) {
  if (!b) return WH_EINVAL;
  if (!b->finalized) return bfail(b, WH_ESTATE, "batch not finalized (call wh_batch_finalize)");
  return WH_OK;
}

}  // namespace

extern "C" {

wh_status wh_batch_create(wh_batch **out, int32_t device, void *stream) {
  if (!out) return WH_EINVAL;
  *out = nullptr;
  wh_batch *b = new (std::nothrow) wh_batch();
  if (!b) return WH_ENOMEM;
  b->device = device;
  b->stream = static_cast<hipStream_t>(stream);
  if (hipSetDevice(device) != hipSuccess ||
      hipHostMalloc((void **)&b->pinned, (size_t)WH_MAX_BATCH * kBatchStride * 8, hipHostMallocDefault) != hipSuccess ||
      hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    if (b->ev) (void)hipEventDestroy(b->ev);
    if (b->own) (void)hipStreamDestroy(b->own);
    if (b->pinned) (void)hipHostFree(b->pinned);
    delete b;
    return WH_EDEVICE;
  }
  *out = b;
  return WH_OK;
}

void wh_batch_destroy(wh_batch *b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->own);
  batch_drop_graphs(b);
  (void)hipEventDestroy(b->ev);
  (void)hipStreamDestroy(b->own);
  (void)hipHostFree(b->pinned);
  delete b;
}

const char *wh_batch_last_error(const wh_batch *b) { return b ? b->err.c_str() : "no batch"; }

wh_status wh_batch_add(wh_batch *b, wh_ctx *c, int32_t *index) {
  if (!b || !c) return WH_EINVAL;
  if (b->finalized) return bfail(b, WH_ESTATE, "batch already finalized");
  if ((int)b->probs.size() >= WH_MAX_BATCH) return bfail(b, WH_EINVAL, "at most %d problems per batch", WH_MAX_BATCH);
  if (!c->grid_set || !c->ws || !c->c2_set || !c->f_set || !c->freq_set)
    return bfail(b, WH_ESTATE, "problem must have grid, workspace, c^2, source and frequency set");
  if (c->implicit) return bfail(b, WH_EINVAL, "the batched solve uses explicit time stepping");
  if (c->dim != 2) return bfail(b, WH_EINVAL, "batches hold 2-D problems");
  if (c->defl_count > 0) return bfail(b, WH_EINVAL, "problems with deflation set cannot be batched");
  if (c->ws_restart < 2) return bfail(b, WH_ENOMEM, "problem workspace must be sized for restart >= 2");
  if (c->device != b->device) return bfail(b, WH_EINVAL, "problem on another device");
  for (wh_ctx *o : b->probs)
    if (o == c) return bfail(b, WH_EINVAL, "problem added twice");
  if (!b->probs.empty() && (c->order != b->order || c->prec != b->prec))
    return bfail(b, WH_EINVAL, "all problems of a batch share order and precision");
  b->order = c->order;
  b->prec = c->prec;
  b->probs.push_back(c);
  if (index) *index = (int32_t)b->probs.size() - 1;
  return WH_OK;
}

wh_status wh_batch_set_tuning(wh_batch *b, int32_t kblock, int32_t tile) {
  if (!b) return WH_EINVAL;
  if (b->finalized) return bfail(b, WH_ESTATE, "batch already finalized");
  if (b->probs.empty()) return bfail(b, WH_ESTATE, "add problems first");
  const bool fp32 = b->prec == WH_FP32_STATE;
  const int K = kblock == 0 ? default_kblock(b->order, fp32) : kblock;
  const int rows = tile == 0 ? wh::block_default_rows(fp32, b->order) : tile;
  if (K < 2 || !wh::block_config_supported(fp32, b->order, K, rows) || rows > 8 * wh::block_rows_per_lane(fp32, b->order))
    return bfail(b, WH_EINVAL, "kblock %d / tile %d not supported for batches", kblock, tile);
  b->K = K;
  b->rows = rows;
  return WH_OK;
}

wh_status wh_batch_workspace_size(wh_batch *b, size_t *bytes) {
  if (!b || !bytes) return WH_EINVAL;
  if (b->probs.empty()) return bfail(b, WH_ESTATE, "add problems first");
  batch_resolve_tuning(b);
  size_t ncoef = 0;
  int red = 0;
  for (wh_ctx *c : b->probs) {
    ncoef += (size_t)batch_passes(c, 2);  // room for any steps-per-launch choice
    red += wh::batch_red_blocks(c->nodes);
  }
  *bytes = batch_layout(b->probs.size(), ncoef, red).total;
  return WH_OK;
}

wh_status wh_batch_finalize(wh_batch *b, void *workspace, size_t bytes) {
  if (!b) return WH_EINVAL;
  if (b->finalized) return bfail(b, WH_ESTATE, "batch already finalized");
  size_t need_bytes = 0;
  WH_TRY(wh_batch_workspace_size(b, &need_bytes));
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return bfail(b, WH_EINVAL, "workspace must be a 256-byte aligned device pointer");
  if (bytes < need_bytes) return bfail(b, WH_ENOMEM, "batch workspace too small: %zu given, %zu needed", bytes, need_bytes);
  WH_BHIP(b, hipSetDevice(b->device));
  if (!is_device_ptr(workspace)) return bfail(b, WH_EINVAL, "workspace is not device memory");
  const size_t P = b->probs.size();
  size_t ncoef = 0;
  int red = 0;
  for (wh_ctx *c : b->probs) {
    ncoef += (size_t)batch_passes(c, 2);
    red += wh::batch_red_blocks(c->nodes);
  }
  const BatchLayout L = batch_layout(P, ncoef, red);
  char *base = static_cast<char *>(workspace);
  b->d_desc = reinterpret_cast<wh::BatchDesc *>(base + L.desc);
  b->d_first = reinterpret_cast<wh::BatchFirst *>(base + L.first);
  b->d_coef = reinterpret_cast<wh::BlockCoef *>(base + L.coef);
  b->d_prefix = reinterpret_cast<int *>(base + L.prefix);
  b->d_vecs = reinterpret_cast<wh::BatchVec *>(base + L.vecs);
  b->d_vecs_e = reinterpret_cast<wh::BatchVec *>(base + L.vecs_e);
  b->d_part = reinterpret_cast<double *>(base + L.part);
  b->d_sc = reinterpret_cast<double *>(base + L.sc);
  WH_TRY(batch_set_k(b, b->K, b->rows));
  b->finalized = true;
  return WH_OK;
}

wh_status wh_batch_apply(wh_batch *b, const double *const *v, double *const *out, int32_t with_forcing) {
  WH_TRY(batch_need(b));
  if (!v || !out) return bfail(b, WH_EINVAL, "pointer arrays are NULL");
  const size_t P = b->probs.size();
  for (size_t i = 0; i < P; ++i)
    if (!v[i] || !out[i] || !is_device_ptr(v[i]) || !is_device_ptr(out[i]) || v[i] == out[i])
      return bfail(b, WH_EINVAL, "problem %zu: input and output must be distinct device arrays", i);
  WH_BHIP(b, hipSetDevice(b->device));
  std::vector<int> all(P);
  for (size_t i = 0; i < P; ++i) all[i] = (int)i;
  WH_TRY(batch_select(b, all, v, out, with_forcing != 0, nullptr, nullptr, b->stream));
  return batch_enqueue_apply(b, with_forcing != 0, wh::FINAL_FILTER, b->stream);
}

// The batched CG; rhs (nullable) gives every problem's right-hand side
// (device FP64 node arrays) instead of b_i = W_h(0, f_i).
static wh_status batch_solve_core(wh_batch *b, const wh_solve_opts *o, double *const *x, wh_solve_info *info,
                                  const double *const *rhs) {
  WH_TRY(batch_need(b));
  if (!o || !x) return bfail(b, WH_EINVAL, "opts or x is NULL");
  if (o->method != WH_SOLVER_CG) return bfail(b, WH_EINVAL, "batches are solved with WH_SOLVER_CG");
  if (o->flags != 0) return bfail(b, WH_EINVAL, "opts.flags must be 0");
  if (o->maxit < 1 || !(o->rtol > 0.0) || !std::isfinite(o->rtol))
    return bfail(b, WH_EINVAL, "maxit must be >= 1 and rtol finite and > 0");
  WH_BHIP(b, hipSetDevice(b->device));
  const size_t P = b->probs.size();
  for (size_t i = 0; i < P; ++i) {
    if (!x[i] || !is_device_ptr(x[i])) return bfail(b, WH_EINVAL, "x[%zu] is not device memory", i);
    if (rhs && (!rhs[i] || !is_device_ptr(rhs[i]))) return bfail(b, WH_EINVAL, "b[%zu] is not device memory", i);
    if (rhs && rhs[i] == x[i]) return bfail(b, WH_EINVAL, "b[%zu] may not alias x[%zu]", i, i);
  }
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = b->own;
  // order after the caller's stream and the problems' own uploads
  for (wh_ctx *c : b->probs) WH_BHIP(b, hipStreamSynchronize(c->stream));
  WH_BHIP(b, hipEventRecord(b->ev, b->stream));
  WH_BHIP(b, hipStreamWaitEvent(s, b->ev, 0));

  std::vector<const double *> zero(P), xin(P), pin(P);
  std::vector<double *> bout(P), qout(P);
  for (size_t i = 0; i < P; ++i) {
    wh_ctx *c = b->probs[i];
    WH_BHIP(b, wh::launch_fill(c->tmp, 0.0, c->nodes, s));
    zero[i] = c->tmp;
    bout[i] = c->b;
    xin[i] = x[i];
    pin[i] = c->V + c->ldv;
    qout[i] = c->V + 2 * c->ldv;
  }
  std::vector<double> sc(P * kBatchStride, 0.0), bnorm(P, 0.0), rel(P, 1.0);
  std::vector<int> iters(P, 0), applies(P, 0);
  std::vector<char> done(P, 0);
  std::vector<int> all(P);
  for (size_t i = 0; i < P; ++i) all[i] = (int)i;
  const bool fp32 = b->prec == WH_FP32_STATE;

  // b_i = W_h(0, f_i) (or the given right-hand side) and ||b_i||: r = b - 0,
  // then <r,r>
  if (rhs) {
    WH_TRY(batch_select(b, all, zero.data(), bout.data(), false, x, nullptr, s));
    for (size_t i = 0; i < P; ++i)
      WH_BHIP(b, hipMemcpyAsync(bout[i], rhs[i], (size_t)b->probs[i]->nodes * 8, hipMemcpyDeviceToDevice, s));
  } else {
    WH_TRY(batch_select(b, all, zero.data(), bout.data(), true, x, nullptr, s));
    WH_TRY(batch_enqueue_apply(b, true, wh::FINAL_FILTER, s));
    for (auto &a : applies) ++a;
  }
  {
    // Euclidean table with q = 0
    std::vector<wh::BatchVec> ve = b->vecs;
    for (size_t t = 0; t < P; ++t) {
      ve[t].c2 = nullptr;
      ve[t].q = b->probs[(size_t)b->ids[t]]->tmp;
    }
    WH_BHIP(b, hipMemcpyAsync(b->d_vecs_e, ve.data(), P * sizeof(wh::BatchVec), hipMemcpyHostToDevice, s));
    WH_BHIP(b, wh::launch_batch_residual(b->d_vecs_e, (int)P, b->red_blocks, s));
    WH_BHIP(b, wh::launch_batch_dot(false, b->d_vecs_e, (int)P, b->red_blocks, 1, b->d_part, b->d_sc + 1,
                                    kBatchStride, s));
    WH_TRY(batch_fetch(b, sc.data(), s));  // synchronises: ve may go
  }
  for (size_t i = 0; i < P; ++i) {
    bnorm[i] = std::sqrt(sc[i * kBatchStride + 1]);
    if (!std::isfinite(bnorm[i])) return bfail(b, WH_ENONFINITE, "problem %zu: ||b|| is not finite", i);
  }

  // r = b - A x, p = r and the slot(k) scalars, for the problems `ids`
  auto restart = [&](const std::vector<int> &ids, int64_t k) -> wh_status {
    WH_TRY(batch_select(b, ids, xin.data(), qout.data(), false, x, nullptr, s));
    WH_TRY(batch_enqueue_apply(b, false, wh::FINAL_A, s));
    const int n = (int)ids.size();
    WH_BHIP(b, wh::launch_batch_residual(b->d_vecs, n, b->red_blocks, s));
    WH_BHIP(b, wh::launch_batch_dot(fp32, b->d_vecs, n, b->red_blocks, 1, b->d_part, b->d_sc + cg_slot(k),
                                    kBatchStride, s));
    WH_BHIP(b, wh::launch_batch_dot(false, b->d_vecs_e, n, b->red_blocks, 1, b->d_part, b->d_sc + cg_slot(k) + 1,
                                    kBatchStride, s));
    WH_TRY(batch_fetch(b, sc.data(), s));
    for (int i : ids) {
      ++applies[(size_t)i];
      const double ee = sc[(size_t)i * kBatchStride + cg_slot(k) + 1];
      rel[(size_t)i] = bnorm[(size_t)i] > 0.0 ? std::sqrt(ee) / bnorm[(size_t)i] : 0.0;
    }
    return WH_OK;
  };

  wh_status st = WH_OK;
  int64_t k = 0;
  WH_TRY(restart(all, k));
  std::vector<int> active;
  for (int i : all)
    if (bnorm[(size_t)i] > 0.0 && rel[(size_t)i] > o->rtol) active.push_back(i);
    else done[(size_t)i] = 1;
  bool reselect = true;
  while (!active.empty() && k < o->maxit) {
    if (reselect) {
      WH_TRY(batch_select(b, active, pin.data(), qout.data(), false, x, sc.data(), s));
      WH_TRY(batch_capture(b));
      reselect = false;
    }
    WH_BHIP(b, hipGraphLaunch(b->exec[k & 1], s));
    ++k;
    WH_TRY(batch_fetch(b, sc.data(), s));
    std::vector<int> hit, keep;
    for (int i : active) {
      const double *row = sc.data() + (size_t)i * kBatchStride;
      ++applies[(size_t)i];
      iters[(size_t)i] = (int)k;
      const double pq = row[0], ee = row[cg_slot(k) + 1];
      if (!std::isfinite(pq) || !std::isfinite(ee)) {
        st = bfail(b, WH_ENONFINITE, "problem %d became non-finite at iteration %lld", i, (long long)k);
        break;
      }
      if (!(pq > 0.0)) {
        st = bfail(b, WH_ENOTCONV, "problem %d: CG breakdown, <p, A p> = %g at iteration %lld", i, pq, (long long)k);
        break;
      }
      rel[(size_t)i] = std::sqrt(ee) / bnorm[(size_t)i];
      (rel[(size_t)i] <= o->rtol ? hit : keep).push_back(i);
    }
    if (st != WH_OK) break;
    if (o->on_iter) {
      double worst = 0.0;
      for (int i : active) worst = std::max(worst, rel[(size_t)i]);
      o->on_iter((int32_t)k, worst, o->user);
    }
    if (!hit.empty()) {
      // confirm with the true residual; problems that drifted continue from it
      WH_TRY(restart(hit, k));
      for (int i : hit)
        if (rel[(size_t)i] <= o->rtol) done[(size_t)i] = 1;
        else keep.push_back(i);
      active = keep;
      reselect = true;
    }
  }
  // problems stopped by maxit report their true residual
  if (st == WH_OK && !active.empty()) WH_TRY(restart(active, k));
  WH_BHIP(b, hipStreamSynchronize(s));
  batch_drop_graphs(b);
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int unconverged = 0;
  for (size_t i = 0; i < P; ++i) {
    unconverged += rel[i] > o->rtol;
    if (!info) continue;
    wh_ctx *c = b->probs[i];
    wh_solve_info &in = info[i];
    std::memset(&in, 0, sizeof in);
    in.iters = iters[i];
    in.applies = applies[i];
    in.rel_res = rel[i];
    in.bnorm = bnorm[i];
    in.scaled_res = rel[i] * bnorm[i] / std::sqrt((double)c->nodes);
    in.cr_last = in.cr_avg = in.ecr = NAN;
    in.mu_pred = NAN;
    in.rel_res_recursive = in.ritz_min = in.ritz_max = NAN;
    in.seconds = secs;
    in.point_steps = applies[i] * point_steps_per_apply(c);
  }
  if (st == WH_OK && unconverged)
    st = bfail(b, WH_ENOTCONV, "%d problems did not reach rtol within maxit = %d", unconverged, o->maxit);
  return st;
}

wh_status wh_batch_solve(wh_batch *b, const wh_solve_opts *o, double *const *x, wh_solve_info *info) {
  return batch_solve_core(b, o, x, info, nullptr);
}

wh_status wh_batch_solve_rhs(wh_batch *b, const wh_solve_opts *o, const double *const *rhs, double *const *x,
                             wh_solve_info *info) {
  if (b && !rhs) return bfail(b, WH_EINVAL, "b is NULL");
  return batch_solve_core(b, o, x, info, rhs);
}

// Residual correction over two batches of the same problems: FP64 residuals
// r_i = b_i - A x_i on `hi`, corrections A d_i = r_i by the batched CG on the
// FP32-state batch `lo` (converged problems get d_i = 0), x_i += d_i.
wh_status wh_batch_solve_mixed(wh_batch *hi, wh_batch *lo, const wh_solve_opts *outer, const wh_solve_opts *inner,
                               double *const *x, wh_solve_info *info) {
  WH_TRY(batch_need(hi));
  if (!lo) return bfail(hi, WH_EINVAL, "lo is NULL");
  if (!lo->finalized) return bfail(hi, WH_ESTATE, "the FP32-state batch is not finalized");
  if (!outer || !inner || !x) return bfail(hi, WH_EINVAL, "opts or x is NULL");
  if (outer->maxit < 1 || !(outer->rtol > 0.0) || !std::isfinite(outer->rtol))
    return bfail(hi, WH_EINVAL, "outer maxit must be >= 1 and outer rtol finite and > 0");
  if (hi->prec != WH_FP64 || lo->prec != WH_FP32_STATE)
    return bfail(hi, WH_EINVAL, "hi must hold WH_FP64 contexts and lo WH_FP32_STATE contexts");
  if (hi->device != lo->device) return bfail(hi, WH_EINVAL, "the batches are on different devices");
  const size_t P = hi->probs.size();
  if (lo->probs.size() != P) return bfail(hi, WH_EINVAL, "the batches hold different numbers of problems");
  for (size_t i = 0; i < P; ++i) {
    const wh_ctx *a = hi->probs[i], *c = lo->probs[i];
    if (a->dim != c->dim || a->order != c->order || a->n[0] != c->n[0] || a->n[1] != c->n[1] ||
        a->tp.nt != c->tp.nt || a->tp.periods != c->tp.periods || a->tp.dt != c->tp.dt || a->tp.alpha != c->tp.alpha)
      return bfail(hi, WH_EINVAL, "problem %zu: the two contexts differ in grid, order or time parameters", i);
    if (!x[i] || !is_device_ptr(x[i])) return bfail(hi, WH_EINVAL, "x[%zu] is not device memory", i);
  }
  WH_BHIP(hi, hipSetDevice(hi->device));
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = hi->own;
  for (wh_ctx *c : hi->probs) WH_BHIP(hi, hipStreamSynchronize(c->stream));
  for (wh_ctx *c : lo->probs) WH_BHIP(hi, hipStreamSynchronize(c->stream));
  WH_BHIP(hi, hipEventRecord(hi->ev, hi->stream));
  WH_BHIP(hi, hipStreamWaitEvent(s, hi->ev, 0));

  std::vector<const double *> zero(P), xin(P), rhs(P);
  std::vector<double *> bout(P), qout(P), d(P);
  for (size_t i = 0; i < P; ++i) {
    wh_ctx *c = hi->probs[i];
    WH_BHIP(hi, wh::launch_fill(c->tmp, 0.0, c->nodes, s));
    zero[i] = c->tmp;
    bout[i] = c->b;
    xin[i] = x[i];
    qout[i] = c->V + 2 * c->ldv;
    d[i] = c->tmp;                            // the correction
    rhs[i] = c->V;                            // r_i of the last residual
  }
  std::vector<double> sc(P * kBatchStride, 0.0), bnorm(P, 0.0), rel(P, 1.0);
  std::vector<int> corr(P, 0), applies(P, 0);
  std::vector<int> all(P);
  for (size_t i = 0; i < P; ++i) all[i] = (int)i;

  // b_i = W_h(0, f_i) in FP64 and ||b_i||
  WH_TRY(batch_select(hi, all, zero.data(), bout.data(), true, x, nullptr, s));
  WH_TRY(batch_enqueue_apply(hi, true, wh::FINAL_FILTER, s));
  for (auto &a : applies) ++a;
  {
    std::vector<wh::BatchVec> ve = hi->vecs;
    for (size_t t = 0; t < P; ++t) {
      ve[t].c2 = nullptr;
      ve[t].q = hi->probs[(size_t)hi->ids[t]]->tmp;
    }
    WH_BHIP(hi, hipMemcpyAsync(hi->d_vecs_e, ve.data(), P * sizeof(wh::BatchVec), hipMemcpyHostToDevice, s));
    WH_BHIP(hi, wh::launch_batch_residual(hi->d_vecs_e, (int)P, hi->red_blocks, s));
    WH_BHIP(hi, wh::launch_batch_dot(false, hi->d_vecs_e, (int)P, hi->red_blocks, 1, hi->d_part, hi->d_sc + 1,
                                     kBatchStride, s));
    WH_TRY(batch_fetch(hi, sc.data(), s));
  }
  for (size_t i = 0; i < P; ++i) {
    bnorm[i] = std::sqrt(sc[i * kBatchStride + 1]);
    if (!std::isfinite(bnorm[i])) return bfail(hi, WH_ENONFINITE, "problem %zu: ||b|| is not finite", i);
  }
  wh_status st = WH_OK;
  std::vector<wh_solve_info> in(P);
  for (int k = 0;; ++k) {
    // FP64 residual r_i = b_i - A x_i (into the r vector of hi's problems)
    WH_TRY(batch_select(hi, all, xin.data(), qout.data(), false, x, nullptr, s));
    WH_TRY(batch_enqueue_apply(hi, false, wh::FINAL_A, s));
    WH_BHIP(hi, wh::launch_batch_residual(hi->d_vecs, (int)P, hi->red_blocks, s));
    WH_BHIP(hi, wh::launch_batch_dot(false, hi->d_vecs_e, (int)P, hi->red_blocks, 1, hi->d_part, hi->d_sc + 1,
                                     kBatchStride, s));
    WH_TRY(batch_fetch(hi, sc.data(), s));
    bool all_done = true;
    double worst = 0.0;
    for (size_t i = 0; i < P; ++i) {
      ++applies[i];
      rel[i] = bnorm[i] > 0.0 ? std::sqrt(sc[i * kBatchStride + 1]) / bnorm[i] : 0.0;
      if (!std::isfinite(rel[i])) return bfail(hi, WH_ENONFINITE, "problem %zu: residual is not finite", i);
      all_done = all_done && rel[i] <= outer->rtol;
      worst = std::max(worst, rel[i]);
    }
    if (outer->on_iter) outer->on_iter(k, worst, outer->user);
    if (all_done || k >= outer->maxit) break;
    // corrections: problems already converged get a zero right-hand side
    for (size_t i = 0; i < P; ++i) {
      WH_BHIP(hi, wh::launch_fill(d[i], 0.0, hi->probs[i]->nodes, s));
      if (rel[i] <= outer->rtol) WH_BHIP(hi, wh::launch_fill(hi->probs[i]->V, 0.0, hi->probs[i]->nodes, s));
    }
    WH_BHIP(hi, hipStreamSynchronize(s));
    const wh_status sl = batch_solve_core(lo, inner, d.data(), in.data(), rhs.data());
    if (sl != WH_OK && sl != WH_ENOTCONV) {
      st = bfail(hi, sl, "inner batched solve failed: %s", lo->err.c_str());
      break;
    }
    for (size_t i = 0; i < P; ++i) {
      applies[i] += in[i].applies;
      if (rel[i] > outer->rtol) ++corr[i];
      WH_BHIP(hi, wh::launch_add(x[i], d[i], x[i], hi->probs[i]->nodes, s));
    }
  }
  WH_BHIP(hi, hipStreamSynchronize(s));
  batch_drop_graphs(hi);
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int unconverged = 0;
  for (size_t i = 0; i < P; ++i) {
    unconverged += rel[i] > outer->rtol;
    if (!info) continue;
    wh_ctx *c = hi->probs[i];
    wh_solve_info &o = info[i];
    std::memset(&o, 0, sizeof o);
    o.iters = corr[i];
    o.applies = applies[i];
    o.rel_res = rel[i];
    o.bnorm = bnorm[i];
    o.scaled_res = rel[i] * bnorm[i] / std::sqrt((double)c->nodes);
    o.cr_last = o.cr_avg = o.ecr = o.mu_pred = NAN;
    o.rel_res_recursive = o.ritz_min = o.ritz_max = NAN;
    o.seconds = secs;
    o.point_steps = applies[i] * point_steps_per_apply(c);
  }
  if (st == WH_OK && unconverged)
    st = bfail(hi, WH_ENOTCONV, "%d problems did not reach rtol within %d corrections", unconverged, outer->maxit);
  return st;
}

wh_status wh_batch_autotune(wh_batch *b, int32_t applies, int32_t *kblock, int32_t *tile, double *ms_per_apply) {
  WH_TRY(batch_need(b));
  if (applies < 1) return bfail(b, WH_EINVAL, "applies must be >= 1");
  WH_BHIP(b, hipSetDevice(b->device));
  const bool fp32 = b->prec == WH_FP32_STATE;
  const size_t P = b->probs.size();
  std::vector<const double *> in(P);
  std::vector<double *> out(P);
  for (size_t i = 0; i < P; ++i) {
    wh_ctx *c = b->probs[i];
    WH_BHIP(b, hipStreamSynchronize(c->stream));
    WH_BHIP(b, wh::launch_fill(c->tmp, 0.0, c->nodes, b->own));
    in[i] = c->tmp;
    out[i] = c->V + 2 * c->ldv;
  }
  std::vector<int> all(P);
  for (size_t i = 0; i < P; ++i) all[i] = (int)i;
  const int rpl = wh::block_rows_per_lane(fp32, b->order);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  WH_BHIP(b, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return bfail(b, WH_EDEVICE, "hipEventCreate failed");
  }
  int bestK = b->K, bestR = b->rows;
  double best = INFINITY;
  wh_status st = WH_OK;
  for (int K = 2; K <= wh::kMaxBlockSteps && st == WH_OK; ++K) {
    for (int r = 0; r < 2 && st == WH_OK; ++r) {
      const int rows = (r == 0 ? 4 : 8) * rpl;
      if (!wh::block_config_supported(fp32, b->order, K, rows)) continue;
      st = batch_set_k(b, K, rows);
      if (st == WH_OK) st = batch_select(b, all, in.data(), out.data(), false, nullptr, nullptr, b->own);
      if (st == WH_OK) st = batch_enqueue_apply(b, false, wh::FINAL_A, b->own);  // warm-up
      if (st != WH_OK) break;
      if (hipEventRecord(e0, b->own) != hipSuccess) st = bfail(b, WH_EDEVICE, "hipEventRecord failed");
      for (int a = 0; a < applies && st == WH_OK; ++a) st = batch_enqueue_apply(b, false, wh::FINAL_A, b->own);
      float ms = 0.0f;
      if (st == WH_OK && (hipEventRecord(e1, b->own) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = bfail(b, WH_EDEVICE, "event timing failed");
      if (st == WH_OK && ms / applies < best) {
        best = ms / applies;
        bestK = K;
        bestR = rows;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  WH_TRY(st);
  WH_TRY(batch_set_k(b, bestK, bestR));
  if (kblock) *kblock = bestK;
  if (tile) *tile = bestR;
  if (ms_per_apply) *ms_per_apply = best;
  return WH_OK;
}

wh_status wh_batch_get_tuning(const wh_batch *b, int32_t *kblock, int32_t *tile) {
  if (!b) return WH_EINVAL;
  if (kblock) *kblock = b->K;
  if (tile) *tile = b->rows;
  return WH_OK;
}

}  // extern "C"
