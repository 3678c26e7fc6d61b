// Configuration queries and routing of the blocked-kernel launches to the
// per-(precision, order) translation units (wh_block_<prec>_p<order>.hip).
#include <hip/hip_runtime.h>

#include "wh_block3d_impl.h"
#include "wh_block_impl.h"

namespace wh {

bool block_config_supported(bool fp32, int order, int K, int rows) {
  if (!(order == 2 || order == 4) || !k_instantiated(order, K)) return false;
  const int rs = block_rows_per_lane(fp32, order);
  if (rows % rs != 0) return false;
  const int nw = rows / rs;
  if (nw != 4 && nw != 8 && !(nw == 10 && !fp32)) return false;
  return rows - 2 * K * (order / 2) > 0 && 64 - 2 * K * (order / 2) > 0;
}

int block_rows_per_lane(bool fp32, int order) {
  if (fp32) return order == 2 ? RowsPerLane<float, 2>::RS : RowsPerLane<float, 4>::RS;
  return order == 2 ? RowsPerLane<double, 2>::RS : RowsPerLane<double, 4>::RS;
}

int block_default_rows(bool fp32, int order) { return (fp32 ? 4 : 8) * block_rows_per_lane(fp32, order); }

void block_tile_shape(bool fp32, int order, int K, int rows, int *owned_x, int *owned_y) {
  const int H = K * (order / 2);
  *owned_x = 64 - 2 * H;
  *owned_y = rows - 2 * H;
}

hipError_t launch_block_steps_2d(bool fp32, const StepGeom &g, int K, int rows, int ksteps, const void *in_prev,
                                 const void *in_cur, void *out_prev, void *out_cur, double *acc, const void *c2,
                                 const void *f, const BlockCoef &coef, int mode, const double *v, double *out,
                                 hipStream_t s) {
  if (ksteps < 1 || ksteps > K || !block_config_supported(fp32, g.order, K, rows)) return hipErrorInvalidValue;
  const int nw = rows / block_rows_per_lane(fp32, g.order);
  const BlockDispatch fn = fp32 ? (g.order == 2 ? block_dispatch_f32_p2 : block_dispatch_f32_p4)
                                 : (g.order == 2 ? block_dispatch_f64_p2 : block_dispatch_f64_p4);
  return fn(g, K, nw, ksteps, in_prev, in_cur, out_prev, out_cur, acc, c2, f, coef, mode, v, out, s);
}

hipError_t launch_batch_block_steps(bool fp32, int order, int K, int rows, bool force, const BatchDesc *descs,
                                    const int *tile_prefix, int nactive, int total_tiles, int pass,
                                    const BlockCoef *coefs, int final_mode, hipStream_t s) {
  if (total_tiles <= 0) return hipSuccess;
  if (!block_config_supported(fp32, order, K, rows)) return hipErrorInvalidValue;
  const int nw = rows / block_rows_per_lane(fp32, order);
  const BatchDispatch fn = fp32 ? (order == 2 ? batch_dispatch_f32_p2 : batch_dispatch_f32_p4)
                                 : (order == 2 ? batch_dispatch_f64_p2 : batch_dispatch_f64_p4);
  return fn(K, nw, force, descs, tile_prefix, nactive, total_tiles, pass, coefs, final_mode, s);
}

// ---- 3-D: z-pipelined blocked kernel ----
int block3d_rows_per_lane(bool fp32) { return fp32 ? Rows3d<float>::RS : Rows3d<double>::RS; }

// LDS of the double-buffered y-halo of all K levels (at most one CU's 160 KB)
static int block3d_lds(bool fp32, int order, int K, int nw) {
  return 2 * K * nw * 2 * (order / 2) * 64 * (fp32 ? 4 : 8);
}

bool block3d_config_supported(bool fp32, int order, int K, int rows) {
  if (!(order == 2 || order == 4) || K < 1 || K > kMaxBlockSteps3d) return false;
  // FP64 p = 4 rings of 3 or more levels do not fit the registers (they spill)
  if (!fp32 && order == 4 && K > 2) return false;
  const int rs = block3d_rows_per_lane(fp32);
  if (rows % rs != 0) return false;
  const int nw = rows / rs;
  if (fp32 ? (nw != 8 && nw != 16) : (nw != 4 && nw != 8)) return false;
  const int H = K * (order / 2);
  return rows - 2 * H > 0 && 64 - 2 * H > 0 && block3d_lds(fp32, order, K, nw) <= kBlock3dMaxLds;
}

// the larger group where it fits (FP32 16 waves, FP64 8)
int block3d_default_rows(bool fp32, int order, int K) {
  const int rs = block3d_rows_per_lane(fp32);
  const int big = (fp32 ? 16 : 8) * rs;
  return block3d_config_supported(fp32, order, K, big) ? big : big / 2;
}

hipError_t launch_block_steps_3d(bool fp32, const StepGeom &g, int K, int rows, const void *in_prev,
                                 const void *in_cur, void *out_prev, void *out_cur, double *acc, const void *c2,
                                 const void *f, const BlockCoef &coef, int mode, const double *v, double *out,
                                 hipStream_t s) {
  if (g.dim != 3 || !block3d_config_supported(fp32, g.order, K, rows)) return hipErrorInvalidValue;
  // node offsets within a plane are 32-bit byte offsets
  if ((double)g.sz * (fp32 ? 4.0 : 8.0) >= 4294967296.0) return hipErrorInvalidValue;
  const int nw = rows / block3d_rows_per_lane(fp32);
  const Block3dDispatch fn = fp32 ? (g.order == 2 ? block3d_dispatch_f32_p2 : block3d_dispatch_f32_p4)
                                   : (g.order == 2 ? block3d_dispatch_f64_p2 : block3d_dispatch_f64_p4);
  return fn(g, K, nw, in_prev, in_cur, out_prev, out_cur, acc, c2, f, coef, mode, v, out, s);
}

}  // namespace wh
