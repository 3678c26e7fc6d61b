// Configuration queries and routing of the blocked-kernel launches to the
// per-(precision, order) translation units (wh_block_<prec>_p<order>.hip).
#include <hip/hip_runtime.h>

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

}  // namespace wh
