// Blocked-kernel instantiations for FP32 state, order 4.
#include <hip/hip_runtime.h>

#include "wh_block_impl.h"

namespace wh {

hipError_t block_dispatch_f32_p4(const StepGeom &g, int K, int nw, int ksteps, const void *in_prev,
                                 const void *in_cur, void *out_prev, void *out_cur, double *acc, const void *c2,
                                 const void *f, const BlockCoef &coef, int mode, const double *v, double *out,
                                 hipStream_t s) {
  return dispatch_k<float, 4>(g, K, nw, ksteps, in_prev, in_cur, out_prev, out_cur, acc, c2, f, coef, mode, v, out, s);
}

hipError_t batch_dispatch_f32_p4(int K, int nw, bool force, const BatchDesc *descs, const int *tile_prefix,
                                 int nactive, int total_tiles, int pass, const BlockCoef *coefs, int final_mode,
                                 hipStream_t s) {
  return batch_k<float, 4>(K, nw, force, descs, tile_prefix, nactive, total_tiles, pass, coefs, final_mode, s);
}

}  // namespace wh
