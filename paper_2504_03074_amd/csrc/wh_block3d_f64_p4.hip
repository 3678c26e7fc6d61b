// 3-D blocked-kernel instantiations for FP64 state, order 4.
#include <hip/hip_runtime.h>

#include "wh_block3d_impl.h"

namespace wh {

hipError_t block3d_dispatch_f64_p4(const StepGeom &g, int K, int nw, const void *in_prev, const void *in_cur,
                                   void *out_prev, void *out_cur, double *acc, const void *c2, const void *f,
                                   const BlockCoef &coef, int mode, const double *v, double *out, hipStream_t s) {
  return dispatch3d_k<double, 4>(g, K, nw, in_prev, in_cur, out_prev, out_cur, acc, c2, f, coef, mode, v, out, s);
}

}  // namespace wh
