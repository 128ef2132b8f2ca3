// Instantiations of the multi-tile fused H-application kernels for float data.
#include "matvec_multi.h"

namespace hs {

int launch_hh_multi_f32(const IndexDev &ix, const double *hh, const void *x, void *y,
                       const double *out_scale, const void *prev, const double *prev_coef,
                       const double *prev_scale, hipStream_t s, bool x2) {
  return launch_hh_multi_impl<float>(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, x2);
}

int launch_hh_short_f32(const IndexDev &ix, const double *hh, const void *x, void *y,
                       const double *out_scale, const void *prev, const double *prev_coef,
                       const double *prev_scale, hipStream_t s, bool x2) {
  return launch_hh_long_impl<float>(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, x2, true);
}

}  // namespace hs
