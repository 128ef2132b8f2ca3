// Instantiations of the multi-tile fused H-application kernels for double data.
#include "matvec_multi.h"

namespace hs {

int launch_hh_multi_f64(const IndexDev &ix, const double *hh, const void *x, void *y,
                       const double *out_scale, const void *prev, const double *prev_coef,
                       const double *prev_scale, hipStream_t s, bool x2) {
  return launch_hh_multi_impl<double>(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, x2);
}

int launch_hh_short_f64(const IndexDev &ix, const double *hh, const void *x, void *y,
                       const double *out_scale, const void *prev, const double *prev_coef,
                       const double *prev_scale, hipStream_t s, bool x2) {
  return launch_hh_long_impl<double>(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, x2, true);
}

}  // namespace hs
