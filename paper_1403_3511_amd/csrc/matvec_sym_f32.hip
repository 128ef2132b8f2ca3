// Instantiations of the symmetrised fused H-application kernels for float data.
#include "matvec_long.h"

namespace hs {

int launch_hh_long_sym_f32(const IndexDev &ix, const double *hh, const void *x, void *y,
                          const double *out_scale, const void *prev, const double *prev_coef,
                          const double *prev_scale, hipStream_t s, bool x2) {
  return launch_hh_long_impl<float, true>(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, x2);
}

}  // namespace hs
