// Instantiations of the fused fourth-order Magnus passes for float data.
#include "matvec_m4.h"

namespace hs {

bool launch_m4_f32(const IndexDev &ix, const double *hh1, const double *hh2, const void *v, void *a,
                  void *d, void *w, const double *in_scale, double g2, const void *prev,
                  const double *prev_coef, const double *prev_scale, hipStream_t s, bool x2,
                  bool dl) {
  return launch_m4_impl<float>(ix, hh1, hh2, v, a, d, w, in_scale, g2, prev, prev_coef, prev_scale, s, x2, dl);
}

}  // namespace hs
