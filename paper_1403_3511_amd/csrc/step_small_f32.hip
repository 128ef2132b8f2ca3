// Instantiations of the one-workgroup small-set step for float Krylov vectors.
#include "step_small.h"

namespace hs {

int launch_step_small_f32(const IndexDev &ix, const double *hh, void *c, void *V, int64_t stride, double h,
                          int m, int reorth, double tol, double *sc, double *t_adv, double *diag, hipStream_t s,
                          bool x2) {
  return launch_step_small_impl<float>(ix, hh, c, V, stride, h, m, reorth, tol, sc, t_adv, diag, s, x2);
}

}  // namespace hs
