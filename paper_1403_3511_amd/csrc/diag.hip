// Local error diagnostics of the fast algorithm (paper Sec. 5.1, eqs. ErrorQuadratureDef and
// ErrorGridReductionDef), at the sizes the GPU holds.
//
//   E^red(v)  = W^pol(X_K) v - Omega(W^pol(X_full) Omega_+(v))
//   E^quad v  = W_{K,pol} v  - W^{GH(K)}_{K,pol} v
// with K_full the box {0..K}^N around the set.  By Lemma 1, W^{GH(K)} on the set is the
// restriction of the fast algorithm on the box; the exact Galerkin product W_{K,pol} v is
// the restriction of the fast algorithm on a box padded by half the polynomial's
// per-axis degree (a polynomial of degree r moves an index by at most r/2 and back, so
// the padded truncation is not seen by rows of the box).  The diagonal D is applied on
// every set and cancels in both differences.
#include <algorithm>
#include <cmath>

#include <string>

#include "hs_internal.h"

namespace hs {

// y_box = Omega_+(x): zero, then the set's entries at their box rows
__global__ void __launch_bounds__(256) k_zero(int64_t n, double2 *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = make_double2(0.0, 0.0);
}
// map entries outside [0, nbox) are skipped (the host checks containment; this keeps a
// wrong map from writing out of bounds)
__global__ void __launch_bounds__(256)
k_scatter(int64_t n, const int32_t *__restrict__ map, int64_t nbox, const double2 *__restrict__ x,
          double2 *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t m = map[i];
  if (m >= 0 && m < nbox) y[m] = x[i];
}
// e = a - b (e may alias a)
__global__ void __launch_bounds__(256)
k_diff(int64_t n, const double2 *a, const double2 *__restrict__ b, double2 *e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 u = a[i], w = b[i];
  e[i] = make_double2(u.x - w.x, u.y - w.y);
}
__global__ void __launch_bounds__(256)
k_gather(int64_t n, const int32_t *__restrict__ map, int64_t nbox, const double2 *__restrict__ ybox,
         double2 *__restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t m = map[i];
  g[i] = (m >= 0 && m < nbox) ? ybox[m] : make_double2(0.0, 0.0);
}

// g = out_scale * ybox[map] - prev_coef * prev_scale * prev (the optional factors when
// non-NULL): the exact operator's result on the rows of the set, in the step's form
__global__ void __launch_bounds__(256)
k_gather_step(int64_t n, const int32_t *__restrict__ map, int64_t nbox, const double2 *__restrict__ ybox,
              const double *__restrict__ out_scale, const double2 *__restrict__ prev,
              const double *__restrict__ prev_coef, const double *__restrict__ prev_scale,
              double2 *__restrict__ g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t m = map[i];
  double2 v = (m >= 0 && m < nbox) ? ybox[m] : make_double2(0.0, 0.0);
  if (out_scale) {
    const double f = *out_scale;
    v = make_double2(f * v.x, f * v.y);
  }
  if (prev) {
    const double pc = *prev_coef * (prev_scale ? *prev_scale : 1.0);
    const double2 q = prev[i];
    v = make_double2(fma(-pc, q.x, v.x), fma(-pc, q.y, v.y));
  }
  g[i] = v;
}

static unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

// workspace of the exact operator: the padded vector in and out, then the padded set's
// own H-application workspace
int64_t exact_apply_workspace_bytes(const hs_index_s *pad, const hs_pot_s *p) {
  const int64_t vb = align_up(std::max<int64_t>(pad->size, 1) * 16, 256);
  return 2 * vb + align_up(apply_workspace_bytes(pad, p, HS_C128), 256);
}

int32_t launch_exact_apply(const hs_index_s *sub, const hs_index_s *pad, const void *pad_dev, const int32_t *map,
                           const hs_pot_s *p, const void *pot_dev, const void *x, void *y, void *ws, hipStream_t s,
                           const double *out_scale, const void *prev, const double *prev_coef,
                           const double *prev_scale) {
  const int64_t n = sub->size;
  if (n == 0) return HS_OK;
  const int64_t vb = align_up(std::max<int64_t>(pad->size, 1) * 16, 256);
  uint8_t *w8 = static_cast<uint8_t *>(ws);
  double2 *xb = (double2 *)w8, *yb = (double2 *)(w8 + vb);
  hipLaunchKernelGGL(k_zero, dim3(nb(pad->size)), dim3(256), 0, s, pad->size, xb);
  hipLaunchKernelGGL(k_scatter, dim3(nb(n)), dim3(256), 0, s, n, map, pad->size, (const double2 *)x, xb);
  const int32_t st = launch_apply(pad, pad_dev, p, pot_dev, HS_C128, xb, yb, w8 + 2 * vb, s, nullptr, nullptr,
                                  nullptr, nullptr);
  if (st != HS_OK) return st;
  hipLaunchKernelGGL(k_gather_step, dim3(nb(n)), dim3(256), 0, s, n, map, pad->size, (const double2 *)yb,
                     out_scale, (const double2 *)prev, prev_coef, prev_scale, (double2 *)y);
  HS_HIP(hipGetLastError());
  return HS_OK;
}

// Whether pad carries the exact Galerkin operator of sub for pot: a box reaching half the
// potential's largest per-axis degree beyond every coordinate of sub (a degree-a factor
// moves an index by at most a/2 past both ends of an entry), or, for a hyperbolic cross,
// the padded cross of the same bound widened by at least that degree.
static int32_t check_exact_pad(const char *who, const hs_index_s *sub, const hs_index_s *pad, const hs_pot_s *p) {
  const std::string w(who);
  if (sub->N != p->N || pad->N != p->N) return fail(HS_E_INVALID, w + ": sets and potential differ in N");
  if (p->form != HS_FORM_PAPER) return fail(HS_E_UNSUPPORTED, w + ": the paper's operator form only");
  int maxdeg = 0;
  for (uint16_t a : p->deg) maxdeg = std::max<int>(maxdeg, a);
  if (pad->kind == HS_SET_PADDED) {
    if (sub->kind != HS_SET_HYPERBOLIC || pad->B - pad->deg != sub->B)
      return fail(HS_E_INVALID, w + ": a padded cross must widen the set itself (same product bound)");
    if (pad->deg < maxdeg) return fail(HS_E_INVALID, w + ": the padded cross must be widened by the largest per-axis degree");
    return HS_OK;
  }
  if (pad->kind != HS_SET_BOX) return fail(HS_E_INVALID, w + ": pad must be a box or a padded cross");
  int64_t top;  // the largest coordinate of sub
  switch (sub->kind) {
    case HS_SET_HYPERBOLIC: case HS_SET_PADDED: top = sub->B - 1; break;
    case HS_SET_BOX: top = sub->kmax; break;
    case HS_SET_TOTAL_DEGREE: top = sub->deg; break;
    default: return fail(HS_E_UNSUPPORTED, w + ": sets given as lists are not served");
  }
  if (pad->kmax < top + (maxdeg + 1) / 2)
    return fail(HS_E_INVALID, w + ": the box must exceed the set by half the largest per-axis degree");
  return HS_OK;
}

struct DiagLayout {
  int64_t big, off_x, off_y, off_g, off_apply, total;
};
static DiagLayout diag_layout(const hs_index_s *sub, const hs_index_s *box, const hs_index_s *pad,
                              const hs_pot_s *p) {
  DiagLayout L;
  L.big = std::max<int64_t>(box->size, pad ? pad->size : 0);
  const int64_t vb = align_up(L.big * 16, 256), vs = align_up(std::max<int64_t>(sub->size, 1) * 16, 256);
  int64_t aws = std::max(apply_workspace_bytes(sub, p, HS_C128), apply_workspace_bytes(box, p, HS_C128));
  if (pad) aws = std::max(aws, apply_workspace_bytes(pad, p, HS_C128));
  L.off_x = 0;
  L.off_y = vb;
  L.off_g = 2 * vb;
  L.off_apply = 2 * vb + vs;
  L.total = L.off_apply + align_up(aws, 256);
  return L;
}

}  // namespace hs

extern "C" int32_t hs_error_split_workspace_bytes(hs_index sub, hs_index box, hs_index pad, hs_pot pot,
                                                  int64_t *bytes) {
  if (!sub || !box || !pot || !bytes) return hs::fail(HS_E_INVALID, "hs_error_split_workspace_bytes: NULL argument");
  *bytes = hs::diag_layout(sub, box, pad, pot).total;
  return HS_OK;
}

extern "C" int32_t hs_error_split(hs_index sub, const void *sub_dev, hs_index box, const void *box_dev,
                                  const int32_t *box_map_dev, hs_index pad, const void *pad_dev,
                                  const int32_t *pad_map_dev, hs_pot pot, const void *pot_dev, const void *v,
                                  void *e_quad, void *e_red, void *ws, void *stream) {
  if (!sub || !box || !pot || !sub_dev || !box_dev || !box_map_dev || !pot_dev || !v || !e_red || !ws)
    return hs::fail(HS_E_INVALID, "hs_error_split: NULL argument");
  if (pad && (!pad_dev || !pad_map_dev || !e_quad))
    return hs::fail(HS_E_INVALID, "hs_error_split: padded box given without its buffers");
  if (v == e_red || (pad && (v == e_quad || e_quad == e_red)))
    return hs::fail(HS_E_INVALID, "hs_error_split: v, e_quad and e_red must be distinct buffers");
  int maxdeg = 0;
  for (uint16_t a : pot->deg) maxdeg = std::max<int>(maxdeg, a);
  // a padded cross in place of the box: e_red becomes the gap to the exact Galerkin product
  const bool gap = box->kind == HS_SET_PADDED;
  if (gap) {
    if (pad) return hs::fail(HS_E_INVALID, "hs_error_split: with a padded cross in place of the box, pad must be NULL");
    if (sub->kind != HS_SET_HYPERBOLIC || box->B - box->deg != sub->B)
      return hs::fail(HS_E_INVALID, "hs_error_split: the padded cross must widen the set (same product bound)");
    if (box->deg < maxdeg)
      return hs::fail(HS_E_INVALID, "hs_error_split: the padded cross must be widened by the largest per-axis degree");
  } else if (box->kind != HS_SET_BOX || (pad && pad->kind != HS_SET_BOX)) {
    return hs::fail(HS_E_INVALID, "hs_error_split: box and pad must be box sets (or box a padded cross)");
  }
  if (sub->N != pot->N || box->N != pot->N || (pad && pad->N != pot->N))
    return hs::fail(HS_E_INVALID, "hs_error_split: sets and potential differ in N");
  if (pad && pad->kmax < box->kmax) return hs::fail(HS_E_INVALID, "hs_error_split: the padded box is smaller than the box");
  if (pot->form != HS_FORM_PAPER) return hs::fail(HS_E_UNSUPPORTED, "hs_error_split: the paper's operator form only");
  // the box must contain the set: its largest coordinate is B - 1 (coordinates stay below B)
  if (!gap && sub->B - 1 > box->kmax) return hs::fail(HS_E_INVALID, "hs_error_split: the box does not contain the set");
  if (pad && pad->kmax - box->kmax < (maxdeg + 1) / 2)
    return hs::fail(HS_E_INVALID, "hs_error_split: the padded box must exceed the box by half the largest degree");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const hs::DiagLayout L = hs::diag_layout(sub, box, pad, pot);
  uint8_t *w8 = static_cast<uint8_t *>(ws);
  double2 *x = (double2 *)(w8 + L.off_x), *y = (double2 *)(w8 + L.off_y), *g = (double2 *)(w8 + L.off_g);
  void *aws = w8 + L.off_apply;
  const int64_t n = sub->size;
  if (n == 0) return HS_OK;
  int32_t st;
  // g = W^{GH(K)} v = Omega(F_box Omega_+(v))   (plus D v)
  hipLaunchKernelGGL(hs::k_zero, dim3(hs::nb(box->size)), dim3(256), 0, s, box->size, x);
  hipLaunchKernelGGL(hs::k_scatter, dim3(hs::nb(n)), dim3(256), 0, s, n, box_map_dev, box->size, (const double2 *)v, x);
  if ((st = hs::launch_apply(box, box_dev, pot, pot_dev, HS_C128, x, y, aws, s, nullptr, nullptr, nullptr, nullptr)) != HS_OK)
    return st;
  hipLaunchKernelGGL(hs::k_gather, dim3(hs::nb(n)), dim3(256), 0, s, n, box_map_dev, box->size, (const double2 *)y, g);
  // E^red = F_K v - g
  if ((st = hs::launch_apply(sub, sub_dev, pot, pot_dev, HS_C128, v, e_red, aws, s, nullptr, nullptr, nullptr, nullptr)) != HS_OK)
    return st;
  hipLaunchKernelGGL(hs::k_diff, dim3(hs::nb(n)), dim3(256), 0, s, n, (const double2 *)e_red, (const double2 *)g,
                     (double2 *)e_red);
  if (pad) {
    // E^quad = Omega(F_pad Omega_+(v)) - g
    hipLaunchKernelGGL(hs::k_zero, dim3(hs::nb(pad->size)), dim3(256), 0, s, pad->size, x);
    hipLaunchKernelGGL(hs::k_scatter, dim3(hs::nb(n)), dim3(256), 0, s, n, pad_map_dev, pad->size, (const double2 *)v, x);
    if ((st = hs::launch_apply(pad, pad_dev, pot, pot_dev, HS_C128, x, y, aws, s, nullptr, nullptr, nullptr, nullptr)) != HS_OK)
      return st;
    hipLaunchKernelGGL(hs::k_gather, dim3(hs::nb(n)), dim3(256), 0, s, n, pad_map_dev, pad->size, (const double2 *)y,
                       (double2 *)e_quad);
    hipLaunchKernelGGL(hs::k_diff, dim3(hs::nb(n)), dim3(256), 0, s, n, (const double2 *)e_quad, (const double2 *)g,
                       (double2 *)e_quad);
  }
  HS_HIP(hipGetLastError());
  return HS_OK;
}

extern "C" int32_t hs_exact_workspace_bytes(hs_index sub, hs_index pad, hs_pot pot, int32_t m, int64_t *bytes) {
  if (!sub || !pad || !pot || !bytes) return hs::fail(HS_E_INVALID, "hs_exact_workspace_bytes: NULL argument");
  if (m < 0 || m > 32) return hs::fail(HS_E_INVALID, "hs_exact_workspace_bytes: m out of range 0..32");
  *bytes = hs::step_exact_workspace_bytes(sub, pad, pot, m);
  return HS_OK;
}

extern "C" int32_t hs_apply_exact(hs_index sub, hs_index pad, const void *pad_dev, const int32_t *pad_map_dev,
                                  hs_pot pot, const void *pot_dev, const void *x, void *y, void *ws, void *stream) {
  if (!sub || !pad || !pad_dev || !pad_map_dev || !pot || !pot_dev || !x || !y || !ws)
    return hs::fail(HS_E_INVALID, "hs_apply_exact: NULL argument");
  if (x == y) return hs::fail(HS_E_INVALID, "hs_apply_exact: x and y must be distinct buffers");
  const int32_t st = hs::check_exact_pad("hs_apply_exact", sub, pad, pot);
  if (st != HS_OK) return st;
  return hs::launch_exact_apply(sub, pad, pad_dev, pad_map_dev, pot, pot_dev, x, y, ws,
                                static_cast<hipStream_t>(stream), nullptr, nullptr, nullptr, nullptr);
}

extern "C" int32_t hs_step_exact(hs_index sub, hs_index pad, const void *pad_dev, const int32_t *pad_map_dev,
                                 hs_pot pot, void *pot_dev, double t, double *t_dev, double h, int32_t m,
                                 int32_t reorth, void *c, void *ws, double *diag_dev, void *stream) {
  if (!sub || !pad || !pad_dev || !pad_map_dev || !pot || !pot_dev || !c || !ws)
    return hs::fail(HS_E_INVALID, "hs_step_exact: NULL argument");
  if (m < 1 || m > 32) return hs::fail(HS_E_INVALID, "hs_step_exact: m out of range 1..32");
  if (!std::isfinite(h) || (!t_dev && !std::isfinite(t))) return hs::fail(HS_E_NONFINITE, "hs_step_exact: t or h not finite");
  const int32_t st = hs::check_exact_pad("hs_step_exact", sub, pad, pot);
  if (st != HS_OK) return st;
  return hs::launch_step_exact(sub, pad, pad_dev, pad_map_dev, pot, pot_dev, t, t_dev, h, m, reorth, c, ws,
                               diag_dev, static_cast<hipStream_t>(stream));
}
