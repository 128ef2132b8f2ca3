// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hs.h"

namespace hs {

// ---- error reporting ----------------------------------------------------------------
void set_error(const std::string &msg);
int32_t fail(int32_t code, const std::string &msg);
int32_t hip_fail(hipError_t e, const char *what);
#define HS_HIP(call)                                             \
  do {                                                           \
    hipError_t e_ = (call);                                      \
    if (e_ != hipSuccess) return ::hs::hip_fail(e_, #call);      \
  } while (0)

inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// ---- index set ------------------------------------------------------------------------
// Device view of the tiled index layout.  All arrays live in one caller buffer.
struct IndexDev {
  int32_t N, d, np;          // dimension, suffix axes per tile, prefix axes (N - d)
  int32_t B;                 // product bound
  int64_t size;              // |K|
  int64_t ntiles, ng;        // tiles, entries of the global suffix list
  const int64_t *tstart;     // [ntiles + 1] first row of each tile
  const int32_t *tlen;       // [ntiles]
  const int32_t *tnbr;       // [ntiles][2 np]: 2l -> prefix - e_l, 2l+1 -> prefix + e_l (-1: none)
  const uint16_t *tpfx;      // [ntiles][np] prefix multi-index
  const int32_t *tpsum;      // [ntiles] sum of prefix coordinates
  const uint16_t *gsidx;     // [ng][d] suffix multi-index (graded order)
  const int32_t *gnbr;       // [ng][2d]: 2a -> s - e_a, 2a+1 -> s + e_a (-1: not in K_d(B))
  const int32_t *gssum;      // [ng] sum of suffix coordinates
  const int32_t *rowtile;    // [size] tile of each row
  const double *wtab;        // [B + 8] sqrt(k / 2)
  const float *wtabf;        // [B + 8] sqrt(k / 2) in float32
};

}  // namespace hs

struct hs_index_s {
  int32_t N = 0, d = 0, np = 0;
  int64_t B = 0, size = 0, ntiles = 0, ng = 0;
  std::vector<uint16_t> tpfx;
  std::vector<int64_t> tstart;
  std::vector<int32_t> tlen, tnbr, tpsum;
  std::vector<uint16_t> gsidx;
  std::vector<int32_t> gnbr, gssum;
  std::vector<int32_t> rowtile;
  // device blob layout (byte offsets)
  int64_t off_tstart = 0, off_tlen = 0, off_tnbr = 0, off_tpfx = 0, off_tpsum = 0,
          off_gsidx = 0, off_gnbr = 0, off_gssum = 0, off_rowtile = 0, off_wtab = 0,
          off_wtabf = 0, dev_bytes = 0;
  std::vector<uint8_t> blob;   // host image of the device block
  void *pinned = nullptr;      // pinned staging for the upload
  hs::IndexDev view(const void *dev) const;
};

namespace hs {

// ---- potential ----------------------------------------------------------------------
constexpr int kMaxTerms = 512;

// Fused class-HH kernel parameters: per outer axis l
//   t_l = X_l ( X_l ( X_l (a3 c) + g2 X_{l+1} c + a2 c ) + g1 X_{l+1} c + a1 c ) + g0' ...
// stored as coefficients of the monomials x_l^a (a = 1..3) and x_l^a x_{l+1} (a = 0..2).
struct HHCoef {
  double a[HS_NMAX][4];   // a[l][p]: coefficient of x_l^p (p = 1..3)
  double g[HS_NMAX][3];   // g[l][p]: coefficient of x_l^p x_{l+1} (p = 0..2)
  double c0;              // constant
};

// Generic program of recurrence passes over whole vectors.
struct PassOp {
  int32_t kind;      // 0: dst = A X_axis(src) + Bc src - C prev ; 1: acc += coef[term] * src
  int32_t axis;      // axis for kind 0
  int32_t src, prev, dst;  // vector slots (-1 none)
  double A, Bc, C;   // recurrence coefficients
  int32_t term;      // kind 1: term index into the coefficient array
};

}  // namespace hs

struct hs_pot_s {
  int32_t N = 0, basis = 0, nterms = 0;
  double scale = 1.0;
  std::vector<uint16_t> deg;          // nterms x N
  std::vector<double> base, amp, freq, phase;
  bool fused = false;
  // fused: compiled monomial coefficient of each HH slot = sum_t M[slot][t] beta_t
  int32_t nslots = 0;
  std::vector<double> M;              // nslots x nterms
  // generic program
  std::vector<hs::PassOp> prog;
  int32_t nslots_vec = 0;             // vector slots used by the program
  // device block: beta[kMaxTerms] | base | amp | freq | phase | M | hh coefficients
  int64_t dev_bytes = 0;
  int64_t off_beta = 0, off_base = 0, off_amp = 0, off_freq = 0, off_phase = 0, off_M = 0,
          off_hh = 0;
};

namespace hs {
int32_t compile_potential(hs_pot_s *p);
// kernels (implemented in the .hip translation units)
int32_t launch_set_time(const hs_pot_s *p, void *pot_dev, double t, const double *t_dev,
                        double dt_offset, hipStream_t s);
int32_t launch_apply_h(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p,
                       const void *pot_dev, int32_t dtype, const void *c, void *y, void *ws,
                       hipStream_t s, double out_scale_unused);
int64_t apply_workspace_bytes(const hs_index_s *idx, const hs_pot_s *p, int32_t dtype);
}  // namespace hs
