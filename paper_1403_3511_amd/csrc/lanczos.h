// Shared declarations of the Lanczos step machinery (single instance and batches).
#pragma once

#include <functional>

#include "hs_internal.h"

namespace hs {

constexpr int kSeg = 4096;        // rows per segment of a reduction
constexpr int kSegThreads = 256;
constexpr int kMaxM = 32;         // largest Krylov dimension
constexpr int kDotChunk = 8;      // inner products per launch
constexpr double kBreakdownTol = 1e-12;  // beta_k <= tol max(1, ||T_{k+1}||_inf) ends the recurrence
constexpr int64_t kSmallStepRowsDefault = 1024;

// one-workgroup step of small sets (step_small.h); 1 if launched
int launch_step_small_f64(const IndexDev &ix, const double *hh, void *c, void *V, int64_t stride, double h,
                          int m, int reorth, double tol, double *sc, double *t_adv, double *diag, hipStream_t s,
                          bool x2);
int launch_step_small_f32(const IndexDev &ix, const double *hh, void *c, void *V, int64_t stride, double h,
                          int m, int reorth, double tol, double *sc, double *t_adv, double *diag, hipStream_t s,
                          bool x2);
constexpr int64_t kSmallStepRowsMax = 1024;  // rows the one-workgroup step can hold
// (N, NP) pairs with an instantiation of the one-workgroup step: the library's default tile dimension for N <= 8
inline bool step_small_supported(int N, int np) {
  switch (N * 32 + np) {
    case 1 * 32 + 0: case 2 * 32 + 0: case 3 * 32 + 1: case 4 * 32 + 2:
    case 5 * 32 + 2: case 6 * 32 + 3: case 7 * 32 + 4: case 8 * 32 + 5:
      return true;
    default:
      return false;
  }
}


// scalar block of one instance (doubles)
struct Scal {
  static constexpr int beta0 = 0, inv0 = 1, stop = 2, meff = 3;
  static constexpr int alpha = 8;                 // [kMaxM]
  static constexpr int beta = alpha + kMaxM;      // [kMaxM]
  static constexpr int inv = beta + kMaxM;        // [kMaxM] 1 / beta_k
  static constexpr int dre = inv + kMaxM;         // [kMaxM + 1] inner products (re)
  static constexpr int dim = dre + kMaxM + 1;     // (im)
  static constexpr int yre = dim + kMaxM + 1;     // [kMaxM] combination weights
  static constexpr int yim = yre + kMaxM;
  static constexpr int size = yim + kMaxM;
};

// y = beta0 exp(-i h T) e1 for the real symmetric tridiagonal T (m <= 32) held in the
// scalar block sc, by scaling and squaring: delta = h / 2^q with h ||T||_inf / 2^q <= 1/2,
// an 18-term Taylor polynomial of exp(-i delta T) (truncation below 1e-22), then q
// squarings.  One thread per matrix element: every thread of a block of kMaxM^2 threads
// calls it, with the same sc.
__device__ __forceinline__ void small_expm_block(double h, double *__restrict__ sc) {
  __shared__ double2 E[kMaxM][kMaxM + 1], P[kMaxM][kMaxM + 1];
  __shared__ double td[kMaxM], to[kMaxM];
  __shared__ double s_delta;
  __shared__ int s_q;
  const int m = (int)sc[Scal::meff];
  if (m <= 0) return;
  const int tid = threadIdx.x;
  const int i = tid / kMaxM, j = tid % kMaxM;
  const bool act = (i < m) && (j < m);
  if (tid < m) {
    td[tid] = sc[Scal::alpha + tid];
    to[tid] = (tid + 1 < m) ? sc[Scal::beta + tid] : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double nrm = 0.0;
    for (int r = 0; r < m; ++r) {
      double row = fabs(td[r]) + fabs(to[r]);
      if (r > 0) row += fabs(to[r - 1]);
      nrm = fmax(nrm, row);
    }
    double rho = fabs(h) * nrm;
    int q = 0;
    while (rho > 0.5 && q < 60) {
      rho *= 0.5;
      ++q;
    }
    s_q = q;
    s_delta = ldexp(h, -q);
  }
  __syncthreads();
  const double delta = s_delta;
  const int q = s_q;
  if (act) {
    const double2 d = make_double2(i == j ? 1.0 : 0.0, 0.0);
    E[i][j] = d;
    P[i][j] = d;
  }
  __syncthreads();
  for (int k = 1; k <= 18; ++k) {
    double2 nv = make_double2(0.0, 0.0);
    if (act) {  // P <- P (-i delta T) / k, T tridiagonal
      double sr = P[i][j].x * td[j], si = P[i][j].y * td[j];
      if (j > 0) {
        sr += P[i][j - 1].x * to[j - 1];
        si += P[i][j - 1].y * to[j - 1];
      }
      if (j + 1 < m) {
        sr += P[i][j + 1].x * to[j];
        si += P[i][j + 1].y * to[j];
      }
      const double f = delta / k;
      nv = make_double2(si * f, -sr * f);
    }
    __syncthreads();
    if (act) {
      P[i][j] = nv;
      E[i][j].x += nv.x;
      E[i][j].y += nv.y;
    }
    __syncthreads();
  }
  for (int r = 0; r < q; ++r) {
    double2 nv = make_double2(0.0, 0.0);
    if (act) {
      double ar = 0.0, ai = 0.0;
      for (int l = 0; l < m; ++l) {
        const double2 a = E[i][l], b = E[l][j];
        ar = fma(a.x, b.x, fma(-a.y, b.y, ar));
        ai = fma(a.x, b.y, fma(a.y, b.x, ai));
      }
      nv = make_double2(ar, ai);
    }
    __syncthreads();
    if (act) E[i][j] = nv;
    __syncthreads();
  }
  if (act && j == 0) {
    const double b0 = sc[Scal::beta0];
    sc[Scal::yre + i] = b0 * E[i][0].x;
    sc[Scal::yim + i] = b0 * E[i][0].y;
  }
}

// Segments of packed vectors: segment s covers rows [row0, row0 + len) of instance inst.
// A single instance uses implicit segments (inst == nullptr).
struct SegView {
  int32_t n;              // instances
  int64_t nseg;
  const int32_t *inst;    // [nseg]
  const int64_t *row0;    // [nseg]
  const int32_t *len;     // [nseg]
  const int64_t *iseg0;   // [n + 1] first segment of each instance
  int64_t size;           // rows of the single instance
  __device__ __forceinline__ void get(int64_t s, int &i, int64_t &r0, int &l) const {
    if (!inst) {
      i = 0;
      r0 = s * kSeg;
      const int64_t rest = size - r0;
      l = (int)(rest < kSeg ? rest : kSeg);
    } else {
      i = inst[s];
      r0 = row0[s];
      l = len[s];
    }
  }
  __device__ __forceinline__ void range(int i, int64_t &s0, int64_t &s1) const {
    if (!inst) {
      s0 = 0;
      s1 = nseg;
    } else {
      s0 = iseg0[i];
      s1 = iseg0[i + 1];
    }
  }
};

struct StepLayout {
  int64_t vec_stride;  // bytes between Krylov vectors
  int64_t off_V, off_W, off_apply, off_part, off_sc, total;
};
StepLayout step_layout(int64_t rows, int64_t nseg, int n, int64_t elem_bytes, int m, int64_t apply_ws);

// What a step needs besides the vector kernels: the coefficient update and H v.
struct StepJob {
  int64_t rows = 0;
  SegView sv{};
  int64_t apply_ws = 0;
  std::function<int32_t(hipStream_t)> set_time;
  // w = H v_k - beta_{k-1} v_{k-1} (vprev == nullptr for k = 0); sc = scalar blocks
  std::function<int32_t(const void *, void *, const void *, int, double *, void *, hipStream_t)> matvec;
};

template <typename T>
int32_t run_step(const StepJob &J, int m, int reorth, double h, void *c, void *ws,
                 const double *t_dev, double *t_adv, double *diag, hipStream_t s);

}  // namespace hs
