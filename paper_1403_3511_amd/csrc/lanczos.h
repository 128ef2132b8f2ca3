// Shared declarations of the Lanczos step machinery (single instance and batches).
#pragma once

#include <functional>

#include "hs_internal.h"

namespace hs {

constexpr int kSeg = 4096;        // rows per segment of a reduction
constexpr int kSegThreads = 256;
constexpr int kMaxM = 32;         // largest Krylov dimension
constexpr int kDotChunk = 8;      // inner products per launch

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
