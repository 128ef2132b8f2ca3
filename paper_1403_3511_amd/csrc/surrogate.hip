// Learned potential coefficients.
//
// (1) Gauss-Hermite projection (the fallback and the accuracy reference): for the potential family
//     W(x) = - sum_i a_i exp(-|x - c_i(t)|^2 / (2 sigma^2)),
//     c_i(t) = base_i + rho (cos(omega t + phi_i) u_i + sin(omega t + phi_i) w_i),
//     alpha_a = <W, H_a> / <H_a, H_a> (weight exp(-|x|^2)) by the product Gauss-Hermite
//     rule with Q nodes per axis (paper Sec. 4.1), |a| <= D.  The Q^N-point sum is
//     factorised over the two halves of the axes: S[mA][aB] = sum_mB F(mA, mB) h_aB(mB)
//     in LDS, then alpha_(aA, aB) = sum_mA h_aA(mA) S[mA][aB].
// (2) A multilayer perceptron in -> hid -> hid -> out with SiLU, trained on those
//     coefficients: BF16 MFMA products (v_mfma_f32_16x16x32_bf16) with FP32
//     accumulation, FP32 master weights, Adam.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "hs_internal.h"

namespace hs {

// ---------------------------------------------------------------------------------------
// Gauss-Hermite rule (host).  The nodes are the eigenvalues of the Jacobi matrix J with zero
// diagonal and off-diagonals sqrt(k/2), k = 1..Q-1 (the matrix X_full of paper Sec. 4.2,
// whose eigen-decomposition U^T Xi U gives the quadrature), i.e. the zeros of the
// orthonormal Hermite polynomial psi_Q.  They are located by Sturm-sequence bisection
// (Wilkinson): for a shift x, the LDL^T pivots of J - x I,
//   q_0 = -x,  q_k = -x - (k/2) / q_{k-1},
// have as many negative entries as J has eigenvalues below x.  Each node is bracketed by
// the Gershgorin interval and bisected until the bracket stops shrinking, then polished by
// one Newton step on psi_Q (psi_Q' = sqrt(2Q) psi_{Q-1}).  The weights come from the
// Christoffel function w_m = 1 / sum_{k<Q} psi_k(x_m)^2 with psi_0 = pi^(-1/4).
// ---------------------------------------------------------------------------------------
// number of eigenvalues of J (order Q) strictly below x
static int gh_sturm_count(int Q, double x) {
  int neg = 0;
  double q = -x;
  for (int k = 1;; ++k) {
    // a zero pivot is replaced by a tiny positive one (a shift of x by a negligible
    // amount), used both for the count and for the next pivot
    if (q == 0.0) q = 1e-300;
    if (q < 0.0) ++neg;
    if (k == Q) break;
    q = -x - 0.5 * k / q;
  }
  return neg;
}

// psi_{Q-1}(x) and psi_Q(x) by the three-term recurrence
//   sqrt((k+1)/2) psi_{k+1} = x psi_k - sqrt(k/2) psi_{k-1}
static void gh_psi_pair(int Q, double x, double &pqm1, double &pq) {
  double pm = 0.0, pc = std::pow(M_PI, -0.25);
  for (int k = 0; k < Q; ++k) {
    const double pn = (x * pc - std::sqrt(0.5 * k) * pm) / std::sqrt(0.5 * (k + 1));
    pm = pc;
    pc = pn;
  }
  pqm1 = pm;
  pq = pc;
}

// nodes x (ascending) and weights w of the Q-point rule for the weight exp(-x^2);
// false if the bisection did not isolate Q distinct nodes
static bool gh_rule(int Q, std::vector<double> &x, std::vector<double> &w) {
  x.assign(Q, 0.0);
  w.assign(Q, 0.0);
  // Gershgorin: every eigenvalue lies in [-g, g]
  double g = 0.0;
  for (int k = 0; k < Q; ++k) {
    const double lo = k > 0 ? std::sqrt(0.5 * k) : 0.0, hi = k + 1 < Q ? std::sqrt(0.5 * (k + 1)) : 0.0;
    g = std::max(g, lo + hi);
  }
  g = g * (1.0 + 1e-12) + 1e-300;
  for (int m = 0; m < Q; ++m) {
    // the (m+1)-th smallest eigenvalue: count(a) <= m < count(b)
    double a = -g, b = g;
    for (int it = 0; it < 2000; ++it) {
      const double mid = 0.5 * (a + b);
      if (mid <= a || mid >= b) break;  // the bracket cannot shrink further
      if (gh_sturm_count(Q, mid) <= m) a = mid; else b = mid;
    }
    double xm = 0.5 * (a + b);
    double pqm1, pq;
    gh_psi_pair(Q, xm, pqm1, pq);
    const double dpq = std::sqrt(2.0 * Q) * pqm1;
    if (dpq != 0.0) {
      const double step = pq / dpq;
      // keep the polish inside the bracket that isolates this node
      if (std::fabs(step) <= (b - a) + 1e-15 * (1.0 + std::fabs(xm))) xm -= step;
    }
    x[m] = xm;
  }
  for (int m = 1; m < Q; ++m)
    if (!(x[m] > x[m - 1])) return false;
  for (int m = 0; m < Q; ++m) {
    double pm = 0.0, pc = std::pow(M_PI, -0.25), s = pc * pc;
    for (int k = 0; k + 1 < Q; ++k) {
      const double pn = (x[m] * pc - std::sqrt(0.5 * k) * pm) / std::sqrt(0.5 * (k + 1));
      pm = pc;
      pc = pn;
      s += pc * pc;
    }
    w[m] = 1.0 / s;
    if (!std::isfinite(w[m]) || !(w[m] > 0.0)) return false;
  }
  return true;
}

// ---------------------------------------------------------------------------------------
// projection kernel
// ---------------------------------------------------------------------------------------
constexpr int kGhMaxQ = 32, kGhMaxG = 4, kGhMaxN = 4, kGhMaxD = 8;
constexpr int kGhThreads = 512;
constexpr int kGhChunk = 4096;                // most leading-grid rows per chunk
constexpr size_t kGhLdsBytes = 64 * 1024;    // LDS budget of one workgroup

struct GhArgs {
  int N, G, D, Q, NA, NB, QA, QB, nB, ncoef, R;
  double xi[kGhMaxQ];
  double hq[kGhMaxD + 1][kGhMaxQ];  // w_m H_n(xi_m) / (sqrt(pi) 2^n n!)
  double base[kGhMaxG][kGhMaxN], u[kGhMaxG][kGhMaxN], w[kGhMaxG][kGhMaxN], phase[kGhMaxG];
};

// LDS layout of the projection kernel (doubles first, then ints)
struct GhLds {
  int64_t F, T, S, hq, xi, dbl_end;  // double offsets
  int bcode, bpos, kA, kB, int_end;  // int offsets after the doubles
  static __host__ __device__ GhLds make(int R, int QB, int Q, int D, int nB, int NB, int ncoef) {
    GhLds L;
    L.F = 0;
    L.T = L.F + (int64_t)R * QB;
    L.S = L.T + (NB == 2 ? (int64_t)R * Q * (D + 1) : 0);
    L.hq = L.S + (int64_t)R * nB;
    L.xi = L.hq + (int64_t)(D + 1) * Q;
    L.dbl_end = L.xi + Q;
    int totB = 1;
    for (int l = 0; l < NB; ++l) totB *= (D + 1);
    L.bcode = 0;
    L.bpos = L.bcode + nB;
    L.kA = L.bpos + totB;
    L.kB = L.kA + ncoef;
    L.int_end = L.kB + ncoef;
    return L;
  }
  __host__ __device__ size_t bytes() const { return sizeof(double) * dbl_end + sizeof(int) * int_end; }
};

// One block per sample; params row: (t, a_1..a_G, sigma, rho, omega).
// V is evaluated at every node of the Q^N grid from its definition (a black box for the
// projection).  Axes split into a leading half A (NA axes) and a trailing half B (NB <= 2
// axes).  For a chunk of R leading-grid points mA:
//   F[r][mB] = W(xi_mA, xi_mB)
//   S[r][b]  = sum_mB F[r][mB] prod_{l in B} hq[aB_l][mB_l]   (b over |aB| <= D; for NB = 2
//              as two 1-D contractions through T[r][mB0][aB1])
//   alpha_(aA, aB) += sum_r prod_{l in A} hq[aA_l][mA_l] S[r][b(aB)]   (one per thread)
// With a box (lo, hi non-null) only samples with some input outside [lo, hi] are
// projected (the others keep what the network wrote); used[s] records the choice.
__global__ void __launch_bounds__(kGhThreads)
k_gh_project(GhArgs A, const double *__restrict__ params, double *__restrict__ coef,
             const float *__restrict__ lo, const float *__restrict__ hi, int32_t *__restrict__ used) {
  extern __shared__ double lds[];
  const GhLds L = GhLds::make(A.R, A.QB, A.Q, A.D, A.nB, A.NB, A.ncoef);
  double *Fc = lds + L.F, *Tc = lds + L.T, *Sc = lds + L.S, *hqs = lds + L.hq, *xis = lds + L.xi;
  int *ib = (int *)(lds + L.dbl_end);
  int *bcode = ib + L.bcode, *bpos = ib + L.bpos, *kA = ib + L.kA, *kB = ib + L.kB;
  const int tid = threadIdx.x;
  const int s = blockIdx.x;
  const int Q = A.Q, DB = A.D + 1;
  const double *p = params + (int64_t)s * (A.G + 4);
  if (lo) {
    bool inside = true;
    for (int k = 0; k < A.G + 4; ++k) inside = inside && p[k] >= (double)lo[k] && p[k] <= (double)hi[k];
    if (tid == 0 && used) used[s] = inside ? 0 : 1;
    if (inside) return;  // uniform over the block: no barrier has been reached yet
  }
  const double t = p[0], sigma = p[A.G + 1], rho = p[A.G + 2], omega = p[A.G + 3];
  const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
  double cen[kGhMaxG][kGhMaxN], amp[kGhMaxG];
#pragma unroll
  for (int i = 0; i < kGhMaxG; ++i) {
    amp[i] = i < A.G ? p[1 + i] : 0.0;
    const double ang = omega * t + A.phase[i];
    const double ca = cos(ang), sa = sin(ang);
#pragma unroll
    for (int l = 0; l < kGhMaxN; ++l) cen[i][l] = A.base[i][l] + rho * (ca * A.u[i][l] + sa * A.w[i][l]);
  }
  for (int e = tid; e < DB * Q; e += kGhThreads) hqs[e] = A.hq[e / Q][e % Q];
  for (int e = tid; e < Q; e += kGhThreads) xis[e] = A.xi[e];
  // multi-index tables, |a| <= D in lexicographic order (last axis fastest), compacted
  // by one wave with ballots
  int totB = 1, tot = 1;
  for (int l = 0; l < A.NB; ++l) totB *= DB;
  for (int l = 0; l < A.N; ++l) tot *= DB;
  if (tid < 64) {
    int nb = 0;
    for (int c0 = 0; c0 < totB; c0 += 64) {
      const int c = c0 + tid;
      int sum = 0, code = 0;
      if (c < totB) {
        int r = c;
        for (int l = A.NB - 1, sh = 0; l >= 0; --l, sh += 4) {
          const int d = r % DB;
          r /= DB;
          sum += d;
          code |= d << sh;
        }
      }
      const bool ok = c < totB && sum <= A.D;
      const unsigned long long mask = __ballot(ok);
      const int pos = nb + __popcll(mask & ((1ull << tid) - 1ull));
      if (ok) {
        bcode[pos] = code;
        bpos[c] = pos;
      }
      nb += __popcll(mask);
    }
  }
  __syncthreads();
  if (tid < 64) {
    int nk = 0;
    for (int c0 = 0; c0 < tot; c0 += 64) {
      const int c = c0 + tid;
      int sum = 0, codeA = 0, cB = c % totB;
      if (c < tot) {
        int r = c;
        for (int l = A.N - 1; l >= 0; --l) {
          const int d = r % DB;
          r /= DB;
          sum += d;
          if (l < A.NA) codeA |= d << (4 * (A.NA - 1 - l));
        }
      }
      const bool ok = c < tot && sum <= A.D;
      const unsigned long long mask = __ballot(ok);
      const int pos = nk + __popcll(mask & ((1ull << tid) - 1ull));
      if (ok) {
        kA[pos] = codeA;
        kB[pos] = bpos[cB];
      }
      nk += __popcll(mask);
    }
  }
  __syncthreads();
  double acc = 0.0;
  int degA[2] = {0, 0}, bk = 0;
  const bool has_k = tid < A.ncoef;
  if (has_k) {
    const int codeA = kA[tid];
    bk = kB[tid];
    degA[0] = A.NA == 2 ? (codeA >> 4) & 15 : codeA & 15;
    degA[1] = codeA & 15;
  }

  for (int mA0 = 0; mA0 < A.QA; mA0 += A.R) {
    const int R = min(A.R, A.QA - mA0);
    // V at the nodes of this chunk
    for (int e = tid; e < R * A.QB; e += kGhThreads) {
      int m = mA0 * A.QB + e;  // grid point index, digits in base Q, last axis fastest
      double xv[kGhMaxN];
#pragma unroll
      for (int l = kGhMaxN - 1; l >= 0; --l) {
        xv[l] = 0.0;
        if (l < A.N) {
          const int q = m / Q;
          xv[l] = xis[m - q * Q];
          m = q;
        }
      }
      double F = 0.0;
#pragma unroll
      for (int i = 0; i < kGhMaxG; ++i) {
        if (i < A.G) {
          double r2 = 0.0;
#pragma unroll
          for (int l = 0; l < kGhMaxN; ++l) {
            if (l < A.N) {
              const double dx = xv[l] - cen[i][l];
              r2 = fma(dx, dx, r2);
            }
          }
          F -= amp[i] * exp(-r2 * inv2s2);
        }
      }
      Fc[e] = F;
    }
    __syncthreads();
    // trailing-half projections
    if (A.NB == 2) {
      // T[r][m0][a1] = sum_m1 F[r][m0 Q + m1] hq[a1][m1]
      for (int e = tid; e < R * Q * DB; e += kGhThreads) {
        const int a1 = e % DB, rm0 = e / DB;
        const double *Fr = Fc + (int64_t)rm0 * Q;
        const double *h = hqs + a1 * Q;
        double sum = 0.0;
        for (int m1 = 0; m1 < Q; ++m1) sum = fma(Fr[m1], h[m1], sum);
        Tc[e] = sum;
      }
      __syncthreads();
      // S[r][b] = sum_m0 hq[a0][m0] T[r][m0][a1]
      for (int e = tid; e < R * A.nB; e += kGhThreads) {
        const int r = e / A.nB, b = e % A.nB;
        const int a0 = (bcode[b] >> 4) & 15, a1 = bcode[b] & 15;
        const double *Tr = Tc + (int64_t)r * Q * DB + a1;
        const double *h = hqs + a0 * Q;
        double sum = 0.0;
        for (int m0 = 0; m0 < Q; ++m0) sum = fma(h[m0], Tr[m0 * DB], sum);
        Sc[e] = sum;
      }
    } else if (A.NB == 1) {
      for (int e = tid; e < R * A.nB; e += kGhThreads) {
        const int r = e / A.nB, b = e % A.nB;
        const double *Fr = Fc + (int64_t)r * Q;
        const double *h = hqs + (bcode[b] & 15) * Q;
        double sum = 0.0;
        for (int m = 0; m < Q; ++m) sum = fma(Fr[m], h[m], sum);
        Sc[e] = sum;
      }
    } else {
      for (int r = tid; r < R; r += kGhThreads) Sc[r] = Fc[r];
    }
    __syncthreads();
    // leading-half projections, accumulated per coefficient
    if (has_k) {
      double sum = 0.0;
      for (int r = 0; r < R; ++r) {
        const int m = mA0 + r;
        double h = Sc[r * A.nB + bk];
        if (A.NA == 2) {
          const int m0 = m / Q;
          h *= hqs[degA[0] * Q + m0] * hqs[degA[1] * Q + (m - m0 * Q)];
        } else {
          h *= hqs[degA[1] * Q + m];
        }
        sum += h;
      }
      acc += sum;
    }
    __syncthreads();
  }
  if (has_k) coef[(int64_t)s * A.ncoef + tid] = acc;
}

static int64_t binom(int n, int k) {
  int64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// ---------------------------------------------------------------------------------------
// BF16 MFMA GEMM with fused epilogues
//   C(i, j) = sum_k A(i, k) B(k, j), A(i, k) = A[i sa0 + k sa1], B(k, j) = B[k sb0 + j sb1]
// FP32 operands in memory, rounded to BF16 when loaded into the MFMA fragments, FP32
// accumulation.  One wave per 16 x 16 output tile; lane l holds A row l%16 and B column
// l%16 for the K slice [8 (l/16), 8 (l/16) + 8) of each 32-wide step, and the outputs
// rows 4 (l/16) .. +3 of column l%16.
// ---------------------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

enum GemmEpi { kEpiStore = 0, kEpiBiasSilu = 1, kEpiSiluGrad = 2 };

// ---------------------------------------------------------------------------------------
// Chebyshev interpolation (paper Sec. 1.3)
// ---------------------------------------------------------------------------------------
constexpr int kChMaxP = 16;                  // R + 1 points per axis
constexpr int kChMaxCoef = 512;
constexpr int kChThreads = 512;
constexpr size_t kChLdsBytes = 64 * 1024;   // grid values and the cosine table

struct ChArgs {
  int N, G, P, grid, ncoef;
  double xk[kChMaxP];              // L cos(theta_k), theta_k = (2k + 1) pi / (2P)
  uint16_t digits[kChMaxCoef];     // requested r, 4 bits per axis (axis 0 highest)
  double base[kGhMaxG][kGhMaxN], u[kGhMaxG][kGhMaxN], w[kGhMaxG][kGhMaxN], phase[kGhMaxG];
};

// One block per sample; params row: (t, a_1..a_G, sigma, rho, omega).  W is evaluated at
// the P^N points of the first-kind Chebyshev grid (grid index with the last axis
// fastest) into LDS; the discrete Chebyshev transform is then taken one axis at a time,
// in place, one fibre per thread (the P inputs of a fibre are held in registers while its
// P outputs are written); the requested coefficients are gathered at the end.
__global__ void __launch_bounds__(kChThreads)
k_cheb_interp(ChArgs A, const double *__restrict__ params, double *__restrict__ coef) {
  extern __shared__ double lds[];
  double *F = lds, *cth = lds + A.grid;
  const int tid = threadIdx.x, s = blockIdx.x, N = A.N, P = A.P;
  for (int e = tid; e < P * P; e += kChThreads) {
    const int r = e / P, k = e - r * P;
    cth[e] = (r == 0 ? 1.0 : 2.0) / P * cos(r * (2.0 * k + 1.0) * M_PI / (2.0 * P));
  }
  const double *p = params + (int64_t)s * (A.G + 4);
  const double t = p[0], sigma = p[A.G + 1], rho = p[A.G + 2], omega = p[A.G + 3];
  const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
  double cen[kGhMaxG][kGhMaxN], amp[kGhMaxG];
#pragma unroll
  for (int i = 0; i < kGhMaxG; ++i) {
    amp[i] = i < A.G ? p[1 + i] : 0.0;
    const double ang = omega * t + A.phase[i];
    const double ca = cos(ang), sa = sin(ang);
#pragma unroll
    for (int l = 0; l < kGhMaxN; ++l) cen[i][l] = A.base[i][l] + rho * (ca * A.u[i][l] + sa * A.w[i][l]);
  }
  for (int m = tid; m < A.grid; m += kChThreads) {
    double xv[kGhMaxN];
    int r = m;
#pragma unroll
    for (int l = kGhMaxN - 1; l >= 0; --l) {
      xv[l] = 0.0;
      if (l < N) {
        const int q = r / P;
        xv[l] = A.xk[r - q * P];
        r = q;
      }
    }
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < kGhMaxG; ++i) {
      if (i < A.G) {
        double d2 = 0.0;
#pragma unroll
        for (int l = 0; l < kGhMaxN; ++l) {
          if (l < N) {
            const double d = xv[l] - cen[i][l];
            d2 = fma(d, d, d2);
          }
        }
        v -= amp[i] * exp(-d2 * inv2s2);
      }
    }
    F[m] = v;
  }
  __syncthreads();
  // axis l has stride P^(N-1-l) in the grid index; grid / P fibres per axis
  int stride = A.grid / P;
  const int nf = A.grid / P;
  for (int l = 0; l < N; ++l) {
    for (int f = tid; f < nf; f += kChThreads) {
      const int hi = f / stride, lo = f - hi * stride;
      double *fb = F + (int64_t)hi * stride * P + lo;
      double v[kChMaxP];
#pragma unroll
      for (int k = 0; k < kChMaxP; ++k) v[k] = k < P ? fb[(int64_t)k * stride] : 0.0;
      for (int r = 0; r < P; ++r) {
        const double *c = cth + r * P;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kChMaxP; ++k)
          if (k < P) acc = fma(c[k], v[k], acc);
        fb[(int64_t)r * stride] = acc;
      }
    }
    __syncthreads();
    stride /= P;
  }
  for (int c = tid; c < A.ncoef; c += kChThreads) {
    const int dg = A.digits[c];
    int m = 0;
    for (int l = 0; l < N; ++l) m = m * P + ((dg >> (4 * (N - 1 - l))) & 15);
    coef[(int64_t)s * A.ncoef + c] = F[m];
  }
}

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_grad_f(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// C = A B (M x N, inner dimension K) with BF16 MFMA tiles 16x16x32 and FP32 accumulation.
// One workgroup per 16x16 output tile; its four waves split the K steps (wave w takes
// steps w, w + 4, ...), and their partial tiles are added in wave order through LDS, so
// the result does not depend on scheduling.  A(i, k) = A[i sa0 + k sa1], B(k, j) =
// B[k sb0 + j sb1].  Epilogues: store (plus bias), bias + SiLU (keeping Z), or the
// product with SiLU'(Zin).
template <int EPI>
__global__ void __launch_bounds__(256)
k_gemm_bf16(int M, int N, int K, const float *__restrict__ A, int64_t sa0, int64_t sa1,
            const float *__restrict__ B, int64_t sb0, int64_t sb1, float *__restrict__ C, int64_t ldc,
            const float *__restrict__ bias, float *__restrict__ Z, float *__restrict__ H,
            const float *__restrict__ Zin) {
  __shared__ float part[4][4][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tiles_n = (N + 15) / 16;
  const int ti = (int)(blockIdx.x / tiles_n), tj = (int)(blockIdx.x % tiles_n);
  const int i = ti * 16 + (lane & 15);   // A row of this lane
  const int j = tj * 16 + (lane & 15);   // B column of this lane
  const int kq = (lane >> 4) * 8;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 32 * wave; k0 < K; k0 += 128) {
    bf16x8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + kq + e;
      const float av = (i < M && k < K) ? A[(int64_t)i * sa0 + (int64_t)k * sa1] : 0.f;
      const float bv = (j < N && k < K) ? B[(int64_t)k * sb0 + (int64_t)j * sb1] : 0.f;
      a[e] = (__bf16)av;
      b[e] = (__bf16)bv;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) part[wave][r][lane] = acc[r];
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int oi = ti * 16 + (lane >> 4) * 4 + r;
    const int oj = tj * 16 + (lane & 15);
    if (oi >= M || oj >= N) continue;
    float v = part[0][r][lane];
    v += part[1][r][lane];
    v += part[2][r][lane];
    v += part[3][r][lane];
    if constexpr (EPI == kEpiStore) {
      if (bias) v += bias[oj];
      C[(int64_t)oi * ldc + oj] = v;
    } else if constexpr (EPI == kEpiBiasSilu) {
      v += bias[oj];
      Z[(int64_t)oi * ldc + oj] = v;
      H[(int64_t)oi * ldc + oj] = silu_f(v);
    } else {
      C[(int64_t)oi * ldc + oj] = v * silu_grad_f(Zin[(int64_t)oi * ldc + oj]);
    }
  }
}

// column sums of X (rows x cols) in a fixed order: out[j] = sum_i X[i][j].  A workgroup
// takes 16 columns; its 16 row groups (rows g, g + 16, ...) sum in parallel, then the
// 16 partial sums of a column are added in group order.
__global__ void __launch_bounds__(256) k_colsum(int rows, int cols, const float *__restrict__ X,
                                                float *__restrict__ out) {
  __shared__ float part[16][16];
  const int c = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int j = blockIdx.x * 16 + c;
  float s = 0.f;
  if (j < cols)
    for (int i = grp; i < rows; i += 16) s += X[(int64_t)i * cols + j];
  part[grp][c] = s;
  __syncthreads();
  if (grp != 0 || j >= cols) return;
  float t = 0.f;
#pragma unroll
  for (int g = 0; g < 16; ++g) t += part[g][c];
  out[j] = t;
}

// tn = (target - mean) / std
__global__ void k_norm_out(int64_t n, int out, const double *__restrict__ tg, const float *__restrict__ mean,
                           const float *__restrict__ sd, float *__restrict__ tn) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int j = (int)(idx % out);
  tn[idx] = (float)((tg[idx] - mean[j]) / sd[j]);
}

// d = y - t; dY = 2 d / n; loss partials: each workgroup sums d^2 over its
// kMseRows elements in a fixed order (k_mse_fin adds the partials in workgroup order)
constexpr int kMseRows = 2048;
__global__ void __launch_bounds__(256) k_mse(int64_t n, const float *__restrict__ y, const float *__restrict__ t,
                                             float *__restrict__ dy, float *__restrict__ part) {
  __shared__ float sh[256];
  float acc = 0.f;
  const float sc = 2.0f / (float)n;
  const int64_t i0 = (int64_t)blockIdx.x * kMseRows;
  const int64_t i1 = i0 + kMseRows < n ? i0 + kMseRows : n;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const float d = y[i] - t[i];
    dy[i] = sc * d;
    acc += d * d;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// loss = (sum of the partials, in order) / n
__global__ void k_mse_fin(int nparts, int64_t n, const float *__restrict__ part, float *__restrict__ loss) {
  if (threadIdx.x != 0 || !loss) return;
  float s = 0.f;
  for (int b = 0; b < nparts; ++b) s += part[b];
  *loss = s / (float)n;
}

// Adam with bias correction; the step counter *tstep is advanced by the next kernel on
// the stream (k_mlp_pack), after every thread here has read it
__global__ void __launch_bounds__(256) k_adam(int64_t n, float *__restrict__ w, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, float lr,
                                              const int32_t *__restrict__ tstep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const int t = *tstep + 1;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.f - powf(b1, (float)t));
  const float vh = vi / (1.f - powf(b2, (float)t));
  w[i] -= lr * mh / (sqrtf(vh) + eps);
}

// ---- fused forward pass ------------------------------------------------------------------
// One workgroup (16 waves) carries 16 samples through the three layers.  Activations stay
// in LDS as BF16, the operand precision of the products, so the result equals that of three
// separate products; weights come from BF16 copies laid out as the fragments need them
// (row j holds the inputs of output j).  The 16-column output tiles of a layer go round-
// robin to the waves (one tile per wave at 256 columns), so a layer costs about one
// memory latency even for a single sample.
constexpr int kFwdRows = 16;
constexpr int kFwdLd0 = 40;  // LDS row stride of the input tile (32 + 8 padding), in bf16

template <class Epi>
__device__ __forceinline__ void dense_layer(const __bf16 *A, int lda, int K, const __bf16 *__restrict__ W,
                                            int ldw, int ncols, Epi &&epi) {
  // 16-column output tiles round-robin over the block's waves; each tile's weight loads
  // for up to kPre K steps are issued together before its MFMAs
  constexpr int kPre = 8;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int row = lane & 15, kq = (lane >> 4) * 8;
  for (int t = wave; t < (ncols >> 4); t += nw) {
    const int col = t * 16 + (lane & 15);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32 * kPre) {
      bf16x8 b[kPre];
#pragma unroll
      for (int q = 0; q < kPre; ++q)
        if (k0 + 32 * q < K) b[q] = *reinterpret_cast<const bf16x8 *>(W + (int64_t)col * ldw + k0 + 32 * q + kq);
#pragma unroll
      for (int q = 0; q < kPre; ++q) {
        if (k0 + 32 * q < K) {
          const bf16x8 a = *reinterpret_cast<const bf16x8 *>(A + row * lda + k0 + 32 * q + kq);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[q], acc, 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) epi((lane >> 4) * 4 + r, col, acc[r]);
  }
}

// TRAIN = false: coef = de-normalised network output (float64).
// TRAIN = true: also writes the normalised input and the pre/post activations (float32)
// that the backward pass reads, and the normalised output y.
template <bool TRAIN>
__global__ void __launch_bounds__(1024)
k_mlp_fwd(int M, int in, int hid, int out, int outp, const double *__restrict__ x, const float *__restrict__ nrm,
          const __bf16 *__restrict__ W1b, const float *__restrict__ b1, const __bf16 *__restrict__ W2b,
          const float *__restrict__ b2, const __bf16 *__restrict__ W3b, const float *__restrict__ b3,
          double *__restrict__ coef, float *__restrict__ xn, float *__restrict__ z1, float *__restrict__ h1,
          float *__restrict__ z2, float *__restrict__ h2, float *__restrict__ yo) {
  extern __shared__ __align__(16) unsigned char fsm[];
  const int ldh = hid + 8;
  __bf16 *A0 = reinterpret_cast<__bf16 *>(fsm);
  __bf16 *H1 = A0 + kFwdRows * kFwdLd0;
  __bf16 *H2 = H1 + kFwdRows * ldh;
  const int i0 = blockIdx.x * kFwdRows;
  const float *lo = nrm, *hi = nrm + in, *mean = nrm + 2 * in, *sd = nrm + 2 * in + out;
  // inputs mapped to [-1, 1], zero beyond `in` and below the last sample
  for (int e = threadIdx.x; e < kFwdRows * 32; e += blockDim.x) {
    const int r = e >> 5, k = e & 31, i = i0 + r;
    float v = 0.f;
    if (i < M && k < in) v = (float)(2.0 * (x[(int64_t)i * in + k] - lo[k]) / ((double)hi[k] - lo[k]) - 1.0);
    A0[r * kFwdLd0 + k] = (__bf16)v;
    if (TRAIN && i < M) xn[(int64_t)i * 32 + k] = v;
  }
  __syncthreads();
  dense_layer(A0, kFwdLd0, 32, W1b, 32, hid, [&](int r, int c, float acc) {
    const float v = acc + b1[c];
    const float h = silu_f(v);
    H1[r * ldh + c] = (__bf16)h;
    const int i = i0 + r;
    if (TRAIN && i < M) {
      z1[(int64_t)i * hid + c] = v;
      h1[(int64_t)i * hid + c] = h;
    }
  });
  __syncthreads();
  dense_layer(H1, ldh, hid, W2b, hid, hid, [&](int r, int c, float acc) {
    const float v = acc + b2[c];
    const float h = silu_f(v);
    H2[r * ldh + c] = (__bf16)h;
    const int i = i0 + r;
    if (TRAIN && i < M) {
      z2[(int64_t)i * hid + c] = v;
      h2[(int64_t)i * hid + c] = h;
    }
  });
  __syncthreads();
  dense_layer(H2, ldh, hid, W3b, hid, outp, [&](int r, int c, float acc) {
    const int i = i0 + r;
    if (i >= M || c >= out) return;
    const float v = acc + b3[c];
    if (TRAIN) yo[(int64_t)i * out + c] = v;
    else coef[(int64_t)i * out + c] = (double)v * (double)sd[c] + (double)mean[c];
  });
}

// BF16 copies of the weights in the fused layout (W1 padded to 32 inputs, W3 to outp
// outputs, zeros there); optionally advances the Adam step counter afterwards.
__global__ void __launch_bounds__(256)
k_mlp_pack(int in, int hid, int out, int outp, const float *__restrict__ w, int64_t oW1, int64_t oW2, int64_t oW3,
           __bf16 *__restrict__ W1b, __bf16 *__restrict__ W2b, __bf16 *__restrict__ W3b, int32_t *tstep) {
  const int64_t n1 = (int64_t)hid * 32, n2 = (int64_t)hid * hid, n3 = (int64_t)outp * hid;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n1 + n2 + n3;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < n1) {
      const int64_t j = e >> 5, k = e & 31;
      W1b[e] = (__bf16)(k < in ? w[oW1 + j * in + k] : 0.f);
    } else if (e < n1 + n2) {
      W2b[e - n1] = (__bf16)w[oW2 + (e - n1)];
    } else {
      const int64_t f = e - n1 - n2;
      W3b[f] = (__bf16)(f / hid < out ? w[oW3 + f] : 0.f);
    }
  }
  if (tstep && blockIdx.x == 0 && threadIdx.x == 0) *tstep += 1;
}

}  // namespace hs

// ---------------------------------------------------------------------------------------
// MLP handle and C ABI
// ---------------------------------------------------------------------------------------
struct hs_mlp_s {
  int32_t in = 0, hid = 0, out = 0, kin = 32, outp = 0;  // outp: out rounded up to 64
  int64_t nparam = 0;
  // parameter offsets (floats) inside one weights array
  int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  // device block layout (bytes) for a given max batch
  int32_t max_batch = 0;
  int64_t off_w = 0, off_m = 0, off_v = 0, off_g = 0, off_norm = 0, off_t = 0, off_loss = 0,
          off_x = 0, off_z1 = 0, off_h1 = 0, off_z2 = 0, off_h2 = 0, off_y = 0, off_tn = 0,
          off_dy = 0, off_dz2 = 0, off_dz1 = 0, off_wb = 0, off_lpart = 0, dev_bytes = 0;
  void layout(int32_t mb) {
    max_batch = mb;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
      int64_t o = off;
      off = hs::align_up(off + std::max<int64_t>(bytes, 1), 256);
      return o;
    };
    off_w = take(4 * nparam);
    off_m = take(4 * nparam);
    off_v = take(4 * nparam);
    off_g = take(4 * nparam);
    off_norm = take(4 * (2 * in + 2 * out));
    off_t = take(4);
    off_loss = take(4);
    off_x = take(4 * (int64_t)mb * kin);
    off_z1 = take(4 * (int64_t)mb * hid);
    off_h1 = take(4 * (int64_t)mb * hid);
    off_z2 = take(4 * (int64_t)mb * hid);
    off_h2 = take(4 * (int64_t)mb * hid);
    off_y = take(4 * (int64_t)mb * out);
    off_tn = take(4 * (int64_t)mb * out);
    off_dy = take(4 * (int64_t)mb * out);
    off_dz2 = take(4 * (int64_t)mb * hid);
    off_dz1 = take(4 * (int64_t)mb * hid);
    off_wb = take(2 * ((int64_t)hid * 32 + (int64_t)hid * hid + (int64_t)outp * hid));
    off_lpart = take(4 * (((int64_t)mb * out + hs::kMseRows - 1) / hs::kMseRows));
    dev_bytes = off;
  }
};

namespace {

inline float *F(void *dev, int64_t off) { return reinterpret_cast<float *>(static_cast<uint8_t *>(dev) + off); }

template <int EPI>
void gemm(hipStream_t s, int M, int N, int K, const float *A, int64_t sa0, int64_t sa1, const float *B,
          int64_t sb0, int64_t sb1, float *C, int64_t ldc, const float *bias = nullptr, float *Z = nullptr,
          float *H = nullptr, const float *Zin = nullptr) {
  const int64_t tiles = (int64_t)((M + 15) / 16) * ((N + 15) / 16);
  hipLaunchKernelGGL((hs::k_gemm_bf16<EPI>), dim3((unsigned)tiles), dim3(256), 0, s, M, N, K, A, sa0, sa1, B,
                     sb0, sb1, C, ldc, bias, Z, H, Zin);
}

__bf16 *WB(void *dev, const hs_mlp_s *p, int layer) {
  __bf16 *b = reinterpret_cast<__bf16 *>(static_cast<uint8_t *>(dev) + p->off_wb);
  if (layer == 1) return b;
  if (layer == 2) return b + (int64_t)p->hid * 32;
  return b + (int64_t)p->hid * 32 + (int64_t)p->hid * p->hid;
}

void mlp_pack(hs_mlp_s *p, void *dev, int32_t *tstep, hipStream_t s) {
  const int64_t n = (int64_t)p->hid * 32 + (int64_t)p->hid * p->hid + (int64_t)p->outp * p->hid;
  const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(hs::k_mlp_pack, dim3(g), dim3(256), 0, s, p->in, p->hid, p->out, p->outp,
                     (const float *)F(dev, p->off_w), p->oW1, p->oW2, p->oW3, WB(dev, p, 1), WB(dev, p, 2),
                     WB(dev, p, 3), tstep);
}

template <bool TRAIN>
void mlp_fwd(hs_mlp_s *p, void *dev, int batch, const double *x, double *coef, hipStream_t s) {
  const float *w = F(dev, p->off_w);
  const size_t lds = sizeof(__bf16) * ((size_t)hs::kFwdRows * hs::kFwdLd0 + 2 * (size_t)hs::kFwdRows * (p->hid + 8));
  hipLaunchKernelGGL((hs::k_mlp_fwd<TRAIN>), dim3((batch + hs::kFwdRows - 1) / hs::kFwdRows), dim3(1024), lds, s,
                     batch, p->in, p->hid, p->out, p->outp, x, (const float *)F(dev, p->off_norm), WB(dev, p, 1),
                     w + p->ob1, WB(dev, p, 2), w + p->ob2, WB(dev, p, 3), w + p->ob3, coef,
                     F(dev, p->off_x), F(dev, p->off_z1), F(dev, p->off_h1), F(dev, p->off_z2), F(dev, p->off_h2),
                     F(dev, p->off_y));
}

}  // namespace

namespace {

int32_t gh_launch(int32_t N, int32_t G, int32_t D, int32_t Q, const double *geometry_host, int32_t nsamp,
                  const double *params_dev, double *coef_dev, const float *lo, const float *hi, int32_t *used,
                  hipStream_t stream) {
  using hs::GhArgs;
  if (N < 1 || N > hs::kGhMaxN || G < 1 || G > hs::kGhMaxG || D < 0 || D > hs::kGhMaxD || Q < 1 ||
      Q > hs::kGhMaxQ || nsamp < 0 || !geometry_host || (nsamp > 0 && (!params_dev || !coef_dev)))
    return hs::fail(HS_E_INVALID, "Gauss-Hermite projection: arguments out of range (N<=4, G<=4, D<=8, Q<=32)");
  GhArgs A;
  std::memset(&A, 0, sizeof(A));
  A.N = N;
  A.G = G;
  A.D = D;
  A.Q = Q;
  A.NA = (N + 1) / 2;
  A.NB = N - A.NA;
  A.QA = 1;
  for (int l = 0; l < A.NA; ++l) A.QA *= Q;
  A.QB = 1;
  for (int l = 0; l < A.NB; ++l) A.QB *= Q;
  A.nB = (int)hs::binom(A.NB + D, A.NB);
  A.ncoef = (int)hs::binom(N + D, N);
  // rows of the leading grid per LDS chunk: as many as fit in the LDS budget
  const size_t fixed = hs::GhLds::make(0, A.QB, Q, D, A.nB, A.NB, A.ncoef).bytes();
  const size_t per_row = sizeof(double) * ((size_t)A.QB + (A.NB == 2 ? (size_t)Q * (D + 1) : 0) + A.nB);
  const int64_t fit = fixed < hs::kGhLdsBytes ? (int64_t)((hs::kGhLdsBytes - fixed) / per_row) : 0;
  A.R = (int)std::min<int64_t>({(int64_t)A.QA, fit, hs::kGhChunk});
  const size_t lds = hs::GhLds::make(A.R, A.QB, Q, D, A.nB, A.NB, A.ncoef).bytes();
  if (A.R < 1 || lds > hs::kGhLdsBytes || A.ncoef > hs::kGhThreads)
    return hs::fail(HS_E_UNSUPPORTED, "Gauss-Hermite projection: workspace exceeds LDS");
  std::vector<double> xi, wq;
  if (!hs::gh_rule(Q, xi, wq))
    return hs::fail(HS_E_NONFINITE, "Gauss-Hermite rule: the bisection did not isolate the nodes");
  for (int m = 0; m < Q; ++m) {
    A.xi[m] = xi[m];
    // H_n(x) by the physicists' recurrence; scaled by w_m / (sqrt(pi) 2^n n!)
    double hm = 0.0, hc = 1.0, fact = 1.0;
    for (int n = 0; n <= D; ++n) {
      if (n > 0) fact *= n;
      A.hq[n][m] = wq[m] * hc / (std::sqrt(M_PI) * std::ldexp(1.0, n) * fact);
      const double hn = 2.0 * xi[m] * hc - 2.0 * n * hm;
      hm = hc;
      hc = hn;
    }
  }
  const double *g = geometry_host;
  for (int i = 0; i < G; ++i)
    for (int l = 0; l < N; ++l) {
      A.base[i][l] = g[i * N + l];
      A.u[i][l] = g[G * N + i * N + l];
      A.w[i][l] = g[2 * G * N + i * N + l];
    }
  for (int i = 0; i < G; ++i) A.phase[i] = g[3 * G * N + i];
  if (nsamp == 0) return HS_OK;
  hipLaunchKernelGGL(hs::k_gh_project, dim3(nsamp), dim3(hs::kGhThreads), lds, stream, A, params_dev, coef_dev,
                     lo, hi, used);
  HS_HIP(hipGetLastError());
  return HS_OK;
}

int32_t cheb_launch(int32_t N, int32_t G, int32_t D, int32_t R, double L, const double *geometry_host,
                    int32_t nsamp, const double *params_dev, double *coef_dev, hipStream_t stream) {
  using hs::ChArgs;
  if (N < 1 || N > hs::kGhMaxN || G < 1 || G > hs::kGhMaxG || D < 0 || R < 0 || R + 1 > hs::kChMaxP ||
      !(L > 0.0) || !std::isfinite(L) || nsamp < 0 || !geometry_host || (nsamp > 0 && (!params_dev || !coef_dev)))
    return hs::fail(HS_E_INVALID, "Chebyshev interpolation: arguments out of range (N<=4, G<=4, R<=15, L>0)");
  ChArgs A;
  std::memset(&A, 0, sizeof(A));
  A.N = N;
  A.G = G;
  A.P = R + 1;
  int64_t grid = 1;
  for (int l = 0; l < N; ++l) grid *= A.P;
  const size_t lds = sizeof(double) * (size_t)(grid + (int64_t)A.P * A.P);
  if (lds > hs::kChLdsBytes) return hs::fail(HS_E_UNSUPPORTED, "Chebyshev interpolation: (R + 1)^N grid exceeds LDS");
  A.grid = (int)grid;
  // requested coefficients: |r| <= D with every r_l <= R, lexicographic order
  int nc = 0;
  std::vector<int> r(N, 0);
  for (int64_t m = 0; m < grid; ++m) {
    int64_t q = m;
    int sum = 0, code = 0;
    for (int l = N - 1; l >= 0; --l) {
      r[l] = (int)(q % A.P);
      q /= A.P;
      sum += r[l];
    }
    if (sum > D) continue;
    for (int l = 0; l < N; ++l) code |= r[l] << (4 * (N - 1 - l));
    if (nc >= hs::kChMaxCoef) return hs::fail(HS_E_UNSUPPORTED, "Chebyshev interpolation: more than 512 coefficients");
    A.digits[nc++] = (uint16_t)code;
  }
  A.ncoef = nc;
  for (int k = 0; k < A.P; ++k) A.xk[k] = L * std::cos((2.0 * k + 1.0) * M_PI / (2.0 * A.P));
  const double *g = geometry_host;
  for (int i = 0; i < G; ++i)
    for (int l = 0; l < N; ++l) {
      A.base[i][l] = g[i * N + l];
      A.u[i][l] = g[G * N + i * N + l];
      A.w[i][l] = g[2 * G * N + i * N + l];
    }
  for (int i = 0; i < G; ++i) A.phase[i] = g[3 * G * N + i];
  if (nsamp == 0) return HS_OK;
  hipLaunchKernelGGL(hs::k_cheb_interp, dim3(nsamp), dim3(hs::kChThreads), lds, stream, A, params_dev, coef_dev);
  HS_HIP(hipGetLastError());
  return HS_OK;
}

}  // namespace

extern "C" {

int32_t hs_cheb_ncoef(int32_t N, int32_t D, int32_t R, int32_t *ncoef) {
  if (!ncoef || N < 1 || N > hs::kGhMaxN || D < 0 || R < 0 || R + 1 > hs::kChMaxP)
    return hs::fail(HS_E_INVALID, "hs_cheb_ncoef: bad arguments");
  int64_t grid = 1, nc = 0;
  for (int l = 0; l < N; ++l) grid *= (R + 1);
  for (int64_t m = 0; m < grid; ++m) {
    int64_t q = m;
    int sum = 0;
    for (int l = 0; l < N; ++l) {
      sum += (int)(q % (R + 1));
      q /= (R + 1);
    }
    if (sum <= D) ++nc;
  }
  *ncoef = (int32_t)nc;
  return HS_OK;
}

int32_t hs_cheb_interp(int32_t N, int32_t G, int32_t D, int32_t R, double L, const double *geometry_host,
                       int32_t nsamp, const double *params_dev, double *coef_dev, void *stream) {
  return cheb_launch(N, G, D, R, L, geometry_host, nsamp, params_dev, coef_dev,
                     static_cast<hipStream_t>(stream));
}

int32_t hs_gh_ncoef(int32_t N, int32_t D, int32_t *ncoef) {
  if (!ncoef || N < 1 || D < 0) return hs::fail(HS_E_INVALID, "hs_gh_ncoef: bad arguments");
  *ncoef = (int32_t)hs::binom(N + D, N);
  return HS_OK;
}

int32_t hs_gh_rule(int32_t Q, double *x_host, double *w_host) {
  if (Q < 1 || Q > hs::kGhMaxQ || !x_host || !w_host) return hs::fail(HS_E_INVALID, "hs_gh_rule: bad arguments");
  std::vector<double> x, w;
  if (!hs::gh_rule(Q, x, w)) return hs::fail(HS_E_NONFINITE, "hs_gh_rule: the bisection did not isolate the nodes");
  std::memcpy(x_host, x.data(), sizeof(double) * Q);
  std::memcpy(w_host, w.data(), sizeof(double) * Q);
  return HS_OK;
}

int32_t hs_gh_project(int32_t N, int32_t G, int32_t D, int32_t Q, const double *geometry_host,
                      int32_t nsamp, const double *params_dev, double *coef_dev, void *stream) {
  return gh_launch(N, G, D, Q, geometry_host, nsamp, params_dev, coef_dev, nullptr, nullptr, nullptr,
                   static_cast<hipStream_t>(stream));
}

int32_t hs_mlp_create(int32_t in, int32_t hidden, int32_t out, hs_mlp *mlp) {
  if (!mlp) return hs::fail(HS_E_INVALID, "hs_mlp_create: out is NULL");
  *mlp = nullptr;
  if (in < 1 || in > 32 || hidden < 64 || hidden > 512 || hidden % 64 || out < 1 || out > 512)
    return hs::fail(HS_E_INVALID, "hs_mlp_create: need in <= 32, hidden a multiple of 64 in 64..512, out <= 512");
  hs_mlp_s *p = new (std::nothrow) hs_mlp_s();
  if (!p) return hs::fail(HS_E_NOMEM, "hs_mlp_create: out of host memory");
  p->in = in;
  p->hid = hidden;
  p->out = out;
  p->outp = (out + 63) / 64 * 64;
  int64_t o = 0;
  p->oW1 = o;
  o += (int64_t)hidden * in;
  p->ob1 = o;
  o += hidden;
  p->oW2 = o;
  o += (int64_t)hidden * hidden;
  p->ob2 = o;
  o += hidden;
  p->oW3 = o;
  o += (int64_t)out * hidden;
  p->ob3 = o;
  o += out;
  p->nparam = o;
  *mlp = p;
  return HS_OK;
}

int32_t hs_mlp_destroy(hs_mlp mlp) {
  delete mlp;
  return HS_OK;
}

int32_t hs_mlp_device_bytes(hs_mlp mlp, int32_t max_batch, int64_t *bytes) {
  if (!mlp || !bytes || max_batch < 1) return hs::fail(HS_E_INVALID, "hs_mlp_device_bytes: bad arguments");
  mlp->layout(max_batch);
  *bytes = mlp->dev_bytes;
  return HS_OK;
}

int32_t hs_mlp_upload_params(hs_mlp mlp, void *dev, const float *weights_host, const float *norm_host,
                             void *stream) {
  if (!mlp || !dev || !weights_host || !norm_host) return hs::fail(HS_E_INVALID, "hs_mlp_upload_params: NULL argument");
  if (mlp->max_batch < 1) return hs::fail(HS_E_INVALID, "hs_mlp_upload_params: call hs_mlp_device_bytes first");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HS_HIP(hipMemcpyAsync(F(dev, mlp->off_w), weights_host, 4 * mlp->nparam, hipMemcpyHostToDevice, s));
  HS_HIP(hipMemcpyAsync(F(dev, mlp->off_norm), norm_host, 4 * (2 * mlp->in + 2 * mlp->out), hipMemcpyHostToDevice, s));
  // Adam moments and the step counter start at zero (fill kernels, no memset nodes)
  std::vector<float> zeros(mlp->nparam, 0.f);
  HS_HIP(hipMemcpyAsync(F(dev, mlp->off_m), zeros.data(), 4 * mlp->nparam, hipMemcpyHostToDevice, s));
  HS_HIP(hipMemcpyAsync(F(dev, mlp->off_v), zeros.data(), 4 * mlp->nparam, hipMemcpyHostToDevice, s));
  HS_HIP(hipMemcpyAsync(F(dev, mlp->off_t), zeros.data(), 4, hipMemcpyHostToDevice, s));
  mlp_pack(mlp, dev, nullptr, s);
  HS_HIP(hipGetLastError());
  HS_HIP(hipStreamSynchronize(s));  // the host staging above is pageable and short-lived
  return HS_OK;
}

int32_t hs_mlp_download_params(hs_mlp mlp, const void *dev, float *weights_host, void *stream) {
  if (!mlp || !dev || !weights_host) return hs::fail(HS_E_INVALID, "hs_mlp_download_params: NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HS_HIP(hipMemcpyAsync(weights_host, F(const_cast<void *>(dev), mlp->off_w), 4 * mlp->nparam,
                        hipMemcpyDeviceToHost, s));
  HS_HIP(hipStreamSynchronize(s));
  return HS_OK;
}

int32_t hs_mlp_predict(hs_mlp mlp, void *dev, int32_t batch, const double *x_dev, double *coef_dev,
                       void *stream) {
  if (!mlp || !dev || !x_dev || !coef_dev) return hs::fail(HS_E_INVALID, "hs_mlp_predict: NULL argument");
  if (batch < 1 || batch > mlp->max_batch) return hs::fail(HS_E_WORKSPACE, "hs_mlp_predict: batch above max_batch");
  hipStream_t s = static_cast<hipStream_t>(stream);
  mlp_fwd<false>(mlp, dev, batch, x_dev, coef_dev, s);  // one launch: normalise, 3 layers, de-normalise
  HS_HIP(hipGetLastError());
  return HS_OK;
}

int32_t hs_sur_coeffs(hs_mlp mlp, void *dev, int32_t N, int32_t G, int32_t D, int32_t Q,
                      const double *geometry_host, int32_t nsamp, const double *params_dev, double *coef_dev,
                      int32_t *used_quad_dev, void *stream) {
  if (!mlp || !dev) return hs::fail(HS_E_INVALID, "hs_sur_coeffs: NULL network");
  if (mlp->in != G + 4 || N < 1 || D < 0 || mlp->out != (int32_t)hs::binom(N + D, N))
    return hs::fail(HS_E_INVALID, "hs_sur_coeffs: network shape does not match (4 + G inputs, C(N+D, N) outputs)");
  if (nsamp == 0) return HS_OK;
  int32_t st = hs_mlp_predict(mlp, dev, nsamp, params_dev, coef_dev, stream);
  if (st != HS_OK) return st;
  const float *nrm = F(dev, mlp->off_norm);
  return gh_launch(N, G, D, Q, geometry_host, nsamp, params_dev, coef_dev, nrm, nrm + mlp->in, used_quad_dev,
                   static_cast<hipStream_t>(stream));
}

int32_t hs_mlp_train_step(hs_mlp mlp, void *dev, int32_t batch, const double *x_dev, const double *target_dev,
                          float lr, float *loss_dev, float *grads_dev, void *stream) {
  if (!mlp || !dev || !x_dev || !target_dev) return hs::fail(HS_E_INVALID, "hs_mlp_train_step: NULL argument");
  if (batch < 1 || batch > mlp->max_batch) return hs::fail(HS_E_WORKSPACE, "hs_mlp_train_step: batch above max_batch");
  if (!std::isfinite(lr)) return hs::fail(HS_E_NONFINITE, "hs_mlp_train_step: lr not finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int in = mlp->in, hid = mlp->hid, out = mlp->out, kin = mlp->kin;
  float *w = F(dev, mlp->off_w), *g = grads_dev ? grads_dev : F(dev, mlp->off_g);
  const float *nrm = F(dev, mlp->off_norm);
  const int64_t ny = (int64_t)batch * out;
  hipLaunchKernelGGL(hs::k_norm_out, dim3((unsigned)((ny + 255) / 256)), dim3(256), 0, s, ny, out, target_dev,
                     nrm + 2 * in, nrm + 2 * in + out, F(dev, mlp->off_tn));
  // forward in one launch, keeping the normalised input and the activations
  mlp_fwd<true>(mlp, dev, batch, x_dev, nullptr, s);
  const int nmse = (int)((ny + hs::kMseRows - 1) / hs::kMseRows);
  hipLaunchKernelGGL(hs::k_mse, dim3(nmse), dim3(256), 0, s, ny, F(dev, mlp->off_y), F(dev, mlp->off_tn),
                     F(dev, mlp->off_dy), F(dev, mlp->off_lpart));
  hipLaunchKernelGGL(hs::k_mse_fin, dim3(1), dim3(64), 0, s, nmse, ny, (const float *)F(dev, mlp->off_lpart),
                     loss_dev ? loss_dev : F(dev, mlp->off_loss));
  float *dy = F(dev, mlp->off_dy), *h2 = F(dev, mlp->off_h2), *h1 = F(dev, mlp->off_h1);
  float *dz2 = F(dev, mlp->off_dz2), *dz1 = F(dev, mlp->off_dz1), *xn = F(dev, mlp->off_x);
  // layer 3: dW3 = dY^T H2, db3 = colsum dY, dZ2 = (dY W3) * silu'(Z2)
  gemm<hs::kEpiStore>(s, out, hid, batch, dy, 1, out, h2, hid, 1, g + mlp->oW3, hid);
  hipLaunchKernelGGL(hs::k_colsum, dim3((out + 15) / 16), dim3(256), 0, s, batch, out, dy, g + mlp->ob3);
  gemm<hs::kEpiSiluGrad>(s, batch, hid, out, dy, out, 1, w + mlp->oW3, hid, 1, dz2, hid, nullptr, nullptr, nullptr,
                         F(dev, mlp->off_z2));
  // layer 2
  gemm<hs::kEpiStore>(s, hid, hid, batch, dz2, 1, hid, h1, hid, 1, g + mlp->oW2, hid);
  hipLaunchKernelGGL(hs::k_colsum, dim3((hid + 15) / 16), dim3(256), 0, s, batch, hid, dz2, g + mlp->ob2);
  gemm<hs::kEpiSiluGrad>(s, batch, hid, hid, dz2, hid, 1, w + mlp->oW2, hid, 1, dz1, hid, nullptr, nullptr, nullptr,
                         F(dev, mlp->off_z1));
  // layer 1
  gemm<hs::kEpiStore>(s, hid, in, batch, dz1, 1, hid, xn, kin, 1, g + mlp->oW1, in);
  hipLaunchKernelGGL(hs::k_colsum, dim3((hid + 15) / 16), dim3(256), 0, s, batch, hid, dz1, g + mlp->ob1);
  // Adam
  const unsigned ab = (unsigned)((mlp->nparam + 255) / 256);
  hipLaunchKernelGGL(hs::k_adam, dim3(ab), dim3(256), 0, s, mlp->nparam, w, (const float *)g, F(dev, mlp->off_m),
                     F(dev, mlp->off_v), lr, (const int32_t *)F(dev, mlp->off_t));
  // refresh the BF16 copies used by the forward pass, then advance the step counter
  mlp_pack(mlp, dev, (int32_t *)F(dev, mlp->off_t), s);
  HS_HIP(hipGetLastError());
  return HS_OK;
}

}  // extern "C"
