// One-workgroup time step for small sets (paper Sec. 2.1 eq. expMPR, Sec. 2.2, Fig. 4):
// the whole Lanczos step -- beta_0 = ||c||, m applications of H by the fused row code,
// the inner products, one classical Gram-Schmidt pass, the breakdown test,
// exp(-i h T_m) e_1 and the combination c <- V_m y -- in a single launch of 1024 threads.
// The general step issues about six launches per Krylov vector; for a set of up to 1024
// rows those launches, not the arithmetic, set the time of a step, and one compute unit
// does the whole step faster (one row per thread, so a row's values stay in registers
// from its H application to the normalised next vector).  The arithmetic is that of the general step
// (the same recurrences and breakdown rule), with the Krylov vectors stored normalised
// and every reduction summed in one fixed order (per wave, then the waves in order), so
// a step repeats bit for bit.
#pragma once

#include "lanczos.h"
#include "matvec_long.h"

namespace hs {

constexpr int kSmallThreads = kMaxM * kMaxM;  // the small exponential maps one thread per entry
constexpr int kSmallWaves = kSmallThreads / 64;
constexpr int kSmallDots = 8;                 // inner products per pass over the rows (16 sums)
constexpr int kSmallRowsPerThread = 1;       // rows per thread: sets of at most 1024 rows

// out[q] = sum over the block of v[q], q < NQ; out is in LDS and visible to every thread
// on return
template <int NQ>
__device__ __forceinline__ void small_sums(const double (&v)[NQ], double *red, double *out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double s = v[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[q * kSmallWaves + wave] = s;
  }
  __syncthreads();
  if (threadIdx.x < NQ) {
    double s = 0.0;
    for (int w = 0; w < kSmallWaves; ++w) s += red[threadIdx.x * kSmallWaves + w];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// out[q] = sum over the block of v[q] for the 2 kSmallDots = 16 values of the inner
// products: a reduce-scatter butterfly inside each wave (at the exchange across lane bit
// b a lane keeps one half of its values and sends the other half, so after bits 5..2 lane
// l holds value (l >> 2) summed over the lanes that differ in those bits; two full
// exchanges over bits 1 and 0 finish the wave), then the wave sums in wave order.
// 17 exchanges instead of the 96 of one butterfly per value; a fixed summation order.
__device__ __forceinline__ void small_sums16(const double (&v)[16], double *red, double *out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double a8[8], a4[4], a2[2];
  {
    const bool hi = (lane & 32) != 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) a8[i] = (hi ? v[i + 8] : v[i]) + __shfl_xor(hi ? v[i] : v[i + 8], 32, 64);
  }
  {
    const bool hi = (lane & 16) != 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) a4[i] = (hi ? a8[i + 4] : a8[i]) + __shfl_xor(hi ? a8[i] : a8[i + 4], 16, 64);
  }
  {
    const bool hi = (lane & 8) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) a2[i] = (hi ? a4[i + 2] : a4[i]) + __shfl_xor(hi ? a4[i] : a4[i + 2], 8, 64);
  }
  const bool hi = (lane & 4) != 0;
  double a1 = (hi ? a2[1] : a2[0]) + __shfl_xor(hi ? a2[0] : a2[1], 4, 64);
  a1 += __shfl_xor(a1, 2, 64);
  a1 += __shfl_xor(a1, 1, 64);
  if ((lane & 3) == 0) red[(lane >> 2) * kSmallWaves + wave] = a1;
  __syncthreads();
  if (threadIdx.x < 16) {
    double s = 0.0;
    for (int w = 0; w < kSmallWaves; ++w) s += red[threadIdx.x * kSmallWaves + w];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// c (complex128, in place) <- one step; V: m vectors of the workspace (stride elements
// apart), written so that the neighbour gathers of the next H application and the final
// combination can read them; sc: the step's scalar block (beta0, m_eff, alpha, beta and y
// are left there as by the general step).  Thread t owns rows t, t + 1024, ... (at most
// kSmallRowsPerThread of them; more per thread spill registers) and keeps their H v_k
// values and tile records in registers from the H application to the normalised next
// vector.
template <typename T, int N, int NP, bool X2>
__global__ void __launch_bounds__(kSmallThreads)
k_step_small(IndexDev ix, const double *__restrict__ hh, double2 *__restrict__ c,
             typename V2<T>::t *__restrict__ V, int64_t stride, double h, int m, int reorth, double tol,
             double *__restrict__ sc, double *__restrict__ t_adv, double *__restrict__ diag) {
  using C = typename V2<T>::t;
  constexpr int RS = rec_stride(NP);
  constexpr int R = kSmallRowsPerThread;
  __shared__ double red[2 * kSmallDots * kSmallWaves];
  __shared__ double res[2 * kSmallDots];
  __shared__ double dre[kMaxM], dim[kMaxM], alpha[kMaxM], beta[kMaxM];
  const int tid = threadIdx.x;
  const int32_t n = (int32_t)ix.size;
  const int32_t *__restrict__ rec[R];
  int32_t off[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int32_t r = tid + j * kSmallThreads;
    rec[j] = nullptr;
    off[j] = 0;
    if (r < n) {
      rec[j] = ix.recs + (int64_t)ix.tile_rec[ix.rowtile[r]] * RS;
      off[j] = r - rec[j][0];
    }
  }

  double a0[1] = {0.0};
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int32_t r = tid + j * kSmallThreads;
    if (r < n) {
      const double2 v = c[r];
      a0[0] = fma(v.x, v.x, fma(v.y, v.y, a0[0]));
    }
  }
  small_sums<1>(a0, red, res);
  const double b0 = sqrt(res[0]);
  int meff = 0;
  if (b0 > 0.0) {
    const double inv0 = 1.0 / b0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int32_t r = tid + j * kSmallThreads;
      if (r < n) {
        const double2 v = c[r];
        C o;
        o.x = (T)(v.x * inv0);
        o.y = (T)(v.y * inv0);
        V[r] = o;
      }
    }
    __syncthreads();
    meff = m;
    for (int k = 0; k < m; ++k) {
      const C *Vk = V + (int64_t)k * stride;
      // w = H v_k, less beta_{k-1} v_{k-1} in the plain recurrence (with the Gram-Schmidt
      // pass the projection removes that component anyway)
      const bool sub_prev = (k > 0) && !reorth;
      const C *prev = sub_prev ? V + (int64_t)(k - 1) * stride : nullptr;
      const T pcoef = sub_prev ? (T)beta[k - 1] : T(0);
      C w[R];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        w[j] = vz<T>();
        if (rec[j]) w[j] = hh_row_value<T, N, NP, X2, false>(ix, hh, Vk, rec[j], off[j], T(1), prev, pcoef);
      }
      // d_q = <v_q, w> for q = lo..k over the thread's own rows (the last step needs
      // alpha_k only)
      const bool last = (k == m - 1);
      const int lo = (reorth && !last) ? 0 : k;
      for (int q0 = lo; q0 <= k; q0 += kSmallDots) {
        const int cnt = min(kSmallDots, k + 1 - q0);
        double p[2 * kSmallDots];
#pragma unroll
        for (int q = 0; q < 2 * kSmallDots; ++q) p[q] = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const int32_t r = tid + j * kSmallThreads;
          if (r < n) {
            const double wr = w[j].x, wi = w[j].y;
#pragma unroll
            for (int q = 0; q < kSmallDots; ++q) {
              if (q < cnt) {
                const C v = V[(int64_t)(q0 + q) * stride + r];
                const double vr = v.x, vi = v.y;
                p[2 * q] = fma(vr, wr, fma(vi, wi, p[2 * q]));
                p[2 * q + 1] = fma(vr, wi, fma(-vi, wr, p[2 * q + 1]));
              }
            }
          }
        }
        small_sums16(p, red, res);
        if (tid < cnt) {
          dre[q0 + tid] = res[2 * tid];
          dim[q0 + tid] = res[2 * tid + 1];
        }
        __syncthreads();
      }
      const double ak = dre[k];  // alpha_k = Re <v_k, w>
      if (tid == 0) alpha[k] = ak;
      if (last) break;
      double a2[1] = {0.0};
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int32_t r = tid + j * kSmallThreads;
        if (r < n) {
          double wr = w[j].x, wi = w[j].y;
          if (reorth) {
            for (int q = lo; q <= k; ++q) {
              const C v = V[(int64_t)q * stride + r];
              const double vr = v.x, vi = v.y;
              wr -= dre[q] * vr - dim[q] * vi;
              wi -= dre[q] * vi + dim[q] * vr;
            }
          } else {
            const C v = V[(int64_t)k * stride + r];
            wr -= ak * (double)v.x;
            wi -= ak * (double)v.y;
          }
          w[j].x = (T)wr;
          w[j].y = (T)wi;
          const double qr = w[j].x, qi = w[j].y;
          a2[0] = fma(qr, qr, fma(qi, qi, a2[0]));
        }
      }
      small_sums<1>(a2, red, res);
      const double b = sqrt(res[0]);
      // breakdown against ||T_{k+1}||_inf (alpha_k taken from dre: alpha[k] is written by
      // one thread and read by the others only after the next barrier)
      double tn = 0.0;
      for (int i = 0; i <= k; ++i) {
        double row = fabs(i == k ? ak : alpha[i]);
        if (i >= 1) row += beta[i - 1];
        if (i < k) row += beta[i];
        tn = fmax(tn, row);
      }
      if (b <= tol * fmax(1.0, tn)) {  // the same value in every thread: a uniform exit
        meff = k + 1;
        break;
      }
      if (tid == 0) beta[k] = b;
      const double ib = 1.0 / b;
      C *Vn = V + (int64_t)(k + 1) * stride;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int32_t r = tid + j * kSmallThreads;
        if (r < n) {
          C o;
          o.x = (T)(w[j].x * ib);
          o.y = (T)(w[j].y * ib);
          Vn[r] = o;
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (tid == 0) {
    sc[Scal::beta0] = b0;
    sc[Scal::meff] = meff;
    for (int i = 0; i < kMaxM; ++i) {
      sc[Scal::alpha + i] = i < meff ? alpha[i] : 0.0;
      sc[Scal::beta + i] = i + 1 < meff ? beta[i] : 0.0;
    }
  }
  __syncthreads();
  small_expm_block(h, sc);  // y = beta0 exp(-i h T_meff) e_1 into sc (nothing for meff = 0)
  __syncthreads();
  if (meff > 0) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const int32_t r = tid + j * kSmallThreads;
      if (r < n) {
        double cr = 0.0, ci = 0.0;
        for (int q = 0; q < meff; ++q) {
          const double yr = sc[Scal::yre + q], yi = sc[Scal::yim + q];
          const C v = V[(int64_t)q * stride + r];
          cr += yr * v.x - yi * v.y;
          ci += yr * v.y + yi * v.x;
        }
        c[r] = make_double2(cr, ci);
      }
    }
  }
  if (tid == 0) {
    if (t_adv) *t_adv += h;
    if (diag) {
      diag[0] = meff;
      for (int i = 0; i < m; ++i) {
        diag[1 + i] = sc[Scal::alpha + i];
        diag[1 + m + i] = sc[Scal::beta + i];
      }
    }
  }
}

// 1 if the step was launched, 0 if this set has no specialised row code (the caller then
// takes the general step)
template <typename T>
int launch_step_small_impl(const IndexDev &ix, const double *hh, void *c, void *V, int64_t stride, double h,
                           int m, int reorth, double tol, double *sc, double *t_adv, double *diag, hipStream_t s,
                           bool x2) {
  using C = typename V2<T>::t;
  if (!ix.tile_rec || ix.rstride != rec_stride(ix.np) || ix.size > (int64_t)kSmallThreads * kSmallRowsPerThread)
    return 0;
  if (m < 1 || m > kMaxM) return 0;
#define HS_SMALL_CASE(NN, PP)                                                                            \
  case NN * 32 + PP:                                                                                     \
    if (x2)                                                                                              \
      hipLaunchKernelGGL((k_step_small<T, NN, PP, true>), dim3(1), dim3(kSmallThreads), 0, s, ix, hh,  \
                         (double2 *)c, (C *)V, stride, h, m, reorth, tol, sc, t_adv, diag);     \
    else                                                                                                 \
      hipLaunchKernelGGL((k_step_small<T, NN, PP, false>), dim3(1), dim3(kSmallThreads), 0, s, ix, hh, \
                         (double2 *)c, (C *)V, stride, h, m, reorth, tol, sc, t_adv, diag);     \
    return 1;
  switch (ix.N * 32 + ix.np) {
    HS_SMALL_CASE(1, 0)
    HS_SMALL_CASE(2, 0)
    HS_SMALL_CASE(3, 1)
    HS_SMALL_CASE(4, 2)
    HS_SMALL_CASE(5, 2)
    HS_SMALL_CASE(6, 3)
    HS_SMALL_CASE(7, 4)
    HS_SMALL_CASE(8, 5)
    default:
      return 0;
  }
#undef HS_SMALL_CASE
}

}  // namespace hs
