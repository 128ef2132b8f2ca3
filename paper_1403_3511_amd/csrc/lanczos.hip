// Short-iterative Lanczos step for the exponential midpoint rule (paper Sec. 2.1 eq.
// expMPR, Sec. 2.2, Fig. 4 time_propagation), for one instance or many at once:
//   coefficients at t + h/2; beta_0 = ||c||, v_1 = c / beta_0;
//   w = H v_k - beta_{k-1} v_{k-1}; alpha_k = Re <v_k, w>;
//   w -= alpha_k v_k  (or, with reorthogonalisation, w -= sum_{i<=k} <v_i, w> v_i);
//   beta_k = ||w||; v_{k+1} = w / beta_k;
//   y = beta_0 exp(-i h T_m) e_1 on the device; c <- V_m y.
// Every scalar stays on the device; no host synchronisation inside a step, so a step
// can be captured into a HIP graph.
//
// Vectors of all instances are packed back to back and cut into segments of at most
// kSeg rows that belong to one instance.  A reduction writes one partial per segment
// and a finishing block per instance adds its segments' partials in a fixed tree, so
// results do not depend on scheduling and repeat bit for bit.
#include <algorithm>
#include <atomic>

#include "lanczos.h"

namespace hs {

// Sum over the block in a fixed order: butterfly inside each wave, then the wave sums in
// wave order.  Every thread receives the result.  sh needs blockDim.x / 64 doubles.
__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r += sh[i];
  __syncthreads();
  return r;
}

// sum of part[s0..s1) by one block in a fixed order
__device__ __forceinline__ double seg_sum(const double *__restrict__ part, int64_t s0, int64_t s1,
                                          double *sh) {
  double acc = 0.0;
  for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) acc += part[s];
  return block_sum(acc, sh);
}

template <typename T> struct CT;
template <> struct CT<double> { using t = double2; };
template <> struct CT<float> { using t = float2; };

// Streaming accesses of the Krylov vectors, marked non-temporal so that they do not
// push the index metadata and the current vector out of the caches between H
// applications.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 nt_ld(const double2 *p) {
  const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(p));
  return make_double2(v[0], v[1]);
}
__device__ __forceinline__ float2 nt_ld(const float2 *p) {
  const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(p));
  return make_float2(v[0], v[1]);
}
__device__ __forceinline__ void nt_st(double2 *p, double2 v) {
  d2v t;
  t[0] = v.x;
  t[1] = v.y;
  __builtin_nontemporal_store(t, reinterpret_cast<d2v *>(p));
}
__device__ __forceinline__ void nt_st(float2 *p, float2 v) {
  f2v t;
  t[0] = v.x;
  t[1] = v.y;
  __builtin_nontemporal_store(t, reinterpret_cast<f2v *>(p));
}

// Krylov vectors are stored unnormalised: v_q = s_q V_q with s_0 = 1 (the start vector
// is normalised when written) and s_q = 1 / beta_{q-1}.
__device__ __forceinline__ double vscale(const double *sc, int q) {
  return q == 0 ? 1.0 : sc[Scal::inv + q - 1];
}

// ---- per-segment kernels -------------------------------------------------------------
__global__ void __launch_bounds__(kSegThreads)
k_snorm2_part(SegView sv, const double2 *__restrict__ c, double *__restrict__ part) {
  __shared__ double sh[kSegThreads];
  int inst, len;
  int64_t r0;
  sv.get(blockIdx.x, inst, r0, len);
  double acc = 0.0;
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    const double2 v = nt_ld(c + r0 + i);
    acc = fma(v.x, v.x, fma(v.y, v.y, acc));
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kSegThreads)
k_sfin_beta0(SegView sv, const double *__restrict__ part, double *__restrict__ scall) {
  __shared__ double sh[kSegThreads];
  int64_t s0, s1;
  sv.range(blockIdx.x, s0, s1);
  const double s = seg_sum(part, s0, s1, sh);
  if (threadIdx.x == 0) {
    double *sc = scall + (int64_t)blockIdx.x * Scal::size;
    const double b = sqrt(s);
    sc[Scal::beta0] = b;
    sc[Scal::inv0] = b > 0.0 ? 1.0 / b : 0.0;
    sc[Scal::stop] = b > 0.0 ? 0.0 : 1.0;
    sc[Scal::meff] = 0.0;
    for (int k = 0; k < kMaxM; ++k) {
      sc[Scal::alpha + k] = 0.0;
      sc[Scal::beta + k] = 0.0;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kSegThreads)
k_sstart(SegView sv, const double2 *__restrict__ c, typename CT<T>::t *__restrict__ v,
         const double *__restrict__ scall) {
  int inst, len;
  int64_t r0;
  sv.get(blockIdx.x, inst, r0, len);
  const double s = scall[(int64_t)inst * Scal::size + Scal::inv0];
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    const double2 a = nt_ld(c + r0 + i);
    typename CT<T>::t o;
    o.x = (T)(a.x * s);
    o.y = (T)(a.y * s);
    v[r0 + i] = o;
  }
}

// partial <V_q, W> = sum conj(V_q) W for q = lo .. lo+cnt-1
template <typename T>
__global__ void __launch_bounds__(kSegThreads)
k_sdots_part(SegView sv, const typename CT<T>::t *__restrict__ V, int64_t stride, int lo, int cnt,
             const typename CT<T>::t *__restrict__ W, double *__restrict__ part,
             const double *__restrict__ scall) {
  __shared__ double sh[kSegThreads];
  int inst, len;
  int64_t r0;
  sv.get(blockIdx.x, inst, r0, len);
  if (scall[(int64_t)inst * Scal::size + Scal::stop] != 0.0) return;
  double ar[kDotChunk], ai[kDotChunk];
#pragma unroll
  for (int q = 0; q < kDotChunk; ++q) ar[q] = ai[q] = 0.0;
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    const int64_t r = r0 + i;
    const typename CT<T>::t wv = nt_ld(W + r);
    const double wr = wv.x, wi = wv.y;
#pragma unroll
    for (int q = 0; q < kDotChunk; ++q) {
      if (q < cnt) {
        const typename CT<T>::t v = nt_ld(V + (int64_t)(lo + q) * stride + r);
        const double vr = v.x, vi = v.y;
        ar[q] = fma(vr, wr, fma(vi, wi, ar[q]));
        ai[q] = fma(vr, wi, fma(-vi, wr, ai[q]));
      }
    }
  }
  for (int q = 0; q < cnt; ++q) {
    const double sr = block_sum(ar[q], sh);
    const double si = block_sum(ai[q], sh);
    if (threadIdx.x == 0) {
      part[(int64_t)(2 * q) * sv.nseg + blockIdx.x] = sr;
      part[(int64_t)(2 * q + 1) * sv.nseg + blockIdx.x] = si;
    }
  }
}

// one block per (instance, partial sum q): q = 2 i + (0: real, 1: imaginary) of
// <V_{lo+i}, W>
__global__ void __launch_bounds__(kSegThreads)
k_sfin_dots(SegView sv, const double *__restrict__ part, int lo, int cnt, int k,
            double *__restrict__ scall) {
  __shared__ double sh[kSegThreads / 64];
  double *sc = scall + (int64_t)blockIdx.x * Scal::size;
  if (sc[Scal::stop] != 0.0) return;
  const int q = blockIdx.y;
  int64_t s0, s1;
  sv.range(blockIdx.x, s0, s1);
  const int idx = lo + q / 2;
  const double s = seg_sum(part + (int64_t)q * sv.nseg, s0, s1, sh) * vscale(sc, idx);
  if (threadIdx.x == 0) {
    if (q & 1) sc[Scal::dim + idx] = s; else sc[Scal::dre + idx] = s;
    if (!(q & 1) && idx == k) sc[Scal::alpha + k] = s;  // alpha_k = Re <v_k, w>
  }
}

// Wout = W - sum_q d_q v_q over q in [lo, k] (reorth) or W - alpha_k v_k, with the
// stored Krylov vectors scaled on read (v_q = s_q V_q); ||Wout||^2 partials.  Wout is the
// next stored Krylov vector: it is never normalised in memory.
template <typename T>
__global__ void __launch_bounds__(kSegThreads)
k_supdate(SegView sv, const typename CT<T>::t *__restrict__ V, int64_t stride, int lo, int k,
          int reorth, const typename CT<T>::t *__restrict__ W, typename CT<T>::t *__restrict__ Wout,
          double *__restrict__ part, const double *__restrict__ scall) {
  using C = typename CT<T>::t;
  __shared__ double sh[kSegThreads / 64];
  __shared__ double cre[kMaxM], cim[kMaxM];
  int inst, len;
  int64_t r0;
  sv.get(blockIdx.x, inst, r0, len);
  const double *sc = scall + (int64_t)inst * Scal::size;
  if (sc[Scal::stop] != 0.0) return;  // uniform over the block (one instance)
  // projection coefficients with the stored vectors' scales folded in: d_q s_q over
  // q = q0 .. q0 + cnt - 1 (reorth), or alpha_k s_k alone
  const int q0 = reorth ? lo : k;
  const int cnt = reorth ? k + 1 - lo : 1;
  if ((int)threadIdx.x < cnt) {
    const int q = q0 + threadIdx.x;
    const double vs = vscale(sc, q);
    cre[threadIdx.x] = (reorth ? sc[Scal::dre + q] : sc[Scal::alpha + k]) * vs;
    cim[threadIdx.x] = reorth ? sc[Scal::dim + q] * vs : 0.0;
  }
  __syncthreads();
  double acc = 0.0;
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    const int64_t r = r0 + i;
    const C wv = nt_ld(W + r);
    double wr = wv.x, wi = wv.y;
    // kDotChunk vectors per round, their loads issued together
    for (int c0 = 0; c0 < cnt; c0 += kDotChunk) {
      C v[kDotChunk];
#pragma unroll
      for (int q = 0; q < kDotChunk; ++q) {
        if (c0 + q < cnt) v[q] = nt_ld(V + (int64_t)(q0 + c0 + q) * stride + r);
        else v[q].x = v[q].y = T(0);
      }
#pragma unroll
      for (int q = 0; q < kDotChunk; ++q) {
        if (c0 + q < cnt) {
          const double dr = cre[c0 + q], di = cim[c0 + q];
          const double vr = v[q].x, vi = v[q].y;
          wr -= dr * vr - di * vi;
          wi -= dr * vi + di * vr;
        }
      }
    }
    C o;
    o.x = (T)wr;
    o.y = (T)wi;
    Wout[r] = o;
    const double qr = o.x, qi = o.y;
    acc = fma(qr, qr, fma(qi, qi, acc));
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// beta_k = ||W||; breakdown test against ||T_{k+1}||_inf
__global__ void __launch_bounds__(kSegThreads)
k_sfin_beta(SegView sv, const double *__restrict__ part, int k, int m, double tol,
            double *__restrict__ scall) {
  __shared__ double sh[kSegThreads];
  double *sc = scall + (int64_t)blockIdx.x * Scal::size;
  if (sc[Scal::stop] != 0.0) return;
  int64_t s0, s1;
  sv.range(blockIdx.x, s0, s1);
  const double s = seg_sum(part, s0, s1, sh);
  if (threadIdx.x == 0) {
    const double b = sqrt(s);
    sc[Scal::meff] = k + 1;
    if (k == m - 1) {
      sc[Scal::stop] = 1.0;  // last step: T_m complete
      return;
    }
    double tn = 0.0;
    for (int i = 0; i <= k; ++i) {
      double row = fabs(sc[Scal::alpha + i]);
      if (i >= 1) row += sc[Scal::beta + i - 1];
      if (i < k) row += sc[Scal::beta + i];
      tn = fmax(tn, row);
    }
    if (b <= tol * fmax(1.0, tn)) {
      sc[Scal::stop] = 1.0;  // breakdown: keep T_{k+1}
      return;
    }
    sc[Scal::beta + k] = b;
    sc[Scal::inv + k] = 1.0 / b;
  }
}

// exp(-i h T) e1 beta0 for instance blockIdx.x
__global__ void __launch_bounds__(1024) k_small_expm(double h, double *__restrict__ scall) {
  small_expm_block(h, scall + (int64_t)blockIdx.x * Scal::size);
}

// c = sum_{k < m_eff} y_k V_k (complex128 result)
template <typename T>
__global__ void __launch_bounds__(kSegThreads)
k_scombine(SegView sv, const typename CT<T>::t *__restrict__ V, int64_t stride, int m,
           double2 *__restrict__ c, const double *__restrict__ scall) {
  int inst, len;
  int64_t r0;
  sv.get(blockIdx.x, inst, r0, len);
  const double *sc = scall + (int64_t)inst * Scal::size;
  const int me = (int)sc[Scal::meff];
  if (me <= 0) return;  // a zero vector stays zero
  for (int i = threadIdx.x; i < len; i += blockDim.x) {
    const int64_t r = r0 + i;
    double cr = 0.0, ci = 0.0;
    for (int k = 0; k < me && k < m; ++k) {
      const double vs = vscale(sc, k);
      const double yr = sc[Scal::yre + k] * vs, yi = sc[Scal::yim + k] * vs;
      const typename CT<T>::t v = nt_ld(V + (int64_t)k * stride + r);
      cr += yr * v.x - yi * v.y;
      ci += yr * v.y + yi * v.x;
    }
    nt_st(c + r, make_double2(cr, ci));
  }
}

__global__ void k_advance_time(double *t_dev, double h, const double *__restrict__ sc,
                               double *__restrict__ diag, int m) {
  if (threadIdx.x != 0) return;
  if (t_dev) *t_dev += h;
  if (diag) {
    diag[0] = sc[Scal::meff];
    for (int k = 0; k < m; ++k) {
      diag[1 + k] = sc[Scal::alpha + k];
      diag[1 + m + k] = sc[Scal::beta + k];
    }
  }
}

// ---- two-stage Gauss-Legendre Magnus operator (paper Sec. 2.1, eq. 2stageMagnus) -------
// With Omega = -i h M, M = (A_1 + A_2)/2 - i g (A_2 A_1 - A_1 A_2), g = sqrt(3) h / 12.
// Given u1 = A_1 v, u2 = A_2 v, z = A_2 u1 and w = A_1 u2 (w is overwritten):
//   w <- (u1 + u2)/2 - i g (z - w) - prev_coef * prev_scale * prev.
// -i g (a + i b) = g b - i g a.
template <typename T>
__global__ void __launch_bounds__(256)
k_m4_combine(int64_t n, const typename CT<T>::t *__restrict__ u1, const typename CT<T>::t *__restrict__ u2,
             const typename CT<T>::t *__restrict__ z, typename CT<T>::t *__restrict__ w, double g,
             const typename CT<T>::t *__restrict__ prev, const double *__restrict__ prev_coef,
             const double *__restrict__ prev_scale) {
  using C = typename CT<T>::t;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const C a = nt_ld(u1 + r), b = nt_ld(u2 + r), zz = nt_ld(z + r), ww = nt_ld(w + r);
  const T gg = (T)g;
  const T dre = zz.x - ww.x, dim = zz.y - ww.y;
  C o;
  o.x = (T)0.5 * (a.x + b.x) + gg * dim;
  o.y = (T)0.5 * (a.y + b.y) - gg * dre;
  if (prev) {
    const T pc = (T)(*prev_coef * (prev_scale ? *prev_scale : 1.0));
    const C pv = nt_ld(prev + r);
    o.x -= pc * pv.x;
    o.y -= pc * pv.y;
  }
  nt_st(w + r, o);
}

// ---- host side --------------------------------------------------------------------------
StepLayout step_layout(int64_t rows, int64_t nseg, int n, int64_t elem_bytes, int m,
                       int64_t apply_ws) {
  StepLayout L;
  L.vec_stride = align_up(rows * elem_bytes, 256);
  int64_t off = 0;
  L.off_V = off;
  off += L.vec_stride * m;
  L.off_W = off;
  off += L.vec_stride;
  L.off_apply = off;
  off += align_up(apply_ws, 256);
  L.off_part = off;
  off += align_up(8 * std::max<int64_t>(nseg, 1) * 2 * kDotChunk, 256);
  L.off_sc = off;
  off += align_up(8 * (int64_t)Scal::size * n, 256);
  L.total = off;
  return L;
}

template <typename T>
int32_t run_step(const StepJob &J, int m, int reorth, double h, void *cvoid, void *ws,
                 const double *t_dev, double *t_adv, double *diag, hipStream_t s) {
  using C = typename CT<T>::t;
  (void)t_dev;
  const StepLayout L = step_layout(J.rows, J.sv.nseg, J.sv.n, sizeof(C), m, J.apply_ws);
  uint8_t *w8 = static_cast<uint8_t *>(ws);
  const int64_t sv_el = L.vec_stride / (int64_t)sizeof(C);
  C *V = (C *)(w8 + L.off_V);
  C *W = (C *)(w8 + L.off_W);
  void *aws = w8 + L.off_apply;
  double *part = (double *)(w8 + L.off_part);
  double *sc = (double *)(w8 + L.off_sc);
  double2 *c = static_cast<double2 *>(cvoid);
  const unsigned nseg = (unsigned)J.sv.nseg, nin = (unsigned)J.sv.n;
  const double tol = kBreakdownTol;

  int32_t st = J.set_time(s);
  if (st != HS_OK) return st;
  if (nseg == 0) return HS_OK;
  hipLaunchKernelGGL(k_snorm2_part, dim3(nseg), dim3(kSegThreads), 0, s, J.sv, (const double2 *)c, part);
  hipLaunchKernelGGL(k_sfin_beta0, dim3(nin), dim3(kSegThreads), 0, s, J.sv, (const double *)part, sc);
  hipLaunchKernelGGL(k_sstart<T>, dim3(nseg), dim3(kSegThreads), 0, s, J.sv, (const double2 *)c, V,
                     (const double *)sc);
  for (int k = 0; k < m; ++k) {
    C *Vk = V + (int64_t)k * sv_el;
    // With the Gram-Schmidt pass against all previous vectors, the projection removes
    // <v_{k-1}, H v_k> v_{k-1} whether or not beta_{k-1} v_{k-1} was subtracted first
    // (and alpha_k = Re <v_k, H v_k> either way), so the H application then skips the
    // previous vector; the plain recurrence subtracts it.
    const bool sub_prev = (k > 0) && !reorth;
    st = J.matvec(Vk, W, sub_prev ? (const void *)(V + (int64_t)(k - 1) * sv_el) : nullptr, k, sc, aws, s);
    if (st != HS_OK) return st;
    // the last step needs alpha_{m-1} only: no orthogonalisation against older vectors
    const bool last = (k == m - 1);
    const int lo = (reorth && !last) ? 0 : k;
    for (int c0 = lo; c0 <= k; c0 += kDotChunk) {
      const int cnt = std::min(kDotChunk, k + 1 - c0);
      hipLaunchKernelGGL(k_sdots_part<T>, dim3(nseg), dim3(kSegThreads), 0, s, J.sv, (const C *)V,
                         sv_el, c0, cnt, (const C *)W, part, (const double *)sc);
      hipLaunchKernelGGL(k_sfin_dots, dim3(nin, 2 * cnt), dim3(kSegThreads), 0, s, J.sv,
                         (const double *)part, c0, cnt, k, sc);
    }
    if (!last) {
      hipLaunchKernelGGL(k_supdate<T>, dim3(nseg), dim3(kSegThreads), 0, s, J.sv, (const C *)V, sv_el,
                         lo, k, reorth, (const C *)W, V + (int64_t)(k + 1) * sv_el, part,
                         (const double *)sc);
    }
    // sets m_eff, and beta_k / breakdown for k < m - 1 (the partial sums are not read at
    // the last step)
    hipLaunchKernelGGL(k_sfin_beta, dim3(nin), dim3(kSegThreads), 0, s, J.sv, (const double *)part,
                       k, m, tol, sc);
  }
  hipLaunchKernelGGL(k_small_expm, dim3(nin), dim3(1024), 0, s, h, sc);
  hipLaunchKernelGGL(k_scombine<T>, dim3(nseg), dim3(kSegThreads), 0, s, J.sv, (const C *)V, sv_el,
                     m, c, (const double *)sc);
  if (t_adv || diag)
    hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(64), 0, s, t_adv, h, (const double *)sc, diag, m);
  HS_HIP(hipGetLastError());
  return HS_OK;
}

template int32_t run_step<double>(const StepJob &, int, int, double, void *, void *, const double *,
                                  double *, double *, hipStream_t);
template int32_t run_step<float>(const StepJob &, int, int, double, void *, void *, const double *,
                                 double *, double *, hipStream_t);

// ---- single instance ----------------------------------------------------------------------
static SegView single_segments(int64_t rows) {
  SegView v{};
  v.n = 1;
  v.size = rows;
  v.nseg = (rows + kSeg - 1) / kSeg;
  return v;
}

int64_t step_workspace_bytes(const hs_index_s *idx, const hs_pot_s *p, int32_t dtype, int m) {
  if (m <= 0) return apply_workspace_bytes(idx, p, dtype);
  const SegView sv = single_segments(idx->size);
  return step_layout(idx->size, sv.nseg, 1, dtype == HS_C64 ? 8 : 16, m,
                     apply_workspace_bytes(idx, p, dtype)).total;
}

// Sets of at most this many rows take the one-workgroup step (hs_set_small_step_rows)
static std::atomic<int64_t> g_small_step_rows{kSmallStepRowsDefault};

void set_small_step_rows(int64_t rows) { g_small_step_rows.store(rows); }
int64_t small_step_rows() { return g_small_step_rows.load(); }

static bool small_step_eligible(const hs_index_s *idx, const hs_pot_s *p, int m) {
  return p->fused && p->form == HS_FORM_PAPER && idx->size > 0 && idx->size <= g_small_step_rows.load() &&
         idx->size <= kSmallStepRowsMax &&
         idx->recs_all && idx->rstride == rec_stride(idx->np) && m >= 1 && m <= kMaxM &&
         step_small_supported(idx->N, idx->np);
}

int32_t launch_step(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p, void *pot_dev,
                    int32_t dtype, double t, double *t_dev, double h, int m, int reorth, void *c,
                    void *ws, double *diag, hipStream_t s) {
  if (small_step_eligible(idx, p, m)) {
    const int64_t elem = dtype == HS_C64 ? 8 : 16;
    const StepLayout L = step_layout(idx->size, single_segments(idx->size).nseg, 1, elem, m,
                                     apply_workspace_bytes(idx, p, dtype));
    uint8_t *w8 = static_cast<uint8_t *>(ws);
    int32_t st = launch_set_time(p, pot_dev, t, t_dev, 0.5 * h, s);
    if (st != HS_OK) return st;
    const IndexDev ix = idx->view(idx_dev);
    const double *hh = (const double *)(static_cast<const uint8_t *>(pot_dev) + p->off_hh);
    double *sc = (double *)(w8 + L.off_sc);
    const int done = dtype == HS_C128
        ? launch_step_small_f64(ix, hh, c, w8 + L.off_V, L.vec_stride / elem, h, m, reorth, kBreakdownTol, sc,
                                t_dev, diag, s, p->x2)
        : launch_step_small_f32(ix, hh, c, w8 + L.off_V, L.vec_stride / elem, h, m, reorth, kBreakdownTol, sc,
                                t_dev, diag, s, p->x2);
    if (done != 1) return fail(HS_E_UNSUPPORTED, "small-set step: no instantiation for this set");
    HS_HIP(hipGetLastError());
    return HS_OK;
  }
  StepJob J;
  J.rows = idx->size;
  J.sv = single_segments(idx->size);
  J.apply_ws = apply_workspace_bytes(idx, p, dtype);
  J.set_time = [&](hipStream_t st) { return launch_set_time(p, pot_dev, t, t_dev, 0.5 * h, st); };
  J.matvec = [&](const void *vk, void *w, const void *vprev, int k, double *sc, void *aws,
                 hipStream_t st) {
    // stored vectors are unnormalised: H v_k = s_k H V_k, v_{k-1} = s_{k-1} V_{k-1}
    return launch_apply(idx, idx_dev, p, pot_dev, dtype, vk, w, aws, st,
                        k > 0 ? sc + Scal::inv + (k - 1) : nullptr, vprev,
                        vprev ? sc + Scal::beta + (k - 1) : nullptr,
                        k > 1 ? sc + Scal::inv + (k - 2) : nullptr);
  };
  if (dtype == HS_C128) return run_step<double>(J, m, reorth, h, c, ws, t_dev, t_dev, diag, s);
  return run_step<float>(J, m, reorth, h, c, ws, t_dev, t_dev, diag, s);
}

// ---- the unperturbed Lanczos process (paper Sec. 6.2): the same step with the exact
// Galerkin operator D + W_{K,pol} in place of the fast algorithm ----------------------------
int64_t step_exact_workspace_bytes(const hs_index_s *sub, const hs_index_s *pad, const hs_pot_s *p, int m) {
  if (m <= 0) return exact_apply_workspace_bytes(pad, p);
  const SegView sv = single_segments(sub->size);
  return step_layout(sub->size, sv.nseg, 1, 16, m, exact_apply_workspace_bytes(pad, p)).total;
}

int32_t launch_step_exact(const hs_index_s *sub, const hs_index_s *pad, const void *pad_dev, const int32_t *map,
                          const hs_pot_s *p, void *pot_dev, double t, double *t_dev, double h, int m, int reorth,
                          void *c, void *ws, double *diag, hipStream_t s) {
  StepJob J;
  J.rows = sub->size;
  J.sv = single_segments(sub->size);
  J.apply_ws = exact_apply_workspace_bytes(pad, p);
  J.set_time = [&](hipStream_t st) { return launch_set_time(p, pot_dev, t, t_dev, 0.5 * h, st); };
  J.matvec = [&](const void *vk, void *w, const void *vprev, int k, double *sc, void *aws, hipStream_t st) {
    return launch_exact_apply(sub, pad, pad_dev, map, p, pot_dev, vk, w, aws, st,
                              k > 0 ? sc + Scal::inv + (k - 1) : nullptr, vprev,
                              vprev ? sc + Scal::beta + (k - 1) : nullptr,
                              k > 1 ? sc + Scal::inv + (k - 2) : nullptr);
  };
  return run_step<double>(J, m, reorth, h, c, ws, t_dev, t_dev, diag, s);
}

// ---- two-stage Gauss-Legendre Magnus scheme (paper Sec. 2.1, eq. 2stageMagnus) ----------
// Nodes c_{1,2} = 1/2 -+ sqrt(3)/6.  Potentials of the fused class take the two fused
// passes of matvec_m4.h; the others (and sets without a specialised kernel) apply M with
// four H applications (A_1 v, A_2 v, A_2 A_1 v, A_1 A_2 v) and one combination pass.
// Scratch: three vectors in front of the H application's own workspace.
static const double kGl2c1 = 0.5 - 0.28867513459481288225;  // sqrt(3) / 6
static const double kGl2c2 = 0.5 + 0.28867513459481288225;

int64_t m4_apply_workspace_bytes(const hs_index_s *idx, const hs_pot_s *p, int32_t dtype) {
  const int64_t vec = align_up(idx->size * (dtype == HS_C64 ? 8 : 16), 256);
  return 3 * vec + apply_workspace_bytes(idx, p, dtype);
}

bool launch_m4_f64(const IndexDev &ix, const double *hh1, const double *hh2, const void *v, void *a,
                   void *d, void *w, const double *in_scale, double g2, const void *prev,
                   const double *prev_coef, const double *prev_scale, hipStream_t s, bool x2,
                   bool dl);
bool launch_m4_f32(const IndexDev &ix, const double *hh1, const double *hh2, const void *v, void *a,
                   void *d, void *w, const double *in_scale, double g2, const void *prev,
                   const double *prev_coef, const double *prev_scale, hipStream_t s, bool x2,
                   bool dl);

template <typename T>
static int32_t m4_apply_impl(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p,
                             const void *pot1, const void *pot2, const void *x, void *y, void *ws,
                             double h, hipStream_t s, const double *in_scale, const void *prev,
                             const double *prev_coef, const double *prev_scale) {
  using C = typename CT<T>::t;
  const int32_t dt = sizeof(T) == 8 ? HS_C128 : HS_C64;
  const int64_t vec = align_up(idx->size * (int64_t)sizeof(C), 256);
  uint8_t *w8 = static_cast<uint8_t *>(ws);
  void *u1 = w8, *u2 = w8 + vec, *z = w8 + 2 * vec, *aws = w8 + 3 * vec;
  if (idx->size == 0) return HS_OK;
  if (p->fused && p->form == HS_FORM_PAPER) {
    // two fused passes: (Abar v, Delta v), then the commutator and combination
    const IndexDev ix = idx->view(idx_dev);
    const double *hh1 = (const double *)((const uint8_t *)pot1 + p->off_hh);
    const double *hh2 = (const double *)((const uint8_t *)pot2 + p->off_hh);
    const double g2 = 2.0 * 1.7320508075688772935 * h / 12.0;
    const bool done = sizeof(T) == 8
        ? launch_m4_f64(ix, hh1, hh2, x, u1, u2, y, in_scale, g2, prev, prev_coef, prev_scale, s, p->x2, p->dyn_linear)
        : launch_m4_f32(ix, hh1, hh2, x, u1, u2, y, in_scale, g2, prev, prev_coef, prev_scale, s, p->x2,
                        p->dyn_linear);
    if (done) {
      HS_HIP(hipGetLastError());
      return HS_OK;
    }
  }
  // four H applications and one combination pass
  int32_t st;
  if ((st = launch_apply(idx, idx_dev, p, pot1, dt, x, u1, aws, s, in_scale, nullptr, nullptr, nullptr)) != HS_OK)
    return st;
  if ((st = launch_apply(idx, idx_dev, p, pot2, dt, x, u2, aws, s, in_scale, nullptr, nullptr, nullptr)) != HS_OK)
    return st;
  if ((st = launch_apply(idx, idx_dev, p, pot2, dt, u1, z, aws, s, nullptr, nullptr, nullptr, nullptr)) != HS_OK)
    return st;
  if ((st = launch_apply(idx, idx_dev, p, pot1, dt, u2, y, aws, s, nullptr, nullptr, nullptr, nullptr)) != HS_OK)
    return st;
  const double g = 1.7320508075688772935 * h / 12.0;
  hipLaunchKernelGGL(k_m4_combine<T>, dim3((unsigned)((idx->size + 255) / 256)), dim3(256), 0, s, idx->size,
                     (const C *)u1, (const C *)u2, (const C *)z, (C *)y, g, (const C *)prev, prev_coef,
                     prev_scale);
  HS_HIP(hipGetLastError());
  return HS_OK;
}

int32_t launch_apply_m4(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p, const void *pot1,
                        const void *pot2, int32_t dtype, double h, const void *x, void *y, void *ws,
                        hipStream_t s) {
  if (dtype == HS_C128)
    return m4_apply_impl<double>(idx, idx_dev, p, pot1, pot2, x, y, ws, h, s, nullptr, nullptr, nullptr, nullptr);
  return m4_apply_impl<float>(idx, idx_dev, p, pot1, pot2, x, y, ws, h, s, nullptr, nullptr, nullptr, nullptr);
}

int64_t step4_workspace_bytes(const hs_index_s *idx, const hs_pot_s *p, int32_t dtype, int m) {
  const SegView sv = single_segments(idx->size);
  return step_layout(idx->size, sv.nseg, 1, dtype == HS_C64 ? 8 : 16, m,
                     m4_apply_workspace_bytes(idx, p, dtype)).total;
}

int32_t launch_step_m4(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p, void *pot1,
                       void *pot2, int32_t dtype, double t, double *t_dev, double h, int m, int reorth,
                       void *c, void *ws, double *diag, hipStream_t s) {
  StepJob J;
  J.rows = idx->size;
  J.sv = single_segments(idx->size);
  J.apply_ws = m4_apply_workspace_bytes(idx, p, dtype);
  // both blocks read t before the step advances it
  J.set_time = [&](hipStream_t st) {
    const int32_t r = launch_set_time(p, pot1, t, t_dev, kGl2c1 * h, st);
    return r != HS_OK ? r : launch_set_time(p, pot2, t, t_dev, kGl2c2 * h, st);
  };
  J.matvec = [&](const void *vk, void *w, const void *vprev, int k, double *sc, void *aws,
                 hipStream_t st) {
    const double *in_scale = k > 0 ? sc + Scal::inv + (k - 1) : nullptr;
    const double *pc = vprev ? sc + Scal::beta + (k - 1) : nullptr;
    const double *ps = k > 1 ? sc + Scal::inv + (k - 2) : nullptr;
    if (dtype == HS_C128)
      return m4_apply_impl<double>(idx, idx_dev, p, pot1, pot2, vk, w, aws, h, st, in_scale, vprev, pc, ps);
    return m4_apply_impl<float>(idx, idx_dev, p, pot1, pot2, vk, w, aws, h, st, in_scale, vprev, pc, ps);
  };
  if (dtype == HS_C128) return run_step<double>(J, m, reorth, h, c, ws, t_dev, t_dev, diag, s);
  return run_step<float>(J, m, reorth, h, c, ws, t_dev, t_dev, diag, s);
}

}  // namespace hs
