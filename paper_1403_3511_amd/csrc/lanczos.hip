// Short-iterative Lanczos step for the exponential midpoint rule (paper Sec. 2.1 eq.
// expMPR, Sec. 2.2, Fig. 4 time_propagation):
//   coefficients at t + h/2; beta_0 = ||c||, v_1 = c / beta_0;
//   w = H v_k - beta_{k-1} v_{k-1}; alpha_k = Re <v_k, w>;
//   w -= alpha_k v_k  (or, with reorthogonalisation, w -= sum_{i<=k} <v_i, w> v_i);
//   beta_k = ||w||; v_{k+1} = w / beta_k;
//   T_m = tridiag(beta, alpha, beta) = Q Lambda Q^T on the device;
//   c <- beta_0 V_m Q exp(-i h Lambda) Q^T e_1.
// Every scalar stays on the device; no host synchronisation inside a step, so a step
// can be captured into a HIP graph.  Reductions are deterministic: fixed grid, per-block
// partials in a fixed slot, one finishing block summing the partials in a fixed tree.
#include "hs_internal.h"

namespace hs {

int32_t launch_apply(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p,
                     const void *pot_dev, int32_t dtype, const void *x, void *y, void *ws,
                     hipStream_t s, const double *out_scale, const void *prev,
                     const double *prev_coef, const double *prev_scale);

constexpr int kRedBlocks = 512;  // fixed partial count of every reduction
constexpr int kRedThreads = 256;
constexpr int kMaxM = 32;
constexpr int kDotChunk = 8;     // vectors per dot-product launch

// scalar block layout (doubles)
struct Scal {
  static constexpr int beta0 = 0, inv0 = 1, stop = 2, meff = 3, tnorm = 4;
  static constexpr int alpha = 8;                 // [kMaxM]
  static constexpr int beta = alpha + kMaxM;      // [kMaxM]
  static constexpr int inv = beta + kMaxM;        // [kMaxM] 1 / beta_k
  static constexpr int dre = inv + kMaxM;         // [kMaxM + 1] dot products (re)
  static constexpr int dim = dre + kMaxM + 1;     // (im)
  static constexpr int yre = dim + kMaxM + 1;     // [kMaxM] combination weights
  static constexpr int yim = yre + kMaxM;
  static constexpr int size = yim + kMaxM;
};

template <typename T> struct CT;
template <> struct CT<double> { using t = double2; };
template <> struct CT<float> { using t = float2; };

__device__ __forceinline__ double block_sum(double v, double *sh) {
  // fixed-order tree over the block
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// ---- ||x||^2 partials (x complex128) ---------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
k_norm2_part(int64_t n, const typename CT<T>::t *__restrict__ x, double *__restrict__ part) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double a = x[i].x, b = x[i].y;
    acc = fma(a, a, fma(b, b, acc));
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// finish ||c||: beta0, inv0; stop if zero
__global__ void k_fin_beta0(const double *__restrict__ part, double *__restrict__ sc) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) acc += part[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) {
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

// v0 = c * inv0 (dtype conversion for the float32 form)
template <typename T>
__global__ void __launch_bounds__(256)
k_start(int64_t n, const double2 *__restrict__ c, typename CT<T>::t *__restrict__ v,
        const double *__restrict__ sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = sc[Scal::inv0];
  typename CT<T>::t o;
  o.x = (T)(c[i].x * s);
  o.y = (T)(c[i].y * s);
  v[i] = o;
}

// partial dot products <V_i, W> = sum conj(V_i) W for i = lo .. lo+cnt-1
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
k_dots_part(int64_t n, const typename CT<T>::t *__restrict__ V, int64_t stride, int lo, int cnt,
            const typename CT<T>::t *__restrict__ W, double *__restrict__ part,
            const double *__restrict__ sc) {
  __shared__ double sh[kRedThreads];
  if (sc[Scal::stop] != 0.0) return;
  double ar[kDotChunk], ai[kDotChunk];
  for (int q = 0; q < kDotChunk; ++q) ar[q] = ai[q] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double wr = W[i].x, wi = W[i].y;
#pragma unroll
    for (int q = 0; q < kDotChunk; ++q) {
      if (q < cnt) {
        const typename CT<T>::t v = V[(int64_t)(lo + q) * stride + i];
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
      part[(2 * q) * kRedBlocks + blockIdx.x] = sr;
      part[(2 * q + 1) * kRedBlocks + blockIdx.x] = si;
    }
  }
}

__global__ void k_fin_dots(const double *__restrict__ part, int lo, int cnt, int k,
                           double *__restrict__ sc) {
  __shared__ double sh[kRedThreads];
  if (sc[Scal::stop] != 0.0) return;
  for (int q = 0; q < 2 * cnt; ++q) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) acc += part[q * kRedBlocks + i];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) {
      const int idx = lo + q / 2;
      if (q & 1) sc[Scal::dim + idx] = s; else sc[Scal::dre + idx] = s;
      if (!(q & 1) && idx == k) sc[Scal::alpha + k] = s;  // alpha_k = Re <v_k, w>
    }
  }
}

// W -= sum_i d_i V_i over i in [lo, k] (reorth) or W -= alpha_k V_k; ||W||^2 partials
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
k_update(int64_t n, const typename CT<T>::t *__restrict__ V, int64_t stride, int lo, int k,
         int reorth, typename CT<T>::t *__restrict__ W, double *__restrict__ part,
         const double *__restrict__ sc) {
  __shared__ double sh[kRedThreads];
  if (sc[Scal::stop] != 0.0) return;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double wr = W[i].x, wi = W[i].y;
    if (reorth) {
      for (int q = lo; q <= k; ++q) {
        const double dr = sc[Scal::dre + q], di = sc[Scal::dim + q];
        const typename CT<T>::t v = V[(int64_t)q * stride + i];
        const double vr = v.x, vi = v.y;
        wr -= dr * vr - di * vi;
        wi -= dr * vi + di * vr;
      }
    } else {
      const double a = sc[Scal::alpha + k];
      const typename CT<T>::t v = V[(int64_t)k * stride + i];
      wr -= a * (double)v.x;
      wi -= a * (double)v.y;
    }
    typename CT<T>::t o;
    o.x = (T)wr;
    o.y = (T)wi;
    W[i] = o;
    const double qr = o.x, qi = o.y;
    acc = fma(qr, qr, fma(qi, qi, acc));
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// beta_k = ||W||; breakdown test against ||T_{k+1}||_inf
__global__ void k_fin_beta(const double *__restrict__ part, int k, int m, double tol,
                           double *__restrict__ sc) {
  __shared__ double sh[kRedThreads];
  if (sc[Scal::stop] != 0.0) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) acc += part[i];
  const double s = block_sum(acc, sh);
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

template <typename T>
__global__ void __launch_bounds__(256)
k_scale_next(int64_t n, const typename CT<T>::t *__restrict__ W, typename CT<T>::t *__restrict__ vn,
             int k, const double *__restrict__ sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || sc[Scal::stop] != 0.0) return;
  const double s = sc[Scal::inv + k];
  typename CT<T>::t o;
  o.x = (T)((double)W[i].x * s);
  o.y = (T)((double)W[i].y * s);
  vn[i] = o;
}

// y = beta0 exp(-i h T) e1 for the real symmetric tridiagonal T (m <= 32) by scaling
// and squaring: delta = h / 2^q with h ||T||_inf / 2^q <= 1/2, an 18-term Taylor
// polynomial of exp(-i delta T) (truncation below 1e-22), then q squarings.  One
// workgroup, one thread per matrix element.
__global__ void __launch_bounds__(1024) k_small_expm(double h, double *__restrict__ sc) {
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
    // P <- P (-i delta T) / k, T tridiagonal
    double2 nv = make_double2(0.0, 0.0);
    if (act) {
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
      nv = make_double2(si * f, -sr * f);  // (-i f) (sr + i si)
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

// c = sum_{k < m_eff} y_k V_k (complex128 result)
template <typename T>
__global__ void __launch_bounds__(256)
k_combine(int64_t n, const typename CT<T>::t *__restrict__ V, int64_t stride, int m,
          double2 *__restrict__ c, const double *__restrict__ sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int me = (int)sc[Scal::meff];
  if (me <= 0) return;  // zero vector stays zero
  double cr = 0.0, ci = 0.0;
  for (int k = 0; k < me && k < m; ++k) {
    const double yr = sc[Scal::yre + k], yi = sc[Scal::yim + k];
    const typename CT<T>::t v = V[(int64_t)k * stride + i];
    cr += yr * v.x - yi * v.y;
    ci += yr * v.y + yi * v.x;
  }
  c[i] = make_double2(cr, ci);
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

// ---- host driver ------------------------------------------------------------------------
struct StepWs {
  int64_t vec_stride;  // bytes between Krylov vectors
  int64_t off_V, off_W, off_apply, off_part, off_sc, total;
};

static StepWs step_layout(const hs_index_s *idx, const hs_pot_s *p, int32_t dtype, int m) {
  StepWs L;
  const int64_t es = dtype == HS_C64 ? 8 : 16;
  L.vec_stride = align_up(idx->size * es, 256);
  int64_t off = 0;
  L.off_V = off;
  off += L.vec_stride * m;
  L.off_W = off;
  off += L.vec_stride;
  L.off_apply = off;
  off += align_up(apply_workspace_bytes(idx, p, dtype), 256);
  L.off_part = off;
  off += align_up(8 * kRedBlocks * 2 * kDotChunk, 256);
  L.off_sc = off;
  off += align_up(8 * Scal::size, 256);
  L.total = off;
  return L;
}

int64_t step_workspace_bytes(const hs_index_s *idx, const hs_pot_s *p, int32_t dtype, int m) {
  if (m <= 0) return apply_workspace_bytes(idx, p, dtype);
  return step_layout(idx, p, dtype, m).total;
}

template <typename T>
static int32_t step_impl(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p,
                         void *pot_dev, int32_t dtype, double t, double *t_dev, double h, int m,
                         int reorth, void *cvoid, void *ws, double *diag, hipStream_t s) {
  using C = typename CT<T>::t;
  const StepWs L = step_layout(idx, p, dtype, m);
  uint8_t *w8 = static_cast<uint8_t *>(ws);
  const int64_t n = idx->size;
  const int64_t sv = L.vec_stride / (int64_t)sizeof(C);
  C *V = (C *)(w8 + L.off_V);
  C *W = (C *)(w8 + L.off_W);
  void *aws = w8 + L.off_apply;
  double *part = (double *)(w8 + L.off_part);
  double *sc = (double *)(w8 + L.off_sc);
  double2 *c = static_cast<double2 *>(cvoid);
  const unsigned g = (unsigned)((n + 255) / 256);
  const double tol = 1e-12;

  int32_t st = launch_set_time(p, pot_dev, t, t_dev, 0.5 * h, s);
  if (st != HS_OK) return st;
  hipLaunchKernelGGL(k_norm2_part<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, s, n,
                     (const double2 *)c, part);
  hipLaunchKernelGGL(k_fin_beta0, dim3(1), dim3(kRedThreads), 0, s, part, sc);
  hipLaunchKernelGGL(k_start<T>, dim3(g), dim3(256), 0, s, n, (const double2 *)c, V, sc);
  for (int k = 0; k < m; ++k) {
    C *Vk = V + (int64_t)k * sv;
    // W = H v_k - beta_{k-1} v_{k-1}
    st = launch_apply(idx, idx_dev, p, pot_dev, dtype, Vk, W, aws, s, nullptr,
                      k > 0 ? (const void *)(V + (int64_t)(k - 1) * sv) : nullptr,
                      k > 0 ? sc + Scal::beta + (k - 1) : nullptr, nullptr);
    if (st != HS_OK) return st;
    const int lo = reorth ? 0 : k;
    for (int c0 = lo; c0 <= k; c0 += kDotChunk) {
      const int cnt = std::min(kDotChunk, k + 1 - c0);
      hipLaunchKernelGGL(k_dots_part<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, s, n,
                         (const C *)V, sv, c0, cnt, (const C *)W, part, (const double *)sc);
      hipLaunchKernelGGL(k_fin_dots, dim3(1), dim3(kRedThreads), 0, s, (const double *)part, c0,
                         cnt, k, sc);
    }
    hipLaunchKernelGGL(k_update<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, s, n, (const C *)V,
                       sv, lo, k, reorth, W, part, (const double *)sc);
    hipLaunchKernelGGL(k_fin_beta, dim3(1), dim3(kRedThreads), 0, s, (const double *)part, k, m,
                       tol, sc);
    if (k + 1 < m)
      hipLaunchKernelGGL(k_scale_next<T>, dim3(g), dim3(256), 0, s, n, (const C *)W,
                         V + (int64_t)(k + 1) * sv, k, (const double *)sc);
  }
  hipLaunchKernelGGL(k_small_expm, dim3(1), dim3(1024), 0, s, h, sc);
  hipLaunchKernelGGL(k_combine<T>, dim3(g), dim3(256), 0, s, n, (const C *)V, sv, m, c,
                     (const double *)sc);
  hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(64), 0, s, t_dev, h, (const double *)sc, diag, m);
  HS_HIP(hipGetLastError());
  return HS_OK;
}

int32_t launch_step(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p, void *pot_dev,
                    int32_t dtype, double t, double *t_dev, double h, int m, int reorth, void *c,
                    void *ws, double *diag, hipStream_t s) {
  if (dtype == HS_C128)
    return step_impl<double>(idx, idx_dev, p, pot_dev, dtype, t, t_dev, h, m, reorth, c, ws, diag, s);
  return step_impl<float>(idx, idx_dev, p, pot_dev, dtype, t, t_dev, h, m, reorth, c, ws, diag, s);
}

}  // namespace hs
