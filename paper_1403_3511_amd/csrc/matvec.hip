// H application y = (D + W^pol(X_K)) c on gfx950 (paper Sec. 3.1-3.2, eq. Horner).
//
// Two kernels families:
//  * hh_rows: one lane per row.  The potential is grouped by outer axis l; the group's
//    operator  X_l(X_l(X_l(a3 c) + a2 c + g2 X_{l+1} c) + a1 c + g1 X_{l+1} c)  is the
//    Horner form of a1 x_l + a2 x_l^2 + a3 x_l^3 + g1 x_l x_{l+1} + g2 x_l^2 x_{l+1} with
//    X_{l+1} applied first, evaluated on the window j + s e_l, |s| <= 3, of the row's
//    axis-l fibre (the layered binary tree of Sec. 5.3 restricted to one layer pair).
//    Truncation at the fibre ends enters through absent edges: the edge between fibre
//    positions k-1 and k carries sqrt(k/2) only if both lie in K (Sec. 3.1: a missing
//    neighbour contributes nothing).
//  * generic passes: one kernel per recurrence step p_{k+1} = A X_l p_k + B p_k - C p_{k-1}
//    over the whole vector, following the program compiled from the term trie.
//
// No MFMA: the operator is a sparse stencil, not a dense contraction.
#include "dev_common.h"

namespace hs {

// specialised fused kernels (compile-time N and prefix axes): 1 = long and short tiles
// launched, 2 = long tiles only, 0 = no specialisation for this (N, NP)
int launch_hh_long_f64(const IndexDev &ix, const double *hh, const void *x, void *y,
                       const double *out_scale, const void *prev, const double *prev_coef,
                       const double *prev_scale, hipStream_t s, bool x2);
int launch_hh_long_f32(const IndexDev &ix, const double *hh, const void *x, void *y,
                       const double *out_scale, const void *prev, const double *prev_coef,
                       const double *prev_scale, hipStream_t s, bool x2);
// the same for the symmetrised operator D + (F + F_rev)/2
int launch_hh_long_sym_f64(const IndexDev &ix, const double *hh, const void *x, void *y,
                           const double *out_scale, const void *prev, const double *prev_coef,
                           const double *prev_scale, hipStream_t s, bool x2);
int launch_hh_long_sym_f32(const IndexDev &ix, const double *hh, const void *x, void *y,
                           const double *out_scale, const void *prev, const double *prev_coef,
                           const double *prev_scale, hipStream_t s, bool x2);

// long tiles by work items of several tiles (0: not served; 1: short tiles too; 2: the
// short tiles left to the caller); short tiles alone by the per-lane-record path of the
// specialised kernel (0: not served)
int launch_hh_multi_f64(const IndexDev &ix, const double *hh, const void *x, void *y,
                         const double *out_scale, const void *prev, const double *prev_coef,
                         const double *prev_scale, hipStream_t s, bool x2);
int launch_hh_multi_f32(const IndexDev &ix, const double *hh, const void *x, void *y,
                         const double *out_scale, const void *prev, const double *prev_coef,
                         const double *prev_scale, hipStream_t s, bool x2);
int launch_hh_short_f64(const IndexDev &ix, const double *hh, const void *x, void *y,
                        const double *out_scale, const void *prev, const double *prev_coef,
                        const double *prev_scale, hipStream_t s, bool x2);
int launch_hh_short_f32(const IndexDev &ix, const double *hh, const void *x, void *y,
                        const double *out_scale, const void *prev, const double *prev_coef,
                        const double *prev_scale, hipStream_t s, bool x2);

struct Pos {
  int32_t t, o;
};

// move one step along axis (0-based) in direction up (1: +e, 0: -e); t < 0 = absent
__device__ __forceinline__ Pos mv(const IndexDev &ix, Pos p, int axis, int up) {
  if (p.t < 0) return p;
  HS_DCHECK(ix, p.t < ix.ntiles && p.o >= 0 && p.o < ix.ng, kDbgPosition);
  if (axis < ix.np) {
    const int32_t t2 = ix.tnbr[(int64_t)p.t * (2 * ix.np) + 2 * axis + up];
    if (t2 < 0 || (up && p.o >= ix.tlen[t2])) return Pos{-1, 0};
    return Pos{t2, p.o};
  }
  const int a = axis - ix.np;
  const int32_t o2 = ix.gnbr[(int64_t)p.o * (2 * ix.d) + 2 * a + up];
  if (o2 < 0 || (up && o2 >= ix.tlen[p.t])) return Pos{-1, 0};
  return Pos{p.t, o2};
}

__device__ __forceinline__ int coord(const IndexDev &ix, Pos p, int axis) {
  return axis < ix.np ? (int)ix.tpfx[(int64_t)p.t * ix.np + axis]
                      : (int)ix.gsidx[(int64_t)p.o * ix.d + (axis - ix.np)];
}

template <typename T>
__device__ __forceinline__ typename V2<T>::t ld(const typename V2<T>::t *__restrict__ c,
                                                const IndexDev &ix, Pos p) {
  if (p.t < 0) return vz<T>();
#ifdef HS_DEBUG_BOUNDS
  // a position outside its tile is counted and not read
  if (!(p.t < ix.ntiles && p.o >= 0 && p.o < ix.tlen[p.t])) {
    debug_flag(ix.dbg, kDbgPosition);
    return vz<T>();
  }
#endif
  return c[ix.tstart[p.t] + p.o];
}

// ---- coefficient update (paper Fig. 4 step (1)) -------------------------------------
// beta_t = base_t + amp_t sin(freq_t (t + dt) + phase_t); hh[s] = sum_t M[s][t] beta_t
__global__ void k_set_time(int nterms, int nslots, const double *__restrict__ base,
                           const double *__restrict__ amp, const double *__restrict__ freq,
                           const double *__restrict__ phase, const double *__restrict__ M,
                           double *__restrict__ beta, double *__restrict__ hh, double t_host,
                           const double *__restrict__ t_dev, double dt) {
  __shared__ double sb[kMaxTerms];
  const double t = (t_dev ? *t_dev : t_host) + dt;
  for (int i = threadIdx.x; i < nterms; i += blockDim.x) {
    const double b = base[i] + amp[i] * sin(freq[i] * t + phase[i]);
    sb[i] = b;
    beta[i] = b;
  }
  __syncthreads();
  for (int s = threadIdx.x; s < nslots; s += blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < nterms; ++i) acc = fma(M[(int64_t)s * nterms + i], sb[i], acc);
    hh[s] = acc;
  }
}

__global__ void k_copy_coeffs(int n, const double *__restrict__ src, double *__restrict__ base,
                              double *__restrict__ amp) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    base[i] = src[i];
    amp[i] = 0.0;
  }
}

// ---- fused row kernel ----------------------------------------------------------------
// y = out_scale * (D + c0 + sum_l G_l) x  -  prev_coef * prev_scale * prev
// out_scale / prev_coef / prev_scale are read from device scalars when given (Lanczos),
// else taken as 1 / 0.
template <typename T>
__global__ void __launch_bounds__(256)
k_hh_rows(IndexDev ix, const double *__restrict__ hh, const typename V2<T>::t *__restrict__ x,
          typename V2<T>::t *__restrict__ y, const double *__restrict__ out_scale,
          const typename V2<T>::t *__restrict__ prev, const double *__restrict__ prev_coef,
          const double *__restrict__ prev_scale, const int32_t *__restrict__ rows, int64_t nrows) {
  using C = typename V2<T>::t;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  const int64_t r = rows ? (int64_t)rows[i] : i;
  const T *wt;
  if constexpr (sizeof(T) == 8) wt = (const T *)ix.wtab; else wt = (const T *)ix.wtabf;
  const int32_t t0 = ix.rowtile[r];
  const Pos p0{t0, (int32_t)(r - ix.tstart[t0])};
  const int N = ix.N;
  const C c0 = x[r];
  const double dval = (double)(ix.tpsum[t0] + ix.gssum[p0.o]) + 0.5 * N + hh[5 * N];
  C acc = scal<T>((T)dval, c0);

  for (int l = 0; l < N; ++l) {
    const T a1 = (T)hh[5 * l + 0], a2 = (T)hh[5 * l + 1], a3 = (T)hh[5 * l + 2];
    const T g1 = (l + 1 < N) ? (T)hh[5 * l + 3] : T(0);
    const T g2 = (l + 1 < N) ? (T)hh[5 * l + 4] : T(0);
    const bool any2 = (a3 != T(0)) || (a2 != T(0)) || (g2 != T(0));
    if (!any2 && a1 == T(0) && g1 == T(0)) continue;  // uniform across the grid
    const int jl = coord(ix, p0, l);
    Pos P[7];
    P[3] = p0;
    P[4] = mv(ix, P[3], l, 1);
    P[2] = mv(ix, P[3], l, 0);
    C u[7];
    u[3] = c0;
    u[4] = ld<T>(x, ix, P[4]);
    u[2] = ld<T>(x, ix, P[2]);
    T e[6];  // e[s + 2] = weight of the edge between window positions s-1 and s
    e[2] = (P[2].t >= 0) ? wt[jl] : T(0);
    e[3] = (P[4].t >= 0) ? wt[jl + 1] : T(0);
    if (any2) {
      P[5] = mv(ix, P[4], l, 1);
      P[1] = mv(ix, P[2], l, 0);
      u[5] = ld<T>(x, ix, P[5]);
      u[1] = ld<T>(x, ix, P[1]);
      e[1] = (P[1].t >= 0) ? wt[jl - 1] : T(0);
      e[4] = (P[5].t >= 0) ? wt[jl + 2] : T(0);
      if (a3 != T(0)) {
        P[6] = mv(ix, P[5], l, 1);
        P[0] = mv(ix, P[1], l, 0);
        u[6] = ld<T>(x, ix, P[6]);
        u[0] = ld<T>(x, ix, P[0]);
        e[0] = (P[0].t >= 0) ? wt[jl - 2] : T(0);
        e[5] = (P[6].t >= 0) ? wt[jl + 3] : T(0);
      } else {
        u[6] = vz<T>();
        u[0] = vz<T>();
        e[0] = e[5] = T(0);
      }
    } else {
      u[5] = u[1] = u[6] = u[0] = vz<T>();
      e[0] = e[1] = e[4] = e[5] = T(0);
    }
    // X_{l+1} c on the window (inner axis applied first)
    C v[5];  // v[s + 2], s = -2..2
    for (int s = 0; s < 5; ++s) v[s] = vz<T>();
    if (g1 != T(0) || g2 != T(0)) {
      const int jn = coord(ix, p0, l + 1);
      const T wlo = wt[jn], whi = wt[jn + 1];
      for (int s = -2; s <= 2; ++s) {
        if ((s & 1) ? (g1 == T(0)) : (g2 == T(0))) continue;
        const Pos q = P[3 + s];
        if (q.t < 0) continue;
        C vs = vz<T>();
        if (jn > 0) fma_rc<T>(vs, wlo, ld<T>(x, ix, mv(ix, q, l + 1, 0)));
        fma_rc<T>(vs, whi, ld<T>(x, ix, mv(ix, q, l + 1, 1)));
        v[s + 2] = vs;
      }
    }
    // Horner along axis l
    C h2[3];  // s = -2, 0, 2
    for (int q = 0; q < 3; ++q) {
      const int s = 2 * q - 2;
      C h = vz<T>();
      if (any2) {
        C xu = vz<T>();
        fma_rc<T>(xu, e[s + 2], u[3 + s - 1]);
        fma_rc<T>(xu, e[s + 3], u[3 + s + 1]);
        h = scal<T>(a3, xu);
        fma_rc<T>(h, a2, u[3 + s]);
        fma_rc<T>(h, g2, v[s + 2]);
      }
      h2[q] = h;
    }
    C h1[2];  // s = -1, 1
    for (int q = 0; q < 2; ++q) {
      const int s = 2 * q - 1;
      C h = vz<T>();
      fma_rc<T>(h, e[s + 2], h2[q]);
      fma_rc<T>(h, e[s + 3], h2[q + 1]);
      fma_rc<T>(h, a1, u[3 + s]);
      fma_rc<T>(h, g1, v[s + 2]);
      h1[q] = h;
    }
    fma_rc<T>(acc, e[2], h1[0]);
    fma_rc<T>(acc, e[3], h1[1]);
  }
  if (out_scale) acc = scal<T>((T)*out_scale, acc);
  if (prev) {
    const T pc = (T)(-(*prev_coef) * (prev_scale ? *prev_scale : 1.0));
    fma_rc<T>(acc, pc, prev[r]);
  }
  y[r] = acc;
}

// ---- long-tile kernel ---------------------------------------------------------------
// One wave per 64-row chunk of one tile: the tile id is uniform, so every move along a
// prefix axis is a scalar chain through the tile-neighbour table and the loads of a
// neighbour tile at the same offsets are contiguous.  Moves along suffix axes read the
// precomputed suffix stencil of the row's offset (no dependent chains).
template <typename T>
__global__ void __launch_bounds__(256)
k_hh_tiles(IndexDev ix, const double *__restrict__ hh, const typename V2<T>::t *__restrict__ x,
           typename V2<T>::t *__restrict__ y, const double *__restrict__ out_scale,
           const typename V2<T>::t *__restrict__ prev, const double *__restrict__ prev_coef,
           const double *__restrict__ prev_scale) {
  using C = typename V2<T>::t;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= ix.nchunks) return;
  const int32_t ri = __builtin_amdgcn_readfirstlane(ix.chunks[2 * wave]);
  const int32_t t = ix.recs[(int64_t)ri * ix.rstride + 3];
  const int32_t o0 = __builtin_amdgcn_readfirstlane(ix.chunks[2 * wave + 1]);
  const int32_t len = ix.tlen[t];
  const int32_t o = o0 + lane;
  if (o >= len) return;
  const T *wt;
  if constexpr (sizeof(T) == 8) wt = (const T *)ix.wtab; else wt = (const T *)ix.wtabf;
  const int N = ix.N, np = ix.np, d = ix.d;
  const int64_t ng = ix.ng;
  const int64_t base = ix.tstart[t];
  const int64_t r = base + o;
  const C c0 = x[r];
  const double dval = (double)(ix.tpsum[t] + ix.gssum[o]) + 0.5 * N + hh[5 * N];
  C acc = scal<T>((T)dval, c0);

  for (int l = 0; l < N; ++l) {
    const T a1 = (T)hh[5 * l + 0], a2 = (T)hh[5 * l + 1], a3 = (T)hh[5 * l + 2];
    const T g1 = (l + 1 < N) ? (T)hh[5 * l + 3] : T(0);
    const T g2 = (l + 1 < N) ? (T)hh[5 * l + 4] : T(0);
    const bool any2 = (a3 != T(0)) || (a2 != T(0)) || (g2 != T(0));
    if (!any2 && a1 == T(0) && g1 == T(0)) continue;
    const int smax = (a3 != T(0)) ? 3 : (any2 ? 2 : 1);
    const bool lp = l < np;
    // window s = -3..3 along axis l: tile Ts (uniform for a prefix axis) and offset Os
    int32_t Ts[7], Os[7];
    bool val[7];
    int jl;
    for (int q = 0; q < 7; ++q) {
      Ts[q] = -1;
      Os[q] = -1;
      val[q] = false;
    }
    Ts[3] = t;
    Os[3] = o;
    val[3] = true;
    if (lp) {
      jl = ix.tpfx[(int64_t)t * np + l];
      int32_t up = t, dn = t;
      for (int s = 1; s <= 3; ++s) {
        if (s > smax) break;
        up = (up >= 0) ? ix.tnbr[(int64_t)up * (2 * np) + 2 * l + 1] : -1;
        dn = (dn >= 0) ? ix.tnbr[(int64_t)dn * (2 * np) + 2 * l] : -1;
        Ts[3 + s] = up;
        Ts[3 - s] = dn;
        Os[3 + s] = o;
        Os[3 - s] = o;
        val[3 + s] = (up >= 0) && (o < ix.tlen[up]);
        val[3 - s] = (dn >= 0);
      }
    } else {
      const int a = l - np;
      jl = ix.gsidx[(int64_t)o * d + a];
      for (int s = 1; s <= 3; ++s) {
        if (s > smax) break;
        const int32_t ou = ix.gst[gst_axis_at(a, s, o, ng)];
        const int32_t od = ix.gst[gst_axis_at(a, -s, o, ng)];
        Ts[3 + s] = t;
        Ts[3 - s] = t;
        Os[3 + s] = ou;
        Os[3 - s] = od;
        val[3 + s] = (ou >= 0) && (ou < len);
        val[3 - s] = (od >= 0);
      }
    }
    C u[7];
    for (int q = 0; q < 7; ++q) u[q] = vz<T>();
    u[3] = c0;
    for (int q = 0; q < 7; q += 2)  // s = -3, -1, 1, 3
      if (val[q]) u[q] = x[ix.tstart[Ts[q]] + Os[q]];
    if (a2 != T(0))
      for (int q = 1; q < 7; q += 4)  // s = -2, +2 only needed for the x_l^2 term
        if (val[q]) u[q] = x[ix.tstart[Ts[q]] + Os[q]];
    T e[6];  // e[s + 2] = weight of the edge between window positions s-1 and s
    for (int s = -2; s <= 3; ++s) e[s + 2] = (val[3 + s - 1] && val[3 + s]) ? wt[jl + s] : T(0);
    // X_{l+1} c on the window (inner axis applied first)
    C v[5];
    for (int q = 0; q < 5; ++q) v[q] = vz<T>();
    if (g1 != T(0) || g2 != T(0)) {
      const int m = l + 1;
      const bool mp = m < np;
      const int jm = mp ? (int)ix.tpfx[(int64_t)t * np + m] : (int)ix.gsidx[(int64_t)o * d + (m - np)];
      const T wlo = wt[jm], whi = wt[jm + 1];
      for (int s = -2; s <= 2; ++s) {
        if ((s & 1) ? (g1 == T(0)) : (g2 == T(0))) continue;
        if (!val[3 + s]) continue;
        C vs = vz<T>();
        for (int r2 = -1; r2 <= 1; r2 += 2) {
          int32_t tq, oq;
          bool ok;
          if (mp) {
            tq = ix.tnbr[(int64_t)Ts[3 + s] * (2 * np) + 2 * m + (r2 > 0)];
            oq = o;
            ok = (tq >= 0) && (r2 < 0 || o < ix.tlen[tq]);
          } else if (lp) {  // l prefix, m the first suffix axis
            tq = Ts[3 + s];
            oq = ix.gst[gst_axis_at(0, r2, o, ng)];
            ok = (oq >= 0) && (oq < ix.tlen[tq]);
          } else {          // both suffix axes
            const int a = l - np;
            tq = t;
            oq = (s == 0) ? ix.gst[gst_axis_at(a + 1, r2, o, ng)]
                          : ix.gst[gst_cross_at(d, a, s, r2, o, ng)];
            ok = (oq >= 0) && (oq < len);
          }
          if (ok) fma_rc<T>(vs, r2 < 0 ? wlo : whi, x[ix.tstart[tq] + oq]);
        }
        v[s + 2] = vs;
      }
    }
    C h2[3];
    for (int q = 0; q < 3; ++q) {
      const int s = 2 * q - 2;
      C h = vz<T>();
      if (any2) {
        C xu = vz<T>();
        fma_rc<T>(xu, e[s + 2], u[3 + s - 1]);
        fma_rc<T>(xu, e[s + 3], u[3 + s + 1]);
        h = scal<T>(a3, xu);
        fma_rc<T>(h, a2, u[3 + s]);
        fma_rc<T>(h, g2, v[s + 2]);
      }
      h2[q] = h;
    }
    C h1[2];
    for (int q = 0; q < 2; ++q) {
      const int s = 2 * q - 1;
      C h = vz<T>();
      fma_rc<T>(h, e[s + 2], h2[q]);
      fma_rc<T>(h, e[s + 3], h2[q + 1]);
      fma_rc<T>(h, a1, u[3 + s]);
      fma_rc<T>(h, g1, v[s + 2]);
      h1[q] = h;
    }
    fma_rc<T>(acc, e[2], h1[0]);
    fma_rc<T>(acc, e[3], h1[1]);
  }
  if (out_scale) acc = scal<T>((T)*out_scale, acc);
  if (prev) {
    const T pc = (T)(-(*prev_coef) * (prev_scale ? *prev_scale : 1.0));
    fma_rc<T>(acc, pc, prev[r]);
  }
  y[r] = acc;
}

// ---- generic passes -------------------------------------------------------------------
// The dense coefficient matrix M[o][i] of the split program's combination, summed from
// the (input, term) table as k_combine_dense sums it; one workgroup, every thread.
__device__ __forceinline__ void comb_matrix_block(int nout, const int32_t *__restrict__ ctab,
                                                  const double *__restrict__ beta, double *__restrict__ M) {
  for (int k = threadIdx.x; k < nout * kCombRegs; k += blockDim.x) M[k] = 0.0;
  __syncthreads();
  const int32_t *cptr = ctab, *cidx = ctab + nout + 1, *cterm = cidx + ctab[nout];
  for (int o = threadIdx.x; o < nout; o += blockDim.x)
    for (int e = cptr[o]; e < cptr[o + 1]; ++e) M[o * kCombRegs + cidx[e]] += beta[cterm[e]];
}

template <typename T>
__global__ void __launch_bounds__(256)
k_diag(IndexDev ix, const typename V2<T>::t *__restrict__ x, typename V2<T>::t *__restrict__ y, int nout,
       const int32_t *__restrict__ ctab, const double *__restrict__ beta, double *__restrict__ M) {
  // block 0 also builds the combination's dense coefficient matrix when M is given
  if (M && blockIdx.x == 0) comb_matrix_block(nout, ctab, beta, M);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ix.size) return;
  const int32_t t0 = ix.rowtile[r];
  const int32_t o = (int32_t)(r - ix.tstart[t0]);
  const double dval = (double)(ix.tpsum[t0] + ix.gssum[o]) + 0.5 * ix.N;
  y[r] = scal<T>((T)dval, x[r]);
}

// dst = A X_axis src + Bc src - C prev + plus ; optionally y += beta[term] dst (term >= 0)
// or y += dst (term == kTermOne)
template <typename T>
__global__ void __launch_bounds__(256)
k_pass(IndexDev ix, int axis, double A, double Bc, double Cc,
       const typename V2<T>::t *__restrict__ src, const typename V2<T>::t *__restrict__ prev,
       const typename V2<T>::t *__restrict__ plus, typename V2<T>::t *__restrict__ dst,
       typename V2<T>::t *__restrict__ y, const double *__restrict__ beta, int term) {
  using C = typename V2<T>::t;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ix.size) return;
  const T *wt;
  if constexpr (sizeof(T) == 8) wt = (const T *)ix.wtab; else wt = (const T *)ix.wtabf;
  const int32_t t0 = ix.rowtile[r];
  const Pos p{t0, (int32_t)(r - ix.tstart[t0])};
  const int j = coord(ix, p, axis);
  C xs = vz<T>();
  if (j > 0) fma_rc<T>(xs, wt[j], ld<T>(src, ix, mv(ix, p, axis, 0)));
  fma_rc<T>(xs, wt[j + 1], ld<T>(src, ix, mv(ix, p, axis, 1)));
  const C s0 = src[r];
  C out = scal<T>((T)A, xs);
  fma_rc<T>(out, (T)Bc, s0);
  if (prev) fma_rc<T>(out, (T)(-Cc), prev[r]);
  if (plus) {
    const C pl = plus[r];
    out.x += pl.x;
    out.y += pl.y;
  }
  dst[r] = out;
  if (term != -1) {
    C yy = y[r];
    fma_rc<T>(yy, term >= 0 ? (T)beta[term] : T(1), out);
    y[r] = yy;
  }
}

// A chain of recurrence passes along one axis (steps s = 0 .. nsteps - 1):
//   out_s = A_s X v_s + B_s v_s - C_s v_{s-1} + plus_s,  v_{s+1} = out_s,
// with v_0 = in0 and v_{-1} = prev0 (no term when prev0 is NULL), evaluated per fibre of
// the axis: one workgroup per batch of fibre segments (hs_index_build_fibres), the
// current vector in LDS (a position's fibre neighbours at the distances del gives),
// each position's own values in registers.  Each step performs the operations of k_pass
// in the same order, so the chain gives the passes' results bit for bit.  Halo positions
// are computed but never stored.
template <typename T>
struct ChainArgs {
  const typename V2<T>::t *in0, *prev0;
  const typename V2<T>::t *plus[kChainMax];
  typename V2<T>::t *out[kChainMax];  // NULL: the step's output is not kept
  double A[kChainMax], B[kChainMax], C[kChainMax];
  int32_t term[kChainMax];            // -1: none, >= 0: y += beta[term] out, kTermOne: y += out
  int32_t nsteps;
};

template <typename T>
__global__ void __launch_bounds__(256)
k_chain(const uint64_t *__restrict__ pos, const uint32_t *__restrict__ del, const int64_t *__restrict__ bat,
        ChainArgs<T> a, const T *__restrict__ wt, typename V2<T>::t *__restrict__ y,
        const double *__restrict__ beta) {
  using C = typename V2<T>::t;
  constexpr int PT = kFibBatch / 256;
  __shared__ C cur[kFibBatch];
  const int64_t p0 = bat[blockIdx.x];
  const int n = (int)(bat[blockIdx.x + 1] - p0);
  uint32_t row[PT], dl[PT];
  int kk[PT], fl[PT];
  C v[PT], o[PT];
#pragma unroll
  for (int j = 0; j < PT; ++j) {
    const int i = threadIdx.x + 256 * j;
    fl[j] = 0;
    row[j] = 0;
    dl[j] = 0;
    kk[j] = 0;
    v[j] = o[j] = vz<T>();
    if (i < n) {
      const uint64_t q = pos[p0 + i];
      row[j] = (uint32_t)q;
      kk[j] = (int)((q >> 32) & 0xFFFF);
      fl[j] = (int)(q >> 48) | 8;  // 8: a position of this batch
      dl[j] = del[p0 + i];
      v[j] = a.in0[row[j]];
      if (a.prev0) o[j] = a.prev0[row[j]];
      cur[i] = v[j];
    }
  }
  // the added vector of each step is loaded one step ahead
  C pn[PT];
#pragma unroll
  for (int j = 0; j < PT; ++j) pn[j] = (a.plus[0] && (fl[j] & 8)) ? a.plus[0][row[j]] : vz<T>();
  __syncthreads();
  for (int s = 0; s < a.nsteps; ++s) {
    const T As = (T)a.A[s], Bs = (T)a.B[s], Cs = (T)(-a.C[s]);
    const bool has_pl = a.plus[s] != nullptr;
    const bool use_prev = s > 0 || a.prev0 != nullptr;
    C pc[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) pc[j] = pn[j];
    if (s + 1 < a.nsteps && a.plus[s + 1]) {
      const C *__restrict__ nx = a.plus[s + 1];
#pragma unroll
      for (int j = 0; j < PT; ++j)
        if (fl[j] & 8) pn[j] = nx[row[j]];
    }
    C nv[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const int i = threadIdx.x + 256 * j;
      nv[j] = vz<T>();
      if (fl[j] & 8) {
        C xs = vz<T>();
        if (kk[j] > 0 && (fl[j] & 1)) fma_rc<T>(xs, wt[kk[j]], cur[i - (int)(dl[j] & 0xFFFF)]);
        fma_rc<T>(xs, wt[kk[j] + 1], (fl[j] & 2) ? cur[i + (int)(dl[j] >> 16)] : vz<T>());
        C out = scal<T>(As, xs);
        fma_rc<T>(out, Bs, v[j]);
        if (use_prev) fma_rc<T>(out, Cs, o[j]);
        if (has_pl) {
          out.x += pc[j].x;
          out.y += pc[j].y;
        }
        nv[j] = out;
      }
    }
    __syncthreads();  // every read of cur for this step is done
    C *__restrict__ dst = a.out[s];
    const int term = a.term[s];
#pragma unroll
    for (int j = 0; j < PT; ++j) {
      const int i = threadIdx.x + 256 * j;
      if (fl[j] & 8) {
        o[j] = v[j];
        v[j] = nv[j];
        cur[i] = nv[j];
        if (fl[j] & 4) {
          if (dst) dst[row[j]] = nv[j];
          if (term != -1) {
            C yy = y[row[j]];
            fma_rc<T>(yy, term >= 0 ? (T)beta[term] : T(1), nv[j]);
            y[row[j]] = yy;
          }
        }
      }
    }
    __syncthreads();
  }
}

// The split program's combination fused with the chains that follow it along one axis
// (hs_pot_s cg_op .. cg_end): one workgroup per fibre batch, one position per thread.
// Each position loads the combination's inputs once and forms any combination output a
// chain needs on the spot, with the operations of k_combine_dense in the same order; the
// chains then run as in k_chain.  Source codes: o >= 0 a combination output, -1 none,
// -2 - i the memory input mem[i].
template <typename T>
struct CombChainArgs {
  const typename V2<T>::t *in[kCombRegs];
  const typename V2<T>::t *mem[kCombChains];
  typename V2<T>::t *wtp[kCombChains];  // combination outputs written through ...
  int32_t wt[kCombChains];               // ... and their indices
  int32_t nin, nout, nchains, nwt;
  int32_t nsteps[kCombChains], src0[kCombChains], prev0[kCombChains];
  int32_t plus[kCombChains][kChainMax], term[kCombChains][kChainMax];
  double A[kCombChains][kChainMax], B[kCombChains][kChainMax], C[kCombChains][kChainMax];
  typename V2<T>::t *out[kCombChains][kChainMax];
};

// M (built by the diagonal's first workgroup) is read with addresses uniform across the
// workgroup (scalar loads, no LDS).  With
// COMB = false the same kernel runs a group of independent chains along one axis whose
// inputs all come from memory (no combination), one after the other on each batch.
template <typename T, bool COMB>
__global__ void __launch_bounds__(256)
k_comb_chains(const uint64_t *__restrict__ pos, const uint32_t *__restrict__ del, const int64_t *__restrict__ bat,
              CombChainArgs<T> a, const double *__restrict__ M, const double *__restrict__ beta,
              const T *__restrict__ wt, typename V2<T>::t *__restrict__ y) {
  using C = typename V2<T>::t;
  __shared__ C cur[kFibBatch];
  const int64_t p0 = bat[blockIdx.x];
  const int n = (int)(bat[blockIdx.x + 1] - p0);
  const int i = threadIdx.x;
  const bool valid = i < n;
  uint32_t row = 0, dl = 0;
  int kk = 0, fl = 0;
  if (valid) {
    const uint64_t q = pos[p0 + i];
    row = (uint32_t)q;
    kk = (int)((q >> 32) & 0xFFFF);
    fl = (int)(q >> 48);
    dl = del[p0 + i];
  }
  constexpr int NI = COMB ? kCombRegs : 1;
  C in[NI];
#pragma unroll
  for (int r = 0; r < NI; ++r) in[r] = (COMB && valid && r < a.nin) ? a.in[r][row] : vz<T>();
  auto comb = [&](int o) {
    C acc = vz<T>();
#pragma unroll
    for (int r = 0; r < NI; ++r) fma_rc<T>(acc, (T)M[o * kCombRegs + r], in[r]);
    return acc;
  };
  auto source = [&](int code) -> C {
    if (COMB && code >= 0) return comb(code);
    if (code < -1 && valid) return a.mem[-2 - code][row];
    return vz<T>();
  };
  if (COMB && valid && (fl & 4))
    for (int w = 0; w < a.nwt; ++w) a.wtp[w][row] = comb(a.wt[w]);
  for (int g = 0; g < a.nchains; ++g) {
    C v = source(a.src0[g]);
    const bool has_prev0 = a.prev0[g] != -1;
    C o = has_prev0 ? source(a.prev0[g]) : vz<T>();
    if (valid) cur[i] = v;
    __syncthreads();
    for (int s = 0; s < a.nsteps[g]; ++s) {
      const bool has_pl = a.plus[g][s] != -1;
      const C pc = has_pl ? source(a.plus[g][s]) : vz<T>();
      C nv = vz<T>();
      if (valid) {
        C xs = vz<T>();
        if (kk > 0 && (fl & 1)) fma_rc<T>(xs, wt[kk], cur[i - (int)(dl & 0xFFFF)]);
        fma_rc<T>(xs, wt[kk + 1], (fl & 2) ? cur[i + (int)(dl >> 16)] : vz<T>());
        C out = scal<T>((T)a.A[g][s], xs);
        fma_rc<T>(out, (T)a.B[g][s], v);
        if (s > 0 || has_prev0) fma_rc<T>(out, (T)(-a.C[g][s]), o);
        if (has_pl) {
          out.x += pc.x;
          out.y += pc.y;
        }
        nv = out;
      }
      __syncthreads();  // every read of cur for this step is done
      if (valid) {
        o = v;
        v = nv;
        cur[i] = nv;
        if (fl & 4) {
          if (a.out[g][s]) a.out[g][s][row] = nv;
          const int term = a.term[g][s];
          if (term != -1) {
            C yy = y[row];
            fma_rc<T>(yy, term >= 0 ? (T)beta[term] : T(1), nv);
            y[row] = yy;
          }
        }
      }
      __syncthreads();
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_accum(int64_t n, const typename V2<T>::t *__restrict__ src, typename V2<T>::t *__restrict__ y,
        const double *__restrict__ beta, int term) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  typename V2<T>::t yy = y[r];
  fma_rc<T>(yy, term >= 0 ? (T)beta[term] : T(1), src[r]);
  y[r] = yy;
}

// Combination of a split program: out_o = sum_{e in [cptr[o], cptr[o+1])} beta[cterm[e]] *
// in_{cidx[e]}, row by row.  Each thread keeps its row's inputs in LDS (64 rows per block).
struct CombSlots {
  int32_t nin, nout;
  int32_t in[kMaxComb], out[kMaxComb];
};

template <typename T>
__global__ void __launch_bounds__(64)
k_combine(int64_t n, CombSlots cs, const typename V2<T>::t *__restrict__ x, typename V2<T>::t *__restrict__ y,
          typename V2<T>::t *__restrict__ ws, int64_t stride, const int32_t *__restrict__ ctab,
          const double *__restrict__ beta) {
  using C = typename V2<T>::t;
  extern __shared__ __align__(16) unsigned char csm[];
  C *V = reinterpret_cast<C *>(csm);
  const int64_t r = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (r >= n) return;  // rows are independent: no barrier below
  auto slot = [&](int k) -> C * {
    if (k == 0) return const_cast<C *>(x);
    if (k == 1) return y;
    return ws + (int64_t)(k - 2) * stride;
  };
  for (int i = 0; i < cs.nin; ++i) V[i * 64 + threadIdx.x] = slot(cs.in[i])[r];
  const int32_t *cptr = ctab, *cidx = ctab + cs.nout + 1, *cterm = cidx + ctab[cs.nout];
  for (int o = 0; o < cs.nout; ++o) {
    C acc = vz<T>();
    for (int e = cptr[o]; e < cptr[o + 1]; ++e) fma_rc<T>(acc, (T)beta[cterm[e]], V[cidx[e] * 64 + threadIdx.x]);
    slot(cs.out[o])[r] = acc;
  }
}

// The same combination for at most kCombRegs inputs, as a dense product: every thread
// loads its row of all inputs into registers at once (the loads overlap), and the block
// first gathers the table into a dense coefficient matrix M[o][i] = sum of beta over the
// entries (o, i) in LDS, read back with one address across the wave.
template <typename T>
__global__ void __launch_bounds__(256)
k_combine_dense(int64_t n, CombSlots cs, const typename V2<T>::t *__restrict__ x, typename V2<T>::t *__restrict__ y,
                typename V2<T>::t *__restrict__ ws, int64_t stride, const int32_t *__restrict__ ctab,
                const double *__restrict__ beta) {
  using C = typename V2<T>::t;
  __shared__ double M[kMaxComb * kCombRegs];
  for (int k = threadIdx.x; k < cs.nout * kCombRegs; k += blockDim.x) M[k] = 0.0;
  __syncthreads();
  const int32_t *cptr = ctab, *cidx = ctab + cs.nout + 1, *cterm = cidx + ctab[cs.nout];
  for (int o = threadIdx.x; o < cs.nout; o += blockDim.x)
    for (int e = cptr[o]; e < cptr[o + 1]; ++e) M[o * kCombRegs + cidx[e]] += beta[cterm[e]];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  auto slot = [&](int k) -> C * {
    if (k == 0) return const_cast<C *>(x);
    if (k == 1) return y;
    return ws + (int64_t)(k - 2) * stride;
  };
  C in[kCombRegs];
#pragma unroll
  for (int i = 0; i < kCombRegs; ++i) in[i] = i < cs.nin ? slot(cs.in[i])[r] : vz<T>();
  for (int o = 0; o < cs.nout; ++o) {
    C acc = vz<T>();
#pragma unroll
    for (int i = 0; i < kCombRegs; ++i) fma_rc<T>(acc, (T)M[o * kCombRegs + i], in[i]);
    slot(cs.out[o])[r] = acc;
  }
}

// y = out_scale * y - prev_coef * prev_scale * prev (epilogue of the generic program)
template <typename T>
__global__ void __launch_bounds__(256)
k_epilogue(int64_t n, typename V2<T>::t *__restrict__ y, const double *__restrict__ out_scale,
           const typename V2<T>::t *__restrict__ prev, const double *__restrict__ prev_coef,
           const double *__restrict__ prev_scale) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  typename V2<T>::t a = y[r];
  if (out_scale) a = scal<T>((T)*out_scale, a);
  if (prev) fma_rc<T>(a, (T)(-(*prev_coef) * (prev_scale ? *prev_scale : 1.0)), prev[r]);
  y[r] = a;
}

// ---- host launchers -------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

int32_t launch_set_time(const hs_pot_s *p, void *pot_dev, double t, const double *t_dev,
                        double dt, hipStream_t s) {
  uint8_t *b = static_cast<uint8_t *>(pot_dev);
  hipLaunchKernelGGL(k_set_time, dim3(1), dim3(256), 0, s, p->nterms, p->fused ? p->nslots : 0,
                     (const double *)(b + p->off_base), (const double *)(b + p->off_amp),
                     (const double *)(b + p->off_freq), (const double *)(b + p->off_phase),
                     (const double *)(b + p->off_M), (double *)(b + p->off_beta),
                     (double *)(b + p->off_hh), t, t_dev, dt);
  HS_HIP(hipGetLastError());
  return HS_OK;
}

int32_t launch_copy_coeffs(const hs_pot_s *p, void *pot_dev, const double *coef, hipStream_t s) {
  uint8_t *b = static_cast<uint8_t *>(pot_dev);
  hipLaunchKernelGGL(k_copy_coeffs, dim3(1), dim3(256), 0, s, p->nterms, coef,
                     (double *)(b + p->off_base), (double *)(b + p->off_amp));
  HS_HIP(hipGetLastError());
  return HS_OK;
}

int64_t apply_workspace_bytes(const hs_index_s *idx, const hs_pot_s *p, int32_t dtype) {
  if (p->fused) return 0;
  const int64_t es = dtype == HS_C64 ? 8 : 16;
  // slots 0 (input) and 1 (output) are the caller's vectors; then the dense coefficient
  // matrix of a combination fused with its chains
  return align_up(idx->size * es, 256) * std::max(0, p->nslots_vec - 2) +
         (p->cg_op >= 0 ? (int64_t)sizeof(double) * kMaxComb * kCombRegs : 0);
}

template <typename T>
static int32_t apply_impl(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p,
                          const void *pot_dev, const void *x, void *y, void *ws, hipStream_t s,
                          const double *out_scale, const void *prev, const double *prev_coef,
                          const double *prev_scale) {
  using C = typename V2<T>::t;
  const IndexDev ix = idx->view(idx_dev);
  const uint8_t *pb = static_cast<const uint8_t *>(pot_dev);
  const double *hh = (const double *)(pb + p->off_hh);
  const double *beta = (const double *)(pb + p->off_beta);
  const unsigned g = nblk(idx->size, 256);
  if (idx->size == 0) return HS_OK;
  if (p->form == HS_FORM_SYM && idx->kind != HS_SET_HYPERBOLIC)
    return fail(HS_E_UNSUPPORTED, "symmetrised form: served on hyperbolic sets only");
  if (p->fused && p->form == HS_FORM_SYM) {
    // the symmetrised operator exists only as the specialised kernel serving every row
    const int done = sizeof(T) == 8
        ? launch_hh_long_sym_f64(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, p->x2)
        : launch_hh_long_sym_f32(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, p->x2);
    if (done != 1)
      return fail(HS_E_UNSUPPORTED, "symmetrised form: no specialised kernel for this index set");
    HS_HIP(hipGetLastError());
    return HS_OK;
  }
  if (p->fused && !p->x2) {
    // long tiles: work items of several tiles (any vector size)
    const int multi = sizeof(T) == 8
        ? launch_hh_multi_f64(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, p->x2)
        : launch_hh_multi_f32(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, p->x2);
    if (multi != 0) {
      if (multi == 2 && ix.nsmall > 0) {
        const int done = sizeof(T) == 8
            ? launch_hh_short_f64(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, p->x2)
            : launch_hh_short_f32(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, p->x2);
        if (done != 1)
          hipLaunchKernelGGL(k_hh_rows<T>, dim3(nblk(ix.nsmall, 256)), dim3(256), 0, s, ix, hh,
                             (const C *)x, (C *)y, out_scale, (const C *)prev, prev_coef, prev_scale,
                             ix.small_rows, ix.nsmall);
      }
      HS_HIP(hipGetLastError());
      return HS_OK;
    }
  }
  if (p->fused) {
    const int done = sizeof(T) == 8
        ? launch_hh_long_f64(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, p->x2)
        : launch_hh_long_f32(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, p->x2);
    if (done == 0 && ix.nchunks > 0)
      hipLaunchKernelGGL(k_hh_tiles<T>, dim3(nblk(ix.nchunks * kChunk, 256)), dim3(256), 0, s, ix, hh,
                         (const C *)x, (C *)y, out_scale, (const C *)prev, prev_coef, prev_scale);
    if (done != 1 && ix.nsmall > 0)
      hipLaunchKernelGGL(k_hh_rows<T>, dim3(nblk(ix.nsmall, 256)), dim3(256), 0, s, ix, hh,
                         (const C *)x, (C *)y, out_scale, (const C *)prev, prev_coef, prev_scale,
                         ix.small_rows, ix.nsmall);
    HS_HIP(hipGetLastError());
    return HS_OK;
  }
  const int64_t stride = align_up(idx->size * (int64_t)sizeof(C), 256);
  auto slot = [&](int k) -> C * {
    if (k == 0) return (C *)x;
    if (k == 1) return (C *)y;
    return (C *)((uint8_t *)ws + (int64_t)(k - 2) * stride);
  };
  // (fibres built after the last upload are not in the device block yet: not used)
  const bool chains = idx->fibres && idx->fibres_uploaded && p->chain.size() == p->prog.size();
  const bool fuse_comb = chains && p->cg_op >= 0 && (int)p->cg_wt.size() <= kCombChains;
  // the fused combination's coefficient matrix, after the slots in the workspace; the
  // diagonal's first workgroup builds it
  double *Mg = fuse_comb ? reinterpret_cast<double *>(static_cast<uint8_t *>(ws) +
                                                       align_up(idx->size * (int64_t)sizeof(C), 256) *
                                                           std::max(0, p->nslots_vec - 2))
                         : nullptr;
  hipLaunchKernelGGL(k_diag<T>, dim3(g), dim3(256), 0, s, ix, (const C *)x, (C *)y, (int)p->cout_slot.size(),
                     (const int32_t *)(pb + p->off_comb), beta, Mg);
  const uint8_t *ib = static_cast<const uint8_t *>(idx_dev);
  const T *wtab = sizeof(T) == 8 ? (const T *)ix.wtab : (const T *)ix.wtabf;
  for (size_t pi = 0; pi < p->prog.size(); ++pi) {
    const PassOp &op = p->prog[pi];
    if (fuse_comb && (int)pi == p->cg_op) {
      // the combination and the chains after it along one axis: one launch
      CombChainArgs<T> ca{};
      ca.nin = (int32_t)p->cin_slot.size();
      ca.nout = (int32_t)p->cout_slot.size();
      for (int r = 0; r < ca.nin; ++r) ca.in[r] = slot(p->cin_slot[r]);
      ca.nwt = (int32_t)p->cg_wt.size();
      for (int w = 0; w < ca.nwt; ++w) {
        ca.wt[w] = p->cg_wt[w];
        ca.wtp[w] = slot(p->cout_slot[p->cg_wt[w]]);
      }
      int nmem = 0;
      auto code = [&](int sl) -> int32_t {
        if (sl < 0) return -1;
        for (int o = 0; o < ca.nout; ++o)
          if (p->cout_slot[o] == sl) return o;
        for (int m = 0; m < nmem; ++m)
          if (ca.mem[m] == slot(sl)) return -2 - m;
        ca.mem[nmem] = slot(sl);
        return -2 - nmem++;
      };
      int g = 0;
      for (int j = p->cg_op + 1; j < p->cg_end; j += p->chain[j], ++g) {
        const int K = p->chain[j];
        ca.nsteps[g] = K;
        ca.src0[g] = code(p->prog[j].src);
        ca.prev0[g] = code(p->prog[j].prev);
        for (int q = 0; q < K; ++q) {
          const PassOp &oq = p->prog[j + q];
          ca.plus[g][q] = code(oq.plus);
          ca.term[g][q] = oq.term;
          ca.A[g][q] = oq.A;
          ca.B[g][q] = oq.Bc;
          ca.C[g][q] = oq.C;
          ca.out[g][q] = p->keep[j + q] ? slot(oq.dst) : nullptr;
        }
      }
      ca.nchains = g;
      const int l = p->prog[p->cg_op + 1].axis;
      const uint64_t *fpos = reinterpret_cast<const uint64_t *>(ib + idx->off_fpos) + idx->fpos0[l];
      const uint32_t *fdel = reinterpret_cast<const uint32_t *>(ib + idx->off_fdel) + idx->fpos0[l];
      const int64_t *fbat = reinterpret_cast<const int64_t *>(ib + idx->off_fbat) + idx->fbat0[l];
      if (idx->fnb[l] > 0)
        hipLaunchKernelGGL((k_comb_chains<T, true>), dim3((unsigned)idx->fnb[l]), dim3(256), 0, s, fpos, fdel, fbat,
                           ca, (const double *)Mg, beta, wtab, (C *)y);
      pi = (size_t)p->cg_end - 1;
      continue;
    }
    if (chains && pi < p->mc_end.size() && p->mc_end[pi] > 0) {
      // independent chains along one axis, reading memory only: one launch
      CombChainArgs<T> ca{};
      int nmem = 0;
      auto code = [&](int sl) -> int32_t {
        if (sl < 0) return -1;
        for (int m = 0; m < nmem; ++m)
          if (ca.mem[m] == slot(sl)) return -2 - m;
        ca.mem[nmem] = slot(sl);
        return -2 - nmem++;
      };
      int g = 0;
      for (int j = (int)pi; j < p->mc_end[pi]; j += p->chain[j], ++g) {
        const int K = p->chain[j];
        ca.nsteps[g] = K;
        ca.src0[g] = code(p->prog[j].src);
        ca.prev0[g] = code(p->prog[j].prev);
        for (int q = 0; q < K; ++q) {
          const PassOp &oq = p->prog[j + q];
          ca.plus[g][q] = code(oq.plus);
          ca.term[g][q] = oq.term;
          ca.A[g][q] = oq.A;
          ca.B[g][q] = oq.Bc;
          ca.C[g][q] = oq.C;
          ca.out[g][q] = p->keep[j + q] ? slot(oq.dst) : nullptr;
        }
      }
      ca.nchains = g;
      const int l = op.axis;
      const uint64_t *fpos = reinterpret_cast<const uint64_t *>(ib + idx->off_fpos) + idx->fpos0[l];
      const uint32_t *fdel = reinterpret_cast<const uint32_t *>(ib + idx->off_fdel) + idx->fpos0[l];
      const int64_t *fbat = reinterpret_cast<const int64_t *>(ib + idx->off_fbat) + idx->fbat0[l];
      if (idx->fnb[l] > 0)
        hipLaunchKernelGGL((k_comb_chains<T, false>), dim3((unsigned)idx->fnb[l]), dim3(256), 0, s, fpos, fdel,
                           fbat, ca, (const double *)nullptr, beta, wtab, (C *)y);
      pi = (size_t)p->mc_end[pi] - 1;
      continue;
    }
    if (chains && p->chain[pi] >= 2) {
      // a chain of passes along op.axis: one launch over the axis's fibre batches
      const int K = p->chain[pi];
      ChainArgs<T> ca{};
      ca.in0 = slot(op.src);
      ca.prev0 = op.prev >= 0 ? slot(op.prev) : nullptr;
      ca.nsteps = K;
      for (int q = 0; q < K; ++q) {
        const PassOp &oq = p->prog[pi + q];
        ca.plus[q] = oq.plus >= 0 ? slot(oq.plus) : nullptr;
        ca.out[q] = p->keep[pi + q] ? slot(oq.dst) : nullptr;
        ca.A[q] = oq.A;
        ca.B[q] = oq.Bc;
        ca.C[q] = oq.C;
        ca.term[q] = oq.term;
      }
      const int l = op.axis;
      const uint64_t *fpos = reinterpret_cast<const uint64_t *>(ib + idx->off_fpos) + idx->fpos0[l];
      const uint32_t *fdel = reinterpret_cast<const uint32_t *>(ib + idx->off_fdel) + idx->fpos0[l];
      const int64_t *fbat = reinterpret_cast<const int64_t *>(ib + idx->off_fbat) + idx->fbat0[l];
      if (idx->fnb[l] > 0)
        hipLaunchKernelGGL(k_chain<T>, dim3((unsigned)idx->fnb[l]), dim3(256), 0, s, fpos, fdel, fbat, ca, wtab,
                           (C *)y, beta);
      pi += K - 1;
      continue;
    }
    if (op.kind == 0) {
      hipLaunchKernelGGL(k_pass<T>, dim3(g), dim3(256), 0, s, ix, op.axis, op.A, op.Bc, op.C,
                         (const C *)slot(op.src), op.prev >= 0 ? (const C *)slot(op.prev) : nullptr,
                         op.plus >= 0 ? (const C *)slot(op.plus) : nullptr, slot(op.dst), (C *)y, beta, op.term);
    } else if (op.kind == 1) {
      hipLaunchKernelGGL(k_accum<T>, dim3(g), dim3(256), 0, s, idx->size, (const C *)slot(op.src),
                         (C *)y, beta, op.term);
    } else {
      CombSlots cs{};
      cs.nin = (int32_t)p->cin_slot.size();
      cs.nout = (int32_t)p->cout_slot.size();
      for (int i = 0; i < cs.nin; ++i) cs.in[i] = p->cin_slot[i];
      for (int i = 0; i < cs.nout; ++i) cs.out[i] = p->cout_slot[i];
      if (cs.nin <= kCombRegs) {
        hipLaunchKernelGGL(k_combine_dense<T>, dim3(g), dim3(256), 0, s, idx->size, cs, (const C *)x, (C *)y,
                           (C *)ws, stride / (int64_t)sizeof(C), (const int32_t *)(pb + p->off_comb), beta);
      } else {
        const size_t lds = sizeof(C) * 64 * (size_t)std::max(cs.nin, 1);
        hipLaunchKernelGGL(k_combine<T>, dim3(nblk(idx->size, 64)), dim3(64), lds, s, idx->size, cs,
                           (const C *)x, (C *)y, (C *)ws, stride / (int64_t)sizeof(C),
                           (const int32_t *)(pb + p->off_comb), beta);
      }
    }
  }
  if (out_scale || prev)
    hipLaunchKernelGGL(k_epilogue<T>, dim3(g), dim3(256), 0, s, idx->size, (C *)y, out_scale,
                       (const C *)prev, prev_coef, prev_scale);
  HS_HIP(hipGetLastError());
  return HS_OK;
}

int32_t launch_apply(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p,
                     const void *pot_dev, int32_t dtype, const void *x, void *y, void *ws,
                     hipStream_t s, const double *out_scale, const void *prev,
                     const double *prev_coef, const double *prev_scale) {
  if (dtype == HS_C128)
    return apply_impl<double>(idx, idx_dev, p, pot_dev, x, y, ws, s, out_scale, prev, prev_coef, prev_scale);
  return apply_impl<float>(idx, idx_dev, p, pot_dev, x, y, ws, s, out_scale, prev, prev_coef, prev_scale);
}

// y = X^(axis) x alone: one pass with A = 1 and nothing added
int32_t launch_apply_x(const hs_index_s *idx, const void *idx_dev, int32_t axis, int32_t dtype,
                       const void *x, void *y, hipStream_t s) {
  if (idx->size == 0) return HS_OK;
  const IndexDev ix = idx->view(idx_dev);
  const unsigned g = nblk(idx->size, 256);
  if (dtype == HS_C128) {
    using C = V2<double>::t;
    hipLaunchKernelGGL(k_pass<double>, dim3(g), dim3(256), 0, s, ix, (int)axis, 1.0, 0.0, 0.0, (const C *)x,
                       nullptr, nullptr, (C *)y, nullptr, nullptr, -1);
  } else {
    using C = V2<float>::t;
    hipLaunchKernelGGL(k_pass<float>, dim3(g), dim3(256), 0, s, ix, (int)axis, 1.0, 0.0, 0.0, (const C *)x,
                       nullptr, nullptr, (C *)y, nullptr, nullptr, -1);
  }
  HS_HIP(hipGetLastError());
  return HS_OK;
}

}  // namespace hs
