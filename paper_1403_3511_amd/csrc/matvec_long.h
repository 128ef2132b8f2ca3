// Fused two-axis H application specialised at compile time on the dimension N and the
// number of prefix axes NP (paper Sec. 3.2, eq. Horner, for the potential class
// a1 x_l + a2 x_l^2 + a3 x_l^3 + g1 x_l x_{l+1} + g2 x_l^2 x_{l+1}).
//
// Long tiles: one wave handles 64 consecutive rows (offsets o0..o0+63) of one tile.  The
// tile's record gives, in one scalar fetch, the first row and length of every neighbour
// tile that the stencil reaches along the prefix axes; there the neighbour of a row is
// the same offset, so those loads are contiguous across the wave.  Neighbours along
// suffix axes come from the per-offset suffix stencil.  Short tiles: one lane per listed
// row, the same code with the record fetched per lane.  Both run in one launch.
//
// X2 = false drops the x_l^2 and x_l x_{l+1} monomials (absent in the Henon-Heiles
// class) at compile time.
//
// SYM = true evaluates the symmetrised operator D + (F + F_rev)/2: the coupling terms
// x_l^a x_{l+1} (a = 1, 2) are averaged over both factor orders.  The reversed order,
// X_{l+1} (X_l^a c), needs c at the same cross positions j + s e_l + r e_{l+1} as the
// paper's order; only which of them count differs (the intermediate j + r e_{l+1} must
// lie in K instead of j + s e_l), and that is decided from the product prod(1 + j_i).
#pragma once

#include "dev_common.h"

namespace hs {

// Complex loads through a structured buffer resource: the element index times the record
// stride (the complex size), checked against the record count.  An absent neighbour gets
// an index beyond every vector (kAbsent), for which the hardware returns zero, so no
// predication or select is needed, and 32-bit indices reach vectors of up to 2^32 - 1
// elements without 64-bit address arithmetic.
constexpr uint32_t kAbsent = 0xFFFFFFFFu;  // element index that is always out of range

typedef int hs_v4i __attribute__((ext_vector_type(4)));
typedef int hs_v2i __attribute__((ext_vector_type(2)));
__device__ hs_v4i hs_struct_load_b128(__amdgpu_buffer_rsrc_t rsrc, int vindex, int voffset, int soffset,
                                      int aux) __asm("llvm.amdgcn.struct.ptr.buffer.load.v4i32");
__device__ hs_v2i hs_struct_load_b64(__amdgpu_buffer_rsrc_t rsrc, int vindex, int voffset, int soffset,
                                     int aux) __asm("llvm.amdgcn.struct.ptr.buffer.load.v2i32");

// The structured loads address element i at byte i * stride, and that product is formed
// in 32 bits: past 2^32 bytes it wraps around, silently, to the start of the vector.  The
// kernels that use them therefore serve only vectors of at most 2^32 bytes; larger ones
// take the kernels with 64-bit addressing.
template <typename T>
inline bool struct_loads_reach(int64_t n) {
  return n * (int64_t)sizeof(typename V2<T>::t) <= (INT64_C(1) << 32);
}

// resource over n complex elements of type V2<T>
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t vec_rsrc(const void *x, int64_t n) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)x, (short)sizeof(typename V2<T>::t), (int)n, 0x00020000);
}

template <typename T> struct BufLoad;
template <> struct BufLoad<double> {
  static __device__ __forceinline__ double2 ld(__amdgpu_buffer_rsrc_t r, uint32_t i) {
    const hs_v4i v = hs_struct_load_b128(r, (int)i, 0, 0, 0);
    double2 d;
    __builtin_memcpy(&d, &v, 16);
    return d;
  }
};
template <> struct BufLoad<float> {
  static __device__ __forceinline__ float2 ld(__amdgpu_buffer_rsrc_t r, uint32_t i) {
    const hs_v2i v = hs_struct_load_b64(r, (int)i, 0, 0, 0);
    float2 d;
    __builtin_memcpy(&d, &v, 8);
    return d;
  }
};

// Window weights sqrt((j + s) / 2), s = -2..3, from the zero-padded table (entry k + 2
// holds sqrt(k / 2)): six consecutive values in two or three vector loads.
template <typename T> struct WinLoad;
template <> struct WinLoad<double> {
  static __device__ __forceinline__ void ld(__amdgpu_buffer_rsrc_t r, int j, double *w) {
    static_for<0, 3>([&](auto I) {
      constexpr int i = decltype(I)::value;
      const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (j + 2 * i) << 3, 0, 0);
      __builtin_memcpy(w + 2 * i, &v, 16);
    });
  }
};
template <> struct WinLoad<float> {
  static __device__ __forceinline__ void ld(__amdgpu_buffer_rsrc_t r, int j, float *w) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, j << 2, 0, 0);
    __builtin_memcpy(w, &v, 16);
    const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, (j + 4) << 2, 0, 0);
    __builtin_memcpy(w + 4, &u, 8);
  }
};

// One group per axis l, skipped as a whole when its coefficients vanish (uniform
// branch).  Coefficients are folded into the edge weights: with u_s = c(j + s e_l) and
// v_s = (X_{l+1} c)(j + s e_l),
//   h2_s = a3 (e_s u_{s-1} + e_{s+1} u_{s+1}) + a2 u_s + g2 v_s      (s = -2, 0, 2)
//   h1_s = e_s h2_{s-1} + e_{s+1} h2_{s+1} + a1 u_s + g1 v_s          (s = -1, 1)
//   G_l  = e_0 h1_{-1} + e_1 h1_1.
// One row (offset o of the tile whose record is rec) of oscale (D + W) x - pcoef prev.
template <typename T, int N, int NP, bool X2, bool SYM>
__device__ __forceinline__ typename V2<T>::t hh_row_value(const IndexDev &ix, const double *__restrict__ hh,
                                                          const typename V2<T>::t *__restrict__ x,
                                                          const int32_t *__restrict__ rec, int32_t o, T oscale,
                                                          const typename V2<T>::t *__restrict__ prev, T pcoef) {
  using C = typename V2<T>::t;
  constexpr int D = N - NP;
  const __amdgpu_buffer_rsrc_t xr = vec_rsrc<T>(x, ix.size);
  const uint32_t base = (uint32_t)rec[0];
  const int32_t len = rec[1];
  HS_DCHECK(ix, rec[0] >= 0 && len >= 0 && (int64_t)rec[0] + len <= ix.size && o >= 0 && o < len &&
                    (int64_t)o < ix.ng, kDbgRecord);
  const T *__restrict__ wt;
  if constexpr (sizeof(T) == 8) wt = (const T *)ix.wtab; else wt = (const T *)ix.wtabf;
  const int64_t ng = ix.ng;
  const int2 *__restrict__ gst2 = reinterpret_cast<const int2 *>(ix.gst);
  const __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc(
      (void *)(sizeof(T) == 8 ? (const void *)ix.wtp : (const void *)ix.wtpf), (short)0,
      (int)((ix.B + 10) * (int)sizeof(T)), 0x00020000);
  int sc[D];
  int ssum = 0;
  {
    const uint64_t pk = ix.gsp[o];  // suffix coordinates, 16 bits each (D <= 4)
    static_for<0, D>([&](auto A) {
      constexpr int a = decltype(A)::value;
      sc[a] = (int)((pk >> (16 * a)) & 0xFFFFu);
      ssum += sc[a];
    });
  }
  const uint32_t self = base + (uint32_t)o;
  const C c0 = x[self];
  // prod(1 + j_i), exact in double (membership tests of the reversed factor order)
  double pj = 1.0;
  if constexpr (SYM) {
    static_for<0, NP>([&](auto I) { pj *= (double)(1 + rec[4 + decltype(I)::value]); });
    static_for<0, D>([&](auto A) { pj *= (double)(1 + sc[decltype(A)::value]); });
  }
  // the previous Lanczos vector is needed only at the end: issue its load now so that
  // its latency overlaps the stencil work
  C pv = vz<T>();
  if (prev) pv = prev[self];
  const double dval = (double)(rec[2] + ssum) + 0.5 * N + hh[5 * N];
  C acc = scal<T>((T)dval, c0);

  // Groups run from axis N down to axis 1.  Group l loads c(j -+ e_l) and the weights
  // sqrt(j_l / 2), sqrt((j_l + 1) / 2) for its own window; group l - 1 needs exactly
  // these as (X_l c)(j) ingredients, so they are carried instead of loaded again.
  C car_lo = vz<T>(), car_hi = vz<T>();
  T car_wlo = T(0), car_whi = T(0);
  bool have_car = false;  // uniform: whether the previous group produced the carry

  static_for<0, N>([&](auto L) {
    constexpr int l = N - 1 - decltype(L)::value;
    constexpr bool inner = (l + 1 < N);
    const T a1 = (T)hh[5 * l + 0], a3 = (T)hh[5 * l + 2];
    const T a2 = X2 ? (T)hh[5 * l + 1] : T(0);
    // symmetrised: each factor order carries half of the coupling coefficient
    const T g1 = (X2 && inner) ? (T)(SYM ? 0.5 * hh[5 * l + 3] : hh[5 * l + 3]) : T(0);
    const T g2 = inner ? (T)(SYM ? 0.5 * hh[5 * l + 4] : hh[5 * l + 4]) : T(0);
    const bool any2 = (a3 != T(0)) || (a2 != T(0)) || (g2 != T(0));
    const bool need3 = (a3 != T(0));
    const bool in_car = have_car;
    const C in_lo = car_lo, in_hi = car_hi;
    const T in_wlo = car_wlo, in_whi = car_whi;
    have_car = false;
    if (!any2 && a1 == T(0) && g1 == T(0)) return;  // uniform: group absent
    // ---- window j + s e_l, s = -3..3: element offset (kAbsent if outside K) ----
    uint32_t id[7];
    bool val[7];
    int32_t stw[7], lnw[7];
    int jl;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      id[q] = kAbsent;
      val[q] = false;
      stw[q] = (int32_t)base;
      lnw[q] = len;
    }
    id[3] = self;
    val[3] = true;
    if constexpr (l < NP) {
      jl = rec[4 + l];
#pragma unroll
      for (int s = -3; s <= 3; ++s) {
        if (s == 0) continue;
        const int p = rec_axis(NP, l, s);
        const int32_t st = rec[p], ln = rec[p + 1];
        HS_DCHECK(ix, ln == 0 || (st >= 0 && ln > 0 && (int64_t)st + ln <= ix.size), kDbgRecord);
        stw[3 + s] = st;
        lnw[3 + s] = ln;
        val[3 + s] = o < ln;
        id[3 + s] = val[3 + s] ? (uint32_t)(st + o) : kAbsent;
      }
    } else {
      constexpr int a = l - NP;
      jl = sc[a];
#pragma unroll
      for (int s = 1; s <= 3; ++s) {
        if (s == 2 && !any2) continue;
        if (s == 3 && !need3) continue;
        const int2 pr = gst2[gst_axis_pair(a, s) * ng + o];  // (-s, +s)
        const int32_t ou = pr.y, od = pr.x;
        HS_DCHECK(ix, (od == -1 || (od >= 0 && od < ng)) && (ou == -1 || (ou >= 0 && ou < ng)), kDbgSuffix);
        val[3 + s] = (uint32_t)ou < (uint32_t)len;
        val[3 - s] = od >= 0;
        id[3 + s] = val[3 + s] ? base + (uint32_t)ou : kAbsent;
        id[3 - s] = val[3 - s] ? base + (uint32_t)od : kAbsent;
      }
    }
    if (!any2) val[1] = val[5] = false;
    if (!need3) val[0] = val[6] = false;
    // edge weights e_s (edge between s-1 and s), a3 folded in for the innermost level
    T raw[6], e[6], ea3[6];
    if constexpr (l >= NP) WinLoad<T>::ld(wr, jl, raw);  // per-lane coordinate
#pragma unroll
    for (int s = -2; s <= 3; ++s) {
      const int k = jl + s;
      if constexpr (l < NP) raw[s + 2] = wt[k > 0 ? k : 0];  // uniform: scalar loads
      const T w = (val[3 + s - 1] && val[3 + s]) ? raw[s + 2] : T(0);
      e[s + 2] = w;
      ea3[s + 2] = w * a3;
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) HS_DCHECK(ix, !val[q] || id[q] < (uint64_t)ix.size, kDbgNeighbour);
    C u[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) u[q] = vz<T>();
    u[3] = c0;
    u[2] = BufLoad<T>::ld(xr, id[2]);
    u[4] = BufLoad<T>::ld(xr, id[4]);
    if (need3) {
      u[0] = BufLoad<T>::ld(xr, id[0]);
      u[6] = BufLoad<T>::ld(xr, id[6]);
    }
    if constexpr (X2) {
      if (a2 != T(0)) {
        u[1] = BufLoad<T>::ld(xr, id[1]);
        u[5] = BufLoad<T>::ld(xr, id[5]);
      }
    }
    // carry for group l - 1: c(j -+ e_l) and the weights at j_l, j_l + 1
    car_lo = u[2];
    car_hi = u[4];
    car_wlo = raw[2];
    car_whi = raw[3];
    have_car = true;
    // ---- h2 at s = -2, 0, 2 ----
    C h2[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int s = 2 * q - 2;
      C h = vz<T>();
      fma_rc<T>(h, ea3[s + 2], u[3 + s - 1]);
      fma_rc<T>(h, ea3[s + 3], u[3 + s + 1]);
      if constexpr (X2) fma_rc<T>(h, a2, u[3 + s]);
      h2[q] = h;
    }
    // inner axis: g2 (X_{l+1} c) at s = -2, 0, 2 into h2; g1 at s = -1, 1 into h1
    C v1[2] = {vz<T>(), vz<T>()};
    if constexpr (inner) {
      if (g1 != T(0) || g2 != T(0)) {
        constexpr int m = l + 1;
        T wlo, whi;
        if (in_car) {
          wlo = in_wlo;
          whi = in_whi;
        } else {
          int jm;
          if constexpr (m < NP) jm = rec[4 + m]; else jm = sc[m - NP];
          wlo = wt[jm];
          whi = wt[jm + 1];
        }
        int32_t o_lo = -1, o_hi = -1;
        if constexpr (m == NP) {  // l prefix, l+1 the first suffix axis
          const int2 pr = gst2[gst_axis_pair(0, 1) * ng + o];
          o_lo = pr.x;
          o_hi = pr.y;
        }
        // symmetrised form: c at j + s e_l -+ e_{l+1}, whether or not j + s e_l is in K
        C xs_lo[5], xs_hi[5];
        if constexpr (SYM) {
#pragma unroll
          for (int q = 0; q < 5; ++q) xs_lo[q] = xs_hi[q] = vz<T>();
        }
#pragma unroll
        for (int s = -2; s <= 2; ++s) {
          if (!X2 && (s & 1)) continue;
          const T gs = (s & 1) ? g1 : g2;
          if (gs == T(0)) continue;
          C vs = vz<T>();
          if (s == 0 && in_car) {
            // (X_{l+1} c)(j) from the carried neighbours
            fma_rc<T>(vs, wlo * gs, in_lo);
            fma_rc<T>(vs, whi * gs, in_hi);
            if constexpr (SYM) {
              xs_lo[2] = in_lo;
              xs_hi[2] = in_hi;
            }
          } else {
            int2 cr = make_int2(-1, -1);  // cross displacements (r = -1, +1) on suffix axes
            if constexpr (m > NP) {
              constexpr int a = l - NP;
              cr = (s == 0) ? gst2[gst_axis_pair(a + 1, 1) * ng + o] : gst2[gst_cross_pair(D, a, s) * ng + o];
            }
            const bool vs_ok = SYM ? true : val[3 + s];
#pragma unroll
            for (int r = -1; r <= 1; r += 2) {
              uint32_t vid;
              if constexpr (m < NP) {
                const int p = rec_pair(NP, l, s, r);
                vid = (vs_ok && o < rec[p + 1]) ? (uint32_t)(rec[p] + o) : kAbsent;
              } else if constexpr (m == NP) {
                const int32_t oq = r < 0 ? o_lo : o_hi;
                vid = (vs_ok && (uint32_t)oq < (uint32_t)lnw[3 + s]) ? (uint32_t)(stw[3 + s] + oq) : kAbsent;
              } else {
                const int32_t oq = r < 0 ? cr.x : cr.y;
                vid = (vs_ok && (uint32_t)oq < (uint32_t)len) ? base + (uint32_t)oq : kAbsent;
              }
              HS_DCHECK(ix, vid == kAbsent || vid < (uint64_t)ix.size, kDbgNeighbour);
              const C xv = BufLoad<T>::ld(xr, vid);
              if constexpr (SYM) {
                if (r < 0) xs_lo[s + 2] = xv; else xs_hi[s + 2] = xv;
              }
              fma_rc<T>(vs, (r < 0 ? wlo : whi) * gs, xv);
            }
            // the paper's order counts (X_{l+1} c)(j + s e_l) only for j + s e_l in K
            if constexpr (SYM) {
              if (!val[3 + s]) vs = vz<T>();
            }
          }
          if (s & 1) v1[(s + 1) / 2] = vs;
          else {
            h2[(s + 2) / 2].x += vs.x;
            h2[(s + 2) / 2].y += vs.y;
          }
        }
        // reversed order: X_{l+1} applied last, to (X_l^a c) at j -+ e_{l+1}.  The lower
        // intermediate lies in K when j_{l+1} >= 1 (its weight wlo is 0 otherwise), the
        // upper one when prod(1 + j_i) (2 + j_{l+1}) / (1 + j_{l+1}) <= B.  The
        // diagonal of X_l^2 at j' counts j' + e_l only when that lies in K.
        if constexpr (SYM) {
          int jm;
          if constexpr (m < NP) jm = rec[4 + m]; else jm = sc[m - NP];
          const double bm = (double)ix.B * (double)(1 + jm), bl = (double)(1 + jl);
          const bool up_in = pj * (double)(2 + jm) <= bm;
          const T wup = up_in ? whi : T(0);
          C rev = vz<T>();
          if (g2 != T(0)) {
            const bool lo_l = jm >= 1 && pj * (double)jm * (double)(2 + jl) <= bm * bl;
            const bool hi_l = up_in && pj * (double)(2 + jm) * (double)(2 + jl) <= bm * bl;
            const T dm = raw[2] * raw[1], dp = raw[3] * raw[4], d0 = raw[2] * raw[2], d1 = raw[3] * raw[3];
            C rl = vz<T>(), rh = vz<T>();
            fma_rc<T>(rl, dm, xs_lo[0]);
            fma_rc<T>(rl, lo_l ? d0 + d1 : d0, xs_lo[2]);
            fma_rc<T>(rl, dp, xs_lo[4]);
            fma_rc<T>(rh, dm, xs_hi[0]);
            fma_rc<T>(rh, hi_l ? d0 + d1 : d0, xs_hi[2]);
            fma_rc<T>(rh, dp, xs_hi[4]);
            fma_rc<T>(rev, wlo * g2, rl);
            fma_rc<T>(rev, wup * g2, rh);
          }
          if constexpr (X2) {
            if (g1 != T(0)) {
              C rl = vz<T>(), rh = vz<T>();
              fma_rc<T>(rl, raw[2], xs_lo[1]);
              fma_rc<T>(rl, raw[3], xs_lo[3]);
              fma_rc<T>(rh, raw[2], xs_hi[1]);
              fma_rc<T>(rh, raw[3], xs_hi[3]);
              fma_rc<T>(rev, wlo * g1, rl);
              fma_rc<T>(rev, wup * g1, rh);
            }
          }
          acc.x += rev.x;
          acc.y += rev.y;
        }
      }
    }
    // ---- h1 at s = -1, 1 and the group's contribution ----
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int s = 2 * q - 1;
      C h = v1[q];
      fma_rc<T>(h, a1, u[3 + s]);
      fma_rc<T>(h, e[s + 2], h2[q]);
      fma_rc<T>(h, e[s + 3], h2[q + 1]);
      fma_rc<T>(acc, e[2 + q], h);  // e_0 for s = -1, e_1 for s = 1
    }
  });
  acc = scal<T>(oscale, acc);
  if (prev) fma_rc<T>(acc, -pcoef, pv);
  return acc;
}

// The same row stored into y.
template <typename T, int N, int NP, bool X2, bool SYM>
__device__ __forceinline__ void hh_row(const IndexDev &ix, const double *__restrict__ hh,
                                       const typename V2<T>::t *__restrict__ x,
                                       typename V2<T>::t *__restrict__ y,
                                       const int32_t *__restrict__ rec, int32_t o, T oscale,
                                       const typename V2<T>::t *__restrict__ prev, T pcoef) {
  const typename V2<T>::t acc = hh_row_value<T, N, NP, X2, SYM>(ix, hh, x, rec, o, oscale, prev, pcoef);
  const uint32_t self = (uint32_t)rec[0] + (uint32_t)o;
  // the result is streamed to its consumers (inner products, update): non-temporal store
  if constexpr (sizeof(T) == 8) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    v2 t;
    t[0] = acc.x;
    t[1] = acc.y;
    __builtin_nontemporal_store(t, reinterpret_cast<v2 *>(y + self));
  } else {
    typedef float v2 __attribute__((ext_vector_type(2)));
    v2 t;
    t[0] = acc.x;
    t[1] = acc.y;
    __builtin_nontemporal_store(t, reinterpret_cast<v2 *>(y + self));
  }
}

// One launch covers both kinds of work.  The grid is kXcd equal ranges; block b runs on
// XCD b % kXcd and takes position b / kXcd of that XCD's range.  Each range holds a
// contiguous share of the long-tile chunks (tiles and their neighbours then share one
// L2), followed by a contiguous share of the packed short-tile rows, so every XCD gets
// the same mix of the two.
template <typename T, int N, int NP, bool X2, bool SYM = false>
__global__ void __launch_bounds__(256)
k_hh_long(IndexDev ix, const double *__restrict__ hh, const typename V2<T>::t *__restrict__ x,
          typename V2<T>::t *__restrict__ y, const double *__restrict__ out_scale,
          const typename V2<T>::t *__restrict__ prev, const double *__restrict__ prev_coef,
          const double *__restrict__ prev_scale, int32_t long_per_xcd, int32_t small_per_xcd) {
  constexpr int RS = rec_stride(NP);
  const int32_t xcd = blockIdx.x % kXcd, j = blockIdx.x / kXcd;
  const T oscale = out_scale ? (T)*out_scale : T(1);
  const T pcoef = prev ? (T)((*prev_coef) * (prev_scale ? *prev_scale : 1.0)) : T(0);
  if (j < long_per_xcd) {
    const int64_t blk = (int64_t)xcd * long_per_xcd + j;
    const int64_t wave = (blk * blockDim.x + threadIdx.x) >> 6;
    if (wave >= ix.nchunks) return;
    const int32_t ri = __builtin_amdgcn_readfirstlane(ix.chunks[2 * wave]);
    const int32_t o0 = __builtin_amdgcn_readfirstlane(ix.chunks[2 * wave + 1]);
    const int32_t *__restrict__ rec = ix.recs + (int64_t)ri * RS;
    const int32_t o = o0 + (int32_t)(threadIdx.x & 63);
    if (o >= rec[1]) return;
    hh_row<T, N, NP, X2, SYM>(ix, hh, x, y, rec, o, oscale, prev, pcoef);
  } else {
    const int64_t blk = (int64_t)xcd * small_per_xcd + (j - long_per_xcd);
    const int64_t i = blk * blockDim.x + threadIdx.x;
    if (i >= ix.nsmall) return;
    const int32_t r = ix.small_rows[i];
    const int32_t *__restrict__ rec = ix.recs + (int64_t)ix.tile_rec[ix.rowtile[r]] * RS;
    hh_row<T, N, NP, X2, SYM>(ix, hh, x, y, rec, r - rec[0], oscale, prev, pcoef);
  }
}

// grid of the combined launch: kXcd ranges of (long share + short share) blocks
inline void long_grid(const IndexDev &ix, bool with_small, int32_t &long_per, int32_t &small_per,
                      unsigned &blocks) {
  const int64_t lb = ix.nchunks > 0 ? (ix.nchunks * kChunk + 255) / 256 : 0;
  const int64_t sb = (with_small && ix.nsmall > 0) ? (ix.nsmall + 255) / 256 : 0;
  long_per = (int32_t)((lb + kXcd - 1) / kXcd);
  small_per = (int32_t)((sb + kXcd - 1) / kXcd);
  blocks = (unsigned)((int64_t)(long_per + small_per) * kXcd);
}

template <typename T, int N, int NP, bool X2, bool SYM>
static void launch_long_pair(const IndexDev &ix, const double *hh, const void *x, void *y,
                             const double *out_scale, const void *prev, const double *prev_coef,
                             const double *prev_scale, hipStream_t s, bool with_small,
                             bool with_long = true) {
  using C = typename V2<T>::t;
  int32_t lp, sp;
  unsigned blocks;
  IndexDev iv = ix;
  if (!with_long) iv.nchunks = 0;
  long_grid(iv, with_small, lp, sp, blocks);
  if (blocks == 0) return;
  hipLaunchKernelGGL((k_hh_long<T, N, NP, X2, SYM>), dim3(blocks), dim3(256), 0, s, iv, hh, (const C *)x,
                     (C *)y, out_scale, (const C *)prev, prev_coef, prev_scale, lp, sp);
}

// Returns 1 if long and short tiles were both launched, 2 if only the long tiles (the
// caller handles the short ones), 0 if (N, NP) has no specialisation.  With short_only,
// only the short tiles are launched (1), or nothing (0) when they lack records.
template <typename T, bool SYM = false>
int launch_hh_long_impl(const IndexDev &ix, const double *hh, const void *x, void *y,
                        const double *out_scale, const void *prev, const double *prev_coef,
                        const double *prev_scale, hipStream_t s, bool x2, bool short_only = false) {
  if (ix.rstride != rec_stride(ix.np)) return 0;
  // row indices are 32-bit and kAbsent must lie beyond every row
  if (ix.size >= (int64_t)INT32_MAX) return 0;
  if (!struct_loads_reach<T>(ix.size)) return 0;
  const bool small = ix.tile_rec != nullptr;
  if (short_only && !small) return 0;
  const bool lng = !short_only;
#define HS_LONG_CASE(NN, PP)                                                                    \
  case NN * 32 + PP:                                                                            \
    if (x2)                                                                                     \
      launch_long_pair<T, NN, PP, true, SYM>(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, small, lng);  \
    else                                                                                        \
      launch_long_pair<T, NN, PP, false, SYM>(ix, hh, x, y, out_scale, prev, prev_coef, prev_scale, s, small, lng); \
    return small ? 1 : 2;
  switch (ix.N * 32 + ix.np) {
    HS_LONG_CASE(1, 0)
    HS_LONG_CASE(2, 0)
    HS_LONG_CASE(2, 1)
    HS_LONG_CASE(3, 0)
    HS_LONG_CASE(3, 1)
    HS_LONG_CASE(3, 2)
    HS_LONG_CASE(4, 0)
    HS_LONG_CASE(4, 1)
    HS_LONG_CASE(4, 2)
    HS_LONG_CASE(4, 3)
    HS_LONG_CASE(5, 2)
    HS_LONG_CASE(5, 4)
    HS_LONG_CASE(6, 2)
    HS_LONG_CASE(6, 3)
    HS_LONG_CASE(6, 5)
    HS_LONG_CASE(7, 4)
    HS_LONG_CASE(7, 6)
    HS_LONG_CASE(8, 5)
    HS_LONG_CASE(8, 7)
    HS_LONG_CASE(9, 5)
    HS_LONG_CASE(10, 6)
    default:
      return 0;
  }
#undef HS_LONG_CASE
}

}  // namespace hs
