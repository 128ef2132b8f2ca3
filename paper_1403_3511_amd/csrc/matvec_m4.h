// Fused passes of the fourth-order Magnus operator (paper Sec. 2.1, eq. 2stageMagnus)
// for potentials of the class served by the fused H kernel.
//
// With Abar = (A_1 + A_2)/2 and Delta = (A_2 - A_1)/2 (the diagonal D cancels in Delta),
// A_2 A_1 - A_1 A_2 = 2 (Delta Abar - Abar Delta), so with g = sqrt(3) h / 12
//   M v = Abar v - 2 i g (Delta a - Abar d),   a = Abar v,  d = Delta v.
// The fast operator is linear in the term coefficients, so Abar and Delta are the fused
// operator with the coefficient tables (hh_1 + hh_2)/2 and (hh_2 - hh_1)/2.
//   pass 1: one gather of v gives a and d (two coefficient sets on the same loads);
//   pass 2: gathers of d (for Abar) and of a (for Delta; usually only the time-dependent
//           terms, so few of its loads are needed) give
//           w = a - 2 i g (Delta a - Abar d) - pcoef prev in the same launch.
// The row, tile and stencil logic is that of hh_row; operator p = 0 is Abar (with D),
// p = 1 is Delta.  Loads that an operator does not need (all of its coefficients on an
// axis vanish) are skipped by uniform branches.  DL = true is the variant for potentials
// whose time-dependent terms are linear in the coordinates (a laser-type drive): Delta
// then has only x_l^1 and constant coefficients, and its other parts vanish at compile
// time.
#pragma once

#include "matvec_long.h"

namespace hs {

template <typename T, int N, int NP, bool X2, bool DL, int MODE>
__device__ __forceinline__ void m4_row(const IndexDev &ix, const double *__restrict__ hh1,
                                       const double *__restrict__ hh2,
                                       const typename V2<T>::t *__restrict__ x0,
                                       const typename V2<T>::t *__restrict__ x1,
                                       typename V2<T>::t *__restrict__ y0,
                                       typename V2<T>::t *__restrict__ y1,
                                       const int32_t *__restrict__ rec, int32_t o, T oscale, T g2,
                                       const typename V2<T>::t *__restrict__ prev, T pcoef) {
  using C = typename V2<T>::t;
  constexpr int D = N - NP;
  // inputs: pass 1 reads v for both operators; pass 2 reads d for Abar and a for Delta
  constexpr int NI = MODE == 1 ? 1 : 2;
  auto inp = [](int p) { return MODE == 1 ? 0 : p; };
  __amdgpu_buffer_rsrc_t xr[NI];
  xr[0] = vec_rsrc<T>(x0, ix.size);
  if constexpr (NI == 2) xr[NI - 1] = vec_rsrc<T>(x1, ix.size);
  const uint32_t base = (uint32_t)rec[0];
  const int32_t len = rec[1];
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
    const uint64_t pk = ix.gsp[o];
    static_for<0, D>([&](auto A) {
      constexpr int a = decltype(A)::value;
      sc[a] = (int)((pk >> (16 * a)) & 0xFFFFu);
      ssum += sc[a];
    });
  }
  const uint32_t self = base + (uint32_t)o;
  C cs[NI];
  cs[0] = x0[self];
  if constexpr (NI == 2) cs[NI - 1] = x1[self];
  C pv = vz<T>();
  if constexpr (MODE == 2) {
    if (prev) pv = prev[self];
  }
  // diagonal: D + constant term for Abar, constant term only for Delta
  const double k0 = 0.5 * (hh1[5 * N] + hh2[5 * N]), k1 = 0.5 * (hh2[5 * N] - hh1[5 * N]);
  C acc[2];
  acc[0] = scal<T>((T)((double)(rec[2] + ssum) + 0.5 * N + k0), cs[inp(0)]);
  acc[1] = scal<T>((T)k1, cs[inp(1)]);

  C car_lo[NI], car_hi[NI];
  T car_wlo = T(0), car_whi = T(0);
  bool have_car = false;  // uniform: the previous group ran and loaded every input's window
#pragma unroll
  for (int i = 0; i < NI; ++i) car_lo[i] = car_hi[i] = vz<T>();

  static_for<0, N>([&](auto L) {
    constexpr int l = N - 1 - decltype(L)::value;
    constexpr bool inner = (l + 1 < N);
    T a1[2], a2[2], a3[2], g1[2], gq[2];
    bool any2p[2], need3p[2], pres[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      auto cf = [&](int k) {
        if (DL && p == 1 && k != 0) return T(0);
        const double u = hh1[5 * l + k], v = hh2[5 * l + k];
        return (T)(p == 0 ? 0.5 * (u + v) : 0.5 * (v - u));
      };
      a1[p] = cf(0);
      a3[p] = cf(2);
      a2[p] = X2 ? cf(1) : T(0);
      g1[p] = (X2 && inner) ? cf(3) : T(0);
      gq[p] = inner ? cf(4) : T(0);
      any2p[p] = (a3[p] != T(0)) || (a2[p] != T(0)) || (gq[p] != T(0));
      need3p[p] = (a3[p] != T(0));
      pres[p] = any2p[p] || (a1[p] != T(0)) || (g1[p] != T(0));
    }
    // what each input must supply (pass 1: the union of both operators)
    bool ipres[NI], ineed3[NI], ix2[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      ipres[i] = ineed3[i] = ix2[i] = false;
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      ipres[inp(p)] = ipres[inp(p)] || pres[p];
      ineed3[inp(p)] = ineed3[inp(p)] || need3p[p];
      ix2[inp(p)] = ix2[inp(p)] || (a2[p] != T(0));
    }
    const bool any2 = any2p[0] || any2p[1];
    const bool need3 = need3p[0] || need3p[1];
    const bool in_car = have_car;
    C in_lo[NI], in_hi[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      in_lo[i] = car_lo[i];
      in_hi[i] = car_hi[i];
    }
    const T in_wlo = car_wlo, in_whi = car_whi;
    have_car = false;
    if (!pres[0] && !pres[1]) return;  // uniform: group absent for both operators
    // ---- window j + s e_l, s = -3..3 ----
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
        const int2 pr = gst2[gst_axis_pair(a, s) * ng + o];
        const int32_t ou = pr.y, od = pr.x;
        val[3 + s] = (uint32_t)ou < (uint32_t)len;
        val[3 - s] = od >= 0;
        id[3 + s] = val[3 + s] ? base + (uint32_t)ou : kAbsent;
        id[3 - s] = val[3 - s] ? base + (uint32_t)od : kAbsent;
      }
    }
    if (!any2) val[1] = val[5] = false;
    if (!need3) val[0] = val[6] = false;
    T raw[6], e[6];
    if constexpr (l >= NP) WinLoad<T>::ld(wr, jl, raw);
#pragma unroll
    for (int s = -2; s <= 3; ++s) {
      const int k = jl + s;
      if constexpr (l < NP) raw[s + 2] = wt[k > 0 ? k : 0];
      e[s + 2] = (val[3 + s - 1] && val[3 + s]) ? raw[s + 2] : T(0);
    }
    C u[NI][7];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
#pragma unroll
      for (int q = 0; q < 7; ++q) u[i][q] = vz<T>();
      u[i][3] = cs[i];
      if (ipres[i]) {
        u[i][2] = BufLoad<T>::ld(xr[i], id[2]);
        u[i][4] = BufLoad<T>::ld(xr[i], id[4]);
        if (ineed3[i]) {
          u[i][0] = BufLoad<T>::ld(xr[i], id[0]);
          u[i][6] = BufLoad<T>::ld(xr[i], id[6]);
        }
        if constexpr (X2) {
          if (ix2[i]) {
            u[i][1] = BufLoad<T>::ld(xr[i], id[1]);
            u[i][5] = BufLoad<T>::ld(xr[i], id[5]);
          }
        }
      }
    }
    // carry for group l - 1 only when every input loaded its window
    bool all_in = true;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      all_in = all_in && ipres[i];
      car_lo[i] = u[i][2];
      car_hi[i] = u[i][4];
    }
    car_wlo = raw[2];
    car_whi = raw[3];
    have_car = all_in;
    // ---- h2 at s = -2, 0, 2 per operator ----
    C h2[2][3];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int i = inp(p);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int s = 2 * q - 2;
        C h = vz<T>();
        if (any2p[p]) {
          fma_rc<T>(h, e[s + 2] * a3[p], u[i][3 + s - 1]);
          fma_rc<T>(h, e[s + 3] * a3[p], u[i][3 + s + 1]);
          if constexpr (X2) fma_rc<T>(h, a2[p], u[i][3 + s]);
        }
        h2[p][q] = h;
      }
    }
    // inner axis: (X_{l+1} x)(j + s e_l) loaded once per input, weighted per operator
    C v1[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p) v1[p][0] = v1[p][1] = vz<T>();
    if constexpr (inner) {
      const bool anyg = (g1[0] != T(0)) || (gq[0] != T(0)) || (g1[1] != T(0)) || (gq[1] != T(0));
      if (anyg) {
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
        if constexpr (m == NP) {
          const int2 pr = gst2[gst_axis_pair(0, 1) * ng + o];
          o_lo = pr.x;
          o_hi = pr.y;
        }
#pragma unroll
        for (int s = -2; s <= 2; ++s) {
          if (!X2 && (s & 1)) continue;
          bool needp[2];
          bool needi[NI];
#pragma unroll
          for (int i = 0; i < NI; ++i) needi[i] = false;
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            needp[p] = ((s & 1) ? g1[p] : gq[p]) != T(0);
            needi[inp(p)] = needi[inp(p)] || needp[p];
          }
          if (!needp[0] && !needp[1]) continue;
          C xl[NI], xh[NI];
          const bool from_car = (s == 0) && in_car;
          int2 cr = make_int2(-1, -1);
          if constexpr (m > NP) {
            constexpr int a = l - NP;
            if (!from_car)
              cr = (s == 0) ? gst2[gst_axis_pair(a + 1, 1) * ng + o] : gst2[gst_cross_pair(D, a, s) * ng + o];
          }
          uint32_t vid[2];
#pragma unroll
          for (int r = -1; r <= 1; r += 2) {
            uint32_t v;
            if constexpr (m < NP) {
              const int pp = rec_pair(NP, l, s, r);
              v = (val[3 + s] && o < rec[pp + 1]) ? (uint32_t)(rec[pp] + o) : kAbsent;
            } else if constexpr (m == NP) {
              const int32_t oq = r < 0 ? o_lo : o_hi;
              v = (val[3 + s] && (uint32_t)oq < (uint32_t)lnw[3 + s]) ? (uint32_t)(stw[3 + s] + oq) : kAbsent;
            } else {
              const int32_t oq = r < 0 ? cr.x : cr.y;
              v = (val[3 + s] && (uint32_t)oq < (uint32_t)len) ? base + (uint32_t)oq : kAbsent;
            }
            vid[(r + 1) / 2] = v;
          }
#pragma unroll
          for (int i = 0; i < NI; ++i) {
            xl[i] = xh[i] = vz<T>();
            if (!needi[i]) continue;
            if (from_car) {
              xl[i] = in_lo[i];
              xh[i] = in_hi[i];
            } else {
              xl[i] = BufLoad<T>::ld(xr[i], vid[0]);
              xh[i] = BufLoad<T>::ld(xr[i], vid[1]);
            }
          }
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            if (!needp[p]) continue;
            const T gs = (s & 1) ? g1[p] : gq[p];
            C vs = vz<T>();
            fma_rc<T>(vs, wlo * gs, xl[inp(p)]);
            fma_rc<T>(vs, whi * gs, xh[inp(p)]);
            if (s & 1) v1[p][(s + 1) / 2] = vs;
            else {
              h2[p][(s + 2) / 2].x += vs.x;
              h2[p][(s + 2) / 2].y += vs.y;
            }
          }
        }
      }
    }
    // ---- h1 at s = -1, 1 and each operator's contribution ----
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (!pres[p]) continue;
      const int i = inp(p);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int s = 2 * q - 1;
        C h = v1[p][q];
        fma_rc<T>(h, a1[p], u[i][3 + s]);
        fma_rc<T>(h, e[s + 2], h2[p][q]);
        fma_rc<T>(h, e[s + 3], h2[p][q + 1]);
        fma_rc<T>(acc[p], e[2 + q], h);
      }
    }
  });
  if constexpr (MODE == 1) {
    y0[self] = scal<T>(oscale, acc[0]);
    y1[self] = scal<T>(oscale, acc[1]);
  } else {
    // w = a - i g2 (Delta a - Abar d) - pcoef prev; -i g2 (x + i y) = g2 y - i g2 x
    const C a = cs[1];
    const T cre = acc[1].x - acc[0].x, cim = acc[1].y - acc[0].y;
    C w;
    w.x = a.x + g2 * cim;
    w.y = a.y - g2 * cre;
    if (prev) fma_rc<T>(w, -pcoef, pv);
    if constexpr (sizeof(T) == 8) {
      typedef double v2 __attribute__((ext_vector_type(2)));
      v2 t;
      t[0] = w.x;
      t[1] = w.y;
      __builtin_nontemporal_store(t, reinterpret_cast<v2 *>(y0 + self));
    } else {
      typedef float v2 __attribute__((ext_vector_type(2)));
      v2 t;
      t[0] = w.x;
      t[1] = w.y;
      __builtin_nontemporal_store(t, reinterpret_cast<v2 *>(y0 + self));
    }
  }
}

// Same grid as k_hh_long: kXcd ranges, each a share of the long-tile chunks followed by a
// share of the packed short-tile rows.
template <typename T, int N, int NP, bool X2, bool DL, int MODE>
__global__ void __launch_bounds__(256)
k_m4_pass(IndexDev ix, const double *__restrict__ hh1, const double *__restrict__ hh2,
          const typename V2<T>::t *__restrict__ x0, const typename V2<T>::t *__restrict__ x1,
          typename V2<T>::t *__restrict__ y0, typename V2<T>::t *__restrict__ y1,
          const double *__restrict__ in_scale, double g2, const typename V2<T>::t *__restrict__ prev,
          const double *__restrict__ prev_coef, const double *__restrict__ prev_scale,
          int32_t long_per_xcd, int32_t small_per_xcd) {
  constexpr int RS = rec_stride(NP);
  const int32_t xcd = blockIdx.x % kXcd, j = blockIdx.x / kXcd;
  const T oscale = in_scale ? (T)*in_scale : T(1);
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
    m4_row<T, N, NP, X2, DL, MODE>(ix, hh1, hh2, x0, x1, y0, y1, rec, o, oscale, (T)g2, prev, pcoef);
  } else {
    const int64_t blk = (int64_t)xcd * small_per_xcd + (j - long_per_xcd);
    const int64_t i = blk * blockDim.x + threadIdx.x;
    if (i >= ix.nsmall) return;
    const int32_t r = ix.small_rows[i];
    const int32_t *__restrict__ rec = ix.recs + (int64_t)ix.tile_rec[ix.rowtile[r]] * RS;
    m4_row<T, N, NP, X2, DL, MODE>(ix, hh1, hh2, x0, x1, y0, y1, rec, r - rec[0], oscale, (T)g2, prev, pcoef);
  }
}

template <typename T, int N, int NP, bool X2, bool DL>
static void launch_m4_passes(const IndexDev &ix, const double *hh1, const double *hh2, const void *v,
                             void *a, void *d, void *w, const double *in_scale, double g2,
                             const void *prev, const double *prev_coef, const double *prev_scale,
                             hipStream_t s) {
  using C = typename V2<T>::t;
  int32_t lp, sp;
  unsigned blocks;
  long_grid(ix, true, lp, sp, blocks);
  if (blocks == 0) return;
  hipLaunchKernelGGL((k_m4_pass<T, N, NP, X2, DL, 1>), dim3(blocks), dim3(256), 0, s, ix, hh1, hh2, (const C *)v,
                     (const C *)v, (C *)a, (C *)d, in_scale, 0.0, (const C *)nullptr, nullptr, nullptr, lp, sp);
  hipLaunchKernelGGL((k_m4_pass<T, N, NP, X2, DL, 2>), dim3(blocks), dim3(256), 0, s, ix, hh1, hh2, (const C *)d,
                     (const C *)a, (C *)w, (C *)nullptr, nullptr, g2, (const C *)prev, prev_coef, prev_scale,
                     lp, sp);
}

// w = M v through the two fused passes (a, d: scratch vectors of |K| elements).  Returns
// false, launching nothing, when (N, NP) has no specialisation or the set has no
// short-tile row list.
template <typename T>
bool launch_m4_impl(const IndexDev &ix, const double *hh1, const double *hh2, const void *v, void *a,
                    void *d, void *w, const double *in_scale, double g2, const void *prev,
                    const double *prev_coef, const double *prev_scale, hipStream_t s, bool x2,
                    bool dl) {
  if (ix.rstride != rec_stride(ix.np)) return false;
  if (ix.size >= (int64_t)INT32_MAX) return false;
  if (!struct_loads_reach<T>(ix.size)) return false;
  if (ix.tile_rec == nullptr && ix.nsmall > 0) return false;
#define HS_M4_CASE(NN, PP)                                                                            \
  case NN * 32 + PP:                                                                                  \
    if (x2)                                                                                           \
      launch_m4_passes<T, NN, PP, true, false>(ix, hh1, hh2, v, a, d, w, in_scale, g2, prev,           \
                                               prev_coef, prev_scale, s);                             \
    else if (dl)                                                                                      \
      launch_m4_passes<T, NN, PP, false, true>(ix, hh1, hh2, v, a, d, w, in_scale, g2, prev,           \
                                               prev_coef, prev_scale, s);                             \
    else                                                                                              \
      launch_m4_passes<T, NN, PP, false, false>(ix, hh1, hh2, v, a, d, w, in_scale, g2, prev,          \
                                                prev_coef, prev_scale, s);                            \
    return true;
  switch (ix.N * 32 + ix.np) {
    HS_M4_CASE(1, 0)
    HS_M4_CASE(2, 0)
    HS_M4_CASE(2, 1)
    HS_M4_CASE(3, 0)
    HS_M4_CASE(3, 1)
    HS_M4_CASE(3, 2)
    HS_M4_CASE(4, 0)
    HS_M4_CASE(4, 1)
    HS_M4_CASE(4, 2)
    HS_M4_CASE(4, 3)
    HS_M4_CASE(5, 2)
    HS_M4_CASE(6, 2)
    HS_M4_CASE(6, 3)
    HS_M4_CASE(7, 4)
    HS_M4_CASE(8, 5)
    HS_M4_CASE(9, 5)
    HS_M4_CASE(10, 6)
    default:
      return false;
  }
#undef HS_M4_CASE
}

}  // namespace hs
