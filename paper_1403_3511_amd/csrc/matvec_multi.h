// Fused two-axis H application over work items of several tiles (paper Sec. 3.2, eq.
// Horner; the potential class a1 x_l + a3 x_l^3 + g2 x_l^2 x_{l+1}, axis N applied first).
//
// A work item is a 64-offset range [o0, o0 + 64) and up to kMultiTiles long tiles that all
// reach past o0.  Every lane owns one offset o.  What depends only on o -- the suffix
// coordinates, the suffix stencil offsets and the suffix edge weights -- is loaded once per
// item and kept in registers for all the item's tiles, so per row only the vector itself
// is read.  Each tile (and each neighbour tile along a prefix axis) is addressed through a
// buffer resource of its own: base = its first row, record count = its length.  The
// hardware then returns zero for an offset past the tile's end (an absent neighbour) and
// the element offsets stay small, so the addressing is 64-bit safe at any vector size.
//
// Truncation at the boundary of K: the Horner nesting along an axis walks the window
// j + s e_l, s = -3..3.  An edge between positions s-1 and s carries the weight
// sqrt((j_l + s) / 2); the edge exists only if its upper end lies in K.  Downward this
// holds exactly when the weight is nonzero (j_l + s >= 1), upward it is tested against
// the tile lengths.  With every edge into a missing position zeroed, nothing computed at
// a missing position can reach the result, so no value needs masking.
#pragma once

#include "matvec_long.h"

namespace hs {

// resource over one tile of a complex vector: elements [start, start + len)
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const typename V2<T>::t *x, int32_t start,
                                                            int32_t len) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)(x + (int64_t)start), (short)sizeof(typename V2<T>::t),
                                           len, 0x00020000);
}

// What one lane (suffix offset o) needs for every tile of the item.
template <typename T, int D>
struct SufMeta {
  int32_t ssum;
  uint32_t off[D > 0 ? D : 1][6];  // offset of s + k e_a, k = -3,-2,-1,1,2,3 (0xFFFFFFFF: none)
  uint32_t cr[D > 1 ? D - 1 : 1][4];  // s + k e_a + r e_{a+1}: (k, r) = (-2,-1), (-2,1), (2,-1), (2,1)
  T E[D > 0 ? D : 1][6];           // sqrt((s_a + k) / 2), k = -2..3 (0 below 0)
};
__device__ __forceinline__ int kidx(int k) { return k < 0 ? k + 3 : k + 2; }

template <typename T, int D>
__device__ __forceinline__ void load_suffix_meta(const IndexDev &ix, int32_t o, SufMeta<T, D> &M) {
  const int64_t ng = ix.ng;
  const int2 *__restrict__ gst2 = reinterpret_cast<const int2 *>(ix.gst);
  const __amdgpu_buffer_rsrc_t wr = __builtin_amdgcn_make_buffer_rsrc(
      (void *)(sizeof(T) == 8 ? (const void *)ix.wtp : (const void *)ix.wtpf), (short)0,
      (int)((ix.B + 10) * (int)sizeof(T)), 0x00020000);
  const uint64_t pk = ix.gsp[o];
  M.ssum = 0;
  static_for<0, D>([&](auto A) {
    constexpr int a = decltype(A)::value;
    const int sa = (int)((pk >> (16 * a)) & 0xFFFFu);
    M.ssum += sa;
    WinLoad<T>::ld(wr, sa, M.E[a]);
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
      const int2 pr = gst2[gst_axis_pair(a, k) * ng + o];  // (-k, +k)
      HS_DCHECK(ix, (pr.x == -1 || (pr.x >= 0 && pr.x < ng)) && (pr.y == -1 || (pr.y >= 0 && pr.y < ng)),
                kDbgSuffix);
      M.off[a][kidx(-k)] = (uint32_t)pr.x;
      M.off[a][kidx(k)] = (uint32_t)pr.y;
    }
    if constexpr (a + 1 < D) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = q == 0 ? -2 : 2;
        const int2 pr = gst2[gst_cross_pair(D, a, k) * ng + o];  // (r = -1, r = +1)
        HS_DCHECK(ix, (pr.x == -1 || (pr.x >= 0 && pr.x < ng)) && (pr.y == -1 || (pr.y >= 0 && pr.y < ng)),
                  kDbgSuffix);
        M.cr[a][2 * q] = (uint32_t)pr.x;
        M.cr[a][2 * q + 1] = (uint32_t)pr.y;
      }
    }
  });
}

// One axis group on one row: given the window u (positions -3, -1, 1, 3 and 0 = c0),
// the coupling values vs at s = -2, 0, 2 (already weighted by g2), the edge weights
// E(-2..3) with the upward ones masked, accumulate
//   G = X (X (X (a3 u) + vs) + a1 u)   at position 0.
template <typename T>
__device__ __forceinline__ void group_value(typename V2<T>::t &acc, const typename V2<T>::t (&u)[7],
                                            const typename V2<T>::t (&vs)[3], const T (&E)[6], T a1,
                                            T a3) {
  using C = typename V2<T>::t;
  // h2 at s = -2, 0, 2: a3 (E(s) u(s-1) + E(s+1) u(s+1)) + vs
  C h2[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int s = 2 * q - 2;
    C xu = vz<T>();
    fma_rc<T>(xu, E[s + 2], u[3 + s - 1]);
    if (s + 1 <= 3) fma_rc<T>(xu, E[s + 3], u[3 + s + 1]);
    C h = vs[q];
    fma_rc<T>(h, a3, xu);
    h2[q] = h;
  }
  // h1 at s = -1, 1: E(s) h2(s-1) + E(s+1) h2(s+1) + a1 u(s); G = E(0) h1(-1) + E(1) h1(1)
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int s = 2 * q - 1;
    C h = vz<T>();
    fma_rc<T>(h, a1, u[3 + s]);
    fma_rc<T>(h, E[s + 2], h2[q]);
    fma_rc<T>(h, E[s + 3], h2[q + 1]);
    fma_rc<T>(acc, E[2 + q], h);
  }
}

// One row (offset o) of tile `rec` for the class without x_l^2 and x_l x_{l+1} terms.
template <typename T, int N, int NP>
__device__ __forceinline__ typename V2<T>::t multi_row(const IndexDev &ix, const double *__restrict__ hh,
                                                       const typename V2<T>::t *__restrict__ x,
                                                       const int32_t *__restrict__ rec, int32_t o,
                                                       const SufMeta<T, N - NP> &M) {
  using C = typename V2<T>::t;
  const int32_t start = rec[0], len = rec[1];
  const __amdgpu_buffer_rsrc_t self = tile_rsrc<T>(x, start, len);
  const T *__restrict__ wt;
  if constexpr (sizeof(T) == 8) wt = (const T *)ix.wtab; else wt = (const T *)ix.wtabf;
  const C c0 = x[(int64_t)start + o];
  const double dval = (double)(rec[2] + M.ssum) + 0.5 * N + hh[5 * N];
  C acc = scal<T>((T)dval, c0);
  // carry from group l + 1: c(j -+ e_{l+1}) and the weights sqrt(j/2), sqrt((j+1)/2) there
  C car_lo = vz<T>(), car_hi = vz<T>();
  T car_wlo = T(0), car_whi = T(0);
  static_for<0, N>([&](auto L) {
    constexpr int l = N - 1 - decltype(L)::value;
    constexpr bool inner = (l + 1 < N);
    const T a1 = (T)hh[5 * l + 0], a3 = (T)hh[5 * l + 2];
    const T g2 = inner ? (T)hh[5 * l + 4] : T(0);
    const C in_lo = car_lo, in_hi = car_hi;
    const T in_wlo = car_wlo, in_whi = car_whi;
    C u[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) u[q] = vz<T>();
    u[3] = c0;
    T E[6];
    T e1raw;  // sqrt((j_l + 1) / 2) before masking: the inner weight of group l - 1's coupling
    C vs[3] = {vz<T>(), vz<T>(), vz<T>()};
    if constexpr (l >= NP) {
      // ---- suffix axis a: neighbours inside the tile, by the suffix stencil ----
      constexpr int a = l - NP;
      const bool m1 = M.off[a][kidx(1)] < (uint32_t)len, m2 = M.off[a][kidx(2)] < (uint32_t)len;
#pragma unroll
      for (int k = 0; k < 6; ++k) E[k] = M.E[a][k];
      e1raw = E[3];
      E[3] = m1 ? E[3] : T(0);
      E[4] = m2 ? E[4] : T(0);
      u[2] = BufLoad<T>::ld(self, M.off[a][kidx(-1)]);
      u[4] = BufLoad<T>::ld(self, M.off[a][kidx(1)]);
      u[0] = BufLoad<T>::ld(self, M.off[a][kidx(-3)]);
      u[6] = BufLoad<T>::ld(self, M.off[a][kidx(3)]);
      if constexpr (inner) {
        C lo[2], hi[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          lo[q] = BufLoad<T>::ld(self, M.cr[a][2 * q]);
          hi[q] = BufLoad<T>::ld(self, M.cr[a][2 * q + 1]);
        }
        const T wl = in_wlo * g2, wh = in_whi * g2;
        fma_rc<T>(vs[1], wl, in_lo);
        fma_rc<T>(vs[1], wh, in_hi);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          fma_rc<T>(vs[2 * q], wl, lo[q]);
          fma_rc<T>(vs[2 * q], wh, hi[q]);
        }
      }
    } else {
      // ---- prefix axis l: the same offset in the neighbour tiles ----
      const int jl = rec[4 + l];
#pragma unroll
      for (int k = -2; k <= 3; ++k) E[k + 2] = (jl + k > 0) ? wt[jl + k] : T(0);
      e1raw = E[3];
      int32_t st[7], ln[7];
#pragma unroll
      for (int k = -3; k <= 3; ++k) {
        if (k == 0) continue;
        const int p = rec_axis(NP, l, k);
        st[3 + k] = rec[p];
        ln[3 + k] = rec[p + 1];
        HS_DCHECK(ix, ln[3 + k] == 0 || (st[3 + k] >= 0 && ln[3 + k] > 0 &&
                                         (int64_t)st[3 + k] + ln[3 + k] <= ix.size), kDbgRecord);
      }
      E[3] = o < ln[4] ? E[3] : T(0);
      E[4] = o < ln[5] ? E[4] : T(0);
      u[2] = BufLoad<T>::ld(tile_rsrc<T>(x, st[2], ln[2]), (uint32_t)o);
      u[4] = BufLoad<T>::ld(tile_rsrc<T>(x, st[4], ln[4]), (uint32_t)o);
      u[0] = BufLoad<T>::ld(tile_rsrc<T>(x, st[0], ln[0]), (uint32_t)o);
      u[6] = BufLoad<T>::ld(tile_rsrc<T>(x, st[6], ln[6]), (uint32_t)o);
      if constexpr (inner) {
        C lo[2], hi[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int k = q == 0 ? -2 : 2;
          if constexpr (l + 1 < NP) {
            // p + k e_l -+ e_{l+1}: two prefix moves, the same offset
            const int pl = rec_pair(NP, l, k, -1), ph = rec_pair(NP, l, k, 1);
            HS_DCHECK(ix, (rec[pl + 1] == 0 || (rec[pl] >= 0 && (int64_t)rec[pl] + rec[pl + 1] <= ix.size)) &&
                              (rec[ph + 1] == 0 || (rec[ph] >= 0 && (int64_t)rec[ph] + rec[ph + 1] <= ix.size)),
                      kDbgRecord);
            lo[q] = BufLoad<T>::ld(tile_rsrc<T>(x, rec[pl], rec[pl + 1]), (uint32_t)o);
            hi[q] = BufLoad<T>::ld(tile_rsrc<T>(x, rec[ph], rec[ph + 1]), (uint32_t)o);
          } else {
            // l + 1 is the first suffix axis: the tile p + k e_l at the offsets of s -+ e_0
            const __amdgpu_buffer_rsrc_t tr = tile_rsrc<T>(x, st[3 + k], ln[3 + k]);
            lo[q] = BufLoad<T>::ld(tr, M.off[0][kidx(-1)]);
            hi[q] = BufLoad<T>::ld(tr, M.off[0][kidx(1)]);
          }
        }
        const T wl = in_wlo * g2, wh = in_whi * g2;
        fma_rc<T>(vs[1], wl, in_lo);
        fma_rc<T>(vs[1], wh, in_hi);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          fma_rc<T>(vs[2 * q], wl, lo[q]);
          fma_rc<T>(vs[2 * q], wh, hi[q]);
        }
      }
    }
    car_lo = u[2];
    car_hi = u[4];
    car_wlo = E[2];
    car_whi = e1raw;
    group_value<T>(acc, u, vs, E, a1, a3);
  });
  return acc;
}

// One work item (the wave's lanes are its 64 offsets): y = oscale H x - pcoef prev on the
// rows of the item's tiles.  x, y and prev point at the first element of the set's vectors.
template <typename T, int N, int NP>
__device__ __forceinline__ void multi_item(const IndexDev &ix, const double *__restrict__ hh,
                                           const typename V2<T>::t *__restrict__ x,
                                           typename V2<T>::t *__restrict__ y, const int32_t *__restrict__ it,
                                           T oscale, const typename V2<T>::t *__restrict__ prev, T pcoef) {
  using C = typename V2<T>::t;
  constexpr int RS = rec_stride(NP);
  const int32_t o0 = __builtin_amdgcn_readfirstlane(it[0]);
  const int32_t nr = __builtin_amdgcn_readfirstlane(it[1]);
  const int32_t o = o0 + (int32_t)(threadIdx.x & 63);
  // the first tile is the longest of the item: lanes past its end have no row at all
  const int32_t len0 = ix.recs[(int64_t)__builtin_amdgcn_readfirstlane(it[2]) * RS + 1];
  HS_DCHECK(ix, o0 >= 0 && (o0 % 64) == 0 && nr >= 1 && nr <= kMultiTiles && o0 < len0, kDbgItem);
  if (o >= len0) return;
  HS_DCHECK(ix, (int64_t)o < ix.ng, kDbgItem);
  SufMeta<T, N - NP> M;
  load_suffix_meta<T, N - NP>(ix, o, M);
  for (int32_t r = 0; r < nr; ++r) {
    const int32_t ri = __builtin_amdgcn_readfirstlane(it[2 + r]);
    const int32_t *__restrict__ rec = ix.recs + (int64_t)ri * RS;
    HS_DCHECK(ix, rec[0] >= 0 && rec[1] >= 0 && (int64_t)rec[0] + rec[1] <= ix.size && rec[1] <= len0,
              kDbgRecord);
    if (o >= rec[1]) continue;
    C acc = multi_row<T, N, NP>(ix, hh, x, rec, o, M);
    const int64_t row = (int64_t)rec[0] + o;
    acc = scal<T>(oscale, acc);
    if (prev) fma_rc<T>(acc, -pcoef, prev[row]);
    if constexpr (sizeof(T) == 8) {
      typedef double v2 __attribute__((ext_vector_type(2)));
      v2 t;
      t[0] = acc.x;
      t[1] = acc.y;
      __builtin_nontemporal_store(t, reinterpret_cast<v2 *>(y + row));
    } else {
      typedef float v2 __attribute__((ext_vector_type(2)));
      v2 t;
      t[0] = acc.x;
      t[1] = acc.y;
      __builtin_nontemporal_store(t, reinterpret_cast<v2 *>(y + row));
    }
  }
}

// One launch: kXcd equal ranges, block b on XCD b % kXcd taking position b / kXcd of its
// range.  A range holds a contiguous share of the work items (contiguous in tile order,
// so neighbouring tiles share an L2; one wave per item), followed, when small_per_xcd > 0,
// by a contiguous share of the short-tile rows (one lane per row, the per-lane records
// of the row kernel), so both kinds of work run side by side.
template <typename T, int N, int NP>
__global__ void __launch_bounds__(256)
k_hh_multi(IndexDev ix, const double *__restrict__ hh, const typename V2<T>::t *__restrict__ x,
           typename V2<T>::t *__restrict__ y, const double *__restrict__ out_scale,
           const typename V2<T>::t *__restrict__ prev, const double *__restrict__ prev_coef,
           const double *__restrict__ prev_scale, int32_t items_per_xcd, int32_t small_per_xcd) {
  constexpr int IS = 2 + kMultiTiles;
  constexpr int RS = rec_stride(NP);
  const int32_t xcd = blockIdx.x % kXcd, j = blockIdx.x / kXcd;
  const T oscale = out_scale ? (T)*out_scale : T(1);
  const T pcoef = prev ? (T)((*prev_coef) * (prev_scale ? *prev_scale : 1.0)) : T(0);
  if (j < items_per_xcd) {
    const int64_t blk = (int64_t)xcd * items_per_xcd + j;
    const int64_t item = (blk * blockDim.x + threadIdx.x) >> 6;
    if (item >= ix.nmitems) return;
    multi_item<T, N, NP>(ix, hh, x, y, ix.mitems + item * IS, oscale, prev, pcoef);
  } else {
    const int64_t blk = (int64_t)xcd * small_per_xcd + (j - items_per_xcd);
    const int64_t i = blk * blockDim.x + threadIdx.x;
    if (i >= ix.nsmall) return;
    const int32_t r = ix.small_rows[i];
    const int32_t *__restrict__ rec = ix.recs + (int64_t)ix.tile_rec[ix.rowtile[r]] * RS;
    hh_row<T, N, NP, false, false>(ix, hh, x, y, rec, r - rec[0], oscale, prev, pcoef);
  }
}

// Whether the long tiles of a set take the multi-tile kernel: potentials without the
// x_l^2 and x_l x_{l+1} monomials, sets with prefix axes and work items, and N <= 6 (for
// larger N its register count caps occupancy and the row kernel is faster), or any N when
// the vector is beyond what the row kernel's structured loads address.
template <typename T>
inline bool multi_serves(const IndexDev &ix, bool x2) {
  if (x2 || ix.nmitems == 0 || ix.np < 1 || ix.rstride != rec_stride(ix.np)) return false;
  return ix.N <= 6 || !struct_loads_reach<T>(ix.size);
}

// Launches the multi-tile kernel.  Returns 0 (nothing launched) when multi_serves is
// false, 1 when the launch also covered the short tiles, 2 when it covered the long
// tiles only (the short tiles need the caller: they lack records, or the vector is beyond
// the row kernel's structured loads).
template <typename T>
int launch_hh_multi_impl(const IndexDev &ix, const double *hh, const void *x, void *y,
                         const double *out_scale, const void *prev, const double *prev_coef,
                         const double *prev_scale, hipStream_t s, bool x2) {
  using C = typename V2<T>::t;
  if (!multi_serves<T>(ix, x2)) return 0;
  // The short tiles join the launch in float32 (measured at N = 6, B = 4096: 197 us per
  // application merged against 204 us as two launches).  In float64 they stay a launch
  // of their own, where the row kernel's low register count keeps its occupancy (248 us
  // against 259 us merged, where they would run at the multi-tile kernel's occupancy).
  const bool small = sizeof(T) == 4 && ix.nsmall > 0 && ix.tile_rec != nullptr &&
                     struct_loads_reach<T>(ix.size) && ix.size < (int64_t)INT32_MAX;
  const int64_t lb = (ix.nmitems * 64 + 255) / 256;
  const int64_t sb = small ? (ix.nsmall + 255) / 256 : 0;
  const int32_t lp = (int32_t)((lb + kXcd - 1) / kXcd), sp = (int32_t)((sb + kXcd - 1) / kXcd);
  const unsigned grid = (unsigned)((int64_t)(lp + sp) * kXcd);
#define HS_MULTI_CASE(NN, PP)                                                                          \
  case NN * 32 + PP:                                                                                   \
    hipLaunchKernelGGL((k_hh_multi<T, NN, PP>), dim3(grid), dim3(256), 0, s, ix, hh, (const C *)x, (C *)y, \
                       out_scale, (const C *)prev, prev_coef, prev_scale, lp, sp);                     \
    return (small || ix.nsmall == 0) ? 1 : 2;
  switch (ix.N * 32 + ix.np) {
    HS_MULTI_CASE(3, 1)
    HS_MULTI_CASE(3, 2)
    HS_MULTI_CASE(4, 1)
    HS_MULTI_CASE(4, 2)
    HS_MULTI_CASE(4, 3)
    HS_MULTI_CASE(5, 2)
    HS_MULTI_CASE(6, 2)
    HS_MULTI_CASE(6, 3)
    HS_MULTI_CASE(7, 4)
    HS_MULTI_CASE(8, 5)
    HS_MULTI_CASE(9, 5)
    HS_MULTI_CASE(10, 6)
    default:
      return 0;
  }
#undef HS_MULTI_CASE
}

}  // namespace hs
