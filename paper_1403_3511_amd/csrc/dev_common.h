// Device helpers shared by the matvec translation units.
#pragma once

#include "hs_internal.h"

namespace hs {

template <typename T> struct V2;
template <> struct V2<double> { using t = double2; };
template <> struct V2<float> { using t = float2; };

template <typename T>
__device__ __forceinline__ typename V2<T>::t vz() {
  typename V2<T>::t r;
  r.x = T(0);
  r.y = T(0);
  return r;
}
template <typename T, typename U>
__device__ __forceinline__ void fma_rc(typename V2<T>::t &acc, U w, const typename V2<T>::t &x) {
  acc.x = fma((T)w, x.x, acc.x);
  acc.y = fma((T)w, x.y, acc.y);
}
template <typename T>
__device__ __forceinline__ typename V2<T>::t scal(T w, const typename V2<T>::t &x) {
  typename V2<T>::t r;
  r.x = w * x.x;
  r.y = w * x.y;
  return r;
}

// Neighbour-index checks of the debug build (HS_DEBUG_BOUNDS): a failed check counts in
// the index's debug words (ix.dbg[0]: number of failed checks, ix.dbg[1]: the first
// check's code), which hs_index_debug_read returns.  The kernels go on as in the release
// build (every load they check is bounded by its buffer resource or its own test), so a
// failed check never faults.  In the release build the checks compile to nothing.
enum DebugCode : uint32_t {
  kDbgRecord = 1,      // a tile record (first row, length) outside the vector
  kDbgItem = 2,        // a work item's offset or tile count out of range
  kDbgSuffix = 3,      // a suffix stencil offset neither absent nor inside the suffix list
  kDbgNeighbour = 4,   // a neighbour element index neither absent nor inside the vector
  kDbgPosition = 5,    // a (tile, offset) position outside its tile
  kDbgRow = 6,         // a row written outside the vector
};
#ifdef HS_DEBUG_BOUNDS
__device__ __forceinline__ void debug_flag(uint32_t *dbg, uint32_t code) {
  if (!dbg) return;
  atomicAdd(dbg, 1u);
  atomicCAS(dbg + 1, 0u, code);
}
#define HS_DCHECK(ix, cond, code)                                 \
  do {                                                            \
    if (!(cond)) ::hs::debug_flag((ix).dbg, (uint32_t)(code));    \
  } while (0)
#else
#define HS_DCHECK(ix, cond, code) \
  do {                            \
  } while (0)
#endif

// MI355X has 8 XCDs with private L2 caches; workgroups are dispatched round-robin
constexpr int kXcd = 8;
// grid size rounded up to a multiple of kXcd (kernels map blocks XCD-contiguously)
inline unsigned xcd_grid(int64_t blocks) { return (unsigned)((blocks + kXcd - 1) / kXcd * kXcd); }

// compile-time loop: f(std::integral_constant<int, I>) for I = B..E-1
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

}  // namespace hs
