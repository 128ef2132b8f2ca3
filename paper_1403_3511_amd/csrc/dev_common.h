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
