// Dual numbers for forward-mode derivatives: a value and one directional
// derivative.  Branches and comparisons act on the value, so code run in dual
// arithmetic differentiates the map with every decision held as taken.
#pragma once

#include <hip/hip_runtime.h>

namespace purse {

template <typename T>
struct Dual {
  T v, d;
  __host__ __device__ Dual() : v(0), d(0) {}
  template <typename S>
  __host__ __device__ Dual(S a) : v((T)a), d(0) {}
  __host__ __device__ Dual(T a, T b) : v(a), d(b) {}
};

template <typename T> __device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <typename T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <typename T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <typename T> __device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <typename T> __device__ __forceinline__ Dual<T> operator/(Dual<T> a, Dual<T> b) {
  T q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <typename T> __device__ __forceinline__ Dual<T> &operator+=(Dual<T> &a, Dual<T> b) { a = a + b; return a; }
template <typename T> __device__ __forceinline__ Dual<T> &operator-=(Dual<T> &a, Dual<T> b) { a = a - b; return a; }
template <typename T> __device__ __forceinline__ Dual<T> &operator*=(Dual<T> &a, Dual<T> b) { a = a * b; return a; }
template <typename T> __device__ __forceinline__ bool operator<(Dual<T> a, Dual<T> b) { return a.v < b.v; }
template <typename T> __device__ __forceinline__ bool operator<=(Dual<T> a, Dual<T> b) { return a.v <= b.v; }
template <typename T> __device__ __forceinline__ bool operator>(Dual<T> a, Dual<T> b) { return a.v > b.v; }
template <typename T> __device__ __forceinline__ bool operator>=(Dual<T> a, Dual<T> b) { return a.v >= b.v; }
template <typename T> __device__ __forceinline__ bool operator==(Dual<T> a, Dual<T> b) { return a.v == b.v; }
template <typename T> __device__ __forceinline__ bool operator!=(Dual<T> a, Dual<T> b) { return a.v != b.v; }

// mixed operands (the scalar is a constant)
#define PURSE_DUAL_MIXED(OP)                                                                         \
  template <typename T> __device__ __forceinline__ auto operator OP(Dual<T> a, T b) { return a OP Dual<T>(b); } \
  template <typename T> __device__ __forceinline__ auto operator OP(T a, Dual<T> b) { return Dual<T>(a) OP b; }
PURSE_DUAL_MIXED(+)
PURSE_DUAL_MIXED(-)
PURSE_DUAL_MIXED(*)
PURSE_DUAL_MIXED(/)
PURSE_DUAL_MIXED(<)
PURSE_DUAL_MIXED(<=)
PURSE_DUAL_MIXED(>)
PURSE_DUAL_MIXED(>=)
#undef PURSE_DUAL_MIXED

template <typename T> __host__ __device__ inline T value_of(T x) { return x; }
template <typename T> __device__ __forceinline__ T value_of(Dual<T> x) { return x.v; }

}  // namespace purse
