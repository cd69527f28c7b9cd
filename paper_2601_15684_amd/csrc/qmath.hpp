// Quaternion arithmetic on the device, [w, x, y, z] with the Hamilton
// product of App. A.2.  Products with a pure quaternion [0, v] are written
// out without the zero component (the compiler may not drop x*0 under IEEE
// rules), which is how the sweep forms every per-edge term.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pgo {

template <typename T>
struct alignas(4 * sizeof(T)) Q4 {
  T w, x, y, z;
};

// A 3-vector and a fourth word in one aligned 16/32-byte record: an edge's
// (tau t~, tau), or the information model's (t~, c_e).  State 3-vectors
// (t, s, z) are stored packed as V3.
template <typename T>
struct alignas(4 * sizeof(T)) P4 {
  T x, y, z, u;
};

template <typename T>
struct V3 {
  T x, y, z;
};

// 3x3 matrix as three packed rows, 9 words (row r = (m[r][0], m[r][1],
// m[r][2])): a quarter fewer bytes to move than padded rows.
template <typename T>
struct R3 {
  V3<T> r[3];
};

template <typename T>
__device__ __forceinline__ Q4<T> qmul(const Q4<T>& a, const Q4<T>& b) {
  return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z,
          a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
          a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x,
          a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}

// [0, a] * b
template <typename T>
__device__ __forceinline__ Q4<T> qmul_pv(const V3<T>& a, const Q4<T>& b) {
  return {-a.x * b.x - a.y * b.y - a.z * b.z,
          a.x * b.w + a.y * b.z - a.z * b.y,
          -a.x * b.z + a.y * b.w + a.z * b.x,
          a.x * b.y - a.y * b.x + a.z * b.w};
}

// a * [0, b]
template <typename T>
__device__ __forceinline__ Q4<T> qmul_vp(const Q4<T>& a, const V3<T>& b) {
  return {-a.x * b.x - a.y * b.y - a.z * b.z,
          a.w * b.x + a.y * b.z - a.z * b.y,
          a.w * b.y - a.x * b.z + a.z * b.x,
          a.w * b.z + a.x * b.y - a.y * b.x};
}

// Im(a * conj(b))
template <typename T>
__device__ __forceinline__ V3<T> im_mul_conj(const Q4<T>& a, const Q4<T>& b) {
  // a * [b.w, -b.x, -b.y, -b.z]
  return {-a.w * b.x + a.x * b.w - a.y * b.z + a.z * b.y,
          -a.w * b.y + a.x * b.z + a.y * b.w - a.z * b.x,
          -a.w * b.z - a.x * b.y + a.y * b.x + a.z * b.w};
}

template <typename T>
__device__ __forceinline__ Q4<T> qconj(const Q4<T>& a) {
  return {a.w, -a.x, -a.y, -a.z};
}

template <typename T>
__device__ __forceinline__ V3<T> im(const Q4<T>& a) {
  return {a.x, a.y, a.z};
}

template <typename T>
__device__ __forceinline__ V3<T> v3(const P4<T>& a) {
  return {a.x, a.y, a.z};
}

template <typename T>
__device__ __forceinline__ V3<T> v3(const V3<T>& a) {
  return a;
}

template <typename T>
__device__ __forceinline__ P4<T> pad3(const V3<T>& v, T u = T(0)) {
  return {v.x, v.y, v.z, u};
}

template <typename T, typename U>
__device__ __forceinline__ Q4<T> cvt(const Q4<U>& a) {
  return {T(a.w), T(a.x), T(a.y), T(a.z)};
}

#ifndef PGO_EDGE_UNROLL
#define PGO_EDGE_UNROLL 2
#endif

// Visits the edges [e0, e1) of one vertex in order.  load(e) issues the
// edge's loads (its record and the neighbour gathers it indexes), use(d)
// does its arithmetic.  U edges are loaded before any is used, so U chains
// of index-then-gather are in flight at once per thread; use runs in edge
// order, so every sum is the same as one edge at a time.
template <int U = PGO_EDGE_UNROLL, typename Load, typename Use>
__device__ __forceinline__ void edge_loop(int e0, int e1, Load&& load, Use&& use) {
  int e = e0;
  if (U > 1) {
    for (; e + U <= e1; e += U) {
      decltype(load(e)) d[U];
#pragma unroll
      for (int k = 0; k < U; ++k) d[k] = load(e + k);
#pragma unroll
      for (int k = 0; k < U; ++k) use(d[k]);
    }
  }
  for (; e < e1; ++e) use(load(e));
}

}  // namespace pgo
