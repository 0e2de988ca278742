// Small device helpers shared by the 2D and 3D step kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace ddcc {

// g(C) = C^2 (C - 1)^2  =>  g'(C) = 2 C (C - 1)(2 C - 1)   (Section 2.1)
template <class R>
__device__ inline R gprime(R C) {
  return R(2) * C * (C - R(1)) * (R(2) * C - R(1));
}

// Periodic wrap of an index into [0, n). Halo indices lie within one period
// of the grid unless the grid is narrower than a tile; those take the
// (slow) integer remainder.
__device__ inline int wrap(int v, int n) {
  if (v >= -n && v < 2 * n) return v < 0 ? v + n : (v >= n ? v - n : v);
  const int m = v % n;
  return m < 0 ? m + n : m;
}

// Element i of a plane: the byte offset is formed in 32 bits, so that the
// plane pointer stays in scalar registers and each access is one global
// load/store with a 32-bit vector offset (planes are at most 4 GiB; the
// library limits grids to 2^29 nodes).
template <class T>
__device__ inline T ldp(const T* plane, unsigned i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(plane) +
                                     i * unsigned(sizeof(T)));
}

// Load of a value that only this node reads in the step (its own history
// and rest populations; in 3D also a pulled population whose row is not
// shifted in x, so that no neighbouring tile touches its cache lines): with
// NT a nontemporal load, which leaves the caches to the rows that
// neighbouring nodes share (in streaming steps: 256^3 3D 1-2 %, 2048^2 2D
// 1-2 % faster). Nontemporal loads of the shared rows too cost 15-35 %.
template <bool NT, class T>
__device__ inline T ldo(const T* plane, unsigned i) {
  if constexpr (NT && sizeof(T) == 2) {
    const unsigned short u = __builtin_nontemporal_load(
        reinterpret_cast<const unsigned short*>(
            reinterpret_cast<const char*>(plane) + i * 2u));
    T v;
    __builtin_memcpy(&v, &u, 2);
    return v;
  } else if constexpr (NT) {
    return __builtin_nontemporal_load(reinterpret_cast<const T*>(
        reinterpret_cast<const char*>(plane) + i * unsigned(sizeof(T))));
  } else {
    return ldp(plane, i);
  }
}

// Plane of the moving population p >= 1 of phase set i: the phase sets keep
// only their Q - 1 moving planes, [N][Q-1][n]; their rest populations live
// in the float64 plane f0.
template <class T>
__host__ __device__ inline T* phase_plane(T* f, int i, int p, int Q,
                                          long long n) {
  return f + ((long long)i * (Q - 1) + (p - 1)) * n;
}

// Store of element i of a plane. NT: a nontemporal (streaming) store, for
// the outputs of a step whose working set is larger than the memory-side
// cache; they are read again only by the next step, after the whole grid
// has gone through the caches.
template <bool NT = false, class T>
__device__ inline void stp(T* plane, unsigned i, T v) {
  T* q = reinterpret_cast<T*>(reinterpret_cast<char*>(plane) +
                              i * unsigned(sizeof(T)));
  if constexpr (NT && sizeof(T) == 2) {
    unsigned short u;
    __builtin_memcpy(&u, &v, 2);
    __builtin_nontemporal_store(u, reinterpret_cast<unsigned short*>(q));
  } else if constexpr (NT) {
    __builtin_nontemporal_store(v, q);
  } else {
    *q = v;
  }
}

}  // namespace ddcc
