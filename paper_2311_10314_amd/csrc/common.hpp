// Small device helpers shared by the 2D and 3D step kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace ddcc {

// g(C) = C^2 (C - 1)^2  =>  g'(C) = 2 C (C - 1)(2 C - 1)   (Section 2.1)
template <class R>
__device__ inline R gprime(R C) {
  return R(2) * C * (C - R(1)) * (R(2) * C - R(1));
}

// Periodic wrap of an index that may lie several periods outside [0, n).
__device__ inline int wrap(int v, int n) {
  int m = v % n;
  return m < 0 ? m + n : m;
}

template <class S, class R>
__device__ inline R ld(const S* p) {
  return static_cast<R>(*p);
}

}  // namespace ddcc
