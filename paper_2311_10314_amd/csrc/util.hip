// Reductions and conversions used by the host API.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace ddcc {

namespace {

constexpr int kMassThreads = 256;
constexpr int kWaves = kMassThreads / 64;

// Per-phase population sums in float64: every thread accumulates a strided
// slice, wavefronts reduce with cross-lane shuffles, the four waves of the
// block through LDS; one partial per block and phase (summed on the host in
// block order, so the result is deterministic).
template <class S>
__global__ __launch_bounds__(kMassThreads) void k_mass(const double* f0,
                                                       const S* f, int N, int Q,
                                                       long long n,
                                                       long long stride_n,
                                                       double* partial,
                                                       int* bad) {
  double acc[kMaxN] = {0.0, 0.0, 0.0, 0.0};
  int nonfinite = 0;
  const long long stride = (long long)gridDim.x * kMassThreads;
  for (long long x = (long long)blockIdx.x * kMassThreads + threadIdx.x; x < n;
       x += stride) {
    for (int i = 0; i < N; ++i) {
      const S* fi = f + (long long)i * Q * stride_n + x;
      double s = f0[(long long)i * stride_n + x];
      for (int p = 1; p < Q; ++p) {
        const double v = double(fi[(long long)p * stride_n]);
        s += v;
      }
      if (!isfinite(s)) nonfinite = 1;
      acc[i] += s;
    }
  }
  for (int i = 0; i < kMaxN; ++i)
    for (int off = 32; off > 0; off >>= 1) acc[i] += __shfl_xor(acc[i], off);
  for (int off = 32; off > 0; off >>= 1) nonfinite |= __shfl_xor(nonfinite, off);
  __shared__ double red[kWaves][kMaxN];
  __shared__ int redbad[kWaves];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    for (int i = 0; i < kMaxN; ++i) red[wave][i] = acc[i];
    redbad[wave] = nonfinite;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int b = 0;
    for (int w = 0; w < kWaves; ++w) b |= redbad[w];
    for (int i = 0; i < N; ++i) {
      double s = 0.0;
      for (int w = 0; w < kWaves; ++w) s += red[w][i];
      partial[(long long)blockIdx.x * N + i] = s;
    }
    bad[blockIdx.x] = b;
  }
}

template <class S>
__global__ void k_convert(const double* src, S* dst, long long count) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
       i < count; i += stride)
    dst[i] = S(src[i]);
}

__global__ void k_fill_u32(unsigned* dst, unsigned v, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = v;
}

}  // namespace

hipError_t launch_fill_u32(unsigned* dst, unsigned v, long long count,
                           hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((count + 255) / 256)),
                     dim3(256), 0, st, dst, v, count);
  return hipGetLastError();
}

template <class S>
hipError_t launch_mass(const double* f0, const S* f, int nphase, int Q,
                       long long n, long long stride_n, double* partial,
                       int* bad, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL((k_mass<S>), dim3(nblocks), dim3(kMassThreads), 0, st, f0,
                     f, nphase, Q, n, stride_n, partial, bad);
  return hipGetLastError();
}

template <class S>
hipError_t launch_convert(const double* src, S* dst, long long count,
                          hipStream_t st) {
  if (count <= 0) return hipSuccess;
  long long blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL((k_convert<S>), dim3((unsigned)blocks), dim3(256), 0, st,
                     src, dst, count);
  return hipGetLastError();
}

template hipError_t launch_mass<double>(const double*, const double*, int, int,
                                         long long, long long, double*,
                                         int*, int, hipStream_t);
template hipError_t launch_mass<float>(const double*, const float*, int, int,
                                         long long, long long, double*,
                                         int*, int, hipStream_t);
template hipError_t launch_mass<_Float16>(const double*, const _Float16*, int, int,
                                         long long, long long, double*,
                                         int*, int, hipStream_t);
template hipError_t launch_mass<__bf16>(const double*, const __bf16*, int, int,
                                         long long, long long, double*,
                                         int*, int, hipStream_t);
template hipError_t launch_convert<double>(const double*, double*, long long,
                                           hipStream_t);
template hipError_t launch_convert<float>(const double*, float*, long long,
                                          hipStream_t);

}  // namespace ddcc
