// Reductions and conversions used by the host API.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace ddcc {

// Workspace of the mass check that allocates nothing (ddcc_mass_noalloc):
// the per-block partial sums [kScratchBlocks][kMaxN] float64, then the
// per-block non-finite flags [kScratchBlocks] int. One copy per GPU, held
// until the process ends; every call on a GPU shares it (calls that overlap
// on one GPU race). Host code never passes this name to a kernel: it takes
// the device address from scratch_address().
static __device__ __align__(256) unsigned char
    scratch[kScratchBlocks * kMaxN * sizeof(double) +
            kScratchBlocks * sizeof(int)];

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
      double s = f0[(long long)i * stride_n + x];
      for (int p = 1; p < Q; ++p) {
        const double v = double(phase_plane(f, i, p, Q, stride_n)[x]);
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

// One wave: if any of the nb block flags is set and *first is still
// negative, *first = t (the time level of the first check that saw a
// non-finite population).
__global__ __launch_bounds__(64) void k_sticky(const int* bad, int nb,
                                               long long* first, long long t) {
  int b = 0;
  for (int i = threadIdx.x; i < nb; i += 64) b |= bad[i];
  for (int off = 32; off > 0; off >>= 1) b |= __shfl_xor(b, off);
  if (threadIdx.x == 0 && b && *first < 0) *first = t;
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

// Wetting weights of K walls (see launch_wet_field). One node per thread.
template <class S>
__global__ void k_wet_field(const double* psik, const double* ctk, int K,
                            int nm1, int nx, int ny, int nz, S* psi_out,
                            S* wet_out, long long stride, long long off) {
  const long long n = (long long)nx * ny * nz;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int x = int(idx % nx);
  const int y = int((idx / nx) % ny);
  const int z = int(idx / ((long long)nx * ny));
  double ps = 1.0;
  double E[kMaxN - 1] = {0.0, 0.0, 0.0};
  for (int kk = 0; kk < K; ++kk) {
    const double* p = psik + kk * n;
    ps *= p[idx];
    double g[3] = {0.0, 0.0, 0.0};
    // isotropic stencil: D2Q9 (1/3 axes, 1/12 diagonals) or D3Q19 (1/6
    // faces, 1/12 edges) weights at d0 = 1/3 over c_s^2 = 1/3
    for (int dz = (nz > 1 ? -1 : 0); dz <= (nz > 1 ? 1 : 0); ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int m = dx * dx + dy * dy + dz * dz;
          if (m == 0 || (nz > 1 && m == 3)) continue;
          const double w = nz > 1 ? (m == 1 ? 1.0 / 6.0 : 1.0 / 12.0)
                                  : (m == 1 ? 1.0 / 3.0 : 1.0 / 12.0);
          const int xs = (x + dx + nx) % nx, ys = (y + dy + ny) % ny;
          const int zs = nz > 1 ? (z + dz + nz) % nz : 0;
          const double v = p[((long long)zs * ny + ys) * nx + xs];
          g[0] += w * dx * v;
          g[1] += w * dy * v;
          g[2] += w * dz * v;
        }
    const double ag = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    for (int i = 0; i < nm1; ++i) {
      const double c = ctk ? ctk[((long long)kk * nm1 + i) * n + idx] : 0.0;
      E[i] += c * ag;
    }
  }
  psi_out[off + idx] = S(ps);
  for (int i = 0; i < nm1; ++i) wet_out[i * stride + off + idx] = S(E[i]);
}

// Per-phase totals from the per-block partials, summed in block order by
// one lane per phase (the order and arithmetic of ddcc_mass's host sum, so
// the two agree bit for bit), and the OR of the block flags.
__global__ __launch_bounds__(64) void k_mass_finish(const double* partial,
                                                    const int* bad, int nb,
                                                    int N, double* out,
                                                    int* nonfinite) {
  const int i = int(threadIdx.x);
  if (i < N) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[(long long)b * N + i];
    out[i] = s;
  }
  if (nonfinite) {
    int f = 0;
    for (int b = i; b < nb; b += 64) f |= bad[b];
    for (int off = 32; off > 0; off >>= 1) f |= __shfl_xor(f, off);
    if (i == 0) *nonfinite = f;
  }
}

}  // namespace

hipError_t scratch_address(int device, void** ptr, size_t* bytes) {
  // Device addresses of `scratch`, looked up once per device with that
  // device current (each GPU holds its own copy at its own address).
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  *ptr = nullptr;
  *bytes = sizeof(scratch);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) {
      const hipError_t e2 = hipSetDevice(prev);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

hipError_t launch_mass_finish(const double* partial, const int* bad, int nb,
                              int N, double* out, int* nonfinite,
                              hipStream_t st) {
  if (nb < 1 || N < 1 || N > kMaxN || !out) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mass_finish, dim3(1), dim3(64), 0, st, partial, bad,
                     nb, N, out, nonfinite);
  return hipGetLastError();
}

template <class S>
hipError_t launch_wet_field(const double* psik, const double* ctk, int K,
                            int nm1, int nx, int ny, int nz, S* psi_out,
                            S* wet_out, long long plane_stride, long long off,
                            hipStream_t st) {
  const long long n = (long long)nx * ny * nz;
  if (n <= 0 || K < 1 || nm1 < 0 || nm1 > kMaxN - 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_wet_field<S>), dim3((unsigned)((n + 255) / 256)),
                     dim3(256), 0, st, psik, ctk, K, nm1, nx, ny, nz, psi_out,
                     wet_out, plane_stride, off);
  return hipGetLastError();
}

template hipError_t launch_wet_field<double>(const double*, const double*, int,
                                             int, int, int, int, double*,
                                             double*, long long, long long,
                                             hipStream_t);
template hipError_t launch_wet_field<float>(const double*, const double*, int,
                                            int, int, int, int, float*, float*,
                                            long long, long long, hipStream_t);

hipError_t launch_sticky(const int* bad, int nb, long long* first,
                         long long t, hipStream_t st) {
  hipLaunchKernelGGL(k_sticky, dim3(1), dim3(64), 0, st, bad, nb, first, t);
  return hipGetLastError();
}

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
