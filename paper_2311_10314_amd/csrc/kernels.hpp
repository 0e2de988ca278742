// Device buffers of one context and the launch entry points of the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "coef.hpp"

namespace ddcc {

enum { MODE_STEP = 0, MODE_INIT = 1, MODE_MOMENTS = 2 };

// Pointers handed to the step/init/moments kernels (by value).
//   fA/gA/TA: current level (read), fB/gB/TB: next level (written);
//   in MODE_INIT the kernels write fB/gB/TB and read inC/inU/inP;
//   in MODE_MOMENTS they write outC/outU/outP and nothing else.
template <class S>
struct Bufs {
  const S* fA;     // phase populations [N][Q][n]; plane p = 0 unused
  S* fB;
  const double* f0A;  // rest populations of the phase sets [N][n], float64
  double* f0B;
  const S* gA;
  S* gB;
  S* hist;
  const S* TA;
  S* TB;
  const S* psi;
  const S* ct;
  const double* inC;
  const double* inU;
  const double* inP;
  double* outC;
  double* outU;
  double* outP;
};

// kd: the float64 constants (fields C, mu, psi, rest populations);
// k: the same constants in the collision arithmetic type R.
template <class S, class R>
hipError_t launch_2d(int nphase, int mode, const Coef<double>& kd,
                     const Coef<R>& k, const Bufs<S>& b, int ty,
                     hipStream_t st);

template <class S, class R>
hipError_t launch_3d(int nphase, int mode, const Coef<double>& kd,
                     const Coef<R>& k, const Bufs<S>& b, int tx, int ty,
                     hipStream_t st);

// Per-phase sums of all populations (rest plane f0 [N][n] plus planes
// p >= 1 of f [N][Q][n]) into partial[block * N + i], plus a non-finite flag
// per block in bad[block].
template <class S>
hipError_t launch_mass(const double* f0, const S* f, int nphase, int Q,
                       long long n, double* partial, int* bad, int nblocks,
                       hipStream_t st);

// dst[i] = S(src[i]) for i < count.
template <class S>
hipError_t launch_convert(const double* src, S* dst, long long count,
                          hipStream_t st);

}  // namespace ddcc
