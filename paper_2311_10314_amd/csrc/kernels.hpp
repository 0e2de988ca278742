// Device buffers of one context and the launch entry points of the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "coef.hpp"

namespace ddcc {

// MODE_STREAM is MODE_STEP with nontemporal stores of everything the step
// writes; the host picks it for grids whose step does not fit the 256 MB
// memory-side cache (there it is 3-6 % faster; on cache-resident grids
// plain stores are, by up to 19 %).
enum { MODE_STEP = 0, MODE_INIT = 1, MODE_MOMENTS = 2, MODE_STREAM = 3 };

// Pointers handed to the step/init/moments kernels (by value).
//   fA/gA/TA: current level (read), fB/gB/TB: next level (written);
//   in MODE_INIT the kernels write fB/gB/TB and read inC/inU/inP;
//   in MODE_MOMENTS they write outC/outU/outP and nothing else.
// Pop is the storage type of the moving populations (f^i_p, p >= 1, and
// g_p); S that of the history, T and geometry fields.
template <class Pop, class S>
struct Bufs {
  const Pop* fA;   // moving phase populations [N][Q-1][n] (phase_plane)
  Pop* fB;
  const double* f0A;  // rest populations of the phase sets [N][n], float64
  double* f0B;
  const Pop* gA;
  Pop* gB;
  S* hist;
  const S* TA;
  S* TB;
  const S* psi;
  // wetting weights E_i = sum_k cos theta^k_iN |grad psi_k| over the walls,
  // [N-1][n] (eqs. 2.9, 2.14; Section 4.5)
  const S* wet;
  const double* inC;
  const double* inU;
  const double* inP;
  double* outC;
  double* outU;
  double* outP;
  double* fC;      // 3D work fields: C_i [N][n] and mu_i [N][n], float64
  double* fmu;
  // device copies of the context's coefficients, Coef<double> and Coef<S>
  // (read by scalar loads instead of kernel arguments: the single-context
  // 2D kernel, and the 3D step kernel for some storage types)
  const void* coef_d;
  const void* coef_r;
};

// A population value v written in a narrower storage type: returns the
// stored value and adds the rounding v - stored to comp, so that the float64
// rest population can take it back and the phase mass stays exact.
template <class Pop, class R>
__device__ inline Pop narrow(R v, double& comp) {
  const Pop s = Pop(v);
  if constexpr (sizeof(Pop) < sizeof(R)) comp += double(v) - double(R(s));
  return s;
}

// kd: the float64 constants (fields C, mu, psi, rest populations);
// k: the same constants in the collision arithmetic type R.
template <class Pop, class S, class R>
hipError_t launch_2d(int nphase, int mode, const Coef<double>& kd,
                     const Coef<R>& k, const Bufs<Pop, S>& b, int ty,
                     hipStream_t st);

// lattice_f: the phase-set lattice id (D3Q15 or D3Q7 of lattice.hpp).
template <class Pop, class S, class R>
hipError_t launch_3d(int nphase, int lattice_f, int mode,
                     const Coef<double>& kd, const Coef<R>& k,
                     const Bufs<Pop, S>& b, int tx, int ty, hipStream_t st);

// Batches of independent 2D boxes: one work-queue entry per tile, and the
// size and node offset of every instance. Each plane of each buffer holds
// every instance, instance i at nodes [off_i, off_i + n_i); the plane stride
// is the total node count (the n of the Coef handed to the batch kernel).
struct BatchTile {
  int inst, x0, y0, pad;
};
struct BatchInst {
  int nx, ny;
  long long n, off;
};

// One step (or initialisation, or moment read-out) of the instances whose
// tiles are listed: a persistent launch of nblocks workgroups that drain the
// tile queue; *counter must be zero at launch. kd, k: device tables of the
// coefficients of every instance.
template <class Pop, class S, class R>
hipError_t launch_2d_batch(int nphase, int mode, const Coef<double>* kd,
                           const Coef<R>* k,
                           const Bufs<Pop, S>& b, const BatchTile* tiles,
                           const BatchInst* insts, unsigned ntiles,
                           unsigned* counter, int nblocks, int ty,
                           hipStream_t st);

// Resident workgroups per compute unit of the batch kernel (0 on error).
template <class Pop, class S, class R>
int batch_blocks_per_cu(int nphase, int ty);

// Geometry from K walls: psi = prod_k psi_k and the wetting weights
// E_i = sum_k cos theta^k_iN |grad psi_k| (i < N-1), the gradient by the
// fixed isotropic stencil (D2Q9 at nz = 1, else D3Q19) on the periodic
// nx x ny x nz box. Inputs float64 on the device: psik [K][n], ctk
// [K][N-1][n] (NULL: 90 degrees). Outputs in S at node off + x of planes of
// plane_stride nodes.
template <class S>
hipError_t launch_wet_field(const double* psik, const double* ctk, int K,
                            int nm1, int nx, int ny, int nz, S* psi_out,
                            S* wet_out, long long plane_stride, long long off,
                            hipStream_t st);

// dst[i] = v for i < count (a kernel, so that it can sit in a captured graph).
hipError_t launch_fill_u32(unsigned* dst, unsigned v, long long count,
                           hipStream_t st);

// Per-phase sums of all populations (rest plane f0 [N][stride_n] plus
// the moving planes of f [N][Q-1][stride_n], nodes [0, n) of each plane) into
// partial[block * N + i], plus a non-finite flag per block in bad[block].
template <class Pop>
hipError_t launch_mass(const double* f0, const Pop* f, int nphase, int Q,
                       long long n, long long stride_n, double* partial,
                       int* bad, int nblocks, hipStream_t st);

// Blocks of the mass kernel whose partials fit the static workspace of the
// allocation-free mass check (the library never launches more).
constexpr int kScratchBlocks = 1024;

// Device address and size of that workspace on `device` (looked up once per
// device, with the device made current for the lookup).
hipError_t scratch_address(int device, void** ptr, size_t* bytes);

// out[i] = sum over blocks b in order of partial[b * N + i] (i < N, float64,
// as ddcc_mass sums them on the host); *nonfinite = OR of bad[0 .. nb) when
// nonfinite is not NULL. One wave.
hipError_t launch_mass_finish(const double* partial, const int* bad, int nb,
                              int N, double* out, int* nonfinite,
                              hipStream_t st);

// *first = t if any of bad[0 .. nb) is set and *first < 0 (one wave).
hipError_t launch_sticky(const int* bad, int nb, long long* first,
                         long long t, hipStream_t st);

// dst[i] = S(src[i]) for i < count.
template <class S>
hipError_t launch_convert(const double* src, S* dst, long long count,
                          hipStream_t st);

}  // namespace ddcc
