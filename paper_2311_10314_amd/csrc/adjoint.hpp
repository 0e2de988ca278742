// Buffers and launch entry points of the adjoint (reverse-time) 2D step.
#pragma once

#include <hip/hip_runtime.h>

#include "coef.hpp"

namespace ddcc {

// Stored forward state of one time level (read only in the reverse sweep),
// laid out as the step's buffers: f [N][8][n] (moving planes), f0 [N][n],
// g [9][n], history [2N + 4][n] (phi C_i u, Y, P), T [n].
template <class S>
struct AdjFwd {
  const S* f;
  const double* f0;
  const S* g;
  const S* hist;
  const S* T;
};

// float64 fields of the level being transposed, recomputed from AdjFwd.
struct AdjWork {
  double* psiC;   // [N][n] phi C_i
  double* tot;    // [n] sum_i phi C_i
  double* C;      // [N][n]
  double* prho;   // [n] phi rho
  double* psimu;  // [N][n] phi mu_i
  double* mu;     // [N][n] mu_i = phi mu_i / psi_hat
};

// Per-node adjoint intermediates: plane offsets in AdjBufs::a (N phases).
template <int N> __host__ __device__ constexpr int adj_gC() { return 0; }
template <int N> __host__ __device__ constexpr int adj_gmu() { return 2 * N; }
template <int N> __host__ __device__ constexpr int adj_gprho() { return 4 * N; }
template <int N> __host__ __device__ constexpr int adj_T() { return 4 * N + 2; }
template <int N> __host__ __device__ constexpr int adj_C() { return 4 * N + 4; }
template <int N> __host__ __device__ constexpr int adj_psimu() { return 5 * N + 4; }
template <int N> __host__ __device__ constexpr int adj_psiC() { return 6 * N + 4; }
template <int N> __host__ __device__ constexpr int adj_psirho() { return 7 * N + 4; }
template <int N> __host__ __device__ constexpr int adj_L() { return 7 * N + 5; }
__host__ __device__ constexpr int adj_planes(int N) { return 8 * N + 5; }

// Adjoint state (float64, R) and the accumulated gradients.
//   lfB/lgB/lTB: adjoint of level n + 1 (read); lfA/lgA/lTA: of level n
//   (written); lf planes [N][9][n] with plane 0 the rest population;
//   lh [2N + 4][n] the history adjoint, updated in place;
//   a [adj_planes(N)][n] intermediates of one reverse step;
//   gE [N-1][n], gpsi [n], ggpsi [2][n]: dJ/dE_i, the pointwise part of
//   dJ/dpsi and the adjoint of grad psi, summed over the steps (float64).
template <class R>
struct AdjBufs {
  const R* lfB;
  R* lfA;
  const R* lgB;
  R* lgA;
  R* lh;
  const R* lTB;
  R* lTA;
  R* a;
  double* gE;
  double* gpsi;
  double* ggpsi;
};

// One reverse step: from the stored state of level n and the adjoint of
// level n + 1, the adjoint of level n, and the gradient sums updated.
template <class S>
hipError_t launch_adj_step(int nphase, const Coef<double>& kd,
                           const AdjFwd<S>& fw, const S* psi, const S* wet,
                           const AdjWork& w, const AdjBufs<double>& ab,
                           hipStream_t st);

// Partial sums (part[2 b], part[2 b + 1]) of w(x) phi C_k(x) and phi C_k(x)
// over nblocks blocks, float64.
template <class S>
hipError_t launch_adj_wsum(const Coef<double>& kd, const AdjFwd<S>& fw,
                           int phase, const double* wgt, double* part,
                           int nblocks, hipStream_t st);

// lf (zeroed by the caller): the adjoint of the final state for
// J = sum w phi C_k / sum phi C_k with value J and phase mass M.
hipError_t launch_adj_seed(const Coef<double>& kd, int phase,
                           const double* wgt, double J, double M, double* lf,
                           hipStream_t st);

// dJ/dcos theta_iN = dJ/dE_i |grad psi| into gcos [N-1][n], and dJ/dpsi
// into gpsi_out [n] (ggpsi is updated in place on the way). psi64 / cos64
// (may be NULL): the float64 psi [n] and cos theta_iN [N-1][n] the wetting
// weights were made from; used for the derivative of E_i in psi instead of
// the stored psi and E_i.
template <class S>
hipError_t launch_adj_finish(const Coef<double>& kd, int nm1, const S* psi,
                             const S* wet, const double* psi64,
                             const double* cos64, const double* gE,
                             double* ggpsi, const double* gpsi, double* gcos,
                             double* gpsi_out, hipStream_t st);

}  // namespace ddcc
