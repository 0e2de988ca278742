// The context behind the opaque ddcc_ctx handle of include/ddcc.h, shared by
// the host files of the library (not installed, not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/ddcc.h"
#include "coef.hpp"

using ddcc::Coef;

struct ddcc_ctx {
  ddcc_params p{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  long long n = 0;
  int Qf = 0, Qg = 0, nhist = 0, nT = 0;
  size_t esz = 8;   // history, T and geometry fields
  size_t pesz = 8;  // moving populations
  void* f[2] = {nullptr, nullptr};
  double* f0[2] = {nullptr, nullptr};  // rest populations, float64
  void* g[2] = {nullptr, nullptr};
  void* T[2] = {nullptr, nullptr};
  void* hist = nullptr;
  void* psi = nullptr;
  void* wet = nullptr;         // wetting weights [N-1][n]
  double* work = nullptr;     // 3D: C_i and mu_i fields, 2 N n float64
  // 2D contexts with one wall: psi [n] and cos theta_iN [N-1][n] in
  // float64, for the adjoint's derivative of the wetting weights
  double* geo64 = nullptr;
  double* staging = nullptr;  // (N + dim + 1) * n float64, lazily
  double* partial = nullptr;
  int* bad = nullptr;
  int mass_blocks = 0;
  int cur = 0;
  bool geom_ok = false, fields_ok = false;
  int nwalls = 0;  // walls of the current geometry
  int64_t t = 0;
  int tile_x = 64, tile_y = 8;
  // steps run as MODE_STREAM (nontemporal stores): what one step moves does
  // not fit the memory-side cache
  bool stream_stores = false;
  // periodic in-stream diagnostics (ddcc_set_diagnostics)
  int diag_every = 0;
  int64_t diag_t = -1;          // time level of the last check
  double* diag_partial = nullptr;
  int* diag_bad = nullptr;
  long long* diag_first = nullptr;  // first level that saw a non-finite value
  std::string err;
  Coef<double> kd{};
  Coef<float> kf{};
  Coef<double>* dkd = nullptr;  // device copies of kd and kf
  Coef<float>* dkf = nullptr;
};

namespace ddcc::detail {

// Record an error message on the context and return code.
int fail(ddcc_ctx* c, int code, const std::string& msg);
// Record a HIP error (DDCC_E_NOMEM for out-of-memory, else DDCC_E_HIP).
int hip_fail(ddcc_ctx* c, hipError_t e, const char* what);
// Launch one forward step on the current buffers (the caller flips cur and
// advances t).
hipError_t step_launch(ddcc_ctx* c);

}  // namespace ddcc::detail
