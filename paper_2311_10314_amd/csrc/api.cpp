// Host side of the C ABI declared in include/ddcc.h: parameter validation,
// derived constants, device buffers (A-B population pairs), kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ddcc.h"
#include "coef.hpp"
#include "ctx.hpp"
#include "kernels.hpp"
#include "lattice.hpp"

using namespace ddcc;

namespace {

const char* kVersion = "ddcc 0.1 (gfx950)";

// Memory-side (Infinity) cache of the chip. A step that moves more than
// this streams its outputs (MODE_STREAM): 256^3 3D and 2048^2 2D steps 3-6 %
// faster; on a 512^2 box, whose step stays in this cache, plain stores are
// 19 % faster.
constexpr size_t kCacheBytes = size_t(256) << 20;

// Bytes one step moves: the populations (one buffer read, the other
// written), T likewise, the in-place history read and written, and the 3D
// work fields written and read.
size_t step_bytes(size_t pops, size_t T, size_t hist, size_t work) {
  return 2 * (pops + T + hist + work);
}

int fail(ddcc_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(ddcc_ctx* c, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(c, e == hipErrorOutOfMemory ? DDCC_E_NOMEM : DDCC_E_HIP, m);
}

#define HIPCHK(ctx, expr, what)                 \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

int lattice_q(int lat) {
  switch (lat) {
    case DDCC_D2Q9:
      return 9;
    case DDCC_D3Q7:
      return 7;
    case DDCC_D3Q15:
      return 15;
    case DDCC_D3Q19:
      return 19;
    default:
      return 0;
  }
}

// Weights w_p(d0) in the velocity order of lattice.hpp (Section 3 tables;
// D3Q19 from the same moment constraints). Returns false if any is <= 0.
bool lattice_weights(int lat, double d0, double* w) {
  double w0, w1, w2 = 0, w3 = 0;
  int q = lattice_q(lat);
  switch (lat) {
    case DDCC_D2Q9:
      w0 = (1 - d0) * (1 - d0);
      w1 = (d0 - d0 * d0) / 2;
      w2 = d0 * d0 / 4;
      for (int p = 0; p < 9; ++p) w[p] = p == 0 ? w0 : (p < 5 ? w1 : w2);
      break;
    case DDCC_D3Q7:
      w0 = 1 - 3 * d0;
      w1 = d0 / 2;
      for (int p = 0; p < 7; ++p) w[p] = p == 0 ? w0 : w1;
      break;
    case DDCC_D3Q15:
      w0 = 1 - 3 * d0 + 2 * d0 * d0;
      w1 = (d0 - d0 * d0) / 2;
      w3 = d0 * d0 / 8;
      for (int p = 0; p < 15; ++p) w[p] = p == 0 ? w0 : (p < 7 ? w1 : w3);
      break;
    case DDCC_D3Q19:
      w0 = 1 - 3 * d0 + 3 * d0 * d0;
      w1 = (d0 - 2 * d0 * d0) / 2;
      w2 = d0 * d0 / 4;
      for (int p = 0; p < 19; ++p) w[p] = p == 0 ? w0 : (p < 7 ? w1 : w2);
      break;
    default:
      return false;
  }
  for (int p = 0; p < q; ++p)
    if (!(w[p] > 0)) return false;
  return true;
}

bool finite(double x) { return std::isfinite(x); }

int validate(const ddcc_params* p, std::string& msg) {
  if (!p) {
    msg = "params is NULL";
    return DDCC_E_INVAL;
  }
  if (p->dim != 2 && p->dim != 3) {
    msg = "dim must be 2 or 3";
    return DDCC_E_INVAL;
  }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) {
    msg = "grid sizes must be >= 1";
    return DDCC_E_INVAL;
  }
  if (p->dim == 2 && p->nz != 1) {
    msg = "nz must be 1 in 2D";
    return DDCC_E_INVAL;
  }
  if ((long long)p->nx * p->ny * p->nz > (1LL << 29)) {
    msg = "grid larger than 2^29 nodes";
    return DDCC_E_INVAL;
  }
  if (p->nphase < 2 || p->nphase > DDCC_MAX_PHASES) {
    msg = "nphase must be in [2, 4]";
    return DDCC_E_INVAL;
  }
  if (p->precision != DDCC_FP64 && p->precision != DDCC_FP32 &&
      p->precision != DDCC_FP16 && p->precision != DDCC_BF16) {
    msg = "precision must be DDCC_FP64, DDCC_FP32, DDCC_FP16 or DDCC_BF16";
    return DDCC_E_INVAL;
  }
  if (p->dim == 2 && (p->lattice_f != DDCC_D2Q9 || p->lattice_g != DDCC_D2Q9)) {
    msg = "2D runs use D2Q9 for both sets";
    return DDCC_E_INVAL;
  }
  if (p->dim == 3 &&
      ((p->lattice_f != DDCC_D3Q15 && p->lattice_f != DDCC_D3Q7) ||
       (p->lattice_g != DDCC_D3Q19 && p->lattice_g != DDCC_D3Q15))) {
    msg = "3D runs use D3Q15/D3Q7 phase sets and a D3Q19/D3Q15 flow set";
    return DDCC_E_INVAL;
  }
  const double scal[] = {p->d0, p->eps, p->m0, p->rho0, p->psi_min, p->lam};
  for (double v : scal)
    if (!finite(v)) {
      msg = "non-finite scalar parameter";
      return DDCC_E_INVAL;
    }
  if (!(p->d0 > 0 && p->d0 < 1)) {
    msg = "d0 must be in (0, 1)";
    return DDCC_E_INVAL;
  }
  double w[19];
  if (!lattice_weights(p->lattice_f, p->d0, w) ||
      !lattice_weights(p->lattice_g, p->d0, w)) {
    msg = "d0 gives a non-positive lattice weight";
    return DDCC_E_INVAL;
  }
  if (!(p->eps > 0) || !(p->m0 > 0) || !(p->psi_min > 0) || !(p->lam >= 0)) {
    msg = "eps, m0, psi_min must be > 0 and lam >= 0";
    return DDCC_E_INVAL;
  }
  const int N = p->nphase;
  for (int i = 0; i < N; ++i) {
    if (!(p->rho[i] > 0) || !finite(p->rho[i]) || !(p->nu[i] > 0) ||
        !finite(p->nu[i]) || !finite(p->eta[i])) {
      msg = "rho_i and nu_i must be finite and > 0";
      return DDCC_E_INVAL;
    }
    for (int j = 0; j < N; ++j) {
      const double s = p->sigma[i][j];
      if (!finite(s) || s != p->sigma[j][i] || (i == j && s != 0) ||
          (i != j && !(s > 0))) {
        msg = "sigma must be symmetric, zero on the diagonal, > 0 elsewhere";
        return DDCC_E_INVAL;
      }
    }
  }
  for (int r = 0; r < 6; ++r) {
    if (!(p->s_f[r] > 0 && p->s_f[r] < 2)) {
      msg = "phase-set rates must be in (0, 2)";
      return DDCC_E_INVAL;
    }
    if ((r != DDCC_S21 && r != DDCC_S22) && !(p->s_g[r] > 0 && p->s_g[r] < 2)) {
      msg = "flow-set rates must be in (0, 2)";
      return DDCC_E_INVAL;
    }
  }
  for (int a = 0; a < 3; ++a)
    if (!finite(p->accel[a]) || !finite(p->force[a])) {
      msg = "non-finite body acceleration or force";
      return DDCC_E_INVAL;
    }
  return DDCC_OK;
}

template <class L>
void fourth_order_q_for(double d0, double q4[3][3]) {
  double w[19];
  lattice_weights(L::ID, d0, w);
  const double cs2 = d0;
  for (int j = 0; j < 3; ++j)
    for (int g = 0; g < 3; ++g) q4[j][g] = 0;
  for (int k = 0; k < L::Q; ++k) {
    const int j = g4_index<L>(k);
    if (j < 0) continue;
    for (int g = 0; g < L::D; ++g) {
      double s = 0;
      for (int p = 0; p < L::Q; ++p) {
        const int cg = g == 0 ? L::c[p].x : (g == 1 ? L::c[p].y : L::c[p].z);
        s += w[p] * row_value<L>(k, p, cs2) * (cg * cg - cs2);
      }
      s /= cs2 - cs2 * cs2;
      q4[j][g] = std::fabs(s) < 1e-14 ? 0.0 : s;
    }
  }
}

// q4 of coef.hpp for the flow lattice.
void fourth_order_q(int lat, double d0, double q4[3][3]) {
  switch (lat) {
    case DDCC_D3Q15:
      fourth_order_q_for<D3Q15>(d0, q4);
      break;
    case DDCC_D3Q19:
      fourth_order_q_for<D3Q19>(d0, q4);
      break;
    default:
      fourth_order_q_for<D2Q9>(d0, q4);
  }
}

template <class R>
void fill_coef(const ddcc_params& p, long long n, Coef<R>& k) {
  std::memset(&k, 0, sizeof(k));
  const int N = p.nphase;
  const double cs2 = p.d0;
  k.nx = p.nx;
  k.ny = p.ny;
  k.nz = p.nz;
  k.n = n;
  k.cs2 = R(cs2);
  k.inv_cs2 = R(1.0 / cs2);
  k.psi_min = R(p.psi_min);
  k.lam = R(p.lam);
  k.rho0 = R(p.rho0);
  k.m0 = R(p.m0);
  for (int i = 0; i < N; ++i) {
    double eta = p.eta[i];
    if (!(eta > 0)) eta = p.m0 / ((1.0 / p.s_f[DDCC_S1] - 0.5) * cs2);  // eq. 17
    k.eta[i] = R(eta);
    k.rho[i] = R(p.rho[i]);
    k.nu[i] = R(p.nu[i]);
    k.sigN[i] = R(p.sigma[i][N - 1]);
    for (int j = 0; j < N; ++j) {
      const double s = p.sigma[i][j];
      k.beta2[i][j] = R(2.0 * 3.0 * s / p.eps);  // beta_ij = 3 sigma_ij / eps
      k.grad34[i][j] = R(0.75 * p.eps * s);
      k.wet3[i][j] = R(3.0 * s);
      k.inv_sig[i][j] = i == j ? R(0) : R(1.0 / s);
    }
  }
  double w[19];
  lattice_weights(p.lattice_f, p.d0, w);
  for (int q = 0; q < lattice_q(p.lattice_f); ++q) k.wf[q] = R(w[q]);
  lattice_weights(p.lattice_g, p.d0, w);
  for (int q = 0; q < lattice_q(p.lattice_g); ++q) k.wg[q] = R(w[q]);
  const double w0g = w[0];
  for (int r = 0; r < 6; ++r) {
    k.sf[r] = R(p.s_f[r]);
    k.sg[r] = R(p.s_g[r]);
  }
  k.two_over_c2mcs2 = R(2.0 / (1.0 - cs2));
  k.h2diag = R(1.0 / (cs2 - cs2 * cs2));
  k.h2off = R(1.0 / (cs2 * cs2));
  k.inv_c2mcs2 = R(1.0 / (1.0 - cs2));
  k.pref = R(cs2 / (1.0 - w0g));
  const double K = w0g / (1.0 - p.d0);  // eq. 19: 1 - d0 (2D), 1 - 2 d0 (3D)
  const double s0 = p.s_g[DDCC_S0];
  k.cgr = R(0.5 + K * (1.0 - p.d0) * (2.0 - s0) / (2.0 * s0));
  k.halfK = R(0.5 * K);
  k.KH = R(p.dim == 2 ? K * (1.0 - 2.0 * p.d0) : K * (3.0 - 7.0 * p.d0) / 2.0);
  k.one_m3cs2 = R(1.0 - 3.0 * cs2);
  for (int a = 0; a < 3; ++a) {
    k.accel[a] = R(p.accel[a]);
    k.force[a] = R(p.force[a]);
  }
  double q4[3][3];
  fourth_order_q(p.lattice_g, p.d0, q4);
  for (int j = 0; j < 3; ++j)
    for (int g = 0; g < 3; ++g) k.q4[j][g] = R(q4[j][g]);
}

template <class Pop, class S>
Bufs<Pop, S> bufs(ddcc_ctx* c, int mode) {
  Bufs<Pop, S> b{};
  const int a = c->cur, o = c->cur ^ 1;
  b.fA = static_cast<const Pop*>(c->f[a]);
  b.f0A = c->f0[a];
  b.gA = static_cast<const Pop*>(c->g[a]);
  b.TA = static_cast<const S*>(c->T[a]);
  if (mode == MODE_INIT) {
    b.fB = static_cast<Pop*>(c->f[a]);
    b.f0B = c->f0[a];
    b.gB = static_cast<Pop*>(c->g[a]);
    b.TB = static_cast<S*>(c->T[a]);
  } else {
    b.fB = static_cast<Pop*>(c->f[o]);
    b.f0B = c->f0[o];
    b.gB = static_cast<Pop*>(c->g[o]);
    b.TB = static_cast<S*>(c->T[o]);
  }
  b.hist = static_cast<S*>(c->hist);
  b.psi = static_cast<const S*>(c->psi);
  b.wet = static_cast<const S*>(c->wet);
  if (c->work) {
    b.fC = c->work;
    b.fmu = c->work + (size_t)c->p.nphase * c->n;
  }
  b.coef_d = c->dkd;
  b.coef_r = sizeof(S) == 8 ? static_cast<const void*>(c->dkd)
                            : static_cast<const void*>(c->dkf);
  return b;
}

template <class Pop, class S, class R>
hipError_t launch_as(ddcc_ctx* c, const Coef<R>& k, int mode,
                     const double* inC, const double* inU, const double* inP,
                     double* oC, double* oU, double* oP) {
  Bufs<Pop, S> b = bufs<Pop, S>(c, mode);
  if (mode == MODE_STEP && c->stream_stores) mode = MODE_STREAM;
  b.inC = inC;
  b.inU = inU;
  b.inP = inP;
  b.outC = oC;
  b.outU = oU;
  b.outP = oP;
  if (c->p.dim == 2)
    return launch_2d<Pop, S, R>(c->p.nphase, mode, c->kd, k, b, c->tile_y,
                                c->stream);
  return launch_3d<Pop, S, R>(c->p.nphase, c->p.lattice_f, mode, c->kd, k, b,
                              c->tile_x, c->tile_y, c->stream);
}

hipError_t launch(ddcc_ctx* c, int mode, const double* inC, const double* inU,
                  const double* inP, double* oC, double* oU, double* oP) {
  switch (c->p.precision) {
    case DDCC_FP64:
      return launch_as<double, double>(c, c->kd, mode, inC, inU, inP, oC, oU,
                                       oP);
    case DDCC_FP16:
      return launch_as<_Float16, float>(c, c->kf, mode, inC, inU, inP, oC, oU,
                                        oP);
    case DDCC_BF16:
      return launch_as<__bf16, float>(c, c->kf, mode, inC, inU, inP, oC, oU,
                                      oP);
    default:
      return launch_as<float, float>(c, c->kf, mode, inC, inU, inP, oC, oU,
                                     oP);
  }
}

int ensure_staging(ddcc_ctx* c) {
  if (c->staging) return DDCC_OK;
  const size_t count = (size_t)(c->p.nphase + c->p.dim + 1) * c->n;
  HIPCHK(c, hipMalloc(&c->staging, count * sizeof(double)), "hipMalloc staging");
  return DDCC_OK;
}

bool all_finite(const double* a, size_t count) {
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

void release(ddcc_ctx* c) {
  void* ptrs[] = {c->f[0],  c->f[1],   c->f0[0],    c->f0[1], c->g[0],
                  c->g[1],  c->T[0],   c->T[1],     c->hist,  c->psi,
                  c->wet,   c->staging, c->partial, c->bad,  c->work,
                  c->diag_partial, c->diag_bad, c->diag_first,
                  c->dkd,   c->dkf,    c->geo64};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

// Launch the per-phase population sums of the current state into
// partial[block * N + i] with non-finite flags bad[block].
hipError_t mass_into(ddcc_ctx* c, double* partial, int* bad) {
  const int N = c->p.nphase;
  const void* f = c->f[c->cur];
  const double* f0 = c->f0[c->cur];
  switch (c->p.precision) {
    case DDCC_FP64:
      return launch_mass(f0, static_cast<const double*>(f), N, c->Qf, c->n,
                         c->n, partial, bad, c->mass_blocks, c->stream);
    case DDCC_FP16:
      return launch_mass(f0, static_cast<const _Float16*>(f), N, c->Qf, c->n,
                         c->n, partial, bad, c->mass_blocks, c->stream);
    case DDCC_BF16:
      return launch_mass(f0, static_cast<const __bf16*>(f), N, c->Qf, c->n,
                         c->n, partial, bad, c->mass_blocks, c->stream);
    default:
      return launch_mass(f0, static_cast<const float*>(f), N, c->Qf, c->n,
                         c->n, partial, bad, c->mass_blocks, c->stream);
  }
}

// Clear the record of the periodic checks (new state or new setting).
int diag_reset(ddcc_ctx* c) {
  c->diag_t = -1;
  if (!c->diag_first) return DDCC_OK;
  const long long none = -1;
  HIPCHK(c, hipMemcpyAsync(c->diag_first, &none, sizeof(none),
                           hipMemcpyHostToDevice, c->stream),
         "clear diagnostics");
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  return DDCC_OK;
}

struct SaveHeader {
  char magic[8];
  int32_t dim, nx, ny, nz, nphase, lattice_f, lattice_g, precision;
  int64_t t;
  int64_t bytes;
};

}  // namespace

namespace ddcc {
bool have_3d();

namespace detail {
int fail(ddcc_ctx* c, int code, const std::string& msg) {
  return ::fail(c, code, msg);
}
int hip_fail(ddcc_ctx* c, hipError_t e, const char* what) {
  return ::hip_fail(c, e, what);
}
hipError_t step_launch(ddcc_ctx* c) {
  return launch(c, MODE_STEP, nullptr, nullptr, nullptr, nullptr, nullptr,
                nullptr);
}
}  // namespace detail
}  // namespace ddcc

extern "C" {

const char* ddcc_version(void) { return kVersion; }

int ddcc_default_params(ddcc_params* p) {
  if (!p) return DDCC_E_INVAL;
  std::memset(p, 0, sizeof(*p));
  p->dim = 2;
  p->nx = 64;
  p->ny = 64;
  p->nz = 1;
  p->nphase = 2;
  p->lattice_f = DDCC_D2Q9;
  p->lattice_g = DDCC_D2Q9;
  p->precision = DDCC_FP64;
  p->d0 = 0.4;
  p->eps = 5.0;
  p->m0 = 0.05;
  p->rho0 = 1.0;
  p->psi_min = 1e-30;
  p->lam = 1.0 / std::pow(2.0 * std::sqrt(2.0) * 1.5, 3);
  for (int i = 0; i < DDCC_MAX_PHASES; ++i) {
    p->rho[i] = 1.0;
    p->nu[i] = 0.1;
    p->eta[i] = 0.0;
    for (int j = 0; j < DDCC_MAX_PHASES; ++j)
      p->sigma[i][j] = i == j ? 0.0 : 0.001;
  }
  const double sf[6] = {1.0, 10.0 / 19.0, 1.2, 1.2, 1.2, 1.2};
  const double sg[6] = {1.0, 1.2, 1.2, 1.2, 1.2, 1.2};
  for (int r = 0; r < 6; ++r) {
    p->s_f[r] = sf[r];
    p->s_g[r] = sg[r];
  }
  return DDCC_OK;
}

int ddcc_create(const ddcc_params* p, void* stream, ddcc_ctx** out) {
  if (!out) return DDCC_E_INVAL;
  *out = nullptr;
  std::string msg;
  int rc = validate(p, msg);
  if (rc != DDCC_OK) return rc;
  ddcc_ctx* c = new (std::nothrow) ddcc_ctx();
  if (!c) return DDCC_E_NOMEM;
  c->p = *p;
  c->n = (long long)p->nx * p->ny * p->nz;
  c->Qf = lattice_q(p->lattice_f);
  c->Qg = lattice_q(p->lattice_g);
  const int d = p->dim;
  // 2D: phi C_i u (2N), Y (3), P; 3D: phi C_i (N), u (3), m^C (3), P
  c->nhist = d == 2 ? 2 * p->nphase + 4 : p->nphase + 7;
  c->nT = d * (d - 1) / 2;
  c->esz = p->precision == DDCC_FP64 ? 8 : 4;
  c->pesz = p->precision == DDCC_FP64 ? 8 : (p->precision == DDCC_FP32 ? 4 : 2);
  // 2D: 64 x 4 tiles for float64 arithmetic (its registers allow three
  // waves per SIMD, which 4-wave workgroups fill; 1-15 % faster than 64 x 8
  // from 4096^2 down to 128^2), 64 x 8 for float; 3D: 64 x 4 columns.
  c->tile_y = d == 2 ? (p->precision == DDCC_FP64 ? 4 : 8) : 4;
  c->tile_x = 64;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return DDCC_E_HIP;
  }
  if (stream) {
    c->stream = static_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return DDCC_E_HIP;
    }
    c->own_stream = true;
  }
  fill_coef<double>(c->p, c->n, c->kd);
  fill_coef<float>(c->p, c->n, c->kf);
  const size_t n = (size_t)c->n;
  const size_t sf = (size_t)p->nphase * (c->Qf - 1) * n * c->pesz;
  const size_t sg = (size_t)c->Qg * n * c->pesz;
  const size_t sT = (size_t)c->nT * n * c->esz;
  hipError_t e = hipSuccess;
  for (int a = 0; a < 2 && e == hipSuccess; ++a) {
    e = hipMalloc(&c->f[a], sf);
    if (e == hipSuccess)
      e = hipMalloc(&c->f0[a], (size_t)p->nphase * n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&c->g[a], sg);
    if (e == hipSuccess) e = hipMalloc(&c->T[a], sT);
  }
  if (e == hipSuccess) e = hipMalloc(&c->hist, (size_t)c->nhist * n * c->esz);
  c->stream_stores =
      step_bytes(sf + sg + (size_t)p->nphase * n * sizeof(double), sT,
                 (size_t)c->nhist * n * c->esz,
                 d == 3 ? (size_t)2 * p->nphase * n * c->esz : 0) > kCacheBytes;
  if (e == hipSuccess) e = hipMalloc(&c->psi, n * c->esz);
  if (e == hipSuccess)
    e = hipMalloc(&c->wet, (size_t)(p->nphase - 1) * n * c->esz);
  if (e == hipSuccess && p->dim == 3)
    e = hipMalloc(&c->work, (size_t)2 * p->nphase * n * sizeof(double));
  long long mb = (c->n + 255) / 256;
  c->mass_blocks = (int)(mb > kScratchBlocks ? kScratchBlocks : mb);
  if (e == hipSuccess)
    e = hipMalloc(&c->partial,
                  (size_t)c->mass_blocks * p->nphase * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&c->bad, (size_t)c->mass_blocks * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&c->dkd, sizeof(Coef<double>));
  if (e == hipSuccess) e = hipMalloc(&c->dkf, sizeof(Coef<float>));
  if (e == hipSuccess)
    e = hipMemcpy(c->dkd, &c->kd, sizeof(Coef<double>), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->dkf, &c->kf, sizeof(Coef<float>), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    release(c);
    delete c;
    return e == hipErrorOutOfMemory ? DDCC_E_NOMEM : DDCC_E_HIP;
  }
  if (p->dim == 3) {
    // The 3D kernels are built per (phase, flow) lattice pair; the host
    // checks the pair here so that create fails early when it is absent.
    if (!((p->lattice_f == DDCC_D3Q15 || p->lattice_f == DDCC_D3Q7) &&
          p->lattice_g == DDCC_D3Q19) ||
        p->nphase > 3 || !have_3d()) {
      release(c);
      delete c;
      return DDCC_E_UNSUPPORTED;
    }
  }
  *out = c;
  return DDCC_OK;
}

// Geometry of K walls from float64 device arrays psik [K][n] and ctk
// [K][N-1][n] (NULL: 90 degrees): psi and the wetting weights in the
// context's field precision.
static int geometry_from_device(ddcc_ctx* c, int K, const double* psik,
                                const double* ctk) {
  const int nm1 = c->p.nphase - 1;
  hipError_t e =
      c->p.precision == DDCC_FP64
          ? launch_wet_field<double>(psik, ctk, K, nm1, c->p.nx, c->p.ny,
                                     c->p.nz, static_cast<double*>(c->psi),
                                     static_cast<double*>(c->wet), c->n, 0,
                                     c->stream)
          : launch_wet_field<float>(psik, ctk, K, nm1, c->p.nx, c->p.ny,
                                    c->p.nz, static_cast<float*>(c->psi),
                                    static_cast<float*>(c->wet), c->n, 0,
                                    c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "geometry kernel");
  // The adjoint's derivative of the wetting weights E_i = cos theta_iN
  // |grad psi| with respect to psi is cos theta_iN grad psi / |grad psi|,
  // taken from the float64 psi and cosines: a float32 psi rounds to 1 a few
  // cells off a wall, where grad psi is small but not zero, and E_i / |grad
  // psi| mixes two evaluations of |grad psi| that differ in their rounding
  // where psi is 1 up to rounding. 2D contexts with one wall (those the
  // adjoint supports) keep the float64 psi and cosines.
  if (c->p.dim == 2 && K == 1) {
    const size_t n = (size_t)c->n;
    if (!c->geo64)
      HIPCHK(c, hipMalloc(&c->geo64, (size_t)(nm1 + 1) * n * sizeof(double)),
             "hipMalloc float64 geometry");
    e = hipMemcpyAsync(c->geo64, psik, n * sizeof(double),
                       hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
      e = ctk ? hipMemcpyAsync(c->geo64 + n, ctk, nm1 * n * sizeof(double),
                               hipMemcpyDeviceToDevice, c->stream)
              : hipMemsetAsync(c->geo64 + n, 0, nm1 * n * sizeof(double),
                               c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "copy float64 geometry");
  }
  c->geom_ok = true;
  c->nwalls = K;
  c->fields_ok = false;
  return DDCC_OK;
}

// Checks K walls on the host (psi_k in [0, 1], cosines in [-1, 1]).
static int check_walls(ddcc_ctx* c, int K, const double* psik,
                       const double* ctk) {
  if (K < 1 || K > DDCC_MAX_WALLS)
    return fail(c, DDCC_E_INVAL, "number of walls must be in [1, 8]");
  if (!psik) return fail(c, DDCC_E_INVAL, "psi is NULL");
  const size_t n = (size_t)c->n;
  for (size_t i = 0; i < (size_t)K * n; ++i)
    if (!(psik[i] >= 0.0 && psik[i] <= 1.0))
      return fail(c, DDCC_E_INVAL, "psi must be finite and in [0, 1]");
  if (ctk)
    for (size_t i = 0; i < (size_t)K * (c->p.nphase - 1) * n; ++i)
      if (!(ctk[i] >= -1.0 && ctk[i] <= 1.0))
        return fail(c, DDCC_E_INVAL, "cos_theta must be finite and in [-1, 1]");
  return DDCC_OK;
}

int ddcc_init_geometry_walls(ddcc_ctx* c, int nwalls, const double* psi,
                             const double* cos_theta) {
  if (!c) return DDCC_E_INVAL;
  int rc = check_walls(c, nwalls, psi, cos_theta);
  if (rc) return rc;
  const size_t n = (size_t)c->n, np = (size_t)nwalls * n;
  const size_t nc = cos_theta ? np * (c->p.nphase - 1) : 0;
  double* d = nullptr;
  HIPCHK(c, hipMalloc(&d, (np + nc) * sizeof(double)), "hipMalloc geometry");
  hipError_t e = hipMemcpyAsync(d, psi, np * sizeof(double),
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && nc)
    e = hipMemcpyAsync(d + np, cos_theta, nc * sizeof(double),
                       hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(c, e, "copy geometry");
  }
  rc = geometry_from_device(c, nwalls, d, nc ? d + np : nullptr);
  e = hipStreamSynchronize(c->stream);
  (void)hipFree(d);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(c, e, "sync");
  return DDCC_OK;
}

int ddcc_init_geometry(ddcc_ctx* c, const double* psi, const double* ct) {
  return ddcc_init_geometry_walls(c, 1, psi, ct);
}

int ddcc_init_geometry_dev(ddcc_ctx* c, const double* psi, const double* ct) {
  if (!c) return DDCC_E_INVAL;
  if (!psi) return fail(c, DDCC_E_INVAL, "psi is NULL");
  return geometry_from_device(c, 1, psi, ct);
}

static int init_fields_common(ddcc_ctx* c, const double* C, const double* u,
                              const double* P) {
  hipError_t e = launch(c, MODE_INIT, C, u, P, nullptr, nullptr, nullptr);
  if (e != hipSuccess) return hip_fail(c, e, "init kernel");
  c->fields_ok = true;
  c->t = 0;
  return diag_reset(c);
}

int ddcc_init_fields(ddcc_ctx* c, const double* C, const double* u,
                     const double* P) {
  if (!c) return DDCC_E_INVAL;
  if (!c->geom_ok) return fail(c, DDCC_E_STATE, "init_geometry first");
  if (!C) return fail(c, DDCC_E_INVAL, "C is NULL");
  const size_t n = (size_t)c->n;
  const int N = c->p.nphase, d = c->p.dim;
  if (!all_finite(C, N * n) || (u && !all_finite(u, d * n)) ||
      (P && !all_finite(P, n)))
    return fail(c, DDCC_E_INVAL, "non-finite initial field");
  int rc = ensure_staging(c);
  if (rc) return rc;
  double* sC = c->staging;
  double* sU = sC + N * n;
  double* sP = sU + d * n;
  HIPCHK(c, hipMemcpyAsync(sC, C, N * n * sizeof(double), hipMemcpyHostToDevice,
                           c->stream),
         "copy C");
  if (u)
    HIPCHK(c, hipMemcpyAsync(sU, u, d * n * sizeof(double),
                             hipMemcpyHostToDevice, c->stream),
           "copy u");
  if (P)
    HIPCHK(c, hipMemcpyAsync(sP, P, n * sizeof(double), hipMemcpyHostToDevice,
                             c->stream),
           "copy P");
  rc = init_fields_common(c, sC, u ? sU : nullptr, P ? sP : nullptr);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  return DDCC_OK;
}

int ddcc_init_fields_dev(ddcc_ctx* c, const double* C, const double* u,
                         const double* P) {
  if (!c) return DDCC_E_INVAL;
  if (!c->geom_ok) return fail(c, DDCC_E_STATE, "init_geometry first");
  if (!C) return fail(c, DDCC_E_INVAL, "C is NULL");
  return init_fields_common(c, C, u, P);
}

int ddcc_step(ddcc_ctx* c, int64_t nsteps) {
  if (!c) return DDCC_E_INVAL;
  if (nsteps < 0) return fail(c, DDCC_E_INVAL, "nsteps < 0");
  if (!c->fields_ok) return fail(c, DDCC_E_STATE, "init_fields first");
  for (int64_t s = 0; s < nsteps; ++s) {
    hipError_t e = launch(c, MODE_STEP, nullptr, nullptr, nullptr, nullptr,
                          nullptr, nullptr);
    if (e != hipSuccess) return hip_fail(c, e, "step kernel");
    c->cur ^= 1;
    ++c->t;
    if (c->diag_every > 0 && c->t % c->diag_every == 0) {
      e = mass_into(c, c->diag_partial, c->diag_bad);
      if (e == hipSuccess)
        e = launch_sticky(c->diag_bad, c->mass_blocks, c->diag_first,
                          (long long)c->t, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "diagnostics");
      c->diag_t = c->t;
    }
  }
  return DDCC_OK;
}

static int moments_common(ddcc_ctx* c, double* C, double* u, double* P) {
  hipError_t e = launch(c, MODE_MOMENTS, nullptr, nullptr, nullptr, C, u, P);
  if (e != hipSuccess) return hip_fail(c, e, "moments kernel");
  return DDCC_OK;
}

int ddcc_read_moments(ddcc_ctx* c, double* C, double* u, double* P) {
  if (!c) return DDCC_E_INVAL;
  if (!c->fields_ok) return fail(c, DDCC_E_STATE, "init_fields first");
  int rc = ensure_staging(c);
  if (rc) return rc;
  const size_t n = (size_t)c->n;
  const int N = c->p.nphase, d = c->p.dim;
  double* sC = c->staging;
  double* sU = sC + N * n;
  double* sP = sU + d * n;
  rc = moments_common(c, sC, sU, sP);
  if (rc) return rc;
  if (C)
    HIPCHK(c, hipMemcpyAsync(C, sC, N * n * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream),
           "copy C");
  if (u)
    HIPCHK(c, hipMemcpyAsync(u, sU, d * n * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream),
           "copy u");
  if (P)
    HIPCHK(c, hipMemcpyAsync(P, sP, n * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream),
           "copy P");
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  return DDCC_OK;
}

int ddcc_read_moments_dev(ddcc_ctx* c, double* C, double* u, double* P) {
  if (!c) return DDCC_E_INVAL;
  if (!c->fields_ok) return fail(c, DDCC_E_STATE, "init_fields first");
  if (!C || !u || !P)
    return fail(c, DDCC_E_INVAL, "device read-out needs all three outputs");
  return moments_common(c, C, u, P);
}

int ddcc_mass(ddcc_ctx* c, double* mass) {
  if (!c || !mass) return fail(c, DDCC_E_INVAL, "NULL argument");
  if (!c->fields_ok) return fail(c, DDCC_E_STATE, "init_fields first");
  const int N = c->p.nphase;
  const hipError_t e = mass_into(c, c->partial, c->bad);
  if (e != hipSuccess) return hip_fail(c, e, "mass kernel");
  std::vector<double> part((size_t)c->mass_blocks * N);
  std::vector<int> bad(c->mass_blocks);
  HIPCHK(c, hipMemcpyAsync(part.data(), c->partial, part.size() * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream),
         "copy partials");
  HIPCHK(c, hipMemcpyAsync(bad.data(), c->bad, bad.size() * sizeof(int),
                           hipMemcpyDeviceToHost, c->stream),
         "copy flags");
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int b = 0; b < c->mass_blocks; ++b) s += part[(size_t)b * N + i];
    mass[i] = s;
  }
  for (int b = 0; b < c->mass_blocks; ++b)
    if (bad[b]) return fail(c, DDCC_E_NONFINITE, "non-finite population");
  return DDCC_OK;
}

int ddcc_mass_noalloc(ddcc_ctx* c, double* mass_dev, int* nonfinite_dev) {
  if (!c || !mass_dev) return fail(c, DDCC_E_INVAL, "NULL argument");
  if (!c->fields_ok) return fail(c, DDCC_E_STATE, "init_fields first");
  const int N = c->p.nphase;
  void* ws = nullptr;
  size_t cap = 0;
  HIPCHK(c, scratch_address(c->device, &ws, &cap), "static workspace address");
  const size_t part_bytes = (size_t)kScratchBlocks * kMaxN * sizeof(double);
  const size_t need_part = (size_t)c->mass_blocks * N * sizeof(double);
  const size_t need_bad = (size_t)c->mass_blocks * sizeof(int);
  if (c->mass_blocks > kScratchBlocks || need_part > part_bytes ||
      part_bytes + need_bad > cap)
    return fail(c, DDCC_E_INVAL,
                "mass check needs more than the static workspace (1024 "
                "blocks of partial sums)");
  double* partial = static_cast<double*>(ws);
  int* bad = reinterpret_cast<int*>(static_cast<char*>(ws) + part_bytes);
  hipError_t e = mass_into(c, partial, bad);
  if (e == hipSuccess)
    e = launch_mass_finish(partial, bad, c->mass_blocks, N, mass_dev,
                           nonfinite_dev, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "mass kernel");
  return DDCC_OK;
}

int64_t ddcc_time(const ddcc_ctx* c) { return c ? c->t : -1; }

int ddcc_save(ddcc_ctx* c, void* buf, size_t* bytes) {
  if (!c || !bytes) return fail(c, DDCC_E_INVAL, "NULL argument");
  if (!c->fields_ok) return fail(c, DDCC_E_STATE, "init_fields first");
  const size_t n = (size_t)c->n;
  const size_t sf = (size_t)c->p.nphase * (c->Qf - 1) * n * c->pesz;
  const size_t sg = (size_t)c->Qg * n * c->pesz;
  const size_t sh = (size_t)c->nhist * n * c->esz;
  const size_t sT = (size_t)c->nT * n * c->esz;
  const size_t s0 = (size_t)c->p.nphase * n * sizeof(double);
  const size_t need = sizeof(SaveHeader) + sf + s0 + sg + sh + sT;
  if (!buf) {
    *bytes = need;
    return DDCC_OK;
  }
  if (*bytes < need) return fail(c, DDCC_E_INVAL, "buffer too small");
  SaveHeader h{};
  std::memcpy(h.magic, "DDCCSAV4", 8);
  h.dim = c->p.dim;
  h.nx = c->p.nx;
  h.ny = c->p.ny;
  h.nz = c->p.nz;
  h.nphase = c->p.nphase;
  h.lattice_f = c->p.lattice_f;
  h.lattice_g = c->p.lattice_g;
  h.precision = c->p.precision;
  h.t = c->t;
  h.bytes = (int64_t)need;
  char* o = static_cast<char*>(buf);
  std::memcpy(o, &h, sizeof(h));
  o += sizeof(h);
  HIPCHK(c, hipMemcpyAsync(o, c->f[c->cur], sf, hipMemcpyDeviceToHost, c->stream),
         "save f");
  o += sf;
  HIPCHK(c, hipMemcpyAsync(o, c->f0[c->cur], s0, hipMemcpyDeviceToHost,
                           c->stream),
         "save f0");
  o += s0;
  HIPCHK(c, hipMemcpyAsync(o, c->g[c->cur], sg, hipMemcpyDeviceToHost, c->stream),
         "save g");
  o += sg;
  HIPCHK(c, hipMemcpyAsync(o, c->hist, sh, hipMemcpyDeviceToHost, c->stream),
         "save hist");
  o += sh;
  if (sT)
    HIPCHK(c, hipMemcpyAsync(o, c->T[c->cur], sT, hipMemcpyDeviceToHost,
                             c->stream),
           "save T");
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  *bytes = need;
  return DDCC_OK;
}

int ddcc_load(ddcc_ctx* c, const void* buf, size_t bytes) {
  if (!c || !buf) return fail(c, DDCC_E_INVAL, "NULL argument");
  if (!c->geom_ok) return fail(c, DDCC_E_STATE, "init_geometry first");
  const size_t n = (size_t)c->n;
  const size_t sf = (size_t)c->p.nphase * (c->Qf - 1) * n * c->pesz;
  const size_t sg = (size_t)c->Qg * n * c->pesz;
  const size_t sh = (size_t)c->nhist * n * c->esz;
  const size_t sT = (size_t)c->nT * n * c->esz;
  const size_t s0 = (size_t)c->p.nphase * n * sizeof(double);
  const size_t need = sizeof(SaveHeader) + sf + s0 + sg + sh + sT;
  if (bytes < need) return fail(c, DDCC_E_INVAL, "checkpoint too small");
  SaveHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, "DDCCSAV4", 8) != 0 || h.dim != c->p.dim ||
      h.nx != c->p.nx || h.ny != c->p.ny || h.nz != c->p.nz ||
      h.nphase != c->p.nphase || h.lattice_f != c->p.lattice_f ||
      h.lattice_g != c->p.lattice_g || h.precision != c->p.precision ||
      h.bytes != (int64_t)need)
    return fail(c, DDCC_E_INVAL, "checkpoint does not match this context");
  const char* s = static_cast<const char*>(buf) + sizeof(h);
  HIPCHK(c, hipMemcpyAsync(c->f[c->cur], s, sf, hipMemcpyHostToDevice, c->stream),
         "load f");
  s += sf;
  HIPCHK(c, hipMemcpyAsync(c->f0[c->cur], s, s0, hipMemcpyHostToDevice,
                           c->stream),
         "load f0");
  s += s0;
  HIPCHK(c, hipMemcpyAsync(c->g[c->cur], s, sg, hipMemcpyHostToDevice, c->stream),
         "load g");
  s += sg;
  HIPCHK(c, hipMemcpyAsync(c->hist, s, sh, hipMemcpyHostToDevice, c->stream),
         "load hist");
  s += sh;
  if (sT)
    HIPCHK(c, hipMemcpyAsync(c->T[c->cur], s, sT, hipMemcpyHostToDevice,
                             c->stream),
           "load T");
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  c->t = h.t;
  c->fields_ok = true;
  return diag_reset(c);
}

int ddcc_sync(ddcc_ctx* c) {
  if (!c) return DDCC_E_INVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  if (c->diag_every > 0) {
    long long first = -1;
    HIPCHK(c, hipMemcpy(&first, c->diag_first, sizeof(first),
                        hipMemcpyDeviceToHost),
           "read diagnostics");
    if (first >= 0)
      return fail(c, DDCC_E_NONFINITE,
                  "non-finite population found by the check at step " +
                      std::to_string(first));
  }
  return DDCC_OK;
}

int ddcc_set_diagnostics(ddcc_ctx* c, int every) {
  if (!c) return DDCC_E_INVAL;
  if (every < 0) return fail(c, DDCC_E_INVAL, "every < 0");
  if (every > 0 && !c->diag_first) {
    const int N = c->p.nphase;
    HIPCHK(c, hipMalloc(&c->diag_partial,
                        (size_t)c->mass_blocks * N * sizeof(double)),
           "hipMalloc diagnostics");
    HIPCHK(c, hipMalloc(&c->diag_bad, (size_t)c->mass_blocks * sizeof(int)),
           "hipMalloc diagnostics");
    HIPCHK(c, hipMalloc(&c->diag_first, sizeof(long long)), "hipMalloc diagnostics");
  }
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  c->diag_every = every;
  return diag_reset(c);
}

int ddcc_diagnostics(ddcc_ctx* c, double* mass, int64_t* t_checked,
                     int64_t* t_nonfinite) {
  if (!c) return DDCC_E_INVAL;
  if (c->diag_every <= 0)
    return fail(c, DDCC_E_STATE, "diagnostics are off (ddcc_set_diagnostics)");
  const int N = c->p.nphase;
  std::vector<double> part((size_t)c->mass_blocks * N);
  long long first = -1;
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  if (c->diag_t >= 0 && mass)
    HIPCHK(c, hipMemcpy(part.data(), c->diag_partial,
                        part.size() * sizeof(double), hipMemcpyDeviceToHost),
           "read diagnostics");
  HIPCHK(c, hipMemcpy(&first, c->diag_first, sizeof(first),
                      hipMemcpyDeviceToHost),
         "read diagnostics");
  if (mass)
    for (int i = 0; i < N; ++i) {
      double sum = 0.0;
      for (int b = 0; b < c->mass_blocks; ++b) sum += part[(size_t)b * N + i];
      mass[i] = c->diag_t >= 0 ? sum : std::nan("");
    }
  if (t_checked) *t_checked = c->diag_t;
  if (t_nonfinite) *t_nonfinite = first;
  return DDCC_OK;
}

int ddcc_set_tile(ddcc_ctx* c, int tx, int ty) {
  if (!c) return DDCC_E_INVAL;
  if (c->p.dim == 2) {
    if (tx != 0 && tx != 64)
      return fail(c, DDCC_E_INVAL, "2D tiles are 64 nodes wide");
    if (ty != 0 && ty != 2 && ty != 4 && ty != 8 && ty != 16)
      return fail(c, DDCC_E_INVAL, "2D tile height must be 2, 4, 8 or 16");
    if (ty) c->tile_y = ty;
  } else {
    if (tx != 0 && tx != 64)
      return fail(c, DDCC_E_INVAL, "3D tiles are 64 nodes wide");
    if (ty != 0 && ty != 2 && ty != 4)
      return fail(c, DDCC_E_INVAL, "3D tile height must be 2 or 4");
    if (tx) c->tile_x = tx;
    if (ty) c->tile_y = ty;
  }
  return DDCC_OK;
}

int ddcc_autotune(ddcc_ctx* c, int steps, int* ty_out) {
  if (!c) return DDCC_E_INVAL;
  if (steps < 1) return fail(c, DDCC_E_INVAL, "steps < 1");
  if (!c->fields_ok) return fail(c, DDCC_E_STATE, "init_fields first");
  // The trial steps change the state: keep a copy of the current level (a
  // step reads populations and T at cur, writes them at cur ^ 1, and updates
  // the history in place).
  const size_t n = (size_t)c->n;
  const int N = c->p.nphase;
  const int cur0 = c->cur;
  const size_t sizes[5] = {(size_t)N * (c->Qf - 1) * n * c->pesz,
                           (size_t)N * n * sizeof(double),
                           (size_t)c->Qg * n * c->pesz,
                           (size_t)c->nT * n * c->esz,
                           (size_t)c->nhist * n * c->esz};
  void* src[5] = {c->f[cur0], c->f0[cur0], c->g[cur0], c->T[cur0], c->hist};
  void* keep[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  hipError_t e = hipSuccess;
  for (int q = 0; q < 5 && e == hipSuccess; ++q) {
    if (!sizes[q] || !src[q]) continue;
    e = hipMalloc(&keep[q], sizes[q]);
    if (e == hipSuccess)
      e = hipMemcpyAsync(keep[q], src[q], sizes[q], hipMemcpyDeviceToDevice,
                         c->stream);
  }
  const int cands2[4] = {2, 4, 8, 16}, cands3[2] = {2, 4};
  const int* cands = c->p.dim == 2 ? cands2 : cands3;
  const int ncand = c->p.dim == 2 ? 4 : 2;
  const int ty0 = c->tile_y;
  float best_ms = 0;
  int best = ty0;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  const int64_t tsave = c->t;
  for (int k = 0; k < ncand && e == hipSuccess; ++k) {
    c->tile_y = cands[k];
    for (int s = 0; s < 2 + steps && e == hipSuccess; ++s) {
      if (s == 2) e = hipEventRecord(t0, c->stream);
      if (e == hipSuccess)
        e = launch(c, MODE_STEP, nullptr, nullptr, nullptr, nullptr, nullptr,
                   nullptr);
      c->cur ^= 1;
    }
    if (e == hipSuccess) e = hipEventRecord(t1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (e == hipSuccess && (k == 0 || ms < best_ms)) {
      best_ms = ms;
      best = cands[k];
    }
  }
  // restore the level the trials started from
  c->cur = cur0;
  c->t = tsave;
  for (int q = 0; q < 5; ++q)
    if (keep[q] && e == hipSuccess)
      e = hipMemcpyAsync(src[q], keep[q], sizes[q], hipMemcpyDeviceToDevice,
                         c->stream);
  const hipError_t es = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = es;
  for (int q = 0; q < 5; ++q)
    if (keep[q]) (void)hipFree(keep[q]);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (e != hipSuccess) {
    c->tile_y = ty0;
    return hip_fail(c, e, "autotune");
  }
  c->tile_y = best;
  if (ty_out) *ty_out = best;
  return DDCC_OK;
}

const char* ddcc_last_error(const ddcc_ctx* c) {
  return c ? c->err.c_str() : "NULL context";
}

void ddcc_destroy(ddcc_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  release(c);
  delete c;
}

}  // extern "C"

// ===========================================================================
// Batches: many independent 2D D2Q9 boxes advanced by one launch per step.
// ===========================================================================
struct ddcc_batch {
  ddcc_params p{};
  int count = 0;
  std::vector<int> nx, ny;
  std::vector<long long> n, off;  // nodes and first node of each instance
  long long ntot = 0;             // plane stride: nodes of all instances
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t esz = 8, pesz = 8;
  void* f[2] = {nullptr, nullptr};
  double* f0[2] = {nullptr, nullptr};
  void* g[2] = {nullptr, nullptr};
  void* T[2] = {nullptr, nullptr};
  void* hist = nullptr;
  void* psi = nullptr;
  void* wet = nullptr;        // wetting weights [N-1][ntot]
  double* staging = nullptr;  // (N + 3) planes of ntot float64
  double* partial = nullptr;
  int* bad = nullptr;
  int mass_blocks = 0;
  BatchTile* tiles = nullptr;
  BatchInst* insts = nullptr;
  std::vector<unsigned> t0, t1;  // tile range of each instance
  unsigned ntiles = 0;
  unsigned* counters = nullptr;  // one per step of a captured graph
  int ty = 8;
  int blocks = 1;                // persistent workgroups per launch
  int graph_steps = 0;           // 0: one launch per step, no graph
  bool stream_stores = false;    // steps as MODE_STREAM (see ddcc_ctx)
  hipGraphExec_t gexec[2] = {nullptr, nullptr};  // by parity of cur
  int cur = 0;
  int cus = 0;
  std::vector<char> geom_ok, fields_ok;
  int64_t t = 0;
  std::string err;
  Coef<double> kd{};
  Coef<float> kf{};
  // device tables of every instance's coefficients (the batch parameters,
  // or an instance's own ones from ddcc_batch_set_params)
  Coef<double>* kds = nullptr;
  Coef<float>* kfs = nullptr;
};

namespace {

constexpr int kMaxGraphSteps = 1024;
constexpr int kBatchQ = 9;

int bfail(ddcc_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  return code;
}

int bhip(ddcc_batch* b, hipError_t e, const char* what) {
  return bfail(b, e == hipErrorOutOfMemory ? DDCC_E_NOMEM : DDCC_E_HIP,
               std::string(what) + ": " + hipGetErrorString(e));
}

#define BHIP(b, expr, what)                            \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return bhip(b, e_, what);    \
  } while (0)

int nhist_of(int N) { return 2 * N + 4; }

void drop_graphs(ddcc_batch* b) {
  for (auto& g : b->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

void batch_release(ddcc_batch* b) {
  drop_graphs(b);
  void* ptrs[] = {b->f[0],   b->f[1], b->f0[0],    b->f0[1],    b->g[0],
                  b->g[1],   b->T[0], b->T[1],     b->hist,     b->psi,
                  b->wet,    b->staging, b->partial, b->bad, b->tiles,
                  b->insts,  b->counters, b->kds, b->kfs};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

// Tile list for tile height ty: instances in order, tiles row-major.
int build_tiles(ddcc_batch* b, int ty) {
  std::vector<BatchTile> tl;
  b->t0.assign(b->count, 0);
  b->t1.assign(b->count, 0);
  for (int i = 0; i < b->count; ++i) {
    b->t0[i] = (unsigned)tl.size();
    for (int y = 0; y < b->ny[i]; y += ty)
      for (int x = 0; x < b->nx[i]; x += 64) tl.push_back(BatchTile{i, x, y, 0});
    b->t1[i] = (unsigned)tl.size();
  }
  if (b->tiles) (void)hipFree(b->tiles);
  b->tiles = nullptr;
  BHIP(b, hipMalloc(&b->tiles, tl.size() * sizeof(BatchTile)), "hipMalloc tiles");
  BHIP(b, hipMemcpyAsync(b->tiles, tl.data(), tl.size() * sizeof(BatchTile),
                         hipMemcpyHostToDevice, b->stream),
       "copy tiles");
  BHIP(b, hipStreamSynchronize(b->stream), "sync");
  b->ntiles = (unsigned)tl.size();
  b->ty = ty;
  // persistent launch: as many workgroups as stay resident at once
  int per_cu = 0;
  switch (b->p.precision) {
    case DDCC_FP64:
      per_cu = batch_blocks_per_cu<double, double, double>(b->p.nphase, ty);
      break;
    case DDCC_FP16:
      per_cu = batch_blocks_per_cu<_Float16, float, float>(b->p.nphase, ty);
      break;
    case DDCC_BF16:
      per_cu = batch_blocks_per_cu<__bf16, float, float>(b->p.nphase, ty);
      break;
    default:
      per_cu = batch_blocks_per_cu<float, float, float>(b->p.nphase, ty);
  }
  b->blocks = (per_cu < 1 ? 1 : per_cu) * (b->cus < 1 ? 1 : b->cus);
  drop_graphs(b);
  return DDCC_OK;
}

template <class Pop, class S>
Bufs<Pop, S> batch_bufs(ddcc_batch* b, int mode) {
  Bufs<Pop, S> r{};
  const int a = b->cur, o = b->cur ^ 1;
  const int w = mode == MODE_INIT ? a : o;
  r.fA = static_cast<const Pop*>(b->f[a]);
  r.fB = static_cast<Pop*>(b->f[w]);
  r.f0A = b->f0[a];
  r.f0B = b->f0[w];
  r.gA = static_cast<const Pop*>(b->g[a]);
  r.gB = static_cast<Pop*>(b->g[w]);
  r.TA = static_cast<const S*>(b->T[a]);
  r.TB = static_cast<S*>(b->T[w]);
  r.hist = static_cast<S*>(b->hist);
  r.psi = static_cast<const S*>(b->psi);
  r.wet = static_cast<const S*>(b->wet);
  return r;
}

template <class Pop, class S, class R>
hipError_t batch_launch_as(ddcc_batch* b, const Coef<R>* k, int mode,
                           unsigned t0, unsigned nt, unsigned* counter,
                           const double* inC, const double* inU,
                           const double* inP, double* oC, double* oU,
                           double* oP) {
  Bufs<Pop, S> r = batch_bufs<Pop, S>(b, mode);
  if (mode == MODE_STEP && b->stream_stores) mode = MODE_STREAM;
  r.inC = inC;
  r.inU = inU;
  r.inP = inP;
  r.outC = oC;
  r.outU = oU;
  r.outP = oP;
  long long nb = b->blocks;
  if (nb > nt) nb = nt;
  if (nb < 1) nb = 1;
  return launch_2d_batch<Pop, S, R>(b->p.nphase, mode, b->kds, k, r,
                                    b->tiles + t0, b->insts, nt, counter,
                                    (int)nb, b->ty, b->stream);
}

// Zero *counter, then run `mode` over tiles [t0, t0 + nt).
hipError_t batch_launch(ddcc_batch* b, int mode, unsigned t0, unsigned nt,
                        unsigned* counter, const double* inC = nullptr,
                        const double* inU = nullptr, const double* inP = nullptr,
                        double* oC = nullptr, double* oU = nullptr,
                        double* oP = nullptr) {
  hipError_t e = launch_fill_u32(counter, 0u, 1, b->stream);
  if (e != hipSuccess) return e;
  switch (b->p.precision) {
    case DDCC_FP64:
      return batch_launch_as<double, double>(b, b->kds, mode, t0, nt, counter,
                                             inC, inU, inP, oC, oU, oP);
    case DDCC_FP16:
      return batch_launch_as<_Float16, float>(b, b->kfs, mode, t0, nt, counter,
                                              inC, inU, inP, oC, oU, oP);
    case DDCC_BF16:
      return batch_launch_as<__bf16, float>(b, b->kfs, mode, t0, nt, counter,
                                            inC, inU, inP, oC, oU, oP);
    default:
      return batch_launch_as<float, float>(b, b->kfs, mode, t0, nt, counter,
                                           inC, inU, inP, oC, oU, oP);
  }
}

// Copies instance i's planes [0, planes) between a host array laid out
// [plane][n_i] and batch-layout device memory [plane][ntot] at off_i.
int copy_planes(ddcc_batch* b, int i, void* dev, const void* host, int planes,
                size_t esz, hipMemcpyKind kind) {
  for (int q = 0; q < planes; ++q) {
    char* d = static_cast<char*>(dev) + ((size_t)q * b->ntot + b->off[i]) * esz;
    const char* h = static_cast<const char*>(host) + (size_t)q * b->n[i] * esz;
    hipError_t e = kind == hipMemcpyHostToDevice
                       ? hipMemcpyAsync(d, h, b->n[i] * esz, kind, b->stream)
                       : hipMemcpyAsync(const_cast<char*>(h), d, b->n[i] * esz,
                                        kind, b->stream);
    if (e != hipSuccess) return bhip(b, e, "plane copy");
  }
  return DDCC_OK;
}

int batch_check(ddcc_batch* b, int i) {
  if (!b) return DDCC_E_INVAL;
  if (i < 0 || i >= b->count) return bfail(b, DDCC_E_INVAL, "instance out of range");
  return DDCC_OK;
}

// One step of every instance; graph replays use counters [0, graph_steps).
int batch_step_direct(ddcc_batch* b) {
  hipError_t e = batch_launch(b, MODE_STEP, 0, b->ntiles, b->counters);
  if (e != hipSuccess) return bhip(b, e, "batch step kernel");
  b->cur ^= 1;
  ++b->t;
  return DDCC_OK;
}

int batch_capture(ddcc_batch* b) {
  const int par = b->cur;
  hipGraph_t graph = nullptr;
  BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal),
       "begin capture");
  hipError_t e = launch_fill_u32(b->counters, 0u, b->graph_steps, b->stream);
  for (int s = 0; s < b->graph_steps && e == hipSuccess; ++s) {
    switch (b->p.precision) {
      case DDCC_FP64:
        e = batch_launch_as<double, double>(b, b->kds, MODE_STEP, 0, b->ntiles,
                                            b->counters + s, nullptr, nullptr,
                                            nullptr, nullptr, nullptr, nullptr);
        break;
      case DDCC_FP16:
        e = batch_launch_as<_Float16, float>(b, b->kfs, MODE_STEP, 0, b->ntiles,
                                             b->counters + s, nullptr, nullptr,
                                             nullptr, nullptr, nullptr, nullptr);
        break;
      case DDCC_BF16:
        e = batch_launch_as<__bf16, float>(b, b->kfs, MODE_STEP, 0, b->ntiles,
                                           b->counters + s, nullptr, nullptr,
                                           nullptr, nullptr, nullptr, nullptr);
        break;
      default:
        e = batch_launch_as<float, float>(b, b->kfs, MODE_STEP, 0, b->ntiles,
                                          b->counters + s, nullptr, nullptr,
                                          nullptr, nullptr, nullptr, nullptr);
    }
    b->cur ^= 1;
  }
  b->cur = par;
  hipError_t e2 = hipStreamEndCapture(b->stream, &graph);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return bhip(b, e != hipSuccess ? e : e2, "graph capture");
  }
  e = hipGraphInstantiate(&b->gexec[par], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    b->gexec[par] = nullptr;
    return bhip(b, e, "graph instantiate");
  }
  return DDCC_OK;
}

}  // namespace

extern "C" {

int ddcc_batch_create(const ddcc_params* p, int count, const int* nx,
                      const int* ny, void* stream, ddcc_batch** out) {
  if (!out) return DDCC_E_INVAL;
  *out = nullptr;
  if (!p || !nx || !ny || count < 1) return DDCC_E_INVAL;
  if (p->dim != 2) return DDCC_E_UNSUPPORTED;
  long long ntot = 0;
  for (int i = 0; i < count; ++i) {
    if (nx[i] < 1 || ny[i] < 1) return DDCC_E_INVAL;
    ntot += (long long)nx[i] * ny[i];
  }
  if (ntot > (1LL << 29)) return DDCC_E_INVAL;
  ddcc_params q = *p;
  q.nx = nx[0];
  q.ny = ny[0];
  q.nz = 1;
  std::string msg;
  int rc = validate(&q, msg);
  if (rc != DDCC_OK) return rc;
  ddcc_batch* b = new (std::nothrow) ddcc_batch();
  if (!b) return DDCC_E_NOMEM;
  b->p = q;
  b->count = count;
  b->nx.assign(nx, nx + count);
  b->ny.assign(ny, ny + count);
  for (int i = 0; i < count; ++i) {
    b->n.push_back((long long)nx[i] * ny[i]);
    b->off.push_back(b->ntot);
    b->ntot += b->n.back();
  }
  b->geom_ok.assign(count, 0);
  b->fields_ok.assign(count, 0);
  b->esz = q.precision == DDCC_FP64 ? 8 : 4;
  b->pesz = q.precision == DDCC_FP64 ? 8 : (q.precision == DDCC_FP32 ? 4 : 2);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount,
                            dev) != hipSuccess) {
    delete b;
    return DDCC_E_HIP;
  }
  // A captured graph cannot use the legacy default stream.
  if (stream) {
    b->stream = static_cast<hipStream_t>(stream);
  } else {
    if (hipStreamCreate(&b->stream) != hipSuccess) {
      delete b;
      return DDCC_E_HIP;
    }
    b->own_stream = true;
  }
  // kernel constants: plane stride ntot; the box sizes come per instance
  ddcc_params qs = q;
  fill_coef<double>(qs, b->ntot, b->kd);
  fill_coef<float>(qs, b->ntot, b->kf);
  const int N = q.nphase;
  const size_t nt = (size_t)b->ntot;
  hipError_t e = hipSuccess;
  for (int a = 0; a < 2 && e == hipSuccess; ++a) {
    e = hipMalloc(&b->f[a], (size_t)N * (kBatchQ - 1) * nt * b->pesz);
    if (e == hipSuccess) e = hipMalloc(&b->f0[a], (size_t)N * nt * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&b->g[a], (size_t)kBatchQ * nt * b->pesz);
    if (e == hipSuccess) e = hipMalloc(&b->T[a], nt * b->esz);
  }
  if (e == hipSuccess) e = hipMalloc(&b->hist, (size_t)nhist_of(N) * nt * b->esz);
  b->stream_stores =
      step_bytes((size_t)N * (kBatchQ - 1) * nt * b->pesz +
                     (size_t)N * nt * sizeof(double) + (size_t)kBatchQ * nt * b->pesz,
                 nt * b->esz, (size_t)nhist_of(N) * nt * b->esz, 0) > kCacheBytes;
  if (e == hipSuccess) e = hipMalloc(&b->psi, nt * b->esz);
  if (e == hipSuccess) e = hipMalloc(&b->wet, (size_t)(N - 1) * nt * b->esz);
  if (e == hipSuccess)
    e = hipMalloc(&b->staging, (size_t)(N + 3) * nt * sizeof(double));
  long long mb = (ntot + 255) / 256;
  b->mass_blocks = (int)(mb > 1024 ? 1024 : mb);
  if (e == hipSuccess)
    e = hipMalloc(&b->partial, (size_t)b->mass_blocks * N * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&b->bad, (size_t)b->mass_blocks * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&b->counters, kMaxGraphSteps * sizeof(unsigned));
  if (e == hipSuccess) {
    std::vector<BatchInst> ins(count);
    for (int i = 0; i < count; ++i) ins[i] = BatchInst{nx[i], ny[i], b->n[i], b->off[i]};
    e = hipMalloc(&b->insts, count * sizeof(BatchInst));
    if (e == hipSuccess)
      e = hipMemcpy(b->insts, ins.data(), count * sizeof(BatchInst),
                    hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) {
    const std::vector<Coef<double>> vd(count, b->kd);
    const std::vector<Coef<float>> vf(count, b->kf);
    e = hipMalloc(&b->kds, count * sizeof(Coef<double>));
    if (e == hipSuccess) e = hipMalloc(&b->kfs, count * sizeof(Coef<float>));
    if (e == hipSuccess)
      e = hipMemcpy(b->kds, vd.data(), count * sizeof(Coef<double>),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(b->kfs, vf.data(), count * sizeof(Coef<float>),
                    hipMemcpyHostToDevice);
  }
  if (e != hipSuccess || build_tiles(b, 8) != DDCC_OK) {
    batch_release(b);
    delete b;
    return e == hipErrorOutOfMemory ? DDCC_E_NOMEM : DDCC_E_HIP;
  }
  *out = b;
  return DDCC_OK;
}

int ddcc_batch_set_params(ddcc_batch* b, int i, const ddcc_params* p) {
  int rc = batch_check(b, i);
  if (rc) return rc;
  if (!p) return bfail(b, DDCC_E_INVAL, "params is NULL");
  if (p->dim != b->p.dim || p->nphase != b->p.nphase ||
      p->lattice_f != b->p.lattice_f || p->lattice_g != b->p.lattice_g ||
      p->precision != b->p.precision)
    return bfail(b, DDCC_E_INVAL,
                 "dim, nphase, lattices and precision must be the batch's");
  ddcc_params q = *p;
  q.nx = b->nx[i];
  q.ny = b->ny[i];
  q.nz = 1;
  std::string msg;
  rc = validate(&q, msg);
  if (rc != DDCC_OK) return bfail(b, rc, msg);
  Coef<double> kd;
  Coef<float> kf;
  fill_coef<double>(q, b->ntot, kd);
  fill_coef<float>(q, b->ntot, kf);
  // the tables are read by kernels on the batch stream
  if (hipStreamSynchronize(b->stream) != hipSuccess ||
      hipMemcpy(b->kds + i, &kd, sizeof(kd), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(b->kfs + i, &kf, sizeof(kf), hipMemcpyHostToDevice) !=
          hipSuccess)
    return bfail(b, DDCC_E_HIP, "copy parameters");
  return DDCC_OK;
}

int ddcc_batch_init_geometry(ddcc_batch* b, int i, const double* psi,
                             const double* ct) {
  int rc = batch_check(b, i);
  if (rc) return rc;
  if (!psi) return bfail(b, DDCC_E_INVAL, "psi is NULL");
  const size_t n = (size_t)b->n[i];
  const int N = b->p.nphase;
  for (size_t k = 0; k < n; ++k)
    if (!(psi[k] >= 0.0 && psi[k] <= 1.0))
      return bfail(b, DDCC_E_INVAL, "psi outside [0, 1]");
  if (ct)
    for (size_t k = 0; k < (size_t)(N - 1) * n; ++k)
      if (!(ct[k] >= -1.0 && ct[k] <= 1.0))
        return bfail(b, DDCC_E_INVAL, "cos theta outside [-1, 1]");
  // psi and the wetting weights of the instance, computed on the device
  const size_t nc = ct ? (size_t)(N - 1) * n : 0;
  double* d = nullptr;
  BHIP(b, hipMalloc(&d, (n + nc) * sizeof(double)), "hipMalloc geometry");
  hipError_t e = hipMemcpyAsync(d, psi, n * sizeof(double),
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess && nc)
    e = hipMemcpyAsync(d + n, ct, nc * sizeof(double), hipMemcpyHostToDevice,
                       b->stream);
  if (e == hipSuccess)
    e = b->p.precision == DDCC_FP64
            ? launch_wet_field<double>(d, nc ? d + n : nullptr, 1, N - 1,
                                       b->nx[i], b->ny[i], 1,
                                       static_cast<double*>(b->psi),
                                       static_cast<double*>(b->wet), b->ntot,
                                       b->off[i], b->stream)
            : launch_wet_field<float>(d, nc ? d + n : nullptr, 1, N - 1,
                                      b->nx[i], b->ny[i], 1,
                                      static_cast<float*>(b->psi),
                                      static_cast<float*>(b->wet), b->ntot,
                                      b->off[i], b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return bhip(b, e, "batch geometry");
  b->geom_ok[i] = 1;
  b->fields_ok[i] = 0;
  return DDCC_OK;
}

int ddcc_batch_init_fields(ddcc_batch* b, int i, const double* C,
                           const double* u, const double* P) {
  int rc = batch_check(b, i);
  if (rc) return rc;
  if (!b->geom_ok[i]) return bfail(b, DDCC_E_STATE, "init_geometry first");
  if (!C) return bfail(b, DDCC_E_INVAL, "C is NULL");
  const int N = b->p.nphase;
  const size_t n = (size_t)b->n[i];
  if (!all_finite(C, N * n) || (u && !all_finite(u, 2 * n)) ||
      (P && !all_finite(P, n)))
    return bfail(b, DDCC_E_INVAL, "non-finite initial field");
  double* sC = b->staging;
  double* sU = sC + (size_t)N * b->ntot;
  double* sP = sU + 2 * (size_t)b->ntot;
  rc = copy_planes(b, i, sC, C, N, sizeof(double), hipMemcpyHostToDevice);
  if (!rc && u) rc = copy_planes(b, i, sU, u, 2, sizeof(double), hipMemcpyHostToDevice);
  if (!rc && P) rc = copy_planes(b, i, sP, P, 1, sizeof(double), hipMemcpyHostToDevice);
  if (rc) return rc;
  // initialisation writes the populations of the current level in place
  hipError_t e = batch_launch(b, MODE_INIT, b->t0[i], b->t1[i] - b->t0[i],
                              b->counters, sC, u ? sU : nullptr,
                              P ? sP : nullptr);
  if (e != hipSuccess) return bhip(b, e, "batch init kernel");
  BHIP(b, hipStreamSynchronize(b->stream), "sync");
  b->fields_ok[i] = 1;
  return DDCC_OK;
}

int ddcc_batch_step(ddcc_batch* b, int64_t nsteps) {
  if (!b) return DDCC_E_INVAL;
  if (nsteps < 0) return bfail(b, DDCC_E_INVAL, "nsteps < 0");
  for (int i = 0; i < b->count; ++i)
    if (!b->fields_ok[i])
      return bfail(b, DDCC_E_STATE, "every instance needs init_fields first");
  int64_t left = nsteps;
  if (b->graph_steps > 0) {
    while (left >= b->graph_steps) {
      if (!b->gexec[b->cur]) {
        int rc = batch_capture(b);
        if (rc) return rc;
      }
      BHIP(b, hipGraphLaunch(b->gexec[b->cur], b->stream), "graph launch");
      // an even number of steps leaves the level parity unchanged
      b->t += b->graph_steps;
      left -= b->graph_steps;
    }
  }
  for (; left > 0; --left) {
    int rc = batch_step_direct(b);
    if (rc) return rc;
  }
  return DDCC_OK;
}

int ddcc_batch_read_moments(ddcc_batch* b, int i, double* C, double* u,
                            double* P) {
  int rc = batch_check(b, i);
  if (rc) return rc;
  if (!b->fields_ok[i]) return bfail(b, DDCC_E_STATE, "init_fields first");
  const int N = b->p.nphase;
  double* sC = b->staging;
  double* sU = sC + (size_t)N * b->ntot;
  double* sP = sU + 2 * (size_t)b->ntot;
  hipError_t e = batch_launch(b, MODE_MOMENTS, b->t0[i], b->t1[i] - b->t0[i],
                              b->counters, nullptr, nullptr, nullptr, sC, sU,
                              sP);
  if (e != hipSuccess) return bhip(b, e, "batch moments kernel");
  if (C) rc = copy_planes(b, i, sC, C, N, sizeof(double), hipMemcpyDeviceToHost);
  if (!rc && u) rc = copy_planes(b, i, sU, u, 2, sizeof(double), hipMemcpyDeviceToHost);
  if (!rc && P) rc = copy_planes(b, i, sP, P, 1, sizeof(double), hipMemcpyDeviceToHost);
  if (rc) return rc;
  BHIP(b, hipStreamSynchronize(b->stream), "sync");
  return DDCC_OK;
}

int ddcc_batch_mass(ddcc_batch* b, int i, double* mass) {
  int rc = batch_check(b, i);
  if (rc) return rc;
  if (!mass) return bfail(b, DDCC_E_INVAL, "mass is NULL");
  if (!b->fields_ok[i]) return bfail(b, DDCC_E_STATE, "init_fields first");
  const int N = b->p.nphase;
  const long long o = b->off[i];
  const double* f0 = b->f0[b->cur] + o;
  hipError_t e;
  switch (b->p.precision) {
    case DDCC_FP64:
      e = launch_mass(f0, static_cast<const double*>(b->f[b->cur]) + o, N,
                      kBatchQ, b->n[i], b->ntot, b->partial, b->bad,
                      b->mass_blocks, b->stream);
      break;
    case DDCC_FP16:
      e = launch_mass(f0, static_cast<const _Float16*>(b->f[b->cur]) + o, N,
                      kBatchQ, b->n[i], b->ntot, b->partial, b->bad,
                      b->mass_blocks, b->stream);
      break;
    case DDCC_BF16:
      e = launch_mass(f0, static_cast<const __bf16*>(b->f[b->cur]) + o, N,
                      kBatchQ, b->n[i], b->ntot, b->partial, b->bad,
                      b->mass_blocks, b->stream);
      break;
    default:
      e = launch_mass(f0, static_cast<const float*>(b->f[b->cur]) + o, N,
                      kBatchQ, b->n[i], b->ntot, b->partial, b->bad,
                      b->mass_blocks, b->stream);
  }
  if (e != hipSuccess) return bhip(b, e, "mass kernel");
  std::vector<double> part((size_t)b->mass_blocks * N);
  std::vector<int> bad(b->mass_blocks);
  BHIP(b, hipMemcpyAsync(part.data(), b->partial, part.size() * sizeof(double),
                         hipMemcpyDeviceToHost, b->stream),
       "copy partials");
  BHIP(b, hipMemcpyAsync(bad.data(), b->bad, bad.size() * sizeof(int),
                         hipMemcpyDeviceToHost, b->stream),
       "copy flags");
  BHIP(b, hipStreamSynchronize(b->stream), "sync");
  for (int k = 0; k < N; ++k) {
    double s = 0.0;
    for (int q = 0; q < b->mass_blocks; ++q) s += part[(size_t)q * N + k];
    mass[k] = s;
  }
  for (int q = 0; q < b->mass_blocks; ++q)
    if (bad[q]) return bfail(b, DDCC_E_NONFINITE, "non-finite population");
  return DDCC_OK;
}

int ddcc_batch_set_tile(ddcc_batch* b, int ty) {
  if (!b) return DDCC_E_INVAL;
  if (ty != 4 && ty != 8 && ty != 16)
    return bfail(b, DDCC_E_INVAL, "batch tile height must be 4, 8 or 16");
  return build_tiles(b, ty);
}

int ddcc_batch_set_graph(ddcc_batch* b, int steps_per_graph) {
  if (!b) return DDCC_E_INVAL;
  if (steps_per_graph < 0 || steps_per_graph > kMaxGraphSteps ||
      steps_per_graph % 2 != 0)
    return bfail(b, DDCC_E_INVAL,
                 "steps per graph must be even and in [0, 1024]");
  drop_graphs(b);
  b->graph_steps = steps_per_graph;
  return DDCC_OK;
}

int ddcc_batch_autotune(ddcc_batch* b, int steps, int* ty_out) {
  if (!b) return DDCC_E_INVAL;
  if (steps < 1) return bfail(b, DDCC_E_INVAL, "steps < 1");
  for (int i = 0; i < b->count; ++i)
    if (!b->fields_ok[i])
      return bfail(b, DDCC_E_STATE, "every instance needs init_fields first");
  // The trial steps change the state: keep a copy of the current level.
  const int N = b->p.nphase;
  const size_t nt = (size_t)b->ntot;
  const size_t sizes[5] = {(size_t)N * (kBatchQ - 1) * nt * b->pesz,
                           (size_t)N * nt * sizeof(double),
                           (size_t)kBatchQ * nt * b->pesz, nt * b->esz,
                           (size_t)nhist_of(N) * nt * b->esz};
  const int cur0 = b->cur;
  void* src[5] = {b->f[cur0], b->f0[cur0], b->g[cur0], b->T[cur0], b->hist};
  void* keep[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  hipError_t e = hipSuccess;
  for (int q = 0; q < 5 && e == hipSuccess; ++q) {
    e = hipMalloc(&keep[q], sizes[q]);
    if (e == hipSuccess)
      e = hipMemcpyAsync(keep[q], src[q], sizes[q], hipMemcpyDeviceToDevice,
                         b->stream);
  }
  const int cands[3] = {4, 8, 16};
  float best_ms = 0;
  int best = b->ty;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  const int64_t tsave = b->t;
  for (int c = 0; c < 3 && e == hipSuccess; ++c) {
    if (build_tiles(b, cands[c]) != DDCC_OK) {
      e = hipErrorUnknown;
      break;
    }
    for (int w = 0; w < 2 && e == hipSuccess; ++w)
      if (batch_step_direct(b) != DDCC_OK) e = hipErrorUnknown;
    if (e == hipSuccess) e = hipEventRecord(t0, b->stream);
    for (int s = 0; s < steps && e == hipSuccess; ++s)
      if (batch_step_direct(b) != DDCC_OK) e = hipErrorUnknown;
    if (e == hipSuccess) e = hipEventRecord(t1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (e == hipSuccess && (c == 0 || ms < best_ms)) {
      best_ms = ms;
      best = cands[c];
    }
  }
  // restore the level the trials started from
  b->cur = cur0;
  b->t = tsave;
  for (int q = 0; q < 5; ++q)
    if (keep[q]) {
      if (e == hipSuccess)
        e = hipMemcpyAsync(src[q], keep[q], sizes[q], hipMemcpyDeviceToDevice,
                           b->stream);
    }
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  for (int q = 0; q < 5; ++q)
    if (keep[q]) (void)hipFree(keep[q]);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (e != hipSuccess) return bhip(b, e, "autotune");
  int rc = build_tiles(b, best);
  if (rc) return rc;
  if (ty_out) *ty_out = best;
  return DDCC_OK;
}

int ddcc_batch_sync(ddcc_batch* b) {
  if (!b) return DDCC_E_INVAL;
  BHIP(b, hipStreamSynchronize(b->stream), "sync");
  return DDCC_OK;
}

int64_t ddcc_batch_time(const ddcc_batch* b) { return b ? b->t : -1; }

const char* ddcc_batch_last_error(const ddcc_batch* b) {
  return b ? b->err.c_str() : "NULL batch";
}

void ddcc_batch_destroy(ddcc_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  batch_release(b);
  delete b;
}

}  // extern "C"
