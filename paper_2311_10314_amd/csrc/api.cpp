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
#include "kernels.hpp"
#include "lattice.hpp"

using namespace ddcc;

struct ddcc_ctx {
  ddcc_params p{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  long long n = 0;
  int Qf = 0, Qg = 0, nhist = 0, nT = 0;
  size_t esz = 8;
  void* f[2] = {nullptr, nullptr};
  double* f0[2] = {nullptr, nullptr};  // rest populations, float64
  void* g[2] = {nullptr, nullptr};
  void* T[2] = {nullptr, nullptr};
  void* hist = nullptr;
  void* psi = nullptr;
  void* ct = nullptr;
  double* staging = nullptr;  // (N + dim + 1) * n float64, lazily
  double* partial = nullptr;
  int* bad = nullptr;
  int mass_blocks = 0;
  int cur = 0;
  bool geom_ok = false, fields_ok = false;
  int64_t t = 0;
  int tile_x = 64, tile_y = 8;
  std::string err;
  Coef<double> kd{};
  Coef<float> kf{};
};

namespace {

const char* kVersion = "ddcc 0.1 (gfx950)";

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
  if ((long long)p->nx * p->ny * p->nz > (1LL << 31)) {
    msg = "grid larger than 2^31 nodes";
    return DDCC_E_INVAL;
  }
  if (p->nphase < 2 || p->nphase > DDCC_MAX_PHASES) {
    msg = "nphase must be in [2, 4]";
    return DDCC_E_INVAL;
  }
  if (p->precision != DDCC_FP64 && p->precision != DDCC_FP32) {
    msg = "precision must be DDCC_FP64 or DDCC_FP32";
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

template <class S>
Bufs<S> bufs(ddcc_ctx* c, int mode) {
  Bufs<S> b{};
  const int a = c->cur, o = c->cur ^ 1;
  b.fA = static_cast<const S*>(c->f[a]);
  b.f0A = c->f0[a];
  b.gA = static_cast<const S*>(c->g[a]);
  b.TA = static_cast<const S*>(c->T[a]);
  if (mode == MODE_INIT) {
    b.fB = static_cast<S*>(c->f[a]);
    b.f0B = c->f0[a];
    b.gB = static_cast<S*>(c->g[a]);
    b.TB = static_cast<S*>(c->T[a]);
  } else {
    b.fB = static_cast<S*>(c->f[o]);
    b.f0B = c->f0[o];
    b.gB = static_cast<S*>(c->g[o]);
    b.TB = static_cast<S*>(c->T[o]);
  }
  b.hist = static_cast<S*>(c->hist);
  b.psi = static_cast<const S*>(c->psi);
  b.ct = static_cast<const S*>(c->ct);
  return b;
}

hipError_t launch(ddcc_ctx* c, int mode, const double* inC, const double* inU,
                  const double* inP, double* oC, double* oU, double* oP) {
  if (c->p.precision == DDCC_FP64) {
    Bufs<double> b = bufs<double>(c, mode);
    b.inC = inC;
    b.inU = inU;
    b.inP = inP;
    b.outC = oC;
    b.outU = oU;
    b.outP = oP;
    if (c->p.dim == 2)
      return launch_2d<double, double>(c->p.nphase, mode, c->kd, c->kd, b,
                                       c->tile_y, c->stream);
    return launch_3d<double, double>(c->p.nphase, mode, c->kd, c->kd, b,
                                     c->tile_x, c->tile_y, c->stream);
  }
  Bufs<float> b = bufs<float>(c, mode);
  b.inC = inC;
  b.inU = inU;
  b.inP = inP;
  b.outC = oC;
  b.outU = oU;
  b.outP = oP;
  if (c->p.dim == 2)
    return launch_2d<float, float>(c->p.nphase, mode, c->kd, c->kf, b,
                                   c->tile_y, c->stream);
  return launch_3d<float, float>(c->p.nphase, mode, c->kd, c->kf, b,
                                 c->tile_x, c->tile_y, c->stream);
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

template <class S>
int upload_as(ddcc_ctx* c, const double* src, void* dst, size_t count) {
  std::vector<S> tmp(count);
  for (size_t i = 0; i < count; ++i) tmp[i] = S(src[i]);
  HIPCHK(c, hipMemcpyAsync(dst, tmp.data(), count * sizeof(S),
                           hipMemcpyHostToDevice, c->stream),
         "hipMemcpyAsync");
  HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return DDCC_OK;
}

int upload(ddcc_ctx* c, const double* src, void* dst, size_t count) {
  return c->p.precision == DDCC_FP64 ? upload_as<double>(c, src, dst, count)
                                     : upload_as<float>(c, src, dst, count);
}

void release(ddcc_ctx* c) {
  void* ptrs[] = {c->f[0],  c->f[1],   c->f0[0],    c->f0[1], c->g[0],
                  c->g[1],  c->T[0],   c->T[1],     c->hist,  c->psi,
                  c->ct,    c->staging, c->partial, c->bad};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
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
}

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
  c->nhist = p->nphase * d + d * (d + 1) / 2 + 1;
  c->nT = d * (d - 1) / 2;
  c->esz = p->precision == DDCC_FP64 ? 8 : 4;
  c->tile_y = d == 2 ? 8 : 4;
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
  const size_t sf = (size_t)p->nphase * c->Qf * n * c->esz;
  const size_t sg = (size_t)c->Qg * n * c->esz;
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
  if (e == hipSuccess) e = hipMalloc(&c->psi, n * c->esz);
  if (e == hipSuccess)
    e = hipMalloc(&c->ct, (size_t)(p->nphase - 1) * n * c->esz);
  long long mb = (c->n + 255) / 256;
  c->mass_blocks = (int)(mb > 1024 ? 1024 : mb);
  if (e == hipSuccess)
    e = hipMalloc(&c->partial,
                  (size_t)c->mass_blocks * p->nphase * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&c->bad, (size_t)c->mass_blocks * sizeof(int));
  if (e != hipSuccess) {
    release(c);
    delete c;
    return e == hipErrorOutOfMemory ? DDCC_E_NOMEM : DDCC_E_HIP;
  }
  if (p->dim == 3) {
    // The 3D kernels are built per (phase, flow) lattice pair; the host
    // checks the pair here so that create fails early when it is absent.
    if (!(p->lattice_f == DDCC_D3Q15 && p->lattice_g == DDCC_D3Q19) ||
        p->nphase > 3 || !have_3d()) {
      release(c);
      delete c;
      return DDCC_E_UNSUPPORTED;
    }
  }
  *out = c;
  return DDCC_OK;
}

int ddcc_init_geometry(ddcc_ctx* c, const double* psi, const double* ct) {
  if (!c) return DDCC_E_INVAL;
  if (!psi) return fail(c, DDCC_E_INVAL, "psi is NULL");
  const size_t n = (size_t)c->n;
  for (size_t i = 0; i < n; ++i)
    if (!(psi[i] >= 0.0 && psi[i] <= 1.0))
      return fail(c, DDCC_E_INVAL, "psi must be finite and in [0, 1]");
  const size_t nct = (size_t)(c->p.nphase - 1) * n;
  std::vector<double> zeros;
  if (ct) {
    for (size_t i = 0; i < nct; ++i)
      if (!(ct[i] >= -1.0 && ct[i] <= 1.0))
        return fail(c, DDCC_E_INVAL, "cos_theta must be finite and in [-1, 1]");
  } else {
    zeros.assign(nct, 0.0);
    ct = zeros.data();
  }
  int rc = upload(c, psi, c->psi, n);
  if (rc) return rc;
  rc = upload(c, ct, c->ct, nct);
  if (rc) return rc;
  c->geom_ok = true;
  c->fields_ok = false;
  return DDCC_OK;
}

int ddcc_init_geometry_dev(ddcc_ctx* c, const double* psi, const double* ct) {
  if (!c) return DDCC_E_INVAL;
  if (!psi) return fail(c, DDCC_E_INVAL, "psi is NULL");
  const long long n = c->n;
  const long long nct = (long long)(c->p.nphase - 1) * n;
  hipError_t e;
  if (c->p.precision == DDCC_FP64) {
    e = launch_convert<double>(psi, static_cast<double*>(c->psi), n, c->stream);
    if (e == hipSuccess) {
      if (ct)
        e = launch_convert<double>(ct, static_cast<double*>(c->ct), nct,
                                   c->stream);
      else
        e = hipMemsetAsync(c->ct, 0, nct * sizeof(double), c->stream);
    }
  } else {
    e = launch_convert<float>(psi, static_cast<float*>(c->psi), n, c->stream);
    if (e == hipSuccess) {
      if (ct)
        e = launch_convert<float>(ct, static_cast<float*>(c->ct), nct,
                                  c->stream);
      else
        e = hipMemsetAsync(c->ct, 0, nct * sizeof(float), c->stream);
    }
  }
  if (e != hipSuccess) return hip_fail(c, e, "init_geometry_dev");
  c->geom_ok = true;
  c->fields_ok = false;
  return DDCC_OK;
}

static int init_fields_common(ddcc_ctx* c, const double* C, const double* u,
                              const double* P) {
  hipError_t e = launch(c, MODE_INIT, C, u, P, nullptr, nullptr, nullptr);
  if (e != hipSuccess) return hip_fail(c, e, "init kernel");
  c->fields_ok = true;
  c->t = 0;
  return DDCC_OK;
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
  hipError_t e =
      c->p.precision == DDCC_FP64
          ? launch_mass<double>(c->f0[c->cur],
                                static_cast<const double*>(c->f[c->cur]), N,
                                c->Qf, c->n, c->partial, c->bad,
                                c->mass_blocks, c->stream)
          : launch_mass<float>(c->f0[c->cur],
                               static_cast<const float*>(c->f[c->cur]), N,
                               c->Qf, c->n, c->partial, c->bad, c->mass_blocks,
                               c->stream);
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

int64_t ddcc_time(const ddcc_ctx* c) { return c ? c->t : -1; }

int ddcc_save(ddcc_ctx* c, void* buf, size_t* bytes) {
  if (!c || !bytes) return fail(c, DDCC_E_INVAL, "NULL argument");
  if (!c->fields_ok) return fail(c, DDCC_E_STATE, "init_fields first");
  const size_t n = (size_t)c->n;
  const size_t sf = (size_t)c->p.nphase * c->Qf * n * c->esz;
  const size_t sg = (size_t)c->Qg * n * c->esz;
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
  std::memcpy(h.magic, "DDCCSAV2", 8);
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
  const size_t sf = (size_t)c->p.nphase * c->Qf * n * c->esz;
  const size_t sg = (size_t)c->Qg * n * c->esz;
  const size_t sh = (size_t)c->nhist * n * c->esz;
  const size_t sT = (size_t)c->nT * n * c->esz;
  const size_t s0 = (size_t)c->p.nphase * n * sizeof(double);
  const size_t need = sizeof(SaveHeader) + sf + s0 + sg + sh + sT;
  if (bytes < need) return fail(c, DDCC_E_INVAL, "checkpoint too small");
  SaveHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, "DDCCSAV2", 8) != 0 || h.dim != c->p.dim ||
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
  return DDCC_OK;
}

int ddcc_sync(ddcc_ctx* c) {
  if (!c) return DDCC_E_INVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
  return DDCC_OK;
}

int ddcc_set_tile(ddcc_ctx* c, int tx, int ty) {
  if (!c) return DDCC_E_INVAL;
  if (c->p.dim == 2) {
    if (tx != 0 && tx != 64)
      return fail(c, DDCC_E_INVAL, "2D tiles are 64 nodes wide");
    if (ty != 0 && ty != 2 && ty != 4 && ty != 8)
      return fail(c, DDCC_E_INVAL, "2D tile height must be 2, 4 or 8");
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
