/* Host-side check of the C ABI for the sanitizer build (AddressSanitizer
 * and UndefinedBehaviorSanitizer on the library's host code): every
 * validation path of include/ddcc.h without a GPU, and with --gpu one small
 * run through each entry point family on the current device. Prints "ok"
 * and returns 0 when every call returned what the header promises. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../include/ddcc.h"

static int failures = 0;

#define EXPECT(cond)                                                \
  do {                                                              \
    if (!(cond)) {                                                  \
      fprintf(stderr, "host_check: %s:%d: %s\n", __FILE__, __LINE__, \
              #cond);                                               \
      ++failures;                                                   \
    }                                                               \
  } while (0)

typedef void (*mutate_fn)(ddcc_params*);
static void m_dim(ddcc_params* p) { p->dim = 4; }
static void m_nx(ddcc_params* p) { p->nx = 0; }
static void m_nz(ddcc_params* p) { p->nz = 3; }
static void m_n1(ddcc_params* p) { p->nphase = 1; }
static void m_n5(ddcc_params* p) { p->nphase = 5; }
static void m_prec(ddcc_params* p) { p->precision = 7; }
static void m_d0(ddcc_params* p) { p->d0 = 1.0; }
static void m_d0n(ddcc_params* p) { p->d0 = NAN; }
static void m_eps(ddcc_params* p) { p->eps = 0.0; }
static void m_m0(ddcc_params* p) { p->m0 = -1.0; }
static void m_psimin(ddcc_params* p) { p->psi_min = 0.0; }
static void m_lam(ddcc_params* p) { p->lam = -1.0; }
static void m_latf(ddcc_params* p) { p->lattice_f = 3; }
static void m_sig(ddcc_params* p) { p->sigma[0][1] = 0.002; }
static void m_sigd(ddcc_params* p) { p->sigma[1][1] = 0.001; }
static void m_rate(ddcc_params* p) { p->s_f[2] = 2.0; }
static void m_rho(ddcc_params* p) { p->rho[0] = 0.0; }
static void m_nu(ddcc_params* p) { p->nu[1] = -0.1; }

static double frand(unsigned* s) {
  *s = *s * 1664525u + 1013904223u;
  return (*s >> 8) * (1.0 / 16777216.0);
}

static void check_validation(void) {
  ddcc_params p;
  EXPECT(ddcc_default_params(&p) == DDCC_OK);
  EXPECT(ddcc_default_params(NULL) == DDCC_E_INVAL);
  EXPECT(ddcc_version() && strlen(ddcc_version()) > 0);
  const mutate_fn bad[] = {m_dim, m_nx,     m_nz,  m_n1,   m_n5,   m_prec,
                           m_d0,  m_d0n,    m_eps, m_m0,   m_psimin, m_lam,
                           m_latf, m_sig,   m_sigd, m_rate, m_rho, m_nu};
  for (size_t i = 0; i < sizeof(bad) / sizeof(bad[0]); ++i) {
    ddcc_params q;
    ddcc_default_params(&q);
    bad[i](&q);
    ddcc_ctx* c = (ddcc_ctx*)&q; /* must be overwritten with NULL */
    EXPECT(ddcc_create(&q, NULL, &c) == DDCC_E_INVAL);
    EXPECT(c == NULL);
  }
  EXPECT(ddcc_create(NULL, NULL, NULL) == DDCC_E_INVAL);
  /* NULL handles */
  ddcc_destroy(NULL);
  EXPECT(ddcc_last_error(NULL) != NULL);
  EXPECT(ddcc_step(NULL, 1) == DDCC_E_INVAL);
  EXPECT(ddcc_time(NULL) == -1);
  EXPECT(ddcc_mass(NULL, NULL) == DDCC_E_INVAL);
  EXPECT(ddcc_mass_noalloc(NULL, NULL, NULL) == DDCC_E_INVAL);
  EXPECT(ddcc_sync(NULL) == DDCC_E_INVAL);
  EXPECT(ddcc_init_fields(NULL, NULL, NULL, NULL) == DDCC_E_INVAL);
  EXPECT(ddcc_init_geometry(NULL, NULL, NULL) == DDCC_E_INVAL);
  EXPECT(ddcc_read_moments(NULL, NULL, NULL, NULL) == DDCC_E_INVAL);
  EXPECT(ddcc_set_tile(NULL, 64, 4) == DDCC_E_INVAL);
  size_t nb = 0;
  EXPECT(ddcc_save(NULL, NULL, &nb) == DDCC_E_INVAL);
  EXPECT(ddcc_load(NULL, NULL, 0) == DDCC_E_INVAL);
  ddcc_batch_destroy(NULL);
  EXPECT(ddcc_batch_last_error(NULL) != NULL);
  EXPECT(ddcc_batch_time(NULL) == -1);
  /* batches: bad counts and sizes are rejected before any device call */
  ddcc_batch* b = (ddcc_batch*)&p;
  const int nx[2] = {64, 0}, ny[2] = {64, 64};
  EXPECT(ddcc_batch_create(&p, 0, nx, ny, NULL, &b) == DDCC_E_INVAL);
  EXPECT(b == NULL);
  EXPECT(ddcc_batch_create(&p, 2, nx, ny, NULL, &b) == DDCC_E_INVAL);
  EXPECT(ddcc_batch_create(&p, 1, NULL, ny, NULL, &b) == DDCC_E_INVAL);
}

/* One small run through every entry point family on the GPU. */
static void check_gpu(void) {
  unsigned seed = 12345u;
  ddcc_params p;
  ddcc_default_params(&p);
  p.nx = 70;
  p.ny = 20;
  p.precision = DDCC_FP32;
  p.lam = 0.5;
  ddcc_ctx* c = NULL;
  EXPECT(ddcc_create(&p, NULL, &c) == DDCC_OK);
  if (!c) return;
  const size_t n = (size_t)p.nx * p.ny;
  double* psi = malloc(n * sizeof(double));
  double* ct = malloc(n * sizeof(double));
  double* C = malloc(2 * n * sizeof(double));
  double* u = malloc(2 * n * sizeof(double));
  double* P = malloc(n * sizeof(double));
  double* w = malloc(n * sizeof(double));
  double* gc = malloc(n * sizeof(double));
  double* gp = malloc(n * sizeof(double));
  for (size_t i = 0; i < n; ++i) {
    const double x = (double)(i % p.nx), y = (double)(i / p.nx);
    const double d = sqrt((x - 35) * (x - 35) + (y - 10) * (y - 10)) - 5.0;
    psi[i] = 0.5 * (1.0 + tanh(d / 2.1));
    ct[i] = 0.4 * frand(&seed) - 0.2;
    const double r = sqrt((x - 20) * (x - 20) + (y - 10) * (y - 10));
    C[i] = 0.5 * (1.0 + tanh(2.0 * (7.0 - r) / 5.0));
    C[n + i] = 1.0 - C[i];
    u[i] = u[n + i] = 0.0;
    P[i] = 0.0;
    w[i] = x;
  }
  EXPECT(ddcc_step(c, 1) == DDCC_E_STATE);
  EXPECT(ddcc_init_geometry(c, psi, ct) == DDCC_OK);
  EXPECT(ddcc_init_fields(c, C, u, P) == DDCC_OK);
  EXPECT(ddcc_step(c, 10) == DDCC_OK);
  EXPECT(ddcc_step(c, -1) == DDCC_E_INVAL);
  EXPECT(ddcc_read_moments(c, C, u, P) == DDCC_OK);
  double m[2];
  EXPECT(ddcc_mass(c, m) == DDCC_OK);
  size_t bytes = 0;
  EXPECT(ddcc_save(c, NULL, &bytes) == DDCC_OK);
  void* buf = malloc(bytes);
  EXPECT(ddcc_save(c, buf, &bytes) == DDCC_OK);
  EXPECT(ddcc_load(c, buf, bytes - 1) == DDCC_E_INVAL);
  EXPECT(ddcc_load(c, buf, bytes) == DDCC_OK);
  free(buf);
  EXPECT(ddcc_set_tile(c, 64, 3) == DDCC_E_INVAL);
  int ty = 0;
  EXPECT(ddcc_autotune(c, 2, &ty) == DDCC_OK);
  EXPECT(ddcc_set_diagnostics(c, 5) == DDCC_OK);
  EXPECT(ddcc_step(c, 11) == DDCC_OK);
  int64_t tc = -2, tn = -2;
  EXPECT(ddcc_diagnostics(c, m, &tc, &tn) == DDCC_OK);
  EXPECT(tn == -1);
  double J = 0.0;
  EXPECT(ddcc_adjoint(c, 6, 4, 0, w, &J, gc, gp) == DDCC_OK);
  EXPECT(ddcc_objective(c, 0, w, &J) == DDCC_OK);
  ddcc_destroy(c);

  /* 3D, FP16 storage */
  ddcc_default_params(&p);
  p.dim = 3;
  p.nx = 66;
  p.ny = 5;
  p.nz = 4;
  p.lattice_f = DDCC_D3Q15;
  p.lattice_g = DDCC_D3Q19;
  p.precision = DDCC_FP16;
  c = NULL;
  EXPECT(ddcc_create(&p, NULL, &c) == DDCC_OK);
  if (c) {
    const size_t n3 = (size_t)p.nx * p.ny * p.nz;
    double* psi3 = malloc(n3 * sizeof(double));
    double* C3 = malloc(2 * n3 * sizeof(double));
    for (size_t i = 0; i < n3; ++i) {
      psi3[i] = 1.0 - 0.5 * frand(&seed);
      C3[i] = frand(&seed);
      C3[n3 + i] = 1.0 - C3[i];
    }
    EXPECT(ddcc_init_geometry(c, psi3, NULL) == DDCC_OK);
    EXPECT(ddcc_init_fields(c, C3, NULL, NULL) == DDCC_OK);
    EXPECT(ddcc_step(c, 3) == DDCC_OK);
    EXPECT(ddcc_read_moments(c, C3, NULL, NULL) == DDCC_OK);
    EXPECT(ddcc_adjoint(c, 2, 1, 0, w, &J, NULL, NULL) == DDCC_E_UNSUPPORTED);
    free(psi3);
    free(C3);
    ddcc_destroy(c);
  }

  /* a batch of three boxes */
  ddcc_default_params(&p);
  p.precision = DDCC_FP32;
  const int bx[3] = {64, 20, 70}, by[3] = {8, 20, 20};
  ddcc_batch* b = NULL;
  EXPECT(ddcc_batch_create(&p, 3, bx, by, NULL, &b) == DDCC_OK);
  if (b) {
    for (int i = 0; i < 3; ++i) {
      const size_t ni = (size_t)bx[i] * by[i];
      double* pi = malloc(ni * sizeof(double));
      double* Ci = malloc(2 * ni * sizeof(double));
      for (size_t k = 0; k < ni; ++k) {
        pi[k] = 1.0;
        Ci[k] = frand(&seed);
        Ci[ni + k] = 1.0 - Ci[k];
      }
      EXPECT(ddcc_batch_init_geometry(b, i, pi, NULL) == DDCC_OK);
      EXPECT(ddcc_batch_init_fields(b, i, Ci, NULL, NULL) == DDCC_OK);
      free(pi);
      free(Ci);
    }
    EXPECT(ddcc_batch_set_graph(b, 4) == DDCC_OK);
    EXPECT(ddcc_batch_step(b, 9) == DDCC_OK);
    EXPECT(ddcc_batch_mass(b, 2, m) == DDCC_OK);
    EXPECT(ddcc_batch_sync(b) == DDCC_OK);
    ddcc_batch_destroy(b);
  }
  free(psi);
  free(ct);
  free(C);
  free(u);
  free(P);
  free(w);
  free(gc);
  free(gp);
}

int main(int argc, char** argv) {
  check_validation();
  if (argc > 1 && strcmp(argv[1], "--gpu") == 0) check_gpu();
  if (failures) {
    fprintf(stderr, "host_check: %d failed checks\n", failures);
    return 1;
  }
  printf("ok\n");
  return 0;
}
