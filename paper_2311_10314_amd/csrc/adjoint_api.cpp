// Host side of ddcc_adjoint (include/ddcc.h): forward sweep with periodic
// checkpoints, objective and seed, reverse sweep segment by segment
// (recomputing each segment's states from its checkpoint, the step kernel
// writing each state straight into its slot), final gradients. The states
// of the next segment are recomputed on a second stream while the reverse
// sweep runs over the current one, into the other of two segment buffers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/ddcc.h"
#include "adjoint.hpp"
#include "ctx.hpp"
#include "kernels.hpp"

using namespace ddcc;
using detail::fail;
using detail::hip_fail;

namespace {

// Device memory released when the call returns.
struct DevMem {
  void* p = nullptr;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 1); }
  template <class T>
  T* as(size_t byte_off = 0) const {
    return reinterpret_cast<T*>(static_cast<char*>(p) + byte_off);
  }
};

// A second stream (default priority) and the events that order the two
// segment buffers between it and the context stream; released on return.
struct Pipe {
  hipStream_t aux = nullptr;
  hipEvent_t ready[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
  hipEvent_t start = nullptr;
  ~Pipe() {
    if (aux) (void)hipStreamSynchronize(aux);
    for (hipEvent_t e : {ready[0], ready[1], freed[0], freed[1], start})
      if (e) (void)hipEventDestroy(e);
    if (aux) (void)hipStreamDestroy(aux);
  }
  hipError_t init() {
    hipError_t e = hipStreamCreateWithFlags(&aux, hipStreamNonBlocking);
    for (hipEvent_t* ev : {&ready[0], &ready[1], &freed[0], &freed[1], &start})
      if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    return e;
  }
};

// Bytes of one stored state in the step's own layout.
struct Layout {
  size_t sf, s0, sg, sh, sT, total;
};

Layout state_layout(const ddcc_ctx* c) {
  Layout L;
  const size_t n = (size_t)c->n;
  L.sf = (size_t)c->p.nphase * (c->Qf - 1) * n * c->pesz;
  L.s0 = (size_t)c->p.nphase * n * sizeof(double);
  L.sg = (size_t)c->Qg * n * c->pesz;
  L.sh = (size_t)c->nhist * n * c->esz;
  L.sT = (size_t)c->nT * n * c->esz;
  // keep every part of every slot 256-byte aligned
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  L.sf = up(L.sf);
  L.s0 = up(L.s0);
  L.sg = up(L.sg);
  L.sh = up(L.sh);
  L.sT = up(L.sT);
  L.total = L.sf + L.s0 + L.sg + L.sh + L.sT;
  return L;
}

// Copy the context's current state (populations, history, T) into a slot.
hipError_t save_state(ddcc_ctx* c, char* slot, const Layout& L) {
  const size_t n = (size_t)c->n;
  struct Part {
    void* dev;
    size_t off, bytes;
  } parts[5] = {
      {c->f[c->cur], 0, (size_t)c->p.nphase * (c->Qf - 1) * n * c->pesz},
      {c->f0[c->cur], L.sf, (size_t)c->p.nphase * n * sizeof(double)},
      {c->g[c->cur], L.sf + L.s0, (size_t)c->Qg * n * c->pesz},
      {c->hist, L.sf + L.s0 + L.sg, (size_t)c->nhist * n * c->esz},
      {c->T[c->cur], L.sf + L.s0 + L.sg + L.sh, (size_t)c->nT * n * c->esz}};
  for (const Part& q : parts) {
    if (!q.bytes) continue;
    hipError_t e = hipMemcpyAsync(slot + q.off, q.dev, q.bytes,
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <class S>
AdjFwd<S> view(const char* slot, const Layout& L) {
  AdjFwd<S> v;
  v.f = reinterpret_cast<const S*>(slot);
  v.f0 = reinterpret_cast<const double*>(slot + L.sf);
  v.g = reinterpret_cast<const S*>(slot + L.sf + L.s0);
  v.hist = reinterpret_cast<const S*>(slot + L.sf + L.s0 + L.sg);
  v.T = reinterpret_cast<const S*>(slot + L.sf + L.s0 + L.sg + L.sh);
  return v;
}

template <class R>
const Coef<R>& coef_of(const ddcc_ctx* c);
template <>
const Coef<double>& coef_of<double>(const ddcc_ctx* c) {
  return c->kd;
}
template <>
const Coef<float>& coef_of<float>(const ddcc_ctx* c) {
  return c->kf;
}

// One forward step from the state stored in slot `from` into slot `to`
// (the history is updated in place, so it is copied over first).
template <class S>
hipError_t step_between(ddcc_ctx* c, const char* from, char* to,
                        const Layout& L, hipStream_t st) {
  const size_t oh = L.sf + L.s0 + L.sg;
  const size_t sh = (size_t)c->nhist * (size_t)c->n * c->esz;
  hipError_t e = hipMemcpyAsync(to + oh, from + oh, sh, hipMemcpyDeviceToDevice,
                                st);
  if (e != hipSuccess) return e;
  Bufs<S, S> b{};
  const AdjFwd<S> a = view<S>(from, L);
  b.fA = a.f;
  b.f0A = a.f0;
  b.gA = a.g;
  b.TA = a.T;
  b.fB = reinterpret_cast<S*>(to);
  b.f0B = reinterpret_cast<double*>(to + L.sf);
  b.gB = reinterpret_cast<S*>(to + L.sf + L.s0);
  b.hist = reinterpret_cast<S*>(to + oh);
  b.TB = reinterpret_cast<S*>(to + oh + L.sh);
  b.psi = static_cast<const S*>(c->psi);
  b.wet = static_cast<const S*>(c->wet);
  b.coef_d = c->dkd;
  b.coef_r = sizeof(S) == 8 ? static_cast<const void*>(c->dkd)
                            : static_cast<const void*>(c->dkf);
  return launch_2d<S, S, S>(c->p.nphase, MODE_STEP, c->kd, coef_of<S>(c), b,
                            c->tile_y, st);
}

int forward_step(ddcc_ctx* c) {
  hipError_t e = detail::step_launch(c);
  if (e != hipSuccess) return hip_fail(c, e, "step kernel");
  c->cur ^= 1;
  ++c->t;
  return DDCC_OK;
}

#define ACHK(expr, what)                              \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return hip_fail(c, e_, what); \
  } while (0)

// Sum of w phi C_k and of phi C_k over the state held by fw.
template <class S>
int weighted_sums(ddcc_ctx* c, const AdjFwd<S>& fw, int phase,
                  const double* wgt, double* part, int wblocks, double& sw,
                  double& sm) {
  ACHK(launch_adj_wsum<S>(c->kd, fw, phase, wgt, part, wblocks, c->stream),
       "objective kernel");
  std::vector<double> hp(2 * (size_t)wblocks);
  ACHK(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double),
                      hipMemcpyDeviceToHost, c->stream),
       "copy objective");
  ACHK(hipStreamSynchronize(c->stream), "sync");
  sw = 0.0;
  sm = 0.0;
  for (int b = 0; b < wblocks; ++b) {
    sw += hp[2 * (size_t)b];
    sm += hp[2 * (size_t)b + 1];
  }
  if (!(std::fabs(sm) > 0.0) || !std::isfinite(sw) || !std::isfinite(sm))
    return fail(c, DDCC_E_NONFINITE, "phase mass is zero or not finite");
  return DDCC_OK;
}

int weight_blocks(long long n) {
  const long long nb = (n + 255) / 256;
  return (int)(nb > 1024 ? 1024 : nb);
}

// S: storage type of the context's forward state; the adjoint is float64.
template <class S>
int adjoint_as(ddcc_ctx* c, int64_t nsteps, int interval, int phase,
               const double* w_host, double* J_out, double* gcos_host,
               double* gpsi_host) {
  using R = double;
  const int N = c->p.nphase;
  const size_t n = (size_t)c->n;
  const Layout L = state_layout(c);
  const int64_t nck = (nsteps + interval - 1) / interval;
  const int64_t seg = nsteps < interval ? nsteps : interval;
  const size_t slots = (size_t)(nck + 2 * seg + 1);

  DevMem store, adj, work, grads, misc;
  ACHK(store.alloc(slots * L.total), "hipMalloc checkpoints");
  auto slot = [&](size_t i) { return store.as<char>(i * L.total); };
  char* ck0 = slot(0);
  char* segbuf[2] = {slot((size_t)nck), slot((size_t)(nck + seg))};
  char* fin = slot((size_t)(nck + 2 * seg));

  const size_t sfl = (size_t)N * 9 * n, sgl = 9 * n, shl = (size_t)c->nhist * n;
  const size_t sal = (size_t)adj_planes(N) * n;
  const size_t adj_count = 2 * sfl + 2 * sgl + shl + 2 * n + sal;
  ACHK(adj.alloc(adj_count * sizeof(R)), "hipMalloc adjoint");
  R* lf[2] = {adj.as<R>(), adj.as<R>() + sfl};
  R* lg[2] = {lf[1] + sfl, lf[1] + sfl + sgl};
  R* lh = lg[1] + sgl;
  R* lT[2] = {lh + shl, lh + shl + n};
  R* a = lT[1] + n;

  ACHK(work.alloc((size_t)(4 * N + 2) * n * sizeof(double)), "hipMalloc work");
  AdjWork w;
  w.psiC = work.as<double>();
  w.tot = w.psiC + (size_t)N * n;
  w.C = w.tot + n;
  w.prho = w.C + (size_t)N * n;
  w.psimu = w.prho + n;
  w.mu = w.psimu + (size_t)N * n;

  const size_t ngrad = (size_t)(N - 1) * n + n + 2 * n + (size_t)(N - 1) * n + n;
  ACHK(grads.alloc(ngrad * sizeof(double)), "hipMalloc gradients");
  double* gE = grads.as<double>();
  double* gpsi = gE + (size_t)(N - 1) * n;
  double* ggpsi = gpsi + n;
  double* gcos = ggpsi + 2 * n;
  double* gpsi_out = gcos + (size_t)(N - 1) * n;
  ACHK(hipMemsetAsync(gE, 0, (size_t)(N + 2) * n * sizeof(double), c->stream),
       "clear gradients");

  const int wblocks = weight_blocks((long long)n);
  ACHK(misc.alloc((n + 2 * (size_t)wblocks) * sizeof(double)), "hipMalloc weights");
  double* wgt = misc.as<double>();
  double* part = wgt + n;
  ACHK(hipMemcpyAsync(wgt, w_host, n * sizeof(double), hipMemcpyHostToDevice,
                      c->stream),
       "copy weights");

  // forward sweep: checkpoint every `interval` steps, keep the final state
  int rc = DDCC_OK;
  for (int64_t s = 0; s < nsteps; ++s) {
    if (s % interval == 0)
      ACHK(save_state(c, slot((size_t)(s / interval)), L), "checkpoint");
    rc = forward_step(c);
    if (rc) return rc;
  }
  ACHK(save_state(c, fin, L), "checkpoint");

  // objective on the final state
  double sw, sm;
  rc = weighted_sums<S>(c, view<S>(fin, L), phase, wgt, part, wblocks, sw,
                            sm);
  if (rc) return rc;
  const double J = sw / sm;
  if (J_out) *J_out = J;

  // lambda at the final level
  ACHK(hipMemsetAsync(adj.p, 0, adj_count * sizeof(R), c->stream), "clear adjoint");
  ACHK(launch_adj_seed(c->kd, phase, wgt, J, sm, lf[0], c->stream), "seed kernel");

  // reverse sweep, one segment at a time. Segment sg's states are in
  // segbuf[(nck - 1 - sg) % 2]; while the context stream runs the reverse
  // steps over them, the second stream recomputes segment sg - 1 into the
  // other buffer, once the reverse sweep of segment sg + 1 has released it.
  Pipe pp;
  ACHK(pp.init(), "adjoint streams");
  auto recompute = [&](int64_t sg, char* dst) -> hipError_t {
    const int64_t s0 = sg * interval;
    const int64_t s1 = s0 + interval < nsteps ? s0 + interval : nsteps;
    hipError_t e = hipMemcpyAsync(dst, ck0 + (size_t)sg * L.total, L.total,
                                  hipMemcpyDeviceToDevice, pp.aux);
    for (int64_t s = s0; s < s1 - 1 && e == hipSuccess; ++s) {
      char* from = dst + (size_t)(s - s0) * L.total;
      e = step_between<S>(c, from, from + L.total, L, pp.aux);
    }
    return e;
  };
  // the checkpoints were written on the context stream (no segment at all
  // when nsteps = 0)
  if (nck > 0) {
    ACHK(hipEventRecord(pp.start, c->stream), "event");
    ACHK(hipStreamWaitEvent(pp.aux, pp.start, 0), "event");
    ACHK(recompute(nck - 1, segbuf[0]), "step kernel");
    ACHK(hipEventRecord(pp.ready[0], pp.aux), "event");
  }
  int la = 0;
  for (int64_t sg = nck - 1; sg >= 0; --sg) {
    const int b = (int)((nck - 1 - sg) % 2);
    if (sg > 0) {
      if (sg + 1 <= nck - 1)
        ACHK(hipStreamWaitEvent(pp.aux, pp.freed[b ^ 1], 0), "event");
      ACHK(recompute(sg - 1, segbuf[b ^ 1]), "step kernel");
      ACHK(hipEventRecord(pp.ready[b ^ 1], pp.aux), "event");
    }
    ACHK(hipStreamWaitEvent(c->stream, pp.ready[b], 0), "event");
    const int64_t s0 = sg * interval;
    const int64_t s1 = s0 + interval < nsteps ? s0 + interval : nsteps;
    for (int64_t s = s1 - 1; s >= s0; --s) {
      AdjBufs<R> ab;
      ab.lfB = lf[la];
      ab.lfA = lf[la ^ 1];
      ab.lgB = lg[la];
      ab.lgA = lg[la ^ 1];
      ab.lh = lh;
      ab.lTB = lT[la];
      ab.lTA = lT[la ^ 1];
      ab.a = a;
      ab.gE = gE;
      ab.gpsi = gpsi;
      ab.ggpsi = ggpsi;
      ACHK(launch_adj_step<S>(N, c->kd,
                              view<S>(segbuf[b] + (size_t)(s - s0) * L.total, L),
                              static_cast<const S*>(c->psi),
                              static_cast<const S*>(c->wet), w, ab, c->stream),
           "adjoint step kernels");
      la ^= 1;
    }
    ACHK(hipEventRecord(pp.freed[b], c->stream), "event");
  }

  // the derivative of the wetting weights in psi from the float64 geometry
  // the weights were made from
  const double* psi64 = c->geo64;
  const double* cos64 = psi64 ? psi64 + n : nullptr;
  ACHK(launch_adj_finish<S>(c->kd, N - 1, static_cast<const S*>(c->psi),
                            static_cast<const S*>(c->wet), psi64, cos64, gE,
                            ggpsi, gpsi, gcos, gpsi_out, c->stream),
       "gradient kernels");
  if (gcos_host)
    ACHK(hipMemcpyAsync(gcos_host, gcos, (size_t)(N - 1) * n * sizeof(double),
                        hipMemcpyDeviceToHost, c->stream),
         "copy gradient");
  if (gpsi_host)
    ACHK(hipMemcpyAsync(gpsi_host, gpsi_out, n * sizeof(double),
                        hipMemcpyDeviceToHost, c->stream),
         "copy gradient");
  // the reverse sweep works on the stored states only: the context still
  // holds the final level of the forward sweep
  ACHK(hipStreamSynchronize(c->stream), "sync");
  return DDCC_OK;
}

template <class S>
int objective_as(ddcc_ctx* c, int phase, const double* w_host, double* J) {
  const size_t n = (size_t)c->n;
  const int wblocks = weight_blocks((long long)n);
  DevMem misc;
  ACHK(misc.alloc((n + 2 * (size_t)wblocks) * sizeof(double)), "hipMalloc weights");
  double* wgt = misc.as<double>();
  ACHK(hipMemcpyAsync(wgt, w_host, n * sizeof(double), hipMemcpyHostToDevice,
                      c->stream),
       "copy weights");
  AdjFwd<S> fw;
  fw.f = static_cast<const S*>(c->f[c->cur]);
  fw.f0 = c->f0[c->cur];
  fw.g = static_cast<const S*>(c->g[c->cur]);
  fw.hist = static_cast<const S*>(c->hist);
  fw.T = static_cast<const S*>(c->T[c->cur]);
  double sw, sm;
  int rc = weighted_sums<S>(c, fw, phase, wgt, wgt + n, wblocks, sw, sm);
  if (rc) return rc;
  *J = sw / sm;
  return DDCC_OK;
}

int check_common(ddcc_ctx* c, int phase, const double* weight) {
  if (!c->fields_ok) return fail(c, DDCC_E_STATE, "init_fields first");
  if (phase < 0 || phase >= c->p.nphase)
    return fail(c, DDCC_E_INVAL, "phase out of range");
  if (!weight) return fail(c, DDCC_E_INVAL, "weight is NULL");
  for (long long i = 0; i < c->n; ++i)
    if (!std::isfinite(weight[i]))
      return fail(c, DDCC_E_INVAL, "non-finite weight");
  if (c->p.dim != 2)
    return fail(c, DDCC_E_UNSUPPORTED, "the adjoint step is two-dimensional");
  return DDCC_OK;
}

}  // namespace

extern "C" int ddcc_objective(ddcc_ctx* c, int phase, const double* weight,
                              double* J) {
  if (!c) return DDCC_E_INVAL;
  if (!J) return fail(c, DDCC_E_INVAL, "J is NULL");
  int rc = check_common(c, phase, weight);
  if (rc) return rc;
  switch (c->p.precision) {
    case DDCC_FP64:
      return objective_as<double>(c, phase, weight, J);
    case DDCC_FP32:
      return objective_as<float>(c, phase, weight, J);
    default:
      return fail(c, DDCC_E_UNSUPPORTED,
                  "the objective runs in FP64 or FP32 contexts");
  }
}

extern "C" int ddcc_adjoint(ddcc_ctx* c, int64_t nsteps, int interval,
                            int phase, const double* weight, double* J,
                            double* grad_cos, double* grad_psi) {
  if (!c) return DDCC_E_INVAL;
  if (nsteps < 0) return fail(c, DDCC_E_INVAL, "nsteps < 0");
  if (interval < 1) return fail(c, DDCC_E_INVAL, "checkpoint interval < 1");
  int rc = check_common(c, phase, weight);
  if (rc) return rc;
  if (c->nwalls != 1)
    return fail(c, DDCC_E_UNSUPPORTED, "the adjoint step needs one wall");
  switch (c->p.precision) {
    case DDCC_FP64:
      return adjoint_as<double>(c, nsteps, interval, phase, weight, J,
                                grad_cos, grad_psi);
    case DDCC_FP32:
      return adjoint_as<float>(c, nsteps, interval, phase, weight, J,
                               grad_cos, grad_psi);
    default:
      return fail(c, DDCC_E_UNSUPPORTED,
                  "the adjoint step runs in FP64 or FP32 contexts");
  }
}
