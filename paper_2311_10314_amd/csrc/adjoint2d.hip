// Reverse-time (adjoint) step of the 2D DD-CCLB scheme for gfx950.
//
// One forward step (Section 3) maps the stored state of level n,
// s^n = (moving populations f^i_p and g_p as written before streaming,
// float64 rest populations f^i_0, history phi C_i u, Y, P at each node, the
// antisymmetric flux T), to s^{n+1}. For an objective J(s^T) the adjoint
// sweep carries lambda^n = (ds^{n+1}/ds^n)^T lambda^{n+1} backwards and
// accumulates the derivatives of J with respect to the static fields every
// step reads: the wetting weights E_i (eq. 2.14 through eq. 2.9) and psi.
// Every stage of the forward step is transposed by hand: pointwise maps by
// their local Jacobians, the isotropic gradient stencil by minus the same
// stencil applied as a divergence, and the two-point div(psi grad .) by
// itself (it is symmetric in the node pair); pull streaming becomes a push.
//
// Kernels of one reverse step (one node per thread, no workgroup barriers):
//   k_adj_frac  forward: phi C_i (pulled), their sum, C_i, phi rho
//   k_adj_mu    forward: phi mu_i (eq. 2.14) and mu_i = phi mu_i / psi_hat
//   k_adj_node  recomputes the node update at x and transposes it: the
//               adjoint of the pulled flow populations (complete, pushed to
//               x - c_p), of the pulled phase populations (direct part), of
//               the history at x, and per-node adjoints of every stencil
//               input (grad C_i, grad mu_i, grad phi rho, div T, grad psi)
//   k_adj_mid   gathers the stencil adjoints, transposes mu = phi mu /
//               psi_hat, phi rho and phi mu_i at the node; the adjoint of T
//               is complete here
//   k_adj_pop   gathers the adjoint of div(psi grad C_j), transposes
//               C_i = phi C_i / sum_j phi C_j and adds the result to every
//               phase population that formed phi C_i
// The adjoint state and arithmetic are float64 for every context; the
// forward states are read in the context's storage type (float32 contexts
// are linearised about their own float32 trajectory).
#include <hip/hip_runtime.h>

#include "adjoint.hpp"
#include "coef.hpp"
#include "common.hpp"
#include "collide.hpp"
#include "lattice.hpp"
#include "lattice_adj.hpp"

namespace ddcc {

namespace {

constexpr int kThreads = 256;
constexpr int Q = 9;

// 3 x 3 neighbourhood of a node on the periodic box; v[dy + 1][dx + 1].
template <class T>
struct P3 {
  T v[3][3];
};

struct Nb3 {
  int xs[3];
  int ys[3];  // row offsets (y * nx)
  __device__ inline unsigned at(int dx, int dy) const {
    return unsigned(ys[dy + 1] + xs[dx + 1]);
  }
  // where population p of this node is pulled from, and where the adjoint of
  // the pulled value is pushed to: x - c_p
  __device__ inline unsigned pull(int p) const {
    return at(-D2Q9::c[p].x, -D2Q9::c[p].y);
  }
};

__device__ inline Nb3 nb3(int gx, int gy, int nx, int ny) {
  Nb3 b;
  b.xs[0] = gx == 0 ? nx - 1 : gx - 1;
  b.xs[1] = gx;
  b.xs[2] = gx == nx - 1 ? 0 : gx + 1;
  b.ys[0] = (gy == 0 ? ny - 1 : gy - 1) * nx;
  b.ys[1] = gy * nx;
  b.ys[2] = (gy == ny - 1 ? 0 : gy + 1) * nx;
  return b;
}

template <class T, class Src>
__device__ inline P3<T> load3(const Src* plane, const Nb3& b) {
  P3<T> p;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx)
      p.v[dy + 1][dx + 1] = T(plane[b.at(dx, dy)]);
  return p;
}

// The fixed isotropic gradient of the step: D2Q9 weights at d0 = 1/3 over
// its c_s^2, 1/3 on the axes and 1/12 on the diagonals.
template <class T>
__device__ inline T gx3(const P3<T>& p) {
  return T(1.0 / 3.0) * (p.v[1][2] - p.v[1][0]) +
         T(1.0 / 12.0) * ((p.v[2][2] + p.v[0][2]) - (p.v[2][0] + p.v[0][0]));
}

template <class T>
__device__ inline T gy3(const P3<T>& p) {
  return T(1.0 / 3.0) * (p.v[2][1] - p.v[0][1]) +
         T(1.0 / 12.0) * ((p.v[2][2] + p.v[2][0]) - (p.v[0][2] + p.v[0][0]));
}

// Transpose of the gradient: for a(x) = (a_x, a_y) the adjoint of the
// field the gradient was taken of is -(Dx a_x + Dy a_y).
template <class T>
__device__ inline T grad_T(const P3<T>& ax, const P3<T>& ay) {
  return -(gx3(ax) + gy3(ay));
}

// Stencil weight of neighbour (dx, dy) in div(psi grad .): 1/3 axes,
// 1/12 diagonals, over c_s^2 = 1/3 of the stencil lattice.
__device__ constexpr double wdiv(int dx, int dy) {
  return (dx != 0 && dy != 0) ? 1.0 / 12.0 : 1.0 / 3.0;
}

// div(psi grad C) in the two-point form of the step.
template <class T>
__device__ inline T div_psi_grad3(const P3<T>& psi, const P3<T>& c) {
  T acc = T(0);
  const T pc = psi.v[1][1], cc = c.v[1][1];
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx)
      if (dx || dy)
        acc += T(wdiv(dx, dy)) * (psi.v[dy + 1][dx + 1] + pc) *
               (c.v[dy + 1][dx + 1] - cc);
  return acc;
}

__device__ inline double gprime2(double C) {  // g''(C), g = C^2 (C - 1)^2
  return 12.0 * C * C - 12.0 * C + 2.0;
}

// ---------------------------------------------------------------------------
// Forward recomputation of the fields of level n
// ---------------------------------------------------------------------------
template <int N, class S>
__global__ __launch_bounds__(kThreads) void k_adj_frac(Coef<double> kd,
                                                       AdjFwd<S> fw,
                                                       const S* psi,
                                                       AdjWork w) {
  const long long n = kd.n;
  const long long x = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (x >= n) return;
  const int gx = int(x % kd.nx), gy = int(x / kd.nx);
  const Nb3 b = nb3(gx, gy, kd.nx, kd.ny);
  double pc[N], tot = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    S mv = S(0);  // moving populations summed as the step sums them
#pragma unroll
    for (int p = 1; p < Q; ++p) mv += phase_plane(fw.f, i, p, Q, n)[b.pull(p)];
    pc[i] = fw.f0[(long long)i * n + x] + double(mv);
    tot += pc[i];
  }
  const double inv = 1.0 / (tot > kd.psi_min ? tot : kd.psi_min);
  double rho = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double C = pc[i] * inv;
    w.psiC[(long long)i * n + x] = pc[i];
    w.C[(long long)i * n + x] = C;
    rho += kd.rho[i] * C;
  }
  w.tot[x] = tot;
  w.prho[x] = double(psi[x]) * rho;
}

template <int N, class S>
__global__ __launch_bounds__(kThreads) void k_adj_mu(Coef<double> kd,
                                                     const S* psi_f,
                                                     const S* wet, AdjWork w) {
  const long long n = kd.n;
  const long long x = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (x >= n) return;
  const int gx = int(x % kd.nx), gy = int(x / kd.nx);
  const Nb3 b = nb3(gx, gy, kd.nx, kd.ny);
  const P3<double> ps = load3<double>(psi_f, b);
  const double psi = ps.v[1][1];
  const double psih = psi > kd.psi_min ? psi : kd.psi_min;
  double C[N], L[N], E[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const P3<double> cp = load3<double>(w.C + (long long)j * n, b);
    C[j] = cp.v[1][1];
    L[j] = div_psi_grad3(ps, cp);
  }
#pragma unroll
  for (int i = 0; i < N - 1; ++i) E[i] = double(wet[(long long)i * n + x]);
  E[N - 1] = 0.0;
  double W[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < N; ++q)
      if (q != j)
        acc += (kd.sigN[j] * E[j] - kd.sigN[q] * E[q]) * kd.inv_sig[j][q] *
               C[j] * C[q];
    W[j] = acc;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double bulk = 0.0, grad = 0.0, wet_t = 0.0;
    const double gi = gprime(C[i]);
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (j != i) {
        bulk += kd.beta2[i][j] * (gi - gprime(C[i] + C[j]));
        grad += kd.grad34[i][j] * L[j];
        wet_t += kd.wet3[i][j] * W[j];
      }
    const double pm = psi * bulk + grad + wet_t;
    w.psimu[(long long)i * n + x] = pm;
    w.mu[(long long)i * n + x] = pm / psih;
  }
}

// ---------------------------------------------------------------------------
// Node update and its transpose
// ---------------------------------------------------------------------------
template <int N, class S, class R>
__global__ __launch_bounds__(kThreads) void k_adj_node(Coef<double> kd,
                                                       Coef<R> k, AdjFwd<S> fw,
                                                       const S* psi_f,
                                                       AdjWork w,
                                                       AdjBufs<R> ab) {
  using D = double;
  const long long n = k.n;
  const long long x = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (x >= n) return;
  const int gx = int(x % k.nx), gy = int(x / k.nx);
  const Nb3 b = nb3(gx, gy, k.nx, k.ny);

  // ---- forward quantities at x, as the step forms them --------------------
  const P3<D> ps = load3<D>(psi_f, b);
  const R psi = R(ps.v[1][1]);
  const D psih_d = ps.v[1][1] > kd.psi_min ? ps.v[1][1] : kd.psi_min;
  const bool psi_floor = !(ps.v[1][1] > kd.psi_min);
  const R gpsi[2] = {R(gx3(ps)), R(gy3(ps))};
  const P3<D> pr = load3<D>(w.prho, b);
  const R psirho = R(pr.v[1][1]);
  const R gprho[2] = {R(gx3(pr)), R(gy3(pr))};
  R C[N], gC[N][2], mu[N], gmu[N][2], psimu[N], psiC[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const P3<D> cp = load3<D>(w.C + (long long)i * n, b);
    C[i] = R(cp.v[1][1]);
    gC[i][0] = R(gx3(cp));
    gC[i][1] = R(gy3(cp));
    const P3<D> mp = load3<D>(w.mu + (long long)i * n, b);
    mu[i] = R(mp.v[1][1]);
    gmu[i][0] = R(gx3(mp));
    gmu[i][1] = R(gy3(mp));
    psimu[i] = R(w.psimu[(long long)i * n + x]);
    psiC[i] = R(w.psiC[(long long)i * n + x]);
  }
  R grho[2] = {R(0), R(0)};
#pragma unroll
  for (int i = 0; i < N; ++i) {
    grho[0] += k.rho[i] * gC[i][0];
    grho[1] += k.rho[i] * gC[i][1];
  }
  R mC[2] = {R(0), R(0)}, Cs[N], sr[N], aj[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    R s = R(0), t = R(0);
#pragma unroll
    for (int q = 0; q < N; ++q)
      if (q != j) {
        s += C[q];
        t += C[q] * (k.rho[j] - k.rho[q]);
      }
    Cs[j] = s;
    sr[j] = t;
    aj[j] = k.m0 * C[j] * t;
    mC[0] -= aj[j] * gmu[j][0];
    mC[1] -= aj[j] * gmu[j][1];
  }
  R gp[Q], jv[2] = {R(0), R(0)}, sum_gm = R(0);
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    gp[p] = R(fw.g[(long long)p * n + b.pull(p)]);
    if (p > 0) sum_gm += gp[p];
    jv[0] += R(D2Q9::c[p].x) * gp[p];
    jv[1] += R(D2Q9::c[p].y) * gp[p];
  }
  const P3<R> tp = load3<R>(fw.T, b);
  const R Pprev = R(fw.hist[(long long)(2 * N + 3) * n + x]);
  R Fp[2];
  Fp[0] = gy3(tp) + Pprev * gpsi[0] + psirho * k.accel[0] + psi * k.force[0];
  Fp[1] = -gx3(tp) + Pprev * gpsi[1] + psirho * k.accel[1] + psi * k.force[1];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    Fp[0] += psimu[i] * gC[i][0];
    Fp[1] += psimu[i] * gC[i][1];
  }
  const R pen = (R(1) - psi) * k.lam;
  const R den = R(1) / (psirho + R(0.5) * pen);
  const R jh[2] = {jv[0] + R(0.5) * Fp[0], jv[1] + R(0.5) * Fp[1]};
  const R u[2] = {jh[0] * den, jh[1] * den};
  const R F[2] = {Fp[0] - pen * u[0], Fp[1] - pen * u[1]};
  const R Y[3] = {psi * mC[0] * u[0],
                  R(0.5) * psi * (mC[0] * u[1] + u[0] * mC[1]),
                  psi * mC[1] * u[1]};
  R dtY[3];
#pragma unroll
  for (int q = 0; q < 3; ++q)
    dtY[q] = Y[q] - R(fw.hist[(long long)(2 * N + q) * n + x]);
  R nu = R(0);
#pragma unroll
  for (int i = 0; i < N; ++i) nu += k.nu[i] * C[i];
  const R s21 = R(1) / (k.two_over_c2mcs2 * nu + R(0.5));
  const R s22 = R(1) / (k.inv_cs2 * nu + R(0.5));
  const R A[3] = {psirho * u[0] * u[0] + Y[0], psirho * u[0] * u[1] + Y[1],
                  psirho * u[1] * u[1] + Y[2]};
  const R s0eq = -k.wg[0] * (A[0] + A[2]) * k.inv_c2mcs2;
  const R ugr = u[0] * grho[0] + u[1] * grho[1];
  const R ugpr = u[0] * gprho[0] + u[1] * gprho[1];
  const R psiP = k.pref * (sum_gm + k.cgr * psi * ugr +
                           k.halfK * (dtY[0] + dtY[2]) +
                           k.KH * (s21 - R(2)) / s21 * ugpr + s0eq);
  const R M[3] = {dtY[0] + R(2) * k.cs2 * u[0] * gprho[0] + k.one_m3cs2 * ugpr,
                  dtY[1] + k.cs2 * (u[0] * gprho[1] + gprho[0] * u[1]),
                  dtY[2] + R(2) * k.cs2 * u[1] * gprho[1] + k.one_m3cs2 * ugpr};
  const R a0 = psi * ugr;
  const R Jm[2] = {psirho * u[0], psirho * u[1]};

  // ---- adjoint of the outputs at x (level n + 1) ---------------------------
  R lX[N][2], lY[3], lP, lTn;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    lX[i][0] = ab.lh[(long long)(2 * i) * n + x];
    lX[i][1] = ab.lh[(long long)(2 * i + 1) * n + x];
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) lY[q] = ab.lh[(long long)(2 * N + q) * n + x];
  lP = ab.lh[(long long)(2 * N + 3) * n + x];
  lTn = ab.lTB[x];

  // adjoint accumulators of the forward intermediates
  R lu[2] = {R(0), R(0)}, lgpsi[2] = {R(0), R(0)}, lgprho[2] = {R(0), R(0)};
  R lgrho[2] = {R(0), R(0)}, lmC[2] = {R(0), R(0)};
  R lC[N], lgC[N][2], lmu[N], lgmu[N][2], lpsimu[N], lpsiC[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    lC[i] = lmu[i] = lpsimu[i] = lpsiC[i] = R(0);
    lgC[i][0] = lgC[i][1] = lgmu[i][0] = lgmu[i][1] = R(0);
  }
  R lpsi = R(0), lpsirho = R(0);

  // ---- phase sets: collision (3.1-3.7) transposed --------------------------
  R lXold[N][2];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R ldel[Q], lfp[Q];
#pragma unroll
    for (int p = 0; p < Q; ++p) {
      const R l = ab.lfB[(long long)(i * Q + p) * n + x];
      ldel[p] = -l;
      lfp[p] = l;  // f*_p = f_p - del_p (the rest population too)
    }
    R lem = R(0), lXi[2] = {lX[i][0], lX[i][1]}, lV[2] = {R(0), R(0)};
    collide_phase_T<D2Q9>(ldel, k.sf, k.cs2, lfp, lem, lXi, lV);
    // pulled moving populations: pushed back to x - c_p; the rest
    // population stays at x (k_adj_pop adds the phi C_i part to both)
    ab.lfA[(long long)(i * Q) * n + x] = lfp[0];
#pragma unroll
    for (int p = 1; p < Q; ++p) ab.lfA[(long long)(i * Q + p) * n + b.pull(p)] = lfp[p];
    lpsimu[i] += k.eta[i] * lem;
    // V = d_t(phi C_i u) + c_s^2 eta (mu_i grad psi - S_i)
    const R ce = k.cs2 * k.eta[i];
    lmu[i] += ce * (lV[0] * gpsi[0] + lV[1] * gpsi[1]);
    lgpsi[0] += ce * mu[i] * lV[0];
    lgpsi[1] += ce * mu[i] * lV[1];
    const R lS[2] = {-ce * lV[0], -ce * lV[1]};
    lXi[0] += lV[0];
    lXi[1] += lV[1];
    lXold[i][0] = -lV[0];
    lXold[i][1] = -lV[1];
    // X = phi C_i u
    lpsiC[i] += lXi[0] * u[0] + lXi[1] * u[1];
    lu[0] += psiC[i] * lXi[0];
    lu[1] += psiC[i] * lXi[1];
    // S_i = psi [(C_i Cs_i - 1) grad mu_i - sum_{j != i} C_i C_j grad mu_j]
    const R cii = C[i] * Cs[i] - R(1);
    lgmu[i][0] += psi * cii * lS[0];
    lgmu[i][1] += psi * cii * lS[1];
    const R g_i = lS[0] * gmu[i][0] + lS[1] * gmu[i][1];
    R bracket = cii * g_i;
    lC[i] += psi * Cs[i] * g_i;
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (j != i) {
        lC[j] += psi * C[i] * g_i;
        const R g_j = lS[0] * gmu[j][0] + lS[1] * gmu[j][1];
        lgmu[j][0] -= psi * C[i] * C[j] * lS[0];
        lgmu[j][1] -= psi * C[i] * C[j] * lS[1];
        lC[i] -= psi * C[j] * g_j;
        lC[j] -= psi * C[i] * g_j;
        bracket -= C[i] * C[j] * g_j;
      }
    lpsi += bracket;
  }

  // ---- flow set: collision (3.2, 3.8-3.12) transposed ----------------------
  R lgp[Q], ldelg[Q];
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    const R l = ab.lgB[(long long)p * n + x];
    ldelg[p] = -l;
    lgp[p] = l;
  }
  R lJ[2] = {R(0), R(0)}, lA[3] = {R(0), R(0), R(0)}, lM[3] = {R(0), R(0), R(0)};
  R lF[2] = {R(0), R(0)}, lpsiP = R(0), la0 = R(0), ls21 = R(0), ls22 = R(0);
  collide_flow_T<D2Q9>(gp, Jm, A, psiP, M, a0, F, s21, s22, k.sg, k.cs2,
                       k.inv_cs2, ldelg, lgp, lJ, lA, lpsiP, lM, la0, lF, ls21,
                       ls22);
  // a0 = psi u.grad rho
  R lugr = psi * la0;
  lpsi += ugr * la0;
  // J = phi rho u
  lpsirho += lJ[0] * u[0] + lJ[1] * u[1];
  lu[0] += psirho * lJ[0];
  lu[1] += psirho * lJ[1];
  // M^{2G} (eq. 3.12)
  R ldtY[3] = {lM[0], lM[1], lM[2]};
  R lugpr = k.one_m3cs2 * (lM[0] + lM[2]);
  lu[0] += R(2) * k.cs2 * gprho[0] * lM[0] + k.cs2 * gprho[1] * lM[1];
  lu[1] += k.cs2 * gprho[0] * lM[1] + R(2) * k.cs2 * gprho[1] * lM[2];
  lgprho[0] += R(2) * k.cs2 * u[0] * lM[0] + k.cs2 * u[1] * lM[1];
  lgprho[1] += k.cs2 * u[0] * lM[1] + R(2) * k.cs2 * u[1] * lM[2];
  // P = phi P / psi_hat (history output)
  lpsiP += R(D(lP) / psih_d);
  if (!psi_floor) lpsi -= R(D(lP) * D(psiP) / (psih_d * psih_d));
  // eq. (19)
  const R Lp = k.pref * lpsiP;
#pragma unroll
  for (int p = 1; p < Q; ++p) lgp[p] += Lp;
  lugr += Lp * k.cgr * psi;
  lpsi += Lp * k.cgr * ugr;
  ldtY[0] += Lp * k.halfK;
  ldtY[2] += Lp * k.halfK;
  ls21 += Lp * k.KH * ugpr * R(2) / (s21 * s21);
  lugpr += Lp * k.KH * (s21 - R(2)) / s21;
  lA[0] -= k.wg[0] * k.inv_c2mcs2 * Lp;
  lA[2] -= k.wg[0] * k.inv_c2mcs2 * Lp;
  // u.grad rho, u.grad(phi rho)
  lu[0] += lugr * grho[0] + lugpr * gprho[0];
  lu[1] += lugr * grho[1] + lugpr * gprho[1];
  lgrho[0] += lugr * u[0];
  lgrho[1] += lugr * u[1];
  lgprho[0] += lugpr * u[0];
  lgprho[1] += lugpr * u[1];
  // A = phi rho u u + Y
  R lYt[3] = {lY[0] + lA[0], lY[1] + lA[1], lY[2] + lA[2]};
  lpsirho += lA[0] * u[0] * u[0] + lA[1] * u[0] * u[1] + lA[2] * u[1] * u[1];
  lu[0] += psirho * (R(2) * u[0] * lA[0] + u[1] * lA[1]);
  lu[1] += psirho * (u[0] * lA[1] + R(2) * u[1] * lA[2]);
  // s21, s22 from nu (eq. 16), nu = sum_i nu_i C_i
  const R lnu = -k.two_over_c2mcs2 * s21 * s21 * ls21 -
                k.inv_cs2 * s22 * s22 * ls22;
#pragma unroll
  for (int i = 0; i < N; ++i) lC[i] += k.nu[i] * lnu;
  // d_t Y = Y - Y^{n-1}
  R lYold[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    lYt[q] += ldtY[q];
    lYold[q] = -ldtY[q];
  }
  // Y and T of phi m^C u
  lmC[0] += psi * (u[0] * lYt[0] + R(0.5) * u[1] * lYt[1] + R(0.5) * u[1] * lTn);
  lmC[1] += psi * (R(0.5) * u[0] * lYt[1] + u[1] * lYt[2] - R(0.5) * u[0] * lTn);
  lu[0] += psi * (mC[0] * lYt[0] + R(0.5) * mC[1] * lYt[1] - R(0.5) * mC[1] * lTn);
  lu[1] += psi * (R(0.5) * mC[0] * lYt[1] + mC[1] * lYt[2] + R(0.5) * mC[0] * lTn);
  lpsi += mC[0] * u[0] * lYt[0] + R(0.5) * (mC[0] * u[1] + u[0] * mC[1]) * lYt[1] +
          mC[1] * u[1] * lYt[2] + R(0.5) * (mC[0] * u[1] - u[0] * mC[1]) * lTn;
  // F = Fp - pen u; u = (j + Fp/2) / (phi rho + pen/2)
  R lFp[2] = {lF[0], lF[1]};
  lu[0] -= pen * lF[0];
  lu[1] -= pen * lF[1];
  R lpen = -(lF[0] * u[0] + lF[1] * u[1]);
  const R lj[2] = {den * lu[0], den * lu[1]};
  lFp[0] += R(0.5) * den * lu[0];
  lFp[1] += R(0.5) * den * lu[1];
  const R lden = lu[0] * jh[0] + lu[1] * jh[1];
  lpsirho -= den * den * lden;
  lpen -= R(0.5) * den * den * lden;
  lpsi -= k.lam * lpen;
#pragma unroll
  for (int p = 0; p < Q; ++p)
    lgp[p] += R(D2Q9::c[p].x) * lj[0] + R(D2Q9::c[p].y) * lj[1];
  // Fp (eq. 3.13)
  const R lPold = lFp[0] * gpsi[0] + lFp[1] * gpsi[1];
  lgpsi[0] += Pprev * lFp[0];
  lgpsi[1] += Pprev * lFp[1];
  lpsirho += k.accel[0] * lFp[0] + k.accel[1] * lFp[1];
  lpsi += k.force[0] * lFp[0] + k.force[1] * lFp[1];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    lpsimu[i] += gC[i][0] * lFp[0] + gC[i][1] * lFp[1];
    lgC[i][0] += psimu[i] * lFp[0];
    lgC[i][1] += psimu[i] * lFp[1];
  }
  // grad rho = sum_i rho_i grad C_i
#pragma unroll
  for (int i = 0; i < N; ++i) {
    lgC[i][0] += k.rho[i] * lgrho[0];
    lgC[i][1] += k.rho[i] * lgrho[1];
  }
  // m^C = -sum_j a_j grad mu_j, a_j = m0 C_j sum_{q != j} C_q (rho_j - rho_q)
#pragma unroll
  for (int j = 0; j < N; ++j) {
    lgmu[j][0] -= aj[j] * lmC[0];
    lgmu[j][1] -= aj[j] * lmC[1];
    const R la = -(lmC[0] * gmu[j][0] + lmC[1] * gmu[j][1]);
    lC[j] += k.m0 * sr[j] * la;
#pragma unroll
    for (int q = 0; q < N; ++q)
      if (q != j) lC[q] += k.m0 * C[j] * (k.rho[j] - k.rho[q]) * la;
  }
  // mu_i = phi mu_i / psi_hat at x
#pragma unroll
  for (int i = 0; i < N; ++i) {
    lpsimu[i] += R(D(lmu[i]) / psih_d);
    if (!psi_floor) lpsi -= R(D(lmu[i]) * D(psimu[i]) / (psih_d * psih_d));
  }

  // ---- writes -------------------------------------------------------------
#pragma unroll
  for (int p = 0; p < Q; ++p) ab.lgA[(long long)p * n + b.pull(p)] = lgp[p];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    ab.lh[(long long)(2 * i) * n + x] = lXold[i][0];
    ab.lh[(long long)(2 * i + 1) * n + x] = lXold[i][1];
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) ab.lh[(long long)(2 * N + q) * n + x] = lYold[q];
  ab.lh[(long long)(2 * N + 3) * n + x] = lPold;
  R* a = ab.a;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    a[(long long)(adj_gC<N>() + 2 * i) * n + x] = lgC[i][0];
    a[(long long)(adj_gC<N>() + 2 * i + 1) * n + x] = lgC[i][1];
    a[(long long)(adj_gmu<N>() + 2 * i) * n + x] = lgmu[i][0];
    a[(long long)(adj_gmu<N>() + 2 * i + 1) * n + x] = lgmu[i][1];
    a[(long long)(adj_C<N>() + i) * n + x] = lC[i];
    a[(long long)(adj_psimu<N>() + i) * n + x] = lpsimu[i];
    a[(long long)(adj_psiC<N>() + i) * n + x] = lpsiC[i];
  }
  a[(long long)(adj_gprho<N>()) * n + x] = lgprho[0];
  a[(long long)(adj_gprho<N>() + 1) * n + x] = lgprho[1];
  // Fp_x = Dy T, Fp_y = -Dx T: the T stencil adjoint (x, y components)
  a[(long long)(adj_T<N>()) * n + x] = -lFp[1];
  a[(long long)(adj_T<N>() + 1) * n + x] = lFp[0];
  a[(long long)(adj_psirho<N>()) * n + x] = lpsirho;
  ab.gpsi[x] += D(lpsi);
  ab.ggpsi[x] += D(lgpsi[0]);
  ab.ggpsi[n + x] += D(lgpsi[1]);
}

// ---------------------------------------------------------------------------
// Gathers of the stencil adjoints; phi mu_i and phi rho transposed
// ---------------------------------------------------------------------------
template <int N, class S, class R>
__global__ __launch_bounds__(kThreads) void k_adj_mid(Coef<double> kd,
                                                      const S* psi_f,
                                                      const S* wet, AdjWork w,
                                                      AdjBufs<R> ab) {
  using D = double;
  const long long n = kd.n;
  const long long x = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (x >= n) return;
  const int gx = int(x % kd.nx), gy = int(x / kd.nx);
  const Nb3 b = nb3(gx, gy, kd.nx, kd.ny);
  const R* a = ab.a;
  auto plane = [&](int q) { return a + (long long)q * n; };
  const D psi = D(psi_f[x]);
  const D psih = psi > kd.psi_min ? psi : kd.psi_min;
  const bool psi_floor = !(psi > kd.psi_min);
  D lpsi = 0.0;
  // adjoint of T^{n-1}: complete
  ab.lTA[x] = grad_T(load3<R>(plane(adj_T<N>()), b),
                     load3<R>(plane(adj_T<N>() + 1), b));
  // phi rho = psi sum_i rho_i C_i
  const D lpr = D(a[(long long)adj_psirho<N>() * n + x]) +
                D(grad_T(load3<R>(plane(adj_gprho<N>()), b),
                         load3<R>(plane(adj_gprho<N>() + 1), b)));
  D C[N], lC[N], lpm[N], E[N];
  D rho = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    C[i] = w.C[(long long)i * n + x];
    rho += kd.rho[i] * C[i];
    lC[i] = D(a[(long long)(adj_C<N>() + i) * n + x]) +
            D(grad_T(load3<R>(plane(adj_gC<N>() + 2 * i), b),
                     load3<R>(plane(adj_gC<N>() + 2 * i + 1), b))) +
            psi * kd.rho[i] * lpr;
    // mu_i = phi mu_i / psi_hat: the stencil part of the adjoint of mu_i
    const D lmu = D(grad_T(load3<R>(plane(adj_gmu<N>() + 2 * i), b),
                           load3<R>(plane(adj_gmu<N>() + 2 * i + 1), b)));
    const D pm = w.psimu[(long long)i * n + x];
    lpm[i] = D(a[(long long)(adj_psimu<N>() + i) * n + x]) + lmu / psih;
    if (!psi_floor) lpsi -= lmu * pm / (psih * psih);
  }
  lpsi += rho * lpr;
#pragma unroll
  for (int i = 0; i < N - 1; ++i) E[i] = D(wet[(long long)i * n + x]);
  E[N - 1] = 0.0;
  // phi mu_i (eq. 2.14): bulk, gradient and wetting terms
  D lL[N], lW[N], lE[N];
#pragma unroll
  for (int j = 0; j < N; ++j) lL[j] = lW[j] = lE[j] = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    D bulk = 0.0, curv = 0.0;
    const D g2i = gprime2(C[i]);
    const D gi = gprime(C[i]);
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (j != i) {
        bulk += kd.beta2[i][j] * (gi - gprime(C[i] + C[j]));
        const D g2ij = gprime2(C[i] + C[j]);
        curv += kd.beta2[i][j] * (g2i - g2ij);
        lC[j] -= psi * lpm[i] * kd.beta2[i][j] * g2ij;
        lL[j] += kd.grad34[i][j] * lpm[i];
        lW[j] += kd.wet3[i][j] * lpm[i];
      }
    lC[i] += psi * lpm[i] * curv;
    lpsi += bulk * lpm[i];
  }
  // W_j = sum_{q != j} c_jq C_j C_q, c_jq = (s_jN E_j - s_qN E_q) / s_jq
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int q = 0; q < N; ++q)
      if (q != j) {
        const D cjq = (kd.sigN[j] * E[j] - kd.sigN[q] * E[q]) * kd.inv_sig[j][q];
        lC[j] += lW[j] * cjq * C[q];
        lC[q] += lW[j] * cjq * C[j];
        const D lc = lW[j] * C[j] * C[q];
        lE[j] += kd.sigN[j] * kd.inv_sig[j][q] * lc;
        lE[q] -= kd.sigN[q] * kd.inv_sig[j][q] * lc;
      }
  R* aw = ab.a;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    aw[(long long)(adj_C<N>() + i) * n + x] = R(lC[i]);
    aw[(long long)(adj_L<N>() + i) * n + x] = R(lL[i]);
  }
#pragma unroll
  for (int i = 0; i < N - 1; ++i) ab.gE[(long long)i * n + x] += lE[i];
  ab.gpsi[x] += lpsi;
}

// ---------------------------------------------------------------------------
// div(psi grad C_j) and C_i = phi C_i / sum_j phi C_j transposed; the phase
// population adjoint
// ---------------------------------------------------------------------------
template <int N, class S, class R>
__global__ __launch_bounds__(kThreads) void k_adj_pop(Coef<double> kd,
                                                      const S* psi_f, AdjWork w,
                                                      AdjBufs<R> ab) {
  using D = double;
  const long long n = kd.n;
  const long long x = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (x >= n) return;
  const int gx = int(x % kd.nx), gy = int(x / kd.nx);
  const Nb3 b = nb3(gx, gy, kd.nx, kd.ny);
  const P3<D> ps = load3<D>(psi_f, b);
  D lC[N], C[N], lpsi = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const P3<D> al = load3<D>(ab.a + (long long)(adj_L<N>() + j) * n, b);
    const P3<D> cp = load3<D>(w.C + (long long)j * n, b);
    C[j] = cp.v[1][1];
    // the two-point operator is symmetric: its transpose is itself
    lC[j] = D(ab.a[(long long)(adj_C<N>() + j) * n + x]) + div_psi_grad3(ps, al);
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx)
        if (dx || dy)
          lpsi += wdiv(dx, dy) * (al.v[1][1] - al.v[dy + 1][dx + 1]) *
                  (cp.v[dy + 1][dx + 1] - cp.v[1][1]);
  }
  const D tot = w.tot[x];
  D lpc[N];
  if (tot > kd.psi_min) {
    D s = 0.0;
#pragma unroll
    for (int k2 = 0; k2 < N; ++k2) s += lC[k2] * C[k2];
#pragma unroll
    for (int i = 0; i < N; ++i) lpc[i] = (lC[i] - s) / tot;
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) lpc[i] = lC[i] / kd.psi_min;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const R l = R(D(ab.a[(long long)(adj_psiC<N>() + i) * n + x]) + lpc[i]);
    // phi C_i = f^i_0(x) + sum_{p >= 1} f^i_p(x - c_p)
    ab.lfA[(long long)(i * Q) * n + x] += l;
#pragma unroll
    for (int p = 1; p < Q; ++p) ab.lfA[(long long)(i * Q + p) * n + b.pull(p)] += l;
  }
  ab.gpsi[x] += lpsi;
}

// ---------------------------------------------------------------------------
// Objective, seed and final gradients
// ---------------------------------------------------------------------------
constexpr int kRedWaves = kThreads / 64;

// Partial sums of w(x) phi C_k(x) and phi C_k(x) over a strided slice per
// block (float64, wavefront shuffles, then LDS): part[2 b], part[2 b + 1].
template <class S>
__global__ __launch_bounds__(kThreads) void k_adj_wsum(Coef<double> kd,
                                                       AdjFwd<S> fw, int phase,
                                                       const double* wgt,
                                                       double* part) {
  const long long n = kd.n;
  double sw = 0.0, sm = 0.0;
  const long long stride = (long long)gridDim.x * kThreads;
  for (long long x = (long long)blockIdx.x * kThreads + threadIdx.x; x < n;
       x += stride) {
    const int gx = int(x % kd.nx), gy = int(x / kd.nx);
    const Nb3 b = nb3(gx, gy, kd.nx, kd.ny);
    S mv = S(0);
    for (int p = 1; p < Q; ++p)
      mv += phase_plane(fw.f, phase, p, Q, n)[b.pull(p)];
    const double pc = fw.f0[(long long)phase * n + x] + double(mv);
    sw += wgt[x] * pc;
    sm += pc;
  }
  for (int off = 32; off > 0; off >>= 1) {
    sw += __shfl_xor(sw, off);
    sm += __shfl_xor(sm, off);
  }
  __shared__ double red[kRedWaves][2];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    red[wave][0] = sw;
    red[wave][1] = sm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int v = 0; v < kRedWaves; ++v) {
      a += red[v][0];
      c += red[v][1];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = c;
  }
}

// lambda^T: dJ / d(stored phase-k population) = (w(x) - J) / M at the node
// whose phi C_k it forms (x for the rest population, x + c_p for p >= 1).
template <class R>
__global__ __launch_bounds__(kThreads) void k_adj_seed(Coef<double> kd,
                                                       int phase,
                                                       const double* wgt,
                                                       double J, double M,
                                                       R* lf) {
  const long long n = kd.n;
  const long long x = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (x >= n) return;
  const int gx = int(x % kd.nx), gy = int(x / kd.nx);
  const Nb3 b = nb3(gx, gy, kd.nx, kd.ny);
  const R v = R((wgt[x] - J) / M);
  lf[(long long)(phase * Q) * n + x] = v;
  for (int p = 1; p < Q; ++p) lf[(long long)(phase * Q + p) * n + b.pull(p)] = v;
}

// E_i = cos theta_iN |grad psi|: dJ/dcos = dJ/dE |grad psi|; and the
// vector field whose negative divergence carries the grad psi adjoint back
// to psi: the accumulated grad psi adjoint plus
// sum_i dJ/dE_i cos theta_iN grad psi / |grad psi| (0 where grad psi = 0).
template <class S>
__global__ __launch_bounds__(kThreads) void k_adj_finish1(Coef<double> kd,
                                                          int nm1,
                                                          const S* psi_f,
                                                          const S* wet,
                                                          const double* gE,
                                                          double* ggpsi,
                                                          double* gcos) {
  const long long n = kd.n;
  const long long x = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (x >= n) return;
  const int gx = int(x % kd.nx), gy = int(x / kd.nx);
  const Nb3 b = nb3(gx, gy, kd.nx, kd.ny);
  const P3<double> ps = load3<double>(psi_f, b);
  const double g0 = gx3(ps), g1 = gy3(ps);
  const double s = g0 * g0 + g1 * g1;
  const double mag = sqrt(s);
  double coef = 0.0;
  for (int i = 0; i < nm1; ++i) {
    const double ge = gE[(long long)i * n + x];
    gcos[(long long)i * n + x] = ge * mag;
    // cos theta_iN / |grad psi| = E_i / |grad psi|^2
    if (s > 0.0) coef += ge * double(wet[(long long)i * n + x]) / s;
  }
  ggpsi[x] += coef * g0;
  ggpsi[n + x] += coef * g1;
}

// The same from the float64 psi and cosines: dE_i / d(grad psi) =
// cos theta_iN grad psi / |grad psi|.
__global__ __launch_bounds__(kThreads) void k_adj_finish1_f64(
    Coef<double> kd, int nm1, const double* psi64, const double* cos64,
    const double* gE, double* ggpsi, double* gcos) {
  const long long n = kd.n;
  const long long x = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (x >= n) return;
  const int gx = int(x % kd.nx), gy = int(x / kd.nx);
  const Nb3 b = nb3(gx, gy, kd.nx, kd.ny);
  const P3<double> ps = load3<double>(psi64, b);
  const double g0 = gx3(ps), g1 = gy3(ps);
  const double mag = sqrt(g0 * g0 + g1 * g1);
  double coef = 0.0;
  for (int i = 0; i < nm1; ++i) {
    const double ge = gE[(long long)i * n + x];
    gcos[(long long)i * n + x] = ge * mag;
    if (mag > 0.0) coef += ge * cos64[(long long)i * n + x] / mag;
  }
  ggpsi[x] += coef * g0;
  ggpsi[n + x] += coef * g1;
}

__global__ __launch_bounds__(kThreads) void k_adj_finish2(Coef<double> kd,
                                                          const double* ggpsi,
                                                          const double* gpsi,
                                                          double* out) {
  const long long n = kd.n;
  const long long x = (long long)blockIdx.x * kThreads + threadIdx.x;
  if (x >= n) return;
  const int gx = int(x % kd.nx), gy = int(x / kd.nx);
  const Nb3 b = nb3(gx, gy, kd.nx, kd.ny);
  out[x] = gpsi[x] + grad_T(load3<double>(ggpsi, b), load3<double>(ggpsi + n, b));
}

inline unsigned blocks_for(long long n) {
  return unsigned((n + kThreads - 1) / kThreads);
}

template <int N, class S>
hipError_t adj_step_n(const Coef<double>& kd, const AdjFwd<S>& fw,
                      const S* psi, const S* wet, const AdjWork& w,
                      const AdjBufs<double>& ab, hipStream_t st) {
  const dim3 g(blocks_for(kd.n)), t(kThreads);
  hipLaunchKernelGGL((k_adj_frac<N, S>), g, t, 0, st, kd, fw, psi, w);
  hipLaunchKernelGGL((k_adj_mu<N, S>), g, t, 0, st, kd, psi, wet, w);
  hipLaunchKernelGGL((k_adj_node<N, S, double>), g, t, 0, st, kd, kd, fw, psi,
                     w, ab);
  hipLaunchKernelGGL((k_adj_mid<N, S, double>), g, t, 0, st, kd, psi, wet, w,
                     ab);
  hipLaunchKernelGGL((k_adj_pop<N, S, double>), g, t, 0, st, kd, psi, w, ab);
  return hipGetLastError();
}

}  // namespace

template <class S>
hipError_t launch_adj_step(int nphase, const Coef<double>& kd,
                           const AdjFwd<S>& fw, const S* psi, const S* wet,
                           const AdjWork& w, const AdjBufs<double>& ab,
                           hipStream_t st) {
  switch (nphase) {
    case 2:
      return adj_step_n<2, S>(kd, fw, psi, wet, w, ab, st);
    case 3:
      return adj_step_n<3, S>(kd, fw, psi, wet, w, ab, st);
    case 4:
      return adj_step_n<4, S>(kd, fw, psi, wet, w, ab, st);
    default:
      return hipErrorInvalidValue;
  }
}

template <class S>
hipError_t launch_adj_wsum(const Coef<double>& kd, const AdjFwd<S>& fw,
                           int phase, const double* wgt, double* part,
                           int nblocks, hipStream_t st) {
  hipLaunchKernelGGL((k_adj_wsum<S>), dim3(nblocks), dim3(kThreads), 0, st, kd,
                     fw, phase, wgt, part);
  return hipGetLastError();
}

hipError_t launch_adj_seed(const Coef<double>& kd, int phase,
                           const double* wgt, double J, double M, double* lf,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_adj_seed<double>), dim3(blocks_for(kd.n)),
                     dim3(kThreads), 0, st, kd, phase, wgt, J, M, lf);
  return hipGetLastError();
}

template <class S>
hipError_t launch_adj_finish(const Coef<double>& kd, int nm1, const S* psi,
                             const S* wet, const double* psi64,
                             const double* cos64, const double* gE,
                             double* ggpsi, const double* gpsi, double* gcos,
                             double* gpsi_out, hipStream_t st) {
  const dim3 g(blocks_for(kd.n)), t(kThreads);
  if (psi64 && cos64)
    hipLaunchKernelGGL(k_adj_finish1_f64, g, t, 0, st, kd, nm1, psi64, cos64,
                       gE, ggpsi, gcos);
  else
    hipLaunchKernelGGL((k_adj_finish1<S>), g, t, 0, st, kd, nm1, psi, wet, gE,
                       ggpsi, gcos);
  hipLaunchKernelGGL(k_adj_finish2, g, t, 0, st, kd, ggpsi, gpsi, gpsi_out);
  return hipGetLastError();
}

#define DDCC_ADJ_INST(S)                                                       \
  template hipError_t launch_adj_step<S>(int, const Coef<double>&,            \
                                         const AdjFwd<S>&, const S*,          \
                                         const S*, const AdjWork&,            \
                                         const AdjBufs<double>&,              \
                                         hipStream_t);                        \
  template hipError_t launch_adj_wsum<S>(const Coef<double>&,                 \
                                         const AdjFwd<S>&, int,               \
                                         const double*, double*, int,         \
                                         hipStream_t);                        \
  template hipError_t launch_adj_finish<S>(                                   \
      const Coef<double>&, int, const S*, const S*, const double*,            \
      const double*, const double*, double*, const double*, double*, double*, \
      hipStream_t);
DDCC_ADJ_INST(double)
DDCC_ADJ_INST(float)

}  // namespace ddcc
