// Fused 3D DD-CCLB step for gfx950: D3Q15 phase sets, D3Q19 flow set.
//
// 2.5-D tiling: a workgroup owns a TX x TY column of nodes (TX = 64, one
// wavefront per row) and marches up a block of ZB planes. Rolling LDS
// windows hold, per plane, the volume fractions C_i and psi on the tile plus
// a 2-node xy halo (4 planes), the chemical potentials mu_i on the tile plus
// a 1-node halo (3 planes) and the lagged flux tensor T (3 planes). Every
// z-iteration computes one new C plane, one new mu plane and one plane of
// output nodes, so each plane's C and mu are evaluated once per workgroup
// column (plus the 2-plane ramp at each end of the block).
//
// Per output node the work is that of the 2D kernel with three components
// (Section 3): gradients from LDS, mobility terms (eqs. 2.5, 3.7), force and
// implicit-penalty velocity (eq. 3.13), pressure (eq. 19 with the 3D
// constants), equilibria and sources (eqs. 3.5-3.12), Hermite collision
// (eqs. 3.1-3.4) with compile-time moment tables, and pull streaming.
//
// Storage as in 2D: float64 rest populations of the phase sets in their own
// plane, g_0 stored as g_0 - rho0, history phi C_i u (3N), Y (6), P in place,
// T (xy, xz, yz) double-buffered. C, mu and psi rho are evaluated in float64.
#include <hip/hip_runtime.h>

#include "coef.hpp"
#include "collide.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "lattice.hpp"

namespace ddcc {

bool have_3d() { return true; }

namespace {

constexpr int TX = 64;

// Fixed isotropic stencil: D3Q19 weights at d0 = 1/3 (1/18 faces, 1/36
// edges) divided by c_s^2 = 1/3, i.e. 1/6 on faces and 1/12 on edges.
template <int q>
constexpr double stencil_w() {
  return (D3Q19::c[q].x * D3Q19::c[q].x + D3Q19::c[q].y * D3Q19::c[q].y +
          D3Q19::c[q].z * D3Q19::c[q].z) == 1
             ? 1.0 / 6.0
             : 1.0 / 12.0;
}

// Accessor forms: at(dx, dy, dz) returns the field at the offset; the sum
// runs over the 18 D3Q19 neighbours with compile-time offsets.
template <int a, class T, class F, int q>
__device__ inline void agrad_term(T& s, F& at) {
  constexpr int cx = D3Q19::c[q].x, cy = D3Q19::c[q].y, cz = D3Q19::c[q].z;
  constexpr int comp = a == 0 ? cx : (a == 1 ? cy : cz);
  if constexpr (comp != 0) s += T(comp * stencil_w<q>()) * at(cx, cy, cz);
}

template <int a, class T, class F, int... q>
__device__ inline T agrad_impl(F& at, std::integer_sequence<int, q...>) {
  T s = T(0);
  (agrad_term<a, T, F, q + 1>(s, at), ...);
  return s;
}

template <int a, class T, class F>
__device__ inline T agrad(F&& at) {
  return agrad_impl<a, T>(at, std::make_integer_sequence<int, 18>{});
}

template <class T, class FP, class FC, int q>
__device__ inline void alap_term(T& s, FP& ps, FC& c, T pc, T cc) {
  constexpr int cx = D3Q19::c[q].x, cy = D3Q19::c[q].y, cz = D3Q19::c[q].z;
  s += T(stencil_w<q>()) * (ps(cx, cy, cz) + pc) * (c(cx, cy, cz) - cc);
}

template <class T, class FP, class FC, int... q>
__device__ inline T alap_impl(FP& ps, FC& c, std::integer_sequence<int, q...>) {
  const T pc = ps(0, 0, 0), cc = c(0, 0, 0);
  T s = T(0);
  (alap_term<T, FP, FC, q + 1>(s, ps, c, pc, cc), ...);
  return s;
}

// div(psi grad C) in conservative two-point-flux form, accessor version.
template <class T, class FP, class FC>
__device__ inline T adiv_psi_grad(FP&& ps, FC&& c) {
  return alap_impl<T>(ps, c, std::make_integer_sequence<int, 18>{});
}

struct Nbr3 {
  int xm, xp, ym, yp, zm, zp, x, y, z, nx, ny;
  // pull: population with velocity c at (x, y, z) comes from x - c
  __device__ inline unsigned src(int cx, int cy, int cz) const {
    const int sx = cx == 1 ? xm : (cx == -1 ? xp : x);
    const int sy = cy == 1 ? ym : (cy == -1 ? yp : y);
    const int sz = cz == 1 ? zm : (cz == -1 ? zp : z);
    return (unsigned(sz) * unsigned(ny) + unsigned(sy)) * unsigned(nx) + unsigned(sx);
  }
};

__device__ inline Nbr3 make_nbr3(int gx, int gy, int gz, int nx, int ny,
                                 int nz) {
  Nbr3 b;
  b.x = gx;
  b.y = gy;
  b.z = gz;
  b.nx = nx;
  b.ny = ny;
  b.xm = gx == 0 ? nx - 1 : gx - 1;
  b.xp = gx == nx - 1 ? 0 : gx + 1;
  b.ym = gy == 0 ? ny - 1 : gy - 1;
  b.yp = gy == ny - 1 ? 0 : gy + 1;
  b.zm = gz == 0 ? nz - 1 : gz - 1;
  b.zp = gz == nz - 1 ? 0 : gz + 1;
  return b;
}

template <int N, class LF, class LG, class S, class R, int MODE, int TY, int ZB>
struct Step3D {
  using D = double;
  static constexpr int QF = LF::Q, QG = LG::Q;
  static constexpr int NT = TX * TY;
  static constexpr int HX = TX + 4, HY = TY + 4;  // C region (xy halo 2)
  static constexpr int MX = TX + 2, MY = TY + 2;  // mu region (xy halo 1)
  static constexpr int NCP = 4, NMP = 3;          // window depths

  struct Smem {
    D C[NCP][N][HY][HX];
    S psi[NCP][HY][HX];
    D mu[NMP][N][MY][MX];
    R T[NMP][3][MY][MX];
  };

  __device__ static inline int slot(int z, int m) {
    const int r = z % m;
    return r < 0 ? r + m : r;
  }

  // C plane z at region coordinates (lx, ly)
  __device__ static inline void node1(Smem& sm, const Coef<D>& k,
                                      const Bufs<S>& b, int x0, int y0, int z,
                                      int lx, int ly) {
    const int gx = wrap(x0 + lx - 2, k.nx), gy = wrap(y0 + ly - 2, k.ny);
    const int gz = wrap(z, k.nz);
    const unsigned idx = (unsigned(gz) * unsigned(k.ny) + unsigned(gy)) * unsigned(k.nx) +
                         unsigned(gx);
    const S psiS = b.psi[idx];
    const D psi = D(psiS);
    D psiC[N];
    if constexpr (MODE == MODE_INIT) {
#pragma unroll
      for (int i = 0; i < N; ++i) psiC[i] = psi * (b.inC + (long long)i * k.n)[idx];
    } else {
      const Nbr3 nb = make_nbr3(gx, gy, gz, k.nx, k.ny, k.nz);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        // phi C_i = sum_p f^i_p (Section 3): moving populations summed in
        // the storage precision, the float64 rest population added last
        const S* f = b.fA + (long long)i * QF * k.n;
        R mv = R(0);
#pragma unroll
        for (int p = 1; p < QF; ++p)
          mv += ld<S, R>(&(f + (long long)p * k.n)[nb.src(LF::c[p].x, LF::c[p].y,
                                                          LF::c[p].z)]);
        psiC[i] = (b.f0A + (long long)i * k.n)[idx] + D(mv);
      }
    }
    // C_i = phi C_i / sum_j phi C_j (keeps sum_j C_j = 1 exact)
    D tot = D(0);
#pragma unroll
    for (int i = 0; i < N; ++i) tot += psiC[i];
    const D inv = D(1) / (tot > k.psi_min ? tot : k.psi_min);
    const int s4 = slot(z, NCP);
#pragma unroll
    for (int i = 0; i < N; ++i) sm.C[s4][i][ly][lx] = psiC[i] * inv;
    sm.psi[s4][ly][lx] = psiS;
  }

  // mu plane z at mu-region coordinates (mx, my): phi mu_i (eq. 2.14)
  __device__ static inline void node2(Smem& sm, const Coef<D>& k,
                                      const Bufs<S>& b, int x0, int y0, int z,
                                      int mx, int my) {
    const int lx = mx + 1, ly = my + 1;
    const int gx = wrap(x0 + mx - 1, k.nx), gy = wrap(y0 + my - 1, k.ny);
    const int gz = wrap(z, k.nz);
    const unsigned idx = (unsigned(gz) * unsigned(k.ny) + unsigned(gy)) * unsigned(k.nx) +
                         unsigned(gx);
    const int sl[3] = {slot(z - 1, NCP), slot(z, NCP), slot(z + 1, NCP)};
    auto psi_at = [&](int dx, int dy, int dz) {
      return D(sm.psi[sl[dz + 1]][ly + dy][lx + dx]);
    };
    const D psi = psi_at(0, 0, 0);
    const D psih = psi > k.psi_min ? psi : k.psi_min;
    const D g0 = agrad<0, D>(psi_at), g1 = agrad<1, D>(psi_at),
            g2 = agrad<2, D>(psi_at);
    const D agp = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
    D C[N], L[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      auto c_at = [&](int dx, int dy, int dz) {
        return sm.C[sl[dz + 1]][j][ly + dy][lx + dx];
      };
      C[j] = c_at(0, 0, 0);
      L[j] = adiv_psi_grad<D>(psi_at, c_at);
    }
    D ct[N];
#pragma unroll
    for (int i = 0; i < N - 1; ++i) ct[i] = ld<S, D>(&(b.ct + (long long)i * k.n)[idx]);
    ct[N - 1] = D(0);
    D W[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      D acc = D(0);
#pragma unroll
      for (int q = 0; q < N; ++q)
        if (q != j) {
          const D cjq = (k.sigN[j] * ct[j] - k.sigN[q] * ct[q]) * k.inv_sig[j][q];
          acc += cjq * C[j] * C[q];
        }
      W[j] = acc;
    }
    const int s3 = slot(z, NMP);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      D bulk = D(0), grad = D(0), wet = D(0);
      const D gi = gprime(C[i]);
#pragma unroll
      for (int j = 0; j < N; ++j)
        if (j != i) {
          bulk += k.beta2[i][j] * (gi - gprime(C[i] + C[j]));
          grad += k.grad34[i][j] * L[j];
          wet += k.wet3[i][j] * W[j];
        }
      sm.mu[s3][i][my][mx] = (psi * bulk + grad + wet * agp) / psih;
    }
    if constexpr (MODE != MODE_INIT) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
        sm.T[s3][c][my][mx] = ld<S, R>(&(b.TA + (long long)c * k.n)[idx]);
    }
  }

  // Output node (tx, ty) of plane z.
  __device__ static inline void node3(const Smem& sm, const Coef<D>& kd,
                                      const Coef<R>& k, const Bufs<S>& b,
                                      int x0, int y0, int z, int tx, int ty) {
    const int gx = x0 + tx, gy = y0 + ty;
    const long long n = k.n;
    const unsigned idx = (unsigned(z) * unsigned(k.ny) + unsigned(gy)) * unsigned(k.nx) +
                         unsigned(gx);
    const int lx = tx + 2, ly = ty + 2, mx = tx + 1, my = ty + 1;
    const Nbr3 nb = make_nbr3(gx, gy, z, k.nx, k.ny, k.nz);

    const int sc[3] = {slot(z - 1, NCP), slot(z, NCP), slot(z + 1, NCP)};
    const int sm3[3] = {slot(z - 1, NMP), slot(z, NMP), slot(z + 1, NMP)};
    auto psi_at = [&](int dx, int dy, int dz) {
      return D(sm.psi[sc[dz + 1]][ly + dy][lx + dx]);
    };
    const D psi_d = psi_at(0, 0, 0);
    const R psi = R(psi_d);
    const D psih_d = psi_d > kd.psi_min ? psi_d : kd.psi_min;
    const R gpsi[3] = {R(agrad<0, D>(psi_at)), R(agrad<1, D>(psi_at)),
                       R(agrad<2, D>(psi_at))};
    // phi rho at a neighbour: psi sum_i rho_i C_i
    auto prho_at = [&](int dx, int dy, int dz) {
      D r = D(0);
#pragma unroll
      for (int i = 0; i < N; ++i)
        r += kd.rho[i] * sm.C[sc[dz + 1]][i][ly + dy][lx + dx];
      return r * psi_at(dx, dy, dz);
    };
    const R psirho = R(prho_at(0, 0, 0));
    const R gprho[3] = {R(agrad<0, D>(prho_at)), R(agrad<1, D>(prho_at)),
                        R(agrad<2, D>(prho_at))};
    R C[N], gC[N][3], mu[N], gmu[N][3];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      auto c_at = [&](int dx, int dy, int dz) {
        return sm.C[sc[dz + 1]][i][ly + dy][lx + dx];
      };
      auto mu_at = [&](int dx, int dy, int dz) {
        return sm.mu[sm3[dz + 1]][i][my + dy][mx + dx];
      };
      C[i] = R(c_at(0, 0, 0));
      gC[i][0] = R(agrad<0, D>(c_at));
      gC[i][1] = R(agrad<1, D>(c_at));
      gC[i][2] = R(agrad<2, D>(c_at));
      mu[i] = R(mu_at(0, 0, 0));
      gmu[i][0] = R(agrad<0, D>(mu_at));
      gmu[i][1] = R(agrad<1, D>(mu_at));
      gmu[i][2] = R(agrad<2, D>(mu_at));
    }
    R grho[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int a = 0; a < 3; ++a) grho[a] += k.rho[i] * gC[i][a];
    D psimu_d[N];
    R psimu[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      psimu_d[i] = D(sm.mu[sm3[1]][i][my][mx]) * psih_d;
      psimu[i] = R(psimu_d[i]);
    }
    // mass flux m^C (eq. 2.5, Section 2.2)
    R mC[3] = {R(0), R(0), R(0)};
    R Cs[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R s = R(0), sr = R(0);
#pragma unroll
      for (int q = 0; q < N; ++q)
        if (q != j) {
          s += C[q];
          sr += C[q] * (k.rho[j] - k.rho[q]);
        }
      Cs[j] = s;
      const R aa = k.m0 * C[j] * sr;
#pragma unroll
      for (int a = 0; a < 3; ++a) mC[a] -= aa * gmu[j][a];
    }

    R u[3], F[3] = {R(0), R(0), R(0)};
    R gp[QG];
    R sum_gm = R(0);
    if constexpr (MODE == MODE_INIT) {
#pragma unroll
      for (int a = 0; a < 3; ++a) u[a] = b.inU ? R((b.inU + a * n)[idx]) : R(0);
    } else {
      R j[3] = {R(0), R(0), R(0)};
#pragma unroll
      for (int p = 0; p < QG; ++p) {
        gp[p] = ld<S, R>(&(b.gA + (long long)p * n)[nb.src(LG::c[p].x, LG::c[p].y,
                                                            LG::c[p].z)]);
        if (p > 0) sum_gm += gp[p];
        if (LG::c[p].x) j[0] += R(LG::c[p].x) * gp[p];
        if (LG::c[p].y) j[1] += R(LG::c[p].y) * gp[p];
        if (LG::c[p].z) j[2] += R(LG::c[p].z) * gp[p];
      }
      // -div T^{n-1} with T antisymmetric, components xy, xz, yz
      auto txy = [&](int dx, int dy, int dz) {
        return sm.T[sm3[dz + 1]][0][my + dy][mx + dx];
      };
      auto txz = [&](int dx, int dy, int dz) {
        return sm.T[sm3[dz + 1]][1][my + dy][mx + dx];
      };
      auto tyz = [&](int dx, int dy, int dz) {
        return sm.T[sm3[dz + 1]][2][my + dy][mx + dx];
      };
      const R divT[3] = {-agrad<1, R>(txy) - agrad<2, R>(txz),
                         agrad<0, R>(txy) - agrad<2, R>(tyz),
                         agrad<0, R>(txz) + agrad<1, R>(tyz)};
      const R Pprev = ld<S, R>(&(b.hist + (long long)(3 * N + 6) * n)[idx]);
      R Fp[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        Fp[a] = -divT[a] + Pprev * gpsi[a] + psirho * k.accel[a] +
                psi * k.force[a];
#pragma unroll
        for (int i = 0; i < N; ++i) Fp[a] += psimu[i] * gC[i][a];
      }
      const R pen = (R(1) - psi) * k.lam;
      const R den = R(1) / (psirho + R(0.5) * pen);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        u[a] = (j[a] + R(0.5) * Fp[a]) * den;
        F[a] = Fp[a] - pen * u[a];
      }
    }

    // Y = sym(phi m^C u): xx, xy, xz, yy, yz, zz; T = antisym: xy, xz, yz
    const R Y[6] = {psi * mC[0] * u[0],
                    R(0.5) * psi * (mC[0] * u[1] + u[0] * mC[1]),
                    R(0.5) * psi * (mC[0] * u[2] + u[0] * mC[2]),
                    psi * mC[1] * u[1],
                    R(0.5) * psi * (mC[1] * u[2] + u[1] * mC[2]),
                    psi * mC[2] * u[2]};
    const R Tn[3] = {R(0.5) * psi * (mC[0] * u[1] - u[0] * mC[1]),
                     R(0.5) * psi * (mC[0] * u[2] - u[0] * mC[2]),
                     R(0.5) * psi * (mC[1] * u[2] - u[1] * mC[2])};
    R dtY[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    if constexpr (MODE != MODE_INIT) {
#pragma unroll
      for (int q = 0; q < 6; ++q)
        dtY[q] = Y[q] - ld<S, R>(&(b.hist + (long long)(3 * N + q) * n)[idx]);
    }
    R nu = R(0);
#pragma unroll
    for (int i = 0; i < N; ++i) nu += k.nu[i] * C[i];
    const R s21 = R(1) / (k.two_over_c2mcs2 * nu + R(0.5));
    const R s22 = R(1) / (k.inv_cs2 * nu + R(0.5));
    // A = phi rho u u + Y, index map as Y
    const R A[6] = {psirho * u[0] * u[0] + Y[0], psirho * u[0] * u[1] + Y[1],
                    psirho * u[0] * u[2] + Y[2], psirho * u[1] * u[1] + Y[3],
                    psirho * u[1] * u[2] + Y[4], psirho * u[2] * u[2] + Y[5]};
    R psiP, P;
    if constexpr (MODE == MODE_INIT) {
      P = b.inP ? R(b.inP[idx]) : R(0);
      psiP = psi * P;
    } else {
      const R s0eq = -k.wg[0] * (A[0] + A[3] + A[5]) * k.inv_c2mcs2;
      const R ugr = u[0] * grho[0] + u[1] * grho[1] + u[2] * grho[2];
      const R ugpr = u[0] * gprho[0] + u[1] * gprho[1] + u[2] * gprho[2];
      psiP = k.pref * (sum_gm + k.cgr * psi * ugr +
                       k.halfK * (dtY[0] + dtY[3] + dtY[5]) +
                       k.KH * (s21 - R(2)) / s21 * ugpr + s0eq);
      P = R(D(psiP) / psih_d);
    }
    const R uvec[3] = {u[0], u[1], u[2]};
    if constexpr (MODE == MODE_MOMENTS) {
#pragma unroll
      for (int i = 0; i < N; ++i) (b.outC + i * n)[idx] = double(C[i]);
#pragma unroll
      for (int a = 0; a < 3; ++a) (b.outU + a * n)[idx] = double(uvec[a]);
      b.outP[idx] = double(P);
      return;
    }

    // ---- flow set: equilibrium (eqs. 3.8, 3.11), source (3.10, 3.12) ---
    if constexpr (MODE == MODE_INIT) {
#pragma unroll
      for (int p = 0; p < QG; ++p) {
        const int cx = LG::c[p].x, cy = LG::c[p].y, cz = LG::c[p].z;
        const R h2 = (A[0] * (R(cx * cx) - k.cs2) + A[3] * (R(cy * cy) - k.cs2) +
                      A[5] * (R(cz * cz) - k.cs2)) *
                         k.h2diag +
                     (A[1] * R(cx * cy) + A[2] * R(cx * cz) + A[4] * R(cy * cz)) *
                         k.h2off;
        R geq = k.wg[p] * ((psiP + psirho * (R(cx) * u[0] + R(cy) * u[1] +
                                               R(cz) * u[2])) *
                               k.inv_cs2 +
                           h2);
        if (p == 0) geq -= psiP * k.inv_cs2;  // stored as g_0 - rho0
        // the buffers hold pre-streaming values: place g_p(x) where the
        // next pull reads it, at x - c_p
        (b.gB + (long long)p * n)[nb.src(cx, cy, cz)] = S(geq);
      }
    } else {
      const R ub = u[0] * gprho[0] + u[1] * gprho[1] + u[2] * gprho[2];
      // M^{2G} (eq. 3.12) with the scalar u.grad(phi rho) on the diagonal
      const R M[6] = {
          dtY[0] + R(2) * k.cs2 * u[0] * gprho[0] + k.one_m3cs2 * ub,
          dtY[1] + k.cs2 * (u[0] * gprho[1] + gprho[0] * u[1]),
          dtY[2] + k.cs2 * (u[0] * gprho[2] + gprho[0] * u[2]),
          dtY[3] + R(2) * k.cs2 * u[1] * gprho[1] + k.one_m3cs2 * ub,
          dtY[4] + k.cs2 * (u[1] * gprho[2] + gprho[1] * u[2]),
          dtY[5] + R(2) * k.cs2 * u[2] * gprho[2] + k.one_m3cs2 * ub};
      const R a0 = psi * (u[0] * grho[0] + u[1] * grho[1] + u[2] * grho[2]);
      const R J[3] = {psirho * u[0], psirho * u[1], psirho * u[2]};
      R del[QG];
      collide_flow<LG>(gp, J, A, psiP, M, a0, F, s21, s22, k.sg, k.q4, k.cs2,
                       k.inv_cs2, del);
#pragma unroll
      for (int p = 0; p < QG; ++p) (b.gB + (long long)p * n)[idx] = S(gp[p] - del[p]);
    }

    // ---- phase sets: equilibrium (3.5), source (3.6, 3.7), collision ---
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const S* fsrc = b.fA + (long long)i * QF * n;
      S* fdst = b.fB + (long long)i * QF * n;
      if constexpr (MODE == MODE_INIT) {
        const D psiC = psi_d * (b.inC + (long long)i * n)[idx];
        const R X[3] = {R(psiC) * u[0], R(psiC) * u[1], R(psiC) * u[2]};
        const R em = k.eta[i] * psimu[i];
        // f^eq_0 = (w_0 - 1) eta phi mu + phi C (float64 rest plane)
        (b.f0B + (long long)i * n)[idx] =
            (kd.wf[0] - D(1)) * kd.eta[i] * psimu_d[i] + psiC;
#pragma unroll
        for (int p = 1; p < QF; ++p) {
          const int cx = LF::c[p].x, cy = LF::c[p].y, cz = LF::c[p].z;
          const R feq = k.wf[p] * (em + (R(cx) * X[0] + R(cy) * X[1] +
                                         R(cz) * X[2]) * k.inv_cs2);
          (fdst + (long long)p * n)[nb.src(cx, cy, cz)] = S(feq);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) (b.hist + (long long)(3 * i + a) * n)[idx] = S(X[a]);
      } else {
        // own phi C_i = sum of the pulled populations (Section 3): moving
        // populations summed in the storage precision, the float64 rest
        // population added last
        R fp[QF];
        fp[0] = R(0);
        R mv = R(0);
#pragma unroll
        for (int p = 1; p < QF; ++p) {
          fp[p] = ld<S, R>(&(fsrc + (long long)p * n)[nb.src(LF::c[p].x, LF::c[p].y,
                                                              LF::c[p].z)]);
          mv += fp[p];
        }
        const D f0 = (b.f0A + (long long)i * n)[idx];
        const R psiC = R(f0 + D(mv));
        const R X[3] = {psiC * u[0], psiC * u[1], psiC * u[2]};
        // S_i (eq. 3.7) and V = d_t(phi C_i u) + c_s^2 eta (mu grad psi - S_i)
        R V[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          R sa = (C[i] * Cs[i] - R(1)) * gmu[i][a];
#pragma unroll
          for (int j = 0; j < N; ++j)
            if (j != i) sa -= C[i] * C[j] * gmu[j][a];
          const R dX = X[a] - ld<S, R>(&(b.hist + (long long)(3 * i + a) * n)[idx]);
          V[a] = dX + k.cs2 * k.eta[i] * (mu[i] * gpsi[a] - psi * sa);
        }
        R del[QF];
        collide_phase<LF>(fp, k.eta[i] * psimu[i], X, V, k.sf, k.cs2, del);
        (b.f0B + (long long)i * n)[idx] = f0 - D(del[0]);
#pragma unroll
        for (int p = 1; p < QF; ++p) (fdst + (long long)p * n)[idx] = S(fp[p] - del[p]);
#pragma unroll
        for (int a = 0; a < 3; ++a) (b.hist + (long long)(3 * i + a) * n)[idx] = S(X[a]);
      }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) (b.hist + (long long)(3 * N + q) * n)[idx] = S(Y[q]);
    (b.hist + (long long)(3 * N + 6) * n)[idx] = S(P);
#pragma unroll
    for (int c = 0; c < 3; ++c) (b.TB + (long long)c * n)[idx] = S(Tn[c]);
  }

  __device__ static void run(const Coef<D>& kd, const Coef<R>& k,
                             const Bufs<S>& b) {
    __shared__ Smem sm;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int z0 = blockIdx.z * ZB;
    const int z1 = z0 + ZB < k.nz ? z0 + ZB : k.nz;
    const bool own = (x0 + tx < k.nx) && (y0 + ty < k.ny);
    for (int zc = z0 - 2; zc <= z1 + 1; ++zc) {
      for (int r = tid; r < HX * HY; r += NT) {
        const int ly = r / HX, lx = r - ly * HX;
        node1(sm, kd, b, x0, y0, zc, lx, ly);
      }
      __syncthreads();
      const int zm = zc - 1;
      if (zm >= z0 - 1) {
        for (int r = tid; r < MX * MY; r += NT) {
          const int my = r / MX, mx = r - my * MX;
          node2(sm, kd, b, x0, y0, zm, mx, my);
        }
      }
      __syncthreads();
      const int zo = zc - 2;
      if (zo >= z0 && own) node3(sm, kd, k, b, x0, y0, zo, tx, ty);
      __syncthreads();
    }
  }
};

template <int N, class S, class R, int MODE, int TY, int ZB>
__global__ __launch_bounds__(TX* TY) void k_step3d(Coef<double> kd, Coef<R> k,
                                                    Bufs<S> b) {
  Step3D<N, D3Q15, D3Q19, S, R, MODE, TY, ZB>::run(kd, k, b);
}

constexpr int kZB = 16;

template <int N, class S, class R, int MODE>
hipError_t launch_3(const Coef<double>& kd, const Coef<R>& k, const Bufs<S>& b,
                    int ty, hipStream_t st) {
  const unsigned gx = (k.nx + TX - 1) / TX;
  const unsigned gz = (k.nz + kZB - 1) / kZB;
  if (ty == 2) {
    dim3 g(gx, (k.ny + 1) / 2, gz);
    hipLaunchKernelGGL((k_step3d<N, S, R, MODE, 2, kZB>), g, dim3(TX * 2), 0,
                       st, kd, k, b);
  } else {
    dim3 g(gx, (k.ny + 3) / 4, gz);
    hipLaunchKernelGGL((k_step3d<N, S, R, MODE, 4, kZB>), g, dim3(TX * 4), 0,
                       st, kd, k, b);
  }
  return hipGetLastError();
}

template <int N, class S, class R>
hipError_t launch_mode3(int mode, const Coef<double>& kd, const Coef<R>& k,
                        const Bufs<S>& b, int ty, hipStream_t st) {
  switch (mode) {
    case MODE_STEP:
      return launch_3<N, S, R, MODE_STEP>(kd, k, b, ty, st);
    case MODE_INIT:
      return launch_3<N, S, R, MODE_INIT>(kd, k, b, ty, st);
    default:
      return launch_3<N, S, R, MODE_MOMENTS>(kd, k, b, ty, st);
  }
}

}  // namespace

template <class S, class R>
hipError_t launch_3d(int nphase, int mode, const Coef<double>& kd,
                     const Coef<R>& k, const Bufs<S>& b, int tx, int ty,
                     hipStream_t st) {
  (void)tx;
  switch (nphase) {
    case 2:
      return launch_mode3<2, S, R>(mode, kd, k, b, ty, st);
    case 3:
      return launch_mode3<3, S, R>(mode, kd, k, b, ty, st);
    default:
      return hipErrorInvalidValue;
  }
}

template hipError_t launch_3d<double, double>(int, int, const Coef<double>&,
                                              const Coef<double>&,
                                              const Bufs<double>&, int, int,
                                              hipStream_t);
template hipError_t launch_3d<float, float>(int, int, const Coef<double>&,
                                            const Coef<float>&,
                                            const Bufs<float>&, int, int,
                                            hipStream_t);

}  // namespace ddcc
