// Fused 2D DD-CCLB step for gfx950 (D2Q9 phase and flow sets).
//
// One workgroup owns a TX x TY tile of nodes (TX = 64: one wavefront per
// row, so every global access of a row is one coalesced 64-wide load).
// Per step and node (Section 3, in order):
//   phase 1  pull f^i from buffer A and sum: phi C_i, C_i = phi C_i / psi_hat
//            on the tile plus a 2-node halo, into LDS with psi and phi rho;
//   phase 2  chemical potential phi mu_i (eq. 2.14) on the tile plus a
//            1-node halo (needs div(psi grad C_j) from LDS and the static
//            wetting weights sum_k cos theta^k_iN |grad psi_k|),
//            mu_i = phi mu_i / psi_hat into LDS, and the lagged flux tensor T;
//   phase 3  own node: gradients from LDS, mobility terms (eqs. 2.5, 3.7),
//            force and velocity (eq. 3.13 with the implicit penalty),
//            pressure (eq. 19), equilibria and sources (eqs. 3.5-3.12),
//            Hermite-moment collision (eqs. 3.1-3.4) in registers, and the
//            post-collision populations written to buffer B at the node
//            (pull streaming: the next step reads them at x - c_p).
// The same kernel body also serves initialisation (populations at
// equilibrium) and moment read-out, selected by a template parameter.
//
// Storage S (float/double), collision arithmetic R (float/double). The
// volume fractions, chemical potentials and the LDS fields (psi, phi rho, C,
// mu) are always float64: mu is a small difference of O(beta) terms near
// equilibrium, and the rest populations of the phase sets (O(1), about
// phi C_i) are kept in a float64 plane f0 so that phase mass does not drift
// with float32 rounding. The rest population of the flow set is stored as
// g_0 - rho0 (small); every other population is raw in S. History per node: phi C_i u (N x 2), the symmetric flux tensor Y
// (xx, xy, yy) and P, updated in place; the antisymmetric tensor T (xy) is
// double-buffered because neighbours read it.
#include <hip/hip_runtime.h>

#include "coef.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "collide.hpp"
#include "lattice.hpp"

namespace ddcc {

namespace {

constexpr int TX = 64;

// Fixed isotropic finite-difference stencil (D2Q9 weights at d0 = 1/3
// divided by its c_s^2 = 1/3): 1/3 on the axes, 1/12 on the diagonals.
// Neighbour order in the 3x3 patch arrays: [dy+1][dx+1].
template <class R>
struct Patch {
  R v[3][3];
};

template <class R>
__device__ inline R grad_x(const Patch<R>& p) {
  return R(1.0 / 3.0) * (p.v[1][2] - p.v[1][0]) +
         R(1.0 / 12.0) * ((p.v[2][2] + p.v[0][2]) - (p.v[2][0] + p.v[0][0]));
}

template <class R>
__device__ inline R grad_y(const Patch<R>& p) {
  return R(1.0 / 3.0) * (p.v[2][1] - p.v[0][1]) +
         R(1.0 / 12.0) * ((p.v[2][2] + p.v[2][0]) - (p.v[0][2] + p.v[0][0]));
}

// div(psi grad C) in conservative two-point-flux form.
template <class R>
__device__ inline R div_psi_grad(const Patch<R>& psi, const Patch<R>& C) {
  const R pc = psi.v[1][1], cc = C.v[1][1];
  R axis = (psi.v[1][2] + pc) * (C.v[1][2] - cc) +
           (psi.v[1][0] + pc) * (C.v[1][0] - cc) +
           (psi.v[2][1] + pc) * (C.v[2][1] - cc) +
           (psi.v[0][1] + pc) * (C.v[0][1] - cc);
  R diag = (psi.v[2][2] + pc) * (C.v[2][2] - cc) +
           (psi.v[2][0] + pc) * (C.v[2][0] - cc) +
           (psi.v[0][2] + pc) * (C.v[0][2] - cc) +
           (psi.v[0][0] + pc) * (C.v[0][0] - cc);
  return R(1.0 / 3.0) * axis + R(1.0 / 12.0) * diag;
}

template <class R, int W, int H>
__device__ inline Patch<R> patch(const R (&a)[H][W], int x, int y) {
  Patch<R> p;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) p.v[dy + 1][dx + 1] = a[y + dy][x + dx];
  return p;
}

// Box a tile belongs to: nx x ny nodes starting at node `off` of planes of
// n nodes (one box: off = 0, n = nx ny; an instance of a batch: its offset in
// planes that hold every instance). The single-box kernel passes its Coef for
// the halo stages (same members nx, ny, n and off = 0), so the sizes stay
// kernel arguments there.
struct Grid {
  int nx, ny;
  long long n;
  unsigned off;
};

// Pull: population p at (gx, gy) comes from (gx - c_px, gy - c_py).
struct Nbr {
  int xm, xp, ym, yp, x, y, nx;
  unsigned off;
  __device__ inline unsigned src(int cx, int cy) const {
    const int sx = cx == 1 ? xm : (cx == -1 ? xp : x);
    const int sy = cy == 1 ? ym : (cy == -1 ? yp : y);
    return off + unsigned(sy * nx + sx);
  }
};

__device__ inline Nbr make_nbr(int gx, int gy, int nx, int ny, unsigned off) {
  Nbr b;
  b.off = off;
  b.x = gx;
  b.y = gy;
  b.nx = nx;
  b.xm = gx == 0 ? nx - 1 : gx - 1;
  b.xp = gx == nx - 1 ? 0 : gx + 1;
  b.ym = gy == 0 ? ny - 1 : gy - 1;
  b.yp = gy == ny - 1 ? 0 : gy + 1;
  return b;
}

template <int N, class Pop, class S, class R, int MODE, int TY>
struct Step2D {
  static constexpr bool STREAM = MODE == MODE_STREAM;  // nontemporal stores
  using D = double;
  static constexpr int Q = 9;
  static constexpr int NT = TX * TY;
  static constexpr int HX = TX + 4, HY = TY + 4;  // C region (halo 2)
  static constexpr int MX = TX + 2, MY = TY + 2;  // mu region (halo 1)
  static constexpr int RING1 = HX * HY - TX * TY;
  static constexpr int RING2 = MX * MY - TX * TY;

  struct Smem {
    D psi[HY][HX];
    D prho[HY][HX];
    D C[N][HY][HX];
    D mu[N][MY][MX];
    R T[MY][MX];
  };

  __device__ static inline void ring1(int r, int& lx, int& ly) {
    if (r < 2 * HX) {
      ly = r / HX;
      lx = r - ly * HX;
    } else if (r < 4 * HX) {
      const int q = r - 2 * HX;
      ly = HY - 2 + q / HX;
      lx = q - (q / HX) * HX;
    } else {
      const int q = r - 4 * HX;
      ly = 2 + (q >> 2);
      const int c = q & 3;
      lx = c < 2 ? c : HX - 4 + c;
    }
  }

  __device__ static inline void ring2(int r, int& mx, int& my) {
    if (r < MX) {
      my = 0;
      mx = r;
    } else if (r < 2 * MX) {
      my = MY - 1;
      mx = r - MX;
    } else {
      const int q = r - 2 * MX;
      my = 1 + (q >> 1);
      mx = (q & 1) ? MX - 1 : 0;
    }
  }

  // Phase 1 at C-region coordinates (lx, ly).
  // Kept: the pulled moving populations (own node) are written to `keep`
  // and handed on to phase 3 in registers instead of being loaded again.
  using Keep = R[N][Q];
  template <bool KEPT = false, class G>
  __device__ static inline void node1(Smem& sm, const Coef<D>& k,
                                      const Bufs<Pop, S>& b, const G& gd, int x0,
                                      int y0, int lx,
                                      int ly, D* psiC_out, Keep* keep = nullptr) {
    const int gx = wrap(x0 + lx - 2, gd.nx), gy = wrap(y0 + ly - 2, gd.ny);
    const unsigned idx = gd.off + unsigned(gy * gd.nx + gx);
    const D psi = D(ldp(b.psi, idx));
    D rho = D(0);
    if constexpr (MODE == MODE_INIT) {
#pragma unroll
      for (int i = 0; i < N; ++i) psiC_out[i] = psi * ldp(b.inC + (long long)(i) * gd.n, idx);
    } else {
      const Nbr nb = make_nbr(gx, gy, gd.nx, gd.ny, gd.off);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        // phi C_i = sum_p f^i_p (Section 3); the rest population does not
        // move and lives in the float64 plane
        // moving populations summed in the storage precision, the float64
        // rest population added last
        R mv = R(0);
#pragma unroll
        for (int p = 1; p < Q; ++p) {
          const R v = R(ldp(phase_plane(b.fA, i, p, Q, gd.n),
                            nb.src(D2Q9::c[p].x, D2Q9::c[p].y)));
          if constexpr (KEPT) (*keep)[i][p] = v;
          mv += v;
        }
        psiC_out[i] = ldp(b.f0A + (long long)(i) * gd.n, idx) + D(mv);
      }
    }
    // C_i = phi C_i / sum_j phi C_j: equal to phi C_i / phi while the
    // constraint sum_j C_j = 1 of Section 2.1 holds, and keeps it exact.
    D tot = D(0);
#pragma unroll
    for (int i = 0; i < N; ++i) tot += psiC_out[i];
    const D inv = D(1) / (tot > k.psi_min ? tot : k.psi_min);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const D C = psiC_out[i] * inv;
      sm.C[i][ly][lx] = C;
      rho += k.rho[i] * C;
    }
    sm.psi[ly][lx] = psi;
    sm.prho[ly][lx] = psi * rho;
  }

  // Phase-2 inputs from global memory, issued in phase 1: the lagged T
  // into LDS and the wetting weights E_i into registers.
  template <class G>
  __device__ static inline void load2(Smem& sm, const Bufs<Pop, S>& b,
                                      const G& gd, int x0, int y0, int mx,
                                      int my, S* E) {
    const int gx = wrap(x0 + mx - 1, gd.nx), gy = wrap(y0 + my - 1, gd.ny);
    const unsigned idx = gd.off + unsigned(gy * gd.nx + gx);
#pragma unroll
    for (int i = 0; i < N - 1; ++i) E[i] = ldp(b.wet + (long long)(i) * gd.n, idx);
    if constexpr (MODE != MODE_INIT) sm.T[my][mx] = R(ldp(b.TA, idx));
  }

  // Phase 2 at mu-region coordinates (mx, my): phi mu_i (eq. 2.14).
  template <bool PRE2 = false, class G>
  __device__ static inline void node2(Smem& sm, const Coef<D>& k,
                                      const Bufs<Pop, S>& b, const G& gd, int x0,
                                      int y0, int mx,
                                      int my, D* psimu_out,
                                      const S* E = nullptr) {
    const int lx = mx + 1, ly = my + 1;
    const int gx = wrap(x0 + mx - 1, gd.nx), gy = wrap(y0 + my - 1, gd.ny);
    const unsigned idx = gd.off + unsigned(gy * gd.nx + gx);
    const Patch<D> ps = patch(sm.psi, lx, ly);
    const D psi = ps.v[1][1];
    const D psih = psi > k.psi_min ? psi : k.psi_min;
    const D ipsih = D(1) / psih;  // one division for the N phases
    D C[N], L[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const Patch<D> cp = patch(sm.C[j], lx, ly);
      C[j] = cp.v[1][1];
      L[j] = div_psi_grad(ps, cp);
    }
    // wetting weights sum_k cos theta^k_jq |grad psi_k| from the stored
    // E_i = sum_k cos theta^k_iN |grad psi_k| (eq. 2.9 is linear in them)
    D ct[N];
#pragma unroll
    for (int i = 0; i < N - 1; ++i)
      ct[i] = PRE2 ? D(E[i]) : D(ldp(b.wet + (long long)(i) * gd.n, idx));
    ct[N - 1] = D(0);
    D W[N];  // sum_{q != j} (sum_k cos theta^k_jq |grad psi_k|) C_j C_q
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
#pragma unroll
    for (int i = 0; i < N; ++i) {
      D bulk = D(0), grad = D(0), wet = D(0);
      const D gi = gprime(C[i]);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if (j != i) {
          bulk += k.beta2[i][j] * (gi - gprime(C[i] + C[j]));
          grad += k.grad34[i][j] * L[j];
          wet += k.wet3[i][j] * W[j];
        }
      }
      const D pm = psi * bulk + grad + wet;
      psimu_out[i] = pm;
      sm.mu[i][my][mx] = pm * ipsih;
    }
    if constexpr (MODE != MODE_INIT && !PRE2) sm.T[my][mx] = R(ldp(b.TA, idx));
  }

  __device__ static void run(const Coef<D>& kd, const Coef<R>& k,
                             const Bufs<Pop, S>& b) {
    // Tile order. Workgroup w is dispatched to XCD w % 8. The row-major tile
    // list is cut into spans of 8 chunks of CH full-width tile rows (64 node
    // rows), and inside a span each XCD takes one contiguous range, about one
    // chunk. The halo lines shared by neighbouring tiles (left, right and
    // below) then sit in one XCD's L2 instead of being fetched by two or
    // three, and the eight XCDs work on adjacent chunks, so the pages in use
    // stay few.
    __shared__ Smem sm;
    int x0, y0;
    {
      constexpr unsigned CH = TY >= 64 ? 1u : 64u / TY;
      const unsigned gx = gridDim.x, total = gx * gridDim.y;
      const unsigned lin = blockIdx.y * gx + blockIdx.x;
      const unsigned span = 8u * CH * gx;
      const unsigned base = lin / span * span;
      const unsigned m = min(span, total - base);
      const unsigned l = lin - base, q = m / 8u, r = m % 8u;
      const unsigned xc = l % 8u, j = l / 8u;
      const unsigned t = base + (xc < r ? xc * (q + 1u) + j
                                        : r * (q + 1u) + (xc - r) * q + j);
      x0 = int(t % gx) * TX;
      y0 = int(t / gx) * TY;
    }
    if constexpr (MODE == MODE_STREAM) {
      body(sm, kd, k, b, Grid{k.nx, k.ny, k.n, 0u}, x0, y0);
      return;
    }
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    D psiC[N], psimu_d[N], dummy[N];
    // The own node's pulled populations stay in registers from phase 1 to
    // the collision (phase 3 would otherwise load them again, after the
    // whole chunk's phase-1 traffic has gone through L2). In float64 that
    // takes the kernel to 187 VGPRs and two waves per SIMD, and is still
    // faster (same GPU, 512^2 N = 3: 48.3 -> 42.4 us; 2048^2: 825 -> 815 us).
    constexpr bool KEEP = MODE == MODE_STEP || MODE == MODE_STREAM;
    Keep fown;
    node1<KEEP>(sm, kd, b, kd, x0, y0, tx + 2, ty + 2, psiC, &fown);
    for (int r = tid; r < RING1; r += NT) {
      int lx, ly;
      ring1(r, lx, ly);
      node1(sm, kd, b, kd, x0, y0, lx, ly, dummy);
    }
    __syncthreads();
    node2(sm, kd, b, kd, x0, y0, tx + 1, ty + 1, psimu_d);
    for (int r = tid; r < RING2; r += NT) {
      int mx, my;
      ring2(r, mx, my);
      node2(sm, kd, b, kd, x0, y0, mx, my, dummy);
    }
    __syncthreads();
    if (x0 + tx < k.nx && y0 + ty < k.ny)
      node3<KEEP>(sm, kd, k, b, Grid{k.nx, k.ny, k.n, 0u}, x0, y0, tx, ty,
                  psiC, psimu_d, &fown);
  }

  // The tile of a streaming step (grids larger than the memory-side cache).
  // Vector-memory completion is counted in issue order, so each phase above
  // waits for its own loads: the pulls in phase 1, T and the wetting weights
  // in phase 2, the flow populations and history in phase 3. Here phase 2's
  // loads go out in phase 1 (T straight into LDS, E_i into registers) and
  // the own node's phase-3 loads before the second barrier, so a tile waits
  // on memory once in phase 1 and once, overlapped by the barrier and the
  // LDS gradients, in phase 3. Same GPU, same results bit for bit, ms per
  // step: porous 2048^2 N = 3 FP32 0.389 -> 0.377, FP64 0.758 -> 0.709;
  // disk 2048^2 N = 2 FP32 0.283 -> 0.265, FP64 0.499 -> 0.496; disk 4096^2
  // FP32 1.136 -> 1.080, FP64 2.130 -> 2.158; 256 batched instances 0.400
  // -> 0.381. On the cache-resident 512^2 box the plain order stays (porous
  // FP32 22.7 -> 24.0 us, FP64 41.3 -> 42.1 us with this one). Phase 2's
  // loads moved alone: porous 2048^2 FP32 0.394, FP64 0.746, batch 0.395.
  __device__ static inline void body(Smem& sm, const Coef<D>& kd,
                                     const Coef<R>& k, const Bufs<Pop, S>& b,
                                     const Grid& gd, int x0, int y0) {
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    constexpr bool KEEP = MODE == MODE_STEP || MODE == MODE_STREAM;
    constexpr int PER2 = (RING2 + NT - 1) / NT;
    D psiC[N], psimu_d[N], dummy[N];
    S Eown[N], Er[PER2][N];
    Keep fown;
    node1<KEEP>(sm, kd, b, gd, x0, y0, tx + 2, ty + 2, psiC, &fown);
    load2(sm, b, gd, x0, y0, tx + 1, ty + 1, Eown);
#pragma unroll
    for (int u = 0; u < PER2; ++u) {
      const int r = tid + u * NT;
      if (r < RING2) {
        int mx, my;
        ring2(r, mx, my);
        load2(sm, b, gd, x0, y0, mx, my, Er[u]);
      }
    }
    for (int r = tid; r < RING1; r += NT) {
      int lx, ly;
      ring1(r, lx, ly);
      node1(sm, kd, b, gd, x0, y0, lx, ly, dummy);
    }
    __syncthreads();
    node2<true>(sm, kd, b, gd, x0, y0, tx + 1, ty + 1, psimu_d, Eown);
#pragma unroll
    for (int u = 0; u < PER2; ++u) {
      const int r = tid + u * NT;
      if (r < RING2) {
        int mx, my;
        ring2(r, mx, my);
        node2<true>(sm, kd, b, gd, x0, y0, mx, my, dummy, Er[u]);
      }
    }
    const bool own = x0 + tx < gd.nx && y0 + ty < gd.ny;
    In3 in3;
    if (own) load3(b, gd, x0, y0, tx, ty, in3);
    __syncthreads();
    if (own)
      node3<KEEP, true>(sm, kd, k, b, gd, x0, y0, tx, ty, psiC, psimu_d,
                        &fown, &in3);
  }

  // One TX x TY tile with its corner at (x0, y0) of box gd. Every thread of
  // the workgroup passes both barriers; there is no early return, so a
  // workgroup can process several tiles in a row.
  __device__ static void tile(const Coef<D>& kd, const Coef<R>& k,
                              const Bufs<Pop, S>& b, const Grid& gd, int x0,
                              int y0) {
    __shared__ Smem sm;
    if constexpr (MODE == MODE_STREAM) {
      body(sm, kd, k, b, gd, x0, y0);
      return;
    }
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    D psiC[N], psimu_d[N], dummy[N];
    // pulled populations kept in registers as in run() (float64, 256
    // instances, 64 x 8 tiles: 0.829 -> 0.756 ms per step, same GPU)
    constexpr bool KEEP = MODE == MODE_STEP || MODE == MODE_STREAM;
    Keep fown;
    node1<KEEP>(sm, kd, b, gd, x0, y0, tx + 2, ty + 2, psiC, &fown);
    for (int r = tid; r < RING1; r += NT) {
      int lx, ly;
      ring1(r, lx, ly);
      node1(sm, kd, b, gd, x0, y0, lx, ly, dummy);
    }
    __syncthreads();
    node2(sm, kd, b, gd, x0, y0, tx + 1, ty + 1, psimu_d);
    for (int r = tid; r < RING2; r += NT) {
      int mx, my;
      ring2(r, mx, my);
      node2(sm, kd, b, gd, x0, y0, mx, my, dummy);
    }
    __syncthreads();
    if (x0 + tx < gd.nx && y0 + ty < gd.ny)
      node3<KEEP>(sm, kd, k, b, gd, x0, y0, tx, ty, psiC, psimu_d, &fown);
  }

  // Phase-3 inputs of the own node from global memory (flow populations,
  // history, float64 rest populations), issued before the second barrier.
  struct In3 {
    Pop g[Q];
    S hX[2 * N], hY[3], hP;
    D f0[N];
  };
  __device__ static inline void load3(const Bufs<Pop, S>& b, const Grid& gd,
                                      int x0, int y0, int tx, int ty, In3& in) {
    if constexpr (MODE != MODE_INIT) {
      const int gx = x0 + tx, gy = y0 + ty;
      const long long n = gd.n;
      const unsigned idx = gd.off + unsigned(gy * gd.nx + gx);
      const Nbr nb = make_nbr(gx, gy, gd.nx, gd.ny, gd.off);
#pragma unroll
      for (int p = 0; p < Q; ++p)
        in.g[p] = ldp(b.gA + (long long)p * n, nb.src(D2Q9::c[p].x, D2Q9::c[p].y));
#pragma unroll
      for (int q = 0; q < 2 * N; ++q) in.hX[q] = ldo<STREAM>(b.hist + (long long)q * n, idx);
#pragma unroll
      for (int q = 0; q < 3; ++q) in.hY[q] = ldo<STREAM>(b.hist + (long long)(2 * N + q) * n, idx);
      in.hP = ldo<STREAM>(b.hist + (long long)(2 * N + 3) * n, idx);
#pragma unroll
      for (int i = 0; i < N; ++i) in.f0[i] = ldp(b.f0A + (long long)(i) * n, idx);
    }
  }

  // Phase 3 for the own node (x0 + tx, y0 + ty) of the tile.
  template <bool KEPT = false, bool PRE3 = false>
  __device__ static inline void node3(const Smem& sm, const Coef<D>& kd,
                                      const Coef<R>& k, const Bufs<Pop, S>& b,
                                      const Grid& gd, int x0, int y0, int tx,
                                      int ty, const D* psiC, const D* psimu_d,
                                      const Keep* kept = nullptr,
                                      const In3* in3 = nullptr) {
    R psimu[N];
#pragma unroll
    for (int i = 0; i < N; ++i) psimu[i] = R(psimu_d[i]);

    const int gx = x0 + tx, gy = y0 + ty;
    const long long n = gd.n;
    const unsigned idx = gd.off + unsigned(gy * gd.nx + gx);
    const int lx = tx + 2, ly = ty + 2, mx = tx + 1, my = ty + 1;

    // ---- gradients from LDS -------------------------------------------
    const Patch<D> ps = patch(sm.psi, lx, ly);
    const R psi = R(ps.v[1][1]);
    const D psih_d = ps.v[1][1] > kd.psi_min ? ps.v[1][1] : kd.psi_min;
    const R gpsi[2] = {R(grad_x(ps)), R(grad_y(ps))};
    const Patch<D> pr = patch(sm.prho, lx, ly);
    const R psirho = R(pr.v[1][1]);
    const R gprho[2] = {R(grad_x(pr)), R(grad_y(pr))};
    R C[N], gC[N][2], mu[N], gmu[N][2];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const Patch<D> cp = patch(sm.C[i], lx, ly);
      C[i] = R(cp.v[1][1]);
      gC[i][0] = R(grad_x(cp));
      gC[i][1] = R(grad_y(cp));
      const Patch<D> mp = patch(sm.mu[i], mx, my);
      mu[i] = R(mp.v[1][1]);
      gmu[i][0] = R(grad_x(mp));
      gmu[i][1] = R(grad_y(mp));
    }
    R grho[2] = {R(0), R(0)};
#pragma unroll
    for (int i = 0; i < N; ++i) {
      grho[0] += k.rho[i] * gC[i][0];
      grho[1] += k.rho[i] * gC[i][1];
    }
    // mass flux m^C = -sum_ij rho_i M_ij grad mu_j, with
    // sum_i rho_i M_ij = m0 C_j sum_{k != j} C_k (rho_j - rho_k)  (eq. 2.5)
    R mC[2] = {R(0), R(0)};
    R Cs[N];  // sum_{k != j} C_k
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
      const R a = k.m0 * C[j] * sr;
      mC[0] -= a * gmu[j][0];
      mC[1] -= a * gmu[j][1];
    }

    R u[2], F[2] = {R(0), R(0)};
    R gp[Q];
    R sum_gm = R(0);
    const Nbr nb = make_nbr(gx, gy, gd.nx, gd.ny, gd.off);
    if constexpr (MODE == MODE_INIT) {
      u[0] = b.inU ? R(ldp(b.inU, idx)) : R(0);
      u[1] = b.inU ? R(ldp(b.inU + n, idx)) : R(0);
    } else {
      R j[2] = {R(0), R(0)};
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        if constexpr (PRE3)
          gp[p] = R(in3->g[p]);
        else
          gp[p] = R(ldp(b.gA + (long long)p * n, nb.src(D2Q9::c[p].x, D2Q9::c[p].y)));
        if (p > 0) sum_gm += gp[p];
        if (D2Q9::c[p].x) j[0] += R(D2Q9::c[p].x) * gp[p];
        if (D2Q9::c[p].y) j[1] += R(D2Q9::c[p].y) * gp[p];
      }
      // force (eq. 3.13): -div T^{n-1} + sum_i phi mu_i grad C_i
      //                   + P^{n-1} grad psi + psi (rho a + G)
      const Patch<R> tp = patch(sm.T, mx, my);
      const R Pprev = R(PRE3 ? in3->hP : ldo<STREAM>(b.hist + (long long)(2 * N + 3) * n, idx));
      R Fp[2];
      Fp[0] = grad_y(tp) + Pprev * gpsi[0] + psirho * k.accel[0] +
              psi * k.force[0];
      Fp[1] = -grad_x(tp) + Pprev * gpsi[1] + psirho * k.accel[1] +
              psi * k.force[1];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        Fp[0] += psimu[i] * gC[i][0];
        Fp[1] += psimu[i] * gC[i][1];
      }
      // phi rho u = j + F/2 with F = Fp - (1 - psi) lam u, solved for u
      const R pen = (R(1) - psi) * k.lam;
      const R den = R(1) / (psirho + R(0.5) * pen);
      u[0] = (j[0] + R(0.5) * Fp[0]) * den;
      u[1] = (j[1] + R(0.5) * Fp[1]) * den;
      F[0] = Fp[0] - pen * u[0];
      F[1] = Fp[1] - pen * u[1];
    }

    // symmetric / antisymmetric flux tensors of phi m^C u
    const R Y[3] = {psi * mC[0] * u[0],
                    R(0.5) * psi * (mC[0] * u[1] + u[0] * mC[1]),
                    psi * mC[1] * u[1]};
    const R Tn = R(0.5) * psi * (mC[0] * u[1] - u[0] * mC[1]);
    R dtY[3] = {R(0), R(0), R(0)};
    if constexpr (MODE != MODE_INIT) {
#pragma unroll
      for (int q = 0; q < 3; ++q)
        dtY[q] = Y[q] - R(PRE3 ? in3->hY[q] : ldo<STREAM>(b.hist + (long long)(2 * N + q) * n, idx));
    }

    // local flow rates from nu (eq. 16)
    R nu = R(0);
#pragma unroll
    for (int i = 0; i < N; ++i) nu += k.nu[i] * C[i];
    const R s21 = R(1) / (k.two_over_c2mcs2 * nu + R(0.5));
    const R s22 = R(1) / (k.inv_cs2 * nu + R(0.5));

    R psiP, P;
    const R A[3] = {psirho * u[0] * u[0] + Y[0], psirho * u[0] * u[1] + Y[1],
                    psirho * u[1] * u[1] + Y[2]};
    if constexpr (MODE == MODE_INIT) {
      P = b.inP ? R(ldp(b.inP, idx)) : R(0);
      psiP = psi * P;
    } else {
      // eq. (19)
      const R s0eq = -k.wg[0] * (A[0] + A[2]) * k.inv_c2mcs2;
      const R ugr = u[0] * grho[0] + u[1] * grho[1];
      const R ugpr = u[0] * gprho[0] + u[1] * gprho[1];
      psiP = k.pref * (sum_gm + k.cgr * psi * ugr + k.halfK * (dtY[0] + dtY[2]) +
                       k.KH * (s21 - R(2)) / s21 * ugpr + s0eq);
      P = R(D(psiP) / psih_d);
    }

    if constexpr (MODE == MODE_MOMENTS) {
#pragma unroll
      for (int i = 0; i < N; ++i) stp<STREAM>(b.outC + (long long)(i) * n, idx, double(C[i]));
      stp<STREAM>(b.outU, idx, double(u[0]));
      stp<STREAM>(b.outU + n, idx, double(u[1]));
      stp<STREAM>(b.outP, idx, double(P));
      return;
    }

    // ---- flow set: equilibrium (eqs. 3.8, 3.11), source (3.10, 3.12) ---
    if constexpr (MODE == MODE_INIT) {
#pragma unroll
      for (int p = 0; p < Q; ++p) {
        const int cx = D2Q9::c[p].x, cy = D2Q9::c[p].y;
        const R h2 = (A[0] * (R(cx * cx) - k.cs2) + A[2] * (R(cy * cy) - k.cs2)) *
                         k.h2diag +
                     A[1] * R(cx * cy) * k.h2off;
        R geq = k.wg[p] * ((psiP + R(cx) * psirho * u[0] + R(cy) * psirho * u[1]) *
                               k.inv_cs2 + h2);
        if (p == 0) geq -= psiP * k.inv_cs2;  // stored as g_0 - rho0
        // the buffers hold pre-streaming values: place g_p(x) where the
        // next pull reads it, at x - c_p
        stp<STREAM>(b.gB + (long long)(p) * n, nb.src(cx, cy), Pop(geq));
      }
    } else {
      const R ub = u[0] * gprho[0] + u[1] * gprho[1];
      // M^{2G} (eq. 3.12), scalar u.grad(phi rho) on the diagonal
      const R M[3] = {dtY[0] + R(2) * k.cs2 * u[0] * gprho[0] + k.one_m3cs2 * ub,
                      dtY[1] + k.cs2 * (u[0] * gprho[1] + gprho[0] * u[1]),
                      dtY[2] + R(2) * k.cs2 * u[1] * gprho[1] + k.one_m3cs2 * ub};
      const R a0 = psi * (u[0] * grho[0] + u[1] * grho[1]);
      R del[Q];
      collide_flow<D2Q9>(gp, A, psiP, M, a0, F, s21, s22, k.sg, k.q4, k.cs2,
                         k.inv_cs2, del);
#pragma unroll
      for (int p = 0; p < Q; ++p) stp<STREAM>(b.gB + (long long)(p) * n, idx, Pop(gp[p] - del[p]));
    }

    // ---- phase sets: equilibrium (3.5), source (3.6, 3.7), collision ---
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const R X[2] = {R(psiC[i]) * u[0], R(psiC[i]) * u[1]};
      const R em = k.eta[i] * psimu[i];
      if constexpr (MODE == MODE_INIT) {
        D comp = D(0);
#pragma unroll
        for (int p = 1; p < Q; ++p) {
          const int cx = D2Q9::c[p].x, cy = D2Q9::c[p].y;
          const R feq = k.wf[p] * (em + (R(cx) * X[0] + R(cy) * X[1]) * k.inv_cs2);
          stp<STREAM>(phase_plane(b.fB, i, p, Q, n), nb.src(cx, cy), narrow<Pop>(feq, comp));
        }
        // f^eq_0 = (w_0 - 1) eta phi mu + phi C (float64 rest plane), plus
        // the storage rounding of the moving populations
        stp<STREAM>(b.f0B + (long long)(i) * n, idx,
            (kd.wf[0] - D(1)) * kd.eta[i] * psimu_d[i] + psiC[i] + comp);
      } else {
        // S_i = psi [(C_i sum_{j!=i} C_j - 1) grad mu_i
        //            - C_i sum_{j != i} C_j grad mu_j]     (eq. 3.7)
        R Sx = (C[i] * Cs[i] - R(1)) * gmu[i][0];
        R Sy = (C[i] * Cs[i] - R(1)) * gmu[i][1];
#pragma unroll
        for (int j = 0; j < N; ++j)
          if (j != i) {
            Sx -= C[i] * C[j] * gmu[j][0];
            Sy -= C[i] * C[j] * gmu[j][1];
          }
        Sx *= psi;
        Sy *= psi;
        const R dX0 = X[0] - R(PRE3 ? in3->hX[2 * i] : ldo<STREAM>(b.hist + (long long)(2 * i) * n, idx));
        const R dX1 = X[1] - R(PRE3 ? in3->hX[2 * i + 1] : ldo<STREAM>(b.hist + (long long)(2 * i + 1) * n, idx));
        const R V[2] = {dX0 + k.cs2 * k.eta[i] * (mu[i] * gpsi[0] - Sx),
                        dX1 + k.cs2 * k.eta[i] * (mu[i] * gpsi[1] - Sy)};
        R fp[Q];
        fp[0] = R(0);
#pragma unroll
        for (int p = 1; p < Q; ++p)
          if constexpr (KEPT)
            fp[p] = (*kept)[i][p];
          else
            fp[p] = R(ldp(phase_plane(b.fA, i, p, Q, n),
                          nb.src(D2Q9::c[p].x, D2Q9::c[p].y)));
        R del[Q];
        collide_phase<D2Q9>(fp, em, X, V, k.sf, k.cs2, del);
        D comp = D(0);
#pragma unroll
        for (int p = 1; p < Q; ++p)
          stp<STREAM>(phase_plane(b.fB, i, p, Q, n), idx,
              narrow<Pop>(fp[p] - del[p], comp));
        stp<STREAM>(b.f0B + (long long)(i) * n, idx,
            (PRE3 ? in3->f0[i] : ldp(b.f0A + (long long)(i) * n, idx)) - D(del[0]) + comp);
      }
      stp<STREAM>(b.hist + (long long)(2 * i) * n, idx, S(X[0]));
      stp<STREAM>(b.hist + (long long)(2 * i + 1) * n, idx, S(X[1]));
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) stp<STREAM>(b.hist + (long long)(2 * N + q) * n, idx, S(Y[q]));
    stp<STREAM>(b.hist + (long long)(2 * N + 3) * n, idx, S(P));
    stp<STREAM>(b.TB, idx, S(Tn));
  }
};

// kd, k: the context's coefficients in device memory. Passed by value the
// two structs (about 1.5 KB) overflow the scalar registers and spill into
// VGPR lanes; read through __restrict__ pointers they are scalar loads where
// used (512^2 N = 3, same GPU: FP32 23.3 -> 22.4 us, FP64 49.2 -> 48.3 us).
template <int N, class Pop, class S, class R, int MODE, int TY>
__global__ __launch_bounds__(TX* TY) void k_step2d(
    const Coef<double>* __restrict__ kd, const Coef<R>* __restrict__ k,
    Bufs<Pop, S> b) {
  Step2D<N, Pop, S, R, MODE, TY>::run(*kd, *k, b);
}

template <int N, class Pop, class S, class R, int MODE>
hipError_t launch_ty(const Coef<double>& kd, const Coef<R>& k,
                     const Bufs<Pop, S>& b, int ty, hipStream_t st) {
  (void)kd;
  const Coef<double>* dk = static_cast<const Coef<double>*>(b.coef_d);
  const Coef<R>* dr = static_cast<const Coef<R>*>(b.coef_r);
  if (!dk || !dr) return hipErrorInvalidValue;
  switch (ty) {
    case 4: {
      dim3 g((k.nx + TX - 1) / TX, (k.ny + 3) / 4);
      hipLaunchKernelGGL((k_step2d<N, Pop, S, R, MODE, 4>), g, dim3(TX * 4), 0, st,
                         dk, dr, b);
      break;
    }
    case 16: {
      dim3 g((k.nx + TX - 1) / TX, (k.ny + 15) / 16);
      hipLaunchKernelGGL((k_step2d<N, Pop, S, R, MODE, 16>), g, dim3(TX * 16), 0, st,
                         dk, dr, b);
      break;
    }
    case 2: {
      dim3 g((k.nx + TX - 1) / TX, (k.ny + 1) / 2);
      hipLaunchKernelGGL((k_step2d<N, Pop, S, R, MODE, 2>), g, dim3(TX * 2), 0, st,
                         dk, dr, b);
      break;
    }
    default: {
      dim3 g((k.nx + TX - 1) / TX, (k.ny + 7) / 8);
      hipLaunchKernelGGL((k_step2d<N, Pop, S, R, MODE, 8>), g, dim3(TX * 8), 0, st,
                         dk, dr, b);
      break;
    }
  }
  return hipGetLastError();
}

template <int N, class Pop, class S, class R>
hipError_t launch_mode(int mode, const Coef<double>& kd, const Coef<R>& k,
                       const Bufs<Pop, S>& b, int ty, hipStream_t st) {
  switch (mode) {
    case MODE_STEP:
      return launch_ty<N, Pop, S, R, MODE_STEP>(kd, k, b, ty, st);
    case MODE_STREAM:
      return launch_ty<N, Pop, S, R, MODE_STREAM>(kd, k, b, ty, st);
    case MODE_INIT:
      return launch_ty<N, Pop, S, R, MODE_INIT>(kd, k, b, ty, st);
    default:
      return launch_ty<N, Pop, S, R, MODE_MOMENTS>(kd, k, b, ty, st);
  }
}

// ---- batches of independent boxes ----------------------------------------
// Persistent step kernel over a work queue of (instance, tile) entries:
// each workgroup takes the next tile index from *counter until the queue is
// empty, then exits. Tiles of one step are independent, so no workgroup ever
// waits for another; the counter must be zero at launch.
// kds / ks: the coefficients of each instance (per-instance parameters),
// read where they are used with the instance index of the tile, which is
// uniform, so the reads are scalar.
template <int N, class Pop, class S, class R, int MODE, int TY>
__global__ __launch_bounds__(TX* TY) void k_step2d_batch(
    const Coef<double>* __restrict__ kds, const Coef<R>* __restrict__ ks,
    Bufs<Pop, S> b, const BatchTile* tiles, const BatchInst* insts,
    unsigned ntiles, unsigned* counter) {
  __shared__ unsigned next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1u);
    __syncthreads();
    // the same value in every lane: make it a scalar so that the tile and
    // instance descriptors are scalar loads
    const unsigned t = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
    if (t >= ntiles) break;
    const BatchTile tl = tiles[t];
    const BatchInst in = insts[tl.inst];
    const Coef<R>& k = ks[tl.inst];
    Step2D<N, Pop, S, R, MODE, TY>::tile(
        kds[tl.inst], k, b, Grid{in.nx, in.ny, k.n, unsigned(in.off)}, tl.x0,
        tl.y0);
  }
}

template <int N, class Pop, class S, class R, int TY>
hipError_t launch_batch_n(int mode, const Coef<double>* kd, const Coef<R>* k,
                          const Bufs<Pop, S>& b, const BatchTile* tiles,
                          const BatchInst* insts, unsigned ntiles,
                          unsigned* counter, int nblocks, hipStream_t st) {
  const dim3 g(nblocks), blk(TX * TY);
  if (mode == MODE_INIT)
    hipLaunchKernelGGL((k_step2d_batch<N, Pop, S, R, MODE_INIT, TY>), g, blk, 0,
                       st, kd, k, b, tiles, insts, ntiles, counter);
  else if (mode == MODE_MOMENTS)
    hipLaunchKernelGGL((k_step2d_batch<N, Pop, S, R, MODE_MOMENTS, TY>), g, blk,
                       0, st, kd, k, b, tiles, insts, ntiles, counter);
  else if (mode == MODE_STREAM)
    hipLaunchKernelGGL((k_step2d_batch<N, Pop, S, R, MODE_STREAM, TY>), g, blk,
                       0, st, kd, k, b, tiles, insts, ntiles, counter);
  else
    hipLaunchKernelGGL((k_step2d_batch<N, Pop, S, R, MODE_STEP, TY>), g, blk, 0,
                       st, kd, k, b, tiles, insts, ntiles, counter);
  return hipGetLastError();
}

template <int N, class Pop, class S, class R, int TY>
int batch_blocks_n() {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(
              &k_step2d_batch<N, Pop, S, R, MODE_STEP, TY>),
          TX * TY, 0) != hipSuccess)
    return 0;
  return per_cu;
}

}  // namespace

template <class Pop, class S, class R>
hipError_t launch_2d(int nphase, int mode, const Coef<double>& kd,
                     const Coef<R>& k, const Bufs<Pop, S>& b, int ty,
                     hipStream_t st) {
  switch (nphase) {
    case 2:
      return launch_mode<2, Pop, S, R>(mode, kd, k, b, ty, st);
    case 3:
      return launch_mode<3, Pop, S, R>(mode, kd, k, b, ty, st);
    case 4:
      return launch_mode<4, Pop, S, R>(mode, kd, k, b, ty, st);
    default:
      return hipErrorInvalidValue;
  }
}

template <class Pop, class S, class R>
hipError_t launch_2d_batch(int nphase, int mode, const Coef<double>* kd,
                           const Coef<R>* k,
                           const Bufs<Pop, S>& b, const BatchTile* tiles,
                           const BatchInst* insts, unsigned ntiles,
                           unsigned* counter, int nblocks, int ty,
                           hipStream_t st) {
#define DDCC_BATCH_TY(NN)                                                      \
  switch (ty) {                                                                \
    case 4:                                                                    \
      return launch_batch_n<NN, Pop, S, R, 4>(mode, kd, k, b, tiles, insts, ntiles,  \
                                               counter, nblocks, st);          \
    case 16:                                                                   \
      return launch_batch_n<NN, Pop, S, R, 16>(mode, kd, k, b, tiles, insts, ntiles, \
                                                counter, nblocks, st);         \
    default:                                                                   \
      return launch_batch_n<NN, Pop, S, R, 8>(mode, kd, k, b, tiles, insts, ntiles,  \
                                               counter, nblocks, st);          \
  }
  switch (nphase) {
    case 2:
      DDCC_BATCH_TY(2)
    case 3:
      DDCC_BATCH_TY(3)
    default:
      return hipErrorInvalidValue;
  }
#undef DDCC_BATCH_TY
}

template <class Pop, class S, class R>
int batch_blocks_per_cu(int nphase, int ty) {
  if (nphase == 2)
    return ty == 4 ? batch_blocks_n<2, Pop, S, R, 4>()
                   : (ty == 16 ? batch_blocks_n<2, Pop, S, R, 16>()
                               : batch_blocks_n<2, Pop, S, R, 8>());
  if (nphase == 3)
    return ty == 4 ? batch_blocks_n<3, Pop, S, R, 4>()
                   : (ty == 16 ? batch_blocks_n<3, Pop, S, R, 16>()
                               : batch_blocks_n<3, Pop, S, R, 8>());
  return 0;
}

#define DDCC_BATCH_INST(P, S, R)                                              \
  template hipError_t launch_2d_batch<P, S, R>(                               \
      int, int, const Coef<double>*, const Coef<R>*, const Bufs<P, S>&,       \
      const BatchTile*, const BatchInst*, unsigned, unsigned*, int, int,      \
      hipStream_t);                                                           \
  template int batch_blocks_per_cu<P, S, R>(int, int);
DDCC_BATCH_INST(double, double, double)
DDCC_BATCH_INST(float, float, float)
DDCC_BATCH_INST(_Float16, float, float)
DDCC_BATCH_INST(__bf16, float, float)
#undef DDCC_BATCH_INST

template hipError_t launch_2d<double, double, double>(
    int, int, const Coef<double>&, const Coef<double>&,
    const Bufs<double, double>&, int, hipStream_t);
template hipError_t launch_2d<float, float, float>(
    int, int, const Coef<double>&, const Coef<float>&,
    const Bufs<float, float>&, int, hipStream_t);
template hipError_t launch_2d<_Float16, float, float>(
    int, int, const Coef<double>&, const Coef<float>&,
    const Bufs<_Float16, float>&, int, hipStream_t);
template hipError_t launch_2d<__bf16, float, float>(
    int, int, const Coef<double>&, const Coef<float>&,
    const Bufs<__bf16, float>&, int, hipStream_t);

}  // namespace ddcc
