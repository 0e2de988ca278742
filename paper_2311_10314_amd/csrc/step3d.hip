// 3D DD-CCLB step for gfx950: D3Q15 or D3Q7 phase sets, D3Q19 flow set.
//
// A step is three kernels on one stream:
//   k_frac3d  pull the phase populations and sum them: phi C_i, then
//             C_i = phi C_i / sum_j phi C_j, written as a field;
//   k_mu3d    phi mu_i (eq. 2.14) from C_j and psi on the 18 D3Q19
//             neighbours (div(psi grad C_j)) and the static wetting weights,
//             mu_i = phi mu_i / psi_hat written as a field (each
//             workgroup marches a column of tiles in z with three planes of
//             C_j and psi in LDS);
//   k_step3d  gradients of C_i, mu_i, psi and psi rho and the divergence of
//             the lagged flux tensor T from the neighbours, mobility terms
//             (eqs. 2.5, 3.7), force and implicit-penalty velocity (eq.
//             3.13), pressure (eq. 19 with the 3D constants), Hermite-moment
//             collision (eqs. 3.1-3.12) of all sets in registers, and the
//             post-collision populations written at the node (pull
//             streaming).
// k_frac3d runs one node per thread. k_mu3d and k_step3d give each
// workgroup a 64 x TY column of nodes over ZB planes and march it in z with
// three planes of their stencil fields (C_j, psi; and mu_i for the step) in
// an LDS ring, so each value is fetched once per tile instead of once per
// neighbour. The C and mu fields (in the field type: float64 for FP64
// contexts, float32 otherwise) cost 4 N values of traffic per node beyond
// the fused minimum; in return no halo is recomputed. (A single z-marching
// kernel that pulls the phase populations of a two-node halo and evaluates
// the chemical potential in LDS was 2.2x slower, and one that only folds
// the chemical potential into the node update 1.25x slower: at the two
// waves per SIMD the node update's registers allow, those stages'
// latencies are not hidden.)
//
// Storage as in 2D: float64 rest populations of the phase sets in their own
// plane, g_0 stored as g_0 - rho0, T (xy, xz, yz) double-buffered. The
// history (in place) holds the factors of the lagged terms rather than the
// products: phi C_i (N), u (3), m^C (3) and P, N + 7 fields instead of the
// 3N + 7 of phi C_i u, Y and P. The next step forms phi C_i u and
// Y = sym(phi m^C u) from them with the expressions (and so the roundings)
// of the step that stored them. C, psi rho and the node update's use of mu
// are evaluated in float64 in every precision; k_mu3d computes the chemical
// potential in the field type (float32 in float contexts, whose C and psi
// fields it reads are float32 already; 256^3 FP32 2.51 -> 2.47 ms per step,
// FP16 1.70 -> 1.67 ms, same GPU, the 1000-step errors unchanged).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "coef.hpp"
#include "collide.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "lattice.hpp"

namespace ddcc {

bool have_3d() { return true; }

namespace {

constexpr int TX = 64;
using G19 = D3Q19;

// Fixed isotropic stencil: D3Q19 weights at d0 = 1/3 (1/18 faces, 1/36
// edges) divided by c_s^2 = 1/3, i.e. 1/6 on faces and 1/12 on edges.
template <int q>
constexpr double stencil_w() {
  return (G19::c[q].x * G19::c[q].x + G19::c[q].y * G19::c[q].y +
          G19::c[q].z * G19::c[q].z) == 1
             ? 1.0 / 6.0
             : 1.0 / 12.0;
}

template <int a, int q>
constexpr int comp() {
  return a == 0 ? G19::c[q].x : (a == 1 ? G19::c[q].y : G19::c[q].z);
}

// Values of a field at the node (v[0]) and its 18 neighbours x + c_q.
template <class T>
struct Star {
  T v[19];
};

template <int a, class T>
__device__ inline T sgrad(const Star<T>& s) {
  T r = T(0);
  static_for<1, 19>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int c = comp<a, q>();
    if constexpr (c != 0) r += T(c * stencil_w<q>()) * s.v[q];
  });
  return r;
}

// div(psi grad C) in conservative two-point-flux form.
template <class T>
__device__ inline T sdiv_psi_grad(const Star<T>& ps, const Star<T>& c) {
  T r = T(0);
  static_for<1, 19>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    r += T(stencil_w<q>()) * (ps.v[q] + ps.v[0]) * (c.v[q] - c.v[0]);
  });
  return r;
}

// History fields of the 3D step (in place, field type S): phi C_i (N), u
// (3), m^C (3), P.
constexpr int H3_C = 0;
template <int N>
constexpr int H3_U = N;
template <int N>
constexpr int H3_M = N + 3;
template <int N>
constexpr int H3_P = N + 6;

// Y = sym(phi m^C u), packed xx, xy, xz, yy, yz, zz. The step that stores
// m^C and u and the next one, which forms its Y again from them, evaluate
// the same expressions.
template <class R>
__device__ inline void sym_flux(R psi, const R* m, const R* u, R* Y) {
  Y[0] = psi * m[0] * u[0];
  Y[1] = R(0.5) * psi * (m[0] * u[1] + u[0] * m[1]);
  Y[2] = R(0.5) * psi * (m[0] * u[2] + u[0] * m[2]);
  Y[3] = psi * m[1] * u[1];
  Y[4] = R(0.5) * psi * (m[1] * u[2] + u[1] * m[2]);
  Y[5] = psi * m[2] * u[2];
}

// Periodic neighbourhood of node (x, y, z).
struct Nbr3 {
  int xs[3], ys[3], zs[3];  // coordinate at offset -1, 0, +1
  int nx, ny;
  // node at x + (dx, dy, dz)
  __device__ inline unsigned at(int dx, int dy, int dz) const {
    return (unsigned(zs[dz + 1]) * unsigned(ny) + unsigned(ys[dy + 1])) *
               unsigned(nx) +
           unsigned(xs[dx + 1]);
  }
  // pull source of the population moving with c: x - c
  __device__ inline unsigned src(int cx, int cy, int cz) const {
    return at(-cx, -cy, -cz);
  }
};

__device__ inline Nbr3 make_nbr3(int x, int y, int z, int nx, int ny, int nz) {
  Nbr3 b;
  b.nx = nx;
  b.ny = ny;
  b.xs[1] = x;
  b.ys[1] = y;
  b.zs[1] = z;
  b.xs[0] = x == 0 ? nx - 1 : x - 1;
  b.xs[2] = x == nx - 1 ? 0 : x + 1;
  b.ys[0] = y == 0 ? ny - 1 : y - 1;
  b.ys[2] = y == ny - 1 ? 0 : y + 1;
  b.zs[0] = z == 0 ? nz - 1 : z - 1;
  b.zs[2] = z == nz - 1 ? 0 : z + 1;
  return b;
}

template <class T, class S>
__device__ inline Star<T> gather(const S* plane, const Nbr3& nb) {
  Star<T> s;
  static_for<0, 19>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    s.v[q] = T(ldp(plane, nb.at(G19::c[q].x, G19::c[q].y, G19::c[q].z)));
  });
  return s;
}

// Node of this thread; false outside the grid. The chip sweeps the box
// plane by plane (workgroups are dispatched z-major; giving each XCD its own
// slab of planes was slower). Within a plane, workgroup w runs on XCD w % 8,
// and each XCD takes one contiguous band of tile rows (when the plane's tile
// count is a multiple of 8), so the rows shared by neighbouring tiles of a
// plane, and of the planes above and below, stay in one L2 (1.4-2.4 %
// faster at 256^3, measured).
template <int TY>
__device__ inline bool node_of(const int nx, const int ny, int& x, int& y,
                               int& z) {
  z = int(blockIdx.z);
  const unsigned gx = gridDim.x, per = gx * gridDim.y;
  unsigned bx = blockIdx.x, by = blockIdx.y;
  if (per % 8u == 0u) {
    const unsigned l = by * gx + bx, q = per / 8u;
    const unsigned t = (l % 8u) * q + l / 8u;
    bx = t % gx;
    by = t / gx;
  }
  y = int(by) * TY + int(threadIdx.x) / TX;
  x = int(bx) * TX + int(threadIdx.x) % TX;
  return x < nx && y < ny;
}

// The C and mu work fields between the kernels are kept in the field type S
// (float64 for FP64 contexts, float32 otherwise): C_i and mu_i are formed in
// float64 and rounded once when stored.
template <class S>
__device__ inline S* work_field(double* p) {
  return reinterpret_cast<S*>(p);
}

// ---- k_frac3d -------------------------------------------------------------
template <int N, class LF, class Pop, class S, class R, int MODE, int TY>
__global__ __launch_bounds__(TX* TY) void k_frac3d(Coef<double> k,
                                                    Bufs<Pop, S> b) {
  using D = double;
  constexpr int QF = LF::Q;
  int x, y, z;
  if (!node_of<TY>(k.nx, k.ny, x, y, z)) return;
  const Nbr3 nb = make_nbr3(x, y, z, k.nx, k.ny, k.nz);
  const unsigned idx = nb.at(0, 0, 0);
  D psiC[N];
  if constexpr (MODE == MODE_INIT) {
    const D psi = D(ldp(b.psi, idx));
#pragma unroll
    for (int i = 0; i < N; ++i) psiC[i] = psi * ldp(b.inC + (long long)i * k.n, idx);
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      // phi C_i = sum_p f^i_p (Section 3): moving populations summed in
      // the storage precision, the float64 rest population added last
      R mv = R(0);
      static_for<1, QF>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        mv += R(ldo<MODE == MODE_STREAM && LF::c[p].x == 0>(
            phase_plane(b.fA, i, p, QF, k.n),
                    nb.src(LF::c[p].x, LF::c[p].y, LF::c[p].z)));
      });
      psiC[i] = ldo<MODE == MODE_STREAM>(b.f0A + (long long)i * k.n, idx) + D(mv);
    }
  }
  // C_i = phi C_i / sum_j phi C_j (keeps sum_j C_j = 1 exact)
  D tot = D(0);
#pragma unroll
  for (int i = 0; i < N; ++i) tot += psiC[i];
  const D inv = D(1) / (tot > k.psi_min ? tot : k.psi_min);
#pragma unroll
  for (int i = 0; i < N; ++i)
    stp<MODE == MODE_STREAM>(work_field<S>(b.fC) + (long long)i * k.n, idx, S(psiC[i] * inv));
}

// ---- k_mu3d ---------------------------------------------------------------
// z-marching: a workgroup owns a TX x TY column of nodes over ZB planes and
// keeps three planes of C_j and psi (tile plus a one-node halo) in an LDS
// ring, so each value is fetched once per tile instead of once per
// neighbour (the 19-point stencil otherwise issues 19 loads per node and
// field through L2). The ring holds the fields in their storage type (float32 in float
// contexts; 256^3 FP32: 196 -> 185 us per launch against a float64 ring,
// same GPU). The step kernel's ring stays float64: typed as the fields it
// took more registers and was slower (FP32 2.69 -> 2.73 ms, FP16 1.89 ->
// 2.81 ms per step).
// Planes per workgroup: each column reloads two halo planes, but more
// columns run at once (same GPU, 256^3 per step, 16 -> 8 planes: FP32 2.86 ->
// 2.80 ms, FP16 and BF16 0.5 % faster, FP64 unchanged; 4 planes: FP32 2.78
// ms, the others 1 % slower than at 16; 32 planes slower for all).
constexpr int ZB = 8;

template <int N, class Pop, class S, int TY, bool NT>
__global__ __launch_bounds__(TX* TY) void k_mu3d(Coef<double> k, Bufs<Pop, S> b) {
  // arithmetic in the field type: float64 in FP64 contexts, float32 otherwise
  using D = std::conditional_t<std::is_same_v<S, double>, double, float>;
  constexpr int HX = TX + 2, HY = TY + 2, HN = HX * HY;
  struct Plane {  // in the field type: float64 <- S conversions are exact
    S c[N][HY][HX];
    S p[HY][HX];
  };
  __shared__ Plane ring[3];
  const int nx = k.nx, ny = k.ny, nz = k.nz;
  // tile of this workgroup (per-plane XCD banding as in node_of)
  const unsigned gx = gridDim.x, per = gx * gridDim.y;
  unsigned bx = blockIdx.x, by = blockIdx.y;
  if (per % 8u == 0u) {
    const unsigned l = by * gx + bx, q = per / 8u;
    const unsigned t = (l % 8u) * q + l / 8u;
    bx = t % gx;
    by = t / gx;
  }
  const int x0 = int(bx) * TX, y0 = int(by) * TY;
  const int z0 = int(blockIdx.z) * ZB;
  const int z1 = z0 + ZB < nz ? z0 + ZB : nz;
  const int tx = int(threadIdx.x) % TX, ty = int(threadIdx.x) / TX;
  const int x = x0 + tx, y = y0 + ty;
  const bool own = x < nx && y < ny;

  auto load = [&](int zz, Plane& pl) {
    const int zw = wrap(zz, nz);
    for (int r = int(threadIdx.x); r < HN; r += TX * TY) {
      const int ly = r / HX, lx = r - ly * HX;
      const unsigned idx = (unsigned(zw) * unsigned(ny) +
                            unsigned(wrap(y0 + ly - 1, ny))) * unsigned(nx) +
                           unsigned(wrap(x0 + lx - 1, nx));
      pl.p[ly][lx] = ldp(b.psi, idx);
#pragma unroll
      for (int j = 0; j < N; ++j)
        pl.c[j][ly][lx] = ldp(work_field<S>(b.fC) + (long long)j * k.n, idx);
    }
  };

  // Plane z + 2 is fetched into registers before plane z is computed and
  // put into the ring after it, so its load latency overlaps that work
  // (256^3 FP32: 184 -> 163 us per launch, same GPU).
  constexpr int PER = (HN + TX * TY - 1) / (TX * TY);  // ring slots per thread
  S pre[PER][N + 1];
  auto fetch = [&](int zz) {
    const int zw = wrap(zz, nz);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int r = int(threadIdx.x) + u * TX * TY;
      if (r < HN) {
        const int ly = r / HX, lx = r - ly * HX;
        const unsigned idx = (unsigned(zw) * unsigned(ny) +
                              unsigned(wrap(y0 + ly - 1, ny))) * unsigned(nx) +
                             unsigned(wrap(x0 + lx - 1, nx));
        pre[u][N] = ldp(b.psi, idx);
#pragma unroll
        for (int j = 0; j < N; ++j)
          pre[u][j] = ldp(work_field<S>(b.fC) + (long long)j * k.n, idx);
      }
    }
  };
  auto put = [&](Plane& pl) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int r = int(threadIdx.x) + u * TX * TY;
      if (r < HN) {
        const int ly = r / HX, lx = r - ly * HX;
        pl.p[ly][lx] = pre[u][N];
#pragma unroll
        for (int j = 0; j < N; ++j) pl.c[j][ly][lx] = pre[u][j];
      }
    }
  };
  load(z0 - 1, ring[(z0 + 2) % 3]);
  load(z0, ring[z0 % 3]);
  load(z0 + 1, ring[(z0 + 1) % 3]);
  __syncthreads();
  for (int z = z0; z < z1; ++z) {
    const bool more = z + 1 < z1;  // the next plane needs plane z + 2
    if (more) fetch(z + 2);
    if (own) {
      const Plane* pz[3] = {&ring[(z + 2) % 3], &ring[z % 3], &ring[(z + 1) % 3]};
      const int lx = tx + 1, ly = ty + 1;
      // value of a staged field at the neighbour x + c_q
      auto at = [&](auto qc, const auto& arr) {
        constexpr int q = decltype(qc)::value;
        return arr(*pz[G19::c[q].z + 1], ly + G19::c[q].y, lx + G19::c[q].x);
      };
      const D psi = pz[1]->p[ly][lx];
      const D psih = psi > D(k.psi_min) ? psi : D(k.psi_min);
      // one division for the N phases (the kernel is VALU-bound: 161 ->
      // 157 us per launch at 256^3 FP32, same GPU)
      const D ipsih = D(1) / psih;
      D C[N], L[N];
      // div(psi grad C_j): the face and the edge terms summed apart and
      // weighted once (1/6, 1/12), psi(x + c_q) + psi shared by the phases
      // (256^3 FP32: 157 -> 151 us per launch, FP64 204 -> 190 us)
      D sf[N], se[N];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        C[j] = pz[1]->c[j][ly][lx];
        sf[j] = D(0);
        se[j] = D(0);
      }
      static_for<1, 19>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const D a = D(at(qc, [](const Plane& pl, int yy, int xx) { return pl.p[yy][xx]; })) + psi;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          const D cq = D(at(qc, [j](const Plane& pl, int yy, int xx) { return pl.c[j][yy][xx]; }));
          if constexpr (stencil_w<q>() > 0.1) sf[j] += a * (cq - C[j]);
          else se[j] += a * (cq - C[j]);
        }
      });
#pragma unroll
      for (int j = 0; j < N; ++j) L[j] = D(1.0 / 6.0) * sf[j] + D(1.0 / 12.0) * se[j];
      const unsigned idx = (unsigned(z) * unsigned(ny) + unsigned(y)) * unsigned(nx) +
                           unsigned(x);
      // wetting weights sum_k cos theta^k_jq |grad psi_k| from the stored
      // E_i = sum_k cos theta^k_iN |grad psi_k| (eq. 2.9 is linear in them)
      D ct[N];
#pragma unroll
      for (int i = 0; i < N - 1; ++i) ct[i] = D(ldp(b.wet + (long long)i * k.n, idx));
      ct[N - 1] = D(0);
      D W[N];  // sum_{q != j} (sum_k cos theta^k_jq |grad psi_k|) C_j C_q
#pragma unroll
      for (int j = 0; j < N; ++j) {
        D acc = D(0);
#pragma unroll
        for (int q = 0; q < N; ++q)
          if (q != j) {
            const D cjq = (D(k.sigN[j]) * ct[j] - D(k.sigN[q]) * ct[q]) * D(k.inv_sig[j][q]);
            acc += cjq * C[j] * C[q];
          }
        W[j] = acc;
      }
#pragma unroll
      for (int i = 0; i < N; ++i) {
        D bulk = D(0), grad = D(0), wet = D(0);
        const D gi = gprime(C[i]);
#pragma unroll
        for (int j = 0; j < N; ++j)
          if (j != i) {
            bulk += D(k.beta2[i][j]) * (gi - gprime(C[i] + C[j]));
            grad += D(k.grad34[i][j]) * L[j];
            wet += D(k.wet3[i][j]) * W[j];
          }
        stp<NT>(work_field<S>(b.fmu) + (long long)i * k.n, idx,
            S((psi * bulk + grad + wet) * ipsih));
      }
    }
    // every read of the slot of plane z - 1 is done: plane z + 2 goes there
    __syncthreads();
    if (more) {
      put(ring[(z + 2) % 3]);
      __syncthreads();
    }
  }
}

// ---- k_step3d -------------------------------------------------------------
// Each workgroup marches a column of tiles in z as k_mu3d does, with three
// planes of C_i, mu_i and psi (tile plus a one-node halo) staged in LDS; the
// node's stencils of these fields read LDS, the rest of its inputs come from
// global memory (256^3 step: FP32 3.17 -> 2.99 ms, FP64 5.52 -> 5.05 ms;
// the 16-bit storages 2-6 % slower than with the gathers from L2).
template <int N, int TY>
struct StepPlane {
  double c[N][TY + 2][TX + 2];
  double m[N][TY + 2][TX + 2];
  double p[TY + 2][TX + 2];
};

// Star of a staged field around LDS position (lx, ly) of the middle plane.
template <class Pl, class F>
__device__ inline Star<double> lds_star(const Pl* const* pz, int lx, int ly,
                                        F get) {
  Star<double> s;
  static_for<0, 19>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    s.v[q] = get(*pz[G19::c[q].z + 1], ly + G19::c[q].y, lx + G19::c[q].x);
  });
  return s;
}

// What the node update reads at its own node, in their storage types: the
// pulled populations of every set, the float64 rest populations and the
// history. With FP32 storage the kernel loads them one plane ahead (below).
template <int N, class LF, class LG, class Pop, class S>
struct NodeIn {
  Pop g[LG::Q];
  Pop f[N][LF::Q - 1];
  double f0[N];
  S hC[N], hU[3], hM[3], hP;
};

template <int N, class LF, class LG, class Pop, class S, int MODE>
__device__ inline void fetch_node(const Bufs<Pop, S>& b, long long n, int nx,
                                  int ny, int nz, int x, int y, int z,
                                  NodeIn<N, LF, LG, Pop, S>& in) {
  if constexpr (MODE != MODE_INIT) {
    constexpr bool NT = MODE == MODE_STREAM;
    constexpr int QF = LF::Q;
    const Nbr3 nb = make_nbr3(x, y, z, nx, ny, nz);
    const unsigned idx = nb.at(0, 0, 0);
    static_for<0, LG::Q>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      in.g[p] = ldo<NT && LG::c[p].x == 0>(
          b.gA + (long long)p * n, nb.src(LG::c[p].x, LG::c[p].y, LG::c[p].z));
    });
#pragma unroll
    for (int i = 0; i < N; ++i) {
      static_for<1, QF>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        in.f[i][p - 1] = ldo<NT && LF::c[p].x == 0>(
            phase_plane(b.fA, i, p, QF, n),
            nb.src(LF::c[p].x, LF::c[p].y, LF::c[p].z));
      });
      in.f0[i] = ldo<NT>(b.f0A + (long long)i * n, idx);
      in.hC[i] = ldo<NT>(b.hist + (long long)(H3_C + i) * n, idx);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      in.hU[a] = ldo<NT>(b.hist + (long long)(H3_U<N> + a) * n, idx);
      in.hM[a] = ldo<NT>(b.hist + (long long)(H3_M<N> + a) * n, idx);
    }
    in.hP = ldo<NT>(b.hist + (long long)(H3_P<N>) * n, idx);
  }
}

template <int N, class LF, class LG, class Pop, class S, class R, int MODE,
          int TY, bool PRE, class PF>
__device__ inline void step3d_node(const Coef<double>& kd, const Coef<R>& k,
                                   const Bufs<Pop, S>& b, int x, int y, int z,
                                   const StepPlane<N, TY>* const* pz, int lx,
                                   int ly, const NodeIn<N, LF, LG, Pop, S>& in,
                                   PF prefetch) {
  using D = double;
  using Pl = StepPlane<N, TY>;
  constexpr int QF = LF::Q, QG = LG::Q;
  constexpr bool NT = MODE == MODE_STREAM;  // streaming stores
  const Nbr3 nb = make_nbr3(x, y, z, k.nx, k.ny, k.nz);
  const unsigned idx = nb.at(0, 0, 0);
  const long long n = k.n;

  // ---- gradients from the neighbours ----------------------------------
  const Star<D> ps = lds_star(pz, lx, ly, [](const Pl& pl, int yy, int xx) {
    return pl.p[yy][xx];
  });
  const D psi_d = ps.v[0];
  const R psi = R(psi_d);
  const D psih_d = psi_d > kd.psi_min ? psi_d : kd.psi_min;
  const R gpsi[3] = {R(sgrad<0>(ps)), R(sgrad<1>(ps)), R(sgrad<2>(ps))};
  Star<D> rs;  // psi rho at the neighbours: psi sum_i rho_i C_i
#pragma unroll
  for (int q = 0; q < 19; ++q) rs.v[q] = D(0);
  R C[N], gC[N][3], mu[N], gmu[N][3];
  D mu_d[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const Star<D> cs = lds_star(pz, lx, ly, [i](const Pl& pl, int yy, int xx) {
      return pl.c[i][yy][xx];
    });
#pragma unroll
    for (int q = 0; q < 19; ++q) rs.v[q] += kd.rho[i] * cs.v[q];
    C[i] = R(cs.v[0]);
    gC[i][0] = R(sgrad<0>(cs));
    gC[i][1] = R(sgrad<1>(cs));
    gC[i][2] = R(sgrad<2>(cs));
    const Star<D> ms = lds_star(pz, lx, ly, [i](const Pl& pl, int yy, int xx) {
      return pl.m[i][yy][xx];
    });
    mu_d[i] = ms.v[0];
    mu[i] = R(ms.v[0]);
    gmu[i][0] = R(sgrad<0>(ms));
    gmu[i][1] = R(sgrad<1>(ms));
    gmu[i][2] = R(sgrad<2>(ms));
  }
#pragma unroll
  for (int q = 0; q < 19; ++q) rs.v[q] *= ps.v[q];
  const R psirho = R(rs.v[0]);
  const R gprho[3] = {R(sgrad<0>(rs)), R(sgrad<1>(rs)), R(sgrad<2>(rs))};
  R grho[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int a = 0; a < 3; ++a) grho[a] += k.rho[i] * gC[i][a];
  // phi mu_i = mu_i psi_hat (the value k_mu3d divided)
  D psimu_d[N];
  R psimu[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    psimu_d[i] = mu_d[i] * psih_d;
    psimu[i] = R(psimu_d[i]);
  }
  // mass flux m^C = -sum_ij rho_i M_ij grad mu_j, with
  // sum_i rho_i M_ij = m0 C_j sum_{k != j} C_k (rho_j - rho_k)  (eq. 2.5)
  R mC[3] = {R(0), R(0), R(0)};
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
    const R aa = k.m0 * C[j] * sr;
#pragma unroll
    for (int a = 0; a < 3; ++a) mC[a] -= aa * gmu[j][a];
  }

  R u[3], F[3] = {R(0), R(0), R(0)};
  R gp[QG];
  R sum_gm = R(0);
  if constexpr (MODE == MODE_INIT) {
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = b.inU ? R(ldp(b.inU + a * n, idx)) : R(0);
  } else {
    // -div T^{n-1}, T antisymmetric with components xy, xz, yz
    const Star<R> txy = gather<R>(b.TA, nb);
    const Star<R> txz = gather<R>(b.TA + n, nb);
    const Star<R> tyz = gather<R>(b.TA + 2 * n, nb);
    const R divT[3] = {-sgrad<1>(txy) - sgrad<2>(txz),
                       sgrad<0>(txy) - sgrad<2>(tyz),
                       sgrad<0>(txz) + sgrad<1>(tyz)};
    // sum_{p != 0} g_p and j = sum_p c_p g_p are accumulated in float64
    // in every precision: both are small differences of populations of
    // either sign (eq. 19, the velocity recovery), where float32 sums lose
    // digits the stored populations still carry
    D sg = D(0), jd[3] = {D(0), D(0), D(0)};
    static_for<0, QG>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      if constexpr (PRE)
        gp[p] = R(in.g[p]);
      else
        gp[p] = R(ldo<NT && LG::c[p].x == 0>(
            b.gA + (long long)p * n, nb.src(LG::c[p].x, LG::c[p].y, LG::c[p].z)));
      if constexpr (p > 0) sg += D(gp[p]);
      if constexpr (LG::c[p].x != 0) jd[0] += D(LG::c[p].x) * D(gp[p]);
      if constexpr (LG::c[p].y != 0) jd[1] += D(LG::c[p].y) * D(gp[p]);
      if constexpr (LG::c[p].z != 0) jd[2] += D(LG::c[p].z) * D(gp[p]);
    });
    sum_gm = R(sg);
    const R j[3] = {R(jd[0]), R(jd[1]), R(jd[2])};
    // force (eq. 3.13): -div T^{n-1} + sum_i phi mu_i grad C_i
    //                   + P^{n-1} grad psi + psi (rho a + G)
    const R Pprev =
        R(PRE ? in.hP : ldo<NT>(b.hist + (long long)(H3_P<N>) * n, idx));
    R Fp[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Fp[a] = -divT[a] + Pprev * gpsi[a] + psirho * k.accel[a] + psi * k.force[a];
#pragma unroll
      for (int i = 0; i < N; ++i) Fp[a] += psimu[i] * gC[i][a];
    }
    // phi rho u = j + F/2 with F = Fp - (1 - psi) lam u, solved for u
    const R pen = (R(1) - psi) * k.lam;
    const R den = R(1) / (psirho + R(0.5) * pen);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      u[a] = (j[a] + R(0.5) * Fp[a]) * den;
      F[a] = Fp[a] - pen * u[a];
    }
  }

  // Y = sym(phi m^C u): xx, xy, xz, yy, yz, zz; T = antisym: xy, xz, yz
  R Y[6];
  sym_flux(psi, mC, u, Y);
  const R Tn[3] = {R(0.5) * psi * (mC[0] * u[1] - u[0] * mC[1]),
                   R(0.5) * psi * (mC[0] * u[2] - u[0] * mC[2]),
                   R(0.5) * psi * (mC[1] * u[2] - u[1] * mC[2])};
  R dtY[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
  if constexpr (MODE != MODE_INIT) {
    R uprev[3], mprev[3], Yprev[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      uprev[a] = R(PRE ? in.hU[a] : ldp(b.hist + (long long)(H3_U<N> + a) * n, idx));
      mprev[a] = R(PRE ? in.hM[a] : ldo<NT>(b.hist + (long long)(H3_M<N> + a) * n, idx));
    }
    sym_flux(psi, mprev, uprev, Yprev);
#pragma unroll
    for (int q = 0; q < 6; ++q) dtY[q] = Y[q] - Yprev[q];
  }
  // local flow rates from nu (eq. 16)
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
    P = b.inP ? R(ldp(b.inP, idx)) : R(0);
    psiP = psi * P;
  } else {
    // eq. (19)
    const R s0eq = -k.wg[0] * (A[0] + A[3] + A[5]) * k.inv_c2mcs2;
    const R ugr = u[0] * grho[0] + u[1] * grho[1] + u[2] * grho[2];
    const R ugpr = u[0] * gprho[0] + u[1] * gprho[1] + u[2] * gprho[2];
    psiP = k.pref * (sum_gm + k.cgr * psi * ugr +
                     k.halfK * (dtY[0] + dtY[3] + dtY[5]) +
                     k.KH * (s21 - R(2)) / s21 * ugpr + s0eq);
    P = R(D(psiP) / psih_d);
  }
  if constexpr (MODE == MODE_MOMENTS) {
#pragma unroll
    for (int i = 0; i < N; ++i) stp<NT>(b.outC + i * n, idx, double(C[i]));
#pragma unroll
    for (int a = 0; a < 3; ++a) stp<NT>(b.outU + a * n, idx, double(u[a]));
    stp<NT>(b.outP, idx, double(P));
    prefetch();
    return;
  }

  // ---- flow set: equilibrium (eqs. 3.8, 3.11), source (3.10, 3.12) ---
  if constexpr (MODE == MODE_INIT) {
    static_for<0, QG>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      constexpr int cx = LG::c[p].x, cy = LG::c[p].y, cz = LG::c[p].z;
      const R h2 = (A[0] * (R(cx * cx) - k.cs2) + A[3] * (R(cy * cy) - k.cs2) +
                    A[5] * (R(cz * cz) - k.cs2)) *
                       k.h2diag +
                   (A[1] * R(cx * cy) + A[2] * R(cx * cz) + A[4] * R(cy * cz)) *
                       k.h2off;
      R geq = k.wg[p] * ((psiP + psirho * (R(cx) * u[0] + R(cy) * u[1] +
                                             R(cz) * u[2])) *
                             k.inv_cs2 +
                         h2);
      if constexpr (p == 0) geq -= psiP * k.inv_cs2;  // stored as g_0 - rho0
      // the buffers hold pre-streaming values: place g_p(x) where the
      // next pull reads it, at x - c_p
      stp<NT>(b.gB + (long long)p * n, nb.src(cx, cy, cz), Pop(geq));
    });
  } else {
    const R ub = u[0] * gprho[0] + u[1] * gprho[1] + u[2] * gprho[2];
    // M^{2G} (eq. 3.12) with the scalar u.grad(phi rho) on the diagonal
    const R M[6] = {dtY[0] + R(2) * k.cs2 * u[0] * gprho[0] + k.one_m3cs2 * ub,
                    dtY[1] + k.cs2 * (u[0] * gprho[1] + gprho[0] * u[1]),
                    dtY[2] + k.cs2 * (u[0] * gprho[2] + gprho[0] * u[2]),
                    dtY[3] + R(2) * k.cs2 * u[1] * gprho[1] + k.one_m3cs2 * ub,
                    dtY[4] + k.cs2 * (u[1] * gprho[2] + gprho[1] * u[2]),
                    dtY[5] + R(2) * k.cs2 * u[2] * gprho[2] + k.one_m3cs2 * ub};
    const R a0 = psi * (u[0] * grho[0] + u[1] * grho[1] + u[2] * grho[2]);
    R del[QG];
    collide_flow<LG>(gp, A, psiP, M, a0, F, s21, s22, k.sg, k.q4, k.cs2,
                     k.inv_cs2, del);
#pragma unroll
    for (int p = 0; p < QG; ++p) stp<NT>(b.gB + (long long)p * n, idx, Pop(gp[p] - del[p]));
  }

  // ---- phase sets: equilibrium (3.5), source (3.6, 3.7), collision ---
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if constexpr (MODE == MODE_INIT) {
      const D psiC = psi_d * ldp(b.inC + (long long)i * n, idx);
      const R X[3] = {R(psiC) * u[0], R(psiC) * u[1], R(psiC) * u[2]};
      const R em = k.eta[i] * psimu[i];
      D comp = D(0);
      static_for<1, QF>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int cx = LF::c[p].x, cy = LF::c[p].y, cz = LF::c[p].z;
        const R feq = k.wf[p] * (em + (R(cx) * X[0] + R(cy) * X[1] +
                                       R(cz) * X[2]) * k.inv_cs2);
        stp<NT>(phase_plane(b.fB, i, p, QF, n), nb.src(cx, cy, cz),
            narrow<Pop>(feq, comp));
      });
      // f^eq_0 = (w_0 - 1) eta phi mu + phi C (float64 rest plane), plus
      // the storage rounding of the moving populations
      stp<NT>(b.f0B + (long long)i * n, idx,
          (kd.wf[0] - D(1)) * kd.eta[i] * psimu_d[i] + psiC + comp);
      stp<NT>(b.hist + (long long)(H3_C + i) * n, idx, S(R(psiC)));
    } else {
      // own phi C_i = sum of the pulled populations (Section 3): moving
      // populations summed in the storage precision, the float64 rest
      // population added last
      R fp[QF];
      fp[0] = R(0);
      R mv = R(0);
      static_for<1, QF>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        if constexpr (PRE)
          fp[p] = R(in.f[i][p - 1]);
        else
          fp[p] = R(ldo<NT && LF::c[p].x == 0>(phase_plane(b.fA, i, p, QF, n),
                        nb.src(LF::c[p].x, LF::c[p].y, LF::c[p].z)));
        mv += fp[p];
      });
      const D f0 = PRE ? in.f0[i] : ldo<NT>(b.f0A + (long long)i * n, idx);
      const R psiC = R(f0 + D(mv));
      // phi C_i u of the previous step from its stored factors (phi C_i is
      // read before this step overwrites it)
      const R psiCprev =
          R(PRE ? in.hC[i] : ldo<NT>(b.hist + (long long)(H3_C + i) * n, idx));
      R Xprev[3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
        Xprev[a] = psiCprev * R(PRE ? in.hU[a]
                                    : ldp(b.hist + (long long)(H3_U<N> + a) * n, idx));
      const R X[3] = {psiC * u[0], psiC * u[1], psiC * u[2]};
      // S_i (eq. 3.7) and V = d_t(phi C_i u) + c_s^2 eta (mu grad psi - S_i)
      R V[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        R sa = (C[i] * Cs[i] - R(1)) * gmu[i][a];
#pragma unroll
        for (int j = 0; j < N; ++j)
          if (j != i) sa -= C[i] * C[j] * gmu[j][a];
        const R dX = X[a] - Xprev[a];
        V[a] = dX + k.cs2 * k.eta[i] * (mu[i] * gpsi[a] - psi * sa);
      }
      R del[QF];
      collide_phase<LF>(fp, k.eta[i] * psimu[i], X, V, k.sf, k.cs2, del);
      D comp = D(0);
#pragma unroll
      for (int p = 1; p < QF; ++p)
        stp<NT>(phase_plane(b.fB, i, p, QF, n), idx,
            narrow<Pop>(fp[p] - del[p], comp));
      stp<NT>(b.f0B + (long long)i * n, idx, f0 - D(del[0]) + comp);
      stp<NT>(b.hist + (long long)(H3_C + i) * n, idx, S(psiC));
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    stp<NT>(b.hist + (long long)(H3_U<N> + a) * n, idx, S(u[a]));
    stp<NT>(b.hist + (long long)(H3_M<N> + a) * n, idx, S(mC[a]));
  }
  stp<NT>(b.hist + (long long)(H3_P<N>) * n, idx, S(P));
#pragma unroll
  for (int c = 0; c < 3; ++c) stp<NT>(b.TB + (long long)c * n, idx, S(Tn[c]));
  // every input of this node has been used: the next plane's node loads go
  // into the same registers
  prefetch();
}

// Waves per SIMD the register allocation aims at: what the LDS ring allows
// (TY waves per workgroup, spread over the CU's four SIMDs), capped at two.
// Left to itself the compiler gives the float64 kernel 256+ registers and
// one wave per SIMD. The float kernels were capped at three while their
// coefficients came as arguments (at two, FP32 was 17 % slower); with the
// coefficient table two is the faster cap (same GPU, 256^3 per step: FP32
// 2.95 -> 2.86 ms, FP16 2.68 -> 1.98 ms, BF16 unchanged).
template <int N, int TY>
constexpr int step3d_waves() {
  constexpr int wgs = int((160u * 1024u) / (3u * sizeof(StepPlane<N, TY>)));
  constexpr int lds_waves = (wgs * TY + 3) / 4;
  constexpr int cap = 2;
  return lds_waves < 1 ? 1 : (lds_waves < cap ? lds_waves : cap);
}

template <int N, class LF, class LG, class Pop, class S, class R, int MODE,
          int TY>
__global__ __launch_bounds__(TX* TY)
__attribute__((amdgpu_waves_per_eu(step3d_waves<N, TY>())))
void k_step3d(Coef<double> kda, Coef<R> ka,
              const Coef<double>* __restrict__ kdp,
              const Coef<R>* __restrict__ kp, Bufs<Pop, S> b) {
  // Coefficients as kernel arguments overflow the scalar registers and spill
  // into VGPR lanes; read from a device table they cost no spills but scalar
  // loads inside the z loop. Which is faster depends on the storage type
  // (same GPU, 256^3: table for BF16 2.79 -> 2.00 ms, FP32 3.00 -> 2.97 ms
  // and FP16 2.68 -> 1.98 ms per step, the last two at two waves per SIMD;
  // arguments for FP64 5.09 vs 5.60 ms).
  constexpr bool TABLE = std::is_same_v<Pop, __bf16> ||
                         std::is_same_v<Pop, float> ||
                         std::is_same_v<Pop, _Float16>;
  const Coef<double>& kd = TABLE ? *kdp : kda;
  const Coef<R>& k = TABLE ? *kp : ka;
  using Pl = StepPlane<N, TY>;
  constexpr int HX = TX + 2, HY = TY + 2, HN = HX * HY;
  __shared__ Pl ring[3];
  const int nx = k.nx, ny = k.ny, nz = k.nz;
  const unsigned gx = gridDim.x, per = gx * gridDim.y;
  unsigned bx = blockIdx.x, by = blockIdx.y;
  if (per % 8u == 0u) {
    const unsigned l = by * gx + bx, q = per / 8u;
    const unsigned t = (l % 8u) * q + l / 8u;
    bx = t % gx;
    by = t / gx;
  }
  const int x0 = int(bx) * TX, y0 = int(by) * TY;
  const int z0 = int(blockIdx.z) * ZB;
  const int z1 = z0 + ZB < nz ? z0 + ZB : nz;
  const int tx = int(threadIdx.x) % TX, ty = int(threadIdx.x) / TX;
  const int x = x0 + tx, y = y0 + ty;
  const bool own = x < nx && y < ny;

  auto load = [&](int zz, Pl& pl) {
    const int zw = wrap(zz, nz);
    for (int r = int(threadIdx.x); r < HN; r += TX * TY) {
      const int ly = r / HX, lx = r - ly * HX;
      const unsigned i0 = (unsigned(zw) * unsigned(ny) +
                           unsigned(wrap(y0 + ly - 1, ny))) * unsigned(nx) +
                          unsigned(wrap(x0 + lx - 1, nx));
      pl.p[ly][lx] = double(ldp(b.psi, i0));
#pragma unroll
      for (int j = 0; j < N; ++j) {
        pl.c[j][ly][lx] = double(ldp(work_field<S>(b.fC) + (long long)j * k.n, i0));
        pl.m[j][ly][lx] = double(ldp(work_field<S>(b.fmu) + (long long)j * k.n, i0));
      }
    }
  };

  // FP32 storage: a software pipeline over the planes of the column. The
  // node's own inputs (NodeIn) for plane z + 1 are loaded at the end of the
  // node update of plane z, into the registers that plane z's inputs have
  // just freed, and plane z + 2 of the ring is fetched into registers before
  // plane z is computed and put into LDS after it. The only loads the node
  // update then issues are the lagged-T gathers (their wait also covers the
  // previous plane's stores and the prefetched inputs, issued before them
  // and by then overlapped with the ring put and the LDS gradients);
  // before, each plane waited for its ring load (behind the previous
  // plane's stores), its gathers and flow populations, then its phase
  // populations. 169 -> 253 VGPRs, still two waves per SIMD; 256^3 FP32
  // 2.476 -> 2.352 ms per step (same GPU, bit for bit the same results).
  // Measured and left out: the node loads alone
  // (2.418 ms), also the T gathers one plane ahead (10 VGPRs spilled, 2.436
  // ms), and the pipeline for the 16-bit storages, whose node update at 161
  // to 165 VGPRs runs three waves per SIMD and drops to two with it (FP16
  // 1.655 -> 1.772 ms, BF16 1.696 -> 1.807 ms). FP64 (253 VGPRs without it)
  // has no room.
  using In = NodeIn<N, LF, LG, Pop, S>;
  constexpr bool PF = std::is_same_v<Pop, float> && MODE != MODE_INIT;
  constexpr bool RF = PF;
  In cur;
  if constexpr (PF)
    if (own) fetch_node<N, LF, LG, Pop, S, MODE>(b, k.n, nx, ny, nz, x, y, z0, cur);
  constexpr int PER = (HN + TX * TY - 1) / (TX * TY);  // ring slots per thread
  S pre[PER][2 * N + 1];
  auto fetch_ring = [&](int zz) {
    const int zw = wrap(zz, nz);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int r = int(threadIdx.x) + u * TX * TY;
      if (r < HN) {
        const int ly = r / HX, lx = r - ly * HX;
        const unsigned i0 = (unsigned(zw) * unsigned(ny) +
                             unsigned(wrap(y0 + ly - 1, ny))) * unsigned(nx) +
                            unsigned(wrap(x0 + lx - 1, nx));
        pre[u][2 * N] = ldp(b.psi, i0);
#pragma unroll
        for (int j = 0; j < N; ++j) {
          pre[u][j] = ldp(work_field<S>(b.fC) + (long long)j * k.n, i0);
          pre[u][N + j] = ldp(work_field<S>(b.fmu) + (long long)j * k.n, i0);
        }
      }
    }
  };
  auto put_ring = [&](Pl& pl) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int r = int(threadIdx.x) + u * TX * TY;
      if (r < HN) {
        const int ly = r / HX, lx = r - ly * HX;
        pl.p[ly][lx] = double(pre[u][2 * N]);
#pragma unroll
        for (int j = 0; j < N; ++j) {
          pl.c[j][ly][lx] = double(pre[u][j]);
          pl.m[j][ly][lx] = double(pre[u][N + j]);
        }
      }
    }
  };

  load(z0 - 1, ring[(z0 + 2) % 3]);
  load(z0, ring[z0 % 3]);
  if constexpr (RF) {
    load(z0 + 1, ring[(z0 + 1) % 3]);
    __syncthreads();
  }
  for (int z = z0; z < z1; ++z) {
    const bool more = z + 1 < z1;
    if constexpr (RF) {
      if (more) fetch_ring(z + 2);
    } else {
      load(z + 1, ring[(z + 1) % 3]);
      __syncthreads();
    }
    if (own) {
      const Pl* pz[3] = {&ring[(z + 2) % 3], &ring[z % 3], &ring[(z + 1) % 3]};
      if constexpr (PF) {
        step3d_node<N, LF, LG, Pop, S, R, MODE, TY, true>(
            kd, k, b, x, y, z, pz, tx + 1, ty + 1, cur, [&] {
              if (more)
                fetch_node<N, LF, LG, Pop, S, MODE>(b, k.n, nx, ny, nz, x, y,
                                                    z + 1, cur);
            });
      } else {
        step3d_node<N, LF, LG, Pop, S, R, MODE, TY, false>(
            kd, k, b, x, y, z, pz, tx + 1, ty + 1, cur, [] {});
      }
    }
    // the slot of plane z - 1 is overwritten next
    __syncthreads();
    if constexpr (RF) {
      if (more) {
        put_ring(ring[(z + 2) % 3]);
        __syncthreads();
      }
    }
  }
}

template <int N, class LF, class Pop, class S, class R, int MODE, int TY>
hipError_t launch_3(const Coef<double>& kd, const Coef<R>& k,
                    const Bufs<Pop, S>& b, hipStream_t st) {
  const dim3 g((k.nx + TX - 1) / TX, (k.ny + TY - 1) / TY, k.nz);
  const dim3 blk(TX * TY);
  hipLaunchKernelGGL((k_frac3d<N, LF, Pop, S, R, MODE, TY>), g, blk, 0, st, kd, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 gm(g.x, g.y, (k.nz + ZB - 1) / ZB);
  hipLaunchKernelGGL((k_mu3d<N, Pop, S, TY, MODE == MODE_STREAM>), gm, blk, 0,
                     st, kd, b);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!b.coef_d || !b.coef_r) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_step3d<N, LF, D3Q19, Pop, S, R, MODE, TY>), gm, blk, 0,
                     st, kd, k, static_cast<const Coef<double>*>(b.coef_d),
                     static_cast<const Coef<R>*>(b.coef_r), b);
  return hipGetLastError();
}

template <int N, class Pop, class S, class R, int MODE>
hipError_t launch_ty3(int lattice_f, const Coef<double>& kd, const Coef<R>& k,
                      const Bufs<Pop, S>& b, int ty, hipStream_t st) {
  if (lattice_f == D3Q7::ID) {
    if (ty == 2) return launch_3<N, D3Q7, Pop, S, R, MODE, 2>(kd, k, b, st);
    return launch_3<N, D3Q7, Pop, S, R, MODE, 4>(kd, k, b, st);
  }
  if (ty == 2) return launch_3<N, D3Q15, Pop, S, R, MODE, 2>(kd, k, b, st);
  return launch_3<N, D3Q15, Pop, S, R, MODE, 4>(kd, k, b, st);
}

template <int N, class Pop, class S, class R>
hipError_t launch_mode3(int mode, int lattice_f, const Coef<double>& kd,
                        const Coef<R>& k, const Bufs<Pop, S>& b, int ty,
                        hipStream_t st) {
  switch (mode) {
    case MODE_STEP:
      return launch_ty3<N, Pop, S, R, MODE_STEP>(lattice_f, kd, k, b, ty, st);
    case MODE_STREAM:
      return launch_ty3<N, Pop, S, R, MODE_STREAM>(lattice_f, kd, k, b, ty, st);
    case MODE_INIT:
      return launch_ty3<N, Pop, S, R, MODE_INIT>(lattice_f, kd, k, b, ty, st);
    default:
      return launch_ty3<N, Pop, S, R, MODE_MOMENTS>(lattice_f, kd, k, b, ty, st);
  }
}

}  // namespace

template <class Pop, class S, class R>
hipError_t launch_3d(int nphase, int lattice_f, int mode,
                     const Coef<double>& kd, const Coef<R>& k,
                     const Bufs<Pop, S>& b, int tx, int ty, hipStream_t st) {
  (void)tx;
  if (!b.fC || !b.fmu) return hipErrorInvalidValue;
  switch (nphase) {
    case 2:
      return launch_mode3<2, Pop, S, R>(mode, lattice_f, kd, k, b, ty, st);
    case 3:
      return launch_mode3<3, Pop, S, R>(mode, lattice_f, kd, k, b, ty, st);
    default:
      return hipErrorInvalidValue;
  }
}

template hipError_t launch_3d<double, double, double>(
    int, int, int, const Coef<double>&, const Coef<double>&,
    const Bufs<double, double>&, int, int, hipStream_t);
template hipError_t launch_3d<float, float, float>(
    int, int, int, const Coef<double>&, const Coef<float>&,
    const Bufs<float, float>&, int, int, hipStream_t);
template hipError_t launch_3d<_Float16, float, float>(
    int, int, int, const Coef<double>&, const Coef<float>&,
    const Bufs<_Float16, float>&, int, int, hipStream_t);
template hipError_t launch_3d<__bf16, float, float>(
    int, int, int, const Coef<double>&, const Coef<float>&,
    const Bufs<__bf16, float>&, int, int, hipStream_t);

}  // namespace ddcc
