// Hermite-moment collision of one node (eqs. 3.1-3.4) with the equilibrium
// and source moments in closed form, so that neither f^eq_p, F_p, g^eq_p nor
// G_p is formed per population.
//
// With Lambda = H^-1 S H the post-collision populations are
//   f* = f - H^-1 [ S (H f - H f^eq) - (I - S/2) H F ],
// and the Hermite moments of the equilibria and sources of eqs. (3.5)-(3.12)
// follow from the orthogonality of the Hermite rows under the weights:
//
// phase set i (eqs. 3.5, 3.6), with B = phi C_i - eta phi mu_i:
//   (H f^eq)_k = B H_k(0) + eta phi mu_i [k = 0] + X_a [k = first order a],
//   (H F)_k    = V_a [k = first order a],  V = d_t(phi C_i u)
//                + c_s^2 eta (mu grad phi - S_i);
//   since (H f)_k contains phi C_i only through A_k0 phi C_i = H_k(0) phi C_i,
//   the O(1) phi C_i cancels exactly: the raw moment r_0 is replaced by
//   eta phi mu_i and nothing large is subtracted.
// flow set (eqs. 3.8, 3.10-3.12), with A = phi rho u u + sym(phi m^C u):
//   (H g^eq)_k = phi rho u_a | A_aa + phi P | A_ab | 0 (third order) |
//                sum_c Q_kc A_cc - H_k(0) phi P / c_s^2 (fourth order),
//   (H G)_k    = phi u.grad rho | F_a | M_aa | M_ab | 0 | sum_c Q_kc M_cc,
//   for the zeroth, first, diagonal / off-diagonal second, third and
//   fourth-order rows (the flow set stores g_0 - rho0, so its zeroth
//   equilibrium moment is 0).
#pragma once

#include <type_traits>
#include <utility>

#include "lattice.hpp"

namespace ddcc {

template <int B, int E, class F>
__host__ __device__ inline void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Index of the diagonal a a / the pair (xy, xz, yz) in the packed symmetric
// tensors (2D: xx xy yy; 3D: xx xy xz yy yz zz).
template <int D>
__host__ __device__ constexpr int sym_diag(int a) {
  return D == 2 ? (a == 0 ? 0 : 2) : (a == 0 ? 0 : (a == 1 ? 3 : 5));
}

template <int D>
__host__ __device__ constexpr int sym_pair(int pr) {
  return D == 2 ? 1 : (pr == 0 ? 1 : (pr == 1 ? 2 : 4));
}

// Phase set. fp[1..Q-1]: pulled moving populations (fp[0] is not read);
// em = eta phi mu; X, V: see above; sf: rates by slot. Returns del with
// f*_p = f_p - del_p (the rest population too).
template <class L, class R>
__device__ inline void collide_phase(const R* fp, R em, const R* X,
                                     const R* V, const R* sf, R cs2, R* del) {
  constexpr int Q = L::Q;
  R d[Q];
  d[0] = R(0);
#pragma unroll
  for (int p = 1; p < Q; ++p) d[p] = fp[p];
  R r[Q], h[Q], ms[Q];
  raw_moments<L>(d, r);
  r[0] = em;
  raw_to_hermite<L>(r, h, cs2);
  static_for<0, Q>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int grp = L::rows[k].group;
    if constexpr (grp == GR0) {
      ms[k] = R(0);
    } else if constexpr (grp == GR1) {
      constexpr int a = row_comp<L>(k);
      const R s = sf[GR1];
      ms[k] = s * (h[k] - X[a]) - (R(1) - R(0.5) * s) * V[a];
    } else {
      ms[k] = sf[grp] * h[k];
    }
  });
  from_hermite<L>(ms, del, cs2);
}

// Flow set. gp: pulled populations (g_0 stored as g_0 - rho0); A, M packed
// symmetric tensors; a0 = phi u.grad rho; F total force; s21, s22 local
// rates, sg the others; q4 fourth-order constants.
// First-order rows: the velocity solves phi rho u = j + F/2 with F the total
// force (penalty included, eq. 3.13), so the first moment of g - g^eq is
// j - phi rho u = -F/2 exactly and the row's post-collision moment
// s (j - phi rho u) - (1 - s/2) F is -F for every rate s. The kernels use
// that value: formed as the difference of j and phi rho u, the rounding of
// phi rho u (relative to u, not to F) repeats with the same sign every step
// where the fields are steady, and adds up in float32.
template <class L, class R>
__device__ inline void collide_flow(const R* gp, const R* A, R psiP,
                                    const R* M, R a0, const R* F, R s21,
                                    R s22, const R* sg, const R (*q4)[3],
                                    R cs2, R inv_cs2, R* del) {
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  R r[Q], h[Q], ms[Q];
  raw_moments<L>(gp, r);
  raw_to_hermite<L>(r, h, cs2);
  static_for<0, Q>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int grp = L::rows[k].group;
    R meq, mg, s;
    if constexpr (grp == GR1) {
      ms[k] = -F[row_comp<L>(k)];  // phi rho u = j + F/2
      return;
    } else if constexpr (grp == GR0) {
      meq = R(0);
      mg = a0;
      s = sg[GR0];
    } else if constexpr (grp == GR21) {
      constexpr int a = row_comp<L>(k);
      meq = A[sym_diag<D>(a)] + psiP;
      mg = M[sym_diag<D>(a)];
      s = s21;
    } else if constexpr (grp == GR22) {
      constexpr int pr = row_pair<L>(k);
      meq = A[sym_pair<D>(pr)];
      mg = M[sym_pair<D>(pr)];
      s = s22;
    } else if constexpr (grp == GR3) {
      meq = R(0);
      mg = R(0);
      s = sg[GR3];
    } else {
      constexpr int j = g4_index<L>(k);
      R qa = R(0), qm = R(0);
#pragma unroll
      for (int c = 0; c < D; ++c) {
        qa += q4[j][c] * A[sym_diag<D>(c)];
        qm += q4[j][c] * M[sym_diag<D>(c)];
      }
      meq = qa - rest_value<L, k>(cs2) * psiP * inv_cs2;
      mg = qm;
      s = sg[GR4];
    }
    ms[k] = s * (h[k] - meq) - (R(1) - R(0.5) * s) * mg;
  });
  from_hermite<L>(ms, del, cs2);
}

}  // namespace ddcc
