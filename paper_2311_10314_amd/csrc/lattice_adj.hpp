// Transposes of the moment transforms of lattice.hpp, for the adjoint
// (reverse-time) step. With H = A(c_s^2) R (A unit lower triangular, R the
// raw monomial matrix):
//   raw_moments_T     ld = R^T lr        (ld_p = sum_k R_kp lr_k, k >= k0)
//   raw_to_hermite_T  lr = A^T lm        (lr_j = lm_j + sum_{k > j} A_kj lm_k)
//   from_hermite_T    lm = A^-T R^-T lo  (back substitution through A^T)
// so that for m = H d, ld = H^T lm, and for o = H^-1 m, lm = H^-T lo.
#pragma once

#include "collide.hpp"
#include "lattice.hpp"

namespace ddcc {

template <class L, int k, int j, class R>
__device__ inline R a_entry(R cs2, R cs4, R cs6) {
  constexpr double a1 = Tab<L>::t.A[1][k][j];
  constexpr double a2 = Tab<L>::t.A[2][k][j];
  constexpr double a3 = Tab<L>::t.A[3][k][j];
  R v = R(0);
  if constexpr (a1 != 0.0) v += R(a1) * cs2;
  if constexpr (a2 != 0.0) v += R(a2) * cs4;
  if constexpr (a3 != 0.0) v += R(a3) * cs6;
  return v;
}

template <class L, int k, int j>
constexpr bool a_nonzero() {
  return Tab<L>::t.A[1][k][j] != 0.0 || Tab<L>::t.A[2][k][j] != 0.0 ||
         Tab<L>::t.A[3][k][j] != 0.0;
}

// ld[p] += sum_{k >= K0} R[k][p] lr[k] for every p.
template <class L, int K0, class R>
__device__ inline void raw_moments_T(const R* lr, R* ld) {
  static_for<0, L::Q>([&](auto pc) {
    constexpr int p = decltype(pc)::value;
    R acc = R(0);
    static_for<K0, L::Q>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      constexpr double v = Tab<L>::t.R[k][p];
      if constexpr (v == 1.0) {
        acc += lr[k];
      } else if constexpr (v == -1.0) {
        acc -= lr[k];
      } else if constexpr (v != 0.0) {
        acc += R(v) * lr[k];
      }
    });
    ld[p] += acc;
  });
}

// lr = A(cs2)^T lm.
template <class L, class R>
__device__ inline void raw_to_hermite_T(const R* lm, R* lr, R cs2) {
  const R cs4 = cs2 * cs2, cs6 = cs4 * cs2;
  static_for<0, L::Q>([&](auto jc) {
    constexpr int j = decltype(jc)::value;
    R acc = lm[j];
    static_for<j + 1, L::Q>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      if constexpr (a_nonzero<L, k, j>())
        acc += a_entry<L, k, j>(cs2, cs4, cs6) * lm[k];
    });
    lr[j] = acc;
  });
}

// lm = A(cs2)^-T R^-T lo.
template <class L, class R>
__device__ inline void from_hermite_T(const R* lo, R* lm, R cs2) {
  constexpr int Q = L::Q;
  R z[Q];
  static_for<0, Q>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    R acc = R(0);
    static_for<0, Q>([&](auto pc) {
      constexpr int p = decltype(pc)::value;
      constexpr double v = Tab<L>::t.Rinv[p][k];
      if constexpr (v == 1.0) {
        acc += lo[p];
      } else if constexpr (v == -1.0) {
        acc -= lo[p];
      } else if constexpr (v != 0.0) {
        acc += R(v) * lo[p];
      }
    });
    z[k] = acc;
  });
  // A^T y = z, A^T unit upper triangular: back substitution
  const R cs4 = cs2 * cs2, cs6 = cs4 * cs2;
  static_for<0, Q>([&](auto rc) {
    constexpr int k = Q - 1 - decltype(rc)::value;
    R acc = z[k];
    static_for<k + 1, Q>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      if constexpr (a_nonzero<L, j, k>())
        acc -= a_entry<L, j, k>(cs2, cs4, cs6) * lm[j];
    });
    lm[k] = acc;
  });
}

// Transpose of collide_phase. ldel: adjoint of del (f*_p = f_p - del_p).
// Accumulates into lfp[1..Q-1] (pulled moving populations), lem
// (eta phi mu), lX and lV.
template <class L, class R>
__device__ inline void collide_phase_T(const R* ldel, const R* sf, R cs2,
                                       R* lfp, R& lem, R* lX, R* lV) {
  constexpr int Q = L::Q;
  R lms[Q], lh[Q], lr[Q];
  from_hermite_T<L>(ldel, lms, cs2);
  static_for<0, Q>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int grp = L::rows[k].group;
    if constexpr (grp == GR0) {
      lh[k] = R(0);
    } else if constexpr (grp == GR1) {
      constexpr int a = row_comp<L>(k);
      const R s = sf[GR1];
      lh[k] = s * lms[k];
      lX[a] -= s * lms[k];
      lV[a] -= (R(1) - R(0.5) * s) * lms[k];
    } else {
      lh[k] = sf[grp] * lms[k];
    }
  });
  raw_to_hermite_T<L>(lh, lr, cs2);
  lem += lr[0];  // the zeroth raw moment is replaced by eta phi mu
  raw_moments_T<L, 1>(lr, lfp);
}

// Transpose of collide_flow for a two-dimensional flow set (no
// fourth-order equilibrium terms from q4). h: Hermite moments of the
// pulled populations; meq/mg as in the forward call. Accumulates into
// lgp, lJ, lA (packed xx xy yy), lpsiP, lM, la0, lF, ls21, ls22.
template <class L, class R>
__device__ inline void collide_flow_T(const R* gp, const R* J, const R* A,
                                      R psiP, const R* M, R a0, const R* F,
                                      R s21, R s22, const R* sg, R cs2,
                                      R inv_cs2, const R* ldel, R* lgp, R* lJ,
                                      R* lA, R& lpsiP, R* lM, R& la0, R* lF,
                                      R& ls21, R& ls22) {
  static_assert(L::D == 2, "two-dimensional flow sets only");
  constexpr int Q = L::Q;
  constexpr int D = L::D;
  R r[Q], h[Q], lms[Q], lh[Q], lr[Q];
  raw_moments<L>(gp, r);
  raw_to_hermite<L>(r, h, cs2);
  from_hermite_T<L>(ldel, lms, cs2);
  static_for<0, Q>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int grp = L::rows[k].group;
    R meq, mg, s;
    if constexpr (grp == GR0) {
      meq = R(0);
      mg = a0;
      s = sg[GR0];
    } else if constexpr (grp == GR1) {
      meq = J[row_comp<L>(k)];
      mg = F[row_comp<L>(k)];
      s = sg[GR1];
    } else if constexpr (grp == GR21) {
      meq = A[sym_diag<D>(row_comp<L>(k))] + psiP;
      mg = M[sym_diag<D>(row_comp<L>(k))];
      s = s21;
    } else if constexpr (grp == GR22) {
      meq = A[sym_pair<D>(row_pair<L>(k))];
      mg = M[sym_pair<D>(row_pair<L>(k))];
      s = s22;
    } else if constexpr (grp == GR3) {
      meq = R(0);
      mg = R(0);
      s = sg[GR3];
    } else {
      meq = -rest_value<L, k>(cs2) * psiP * inv_cs2;
      mg = R(0);
      s = sg[GR4];
    }
    // ms = s (h - meq) - (1 - s/2) mg
    const R l = lms[k];
    lh[k] = s * l;
    const R lmeq = -s * l;
    const R lmg = -(R(1) - R(0.5) * s) * l;
    const R ls = l * (h[k] - meq + R(0.5) * mg);
    if constexpr (grp == GR0) {
      la0 += lmg;
    } else if constexpr (grp == GR1) {
      lJ[row_comp<L>(k)] += lmeq;
      lF[row_comp<L>(k)] += lmg;
    } else if constexpr (grp == GR21) {
      lA[sym_diag<D>(row_comp<L>(k))] += lmeq;
      lpsiP += lmeq;
      lM[sym_diag<D>(row_comp<L>(k))] += lmg;
      ls21 += ls;
    } else if constexpr (grp == GR22) {
      lA[sym_pair<D>(row_pair<L>(k))] += lmeq;
      lM[sym_pair<D>(row_pair<L>(k))] += lmg;
      ls22 += ls;
    } else if constexpr (grp == GR4) {
      lpsiP -= rest_value<L, k>(cs2) * inv_cs2 * lmeq;
    }
  });
  raw_to_hermite_T<L>(lh, lr, cs2);
  raw_moments_T<L, 0>(lr, lgp);
}

}  // namespace ddcc
