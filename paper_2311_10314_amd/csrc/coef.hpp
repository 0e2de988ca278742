// Per-run constants handed to every kernel by value (kernel arguments),
// derived on the host from ddcc_params. R is the arithmetic type.
#pragma once

#include <cstdint>

namespace ddcc {

constexpr int kMaxN = 4;

template <class R>
struct Coef {
  int nx, ny, nz;
  long long n;          // nodes (plane stride)
  static constexpr unsigned off = 0;  // first node of the box in each plane
  R cs2, inv_cs2;       // c_s^2 = d0 (c = 1)
  R psi_min, lam, rho0;
  R m0;
  R beta2[kMaxN][kMaxN];  // 2 beta_ij = 6 sigma_ij / eps   (Section 2.1)
  R grad34[kMaxN][kMaxN]; // (3 eps / 4) sigma_ij           (eq. 2.14)
  R wet3[kMaxN][kMaxN];   // 3 sigma_ij                     (eq. 2.14)
  R sigN[kMaxN];          // sigma_iN                       (eq. 2.9)
  R inv_sig[kMaxN][kMaxN];// 1 / sigma_ij, 0 on the diagonal
  R rho[kMaxN], nu[kMaxN], eta[kMaxN];
  R wf[19], wg[19];       // weights of the phase / flow velocity sets
  R sf[6], sg[6];         // rates per relaxation slot (s0 s1 s21 s22 s3 s4)
  R two_over_c2mcs2;      // 2 / (c^2 - c_s^2)  (eq. 16, s21)
  R h2diag;               // 1 / (c^2 c_s^2 - c_s^4)   (eqs. 3.10, 3.11)
  R h2off;                // 1 / c_s^4
  R inv_c2mcs2;           // 1 / (c^2 - c_s^2)  (s_0 of eq. 3.11)
  R pref;                 // c_s^2 / (1 - w_0)          (eq. 19)
  R cgr;                  // 1/2 + K (1 - d0)(2 - s0) / (2 s0)   (eq. 19)
  R halfK;                // K / (2 c^2)                (eq. 19)
  R KH;                   // K * (1 - 2 d0) in 2D, K (3 - 7 d0)/2 in 3D
  R one_m3cs2;            // c^2 - 3 c_s^2              (eq. 3.12)
  // Fourth-order Hermite moments of the second-order expansion used in the
  // flow equilibrium and source (eqs. 3.10, 3.11): for the j-th fourth-order
  // row k of the flow set, q4[j][g] = sum_p w_p H_k(c_p) (c_pg^2 - c_s^2) /
  // (c^2 c_s^2 - c_s^4). Zero on D2Q9.
  R q4[3][3];
  R accel[3];             // body acceleration: force psi rho a
  R force[3];             // body force density: force psi G
};

}  // namespace ddcc
