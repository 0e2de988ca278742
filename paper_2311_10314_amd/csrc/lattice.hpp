// Lattice traits of the HIP path: velocity sets, Hermite rows of the
// collision matrix and compile-time moment tables.
//
// Velocity sets and weights: Section 3 lattice tables (D2Q9, D3Q7, D3Q15);
// D3Q19 weights solve the same moment constraints (sum w = 1,
// sum w c_x^2 = d0, sum w c_x^2 c_y^2 = d0^2). Hermite rows (eq. 3.4's H,
// not printed in the paper): products of 1, c_a and c_a^2 - c_s^2 ordered as
// the printed relaxation matrices S.
//
// The transform m = H d is done as m = A(c_s^2) (R d): R is H at c_s^2 = 0
// (integer "raw" monomials, applied as sparse adds), A(c_s^2) is unit lower
// triangular with integer polynomial entries. The inverse uses forward
// substitution through A and the constant R^-1, all with compile-time
// sparsity, so no runtime matrix is stored.
#pragma once

#include <utility>

namespace ddcc {

struct Vel {
  int x, y, z;
};

// Per-axis factor codes of a Hermite term: 0 -> 1, 1 -> c_a,
// 2 -> c_a^2 - c_s^2.
struct Term {
  int f[3];
};

struct Row {
  int nterm;
  Term t[3];
  int group;  // relaxation slot: 0 s0, 1 s1, 2 s21, 3 s22, 4 s3, 5 s4
};

enum { GR0 = 0, GR1 = 1, GR21 = 2, GR22 = 3, GR3 = 4, GR4 = 5 };

// Weight shells: index = c.c (0 rest, 1 face, 2 edge, 3 corner).
struct D2Q9 {
  static constexpr int Q = 9, D = 2, ID = 0;
  static constexpr Vel c[Q] = {{0, 0, 0},  {1, 0, 0},   {0, 1, 0},
                               {-1, 0, 0}, {0, -1, 0},  {1, 1, 0},
                               {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
  static constexpr Row rows[Q] = {
      {1, {{{0, 0, 0}}}, GR0},  {1, {{{1, 0, 0}}}, GR1},
      {1, {{{0, 1, 0}}}, GR1},  {1, {{{2, 0, 0}}}, GR21},
      {1, {{{0, 2, 0}}}, GR21}, {1, {{{1, 1, 0}}}, GR22},
      {1, {{{2, 1, 0}}}, GR3},  {1, {{{1, 2, 0}}}, GR3},
      {1, {{{2, 2, 0}}}, GR4}};
};

struct D3Q7 {
  static constexpr int Q = 7, D = 3, ID = 1;
  static constexpr Vel c[Q] = {{0, 0, 0},  {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                               {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
  static constexpr Row rows[Q] = {
      {1, {{{0, 0, 0}}}, GR0},  {1, {{{1, 0, 0}}}, GR1},
      {1, {{{0, 1, 0}}}, GR1},  {1, {{{0, 0, 1}}}, GR1},
      {1, {{{2, 0, 0}}}, GR21}, {1, {{{0, 2, 0}}}, GR21},
      {1, {{{0, 0, 2}}}, GR21}};
};

struct D3Q15 {
  static constexpr int Q = 15, D = 3, ID = 2;
  static constexpr Vel c[Q] = {
      {0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
      {0, 0, 1},   {0, 0, -1},  {1, 1, 1},   {1, 1, -1}, {1, -1, 1},
      {1, -1, -1}, {-1, 1, 1},  {-1, 1, -1}, {-1, -1, 1}, {-1, -1, -1}};
  static constexpr Row rows[Q] = {
      {1, {{{0, 0, 0}}}, GR0},
      {1, {{{1, 0, 0}}}, GR1},
      {1, {{{0, 1, 0}}}, GR1},
      {1, {{{0, 0, 1}}}, GR1},
      {1, {{{2, 0, 0}}}, GR21},
      {1, {{{0, 2, 0}}}, GR21},
      {1, {{{0, 0, 2}}}, GR21},
      {1, {{{1, 1, 0}}}, GR22},
      {1, {{{1, 0, 1}}}, GR22},
      {1, {{{0, 1, 1}}}, GR22},
      {2, {{{1, 2, 0}}, {{1, 0, 2}}}, GR3},
      {2, {{{2, 1, 0}}, {{0, 1, 2}}}, GR3},
      {2, {{{2, 0, 1}}, {{0, 2, 1}}}, GR3},
      {1, {{{1, 1, 1}}}, GR3},
      {3, {{{2, 2, 0}}, {{2, 0, 2}}, {{0, 2, 2}}}, GR4}};
};

struct D3Q19 {
  static constexpr int Q = 19, D = 3, ID = 3;
  static constexpr Vel c[Q] = {
      {0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
      {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {1, -1, 0},  {-1, 1, 0},
      {-1, -1, 0}, {1, 0, 1}, {1, 0, -1}, {-1, 0, 1},  {-1, 0, -1},
      {0, 1, 1},  {0, 1, -1}, {0, -1, 1}, {0, -1, -1}};
  static constexpr Row rows[Q] = {
      {1, {{{0, 0, 0}}}, GR0},  {1, {{{1, 0, 0}}}, GR1},
      {1, {{{0, 1, 0}}}, GR1},  {1, {{{0, 0, 1}}}, GR1},
      {1, {{{2, 0, 0}}}, GR21}, {1, {{{0, 2, 0}}}, GR21},
      {1, {{{0, 0, 2}}}, GR21}, {1, {{{1, 1, 0}}}, GR22},
      {1, {{{1, 0, 1}}}, GR22}, {1, {{{0, 1, 1}}}, GR22},
      {1, {{{2, 1, 0}}}, GR3},  {1, {{{2, 0, 1}}}, GR3},
      {1, {{{1, 2, 0}}}, GR3},  {1, {{{0, 2, 1}}}, GR3},
      {1, {{{1, 0, 2}}}, GR3},  {1, {{{0, 1, 2}}}, GR3},
      {1, {{{2, 2, 0}}}, GR4},  {1, {{{2, 0, 2}}}, GR4},
      {1, {{{0, 2, 2}}}, GR4}};
};

// ---------------------------------------------------------------------------
// Compile-time tables
// ---------------------------------------------------------------------------
constexpr int kMaxQ = 19;

struct Tables {
  int Q;
  double R[kMaxQ][kMaxQ];     // raw monomial matrix (H at c_s^2 = 0)
  double Rinv[kMaxQ][kMaxQ];  // its inverse (multiples of 1/192)
  double A[4][kMaxQ][kMaxQ];  // H = (I + sum_d cs2^d A[d]) R, A[0] unused
  double shell[kMaxQ];        // c.c of each velocity
};

constexpr double cabs(double x) { return x < 0 ? -x : x; }

constexpr double cround(double x, double q) {
  double y = x * q;
  long long i = static_cast<long long>(y + (y >= 0 ? 0.5 : -0.5));
  return static_cast<double>(i) / q;
}

// Polynomial in cs2 (degree <= 3) of one factor code at one component.
struct Poly {
  double a[4];
};

constexpr Poly poly_factor(int code, int comp) {
  Poly p{{0, 0, 0, 0}};
  if (code == 0) {
    p.a[0] = 1;
  } else if (code == 1) {
    p.a[0] = comp;
  } else {
    p.a[0] = comp * comp;
    p.a[1] = -1;
  }
  return p;
}

constexpr Poly poly_mul(Poly x, Poly y) {
  Poly r{{0, 0, 0, 0}};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; i + j < 4; ++j) r.a[i + j] += x.a[i] * y.a[j];
  return r;
}

template <class L>
constexpr Tables make_tables() {
  Tables t{};
  const int Q = L::Q;
  t.Q = Q;
  double P[4][kMaxQ][kMaxQ] = {};
  for (int k = 0; k < Q; ++k)
    for (int p = 0; p < Q; ++p) {
      const int cc[3] = {L::c[p].x, L::c[p].y, L::c[p].z};
      for (int m = 0; m < L::rows[k].nterm; ++m) {
        Poly acc{{1, 0, 0, 0}};
        for (int a = 0; a < 3; ++a)
          acc = poly_mul(acc, poly_factor(L::rows[k].t[m].f[a], cc[a]));
        for (int d = 0; d < 4; ++d) P[d][k][p] += acc.a[d];
      }
    }
  for (int p = 0; p < Q; ++p)
    t.shell[p] = L::c[p].x * L::c[p].x + L::c[p].y * L::c[p].y +
                 L::c[p].z * L::c[p].z;
  // R = P[0]; invert by Gauss-Jordan with partial pivoting.
  double M[kMaxQ][2 * kMaxQ] = {};
  for (int i = 0; i < Q; ++i) {
    for (int j = 0; j < Q; ++j) {
      t.R[i][j] = P[0][i][j];
      M[i][j] = P[0][i][j];
    }
    M[i][Q + i] = 1;
  }
  for (int col = 0; col < Q; ++col) {
    int piv = col;
    for (int r = col + 1; r < Q; ++r)
      if (cabs(M[r][col]) > cabs(M[piv][col])) piv = r;
    for (int j = 0; j < 2 * Q; ++j) {
      double tmp = M[col][j];
      M[col][j] = M[piv][j];
      M[piv][j] = tmp;
    }
    double inv = 1.0 / M[col][col];
    for (int j = 0; j < 2 * Q; ++j) M[col][j] *= inv;
    for (int r = 0; r < Q; ++r) {
      if (r == col) continue;
      double f = M[r][col];
      if (f == 0) continue;
      for (int j = 0; j < 2 * Q; ++j) M[r][j] -= f * M[col][j];
    }
  }
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j) t.Rinv[i][j] = cround(M[i][Q + j], 192.0);
  // A[d] = P[d] R^-1 (integer entries)
  for (int d = 1; d < 4; ++d)
    for (int i = 0; i < Q; ++i)
      for (int j = 0; j < Q; ++j) {
        double s = 0;
        for (int k = 0; k < Q; ++k) s += P[d][i][k] * t.Rinv[k][j];
        t.A[d][i][j] = cround(s, 1.0);
      }
  return t;
}

template <class L>
constexpr bool check_tables(const Tables& t) {
  const int Q = L::Q;
  // R Rinv == I to rounding (entries are k/192)
  for (int i = 0; i < Q; ++i)
    for (int j = 0; j < Q; ++j) {
      double s = 0;
      for (int k = 0; k < Q; ++k) s += t.R[i][k] * t.Rinv[k][j];
      if (cabs(s - (i == j ? 1.0 : 0.0)) > 1e-12) return false;
    }
  // A strictly lower triangular (rows are graded by polynomial degree)
  for (int d = 1; d < 4; ++d)
    for (int i = 0; i < Q; ++i)
      for (int j = i; j < Q; ++j)
        if (t.A[d][i][j] != 0) return false;
  return true;
}

template <class L>
struct Tab {
  static constexpr Tables t = make_tables<L>();
  static_assert(check_tables<L>(t), "lattice tables inconsistent");
};

// ---------------------------------------------------------------------------
// Sparse unrolled transforms (R: arithmetic type)
// ---------------------------------------------------------------------------
template <class L, int k, int p, class R>
__host__ __device__ inline void raw_term(R& acc, const R* d) {
  constexpr double v = Tab<L>::t.R[k][p];
  if constexpr (v == 1.0) {
    acc += d[p];
  } else if constexpr (v == -1.0) {
    acc -= d[p];
  } else if constexpr (v != 0.0) {
    acc += R(v) * d[p];
  }
}

template <class L, int k, class R, int... p>
__host__ __device__ inline R raw_row(const R* d,
                                     std::integer_sequence<int, p...>) {
  R acc = R(0);
  (raw_term<L, k, p>(acc, d), ...);
  return acc;
}

template <class L, int k, int j, class R>
__host__ __device__ inline void herm_term(R& acc, const R* r, R cs2, R cs4,
                                          R cs6) {
  constexpr double a1 = Tab<L>::t.A[1][k][j];
  constexpr double a2 = Tab<L>::t.A[2][k][j];
  constexpr double a3 = Tab<L>::t.A[3][k][j];
  if constexpr (a1 != 0.0) acc += R(a1) * cs2 * r[j];
  if constexpr (a2 != 0.0) acc += R(a2) * cs4 * r[j];
  if constexpr (a3 != 0.0) acc += R(a3) * cs6 * r[j];
}

template <class L, int k, class R, int... j>
__host__ __device__ inline R herm_row(const R* r, R cs2, R cs4, R cs6,
                                      std::integer_sequence<int, j...>) {
  R acc = r[k];
  (herm_term<L, k, j>(acc, r, cs2, cs4, cs6), ...);
  return acc;
}

template <class L, class R, int... k>
__host__ __device__ inline void to_hermite_impl(const R* d, R* m, R cs2,
                                                std::integer_sequence<int, k...>) {
  R r[L::Q];
  ((r[k] = raw_row<L, k>(d, std::make_integer_sequence<int, L::Q>{})), ...);
  const R cs4 = cs2 * cs2, cs6 = cs4 * cs2;
  ((m[k] = herm_row<L, k>(r, cs2, cs4, cs6,
                          std::make_integer_sequence<int, k>{})), ...);
}

// m = H d
template <class L, class R>
__host__ __device__ inline void to_hermite(const R* d, R* m, R cs2) {
  to_hermite_impl<L>(d, m, cs2, std::make_integer_sequence<int, L::Q>{});
}

template <class L, int k, int j, class R>
__host__ __device__ inline void unherm_term(R& acc, const R* r, R cs2, R cs4,
                                            R cs6) {
  constexpr double a1 = Tab<L>::t.A[1][k][j];
  constexpr double a2 = Tab<L>::t.A[2][k][j];
  constexpr double a3 = Tab<L>::t.A[3][k][j];
  if constexpr (a1 != 0.0) acc -= R(a1) * cs2 * r[j];
  if constexpr (a2 != 0.0) acc -= R(a2) * cs4 * r[j];
  if constexpr (a3 != 0.0) acc -= R(a3) * cs6 * r[j];
}

template <class L, int k, class R, int... j>
__host__ __device__ inline void unherm_row(const R* m, R* r, R cs2, R cs4,
                                           R cs6,
                                           std::integer_sequence<int, j...>) {
  R acc = m[k];
  (unherm_term<L, k, j>(acc, r, cs2, cs4, cs6), ...);
  r[k] = acc;
}

template <class L, int p, int k, class R>
__host__ __device__ inline void inv_term(R& acc, const R* r) {
  constexpr double v = Tab<L>::t.Rinv[p][k];
  if constexpr (v == 1.0) {
    acc += r[k];
  } else if constexpr (v == -1.0) {
    acc -= r[k];
  } else if constexpr (v != 0.0) {
    acc += R(v) * r[k];
  }
}

template <class L, int p, class R, int... k>
__host__ __device__ inline R inv_row(const R* r,
                                     std::integer_sequence<int, k...>) {
  R acc = R(0);
  (inv_term<L, p, k>(acc, r), ...);
  return acc;
}

template <class L, class R, int... k>
__host__ __device__ inline void from_hermite_impl(const R* m, R* out, R cs2,
                                                  std::integer_sequence<int, k...>) {
  R r[L::Q];
  const R cs4 = cs2 * cs2, cs6 = cs4 * cs2;
  // forward substitution through the unit lower-triangular A(cs2)
  (unherm_row<L, k>(m, r, cs2, cs4, cs6, std::make_integer_sequence<int, k>{}),
   ...);
  ((out[k] = inv_row<L, k>(r, std::make_integer_sequence<int, L::Q>{})), ...);
}

// out = H^-1 m
template <class L, class R>
__host__ __device__ inline void from_hermite(const R* m, R* out, R cs2) {
  from_hermite_impl<L>(m, out, cs2, std::make_integer_sequence<int, L::Q>{});
}

template <class L, class R, int... k>
__host__ __device__ inline void raw_impl(const R* d, R* r,
                                         std::integer_sequence<int, k...>) {
  ((r[k] = raw_row<L, k>(d, std::make_integer_sequence<int, L::Q>{})), ...);
}

// r = R d: raw monomial moments (integer coefficients, sparse adds)
template <class L, class R>
__host__ __device__ inline void raw_moments(const R* d, R* r) {
  raw_impl<L>(d, r, std::make_integer_sequence<int, L::Q>{});
}

template <class L, class R, int... k>
__host__ __device__ inline void r2h_impl(const R* r, R* m, R cs2,
                                         std::integer_sequence<int, k...>) {
  const R cs4 = cs2 * cs2, cs6 = cs4 * cs2;
  ((m[k] = herm_row<L, k>(r, cs2, cs4, cs6,
                          std::make_integer_sequence<int, k>{})), ...);
}

// m = A(cs2) r: Hermite moments from raw moments
template <class L, class R>
__host__ __device__ inline void raw_to_hermite(const R* r, R* m, R cs2) {
  r2h_impl<L>(r, m, cs2, std::make_integer_sequence<int, L::Q>{});
}

// Order of a Hermite row (number of c factors, counting c^2 - cs2 as two).
template <class L>
__host__ __device__ constexpr int row_order(int k) {
  int o = 0;
  for (int a = 0; a < 3; ++a) o += L::rows[k].t[0].f[a];
  return o;
}

// Value of Hermite row k at c = 0 divided by (-cs2)^(order/2): the product
// of its (c_a^2 - cs2) factors is (-cs2)^m, summed over the row's terms,
// and rows with a bare c_a factor vanish there. Returns the integer
// multiplicity (0 for rows that vanish at rest).
template <class L>
__host__ __device__ constexpr int rest_multiplicity(int k) {
  int mult = 0;
  for (int t = 0; t < L::rows[k].nterm; ++t) {
    bool zero = false;
    for (int a = 0; a < 3; ++a)
      if (L::rows[k].t[t].f[a] == 1) zero = true;
    if (!zero) ++mult;
  }
  return mult;
}

// Value of Hermite row k at c = 0, a polynomial in cs2.
template <class L, int k, class R>
__host__ __device__ inline R rest_value(R cs2) {
  R v = R(0);
#pragma unroll
  for (int t = 0; t < L::rows[k].nterm; ++t) {
    R prod = R(1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int f = L::rows[k].t[t].f[a];
      if (f == 1) prod = R(0);
      if (f == 2) prod *= -cs2;
    }
    v += prod;
  }
  return v;
}

// Hermite row k evaluated at velocity c (host-side, for derived constants).
template <class L>
inline double row_value(int k, int p, double cs2) {
  const int cc[3] = {L::c[p].x, L::c[p].y, L::c[p].z};
  double v = 0;
  for (int t = 0; t < L::rows[k].nterm; ++t) {
    double prod = 1;
    for (int a = 0; a < 3; ++a) {
      const int f = L::rows[k].t[t].f[a];
      if (f == 1) prod *= cc[a];
      if (f == 2) prod *= cc[a] * cc[a] - cs2;
    }
    v += prod;
  }
  return v;
}

// Index among the fourth-order rows (0, 1, 2) of row k, -1 otherwise.
template <class L>
__host__ __device__ constexpr int g4_index(int k) {
  int j = -1;
  for (int q = 0; q <= k; ++q)
    if (L::rows[q].group == GR4) ++j;
  return L::rows[k].group == GR4 ? j : -1;
}

// Component of a first-order row / diagonal second-order row, and the pair
// index (xy, xz, yz) of an off-diagonal second-order row.
template <class L>
__host__ __device__ constexpr int row_comp(int k) {
  for (int a = 0; a < 3; ++a)
    if (L::rows[k].t[0].f[a] != 0) return a;
  return -1;
}

template <class L>
__host__ __device__ constexpr int row_pair(int k) {
  // (x, y) -> 0, (x, z) -> 1, (y, z) -> 2
  const int* f = L::rows[k].t[0].f;
  if (f[0] && f[1]) return 0;
  if (f[0] && f[2]) return 1;
  return 2;
}

// Relaxation slot of Hermite row k.
template <class L>
__host__ __device__ constexpr int row_group(int k) {
  return L::rows[k].group;
}

}  // namespace ddcc
