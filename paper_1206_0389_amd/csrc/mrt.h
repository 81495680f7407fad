// D3Q19 MRT collision with a Smagorinsky eddy viscosity, for gfx950.
//
// Eq. (12) read as a relaxation, f* = f - M^-1 S (M f - m_eq), m_eq = M f_eq
// with the incompressible equilibrium of Eq. (2) (deviation form, rho0 = 1).
// The shear rows relax with 1/tau_total from the closed form Eqs. (20)-(21),
// Q = sqrt(2 Pi:Pi), Pi = sum_i e_i e_i (f_i - f_eq_i) (Eq. (19)).
//
// Both moment bases and their inverses are built at compile time; the
// kernels unroll every matrix-vector product so that zero entries vanish and
// +-1 entries become additions. Only the shear rate is per node.
#pragma once

#include "stencil.h"

namespace lbm {

// One moment row: a radial polynomial r0 + r1 |e|^2 + r2 |e|^4 times a sum
// of monomials coef * ex^a ey^b ez^c.
struct Mono {
  double coef;
  int a, b, c;
};
struct Row {
  double r[3];
  int n;
  Mono t[3];
  int group;  // 0 conserved, 1 shear (1/tau_total), 2+k runtime rate k
};

constexpr double ipow_c(int v, int p) {
  double r = 1.0;
  for (int k = 0; k < p; ++k) r *= v;
  return r;
}

// Moments grouped as in Table 1 (the s1..s7 groups that exist on D3Q19).
constexpr Row kTable1Rows[19] = {
    {{1, 0, 0}, 1, {{1, 0, 0, 0}}, 0},
    {{1, 0, 0}, 1, {{1, 1, 0, 0}}, 0},
    {{1, 0, 0}, 1, {{1, 0, 1, 0}}, 0},
    {{1, 0, 0}, 1, {{1, 0, 0, 1}}, 0},
    {{1, 0, 0}, 1, {{1, 1, 1, 0}}, 1},                         // mu_12
    {{1, 0, 0}, 1, {{1, 1, 0, 1}}, 1},                         // mu_13
    {{1, 0, 0}, 1, {{1, 0, 1, 1}}, 1},                         // mu_23
    {{1, 0, 0}, 2, {{1, 2, 0, 0}, {-1, 0, 2, 0}}, 1},          // mu_11 - mu_22
    {{1, 0, 0}, 2, {{1, 2, 0, 0}, {-1, 0, 0, 2}}, 1},          // mu_11 - mu_33
    {{0, 1, 0}, 1, {{1, 0, 0, 0}}, 2},                         // s2: trace
    {{1, 0, 0}, 2, {{1, 1, 2, 0}, {1, 1, 0, 2}}, 3},           // s3
    {{1, 0, 0}, 2, {{1, 2, 1, 0}, {1, 0, 1, 2}}, 3},
    {{1, 0, 0}, 2, {{1, 2, 0, 1}, {1, 0, 2, 1}}, 3},
    {{1, 0, 0}, 2, {{1, 1, 2, 0}, {-1, 1, 0, 2}}, 4},          // s4
    {{1, 0, 0}, 2, {{1, 2, 1, 0}, {-1, 0, 1, 2}}, 4},
    {{1, 0, 0}, 2, {{1, 2, 0, 1}, {-1, 0, 2, 1}}, 4},
    {{1, 0, 0}, 3, {{1, 2, 2, 0}, {-2, 2, 0, 2}, {1, 0, 2, 2}}, 5},  // s7
    {{1, 0, 0}, 3, {{1, 2, 2, 0}, {1, 2, 0, 2}, {-2, 0, 2, 2}}, 5},
    {{1, 0, 0}, 3, {{1, 2, 2, 0}, {1, 2, 0, 2}, {1, 0, 2, 2}}, 5},
};

// d'Humieres, Ginzburg, Krafczyk, Lallemand & Luo (2002) orthogonal D3Q19
// basis: energy, energy squared, heat flux, viscous stress, 4th-order
// stress and the antisymmetric 3rd-order moments.
constexpr Row kDhumieresRows[19] = {
    {{1, 0, 0}, 1, {{1, 0, 0, 0}}, 0},
    {{-30, 19, 0}, 1, {{1, 0, 0, 0}}, 2},                       // e
    {{12, -26.5, 10.5}, 1, {{1, 0, 0, 0}}, 3},                  // eps
    {{1, 0, 0}, 1, {{1, 1, 0, 0}}, 0},                          // j_x
    {{-9, 5, 0}, 1, {{1, 1, 0, 0}}, 4},                         // q_x
    {{1, 0, 0}, 1, {{1, 0, 1, 0}}, 0},                          // j_y
    {{-9, 5, 0}, 1, {{1, 0, 1, 0}}, 4},                         // q_y
    {{1, 0, 0}, 1, {{1, 0, 0, 1}}, 0},                          // j_z
    {{-9, 5, 0}, 1, {{1, 0, 0, 1}}, 4},                         // q_z
    {{1, 0, 0}, 3, {{2, 2, 0, 0}, {-1, 0, 2, 0}, {-1, 0, 0, 2}}, 1},   // 3 p_xx
    {{-5, 3, 0}, 3, {{2, 2, 0, 0}, {-1, 0, 2, 0}, {-1, 0, 0, 2}}, 5},  // 3 pi_xx
    {{1, 0, 0}, 2, {{1, 0, 2, 0}, {-1, 0, 0, 2}}, 1},           // p_ww
    {{-5, 3, 0}, 2, {{1, 0, 2, 0}, {-1, 0, 0, 2}}, 5},          // pi_ww
    {{1, 0, 0}, 1, {{1, 1, 1, 0}}, 1},                          // p_xy
    {{1, 0, 0}, 1, {{1, 0, 1, 1}}, 1},                          // p_yz
    {{1, 0, 0}, 1, {{1, 1, 0, 1}}, 1},                          // p_xz
    {{1, 0, 0}, 2, {{1, 1, 2, 0}, {-1, 1, 0, 2}}, 6},           // m_x
    {{1, 0, 0}, 2, {{1, 0, 1, 2}, {-1, 2, 1, 0}}, 6},           // m_y
    {{1, 0, 0}, 2, {{1, 2, 0, 1}, {-1, 0, 2, 1}}, 6},           // m_z
};

struct Mat19 {
  double a[19][19];
};

constexpr double eval_row(const Row& r, int i) {
  const double e2 = cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i);
  double s = 0.0;
  for (int k = 0; k < r.n; ++k)
    s += r.t[k].coef * ipow_c(cx(i), r.t[k].a) * ipow_c(cy(i), r.t[k].b) *
         ipow_c(cz(i), r.t[k].c);
  return (r.r[0] + r.r[1] * e2 + r.r[2] * e2 * e2) * s;
}

constexpr Mat19 build_basis(int basis) {
  Mat19 M{};
  for (int k = 0; k < 19; ++k)
    for (int i = 0; i < 19; ++i)
      M.a[k][i] = eval_row(basis == 0 ? kTable1Rows[k] : kDhumieresRows[k], i);
  return M;
}

constexpr double abs_c(double v) { return v < 0 ? -v : v; }

// Gauss-Jordan inverse with partial pivoting, evaluated by the compiler.
constexpr Mat19 invert19(const Mat19& A) {
  double w[19][38] = {};
  for (int r = 0; r < 19; ++r) {
    for (int c = 0; c < 19; ++c) w[r][c] = A.a[r][c];
    w[r][19 + r] = 1.0;
  }
  for (int c = 0; c < 19; ++c) {
    int p = c;
    for (int r = c + 1; r < 19; ++r)
      if (abs_c(w[r][c]) > abs_c(w[p][c])) p = r;
    if (p != c)
      for (int k = 0; k < 38; ++k) {
        const double t = w[c][k];
        w[c][k] = w[p][k];
        w[p][k] = t;
      }
    const double piv = w[c][c];
    for (int k = 0; k < 38; ++k) w[c][k] /= piv;
    for (int r = 0; r < 19; ++r)
      if (r != c && w[r][c] != 0.0) {
        const double l = w[r][c];
        for (int k = 0; k < 38; ++k) w[r][k] -= l * w[c][k];
      }
  }
  Mat19 R{};
  for (int r = 0; r < 19; ++r)
    for (int c = 0; c < 19; ++c) R.a[r][c] = w[r][19 + c];
  return R;
}

constexpr int row_group(int basis, int k) {
  return basis == 0 ? kTable1Rows[k].group : kDhumieresRows[k].group;
}

template <int BASIS>
struct MrtTables {
  static constexpr Mat19 M = build_basis(BASIS);
  static constexpr Mat19 Minv = invert19(M);
};

// Entries below this magnitude are exact zeros of the rational inverse.
constexpr bool is_nonzero(double v) { return abs_c(v) > 1e-12; }

struct MrtParams {
  double tau0;     // 3 nu + 1/2
  double cs18;     // 18 C_S^2
  double rates[5]; // runtime non-shear rates (groups 2+k)
};

template <typename real, int BASIS>
__device__ __forceinline__ void mrt_collide(real (&f)[19], const MrtParams& p) {
  using T = MrtTables<BASIS>;
  real drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    drho += f[i];
    if (cx(i)) jx += cx(i) > 0 ? f[i] : -f[i];
    if (cy(i)) jy += cy(i) > 0 ? f[i] : -f[i];
    if (cz(i)) jz += cz(i) > 0 ? f[i] : -f[i];
  }
  const real uu = jx * jx + jy * jy + jz * jz;
  // d_i = f_i - f_eq_i (Eq. (2), rho0 = 1, u = j)
  real d[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const real eu = real(cx(i)) * jx + real(cy(i)) * jy + real(cz(i)) * jz;
    const real feq = real(weight<19>(i)) *
                     (drho + real(3) * eu + real(4.5) * eu * eu - real(1.5) * uu);
    d[i] = f[i] - feq;
  }
  // non-equilibrium momentum flux and the strain-dependent tau
  real pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    if (cx(i)) pxx += d[i];
    if (cy(i)) pyy += d[i];
    if (cz(i)) pzz += d[i];
    if (cx(i) * cy(i)) pxy += cx(i) * cy(i) > 0 ? d[i] : -d[i];
    if (cx(i) * cz(i)) pxz += cx(i) * cz(i) > 0 ? d[i] : -d[i];
    if (cy(i) * cz(i)) pyz += cy(i) * cz(i) > 0 ? d[i] : -d[i];
  }
  const real pi2 = pxx * pxx + pyy * pyy + pzz * pzz +
                   real(2) * (pxy * pxy + pxz * pxz + pyz * pyz);
  const real Qs = sqrt(real(2) * pi2);
  const real tau0 = real(p.tau0);
  const real tau = real(0.5) * (tau0 + sqrt(tau0 * tau0 + real(p.cs18) * Qs));
  const real s_shear = real(1) / tau;
  real rate[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) rate[k] = real(p.rates[k]);
  // relaxed moment differences S (M d)
  real dm[19];
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    dm[k] = 0;
    if (row_group(BASIS, k) == 0) continue;
    real acc = 0;
#pragma unroll
    for (int i = 0; i < 19; ++i)
      if (is_nonzero(T::M.a[k][i])) acc += real(T::M.a[k][i]) * d[i];
    const int g = row_group(BASIS, k);
    dm[k] = acc * (g == 1 ? s_shear : rate[g - 2]);
  }
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    real c = 0;
#pragma unroll
    for (int k = 0; k < 19; ++k)
      if (row_group(BASIS, k) != 0 && is_nonzero(T::Minv.a[i][k]))
        c += real(T::Minv.a[i][k]) * dm[k];
    f[i] -= c;
  }
}

}  // namespace lbm
