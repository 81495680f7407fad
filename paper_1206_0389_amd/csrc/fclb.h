// D3Q27 factorized cascaded (FCLB) collision for gfx950.
//
// Central moments (Eqs. (14)-(15)) are taken per unit mass about the local
// velocity u = j / rho (Eqs. (6)-(8)). The shear part of the second order
// relaxes with omega = 1/tau0, every other group with rate 1 (Section 2:
// s_i = 1 for i != 1): the trace goes to 1, orders 3 and 5 to 0, and the
// fourth and sixth orders to the factorized equilibria of Table 2, products
// of the relaxed second-order central moments. The whole post-collision
// moment set is recomputed and transformed back (the paper's "recompute"
// variant).
//
// Both transforms factor over the axes: with D3Q27 = {-1,0,1}^3 the central
// moment matrix is a Kronecker product of three 3x3 matrices, so each
// transform is three sweeps of nine 3-point transforms held in registers.
// The arithmetic runs on deviations f_i - w_i: the rest weights factor as
// w = phi(ex) phi(ey) phi(ez) with phi = (1/6, 2/3, 1/6), whose central
// moments about u are c0 = 1, c1 = -u, c2 = 1/3 + u^2, so the rest part is
// added in closed form and every quantity in the registers stays small.
// That keeps FP32 arithmetic at the accuracy of FP32 storage.
#pragma once

#include "stencil.h"

namespace lbm {

// (f(-1), f(0), f(+1)) -> central moments of order 0, 1, 2 about u.
template <typename real>
__device__ __forceinline__ void central3(real& a0, real& a1, real& a2, real u) {
  const real s = a0 + a1 + a2;
  const real dif = a2 - a0;
  const real sum = a2 + a0;
  a0 = s;
  a1 = dif - u * s;
  a2 = sum - real(2) * u * dif + u * u * s;
}

// Inverse of central3.
template <typename real>
__device__ __forceinline__ void uncentral3(real& a0, real& a1, real& a2, real u) {
  const real m1 = a1 + u * a0;
  const real m2 = a2 + u * (real(2) * a1 + u * a0);
  const real m0 = a0;
  a0 = real(0.5) * (m2 - m1);
  a1 = m0 - m2;
  a2 = real(0.5) * (m2 + m1);
}

// Macroscopic quantities and relaxed second-order central moments of one
// node: everything the post-collision moment set depends on.
template <typename real>
struct FclbState {
  real drho, inv, ux, uy, uz;
  real ax, ay, az, bxy, bxz, byz;  // relaxed rho (kappa_aa - T/3), rho kappa_ab
};

// Forward central transform of the deviations (only the second order is
// used: every other group relaxes with rate 1) and the shear relaxation.
template <typename real>
__device__ __forceinline__ FclbState<real> fclb_relax(const real (&f)[27], real omega) {
  real A[3][3][3];
  real drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    A[cx(i) + 1][cy(i) + 1][cz(i) + 1] = f[i];
    drho += f[i];
    if (cx(i)) jx += cx(i) > 0 ? f[i] : -f[i];
    if (cy(i)) jy += cy(i) > 0 ? f[i] : -f[i];
    if (cz(i)) jz += cz(i) > 0 ? f[i] : -f[i];
  }
  FclbState<real> s;
  s.drho = drho;
  const real rho = real(1) + drho;
  s.inv = real(1) / rho;
  s.ux = jx * s.inv;
  s.uy = jy * s.inv;
  s.uz = jz * s.inv;
  const real ux = s.ux, uy = s.uy, uz = s.uz;

  // Central moments D_abc of the deviations about u.
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) central3(A[a][b][0], A[a][b][1], A[a][b][2], uz);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) central3(A[a][0][c], A[a][1][c], A[a][2][c], uy);
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) central3(A[0][b][c], A[1][b][c], A[2][b][c], ux);

  const real third = real(1.0 / 3.0);
  const real omc = real(1) - omega;
  const real uu = ux * ux + uy * uy + uz * uz;
  const real dtr = A[2][0][0] + A[0][2][0] + A[0][0][2];
  // rho (kappa_aa - T/3) relaxed with omega; rho kappa_ab relaxed with omega
  s.ax = omc * ((ux * ux + A[2][0][0]) - third * (uu + dtr));
  s.ay = omc * ((uy * uy + A[0][2][0]) - third * (uu + dtr));
  s.az = omc * ((uz * uz + A[0][0][2]) - third * (uu + dtr));
  s.bxy = omc * (ux * uy + A[1][1][0]);
  s.bxz = omc * (ux * uz + A[1][0][1]);
  s.byz = omc * (uy * uz + A[0][1][1]);
  return s;
}

// Post-collision central moments G = rho kappa* minus the central moments
// of the rest weights about u, then the inverse transform to deviations.
// GAUSS: the cascaded scheme before the factorization (CLB): orders 4 and 6
// relax to the Gaussian's central moments (rho/9, 0, rho/27) instead of the
// products of the relaxed second order.
template <typename real, bool GAUSS = false>
__device__ __forceinline__ void fclb_post(const FclbState<real>& s, real (&A)[3][3][3]) {
  const real drho = s.drho, inv = s.inv, ux = s.ux, uy = s.uy, uz = s.uz;
  const real ax = s.ax, ay = s.ay, az = s.az, bxy = s.bxy, bxz = s.bxz, byz = s.byz;
  const real third = real(1.0 / 3.0);
  const real ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  const real uu = ux2 + uy2 + uz2;
  const real c2x = third + ux2, c2y = third + uy2, c2z = third + uz2;
  A[0][0][0] = drho;
  A[1][0][0] = ux;
  A[0][1][0] = uy;
  A[0][0][1] = uz;
  A[2][0][0] = third * drho + ax - ux2;
  A[0][2][0] = third * drho + ay - uy2;
  A[0][0][2] = third * drho + az - uz2;
  A[1][1][0] = bxy - ux * uy;
  A[1][0][1] = bxz - ux * uz;
  A[0][1][1] = byz - uy * uz;
  A[2][1][0] = c2x * uy;
  A[2][0][1] = c2x * uz;
  A[1][2][0] = ux * c2y;
  A[0][2][1] = c2y * uz;
  A[1][0][2] = ux * c2z;
  A[0][1][2] = uy * c2z;
  A[1][1][1] = ux * uy * uz;
  const real ninth = real(1.0 / 9.0);
  if constexpr (GAUSS) {
    A[2][2][0] = ninth * drho - third * (ux2 + uy2) - ux2 * uy2;
    A[2][0][2] = ninth * drho - third * (ux2 + uz2) - ux2 * uz2;
    A[0][2][2] = ninth * drho - third * (uy2 + uz2) - uy2 * uz2;
    A[2][1][1] = -(third + ux2) * uy * uz;
    A[1][2][1] = -(third + uy2) * ux * uz;
    A[1][1][2] = -(third + uz2) * ux * uy;
  } else {
    A[2][2][0] = ninth * drho + third * (ax + ay - ux2 - uy2) + ax * ay * inv - ux2 * uy2;
    A[2][0][2] = ninth * drho + third * (ax + az - ux2 - uz2) + ax * az * inv - ux2 * uz2;
    A[0][2][2] = ninth * drho + third * (ay + az - uy2 - uz2) + ay * az * inv - uy2 * uz2;
    A[2][1][1] = third * (byz - uy * uz) + ax * inv * byz - ux2 * uy * uz;
    A[1][2][1] = third * (bxz - ux * uz) + ay * inv * bxz - uy2 * ux * uz;
    A[1][1][2] = third * (bxy - ux * uy) + az * inv * bxy - uz2 * ux * uy;
  }
  A[2][2][1] = c2x * c2y * uz;
  A[2][1][2] = c2x * uy * c2z;
  A[1][2][2] = ux * c2y * c2z;
  if constexpr (GAUSS)
    A[2][2][2] = real(1.0 / 27.0) * drho - ninth * uu -
                 third * (ux2 * uy2 + ux2 * uz2 + uy2 * uz2) - ux2 * uy2 * uz2;
  else
    A[2][2][2] = real(1.0 / 27.0) * drho + ninth * (ax + ay + az - uu) +
                 third * inv * (ax * ay + ax * az + ay * az) + ax * ay * az * inv * inv -
                 third * (ux2 * uy2 + ux2 * uz2 + uy2 * uz2) - ux2 * uy2 * uz2;

#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) uncentral3(A[0][b][c], A[1][b][c], A[2][b][c], ux);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) uncentral3(A[a][0][c], A[a][1][c], A[a][2][c], uy);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) uncentral3(A[a][b][0], A[a][b][1], A[a][b][2], uz);
}

template <typename real, bool GAUSS = false>
__device__ __forceinline__ void fclb_collide(real (&f)[27], real omega) {
  const FclbState<real> s = fclb_relax(f, omega);
  real A[3][3][3];
  fclb_post<real, GAUSS>(s, A);
#pragma unroll
  for (int i = 0; i < 27; ++i) f[i] = A[cx(i) + 1][cy(i) + 1][cz(i) + 1];
}

}  // namespace lbm
