// Discrete adjoint of the D3Q27 FCLB and D3Q19 MRT-LES collide-and-stream
// steps for gfx950.
//
// One step maps the pre-collision state f_t to f_{t+1} = S(C(f_t); u_in):
// collide every node, then stream with the boundary rules (periodic wrap,
// halfway bounce-back with 6 w_i e_i.u at WALL and INLET faces, zero-gradient
// copy at an OUTFLOW face). For an objective J(f_T) the adjoint runs
//   mu = S^T lambda_{t+1},   lambda_t = J_C(f_t)^T mu,
// node by node, and the inlet velocity's gradient collects the bounce-back
// terms: dJ/du_in(x) += sum over inlet-crossing i of 6 w_i e_i lambda_{t+1,i}(x).
//
// S^T is taken in gather form, one thread per node x: population i of x went
// to x + e_i (in the domain), or back to x as opp(i) (a WALL/INLET face lies
// beyond), or nowhere (only an OUTFLOW face beyond); a node on the outflow
// plane also feeds the ghost copy read by its in-plane neighbour x + e_i with
// the normal component dropped. These are the forward pull rules read from
// the source side.
//
// J_C^T is the hand-derived reverse mode of the factorized collision in
// fclb.h: the inverse transform is a Kronecker product of three 3-point maps
// o = R S(u) a along the axes, so its transpose is three sweeps of
// a_bar = S(u)^T R^T o_bar, and because the three axis maps commute, its
// derivative in u_x is (R N R^-1 along x) applied to the outputs, N the
// derivation m_k -> k m_{k-1} of raw moments: no intermediate stage has to
// be kept. Then the post-collision moment formulas, the shear relaxation,
// the second-order central moments (dD_ab/du from the first central moments,
// which for deviations equal u) and u = j / rho are differentiated by hand.
//
// The MRT-LES collision (Eq. 12 with the relaxation time of Eqs. 16-21) is
// reversed the same way in mrt_vjp: the moment relaxation is a fixed linear
// map apart from the shear rate 1/tau, whose dependence on the node runs
// through the strain magnitude Q of the non-equilibrium momentum flux.
#pragma once

#include "fclb.h"
#include "kernels.h"
#include "mrt.h"

namespace lbm {

// Transpose of uncentral3's linear map, in place on (o0, o1, o2).
template <typename real>
__device__ __forceinline__ void uncentral3_t(real& a0, real& a1, real& a2, real u) {
  const real m0 = a1;
  const real m1 = real(0.5) * (a2 - a0);
  const real m2 = real(0.5) * (a0 + a2) - a1;
  a0 = m0 + u * (m1 + u * m2);
  a1 = m1 + real(2) * u * m2;
  a2 = m2;
}

// <g, d(uncentral3 line)/du> from the line's outputs o: with raw moments
// m0 = o0 + o1 + o2, m1 = o2 - o0 the derivative is R (0, m0, 2 m1).
template <typename real>
__device__ __forceinline__ real uncentral3_du(real o0, real o1, real o2, real g0, real g1,
                                              real g2) {
  return (o2 - o0) * (g0 - real(2) * g1 + g2) + real(0.5) * (o0 + o1 + o2) * (g2 - g0);
}

// g <- J_C(f)^T g for the FCLB collision of one node (deviation form).
template <typename real>
__device__ __forceinline__ void fclb_vjp(const real (&f)[27], real (&g)[27], real omega) {
  const FclbState<real> s = fclb_relax(f, omega);
  const real ux = s.ux, uy = s.uy, uz = s.uz, inv = s.inv;
  const real ax = s.ax, ay = s.ay, az = s.az, bxy = s.bxy, bxz = s.bxz, byz = s.byz;
  real B[3][3][3];
#pragma unroll
  for (int i = 0; i < 27; ++i) B[cx(i) + 1][cy(i) + 1][cz(i) + 1] = g[i];

  // u-derivative of the inverse transform, from its outputs
  real ubx = 0, uby = 0, ubz = 0;
  {
    real A[3][3][3];
    fclb_post(s, A);
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        ubx += uncentral3_du(A[0][p][q], A[1][p][q], A[2][p][q], B[0][p][q], B[1][p][q],
                             B[2][p][q]);
        uby += uncentral3_du(A[p][0][q], A[p][1][q], A[p][2][q], B[p][0][q], B[p][1][q],
                             B[p][2][q]);
        ubz += uncentral3_du(A[p][q][0], A[p][q][1], A[p][q][2], B[p][q][0], B[p][q][1],
                             B[p][q][2]);
      }
  }
  // G_bar: transpose of the inverse transform (the axis maps commute)
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c) uncentral3_t(B[0][b][c], B[1][b][c], B[2][b][c], ux);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) uncentral3_t(B[a][0][c], B[a][1][c], B[a][2][c], uy);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) uncentral3_t(B[a][b][0], B[a][b][1], B[a][b][2], uz);

  const real third = real(1.0 / 3.0), ninth = real(1.0 / 9.0);
  const real two3 = real(2.0 / 3.0), two9 = real(2.0 / 9.0);
  const real ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
  const real c2x = third + ux2, c2y = third + uy2, c2z = third + uz2;
  const real B222 = B[2][2][2];
  // adjoints of the post-collision formulas' inputs
  const real drb = B[0][0][0] + third * (B[2][0][0] + B[0][2][0] + B[0][0][2]) +
                   ninth * (B[2][2][0] + B[2][0][2] + B[0][2][2]) + real(1.0 / 27.0) * B222;
  const real t222 = ninth * B222;
  const real ii = inv * inv;
  const real axb = B[2][0][0] + third * (B[2][2][0] + B[2][0][2]) +
                   inv * (ay * B[2][2][0] + az * B[2][0][2] + byz * B[2][1][1]) + t222 +
                   (third * inv * (ay + az) + ay * az * ii) * B222;
  const real ayb = B[0][2][0] + third * (B[2][2][0] + B[0][2][2]) +
                   inv * (ax * B[2][2][0] + az * B[0][2][2] + bxz * B[1][2][1]) + t222 +
                   (third * inv * (ax + az) + ax * az * ii) * B222;
  const real azb = B[0][0][2] + third * (B[2][0][2] + B[0][2][2]) +
                   inv * (ax * B[2][0][2] + ay * B[0][2][2] + bxy * B[1][1][2]) + t222 +
                   (third * inv * (ax + ay) + ax * ay * ii) * B222;
  const real bxyb = B[1][1][0] + (third + az * inv) * B[1][1][2];
  const real bxzb = B[1][0][1] + (third + ay * inv) * B[1][2][1];
  const real byzb = B[0][1][1] + (third + ax * inv) * B[2][1][1];
  const real invb = ax * ay * B[2][2][0] + ax * az * B[2][0][2] + ay * az * B[0][2][2] +
                    ax * byz * B[2][1][1] + ay * bxz * B[1][2][1] + az * bxy * B[1][1][2] +
                    (third * (ax * ay + ax * az + ay * az) + real(2) * ax * ay * az * inv) * B222;
  // direct dependence of the formulas on u
  ubx += B[1][0][0] - real(2) * ux * B[2][0][0] - uy * B[1][1][0] - uz * B[1][0][1] +
         real(2) * ux * (uy * B[2][1][0] + uz * B[2][0][1]) + c2y * B[1][2][0] +
         c2z * B[1][0][2] + uy * uz * B[1][1][1] - (two3 + real(2) * uy2) * ux * B[2][2][0] -
         (two3 + real(2) * uz2) * ux * B[2][0][2] - real(2) * ux * uy * uz * B[2][1][1] -
         (third + uy2) * uz * B[1][2][1] - (third + uz2) * uy * B[1][1][2] +
         real(2) * ux * (c2y * uz * B[2][2][1] + uy * c2z * B[2][1][2]) + c2y * c2z * B[1][2][2] -
         (two9 + two3 * (uy2 + uz2) + real(2) * uy2 * uz2) * ux * B222;
  uby += B[0][1][0] - real(2) * uy * B[0][2][0] - ux * B[1][1][0] - uz * B[0][1][1] +
         c2x * B[2][1][0] + real(2) * uy * (ux * B[1][2][0] + uz * B[0][2][1]) +
         c2z * B[0][1][2] + ux * uz * B[1][1][1] - (two3 + real(2) * ux2) * uy * B[2][2][0] -
         (two3 + real(2) * uz2) * uy * B[0][2][2] - (third + ux2) * uz * B[2][1][1] -
         real(2) * ux * uy * uz * B[1][2][1] - (third + uz2) * ux * B[1][1][2] +
         real(2) * uy * (c2x * uz * B[2][2][1] + ux * c2z * B[1][2][2]) + c2x * c2z * B[2][1][2] -
         (two9 + two3 * (ux2 + uz2) + real(2) * ux2 * uz2) * uy * B222;
  ubz += B[0][0][1] - real(2) * uz * B[0][0][2] - ux * B[1][0][1] - uy * B[0][1][1] +
         c2x * B[2][0][1] + c2y * B[0][2][1] + real(2) * uz * (ux * B[1][0][2] + uy * B[0][1][2]) +
         ux * uy * B[1][1][1] - (two3 + real(2) * ux2) * uz * B[2][0][2] -
         (two3 + real(2) * uy2) * uz * B[0][2][2] - (third + ux2) * uy * B[2][1][1] -
         (third + uy2) * ux * B[1][2][1] - real(2) * ux * uy * uz * B[1][1][2] +
         c2x * c2y * B[2][2][1] + real(2) * uz * (c2x * uy * B[2][1][2] + ux * c2y * B[1][2][2]) -
         (two9 + two3 * (ux2 + uy2) + real(2) * ux2 * uy2) * uz * B222;
  // shear relaxation: a_x = (1-omega)((u_x^2 + D200) - (|u|^2 + tr D)/3), ...
  const real omc = real(1) - omega;
  const real asum = axb + ayb + azb;
  const real D200b = omc * (axb - third * asum);
  const real D020b = omc * (ayb - third * asum);
  const real D002b = omc * (azb - third * asum);
  const real D110b = omc * bxyb, D101b = omc * bxzb, D011b = omc * byzb;
  ubx += omc * (real(2) * ux * axb - two3 * ux * asum + uy * bxyb + uz * bxzb);
  uby += omc * (real(2) * uy * ayb - two3 * uy * asum + ux * bxyb + uz * byzb);
  ubz += omc * (real(2) * uz * azb - two3 * uz * asum + ux * bxzb + uy * byzb);
  // second-order central moments of the deviations about u
  ubx -= real(2) * ux * D200b + uy * D110b + uz * D101b;
  uby -= real(2) * uy * D020b + ux * D110b + uz * D011b;
  ubz -= real(2) * uz * D002b + ux * D101b + uy * D011b;
  // u = j / rho, inv = 1 / rho, rho = 1 + sum f
  const real d0 = drb - ii * invb;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const real dx = real(cx(i)) - ux, dy = real(cy(i)) - uy, dz = real(cz(i)) - uz;
    g[i] = d0 + inv * (ubx * dx + uby * dy + ubz * dz) + D200b * dx * dx + D020b * dy * dy +
           D002b * dz * dz + D110b * dx * dy + D101b * dx * dz + D011b * dy * dz;
  }
}

// g <- J_C(f)^T g for the MRT-LES collision of one node (deviation form),
// the reverse of mrt_collide: with d = f - f_eq(f), acc_k = (M d)_k and
// f* = f - M^-1 S(tau(d)) M d,
//   acc_bar_k = -s_k (M^-T g)_k,  s_bar = -sum over shear rows of (M^-T g)_k acc_k,
//   d_bar = M^T acc_bar + dPi/dd^T Pi_bar,  Pi_bar from s = 1/tau, Eq. (21) for
//   tau(Q) and Q = sqrt(2 Pi:Pi) (no strain term where Q = 0),
//   g <- g + d_bar - J_eq^T d_bar,  J_eq the Jacobian of the incompressible
//   equilibrium in (drho, j).
template <typename real, int BASIS>
__device__ __forceinline__ void mrt_vjp(const real (&f)[19], real (&g)[19], const MrtParams& p) {
  using T = MrtTables<BASIS>;
  // forward recomputation: j, d, Pi, Q and tau as in mrt_collide
  real drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    drho += f[i];
    if (cx(i)) jx += cx(i) > 0 ? f[i] : -f[i];
    if (cy(i)) jy += cy(i) > 0 ? f[i] : -f[i];
    if (cz(i)) jz += cz(i) > 0 ? f[i] : -f[i];
  }
  const real uu = jx * jx + jy * jy + jz * jz;
  real d[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const real eu = real(cx(i)) * jx + real(cy(i)) * jy + real(cz(i)) * jz;
    const real feq = real(weight<19>(i)) *
                     (drho + real(3) * eu + real(4.5) * eu * eu - real(1.5) * uu);
    d[i] = f[i] - feq;
  }
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
  const real root = sqrt(tau0 * tau0 + real(p.cs18) * Qs);
  const real tau = real(0.5) * (tau0 + root);
  const real s_shear = real(1) / tau;
  real rate[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) rate[k] = real(p.rates[k]);
  // reverse of the relaxation: h = M^-T g over the relaxed rows
  real db[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) db[i] = 0;
  real sb = 0;
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    const int grp = row_group(BASIS, k);
    if (grp == 0) continue;
    real h = 0;
#pragma unroll
    for (int i = 0; i < 19; ++i)
      if (is_nonzero(T::Minv.a[i][k])) h += real(T::Minv.a[i][k]) * g[i];
    if (grp == 1) {
      real acc = 0;
#pragma unroll
      for (int i = 0; i < 19; ++i)
        if (is_nonzero(T::M.a[k][i])) acc += real(T::M.a[k][i]) * d[i];
      sb -= h * acc;
    }
    const real ab = -h * (grp == 1 ? s_shear : rate[grp - 2]);
#pragma unroll
    for (int i = 0; i < 19; ++i)
      if (is_nonzero(T::M.a[k][i])) db[i] += real(T::M.a[k][i]) * ab;
  }
  // s = 1/tau, tau = (tau0 + sqrt(tau0^2 + cs18 Q)) / 2, Q = sqrt(2 pi2)
  if (Qs > real(0)) {
    const real taub = -sb * s_shear * s_shear;
    const real qb = taub * real(p.cs18) / (real(4) * root);
    const real pb = qb / Qs;  // d pi2 -> d Q: 1 / Q
    const real bxx = real(2) * pxx * pb, byy = real(2) * pyy * pb, bzz = real(2) * pzz * pb;
    const real bxy = real(4) * pxy * pb, bxz = real(4) * pxz * pb, byz = real(4) * pyz * pb;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      real v = 0;
      if (cx(i)) v += bxx;
      if (cy(i)) v += byy;
      if (cz(i)) v += bzz;
      if (cx(i) * cy(i)) v += cx(i) * cy(i) > 0 ? bxy : -bxy;
      if (cx(i) * cz(i)) v += cx(i) * cz(i) > 0 ? bxz : -bxz;
      if (cy(i) * cz(i)) v += cy(i) * cz(i) > 0 ? byz : -byz;
      db[i] += v;
    }
  }
  // d = f - f_eq(drho, j): the equilibrium's inputs receive -d_bar
  real rb = 0, jbx = 0, jby = 0, jbz = 0;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const real eu = real(cx(i)) * jx + real(cy(i)) * jy + real(cz(i)) * jz;
    const real wq = real(weight<19>(i)) * db[i];
    rb += wq;
    const real c = wq * (real(3) + real(9) * eu);
    if (cx(i)) jbx += cx(i) > 0 ? c : -c;
    if (cy(i)) jby += cy(i) > 0 ? c : -c;
    if (cz(i)) jbz += cz(i) > 0 ? c : -c;
  }
  jbx -= real(3) * jx * rb;
  jby -= real(3) * jy * rb;
  jbz -= real(3) * jz * rb;
#pragma unroll
  for (int i = 0; i < 19; ++i)
    g[i] += db[i] - rb - (real(cx(i)) * jbx + real(cy(i)) * jby + real(cz(i)) * jbz);
}

// One adjoint step over the rows selected by r. f: natural pre-collision
// state at t; ln: adjoint at t+1; l: adjoint at t (all [27][N]); grad:
// [3][nb][na] inlet-velocity gradient, accumulated by the inlet-plane nodes
// (each owns its own entry: at most one inlet face).
template <int KIND, typename real, int BCM, int ROWS>
__global__ __launch_bounds__(256) void adjoint_kernel(const LatArgs a, const Rows r,
                                                      const real* __restrict__ f,
                                                      const real* __restrict__ ln,
                                                      real* __restrict__ l,
                                                      double* __restrict__ grad) {
  static_assert(KIND >= 0 && KIND <= 2, "the adjoint covers MRT-LES and FCLB");
  constexpr int Q = Model<KIND>::Q;
  int x, y, z;
  if (!row_coords<ROWS>(a, r, x, y, z)) return;
  const Node n = make_node(a, x, y, z);
  const size_t N = (size_t)a.N;
  // 32-bit byte offsets from per-population bases (see ldo); the wall rows
  // select between a population and its opposite from the lower slab
  const uint32_t sz = sizeof(real);
  const uint32_t self_off = (uint32_t)n.self * sz;
  real fv[Q], m[Q];
  static_for<0, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    fv[I] = ldo<real, true>(f + (size_t)I * N, self_off);
  });
  double gin[3] = {0, 0, 0};
  if constexpr (BCM == BC_NONE) {
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      m[I] = ldo<real, cx(I) == 0>(ln + (size_t)I * N,
                                   (uint32_t)n.at(cx(I), cy(I), cz(I)) * sz);
    });
  } else if constexpr (BCM == BC_WALLS) {
    // wall rows: a population pushed through an x or y wall returns as
    // opp(I) at the node itself (the wall term is a constant)
    const uint32_t slab = (uint32_t)N * sz;
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      constexpr int IO = opposite<Q>(I);
      constexpr uint32_t WB = push_faces(I) & 15u;
      const uint32_t nb = (uint32_t)n.at(cx(I), cy(I), cz(I)) * sz;
      if constexpr (WB == 0) {
        m[I] = ldo<real, true>(ln + (size_t)I * N, nb);
      } else {
        constexpr int LO = I < IO ? I : IO;
        const bool bb = (n.atface & WB) != 0;
        const uint32_t off = bb ? (IO - LO) * slab + self_off : (I - LO) * slab + nb;
        m[I] = ldo<real, cx(I) == 0>(ln + (size_t)LO * N, off);
      }
    });
  } else {
    const uint32_t bbf = a.bc.wall | a.bc.inlet;
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      constexpr int IO = opposite<Q>(I);
      const uint32_t cross = n.atface & push_faces(I);
      const bool bb = (cross & bbf) != 0;
      const real v = ln[bb ? (size_t)IO * N + n.self
                           : (size_t)I * N + n.at(cx(I), cy(I), cz(I))];
      m[I] = (cross != 0 && !bb) ? real(0) : v;
    });
    if (n.atface & a.bc.inlet) {
      static_for<0, Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        const uint32_t cross = n.atface & push_faces(I);
        if ((cross & a.bc.inlet) && !(cross & a.bc.wall)) {
          const double t = -6.0 * weight<Q>(I) * (double)m[I];
          gin[0] += cx(I) * t;
          gin[1] += cy(I) * t;
          gin[2] += cz(I) * t;
        }
      });
    }
    if (n.atface & a.bc.outflow) {
      static_for<0, Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        if ((n.atface & a.bc.outflow & pull_faces(I)) && (n.atface & push_faces(I)) == 0)
          m[I] += ln[(size_t)I * N + n.at(cx(I), cy(I), 0)];
      });
    }
  }
  if constexpr (KIND == 2)
    fclb_vjp<real>(fv, m, real(a.omega));
  else
    mrt_vjp<real, KIND>(fv, m, a.mrt);
  static_for<0, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    sto<BCM != BC_GENERAL>(l + (size_t)I * N, self_off, m[I]);
  });
  if constexpr (BCM == BC_GENERAL) {
    if (grad && (n.atface & a.bc.inlet)) {
      const int coord[3] = {n.x, n.y, n.z};
      const int A = coord[a.bc.inlet_axis == 0 ? 1 : 0];
      const int Bc = coord[a.bc.inlet_axis == 2 ? 1 : 2];
      const size_t nf = (size_t)a.bc.inlet_na * a.bc.inlet_nb;
      const size_t idx = (size_t)Bc * a.bc.inlet_na + A;
      for (int c = 0; c < 3; ++c) grad[c * nf + idx] += gin[c];
    }
  }
}

// Probe objective: J = sum over the box [lo, hi) of |j|^2 / (2 rho), times
// scale (1 / nodes of the box for the mean), of the natural pre-collision
// state; rho = 1 + sum f for FCLB, 1 for the incompressible MRT model.
// Writes dJ/df into lam (zero outside the box) if lam is not null, and one
// row of 5 partial sums per block (J in column 0) for reduce_final_kernel.
template <int KIND, typename S, bool BC, typename O>
__global__ __launch_bounds__(256) void probe_kernel(const LatArgs a, int parity, long long t,
                                                    int3 lo, int3 hi, double scale, O* lam,
                                                    double* partial) {
  constexpr int Q = Model<KIND>::Q;
  __shared__ double sh[256];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int nthreads = blockDim.x * blockDim.y;
  double v = 0.0;
  int x, y, z;
  if (node_coords(a, x, y, z)) {
    const Node n = make_node(a, x, y, z);
    const size_t N = (size_t)a.N;
    const bool in = x >= lo.x && x < hi.x && y >= lo.y && y < hi.y && z >= lo.z && z < hi.z;
    double f[Q];
    double d = 0, j[3] = {0, 0, 0};
    if (in) {
      fetch_natural<Q, S, BC>(a, n, parity, t, f);
      for (int i = 0; i < Q; ++i) {
        d += f[i];
        j[0] += cx(i) * f[i];
        j[1] += cy(i) * f[i];
        j[2] += cz(i) * f[i];
      }
    }
    const double rinv = (KIND == 2) ? 1.0 / (1.0 + d) : 1.0;
    const double jj = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
    if (in) v = 0.5 * jj * rinv * scale;
    if (lam) {
      const double c0 = (KIND == 2) ? -0.5 * jj * rinv * rinv : 0.0;
      for (int i = 0; i < Q; ++i) {
        const double ej = cx(i) * j[0] + cy(i) * j[1] + cz(i) * j[2];
        lam[(size_t)i * N + n.self] = in ? O((ej * rinv + c0) * scale) : O(0);
      }
    }
  }
  sh[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s && tid + s < nthreads) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    const size_t b = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    partial[b * 5] = sh[0];
    for (int k = 1; k < 5; ++k) partial[b * 5 + k] = 0.0;
  }
}

}  // namespace lbm
