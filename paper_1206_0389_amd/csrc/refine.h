// gfx950 kernels of the nested time refinement on a hierarchical block grid
// (block grid with nested time steps, Section 1, and the refinement levels
// of the numerical set-up, Section 3; interface interpolation and rescaling
// after Yu et al., cited there without formulas).
//
// Geometry: level l has spacing and time step 2^-l of level 0 and cell-
// centred 2:1 nesting, level-(l+1) node j sitting at level-l coordinate
// j/2 - 1/4 (a parent node's cell holds the children 2i, 2i+1 per axis), so
// halfway walls and faces coincide on every level. Each level is stored
// densely over a box (its refined region plus a ghost layer); the box's x
// origin is a multiple of 64 nodes and its row pitch M[0] a multiple of 64,
// so 64-node row segments are aligned. A type byte per box node says what a
// kernel does with it:
//   0 unused, 1 fluid, 2 band (inside the next level's region, read by that
//   level's ghost interpolation, so updated on this level), 3 covered
//   (inside the next level's region, receives the mean of its children),
//   4 ghost (filled from the parent level), 5 solid (never updated).
//
// Every level holds post-collision populations in two arrays and advances
// by pull and collide (f_i(x, t+1) = f*_i(x - e_i, t), then the collision).
// A level step runs over lists of tiles (row segments of up to 256 nodes) that contain
// fluid or band nodes: tiles whose nodes read only in-box neighbours without
// wrapping take the plain kernel, tiles with x or y WALL faces besides that
// the wall kernel (the wall-row rule of the uniform lattice), the others the
// general one (periodic wrap, every face rule).
//
// Interface per parent step t (dt_parent = 2 dt_child):
//   G(t+1) = parent state at t+1 interpolated at the child's ghosts (tensor
//            4-point cubic Lagrange at the child positions, windows kept
//            inside non-periodic domains);
//   child substep 1 reads ghosts rescale(G(t)), substep 2 reads
//   rescale(-1/8 G(t-1) + 3/4 G(t) + 3/8 G(t+1)) (linear, 1/2 G(t) + 1/2
//   G(t+1), on the first step after a state change);
//   rescale: the non-equilibrium part scaled per Chapman-Enskog (FCLB one
//   ratio r = (tau_f - 1)/(2 (tau_c - 1)); MRT per moment group, the shear
//   group with the total relaxation times of Eq. (20));
//   the covered parent nodes that parent-updated nodes pull from take the
//   rescaled mean of their eight children once the two child substeps are
//   done (no other covered node is read by anything).
// Solid nodes: before each step a pre-pass writes into each solid node's
// slot i the value its fluid neighbour x = s + e_i pulls from it (halfway
// bounce-back, or Bouzidi's interpolation along a curved link), so the step
// itself reads solid sources like any other neighbour.
#pragma once

#include "kernels.h"

namespace lbm {

enum : uint8_t { RT_UNUSED = 0, RT_FLUID = 1, RT_BAND = 2, RT_COVERED = 3, RT_GHOST = 4,
                 RT_SOLID = 5 };

struct Lev {
  void* a;              // [Q][Nbox] state read by the next step
  void* b;              // [Q][Nbox] state written by it
  const uint8_t* type;  // [Nbox]
  int o[3];             // box origin (level coordinates); o[0] % 64 == 0
  int M[3];             // box extent; M[0] (the row pitch) % 64 == 0
  int n[3];             // domain extent of the level
  uint32_t span;        // bit d: the box spans periodic axis d (wraps at n[d])
  int tw_shift;         // log2 of the tile width (64, 128 or 256 nodes)
  long long Nbox;
  MrtParams mrt;
  double omega;
  BcArgs bc;
};

// Injection into a parent level: the covered parent nodes that parent-
// updated nodes pull from receive the rescaled mean of their eight children
// once the two child substeps are done (no other covered node is read).
struct InjArgs {
  void* dst;            // parent array being written this parent step
  const int* nodes;     // parent box indices of the nodes to inject
  long long n;
  int po[3], pM[3];     // parent box
  long long pN;
  const void* src;      // child state after its two substeps
  int co[3], cM[3];     // child box
  long long cN;
};

// One interface ratio set (parent c -> child f).
struct RescaleArgs {
  double tau0_c, tau0_f, cs;  // molecular relaxation times, Smagorinsky C_S
  double r;                   // FCLB ratio (tau0_f - 1)/(2 (tau0_c - 1))
  double rates[5];            // MRT non-shear rates (both levels)
};

// ---------------------------------------------------------------- rescale
// Total relaxation time of an MRT-LES post-collision state from the
// traceless part T of its non-equilibrium stress: Qp = sqrt(2 T:T) = Q |1 -
// 1/tau| with Q the pre-collision strain measure of Eq. (21); with Eq. (20)
// the root tending to tau0 as Qp -> 0 is tau = (1 + tau0 -+ sqrt((1 -
// tau0)^2 -+ 18 C_S^2 Qp)) / 2 (upper signs for tau0 < 1, radicand clamped
// at 0).
template <typename R>
__device__ __forceinline__ R tau_from_post(const R (&d)[19], R tau0, R cs) {
  R pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    if (cx(i)) pxx += d[i];
    if (cy(i)) pyy += d[i];
    if (cz(i)) pzz += d[i];
    if (cx(i) * cy(i)) pxy += cx(i) * cy(i) > 0 ? d[i] : -d[i];
    if (cx(i) * cz(i)) pxz += cx(i) * cz(i) > 0 ? d[i] : -d[i];
    if (cy(i) * cz(i)) pyz += cy(i) * cz(i) > 0 ? d[i] : -d[i];
  }
  const R tr = (pxx + pyy + pzz) / R(3);
  const R a = pxx - tr, b = pyy - tr, c = pzz - tr;
  const R t2 = a * a + b * b + c * c + R(2) * (pxy * pxy + pxz * pxz + pyz * pyz);
  const R k = R(18) * cs * cs * sqrt(R(2) * t2);
  if (tau0 < R(1)) {
    R rad = (R(1) - tau0) * (R(1) - tau0) - k;
    rad = rad < R(0) ? R(0) : rad;
    return R(0.5) * (R(1) + tau0 - sqrt(rad));
  }
  return R(0.5) * (R(1) + tau0 + sqrt((tau0 - R(1)) * (tau0 - R(1)) + k));
}

// f := f_eq + rescaled (f - f_eq) in place, for one node. DIR > 0: a parent
// state to the child level; DIR < 0: back.
template <int KIND, int DIR, typename R>
__device__ __forceinline__ void rescale_node(R (&f)[Model<KIND>::Q], double tau0_c,
                                             double tau0_f, double cs, double r,
                                             const double (&rates)[5]) {
  constexpr int Q = Model<KIND>::Q;
  R d = 0, j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    d += f[i];
    j[0] += R(cx(i)) * f[i];
    j[1] += R(cy(i)) * f[i];
    j[2] += R(cz(i)) * f[i];
  }
  R neq[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R feq = equilibrium_one<KIND, R>(d, j, cx(i), cy(i), cz(i));
    neq[i] = f[i] - feq;
    f[i] = feq;
  }
  if constexpr (Q == 27) {
    const R s = DIR > 0 ? R(r) : R(1.0 / r);
#pragma unroll
    for (int i = 0; i < 27; ++i) f[i] += s * neq[i];
  } else {
    constexpr int BASIS = KIND;
    using T = MrtTables<BASIS>;
    R tc, tf;
    if constexpr (DIR > 0) {
      tc = tau_from_post<R>(neq, R(tau0_c), R(cs));
      tf = R(tau0_f) + R(0.5) * (tc - R(tau0_c));
    } else {
      tf = tau_from_post<R>(neq, R(tau0_f), R(cs));
      tc = R(tau0_c) + R(2) * (tf - R(tau0_f));
    }
    const R rs = DIR > 0 ? (tf - R(1)) / (R(2) * (tc - R(1))) : (R(2) * (tc - R(1))) / (tf - R(1));
    R m[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) {
      m[k] = 0;
      const int g = row_group(BASIS, k);
      if (g == 0) continue;
      R acc = 0;
#pragma unroll
      for (int i = 0; i < 19; ++i)
        if (is_nonzero(T::M.a[k][i])) acc += R(T::M.a[k][i]) * neq[i];
      // shear: the ratio of the total times; other groups keep their rate on
      // both levels: 1/2 (2 back), none left where the rate is 1
      const R sk = g == 1 ? rs
                          : (rates[g - 2] == 1.0 ? R(0) : (DIR > 0 ? R(0.5) : R(2)));
      m[k] = sk * acc;
    }
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      R c = 0;
#pragma unroll
      for (int k = 0; k < 19; ++k)
        if (row_group(BASIS, k) != 0 && is_nonzero(T::Minv.a[i][k]))
          c += R(T::Minv.a[i][k]) * m[k];
      f[i] += c;
    }
  }
}

// ------------------------------------------------------------- addressing
struct BoxNode {
  int g[3];                 // level coordinates
  int self;                 // box index
  int xo[3], yo[3], zo[3];  // box offsets of coordinates c-1, c, c+1 (wrapped)
  uint32_t atface;          // non-periodic domain faces the node lies on
  __device__ __forceinline__ int at(int dx, int dy, int dz) const {
    return zo[dz + 1] + yo[dy + 1] + xo[dx + 1];
  }
};

// Box coordinate of level coordinate g + d on axis ax: wrapped at the
// domain extent on a spanned periodic axis; otherwise (valid geometries
// never leave the box there) kept inside the box.
__device__ __forceinline__ int box_coord(const Lev& L, int ax, int g, int d) {
  int v = g + d;
  if ((L.span >> ax) & 1u) v = v < 0 ? v + L.n[ax] : (v >= L.n[ax] ? v - L.n[ax] : v);
  v -= L.o[ax];
  return v < 0 ? 0 : (v >= L.M[ax] ? L.M[ax] - 1 : v);
}

__device__ __forceinline__ BoxNode make_box_node(const Lev& L, const int (&g)[3]) {
  BoxNode n;
  const int stride[3] = {1, L.M[0], L.M[0] * L.M[1]};
  int* off[3] = {n.xo, n.yo, n.zo};
  uint32_t m = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
#pragma unroll
    for (int k = -1; k <= 1; ++k) off[d][k + 1] = box_coord(L, d, g[d], k) * stride[d];
    n.g[d] = g[d];
    if (g[d] == 0) m |= 1u << (2 * d);
    if (g[d] == L.n[d] - 1) m |= 1u << (2 * d + 1);
  }
  n.atface = m & L.bc.nonper;
  n.self = n.zo[1] + n.yo[1] + n.xo[1];
  return n;
}

// General pull source of population I: the source node's slot I; across a
// WALL/INLET face the node's own slot opp(I) (plus the bounce-back term);
// across a PRESSURE face the same slot (completed by gen_pressure); across
// FREESLIP faces slot k (I mirrored) of the source with the crossed
// coordinates kept; across an OUTFLOW face slot I of that source.
template <int Q, int I, typename S>
__device__ __forceinline__ const S* gen_pull_addr(const Lev& L, const S* A, const BoxNode& n) {
  constexpr int IO = opposite<Q>(I);
  const size_t N = (size_t)L.Nbox;
  const uint32_t crossed = n.atface & pull_faces(I);
  const S* normal = A + (size_t)I * N + n.at(-cx(I), -cy(I), -cz(I));
  const S* own = A + (size_t)IO * N + n.self;
  const int kx = (crossed & 3u) ? 0 : -cx(I);
  const int ky = (crossed & 12u) ? 0 : -cy(I);
  const int kz = (crossed & 48u) ? 0 : -cz(I);
  const S* outflow = A + (size_t)I * N + n.at(kx, ky, kz);
  const bool bb = (crossed & (L.bc.wall | L.bc.inlet | L.bc.pressure)) != 0;
  const uint32_t fs = crossed & L.bc.freeslip;
  const S* slip = A + (size_t)mirror_slot<Q, I, false>(slip_axes(fs)) * N + n.at(kx, ky, kz);
  return bb ? own : (fs ? slip : (crossed ? outflow : normal));
}

// Completes the pull at a node on PRESSURE faces: f_I = -f*_opp(I) +
// feq_I + feq_opp(I) at the face density and the node's velocity of its
// post-collision state (slot K holds f*_K), for the directions entering
// through a PRESSURE and no WALL or INLET face.
template <int KIND, typename real, typename S>
__device__ __forceinline__ void gen_pressure(const Lev& L, const S* A, const BoxNode& n,
                                             real (&f)[Model<KIND>::Q]) {
  constexpr int Q = Model<KIND>::Q;
  const size_t N = (size_t)L.Nbox;
  real d = 0, j[3] = {0, 0, 0};
  static_for<0, Q>([&](auto kc) {
    constexpr int K = decltype(kc)::value;
    const real v = ld<real>(A + (size_t)K * N + n.self);
    d += v;
    j[0] += real(cx(K)) * v;
    j[1] += real(cy(K)) * v;
    j[2] += real(cz(K)) * v;
  });
  const real rho = Q == 27 ? real(1) + d : real(1);
  const real u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
  static_for<0, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    const uint32_t crossed = n.atface & pull_faces(I);
    if ((crossed & L.bc.pressure) && !(crossed & (L.bc.wall | L.bc.inlet)))
      f[I] = -f[I] + pressure_pair<Q == 27 ? 2 : 0, I, real>(
                         real(pressure_drho(L.bc, crossed & L.bc.pressure)), u);
  });
}

// Lane -> node of a tile of TW x (256 / TW) nodes (TW = 2^tw_shift, 64 to
// 256; x fastest): whole row segments per workgroup, so each population is
// read and written in runs of TW nodes (the widest runs move the most bytes
// per second).
__device__ __forceinline__ void tile_node(const Lev& L, const int* tiles, int (&g)[3]) {
  const int* t = tiles + 3 * (size_t)blockIdx.x;
  const int lane = threadIdx.x;
  g[0] = t[0] + (lane & ((1 << L.tw_shift) - 1));
  g[1] = t[1] + (lane >> L.tw_shift);
  g[2] = t[2];
}

__device__ __forceinline__ bool in_box(const Lev& L, const int (&g)[3], int& self) {
  const int b0 = g[0] - L.o[0], b1 = g[1] - L.o[1], b2 = g[2] - L.o[2];
  if (b0 < 0 || b1 < 0 || b2 < 0 || b0 >= L.M[0] || b1 >= L.M[1] || b2 >= L.M[2]) return false;
  self = (b2 * L.M[1] + b1) * L.M[0] + b0;
  return true;
}

// Pull of population I at a node whose sources lie in the box without
// wrapping except across x or y WALL faces (wall tiles): across such a face
// the node's own slot opp(I) plus the wall term 6 w_I e_I.u_w (the x face
// first where a node lies on both); both candidate slots are offsets from
// the lower of the two population slabs, so one scalar-base load serves.
template <int Q, int I, typename real, typename S>
__device__ __forceinline__ real walls_pull(const Lev& L, const S* A, int self, int src,
                                           uint32_t atface) {
  constexpr int IO = opposite<Q>(I);
  constexpr uint32_t XB = pull_faces(I) & 3u, YB = pull_faces(I) & 12u;
  const uint32_t sz = sizeof(S);
  if constexpr ((XB | YB) == 0) {
    return ldo<real, cx(I) == 0>(A + (size_t)I * L.Nbox, (uint32_t)src * sz);
  } else {
    constexpr int LO = I < IO ? I : IO;
    const uint32_t slab = (uint32_t)L.Nbox * sz;
    const bool bx = (atface & XB) != 0, by = (atface & YB) != 0;
    const bool bb = bx || by;
    const uint32_t off = bb ? (uint32_t)(IO - LO) * slab + (uint32_t)self * sz
                            : (uint32_t)(I - LO) * slab + (uint32_t)src * sz;
    const real v = ldo<real, cx(I) == 0>(A + (size_t)LO * L.Nbox, off);
    const real term =
        wall_row_term<I, real, XB, YB>(L.bc, bx, cx(I) > 0 ? 0 : 1, cy(I) > 0 ? 2 : 3);
    return bb ? v + term : v;
  }
}

// ------------------------------------------------------------- level step
enum { TILE_PLAIN = 0, TILE_WALLS = 1, TILE_GENERAL = 2 };

// One pull-and-collide step of level L at its step index t over a tile
// list. KINDT: TILE_PLAIN (every source of the tile's active nodes lies in
// the box without wrapping, no node on a domain face), TILE_WALLS (as plain
// but with x or y WALL faces, the wall-row rule) or TILE_GENERAL (periodic
// wrap and every face rule).
template <int KIND, typename S, int KINDT>
__global__ __launch_bounds__(256) void level_step_kernel(const Lev L, const int* tiles,
                                                         long long t) {
  using M = Model<KIND>;
  using real = typename Compute<S>::type;
  constexpr int Q = M::Q;
  int g[3], self = 0;
  tile_node(L, tiles, g);
  bool active = in_box(L, g, self);
  if (active) {
    const uint8_t ty = L.type[self];
    active = ty == RT_FLUID || ty == RT_BAND;
  }
  if (!active) return;
  const S* A = (const S*)L.a;
  S* B = (S*)L.b;
  const size_t N = (size_t)L.Nbox;
  real f[Q];
  if (active) {
    if constexpr (KINDT == TILE_GENERAL) {
      const BoxNode n = make_box_node(L, g);
      static_for<0, Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        f[I] = ld<real>(gen_pull_addr<Q, I, S>(L, A, n));
      });
      if (n.atface) {
        double uin[3] = {0, 0, 0};
        if (n.atface & L.bc.inlet) inlet_velocity(L.bc, g[0], g[1], g[2], t, uin);
        const real up[3] = {real(uin[0]), real(uin[1]), real(uin[2])};
        static_for<0, Q>([&](auto ic) {
          constexpr int I = decltype(ic)::value;
          f[I] += pull_term<Q, I, real>(L.bc, n.atface, up);
        });
        if (n.atface & L.bc.pressure) gen_pressure<KIND, real, S>(L, A, n, f);
      }
    } else if constexpr (KINDT == TILE_WALLS) {
      const int sy = L.M[0], sz = L.M[0] * L.M[1];
      uint32_t m = 0;
      m |= g[0] == 0 ? 1u : 0u;
      m |= g[0] == L.n[0] - 1 ? 2u : 0u;
      m |= g[1] == 0 ? 4u : 0u;
      m |= g[1] == L.n[1] - 1 ? 8u : 0u;
      m &= L.bc.wall;
      static_for<0, Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        const int src = self - cx(I) - cy(I) * sy - cz(I) * sz;
        f[I] = walls_pull<Q, I, real, S>(L, A, self, src, m);
      });
    } else {
      const int sy = L.M[0], sz = L.M[0] * L.M[1];
      static_for<0, Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        const int src = self - cx(I) - cy(I) * sy - cz(I) * sz;
        f[I] = ldo<real, cx(I) == 0>(A + (size_t)I * N, (uint32_t)src * (uint32_t)sizeof(S));
      });
    }
    M::collide(f, L);
    const uint32_t so = (uint32_t)self * (uint32_t)sizeof(S);
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      sto<true>(B + (size_t)I * N, so, f[I]);
    });
  }
}

// Covered parent nodes := f_eq + rescaled-back (m - f_eq), m = the mean of
// the eight children (summed x fastest, then y, then z).
template <int KIND, typename S>
__global__ __launch_bounds__(256) void inject_kernel(const InjArgs ia, const RescaleArgs ra) {
  using R = typename Compute<S>::type;
  constexpr int Q = Model<KIND>::Q;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ia.n) return;
  const int pi = ia.nodes[e];
  const int b0 = pi % ia.pM[0], b1 = (pi / ia.pM[0]) % ia.pM[1], b2 = pi / (ia.pM[0] * ia.pM[1]);
  const int c0 = 2 * (b0 + ia.po[0]) - ia.co[0], c1 = 2 * (b1 + ia.po[1]) - ia.co[1],
            c2 = 2 * (b2 + ia.po[2]) - ia.co[2];
  const S* C = (const S*)ia.src;
  R m[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) m[q] = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const size_t k = ((size_t)(c2 + (c >> 2)) * ia.cM[1] + (c1 + ((c >> 1) & 1))) * ia.cM[0] +
                     (c0 + (c & 1));
#pragma unroll
    for (int q = 0; q < Q; ++q) m[q] += ld<R>(C + (size_t)q * (size_t)ia.cN + k);
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) m[q] *= R(0.125);
  rescale_node<KIND, -1, R>(m, ra.tau0_c, ra.tau0_f, ra.cs, ra.r, ra.rates);
  S* P = (S*)ia.dst;
#pragma unroll
  for (int q = 0; q < Q; ++q) st(P + (size_t)q * (size_t)ia.pN + pi, m[q]);
}

// --------------------------------------------------------- solid pre-pass
// Before a step: for every listed fluid node x and direction i whose source
// s = x - e_i is solid, write into slot i of s the value x pulls from it,
// from the post-collision state in A (k = opp(i), the link towards the
// wall at the fraction q of it; q = 1/2 or a link without a fluid node
// behind x is the halfway rule):
//   halfway:   f*_k(x)
//   q <  1/2:  2q f*_k(x) + (1 - 2q) f*_k(x + e_i)
//   q >= 1/2:  f*_k(x) / (2q) + (2q - 1)/(2q) f*_i(x)
// Slot i of s has this one writer, and nothing the pass reads is written.
template <int Q, typename S>
__global__ __launch_bounds__(256) void solid_prepass_kernel(const Lev L, const int* nodes,
                                                            const uint32_t* dirs, const float* q,
                                                            long long n) {
  using real = typename Compute<S>::type;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int self = nodes[e];
  const uint32_t m = dirs[e];
  const int M0 = L.M[0], M1 = L.M[1];
  const int b[3] = {self % M0, (self / M0) % M1, self / (M0 * M1)};
  const int g[3] = {b[0] + L.o[0], b[1] + L.o[1], b[2] + L.o[2]};
  const BoxNode nd = make_box_node(L, g);
  S* A = (S*)L.a;
  const size_t N = (size_t)L.Nbox;
  static_for<1, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    constexpr int K = opposite<Q>(I);
    if ((m >> I) & 1u) {
      const real fk = ld<real>(A + (size_t)K * N + self);
      const real qq = real(q[(size_t)e * Q + K]);
      real v = fk;
      if (qq < real(0.5)) {
        v = real(2) * qq * fk + (real(1) - real(2) * qq) * ld<real>(A + (size_t)K * N + nd.at(cx(I), cy(I), cz(I)));
      } else if (qq > real(0.5)) {
        v = fk / (real(2) * qq) + (real(2) * qq - real(1)) / (real(2) * qq) *
                                      ld<real>(A + (size_t)I * N + self);
      }
      st(A + (size_t)I * N + nd.at(-cx(I), -cy(I), -cz(I)), v);
    }
  });
}

// ------------------------------------------------------------- interface
struct GhostArgs {
  const int* ghosts;  // child box indices of the ghost nodes (group order)
  long long ng;
  const int* groups;  // GhostGroup records
  const int* gcode;   // per ghost: stencil start and code per axis
  long long ngroups;
  const int* unodes;  // parent box indices read by the stencils (nu)
  long long nu;
  const int* pidx;    // per group patch node: index into unodes, or -1
  // parent box
  int po[3], pM[3], pn[3];
  uint32_t pspan;
  long long pN, cN;   // parent and child box sizes
};

// Ghosts are grouped by the parent cube of kGhostCube^3 nodes holding their
// stencil starts (at most kGhostMax per group); a group's stencils read the
// parent patch [lo, lo + m) (level coordinates, wrapped on spanned periodic
// axes; m <= kGhostCube + 3 per axis), staged in LDS by one workgroup from
// a compact node-major copy of the parent nodes the stencils read (patch
// node p of a group: entry pidx[poff + p] of that copy, x fastest). A
// ghost's code holds per axis d, in bits 6d..6d+5, the stencil start
// relative to lo (3 bits) and the stencil code c (3 bits): the child lies at
// t = (2c - 1)/4 of the window s..s+3.
constexpr int kGhostCube = 4;
constexpr int kGhostMax = 64;
constexpr int kPatchEdge = kGhostCube + 3;
constexpr int kPatchMax = kPatchEdge * kPatchEdge * kPatchEdge;
struct GhostGroup {
  int gbeg, gend;
  int lo[3], m[3];
  int poff;
};

// Cubic Lagrange weights (dyadic, exact) at t = (2c - 1)/4, c = 0..7, on
// the nodes 0..3 of a window.
template <typename T>
__host__ __device__ inline void stencil_weights(int c, T w[4]) {
  // exact in FP32 too: dyadic values with a few bits, the division by 6 of
  // a multiple of 3 correctly rounded
  const T t = (T(2) * T(c) - T(1)) * T(0.25);
  w[0] = -(t - T(1)) * (t - T(2)) * (t - T(3)) / T(6);
  w[1] = t * (t - T(2)) * (t - T(3)) / T(2);
  w[2] = -t * (t - T(1)) * (t - T(3)) / T(2);
  w[3] = t * (t - T(1)) * (t - T(2)) / T(6);
}

// Window start s and code c of child coordinate j on a parent axis of n
// nodes: s = floor(j/2 - 1/4) - 1, moved inside [0, n - 4] on a
// non-periodic axis; c = j - 2 s.
__host__ __device__ inline int child_window(int j, int n, bool periodic, int& s) {
  int f = (2 * j - 1) >= 0 ? (2 * j - 1) / 4 : -((-(2 * j - 1) + 3) / 4);  // floor((2j-1)/4)
  s = f - 1;
  if (!periodic) s = s < 0 ? 0 : (s > n - 4 ? n - 4 : s);
  return j - 2 * s;
}

// Tensor interpolation from a staged patch (x fastest): 4 x 4 x 4 nodes,
// summation z, then y, then x.
template <typename S, typename R>
__device__ __forceinline__ R patch_interp(const S* sp, int code, int m0, int m01) {
  int a[3];
  R w[3][4];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int cd = (code >> (6 * d)) & 63;
    a[d] = cd & 7;
    stencil_weights(cd >> 3, w[d]);
  }
  R s = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const R wbc = w[1][b] * w[2][c];
      const S* row = sp + (a[2] + c) * m01 + (a[1] + b) * m0 + a[0];
#pragma unroll
      for (int x = 0; x < 4; ++x) s += w[0][x] * wbc * R(row[x]);
    }
  return s;
}

// The parent nodes the stencils read, node-major: Pc[u][q] = fp[q][unodes[u]]
// (rows of the parent box read once, where the group patches overlap and
// cover only part of each memory line).
template <int KIND, typename S>
__global__ __launch_bounds__(256) void ghost_gather_kernel(const GhostArgs ga, const S* fp,
                                                           S* Pc) {
  constexpr int Q = Model<KIND>::Q;
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= ga.nu) return;
  const size_t k = (size_t)ga.unodes[u];
  S v[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) v[q] = fp[(size_t)q * (size_t)ga.pN + k];
#pragma unroll
  for (int q = 0; q < Q; ++q) Pc[(size_t)u * Q + q] = v[q];
}

// Interface interpolation of one ghost group per workgroup (launched with
// 256 threads): the parent patch is staged in LDS from the gathered copy Pc,
// every (ghost, population) is interpolated from it into Gn (kept for the
// following steps), and the time combination c0 Gm + c1 Gc + c2 Gn (Gm, Gc
// not read where their weight is 0; G* are [Q][ng]) goes back to LDS with
// Gn itself; one thread per ghost rescales the combination into the child
// array ff (the next substep's ghosts) and, if fn is given, another rescales
// Gn into the child array fn (the ghosts of the first substep of the next
// parent step).
template <int KIND, typename S, typename R>
__global__ __launch_bounds__(256) void ghost_patch_kernel(const GhostArgs ga, const S* Pc, R* Gn,
                                                          const R* Gc, const R* Gm, double c0,
                                                          double c1, double c2,
                                                          const RescaleArgs ra, S* ff, S* fn) {
  static_assert(2 * kGhostMax <= 256, "one thread per ghost and value set");
  constexpr int Q = Model<KIND>::Q;
  // the patch, then (after it is read) the ghosts' combined and new values
  constexpr size_t kPatchBytes = sizeof(S) * Q * kPatchMax;
  constexpr size_t kHBytes = sizeof(R) * Q * kGhostMax;
  __shared__ __align__(16) unsigned char
      lds[kPatchBytes > 2 * kHBytes ? kPatchBytes : 2 * kHBytes];
  S(&sp)[Q][kPatchMax] = *reinterpret_cast<S(*)[Q][kPatchMax]>(lds);
  R(&hs)[Q][kGhostMax] = *reinterpret_cast<R(*)[Q][kGhostMax]>(lds);
  R(&gs)[Q][kGhostMax] = *reinterpret_cast<R(*)[Q][kGhostMax]>(lds + kHBytes);
  const GhostGroup* grp = (const GhostGroup*)ga.groups + blockIdx.x;
  const long long gbeg = grp->gbeg;
  const int ngg = grp->gend - grp->gbeg;
  const int m0 = grp->m[0], m1 = grp->m[1], m01 = m0 * m1;
  const int P = m01 * grp->m[2];
  const int* pidx = ga.pidx + grp->poff;
  // this thread's (population, ghost) items: k = threadIdx.x + 256 it, their
  // history values loaded ahead of the staging so the latencies overlap
  constexpr int kItems = (Q * kGhostMax + 255) / 256;
  R hist[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int k = threadIdx.x + 256 * it;
    const int q = k / kGhostMax, gl = k % kGhostMax;
    hist[it] = R(0);
    if (k < Q * kGhostMax && gl < ngg) {
      const size_t kk = (size_t)q * ga.ng + gbeg + gl;
      if (c1 != 0.0) hist[it] = R(c1) * Gc[kk];
      if (c0 != 0.0) hist[it] += R(c0) * Gm[kk];
    }
  }
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    const int u = pidx[p];
    const S* src = Pc + (size_t)(u < 0 ? 0 : u) * Q;
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      sp[I][p] = u < 0 ? S(0) : src[I];
    });
  }
  __syncthreads();
  R h[kItems], g[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int k = threadIdx.x + 256 * it;
    const int q = k / kGhostMax, gl = k % kGhostMax;
    h[it] = R(0);
    g[it] = R(0);
    if (k >= Q * kGhostMax || gl >= ngg) continue;
    const long long gi = gbeg + gl;
    const R v = patch_interp<S, R>(sp[q], ga.gcode[gi], m0, m01);
    Gn[(size_t)q * ga.ng + gi] = v;
    g[it] = v;
    h[it] = R(c2) * v + hist[it];
  }
  __syncthreads();  // the patch is read: its space takes the ghosts' values
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int k = threadIdx.x + 256 * it;
    if (k < Q * kGhostMax) {
      hs[k / kGhostMax][k % kGhostMax] = h[it];
      gs[k / kGhostMax][k % kGhostMax] = g[it];
    }
  }
  __syncthreads();
  // threads [0, ngg): the combined values into ff; threads [kGhostMax,
  // kGhostMax + ngg): the new values into fn (when given)
  const int tl = threadIdx.x;
  const bool second = tl >= kGhostMax;
  const int gl = second ? tl - kGhostMax : tl;
  if (gl < ngg && (!second || fn != nullptr)) {
    R f[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) f[q] = second ? gs[q][gl] : hs[q][gl];
    rescale_node<KIND, +1, R>(f, ra.tau0_c, ra.tau0_f, ra.cs, ra.r, ra.rates);
    const int l = ga.ghosts[gbeg + gl];
    S* dst = second ? fn : ff;
#pragma unroll
    for (int q = 0; q < Q; ++q) st(dst + (size_t)q * (size_t)ga.cN + l, f[q]);
  }
}

// ------------------------------------------------------------- reductions
// FP64 partial sums over the nodes of a level box of type want, each
// weighted by w (the node's volume in level-0 cells).
template <int KIND, typename S>
__global__ __launch_bounds__(256) void level_reduce_kernel(const Lev L, int want, double w,
                                                           double* partial) {
  constexpr int Q = Model<KIND>::Q;
  __shared__ double sh[5][256];
  const int tid = threadIdx.x;
  double v[5] = {0, 0, 0, 0, 0};
  const long long self = (long long)blockIdx.x * blockDim.x + tid;
  if (self < L.Nbox && L.type[self] == want) {
    const S* A = (const S*)L.a;
    double d = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
      const double fi = ld<double>(A + (size_t)i * (size_t)L.Nbox + self);
      d += fi;
      j[0] += cx(i) * fi;
      j[1] += cy(i) * fi;
      j[2] += cz(i) * fi;
    }
    const double r = (Q == 27) ? 1.0 + d : 1.0;
    v[0] = w * d;
    v[1] = w * j[0];
    v[2] = w * j[1];
    v[3] = w * j[2];
    v[4] = w * 0.5 * (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / r;
  }
  for (int k = 0; k < 5; ++k) sh[k][tid] = v[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s)
      for (int k = 0; k < 5; ++k) sh[k][tid] += sh[k][tid + s];
    __syncthreads();
  }
  if (tid == 0)
    for (int k = 0; k < 5; ++k) partial[(size_t)blockIdx.x * 5 + k] = sh[k][0];
}

}  // namespace lbm
