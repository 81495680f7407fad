// gfx950 kernels of the two-level nested time refinement (hierarchical block
// grid with nested time steps, Section 1 and the numerical set-up of
// Section 3; interface treatment after Yu et al., cited there).
//
// Geometry: 2:1 vertex-centred nesting. Fine node j (global fine index) sits
// at coarse coordinate j/2; a refined coarse block of B^3 nodes carries
// (2B)^3 fine nodes. Each level is stored densely over a box: the coarse box
// is the whole domain, the fine box the refined blocks' bounding box plus
// one ghost layer on every side that is not a domain face. A per-node type
// byte marks what a kernel updates: coarse 0 = outside the refined region,
// 1 = refined but read by a ghost stencil ("band"), 2 = covered (overwritten
// from the fine level); fine 0 = unused, 1 = fluid, 2 = ghost.
//
// Both levels hold post-collision populations and advance by a two-array
// pull-and-collide (f_i(x,t+1) = f*_i(x - e_i, t), then collide): the fine
// level reads interpolated ghosts between the two arrays, so the in-place
// AA parity bookkeeping of the uniform kernels is not used here; the bytes
// moved per node update are the same.
//
// Per coarse step t (dt_c = 2 dt_f, nu_f = 2 nu_c in lattice units):
//   G0 = coarse values interpolated at the ghosts (tensor 4-point cubic
//        Lagrange, one-sided near non-periodic faces), fill ghosts with
//        rescale(G0): f = f_eq + r (g - f_eq), r = (tau_f - 1)/(2(tau_c - 1))
//   coarse pull-collide (skips covered nodes)
//   fine pull-collide at fine time 2t
//   G1 = interpolation of the new coarse state; ghosts = rescale((G0+G1)/2)
//   fine pull-collide at fine time 2t+1
//   covered coarse nodes = f_eq + (f_fine - f_eq)/r of the coincident node.
#pragma once

#include "kernels.h"

namespace lbm {

struct Level {
  void* a;              // [Q][Nbox] state read by a step
  void* b;              // [Q][Nbox] state written by a step
  const uint8_t* type;  // [Nbox]
  int lo[3];            // box origin in this level's global coordinates
  int M[3];             // box extent
  int n[3];             // domain extent of this level
  long long Nbox;
  MrtParams mrt;
  double omega;
  BcArgs bc;
  // Injection into the covered coarse nodes, done by the last fine substep
  // of a coarse step (cinj null otherwise): the fine node coincident with a
  // covered coarse node (all global fine coordinates even, coarse type 2)
  // writes f_eq + rinv (f - f_eq) of its post-collision state into cinj.
  void* cinj;
  const uint8_t* ctype;
  int cn[3];
  long long Nc;
  double rinv;
};

// 1-D interpolation stencil for fine coordinate j on an axis of n >= 4
// coarse nodes. Code 0: one node, j/2 (j even, weight 1). Codes 1-4: the
// four nodes s..s+3, s = (j-1)/2 - 1 (moved inside [0, n) on a non-periodic
// axis), with the cubic Lagrange weights at t = j/2 - s = 1/2, 3/2, 5/2,
// 7/2 (3/2 inside, the others next to a face). start is the first node
// before wrapping on a periodic axis.
__host__ __device__ inline int stencil_code(int j, int n, bool periodic, int& start) {
  if ((j & 1) == 0) {
    start = j / 2;
    return 0;
  }
  int s = (j - 1) / 2 - 1;
  if (!periodic) s = s < 0 ? 0 : (s > n - 4 ? n - 4 : s);
  start = s;
  return (j - 2 * s + 1) / 2;  // 2t = 1, 3, 5, 7
}

// Weights of a stencil code (dyadic, exact in every precision used).
__host__ __device__ inline void stencil_weights(int code, double w[4]) {
  switch (code) {
    case 0: w[0] = 1.0; w[1] = 0.0; w[2] = 0.0; w[3] = 0.0; break;
    case 1: w[0] = 5.0 / 16; w[1] = 15.0 / 16; w[2] = -5.0 / 16; w[3] = 1.0 / 16; break;
    case 2: w[0] = -1.0 / 16; w[1] = 9.0 / 16; w[2] = 9.0 / 16; w[3] = -1.0 / 16; break;
    case 3: w[0] = 1.0 / 16; w[1] = -5.0 / 16; w[2] = 15.0 / 16; w[3] = 5.0 / 16; break;
    default: w[0] = -5.0 / 16; w[1] = 21.0 / 16; w[2] = -35.0 / 16; w[3] = 35.0 / 16; break;
  }
}

// Nodes (wrapped) and weights of the stencil; returns the node count.
__host__ __device__ inline int interp_stencil(int j, int n, bool periodic, int idx[4],
                                              double w[4]) {
  int s;
  const int code = stencil_code(j, n, periodic, s);
  stencil_weights(code, w);
  const int cnt = code == 0 ? 1 : 4;
  for (int a = 0; a < cnt; ++a) idx[a] = periodic ? (((s + a) % n) + n) % n : s + a;
  return cnt;
}

struct BoxNode {
  int g[3];                 // global coordinates
  int self;                 // box index
  int xo[3], yo[3], zo[3];  // box-local linear offsets of coordinates c-1, c, c+1
  uint32_t atface;          // non-periodic domain faces the node lies on
  __device__ __forceinline__ int at(int dx, int dy, int dz) const {
    return zo[dz + 1] + yo[dy + 1] + xo[dx + 1];
  }
};

// Neighbour coordinate in the box: wrapped on a periodic axis the box spans,
// otherwise kept inside the box (valid configurations never need the clamp:
// fluid nodes only read fluid or ghost neighbours or cross a domain face).
__device__ __forceinline__ int box_nbr(int c, int d, int M, bool wrap) {
  const int v = c + d;
  if (wrap) return v < 0 ? M - 1 : (v >= M ? 0 : v);
  return v < 0 ? 0 : (v >= M ? M - 1 : v);
}

__device__ __forceinline__ BoxNode make_box_node(const Level& L, int lx, int ly, int lz) {
  BoxNode n;
  const int l3[3] = {lx, ly, lz};
  const int stride[3] = {1, L.M[0], L.M[0] * L.M[1]};
  int* off[3] = {n.xo, n.yo, n.zo};
  uint32_t m = 0;
  for (int d = 0; d < 3; ++d) {
    const bool wrap = ((L.bc.nonper >> (2 * d)) & 1u) == 0;
    for (int k = -1; k <= 1; ++k) off[d][k + 1] = box_nbr(l3[d], k, L.M[d], wrap) * stride[d];
    n.g[d] = l3[d] + L.lo[d];
    if (n.g[d] == 0) m |= 1u << (2 * d);
    if (n.g[d] == L.n[d] - 1) m |= 1u << (2 * d + 1);
  }
  n.atface = m & L.bc.nonper;
  n.self = n.zo[1] + n.yo[1] + n.xo[1];
  return n;
}

// Pull of population I in two-array post-collision storage: the source
// node's own slot I; across a WALL/INLET face the node's slot opp(I) (plus
// the bounce-back term, pull_term); across a PRESSURE face the same slot
// (completed by ab_pressure); across FREESLIP faces slot k (I mirrored
// across them) of the source with the crossed coordinates kept; across an
// OUTFLOW face slot I of that source.
template <int Q, int I, typename S>
__device__ __forceinline__ const S* ab_pull_addr(const Level& L, const S* A, const BoxNode& n) {
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
// feq_I + feq_opp(I) (anti-bounce-back at the face density) for the
// directions entering through one and through no WALL or INLET face, with
// the node's velocity of its post-collision state, slot K holding f*_K.
template <int Q, typename real, typename S>
__device__ __forceinline__ void ab_pressure(const Level& L, const S* A, const BoxNode& n,
                                            real (&f)[Q]) {
  constexpr int KQ = Q == 27 ? 2 : 0;
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
      f[I] = -f[I] + pressure_pair<KQ, I, real>(
                         real(pressure_drho(L.bc, crossed & L.bc.pressure)), u);
  });
}

// Wall-row pull (rows off every non-periodic z face and off y faces that are
// not walls; x and y faces WALL or periodic): population I entering through
// an x or y wall is the node's own opposite slot plus a per-direction wall
// term (the x face first where a node lies on both). Both sources are
// offsets from the lower of the two slabs (one scalar-base load).
template <int Q, int I, typename real, bool NT, typename S>
__device__ __forceinline__ real ab_pull_walls(const Level& L, const S* A, const BoxNode& n) {
  constexpr int IO = opposite<Q>(I);
  constexpr uint32_t XB = pull_faces(I) & 3u, YB = pull_faces(I) & 12u;
  const uint32_t sz = sizeof(S);
  const uint32_t nb = (uint32_t)n.at(-cx(I), -cy(I), -cz(I)) * sz;
  if constexpr ((XB | YB) == 0) {
    return ldo<real, NT>(A + (size_t)I * L.Nbox, nb);
  } else {
    constexpr int LO = I < IO ? I : IO;
    const uint32_t slab = (uint32_t)L.Nbox * sz;
    const bool bx = (n.atface & XB) != 0, by = (n.atface & YB) != 0;
    const bool bb = bx || by;
    const uint32_t off = bb ? (IO - LO) * slab + (uint32_t)n.self * sz : (I - LO) * slab + nb;
    const real v = ldo<real, NT>(A + (size_t)LO * L.Nbox, off);
    const real term =
        wall_row_term<I, real, XB, YB>(L.bc, bx, cx(I) > 0 ? 0 : 1, cy(I) > 0 ? 2 : 3);
    return bb ? v + term : v;
  }
}

// Equilibrium of the model (deviation form) for the moments of f.
template <int KIND, typename R>
__device__ __forceinline__ void equilibrium_dev(const R (&f)[Model<KIND>::Q],
                                                R (&feq)[Model<KIND>::Q]) {
  constexpr int Q = Model<KIND>::Q;
  R d = 0, j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    d += f[i];
    j[0] += R(cx(i)) * f[i];
    j[1] += R(cy(i)) * f[i];
    j[2] += R(cz(i)) * f[i];
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) feq[i] = equilibrium_one<KIND, R>(d, j, cx(i), cy(i), cz(i));
}

// One pull-and-collide update of a level at time t over the rows r (box-
// local coordinates). mode 0 updates every node whose type is not 2
// (coarse), mode 1 only type-1 nodes (fine). BCM: BC_NONE (no non-periodic
// face), BC_WALLS (wall rows, see ab_pull_walls) or BC_GENERAL.
template <int KIND, typename S, int BCM, int ROWS>
__global__ __launch_bounds__(256) void ab_step_kernel(const Level L, const Rows r, int mode,
                                                      long long t) {
  using M = Model<KIND>;
  using real = typename Compute<S>::type;
  constexpr int Q = M::Q;
  int lx, ly, lz;
  {
    LatArgs dims;
    dims.nx = L.M[0];
    dims.ny = L.M[1];
    dims.nz = L.M[2];
    if (!row_coords<ROWS>(dims, r, lx, ly, lz)) return;
  }
  const int self = (lz * L.M[1] + ly) * L.M[0] + lx;
  const uint8_t ty = L.type[self];
  if (mode == 0 ? ty == 2 : ty != 1) return;
  const BoxNode n = make_box_node(L, lx, ly, lz);
  const S* A = (const S*)L.a;
  S* B = (S*)L.b;
  real f[Q];
  if constexpr (BCM == BC_GENERAL) {
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      f[I] = ld<real>(ab_pull_addr<Q, I, S>(L, A, n));
    });
    if (n.atface) {
      double uin[3] = {0, 0, 0};
      if (n.atface & L.bc.inlet) inlet_velocity(L.bc, n.g[0], n.g[1], n.g[2], t, uin);
      const real up[3] = {real(uin[0]), real(uin[1]), real(uin[2])};
      static_for<0, Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        f[I] += pull_term<Q, I, real>(L.bc, n.atface, up);
      });
      if (n.atface & L.bc.pressure) ab_pressure<Q, real, S>(L, A, n, f);
    }
  } else if constexpr (BCM == BC_WALLS) {
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      f[I] = ab_pull_walls<Q, I, real, cx(I) == 0>(L, A, n);
    });
  } else {
    const size_t N = (size_t)L.Nbox;
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      f[I] = ldo<real, cx(I) == 0>(A + (size_t)I * N,
                                   (uint32_t)n.at(-cx(I), -cy(I), -cz(I)) * (uint32_t)sizeof(S));
    });
  }
  M::collide(f, L);
  const size_t N = (size_t)L.Nbox;
  if constexpr (BCM == BC_GENERAL) {
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      st(B + (size_t)I * N + self, f[I]);
    });
  } else {
    const uint32_t self_off = (uint32_t)self * (uint32_t)sizeof(S);
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      sto<true>(B + (size_t)I * N, self_off, f[I]);
    });
  }
  if (L.cinj != nullptr && ((n.g[0] | n.g[1] | n.g[2]) & 1) == 0) {
    const size_t ci = ((size_t)(n.g[2] >> 1) * L.cn[1] + (n.g[1] >> 1)) * L.cn[0] + (n.g[0] >> 1);
    if (L.ctype[ci] == 2) {
      real g[Q], feq[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) g[q] = real(S(f[q]));  // the stored value
      equilibrium_dev<KIND, real>(g, feq);
      S* C = (S*)L.cinj;
#pragma unroll
      for (int q = 0; q < Q; ++q)
        st(C + (size_t)q * (size_t)L.Nc + ci, feq[q] + real(L.rinv) * (g[q] - feq[q]));
    }
  }
}

struct GhostArgs {
  const int* ghosts;  // fine box indices of the ghost nodes
  long long ng;
  // ghost groups (see GhostGroup) and per-ghost stencil codes
  const int* groups;
  const int* gcode;
  long long ngroups;
  long long Nc, Nf;
  int cn[3];          // coarse domain extent
};

// The ghosts are grouped by the coarse cube of kGhostCube^3 cells that holds
// them (at most kGhostMax ghosts per group; ghosts [gbeg, gend) of the
// list). A group's stencils read the coarse patch [lo, lo + m) (unwrapped
// coordinates, wrapped on periodic axes; m <= kGhostCube + 3 per axis),
// which one workgroup stages in LDS. A ghost's code holds, per axis d in
// bits 6d..6d+5, its stencil's first node relative to lo (3 bits) and its
// stencil code (3 bits).
constexpr int kGhostCube = 4;
constexpr int kGhostMax = 64;
constexpr int kPatchEdge = kGhostCube + 3;
constexpr int kPatchMax = kPatchEdge * kPatchEdge * kPatchEdge;
struct GhostGroup {
  int gbeg, gend;
  int lo[3], m[3];
};

// Tensor interpolation from a staged patch (x fastest, rows of m0 nodes,
// planes of m01). The stencil shape is a compile-time count per axis so
// the LDS reads are unrolled; summation order z, then y, then x.
template <int C0, int C1, int C2, typename S, typename R>
__device__ __forceinline__ R patch_interp_fixed(const S* sp, const int (&a)[3],
                                                const double (&w)[3][4], int m0, int m01) {
  R s = 0;
#pragma unroll
  for (int c = 0; c < C2; ++c)
#pragma unroll
    for (int b = 0; b < C1; ++b) {
      const R wbc = R(w[1][b] * w[2][c]);
      const S* row = sp + (a[2] + c) * m01 + (a[1] + b) * m0 + a[0];
#pragma unroll
      for (int x = 0; x < C0; ++x) s += R(w[0][x]) * wbc * R(row[x]);
    }
  return s;
}

template <typename S, typename R>
__device__ __forceinline__ R patch_interp(const S* sp, int code, int m0, int m01) {
  int a[3], shape = 0;
  double w[3][4];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int cd = (code >> (6 * d)) & 63;
    a[d] = cd & 7;
    stencil_weights(cd >> 3, w[d]);
    shape |= (cd >> 3) != 0 ? 1 << d : 0;
  }
  switch (shape) {
    case 0: return patch_interp_fixed<1, 1, 1, S, R>(sp, a, w, m0, m01);
    case 1: return patch_interp_fixed<4, 1, 1, S, R>(sp, a, w, m0, m01);
    case 2: return patch_interp_fixed<1, 4, 1, S, R>(sp, a, w, m0, m01);
    case 3: return patch_interp_fixed<4, 4, 1, S, R>(sp, a, w, m0, m01);
    case 4: return patch_interp_fixed<1, 1, 4, S, R>(sp, a, w, m0, m01);
    case 5: return patch_interp_fixed<4, 1, 4, S, R>(sp, a, w, m0, m01);
    case 6: return patch_interp_fixed<1, 4, 4, S, R>(sp, a, w, m0, m01);
    default: return patch_interp_fixed<4, 4, 4, S, R>(sp, a, w, m0, m01);
  }
}

// Rescaled ghost populations of one group: lanes take (ghost, population)
// pairs population-major, v = c0 G0 + c1 G (G0 may be null), with the
// moments of each ghost shared through LDS; every lane evaluates the
// equilibrium of its own population and writes feq + r (v - feq) to ff
// (Yu's rescaling of the non-equilibrium part).
template <int KIND, typename S, typename R>
__device__ __forceinline__ void rescale_group(const GhostArgs& ga, long long gbeg, int ngg,
                                              R (&sv)[Model<KIND>::Q][kGhostMax],
                                              const int (&se)[Model<KIND>::Q][3], double r,
                                              S* ff) {
  constexpr int Q = Model<KIND>::Q;
  for (int k = threadIdx.x; k < Q * kGhostMax; k += blockDim.x) {
    const int q = k / kGhostMax, gl = k % kGhostMax;
    if (gl >= ngg) continue;
    R d = 0, j[3] = {0, 0, 0};
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      const R f = sv[I][gl];
      d += f;
      j[0] += R(cx(I)) * f;
      j[1] += R(cy(I)) * f;
      j[2] += R(cz(I)) * f;
    });
    const R feq = equilibrium_one<KIND, R>(d, j, se[q][0], se[q][1], se[q][2]);
    const int l = ga.ghosts[gbeg + gl];
    st(ff + (size_t)q * (size_t)ga.Nf + l, feq + R(r) * (sv[q][gl] - feq));
  }
}

template <int Q>
__device__ __forceinline__ void velocity_table(int (&se)[Q][3]) {
  const int t = threadIdx.x;
  if (t < Q) {
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      if (t == I) {
        se[I][0] = cx(I);
        se[I][1] = cy(I);
        se[I][2] = cz(I);
      }
    });
  }
}

// Interface update of one ghost group per workgroup: the coarse patch
// (all populations of the coarse state fc) is staged in LDS, each ghost
// population is interpolated from it (G, kept for the next coarse step),
// and the ghosts of ff receive the rescaled c0 G0 + c1 G.
template <int KIND, typename S, typename R>
__global__ __launch_bounds__(256) void ghost_patch_kernel(const GhostArgs ga, const S* fc, R* G,
                                                          const R* G0, double c0, double c1,
                                                          double r, S* ff) {
  constexpr int Q = Model<KIND>::Q;
  __shared__ S sp[Q][kPatchMax];
  __shared__ R sv[Q][kGhostMax];
  __shared__ int se[Q][3];
  const GhostGroup* grp = (const GhostGroup*)ga.groups + blockIdx.x;
  const long long gbeg = grp->gbeg;
  const int ngg = grp->gend - grp->gbeg;
  const int lo[3] = {grp->lo[0], grp->lo[1], grp->lo[2]};
  const int m0 = grp->m[0], m1 = grp->m[1], m01 = m0 * m1;
  const int P = m01 * grp->m[2];
  velocity_table<Q>(se);
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    const int pz = p / m01, rem = p - pz * m01, py = rem / m0, px = rem - py * m0;
    const int g3[3] = {lo[0] + px, lo[1] + py, lo[2] + pz};
    int c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
      c[d] = g3[d] < 0 ? g3[d] + ga.cn[d] : (g3[d] >= ga.cn[d] ? g3[d] - ga.cn[d] : g3[d]);
    const size_t idx = ((size_t)c[2] * ga.cn[1] + c[1]) * ga.cn[0] + c[0];
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      sp[I][p] = fc[(size_t)I * (size_t)ga.Nc + idx];
    });
  }
  __syncthreads();
  for (int k = threadIdx.x; k < Q * kGhostMax; k += blockDim.x) {
    const int q = k / kGhostMax, gl = k % kGhostMax;
    if (gl >= ngg) continue;
    const long long gi = gbeg + gl;
    const R g = patch_interp<S, R>(sp[q], ga.gcode[gi], m0, m01);
    const size_t kk = (size_t)q * ga.ng + gi;
    G[kk] = g;
    sv[q][gl] = G0 ? R(c0) * G0[kk] + R(c1) * g : R(c1) * g;
  }
  __syncthreads();
  rescale_group<KIND, S, R>(ga, gbeg, ngg, sv, se, r, ff);
}

// Ghosts of ff := rescale(c1 G) from stored interpolated values, by group.
template <int KIND, typename S, typename R>
__global__ __launch_bounds__(256) void ghost_rescale_kernel(const GhostArgs ga, const R* G,
                                                            double c1, double r, S* ff) {
  constexpr int Q = Model<KIND>::Q;
  __shared__ R sv[Q][kGhostMax];
  __shared__ int se[Q][3];
  const GhostGroup* grp = (const GhostGroup*)ga.groups + blockIdx.x;
  const long long gbeg = grp->gbeg;
  const int ngg = grp->gend - grp->gbeg;
  velocity_table<Q>(se);
  for (int k = threadIdx.x; k < Q * kGhostMax; k += blockDim.x) {
    const int q = k / kGhostMax, gl = k % kGhostMax;
    if (gl < ngg) sv[q][gl] = R(c1) * G[(size_t)q * ga.ng + gbeg + gl];
  }
  __syncthreads();
  rescale_group<KIND, S, R>(ga, gbeg, ngg, sv, se, r, ff);
}

// FP64 partial sums over the nodes of a level box whose type equals want,
// each weighted by w (the node's volume in coarse cells).
template <int KIND, typename S>
__global__ __launch_bounds__(256) void masked_reduce_kernel(const Level L, int want, double w,
                                                            double* partial) {
  constexpr int Q = Model<KIND>::Q;
  __shared__ double sh[5][256];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int nthreads = blockDim.x * blockDim.y;
  double v[5] = {0, 0, 0, 0, 0};
  const int lx = blockIdx.x * blockDim.x + threadIdx.x;
  const int ly = blockIdx.y * blockDim.y + threadIdx.y;
  const int lz = blockIdx.z;
  if (lx < L.M[0] && ly < L.M[1]) {
    const size_t self = ((size_t)lz * L.M[1] + ly) * L.M[0] + lx;
    if (L.type[self] == want) {
      const S* A = (const S*)L.a;
      double d = 0, j[3] = {0, 0, 0};
      for (int i = 0; i < Q; ++i) {
        const double fi = ld<double>(A + (size_t)i * (size_t)L.Nbox + self);
        d += fi;
        j[0] += cx(i) * fi;
        j[1] += cy(i) * fi;
        j[2] += cz(i) * fi;
      }
      const double r = (Model<KIND>::Q == 27) ? 1.0 + d : 1.0;
      v[0] = w * d;
      v[1] = w * j[0];
      v[2] = w * j[1];
      v[3] = w * j[2];
      v[4] = w * 0.5 * (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / r;
    }
  }
  for (int k = 0; k < 5; ++k) sh[k][tid] = v[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s && tid + s < nthreads)
      for (int k = 0; k < 5; ++k) sh[k][tid] += sh[k][tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    const size_t b = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    for (int k = 0; k < 5; ++k) partial[b * 5 + k] = sh[k][0];
  }
}

}  // namespace lbm
