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

// 1-D interpolation stencil for fine coordinate j on an axis of n coarse
// nodes: one node (weight 1) if j is even, else 4-point Lagrange weights at
// j/2 on nodes s..s+3, s = (j-1)/2 - 1, wrapped on periodic axes and moved
// inside [0, n) otherwise.
__host__ __device__ inline int interp_stencil(int j, int n, bool periodic, int idx[4],
                                              double w[4]) {
  if ((j & 1) == 0) {
    int c = j / 2;
    if (periodic) c = ((c % n) + n) % n;
    idx[0] = c;
    w[0] = 1.0;
    return 1;
  }
  // The target j/2 lies at t = j/2 - s from the first node: 3/2 inside,
  // 1/2, 5/2 or 7/2 where the window is moved inside a non-periodic face.
  // The cubic Lagrange weights at these t are dyadic (written out exactly);
  // any other t falls back to the product formula.
  int s = (j - 1) / 2 - 1;
  if (!periodic) s = s < 0 ? 0 : (s > n - 4 ? n - 4 : s);
  const int k2 = j - 2 * s;  // 2t
  if (k2 == 3) {
    w[0] = -1.0 / 16; w[1] = 9.0 / 16; w[2] = 9.0 / 16; w[3] = -1.0 / 16;
  } else if (k2 == 1) {
    w[0] = 5.0 / 16; w[1] = 15.0 / 16; w[2] = -5.0 / 16; w[3] = 1.0 / 16;
  } else if (k2 == 5) {
    w[0] = 1.0 / 16; w[1] = -5.0 / 16; w[2] = 15.0 / 16; w[3] = 5.0 / 16;
  } else if (k2 == 7) {
    w[0] = -5.0 / 16; w[1] = 21.0 / 16; w[2] = -35.0 / 16; w[3] = 35.0 / 16;
  } else {
    const double p = 0.5 * j;
    for (int a = 0; a < 4; ++a) {
      double v = 1.0;
      for (int b = 0; b < 4; ++b)
        if (b != a) v *= (p - (double)(s + b)) / (double)(a - b);
      w[a] = v;
    }
  }
  for (int a = 0; a < 4; ++a) idx[a] = periodic ? (((s + a) % n) + n) % n : s + a;
  return 4;
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
// the bounce-back term, pull_term); across an OUTFLOW face slot I of the
// source with the crossed coordinates kept.
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
  const bool bb = (crossed & (L.bc.wall | L.bc.inlet)) != 0;
  return bb ? own : (crossed ? outflow : normal);
}

// x-wall-only pull for rows off every non-periodic y/z face: population I
// enters through x- (e_Ix = +1 at global x = 0) or x+ (e_Ix = -1 at x =
// n_x - 1), where it is the node's own opposite slot plus a per-direction
// wall term. Both sources are offsets from the lower of the two slabs (one
// scalar-base load).
template <int Q, int I, typename real, bool NT, typename S>
__device__ __forceinline__ real ab_pull_xwall(const Level& L, const S* A, const BoxNode& n) {
  constexpr int IO = opposite<Q>(I);
  const uint32_t sz = sizeof(S);
  const uint32_t nb = (uint32_t)n.at(-cx(I), -cy(I), -cz(I)) * sz;
  if constexpr (cx(I) == 0) {
    return ldo<real, NT>(A + (size_t)I * L.Nbox, nb);
  } else {
    constexpr int LO = I < IO ? I : IO;
    const uint32_t slab = (uint32_t)L.Nbox * sz;
    constexpr int F_ = cx(I) > 0 ? 0 : 1;
    const bool bb = (n.atface & (1u << F_)) != 0;
    const uint32_t off = bb ? (IO - LO) * slab + (uint32_t)n.self * sz : (I - LO) * slab + nb;
    const real v = ldo<real, NT>(A + (size_t)LO * L.Nbox, off);
    return bb ? v + xterm<real>(L.bc, F_, I) : v;
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
  if constexpr (Q == 19) {
    const R uu = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const R eu = R(cx(i)) * j[0] + R(cy(i)) * j[1] + R(cz(i)) * j[2];
      feq[i] = R(weight<19>(i)) * (d + R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu);
    }
  } else {
    // rho prod_a phi(e_a; u_a) - w with phi(0) = 2/3 - u^2,
    // phi(+-1) = (1/3 + u^2 +- u)/2, expanded about the rest factors
    const R rho = R(1) + d;
    R dp[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const R u = j[c] / rho, q = u * u;
      dp[c][0] = R(0.5) * (q - u);
      dp[c][1] = -q;
      dp[c][2] = R(0.5) * (q + u);
    }
    const R p0[3] = {R(1.0 / 6.0), R(2.0 / 3.0), R(1.0 / 6.0)};
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      const R a0 = p0[cx(i) + 1], b0 = p0[cy(i) + 1], c0 = p0[cz(i) + 1];
      const R da = dp[0][cx(i) + 1], db = dp[1][cy(i) + 1], dc = dp[2][cz(i) + 1];
      const R dev = da * b0 * c0 + a0 * db * c0 + a0 * b0 * dc + da * db * c0 + da * b0 * dc +
                    a0 * db * dc + da * db * dc;
      feq[i] = dev + d * (a0 * b0 * c0 + dev);
    }
  }
}

// One pull-and-collide update of a level at time t over the rows r (box-
// local coordinates). mode 0 updates every node whose type is not 2
// (coarse), mode 1 only type-1 nodes (fine). BCM: BC_NONE (no non-periodic
// face), BC_XWALL (rows off the y/z faces, x faces walls) or BC_GENERAL.
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
    }
  } else if constexpr (BCM == BC_XWALL) {
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      f[I] = ab_pull_xwall<Q, I, real, cx(I) == 0>(L, A, n);
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
  int fM[3], flo[3];  // fine box extent and origin
  int cn[3];          // coarse domain extent
  uint32_t cper;      // periodic axes (bit d)
  long long Nc, Nf;
};

// G[q][g] = spatial interpolation of the coarse post-collision field at
// ghost g; one thread per (ghost, population), population-major so that a
// wave reads the stencils of neighbouring ghosts in one population array.
// Tensor interpolation stencil of one ghost (per axis: 1 or 4 coarse nodes).
struct GhostStencil {
  int cnt[3];
  int idx[3][4];
  double w[3][4];
};

__device__ __forceinline__ void ghost_stencil(const GhostArgs& ga, long long gi, GhostStencil& st) {
  const int l = ga.ghosts[gi];
  const int lx = l % ga.fM[0], ly = (l / ga.fM[0]) % ga.fM[1], lz = l / (ga.fM[0] * ga.fM[1]);
  const int j[3] = {lx + ga.flo[0], ly + ga.flo[1], lz + ga.flo[2]};
  for (int d = 0; d < 3; ++d)
    st.cnt[d] = interp_stencil(j[d], ga.cn[d], (ga.cper >> d) & 1u, st.idx[d], st.w[d]);
}

template <typename S, typename R, typename ST>
__device__ __forceinline__ R interp_apply(const GhostArgs& ga, const S* fc, int q, const ST& st) {
  const S* fq = fc + (size_t)q * (size_t)ga.Nc;
  R s = 0;
  for (int c = 0; c < st.cnt[2]; ++c)
    for (int b = 0; b < st.cnt[1]; ++b) {
      const R wbc = R(st.w[1][b] * st.w[2][c]);
      const size_t row = ((size_t)st.idx[2][c] * ga.cn[1] + st.idx[1][b]) * ga.cn[0];
      for (int a = 0; a < st.cnt[0]; ++a)
        s += R(st.w[0][a]) * wbc * ld<R>(fq + row + st.idx[0][a]);
    }
  return s;
}

template <typename S, typename R>
__device__ __forceinline__ R interp_value(const GhostArgs& ga, const S* fc, int q, long long gi) {
  GhostStencil st;
  ghost_stencil(ga, gi, st);
  return interp_apply<S, R>(ga, fc, q, st);
}

template <int Q, typename S, typename R>
__global__ __launch_bounds__(256) void interp_kernel(const GhostArgs ga, const S* fc, R* G) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ga.ng * Q) return;
  const int q = (int)(k / ga.ng);
  const long long gi = k - (long long)q * ga.ng;
  G[(size_t)q * ga.ng + gi] = interp_value<S, R>(ga, fc, q, gi);
}

// Ghost populations = rescale(c0 G0 + c1 G1) into the fine state ff.
template <int KIND, typename S, typename R>
__global__ __launch_bounds__(256) void fill_kernel(const GhostArgs ga, const R* G0, const R* G1,
                                                   double c0, double c1, double r, S* ff) {
  constexpr int Q = Model<KIND>::Q;
  const long long gi = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= ga.ng) return;
  R g[Q], feq[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q)
    g[q] = R(c0) * G0[(size_t)q * ga.ng + gi] + R(c1) * G1[(size_t)q * ga.ng + gi];
  equilibrium_dev<KIND, R>(g, feq);
  const int l = ga.ghosts[gi];
#pragma unroll
  for (int q = 0; q < Q; ++q)
    st(ff + (size_t)q * (size_t)ga.Nf + l, feq[q] + R(r) * (g[q] - feq[q]));
}

// Half-step interface update in one launch: G1 = interpolation of the
// coarse state at t+1 (kept for the next coarse step), the ghosts of the
// second fine substep = rescale(G0/2 + G1/2) into ff_half, and the ghosts
// of the next coarse step's first substep = rescale(G1) into ff_next (that
// array's ghost slots are not written by the second substep). A workgroup
// takes GT ghosts x Q populations, population-major; the rescaling needs
// each ghost's moments, shared through LDS. Same arithmetic as
// interp_kernel followed by fill_kernel.
template <int KIND, typename S, typename R>
__global__ __launch_bounds__(1024) void interp_fill_kernel(const GhostArgs ga, const S* fc,
                                                           R* G1, const R* G0, double r,
                                                           S* ff_half, S* ff_next) {
  constexpr int Q = Model<KIND>::Q;
  constexpr int GT = 1024 / Q;
  __shared__ R sv[2][Q][GT];
  __shared__ R se[2][Q][GT];
  __shared__ GhostStencil sst[GT];
  const int t = threadIdx.x;
  const int q = t / GT, gl = t - q * GT;
  const long long g0 = (long long)blockIdx.x * GT;
  const long long gi = g0 + gl;
  const bool act = q < Q && gi < ga.ng;
  if (t < GT && g0 + t < ga.ng) ghost_stencil(ga, g0 + t, sst[t]);
  __syncthreads();
  if (act) {
    const R g1 = interp_apply<S, R>(ga, fc, q, sst[gl]);
    G1[(size_t)q * ga.ng + gi] = g1;
    sv[0][q][gl] = R(0.5) * G0[(size_t)q * ga.ng + gi] + R(0.5) * g1;
    sv[1][q][gl] = g1;
  }
  __syncthreads();
  if (t < 2 * GT) {
    const int w = t / GT, g = t - w * GT;
    if (g0 + g < ga.ng) {
      R v[Q], feq[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) v[i] = sv[w][i][g];
      equilibrium_dev<KIND, R>(v, feq);
#pragma unroll
      for (int i = 0; i < Q; ++i) se[w][i][g] = feq[i];
    }
  }
  __syncthreads();
  if (act) {
    const int l = ga.ghosts[gi];
    const R e0 = se[0][q][gl], e1 = se[1][q][gl];
    st(ff_half + (size_t)q * (size_t)ga.Nf + l, e0 + R(r) * (sv[0][q][gl] - e0));
    st(ff_next + (size_t)q * (size_t)ga.Nf + l, e1 + R(r) * (sv[1][q][gl] - e1));
  }
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
      const double r = (KIND == 2) ? 1.0 + d : 1.0;
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
