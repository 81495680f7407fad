// gfx950 kernels of the uniform lattice: fused collide-and-stream with
// in-place AA-pattern streaming, boundary rules, initialisation, readouts
// and FP64 reductions.
//
// Storage: one array per population, f[q][z][y][x] (x fastest), deviations
// f_i - w_i in S = double, float or _Float16; arithmetic in double for
// double storage and float otherwise. One thread per node, x-rows mapped
// to consecutive lanes so every population access is a coalesced row
// segment.
//
// AA pattern (two step kinds, one array):
//   even step: node x reads slot i of its own node (= f_i(x, t)), collides
//              and writes f*_i into slot opp(i) of its own node;
//   odd step:  node x reads f_i(x, t) = f*_i(x - e_i, t-1) from slot opp(i)
//              of node x - e_i, collides and writes f*_i into slot i of
//              node x + e_i, which is where that node reads it next.
// Every node reads and writes the same set of locations within a step, so
// the update is race-free in place and moves Q values in and Q values out.
//
// Boundaries (left side of Eq. (1), pull form f_i(x) = f*_i(x - e_i)):
// a population whose source lies beyond a non-periodic face is
//   WALL/INLET: bounced back at the half-way point with the wall or inlet
//               velocity, f_i(x) = f*_opp(i)(x) + 6 w_i e_i.u;
//   PRESSURE:   anti-bounce-back, f_i(x) = -f*_opp(i)(x) + feq_i + feq_opp(i)
//               with the model's equilibrium at the face's density and the
//               node's velocity (of its state at t): fixed pressure;
//   FREESLIP:   reflected specularly at the half-way point, f_i(x) =
//               f*_k(s), k = i with the normal component reversed, s = x -
//               e_i with the crossed coordinates kept;
//   OUTFLOW:    (a z face) copied from the boundary plane, f_i(x) = f*_i(s),
//               s = x - e_i with the z coordinate kept (a ghost layer equal
//               to the last plane: zero normal gradient).
// (WALL before INLET before PRESSURE before FREESLIP before OUTFLOW where
// faces meet.)
// In AA form the bounce-back reads/writes the node's own opposite slot. The
// outflow copy needs f*_i(s) twice (normal streaming and the ghost), so even
// steps also store the inward populations of the outflow plane in a small
// ghost plane buffer that odd steps read; odd steps write the ghost copies
// straight into the (otherwise unwritten) inward slots of the plane.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fclb.h"
#include "mrt.h"
#include "stencil.h"

namespace lbm {

struct BcArgs {
  uint32_t nonper;   // bits of non-periodic faces
  uint32_t wall;     // bits of WALL faces
  uint32_t inlet;    // bit of the INLET face (0 if none)
  uint32_t outflow;  // bit of the OUTFLOW face (0 if none)
  uint32_t freeslip; // bits of FREESLIP faces
  uint32_t pressure; // bits of PRESSURE faces
  double face_drho[6];  // density deviation of PRESSURE faces
  double face_u[6][3];
  const void* inlet_u;
  const uint8_t* inlet_mask;
  double inlet_amp;
  uint64_t seed;
  int inlet_f64;
  int inlet_axis;
  int inlet_na, inlet_nb;
  long long ghost_n; // nodes of a z plane (the outflow face is a z face)
  // 6 w_J (e_J . u_F) for population J entering through x or y face F (0:
  // x-, 1: x+, 2: y-, 3: y+), set on the host with the face velocities
  double wterm[4][27];
  float wterm_f[4][27];
};

struct LatArgs {
  void* f;      // [Q][N]
  void* ghost;  // [Q][ghost_n]
  // interior solid nodes (null if none): per node, bit i set if the pull
  // source x - e_i is a solid node inside the domain, bit 31 if the node
  // itself is solid (see solid_mask_kernel)
  const uint32_t* solid_nb;
  int nx, ny, nz;
  long long N;
  MrtParams mrt;
  double omega;  // FCLB shear rate
  BcArgs bc;
};

// Which rows (fixed y, z; all x) a launch covers. BOX: y in [y0, y0+ny_in),
// z in [z0, z0+nz_in) with blockIdx.z = z - z0. LIST: the rows lying on a
// non-periodic y or z face, enumerated as the zb planes first, then the yb
// rows of every other z; blockIdx.y is the row number.
struct Rows {
  int y0, ny_in, z0, nz_in;
  int zb_n, zb[2];
  int yb_n, yb[2];
  int zi0;
};
enum { ROWS_BOX = 0, ROWS_LIST = 1 };
// Boundary handling of a step kernel: none (all faces periodic), general
// (any face type, any node), or walls only (rows off every non-periodic z
// face and off y faces that are not walls; x and y faces WALL or periodic).
enum { BC_NONE = 0, BC_GENERAL = 1, BC_WALLS = 2 };

// ---------------------------------------------------------------- storage
template <typename S>
struct Compute {
  using type = float;
};
template <>
struct Compute<double> {
  using type = double;
};

// NT: non-temporal (streaming) hint. The step kernels touch every population
// once per step, so nothing they load or store is reused from cache except
// the partial lines at the ends of one-element x shifts; the hint is applied
// where accesses are aligned to the row (measured: +8 % on the even step,
// +3 % on the odd step's x-aligned directions, nothing on shifted ones).
template <typename R, bool NT = false, typename S>
__device__ __forceinline__ R ld(const S* p) {
  if constexpr (NT)
    return R(__builtin_nontemporal_load(p));
  else
    return R(*p);
}
template <bool NT = false, typename S, typename R>
__device__ __forceinline__ void st(S* p, R v) {
  if constexpr (NT)
    __builtin_nontemporal_store(S(v), p);
  else
    *p = S(v);
}

// Population slabs are addressed as a uniform base pointer (SGPRs) plus a
// 32-bit byte offset of the node: the loads and stores then take the
// scalar-base form and need no 64-bit address arithmetic per lane. A slab
// (one population, all nodes) is below 4 GiB (checked at creation); offsets
// from the lower slab of a population and its opposite (up to 7 slabs apart
// in the paper's order) are used only while that span stays below 4 GiB.
template <typename R, bool NT = false, typename S>
__device__ __forceinline__ R ldo(const S* base, uint32_t off) {
  return ld<R, NT>((const S*)((const char*)base + off));
}
template <bool NT = false, typename S, typename R>
__device__ __forceinline__ void sto(S* base, uint32_t off, R v) {
  st<NT>((S*)((char*)base + off), v);
}
// Host: 6 w_J (e_J . u_F) for the x and y faces, per model (the weights
// differ).
inline void fill_wall_terms(BcArgs& b, int Q) {
  for (int F = 0; F < 4; ++F)
    for (int j = 0; j < 27; ++j) {
      double v = 0.0;
      if (j < Q) {
        const double w = Q == 27 ? weight<27>(j) : weight<19>(j);
        v = 6.0 * w * (cx(j) * b.face_u[F][0] + cy(j) * b.face_u[F][1] + cz(j) * b.face_u[F][2]);
      }
      b.wterm[F][j] = v;
      b.wterm_f[F][j] = (float)v;
    }
}

template <typename T>
__device__ __forceinline__ T wterm(const BcArgs& b, int face, int i) {
  if constexpr (sizeof(T) == sizeof(double))
    return b.wterm[face][i];
  else
    return T(b.wterm_f[face][i]);
}

// Wall term of direction I at a wall-row node whose crossed x face is
// FX (if bx) and y face FY (if by): the x face comes first, as in wall_term.
template <int I, typename real, uint32_t XB, uint32_t YB>
__device__ __forceinline__ real wall_row_term(const BcArgs& b, bool bx, int FX, int FY) {
  if constexpr (XB == 0)
    return wterm<real>(b, FY, I);
  else if constexpr (YB == 0)
    return wterm<real>(b, FX, I);
  else
    return bx ? wterm<real>(b, FX, I) : wterm<real>(b, FY, I);
}

// ------------------------------------------------------------------ models
template <int KIND>
struct Model;
// Args: any struct with the level's physics (fields mrt and omega).
template <>
struct Model<0> {  // D3Q19 MRT-LES, Table 1 basis
  static constexpr int Q = 19;
  template <typename real, typename Args>
  __device__ static void collide(real (&f)[19], const Args& a) {
    mrt_collide<real, 0>(f, a.mrt);
  }
};
template <>
struct Model<1> {  // D3Q19 MRT-LES, d'Humieres basis
  static constexpr int Q = 19;
  template <typename real, typename Args>
  __device__ static void collide(real (&f)[19], const Args& a) {
    mrt_collide<real, 1>(f, a.mrt);
  }
};
template <>
struct Model<2> {  // D3Q27 FCLB
  static constexpr int Q = 27;
  template <typename real, typename Args>
  __device__ static void collide(real (&f)[27], const Args& a) {
    fclb_collide<real>(f, real(a.omega));
  }
};
template <>
struct Model<3> {  // D3Q27 CLB: Gaussian fourth- and sixth-order equilibria
  static constexpr int Q = 27;
  template <typename real, typename Args>
  __device__ static void collide(real (&f)[27], const Args& a) {
    fclb_collide<real, true>(f, real(a.omega));
  }
};

// Compile-time loop: calls fn(integral_constant<int, I>) for I = 0..N-1.
template <int I, int N, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (I < N) {
    fn(std::integral_constant<int, I>{});
    static_for<I + 1, N>(fn);
  }
}

// --------------------------------------------------------------- geometry
struct Node {
  int x, y, z;
  int self;
  int xo[3], yo[3], zo[3];  // linear offsets of coordinate c-1, c, c+1
  uint32_t atface;          // non-periodic faces the node lies on
  __device__ __forceinline__ int at(int dx, int dy, int dz) const {
    return zo[dz + 1] + yo[dy + 1] + xo[dx + 1];
  }
};

__device__ __forceinline__ int wrap_dn(int c, int n) { return c == 0 ? n - 1 : c - 1; }
__device__ __forceinline__ int wrap_up(int c, int n) { return c == n - 1 ? 0 : c + 1; }

__device__ __forceinline__ Node make_node(const LatArgs& a, int x, int y, int z) {
  Node n;
  n.x = x;
  n.y = y;
  n.z = z;
  const int sy = a.nx, sz = a.nx * a.ny;
  n.xo[0] = wrap_dn(x, a.nx);
  n.xo[1] = x;
  n.xo[2] = wrap_up(x, a.nx);
  n.yo[0] = wrap_dn(y, a.ny) * sy;
  n.yo[1] = y * sy;
  n.yo[2] = wrap_up(y, a.ny) * sy;
  n.zo[0] = wrap_dn(z, a.nz) * sz;
  n.zo[1] = z * sz;
  n.zo[2] = wrap_up(z, a.nz) * sz;
  n.self = n.zo[1] + n.yo[1] + x;
  uint32_t m = 0;
  m |= (x == 0) ? 1u : 0u;
  m |= (x == a.nx - 1) ? 2u : 0u;
  m |= (y == 0) ? 4u : 0u;
  m |= (y == a.ny - 1) ? 8u : 0u;
  m |= (z == 0) ? 16u : 0u;
  m |= (z == a.nz - 1) ? 32u : 0u;
  n.atface = m & a.bc.nonper;
  return n;
}

// SplitMix64 (Steele, Lea & Flood 2014): one output for a given state.
__device__ __forceinline__ uint64_t splitmix64(uint64_t s) {
  uint64_t z = s + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Velocity of an inlet-face node at step t (base profile + seeded draw).
__device__ __forceinline__ void inlet_velocity(const BcArgs& b, int x, int y, int z, long long t,
                                               double u[3]) {
  const int coord[3] = {x, y, z};
  const int A = coord[b.inlet_axis == 0 ? 1 : 0];
  const int B = coord[b.inlet_axis == 2 ? 1 : 2];
  const long idx = (long)B * b.inlet_na + A;
  const long nf = (long)b.inlet_na * b.inlet_nb;
  const bool pert = b.inlet_mask != nullptr && b.inlet_mask[idx] != 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double v = b.inlet_f64 ? ((const double*)b.inlet_u)[c * nf + idx]
                           : (double)((const float*)b.inlet_u)[c * nf + idx];
    if (pert) {
      const uint64_t key = b.seed ^ (((uint64_t)t << 32) | ((uint64_t)c << 28) |
                                     ((uint64_t)B << 14) | (uint64_t)A);
      const double U = (double)(splitmix64(key) >> 11) * (1.0 / 9007199254740992.0);
      v += b.inlet_amp * (2.0 * U - 1.0);
    }
    u[c] = v;
  }
}

// Bounce-back term 6 w_I e_I.u_w of the first (lowest face index) WALL face
// that x - e_I crosses, selected without branches; 0 if none.
template <int Q, int I, typename real>
__device__ __forceinline__ real wall_term(const BcArgs& b, uint32_t cw) {
  real term = real(0);
#pragma unroll
  for (int d = 2; d >= 0; --d) {
    const int e = c_axis(I, d);
    if (e == 0) continue;
    const int F = e > 0 ? 2 * d : 2 * d + 1;
    const real dot = real(6.0 * weight<Q>(I) *
                          (cx(I) * b.face_u[F][0] + cy(I) * b.face_u[F][1] + cz(I) * b.face_u[F][2]));
    term = ((cw >> F) & 1u) ? dot : term;
  }
  return term;
}

// Equilibrium (deviation form) of the population with velocity (ex, ey,
// ez) for the moments d = sum f, j = sum e f: the incompressible
// polynomial of Eq. (2) for D3Q19 MRT, the product form rho prod_a
// phi(e_a; u_a) - w of the factorized model for D3Q27 (phi(0) = 2/3 - u^2,
// phi(+-1) = (1/3 + u^2 +- u)/2, expanded about the rest factors).
template <int KIND, typename R>
__device__ __forceinline__ R equilibrium_one(R d, const R (&j)[3], int ex, int ey, int ez) {
  if constexpr (Model<KIND>::Q == 19) {
    const R uu = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
    const R eu = R(ex) * j[0] + R(ey) * j[1] + R(ez) * j[2];
    const int e2 = ex * ex + ey * ey + ez * ez;
    const R w = e2 == 0 ? R(1.0 / 3.0) : (e2 == 1 ? R(1.0 / 18.0) : R(1.0 / 36.0));
    return w * (d + R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu);
  } else {
    const R rho = R(1) + d;
    const int e[3] = {ex, ey, ez};
    R p[3], dp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const R u = j[c] / rho, q = u * u;
      p[c] = e[c] == 0 ? R(2.0 / 3.0) : R(1.0 / 6.0);
      dp[c] = e[c] == 0 ? -q : (e[c] < 0 ? R(0.5) * (q - u) : R(0.5) * (q + u));
    }
    const R a0 = p[0], b0 = p[1], c0 = p[2], da = dp[0], db = dp[1], dc = dp[2];
    const R dev = da * b0 * c0 + a0 * db * c0 + a0 * b0 * dc + da * db * c0 + da * b0 * dc +
                  a0 * db * dc + da * db * dc;
    return dev + d * (a0 * b0 * c0 + dev);
  }
}

// The fixed-pressure (anti-bounce-back) part of direction I at a PRESSURE
// face: feq_I + feq_opp(I) at density deviation dout and velocity u.
template <int KIND, int I, typename real>
__device__ __forceinline__ real pressure_pair(real dout, const real (&u)[3]) {
  constexpr int IO = opposite<Model<KIND>::Q>(I);
  const real s = (Model<KIND>::Q == 19) ? real(1) : real(1) + dout;
  const real j[3] = {s * u[0], s * u[1], s * u[2]};
  return equilibrium_one<KIND, real>(dout, j, cx(I), cy(I), cz(I)) +
         equilibrium_one<KIND, real>(dout, j, cx(IO), cy(IO), cz(IO));
}

// Density deviation of the lowest face in the mask of crossed PRESSURE faces.
__device__ __forceinline__ double pressure_drho(const BcArgs& b, uint32_t crossed) {
  double d = 0.0;
#pragma unroll
  for (int F = 5; F >= 0; --F) d = ((crossed >> F) & 1u) ? b.face_drho[F] : d;
  return d;
}

// Compile-time table of the images of I across the axes of mask m (bit d:
// axis d), selected at run time without an indexed array.
template <int Q, int I, bool OPP>
__device__ __forceinline__ int mirror_slot(int m) {
  int k = OPP ? opposite<Q>(I) : I;
  static_for<1, 8>([&](auto mc) {
    constexpr int M = decltype(mc)::value;
    constexpr int J = mirror_index(I, M);
    constexpr int V = J < 0 ? 0 : (OPP ? opposite<Q>(J) : J);
    k = m == M ? V : k;
  });
  return k;
}

// Axes (bit d) of the FREESLIP faces in a crossed-face set.
__device__ __forceinline__ int slip_axes(uint32_t fs) {
  return ((fs & 3u) ? 1 : 0) | ((fs & 12u) ? 2 : 0) | ((fs & 48u) ? 4 : 0);
}

// Where f_I(x, t) lives at odd parity: slot opp(I) of node x - e_I (the
// pull through the post-collision slots), the node's own slot I (WALL or
// INLET bounce-back, see pull_term) or the outflow ghost plane (index of
// x - e_I in the z plane). Selects only, no branches, so the loads of all
// directions can be issued back to back.
// EXT: interior solids or FREESLIP faces may be present (the rules for
// them are compiled only then: they cost registers in the general kernel).
template <int Q, int I, typename S, bool BC, bool EXT = true>
__device__ __forceinline__ const S* pull_addr(const LatArgs& a, const S* F, const Node& n,
                                              uint32_t sb) {
  constexpr int IO = opposite<Q>(I);
  const size_t N = (size_t)a.N;
  const S* normal = F + (size_t)IO * N + n.at(-cx(I), -cy(I), -cz(I));
  if constexpr (!BC) {
    return normal;
  } else {
    // a solid source bounces back like a WALL face at rest (pull_term adds
    // nothing: no face is crossed)
    const uint32_t crossed = n.atface & pull_faces(I);
    const bool bb = (crossed & (a.bc.wall | a.bc.inlet)) != 0 || (EXT && ((sb >> I) & 1u) != 0);
    const S* own = F + (size_t)I * N + n.self;
    const S* ghost = (const S*)a.ghost + (size_t)I * (size_t)a.bc.ghost_n +
                     (n.yo[1 - cy(I)] + n.xo[1 - cx(I)]);
    if constexpr (!EXT) return bb ? own : (crossed ? ghost : normal);
    // specular: f*_k(s) sits in slot opp(k) of s since the even step; where
    // the OUTFLOW face is crossed too (s on the outflow plane, k inward),
    // that slot has a second reader that rewrites it within the odd step,
    // so the value comes from the ghost plane the even step filled
    const uint32_t fs = crossed & a.bc.freeslip;
    const int axes = slip_axes(fs);
    const S* slip = F + (size_t)mirror_slot<Q, I, true>(axes) * N +
                    n.at((crossed & 3u) ? 0 : -cx(I), (crossed & 12u) ? 0 : -cy(I),
                         (crossed & 48u) ? 0 : -cz(I));
    const S* slip_ghost = (const S*)a.ghost +
                          (size_t)mirror_slot<Q, I, false>(axes) * (size_t)a.bc.ghost_n +
                          (n.yo[(crossed & 12u) ? 1 : 1 - cy(I)] +
                           n.xo[(crossed & 3u) ? 1 : 1 - cx(I)]);
    const bool edge = (crossed & a.bc.outflow) != 0;
    // PRESSURE: anti-bounce-back from the own slot, where the store that
    // filled it (either parity) left the completed value
    const bool pr = (crossed & a.bc.pressure) != 0;
    return (bb || pr) ? own : (fs ? (edge ? slip_ghost : slip) : (crossed ? ghost : normal));
  }
}

// Bounce-back term added to the value read by pull_addr: 6 w_I e_I.u with
// the wall's velocity (first WALL face crossed) or the inlet velocity.
template <int Q, int I, typename real>
__device__ __forceinline__ real pull_term(const BcArgs& b, uint32_t atface, const real* uin) {
  const uint32_t crossed = atface & pull_faces(I);
  const uint32_t cw = crossed & b.wall;
  const uint32_t ci = crossed & b.inlet;
  const real tw = wall_term<Q, I, real>(b, cw);
  const real ti = real(6.0 * weight<Q>(I)) *
                  (real(cx(I)) * uin[0] + real(cy(I)) * uin[1] + real(cz(I)) * uin[2]);
  return cw ? tw : (ci ? ti : real(0));
}

// Store f*_I(x, t) at the end of an odd step (push to x + e_I), with the
// bounce-back rule (own slot opp(I), minus the term) and the outflow rule
// (dropped; a node on the outflow plane also writes the inward population
// I of its in-plane neighbour, the ghost copy of the next pull).
template <int Q, int I, typename real, typename S, bool BC, bool EXT = true>
__device__ __forceinline__ void push(const LatArgs& a, S* F, const Node& n, real v,
                                     const real* uin, uint32_t sb, const real* unode) {
  constexpr int IO = opposite<Q>(I);
  const size_t N = (size_t)a.N;
  if constexpr (!BC) {
    sto<cx(I) == 0>(F + (size_t)I * N, (uint32_t)n.at(cx(I), cy(I), cz(I)) * (uint32_t)sizeof(S),
                    v);
  } else {
    S* normal = F + (size_t)I * N + n.at(cx(I), cy(I), cz(I));
    const uint32_t crossed = n.atface & push_faces(I);
    const uint32_t cw = crossed & a.bc.wall;
    const uint32_t ci = crossed & a.bc.inlet;
    // the bounce-back of direction I is the pull of opp(I) seen from here
    const real tw = wall_term<Q, IO, real>(a.bc, cw);
    const real ti = real(6.0 * weight<Q>(I)) * (real(cx(IO)) * uin[0] + real(cy(IO)) * uin[1] +
                                                real(cz(IO)) * uin[2]);
    const real term = cw ? tw : (ci ? ti : real(0));
    // x + e_I solid (the pull source of opp(I)): bounce back, no term
    const bool bb = (cw | ci) != 0 || (EXT && ((sb >> IO) & 1u) != 0);
    S* own = F + (size_t)IO * N + n.self;
    if constexpr (!EXT) {
      if (bb || !crossed) st(bb ? own : normal, bb ? v + term : v);
      if ((n.atface & a.bc.outflow & pull_faces(I)) && (n.atface & push_faces(I)) == 0)
        st(F + (size_t)I * N + n.at(cx(I), cy(I), 0), v);
      return;
    }
    // leaving through a PRESSURE face: returns as opp(I) into the own slot,
    // -f*_I + feq_I + feq_opp(I) at the node's velocity
    if ((crossed & a.bc.pressure) && !bb) {
      constexpr int KQ = Q == 27 ? 2 : 0;
      const real u[3] = {unode[0], unode[1], unode[2]};
      const real dp = real(pressure_drho(a.bc, crossed & a.bc.pressure));
      st(own, -v + pressure_pair<KQ, I, real>(dp, u));
      return;
    }
    // leaving through FREESLIP faces only (no OUTFLOW): the image k of I
    // arrives at x + e_I with the crossed coordinates kept, slot k
    const uint32_t fs = crossed & a.bc.freeslip;
    const bool slip = !bb && fs != 0 && (crossed & a.bc.outflow) == 0;
    S* mirrored = F + (size_t)mirror_slot<Q, I, false>(slip_axes(fs)) * N +
                  n.at((crossed & 3u) ? 0 : cx(I), (crossed & 12u) ? 0 : cy(I),
                       (crossed & 48u) ? 0 : cz(I));
    if (bb || !crossed || slip) st(bb ? own : (slip ? mirrored : normal), bb ? v + term : v);
    // on the outflow plane, a population entering through the outflow face
    // and leaving through FREESLIP faces is also the image arriving at the
    // in-plane node (z kept): the source of the edge rule (free slip, then
    // the outflow's kept coordinate), a second copy as for the ghost plane
    if (slip && (n.atface & a.bc.outflow & pull_faces(I)))
      st(F + (size_t)mirror_slot<Q, I, false>(slip_axes(fs)) * N +
             n.at((crossed & 3u) ? 0 : cx(I), (crossed & 12u) ? 0 : cy(I), 0),
         v);
    if ((n.atface & a.bc.outflow & pull_faces(I)) && (n.atface & push_faces(I)) == 0)
      st(F + (size_t)I * N + n.at(cx(I), cy(I), 0), v);
  }
}

// Wall rows: rows off every non-periodic z face (and off y faces that are
// not walls), whose x and y faces are WALL or periodic. Population I enters
// through x- (e_Ix = +1 at x = 0), x+ (e_Ix = -1 at x = nx-1), y- or y+ in
// the same way, where it is the node's own slot I plus a per-direction wall
// term (the x face first where a node lies on both). The bounce-back source
// (slot I of the node itself) and the normal source (slot opp(I) of x - e_I)
// are selected as offsets from the lower of the two slabs, so one
// scalar-base load serves both.
// SOLID: interior solid nodes present (sb: the node's solid-neighbour
// mask); a solid source bounces back like a wall at rest, without a term.
template <int Q, int I, typename real, bool NT, bool SOLID, typename S>
__device__ __forceinline__ real pull_walls(const LatArgs& a, const S* F, const Node& n,
                                           uint32_t sb) {
  constexpr int IO = opposite<Q>(I);
  constexpr uint32_t XB = pull_faces(I) & 3u, YB = pull_faces(I) & 12u;
  const uint32_t sz = sizeof(S);
  const uint32_t nb = (uint32_t)n.at(-cx(I), -cy(I), -cz(I)) * sz;
  if constexpr ((XB | YB) == 0 && (!SOLID || I == 0)) {
    return ldo<real, NT>(F + (size_t)IO * a.N, nb);
  } else {
    constexpr int LO = I < IO ? I : IO;
    const uint32_t slab = (uint32_t)a.N * sz;
    const bool bx = (n.atface & XB) != 0, by = (n.atface & YB) != 0;
    const bool bs = SOLID && ((sb >> I) & 1u) != 0;
    const bool bb = bx || by || bs;
    const uint32_t off = bb ? (I - LO) * slab + (uint32_t)n.self * sz : (IO - LO) * slab + nb;
    const real v = ldo<real, NT>(F + (size_t)LO * a.N, off);
    if constexpr ((XB | YB) == 0) {
      return v;
    } else {
      const real term =
          wall_row_term<I, real, XB, YB>(a.bc, bx, cx(I) > 0 ? 0 : 1, cy(I) > 0 ? 2 : 3);
      return (bx || by) ? v + term : v;
    }
  }
}

template <int Q, int I, typename real, bool NT, bool SOLID, typename S>
__device__ __forceinline__ void push_walls(const LatArgs& a, S* F, const Node& n, real v,
                                           uint32_t sb) {
  constexpr int IO = opposite<Q>(I);
  constexpr uint32_t XB = push_faces(I) & 3u, YB = push_faces(I) & 12u;
  const uint32_t sz = sizeof(S);
  const uint32_t nb = (uint32_t)n.at(cx(I), cy(I), cz(I)) * sz;
  if constexpr ((XB | YB) == 0 && (!SOLID || I == 0)) {
    sto<NT>(F + (size_t)I * a.N, nb, v);
  } else {
    // leaving through a wall, I returns as opp(I), entering through the
    // same face: the term is that of opp(I) at that face; a solid target
    // (the pull source of opp(I)) returns it without a term
    constexpr int LO = I < IO ? I : IO;
    const uint32_t slab = (uint32_t)a.N * sz;
    const bool bx = (n.atface & XB) != 0, by = (n.atface & YB) != 0;
    const bool bs = SOLID && ((sb >> IO) & 1u) != 0;
    const bool bb = bx || by || bs;
    const uint32_t off = bb ? (IO - LO) * slab + (uint32_t)n.self * sz : (I - LO) * slab + nb;
    if constexpr ((XB | YB) == 0) {
      sto<NT>(F + (size_t)LO * a.N, off, v);
    } else {
      const real term =
          wall_row_term<IO, real, XB, YB>(a.bc, bx, cx(I) > 0 ? 1 : 0, cy(I) > 0 ? 3 : 2);
      sto<NT>(F + (size_t)LO * a.N, off, (bx || by) ? v + term : v);
    }
  }
}

// --------------------------------------------------------------- kernels
__device__ __forceinline__ bool node_coords(const LatArgs& a, int& x, int& y, int& z) {
  x = blockIdx.x * blockDim.x + threadIdx.x;
  y = blockIdx.y * blockDim.y + threadIdx.y;
  z = blockIdx.z;
  return x < a.nx && y < a.ny;
}

template <int ROWS>
__device__ __forceinline__ bool row_coords(const LatArgs& a, const Rows& r, int& x, int& y,
                                           int& z) {
  x = blockIdx.x * blockDim.x + threadIdx.x;
  if constexpr (ROWS == ROWS_BOX) {
    y = r.y0 + (int)(blockIdx.y * blockDim.y + threadIdx.y);
    z = r.z0 + (int)blockIdx.z;
    return x < a.nx && y < r.y0 + r.ny_in;
  } else {
    const int row = blockIdx.y;
    if (row < r.zb_n * a.ny) {
      z = r.zb[row / a.ny];
      y = row % a.ny;
    } else {
      const int k = row - r.zb_n * a.ny;
      y = r.yb[k % r.yb_n];
      z = r.zi0 + k / r.yb_n;
    }
    return x < a.nx;
  }
}

// One collide-and-stream step at time t over the rows selected by r. If rec
// is not null, the natural pre-collision state the step collides is also
// written to rec ([Q][N] in the compute type). The record is a runtime
// switch, so recording and plain steps run the same code and round alike.
// EXT: interior solids (wall rows and general kernel) or FREESLIP faces
// (general kernel) present.
template <int KIND, typename S, bool ODD, int BCM, int ROWS, bool EXT = false>
__global__ __launch_bounds__(256) void step_kernel(const LatArgs a, const Rows r, long long t,
                                                   typename Compute<S>::type* rec) {
  using M = Model<KIND>;
  using real = typename Compute<S>::type;
  constexpr int Q = M::Q;
  constexpr bool BC = BCM == BC_GENERAL;
  int x, y, z;
  if (!row_coords<ROWS>(a, r, x, y, z)) return;
  const Node n = make_node(a, x, y, z);
  S* __restrict__ F = (S*)a.f;
  const size_t N = (size_t)a.N;
  // interior solids: solid nodes are skipped (the even step runs this only
  // with PRESSURE faces; otherwise solid nodes run it harmlessly on their own
  // slots, which nothing reads)
  uint32_t sb = 0;
  if constexpr (BC && EXT) {
    if (a.solid_nb) {
      sb = a.solid_nb[n.self];
      if (sb >> 31) return;
    }
  } else if constexpr (BCM == BC_WALLS && EXT) {
    sb = a.solid_nb[n.self];
    if (sb >> 31) return;
  }
  double uin_prev[3] = {0, 0, 0}, uin_now[3] = {0, 0, 0};
  if constexpr (BC && ODD) {
    if (n.atface & a.bc.inlet) {
      inlet_velocity(a.bc, n.x, n.y, n.z, t - 1, uin_prev);
      inlet_velocity(a.bc, n.x, n.y, n.z, t, uin_now);
    }
  }
  const uint32_t self_off = (uint32_t)n.self * (uint32_t)sizeof(S);
  real f[Q];
  if constexpr (!ODD) {
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      f[I] = ldo<real, true>(F + (size_t)I * N, self_off);
    });
  } else {
    if constexpr (BCM == BC_WALLS) {
      static_for<0, Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        f[I] = pull_walls<Q, I, real, cx(I) == 0, EXT>(a, F, n, sb);
      });
    } else if constexpr (BCM == BC_NONE) {
      static_for<0, Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        f[I] = ldo<real, cx(I) == 0>(F + (size_t)opposite<Q>(I) * N,
                                     (uint32_t)n.at(-cx(I), -cy(I), -cz(I)) * (uint32_t)sizeof(S));
      });
    } else {
      static_for<0, Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        f[I] = ld<real, !BC && cx(I) == 0>(pull_addr<Q, I, S, BC, EXT>(a, F, n, sb));
      });
      if constexpr (BC) {
        const real up[3] = {real(uin_prev[0]), real(uin_prev[1]), real(uin_prev[2])};
        static_for<0, Q>([&](auto ic) {
          constexpr int I = decltype(ic)::value;
          f[I] += pull_term<Q, I, real>(a.bc, n.atface, up);
        });
      }
    }
  }
  if (rec != nullptr) {
    const uint32_t roff = (uint32_t)n.self * (uint32_t)sizeof(real);
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      sto<true>(rec + (size_t)I * N, roff, f[I]);
    });
  }
  // the node's velocity (kept by the collision) for PRESSURE faces
  real unode[3] = {0, 0, 0};
  if constexpr (BC && EXT) {
    if (n.atface & a.bc.pressure) {
      real d = 0, j[3] = {0, 0, 0};
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        d += f[i];
        j[0] += real(cx(i)) * f[i];
        j[1] += real(cy(i)) * f[i];
        j[2] += real(cz(i)) * f[i];
      }
      const real rho = Q == 27 ? real(1) + d : real(1);
      unode[0] = j[0] / rho;
      unode[1] = j[1] / rho;
      unode[2] = j[2] / rho;
    }
  }
  M::collide(f, a);
  if constexpr (!ODD) {
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      real v = f[I];
      // leaving through a PRESSURE face: the own slot opp(I) takes the
      // anti-bounce-back value the next pull reads as it is
      if constexpr (BC && EXT) {
        constexpr int KQ = Q == 27 ? 2 : 0;
        const uint32_t crossed = n.atface & push_faces(I);
        if ((crossed & a.bc.pressure) && !(crossed & (a.bc.wall | a.bc.inlet)))
          v = -v + pressure_pair<KQ, I, real>(
                       real(pressure_drho(a.bc, crossed & a.bc.pressure)), unode);
      }
      sto<true>(F + (size_t)opposite<Q>(I) * N, self_off, v);
    });
    if constexpr (BC) {
      if (n.atface & a.bc.outflow) {
        S* G = (S*)a.ghost;
        const long long g = n.yo[1] + n.xo[1];
        static_for<0, Q>([&](auto ic) {
          constexpr int I = decltype(ic)::value;
          if (n.atface & a.bc.outflow & pull_faces(I))
            st(G + (size_t)I * (size_t)a.bc.ghost_n + g, f[I]);
        });
      }
    }
  } else {
    if constexpr (BCM == BC_WALLS) {
      static_for<0, Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        push_walls<Q, I, real, cx(I) == 0, EXT>(a, F, n, f[I], sb);
      });
    } else {
      const real un[3] = {real(uin_now[0]), real(uin_now[1]), real(uin_now[2])};
      static_for<0, Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        push<Q, I, real, S, BC, EXT>(a, F, n, f[I], un, sb, unode);
      });
    }
  }
}

// Even step of FP16 storage with two x-neighbouring nodes per lane (x even):
// one 4-byte load and store per population serve both, where one node per
// lane moves 2 bytes per access. Each node collides in FP32 exactly as in
// step_kernel (bitwise the same result). No solids, links, pressure faces or
// recording (those lattices take step_kernel).
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
template <int KIND, bool BC>
__global__ __launch_bounds__(256) void step_even_pair_kernel(const LatArgs a) {
  using M = Model<KIND>;
  constexpr int Q = M::Q;
  const int x = 2 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const int y = (int)(blockIdx.y * blockDim.y + threadIdx.y);
  const int z = (int)blockIdx.z;
  if (x >= a.nx || y >= a.ny) return;
  _Float16* __restrict__ F = (_Float16*)a.f;
  const size_t N = (size_t)a.N;
  const uint32_t off = (uint32_t)((((size_t)z * a.ny + y) * a.nx + x) * sizeof(_Float16));
  half2_t v[Q];
  static_for<0, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    v[I] = __builtin_nontemporal_load((const half2_t*)((const char*)(F + (size_t)I * N) + off));
  });
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    float f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = float(v[i][k]);
    M::collide(f, a);
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i][k] = _Float16(f[i]);
    if constexpr (BC) {
      const Node n = make_node(a, x + k, y, z);
      if (n.atface & a.bc.outflow) {
        _Float16* G = (_Float16*)a.ghost;
        const long long g = n.yo[1] + n.xo[1];
        static_for<0, Q>([&](auto ic) {
          constexpr int I = decltype(ic)::value;
          if (n.atface & a.bc.outflow & pull_faces(I))
            st(G + (size_t)I * (size_t)a.bc.ghost_n + g, f[I]);
        });
      }
    }
  }
  static_for<0, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    __builtin_nontemporal_store(v[I],
                                (half2_t*)((char*)(F + (size_t)opposite<Q>(I) * N) + off));
  });
}

// Natural (pre-collision) populations of a node in double precision; zero
// (the rest state) at a solid node, whose populations are not updated.
template <int Q, typename S, bool BC>
__device__ __forceinline__ void fetch_natural(const LatArgs& a, const Node& n, int parity,
                                              long long t, double (&f)[Q]) {
  const S* F = (const S*)a.f;
  const size_t N = (size_t)a.N;
  uint32_t sb = 0;
  if constexpr (BC) {
    if (a.solid_nb) {
      sb = a.solid_nb[n.self];
      if (sb >> 31) {
        for (int i = 0; i < Q; ++i) f[i] = 0.0;
        return;
      }
    }
  }
  if (parity == 0) {
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      f[I] = ld<double, true>(F + (size_t)I * N + n.self);
    });
  } else {
    double uin[3] = {0, 0, 0};
    if constexpr (BC) {
      if (n.atface & a.bc.inlet) inlet_velocity(a.bc, n.x, n.y, n.z, t - 1, uin);
    }
    static_for<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      f[I] = ld<double>(pull_addr<Q, I, S, BC>(a, F, n, sb));
      if constexpr (BC) f[I] += pull_term<Q, I, double>(a.bc, n.atface, uin);
    });
  }
}

// Solid-neighbour masks of the nodes (LatArgs::solid_nb) from a solid flag
// per node; flag[0] := 1 if a solid node lies on an OUTFLOW face (the
// outflow copy would read it).
template <int Q>
__global__ __launch_bounds__(256) void solid_mask_kernel(const LatArgs a, const uint8_t* solid,
                                                         uint32_t* out, int* flag) {
  int x, y, z;
  if (!node_coords(a, x, y, z)) return;
  const Node n = make_node(a, x, y, z);
  uint32_t m = solid[n.self] ? (1u << 31) : 0u;
  static_for<1, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    if ((n.atface & pull_faces(I)) == 0 && solid[n.at(-cx(I), -cy(I), -cz(I))]) m |= 1u << I;
  });
  out[n.self] = m;
  if ((m >> 31) && (n.atface & a.bc.outflow)) flag[0] = 1;
}

// Bouzidi's linear interpolated bounce-back (the curved no-slip walls of
// the paper's nozzle, Section 3) on the links from listed fluid nodes x to
// solid neighbours x + e_K, run right after a step over the slot the halfway
// rule filled. With q the wall's distance along the link (fraction of it)
// and I = opp(K) the returning direction:
//   q < 1/2:  f_I(x) = 2q f*_K(x) + (1 - 2q) f*_K(x - e_K)
//   q >= 1/2: f_I(x) = f*_K(x) / (2q) + (2q - 1)/(2q) f*_I(x)
// In AA form each value sits in a known slot: f*_K(x) in slot opp(K) of x
// (the halfway value, replaced here) after either step; after an even step
// f*_K(x - e_K) is in slot opp(K) of x - e_K and f*_I(x) in slot K of x,
// after an odd step the other way round. A link needs x - e_K to be a fluid
// node inside the domain, else the halfway value stays. No other node's
// links touch these slots (x + e_K is solid), and a node reads all its
// links' values before it writes any (a link reads the slot the opposite
// link writes).
// One 32-lane group per listed node, lane K handling direction K: a block
// of 256 threads holds 8 whole nodes, and its barrier puts every read of
// the block before any write.
template <int Q, typename S, bool AFTER_ODD>
__global__ __launch_bounds__(256) void link_kernel(const LatArgs a, const int32_t* nodes,
                                                   const float* q, long long n) {
  using real = typename Compute<S>::type;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long k = t >> 5;
  const int K = (int)(t & 31);
  // the lane's direction, selected from the compile-time tables
  int ex = 0, ey = 0, ez = 0, ko = 0;
  uint32_t pf = 0;
  static_for<1, Q>([&](auto kc) {
    constexpr int D = decltype(kc)::value;
    if (K == D) {
      ex = cx(D);
      ey = cy(D);
      ez = cz(D);
      ko = opposite<Q>(D);
      pf = pull_faces(D);
    }
  });
  S* F = (S*)a.f;
  const size_t N = (size_t)a.N;
  bool link = false;
  real v = 0;
  int self = 0;
  if (k < n && K >= 1 && K < Q) {
    self = nodes[k];
    if (self >= 0 && (long long)self < a.N) {
      const uint32_t sb = a.solid_nb[self];
      const float d = q[(size_t)k * Q + K];
      if (!(sb >> 31) && ((sb >> ko) & 1u) && !((sb >> K) & 1u) && d > 0.f && d <= 1.f &&
          d != 0.5f) {
        const Node nd = make_node(a, self % a.nx, (self / a.nx) % a.ny, self / (a.nx * a.ny));
        if ((nd.atface & pf) == 0) {
          link = true;
          const int b = nd.at(-ex, -ey, -ez);
          const real A = ld<real>(F + (size_t)ko * N + self);
          const real B = ld<real>(AFTER_ODD ? F + (size_t)K * N + self : F + (size_t)ko * N + b);
          const real C = ld<real>(AFTER_ODD ? F + (size_t)ko * N + b : F + (size_t)K * N + self);
          const real tq = real(2) * real(d);
          v = d < 0.5f ? tq * A + (real(1) - tq) * B : A / tq + (tq - real(1)) / tq * C;
        }
      }
    }
  }
  __syncthreads();
  if (link) st(F + (size_t)ko * N + self, v);
}

template <int Q, typename S, bool BC, typename O>
__global__ __launch_bounds__(256) void get_populations_kernel(const LatArgs a, int parity,
                                                              long long t, O* out) {
  int x, y, z;
  if (!node_coords(a, x, y, z)) return;
  const Node n = make_node(a, x, y, z);
  double f[Q];
  fetch_natural<Q, S, BC>(a, n, parity, t, f);
  for (int i = 0; i < Q; ++i) out[(size_t)i * a.N + n.self] = O(f[i]);
}

template <int Q, typename S, typename O>
__global__ __launch_bounds__(256) void set_populations_kernel(const LatArgs a, const O* in) {
  int x, y, z;
  if (!node_coords(a, x, y, z)) return;
  const int self = (z * a.ny + y) * a.nx + x;
  S* F = (S*)a.f;
  for (int i = 0; i < Q; ++i)
    F[(size_t)i * a.N + self] = S((double)in[(size_t)i * a.N + self]);
}

// Equilibrium deviations of the model for (drho, u), computed in double:
// MRT Eq. (2); FCLB the product equilibrium rho prod phi(e_a; u_a), whose
// central moments are the Table 2 equilibria.
template <int KIND, typename S, typename I>
__global__ __launch_bounds__(256) void init_equilibrium_kernel(const LatArgs a, const I* drho,
                                                               const I* u) {
  constexpr int Q = Model<KIND>::Q;
  int x, y, z;
  if (!node_coords(a, x, y, z)) return;
  const size_t self = ((size_t)z * a.ny + y) * a.nx + x;
  const size_t N = (size_t)a.N;
  const double d = drho[self];
  const double ux = u[self], uy = u[N + self], uz = u[2 * N + self];
  S* F = (S*)a.f;
  if constexpr (Q == 19) {
    const double uu = ux * ux + uy * uy + uz * uz;
    static_for<0, 19>([&](auto ic) {
      constexpr int I2 = decltype(ic)::value;
      const double eu = cx(I2) * ux + cy(I2) * uy + cz(I2) * uz;
      F[(size_t)I2 * N + self] = S(weight<19>(I2) * (d + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
    });
  } else {
    // phi(0) = 2/3 - u^2, phi(+-1) = (1/3 + u^2 +- u)/2; deviation from the
    // rest factors (2/3, 1/6) expanded so no O(1) terms cancel.
    const double uv[3] = {ux, uy, uz};
    double ph[3][3], ph0[3];  // ph[d][e+1] = phi, ph0 = rest factor
    for (int c = 0; c < 3; ++c) {
      const double q = uv[c] * uv[c];
      ph[c][1] = 2.0 / 3.0 - q;
      ph[c][0] = 0.5 * (1.0 / 3.0 + q - uv[c]);
      ph[c][2] = 0.5 * (1.0 / 3.0 + q + uv[c]);
    }
    ph0[0] = 1.0 / 6.0;
    ph0[1] = 2.0 / 3.0;
    ph0[2] = 1.0 / 6.0;
    static_for<0, 27>([&](auto ic) {
      constexpr int I2 = decltype(ic)::value;
      const double a0 = ph0[cx(I2) + 1], b0 = ph0[cy(I2) + 1], c0 = ph0[cz(I2) + 1];
      const double da = ph[0][cx(I2) + 1] - a0, db = ph[1][cy(I2) + 1] - b0,
                   dc = ph[2][cz(I2) + 1] - c0;
      // (a0+da)(b0+db)(c0+dc)(1+d) - a0 b0 c0
      const double prod_dev = da * b0 * c0 + a0 * db * c0 + a0 * b0 * dc + da * db * c0 +
                              da * b0 * dc + a0 * db * dc + da * db * dc;
      const double full = a0 * b0 * c0 + prod_dev;
      F[(size_t)I2 * N + self] = S(prod_dev + d * full);
    });
  }
}

template <int KIND, typename S, bool BC, typename O>
__global__ __launch_bounds__(256) void macroscopic_kernel(const LatArgs a, int parity, long long t,
                                                          O* rho, O* u, int rho_mode) {
  constexpr int Q = Model<KIND>::Q;
  int x, y, z;
  if (!node_coords(a, x, y, z)) return;
  const Node n = make_node(a, x, y, z);
  double f[Q];
  fetch_natural<Q, S, BC>(a, n, parity, t, f);
  double d = 0, j[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i) {
    d += f[i];
    j[0] += cx(i) * f[i];
    j[1] += cy(i) * f[i];
    j[2] += cz(i) * f[i];
  }
  const double r = (Model<KIND>::Q == 27) ? 1.0 + d : 1.0;
  if (rho) rho[n.self] = O(rho_mode == 0 ? 1.0 + d : d);
  if (u) {
    const size_t N = (size_t)a.N;
    u[n.self] = O(j[0] / r);
    u[N + n.self] = O(j[1] / r);
    u[2 * N + n.self] = O(j[2] / r);
  }
}

// Running sums for time averages of the velocity (the jet statistics of
// Section 3: mean velocity and the turbulent intensity of Eq. (25)): adds u
// and the squares u_a^2 of the current natural state (u as in
// macroscopic_kernel) to sums [6][N] in FP64; each node owns its entries.
template <int KIND, typename S, bool BC>
__global__ __launch_bounds__(256) void stats_accumulate_kernel(const LatArgs a, int parity,
                                                               long long t, double* sums) {
  constexpr int Q = Model<KIND>::Q;
  int x, y, z;
  if (!node_coords(a, x, y, z)) return;
  const Node n = make_node(a, x, y, z);
  double f[Q];
  fetch_natural<Q, S, BC>(a, n, parity, t, f);
  double d = 0, j[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i) {
    d += f[i];
    j[0] += cx(i) * f[i];
    j[1] += cy(i) * f[i];
    j[2] += cz(i) * f[i];
  }
  const double r = (Model<KIND>::Q == 27) ? 1.0 + d : 1.0;
  const size_t N = (size_t)a.N;
  // the running sums are streamed once per call (non-temporal hint)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double u = j[c] / r;
    double* s1 = sums + c * N + n.self;
    double* s2 = sums + (3 + c) * N + n.self;
    st<true>(s1, ld<double, true>(s1) + u);
    st<true>(s2, ld<double, true>(s2) + u * u);
  }
}

// Time averages from count accumulated states: mean = sums / count, rms =
// sqrt(<u_a^2> - <u_a>^2) (0 where rounding makes it negative) and, if ti
// is not null, the turbulent intensity of Eq. (25): the rms of the
// streamwise component (axis ax) over the mean streamwise velocity at the
// jet-axis point (p0, p1) of the node's cross-section (the two other
// coordinates in increasing order).
template <typename O>
__global__ __launch_bounds__(256) void stats_finalize_kernel(const LatArgs a, const double* sums,
                                                             double inv_count, O* mean, O* rms,
                                                             O* ti, int ax, int p0, int p1) {
  int x, y, z;
  if (!node_coords(a, x, y, z)) return;
  const size_t N = (size_t)a.N;
  const size_t self = ((size_t)z * a.ny + y) * a.nx + x;
  double m[3], v[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    m[c] = sums[c * N + self] * inv_count;
    const double var = sums[(3 + c) * N + self] * inv_count - m[c] * m[c];
    v[c] = var > 0.0 ? sqrt(var) : 0.0;
    mean[c * N + self] = O(m[c]);
    rms[c * N + self] = O(v[c]);
  }
  if (ti) {
    int g[3] = {x, y, z};
    const int o0 = ax == 0 ? 1 : 0, o1 = ax == 2 ? 1 : 2;
    g[o0] = p0;
    g[o1] = p1;
    const size_t axis_node = ((size_t)g[2] * a.ny + g[1]) * a.nx + g[0];
    ti[self] = O(v[ax] / (sums[ax * N + axis_node] * inv_count));
  }
}

// Per-block FP64 partial sums (mass deviation, momentum, kinetic energy) in
// a fixed tree order, one row of 5 per block of the launch grid.
template <int KIND, typename S, bool BC>
__global__ __launch_bounds__(256) void reduce_partial_kernel(const LatArgs a, int parity,
                                                             long long t, double* partial) {
  constexpr int Q = Model<KIND>::Q;
  __shared__ double sh[5][256];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int nthreads = blockDim.x * blockDim.y;
  double v[5] = {0, 0, 0, 0, 0};
  int x, y, z;
  // a block sums the planes z = blockIdx.z + k gridDim.z (one plane when the
  // grid spans every plane)
  if (node_coords(a, x, y, z)) {
    for (; z < a.nz; z += gridDim.z) {
      const Node n = make_node(a, x, y, z);
      double f[Q];
      fetch_natural<Q, S, BC>(a, n, parity, t, f);
      double d = 0, j[3] = {0, 0, 0};
      for (int i = 0; i < Q; ++i) {
        d += f[i];
        j[0] += cx(i) * f[i];
        j[1] += cy(i) * f[i];
        j[2] += cz(i) * f[i];
      }
      const double r = (Model<KIND>::Q == 27) ? 1.0 + d : 1.0;
      v[0] += d;
      v[1] += j[0];
      v[2] += j[1];
      v[3] += j[2];
      v[4] += 0.5 * (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / r;
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

static __global__ __launch_bounds__(256) void reduce_final_kernel(const double* partial, size_t nb,
                                                           double* out) {
  __shared__ double sh[5][256];
  const int tid = threadIdx.x;
  double v[5] = {0, 0, 0, 0, 0};
  for (size_t b = tid; b < nb; b += 256)
    for (int k = 0; k < 5; ++k) v[k] += partial[b * 5 + k];
  for (int k = 0; k < 5; ++k) sh[k][tid] = v[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s)
      for (int k = 0; k < 5; ++k) sh[k][tid] += sh[k][tid + s];
    __syncthreads();
  }
  if (tid == 0)
    for (int k = 0; k < 5; ++k) out[k] = sh[k][0];
}

// Plain vectorised copy, one 16-byte element per thread with the streaming
// hint: the achievable-bandwidth probe.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
static __global__ __launch_bounds__(256) void copy_kernel(u32x4* __restrict__ dst,
                                                   const u32x4* __restrict__ src, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace lbm
