// Host runtime of the refined lattice (lbm_refined_* in include/lbm.h):
// geometry of the nested block-refined levels, memory layout inside the
// caller's block, and the recursive launch sequence of a level-0 step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lbm.h"
#include "refine.h"
#include "trace.h"

using namespace lbm;

namespace {

constexpr int kMaxLevels = 8;

struct HostLevel {
  int o[3] = {0, 0, 0}, M[3] = {0, 0, 0}, n[3] = {0, 0, 0};
  uint32_t span = 0;
  size_t Nbox = 0;
  std::vector<uint8_t> type;
  // tiles (3 ints each) by class: general, walls, plain
  std::vector<int32_t> tiles;
  size_t nt[3] = {0, 0, 0};
  std::vector<int32_t> inj;  // covered nodes read by this level's steps
  std::vector<int32_t> ghosts, gcode;
  std::vector<GhostGroup> groups;
  std::vector<uint8_t> solid;               // host copy over the box (empty: none)
  std::vector<int32_t> link_nodes;          // user links: box indices
  std::vector<float> link_q;                // [n][Q]
  std::vector<int32_t> pre_nodes;           // solid pre-pass list
  std::vector<uint32_t> pre_dirs;
  std::vector<float> pre_q;
  std::vector<int32_t> unodes;              // parent box indices the ghost stencils read
  std::vector<int32_t> pidx;                // per group patch: indices into unodes
  // device offsets
  size_t off_a = 0, off_b = 0, off_c = 0, off_type = 0, off_tiles = 0, off_ghosts = 0, off_gcode = 0,
         off_groups = 0, off_G[3] = {0, 0, 0}, off_pre_nodes = 0, off_pre_dirs = 0,
         off_pre_q = 0, off_inj = 0, off_unodes = 0, off_pidx = 0, off_pc = 0;
  int gi[3] = {0, 1, 2};  // history buffers holding G(t-1), G(t), G(t+1)
  bool have_cur = false, have_prev = false;
  // The level's three state arrays rotate over its steps: dev.a is read, dev.b
  // written, c3 is the array the step after next reads (its ghosts are
  // written ahead by the interpolation of the parent's step).
  void* c3 = nullptr;
  bool tail_pending = false;   // injection into this level queued on its stream
  Lev dev;
  double tau0 = 0.5;
};

int hip_fail(hipError_t e);
}  // namespace

struct lbm_refined {
  lbm_config cfg;
  int kind = 0, Q = 27;
  size_t elem = 4, relem = 4;
  int B = 16, nb[3] = {0, 0, 0}, L = 1;
  std::vector<uint8_t> map;
  HostLevel lev[kMaxLevels];
  BcArgs bc;
  const void* inlet_u[kMaxLevels] = {nullptr};
  const uint8_t* inlet_mask[kMaxLevels] = {nullptr};
  bool geometry_ok = false;
  char* base = nullptr;
  size_t req = 0, off_partial = 0, off_result = 0, max_rblocks = 1;
  hipStream_t stream = nullptr;
  // One more stream per parent level l (default priority), created at the
  // first step: level l's step and its child's interface work run there
  // beside the child's first substep on the lattice's stream, joined by
  // events (see advance).
  hipStream_t aux[kMaxLevels] = {nullptr};
  hipEvent_t ev_fork[kMaxLevels] = {nullptr};   // lattice stream -> aux[l]
  hipEvent_t ev_done[kMaxLevels] = {nullptr};   // aux[l]: step and interface done
  hipEvent_t ev_sub2[kMaxLevels] = {nullptr};   // lattice stream: child substep 2 done
  hipEvent_t ev_tail[kMaxLevels] = {nullptr};   // aux[l]: injection into level l done
  bool aux_tried = false;
  int64_t t = 0;
  // per-launch timing (LBM_TRACE=1 at creation)
  std::unique_ptr<Tracer> tracer = std::make_unique<Tracer>();
};

namespace {

thread_local std::string g_msg;

int hip_fail(hipError_t e) {
  g_msg = std::string("HIP error: ") + hipGetErrorString(e);
  return LBM_EHIP;
}

int check_launch() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LBM_OK : hip_fail(e);
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

bool periodic_axis(const lbm_refined* R, int d) { return ((R->bc.nonper >> (2 * d)) & 1u) == 0; }

int block_level(const lbm_refined* R, int bx, int by, int bz) {
  return R->map[((size_t)bz * R->nb[1] + by) * R->nb[0] + bx];
}

// Is level-l node g (level coordinates, inside the domain) in R_m?
bool in_region(const lbm_refined* R, int l, int m, const int g[3]) {
  const int s = R->B << l;
  return block_level(R, g[0] / s, g[1] / s, g[2] / s) >= m;
}

// Neighbour of g by d on level l: periodic axes wrap; false beyond a
// non-periodic face.
bool neighbour(const lbm_refined* R, int l, const int g[3], const int d[3], int y[3]) {
  const HostLevel& V = R->lev[l];
  for (int a = 0; a < 3; ++a) {
    y[a] = g[a] + d[a];
    if (y[a] >= 0 && y[a] < V.n[a]) continue;
    if (!periodic_axis(R, a)) return false;
    y[a] = (y[a] + V.n[a]) % V.n[a];
  }
  return true;
}

// Box index of level coordinates g (inside the box), or -1.
long box_index(const HostLevel& V, const int g[3]) {
  int b[3];
  for (int d = 0; d < 3; ++d) {
    b[d] = g[d] - V.o[d];
    if (b[d] < 0 || b[d] >= V.M[d]) return -1;
  }
  return ((long)b[2] * V.M[1] + b[1]) * V.M[0] + b[0];
}

void box_coords(const HostLevel& V, long k, int g[3]) {
  g[0] = (int)(k % V.M[0]) + V.o[0];
  g[1] = (int)((k / V.M[0]) % V.M[1]) + V.o[1];
  g[2] = (int)(k / ((long)V.M[0] * V.M[1])) + V.o[2];
}

// Parent window of child coordinate j on axis d of level l-1.
void child_stencil(const lbm_refined* R, int lp, int d, int j, int idx[4], int& start, int& code) {
  const HostLevel& P = R->lev[lp];
  const bool per = periodic_axis(R, d);
  code = child_window(j, P.n[d], per, start);
  for (int a = 0; a < 4; ++a) idx[a] = per ? (((start + a) % P.n[d]) + P.n[d]) % P.n[d] : start + a;
}

// Ghost groups of level l (parent cube of the stencil starts, then box
// index), their parent patches and each ghost's stencil code.
void group_ghosts(lbm_refined* R, int l) {
  HostLevel& V = R->lev[l];
  struct Item {
    std::tuple<int, int, int> cube;
    int32_t k;
    int start[3], code[3];
  };
  std::vector<Item> it(V.ghosts.size());
  for (size_t gi = 0; gi < V.ghosts.size(); ++gi) {
    int g[3];
    box_coords(V, V.ghosts[gi], g);
    Item& e = it[gi];
    e.k = V.ghosts[gi];
    int idx[4];
    for (int d = 0; d < 3; ++d) child_stencil(R, l - 1, d, g[d], idx, e.start[d], e.code[d]);
    e.cube = std::make_tuple(floor_div(e.start[2], kGhostCube), floor_div(e.start[1], kGhostCube),
                             floor_div(e.start[0], kGhostCube));
  }
  std::stable_sort(it.begin(), it.end(), [](const Item& a, const Item& b) {
    return a.cube < b.cube || (a.cube == b.cube && a.k < b.k);
  });
  V.gcode.assign(it.size(), 0);
  V.groups.clear();
  auto add = [&](size_t b, size_t e) {
    GhostGroup gr;
    gr.gbeg = (int)b;
    gr.gend = (int)e;
    for (int d = 0; d < 3; ++d) {
      int lo = it[b].start[d], hi = it[b].start[d] + 3;
      for (size_t k = b; k < e; ++k) {
        lo = std::min(lo, it[k].start[d]);
        hi = std::max(hi, it[k].start[d] + 3);
      }
      gr.lo[d] = lo;
      gr.m[d] = hi - lo + 1;
    }
    for (size_t k = b; k < e; ++k) {
      int c = 0;
      for (int d = 0; d < 3; ++d) c |= ((it[k].start[d] - gr.lo[d]) | (it[k].code[d] << 3)) << (6 * d);
      V.gcode[k] = c;
    }
    V.groups.push_back(gr);
    return gr.m[0] <= kPatchEdge && gr.m[1] <= kPatchEdge && gr.m[2] <= kPatchEdge;
  };
  size_t b = 0;
  while (b < it.size()) {
    size_t e = b;
    while (e < it.size() && it[e].cube == it[b].cube && e - b < (size_t)kGhostMax) ++e;
    if (!add(b, e)) {
      V.groups.pop_back();
      for (size_t k = b; k < e; ++k) add(k, k + 1);
    }
    b = e;
  }
  for (size_t gi = 0; gi < it.size(); ++gi) V.ghosts[gi] = it[gi].k;
  // The parent nodes of the stencils (union, in parent box order) and each
  // group's patch as indices into it (-1: a patch node no stencil reads).
  const HostLevel& P = R->lev[l - 1];
  std::vector<int32_t> umap(P.Nbox, -1);
  for (size_t gi = 0; gi < it.size(); ++gi) {
    int g[3], idx[3][4], st, cd;
    box_coords(V, V.ghosts[gi], g);
    for (int d = 0; d < 3; ++d) child_stencil(R, l - 1, d, g[d], idx[d], st, cd);
    for (int c = 0; c < 64; ++c) {
      const int h[3] = {idx[0][c & 3], idx[1][(c >> 2) & 3], idx[2][c >> 4]};
      const long pb = box_index(P, h);
      if (pb >= 0) umap[pb] = 0;
    }
  }
  V.unodes.clear();
  for (size_t k = 0; k < P.Nbox; ++k)
    if (umap[k] == 0) {
      umap[k] = (int32_t)V.unodes.size();
      V.unodes.push_back((int32_t)k);
    }
  V.pidx.clear();
  for (GhostGroup& gr : V.groups) {
    gr.poff = (int)V.pidx.size();
    for (int pz = 0; pz < gr.m[2]; ++pz)
      for (int py = 0; py < gr.m[1]; ++py)
        for (int px = 0; px < gr.m[0]; ++px) {
          int h[3] = {gr.lo[0] + px, gr.lo[1] + py, gr.lo[2] + pz};
          for (int d = 0; d < 3; ++d)
            if ((P.span >> d) & 1u) h[d] = (h[d] % P.n[d] + P.n[d]) % P.n[d];
          const long pb = box_index(P, h);
          V.pidx.push_back(pb >= 0 ? umap[pb] : -1);
        }
  }
}

// log2 of the tile width of a level: the widest power-of-two row run up to
// 256 nodes that divides the row pitch (a multiple of 64), so that no tile
// hangs over the end of a row.
int tile_shift(const HostLevel& V) { return V.M[0] % 256 == 0 ? 8 : (V.M[0] % 128 == 0 ? 7 : 6); }

// Tile lists of level l: tiles of TW x (256 / TW) x 1 nodes holding fluid or
// band nodes, by class: plain (every active node reads only in-box neighbours
// without wrapping and lies on no domain face), walls (as plain except that
// sources may lie beyond x or y WALL faces; no node on a z face), general.
void build_tiles(lbm_refined* R, int l) {
  HostLevel& V = R->lev[l];
  std::vector<int32_t> lists[3];
  const uint32_t np = R->bc.nonper, wall = R->bc.wall;
  // the wall kernel addresses a population and its opposite from the lower
  // slab with 32-bit offsets
  const double span = 1.0 + (R->Q == 27 ? max_opposite_distance<27>() : max_opposite_distance<19>());
  const bool o32 = span * (double)V.Nbox * (double)R->elem < 4294967296.0;
  const int sh = tile_shift(V), tw = 1 << sh, th = 256 / tw;
  for (int tz = V.o[2]; tz < V.o[2] + V.M[2]; ++tz)
    for (int ty = V.o[1]; ty < V.o[1] + V.M[1]; ty += th)
      for (int tx = V.o[0]; tx < V.o[0] + V.M[0]; tx += tw) {
        bool any = false, plain = true, walls = o32;
        for (int k = 0; k < 256; ++k) {
          const int g[3] = {tx + (k & (tw - 1)), ty + (k >> sh), tz};
          const long bi = box_index(V, g);
          if (bi < 0) continue;
          const uint8_t ty_ = V.type[bi];
          if (ty_ != RT_FLUID && ty_ != RT_BAND) continue;
          any = true;
          for (int c = 0; c < 27; ++c) {
            const int d[3] = {c % 3 - 1, (c / 3) % 3 - 1, c / 9 - 1};
            const int h[3] = {g[0] + d[0], g[1] + d[1], g[2] + d[2]};
            uint32_t crossed = 0;
            for (int a = 0; a < 3; ++a) {
              if (h[a] < 0) crossed |= 1u << (2 * a);
              if (h[a] >= V.n[a]) crossed |= 1u << (2 * a + 1);
            }
            if (crossed) {
              plain = false;
              // beyond x/y WALL faces only
              if ((crossed & 48u) || (crossed & ~(np & wall))) walls = false;
            } else if (box_index(V, h) < 0) {
              plain = walls = false;
            }
          }
          if ((np & 48u) && (g[2] == 0 || g[2] == V.n[2] - 1)) walls = false;
        }
        if (!any) continue;
        const int which = plain ? 2 : (walls ? 1 : 0);
        lists[which].push_back(tx);
        lists[which].push_back(ty);
        lists[which].push_back(tz);
      }
  V.tiles.clear();
  for (int k = 0; k < 3; ++k) {
    V.nt[k] = lists[k].size() / 3;
    V.tiles.insert(V.tiles.end(), lists[k].begin(), lists[k].end());
  }
}

// Covered nodes of level l that its fluid or band nodes pull from (their
// 26 neighbourhoods); their eight children must be fluid or band.
bool build_inject(lbm_refined* R, int l) {
  HostLevel& V = R->lev[l];
  V.inj.clear();
  if (l + 1 >= R->L) return true;
  const HostLevel& C = R->lev[l + 1];
  std::vector<uint8_t> mark(V.Nbox, 0);
  for (size_t k = 0; k < V.Nbox; ++k) {
    if (V.type[k] != RT_FLUID && V.type[k] != RT_BAND) continue;
    int g[3];
    box_coords(V, (long)k, g);
    for (int c = 0; c < 27; ++c) {
      const int d[3] = {c % 3 - 1, (c / 3) % 3 - 1, c / 9 - 1};
      int y[3];
      if (!neighbour(R, l, g, d, y)) continue;
      const long yi = box_index(V, y);
      if (yi >= 0 && V.type[yi] == RT_COVERED) mark[yi] = 1;
    }
  }
  for (size_t k = 0; k < V.Nbox; ++k) {
    if (!mark[k]) continue;
    int g[3];
    box_coords(V, (long)k, g);
    for (int c = 0; c < 8; ++c) {
      const int z[3] = {2 * g[0] + (c & 1), 2 * g[1] + ((c >> 1) & 1), 2 * g[2] + (c >> 2)};
      const long zi = box_index(C, z);
      if (zi < 0 || (C.type[zi] != RT_FLUID && C.type[zi] != RT_BAND)) return false;
    }
    V.inj.push_back((int32_t)k);
  }
  return true;
}

// Geometry of every level from the block map, the periodic axes, the solids
// and the links. Returns false for an invalid configuration.
bool build_geometry(lbm_refined* R) {
  const int L = R->L, B = R->B, Q = R->Q;
  const int n0[3] = {R->cfg.nx, R->cfg.ny, R->cfg.nz};
  // nesting: the neighbours of a block at level m >= 2 are at level >= m - 1
  for (int bz = 0; bz < R->nb[2]; ++bz)
    for (int by = 0; by < R->nb[1]; ++by)
      for (int bx = 0; bx < R->nb[0]; ++bx) {
        const int m = block_level(R, bx, by, bz);
        if (m >= L) return false;
        if (m < 2) continue;
        for (int c = 0; c < 27; ++c) {
          int b[3] = {bx + c % 3 - 1, by + (c / 3) % 3 - 1, bz + c / 9 - 1};
          bool inside = true;
          for (int d = 0; d < 3; ++d) {
            if (b[d] >= 0 && b[d] < R->nb[d]) continue;
            if (!periodic_axis(R, d)) inside = false;
            b[d] = (b[d] + R->nb[d]) % R->nb[d];
          }
          if (inside && block_level(R, b[0], b[1], b[2]) < m - 1) return false;
        }
      }
  for (int l = 0; l < L; ++l) {
    HostLevel& V = R->lev[l];
    int blo[3] = {R->nb[0], R->nb[1], R->nb[2]}, bhi[3] = {-1, -1, -1};
    for (int bz = 0; bz < R->nb[2]; ++bz)
      for (int by = 0; by < R->nb[1]; ++by)
        for (int bx = 0; bx < R->nb[0]; ++bx)
          if (block_level(R, bx, by, bz) >= l) {
            const int b3[3] = {bx, by, bz};
            for (int d = 0; d < 3; ++d) {
              blo[d] = std::min(blo[d], b3[d]);
              bhi[d] = std::max(bhi[d], b3[d] + 1);
            }
          }
    V.span = 0;
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      V.n[d] = n0[d] << l;
      if (bhi[0] < 0) {  // nothing on this level
        lo[d] = hi[d] = 0;
        continue;
      }
      const int s = B << l;
      const bool full = blo[d] == 0 && bhi[d] == R->nb[d];
      if (periodic_axis(R, d)) {
        if (full) {
          V.span |= 1u << d;
          lo[d] = 0;
          hi[d] = V.n[d];
          continue;
        }
        if (blo[d] == 0 || bhi[d] == R->nb[d]) return false;  // touches a periodic end
      }
      lo[d] = std::max(0, blo[d] * s - 1);
      hi[d] = std::min(V.n[d], bhi[d] * s + 1);
    }
    V.o[0] = floor_div(lo[0], 64) * 64;
    V.M[0] = hi[0] > lo[0] ? ((hi[0] - V.o[0] + 63) / 64) * 64 : 0;
    V.o[1] = lo[1];
    V.M[1] = hi[1] - lo[1];
    V.o[2] = lo[2];
    V.M[2] = hi[2] - lo[2];
    if (V.M[0] == 0 || V.M[1] == 0 || V.M[2] == 0) V.M[0] = V.M[1] = V.M[2] = 0;
    V.Nbox = (size_t)V.M[0] * V.M[1] * V.M[2];
    if ((double)V.Nbox * 8.0 >= 2147483647.0) return false;  // 32-bit box offsets
    V.type.assign(V.Nbox, RT_UNUSED);
    V.ghosts.clear();
    for (size_t k = 0; k < V.Nbox; ++k) {
      int g[3];
      box_coords(V, (long)k, g);
      if (g[0] >= V.n[0]) continue;
      if (in_region(R, l, l, g)) {
        V.type[k] = (l + 1 < L && in_region(R, l, l + 1, g)) ? RT_COVERED : RT_FLUID;
        continue;
      }
      for (int c = 0; c < 27; ++c) {
        const int d[3] = {c % 3 - 1, (c / 3) % 3 - 1, c / 9 - 1};
        int y[3];
        if (neighbour(R, l, g, d, y) && in_region(R, l, l, y)) {
          V.type[k] = RT_GHOST;
          V.ghosts.push_back((int32_t)k);
          break;
        }
      }
    }
  }
  // band: parent nodes read by a child's ghost stencils stay parent-updated
  for (int l = 1; l < L; ++l) {
    HostLevel& V = R->lev[l];
    HostLevel& P = R->lev[l - 1];
    for (int32_t gk : V.ghosts) {
      int g[3], idx[3][4], s, c;
      box_coords(V, gk, g);
      for (int d = 0; d < 3; ++d) child_stencil(R, l - 1, d, g[d], idx[d], s, c);
      for (int cz = 0; cz < 4; ++cz)
        for (int cy = 0; cy < 4; ++cy)
          for (int cx_ = 0; cx_ < 4; ++cx_) {
            const int pg[3] = {idx[0][cx_], idx[1][cy], idx[2][cz]};
            const long pi = box_index(P, pg);
            if (pi < 0) return false;
            uint8_t& t = P.type[pi];
            if (t == RT_COVERED) t = RT_BAND;
            if (t != RT_FLUID && t != RT_BAND) return false;
          }
    }
  }
  // solids: off the interface
  for (int l = 0; l < L; ++l) {
    HostLevel& V = R->lev[l];
    if (V.solid.empty()) continue;
    for (size_t k = 0; k < V.Nbox; ++k) {
      if (!V.solid[k]) continue;
      uint8_t& t = V.type[k];
      if (t == RT_GHOST || t == RT_BAND) return false;
      if (t == RT_FLUID || t == RT_COVERED) t = RT_SOLID;
    }
  }
  for (int l = 0; l < L; ++l) {
    HostLevel& V = R->lev[l];
    const bool child = l + 1 < L;
    for (size_t k = 0; k < V.Nbox; ++k) {
      if (V.type[k] != RT_FLUID && V.type[k] != RT_BAND) continue;
      int g[3];
      box_coords(V, (long)k, g);
      for (int i = 0; i < 27; ++i) {
        const int d[3] = {i % 3 - 1, (i / 3) % 3 - 1, i / 9 - 1};
        int y[3];
        if (!neighbour(R, l, g, d, y)) continue;
        const long yi = box_index(V, y);
        if (yi < 0 || V.type[yi] == RT_UNUSED) return false;
        if (!child) continue;
        if (V.type[yi] == RT_SOLID && in_region(R, l, l + 1, y)) return false;
        if (V.type[yi] != RT_COVERED || R->lev[l + 1].solid.empty()) continue;
        const HostLevel& C = R->lev[l + 1];
        for (int c = 0; c < 8; ++c) {
          const int z[3] = {2 * y[0] + (c & 1), 2 * y[1] + ((c >> 1) & 1), 2 * y[2] + (c >> 2)};
          const long zi = box_index(C, z);
          if (zi >= 0 && C.solid[zi]) return false;
        }
      }
    }
    if (l > 0 && !V.solid.empty())
      for (int32_t gk : V.ghosts) {
        int g[3];
        box_coords(V, gk, g);
        for (int c = 0; c < 27; ++c) {
          const int d[3] = {c % 3 - 1, (c / 3) % 3 - 1, c / 9 - 1};
          int y[3];
          if (!neighbour(R, l, g, d, y)) continue;
          const long yi = box_index(V, y);
          if (yi >= 0 && V.solid[yi]) return false;
        }
      }
  }
  // solid pre-pass lists (with the curved links' distances)
  for (int l = 0; l < L; ++l) {
    HostLevel& V = R->lev[l];
    V.pre_nodes.clear();
    V.pre_dirs.clear();
    V.pre_q.clear();
    if (V.solid.empty()) continue;
    std::map<int32_t, size_t> lk;
    for (size_t j = 0; j < V.link_nodes.size(); ++j) lk[V.link_nodes[j]] = j;
    for (size_t k = 0; k < V.Nbox; ++k) {
      if (V.type[k] != RT_FLUID && V.type[k] != RT_BAND) continue;
      int g[3];
      box_coords(V, (long)k, g);
      uint32_t dirs = 0;
      float q[27];
      for (int i = 0; i < 27; ++i) q[i] = 0.5f;
      auto it = lk.find((int32_t)k);
      for (int i = 1; i < Q; ++i) {
        const int d[3] = {-cx(i), -cy(i), -cz(i)};
        int s[3];
        if (!neighbour(R, l, g, d, s)) continue;
        if (V.type[box_index(V, s)] != RT_SOLID) continue;
        dirs |= 1u << i;
        const int kdir = Q == 27 ? opposite<27>(i) : opposite<19>(i);
        if (it == lk.end()) continue;
        const float qq = V.link_q[it->second * Q + kdir];
        if (!(qq > 0.0f && qq <= 1.0f)) continue;
        // the node behind x along the link (x + e_i) must be a fluid node
        // inside the domain, else the halfway rule stays (either branch)
        const int db[3] = {cx(i), cy(i), cz(i)};
        int bh[3];
        if (!neighbour(R, l, g, db, bh)) continue;
        const uint8_t tb = V.type[box_index(V, bh)];
        if (tb == RT_SOLID || tb == RT_UNUSED) continue;
        q[kdir] = qq;
      }
      if (!dirs) continue;
      V.pre_nodes.push_back((int32_t)k);
      V.pre_dirs.push_back(dirs);
      V.pre_q.insert(V.pre_q.end(), q, q + Q);
    }
  }
  for (int l = 0; l < L; ++l) build_tiles(R, l);
  for (int l = 0; l < L; ++l)
    if (!build_inject(R, l)) return false;
  for (int l = 1; l < L; ++l) group_ghosts(R, l);
  return true;
}

void layout(lbm_refined* R) {
  size_t o = 0;
  R->max_rblocks = 1;
  for (int l = 0; l < R->L; ++l) {
    HostLevel& V = R->lev[l];
    const size_t pa = align256(V.Nbox * R->Q * R->elem);
    const size_t ng = V.ghosts.size();
    V.off_a = o; o += pa;
    V.off_b = o; o += pa;
    V.off_c = o; o += pa;
    V.off_type = o; o += align256(V.Nbox);
    V.off_tiles = o; o += align256(V.tiles.size() * 4);
    V.off_ghosts = o; o += align256(ng * 4);
    V.off_gcode = o; o += align256(ng * 4);
    V.off_groups = o; o += align256(V.groups.size() * sizeof(GhostGroup));
    for (int k = 0; k < 3; ++k) {
      V.off_G[k] = o;
      o += align256(ng * R->Q * R->relem);
    }
    V.off_inj = o; o += align256(V.inj.size() * 4);
    V.off_unodes = o; o += align256(V.unodes.size() * 4);
    V.off_pidx = o; o += align256(V.pidx.size() * 4);
    V.off_pc = o; o += align256(V.unodes.size() * R->Q * R->elem);
    V.off_pre_nodes = o; o += align256(V.pre_nodes.size() * 4);
    V.off_pre_dirs = o; o += align256(V.pre_dirs.size() * 4);
    V.off_pre_q = o; o += align256(V.pre_q.size() * 4);
    R->max_rblocks = std::max(R->max_rblocks, (V.Nbox + 255) / 256);
  }
  R->off_partial = o;
  o += align256(R->max_rblocks * 5 * sizeof(double));
  R->off_result = o;
  o += 256;
  R->req = o;
}

void level_physics(const lbm_refined* R, int l, Lev& D) {
  const lbm_config& c = R->cfg;
  const double nu = c.nu * (double)(1 << l);
  const double tau0 = 3.0 * nu + 0.5;
  D.mrt.tau0 = tau0;
  D.mrt.cs18 = 18.0 * c.cs_smag * c.cs_smag;
  D.omega = 1.0 / tau0;
  const double dh[5] = {1.19, 1.4, 1.2, 1.4, 1.98};
  for (int k = 0; k < 5; ++k)
    D.mrt.rates[k] = c.use_default_rates ? (c.mrt_basis == LBM_BASIS_TABLE1 ? 1.0 : dh[k])
                                         : c.rates[k];
}

// Kernel arguments of every level (after bind or a change of boundaries).
void make_levels(lbm_refined* R) {
  for (int l = 0; l < R->L; ++l) {
    HostLevel& V = R->lev[l];
    Lev& D = V.dev;
    std::memset(&D, 0, sizeof(Lev));
    D.a = R->base ? R->base + V.off_a : nullptr;
    D.b = R->base ? R->base + V.off_b : nullptr;
    V.c3 = R->base ? R->base + V.off_c : nullptr;
    D.type = R->base ? (const uint8_t*)(R->base + V.off_type) : nullptr;
    for (int d = 0; d < 3; ++d) {
      D.o[d] = V.o[d];
      D.M[d] = V.M[d];
      D.n[d] = V.n[d];
    }
    D.span = V.span;
    D.tw_shift = tile_shift(V);
    D.Nbox = (long long)V.Nbox;
    level_physics(R, l, D);
    V.tau0 = D.mrt.tau0;
    BcArgs b = R->bc;
    if (b.inlet) {
      const int ax = b.inlet_axis;
      b.inlet_u = R->inlet_u[l];
      b.inlet_mask = R->inlet_mask[l];
      b.inlet_na = V.n[ax == 0 ? 1 : 0];
      b.inlet_nb = V.n[ax == 2 ? 1 : 2];
      b.seed = R->bc.seed + (uint64_t)l;  // each level draws its own perturbation
    }
    fill_wall_terms(b, R->Q);
    D.bc = b;
    V.have_cur = V.have_prev = false;
  }
}

template <typename Fn>
void with_kind_s(const lbm_refined* R, Fn&& fn) {
  auto by_s = [&](auto kc) {
    switch (R->cfg.storage) {
      case LBM_F64: fn(kc, std::type_identity<double>{}); break;
      case LBM_F32: fn(kc, std::type_identity<float>{}); break;
      default: fn(kc, std::type_identity<_Float16>{}); break;
    }
  };
  switch (R->kind) {
    case 0: by_s(std::integral_constant<int, 0>{}); break;
    case 1: by_s(std::integral_constant<int, 1>{}); break;
    case 3: by_s(std::integral_constant<int, 3>{}); break;
    default: by_s(std::integral_constant<int, 2>{}); break;
  }
}

unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

GhostArgs ghost_args(const lbm_refined* R, int l) {
  const HostLevel& V = R->lev[l];
  const HostLevel& P = R->lev[l - 1];
  GhostArgs g;
  g.ghosts = (const int*)(R->base + V.off_ghosts);
  g.ng = (long long)V.ghosts.size();
  g.gcode = (const int*)(R->base + V.off_gcode);
  g.groups = (const int*)(R->base + V.off_groups);
  g.ngroups = (long long)V.groups.size();
  g.unodes = (const int*)(R->base + V.off_unodes);
  g.nu = (long long)V.unodes.size();
  g.pidx = (const int*)(R->base + V.off_pidx);
  for (int d = 0; d < 3; ++d) {
    g.po[d] = P.o[d];
    g.pM[d] = P.M[d];
    g.pn[d] = P.n[d];
  }
  g.pspan = P.span;
  g.pN = (long long)P.Nbox;
  g.cN = (long long)V.Nbox;
  return g;
}

RescaleArgs rescale_args(const lbm_refined* R, int l) {
  RescaleArgs a;
  a.tau0_c = R->lev[l - 1].tau0;
  a.tau0_f = R->lev[l].tau0;
  a.cs = R->cfg.cs_smag;
  a.r = (a.tau0_f - 1.0) / (2.0 * (a.tau0_c - 1.0));
  for (int k = 0; k < 5; ++k) a.rates[k] = R->lev[l].dev.mrt.rates[k];
  return a;
}


// Child level l's ghosts in array ff := rescale(c0 G(t-1) + c1 G(t) + c2
// Gnew), Gnew = the interpolation of parent state fp, kept as G(t+1) (or as
// G(t) when `init`), and, if fn is given, in array fn := rescale(Gnew).
template <int KIND, typename S>
void ghost_patch(lbm_refined* R, int l, const void* fp, void* ff, void* fn, double c0, double c1,
                 double c2, bool init, hipStream_t stream) {
  using Rt = typename Compute<S>::type;
  HostLevel& V = R->lev[l];
  if (V.groups.empty()) return;
  const GhostArgs ga = ghost_args(R, l);
  void* Gn = R->base + V.off_G[V.gi[init ? 1 : 2]];
  S* Pc = (S*)(R->base + V.off_pc);
  {
    TraceScope ts(R->tracer.get(), stream, "ghost_gather_kernel", l);
    hipLaunchKernelGGL((ghost_gather_kernel<KIND, S>), dim3(blocks_for(ga.nu)), dim3(256), 0,
                       stream, ga, (const S*)fp, Pc);
  }
  TraceScope ts(R->tracer.get(), stream, "ghost_patch_kernel", l);
  hipLaunchKernelGGL((ghost_patch_kernel<KIND, S, Rt>), dim3((unsigned)V.groups.size()),
                     dim3(256), 0, stream, ga, (const S*)Pc, (Rt*)Gn,
                     (const Rt*)(R->base + V.off_G[V.gi[1]]),
                     (const Rt*)(R->base + V.off_G[V.gi[0]]), c0, c1, c2, rescale_args(R, l),
                     (S*)ff, (S*)fn);
}

// Covered nodes of level l read by its steps := the rescaled mean of their
// children in level l+1's current state.
template <int KIND, typename S>
void inject(lbm_refined* R, int l, hipStream_t stream) {
  HostLevel& V = R->lev[l];
  const HostLevel& C = R->lev[l + 1];
  if (V.inj.empty()) return;
  InjArgs ia;
  ia.dst = V.dev.b;
  ia.nodes = (const int*)(R->base + V.off_inj);
  ia.n = (long long)V.inj.size();
  ia.src = C.dev.a;
  for (int d = 0; d < 3; ++d) {
    ia.po[d] = V.o[d];
    ia.pM[d] = V.M[d];
    ia.co[d] = C.o[d];
    ia.cM[d] = C.M[d];
  }
  ia.pN = (long long)V.Nbox;
  ia.cN = (long long)C.Nbox;
  TraceScope ts(R->tracer.get(), stream, "inject_kernel", l);
  hipLaunchKernelGGL((inject_kernel<KIND, S>), dim3(blocks_for(ia.n)), dim3(256), 0, stream, ia,
                     rescale_args(R, l + 1));
}

// One step of level l on stream st: the solid pre-pass, then the tile
// classes.
template <int KIND, typename S>
void level_step(lbm_refined* R, int l, long long t, hipStream_t st) {
  HostLevel& V = R->lev[l];
  if (V.Nbox == 0) return;
  const Lev& D = V.dev;
  if (!V.pre_nodes.empty()) {
    constexpr int Q = Model<KIND>::Q;
    TraceScope ts(R->tracer.get(), st, "solid_prepass_kernel", l);
    hipLaunchKernelGGL((solid_prepass_kernel<Q, S>), dim3(blocks_for((long long)V.pre_nodes.size())),
                       dim3(256), 0, st, D, (const int*)(R->base + V.off_pre_nodes),
                       (const uint32_t*)(R->base + V.off_pre_dirs),
                       (const float*)(R->base + V.off_pre_q), (long long)V.pre_nodes.size());
  }
  const int* tiles = (const int*)(R->base + V.off_tiles);
  size_t start = 0;
  for (int k = 0; k < 3; ++k) {
    const size_t n = V.nt[k];
    const int* tl = tiles + 3 * start;
    start += n;
    if (n == 0) continue;
    const dim3 grid((unsigned)n), block(256);
    static const char* const names[3] = {"level_step_kernel (general tiles)",
                                         "level_step_kernel (wall tiles)",
                                         "level_step_kernel (plain tiles)"};
    TraceScope ts(R->tracer.get(), st, names[k], l);
    if (k == 0)
      hipLaunchKernelGGL((level_step_kernel<KIND, S, TILE_GENERAL>), grid, block, 0, st, D, tl, t);
    else if (k == 1)
      hipLaunchKernelGGL((level_step_kernel<KIND, S, TILE_WALLS>), grid, block, 0, st, D, tl, t);
    else
      hipLaunchKernelGGL((level_step_kernel<KIND, S, TILE_PLAIN>), grid, block, 0, st, D, tl, t);
  }
}

// After a step of level V: the array written becomes the one read, the one
// the step after next reads becomes the one written.
void rotate_arrays(HostLevel& V) {
  void* read = V.dev.a;
  V.dev.a = V.dev.b;
  V.dev.b = V.c3;
  V.c3 = read;
}

// Advance level l by one of its steps (index t), and recursively the finer
// levels by two steps each, on the lattice's stream M. The child's first
// substep reads only ghosts prepared from the parent's state before this
// step, so with the parent's own stream X = aux[l] the parent's work runs
// there beside the child's substeps:
//   X: parent step, interpolation of the ghosts for substep 2 (into the
//      array substep 1 writes and substep 2 reads) and of the ghosts of the
//      next parent step's first substep (into the child's third array, which
//      substep 2 writes and nothing reads before that step);
//   M: substep 1;
//   M: after the interpolation, substep 2;
//   X: after substep 2, injection into the parent (beside the next first
//      substep on M, which does not read the parent).
// Ghost slots are written only by the interface kernels, fluid slots only
// by the steps, covered slots only by the injection.
template <int KIND, typename S>
void advance(lbm_refined* R, int l, long long t) {
  HostLevel& V = R->lev[l];
  hipStream_t M = R->stream;
  const bool child = l + 1 < R->L && R->lev[l + 1].Nbox > 0;
  if (!child) {
    level_step<KIND, S>(R, l, t, M);
    rotate_arrays(V);
    return;
  }
  HostLevel& C = R->lev[l + 1];
  if (!C.have_cur) {
    ghost_patch<KIND, S>(R, l + 1, V.dev.a, C.dev.a, nullptr, 0.0, 0.0, 1.0, true, M);
    C.have_cur = true;
    C.have_prev = false;
  }
  hipStream_t X = R->aux[l] ? R->aux[l] : M;
  const bool two = X != M;
  auto to = [&](hipStream_t from, hipStream_t dst, hipEvent_t e) {
    if (!two) return;
    (void)hipEventRecord(e, from);
    (void)hipStreamWaitEvent(dst, e, 0);
  };
  to(M, X, R->ev_fork[l]);
  level_step<KIND, S>(R, l, t, X);
  const double c0 = C.have_prev ? -0.125 : 0.0, c1 = C.have_prev ? 0.75 : 0.5,
               c2 = C.have_prev ? 0.375 : 0.5;
  ghost_patch<KIND, S>(R, l + 1, V.dev.b, C.dev.b, C.c3, c0, c1, c2, false, X);
  if (two) (void)hipEventRecord(R->ev_done[l], X);
  advance<KIND, S>(R, l + 1, 2 * t);
  if (two) (void)hipStreamWaitEvent(M, R->ev_done[l], 0);
  advance<KIND, S>(R, l + 1, 2 * t + 1);
  to(M, X, R->ev_sub2[l]);
  inject<KIND, S>(R, l, X);
  if (two) {
    (void)hipEventRecord(R->ev_tail[l], X);
    V.tail_pending = true;
  }
  const int old = C.gi[0];
  C.gi[0] = C.gi[1];
  C.gi[1] = C.gi[2];
  C.gi[2] = old;
  C.have_prev = true;
  rotate_arrays(V);
}

void destroy_streams(lbm_refined* R) {
  for (int l = 0; l < kMaxLevels; ++l) {
    if (R->aux[l]) {
      (void)hipStreamSynchronize(R->aux[l]);
      (void)hipStreamDestroy(R->aux[l]);
    }
    for (hipEvent_t* e : {&R->ev_fork[l], &R->ev_done[l], &R->ev_sub2[l], &R->ev_tail[l]})
      if (*e) (void)hipEventDestroy(*e);
    R->aux[l] = nullptr;
    R->ev_fork[l] = R->ev_done[l] = R->ev_sub2[l] = R->ev_tail[l] = nullptr;
  }
}

// The parent levels' streams and events; without them every kernel runs in
// order on the lattice's stream.
void create_streams(lbm_refined* R) {
  bool ok = true;
  for (int l = 0; l < R->L && ok; ++l) {
    for (hipEvent_t* e : {&R->ev_fork[l], &R->ev_done[l], &R->ev_sub2[l], &R->ev_tail[l]})
      ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
    if (l + 1 < R->L)
      ok = ok && hipStreamCreateWithFlags(&R->aux[l], hipStreamNonBlocking) == hipSuccess;
  }
  if (!ok) {
    destroy_streams(R);
    (void)hipGetLastError();
  }
}

bool valid_dtype(int d) { return d == LBM_DTYPE_F64 || d == LBM_DTYPE_F32; }

// A LatArgs view of one level's current state box (the uniform lattice's
// init/set/get/macroscopic kernels, parity 0, no boundary pulls).
LatArgs level_view(const lbm_refined* R, int level) {
  const HostLevel& V = R->lev[level];
  LatArgs a;
  std::memset(&a, 0, sizeof(a));
  a.f = V.dev.a;
  a.nx = V.M[0];
  a.ny = V.M[1];
  a.nz = V.M[2];
  a.N = (long long)V.Nbox;
  a.mrt = V.dev.mrt;
  a.omega = V.dev.omega;
  a.bc.ghost_n = 1;
  return a;
}

void view_launch(const LatArgs& a, dim3& grid, dim3& block) {
  int bx = a.nx < 256 ? a.nx : 256;
  if (bx < 1) bx = 1;
  int by = 256 / bx;
  if (by > a.ny) by = a.ny;
  if (by < 1) by = 1;
  block = dim3(bx, by, 1);
  grid = dim3((a.nx + bx - 1) / bx, (a.ny + by - 1) / by, a.nz);
}

int upload(lbm_refined* R, size_t off, const void* src, size_t bytes) {
  if (bytes == 0) return LBM_OK;
  const hipError_t e = hipMemcpyAsync(R->base + off, src, bytes, hipMemcpyHostToDevice, R->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e);
}

void invalidate_history(lbm_refined* R) {
  for (int l = 0; l < R->L; ++l) R->lev[l].have_cur = R->lev[l].have_prev = false;
}

bool level_ok(const lbm_refined* R, int level) { return level >= 0 && level < R->L; }

}  // namespace

extern "C" {

int lbm_refined_create(const lbm_config* cfg, int32_t block, int32_t nlevels,
                       const uint8_t* level_map, lbm_refined** out) {
  if (!cfg || !level_map || !out) return LBM_EINVAL;
  const lbm_config& c = *cfg;
  if (c.model != LBM_D3Q19_MRT_LES && c.model != LBM_D3Q27_FCLB && c.model != LBM_D3Q27_CLB)
    return LBM_EINVAL;
  if (c.storage != LBM_F64 && c.storage != LBM_F32 && c.storage != LBM_F16) return LBM_EINVAL;
  if (nlevels < 1 || nlevels > kMaxLevels) return LBM_EINVAL;
  if (block < 2 || (nlevels >= 3 && block < 3)) return LBM_EINVAL;
  if (c.nx < 1 || c.ny < 1 || c.nz < 1 || c.nx % block || c.ny % block || c.nz % block)
    return LBM_EINVAL;
  if (!(c.nu > 0.0) || !std::isfinite(c.nu) || !(c.cs_smag >= 0.0)) return LBM_EINVAL;
  if (c.model == LBM_D3Q19_MRT_LES && c.mrt_basis != LBM_BASIS_TABLE1 &&
      c.mrt_basis != LBM_BASIS_DHUMIERES)
    return LBM_EINVAL;
  for (int l = 0; l < nlevels; ++l) {
    const double tau = 3.0 * c.nu * (double)(1 << l) + 0.5;
    if (nlevels > 1 && std::fabs(tau - 1.0) < 1e-6) return LBM_EINVAL;
    if (1.0 / tau >= 2.0) return LBM_EINVAL;
  }
  lbm_refined* R = new (std::nothrow) lbm_refined();
  if (!R) return LBM_EINVAL;
  R->cfg = c;
  R->kind = c.model == LBM_D3Q27_FCLB ? 2
            : c.model == LBM_D3Q27_CLB  ? 3
                                        : (c.mrt_basis == LBM_BASIS_TABLE1 ? 0 : 1);
  R->Q = c.model == LBM_D3Q19_MRT_LES ? 19 : 27;
  R->elem = c.storage == LBM_F64 ? 8 : (c.storage == LBM_F32 ? 4 : 2);
  R->relem = c.storage == LBM_F64 ? 8 : 4;
  R->B = block;
  R->L = nlevels;
  R->nb[0] = c.nx / block;
  R->nb[1] = c.ny / block;
  R->nb[2] = c.nz / block;
  R->map.assign(level_map, level_map + (size_t)R->nb[0] * R->nb[1] * R->nb[2]);
  R->stream = (hipStream_t)c.stream;
  std::memset(&R->bc, 0, sizeof(BcArgs));
  R->bc.inlet_axis = 2;
  R->bc.ghost_n = 1;
  // all faces periodic until boundaries are set; a configuration that is
  // only valid with other boundaries waits for them before binding
  R->geometry_ok = build_geometry(R);
  if (!R->geometry_ok) {
    // one-sided windows need 4 nodes on non-periodic axes
    for (int d = 0; d < 3; ++d) {
      const int n = d == 0 ? c.nx : (d == 1 ? c.ny : c.nz);
      if (n < 4) {
        delete R;
        return LBM_EINVAL;
      }
    }
    R->bc.nonper = 0x3Fu;
    const bool ok = build_geometry(R);
    R->bc.nonper = 0;
    if (!ok) {
      delete R;
      return LBM_EINVAL;
    }
    for (int l = 0; l < R->L; ++l) R->lev[l].type.clear();
  }
  make_levels(R);
  layout(R);
  *out = R;
  return LBM_OK;
}

int lbm_refined_geometry(const lbm_refined* R, int32_t level, int32_t lo[3], int32_t dims[3],
                         int64_t counts[5]) {
  if (!R || !lo || !dims || !counts || !level_ok(R, level)) return LBM_EINVAL;
  if (!R->geometry_ok) return LBM_ESTATE;
  const HostLevel& V = R->lev[level];
  for (int d = 0; d < 3; ++d) {
    lo[d] = V.o[d];
    dims[d] = V.M[d];
  }
  for (int k = 0; k < 5; ++k) counts[k] = 0;
  for (uint8_t t : V.type) {
    if (t == RT_FLUID) ++counts[0];
    if (t == RT_BAND) ++counts[1];
    if (t == RT_COVERED) ++counts[2];
    if (t == RT_GHOST) ++counts[3];
    if (t == RT_SOLID) ++counts[4];
  }
  return LBM_OK;
}

int lbm_refined_types(const lbm_refined* R, int32_t level, uint8_t* types) {
  if (!R || !types || !level_ok(R, level)) return LBM_EINVAL;
  if (!R->geometry_ok) return LBM_ESTATE;
  std::memcpy(types, R->lev[level].type.data(), R->lev[level].type.size());
  return LBM_OK;
}

int lbm_refined_required_bytes(const lbm_refined* R, size_t* bytes) {
  if (!R || !bytes) return LBM_EINVAL;
  *bytes = R->req;
  return LBM_OK;
}

int lbm_refined_bind_memory(lbm_refined* R, void* dev, size_t bytes) {
  if (!R || !dev || ((uintptr_t)dev & 255) != 0) return LBM_EINVAL;
  if (!R->geometry_ok) return LBM_ESTATE;
  if (bytes < R->req) return LBM_ENOMEM;
  R->base = (char*)dev;
  R->t = 0;
  make_levels(R);
  for (int l = 0; l < R->L; ++l) {
    HostLevel& V = R->lev[l];
    int rc = upload(R, V.off_type, V.type.data(), V.Nbox);
    if (!rc) rc = upload(R, V.off_tiles, V.tiles.data(), V.tiles.size() * 4);
    if (!rc) rc = upload(R, V.off_ghosts, V.ghosts.data(), V.ghosts.size() * 4);
    if (!rc) rc = upload(R, V.off_gcode, V.gcode.data(), V.gcode.size() * 4);
    if (!rc) rc = upload(R, V.off_groups, V.groups.data(), V.groups.size() * sizeof(GhostGroup));
    if (!rc) rc = upload(R, V.off_pre_nodes, V.pre_nodes.data(), V.pre_nodes.size() * 4);
    if (!rc) rc = upload(R, V.off_pre_dirs, V.pre_dirs.data(), V.pre_dirs.size() * 4);
    if (!rc) rc = upload(R, V.off_pre_q, V.pre_q.data(), V.pre_q.size() * 4);
    if (!rc) rc = upload(R, V.off_inj, V.inj.data(), V.inj.size() * 4);
    if (!rc) rc = upload(R, V.off_unodes, V.unodes.data(), V.unodes.size() * 4);
    if (!rc) rc = upload(R, V.off_pidx, V.pidx.data(), V.pidx.size() * 4);
    if (rc) {
      R->base = nullptr;
      return rc;
    }
  }
  const hipError_t e = hipStreamSynchronize(R->stream);
  if (e != hipSuccess) {
    R->base = nullptr;
    return hip_fail(e);
  }
  return LBM_OK;
}

int lbm_refined_set_boundaries(lbm_refined* R, const lbm_boundaries* bc,
                               const void* const* level_inlet_u,
                               const uint8_t* const* level_inlet_mask) {
  if (!R || !bc) return LBM_EINVAL;
  if (R->base) return LBM_ESTATE;  // the layout depends on the boundaries
  BcArgs b;
  std::memset(&b, 0, sizeof(b));
  b.inlet_axis = 2;
  b.ghost_n = 1;
  int n_inlet = 0, n_out = 0;
  for (int f = 0; f < 6; ++f) {
    const int ty = bc->face_type[f];
    if (ty < LBM_PERIODIC || ty > LBM_PRESSURE) return LBM_EINVAL;
    if (ty != LBM_PERIODIC) b.nonper |= 1u << f;
    for (int k = 0; k < 3; ++k) {
      if (!std::isfinite(bc->face_u[f][k])) return LBM_EINVAL;
      b.face_u[f][k] = bc->face_u[f][k];
    }
    if (ty == LBM_WALL) b.wall |= 1u << f;
    if (ty == LBM_INLET) {
      b.inlet |= 1u << f;
      b.inlet_axis = f / 2;
      ++n_inlet;
    }
    if (ty == LBM_OUTFLOW) {
      b.outflow |= 1u << f;
      ++n_out;
    }
    if (ty == LBM_FREESLIP) b.freeslip |= 1u << f;
    if (ty == LBM_PRESSURE) {
      if (!std::isfinite(bc->face_drho[f]) || !(bc->face_drho[f] > -1.0)) return LBM_EINVAL;
      b.pressure |= 1u << f;
      b.face_drho[f] = bc->face_drho[f];
    }
  }
  for (int d = 0; d < 3; ++d)
    if (((b.nonper >> (2 * d)) & 1u) != ((b.nonper >> (2 * d + 1)) & 1u)) return LBM_EINVAL;
  const int n3[3] = {R->cfg.nx, R->cfg.ny, R->cfg.nz};
  for (int d = 0; d < 3; ++d)
    if (((b.nonper >> (2 * d)) & 1u) && n3[d] < 4) return LBM_EINVAL;
  if (n_inlet > 1 || n_out > 1) return LBM_EINVAL;
  const void* iu[kMaxLevels] = {nullptr};
  const uint8_t* im[kMaxLevels] = {nullptr};
  if (n_inlet) {
    if (!bc->inlet_u || (bc->inlet_dtype != LBM_DTYPE_F64 && bc->inlet_dtype != LBM_DTYPE_F32))
      return LBM_EINVAL;
    if (!std::isfinite(bc->inlet_amp)) return LBM_EINVAL;
    const int d = b.inlet_axis;
    b.inlet_f64 = bc->inlet_dtype == LBM_DTYPE_F64;
    b.inlet_amp = bc->inlet_amp;
    b.seed = bc->seed;
    iu[0] = bc->inlet_u;
    im[0] = bc->inlet_mask;
    for (int l = 1; l < R->L; ++l) {
      if (!level_inlet_u || !level_inlet_u[l]) return LBM_EINVAL;
      iu[l] = level_inlet_u[l];
      im[l] = (bc->inlet_mask && level_inlet_mask) ? level_inlet_mask[l] : nullptr;
      if ((n3[d == 0 ? 1 : 0] << l) >= 16384 || (n3[d == 2 ? 1 : 2] << l) >= 16384)
        return LBM_EINVAL;
    }
  }
  const BcArgs keep = R->bc;
  R->bc = b;
  if (!build_geometry(R)) {
    R->bc = keep;
    R->geometry_ok = build_geometry(R);
    return LBM_EINVAL;
  }
  R->geometry_ok = true;
  for (int l = 0; l < kMaxLevels; ++l) {
    R->inlet_u[l] = iu[l];
    R->inlet_mask[l] = im[l];
  }
  make_levels(R);
  layout(R);
  return LBM_OK;
}

int lbm_refined_set_solids(lbm_refined* R, int32_t level, const uint8_t* solid) {
  if (!R || !level_ok(R, level)) return LBM_EINVAL;
  if (R->base) return LBM_ESTATE;
  if (!R->geometry_ok) return LBM_ESTATE;
  HostLevel& V = R->lev[level];
  std::vector<uint8_t> keep;
  keep.swap(V.solid);
  if (solid) V.solid.assign(solid, solid + V.Nbox);
  if (!build_geometry(R)) {
    V.solid.swap(keep);
    build_geometry(R);
    return LBM_EINVAL;
  }
  V.link_nodes.clear();  // new solids clear the links
  V.link_q.clear();
  build_geometry(R);
  make_levels(R);
  layout(R);
  return LBM_OK;
}

int lbm_refined_set_links(lbm_refined* R, int32_t level, const int32_t* nodes, const float* q,
                          int64_t n) {
  if (!R || !level_ok(R, level) || n < 0 || n >= ((int64_t)1 << 31)) return LBM_EINVAL;
  if (R->base) return LBM_ESTATE;
  if (!R->geometry_ok) return LBM_ESTATE;
  HostLevel& V = R->lev[level];
  if (n > 0 && (!nodes || !q || V.solid.empty())) return LBM_EINVAL;
  V.link_nodes.assign(nodes, nodes + n);
  V.link_q.assign(q, q + (size_t)n * R->Q);
  for (int32_t k : V.link_nodes)
    if (k < 0 || (size_t)k >= V.Nbox) {
      V.link_nodes.clear();
      V.link_q.clear();
      build_geometry(R);
      return LBM_EINVAL;
    }
  build_geometry(R);
  layout(R);
  return LBM_OK;
}

int lbm_refined_init_equilibrium(lbm_refined* R, int level, const void* drho, const void* u,
                                 int dtype, int64_t t0) {
  if (!R || !level_ok(R, level) || !drho || !u || !valid_dtype(dtype)) return LBM_EINVAL;
  if (!R->base) return LBM_EUNBOUND;
  R->t = t0;
  invalidate_history(R);
  if (R->lev[level].Nbox == 0) return LBM_OK;
  const LatArgs a = level_view(R, level);
  dim3 grid, block;
  view_launch(a, grid, block);
  with_kind_s(R, [&](auto kc, auto st_) {
    constexpr int KIND = decltype(kc)::value;
    using S = typename decltype(st_)::type;
    if (dtype == LBM_DTYPE_F64)
      hipLaunchKernelGGL((init_equilibrium_kernel<KIND, S, double>), grid, block, 0, R->stream, a,
                         (const double*)drho, (const double*)u);
    else
      hipLaunchKernelGGL((init_equilibrium_kernel<KIND, S, float>), grid, block, 0, R->stream, a,
                         (const float*)drho, (const float*)u);
  });
  return check_launch();
}

int lbm_refined_set_populations(lbm_refined* R, int level, const void* f, int dtype, int64_t t0) {
  if (!R || !level_ok(R, level) || !f || !valid_dtype(dtype)) return LBM_EINVAL;
  if (!R->base) return LBM_EUNBOUND;
  R->t = t0;
  invalidate_history(R);
  if (R->lev[level].Nbox == 0) return LBM_OK;
  const LatArgs a = level_view(R, level);
  dim3 grid, block;
  view_launch(a, grid, block);
  with_kind_s(R, [&](auto kc, auto st_) {
    constexpr int Q = Model<decltype(kc)::value>::Q;
    using S = typename decltype(st_)::type;
    if (dtype == LBM_DTYPE_F64)
      hipLaunchKernelGGL((set_populations_kernel<Q, S, double>), grid, block, 0, R->stream, a,
                         (const double*)f);
    else
      hipLaunchKernelGGL((set_populations_kernel<Q, S, float>), grid, block, 0, R->stream, a,
                         (const float*)f);
  });
  return check_launch();
}

int lbm_refined_get_populations(lbm_refined* R, int level, void* f, int dtype) {
  if (!R || !level_ok(R, level) || !f || !valid_dtype(dtype)) return LBM_EINVAL;
  if (!R->base) return LBM_EUNBOUND;
  if (R->lev[level].Nbox == 0) return LBM_OK;
  const LatArgs a = level_view(R, level);
  dim3 grid, block;
  view_launch(a, grid, block);
  with_kind_s(R, [&](auto kc, auto st_) {
    constexpr int Q = Model<decltype(kc)::value>::Q;
    using S = typename decltype(st_)::type;
    if (dtype == LBM_DTYPE_F64)
      hipLaunchKernelGGL((get_populations_kernel<Q, S, false, double>), grid, block, 0, R->stream,
                         a, 0, 0LL, (double*)f);
    else
      hipLaunchKernelGGL((get_populations_kernel<Q, S, false, float>), grid, block, 0, R->stream,
                         a, 0, 0LL, (float*)f);
  });
  return check_launch();
}

int lbm_refined_get_macroscopic(lbm_refined* R, int level, void* rho, void* u, int dtype,
                                int rho_mode) {
  if (!R || !level_ok(R, level) || !valid_dtype(dtype)) return LBM_EINVAL;
  if (rho_mode != LBM_RHO_FULL && rho_mode != LBM_RHO_DEVIATION) return LBM_EINVAL;
  if (!R->base) return LBM_EUNBOUND;
  if ((!rho && !u) || R->lev[level].Nbox == 0) return LBM_OK;
  const LatArgs a = level_view(R, level);
  dim3 grid, block;
  view_launch(a, grid, block);
  with_kind_s(R, [&](auto kc, auto st_) {
    constexpr int KIND = decltype(kc)::value;
    using S = typename decltype(st_)::type;
    if (dtype == LBM_DTYPE_F64)
      hipLaunchKernelGGL((macroscopic_kernel<KIND, S, false, double>), grid, block, 0, R->stream,
                         a, 0, 0LL, (double*)rho, (double*)u, rho_mode);
    else
      hipLaunchKernelGGL((macroscopic_kernel<KIND, S, false, float>), grid, block, 0, R->stream, a,
                         0, 0LL, (float*)rho, (float*)u, rho_mode);
  });
  return check_launch();
}

int lbm_refined_step(lbm_refined* R, int64_t n) {
  if (!R || n < 0) return LBM_EINVAL;
  if (!R->base) return LBM_EUNBOUND;
  if (!R->aux_tried && R->L > 1) {
    R->aux_tried = true;
    create_streams(R);
  }
  for (int64_t k = 0; k < n; ++k) {
    with_kind_s(R, [&](auto kc, auto st_) {
      advance<decltype(kc)::value, typename decltype(st_)::type>(R, 0, (long long)R->t);
    });
    R->t += 1;
  }
  // callers see single-stream semantics: join the work still queued on the
  // parent levels' streams
  for (int l = 0; l < R->L; ++l) {
    if (R->lev[l].tail_pending) {
      (void)hipStreamWaitEvent(R->stream, R->ev_tail[l], 0);
      R->lev[l].tail_pending = false;
    }
  }
  return check_launch();
}

int lbm_refined_reduce(lbm_refined* R, double out[5]) {
  if (!R || !out) return LBM_EINVAL;
  if (!R->base) return LBM_EUNBOUND;
  double acc[5] = {0, 0, 0, 0, 0};
  double* partial = (double*)(R->base + R->off_partial);
  double* result = (double*)(R->base + R->off_result);
  for (int l = 0; l < R->L; ++l) {
    const HostLevel& V = R->lev[l];
    if (V.Nbox == 0) continue;
    const unsigned nb = blocks_for((long long)V.Nbox);
    with_kind_s(R, [&](auto kc, auto st_) {
      constexpr int KIND = decltype(kc)::value;
      using S = typename decltype(st_)::type;
      hipLaunchKernelGGL((level_reduce_kernel<KIND, S>), dim3(nb), dim3(256), 0, R->stream, V.dev,
                         (int)RT_FLUID, std::ldexp(1.0, -3 * l), partial);
    });
    int rc = check_launch();
    if (rc) return rc;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, R->stream, partial,
                       (size_t)nb, result);
    rc = check_launch();
    if (rc) return rc;
    double part[5];
    hipError_t e = hipMemcpyAsync(part, result, 5 * sizeof(double), hipMemcpyDeviceToHost,
                                  R->stream);
    if (e != hipSuccess) return hip_fail(e);
    e = hipStreamSynchronize(R->stream);
    if (e != hipSuccess) return hip_fail(e);
    for (int k = 0; k < 5; ++k) acc[k] += part[k];
  }
  for (int k = 0; k < 5; ++k) out[k] = acc[k];
  for (int k = 0; k < 5; ++k)
    if (!std::isfinite(out[k])) return LBM_ENONFINITE;
  return LBM_OK;
}

int lbm_refined_get_time(const lbm_refined* R, int64_t* t) {
  if (!R || !t) return LBM_EINVAL;
  *t = R->t;
  return LBM_OK;
}

int lbm_refined_set_stream(lbm_refined* R, void* stream) {
  if (!R) return LBM_EINVAL;
  R->stream = (hipStream_t)stream;
  return LBM_OK;
}

int lbm_refined_destroy(lbm_refined* R) {
  if (R) R->tracer->report("refined lattice");
  if (R) destroy_streams(R);
  delete R;
  return LBM_OK;
}

}  // extern "C"
