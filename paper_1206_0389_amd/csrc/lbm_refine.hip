// Host runtime of the two-level refined lattice (lbm_refined_* in
// include/lbm.h): geometry of the block-refined region, memory layout inside
// the caller's block, and the per-coarse-step launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "refine.h"

using namespace lbm;

struct lbm_refined {
  lbm_config cfg;
  int kind, Q;
  size_t elem, relem;  // bytes per stored value / per compute value
  int B, nb[3];
  std::vector<uint8_t> mask;
  int lo[3], M[3];
  size_t Nc, Nf;
  std::vector<uint8_t> ctype, ftype;
  std::vector<int32_t> ghosts, covered;
  std::vector<int32_t> gcode;       // per ghost: stencil code (GhostGroup)
  std::vector<GhostGroup> groups;   // ghost groups staged by one workgroup
  double r;
  hipStream_t stream;
  // second stream (default priority, non-blocking) on which the coarse step
  // runs concurrently with the first fine substep, joined by events
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr, sub1_ev = nullptr;
  bool side_tried = false;
  // device layout
  char* base = nullptr;
  size_t off[14] = {0};
  size_t req = 0;
  Level Lc, Lf;
  void *g0 = nullptr, *g1 = nullptr;
  double* partial = nullptr;
  double* result = nullptr;
  size_t nblocks_c = 0, nblocks_f = 0;
  dim3 grid_c, block_c, grid_f, block_f;
  bool g0_valid = false;
  int64_t t = 0;
  bool has_bc = false;
  bool geometry_ok = false;  // false until a valid boundary set is known
  // per level (0 coarse, 1 fine): wall rows (off the non-periodic z domain
  // faces and off y faces that are not walls; wall kernel) and the rows on
  // those faces (general kernel)
  struct Plan {
    int mode;  // 0: no boundary logic, 1: wall rows + face rows, 2: general
    Rows all, inner, face;
    dim3 grid_all, grid_inner, grid_face, block, block_face;
  } plan[2];
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

void shape_for(int nx, int ny, int nz, dim3& grid, dim3& block, size_t& nblocks) {
  int bx = nx < 256 ? nx : 256;
  if (bx < 1) bx = 1;
  int by = 256 / bx;
  if (by > ny) by = ny;
  if (by < 1) by = 1;
  block = dim3(bx, by, 1);
  grid = dim3((nx + bx - 1) / bx, (ny + by - 1) / by, nz);
  nblocks = (size_t)grid.x * grid.y * grid.z;
}

bool block_refined(const lbm_refined* R, int bx, int by, int bz) {
  return R->mask[((size_t)bz * R->nb[1] + by) * R->nb[0] + bx] != 0;
}

// Is fine global node j inside the refined region?
bool fine_refined(const lbm_refined* R, const int j[3]) {
  const int n3[3] = {R->cfg.nx, R->cfg.ny, R->cfg.nz};
  int b[3];
  for (int d = 0; d < 3; ++d) {
    if (j[d] < 0 || j[d] >= 2 * n3[d]) return false;
    b[d] = j[d] / (2 * R->B);
  }
  return block_refined(R, b[0], b[1], b[2]);
}

// Orders the ghost list by group (coarse cube of kGhostCube^3 cells, then
// stencil shape, then box index: the lanes of a wave mostly share one
// shape), splits each cube into groups of at most kGhostMax ghosts, and sets
// each group's coarse patch and each ghost's stencil code relative to it. A
// group whose patch would exceed kPatchEdge on an axis is split into single
// ghosts (patches of at most 4 nodes per axis).
void group_ghosts(lbm_refined* R, uint32_t nonper) {
  const int n3[3] = {R->cfg.nx, R->cfg.ny, R->cfg.nz};
  const size_t ng = R->ghosts.size();
  struct Item {
    long long key;
    int32_t l;
    int start[3], code[3];
  };
  std::vector<Item> it(ng);
  int ncube[3];
  for (int d = 0; d < 3; ++d) ncube[d] = (n3[d] + kGhostCube - 1) / kGhostCube;
  for (size_t g = 0; g < ng; ++g) {
    const int32_t l = R->ghosts[g];
    const int lx = l % R->M[0], ly = (l / R->M[0]) % R->M[1], lz = l / (R->M[0] * R->M[1]);
    const int j[3] = {lx + R->lo[0], ly + R->lo[1], lz + R->lo[2]};
    Item& e = it[g];
    e.l = l;
    int cube[3], shape = 0;
    for (int d = 0; d < 3; ++d) {
      e.code[d] = stencil_code(j[d], n3[d], ((nonper >> (2 * d)) & 1u) == 0, e.start[d]);
      cube[d] = (j[d] >> 1) / kGhostCube;
      shape |= e.code[d] != 0 ? 1 << d : 0;
    }
    const long long c = ((long long)cube[2] * ncube[1] + cube[1]) * ncube[0] + cube[0];
    e.key = (c * 8 + shape) * (1ll << 32) + l;
  }
  std::sort(it.begin(), it.end(), [](const Item& a, const Item& b) { return a.key < b.key; });
  R->gcode.assign(ng, 0);
  R->groups.clear();
  auto add_group = [&](size_t b, size_t e) {
    GhostGroup gr;
    gr.gbeg = (int)b;
    gr.gend = (int)e;
    for (int d = 0; d < 3; ++d) {
      int lo = it[b].start[d], hi = lo;
      for (size_t k = b; k < e; ++k) {
        lo = std::min(lo, it[k].start[d]);
        hi = std::max(hi, it[k].start[d] + (it[k].code[d] ? 3 : 0));
      }
      gr.lo[d] = lo;
      gr.m[d] = hi - lo + 1;
    }
    for (size_t k = b; k < e; ++k) {
      int code = 0;
      for (int d = 0; d < 3; ++d) code |= ((it[k].start[d] - gr.lo[d]) | (it[k].code[d] << 3)) << (6 * d);
      R->gcode[k] = code;
    }
    R->groups.push_back(gr);
    return gr.m[0] <= kPatchEdge && gr.m[1] <= kPatchEdge && gr.m[2] <= kPatchEdge;
  };
  size_t b = 0;
  while (b < ng) {
    const long long cube = it[b].key >> 35;
    size_t e = b;
    while (e < ng && (it[e].key >> 35) == cube && e - b < (size_t)kGhostMax) ++e;
    if (!add_group(b, e)) {
      R->groups.pop_back();
      for (size_t k = b; k < e; ++k) add_group(k, k + 1);
    }
    b = e;
  }
  for (size_t g = 0; g < ng; ++g) R->ghosts[g] = it[g].l;
}

// Box, node types, ghost and covered lists. Returns false if a refined
// region touches a periodic axis without spanning it.
bool build_geometry(lbm_refined* R, const uint32_t nonper) {
  const int n3[3] = {R->cfg.nx, R->cfg.ny, R->cfg.nz};
  int blo[3] = {R->nb[0], R->nb[1], R->nb[2]}, bhi[3] = {0, 0, 0};
  bool any = false;
  for (int bz = 0; bz < R->nb[2]; ++bz)
    for (int by = 0; by < R->nb[1]; ++by)
      for (int bx = 0; bx < R->nb[0]; ++bx) {
        if (!block_refined(R, bx, by, bz)) continue;
        any = true;
        const int b[3] = {bx, by, bz};
        for (int d = 0; d < 3; ++d) {
          blo[d] = std::min(blo[d], b[d]);
          bhi[d] = std::max(bhi[d], b[d] + 1);
        }
      }
  for (int d = 0; d < 3; ++d) {
    if (!any) {
      R->lo[d] = 0;
      R->M[d] = 0;
      continue;
    }
    const bool periodic = ((nonper >> (2 * d)) & 1u) == 0;
    if (periodic && !((blo[d] == 0 && bhi[d] == R->nb[d]) || (blo[d] > 0 && bhi[d] < R->nb[d])))
      return false;
    int a = 2 * R->B * blo[d], b = 2 * R->B * bhi[d];
    if (a > 0) --a;
    if (b < 2 * n3[d]) ++b;
    R->lo[d] = a;
    R->M[d] = b - a;
  }
  R->Nf = (size_t)R->M[0] * R->M[1] * R->M[2];
  R->ftype.assign(R->Nf, 0);
  R->ghosts.clear();
  for (int lz = 0; lz < R->M[2]; ++lz)
    for (int ly = 0; ly < R->M[1]; ++ly)
      for (int lx = 0; lx < R->M[0]; ++lx) {
        const int j[3] = {lx + R->lo[0], ly + R->lo[1], lz + R->lo[2]};
        const size_t l = ((size_t)lz * R->M[1] + ly) * R->M[0] + lx;
        if (fine_refined(R, j)) {
          R->ftype[l] = 1;
          continue;
        }
        bool near = false;
        for (int k = 0; k < 27 && !near; ++k) {
          const int jj[3] = {j[0] + k % 3 - 1, j[1] + (k / 3) % 3 - 1, j[2] + k / 9 - 1};
          near = fine_refined(R, jj);
        }
        if (near) {
          R->ftype[l] = 2;
          R->ghosts.push_back((int32_t)l);
        }
      }
  group_ghosts(R, nonper);
  R->ctype.assign(R->Nc, 0);
  for (int z = 0; z < n3[2]; ++z)
    for (int y = 0; y < n3[1]; ++y)
      for (int x = 0; x < n3[0]; ++x)
        if (block_refined(R, x / R->B, y / R->B, z / R->B))
          R->ctype[((size_t)z * n3[1] + y) * n3[0] + x] = 2;
  // nodes read by a ghost stencil stay coarse-updated ("band")
  for (int32_t l : R->ghosts) {
    const int lx = l % R->M[0], ly = (l / R->M[0]) % R->M[1], lz = l / (R->M[0] * R->M[1]);
    const int j[3] = {lx + R->lo[0], ly + R->lo[1], lz + R->lo[2]};
    int idx[3][4], cnt[3];
    double w[3][4];
    for (int d = 0; d < 3; ++d)
      cnt[d] = interp_stencil(j[d], n3[d], ((nonper >> (2 * d)) & 1u) == 0, idx[d], w[d]);
    for (int c = 0; c < cnt[2]; ++c)
      for (int b = 0; b < cnt[1]; ++b)
        for (int a = 0; a < cnt[0]; ++a) {
          uint8_t& t = R->ctype[((size_t)idx[2][c] * n3[1] + idx[1][b]) * n3[0] + idx[0][a]];
          if (t == 2) t = 1;
        }
  }
  R->covered.clear();
  for (size_t i = 0; i < R->Nc; ++i)
    if (R->ctype[i] == 2) R->covered.push_back((int32_t)i);
  return true;
}

void layout(lbm_refined* R) {
  const size_t pc = align256(R->Nc * R->Q * R->elem), pf = align256(R->Nf * R->Q * R->elem);
  const size_t ng = R->ghosts.size();
  size_t o = 0;
  R->off[0] = o; o += pc;                                    // coarse A
  R->off[1] = o; o += pc;                                    // coarse B
  R->off[2] = o; o += pf;                                    // fine A
  R->off[3] = o; o += pf;                                    // fine B
  R->off[4] = o; o += align256(R->Nc);                       // coarse types
  R->off[5] = o; o += align256(R->Nf);                       // fine types
  R->off[6] = o; o += align256(ng * 4);                      // ghosts
  R->off[7] = o; o += align256(R->covered.size() * 4);       // covered
  R->off[8] = o; o += align256(ng * R->Q * R->relem);        // G0
  R->off[9] = o; o += align256(ng * R->Q * R->relem);        // G1
  R->off[12] = o; o += align256(ng * 4);                     // stencil codes
  R->off[13] = o; o += align256(R->groups.size() * sizeof(GhostGroup));  // groups
  const size_t nbmax = std::max(R->nblocks_c, R->nblocks_f);
  R->off[10] = o; o += align256(nbmax * 5 * sizeof(double));  // partials
  R->off[11] = o; o += 256;                                  // result
  R->req = o;
}

void level_physics(Level& L, const lbm_config& c, double nu) {
  const double tau0 = 3.0 * nu + 0.5;
  L.mrt.tau0 = tau0;
  L.mrt.cs18 = 18.0 * c.cs_smag * c.cs_smag;
  L.omega = 1.0 / tau0;
  const double t1[5] = {1, 1, 1, 1, 1}, dh[5] = {1.19, 1.4, 1.2, 1.4, 1.98};
  for (int k = 0; k < 5; ++k)
    L.mrt.rates[k] = c.use_default_rates ? (c.mrt_basis == LBM_BASIS_TABLE1 ? t1[k] : dh[k])
                                         : c.rates[k];
}

GhostArgs ghost_args(const lbm_refined* R) {
  GhostArgs g;
  g.ghosts = (const int*)(R->base + R->off[6]);
  g.ng = (long long)R->ghosts.size();
  g.gcode = (const int*)(R->base + R->off[12]);
  g.groups = (const int*)(R->base + R->off[13]);
  g.ngroups = (long long)R->groups.size();
  g.cn[0] = R->cfg.nx;
  g.cn[1] = R->cfg.ny;
  g.cn[2] = R->cfg.nz;
  g.Nc = (long long)R->Nc;
  g.Nf = (long long)R->Nf;
  return g;
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

// Row sets of one level's box: the wall rows (global z on no non-periodic
// domain face, global y on no non-periodic y face other than a wall), and
// the other rows (listed as whole z planes first, then single y rows).
void plan_level(lbm_refined::Plan& p, const Level& L, dim3 block, size_t elem, int Q) {
  const uint32_t np = L.bc.nonper;
  const int Mx = L.M[0], My = L.M[1], Mz = L.M[2];
  Rows all{};
  all.ny_in = My;
  all.nz_in = Mz;
  p.all = all;
  p.block = block;
  p.grid_all = dim3((Mx + block.x - 1) / block.x, (My + block.y - 1) / block.y, Mz);
  Rows in = all, f{};
  // y faces that are walls stay in the wall rows
  const bool ywall = (L.bc.wall & 12u) == 12u;
  const bool ylo = !ywall && (np & 4u) && L.lo[1] == 0;
  const bool yhi = !ywall && (np & 8u) && L.lo[1] + My == L.n[1];
  const bool zlo = (np & 16u) && L.lo[2] == 0, zhi = (np & 32u) && L.lo[2] + Mz == L.n[2];
  if (ylo) f.yb[f.yb_n++] = 0;
  if (yhi) f.yb[f.yb_n++] = My - 1;
  if (zlo) f.zb[f.zb_n++] = 0;
  if (zhi) f.zb[f.zb_n++] = Mz - 1;
  in.y0 = ylo ? 1 : 0;
  in.ny_in = My - (ylo ? 1 : 0) - (yhi ? 1 : 0);
  in.z0 = zlo ? 1 : 0;
  in.nz_in = Mz - (zlo ? 1 : 0) - (zhi ? 1 : 0);
  f.zi0 = zlo ? 1 : 0;
  p.inner = in;
  p.face = f;
  const long long nrows = (long long)f.zb_n * My + (long long)f.yb_n * (Mz - f.zb_n);
  p.grid_inner = dim3((Mx + block.x - 1) / block.x,
                      in.ny_in > 0 ? (in.ny_in + block.y - 1) / block.y : 0,
                      in.nz_in > 0 ? in.nz_in : 0);
  const int bbx = Mx < 256 ? (Mx > 0 ? Mx : 1) : 256;
  p.block_face = dim3(bbx, 1, 1);
  p.grid_face = dim3((Mx + bbx - 1) / bbx, (unsigned)(nrows > 0 ? nrows : 0), 1);
  const bool x_walls = (L.bc.inlet & 3u) == 0 && ((np & 3u) == 0 || (L.bc.wall & 3u) == 3u);
  // the box and wall-row kernels address a population and its opposite from
  // the lower slab with 32-bit byte offsets; larger boxes take the general
  // kernel
  const double span = 1.0 + (Q == 27 ? max_opposite_distance<27>() : max_opposite_distance<19>());
  const bool o32 = span * (double)L.Nbox * (double)elem < 4294967296.0;
  if (!o32)
    p.mode = 2;
  else if (np == 0)
    p.mode = 0;
  else if (x_walls && nrows <= 65535)
    p.mode = 1;
  else
    p.mode = 2;
}

template <int KIND, typename S>
void level_step(const lbm_refined* R, hipStream_t stream, const Level& L,
                const lbm_refined::Plan& p, int mode,
                long long t) {
  if (L.Nbox == 0) return;
  if (p.mode == 0) {
    hipLaunchKernelGGL((ab_step_kernel<KIND, S, BC_NONE, ROWS_BOX>), p.grid_all, p.block, 0,
                       stream, L, p.all, mode, t);
  } else if (p.mode == 2) {
    hipLaunchKernelGGL((ab_step_kernel<KIND, S, BC_GENERAL, ROWS_BOX>), p.grid_all, p.block, 0,
                       stream, L, p.all, mode, t);
  } else {
    if (p.grid_inner.y > 0 && p.grid_inner.z > 0)
      hipLaunchKernelGGL((ab_step_kernel<KIND, S, BC_WALLS, ROWS_BOX>), p.grid_inner, p.block, 0,
                         stream, L, p.inner, mode, t);
    if (p.grid_face.y > 0)
      hipLaunchKernelGGL((ab_step_kernel<KIND, S, BC_GENERAL, ROWS_LIST>), p.grid_face,
                         p.block_face, 0, stream, L, p.face, mode, t);
  }
}

// Ghosts of the fine array ff := rescale(c0 G0 + c1 G), G = the
// interpolation of the coarse state fc (stored into G); G0 may be null
// (then c0 is unused).
template <int KIND, typename S>
void ghost_patch(const lbm_refined* R, hipStream_t stream, const GhostArgs& ga, const void* fc,
                 void* G, const void* G0, double c0, double c1, void* ff) {
  using Rt = typename Compute<S>::type;
  if (ga.ngroups == 0) return;
  hipLaunchKernelGGL((ghost_patch_kernel<KIND, S, Rt>), dim3((unsigned)ga.ngroups), dim3(256), 0,
                     stream, ga, (const S*)fc, (Rt*)G, (const Rt*)G0, c0, c1, R->r, (S*)ff);
}

// Ghosts of ff := rescale(G) from the stored interpolation G.
template <int KIND, typename S>
void ghost_rescale(const lbm_refined* R, hipStream_t stream, const GhostArgs& ga, const void* G,
                   void* ff) {
  using Rt = typename Compute<S>::type;
  if (ga.ngroups == 0) return;
  hipLaunchKernelGGL((ghost_rescale_kernel<KIND, S, Rt>), dim3((unsigned)ga.ngroups), dim3(256),
                     0, stream, ga, (const Rt*)G, 1.0, R->r, (S*)ff);
}

// One coarse step: the coarse update (Lc.a -> Lc.b), two fine substeps
// (Lf.a -> Lf.b -> Lf.a) and the interface. Ghost slots are written only by
// the interface kernels and fluid slots only by the fine updates, so with
// the side stream the work runs as two chains:
//   main: fine substep 1 ............ [wait interp] fine substep 2 + injection
//   side: coarse step -> G1, half-step ghosts of Lf.b -> [wait substep 1]
//         next-step ghosts of Lf.a
// (the half-step ghosts rescale(G0/2 + G1/2) are read only by substep 2; the
// next-step ghosts rescale(G1) go into Lf.a, which substep 1 reads, so they
// wait for it). The main stream joins the side stream at the end.
template <int KIND, typename S>
void one_coarse_step(lbm_refined* R, long long t) {
  const GhostArgs ga = ghost_args(R);
  const bool fine = R->Nf > 0;
  // The ghosts of the first fine substep come from the previous coarse
  // step; after a change of state they are rebuilt.
  if (fine && !R->g0_valid)
    ghost_patch<KIND, S>(R, R->stream, ga, R->Lc.a, R->g0, nullptr, 0.0, 1.0, R->Lf.a);
  const bool fork = fine && R->side != nullptr;
  hipStream_t side = fork ? R->side : R->stream;
  if (fork) {
    (void)hipEventRecord(R->fork_ev, R->stream);
    (void)hipStreamWaitEvent(R->side, R->fork_ev, 0);
  }
  level_step<KIND, S>(R, side, R->Lc, R->plan[0], 0, t);
  if (!fine) {
    std::swap(R->Lc.a, R->Lc.b);
    R->g0_valid = false;
    return;
  }
  ghost_patch<KIND, S>(R, side, ga, R->Lc.b, R->g1, R->g0, 0.5, 0.5, R->Lf.b);
  if (fork) (void)hipEventRecord(R->join_ev, R->side);
  level_step<KIND, S>(R, R->stream, R->Lf, R->plan[1], 1, 2 * t);
  // the last fine substep also injects into the covered nodes of the
  // coarse state at t + 1 (read by no ghost stencil)
  Level L2 = R->Lf;
  std::swap(L2.a, L2.b);
  if (!R->covered.empty()) {
    L2.cinj = R->Lc.b;
    L2.ctype = R->Lc.type;
    for (int d = 0; d < 3; ++d) L2.cn[d] = R->Lc.n[d];
    L2.Nc = (long long)R->Nc;
    L2.rinv = 1.0 / R->r;
  }
  if (fork) {
    (void)hipEventRecord(R->sub1_ev, R->stream);
    (void)hipStreamWaitEvent(R->stream, R->join_ev, 0);
    level_step<KIND, S>(R, R->stream, L2, R->plan[1], 1, 2 * t + 1);
    (void)hipStreamWaitEvent(R->side, R->sub1_ev, 0);
    ghost_rescale<KIND, S>(R, R->side, ga, R->g1, R->Lf.a);
    (void)hipEventRecord(R->join_ev, R->side);
    (void)hipStreamWaitEvent(R->stream, R->join_ev, 0);
  } else {
    ghost_rescale<KIND, S>(R, R->stream, ga, R->g1, R->Lf.a);
    level_step<KIND, S>(R, R->stream, L2, R->plan[1], 1, 2 * t + 1);
  }
  std::swap(R->Lc.a, R->Lc.b);
  std::swap(R->g0, R->g1);
  R->g0_valid = true;
}

bool valid_dtype(int d) { return d == LBM_DTYPE_F64 || d == LBM_DTYPE_F32; }

// A LatArgs view of one level's current state (for the uniform-lattice
// init/set/get/macroscopic kernels, parity 0, no boundary pulls).
LatArgs level_view(const lbm_refined* R, int level) {
  const Level& L = level == 0 ? R->Lc : R->Lf;
  LatArgs a;
  std::memset(&a, 0, sizeof(a));
  a.f = L.a;
  a.nx = L.M[0];
  a.ny = L.M[1];
  a.nz = L.M[2];
  a.N = L.Nbox;
  a.mrt = L.mrt;
  a.omega = L.omega;
  a.bc.ghost_n = 1;
  return a;
}

}  // namespace

extern "C" {

int lbm_refined_create(const lbm_config* cfg, int32_t block, const uint8_t* mask,
                       lbm_refined** out) {
  if (!cfg || !mask || !out) return LBM_EINVAL;
  const lbm_config& c = *cfg;
  if (c.model != LBM_D3Q19_MRT_LES && c.model != LBM_D3Q27_FCLB && c.model != LBM_D3Q27_CLB)
    return LBM_EINVAL;
  if (c.storage != LBM_F64 && c.storage != LBM_F32 && c.storage != LBM_F16) return LBM_EINVAL;
  if (block < 2 || c.nx < 4 || c.ny < 4 || c.nz < 4) return LBM_EINVAL;
  if (c.nx % block || c.ny % block || c.nz % block) return LBM_EINVAL;
  if ((double)c.nx * c.ny * c.nz * 8.0 >= 2147483648.0) return LBM_EINVAL;
  if (2 * c.nz > 65535) return LBM_EINVAL;
  if (!(c.nu > 0.0) || !std::isfinite(c.nu) || !(c.cs_smag >= 0.0)) return LBM_EINVAL;
  if (c.model == LBM_D3Q19_MRT_LES && c.mrt_basis != LBM_BASIS_TABLE1 &&
      c.mrt_basis != LBM_BASIS_DHUMIERES)
    return LBM_EINVAL;
  const double tc = 3.0 * c.nu + 0.5, tf = 6.0 * c.nu + 0.5;
  if (std::fabs(tc - 1.0) < 1e-6 || std::fabs(tf - 1.0) < 1e-6) return LBM_EINVAL;
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
  R->nb[0] = c.nx / block;
  R->nb[1] = c.ny / block;
  R->nb[2] = c.nz / block;
  R->mask.assign(mask, mask + (size_t)R->nb[0] * R->nb[1] * R->nb[2]);
  R->Nc = (size_t)c.nx * c.ny * c.nz;
  R->r = (tf - 1.0) / (2.0 * (tc - 1.0));
  R->stream = (hipStream_t)c.stream;
  // all faces periodic until boundaries are set; a region that touches a
  // periodic axis without spanning it needs boundaries before binding
  R->geometry_ok = build_geometry(R, 0u);
  if (!R->geometry_ok) build_geometry(R, 0x3Fu);
  std::memset(&R->Lc, 0, sizeof(Level));
  std::memset(&R->Lf, 0, sizeof(Level));
  level_physics(R->Lc, c, c.nu);
  level_physics(R->Lf, c, 2.0 * c.nu);
  R->Lc.n[0] = R->Lc.M[0] = c.nx;
  R->Lc.n[1] = R->Lc.M[1] = c.ny;
  R->Lc.n[2] = R->Lc.M[2] = c.nz;
  R->Lc.Nbox = (long long)R->Nc;
  R->Lf.n[0] = 2 * c.nx;
  R->Lf.n[1] = 2 * c.ny;
  R->Lf.n[2] = 2 * c.nz;
  for (int d = 0; d < 3; ++d) {
    R->Lf.lo[d] = R->lo[d];
    R->Lf.M[d] = R->M[d];
  }
  R->Lf.Nbox = (long long)R->Nf;
  shape_for(c.nx, c.ny, c.nz, R->grid_c, R->block_c, R->nblocks_c);
  shape_for(R->M[0], R->M[1], R->M[2], R->grid_f, R->block_f, R->nblocks_f);
  layout(R);
  plan_level(R->plan[0], R->Lc, R->block_c, R->elem, R->Q);
  plan_level(R->plan[1], R->Lf, R->block_f, R->elem, R->Q);
  *out = R;
  return LBM_OK;
}

int lbm_refined_geometry(const lbm_refined* R, int32_t lo[3], int32_t dims[3],
                         int64_t counts[4]) {
  if (!R || !lo || !dims || !counts) return LBM_EINVAL;
  for (int d = 0; d < 3; ++d) {
    lo[d] = R->lo[d];
    dims[d] = R->M[d];
  }
  int64_t nf = 0, nb = 0;
  for (uint8_t t : R->ftype) nf += t == 1;
  for (uint8_t t : R->ctype) nb += t == 1;
  counts[0] = nf;
  counts[1] = (int64_t)R->ghosts.size();
  counts[2] = (int64_t)R->covered.size();
  counts[3] = nb;
  return LBM_OK;
}

int lbm_refined_required_bytes(const lbm_refined* R, size_t* bytes) {
  if (!R || !bytes) return LBM_EINVAL;
  *bytes = R->req;
  return LBM_OK;
}

static int upload_geometry(lbm_refined* R) {
  hipError_t e;
  e = hipMemcpyAsync(R->base + R->off[4], R->ctype.data(), R->Nc, hipMemcpyHostToDevice, R->stream);
  if (e != hipSuccess) return hip_fail(e);
  if (R->Nf) {
    e = hipMemcpyAsync(R->base + R->off[5], R->ftype.data(), R->Nf, hipMemcpyHostToDevice,
                       R->stream);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (!R->ghosts.empty()) {
    e = hipMemcpyAsync(R->base + R->off[6], R->ghosts.data(), R->ghosts.size() * 4,
                       hipMemcpyHostToDevice, R->stream);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (!R->covered.empty()) {
    e = hipMemcpyAsync(R->base + R->off[7], R->covered.data(), R->covered.size() * 4,
                       hipMemcpyHostToDevice, R->stream);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (!R->ghosts.empty()) {
    e = hipMemcpyAsync(R->base + R->off[12], R->gcode.data(), R->gcode.size() * 4,
                       hipMemcpyHostToDevice, R->stream);
    if (e != hipSuccess) return hip_fail(e);
    e = hipMemcpyAsync(R->base + R->off[13], R->groups.data(),
                       R->groups.size() * sizeof(GhostGroup), hipMemcpyHostToDevice, R->stream);
    if (e != hipSuccess) return hip_fail(e);
  }
  e = hipStreamSynchronize(R->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e);
}

int lbm_refined_bind_memory(lbm_refined* R, void* dev, size_t bytes) {
  if (!R || !dev || ((uintptr_t)dev & 255) != 0) return LBM_EINVAL;
  if (!R->geometry_ok) return LBM_ESTATE;
  if (bytes < R->req) return LBM_ENOMEM;
  R->base = (char*)dev;
  R->Lc.a = R->base + R->off[0];
  R->Lc.b = R->base + R->off[1];
  R->Lf.a = R->base + R->off[2];
  R->Lf.b = R->base + R->off[3];
  R->Lc.type = (const uint8_t*)(R->base + R->off[4]);
  R->Lf.type = (const uint8_t*)(R->base + R->off[5]);
  R->g0 = R->base + R->off[8];
  R->g1 = R->base + R->off[9];
  R->partial = (double*)(R->base + R->off[10]);
  R->result = (double*)(R->base + R->off[11]);
  R->t = 0;
  R->g0_valid = false;
  return upload_geometry(R);
}

int lbm_refined_set_boundaries(lbm_refined* R, const lbm_boundaries* bc,
                               const void* fine_inlet_u, const uint8_t* fine_inlet_mask) {
  if (!R || !bc) return LBM_EINVAL;
  if (R->base) return LBM_ESTATE;  // the layout depends on the boundaries
  const int n3[3] = {R->cfg.nx, R->cfg.ny, R->cfg.nz};
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
  if (n_inlet > 1 || n_out > 1) return LBM_EINVAL;
  BcArgs bf = b;
  if (n_inlet) {
    if (!bc->inlet_u || !fine_inlet_u || (bc->inlet_dtype != LBM_DTYPE_F64 &&
                                          bc->inlet_dtype != LBM_DTYPE_F32))
      return LBM_EINVAL;
    const int d = b.inlet_axis;
    b.inlet_u = bc->inlet_u;
    b.inlet_f64 = bc->inlet_dtype == LBM_DTYPE_F64;
    b.inlet_mask = bc->inlet_mask;
    b.inlet_amp = bc->inlet_amp;
    b.seed = bc->seed;
    b.inlet_na = n3[d == 0 ? 1 : 0];
    b.inlet_nb = n3[d == 2 ? 1 : 2];
    bf.inlet_u = fine_inlet_u;
    bf.inlet_f64 = b.inlet_f64;
    bf.inlet_mask = fine_inlet_mask;
    bf.inlet_amp = bc->inlet_amp;
    bf.seed = bc->seed + 1;  // the fine level draws its own perturbations
    bf.inlet_na = 2 * b.inlet_na;
    bf.inlet_nb = 2 * b.inlet_nb;
    if (bf.inlet_na >= 16384 || bf.inlet_nb >= 16384) return LBM_EINVAL;
  }
  // the geometry depends on which axes are periodic
  if (!build_geometry(R, b.nonper)) {
    R->geometry_ok = build_geometry(R, R->Lc.bc.nonper);
    return LBM_EINVAL;
  }
  R->geometry_ok = true;
  for (int d = 0; d < 3; ++d) {
    R->Lf.lo[d] = R->lo[d];
    R->Lf.M[d] = R->M[d];
  }
  R->Lf.Nbox = (long long)R->Nf;
  shape_for(R->M[0], R->M[1], R->M[2], R->grid_f, R->block_f, R->nblocks_f);
  layout(R);
  fill_wall_terms(b, R->Q);
  fill_wall_terms(bf, R->Q);
  R->Lc.bc = b;
  R->Lf.bc = bf;
  R->has_bc = b.nonper != 0;
  R->g0_valid = false;
  plan_level(R->plan[0], R->Lc, R->block_c, R->elem, R->Q);
  plan_level(R->plan[1], R->Lf, R->block_f, R->elem, R->Q);
  return LBM_OK;
}

int lbm_refined_init_equilibrium(lbm_refined* R, int level, const void* drho, const void* u,
                                 int dtype, int64_t t0) {
  if (!R || (level != 0 && level != 1) || !drho || !u || !valid_dtype(dtype)) return LBM_EINVAL;
  if (!R->base) return LBM_EUNBOUND;
  if (level == 1 && R->Nf == 0) return LBM_OK;
  const LatArgs a = level_view(R, level);
  const dim3 grid = level == 0 ? R->grid_c : R->grid_f, block = level == 0 ? R->block_c : R->block_f;
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
  R->t = t0;
  R->g0_valid = false;
  return check_launch();
}

int lbm_refined_set_populations(lbm_refined* R, int level, const void* f, int dtype, int64_t t0) {
  if (!R || (level != 0 && level != 1) || !f || !valid_dtype(dtype)) return LBM_EINVAL;
  if (!R->base) return LBM_EUNBOUND;
  if (level == 1 && R->Nf == 0) return LBM_OK;
  const LatArgs a = level_view(R, level);
  const dim3 grid = level == 0 ? R->grid_c : R->grid_f, block = level == 0 ? R->block_c : R->block_f;
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
  R->t = t0;
  R->g0_valid = false;
  return check_launch();
}

int lbm_refined_get_populations(lbm_refined* R, int level, void* f, int dtype) {
  if (!R || (level != 0 && level != 1) || !f || !valid_dtype(dtype)) return LBM_EINVAL;
  if (!R->base) return LBM_EUNBOUND;
  if (level == 1 && R->Nf == 0) return LBM_OK;
  const LatArgs a = level_view(R, level);
  const dim3 grid = level == 0 ? R->grid_c : R->grid_f, block = level == 0 ? R->block_c : R->block_f;
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
  if (!R || (level != 0 && level != 1) || !valid_dtype(dtype)) return LBM_EINVAL;
  if (rho_mode != LBM_RHO_FULL && rho_mode != LBM_RHO_DEVIATION) return LBM_EINVAL;
  if (!R->base) return LBM_EUNBOUND;
  if ((!rho && !u) || (level == 1 && R->Nf == 0)) return LBM_OK;
  const LatArgs a = level_view(R, level);
  const dim3 grid = level == 0 ? R->grid_c : R->grid_f, block = level == 0 ? R->block_c : R->block_f;
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
  if (!R->side_tried) {
    // without the side stream the coarse step simply runs in order
    R->side_tried = true;
    if (hipStreamCreateWithFlags(&R->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&R->fork_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&R->join_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&R->sub1_ev, hipEventDisableTiming) != hipSuccess) {
      if (R->side) (void)hipStreamDestroy(R->side);
      if (R->fork_ev) (void)hipEventDestroy(R->fork_ev);
      if (R->join_ev) (void)hipEventDestroy(R->join_ev);
    if (R->sub1_ev) (void)hipEventDestroy(R->sub1_ev);
      R->side = nullptr;
      R->fork_ev = R->join_ev = R->sub1_ev = nullptr;
      (void)hipGetLastError();
    }
  }
  for (int64_t k = 0; k < n; ++k) {
    with_kind_s(R, [&](auto kc, auto st_) {
      one_coarse_step<decltype(kc)::value, typename decltype(st_)::type>(R, (long long)R->t);
    });
    R->t += 1;
  }
  return check_launch();
}

int lbm_refined_reduce(lbm_refined* R, double out[5]) {
  if (!R || !out) return LBM_EINVAL;
  if (!R->base) return LBM_EUNBOUND;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int level = 0; level < 2; ++level) {
    const Level& L = level == 0 ? R->Lc : R->Lf;
    if (L.Nbox == 0) continue;
    const dim3 grid = level == 0 ? R->grid_c : R->grid_f, block = level == 0 ? R->block_c : R->block_f;
    const size_t nb = level == 0 ? R->nblocks_c : R->nblocks_f;
    with_kind_s(R, [&](auto kc, auto st_) {
      constexpr int KIND = decltype(kc)::value;
      using S = typename decltype(st_)::type;
      hipLaunchKernelGGL((masked_reduce_kernel<KIND, S>), grid, block, 0, R->stream, L,
                         level == 0 ? 0 : 1, level == 0 ? 1.0 : 0.125, R->partial);
    });
    int rc = check_launch();
    if (rc) return rc;
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, R->stream, R->partial, nb,
                       R->result);
    rc = check_launch();
    if (rc) return rc;
    double part[5];
    hipError_t e =
        hipMemcpyAsync(part, R->result, 5 * sizeof(double), hipMemcpyDeviceToHost, R->stream);
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
  if (R) {
    if (R->side) {
      (void)hipStreamSynchronize(R->side);
      (void)hipStreamDestroy(R->side);
    }
    if (R->fork_ev) (void)hipEventDestroy(R->fork_ev);
    if (R->join_ev) (void)hipEventDestroy(R->join_ev);
  }
  delete R;
  return LBM_OK;
}

}  // extern "C"
