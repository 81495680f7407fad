// Host runtime of the C ABI declared in include/lbm.h: validation, memory
// layout inside the caller's block, launch configuration and dispatch over
// model x storage x step parity x boundary handling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>

#include "../../include/lbm.h"
#include "adjoint.h"
#include "jetprofile.h"
#include "kernels.h"
#include "trace.h"

using namespace lbm;

struct lbm_lattice {
  lbm_config cfg;
  int kind;  // 0 MRT Table 1, 1 MRT d'Humieres, 2 FCLB
  int Q;
  size_t N;
  size_t elem;  // bytes per stored value
  hipStream_t stream;
  // bound memory
  char* base = nullptr;
  size_t bytes = 0;
  size_t off_ghost = 0, off_partial = 0, off_result = 0, req = 0;
  size_t ghost_n_max = 0;
  size_t nblocks = 0;
  // state
  int64_t t = 0;
  int parity = 0;
  bool has_bc = false;
  bool solids = false;  // interior solid nodes set (general kernel only)
  // interpolated bounce-back links (caller-owned device buffers)
  const int32_t* link_nodes = nullptr;
  const float* link_q = nullptr;
  long long nlinks = 0;
  LatArgs args;
  dim3 grid, block;
  // odd steps with boundaries split into wall rows (x and y faces walls or
  // periodic, see pull_walls) and the rows on the other non-periodic faces
  bool split_odd = false;
  Rows rows_all, rows_inner, rows_bnd;
  dim3 grid_inner, grid_bnd, block_bnd;
  // health check inside lbm_step (lbm_set_check)
  int64_t check_every = 0;
  double check_tol = -1.0, check_m0 = 0.0;
  // per-launch timing (LBM_TRACE=1 at creation)
  std::unique_ptr<Tracer> tracer = std::make_unique<Tracer>();
};

namespace {

thread_local std::string g_hip_msg;

int hip_fail(hipError_t e) {
  g_hip_msg = std::string("HIP error: ") + hipGetErrorString(e);
  return LBM_EHIP;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

void launch_shape(lbm_lattice* L) {
  const int nx = L->cfg.nx, ny = L->cfg.ny, nz = L->cfg.nz;
  int bx = nx < 256 ? nx : 256;
  int by = 256 / bx;
  if (by > ny) by = ny;
  if (by < 1) by = 1;
  L->block = dim3(bx, by, 1);
  L->grid = dim3((nx + bx - 1) / bx, (ny + by - 1) / by, nz);
  L->nblocks = (size_t)L->grid.x * L->grid.y * L->grid.z;
}

template <int KIND, typename S, bool ODD, int BCM, int ROWS, bool EXT = false>
void launch_step(const lbm_lattice* L, dim3 grid, dim3 block, const Rows& r, long long t,
                 void* rec) {
  TraceScope ts(L->tracer.get(), L->stream, LBM_TRACE_LABEL("step_kernel"));
  hipLaunchKernelGGL((step_kernel<KIND, S, ODD, BCM, ROWS, EXT>), grid, block, 0, L->stream,
                     L->args, r, t, (typename Compute<S>::type*)rec);
}

template <int KIND, typename S, bool EXT>
void step_model_ext(const lbm_lattice* L, bool odd, long long t, void* rec) {
  if (!L->has_bc) {
    if (odd)
      launch_step<KIND, S, true, BC_NONE, ROWS_BOX>(L, L->grid, L->block, L->rows_all, t, rec);
    else
      launch_step<KIND, S, false, BC_NONE, ROWS_BOX>(L, L->grid, L->block, L->rows_all, t, rec);
  } else if (!odd) {
    launch_step<KIND, S, false, BC_GENERAL, ROWS_BOX, EXT>(L, L->grid, L->block, L->rows_all, t,
                                                           rec);
  } else if (!L->split_odd) {
    launch_step<KIND, S, true, BC_GENERAL, ROWS_BOX, EXT>(L, L->grid, L->block, L->rows_all, t,
                                                          rec);
  } else {
    // wall rows: the solid variant only with solids (free slip never
    // reaches them)
    if (L->grid_inner.y > 0 && L->grid_inner.z > 0) {
      if (L->solids)
        launch_step<KIND, S, true, BC_WALLS, ROWS_BOX, true>(L, L->grid_inner, L->block,
                                                             L->rows_inner, t, rec);
      else
        launch_step<KIND, S, true, BC_WALLS, ROWS_BOX>(L, L->grid_inner, L->block,
                                                       L->rows_inner, t, rec);
    }
    if (L->grid_bnd.y > 0)
      launch_step<KIND, S, true, BC_GENERAL, ROWS_LIST, EXT>(L, L->grid_bnd, L->block_bnd,
                                                             L->rows_bnd, t, rec);
  }
}

// Lattices without interior solids, FREESLIP or PRESSURE faces run the
// general kernel compiled without their rules. The even step touches only
// each node's own slots, which no other node reads: solid nodes may run it
// (their populations are never read) and free slip has no even-step rule,
// so there the rules are compiled in only for PRESSURE faces.
template <int KIND, typename S>
void step_model(const lbm_lattice* L, bool odd, long long t, void* rec) {
  const bool ext = odd ? (L->solids || L->args.bc.freeslip || L->args.bc.pressure)
                       : L->args.bc.pressure != 0;
  if constexpr (std::is_same_v<S, _Float16>) {
    // FP16 even steps: two nodes per lane (the pair kernel's rows)
    if (!odd && !ext && rec == nullptr && L->cfg.nx % 2 == 0) {
      const int hx = L->cfg.nx / 2;
      const int bx = hx < 256 ? hx : 256;
      int by = 256 / bx;
      if (by > L->cfg.ny) by = L->cfg.ny;
      const dim3 block(bx, by, 1);
      const dim3 grid((hx + bx - 1) / bx, (L->cfg.ny + by - 1) / by, L->cfg.nz);
      TraceScope ts(L->tracer.get(), L->stream,
                    L->has_bc ? "step_even_pair_kernel (FP16, boundaries)"
                              : "step_even_pair_kernel (FP16)");
      if (L->has_bc)
        hipLaunchKernelGGL((step_even_pair_kernel<KIND, true>), grid, block, 0, L->stream,
                           L->args);
      else
        hipLaunchKernelGGL((step_even_pair_kernel<KIND, false>), grid, block, 0, L->stream,
                           L->args);
      return;
    }
  }
  if (ext)
    step_model_ext<KIND, S, true>(L, odd, t, rec);
  else
    step_model_ext<KIND, S, false>(L, odd, t, rec);
}

template <typename S>
void step_dispatch_s(lbm_lattice* L, bool odd, long long t) {
  switch (L->kind) {
    case 0: step_model<0, S>(L, odd, t, nullptr); break;
    case 1: step_model<1, S>(L, odd, t, nullptr); break;
    case 3: step_model<3, S>(L, odd, t, nullptr); break;
    default: step_model<2, S>(L, odd, t, nullptr); break;
  }
}

void step_dispatch(lbm_lattice* L, bool odd, long long t) {
  switch (L->cfg.storage) {
    case LBM_F64: step_dispatch_s<double>(L, odd, t); break;
    case LBM_F32: step_dispatch_s<float>(L, odd, t); break;
    default: step_dispatch_s<_Float16>(L, odd, t); break;
  }
}

// Interpolated bounce-back over the link list after a step.
template <typename S>
void links_dispatch_s(const lbm_lattice* L, bool after_odd) {
  const dim3 grid((unsigned)((L->nlinks + 7) / 8)), block(256);  // 32 lanes per node
  TraceScope ts(L->tracer.get(), L->stream, "link_kernel (interpolated bounce-back)");
  auto go = [&](auto q_c, auto odd_c) {
    constexpr int Q = decltype(q_c)::value;
    constexpr bool ODD = decltype(odd_c)::value;
    hipLaunchKernelGGL((link_kernel<Q, S, ODD>), grid, block, 0, L->stream, L->args,
                       L->link_nodes, L->link_q, L->nlinks);
  };
  if (L->Q == 27) {
    if (after_odd) go(std::integral_constant<int, 27>{}, std::true_type{});
    else go(std::integral_constant<int, 27>{}, std::false_type{});
  } else {
    if (after_odd) go(std::integral_constant<int, 19>{}, std::true_type{});
    else go(std::integral_constant<int, 19>{}, std::false_type{});
  }
}

void links_dispatch(const lbm_lattice* L, bool after_odd) {
  switch (L->cfg.storage) {
    case LBM_F64: links_dispatch_s<double>(L, after_odd); break;
    case LBM_F32: links_dispatch_s<float>(L, after_odd); break;
    default: links_dispatch_s<_Float16>(L, after_odd); break;
  }
}

// One FCLB or MRT-LES step that also records the pre-collision state (FP64
// and FP32 storage: the adjoint's recomputation).
template <int KIND>
void step_record_kind(lbm_lattice* L, bool odd, long long t, void* rec) {
  if (L->cfg.storage == LBM_F64)
    step_model<KIND, double>(L, odd, t, rec);
  else
    step_model<KIND, float>(L, odd, t, rec);
}

void step_record_dispatch(lbm_lattice* L, bool odd, long long t, void* rec) {
  switch (L->kind) {
    case 0: step_record_kind<0>(L, odd, t, rec); break;
    case 1: step_record_kind<1>(L, odd, t, rec); break;
    default: step_record_kind<2>(L, odd, t, rec); break;
  }
}

// Slabs spanned by a population and its opposite (see max_opposite_distance).
double slab_span(int Q) {
  return 1.0 + (Q == 27 ? max_opposite_distance<27>() : max_opposite_distance<19>());
}

// Row sets of the split odd step for the current boundary description.
void plan_rows(lbm_lattice* L) {
  const int nx = L->cfg.nx, ny = L->cfg.ny, nz = L->cfg.nz;
  const uint32_t np = L->args.bc.nonper;
  Rows all{};
  all.y0 = 0;
  all.ny_in = ny;
  all.z0 = 0;
  all.nz_in = nz;
  L->rows_all = all;
  const bool znp = (np & 48u) != 0;
  // y faces that are walls stay in the wall rows; other non-periodic y
  // faces go to the row list
  const bool ynp = (np & 12u) != 0 && (L->args.bc.wall & 12u) != 12u;
  Rows in = all;
  if (ynp) {
    in.y0 = 1;
    in.ny_in = ny - 2;
  }
  if (znp) {
    in.z0 = 1;
    in.nz_in = nz - 2;
  }
  L->rows_inner = in;
  Rows b{};
  if (znp) {
    b.zb_n = 2;
    b.zb[0] = 0;
    b.zb[1] = nz - 1;
  }
  if (ynp) {
    b.yb_n = 2;
    b.yb[0] = 0;
    b.yb[1] = ny - 1;
  }
  b.zi0 = znp ? 1 : 0;
  const long long nrows = (long long)b.zb_n * ny + (long long)b.yb_n * (nz - b.zb_n);
  L->rows_bnd = b;
  const uint32_t xbits = np & 3u;
  const bool x_ok = (L->args.bc.inlet & 3u) == 0 && (xbits == 0 || (L->args.bc.wall & 3u) == 3u);
  // the wall rows address a population and its opposite from the lower
  // slab with 32-bit offsets: the span of slabs must stay below 4 GiB
  const bool span_ok = slab_span(L->Q) * (double)L->N * (double)L->elem < 4294967296.0;
  L->split_odd = L->has_bc && x_ok && nrows <= 65535 && span_ok;
  const int bx = L->block.x, by = L->block.y;
  L->grid_inner = dim3((nx + bx - 1) / bx, in.ny_in > 0 ? (in.ny_in + by - 1) / by : 0,
                       in.nz_in > 0 ? in.nz_in : 0);
  const int bbx = nx < 256 ? nx : 256;
  L->block_bnd = dim3(bbx, 1, 1);
  L->grid_bnd = dim3((nx + bbx - 1) / bbx, (unsigned)(nrows > 0 ? nrows : 0), 1);
}

// Runs fn<KIND, S, BC>() for the lattice's configuration.
template <typename Fn>
void with_config(const lbm_lattice* L, Fn&& fn) {
  auto by_s = [&](auto kind_c) {
    constexpr int KIND = decltype(kind_c)::value;
    auto by_bc = [&](auto s_tag) {
      using S = typename decltype(s_tag)::type;
      if (L->has_bc)
        fn(std::integral_constant<int, KIND>{}, s_tag, std::true_type{});
      else
        fn(std::integral_constant<int, KIND>{}, s_tag, std::false_type{});
    };
    switch (L->cfg.storage) {
      case LBM_F64: by_bc(std::type_identity<double>{}); break;
      case LBM_F32: by_bc(std::type_identity<float>{}); break;
      default: by_bc(std::type_identity<_Float16>{}); break;
    }
  };
  switch (L->kind) {
    case 0: by_s(std::integral_constant<int, 0>{}); break;
    case 1: by_s(std::integral_constant<int, 1>{}); break;
    case 3: by_s(std::integral_constant<int, 3>{}); break;
    default: by_s(std::integral_constant<int, 2>{}); break;
  }
}

int check_launch() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? LBM_OK : hip_fail(e);
}

bool valid_dtype(int d) { return d == LBM_DTYPE_F64 || d == LBM_DTYPE_F32; }

void default_bc(BcArgs& b) {
  std::memset(&b, 0, sizeof(b));
  b.inlet_axis = 2;
  b.ghost_n = 1;
}

// FP64 sums of the current state (lbm_reduce's definition), blocking.
int reduce_now(lbm_lattice* L, double out[5]) {
  double* partial = (double*)(L->base + L->off_partial);
  double* result = (double*)(L->base + L->off_result);
  {
    TraceScope ts(L->tracer.get(), L->stream, "reduce_partial_kernel + reduce_final_kernel");
    with_config(L, [&](auto kind_c, auto s_tag, auto bc_c) {
      constexpr int KIND = decltype(kind_c)::value;
      using S = typename decltype(s_tag)::type;
      constexpr bool BC = decltype(bc_c)::value;
      hipLaunchKernelGGL((reduce_partial_kernel<KIND, S, BC>), L->grid, L->block, 0, L->stream,
                         L->args, L->parity, (long long)L->t, partial);
    });
    hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, L->stream, partial,
                       L->nblocks, result);
  }
  const int rc = check_launch();
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(out, result, 5 * sizeof(double), hipMemcpyDeviceToHost,
                                L->stream);
  if (e != hipSuccess) return hip_fail(e);
  e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e);
  for (int k = 0; k < 5; ++k)
    if (!std::isfinite(out[k])) return LBM_ENONFINITE;
  return LBM_OK;
}

// The check of lbm_set_check after a step.
int run_check(lbm_lattice* L) {
  double out[5];
  const int rc = reduce_now(L, out);
  if (rc) return rc;
  if (L->check_tol >= 0.0 && std::fabs(out[0] - L->check_m0) > L->check_tol)
    return LBM_EMASS;
  return LBM_OK;
}

}  // namespace

// Library-owned partial sums for lbm_reduce_static: one row of five per block
// of an x-y plane of the reduce launch, then the five results. Each device
// holds its own copy for the life of the process; every call on a device
// shares it.
constexpr size_t kStaticPartials = 16384;
static __device__ __align__(256) double scratch[kStaticPartials * 5 + 8];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {nullptr};

// The device address of the scratch array on the device that runs the
// lattice's stream (the current device for the null stream), looked up once
// per device with that device current (the array's name in host code is not
// a device address).
int static_scratch(hipStream_t stream, double** out) {
  int cur = 0, dev = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e);
  dev = cur;
  if (stream) {
    e = hipStreamGetDevice(stream, &dev);
    if (e != hipSuccess) return hip_fail(e);
  }
  if (dev < 0 || dev >= kMaxDevices) return LBM_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess) return hip_fail(e);
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (dev != cur) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e);
    g_scratch_ptr[dev] = (double*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_strerror(int status) {
  switch (status) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument or configuration";
    case LBM_ENOMEM: return "bound device block is smaller than required";
    case LBM_EUNBOUND: return "no device memory bound";
    case LBM_EHIP: return g_hip_msg.empty() ? "HIP error" : g_hip_msg.c_str();
    case LBM_ENONFINITE: return "non-finite global sum";
    case LBM_ESTATE: return "call not valid in the current lattice state";
    case LBM_EMASS: return "mass deviation drifted beyond the check tolerance";
    default: return "unknown status";
  }
}

int lbm_create_lattice(const lbm_config* cfg, lbm_lattice** out) {
  if (!cfg || !out) return LBM_EINVAL;
  const lbm_config& c = *cfg;
  if (c.model != LBM_D3Q19_MRT_LES && c.model != LBM_D3Q27_FCLB && c.model != LBM_D3Q27_CLB)
    return LBM_EINVAL;
  if (c.storage != LBM_F64 && c.storage != LBM_F32 && c.storage != LBM_F16) return LBM_EINVAL;
  if (c.nx < 1 || c.ny < 1 || c.nz < 1) return LBM_EINVAL;
  const double nnodes = (double)c.nx * c.ny * c.nz;
  if (nnodes >= 2147483648.0) return LBM_EINVAL;
  if (c.nz > 65535 || c.ny > 65535 * 256) return LBM_EINVAL;  // launch grid limits
  // one population slab (all nodes) below 4 GiB: the kernels address it with
  // 32-bit byte offsets
  const size_t elem_bytes = c.storage == LBM_F64 ? 8 : (c.storage == LBM_F32 ? 4 : 2);
  if (nnodes * (double)elem_bytes >= 4294967296.0) return LBM_EINVAL;
  if (!(c.nu > 0.0) || !std::isfinite(c.nu)) return LBM_EINVAL;
  if (!(c.cs_smag >= 0.0) || !std::isfinite(c.cs_smag)) return LBM_EINVAL;
  if (c.model == LBM_D3Q19_MRT_LES &&
      c.mrt_basis != LBM_BASIS_TABLE1 && c.mrt_basis != LBM_BASIS_DHUMIERES)
    return LBM_EINVAL;
  if (c.model == LBM_D3Q19_MRT_LES && !c.use_default_rates) {
    const int nr = c.mrt_basis == LBM_BASIS_TABLE1 ? 4 : 5;
    for (int k = 0; k < nr; ++k)
      if (!(c.rates[k] > 0.0 && c.rates[k] < 2.0)) return LBM_EINVAL;
  }
  lbm_lattice* L = new (std::nothrow) lbm_lattice();
  if (!L) return LBM_EINVAL;
  L->cfg = c;
  L->kind = c.model == LBM_D3Q27_FCLB ? 2
            : c.model == LBM_D3Q27_CLB  ? 3
                                        : (c.mrt_basis == LBM_BASIS_TABLE1 ? 0 : 1);
  L->Q = c.model == LBM_D3Q19_MRT_LES ? 19 : 27;
  L->N = (size_t)c.nx * c.ny * c.nz;
  L->elem = c.storage == LBM_F64 ? 8 : (c.storage == LBM_F32 ? 4 : 2);
  L->stream = (hipStream_t)c.stream;
  launch_shape(L);
  // memory layout: populations | outflow ghost plane (one z plane) |
  // reduction partials | result
  const size_t face = (size_t)c.nx * c.ny;
  L->ghost_n_max = face;
  L->off_ghost = align256(L->N * L->Q * L->elem);
  L->off_partial = L->off_ghost + align256(face * L->Q * L->elem);
  L->off_result = L->off_partial + align256(L->nblocks * 5 * sizeof(double));
  L->req = L->off_result + 256;
  // arguments
  LatArgs& a = L->args;
  std::memset(&a, 0, sizeof(a));
  a.nx = c.nx;
  a.ny = c.ny;
  a.nz = c.nz;
  a.N = (long long)L->N;
  const double tau0 = 3.0 * c.nu + 0.5;
  a.mrt.tau0 = tau0;
  a.mrt.cs18 = 18.0 * c.cs_smag * c.cs_smag;
  a.omega = 1.0 / tau0;
  if (c.model == LBM_D3Q19_MRT_LES) {
    if (c.use_default_rates) {
      const double t1[5] = {1.0, 1.0, 1.0, 1.0, 1.0};
      const double dh[5] = {1.19, 1.4, 1.2, 1.4, 1.98};
      for (int k = 0; k < 5; ++k)
        a.mrt.rates[k] = c.mrt_basis == LBM_BASIS_TABLE1 ? t1[k] : dh[k];
    } else {
      for (int k = 0; k < 5; ++k) a.mrt.rates[k] = c.rates[k];
    }
  }
  default_bc(a.bc);
  plan_rows(L);
  *out = L;
  return LBM_OK;
}

int lbm_required_bytes(const lbm_lattice* L, size_t* bytes) {
  if (!L || !bytes) return LBM_EINVAL;
  *bytes = L->req;
  return LBM_OK;
}

int lbm_bind_memory(lbm_lattice* L, void* dev, size_t bytes) {
  if (!L || !dev) return LBM_EINVAL;
  if (((uintptr_t)dev & 255) != 0) return LBM_EINVAL;
  if (bytes < L->req) return LBM_ENOMEM;
  L->base = (char*)dev;
  L->bytes = bytes;
  L->args.f = L->base;
  L->args.ghost = L->base + L->off_ghost;
  L->t = 0;
  L->parity = 0;
  return LBM_OK;
}

int lbm_set_stream(lbm_lattice* L, void* stream) {
  if (!L) return LBM_EINVAL;
  L->stream = (hipStream_t)stream;
  return LBM_OK;
}

int lbm_set_boundaries(lbm_lattice* L, const lbm_boundaries* bc) {
  if (!L || !bc) return LBM_EINVAL;
  if (L->parity != 0) return LBM_ESTATE;
  const int n3[3] = {L->cfg.nx, L->cfg.ny, L->cfg.nz};
  BcArgs b;
  default_bc(b);
  int n_inlet = 0, n_out = 0;
  for (int f = 0; f < 6; ++f) {
    const int ty = bc->face_type[f];
    if (ty < LBM_PERIODIC || ty > LBM_PRESSURE) return LBM_EINVAL;
    if (ty != LBM_PERIODIC) {
      b.nonper |= 1u << f;
      if (n3[f / 2] < 2) return LBM_EINVAL;
    }
    for (int k = 0; k < 3; ++k) {
      if (!std::isfinite(bc->face_u[f][k])) return LBM_EINVAL;
      b.face_u[f][k] = bc->face_u[f][k];
    }
    if (ty == LBM_WALL) b.wall |= 1u << f;
    if (ty == LBM_FREESLIP) b.freeslip |= 1u << f;
    if (ty == LBM_PRESSURE) {
      if (!std::isfinite(bc->face_drho[f]) || !(bc->face_drho[f] > -1.0)) return LBM_EINVAL;
      b.pressure |= 1u << f;
      b.face_drho[f] = bc->face_drho[f];
    }
    if (ty == LBM_INLET) {
      b.inlet |= 1u << f;
      b.inlet_axis = f / 2;
      ++n_inlet;
    }
    if (ty == LBM_OUTFLOW) {
      if (f / 2 != 2) return LBM_EINVAL;  // outflow faces are z faces
      b.outflow |= 1u << f;
      ++n_out;
    }
  }
  for (int d = 0; d < 3; ++d) {
    const bool lo = (b.nonper >> (2 * d)) & 1u, hi = (b.nonper >> (2 * d + 1)) & 1u;
    if (lo != hi) return LBM_EINVAL;  // faces of one axis: both periodic or neither
  }
  if (n_inlet > 1 || n_out > 1) return LBM_EINVAL;
  if (n_inlet) {
    if (!bc->inlet_u || !valid_dtype(bc->inlet_dtype)) return LBM_EINVAL;
    if (!std::isfinite(bc->inlet_amp)) return LBM_EINVAL;
    b.inlet_u = bc->inlet_u;
    b.inlet_f64 = bc->inlet_dtype == LBM_DTYPE_F64;
    b.inlet_mask = bc->inlet_mask;
    b.inlet_amp = bc->inlet_amp;
    b.seed = bc->seed;
    const int d = b.inlet_axis;
    b.inlet_na = n3[d == 0 ? 1 : 0];
    b.inlet_nb = n3[d == 2 ? 1 : 2];
    if (b.inlet_na >= 16384 || b.inlet_nb >= 16384) return LBM_EINVAL;
  }
  if (n_out) b.ghost_n = (long long)n3[0] * n3[1];
  fill_wall_terms(b, L->Q);
  L->args.bc = b;
  L->args.solid_nb = nullptr;  // new boundaries clear the solids and links
  L->solids = false;
  L->link_nodes = nullptr;
  L->link_q = nullptr;
  L->nlinks = 0;
  L->has_bc = b.nonper != 0;
  plan_rows(L);
  return LBM_OK;
}

int lbm_init_equilibrium(lbm_lattice* L, const void* drho, const void* u, int dtype,
                         int64_t t0) {
  if (!L || !drho || !u || !valid_dtype(dtype)) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  with_config(L, [&](auto kind_c, auto s_tag, auto) {
    constexpr int KIND = decltype(kind_c)::value;
    using S = typename decltype(s_tag)::type;
    if (dtype == LBM_DTYPE_F64)
      hipLaunchKernelGGL((init_equilibrium_kernel<KIND, S, double>), L->grid, L->block, 0,
                         L->stream, L->args, (const double*)drho, (const double*)u);
    else
      hipLaunchKernelGGL((init_equilibrium_kernel<KIND, S, float>), L->grid, L->block, 0,
                         L->stream, L->args, (const float*)drho, (const float*)u);
  });
  const int rc = check_launch();
  if (rc) return rc;
  L->t = t0;
  L->parity = 0;
  return LBM_OK;
}

int lbm_set_populations(lbm_lattice* L, const void* f, int dtype, int64_t t0) {
  if (!L || !f || !valid_dtype(dtype)) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  with_config(L, [&](auto kind_c, auto s_tag, auto) {
    constexpr int Q = Model<decltype(kind_c)::value>::Q;
    using S = typename decltype(s_tag)::type;
    if (dtype == LBM_DTYPE_F64)
      hipLaunchKernelGGL((set_populations_kernel<Q, S, double>), L->grid, L->block, 0,
                         L->stream, L->args, (const double*)f);
    else
      hipLaunchKernelGGL((set_populations_kernel<Q, S, float>), L->grid, L->block, 0,
                         L->stream, L->args, (const float*)f);
  });
  const int rc = check_launch();
  if (rc) return rc;
  L->t = t0;
  L->parity = 0;
  return LBM_OK;
}

int lbm_get_populations(lbm_lattice* L, void* f, int dtype) {
  if (!L || !f || !valid_dtype(dtype)) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  with_config(L, [&](auto kind_c, auto s_tag, auto bc_c) {
    constexpr int Q = Model<decltype(kind_c)::value>::Q;
    using S = typename decltype(s_tag)::type;
    constexpr bool BC = decltype(bc_c)::value;
    if (dtype == LBM_DTYPE_F64)
      hipLaunchKernelGGL((get_populations_kernel<Q, S, BC, double>), L->grid, L->block, 0,
                         L->stream, L->args, L->parity, (long long)L->t, (double*)f);
    else
      hipLaunchKernelGGL((get_populations_kernel<Q, S, BC, float>), L->grid, L->block, 0,
                         L->stream, L->args, L->parity, (long long)L->t, (float*)f);
  });
  return check_launch();
}

int lbm_step(lbm_lattice* L, int64_t n) {
  if (!L || n < 0) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  for (int64_t k = 0; k < n; ++k) {
    step_dispatch(L, L->parity == 1, (long long)L->t);
    if (L->nlinks > 0) links_dispatch(L, L->parity == 1);
    L->t += 1;
    L->parity ^= 1;
    if (L->check_every > 0 && L->t % L->check_every == 0) {
      const int rc = run_check(L);
      if (rc) return rc;
    }
  }
  return check_launch();
}

int lbm_step_record(lbm_lattice* L, void* rec, int dtype) {
  if (!L || !rec || !valid_dtype(dtype)) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  if (L->kind > 2 || L->cfg.storage == LBM_F16 || L->solids || L->args.bc.freeslip ||
      L->args.bc.pressure)
    return LBM_EINVAL;
  if (dtype != (L->cfg.storage == LBM_F64 ? LBM_DTYPE_F64 : LBM_DTYPE_F32)) return LBM_EINVAL;
  step_record_dispatch(L, L->parity == 1, (long long)L->t, rec);
  L->t += 1;
  L->parity ^= 1;
  return check_launch();
}

int lbm_get_macroscopic(lbm_lattice* L, void* rho, void* u, int dtype, int rho_mode) {
  if (!L || !valid_dtype(dtype)) return LBM_EINVAL;
  if (rho_mode != LBM_RHO_FULL && rho_mode != LBM_RHO_DEVIATION) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  if (!rho && !u) return LBM_OK;
  with_config(L, [&](auto kind_c, auto s_tag, auto bc_c) {
    constexpr int KIND = decltype(kind_c)::value;
    using S = typename decltype(s_tag)::type;
    constexpr bool BC = decltype(bc_c)::value;
    if (dtype == LBM_DTYPE_F64)
      hipLaunchKernelGGL((macroscopic_kernel<KIND, S, BC, double>), L->grid, L->block, 0,
                         L->stream, L->args, L->parity, (long long)L->t, (double*)rho,
                         (double*)u, rho_mode);
    else
      hipLaunchKernelGGL((macroscopic_kernel<KIND, S, BC, float>), L->grid, L->block, 0,
                         L->stream, L->args, L->parity, (long long)L->t, (float*)rho,
                         (float*)u, rho_mode);
  });
  return check_launch();
}

int lbm_set_solids(lbm_lattice* L, const uint8_t* solid, uint32_t* masks) {
  if (!L) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  if (L->parity != 0) return LBM_ESTATE;
  L->args.solid_nb = nullptr;
  L->solids = false;
  L->link_nodes = nullptr;  // new solids clear the links
  L->link_q = nullptr;
  L->nlinks = 0;
  L->has_bc = L->args.bc.nonper != 0;
  if (solid) {
    if (!masks) return LBM_EINVAL;
    int* flag = (int*)(L->base + L->off_result);
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), L->stream);
    if (e != hipSuccess) return hip_fail(e);
    if (L->Q == 27)
      hipLaunchKernelGGL((solid_mask_kernel<27>), L->grid, L->block, 0, L->stream, L->args, solid,
                         masks, flag);
    else
      hipLaunchKernelGGL((solid_mask_kernel<19>), L->grid, L->block, 0, L->stream, L->args, solid,
                         masks, flag);
    const int rc = check_launch();
    if (rc) return rc;
    int bad = 0;
    e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, L->stream);
    if (e != hipSuccess) return hip_fail(e);
    e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return hip_fail(e);
    if (bad) {
      plan_rows(L);
      return LBM_EINVAL;
    }
    L->args.solid_nb = masks;
    L->solids = true;
    L->has_bc = true;
  }
  plan_rows(L);
  return LBM_OK;
}

int lbm_set_links(lbm_lattice* L, const int32_t* nodes, const float* q, int64_t n) {
  if (!L || n < 0 || n >= ((int64_t)1 << 31)) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  if (L->parity != 0) return LBM_ESTATE;
  if (n > 0 && (!nodes || !q || !L->solids)) return LBM_EINVAL;
  L->link_nodes = n > 0 ? nodes : nullptr;
  L->link_q = n > 0 ? q : nullptr;
  L->nlinks = n;
  return LBM_OK;
}

int lbm_stats_accumulate(lbm_lattice* L, double* sums) {
  if (!L || !sums) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  with_config(L, [&](auto kind_c, auto s_tag, auto bc_c) {
    constexpr int KIND = decltype(kind_c)::value;
    using S = typename decltype(s_tag)::type;
    constexpr bool BC = decltype(bc_c)::value;
    hipLaunchKernelGGL((stats_accumulate_kernel<KIND, S, BC>), L->grid, L->block, 0, L->stream,
                       L->args, L->parity, (long long)L->t, sums);
  });
  return check_launch();
}

int lbm_stats_finalize(const lbm_lattice* L, const double* sums, int64_t count, void* mean,
                       void* rms, void* ti, int dtype, int axis, int p0, int p1) {
  if (!L || !sums || !mean || !rms || !valid_dtype(dtype) || count < 1) return LBM_EINVAL;
  if (axis < 0 || axis > 2) return LBM_EINVAL;
  const int n3[3] = {L->cfg.nx, L->cfg.ny, L->cfg.nz};
  const int o0 = axis == 0 ? 1 : 0, o1 = axis == 2 ? 1 : 2;
  if (ti && (p0 < 0 || p0 >= n3[o0] || p1 < 0 || p1 >= n3[o1])) return LBM_EINVAL;
  const double inv = 1.0 / (double)count;
  if (dtype == LBM_DTYPE_F64)
    hipLaunchKernelGGL((stats_finalize_kernel<double>), L->grid, L->block, 0, L->stream, L->args,
                       sums, inv, (double*)mean, (double*)rms, (double*)ti, axis, p0, p1);
  else
    hipLaunchKernelGGL((stats_finalize_kernel<float>), L->grid, L->block, 0, L->stream, L->args,
                       sums, inv, (float*)mean, (float*)rms, (float*)ti, axis, p0, p1);
  return check_launch();
}

int lbm_jet_profile(const lbm_lattice* L, const void* mean, int dtype, int axis, double c0,
                    double c1, int ndir, double dr, int nr, double* um, double* re,
                    double* prof) {
  if (!L || !mean || !um || !re || !valid_dtype(dtype)) return LBM_EINVAL;
  if (axis < 0 || axis > 2 || ndir < 1 || ndir > 65536 || nr < 2 || nr > 65536) return LBM_EINVAL;
  if (!std::isfinite(dr) || !(dr > 0.0)) return LBM_EINVAL;
  const long long nx = L->cfg.nx, ny = L->cfg.ny, nz = L->cfg.nz;
  JetSections s{};
  s.comp = axis * nx * ny * nz;
  if (axis == 2) {
    s.sp = nx * ny, s.sa = 1, s.sb = nx, s.np = (int)nz, s.na = (int)nx, s.nb = (int)ny;
  } else if (axis == 1) {
    s.sp = nx, s.sa = 1, s.sb = nx * ny, s.np = (int)ny, s.na = (int)nx, s.nb = (int)nz;
  } else {
    s.sp = 1, s.sa = nx, s.sb = nx * ny, s.np = (int)nx, s.na = (int)ny, s.nb = (int)nz;
  }
  if (s.na < 2 || s.nb < 2) return LBM_EINVAL;
  if (!(c0 >= 0.0 && c0 <= s.na - 1 && c1 >= 0.0 && c1 <= s.nb - 1)) return LBM_EINVAL;
  if (dtype == LBM_DTYPE_F64)
    hipLaunchKernelGGL((jet_profile_kernel<double>), dim3(s.np), dim3(256), 0, L->stream,
                       (const double*)mean, s, c0, c1, ndir, dr, nr, um, re, prof);
  else
    hipLaunchKernelGGL((jet_profile_kernel<float>), dim3(s.np), dim3(256), 0, L->stream,
                       (const float*)mean, s, c0, c1, ndir, dr, nr, um, re, prof);
  return check_launch();
}

int lbm_jet_fit(const lbm_lattice* L, const double* um, const double* re, const double* prof,
                int np, int nr, double dr, double x0, double u0, double d, int p0, int p1,
                double* out) {
  if (!L || !um || !re || !prof || !out) return LBM_EINVAL;
  if (np < 1 || nr < 1 || p0 < 0 || p1 > np || p0 >= p1) return LBM_EINVAL;
  if (!std::isfinite(dr) || !(dr > 0.0) || !std::isfinite(x0) || !std::isfinite(u0) ||
      !(u0 != 0.0) || !std::isfinite(d) || !(d > 0.0))
    return LBM_EINVAL;
  hipLaunchKernelGGL(jet_fit_kernel, dim3(1), dim3(256), 0, L->stream, um, re, prof, np, nr, dr,
                     x0, u0, d, p0, p1, out);
  return check_launch();
}

int lbm_reduce(lbm_lattice* L, double out[5]) {
  if (!L || !out) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  return reduce_now(L, out);
}

int lbm_set_check(lbm_lattice* L, int64_t every, double mass_tol) {
  if (!L || every < 0 || std::isnan(mass_tol)) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  L->check_every = every;
  L->check_tol = mass_tol;
  L->check_m0 = 0.0;
  if (every > 0) {  // the current state is checked at once
    double out[5];
    const int rc = reduce_now(L, out);
    if (rc) {
      L->check_every = 0;
      return rc;
    }
    L->check_m0 = out[0];
  }
  return LBM_OK;
}

int lbm_reduce_static(lbm_lattice* L, double* out) {
  if (!L || !out) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  // fold z planes into the blocks of one plane so the partials fit
  const size_t plane = (size_t)L->grid.x * L->grid.y;
  if (plane > kStaticPartials) return LBM_EINVAL;
  double* partial = nullptr;
  int rc = static_scratch(L->stream, &partial);
  if (rc) return rc;
  size_t gz = kStaticPartials / plane;
  if (gz > (size_t)L->grid.z) gz = L->grid.z;
  const dim3 grid(L->grid.x, L->grid.y, (unsigned)gz);
  with_config(L, [&](auto kind_c, auto s_tag, auto bc_c) {
    constexpr int KIND = decltype(kind_c)::value;
    using S = typename decltype(s_tag)::type;
    constexpr bool BC = decltype(bc_c)::value;
    hipLaunchKernelGGL((reduce_partial_kernel<KIND, S, BC>), grid, L->block, 0, L->stream,
                       L->args, L->parity, (long long)L->t, partial);
  });
  rc = check_launch();
  if (rc) return rc;
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, L->stream, partial,
                     plane * gz, out);
  return check_launch();
}

int lbm_state_bytes(const lbm_lattice* L, size_t* bytes) {
  if (!L || !bytes) return LBM_EINVAL;
  *bytes = L->off_partial;
  return LBM_OK;
}

int lbm_save_state(lbm_lattice* L, void* dev, size_t bytes, int64_t* t, int32_t* parity) {
  if (!L || !dev) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  if (bytes < L->off_partial) return LBM_ENOMEM;
  const hipError_t e =
      hipMemcpyAsync(dev, L->base, L->off_partial, hipMemcpyDeviceToDevice, L->stream);
  if (e != hipSuccess) return hip_fail(e);
  if (t) *t = L->t;
  if (parity) *parity = L->parity;
  return LBM_OK;
}

int lbm_load_state(lbm_lattice* L, const void* dev, size_t bytes, int64_t t, int32_t parity) {
  if (!L || !dev || (parity != 0 && parity != 1)) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  if (bytes < L->off_partial) return LBM_ENOMEM;
  const hipError_t e =
      hipMemcpyAsync(L->base, dev, L->off_partial, hipMemcpyDeviceToDevice, L->stream);
  if (e != hipSuccess) return hip_fail(e);
  L->t = t;
  L->parity = parity;
  return LBM_OK;
}

int lbm_get_time(const lbm_lattice* L, int64_t* t) {
  if (!L || !t) return LBM_EINVAL;
  *t = L->t;
  return LBM_OK;
}

int lbm_destroy(lbm_lattice* L) {
  if (L) L->tracer->report("lattice");
  delete L;
  return LBM_OK;
}

int lbm_probe_ke(lbm_lattice* L, const int32_t lo[3], const int32_t hi[3], void* lambda,
                 int dtype, double* J) {
  if (!L || !lo || !hi || !J || !valid_dtype(dtype)) return LBM_EINVAL;
  if (!L->base) return LBM_EUNBOUND;
  const int n3[3] = {L->cfg.nx, L->cfg.ny, L->cfg.nz};
  for (int d = 0; d < 3; ++d)
    if (lo[d] < 0 || hi[d] > n3[d] || lo[d] >= hi[d]) return LBM_EINVAL;
  const double scale = 1.0 / ((double)(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]));
  double* partial = (double*)(L->base + L->off_partial);
  double* result = (double*)(L->base + L->off_result);
  const int3 l3 = make_int3(lo[0], lo[1], lo[2]), h3 = make_int3(hi[0], hi[1], hi[2]);
  with_config(L, [&](auto kind_c, auto s_tag, auto bc_c) {
    constexpr int KIND = decltype(kind_c)::value;
    using S = typename decltype(s_tag)::type;
    constexpr bool BC = decltype(bc_c)::value;
    if (dtype == LBM_DTYPE_F64)
      hipLaunchKernelGGL((probe_kernel<KIND, S, BC, double>), L->grid, L->block, 0, L->stream,
                         L->args, L->parity, (long long)L->t, l3, h3, scale, (double*)lambda,
                         partial);
    else
      hipLaunchKernelGGL((probe_kernel<KIND, S, BC, float>), L->grid, L->block, 0, L->stream,
                         L->args, L->parity, (long long)L->t, l3, h3, scale, (float*)lambda,
                         partial);
  });
  int rc = check_launch();
  if (rc) return rc;
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, L->stream, partial,
                     L->nblocks, result);
  rc = check_launch();
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(J, result, sizeof(double), hipMemcpyDeviceToHost, L->stream);
  if (e != hipSuccess) return hip_fail(e);
  e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_fail(e);
  return std::isfinite(*J) ? LBM_OK : LBM_ENONFINITE;
}

int lbm_adjoint_step(lbm_lattice* L, const void* f_t, const void* lambda_next, void* lambda,
                     int dtype, double* grad_inlet) {
  if (!L || !f_t || !lambda_next || !lambda || !valid_dtype(dtype)) return LBM_EINVAL;
  if (L->kind > 2 || L->solids || L->args.bc.freeslip || L->args.bc.pressure)
    return LBM_EINVAL;
  if (lambda == lambda_next || lambda == f_t) return LBM_EINVAL;
  // the kernels address the adjoint arrays with 32-bit byte offsets: one
  // slab must stay below 4 GiB, and the wall rows (a population and its
  // opposite from the lower slab) need the whole span below 4 GiB, else the
  // general kernel takes every row
  const double rsz = dtype == LBM_DTYPE_F64 ? 8.0 : 4.0;
  if ((double)L->N * rsz >= 4294967296.0) return LBM_EINVAL;
  const int Q = L->kind == 2 ? 27 : 19;
  const bool split = L->split_odd && slab_span(Q) * (double)L->N * rsz < 4294967296.0;
  TraceScope ts(L->tracer.get(), L->stream, "adjoint step (adjoint_kernel launches)");
  auto run = [&](auto kind_c, auto real_tag) {
    constexpr int K = decltype(kind_c)::value;
    using R = typename decltype(real_tag)::type;
    const R* f = (const R*)f_t;
    const R* ln = (const R*)lambda_next;
    R* l = (R*)lambda;
    if (!L->has_bc) {
      hipLaunchKernelGGL((adjoint_kernel<K, R, BC_NONE, ROWS_BOX>), L->grid, L->block, 0,
                         L->stream, L->args, L->rows_all, f, ln, l, grad_inlet);
    } else if (!split) {
      hipLaunchKernelGGL((adjoint_kernel<K, R, BC_GENERAL, ROWS_BOX>), L->grid, L->block, 0,
                         L->stream, L->args, L->rows_all, f, ln, l, grad_inlet);
    } else {
      if (L->grid_inner.y > 0 && L->grid_inner.z > 0)
        hipLaunchKernelGGL((adjoint_kernel<K, R, BC_WALLS, ROWS_BOX>), L->grid_inner, L->block,
                           0, L->stream, L->args, L->rows_inner, f, ln, l, grad_inlet);
      if (L->grid_bnd.y > 0)
        hipLaunchKernelGGL((adjoint_kernel<K, R, BC_GENERAL, ROWS_LIST>), L->grid_bnd,
                           L->block_bnd, 0, L->stream, L->args, L->rows_bnd, f, ln, l,
                           grad_inlet);
    }
  };
  auto by_type = [&](auto kind_c) {
    if (dtype == LBM_DTYPE_F64)
      run(kind_c, std::type_identity<double>{});
    else
      run(kind_c, std::type_identity<float>{});
  };
  switch (L->kind) {
    case 0: by_type(std::integral_constant<int, 0>{}); break;
    case 1: by_type(std::integral_constant<int, 1>{}); break;
    default: by_type(std::integral_constant<int, 2>{}); break;
  }
  return check_launch();
}

int lbm_stream_copy(void* dst, const void* src, size_t n, void* stream) {
  if (!dst || !src || (((uintptr_t)dst | (uintptr_t)src | n) & 15) != 0) return LBM_EINVAL;
  const size_t n16 = n / 16;
  if (n16 == 0) return LBM_OK;
  const size_t blocks = (n16 + 255) / 256;
  if (blocks > 0x7fffffffu) return LBM_EINVAL;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     (u32x4*)dst, (const u32x4*)src, n16);
  return check_launch();
}

}  // extern "C"
