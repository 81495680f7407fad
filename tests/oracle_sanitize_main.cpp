// Drives every entry of the FP64 oracle on small seeded cases so that a build
// with the address and undefined-behaviour sanitizers can watch each code
// path: uniform steps of the four collision set-ups on a periodic box, the
// jet faces (walls moving with the co-flow, perturbed inlet, outflow), free
// slip and fixed-pressure faces, interior solids with curved links, the
// adjoint and tangent steps with the kinetic-energy probe, and nested
// refinement on two and three levels (steps, ghosts, rescaling, half-step
// values, reductions). Prints one line per case and "ok" at the end; any
// sanitizer report aborts the run (-fno-sanitize-recover).
//
// Test infrastructure: built and run by tests/test_oracle_sanitize.py only.
#include "../oracle/lbm_oracle.cpp"

#include <cstdio>
#include <random>
#include <vector>

namespace {

std::mt19937_64 rng(1206);

std::vector<double> noise(size_t n, double amp) {
  std::uniform_real_distribution<double> u(-amp, amp);
  std::vector<double> v(n);
  for (double& x : v) x = u(rng);
  return v;
}

orc_params params(int model, int basis, int nx, int ny, int nz) {
  orc_params p;
  std::memset(&p, 0, sizeof(p));
  p.model = model;
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.nu = 0.02;
  p.cs_smag = model == ORC_MRT19 ? 0.1 : 0.0;
  p.mrt_basis = basis;
  const double dh[5] = {1.19, 1.4, 1.2, 1.4, 1.98};
  for (int k = 0; k < 5; ++k) p.rates[k] = basis == ORC_BASIS_DHUMIERES ? dh[k] : 1.0;
  return p;
}

long nodes(const orc_params& p) { return (long)p.nx * p.ny * p.nz; }

void steps(const char* what, const orc_params& p, int n) {
  const int Q = nq(p.model);
  std::vector<double> f = noise((size_t)Q * nodes(p), 1e-2);
  const int bad = orc_run(&p, f.data(), 0, n);
  std::vector<double> drho(nodes(p)), u(3 * nodes(p));
  orc_macroscopic(&p, f.data(), drho.data(), u.data());
  double out[5];
  orc_reduce(&p, f.data(), out);
  std::printf("%-28s Q=%d bad=%d mass=%.3e\n", what, Q, bad, out[0]);
}

}  // namespace

int main() {
  orc_set_threads(2);
  const int models[4][2] = {{ORC_MRT19, ORC_BASIS_TABLE1},
                            {ORC_MRT19, ORC_BASIS_DHUMIERES},
                            {ORC_FCLB27, 0},
                            {ORC_CLB27, 0}};
  for (const auto& m : models) steps("periodic", params(m[0], m[1], 6, 5, 7), 3);

  // jet faces
  const int nx = 8, ny = 8, nz = 10;
  std::vector<double> inlet((size_t)3 * nx * ny, 0.0);
  std::vector<uint8_t> mask((size_t)nx * ny, 0);
  for (int b = 0; b < ny; ++b)
    for (int a = 0; a < nx; ++a) {
      const double r2 = (a - 3.5) * (a - 3.5) + (b - 3.5) * (b - 3.5);
      const bool in = r2 <= 4.0;
      inlet[(size_t)2 * nx * ny + (size_t)b * nx + a] = in ? 0.05 : 0.002;
      mask[(size_t)b * nx + a] = in;
    }
  for (const auto& m : models) {
    orc_params p = params(m[0], m[1], nx, ny, nz);
    const int ft[6] = {ORC_WALL, ORC_WALL, ORC_WALL, ORC_WALL, ORC_INLET, ORC_OUTFLOW};
    for (int k = 0; k < 6; ++k) p.face_type[k] = ft[k];
    for (int k = 0; k < 4; ++k) p.face_u[k][2] = 0.002;
    p.inlet_u = inlet.data();
    p.inlet_mask = mask.data();
    p.inlet_amp = 1e-3;
    p.seed = 7;
    p.inlet_na = nx;
    p.inlet_nb = ny;
    steps("jet faces", p, 3);
  }

  // free slip and fixed pressure
  for (const auto& m : models) {
    orc_params p = params(m[0], m[1], 6, 7, 8);
    const int ft[6] = {ORC_FREESLIP, ORC_FREESLIP, ORC_WALL, ORC_WALL, ORC_PRESSURE,
                       ORC_PRESSURE};
    for (int k = 0; k < 6; ++k) p.face_type[k] = ft[k];
    p.face_drho[4] = 0.001;
    p.face_drho[5] = -0.001;
    steps("free slip / pressure", p, 3);
  }

  // interior solids with curved links
  {
    orc_params p = params(ORC_FCLB27, 0, 8, 8, 8);
    std::vector<uint8_t> solid(nodes(p), 0);
    for (int z = 3; z < 5; ++z)
      for (int y = 3; y < 5; ++y)
        for (int x = 3; x < 5; ++x) solid[((long)z * 8 + y) * 8 + x] = 1;
    std::vector<double> q((size_t)27 * nodes(p), 0.0);
    std::uniform_real_distribution<double> uq(0.05, 0.95);
    for (double& v : q) v = uq(rng);
    p.solid = solid.data();
    p.link_q = q.data();
    steps("solids and links", p, 3);
  }

  // adjoint, tangent and probe
  {
    orc_params p = params(ORC_FCLB27, 0, nx, ny, nz);
    const int ft[6] = {ORC_WALL, ORC_WALL, ORC_WALL, ORC_WALL, ORC_INLET, ORC_OUTFLOW};
    for (int k = 0; k < 6; ++k) p.face_type[k] = ft[k];
    p.inlet_u = inlet.data();
    p.inlet_na = nx;
    p.inlet_nb = ny;
    const size_t n = (size_t)27 * nodes(p);
    std::vector<double> f = noise(n, 1e-2), v = noise(n, 1.0), out(n), lam(n), lam2(n);
    std::vector<double> grad((size_t)3 * nx * ny, 0.0);
    const int32_t lo[3] = {2, 2, 3}, hi[3] = {6, 6, 7};
    const double J = orc_probe_ke(&p, f.data(), lo, hi, lam.data());
    orc_adjoint_step(&p, f.data(), lam.data(), lam2.data(), grad.data());
    orc_tangent_step(&p, f.data(), v.data(), out.data());
    std::vector<double> jv(27);
    orc_collide_jvp(&p, f.data(), v.data(), jv.data());
    std::printf("%-28s J=%.3e\n", "adjoint / tangent", J);
  }

  // nested refinement: the slab of two and three levels, and a jet
  for (int levels = 2; levels <= 3; ++levels) {
    for (const auto& m : models) {
      if (m[0] == ORC_CLB27) continue;
      orc_params p = params(m[0], m[1], 4, 4, 64);
      std::vector<uint8_t> map(16, 0);
      for (int k = 6; k < 10; ++k) map[k] = 1;
      if (levels == 3) {
        for (int k = 4; k < 12; ++k) map[k] = 1;
        map[7] = map[8] = 2;
      }
      void* h = orc_mlref_create(&p, 4, levels, map.data(), nullptr, nullptr, nullptr, nullptr);
      if (!h) {
        std::printf("refinement create failed\n");
        return 1;
      }
      for (int l = 0; l < levels; ++l) {
        int32_t n3[3], box[6];
        int64_t counts[6];
        orc_mlref_info(h, l, n3, box, counts);
        const size_t N = (size_t)n3[0] * n3[1] * n3[2];
        std::vector<uint8_t> type(N);
        orc_mlref_types(h, l, type.data());
        std::vector<double> f = noise((size_t)nq(p.model) * N, 1e-2);
        orc_mlref_set_state(h, l, f.data());
      }
      const int64_t bad = orc_mlref_run(h, 0, 2);
      for (int l = 1; l < levels; ++l) {
        int32_t n3[3], box[6];
        int64_t counts[6];
        orc_mlref_info(h, l - 1, n3, box, counts);
        const int Q = nq(p.model);
        std::vector<double> parent((size_t)Q * n3[0] * n3[1] * n3[2]);
        orc_mlref_get_state(h, l - 1, parent.data());
        const int64_t ng = orc_mlref_ghost_count(h, l);
        std::vector<int32_t> coords((size_t)3 * ng);
        std::vector<double> g((size_t)Q * ng), hs((size_t)Q * ng), one(Q), res(Q);
        orc_mlref_ghosts(h, l, coords.data(), parent.data(), g.data());
        orc_mlref_half_step(h, l, g.data(), g.data(), g.data(), 1, hs.data());
        for (int q = 0; q < Q; ++q) one[q] = parent[(size_t)q * (parent.size() / Q)];
        orc_mlref_rescale(h, l, one.data(), 1, res.data());
        orc_mlref_rescale(h, l, res.data(), -1, one.data());
      }
      double out[5];
      orc_mlref_reduce(h, out);
      orc_mlref_destroy(h);
      std::printf("%-28s levels=%d Q=%d bad=%lld\n", "refinement slab", levels, nq(p.model),
                  (long long)bad);
    }
  }
  std::printf("ok\n");
  return 0;
}
