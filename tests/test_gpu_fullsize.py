"""Parity at the benchmark's full size and launch configuration.

The 256 x 256 x 512 round jet is built exactly as bench.py builds it (same
lattice, boundaries, inlet field and perturbation seed), loaded with a seeded
noise state from synth (far from equilibrium, so every collision term is
exercised) and stepped three times (even, odd, even parity: both row splits
of the odd step run). Sampled 8^3 boxes are then compared element by element
with the FP64 oracle run on the same box padded by the light cone (three
nodes per side; cut sides are made periodic in the oracle, which only
corrupts the padding). The boxes cover the interior, both row ends (x walls),
a y wall, the inlet disk with its perturbation, the inlet-wall corner, the
outflow plane and the outflow-wall corner.

Tolerances per step, as in the small-lattice parity tests: FP64 1e-12, FP32
4e-6, FP16 2e-3 of the largest population; the oracle starts from the state
rounded to the storage precision, exactly as the GPU stored it.

The same is done for the jet with the round nozzle tube as curved walls
(interpolated bounce-back), in boxes across the tube.

The two-level refined workload of the benchmark is compared at full size with
the oracle's refined lattice (FP64 storage, two level-0 steps from noise) and
keeps a uniform co-flow exactly uniform.
A 512 x 512 x 256 FP64 lattice checks the path taken when 32-bit offsets
cannot span a population and its opposite. The velocity time averages of
the FCLB FP32 jet are checked in four of the boxes.
"""
import numpy as np
import pytest

import oracle
import synth
from lbm_cases import MODELS, oracle_lattice, rel_err, window

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

W, I, O = oracle.WALL, oracle.INLET, oracle.OUTFLOW
JET = [W, W, W, W, I, O]
STEPS, T0, SEED, AMP = 3, 0, 20120389, 1e-2
BOXES = [  # (lo, hi) in (x, y, z)
    ((124, 124, 250), (132, 132, 258)),  # interior
    ((0, 100, 100), (8, 108, 108)),      # row starts at the x- wall
    ((248, 100, 100), (256, 108, 108)),  # row ends at the x+ wall
    ((100, 0, 300), (108, 8, 308)),      # y- wall (face rows of the odd step)
    ((124, 124, 0), (132, 132, 8)),      # inlet disk, perturbed
    ((0, 248, 0), (8, 256, 8)),          # x- wall, y+ wall, inlet corner
    ((120, 0, 504), (128, 8, 512)),      # outflow plane, y- wall
    ((248, 248, 504), (256, 256, 512)),  # x+, y+, outflow corner
]
TOL = {"f64": 1e-12, "f32": 4e-6, "f16": 2e-3}
ROUND = {"f64": np.float64, "f32": np.float32, "f16": np.float16}


@pytest.mark.parametrize("workload", ["jet256-fclb-f32", "jet256-mrt-f32", "jet256-fclb-f16",
                                      "jet256-fclb-f64", "jet256-clb-f32"])
def test_jet256_boxes_against_oracle(workload):
    import bench
    import paper_1206_0389_amd as P
    print("case full size", workload, flush=True)
    model, storage, shape, _ = bench.workload(workload)
    nx, ny, nz = shape
    name = "mrt_table1" if model == "mrt" else model
    Q = 19 if model == "mrt" else 27
    lat, _ = bench.make_lattice(workload, P, torch, synth)
    js = bench.jet_setup(nx, ny, synth)
    f = torch.empty((Q, nz, ny, nx), dtype=torch.float64, device="cuda")
    for q in range(Q):
        f[q] = torch.from_numpy(synth.tiled_populations(Q, (nz, ny, nx), AMP, SEED,
                                                        qs=[q])[0]).cuda()
    lat.set_populations(f, t0=T0)
    del f
    lat.step(STEPS)
    torch.cuda.synchronize()
    got = lat.populations()
    worst = 0.0
    for lo, hi in BOXES:
        wlo, whi, wf, inner = window((nx, ny, nz), JET, lo, hi, STEPS)
        f0 = synth.tiled_populations(Q, (nz, ny, nx), AMP, SEED, lo=wlo, hi=whi)
        f0 = f0.astype(ROUND[storage]).astype(np.float64)
        o = oracle_lattice(name, tuple(b - a for a, b in zip(wlo, whi)), js["nu"],
                           cs=js["cs"] if model == "mrt" else 0.0, faces=wf,
                           face_u=js["face_u"], inlet=(js["inlet_u"], js["inlet_mask"]),
                           amp=js["inlet_amp"], seed=js["seed"], origin=tuple(wlo),
                           extent=(nx, ny))
        ref = o.run(f0, T0, STEPS)[:, inner[2], inner[1], inner[0]]
        g = got[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].cpu().numpy()
        err = rel_err(g, ref)
        worst = max(worst, err)
        assert err <= STEPS * TOL[storage], (lo, hi, err)
    print(workload, "worst box error", worst, flush=True)


NOZZLE_BOXES = [  # across the tube wall, at the tube's end, on its diagonal at the inlet
    ((106, 124, 4), (114, 132, 12)),
    ((106, 124, 12), (114, 132, 20)),
    ((112, 112, 0), (120, 120, 8)),
    ((140, 124, 4), (148, 132, 12)),
]


def test_nozzlecurved256_boxes_against_oracle():
    """The jet with the round nozzle tube as curved walls (solid nodes plus
    interpolated bounce-back on every fluid-solid link), built as bench.py
    builds it, three steps from the noise state; boxes across the tube's
    wall, its end and its diagonal at the inlet against the oracle window
    with the same solid nodes and link distances."""
    import bench
    import paper_1206_0389_amd as P
    workload = "nozzlecurved256-fclb-f32"
    print("case full size", workload, flush=True)
    model, storage, shape, _ = bench.workload(workload)
    nx, ny, nz = shape
    lat, _ = bench.make_lattice(workload, P, torch, synth)
    js = bench.jet_setup(nx, ny, synth)
    f = torch.empty((27, nz, ny, nx), dtype=torch.float64, device="cuda")
    for q in range(27):
        f[q] = torch.from_numpy(synth.tiled_populations(27, (nz, ny, nx), AMP, SEED,
                                                        qs=[q])[0]).cuda()
    lat.set_populations(f, t0=T0)
    del f
    lat.step(STEPS)
    torch.cuda.synchronize()
    got = lat.populations()
    body = synth.nozzle_tube(nx, ny, js["diameter"], 2.0, 16.0)
    worst = 0.0
    for lo, hi in NOZZLE_BOXES:
        wlo, whi, wf, inner = window((nx, ny, nz), JET, lo, hi, STEPS)
        wsh = (whi[2] - wlo[2], whi[1] - wlo[1], whi[0] - wlo[0])
        solid, nodes, q = synth.link_distances(body, wsh, P.VELOCITIES, origin=tuple(wlo),
                                               full_shape=(nz, ny, nx))
        lq = np.zeros((27,) + wsh)
        z, r = np.divmod(nodes, nx * ny)
        y, x = np.divmod(r, nx)
        lq[:, z - wlo[2], y - wlo[1], x - wlo[0]] = q.T.astype(np.float64)
        f0 = synth.tiled_populations(27, (nz, ny, nx), AMP, SEED, lo=wlo, hi=whi)
        f0 = f0.astype(np.float32).astype(np.float64)
        o = oracle.Lattice(oracle.FCLB27, wsh[2], wsh[1], wsh[0], nu=js["nu"], faces=wf,
                           face_u=js["face_u"], inlet_u=js["inlet_u"],
                           inlet_mask=js["inlet_mask"], inlet_amp=js["inlet_amp"],
                           seed=js["seed"], origin=tuple(wlo), inlet_extent=(nx, ny),
                           solid=solid, link_q=lq)
        ref = o.run(f0, T0, STEPS)[:, inner[2], inner[1], inner[0]]
        g = got[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].cpu().numpy()
        fl = solid[inner[2], inner[1], inner[0]] == 0
        assert (~fl).any() or lo[2] >= 12  # the boxes cut the tube (or its end)
        err = rel_err(g[:, fl], ref[:, fl])
        worst = max(worst, err)
        print("nozzle box", lo, "links", len(nodes), "error", err, flush=True)
        assert err <= STEPS * TOL[storage], (lo, hi, err)
    print(workload, "worst box error", worst, flush=True)


def test_jet256_statistics_boxes():
    """Time averages (lbm_stats_accumulate after each of the 3 steps of the
    full-size FCLB FP32 jet, bench launch configuration) in the sampled boxes
    against the oracle's two-pass statistics of its own states, with the
    bounds of test_gpu_stats.py (per-step state error 4e-6 relative)."""
    import bench
    import paper_1206_0389_amd as P
    workload = "jet256-fclb-f32"
    print("case full size statistics", workload, flush=True)
    model, storage, shape, _ = bench.workload(workload)
    nx, ny, nz = shape
    lat, _ = bench.make_lattice(workload, P, torch, synth)
    js = bench.jet_setup(nx, ny, synth)
    f = torch.empty((27, nz, ny, nx), dtype=torch.float64, device="cuda")
    for q in range(27):
        f[q] = torch.from_numpy(synth.tiled_populations(27, (nz, ny, nx), AMP, SEED,
                                                        qs=[q])[0]).cuda()
    lat.set_populations(f, t0=T0)
    del f
    sums = lat.stats_buffer()
    for _ in range(STEPS):
        lat.step(1)
        lat.stats_accumulate(sums)
    mean, rms, _ = lat.stats_finalize(sums, STEPS)
    del sums
    e = TOL["f32"]
    for lo, hi in BOXES[:4]:
        wlo, whi, wf, inner = window((nx, ny, nz), JET, lo, hi, STEPS)
        f0 = synth.tiled_populations(27, (nz, ny, nx), AMP, SEED, lo=wlo, hi=whi)
        f0 = f0.astype(np.float32).astype(np.float64)
        o = oracle_lattice("fclb", tuple(b - a for a, b in zip(wlo, whi)), js["nu"], faces=wf,
                           face_u=js["face_u"], inlet=(js["inlet_u"], js["inlet_mask"]),
                           amp=js["inlet_amp"], seed=js["seed"], origin=tuple(wlo),
                           extent=(nx, ny))
        us, fo = [], f0
        for k in range(STEPS):
            fo = o.run(fo, T0 + k, 1)
            us.append(o.macroscopic(fo)[1][:, inner[2], inner[1], inner[0]])
        m_o, r_o, _ = oracle.velocity_statistics(us)
        sl = (slice(None), slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        m_g, r_g = mean[sl].cpu().numpy(), rms[sl].cpu().numpy()
        u2max = float((m_o ** 2 + r_o ** 2).max())
        dm = float(np.abs(m_g - m_o).max())
        dv = float(np.abs(r_g ** 2 - r_o ** 2).max())
        print("statistics box", lo, "mean", dm / np.abs(m_o).max(), "var", dv / u2max, flush=True)
        assert dm <= STEPS * e * float(np.abs(m_o).max()), (lo, dm)
        assert dv <= 4 * STEPS * e * u2max, (lo, dv)


def _bench_refined(model, storage, u0=None):
    """The benchmark's two-level 128 x 128 x 256 jet (16^3 blocks, 416 of 1024
    refined); with u0 a uniform co-flow inlet instead of the jet's."""
    import bench
    import paper_1206_0389_amd as P
    nx, ny, nz, B = 128, 128, 256, 16
    mask = bench.refined_jet_mask(nx, ny, nz, B)
    fu = [[0.0, 0.0, 0.002]] * 4 + [[0.0, 0.0, 0.0]] * 2
    if u0 is None:
        iu, im = synth.jet_inlet(nx, ny, 16.0, 0.05, 0.002)
        fiu, fim = synth.jet_inlet(2 * nx, 2 * ny, 32.0, 0.05, 0.002)
        amp = 5e-4
    else:
        iu = np.zeros((3, ny, nx))
        iu[2] = u0
        fiu = np.zeros((3, 2 * ny, 2 * nx))
        fiu[2] = u0
        im = fim = None
        amp = 0.0
        fu = [[0.0, 0.0, u0]] * 4 + [[0.0, 0.0, 0.0]] * 2
    lat = P.RefinedLattice(model=model, storage=storage, shape=(nx, ny, nz), nu=1e-4,
                           cs_smag=0.1, block=B, mask=mask,
                           faces=[P.WALL] * 4 + [P.INLET, P.OUTFLOW], face_u=fu,
                           inlet_u=torch.from_numpy(iu),
                           inlet_mask=None if im is None else torch.from_numpy(im),
                           fine_inlet_u=torch.from_numpy(fiu),
                           fine_inlet_mask=None if fim is None else torch.from_numpy(fim),
                           inlet_amp=amp, seed=12060389)
    return lat, (nx, ny, nz, B, mask, fu, iu, im, fiu, fim, amp)


@pytest.mark.parametrize("model", ["fclb", "mrt"])
def test_refined_jet_full_size_uniform_flow(model):
    """The 128 x 128 x 256 two-level jet of the benchmark: a uniform co-flow
    through the whole configuration (inlet at the co-flow speed everywhere,
    walls moving with it) stays exactly uniform on both levels in FP64."""
    print("case refined full size uniform", model, flush=True)
    u0 = 0.002
    lat, _ = _bench_refined(model, "f64", u0=u0)
    for level in (0, 1):
        d, u = synth.uniform_fields(*lat.shape3(level)[::-1], u=(0.0, 0.0, u0))
        lat.init_equilibrium(level, torch.from_numpy(d), torch.from_numpy(u))
    f0 = [lat.populations(level) for level in (0, 1)]
    lat.step(3)
    for level in (0, 1):
        live = torch.from_numpy(np.isin(lat.types(level), (1, 2))).cuda()
        d, u = lat.macroscopic(level)
        f1 = lat.populations(level)
        assert float((f1 - f0[level])[:, live].abs().max()) < 1e-15, level
        assert float((u[2][live] - u0).abs().max()) < 1e-15
        assert float(d[live].abs().max()) < 1e-15
    del lat, f0
    torch.cuda.empty_cache()


@pytest.mark.parametrize("model", ["fclb", "mrt"])
def test_refined_jet_full_size_against_oracle(model):
    """The benchmark's two-level jet (13.6 M fine nodes, 3,000+ ghost groups,
    the full interface) in FP64 storage from a seeded noise state on both
    levels, two level-0 steps, against the oracle's refined lattice element
    by element on both levels (fluid and band nodes, the covered nodes they
    read) to 1e-12 relative."""
    print("case refined full size vs oracle", model, flush=True)
    lat, (nx, ny, nz, B, mask, fu, iu, im, fiu, fim, amp) = _bench_refined(model, "f64")
    code = oracle.FCLB27 if model == "fclb" else oracle.MRT19
    c = oracle.Lattice(code, nx, ny, nz, nu=1e-4, cs_smag=0.1,
                       faces=[W, W, W, W, I, O], face_u=fu, inlet_u=iu, inlet_mask=im,
                       inlet_amp=amp, seed=12060389)
    R = oracle.Refined(c, B, mask, 2, inlet_u=[None, fiu], inlet_mask=[None, fim])
    Q = c.Q
    for level in (0, 1):
        assert np.array_equal(lat.types(level), lat.to_box(level, R.types(level))), level
        shape = lat.shape3(level)
        f = synth.random_populations(Q, shape, 1e-2, seed=SEED + level)
        lat.set_populations(level, torch.from_numpy(f), T0)
        full = np.zeros((Q,) + R.levels[level]["shape"])
        sz, sy, sx, wx = lat.box_slices(level)
        full[:, sz, sy, sx] = f[..., :wx]
        R.set_state(level, full)
        del f, full
    lat.step(2)
    R.run(T0, 2)
    from lbm_cases import read_covered
    for level in (0, 1):
        keep = np.isin(lat.types(level), (1, 2))
        if level == 0:
            keep |= lat.to_box(0, read_covered(R.types(0), [W, W, W, W, I, O])).astype(bool)
        got = lat.populations(level).cpu().numpy()[:, keep]
        want = lat.to_box(level, R.state(level))[:, keep]
        err = rel_err(got, want)
        print("refined full size", model, "level", level, "nodes", int(keep.sum()),
              "error", err, flush=True)
        assert err <= 1e-12, (level, err)
    del lat, R
    torch.cuda.empty_cache()


def test_lattice_beyond_the_offset_span_takes_the_general_path():
    """512 x 512 x 256 nodes in FP64: eight population slabs are exactly
    4 GiB, so the x-wall rows of the odd step (which address a corner
    population and its opposite, 7 slabs apart, with 32-bit offsets) must run
    through the general kernel. Boxes at the x walls and the interior against
    the oracle after 3 steps."""
    import bench
    import paper_1206_0389_amd as P
    nx, ny, nz = 512, 512, 256
    print("case beyond offset span", (nx, ny, nz), flush=True)
    js = bench.jet_setup(nx, ny, synth)
    lat = P.Lattice(model="fclb", storage="f64", shape=(nx, ny, nz), nu=js["nu"])
    faces = [P.WALL] * 4 + [P.INLET, P.OUTFLOW]
    lat.set_boundaries(faces, face_u=js["face_u"], inlet_u=torch.from_numpy(js["inlet_u"]),
                       inlet_mask=torch.from_numpy(js["inlet_mask"]),
                       inlet_amp=js["inlet_amp"], seed=js["seed"])
    f = torch.empty((27, nz, ny, nx), dtype=torch.float64, device="cuda")
    for q in range(27):
        f[q] = torch.from_numpy(synth.tiled_populations(27, (nz, ny, nx), AMP, SEED,
                                                        qs=[q])[0]).cuda()
    lat.set_populations(f, t0=T0)
    del f
    lat.step(STEPS)
    boxes = [((0, 200, 100), (8, 208, 108)), ((504, 300, 120), (512, 308, 128)),
             ((250, 250, 60), (258, 258, 68)), ((0, 0, 0), (8, 8, 8))]
    full = lat.populations()
    worst = 0.0
    for lo, hi in boxes:
        wlo, whi, wf, inner = window((nx, ny, nz), JET, lo, hi, STEPS)
        f0 = synth.tiled_populations(27, (nz, ny, nx), AMP, SEED, lo=wlo, hi=whi)
        o = oracle_lattice("fclb", tuple(b - a for a, b in zip(wlo, whi)), js["nu"], faces=wf,
                           face_u=js["face_u"], inlet=(js["inlet_u"], js["inlet_mask"]),
                           amp=js["inlet_amp"], seed=js["seed"], origin=tuple(wlo),
                           extent=(nx, ny))
        ref = o.run(f0, T0, STEPS)[:, inner[2], inner[1], inner[0]]
        g = full[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].cpu().numpy()
        err = rel_err(g, ref)
        worst = max(worst, err)
        assert err <= STEPS * TOL["f64"], (lo, hi, err)
    print("beyond offset span: worst box error", worst, flush=True)
