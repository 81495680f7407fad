"""HIP path vs the FP64 oracle, element by element, through the C ABI.

FP64 storage: max |f_gpu - f_oracle| / max |f_oracle| <= 1e-12 (the two
differ only in rounding order: FMA contraction on the GPU, a factorised
central-moment transform vs the oracle's dense 27x27 solve).
FP32 / FP16 storage: the per-step error is dominated by rounding the
stored deviations (2^-24 and 2^-11 relative) plus FP32 arithmetic; the
bounds below allow a few units of that per step.
"""
import numpy as np
import pytest

import oracle
import synth
from lbm_cases import (JET_FACES, MODELS, O, P, W, I, face_velocities, gpu_lattice,
                       oracle_lattice, rel_err)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

TOL = {"f64": 1e-12, "f32": 4e-6, "f16": 2e-3}
F = oracle.FREESLIP
PR = oracle.PRESSURE
NAMES = list(MODELS)


def _say(*a):
    print(*a, flush=True)


def _run_pair(name, storage, shape, nu, steps, cs=0.1, faces=None, face_u=None, inlet=None,
              amp=0.0, seed=0, t0=0, f0=None, rates=None, face_drho=None):
    nx, ny, nz = shape
    Q = 19 if MODELS[name][0] == oracle.MRT19 else 27
    _say("case", name, storage, shape, "steps", steps, "faces", faces)
    f = f0 if f0 is not None else synth.random_populations(Q, (nz, ny, nx), amp=1e-2, seed=11)
    g = gpu_lattice(name, storage, shape, nu, cs=cs, rates=rates, faces=faces, face_u=face_u,
                    inlet=inlet, amp=amp, seed=seed, face_drho=face_drho)
    o = oracle_lattice(name, shape, nu, cs=cs, rates=rates, faces=faces, face_u=face_u,
                       inlet=inlet, amp=amp, seed=seed, face_drho=face_drho)
    g.set_populations(torch.from_numpy(f), t0)
    snaps = []
    for k in steps:
        g.step(k - (g.time - t0))
        snaps.append((k, g.populations().cpu().numpy()))
    out, ref, done = [], f.copy(), 0
    for k, gp in snaps:
        ref = o.run(ref, t0 + done, k - done)
        done = k
        out.append(rel_err(gp, ref))
    return out


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 10, 9), (1, 16, 3), (16, 12, 1), (7, 1, 1)])
def test_periodic_step_parity_fp64(name, shape):
    errs = _run_pair(name, "f64", shape, 0.02, [1, 2, 5])
    assert max(errs) <= TOL["f64"], errs


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("layout", ["jet", "zoutflow_lo", "x_inlet", "y_inlet_walls",
                                    "xwalls_only", "channel_thin", "freeslip_y", "jet_slip_top",
                                    "slip_x_edges", "slip_box", "jet_pressure", "pressure_x",
                                    "pressure_slip_outflow", "pressure_box"])
def test_boundary_step_parity_fp64(name, layout):
    fu = face_velocities(0.002)
    fu[4] = [0.0, 0.0, 0.0]
    fu[0] = [0.0, 0.001, 0.002]
    shape = (10, 8, 9)
    nx, ny, nz = shape
    if layout == "jet":
        faces, inlet = JET_FACES, synth.jet_inlet(nx, ny, 4.0, 0.05, 0.002)
    elif layout == "zoutflow_lo":
        faces, inlet = [P, P, W, W, O, I], synth.jet_inlet(nx, ny, 4.0, 0.04, 0.001)
    elif layout == "x_inlet":
        faces, inlet = [I, W, P, P, W, O], synth.jet_inlet(ny, nz, 3.0, 0.04, 0.001, axis=0)
    elif layout == "y_inlet_walls":
        faces, inlet = [W, W, W, I, O, W], synth.jet_inlet(nx, nz, 3.0, 0.04, 0.001, axis=1)
    elif layout == "xwalls_only":
        faces, inlet = [W, W, P, P, P, P], None
    elif layout == "freeslip_y":
        faces, inlet = [P, P, F, F, P, P], None
    elif layout == "jet_slip_top":  # free slip meets walls, the inlet and the outflow
        faces, inlet = [W, W, W, F, I, O], synth.jet_inlet(nx, ny, 4.0, 0.05, 0.002)
    elif layout == "slip_x_edges":  # free-slip / free-slip and free-slip / outflow edges
        faces, inlet = [F, F, F, W, I, O], synth.jet_inlet(nx, ny, 4.0, 0.05, 0.002)
    elif layout == "slip_box":
        faces, inlet = [F] * 6, None
    elif layout == "jet_pressure":  # fixed-pressure outlet, edges with walls and the inlet
        faces, inlet = [W, W, W, W, I, PR], synth.jet_inlet(nx, ny, 4.0, 0.05, 0.002)
    elif layout == "pressure_x":  # pressure drop along x, edges with walls and the outflow
        faces, inlet = [PR, PR, P, P, W, O], None
    elif layout == "pressure_slip_outflow":  # pressure meets free slip, a wall, the outflow
        faces, inlet = [PR, W, F, F, O, PR], None
    elif layout == "pressure_box":
        faces, inlet = [PR] * 6, None
    else:  # walls two nodes apart in y: no interior rows at all
        faces, inlet = [W, W, W, W, I, O], synth.jet_inlet(nx, 2, 2.0, 0.04, 0.001)
        shape = (nx, 2, nz)
    errs = _run_pair(name, "f64", shape, 0.02, [1, 2, 6], faces=faces, face_u=fu, inlet=inlet,
                     amp=5e-4, seed=12060389, t0=3,
                     face_drho=[0.002, -0.001, 0.003, -0.002, 0.001, -0.003])
    assert max(errs) <= TOL["f64"], errs


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_reduced_storage_within_stated_tolerance(name, storage):
    errs = _run_pair(name, storage, (16, 12, 10), 0.02, [1, 3], faces=JET_FACES,
                     face_u=face_velocities(0.002), inlet=synth.jet_inlet(16, 12, 6.0, 0.05, 0.002),
                     amp=5e-4, seed=3)
    assert errs[0] <= TOL[storage], errs
    assert errs[1] <= 3 * TOL[storage], errs


@pytest.mark.parametrize("name", ["fclb", "mrt_table1"])
@pytest.mark.parametrize("storage", ["f32", "f16"])
@pytest.mark.parametrize("layout", ["pressure_slip_outflow", "jet_pressure", "slip_box"])
def test_reduced_storage_free_slip_and_pressure(name, storage, layout):
    """The free-slip and fixed-pressure rules with FP32 and FP16 storage:
    the stored value of a completed anti-bounce-back population is rounded
    like any other, so the bound is the one of the plain jet."""
    nx, ny, nz = 16, 12, 10
    inlet = None
    if layout == "pressure_slip_outflow":
        faces = [PR, W, F, F, O, PR]
    elif layout == "jet_pressure":
        faces, inlet = [W, W, W, W, I, PR], synth.jet_inlet(nx, ny, 6.0, 0.05, 0.002)
    else:
        faces = [F] * 6
    errs = _run_pair(name, storage, (nx, ny, nz), 0.02, [1, 3], faces=faces,
                     face_u=face_velocities(0.002), inlet=inlet, amp=5e-4, seed=3,
                     face_drho=[0.002, -0.001, 0.003, -0.002, 0.001, -0.003])
    assert errs[0] <= TOL[storage], errs
    assert errs[1] <= 3 * TOL[storage], errs


@pytest.mark.parametrize("name", ["mrt_table1", "fclb"])
def test_pressure_driven_channel_flow(name):
    """Physics of the fixed-pressure faces, at any size: a density drop
    between two PRESSURE faces (x) drives the flow between two WALL faces
    (y). Mid-channel, the settled flow is the plane Poiseuille profile u(y) =
    G (y + 1/2)(H - 1/2 - y) / (2 nu) for the local gradient G = -c_s^2
    d(rho)/dx (walls half a link outside the end nodes, H = ny), within 0.5 %;
    that gradient is the imposed drop over the length, c_s^2 (rho_in -
    rho_out) / nx, within 5 % (the faces fix the density of a non-uniform
    profile only on average: an O(1/nx) end effect, 3.5 % at nx = 48 and
    half that at nx = 96 in the oracle). The same run of the oracle gives the
    same figures."""
    nx, ny, nz = 48, 17, 1
    nu, d_in, d_out = 0.1, 0.0015, -0.0015
    faces = [PR, PR, W, W, P, P]
    g = gpu_lattice(name, "f64", (nx, ny, nz), nu, faces=faces, face_u=[[0.0] * 3] * 6,
                    face_drho=[d_in, d_out, 0, 0, 0, 0])
    d0, u0 = synth.uniform_fields(nx, ny, nz)
    g.init_equilibrium(torch.from_numpy(d0), torch.from_numpy(u0))
    g.step(12000)
    d, u = (t.cpu().numpy() for t in g.macroscopic())
    dc = d[0, ny // 2, :]
    G = -(dc[nx // 2 + 5] - dc[nx // 2 - 5]) / 10 / 3.0
    G_nominal = (d_in - d_out) / 3.0 / nx
    y = np.arange(ny)
    ux = u[0, 0, :, nx // 2]
    exact = G * (y + 0.5) * (ny - 0.5 - y) / (2 * nu)
    err = np.abs(ux - exact).max() / exact.max()
    print(name, "Poiseuille error", err, "gradient / nominal", G / G_nominal, flush=True)
    assert err <= 5e-3, err
    assert abs(G / G_nominal - 1) <= 0.05
    # no cross flow mid-channel, and the profile is symmetric
    assert np.abs(u[1, 0, :, nx // 2]).max() <= 1e-4 * exact.max()
    assert np.abs(ux - ux[::-1]).max() <= 1e-6 * exact.max()


@pytest.mark.parametrize("name", ["mrt_table1", "fclb"])
def test_free_slip_top_halves_the_channel(name):
    """Physics of the free-slip faces: the pressure-driven channel of
    test_pressure_driven_channel_flow with a FREESLIP top instead of a wall
    is the lower half of a channel twice as high (no shear at the plane
    half a link above the last node): u(y) = G (y + 1/2)(2 ny - y - 1/2) /
    (2 nu) for the local gradient G, within 0.5 % mid-channel."""
    nx, ny, nz = 48, 9, 1
    nu, d_in, d_out = 0.1, 0.0015, -0.0015
    faces = [PR, PR, W, F, P, P]
    g = gpu_lattice(name, "f64", (nx, ny, nz), nu, faces=faces, face_u=[[0.0] * 3] * 6,
                    face_drho=[d_in, d_out, 0, 0, 0, 0])
    d0, u0 = synth.uniform_fields(nx, ny, nz)
    g.init_equilibrium(torch.from_numpy(d0), torch.from_numpy(u0))
    g.step(12000)
    d, u = (t.cpu().numpy() for t in g.macroscopic())
    dc = d[0, ny // 2, :]
    G = -(dc[nx // 2 + 5] - dc[nx // 2 - 5]) / 10 / 3.0
    y = np.arange(ny)
    ux = u[0, 0, :, nx // 2]
    exact = G * (y + 0.5) * (2 * ny - y - 0.5) / (2 * nu)
    err = np.abs(ux - exact).max() / exact.max()
    print(name, "half-channel error", err, flush=True)
    assert err <= 5e-3, err
    assert np.abs(u[1, 0, :, nx // 2]).max() <= 1e-4 * exact.max()


@pytest.mark.parametrize("name", NAMES)
def test_equilibrium_macroscopic_and_reductions(name):
    shape = (16, 8, 6)
    nx, ny, nz = shape
    _say("case init/macro/reduce", name)
    drho, u = synth.smooth_random_fields(nx, ny, nz, 0.05, 0.02, seed=5)
    g = gpu_lattice(name, "f64", shape, 0.01, cs=0.1)
    o = oracle_lattice(name, shape, 0.01, cs=0.1)
    g.init_equilibrium(torch.from_numpy(drho), torch.from_numpy(u))
    ref = o.init_equilibrium(drho, u)
    err = rel_err(g.populations().cpu().numpy(), ref)
    assert err <= 1e-12, err
    for k in (3, 1):  # odd and even parity readouts
        g.step(k)
        ref = o.run(ref, g.time - k, k)
        d_g, u_g = g.macroscopic()
        d_o, u_o = o.macroscopic(ref)
        ed = float(np.abs(d_g.cpu().numpy() - d_o).max())
        eu = float(np.abs(u_g.cpu().numpy() - u_o).max())
        assert ed <= 1e-14 and eu <= 1e-14, (ed, eu)
        rg, ro = np.array(g.reduce()), o.reduce(ref)
        scale = np.array([np.abs(d_o).sum(), *np.abs(u_o).sum(axis=(1, 2, 3)), ro[4]])
        assert np.all(np.abs(rg - ro) <= 1e-12 * scale + 1e-300)
    rho_full, _ = g.macroscopic(rho_mode=0)
    assert float(np.abs(rho_full.cpu().numpy() - 1 - d_g.cpu().numpy()).max()) <= 1e-15


def test_nonfinite_state_is_reported():
    g = gpu_lattice("fclb", "f32", (8, 8, 8), 0.01)
    f = np.zeros((27, 8, 8, 8))
    f[3, 2, 2, 2] = np.nan
    g.set_populations(torch.from_numpy(f))
    import paper_1206_0389_amd as Pk
    _, rc = Pk.reduce(g.h, check=False)
    assert rc == Pk.ENONFINITE


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_save_load_is_bit_identical(storage):
    _say("case save/load", storage)
    shape = (16, 8, 12)
    g = gpu_lattice("fclb", storage, shape, 0.01, faces=JET_FACES,
                    face_u=face_velocities(0.002), inlet=synth.jet_inlet(16, 8, 4.0, 0.05, 0.002),
                    amp=5e-4, seed=9)
    d, u = synth.smooth_random_fields(*shape, 0.05, 0.01, seed=2)
    g.init_equilibrium(torch.from_numpy(d), torch.from_numpy(u))
    g.step(3)  # odd parity snapshot
    buf, t, p = g.save_state()
    buf = buf.clone()
    g.step(5)
    a = g.populations().cpu().numpy()
    g.load_state(buf, t, p)
    g.step(5)
    b = g.populations().cpu().numpy()
    assert bool(np.array_equal(a, b))


def test_zero_steps_and_time():
    g = gpu_lattice("mrt_table1", "f32", (8, 4, 4), 0.01)
    g.set_populations(torch.zeros(19, 4, 4, 8, dtype=torch.float64), 7)
    g.step(0)
    assert g.time == 7
    g.step(3)
    assert g.time == 10


def test_c1_taylor_green_dhumieres_fp64_against_oracle():
    """32^3 periodic Taylor-Green, u0 = 0.05, nu = 0.005, C_S = 0.1, the
    d'Humieres rates, FP64, 100 steps: every population vs the oracle, and
    the energy decay at least the molecular rate -6 nu k0^2."""
    n, u0, nu, cs, steps = 32, 0.05, 0.005, 0.1, 100
    _say("case C1 TGV 32^3")
    drho, u = synth.taylor_green(n, u0)
    g = gpu_lattice("mrt_dhumieres", "f64", (n, n, n), nu, cs=cs)
    o = oracle_lattice("mrt_dhumieres", (n, n, n), nu, cs=cs)
    g.init_equilibrium(torch.from_numpy(drho), torch.from_numpy(u))
    ref = o.init_equilibrium(drho, u)
    E = [g.reduce()[4]]
    for _ in range(steps // 10):
        g.step(10)
        E.append(g.reduce()[4])
    ref = o.run(ref, 0, steps)
    err = rel_err(g.populations().cpu().numpy(), ref)
    assert err <= 1e-12, err
    assert E[-1] == pytest.approx(o.reduce(ref)[4], rel=1e-12)
    k0 = 2 * np.pi / n
    rate = np.log(E[-1] / E[5]) / 50.0
    assert rate < -6 * nu * k0 * k0 * 0.97


def test_bgk_as_mrt_with_equal_rates():
    """The BGK collision of Eq. (1) is the Table-1 MRT with every non-shear
    rate equal to the shear rate omega = 1/tau and C_S = 0 (the oracle's
    reduction is pinned in test_oracle_pins.py). Through the explicit rate
    override: against the oracle on the jet layout (FP64, 1-2-5 steps), and
    one periodic step against a direct numpy evaluation of Eq. (1) with
    Eq. (2) and pull streaming by array rolls."""
    nu = 0.02
    omega = 1.0 / (3.0 * nu + 0.5)
    errs = _run_pair("mrt_table1", "f64", (12, 10, 9), nu, [1, 2, 5], cs=0.0,
                     rates=[omega] * 4, faces=JET_FACES, face_u=face_velocities(0.002),
                     inlet=synth.jet_inlet(12, 10, 4.0, 0.05, 0.002), amp=5e-4, seed=3)
    assert max(errs) <= TOL["f64"], errs
    nx, ny, nz = 8, 6, 5
    f = synth.random_populations(19, (nz, ny, nx), amp=1e-2, seed=31)
    g = gpu_lattice("mrt_table1", "f64", (nx, ny, nz), nu, rates=[omega] * 4)
    g.set_populations(torch.from_numpy(f), 0)
    g.step(1)
    e, w, _ = oracle.stencil(19)
    d = f.sum(axis=0)
    j = np.einsum("ia,izyx->azyx", e.astype(np.float64), f)
    eu = np.einsum("ia,azyx->izyx", e.astype(np.float64), j)
    feq = w[:, None, None, None] * (d + 3 * eu + 4.5 * eu ** 2 - 1.5 * (j ** 2).sum(axis=0))
    post = f - omega * (f - feq)
    ref = np.stack([np.roll(post[i], shift=(e[i][2], e[i][1], e[i][0]), axis=(0, 1, 2))
                    for i in range(19)])
    assert rel_err(g.populations().cpu().numpy(), ref) <= 1e-13


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("faces", [None, "jet"])
def test_fp16_even_step_two_nodes_per_lane_is_the_one_node_step(name, faces):
    """The FP16 even step runs two x-neighbouring nodes per lane when the x
    extent is even and one node per lane otherwise. An even step touches only
    each node's own slots, so on a 32-wide lattice and a 33-wide one holding
    the same populations in x < 32 it must give the same values there (read
    back away from x = 0 and 31, whose natural populations come from the
    wrapped neighbours after the step), up to the final rounding to FP16: the
    compiler may fuse the last FP32 operation with the conversion (one
    rounding instead of two), so the two kernels may differ by one FP16 unit
    in the last place, no more."""
    Q = 19 if MODELS[name][0] == oracle.MRT19 else 27
    ny, nz = 8, 6
    f33 = synth.random_populations(Q, (nz, ny, 33), 1e-2, seed=17)
    iu, im = synth.jet_inlet(33, ny, 3.0, 0.05, 0.002)  # one inlet field for both
    out = {}
    for nx in (32, 33):
        kw = {}
        if faces == "jet":
            kw = dict(faces=JET_FACES, face_u=face_velocities(),
                      inlet=(np.ascontiguousarray(iu[..., :nx]),
                             np.ascontiguousarray(im[..., :nx])))
        _say("case fp16 even step", name, nx, faces)
        g = gpu_lattice(name, "f16", (nx, ny, nz), 0.02, cs=0.1, **kw)
        g.set_populations(torch.from_numpy(np.ascontiguousarray(f33[..., :nx])))
        g.step(1)
        out[nx] = g.populations().cpu().numpy()
    a, b = out[32][..., 1:31], out[33][..., 1:31]
    ulp = np.spacing(np.maximum(np.abs(a), np.abs(b)).astype(np.float16)).astype(np.float64)
    d = np.abs(a - b)
    print(name, faces, "values differing:", int((d > 0).sum()), "of", d.size, flush=True)
    assert np.all(d <= ulp), float((d / ulp).max())
