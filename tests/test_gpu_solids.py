"""Interior solid nodes on the GPU (lbm_set_solids) against the oracle.

Fluid nodes are compared element by element after 1, 2 and 5 steps with the
bounds of test_gpu_parity.py (FP64 1e-12, FP32 4e-6 per step of the largest
population); solid nodes read back as zeros and as the rest state. Layouts:
an obstacle block in a periodic box, and a nozzle plate with a hole on the
inlet side of a jet (walls, inlet, outflow). A channel bounded by solid
layers runs the general kernel and matches the same channel bounded by WALL
faces, which runs the wall-row kernel.
"""
import numpy as np
import pytest

import oracle
import synth
from lbm_cases import JET_FACES, MODELS, P, W, face_velocities, gpu_lattice

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

TOL = {"f64": 1e-12, "f32": 4e-6}


def _layout(kind):
    if kind == "periodic_obstacle":
        shape = (12, 10, 9)
        nx, ny, nz = shape
        solid = np.zeros((nz, ny, nx), np.uint8)
        solid[3:6, 4:7, 2:9] = 1
        return shape, solid, {}
    shape = (16, 12, 10)
    nx, ny, nz = shape
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[0:3] = 1
    solid[0:3, 3:9, 5:11] = 0  # the hole over the inlet disk
    kw = dict(faces=JET_FACES, face_u=face_velocities(0.002),
              inlet=synth.jet_inlet(nx, ny, 6.0, 0.05, 0.002), amp=5e-4, seed=9)
    return shape, solid, kw


@pytest.mark.parametrize("name", ["fclb", "mrt_table1"])
@pytest.mark.parametrize("kind", ["periodic_obstacle", "jet_nozzle_plate"])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_solids_against_oracle(name, kind, storage):
    shape, solid, kw = _layout(kind)
    nx, ny, nz = shape
    Q = 19 if MODELS[name][0] == oracle.MRT19 else 27
    print("case solids", name, kind, storage, shape, flush=True)
    f0 = synth.random_populations(Q, (nz, ny, nx), amp=1e-2, seed=23)
    f0 = f0.astype(np.float32 if storage == "f32" else np.float64).astype(np.float64)
    g = gpu_lattice(name, storage, shape, 0.02, cs=0.1, **kw)
    g.set_solids(torch.from_numpy(solid))
    g.set_populations(torch.from_numpy(f0), 2)
    o = oracle.Lattice(MODELS[name][0], nx, ny, nz, nu=0.02, cs_smag=0.1,
                       basis=MODELS[name][1], solid=solid, **_oracle_kw(kw))
    fluid = solid == 0
    ref, done = f0.copy(), 0
    for k in (1, 2, 5):
        g.step(k - done)
        ref = o.run(ref, 2 + done, k - done)
        done = k
        got = g.populations().cpu().numpy()
        err = float(np.abs(got[:, fluid] - ref[:, fluid]).max() / np.abs(ref[:, fluid]).max())
        assert err <= k * TOL[storage], (k, err)
        assert np.all(got[:, ~fluid] == 0.0)
    drho, u = (t.cpu().numpy() for t in g.macroscopic())
    assert np.all(drho[~fluid] == 0.0) and np.all(u[:, ~fluid] == 0.0)
    print(name, kind, storage, "after 5 steps", err, flush=True)


def _oracle_kw(kw):
    if not kw:
        return {}
    iu, im = kw["inlet"]
    return dict(faces=kw["faces"], face_u=kw["face_u"], inlet_u=iu, inlet_mask=im,
                inlet_amp=kw["amp"], seed=kw["seed"])


@pytest.mark.parametrize("name", ["fclb", "mrt_table1"])
def test_solid_layers_match_wall_faces(name):
    nx, ny, nz = 16, 9, 6
    Q = 19 if MODELS[name][0] == oracle.MRT19 else 27
    print("case solid channel", name, flush=True)
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 0] = 1
    solid[:, ny - 1] = 1
    f0 = synth.random_populations(Q, (nz, ny, nx), amp=1e-2, seed=29)
    a = gpu_lattice(name, "f64", (nx, ny, nz), 0.02, cs=0.1)
    a.set_solids(torch.from_numpy(solid))
    a.set_populations(torch.from_numpy(f0), 0)
    b = gpu_lattice(name, "f64", (nx, ny - 2, nz), 0.02, cs=0.1, faces=[P, P, W, W, P, P],
                    face_u=[[0.0, 0.0, 0.0]] * 6)
    b.set_populations(torch.from_numpy(np.ascontiguousarray(f0[:, :, 1:ny - 1])), 0)
    for _ in range(5):
        a.step(1)
        b.step(1)
        fa = a.populations().cpu().numpy()[:, :, 1:ny - 1]
        fb = b.populations().cpu().numpy()
        assert float(np.abs(fa - fb).max()) <= 1e-13 * float(np.abs(fb).max())


def test_solid_errors_and_clearing():
    import paper_1206_0389_amd as Pk
    nx, ny, nz = 16, 12, 10
    print("case solid errors", flush=True)
    kw = dict(faces=JET_FACES, face_u=face_velocities(0.002),
              inlet=synth.jet_inlet(nx, ny, 6.0, 0.05, 0.002), amp=5e-4, seed=9)
    g = gpu_lattice("fclb", "f32", (nx, ny, nz), 0.02, **kw)
    bad = np.zeros((nz, ny, nx), np.uint8)
    bad[nz - 1, 5, 5] = 1  # on the outflow plane
    with pytest.raises(Pk.LbmError):
        g.set_solids(torch.from_numpy(bad))
    ok = np.zeros_like(bad)
    ok[4, 5, 5] = 1
    g.set_solids(torch.from_numpy(ok))
    lam = torch.zeros((27, nz, ny, nx), dtype=torch.float32, device="cuda")
    with pytest.raises(Pk.LbmError):
        g.step_record(lam)
    # clearing restores the plain lattice: same result as one never given solids
    g.set_solids(None)
    h = gpu_lattice("fclb", "f32", (nx, ny, nz), 0.02, **kw)
    f0 = torch.from_numpy(synth.random_populations(27, (nz, ny, nx), amp=1e-2, seed=2))
    g.set_populations(f0, 0)
    h.set_populations(f0, 0)
    g.step(3)
    h.step(3)
    assert torch.equal(g.populations(), h.populations())
