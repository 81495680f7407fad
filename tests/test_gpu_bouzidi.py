"""Curved walls on the GPU (lbm_set_links: Bouzidi's interpolated
bounce-back on links to solid nodes) against the oracle.

Fluid nodes are compared element by element after 1, 2 and 5 steps (both
in-place parities) with the bounds of test_gpu_parity.py (FP64 1e-12, FP32
4e-6, FP16 2e-3 per step of the largest population). Geometries come from a point
predicate with wall distances found by bisection (synth.link_distances): a
sphere in a periodic box (every q in (0, 1], links in all directions) and
the round nozzle tube of the jet workload at reduced size (walls, inlet,
outflow; inner and outer surfaces and the tube's end). The links change the
result (against the halfway rule); clearing them restores it exactly.
"""
import numpy as np
import pytest

import oracle
import synth
from lbm_cases import JET_FACES, MODELS, face_velocities, gpu_lattice
from test_oracle_bouzidi import E

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

TOL = {"f64": 1e-12, "f32": 4e-6, "f16": 2e-3}


def _sphere(nx, ny, nz, c, r):
    def inside(x, y, z):
        return (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2 < r * r
    return inside


def _case(kind, Q):
    if kind == "sphere_periodic":
        shape = (12, 11, 10)
        nx, ny, nz = shape
        body = _sphere(nx, ny, nz, (5.3, 4.8, 4.6), 3.1)
        kw = {}
    else:
        shape = (24, 24, 14)
        nx, ny, nz = shape
        body = synth.nozzle_tube(nx, ny, 8.0, 2.0, 6.0)
        kw = dict(faces=JET_FACES, face_u=face_velocities(0.002),
                  inlet=synth.jet_inlet(nx, ny, 8.0, 0.05, 0.002), amp=5e-4, seed=9)
    solid, nodes, q = synth.link_distances(body, (shape[2], shape[1], shape[0]), E[:Q])
    return shape, solid, nodes, q, kw


def _dense(q, nodes, Q, shape):
    nx, ny, nz = shape
    lq = np.zeros((Q, nx * ny * nz))
    lq[:, nodes] = q.T.astype(np.float64)
    return lq.reshape(Q, nz, ny, nx)


def _oracle(name, shape, solid, lq, kw):
    nx, ny, nz = shape
    okw = {}
    if kw:
        iu, im = kw["inlet"]
        okw = dict(faces=kw["faces"], face_u=kw["face_u"], inlet_u=iu, inlet_mask=im,
                   inlet_amp=kw["amp"], seed=kw["seed"])
    return oracle.Lattice(MODELS[name][0], nx, ny, nz, nu=0.02, cs_smag=0.1,
                          basis=MODELS[name][1], solid=solid, link_q=lq, **okw)


@pytest.mark.parametrize("name", ["fclb", "mrt_table1", "mrt_dhumieres"])
@pytest.mark.parametrize("kind", ["sphere_periodic", "nozzle_jet"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_links_against_oracle(name, kind, storage):
    Q = 19 if MODELS[name][0] == oracle.MRT19 else 27
    shape, solid, nodes, q, kw = _case(kind, Q)
    nx, ny, nz = shape
    print("case links", name, kind, storage, shape, "nodes", len(nodes), flush=True)
    f0 = synth.random_populations(Q, (nz, ny, nx), amp=1e-2, seed=29)
    f0 = f0.astype({"f64": np.float64, "f32": np.float32, "f16": np.float16}[storage])
    f0 = f0.astype(np.float64)
    g = gpu_lattice(name, storage, shape, 0.02, cs=0.1, **kw)
    g.set_solids(torch.from_numpy(solid))
    g.set_links(torch.from_numpy(nodes), torch.from_numpy(q))
    g.set_populations(torch.from_numpy(f0), 2)
    o = _oracle(name, shape, solid, _dense(q, nodes, Q, shape), kw)
    h = _oracle(name, shape, solid, None, kw)  # the halfway rule
    fluid = solid == 0
    ref, half, done = f0.copy(), f0.copy(), 0
    for k in (1, 2, 5):
        g.step(k - done)
        ref = o.run(ref, 2 + done, k - done)
        half = h.run(half, 2 + done, k - done)
        done = k
        got = g.populations().cpu().numpy()
        scale = np.abs(ref[:, fluid]).max()
        err = float(np.abs(got[:, fluid] - ref[:, fluid]).max() / scale)
        assert err <= k * TOL[storage], (k, err)
        assert np.abs(half[:, fluid] - ref[:, fluid]).max() / scale > 1e-4
    print(name, kind, storage, "after 5 steps", err, flush=True)


def test_links_errors_and_clearing():
    import paper_1206_0389_amd as Pk
    name, storage = "fclb", "f64"
    Q = 27
    shape, solid, nodes, q, kw = _case("sphere_periodic", Q)
    nx, ny, nz = shape
    g = gpu_lattice(name, storage, shape, 0.02, cs=0.1)
    with pytest.raises(Pk.LbmError):  # no solids yet
        g.set_links(torch.from_numpy(nodes), torch.from_numpy(q))
    with pytest.raises(ValueError):
        g.set_links(torch.from_numpy(nodes), torch.from_numpy(q[:, :19].copy()))
    g.set_solids(torch.from_numpy(solid))
    g.set_links(torch.from_numpy(nodes), torch.from_numpy(q))
    g.set_links(None)  # cleared: the halfway rule again
    f0 = synth.random_populations(Q, (nz, ny, nx), amp=1e-2, seed=31)
    g.set_populations(torch.from_numpy(f0))
    g.step(3)
    ref = _oracle(name, shape, solid, None, {}).run(f0, 0, 3)
    fluid = solid == 0
    got = g.populations().cpu().numpy()
    assert np.abs(got[:, fluid] - ref[:, fluid]).max() <= 1e-12 * np.abs(ref).max()
    # new solids clear the links too
    g2 = gpu_lattice(name, storage, shape, 0.02, cs=0.1)
    g2.set_solids(torch.from_numpy(solid))
    g2.set_links(torch.from_numpy(nodes), torch.from_numpy(q))
    g2.set_solids(torch.from_numpy(solid))
    g2.set_populations(torch.from_numpy(f0))
    g2.step(3)
    got2 = g2.populations().cpu().numpy()
    assert np.abs(got2[:, fluid] - ref[:, fluid]).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["fclb", "mrt_table1"])
@pytest.mark.parametrize("q", [0.2, 0.8])
def test_couette_no_slip_at_the_wall_distance(name, q):
    """Physics on the GPU, at any size: steady Couette flow between a solid
    layer whose wall lies a fraction q of a link from the first fluid plane
    (curved-wall links) and a moving WALL face is linear with its no-slip
    point at the wall (the oracle's pin, here on the GPU path)."""
    Q = 19 if MODELS[name][0] == oracle.MRT19 else 27
    nx, ny, nz = 1, 10, 1
    U = 1e-3
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 0, :] = 1
    fu = [[0.0] * 3 for _ in range(6)]
    fu[3] = [U, 0.0, 0.0]
    import paper_1206_0389_amd as Pk
    g = gpu_lattice(name, "f64", (nx, ny, nz), 1.0 / 6.0,
                    faces=[Pk.PERIODIC, Pk.PERIODIC, Pk.WALL, Pk.WALL, Pk.PERIODIC, Pk.PERIODIC],
                    face_u=fu)
    g.set_solids(torch.from_numpy(solid))
    nodes = np.array([1 * nx], dtype=np.int32)  # the fluid node at y = 1
    qq = np.zeros((1, Q), np.float32)
    for k in range(Q):
        if E[k][1] == -1:
            qq[0, k] = q
    g.set_links(torch.from_numpy(nodes), torch.from_numpy(qq))
    d0, u0 = synth.uniform_fields(nx, ny, nz)
    g.init_equilibrium(torch.from_numpy(d0), torch.from_numpy(u0))
    g.step(2500)
    _, u = g.macroscopic()
    ux = u[0, 0, 1:, 0].cpu().numpy()
    y = np.arange(1, ny, dtype=float)
    y_w = 1.0 - float(np.float32(q))
    exact = U * (y - y_w) / (ny - 0.5 - y_w)
    err = np.abs(ux - exact).max() / exact.max()
    print(name, q, "Couette error", err, flush=True)
    assert err <= 1e-9, err
