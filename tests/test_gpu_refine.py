"""Two-level refined lattice on the GPU vs the FP64 oracle, through the C ABI.

FP64 storage: both levels element by element to 1e-12 relative (rounding
order only). FP32 storage: a few units of FP32 rounding per step. On the
fine level the ghost nodes are interface scratch (the library prepares the
next substep's ghosts ahead of time), so they are left out of the
comparison; every fluid node next to a ghost pulls from it, so a wrong ghost
value shows up in the fluid nodes one substep later.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
pytest.skip("the GPU refined lattice still has the two-level vertex-centred layout; the "
            "oracle moved to cell-centred multi-level nesting", allow_module_level=True)

import oracle  # noqa: E402
import synth  # noqa: E402
from lbm_cases import MODELS, REFINED_MODELS, rel_err  # noqa: E402

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

W, I, O, P = oracle.WALL, oracle.INLET, oracle.OUTFLOW, oracle.PERIODIC
FACE_U = [[0.0, 0.001, 0.002], [0.0, 0.0, 0.002], [0.001, 0.0, 0.002], [0.0, 0.0, 0.002],
          [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]]


def _pair(name, storage, jet=True, nu=0.02, cs=0.1, faces=None, face_drho=None):
    import paper_1206_0389_amd as Pk
    model, basis = MODELS[name]
    print("case refine", name, storage, "jet" if jet else "slab", faces, flush=True)
    if jet:
        n, nz, B, mask = _jet_case(model)
        nx = ny = n
        faces = faces or [W, W, W, W, I, O]
        iu, im = synth.jet_inlet(n, n, 4.0, 0.05, 0.002)
        fiu, fim = synth.jet_inlet(2 * n, 2 * n, 8.0, 0.05, 0.002)
    else:
        nx = ny = B = 4
        nz = 64
        mask = np.zeros((16, 1, 1), dtype=np.uint8)
        mask[6:10] = 1
        faces = faces or [P] * 6
        iu = im = fiu = fim = None
    g = Pk.RefinedLattice(model=model, storage=storage, shape=(nx, ny, nz), nu=nu, cs_smag=cs,
                          mrt_basis=basis, block=B, mask=mask, faces=faces, face_u=FACE_U,
                          inlet_u=None if iu is None else torch.from_numpy(iu),
                          inlet_mask=None if im is None else torch.from_numpy(im),
                          fine_inlet_u=None if fiu is None else torch.from_numpy(fiu),
                          fine_inlet_mask=None if fim is None else torch.from_numpy(fim),
                          inlet_amp=5e-4, seed=11, face_drho=face_drho)
    c = oracle.Lattice(model, nx, ny, nz, nu=nu, cs_smag=cs, basis=basis, faces=faces,
                       face_u=FACE_U, inlet_u=iu, inlet_mask=im, inlet_amp=5e-4, seed=11,
                       face_drho=face_drho)
    R = oracle.Refined(c, B, mask, fiu, fim)
    assert g.fine_lo == R.lo and g.fine_dims == R.M
    assert g.counts == R.counts
    return g, R, c


def _oracle_reduce(R, c, fc, ff):
    ct, ft = R.types()
    out = np.zeros(5)
    fl = R.fine_lattice()
    for lat, f, types, want, w in ((c, fc, ct, 0, 1.0), (fl, ff, ft, 1, 0.125)):
        d, u = lat.macroscopic(f)
        rho = 1.0 if lat.model == oracle.MRT19 else 1.0 + d
        j = u * rho
        m = types == want
        out[0] += w * d[m].sum()
        for a in range(3):
            out[1 + a] += w * j[a][m].sum()
        out[4] += w * (0.5 * (j * j).sum(axis=0) / rho)[m].sum() if np.ndim(rho) else \
            w * (0.5 * (j * j).sum(axis=0))[m].sum()
    return out


@pytest.mark.parametrize("name", REFINED_MODELS)
@pytest.mark.parametrize("jet", [True, False, "slip_pressure", "slab_slip_pressure"])
def test_refined_step_parity_fp64(name, jet):
    F, PR = oracle.FREESLIP, oracle.PRESSURE
    if jet == "slip_pressure":  # a free-slip top and a fixed-pressure outlet (coarse level)
        g, R, c = _pair(name, "f64", jet=True, faces=[W, W, W, F, I, PR],
                        face_drho=[0, 0, 0, 0, 0, -0.002])
    elif jet == "slab_slip_pressure":  # the fine slab spans free-slip x and pressure y faces
        g, R, c = _pair(name, "f64", jet=False, faces=[F, F, PR, PR, P, P],
                        face_drho=[0, 0, 0.001, -0.001, 0, 0])
    else:
        g, R, c = _pair(name, "f64", jet=jet)
    Q = c.Q
    fc = synth.random_populations(Q, c.shape, 1e-2, seed=1)
    ff = synth.random_populations(Q, R.fine_shape, 1e-2, seed=2)
    g.set_populations(0, torch.from_numpy(fc), 4)
    g.set_populations(1, torch.from_numpy(ff), 4)
    oc, of = fc, ff
    keep = R.types()[1] != 2
    for k in range(3):
        g.step(1)
        oc, of = R.run(oc, of, 4 + k, 1)
        ec = rel_err(g.populations(0).cpu().numpy(), oc)
        ef = rel_err(g.populations(1).cpu().numpy()[:, keep], of[:, keep])
        assert ec <= 1e-12 and ef <= 1e-12, (k, ec, ef)
    rg = np.array(g.reduce())
    ro = _oracle_reduce(R, c, oc, of)
    scale = np.abs(ro).max() + 1.0
    assert float(np.abs(rg - ro).max()) <= 1e-12 * scale


@pytest.mark.parametrize("name", ["fclb", "mrt_table1"])
def test_refined_fp32_within_tolerance(name):
    g, R, c = _pair(name, "f32", jet=True)
    fc = synth.random_populations(c.Q, c.shape, 1e-2, seed=3)
    ff = synth.random_populations(c.Q, R.fine_shape, 1e-2, seed=4)
    g.set_populations(0, torch.from_numpy(fc))
    g.set_populations(1, torch.from_numpy(ff))
    g.step(2)
    oc, of = R.run(fc, ff, 0, 2)
    keep = R.types()[1] != 2
    ec = rel_err(g.populations(0).cpu().numpy(), oc)
    ef = rel_err(g.populations(1).cpu().numpy()[:, keep], of[:, keep])
    assert ec <= 1e-5 and ef <= 1e-5, (ec, ef)


@pytest.mark.parametrize("name", REFINED_MODELS)
def test_refined_uniform_flow_and_readouts(name):
    """Uniform co-flow through walls moving with it, a uniform inlet and the
    outflow stays exactly uniform on both levels; macroscopic readouts of
    each level return it."""
    import paper_1206_0389_amd as Pk
    model, basis = MODELS[name]
    n, nz, B, mask = _jet_case(model)
    u0 = 0.002
    iu = np.zeros((3, n, n))
    iu[2] = u0
    fiu = np.zeros((3, 2 * n, 2 * n))
    fiu[2] = u0
    fu = [[0, 0, u0]] * 4 + [[0, 0, 0]] * 2
    g = Pk.RefinedLattice(model=model, storage="f64", shape=(n, n, nz), nu=0.02, cs_smag=0.1,
                          mrt_basis=basis, block=B, mask=mask, faces=[W, W, W, W, I, O],
                          face_u=fu, inlet_u=torch.from_numpy(iu),
                          fine_inlet_u=torch.from_numpy(fiu))
    for level in (0, 1):
        d, u = synth.uniform_fields(*g.shape3(level)[::-1], u=(0, 0, u0))
        g.init_equilibrium(level, torch.from_numpy(d), torch.from_numpy(u))
    f0 = [g.populations(level).cpu().numpy() for level in (0, 1)]
    g.step(5)
    ct, ft = oracle.Refined(oracle.Lattice(model, n, n, nz, nu=0.02,
                                           faces=[W, W, W, W, I, O], face_u=fu, inlet_u=iu),
                            B, mask, fiu).types()
    f1 = [g.populations(level).cpu().numpy() for level in (0, 1)]
    assert float(np.abs((f1[0] - f0[0])[:, ct != 2]).max()) < 1e-15
    assert float(np.abs((f1[1] - f0[1])[:, ft == 1]).max()) < 1e-15
    for level in (0, 1):
        d, u = g.macroscopic(level)
        types = ct if level == 0 else ft
        live = types != 2 if level == 0 else types == 1
        assert float(np.abs(u[2].cpu().numpy()[live] - u0).max()) < 1e-15


@pytest.mark.parametrize("name", ["fclb", "mrt_table1"])
def test_refined_with_empty_mask_is_the_coarse_lattice(name):
    """No refined block: no fine level, no ghosts, no covered nodes; the
    coarse level steps exactly as the oracle's uniform lattice."""
    import paper_1206_0389_amd as Pk
    model, basis = MODELS[name]
    n, nz, B = 16, 32, 4
    mask = np.zeros((nz // B, n // B, n // B), dtype=np.uint8)
    iu, im = synth.jet_inlet(n, n, 4.0, 0.05, 0.002)
    fiu, fim = synth.jet_inlet(2 * n, 2 * n, 8.0, 0.05, 0.002)
    faces = [W, W, W, W, I, O]
    g = Pk.RefinedLattice(model=model, storage="f64", shape=(n, n, nz), nu=0.02, cs_smag=0.1,
                          mrt_basis=basis, block=B, mask=mask, faces=faces, face_u=FACE_U,
                          inlet_u=torch.from_numpy(iu), inlet_mask=torch.from_numpy(im),
                          fine_inlet_u=torch.from_numpy(fiu), fine_inlet_mask=torch.from_numpy(fim),
                          inlet_amp=5e-4, seed=11)
    assert g.counts["fluid"] == 0 and g.counts["ghost"] == 0 and g.counts["covered"] == 0
    c = oracle.Lattice(model, n, n, nz, nu=0.02, cs_smag=0.1, basis=basis, faces=faces,
                       face_u=FACE_U, inlet_u=iu, inlet_mask=im, inlet_amp=5e-4, seed=11)
    fc = synth.random_populations(c.Q, c.shape, 1e-2, seed=5)
    g.set_populations(0, torch.from_numpy(fc), 2)
    g.step(3)
    # post-collision (refined storage) vs the oracle's uniform pre-collision
    # run: compare through the refined oracle, pinned equal to the uniform
    # lattice for an empty mask
    R = oracle.Refined(c, B, mask, fiu, fim)
    oc, _ = R.run(fc, np.zeros((c.Q,) + R.fine_shape), 2, 3)
    err = rel_err(g.populations(0).cpu().numpy(), oc)
    assert err <= 1e-12, err
