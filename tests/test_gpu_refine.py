"""Refined lattice (nested levels) on the GPU vs the FP64 oracle, through the
C ABI.

FP64 storage: every level element by element to 1e-12 relative (rounding
order only). FP32 storage: a few units of FP32 rounding per step. Compared
nodes: fluid and band nodes, and the covered nodes they read (the library
injects into those only: no other covered node is read); ghost nodes hold interface values
prepared ahead for the next substep, so they are left out, but every fluid
node next to a ghost pulls from it, so a wrong ghost value shows up in the
fluid nodes one substep later. The node types of every level are compared
with the oracle's geometry exactly.
"""
import numpy as np
import pytest

import oracle
import synth
from lbm_cases import (MODELS, REFINED_CASES as CASES, REFINED_FACE_U as FACE_U,  # noqa: F401
                       REFINED_MODELS, REFINED_NU, jet_map, read_covered, refined_jet_geometry,
                       rel_err, slab_map)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

W, I, O, P = oracle.WALL, oracle.INLET, oracle.OUTFLOW, oracle.PERIODIC
F, PR = oracle.FREESLIP, oracle.PRESSURE


def make_pair(name, storage, case, nu=0.02, cs=0.1, solids=None, links=None):
    import paper_1206_0389_amd as Pk
    model, basis = MODELS[name]
    levels, jet, faces, drho = CASES[case]
    nu = REFINED_NU.get(case, nu)
    print("case refine", name, storage, case, "nu", nu, flush=True)
    if jet:
        n, nz, B, m = refined_jet_geometry(case)
        nx = ny = n
        iu, im = synth.jet_inlet(n, n, 4.0, 0.05, 0.002)
        lius, lims = [None], [None]
        for l in range(1, levels):
            a, b = synth.jet_inlet(n << l, n << l, 4.0 * 2 ** l, 0.05, 0.002)
            lius.append(a)
            lims.append(b)
    else:
        nx = ny = B = 4
        nz = 64
        m = slab_map(levels)
        iu = im = None
        lius = lims = None
    g = Pk.RefinedLattice(
        model=model, storage=storage, shape=(nx, ny, nz), nu=nu, cs_smag=cs, mrt_basis=basis,
        block=B, level_map=m, nlevels=levels, faces=faces, face_u=FACE_U,
        inlet_u=None if iu is None else torch.from_numpy(iu),
        inlet_mask=None if im is None else torch.from_numpy(im),
        level_inlet_u=None if lius is None else [None] + [torch.from_numpy(a) for a in lius[1:]],
        level_inlet_mask=None if lims is None else [None] + [torch.from_numpy(a)
                                                             for a in lims[1:]],
        inlet_amp=5e-4, seed=11, face_drho=drho, solids=solids, links=links)
    c = oracle.Lattice(model, nx, ny, nz, nu=nu, cs_smag=cs, basis=basis, faces=faces,
                       face_u=FACE_U, inlet_u=iu, inlet_mask=im, inlet_amp=5e-4, seed=11,
                       face_drho=drho)
    lq = None
    if links is not None:
        lq = []
        for l, lk in enumerate(links):
            if lk is None:
                lq.append(None)
                continue
            nxl, nyl, nzl = nx << l, ny << l, nz << l
            a = np.zeros((c.Q, nzl * nyl * nxl))
            a[:, lk[0]] = np.asarray(lk[1], np.float64).T
            lq.append(a.reshape(c.Q, nzl, nyl, nxl))
    R = oracle.Refined(c, B, m, levels, inlet_u=lius, inlet_mask=lims, solid=solids, link_q=lq)
    for l in range(levels):
        assert np.array_equal(g.types(l), g.to_box(l, R.types(l))), l
    return g, R


def compared(g, R, l, faces):
    """Box mask of the nodes compared on level l: fluid and band nodes and
    the covered nodes they read."""
    keep = np.isin(g.types(l), (1, 2))
    if l + 1 < R.L:
        keep |= g.to_box(l, read_covered(R.types(l), faces)).astype(bool)
    return keep


def seed_states(g, R, seed):
    fs = []
    for l in range(R.L):
        f = synth.random_populations(R.Q, R.levels[l]["shape"], 1e-2, seed=seed + l)
        R.set_state(l, f)
        fs.append(f)
    for l in range(R.L):
        g.set_populations(l, torch.from_numpy(g.to_box(l, fs[l])), 4)


def level_errors(g, R):
    out = []
    faces = [int(R.coarse.p.face_type[k]) for k in range(6)]
    for l in range(R.L):
        keep = compared(g, R, l, faces)
        got = g.populations(l).cpu().numpy()[:, keep]
        want = g.to_box(l, R.state(l))[:, keep]
        out.append(rel_err(got, want))
    return out


@pytest.mark.parametrize("name", REFINED_MODELS)
@pytest.mark.parametrize("case", list(CASES))
def test_refined_step_parity_fp64(name, case):
    g, R = make_pair(name, "f64", case)
    seed_states(g, R, 1)
    for k in range(3):
        g.step(1)
        R.run(4 + k, 1)
        errs = level_errors(g, R)
        assert max(errs) <= 1e-12, (k, errs)
    rg = np.array(g.reduce())
    ro = R.reduce()
    scale = np.abs(ro).max() + 1.0
    assert float(np.abs(rg - ro).max()) <= 1e-12 * scale


def _tube(n, diam, length, level):
    """The nozzle tube (inner radius D/2, wall 2 coarse nodes) on level l's
    whole domain, from the same point predicate at that resolution."""
    s = 2 ** level
    return synth.nozzle_tube(n * s, n * s, diam * s, 2.0 * s, length * s)


@pytest.mark.parametrize("name", ["fclb", "mrt_table1", "mrt_dhumieres"])
@pytest.mark.parametrize("curved", [False, True])
def test_refined_nozzle_inside_the_fine_level_fp64(name, curved):
    """The paper's nozzle sits inside the refined region (Section 3): a solid
    tube on level 1 of the two-level jet, halfway walls or curved links."""
    n, nz = 24, 32
    model, _ = MODELS[name]
    Q = 19 if model == oracle.MRT19 else 27
    body = _tube(n, 4.0, 3.0, 1)
    dirs = oracle.stencil(Q)[0].tolist()
    sm, nodes, q = synth.link_distances(body, (2 * nz, 2 * n, 2 * n), dirs)
    solids = [None, sm]
    links = [None, (nodes, q)] if curved else None
    g, R = make_pair(name, "f64", "jet2wide", solids=solids, links=links)
    assert g.levels[1]["counts"]["solid"] > 0
    seed_states(g, R, 7)
    for k in range(3):
        g.step(1)
        R.run(4 + k, 1)
        errs = level_errors(g, R)
        assert max(errs) <= 1e-12, (k, errs)


def test_refined_solids_on_the_interface_are_refused():
    import paper_1206_0389_amd as Pk
    n, nz = 16, 32
    sm = np.zeros((2 * nz, 2 * n, 2 * n), dtype=np.uint8)
    sm[4:6, 6:8, :] = 1  # a bar through the level-1 ghost layer
    with pytest.raises(Pk.LbmError):
        make_pair("fclb", "f64", "jet2", solids=[None, sm])


@pytest.mark.parametrize("name", ["fclb", "mrt_table1"])
@pytest.mark.parametrize("case", ["jet2", "jet3"])
def test_refined_fp32_within_tolerance(name, case):
    g, R = make_pair(name, "f32", case)
    seed_states(g, R, 3)
    g.step(2)
    R.run(4, 2)
    errs = level_errors(g, R)
    assert max(errs) <= 1e-5, errs


@pytest.mark.parametrize("name", ["fclb", "mrt_table1"])
@pytest.mark.parametrize("case", ["jet2", "jet3"])
def test_refined_fp16_within_tolerance(name, case):
    """FP16 storage of the deviations (FP32 arithmetic, FP32 interface
    buffers): each stored value carries 2^-11 relative rounding, a few units
    of it per step against the largest deviation."""
    g, R = make_pair(name, "f16", case)
    seed_states(g, R, 3)
    g.step(2)
    R.run(4, 2)
    errs = level_errors(g, R)
    assert max(errs) <= 3e-3, errs


@pytest.mark.parametrize("name", REFINED_MODELS)
@pytest.mark.parametrize("levels", [2, 3])
def test_refined_uniform_flow_and_readouts(name, levels):
    """Uniform co-flow through walls moving with it, a uniform inlet and the
    outflow stays exactly uniform on every level; macroscopic readouts of
    each level return it."""
    import paper_1206_0389_amd as Pk
    model, basis = MODELS[name]
    n, nz, B = (16 if levels == 2 else 24), 32, 4
    m = jet_map(n, nz, B, levels)
    u0 = 0.002
    iu = np.zeros((3, n, n))
    iu[2] = u0
    lius = [None] + [torch.from_numpy(np.stack([np.zeros((n << l, n << l))] * 2 +
                                               [np.full((n << l, n << l), u0)]))
                     for l in range(1, levels)]
    fu = [[0, 0, u0]] * 4 + [[0, 0, 0]] * 2
    g = Pk.RefinedLattice(model=model, storage="f64", shape=(n, n, nz), nu=0.02, cs_smag=0.1,
                          mrt_basis=basis, block=B, level_map=m, faces=[W, W, W, W, I, O],
                          face_u=fu, inlet_u=torch.from_numpy(iu), level_inlet_u=lius)
    for level in range(levels):
        d, u = synth.uniform_fields(*g.shape3(level)[::-1], u=(0, 0, u0))
        g.init_equilibrium(level, torch.from_numpy(d), torch.from_numpy(u))
    f0 = [g.populations(level).cpu().numpy() for level in range(levels)]
    g.step(4)
    for level in range(levels):
        live = np.isin(g.types(level), (1, 2))
        f1 = g.populations(level).cpu().numpy()
        # the post-collision uniform state is the equilibrium itself
        assert float(np.abs((f1 - f0[level])[:, live]).max()) < 1e-15, level
        d, u = g.macroscopic(level)
        assert float(np.abs(u[2].cpu().numpy()[live] - u0).max()) < 1e-15


@pytest.mark.parametrize("name", ["fclb", "mrt_table1"])
def test_refined_with_nothing_refined_is_the_coarse_lattice(name):
    """No refined block: one level stepping as the oracle (pinned equal to
    the uniform lattice when nothing is refined)."""
    import paper_1206_0389_amd as Pk
    model, basis = MODELS[name]
    n, nz, B = 16, 32, 4
    m = np.zeros((nz // B, n // B, n // B), dtype=np.uint8)
    iu, im = synth.jet_inlet(n, n, 4.0, 0.05, 0.002)
    faces = [W, W, W, W, I, O]
    g = Pk.RefinedLattice(model=model, storage="f64", shape=(n, n, nz), nu=0.02, cs_smag=0.1,
                          mrt_basis=basis, block=B, level_map=m, nlevels=1, faces=faces,
                          face_u=FACE_U, inlet_u=torch.from_numpy(iu),
                          inlet_mask=torch.from_numpy(im), inlet_amp=5e-4, seed=11)
    c = oracle.Lattice(model, n, n, nz, nu=0.02, cs_smag=0.1, basis=basis, faces=faces,
                       face_u=FACE_U, inlet_u=iu, inlet_mask=im, inlet_amp=5e-4, seed=11)
    R = oracle.Refined(c, B, m, 1)
    fc = synth.random_populations(c.Q, c.shape, 1e-2, seed=5)
    R.set_state(0, fc)
    g.set_populations(0, torch.from_numpy(g.to_box(0, fc)), 2)
    g.step(3)
    R.run(2, 3)
    live = g.types(0) == 1
    err = rel_err(g.populations(0).cpu().numpy()[:, live], g.to_box(0, R.state(0))[:, live])
    assert err <= 1e-12, err
