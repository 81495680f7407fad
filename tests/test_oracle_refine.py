"""Pins of the oracle's nested time refinement (hierarchical block grid).

The paper cites the refinement method (Yu et al.) without printing its
formulas; these tests pin the oracle's reading against facts that hold
independently of the implementation: the nesting geometry, polynomial
exactness of the space and time interpolants at the cell-centred child
positions, the Chapman-Enskog scaling of every moment group's
non-equilibrium part between levels (with and without the Smagorinsky eddy
viscosity), exact preservation of uniform flow, steady Couette flow whose
refined levels see the walls where the coarse level does, reduction to the
uniform lattice (nothing refined, or everything refined), and the viscous
decay of a shear wave crossing one and two nested interfaces.
"""
import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import _DH_ROWS, _T1_ROWS, _typed_basis

W, I, O, P = oracle.WALL, oracle.INLET, oracle.OUTFLOW, oracle.PERIODIC
MODELS = [oracle.MRT19, oracle.FCLB27]


def _slab_map(nz, B, ranges):
    """Periodic 1 x 1 x (nz/B) block map; ranges: [(lo, hi, level), ...]."""
    m = np.zeros((nz // B, 1, 1), dtype=np.uint8)
    for lo, hi, lev in ranges:
        m[lo:hi] = np.maximum(m[lo:hi], lev)
    return m


def _jet_map(n, nz, B, levels=2):
    """Blocks of the first four z layers within a radius of the axis refined
    once (two levels: 16 x 16 x 32, radius^2 40; three levels: 24 x 24 x 32,
    the centre 4 x 4 blocks, and its inner 2 x 2 blocks of the first two
    layers refined again)."""
    m = np.zeros((nz // B, n // B, n // B), dtype=np.uint8)
    r2 = 40.0 if levels == 2 else 72.0
    for bz in range(4):
        for by in range(n // B):
            for bx in range(n // B):
                cx, cy = (bx + 0.5) * B - n / 2, (by + 0.5) * B - n / 2
                if cx * cx + cy * cy <= r2:
                    m[bz, by, bx] = 1
    if levels == 3:
        h = n // B // 2
        m[0:2, h - 1:h + 1, h - 1:h + 1] = 2
    return m


def _jet_inlets(n, L, diam=4.0, u=0.05, co=0.002):
    ius, ims = [None], [None]
    for l in range(1, L):
        iu, im = synth.jet_inlet(n << l, n << l, diam * 2 ** l, u, co)
        ius.append(iu)
        ims.append(im)
    return ius, ims


def _jet(model, levels=2, nu=0.02, cs=0.1):
    n, nz, B = (16 if levels == 2 else 24), 32, 4
    m = _jet_map(n, nz, B, levels)
    iu, im = synth.jet_inlet(n, n, 4.0, 0.05, 0.002)
    fu = [[0, 0, 0.002]] * 4 + [[0, 0, 0]] * 2
    c = oracle.Lattice(model, n, n, nz, nu=nu, cs_smag=cs, faces=[W, W, W, W, I, O],
                       face_u=fu, inlet_u=iu, inlet_mask=im, inlet_amp=5e-4, seed=9)
    ius, ims = _jet_inlets(n, levels)
    return oracle.Refined(c, B, m, levels, inlet_u=ius, inlet_mask=ims), m


@pytest.mark.parametrize("levels", [2, 3])
def test_geometry_invariants(levels):
    R, m = _jet(oracle.FCLB27, levels)
    B = R.B
    for l in range(levels):
        t = R.types(l)
        c = R.levels[l]["counts"]
        inside = int((m >= l).sum()) * (B << l) ** 3
        assert c["fluid"] + c["band"] + c["covered"] + c["solid"] == inside
        if l + 1 < levels:
            # the next level's region is exactly this level's band and covered nodes
            fine = np.kron((m >= l + 1).astype(np.uint8),
                           np.ones((B << l,) * 3, dtype=np.uint8))
            assert np.array_equal(np.isin(t, (2, 3)), fine > 0)
            assert c["band"] > 0 and c["covered"] > 0
        else:
            assert c["band"] == 0 and c["covered"] == 0
        if l == 0:
            assert c["ghost"] == 0 and c["unused"] == 0
            continue
        # ghosts: exactly the layer of nodes outside R_l next to it
        reg = np.kron((m >= l).astype(np.uint8), np.ones((B << l,) * 3, dtype=np.uint8)) > 0
        near = np.zeros_like(reg)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    sh = np.zeros_like(reg)
                    src = reg[max(0, -dz):reg.shape[0] - max(0, dz),
                              max(0, -dy):reg.shape[1] - max(0, dy),
                              max(0, -dx):reg.shape[2] - max(0, dx)]
                    sh[max(0, dz):reg.shape[0] - max(0, -dz),
                       max(0, dy):reg.shape[1] - max(0, -dy),
                       max(0, dx):reg.shape[2] - max(0, -dx)] = src
                    near |= sh
        assert np.array_equal(t == 4, near & ~reg)


def test_invalid_nestings_are_refused():
    n, nz, B = 16, 32, 4
    c = oracle.Lattice(oracle.FCLB27, n, n, nz, nu=0.02, faces=[W] * 6)
    m = np.zeros((nz // B, n // B, n // B), dtype=np.uint8)
    m[3, 1, 1] = 2  # a level-2 block whose neighbours are level 0
    with pytest.raises(ValueError):
        oracle.Refined(c, B, m, 3)
    m[2:5, 0:3, 0:3] = 1
    oracle.Refined(c, B, m, 3)  # surrounded by level-1 blocks: valid
    cp = oracle.Lattice(oracle.FCLB27, n, n, nz, nu=0.02)  # periodic
    m2 = np.zeros_like(m)
    m2[0:2] = 1  # touches the periodic z ends without spanning z
    with pytest.raises(ValueError):
        oracle.Refined(cp, B, m2, 2)
    c1 = oracle.Lattice(oracle.FCLB27, n, n, nz, nu=1.0 / 6.0, faces=[W] * 6)  # tau = 1
    with pytest.raises(ValueError):
        oracle.Refined(c1, B, m, 2)


@pytest.mark.parametrize("levels", [2, 3])
def test_interpolation_reproduces_cubics_at_cell_centred_children(levels):
    """Ghost values of level l are the parent field's tensor cubic evaluated
    at the child positions j/2 - 1/4 in parent node units (the cell-centred
    nesting), including the one-sided windows at the walls and the inlet."""
    R, _ = _jet(oracle.MRT19, levels)
    rng = np.random.default_rng(3)
    for l in range(1, levels):
        nz, ny, nx = R.levels[l - 1]["shape"]
        Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        coef = rng.normal(size=(R.Q, 3, 4))

        def poly(q, x, y, z):
            px = sum(coef[q, 0, k] * (x / nx) ** k for k in range(4))
            py = sum(coef[q, 1, k] * (y / ny) ** k for k in range(4))
            pz = sum(coef[q, 2, k] * (z / nz) ** k for k in range(4))
            return px * py * pz

        fp = np.stack([poly(q, X, Y, Z) for q in range(R.Q)])
        coords, g = R.ghosts(l, fp)
        assert len(coords) > 0
        j = coords / 2.0 - 0.25
        expect = np.stack([poly(q, j[:, 0], j[:, 1], j[:, 2]) for q in range(R.Q)])
        assert np.abs(g - expect).max() < 1e-12 * np.abs(expect).max()
        # windows at the non-periodic faces were exercised
        assert (coords[:, 2] <= 1).any()


@pytest.mark.parametrize("model", MODELS)
def test_half_step_ghosts_are_quadratic_in_time(model):
    """Parent states at rest with a density deviation that is cubic in space
    and quadratic in time (equilibria: the rescaling leaves them alone) give
    half-step ghosts equal to the equilibrium of the density at the child's
    position and t + 1/2; without the state at t-1 the fill is linear."""
    R, _ = _jet(model, 2, cs=0.0)
    lat0 = R.level_lattice(0)
    nz, ny, nx = R.levels[0]["shape"]
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")

    def drho(x, y, z, t):
        s = 1e-3 * (1 + 0.3 * x / nx - 0.2 * (y / ny) ** 2 + 0.1 * (z / nz) ** 3)
        return s * (1.0 + 0.4 * t - 0.7 * t * t)

    zero = np.zeros((3,) + X.shape)
    gs = []
    for t in (-1, 0, 1):
        f = lat0.init_equilibrium(drho(X, Y, Z, t), zero)
        coords, g = R.ghosts(1, f)
        gs.append(g)
    x, y, z = coords[:, 0] / 2 - 0.25, coords[:, 1] / 2 - 0.25, coords[:, 2] / 2 - 0.25
    for have_prev, want_t in ((True, 0.5), (False, None)):
        out = R.half_step(1, gs[0], gs[1], gs[2], have_prev=have_prev)
        if want_t is None:  # linear: the mean of the states at t and t + 1
            d = 0.5 * (drho(x, y, z, 0) + drho(x, y, z, 1))
        else:
            d = drho(x, y, z, want_t)
        want = np.stack([_feq(model, v) for v in d], axis=1)
        assert np.abs(out - want).max() < 1e-12 * np.abs(want).max()


def _feq(model, drho):
    """Equilibrium at rest of one node with density deviation drho."""
    if model == oracle.MRT19:
        return oracle.feq_incomp(19, drho, np.zeros(3))
    _, w, _ = oracle.stencil(27)
    return oracle.feq_product(1.0 + drho, np.zeros(3)) - w


def _ce_state(model, tau_shear, S, basis=oracle.BASIS_TABLE1, rates=None):
    """Post-collision Chapman-Enskog state at rest for a traceless lattice
    strain S. The first-order source is the BGK one, f_src = 3 w (e e -
    I/3):S; each moment group k relaxes it with its own time tau_k = 1/s_k,
    so the state after the collision is -M^-1 diag(tau_k - 1) M f_src (the
    shear group at tau_shear, conserved rows empty), M the test's own typed
    basis. The FCLB relaxes every non-shear central moment with rate 1 and
    its shear moments at tau: -3 (tau - 1) w (e e - I/3):S."""
    Q = 19 if model == oracle.MRT19 else 27
    e, w, _ = oracle.stencil(Q)
    e = e.astype(float)
    Qi = np.einsum("ia,ib->iab", e, e) - np.eye(3) / 3
    src = 3 * w * np.einsum("iab,ab->i", Qi, S)
    if model != oracle.MRT19:
        return -(tau_shear - 1) * src
    rows = _T1_ROWS if basis == oracle.BASIS_TABLE1 else _DH_ROWS
    names = ("s2", "s3", "s4", "s7") if basis == oracle.BASIS_TABLE1 else \
        ("s_e", "s_eps", "s_q", "s_pi", "s_m")
    if rates is None:
        rates = oracle.TABLE1_RATES if basis == oracle.BASIS_TABLE1 else oracle.DHUMIERES_RATES
    named = dict(zip(names, rates))
    Mt = _typed_basis(rows)
    tk = np.array([0.0 if r[-1] is None else
                   (tau_shear if r[-1] in ("s1", "nu") else 1.0 / named[r[-1]]) for r in rows])
    diag = np.where(tk == 0.0, 0.0, tk - 1.0)
    return -np.linalg.solve(Mt, diag * (Mt @ src))


@pytest.mark.parametrize("model,basis,cs", [
    (oracle.MRT19, oracle.BASIS_TABLE1, 0.0), (oracle.MRT19, oracle.BASIS_TABLE1, 0.1),
    (oracle.MRT19, oracle.BASIS_TABLE1, 0.18), (oracle.MRT19, oracle.BASIS_DHUMIERES, 0.1),
    (oracle.FCLB27, oracle.BASIS_TABLE1, 0.0)])
def test_rescale_maps_chapman_enskog_states_between_levels(model, basis, cs):
    """A parent post-collision CE state of strain S (shear group relaxed with
    the total time tau_c = tau0_c + 3 C_S^2 |S|, the closed form of Eq. (20)
    for this state) maps to the child's CE state of the same physical strain,
    S/2 in child lattice units, with tau_f = tau0_f + 3 C_S^2 |S| / 2; and
    back. Two and three levels (each interface)."""
    nu = 0.02
    for levels in (2, 3):
        nz = 16 if levels == 2 else 32
        c = oracle.Lattice(model, 4, 4, nz, nu=nu, cs_smag=cs, basis=basis)
        ranges = [(1, 3, 1)] if levels == 2 else [(1, 7, 1), (3, 5, 2)]
        R = oracle.Refined(c, 4, _slab_map(nz, 4, ranges), levels)
        rng = np.random.default_rng(4)
        for l in range(1, levels):
            A = rng.normal(size=(3, 3)) * 1e-3
            S = 0.5 * (A + A.T)
            S -= np.trace(S) / 3 * np.eye(3)
            Smag = np.sqrt(2 * np.sum(S * S))
            nu_c, nu_f = nu * 2 ** (l - 1), nu * 2 ** l
            tc = 3 * nu_c + 0.5 + (3 * cs * cs * Smag if model == oracle.MRT19 else 0.0)
            tf = 3 * nu_f + 0.5 + (3 * cs * cs * Smag / 2 if model == oracle.MRT19 else 0.0)
            fc = _ce_state(model, tc, S, basis)
            ff = _ce_state(model, tf, S / 2, basis)
            got, r = R.rescale(l, fc, +1)
            assert r == pytest.approx((tf - 1) / (2 * (tc - 1)), rel=1e-12)
            assert np.abs(got - ff).max() < 1e-12 * np.abs(ff).max()
            back, _ = R.rescale(l, ff, -1)
            assert np.abs(back - fc).max() < 1e-12 * np.abs(fc).max()


@pytest.mark.parametrize("basis,rows", [(oracle.BASIS_DHUMIERES, _DH_ROWS),
                                        (oracle.BASIS_TABLE1, _T1_ROWS)])
def test_rescale_scales_each_moment_group(basis, rows):
    """Chapman-Enskog per moment group: a non-equilibrium part in one group
    of rate s (fixed on both levels) after the collision is (1 - s)/s times
    a source proportional to the time step, so it halves from parent to
    child; groups relaxed with rate 1 carry none and are set to zero. The
    groups come from the test's own typed bases."""
    nu, n = 0.02, 16
    rates = [1.1, 1.0, 1.3, 1.6, 1.9] if basis == oracle.BASIS_DHUMIERES else [1.0, 1.2, 1.5, 1.7]
    c = oracle.Lattice(oracle.MRT19, 4, 4, n, nu=nu, cs_smag=0.0, basis=basis, rates=rates)
    R = oracle.Refined(c, 4, _slab_map(n, 4, [(1, 3, 1)]), 2)
    Mt = _typed_basis(rows)
    names = ("s_e", "s_eps", "s_q", "s_pi", "s_m") if basis == oracle.BASIS_DHUMIERES else \
        ("s2", "s3", "s4", "s7")
    named = dict(zip(names, rates))
    for k, row in enumerate(rows):
        rate = row[-1]
        if rate is None or rate in ("nu", "s1"):
            continue
        m = np.zeros(19)
        m[k] = 1e-3
        f = np.linalg.solve(Mt, m)
        got, _ = R.rescale(1, f, +1)
        want = 0.0 if named[rate] == 1.0 else 0.5
        mg = Mt @ got
        expect = np.zeros(19)
        expect[k] = want * 1e-3
        assert np.abs(mg - expect).max() < 1e-15, (k, rate)


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("levels", [2, 3])
def test_uniform_flow_is_preserved_through_interfaces(model, levels):
    u0 = 0.002
    n, nz, B = (16 if levels == 2 else 24), 32, 4
    m = _jet_map(n, nz, B, levels)
    fu = [[0, 0, u0]] * 4 + [[0, 0, 0]] * 2
    iu = np.zeros((3, n, n))
    iu[2] = u0
    c = oracle.Lattice(model, n, n, nz, nu=0.02, cs_smag=0.1, faces=[W, W, W, W, I, O],
                       face_u=fu, inlet_u=iu)
    ius = [None] + [np.stack([np.zeros((n << l, n << l)), np.zeros((n << l, n << l)),
                              np.full((n << l, n << l), u0)]) for l in range(1, levels)]
    R = oracle.Refined(c, B, m, levels, inlet_u=ius)
    f0 = []
    for l in range(levels):
        lat = R.level_lattice(l)
        d, u = synth.uniform_fields(*R.levels[l]["n"], u=(0, 0, u0))
        f0.append(lat.collide(lat.init_equilibrium(d, u)))
        R.set_state(l, f0[-1])
    R.run(0, 3)
    for l in range(levels):
        t = R.types(l)
        act = np.isin(t, (1, 2))
        assert np.abs((R.state(l) - f0[l])[:, act]).max() < 1e-15, l


@pytest.mark.parametrize("model", MODELS)
def test_uniform_flow_through_four_levels(model):
    """A periodic 4 x 4 x 64 slab with three nested refined z bands (levels
    1-3, level 3 eight times finer) keeps a uniform flow crossing every
    interface exactly, on every level, over two level-0 steps (16 level-3
    steps)."""
    u0 = 0.002
    c = oracle.Lattice(model, 4, 4, 64, nu=0.02, cs_smag=0.1)
    m = _slab_map(64, 4, [(2, 14, 1), (5, 11, 2), (7, 9, 3)])
    R = oracle.Refined(c, 4, m, 4)
    f0 = []
    for l in range(4):
        lat = R.level_lattice(l)
        d, u = synth.uniform_fields(*R.levels[l]["n"], u=(0.0005, -0.001, u0))
        f0.append(lat.collide(lat.init_equilibrium(d, u)))
        R.set_state(l, f0[-1])
    R.run(0, 2)
    for l in range(4):
        act = np.isin(R.types(l), (1, 2))
        assert act.any(), l
        assert np.abs((R.state(l) - f0[l])[:, act]).max() < 1e-15, l


@pytest.mark.parametrize("model", MODELS)
def test_nothing_refined_is_the_uniform_lattice(model):
    n = 8
    faces = [W, W, P, P, I, O]
    iu, im = synth.jet_inlet(n, n, 3.0, 0.04, 0.001)
    c = oracle.Lattice(model, n, n, n, nu=0.02, cs_smag=0.1, faces=faces,
                       face_u=[[0, 0, 0.001]] * 6, inlet_u=iu, inlet_mask=im,
                       inlet_amp=1e-3, seed=5)
    f0 = synth.random_populations(c.Q, (n, n, n), amp=1e-2, seed=6)
    ref = c.collide(c.run(f0, 3, 4))
    for levels in (1, 2):
        ius, ims = _jet_inlets(n, levels, 3.0, 0.04, 0.001)
        R = oracle.Refined(c, 4, np.zeros((2, 2, 2), dtype=np.uint8), levels,
                           inlet_u=ius, inlet_mask=ims)
        R.set_state(0, c.collide(f0))
        R.run(3, 4)
        assert np.abs(R.state(0) - ref).max() < 1e-16


@pytest.mark.parametrize("model", MODELS)
def test_everything_refined_is_the_fine_uniform_lattice(model):
    """With every block refined there is no interface: the finest level is a
    uniform lattice at 2^l times the resolution (viscosity 2^l nu, seed + l,
    step indices 2^l t + k), solids and curved links included."""
    n, levels = 4, 3
    nf = n << (levels - 1)
    faces = [W, W, P, P, I, O]
    fu = [[0, 0, 0.001]] * 6
    iu, im = synth.jet_inlet(n, n, 2.0, 0.04, 0.001)
    c = oracle.Lattice(model, n, n, n, nu=0.01, cs_smag=0.1, faces=faces, face_u=fu,
                       inlet_u=iu, inlet_mask=im, inlet_amp=1e-3, seed=5)
    ius, ims = _jet_inlets(n, levels, 2.0, 0.04, 0.001)
    def body(x, y, z):  # a sphere on the finest level
        return (x - 5.5) ** 2 + (y - 7.5) ** 2 + (z - 6.0) ** 2 < 4.0

    sm, nodes, q = synth.link_distances(body, (nf, nf, nf),
                                        oracle.stencil(c.Q)[0].tolist())
    lq = np.zeros((c.Q, nf, nf, nf))
    lq.reshape(c.Q, -1)[:, nodes] = q.T
    solids = [None] * (levels - 1) + [sm]
    links = [None] * (levels - 1) + [lq]
    R = oracle.Refined(c, 4, np.full((1, 1, 1), levels - 1, dtype=np.uint8), levels,
                       inlet_u=ius, inlet_mask=ims, solid=solids, link_q=links)
    fine = oracle.Lattice(model, nf, nf, nf, nu=0.01 * 2 ** (levels - 1), cs_smag=0.1,
                          faces=faces, face_u=fu, inlet_u=ius[-1], inlet_mask=ims[-1],
                          inlet_amp=1e-3, seed=5 + levels - 1, solid=sm, link_q=lq)
    f0 = synth.random_populations(c.Q, (nf, nf, nf), amp=1e-2, seed=6)
    k = 2 ** (levels - 1)
    for l in range(levels):
        lat = R.level_lattice(l)
        d, u = synth.uniform_fields(*R.levels[l]["n"])
        R.set_state(l, lat.init_equilibrium(d, u))
    R.set_state(levels - 1, fine.collide(f0))
    R.run(1, 2)
    ref = fine.collide(fine.run(f0, k, 2 * k))
    got = R.state(levels - 1)
    fl = sm == 0
    assert np.abs((got - ref)[:, fl]).max() < 1e-15


@pytest.mark.parametrize("model", MODELS)
def test_couette_flow_sees_the_walls_at_the_same_place_on_every_level(model):
    """Steady Couette flow between a wall at rest (y-) and one moving at u_w
    (y+), both halfway between nodes, with the blocks next to both walls
    refined (two levels): u(y) = u_w (y + 1/2) / n_y in level-0 units on
    every level, level-l node j lying at (j + 1/2) / 2^l - 1/2."""
    B, ny, uw = 4, 16, 1e-3
    c = oracle.Lattice(model, B, ny, B, nu=0.1, faces=[P, P, W, W, P, P],
                       face_u=[[0, 0, 0]] * 3 + [[uw, 0, 0]] + [[0, 0, 0]] * 2)
    m = np.zeros((1, ny // B, 1), dtype=np.uint8)
    m[0, 0, 0] = m[0, -1, 0] = 1
    R = oracle.Refined(c, B, m, 2)
    for l in range(2):
        lat = R.level_lattice(l)
        nx, nyl, nz = R.levels[l]["n"]
        y = (np.arange(nyl) + 0.5) / 2 ** l - 0.5
        u = np.zeros((3, nz, nyl, nx))
        u[0] = (uw * (y + 0.5) / ny)[None, :, None]
        R.set_state(l, lat.collide(lat.init_equilibrium(np.zeros((nz, nyl, nx)), u)))
    R.run(0, 3000)
    for l in range(2):
        lat = R.level_lattice(l)
        _, u = lat.macroscopic(R.state(l))
        t = R.types(l)
        nyl = R.levels[l]["n"][1]
        y = (np.arange(nyl) + 0.5) / 2 ** l - 0.5
        want = uw * (y + 0.5) / ny
        act = np.isin(t, (1, 2))[0, :, 0]
        err = np.abs(u[0, 0, :, 0] - want)[act].max()
        assert err < 1e-4 * uw, (l, err)


def _shear_wave(model, levels, nz=32, B=2, nu=0.05, u0=1e-4, steps=300):
    ranges = [(6, 10, 1)] if levels == 2 else [(4, 12, 1), (6, 10, 2)]
    c = oracle.Lattice(model, B, B, nz, nu=nu)
    R = oracle.Refined(c, B, _slab_map(nz, B, ranges), levels)
    for l in range(levels):
        lat = R.level_lattice(l)
        nx, ny, nzl = R.levels[l]["n"]
        z = (np.arange(nzl) + 0.5) / 2 ** l - 0.5
        u = np.zeros((3, nzl, ny, nx))
        u[0] = (u0 * np.sin(2 * np.pi * z / nz))[:, None, None]
        R.set_state(l, lat.collide(lat.init_equilibrium(np.zeros((nzl, ny, nx)), u)))
    k = 2 * np.pi / nz
    zc = np.arange(nz)
    out0 = R.types(0)[:, 0, 0] == 1
    c0 = R.level_lattice(0)

    def amp():
        _, uu = c0.macroscopic(R.state(0))
        s = np.sin(k * zc)
        return np.sum((uu[0, :, 0, 0] * s)[out0]) / np.sum((s * s)[out0])

    R.run(0, 100)
    a0, m0 = amp(), R.reduce()[0]
    R.run(100, steps)
    return np.log(a0 / amp()) / steps, nu * k * k, R.reduce()[0] - m0, c0.N * u0


@pytest.mark.parametrize("model", MODELS)
@pytest.mark.parametrize("levels", [2, 3])
def test_shear_wave_crossing_nested_interfaces(model, levels):
    """u_x = u0 sin(2 pi z / nz) across one refined slab (two levels) or two
    nested slabs (three levels) decays as exp(-nu k^2 t) with the physical
    (level-0) viscosity; the interfaces are not conservative, but the mass
    drift stays tiny."""
    rate, want, drift, scale = _shear_wave(model, levels)
    assert rate == pytest.approx(want, rel=0.03)
    assert abs(drift) < 1e-3 * scale


def test_reduce_weights_levels_by_volume():
    """Uniform density deviation d and velocity u on every level: the sums
    are the domain volume (in level-0 cells) times d, d u and |u|^2/2."""
    R, _ = _jet(oracle.MRT19, 3)
    d0, u0 = 1e-3, (0.0, 0.001, 0.002)
    for l in range(3):
        lat = R.level_lattice(l)
        d, u = synth.uniform_fields(*R.levels[l]["n"], u=u0)
        R.set_state(l, lat.init_equilibrium(d + d0, u))
    V = 24 * 24 * 32
    out = R.reduce()
    assert out[0] == pytest.approx(V * d0, rel=1e-12)
    assert out[2] == pytest.approx(V * 0.001, rel=1e-12)
    assert out[3] == pytest.approx(V * 0.002, rel=1e-12)
    assert out[4] == pytest.approx(V * 0.5 * (0.001 ** 2 + 0.002 ** 2), rel=1e-12)
