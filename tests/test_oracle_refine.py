"""Pins of the oracle's two-level nested time refinement.

The paper cites the refinement method (Yu et al.) without printing its
formulas; these tests pin the oracle's reading against facts that hold
independently of the implementation: polynomial exactness of the
interpolant, the Chapman-Enskog scaling of the non-equilibrium part between
levels, exact preservation of uniform flow, reduction to the uniform lattice
when nothing is refined, and the viscous decay of a shear wave crossing the
interface.
"""
import numpy as np
import pytest

import oracle
import synth

W, I, O, P = oracle.WALL, oracle.INLET, oracle.OUTFLOW, oracle.PERIODIC


def _slab(model, nu=0.05, nz=64, B=4, zr=(6, 10), cs=0.0):
    """Coarse 4x4xnz periodic lattice with the z-block range zr refined."""
    mask = np.zeros((nz // B, 1, 1), dtype=np.uint8)
    mask[zr[0]:zr[1]] = 1
    c = oracle.Lattice(model, B, B, nz, nu=nu, cs_smag=cs)
    return oracle.Refined(c, B, mask)


def _jet_case(model, nu=0.02):
    """Coarse 16x16x32 with walls, inlet z-, outflow z+, blocks of 4, the
    first four z-block layers refined inside a radius: touches the inlet and
    the side walls, has lateral and top interfaces."""
    n, nz, B = 16, 32, 4
    mask = np.zeros((nz // B, n // B, n // B), dtype=np.uint8)
    for bz in range(4):
        for by in range(n // B):
            for bx in range(n // B):
                cx, cy = (bx + 0.5) * B - n / 2, (by + 0.5) * B - n / 2
                if cx * cx + cy * cy <= 36.0:
                    mask[bz, by, bx] = 1
    return n, nz, B, mask


def test_geometry_invariants():
    for model in (oracle.MRT19, oracle.FCLB27):
        n, nz, B, mask = _jet_case(model)
        iu, im = synth.jet_inlet(n, n, 4.0, 0.05, 0.002)
        fiu, fim = synth.jet_inlet(2 * n, 2 * n, 8.0, 0.05, 0.002)
        c = oracle.Lattice(model, n, n, nz, nu=0.02, faces=[W, W, W, W, I, O],
                           inlet_u=iu, inlet_mask=im)
        R = oracle.Refined(c, B, mask, fiu, fim)
        ct, ft = R.types()
        assert R.counts["fluid"] == int(mask.sum()) * (2 * B) ** 3
        assert R.counts["ghost"] > 0 and R.counts["covered"] > 0 and R.counts["band"] > 0
        # every fluid node's in-domain neighbours are fluid or ghost
        lo, (Mx, My, Mz) = R.lo, R.M
        fl = np.argwhere(ft == 1)
        for lz, ly, lx in fl[:: max(1, len(fl) // 2000)]:
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        jz, jy, jx = lz + dz + lo[2], ly + dy + lo[1], lx + dx + lo[0]
                        if 0 <= jx < 2 * n and 0 <= jy < 2 * n and 0 <= jz < 2 * nz:
                            assert ft[lz + dz, ly + dy, lx + dx] in (1, 2)
        # covered / band nodes are exactly the refined coarse nodes
        refined = np.kron(mask, np.ones((B, B, B), dtype=np.uint8))
        assert np.array_equal(ct > 0, refined > 0)


@pytest.mark.parametrize("model", [oracle.MRT19, oracle.FCLB27])
def test_interpolation_reproduces_cubics(model):
    n, nz, B, mask = _jet_case(model)
    c = oracle.Lattice(model, n, n, nz, nu=0.02, faces=[W, W, W, W, W, W])
    R = oracle.Refined(c, B, mask)
    rng = np.random.default_rng(3)
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(n), np.arange(n), indexing="ij")
    coef = rng.normal(size=(R.Q, 3, 4))

    def poly(q, x, y, z):
        px = sum(coef[q, 0, k] * (x / n) ** k for k in range(4))
        py = sum(coef[q, 1, k] * (y / n) ** k for k in range(4))
        pz = sum(coef[q, 2, k] * (z / nz) ** k for k in range(4))
        return px * py * pz

    fc = np.stack([poly(q, X, Y, Z) for q in range(R.Q)])
    coords, g = R.ghosts(fc)
    j = coords / 2.0
    expect = np.stack([poly(q, j[:, 0], j[:, 1], j[:, 2]) for q in range(R.Q)])
    assert np.abs(g - expect).max() < 1e-12 * np.abs(expect).max()


@pytest.mark.parametrize("model", [oracle.MRT19, oracle.FCLB27])
def test_rescale_chapman_enskog_and_inverse(model):
    """A coarse post-collision Chapman-Enskog state f = f_eq - 3 (tau_c - 1)
    w (e e - I/3):S maps to the fine one for the same physical strain, which
    is S/2 in fine lattice units: f_eq - 3 (tau_f - 1) w (e e - I/3):S/2."""
    nu = 0.02
    R = _slab(model, nu=nu)
    Q = R.Q
    e, w, _ = oracle.stencil(Q)
    e = e.astype(float)
    tc, tf = 3 * nu + 0.5, 6 * nu + 0.5
    assert R.r == pytest.approx((tf - 1) / (2 * (tc - 1)), rel=1e-15)
    rng = np.random.default_rng(4)
    A = rng.normal(size=(3, 3)) * 1e-3
    S = 0.5 * (A + A.T)
    S -= np.trace(S) / 3 * np.eye(3)
    Qi = np.einsum("ia,ib->iab", e, e) - np.eye(3) / 3
    drho, u = 0.01, np.array([0.02, -0.01, 0.03])
    if model == oracle.MRT19:
        feq = oracle.feq_incomp(19, drho, u)
    else:
        feq = oracle.feq_product(1 + drho, u) - w
    fc = feq - 3 * (tc - 1) * w * np.einsum("iab,ab->i", Qi, S)
    ff = feq - 3 * (tf - 1) * w * np.einsum("iab,ab->i", Qi, S / 2)
    got = R.rescale(fc, R.r)
    assert np.abs(got - ff).max() < 1e-15
    assert np.abs(R.rescale(got, 1 / R.r) - fc).max() < 1e-15


@pytest.mark.parametrize("model", [oracle.MRT19, oracle.FCLB27])
def test_uniform_flow_is_preserved_through_interfaces(model):
    n, nz, B, mask = _jet_case(model)
    u0 = 0.002
    fu = [[0, 0, u0]] * 4 + [[0, 0, 0]] * 2
    iu = np.zeros((3, n, n))
    iu[2] = u0
    fiu = np.zeros((3, 2 * n, 2 * n))
    fiu[2] = u0
    c = oracle.Lattice(model, n, n, nz, nu=0.02, cs_smag=0.1, faces=[W, W, W, W, I, O],
                       face_u=fu, inlet_u=iu)
    R = oracle.Refined(c, B, mask, fiu, None)
    d, u = synth.uniform_fields(n, n, nz, u=(0, 0, u0))
    fc = c.init_equilibrium(d, u)
    fl = R.fine_lattice()
    df, uf = synth.uniform_fields(*R.M, u=(0, 0, u0))
    ff = fl.init_equilibrium(df, uf)
    ct, ft = R.types()
    fc1, ff1 = R.run(fc, ff, 0, 4)
    act = ct != 2
    assert np.abs((fc1 - fc)[:, act]).max() < 1e-15
    assert np.abs((ff1 - ff)[:, ft == 1]).max() < 1e-15


@pytest.mark.parametrize("model", [oracle.MRT19, oracle.FCLB27])
def test_empty_mask_is_the_uniform_lattice(model):
    n = 8
    faces = [W, W, P, P, I, O]
    iu, im = synth.jet_inlet(n, n, 3.0, 0.04, 0.001)
    c = oracle.Lattice(model, n, n, n, nu=0.02, cs_smag=0.1, faces=faces,
                       face_u=[[0, 0, 0.001]] * 6, inlet_u=iu, inlet_mask=im,
                       inlet_amp=1e-3, seed=5)
    R = oracle.Refined(c, 4, np.zeros((2, 2, 2), dtype=np.uint8))
    f0 = synth.random_populations(c.Q, (n, n, n), amp=1e-2, seed=6)
    fc, _ = R.run(c.collide(f0), np.zeros((c.Q, 0, 0, 0)), 3, 4)
    ref = c.collide(c.run(f0, 3, 4))
    assert np.abs(fc - ref).max() < 1e-16


@pytest.mark.parametrize("model", [oracle.MRT19, oracle.FCLB27])
def test_shear_wave_crossing_the_interface(model):
    """u_x = u0 sin(2 pi z / nz) across a refined z slab decays as
    exp(-nu k^2 t) with the physical (coarse-level) viscosity."""
    nz, B, nu, u0 = 64, 4, 0.05, 1e-4
    R = _slab(model, nu=nu, nz=nz, B=B)
    c = R.coarse
    d, u = synth.shear_wave(B, B, nz, u0, axis_u=0, axis_k=2)
    fc = c.init_equilibrium(d, u)
    fl = R.fine_lattice()
    Mx, My, Mz = R.M
    zf = (np.arange(Mz) + R.lo[2]) / 2.0
    uf = np.zeros((3, Mz, My, Mx))
    uf[0] = (u0 * np.sin(2 * np.pi * zf / nz))[:, None, None]
    ff = fl.init_equilibrium(np.zeros((Mz, My, Mx)), uf)
    ct, ft = R.types()
    k = 2 * np.pi / nz
    z = np.arange(nz)
    outside = ct[:, 0, 0] == 0

    def amp(f):
        _, uu = c.macroscopic(f)
        ux = uu[0, :, 0, 0]
        s = np.sin(k * z)
        return np.sum((ux * s)[outside]) / np.sum((s * s)[outside])

    steps = 400
    fc, ff = R.run(fc, ff, 0, 100)
    a0 = amp(fc)
    m0 = c.reduce(fc)[0]
    fc, ff = R.run(fc, ff, 100, steps)
    rate = np.log(a0 / amp(fc)) / steps
    assert rate == pytest.approx(nu * k * k, rel=0.03)
    # the interface is not conservative, but the drift stays tiny
    assert abs(c.reduce(fc)[0] - m0) < 1e-3 * u0 * c.N
