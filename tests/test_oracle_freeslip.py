"""Pins of the oracle's FREESLIP faces (halfway specular reflection, the
free-slip top of the paper's tank, Section 3).

* Mirror symmetry: a lattice with free-slip faces at y- and y+ evolves as
  the upper half of a periodic lattice twice as high started from the
  mirror-symmetric state (node y -> -1 - y, populations with e_y reversed):
  the mirror planes of the doubled lattice sit half a node outside the
  free-slip faces, exactly where the reflection happens. Checked with
  random far-from-equilibrium states, both models, periodic in x and z, to
  the rounding of mirrored collisions (1e-13).
* A uniform flow along the faces is kept exactly (no friction), while WALL
  faces at rest slow it down.
"""
import numpy as np
import pytest

import oracle
import synth

P, W, F = oracle.PERIODIC, oracle.WALL, oracle.FREESLIP
MODELS = [(oracle.FCLB27, 27), (oracle.MRT19, 19)]


def _mirror_index(Q):
    e, _, _ = oracle.stencil(Q)
    return np.array([int(np.where((e == [a, -b, c]).all(axis=1))[0][0]) for a, b, c in e])


@pytest.mark.parametrize("model,Q", MODELS)
def test_freeslip_faces_are_mirror_planes(model, Q):
    nx, ny, nz = 5, 4, 6
    f = synth.random_populations(Q, (nz, ny, nx), amp=1e-2, seed=41)
    r = _mirror_index(Q)
    # doubled periodic lattice: rows ny..2ny-1 = f, rows ny-1-y = mirror of row y
    big = np.zeros((Q, nz, 2 * ny, nx))
    big[:, :, ny:] = f
    big[:, :, :ny] = f[r][:, :, ::-1, :]
    a = oracle.Lattice(model, nx, ny, nz, nu=0.02, cs_smag=0.1, faces=[P, P, F, F, P, P])
    b = oracle.Lattice(model, nx, 2 * ny, nz, nu=0.02, cs_smag=0.1)
    fa, fb = f.copy(), big
    for t in range(5):
        fa, fb = a.run(fa, t, 1), b.run(fb, t, 1)
        d = np.abs(fa - fb[:, :, ny:]).max()
        assert d <= 1e-13 * np.abs(fa).max(), (t, d)
        # the doubled state stays mirror symmetric (to the rounding of a
        # mirrored collision, which is not bitwise the mirrored result)
        sym = np.abs(fb[:, :, :ny] - fb[r][:, :, ::-1][:, :, :ny]).max()
        assert sym <= 1e-13 * np.abs(fb).max(), (t, sym)


@pytest.mark.parametrize("model,Q", MODELS)
def test_uniform_tangential_flow_is_kept(model, Q):
    nx, ny, nz = 4, 6, 4
    d = np.zeros((nz, ny, nx))
    u = np.zeros((3, nz, ny, nx))
    u[0] = 0.04
    u[2] = -0.01
    for faces, slip in (([P, P, F, F, P, P], True), ([P, P, W, W, P, P], False)):
        o = oracle.Lattice(model, nx, ny, nz, nu=0.02, faces=faces)
        f0 = o.init_equilibrium(d, u)
        f = o.run(f0, 0, 10)
        _, v = o.macroscopic(f)
        if slip:
            # the periodic lattice drifts by the same 1e-13 (rounding of the
            # equilibrium fixed point over 10 steps)
            assert np.abs(f - f0).max() <= 1e-12 * np.abs(f0).max()
        else:
            assert np.abs(v[0] - 0.04).max() > 1e-3


def test_free_slip_top_halves_a_pressure_driven_channel():
    """A pressure-driven channel with a FREESLIP top is the lower half of a
    channel twice as high: no shear at the plane half a link above the last
    node, u = G (y + 1/2)(2 ny - y - 1/2) / (2 nu) mid-channel (0.5 %)."""
    P, W, PR, F = oracle.PERIODIC, oracle.WALL, oracle.PRESSURE, oracle.FREESLIP
    nx, ny, nz, nu = 48, 9, 1, 0.1
    o = oracle.Lattice(oracle.MRT19, nx, ny, nz, nu=nu, faces=[PR, PR, W, F, P, P],
                       face_drho=[0.0015, -0.0015, 0, 0, 0, 0])
    f = o.run(o.init_equilibrium(np.zeros((nz, ny, nx)), np.zeros((3, nz, ny, nx))), 0, 12000)
    d, u = o.macroscopic(f)
    dc = d[0, ny // 2, :]
    G = -(dc[nx // 2 + 5] - dc[nx // 2 - 5]) / 10 / 3.0
    y = np.arange(ny)
    exact = G * (y + 0.5) * (2 * ny - y - 0.5) / (2 * nu)
    assert np.abs(u[0, 0, :, nx // 2] - exact).max() <= 5e-3 * exact.max()
