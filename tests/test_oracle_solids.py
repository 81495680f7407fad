"""Pins of the oracle's interior solid nodes (halfway bounce-back off solid
neighbours, the rule of a WALL face at rest).

* A channel bounded by two solid layers is the channel bounded by two WALL
  faces at rest: the fluid nodes of the first equal every node of the
  second, step by step, for both models.
* Two solid slabs across a periodic box cut it into two chambers: the mass
  of each chamber is conserved exactly (nothing crosses a solid), while the
  same box without the slabs exchanges mass between the two regions.
"""
import numpy as np
import pytest

import oracle
import synth

P, W = oracle.PERIODIC, oracle.WALL
MODELS = [(oracle.FCLB27, 27), (oracle.MRT19, 19)]


@pytest.mark.parametrize("model,Q", MODELS)
def test_solid_layers_equal_wall_faces(model, Q):
    nx, ny, nz = 6, 7, 5
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    f = synth.random_populations(Q, (nz, ny, nx), amp=1e-2, seed=13)
    a = oracle.Lattice(model, nx, ny, nz, nu=0.02, cs_smag=0.1, solid=solid)
    b = oracle.Lattice(model, nx, ny - 2, nz, nu=0.02, cs_smag=0.1, faces=[P, P, W, W, P, P])
    fa, fb = f.copy(), np.ascontiguousarray(f[:, :, 1:ny - 1, :])
    for t in range(4):
        fa, fb = a.run(fa, t, 1), b.run(fb, t, 1)
        d = np.abs(fa[:, :, 1:ny - 1, :] - fb).max()
        assert d <= 1e-16 * np.abs(fb).max(), (t, d)
        # solid nodes keep their populations
        assert np.array_equal(fa[:, :, 0, :], f[:, :, 0, :])


@pytest.mark.parametrize("model,Q", MODELS)
def test_solid_slabs_separate_chambers(model, Q):
    nx, ny, nz = 5, 4, 12
    f = synth.random_populations(Q, (nz, ny, nx), amp=1e-2, seed=17)
    solid = np.zeros((nz, ny, nx), np.uint8)
    solid[0] = 1
    solid[6] = 1
    first, second = slice(1, 6), slice(7, 12)
    a = oracle.Lattice(model, nx, ny, nz, nu=0.02, solid=solid)
    b = oracle.Lattice(model, nx, ny, nz, nu=0.02)
    fa = a.run(f, 0, 20)
    fb = b.run(f, 0, 20)
    for sl in (first, second):
        m0 = f[:, sl].sum()
        assert abs(fa[:, sl].sum() - m0) <= 1e-14 * np.abs(f).sum()
    # without the slabs the regions do exchange mass
    assert abs(fb[:, first].sum() - f[:, first].sum()) > 1e-6
