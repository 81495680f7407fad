"""Pins of the oracle's interpolated bounce-back (Bouzidi's linear rule on
links from fluid nodes to interior solid nodes, the curved no-slip walls of
the paper's nozzle, Section 3).

* q = 1/2 on every link is the halfway rule: identical results, step by
  step, to the lattice without link distances.
* Where the fluid node behind x along the link is missing (a one-node gap
  between solids), the halfway rule stays for q < 1/2.
* Steady Couette flow between a solid layer whose wall lies a fraction q
  of a link from the first fluid plane and a moving WALL face: the velocity
  is linear and vanishes at the wall's position (y_w = 1 - q), to the
  rounding of a nearly converged state; the halfway rule on the same
  lattice puts the no-slip point half a link out instead.
"""
import numpy as np
import pytest

import oracle
import synth

P, W = oracle.PERIODIC, oracle.WALL
MODELS = [(oracle.FCLB27, 27, oracle.BASIS_TABLE1), (oracle.MRT19, 19, oracle.BASIS_TABLE1),
          (oracle.MRT19, 19, oracle.BASIS_DHUMIERES)]


def _links_towards(Q, shape, solid, q):
    """link_q = q on every link from a fluid node to a solid node."""
    nz, ny, nx = shape
    lq = np.zeros((Q, nz, ny, nx))
    for i in range(Q):
        ex, ey, ez = E[i]
        nb = np.roll(solid, shift=(-ez, -ey, -ex), axis=(0, 1, 2))  # solid at x + e_i
        lq[i][(nb != 0) & (solid == 0)] = q
    return lq


E = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
     (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
     (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1), (1, 1, 1), (-1, 1, 1),
     (1, -1, 1), (1, 1, -1), (-1, -1, 1), (-1, 1, -1), (1, -1, -1), (-1, -1, -1)]


def _block(shape):
    nz, ny, nx = shape
    solid = np.zeros(shape, np.uint8)
    solid[2:5, 2:4, 1:4] = 1
    return solid


@pytest.mark.parametrize("model,Q,basis", MODELS)
def test_half_link_is_the_halfway_rule(model, Q, basis):
    shape = (7, 6, 6)
    nz, ny, nx = shape
    solid = _block(shape)
    f = synth.random_populations(Q, shape, amp=1e-2, seed=21)
    a = oracle.Lattice(model, nx, ny, nz, nu=0.02, cs_smag=0.1, basis=basis, solid=solid,
                       link_q=_links_towards(Q, shape, solid, 0.5))
    b = oracle.Lattice(model, nx, ny, nz, nu=0.02, cs_smag=0.1, basis=basis, solid=solid)
    fa, fb = f.copy(), f.copy()
    for t in range(3):
        fa, fb = a.run(fa, t, 1), b.run(fb, t, 1)
        assert np.array_equal(fa, fb), t
    # another distance changes the populations next to the block only
    c = oracle.Lattice(model, nx, ny, nz, nu=0.02, cs_smag=0.1, basis=basis, solid=solid,
                       link_q=_links_towards(Q, shape, solid, 0.3))
    fc = c.run(f, 0, 1)
    near = np.zeros(shape, bool)
    for ex, ey, ez in E[:Q]:
        near |= np.roll(solid, shift=(ez, ey, ex), axis=(0, 1, 2)) != 0
    far = ~near & (solid == 0)
    fb1 = b.run(f, 0, 1)
    assert np.array_equal(fc[:, far], fb1[:, far])
    assert np.abs(fc[:, near & (solid == 0)] - fb1[:, near & (solid == 0)]).max() > 1e-6


@pytest.mark.parametrize("model,Q,basis", MODELS[:2])
def test_one_node_gap_keeps_halfway(model, Q, basis):
    shape = (4, 5, 4)
    nz, ny, nx = shape
    solid = np.zeros(shape, np.uint8)
    solid[:, 1, :] = 1
    solid[:, 3, :] = 1  # fluid plane y = 2 between two solid planes; y = 0, 4 fluid
    f = synth.random_populations(Q, shape, amp=1e-2, seed=5)
    lq = np.zeros((Q, nz, ny, nx))
    for i in range(Q):
        if E[i][1] != 0:
            lq[i, :, 2, :] = 0.3  # behind the gap node lies the other solid
    a = oracle.Lattice(model, nx, ny, nz, nu=0.05, solid=solid, link_q=lq)
    b = oracle.Lattice(model, nx, ny, nz, nu=0.05, solid=solid)
    assert np.array_equal(a.run(f, 0, 2), b.run(f, 0, 2))


def _couette(model, Q, basis, q, use_links, steps=2500, U=1e-3, ny=10):
    nx = nz = 1
    shape = (nz, ny, nx)
    solid = np.zeros(shape, np.uint8)
    solid[:, 0, :] = 1
    face_u = [[0.0] * 3 for _ in range(6)]
    face_u[3] = [U, 0.0, 0.0]
    kw = dict(solid=solid, faces=[P, P, W, W, P, P], face_u=face_u, basis=basis)
    if use_links:
        kw["link_q"] = _links_towards(Q, shape, solid, q)
    lat = oracle.Lattice(model, nx, ny, nz, nu=1.0 / 6.0, **kw)
    d0 = np.zeros(shape)
    u0 = np.zeros((3,) + shape)
    f = lat.init_equilibrium(d0, u0)
    f = lat.run(f, 0, steps)
    _, u = lat.macroscopic(f)
    y = np.arange(1, ny, dtype=float)
    ux = u[0, 0, 1:, 0]
    # the exact profile: zero at y_w, U at the moving face y = ny - 1/2
    y_w = 1.0 - q
    exact = U * (y - y_w) / (ny - 0.5 - y_w)
    return ux, exact


@pytest.mark.parametrize("model,Q,basis", MODELS)
@pytest.mark.parametrize("q", [0.2, 0.5, 0.8])
def test_couette_no_slip_at_the_wall_distance(model, Q, basis, q):
    ux, exact = _couette(model, Q, basis, q, True)
    err = np.abs(ux - exact).max() / exact.max()
    assert err <= 1e-10, err
    if q != 0.5:  # the halfway rule puts the wall half a link out
        ux_h, _ = _couette(model, Q, basis, q, False)
        assert np.abs(ux_h - exact).max() / exact.max() > 1e-2
