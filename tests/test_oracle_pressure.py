"""Pins of the oracle's PRESSURE faces (the fixed-pressure outflow of the
paper's numerical set-up, Section 3; read as anti-bounce-back with the
model's equilibrium at the face's density and the node's velocity).

* Plug flow from a velocity inlet to a pressure outlet (periodic sides) is a
  fixed point: the anti-bounce-back of an equilibrium state returns that
  state (its even part is what the rule imposes), as the inlet's Ladd
  bounce-back does for its odd part. Exact for the incompressible MRT at any
  outlet density; for the FCLB at rho = 1, to the rounding of its fixed
  point (the periodic lattice drifts by the same 1e-13).
* A closed box at rest with a density excess relaxes toward the outlet's
  density through the pressure face (the excess leaves as sound).
"""
import numpy as np
import pytest

import oracle

P, W, I, PR = oracle.PERIODIC, oracle.WALL, oracle.INLET, oracle.PRESSURE


@pytest.mark.parametrize("model,drho_out,tol", [(oracle.MRT19, 0.0, 1e-14),
                                                 (oracle.MRT19, 0.003, 1e-14),
                                                 (oracle.FCLB27, 0.0, 1e-12)])
def test_plug_flow_is_a_fixed_point(model, drho_out, tol):
    nx, ny, nz = 4, 4, 12
    iu = np.zeros((3, ny, nx))
    iu[2] = 0.02
    o = oracle.Lattice(model, nx, ny, nz, nu=0.02, faces=[P, P, P, P, I, PR], inlet_u=iu,
                       face_drho=[0, 0, 0, 0, 0, drho_out])
    d = np.full((nz, ny, nx), drho_out)
    u = np.zeros((3, nz, ny, nx))
    u[2] = 0.02
    f0 = o.init_equilibrium(d, u)
    f = o.run(f0, 0, 20)
    assert np.abs(f - f0).max() <= tol * np.abs(f0).max()


@pytest.mark.parametrize("model", [oracle.MRT19, oracle.FCLB27])
def test_closed_box_relaxes_to_outlet_density(model):
    nx, ny, nz = 8, 8, 16
    o = oracle.Lattice(model, nx, ny, nz, nu=0.02, faces=[W, W, W, W, W, PR])
    f = o.init_equilibrium(np.full((nz, ny, nx), 0.01), np.zeros((3, nz, ny, nx)))
    f = o.run(f, 0, 400)
    drho, u = o.macroscopic(f)
    assert np.all(np.isfinite(f))
    assert np.abs(drho).max() < 1e-3          # from 1e-2
    # a closed box keeps its mass: walls alone do not relax it
    c = oracle.Lattice(model, nx, ny, nz, nu=0.02, faces=[W] * 6)
    g = c.run(c.init_equilibrium(np.full((nz, ny, nx), 0.01), np.zeros((3, nz, ny, nx))), 0, 400)
    assert abs(c.macroscopic(g)[0].mean() - 0.01) < 1e-12


def _channel():
    """Pressure-driven flow between PRESSURE faces at x and WALL faces at y
    (MRT, 12000 steps from rest): the mid-channel velocity profile and the
    local gradient G = -c_s^2 d(rho)/dx."""
    nx, ny, nz = 48, 17, 1
    nu = 0.1
    o = oracle.Lattice(oracle.MRT19, nx, ny, nz, nu=nu, faces=[PR, PR, W, W, P, P],
                       face_drho=[0.0015, -0.0015, 0, 0, 0, 0])
    f = o.run(o.init_equilibrium(np.zeros((nz, ny, nx)), np.zeros((3, nz, ny, nx))), 0, 12000)
    d, u = o.macroscopic(f)
    dc = d[0, ny // 2, :]
    G = -(dc[nx // 2 + 5] - dc[nx // 2 - 5]) / 10 / 3.0
    return u[0, 0, :, nx // 2], u[1, 0, :, nx // 2], G, nu, ny, nx


def test_pressure_drop_drives_plane_poiseuille_flow():
    """Mid-channel, the settled flow between walls half a link outside the
    end nodes is u = G (y + 1/2)(H - 1/2 - y) / (2 nu) for the local gradient
    (within 0.5 %); that gradient is the imposed drop over the length to
    within 5 % (an end effect of the faces, O(1/nx))."""
    ux, uy, G, nu, ny, nx = _channel()
    y = np.arange(ny)
    exact = G * (y + 0.5) * (ny - 0.5 - y) / (2 * nu)
    assert np.abs(ux - exact).max() <= 5e-3 * exact.max()
    assert abs(G / (0.003 / 3.0 / nx) - 1) <= 0.05
    assert np.abs(uy).max() <= 1e-4 * exact.max()
