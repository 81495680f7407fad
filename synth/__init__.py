"""Seeded synthetic inputs shared by the HIP path and the FP64 oracle.

This module only draws numbers and lays out fields. It holds none of the
lattice Boltzmann arithmetic: no equilibria, moments, collisions or
streaming. Each side turns these fields into populations with its own code.

Layouts
-------
* scalar field: float64 array of shape (nz, ny, nx), x fastest.
* vector field: float64 array of shape (3, nz, ny, nx).
* populations:  float64 array of shape (Q, nz, ny, nx), the deviations
  f_i - w_i, population index in the order of the velocity tables of
  Section 2 of the paper.
* inlet face fields: index (b, a) over the two tangential axes of the face
  in increasing axis order (for a z face: shape (ny, nx)).
"""
from __future__ import annotations

import numpy as np


def random_populations(q: int, shape, amp: float = 1e-2, seed: int = 0):
    """Uniform noise in [-amp, amp] for every population deviation.

    The state is far from equilibrium, which both collisions accept; it
    exercises every term of a collision at once.
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    return rng.uniform(-amp, amp, size=(q, nz, ny, nx))


def taylor_green(n, u0: float):
    """Taylor-Green vortex on an n^3 periodic box (x = 2 pi i / n).

    u = u0 sin x cos y cos z, v = -u0 cos x sin y cos z, w = 0 and the
    incompressible pressure p' = u0^2/16 (cos 2x + cos 2y)(cos 2z + 2);
    returns (drho, u) with drho = 3 p' (lattice sound speed squared 1/3).
    """
    if np.isscalar(n):
        nx = ny = nz = int(n)
    else:
        nx, ny, nz = (int(v) for v in n)
    x = 2.0 * np.pi * np.arange(nx) / nx
    y = 2.0 * np.pi * np.arange(ny) / ny
    z = 2.0 * np.pi * np.arange(nz) / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    u = np.empty((3, nz, ny, nx))
    u[0] = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    u[1] = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    u[2] = 0.0
    p = (u0 * u0 / 16.0) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    return 3.0 * p, u


def shear_wave(nx, ny, nz, u0: float, axis_u: int = 0, axis_k: int = 1, m: int = 1):
    """u_{axis_u} = u0 sin(2 pi m x_{axis_k} / n_{axis_k}), drho = 0."""
    n = (nx, ny, nz)
    coords = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    c = {0: coords[2], 1: coords[1], 2: coords[0]}[axis_k]
    u = np.zeros((3, nz, ny, nx))
    u[axis_u] = u0 * np.sin(2.0 * np.pi * m * c / n[axis_k])
    return np.zeros((nz, ny, nx)), u


def jet_inlet(na: int, nb: int, diameter: float, u_jet: float, u_coflow: float,
              axis: int = 2):
    """Top-hat round-jet inlet on a face of na x nb nodes.

    Nodes whose centre lies within diameter/2 of the face centre
    ((na-1)/2, (nb-1)/2) get u_jet along the face normal ``axis``, the rest
    the co-flow u_coflow.  Returns (u_face[3, nb, na], disk_mask[nb, na]).
    """
    a = np.arange(na) - 0.5 * (na - 1)
    b = np.arange(nb) - 0.5 * (nb - 1)
    B, A = np.meshgrid(b, a, indexing="ij")
    mask = (A * A + B * B) <= (0.5 * diameter) ** 2
    u = np.zeros((3, nb, na))
    u[axis] = np.where(mask, u_jet, u_coflow)
    return u, mask.astype(np.uint8)


def uniform_fields(nx, ny, nz, u=(0.0, 0.0, 0.0), drho: float = 0.0, dtype=np.float64):
    """Uniform (drho, u) fields."""
    f = np.full((nz, ny, nx), float(drho), dtype=dtype)
    uu = np.empty((3, nz, ny, nx), dtype=dtype)
    for c in range(3):
        uu[c] = u[c]
    return f, uu


def gaussian_field(shape, sigma: float, seed: int):
    """Seeded N(0, sigma^2) field (numpy PCG64 + its standard normal)."""
    rng = np.random.default_rng(seed)
    return sigma * rng.standard_normal(size=shape)


def smooth_random_fields(nx, ny, nz, u_amp: float, rho_amp: float, seed: int,
                         modes: int = 3):
    """A smooth periodic (drho, u) field: a few random low Fourier modes."""
    rng = np.random.default_rng(seed)
    Z, Y, X = np.meshgrid(np.arange(nz) / nz, np.arange(ny) / ny,
                          np.arange(nx) / nx, indexing="ij")
    def field(amp):
        out = np.zeros((nz, ny, nx))
        for _ in range(modes):
            k = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            a = rng.uniform(-1, 1)
            out += a * np.cos(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
        return amp * out / modes
    drho = field(rho_amp)
    u = np.stack([field(u_amp), field(u_amp), field(u_amp)])
    return drho, u


def jet_adjoint_case(n: int = 128, nz: int = 256, diameter: int = 16, u_jet: float = 0.05,
                     u_coflow: float = 0.002, sigma: float = 0.005, seed: int = 389):
    """Round jet for the inlet-sensitivity study: a top-hat inlet of the given
    diameter centred on the z- face of an n x n x nz box, with a static
    perturbation of u_z on the nozzle's bounding square (diameter x diameter
    nodes, including the corners outside the disk), drawn from N(0, sigma^2),
    and a probe box of (2 diameter)^3 nodes centred on the axis, starting 5
    diameters downstream.

    Returns a dict: ``inlet_u`` [3, n, n] (base + perturbation), ``base_u``,
    ``square`` = (b0, b1, a0, a1) index bounds of the perturbed square on the
    face, ``delta`` [diameter, diameter], ``probe_lo`` / ``probe_hi`` (x, y, z).
    """
    base, disk = jet_inlet(n, n, float(diameter), u_jet, u_coflow)
    c0 = n // 2 - diameter // 2
    square = (c0, c0 + diameter, c0, c0 + diameter)
    delta = gaussian_field((diameter, diameter), sigma, seed)
    u = base.copy()
    u[2, square[0]:square[1], square[2]:square[3]] += delta
    p0 = n // 2 - diameter
    lo = (p0, p0, 5 * diameter)
    hi = (p0 + 2 * diameter, p0 + 2 * diameter, 7 * diameter)
    return {"inlet_u": u, "base_u": base, "disk": disk, "square": square, "delta": delta,
            "probe_lo": lo, "probe_hi": hi}


def tiled_populations(q: int, shape, amp: float = 1e-2, seed: int = 0, period=(31, 29, 37),
                      lo=(0, 0, 0), hi=None, qs=None):
    """Seeded uniform-noise populations on a large lattice, cheap to evaluate
    on any sub-box: a random block of `period` = (pz, py, px) nodes repeated
    periodically. shape = (nz, ny, nx) of the whole lattice; lo, hi = (x, y,
    z) bounds of the sub-box returned ([q][z][y][x]); qs selects populations
    (default all). The odd periods make row ends, walls and corners see
    different values."""
    nz, ny, nx = shape
    if hi is None:
        hi = (nx, ny, nz)
    base = random_populations(q, period, amp, seed)
    zs = np.arange(lo[2], hi[2]) % period[0]
    ys = np.arange(lo[1], hi[1]) % period[1]
    xs = np.arange(lo[0], hi[0]) % period[2]
    qsel = range(q) if qs is None else qs
    return np.stack([base[k][np.ix_(zs, ys, xs)] for k in qsel])


def link_distances(is_solid, shape, dirs, iters: int = 40, origin=(0, 0, 0), full_shape=None):
    """Solid nodes and wall distances of a body given by a point predicate.

    is_solid(x, y, z) takes float coordinate arrays (node (i, j, k) sits at
    (i, j, k)) and returns a bool array. dirs: the velocity table, a list of
    (ex, ey, ez). A link runs from a fluid node p to an in-domain solid
    neighbour p + e (no wrap); its distance q in (0, 1] is where the segment
    first enters the body, found by bisection. Returns (solid uint8
    [nz][ny][nx], nodes int32 [n] linear indices x + nx (y + ny z), q
    float32 [n][len(dirs)], zero where there is no link).
    A sub-box of a larger lattice (full_shape = (NZ, NY, NX)) starting at
    node origin = (x0, y0, z0) gives the same links if the body stays one
    node inside it (or touches only the lattice's own faces); the node
    indices are then those of the larger lattice and solid covers the box."""
    nz, ny, nx = shape
    x0, y0, z0 = origin
    NZ, NY, NX = full_shape if full_shape is not None else shape
    z, y, x = np.meshgrid(np.arange(z0, z0 + nz), np.arange(y0, y0 + ny), np.arange(x0, x0 + nx),
                          indexing="ij")
    solid = is_solid(x.astype(float), y.astype(float), z.astype(float))
    n = nx * ny * nz
    qfull = np.zeros((len(dirs), n), np.float32)
    fluid = ~solid
    for k, (ex, ey, ez) in enumerate(dirs):
        if ex == ey == ez == 0:
            continue
        xs, ys, zs = x - x0 + ex, y - y0 + ey, z - z0 + ez
        inside = (xs >= 0) & (xs < nx) & (ys >= 0) & (ys < ny) & (zs >= 0) & (zs < nz)
        cand = fluid & inside
        cand[cand] = solid[zs[cand], ys[cand], xs[cand]]
        if not cand.any():
            continue
        px, py, pz = x[cand].astype(float), y[cand].astype(float), z[cand].astype(float)
        lo = np.zeros(px.shape)
        hi = np.ones(px.shape)
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            s = is_solid(px + mid * ex, py + mid * ey, pz + mid * ez)
            hi = np.where(s, mid, hi)
            lo = np.where(s, lo, mid)
        qfull[k][cand.reshape(-1)] = hi.astype(np.float32)
    local = np.nonzero((qfull != 0).any(axis=0))[0]
    nodes = ((z.reshape(-1)[local] * NY + y.reshape(-1)[local]) * NX +
             x.reshape(-1)[local]).astype(np.int32)
    return solid.astype(np.uint8), nodes, np.ascontiguousarray(qfull[:, local].T)


def nozzle_tube(nx: int, ny: int, diameter: float, wall: float, length: float):
    """Point predicate of a round tube along z around the lattice's centre
    line (x, y) = (nx/2 - 1/2, ny/2 - 1/2): inner radius diameter/2,
    thickness wall, from z = -1/2 to z = length - 1/2."""
    cx, cy, r0 = nx / 2.0 - 0.5, ny / 2.0 - 0.5, diameter / 2.0

    def inside(x, y, z):
        r = np.hypot(x - cx, y - cy)
        return (r >= r0) & (r < r0 + wall) & (z < length - 0.5)
    return inside
