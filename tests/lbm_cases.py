"""Shared set-up for GPU-vs-oracle parity tests: builds the same lattice on
both sides from the same seeded inputs (synth) and compares them."""
import numpy as np

import oracle
import synth

MODELS = {  # name: (model code, mrt basis)
    "fclb": (oracle.FCLB27, oracle.BASIS_TABLE1),
    "mrt_table1": (oracle.MRT19, oracle.BASIS_TABLE1),
    "mrt_dhumieres": (oracle.MRT19, oracle.BASIS_DHUMIERES),
    "clb": (oracle.CLB27, oracle.BASIS_TABLE1),
}
# the models the refined lattice runs (all of them)
REFINED_MODELS = list(MODELS)
W, I, O, P = oracle.WALL, oracle.INLET, oracle.OUTFLOW, oracle.PERIODIC
JET_FACES = [W, W, W, W, I, O]


def face_velocities(coflow=0.002, axis=2):
    fu = [[0.0, 0.0, 0.0] for _ in range(6)]
    for k in range(4):
        fu[k][axis] = coflow
    return fu


def gpu_lattice(name, storage, shape, nu, cs=0.0, rates=None, faces=None, face_u=None,
                inlet=None, amp=0.0, seed=0, face_drho=None):
    import torch
    import paper_1206_0389_amd as P
    model, basis = MODELS[name]
    lat = P.Lattice(model=model, storage=storage, shape=shape, nu=nu, cs_smag=cs,
                    mrt_basis=basis, rates=rates)
    if faces is not None:
        iu = im = None
        if inlet is not None:
            iu = torch.from_numpy(np.ascontiguousarray(inlet[0], dtype=np.float64))
            im = torch.from_numpy(np.ascontiguousarray(inlet[1], dtype=np.uint8))
        lat.set_boundaries(faces, face_u=face_u, inlet_u=iu, inlet_mask=im, inlet_amp=amp,
                           seed=seed, face_drho=face_drho)
    return lat


def oracle_lattice(name, shape, nu, cs=0.0, rates=None, faces=None, face_u=None, inlet=None,
                   amp=0.0, seed=0, origin=(0, 0, 0), extent=None, face_drho=None):
    model, basis = MODELS[name]
    nx, ny, nz = shape
    kw = {}
    if faces is not None:
        kw = dict(faces=faces, face_u=face_u, inlet_amp=amp, seed=seed, origin=origin)
        if face_drho is not None:
            kw["face_drho"] = face_drho
        if inlet is not None:
            kw.update(inlet_u=inlet[0], inlet_mask=inlet[1])
            if extent is not None:
                kw["inlet_extent"] = extent
    return oracle.Lattice(model, nx, ny, nz, nu=nu, cs_smag=cs, basis=basis, rates=rates, **kw)


def rel_err(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def window(shape, faces, lo, hi, margin):
    """Oracle window [lo, hi) (+margin on cut sides) of a global lattice.

    Returns (wlo, whi, wfaces, inner) where inner are the slices of the
    window that hold exact values after `margin` steps.
    """
    wlo, whi, wf, inner = [], [], [], []
    for d in range(3):
        n = shape[d]
        a = max(lo[d] - margin, 0)
        b = min(hi[d] + margin, n)
        per = faces[2 * d] == P
        if per and (lo[d] - margin < 0 or hi[d] + margin > n):
            a, b = 0, n  # periodic axis: take it whole
        wlo.append(a)
        whi.append(b)
        f_lo = faces[2 * d] if a == 0 else P
        f_hi = faces[2 * d + 1] if b == n else P
        if per and (a, b) == (0, n):
            f_lo = f_hi = P
        wf += [f_lo, f_hi]
        inner.append(slice(lo[d] - a, hi[d] - a))
    return wlo, whi, wf, inner


# ------------------------------------------------ refined-lattice cases
F, PR = oracle.FREESLIP, oracle.PRESSURE
REFINED_FACE_U = [[0.0, 0.001, 0.002], [0.0, 0.0, 0.002], [0.001, 0.0, 0.002], [0.0, 0.0, 0.002],
          [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]]


def jet_map(n, nz, B, levels, r2=None):
    """First four z block layers within a radius refined (two levels: 16 x 16
    x 32, radius^2 40; three: 24 x 24 x 32, the centre 4 x 4 blocks, and the
    inner 2 x 2 blocks of the first two layers once more)."""
    m = np.zeros((nz // B, n // B, n // B), dtype=np.uint8)
    if r2 is None:
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


REFINED_CASES = {
    # name: (levels, jet, faces, face_drho)
    "jet2": (2, True, [W, W, W, W, I, O], None),
    "jet3": (3, True, [W, W, W, W, I, O], None),
    "slab": (2, False, [P] * 6, None),
    "slab3": (3, False, [P] * 6, None),
    # four nested z bands (level 3 has eight times the resolution)
    "slab4": (4, False, [P] * 6, None),
    "slip_pressure": (2, True, [W, W, W, F, I, PR], [0, 0, 0, 0, 0, -0.002]),
    "slab_slip_pressure": (2, False, [F, F, PR, PR, P, P], [0, 0, 0.001, -0.001, 0, 0]),
    # 24 x 24 x 32 with the centre 4 x 4 blocks of the first four layers
    # refined: room for a nozzle inside the fine level
    "jet2wide": (2, True, [W, W, W, W, I, O], None),
    # the paper's 11^3 blocks: 44 x 44 x 44, three levels
    "jet3b11": (3, True, [W, W, W, W, I, O], None),
}


# Level-0 viscosity per case (default 0.02). With four levels tau doubles its
# excess over 1/2 three times: at 0.02 the finest level has tau = 0.98, where
# the rescaling of the non-equilibrium parts from it back to level 2 (the
# injection) multiplies them, and their rounding, by 2 (tau_c - 1) / (tau_f -
# 1) = 26; at 0.005 the levels have tau = 0.515, 0.53, 0.56, 0.62 and the
# factor is 2.3.
REFINED_NU = {"slab4": 0.005}


def slab_map(levels):
    """Level map of the 4 x 4 x 64 slab (blocks of 4): nested bands in z."""
    m = np.zeros((16, 1, 1), dtype=np.uint8)
    if levels == 2:
        m[6:10] = 1
    elif levels == 3:
        m[4:12] = 1
        m[7:9] = 2
    else:
        m[2:14] = 1
        m[5:11] = 2
        m[7:9] = 3
    return m


def refined_jet_geometry(case):
    """(n, nz, B, level map) of a jet case."""
    levels = REFINED_CASES[case][0]
    if case == "jet3b11":
        # level 1 over the whole cross-section of the first three block
        # layers, level 2 on the inner 2 x 2 blocks of the first two
        m = np.zeros((4, 4, 4), dtype=np.uint8)
        m[0:3] = 1
        m[0:2, 1:3, 1:3] = 2
        return 44, 44, 11, m
    n = 16 if (levels == 2 and case != "jet2wide") else 24
    r2 = 72.0 if case == "jet2wide" else None
    return n, 32, 4, jet_map(n, 32, 4, levels, r2)


def read_covered(types, faces):
    """Covered nodes (type 3) in the 26-neighbourhood of fluid or band nodes
    (types 1, 2) of a level's whole domain: the covered nodes a refined
    step reads, the ones the library injects into. faces: the six face types
    (periodic axes wrap)."""
    act = np.isin(types, (1, 2))
    near = np.zeros_like(act)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                sh = act
                for ax, d in ((0, dz), (1, dy), (2, dx)):
                    if d == 0:
                        continue
                    per = faces[2 * (2 - ax)] == P
                    sh = np.roll(sh, d, axis=ax)
                    if not per:  # no wrap: clear the layer rolled in
                        idx = [slice(None)] * 3
                        idx[ax] = 0 if d > 0 else -1
                        sh[tuple(idx)] = False
                near |= sh
    return near & (types == 3)
