"""ctypes binding of the FP64 CPU oracle (``oracle/lbm_oracle.cpp``).

TEST INFRASTRUCTURE. Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The GPU
library and its Python binding never import it, and it never imports them.

Parity status of each oracle function (what pins it, see tests/):
  stencil, weights            golden table typed from Section 2 + isotropy
  feq_incomp (Eq. 2)          closed-form moments
  mrt_collide (Eq. 12)        conservation, fixed point, all-rates-1 and BGK
                              reductions, basis orthogonality (d'Humieres)
  smagorinsky_tau (Eqs.16-21) Chapman-Enskog strain state, quadratic identity
  central_moments (Eq. 15)    Table 2 printed raw->central polynomials
  fclb_collide                conservation, product-equilibrium fixed point,
                              omega = 1 map, moment self-consistency, symmetry
  clb_collide (CLB27)         conservation, fixed point, equal to the FCLB at
                              omega = 1, post-collision central moments of
                              orders 4 and 6 those of the Gaussian (computed
                              from the populations), shear-wave decay rate
  run (streaming + BCs)       exact first-moment transport law, shear-wave
                              and Taylor-Green decay rates, Couette profile
  splitmix64                  published test vector
  Refined (two-level nesting) polynomial exactness of the interpolant,
                              Chapman-Enskog rescaling, uniform flow kept,
                              reduction to the uniform lattice, shear-wave decay
  collide_jvp (FCLB)          central differences, rest-state relaxation
                              spectrum (1 - omega shear, trace removed),
                              conservation, equilibrium tangent fixed
  collide_jvp (MRT-LES)       central differences in both bases with the
                              eddy viscosity on (and differing from the
                              product without it), rest-state spectrum (each
                              non-conserved moment mode scaled by 1 - s_k,
                              Table 1 multiplicities), conservation, the
                              incompressible equilibrium tangent fixed
  tangent_step / adjoint_step central differences of run; dot-product identity;
                              periodic mass/momentum adjoint invariants
  probe_ke, inlet_gradient    central differences of J through many steps
  velocity_statistics         constant and two-level sequences, the variance
                              (K^2 - 1)/12 of a ramp, Eq. (25) on fields
                              with known values
  solid nodes (run)           a channel bounded by solid layers equals the
                              channel bounded by WALL faces; a solid slab
                              across a periodic box blocks all transport
  FREESLIP faces (run)        free-slip y faces equal the mirror-symmetric
                              half of a periodic lattice twice as high;
                              uniform tangential flow is kept exactly; a
                              free-slip top halves a pressure-driven channel
  PRESSURE faces (run)        plug flow from a velocity inlet to a pressure
                              outlet is a fixed point; a closed box with a
                              pressure face relaxes to the face's density;
                              a pressure drop drives plane Poiseuille flow
  jet_profile (Eqs. 23-24)    a field linear in the section (bilinear
                              exact): closed-form crossing radii; Gaussian
                              and elliptic jets: r_e at the e-folding radius
                              of each axis; axis permutations agree
  jet_fit (Eqs. 22-24)        exact power laws and Gaussian profiles give
                              their constants and zero residual; a known
                              profile offset gives that residual
  interpolated bounce-back    q = 1/2 is the halfway rule; steady Couette
  (run, link_q)               flow puts the no-slip point at the wall's
                              distance q (halfway: at 1/2)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.cpp")
LIB = os.path.join(HERE, "liblbm_oracle.so")

MRT19, FCLB27, CLB27 = 1, 2, 3
BASIS_TABLE1, BASIS_DHUMIERES = 0, 1
PERIODIC, WALL, INLET, OUTFLOW, FREESLIP, PRESSURE = 0, 1, 2, 3, 4, 5

DHUMIERES_RATES = (1.19, 1.4, 1.2, 1.4, 1.98)
TABLE1_RATES = (1.0, 1.0, 1.0, 1.0)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["g++", "-std=c++17", "-O3", "-fopenmp", "-ffp-contract=off",
               "-shared", "-fPIC", "-o", LIB + ".tmp", SRC]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("nu", ctypes.c_double),
        ("cs_smag", ctypes.c_double),
        ("mrt_basis", ctypes.c_int32),
        ("pad0", ctypes.c_int32),
        ("rates", ctypes.c_double * 8),
        ("face_type", ctypes.c_int32 * 6),
        ("face_u", (ctypes.c_double * 3) * 6),
        ("inlet_u", ctypes.POINTER(ctypes.c_double)),
        ("inlet_mask", ctypes.POINTER(ctypes.c_uint8)),
        ("inlet_amp", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("origin", ctypes.c_int32 * 3),
        ("inlet_na", ctypes.c_int32), ("inlet_nb", ctypes.c_int32),
        ("solid", ctypes.POINTER(ctypes.c_uint8)),
        ("face_drho", ctypes.c_double * 6),
        ("link_q", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        pp = ctypes.POINTER(Params)
        L.orc_stencil.argtypes = [ctypes.c_int, ip, dp, ip]
        L.orc_feq_incomp.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_feq_product.argtypes = [ctypes.c_double, dp, dp]
        L.orc_mrt_basis.argtypes = [ctypes.c_int, dp]
        L.orc_smagorinsky_tau.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_smagorinsky_tau.restype = ctypes.c_double
        L.orc_mrt_collide.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                      dp, dp, dp]
        L.orc_central_moments.argtypes = [dp, dp, dp, dp]
        L.orc_fclb_collide.argtypes = [dp, ctypes.c_double, dp]
        L.orc_clb_collide.argtypes = [dp, ctypes.c_double, dp]
        L.orc_splitmix64.argtypes = [ctypes.c_uint64]
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_inlet_uniform.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int]
        L.orc_inlet_uniform.restype = ctypes.c_double
        L.orc_collide_lattice.argtypes = [pp, dp, dp]
        L.orc_run.argtypes = [pp, dp, ctypes.c_int64, ctypes.c_int64]
        L.orc_macroscopic.argtypes = [pp, dp, dp, dp]
        L.orc_init_equilibrium.argtypes = [pp, dp, dp, dp]
        L.orc_reduce.argtypes = [pp, dp, dp]
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.orc_collide_jvp.argtypes = [pp, dp, dp, dp]
        L.orc_tangent_step.argtypes = [pp, dp, dp, dp]
        L.orc_adjoint_step.argtypes = [pp, dp, dp, dp, dp]
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.orc_probe_ke.argtypes = [pp, dp, i32p, i32p, dp]
        L.orc_probe_ke.restype = ctypes.c_double
        L.orc_mlref_info.argtypes = [ctypes.c_void_p, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int64)]
        L.orc_mlref_types.argtypes = [ctypes.c_void_p, ctypes.c_int, u8p]
        L.orc_mlref_set_state.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
        L.orc_mlref_get_state.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
        L.orc_mlref_ghosts.argtypes = [ctypes.c_void_p, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int32), dp, dp]
        L.orc_mlref_rescale.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, ctypes.c_int, dp]
        L.orc_mlref_reduce.argtypes = [ctypes.c_void_p, dp]
        L.orc_mlref_half_step.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp, dp,
                                          ctypes.c_int, dp]
        L.orc_mlref_destroy.argtypes = [ctypes.c_void_p]
        L.orc_mlref_ghost_count.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n):
    """OpenMP team size of the oracle's loops (timing only)."""
    lib().orc_set_threads(int(n))


def max_threads():
    return int(lib().orc_max_threads())


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def q_of(model):
    return 19 if model == MRT19 else 27


def stencil(Q):
    e = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    opp = np.zeros(Q, dtype=np.int32)
    ip = ctypes.POINTER(ctypes.c_int)
    rc = lib().orc_stencil(Q, e.ctypes.data_as(ip), _dp(w), opp.ctypes.data_as(ip))
    assert rc == 0
    return e, w, opp


def feq_incomp(Q, drho, u):
    out = np.zeros(Q)
    lib().orc_feq_incomp(Q, float(drho), _dp(_f64(u)), _dp(out))
    return out


def feq_product(rho, u):
    out = np.zeros(27)
    lib().orc_feq_product(float(rho), _dp(_f64(u)), _dp(out))
    return out


def mrt_basis(basis):
    M = np.zeros((19, 19))
    lib().orc_mrt_basis(basis, _dp(M))
    return M


def smagorinsky_tau(f19, tau0, cs):
    Q = np.zeros(1)
    t = lib().orc_smagorinsky_tau(_dp(_f64(f19)), tau0, cs, _dp(Q))
    return t, float(Q[0])


def mrt_collide(f19, tau0, cs=0.0, basis=BASIS_TABLE1, rates=None):
    if rates is None:
        rates = TABLE1_RATES if basis == BASIS_TABLE1 else DHUMIERES_RATES
    r = np.zeros(8)
    r[:len(rates)] = rates
    out = np.zeros(19)
    tau = np.zeros(1)
    lib().orc_mrt_collide(_dp(_f64(f19)), tau0, cs, basis, _dp(r), _dp(out), _dp(tau))
    return out, float(tau[0])


def central_moments(F):
    rho = np.zeros(1)
    u = np.zeros(3)
    k = np.zeros(27)
    lib().orc_central_moments(_dp(_f64(F)), _dp(rho), _dp(u), _dp(k))
    return float(rho[0]), u, k.reshape(3, 3, 3)


def fclb_collide(f27, omega):
    out = np.zeros(27)
    lib().orc_fclb_collide(_dp(_f64(f27)), float(omega), _dp(out))
    return out


def clb_collide(f27, omega):
    """The cascaded collision with Gaussian higher-order equilibria."""
    out = np.zeros(27)
    lib().orc_clb_collide(_dp(_f64(f27)), float(omega), _dp(out))
    return out


def splitmix64(state):
    return int(lib().orc_splitmix64(ctypes.c_uint64(state & 0xFFFFFFFFFFFFFFFF)))


def inlet_uniform(seed, t, a, b, c):
    return float(lib().orc_inlet_uniform(seed, t, a, b, c))


def velocity_statistics(us, axis=2, point=None):
    """Time averages of a sequence of velocity fields (the jet statistics of
    Section 3). us: iterable of K arrays [3][nz][ny][nx]. Returns mean, rms
    and, if point is given, the turbulent intensity of Eq. (25).

    mean = (1/K) sum_k u_k; rms = sqrt((1/K) sum_k (u_k - mean)^2) (the
    fluctuation about the mean, population normalisation); ti = rms of the
    streamwise component (axis) over the mean streamwise velocity at the jet
    axis point of the same cross-section (point: the two other coordinates in
    increasing order)."""
    us = [np.asarray(u, dtype=np.float64) for u in us]
    K = len(us)
    mean = sum(us) / K
    var = sum((u - mean) ** 2 for u in us) / K
    rms = np.sqrt(var)
    if point is None:
        return mean, rms, None
    m = np.moveaxis(mean[axis], 2 - axis, 0)  # streamwise index first
    # [stream][a][b] with (a, b) the other coordinates, slowest first
    axis_mean = m[:, point[1], point[0]]
    shape = [1, 1, 1]
    shape[2 - axis] = -1
    ti = rms[axis] / axis_mean.reshape(shape)
    return mean, rms, ti


# Fraction of the axis velocity at the radius r_e that defines the spreading
# width (Eqs. (23)-(24): u = 0.368 u_m at half the width).
SPREAD_FRACTION = 0.368


def jet_profile(mean, axis, center, ndir, dr, nr):
    """Spreading of a jet from its time-averaged velocity (Section 3: the
    width of Eq. (23) and the profile of Eq. (24)), on every cross-section.

    mean: [3][nz][ny][nx]; axis: the jet axis; center: the jet centre (a, b)
    in the two other coordinates in increasing axis order (node units). On
    cross-section p, the streamwise mean u is interpolated bilinearly in
    (a, b); u_m = u at the centre. Rays leave the centre at the angles 2 pi
    j / ndir (from the a axis towards b), sampled at r_k = k dr, k < nr,
    while the sample lies within the cross-section's nodes. The radius r_e
    of a ray is the first point where u falls to SPREAD_FRACTION u_m,
    interpolated linearly between the two samples around it.

    Returns um [np], re [3][np] (minimum, maximum and mean of r_e over the
    rays that reach it; NaN if none does) and prof [np][nr], the mean of
    u(r_k) / u_m over the rays whose sample k lies within the section (NaN
    if none)."""
    u = np.moveaxis(np.asarray(mean, dtype=np.float64)[axis], 2 - axis, 0)  # [p][b][a]
    npl, nb, na = u.shape
    c0, c1 = float(center[0]), float(center[1])

    def bilinear(P, a, b):
        i = min(int(np.floor(a)), na - 2)
        j = min(int(np.floor(b)), nb - 2)
        fa, fb = a - i, b - j
        return ((1 - fa) * (1 - fb) * P[j, i] + fa * (1 - fb) * P[j, i + 1] +
                (1 - fa) * fb * P[j + 1, i] + fa * fb * P[j + 1, i + 1])

    def inside(a, b):
        return 0.0 <= a <= na - 1 and 0.0 <= b <= nb - 1

    um = np.zeros(npl)
    re = np.full((3, npl), np.nan)
    prof = np.full((npl, nr), np.nan)
    for p in range(npl):
        P = u[p]
        um[p] = bilinear(P, c0, c1)
        thr = SPREAD_FRACTION * um[p]
        radii = []
        sums, counts = np.zeros(nr), np.zeros(nr)
        for j in range(ndir):
            th = 2.0 * np.pi * j / ndir
            ca, sa = np.cos(th), np.sin(th)
            prev, found = um[p], False
            for k in range(nr):
                a, b = c0 + k * dr * ca, c1 + k * dr * sa
                if not inside(a, b):
                    break
                v = bilinear(P, a, b)
                sums[k] += v / um[p]
                counts[k] += 1
                if k > 0 and not found and v <= thr:
                    radii.append((k - 1) * dr + dr * (prev - thr) / (prev - v))
                    found = True
                prev = v
        if radii:
            re[:, p] = (min(radii), max(radii), sum(radii) / len(radii))
        ok = counts > 0
        prof[p, ok] = sums[ok] / counts[ok]
    return um, re, prof


def jet_fit(um, re, prof, dr, x0, u0, d, p0, p1):
    """The jet laws of Section 3 fitted to a jet_profile result over the
    cross-sections p0 <= p < p1 downstream of the nozzle exit x0 (distance
    x = p - x0 > 0; sections with a NaN input are skipped).

    k_par: least squares of u_m = u0 k_par d / x (Eq. (22)); k_perp: least
    squares of b_g = k_perp x (Eq. (23)) with b_g the mean radius r_e (where
    the velocity is 0.368 u_m); res: root mean square over those sections
    and the radii r_k = k dr <= 2 r_e of prof - 0.938 exp(-0.944 (r_k /
    r_e)^2) (Eq. (24)). Returns (k_par, k_perp, res, number of profile
    samples); NaN where nothing enters a fit."""
    um, re, prof = (np.asarray(a, dtype=np.float64) for a in (um, re, prof))
    s1 = s2 = s3 = s4 = s5 = 0.0
    n = 0
    for p in range(p0, p1):
        x = p - x0
        if x <= 0:
            continue
        if not np.isnan(um[p]):
            a = u0 * d / x
            s1 += um[p] * a
            s2 += a * a
        r_e = re[2, p]
        if np.isnan(r_e):
            continue
        s3 += r_e * x
        s4 += x * x
        for k in range(prof.shape[1]):
            r = k * dr
            if r > 2.0 * r_e or np.isnan(prof[p, k]):
                continue
            g = 0.938 * np.exp(-0.944 * (r / r_e) ** 2)
            s5 += (prof[p, k] - g) ** 2
            n += 1
    k_par = s1 / s2 if s2 > 0 else np.nan
    k_perp = s3 / s4 if s4 > 0 else np.nan
    res = np.sqrt(s5 / n) if n > 0 else np.nan
    return k_par, k_perp, res, n


class Lattice:
    """Configuration of an oracle lattice (or window of one).

    faces: six of PERIODIC/WALL/INLET/OUTFLOW for x-, x+, y-, y+, z-, z+.
    face_drho: density deviation of PRESSURE faces (six values).
    solid: optional [nz][ny][nx] mask of interior solid nodes; a population
    whose source is solid bounces back off a wall at rest, and solid nodes
    keep their (meaningless) populations unchanged.
    link_q: optional [Q][nz][ny][nx] wall distances of the links from fluid
    node x towards solid x + e_i, as fractions of the link (0: halfway);
    those links bounce back with Bouzidi's linear interpolation.
    """

    def __init__(self, model, nx, ny, nz, nu, cs_smag=0.0, basis=BASIS_TABLE1,
                 rates=None, faces=(PERIODIC,) * 6, face_u=None, inlet_u=None,
                 inlet_mask=None, inlet_amp=0.0, seed=0, origin=(0, 0, 0),
                 inlet_extent=None, solid=None, face_drho=None, link_q=None):
        p = Params()
        p.model = model
        p.nx, p.ny, p.nz = nx, ny, nz
        p.nu = nu
        p.cs_smag = cs_smag
        p.mrt_basis = basis
        if rates is None:
            rates = TABLE1_RATES if basis == BASIS_TABLE1 else DHUMIERES_RATES
        for k, v in enumerate(rates):
            p.rates[k] = v
        for k in range(6):
            p.face_type[k] = faces[k]
        if face_u is not None:
            for k in range(6):
                for c in range(3):
                    p.face_u[k][c] = face_u[k][c]
        self._keep = []
        if inlet_u is not None:
            iu = _f64(inlet_u)
            self._keep.append(iu)
            p.inlet_u = _dp(iu)
            p.inlet_nb, p.inlet_na = iu.shape[1], iu.shape[2]
        if inlet_extent is not None:
            p.inlet_na, p.inlet_nb = inlet_extent
        if inlet_mask is not None:
            im = np.ascontiguousarray(inlet_mask, dtype=np.uint8)
            self._keep.append(im)
            p.inlet_mask = im.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        p.inlet_amp = inlet_amp
        p.seed = seed
        for k in range(3):
            p.origin[k] = origin[k]
        if face_drho is not None:
            for k in range(6):
                p.face_drho[k] = face_drho[k]
        self.solid = None
        if solid is not None:
            sm = np.ascontiguousarray(solid, dtype=np.uint8)
            assert sm.shape == (nz, ny, nx)
            self._keep.append(sm)
            self.solid = sm
            p.solid = sm.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        if link_q is not None:
            lq = _f64(link_q)
            assert lq.shape == (q_of(model), nz, ny, nx)
            self._keep.append(lq)
            p.link_q = _dp(lq)
        self.p = p
        self.model = model
        self.Q = q_of(model)
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz

    def run(self, f, t0, nsteps):
        f = _f64(f).copy()
        assert f.shape == (self.Q,) + self.shape
        lib().orc_run(ctypes.byref(self.p), _dp(f), int(t0), int(nsteps))
        return f

    def collide(self, f):
        f = _f64(f)
        out = np.empty_like(f)
        lib().orc_collide_lattice(ctypes.byref(self.p), _dp(f), _dp(out))
        return out

    def macroscopic(self, f):
        f = _f64(f)
        drho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        lib().orc_macroscopic(ctypes.byref(self.p), _dp(f), _dp(drho), _dp(u))
        return drho, u

    def init_equilibrium(self, drho, u):
        f = np.zeros((self.Q,) + self.shape)
        lib().orc_init_equilibrium(ctypes.byref(self.p), _dp(_f64(drho)), _dp(_f64(u)),
                                   _dp(f))
        return f

    def reduce(self, f):
        out = np.zeros(5)
        lib().orc_reduce(ctypes.byref(self.p), _dp(_f64(f)), _dp(out))
        return out

    # ---- adjoint of the FCLB and MRT-LES models (exact Jacobian-vector
    # products by dual numbers; the transpose of streaming is the scatter of
    # the pull) ----
    def _need_adjoint(self):
        if self.model not in (FCLB27, MRT19):
            raise ValueError("the oracle's adjoint covers the FCLB and MRT-LES models only")
        if self.solid is not None:
            raise ValueError("the oracle's adjoint has no interior solids")
        if FREESLIP in tuple(self.p.face_type) or PRESSURE in tuple(self.p.face_type):
            raise ValueError("the oracle's adjoint has no free-slip or pressure faces")

    def collide_jvp(self, f, v):
        self._need_adjoint()
        out = np.zeros(self.Q)
        lib().orc_collide_jvp(ctypes.byref(self.p), _dp(_f64(f)), _dp(_f64(v)), _dp(out))
        return out

    def tangent_step(self, f, v):
        self._need_adjoint()
        out = np.zeros((self.Q,) + self.shape)
        lib().orc_tangent_step(ctypes.byref(self.p), _dp(_f64(f)), _dp(_f64(v)), _dp(out))
        return out

    def adjoint_step(self, f, lam_next, grad):
        """Adjoint at t from the state f_t and the adjoint at t+1; grad
        ([3][nb][na], float64) is accumulated in place."""
        self._need_adjoint()
        lam = np.zeros((self.Q,) + self.shape)
        assert grad.dtype == np.float64 and grad.flags.c_contiguous
        lib().orc_adjoint_step(ctypes.byref(self.p), _dp(_f64(f)), _dp(_f64(lam_next)), _dp(lam),
                               _dp(grad))
        return lam

    def probe_ke(self, f, lo, hi, grad=False):
        i32p = ctypes.POINTER(ctypes.c_int32)
        lo = np.ascontiguousarray(lo, dtype=np.int32)
        hi = np.ascontiguousarray(hi, dtype=np.int32)
        lam = np.zeros((self.Q,) + self.shape) if grad else None
        J = lib().orc_probe_ke(ctypes.byref(self.p), _dp(_f64(f)), lo.ctypes.data_as(i32p),
                               hi.ctypes.data_as(i32p), _dp(lam) if grad else None)
        return (J, lam) if grad else J

    def inlet_gradient(self, f0, t0, nsteps, lo, hi, every=20):
        """Probe kinetic energy J after nsteps from the pre-collision state f0
        at time t0, and dJ/du_in ([3][nb][na]) of a static additive inlet
        velocity, by the discrete adjoint. States are checkpointed every
        `every` steps and recomputed segment by segment in reverse."""
        self._need_adjoint()
        ckpt = {}
        f = _f64(f0).copy()
        for t in range(nsteps):
            if t % every == 0:
                ckpt[t] = f
            f = self.run(f, t0 + t, 1)
        J, lam = self.probe_ke(f, lo, hi, grad=True)
        grad = np.zeros((3, self.p.inlet_nb, self.p.inlet_na))
        for s in sorted(ckpt, reverse=True):
            states = [ckpt[s]]
            for t in range(s, min(s + every, nsteps) - 1):
                states.append(self.run(states[-1], t0 + t, 1))
            for fs in reversed(states):
                lam = self.adjoint_step(fs, lam, grad)
        return J, grad, lam


class Refined:
    """Nested time refinement in the oracle: post-collision storage, every
    level held over its whole domain (see the refinement section of
    lbm_oracle.cpp for the readings).

    coarse: a :class:`Lattice` for level 0 (faces, inlet, seed, model).
    block: block edge B in level-0 nodes. level_map: uint8 [nz/B][ny/B][nx/B],
    the finest level of each block (a 0/1 mask gives two levels).
    nlevels: number of levels (default: largest map entry + 1).
    Per-level lists indexed by level (entries may be None): inlet_u
    [3][nb][na] and inlet_mask [nb][na] at that level's resolution (levels
    >= 1 need them when level 0 has an inlet face), solid [nz][ny][nx] masks
    and link_q [Q][nz][ny][nx] wall distances over the level's whole domain.
    """

    def __init__(self, coarse: Lattice, block: int, level_map, nlevels=None, inlet_u=None,
                 inlet_mask=None, solid=None, link_q=None):
        self.coarse = coarse
        self.map = np.ascontiguousarray(level_map, dtype=np.uint8)
        self.L = int(nlevels) if nlevels is not None else int(self.map.max()) + 1
        self.B = int(block)
        self.Q = coarse.Q
        L = self.L
        u8p = ctypes.POINTER(ctypes.c_uint8)
        self._keep = [self.map]

        def arr(vals, conv, ptype):
            if vals is None:
                return None
            a = (ptype * L)()
            for l in range(min(L, len(vals))):
                if vals[l] is not None:
                    v = conv(vals[l])
                    self._keep.append(v)
                    a[l] = v.ctypes.data_as(ptype)
            return a

        u8 = lambda v: np.ascontiguousarray(v, dtype=np.uint8)
        dp = ctypes.POINTER(ctypes.c_double)
        lib().orc_mlref_create.restype = ctypes.c_void_p
        lib().orc_mlref_create.argtypes = [ctypes.POINTER(Params), ctypes.c_int, ctypes.c_int,
                                           u8p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]
        self.h = lib().orc_mlref_create(ctypes.byref(coarse.p), self.B, L,
                                        self.map.ctypes.data_as(u8p),
                                        arr(inlet_u, _f64, dp), arr(inlet_mask, u8, u8p),
                                        arr(solid, u8, u8p), arr(link_q, _f64, dp))
        if not self.h:
            raise ValueError("invalid refinement configuration")
        self.levels = []
        for l in range(L):
            n = (ctypes.c_int32 * 3)()
            box = (ctypes.c_int32 * 6)()
            cnt = (ctypes.c_int64 * 6)()
            lib().orc_mlref_info(ctypes.c_void_p(self.h), l, n, box, cnt)
            self.levels.append({
                "n": tuple(n), "shape": (n[2], n[1], n[0]), "lo": tuple(box[:3]),
                "hi": tuple(box[3:]),
                "counts": dict(zip(("fluid", "band", "covered", "ghost", "solid", "unused"),
                                   tuple(cnt)))})

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_mlref_destroy(ctypes.c_void_p(self.h))
            self.h = None

    def types(self, l):
        """Node types of level l: 0 unused, 1 fluid, 2 band (inside the next
        level's region, updated on this level), 3 covered, 4 ghost, 5 solid."""
        t = np.zeros(self.levels[l]["shape"], dtype=np.uint8)
        lib().orc_mlref_types(ctypes.c_void_p(self.h), l,
                              t.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        return t

    def set_state(self, l, f):
        f = _f64(f)
        assert f.shape == (self.Q,) + self.levels[l]["shape"]
        lib().orc_mlref_set_state(ctypes.c_void_p(self.h), l, _dp(f))

    def state(self, l):
        f = np.zeros((self.Q,) + self.levels[l]["shape"])
        lib().orc_mlref_get_state(ctypes.c_void_p(self.h), l, _dp(f))
        return f

    def run(self, t0, n):
        lib().orc_mlref_run.restype = ctypes.c_int64
        bad = lib().orc_mlref_run(ctypes.c_void_p(self.h), ctypes.c_int64(int(t0)),
                                  ctypes.c_int64(int(n)))
        if bad:
            raise RuntimeError("refinement geometry error: %d pulls from unused nodes" % bad)

    def ghosts(self, l, parent=None):
        """Ghost coordinates of level l >= 1 ([ng][3], x y z) and the raw
        spatial interpolation of a level l-1 field parent ([Q][...]) at them."""
        lib().orc_mlref_ghost_count.restype = ctypes.c_int64
        ng = int(lib().orc_mlref_ghost_count(ctypes.c_void_p(self.h), l))
        coords = np.zeros((ng, 3), dtype=np.int32)
        i32p = ctypes.POINTER(ctypes.c_int32)
        if parent is None:
            lib().orc_mlref_ghosts(ctypes.c_void_p(self.h), l, coords.ctypes.data_as(i32p),
                                   None, None)
            return coords, None
        g = np.zeros((self.Q, ng))
        lib().orc_mlref_ghosts(ctypes.c_void_p(self.h), l, coords.ctypes.data_as(i32p),
                               _dp(_f64(parent)), _dp(g))
        return coords, g

    def rescale(self, l, f, direction):
        """Non-equilibrium rescaling of one node between level l-1 and level l
        (direction +1: a level l-1 state to level l; -1: back). Returns the
        rescaled populations and the shear ratio."""
        out = np.zeros(self.Q)
        lib().orc_mlref_rescale.restype = ctypes.c_double
        r = lib().orc_mlref_rescale(ctypes.c_void_p(self.h), l, _dp(_f64(f)), int(direction),
                                    _dp(out))
        return out, float(r)

    def half_step(self, l, gm1, g0, gp1, have_prev=True):
        """Half-step ghost values of level l from raw parent interpolations at
        t-1, t and t+1 ([Q][ng] each), as a refined step fills them."""
        ng = g0.shape[1]
        out = np.zeros((self.Q, ng))
        lib().orc_mlref_half_step(ctypes.c_void_p(self.h), l, _dp(_f64(gm1)), _dp(_f64(g0)),
                                  _dp(_f64(gp1)), int(bool(have_prev)), _dp(out))
        return out

    def reduce(self):
        out = np.zeros(5)
        lib().orc_mlref_reduce(ctypes.c_void_p(self.h), _dp(out))
        return out

    def level_lattice(self, l):
        """An oracle Lattice with level l's parameters (viscosity 2^l nu_0)
        over its whole domain, for equilibria and macroscopic readouts."""
        c = self.coarse
        nx, ny, nz = self.levels[l]["n"]
        return Lattice(c.model, nx, ny, nz, nu=c.p.nu * 2 ** l, cs_smag=c.p.cs_smag,
                       basis=c.p.mrt_basis, rates=list(c.p.rates)[:5])
