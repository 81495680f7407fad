"""Pins of the oracle's discrete adjoint of the FCLB and MRT-LES
collide-and-stream maps.

The collision's Jacobian-vector products come from dual numbers run through
the collision itself; the transpose of streaming is the scatter of the pull
rule. They are pinned against facts that do not depend on that code: central
differences of the forward map, the linear relaxation spectrum of the
collision at rest (shear moments scale by 1 - omega, the trace is relaxed to
equilibrium, conserved moments are kept), the tangent of the equilibrium
manifold as a fixed direction, the dot-product identity between the tangent
and the adjoint, adjoint invariants from mass and momentum conservation on a
periodic lattice, and finite differences of the probe objective through many
steps with respect to the inlet velocity. For the MRT-LES collision (Eq. 12
with the Smagorinsky relaxation time of Eqs. 16-21) the rest-state spectrum
is that of the moment relaxation: the four conserved modes keep eigenvalue 1
and every other moment mode M^-1 e_k is scaled by 1 - s_k, with the
multiplicities of the paper's Table 1 (and of the d'Humieres basis).
"""
import numpy as np
import pytest

import oracle
import synth

W, I, O, P = oracle.WALL, oracle.INLET, oracle.OUTFLOW, oracle.PERIODIC
FACE_U = [[0.0, 0.001, 0.002], [0.0, 0.0, 0.002], [0.001, 0.0, 0.002], [0.0, 0.0, 0.002],
          [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]]


def _moving_state(seed, amp=1e-2):
    """One node's deviations: equilibrium of a moving fluid plus noise."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.02 * rng.uniform(-1, 1)
    u = 0.05 * rng.uniform(-1, 1, size=3)
    _, w, _ = oracle.stencil(27)
    return oracle.feq_product(rho, u) - w + amp * rng.uniform(-1, 1, size=27)


def _lat(nu=0.02, faces=(P,) * 6, n=(6, 5, 7), model="fclb", **kw):
    code, basis, cs = MODELS[model]
    return oracle.Lattice(code, *n, nu=nu, faces=list(faces), face_u=FACE_U, cs_smag=cs,
                          basis=basis, **kw)


# name: (model, MRT basis, Smagorinsky constant)
MODELS = {
    "fclb": (oracle.FCLB27, oracle.BASIS_TABLE1, 0.0),
    "mrt_table1": (oracle.MRT19, oracle.BASIS_TABLE1, 0.1),
    "mrt_dhumieres": (oracle.MRT19, oracle.BASIS_DHUMIERES, 0.1),
}


def test_jvp_matches_central_difference():
    lat = _lat()
    omega = 1.0 / (3 * 0.02 + 0.5)
    rng = np.random.default_rng(3)
    for seed in range(5):
        f = _moving_state(seed)
        v = rng.standard_normal(27)
        h = 1e-6
        fd = (oracle.fclb_collide(f + h * v, omega) - oracle.fclb_collide(f - h * v, omega)) / (2 * h)
        jv = lat.collide_jvp(f, v)
        assert np.abs(jv - fd).max() <= 1e-8 * np.abs(fd).max()


def test_jvp_keeps_mass_and_momentum():
    lat = _lat()
    e, _, _ = oracle.stencil(27)
    rng = np.random.default_rng(4)
    for seed in range(5):
        f = _moving_state(seed)
        v = rng.standard_normal(27)
        jv = lat.collide_jvp(f, v)
        assert abs(jv.sum() - v.sum()) <= 1e-13 * np.abs(v).sum()
        assert np.abs(e.T @ jv - e.T @ v).max() <= 1e-13 * np.abs(v).sum()


def test_linear_spectrum_at_rest():
    """Around the rest state the collision is a linear relaxation: shear
    perturbations w_i e_ix e_iy and w_i (e_ix^2 - e_iy^2) scale by 1 - omega,
    the trace perturbation w_i (|e_i|^2 - 1) is removed (rate 1), and
    perturbations of density and momentum pass unchanged."""
    nu = 0.02
    omega = 1.0 / (3 * nu + 0.5)
    lat = _lat(nu=nu)
    e, w, _ = oracle.stencil(27)
    f0 = np.zeros(27)
    shear = [w * e[:, 0] * e[:, 1], w * e[:, 1] * e[:, 2], w * (e[:, 0] ** 2 - e[:, 1] ** 2)]
    for v in shear:
        np.testing.assert_allclose(lat.collide_jvp(f0, v), (1 - omega) * v, atol=1e-15)
    trace = w * ((e * e).sum(axis=1) - 1.0)
    np.testing.assert_allclose(lat.collide_jvp(f0, trace), 0.0, atol=1e-15)
    for v in (w, w * e[:, 0], w * e[:, 2]):
        jv = lat.collide_jvp(f0, v)
        # conserved moments kept; the first-order perturbation also carries its
        # equilibrium second moments, which a rest-state linearisation sets to 0
        assert abs(jv.sum() - v.sum()) <= 1e-15
        np.testing.assert_allclose(e.T @ jv, e.T @ v, atol=1e-15)


def test_equilibrium_tangent_is_fixed():
    """Equilibria are fixed points for every (rho, u), so the collision's
    Jacobian maps a tangent of the equilibrium family onto itself."""
    lat = _lat()
    _, w, _ = oracle.stencil(27)
    rng = np.random.default_rng(5)
    for _ in range(4):
        rho = 1.0 + 0.02 * rng.uniform(-1, 1)
        u = 0.05 * rng.uniform(-1, 1, size=3)
        d = rng.standard_normal(4)
        h = 1e-5
        t = (oracle.feq_product(rho + h * d[0], u + h * d[1:]) -
             oracle.feq_product(rho - h * d[0], u - h * d[1:])) / (2 * h)
        jv = lat.collide_jvp(oracle.feq_product(rho, u) - w, t)
        assert np.abs(jv - t).max() <= 1e-9 * np.abs(t).max()


JET = [W, W, W, W, I, O]
FACE_SETS = {
    "periodic": [P] * 6,
    "jet": JET,
    "closed": [W] * 6,
    "channel": [P, P, W, W, I, O],
    "outflow_both": [W, W, P, P, O, O],
}


def _inlet(nx, ny):
    iu, im = synth.jet_inlet(nx, ny, 2.0, 0.05, 0.002)
    return iu, im


@pytest.mark.parametrize("model", list(MODELS))
@pytest.mark.parametrize("faces", list(FACE_SETS))
def test_tangent_step_matches_finite_difference(faces, model):
    n = (6, 5, 7)
    iu, im = _inlet(n[0], n[1])
    lat = _lat(faces=FACE_SETS[faces], n=n, inlet_u=iu, inlet_mask=im, inlet_amp=1e-3, seed=2,
               model=model)
    f = synth.random_populations(lat.Q, lat.shape, 1e-2, seed=6)
    v = synth.random_populations(lat.Q, lat.shape, 1.0, seed=7)
    h = 1e-6
    fd = (lat.run(f + h * v, 5, 1) - lat.run(f - h * v, 5, 1)) / (2 * h)
    tv = lat.tangent_step(f, v)
    assert np.abs(tv - fd).max() <= 1e-8 * np.abs(fd).max()


@pytest.mark.parametrize("model", list(MODELS))
@pytest.mark.parametrize("faces", list(FACE_SETS))
def test_adjoint_dot_product(faces, model):
    """<S J v, w> = <v, J^T S^T w> to rounding for the one-step map."""
    n = (6, 5, 7)
    iu, im = _inlet(n[0], n[1])
    lat = _lat(faces=FACE_SETS[faces], n=n, inlet_u=iu, inlet_mask=im, model=model)
    f = synth.random_populations(lat.Q, lat.shape, 1e-2, seed=8)
    for s in range(3):
        v = synth.random_populations(lat.Q, lat.shape, 1.0, seed=10 + s)
        w = synth.random_populations(lat.Q, lat.shape, 1.0, seed=20 + s)
        g = np.zeros((3, n[1], n[0]))
        lhs = float((lat.tangent_step(f, v) * w).sum())
        rhs = float((v * lat.adjoint_step(f, w, g)).sum())
        assert abs(lhs - rhs) <= 1e-12 * (np.abs(v).sum() + np.abs(w).sum())


@pytest.mark.parametrize("model", list(MODELS))
def test_periodic_adjoint_invariants(model):
    """On a periodic lattice streaming only permutes populations and the
    collision keeps mass and momentum, so the adjoint fields 1 (total mass)
    and e_i (total momentum) are reproduced exactly by every step."""
    lat = _lat(n=(5, 6, 4), model=model)
    Q = lat.Q
    e, _, _ = oracle.stencil(Q)
    f = synth.random_populations(Q, lat.shape, 1e-2, seed=9)
    g = np.zeros((3, 1, 1))
    one = np.ones((Q,) + lat.shape)
    assert np.abs(lat.adjoint_step(f, one, g) - 1.0).max() <= 1e-13
    for a in range(3):
        lam = np.broadcast_to(e[:, a].reshape(Q, 1, 1, 1), one.shape)
        assert np.abs(lat.adjoint_step(f, lam, g) - lam).max() <= 1e-13


def test_probe_gradient_matches_finite_difference():
    lat = _lat(n=(6, 6, 8))
    f = synth.random_populations(27, lat.shape, 1e-2, seed=12)
    lo, hi = (1, 2, 3), (4, 5, 6)
    J, lam = lat.probe_ke(f, lo, hi, grad=True)
    assert J > 0
    rng = np.random.default_rng(13)
    h = 1e-7
    for _ in range(20):
        i, z, y, x = rng.integers(27), rng.integers(8), rng.integers(6), rng.integers(6)
        fp, fm = f.copy(), f.copy()
        fp[i, z, y, x] += h
        fm[i, z, y, x] -= h
        fd = (lat.probe_ke(fp, lo, hi) - lat.probe_ke(fm, lo, hi)) / (2 * h)
        assert abs(fd - lam[i, z, y, x]) <= 1e-8 * (abs(fd) + 1e-6)
    # zero outside the probe
    mask = np.zeros(lat.shape, dtype=bool)
    mask[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = True
    assert np.abs(lam[:, ~mask]).max() == 0.0


def _jet_lattice(model, n, nz, nu, u_face):
    code, basis, cs = MODELS[model]
    return oracle.Lattice(code, n, n, nz, nu=nu, faces=JET, face_u=FACE_U, inlet_u=u_face,
                          cs_smag=cs, basis=basis)


def _jet_objective(case, n, nz, nsteps, nu, u_face, model="fclb"):
    lat = _jet_lattice(model, n, nz, nu, u_face)
    f = np.zeros((lat.Q, nz, n, n))
    f = lat.run(f, 0, nsteps)
    return lat.probe_ke(f, case["probe_lo"], case["probe_hi"])


@pytest.mark.parametrize("model", ["fclb", "mrt_table1"])
def test_inlet_gradient_matches_finite_difference(model):
    """dJ/du_in from the adjoint through 24 steps of a small jet against
    central differences of J, for every component on the perturbed square and
    two points outside it; the checkpoint spacing does not change it. The
    MRT case runs with the eddy viscosity on (C_S = 0.1)."""
    n, nz, D, nsteps, nu = 8, 16, 2, 24, 0.01
    case = synth.jet_adjoint_case(n, nz, D, u_jet=0.05, u_coflow=0.002, sigma=0.005, seed=3)
    case["probe_lo"], case["probe_hi"] = (2, 2, 5), (6, 6, 9)
    lat = _jet_lattice(model, n, nz, nu, case["inlet_u"])
    f0 = np.zeros((lat.Q, nz, n, n))
    J, grad, _ = lat.inlet_gradient(f0, 0, nsteps, case["probe_lo"], case["probe_hi"], every=5)
    J2, grad2, _ = lat.inlet_gradient(f0, 0, nsteps, case["probe_lo"], case["probe_hi"],
                                      every=100)
    assert J == J2 and np.array_equal(grad, grad2)
    assert abs(J - _jet_objective(case, n, nz, nsteps, nu, case["inlet_u"], model)) <= \
        1e-16 * J + 1e-300
    b0, b1, a0, a1 = case["square"]
    points = [(b, a) for b in range(b0, b1) for a in range(a0, a1)] + [(0, 0), (b0 - 1, a1)]
    h = 1e-6
    fd = np.zeros((3, len(points)))
    for k, (b, a) in enumerate(points):
        for c in range(3):
            up, um = case["inlet_u"].copy(), case["inlet_u"].copy()
            up[c, b, a] += h
            um[c, b, a] -= h
            fd[c, k] = (_jet_objective(case, n, nz, nsteps, nu, up, model) -
                        _jet_objective(case, n, nz, nsteps, nu, um, model)) / (2 * h)
    adj = np.array([[grad[c, b, a] for (b, a) in points] for c in range(3)])
    assert np.abs(fd).max() > 0
    assert np.linalg.norm(adj - fd) <= 1e-6 * np.linalg.norm(fd)


def test_adjoint_rejects_other_models():
    lat = oracle.Lattice(oracle.CLB27, 4, 4, 4, nu=0.02)
    with pytest.raises(ValueError):
        lat.tangent_step(np.zeros((27, 4, 4, 4)), np.zeros((27, 4, 4, 4)))


# ------------------------------------------------ MRT-LES collision
BASES = {"table1": oracle.BASIS_TABLE1, "dhumieres": oracle.BASIS_DHUMIERES}
# distinct free rates so that the spectrum shows each group's multiplicity
FREE_RATES = {"table1": (1.3, 1.1, 1.7, 0.9), "dhumieres": (1.19, 1.4, 1.2, 1.6, 1.98)}
# (rate index or "shear", number of moments) per group: Table 1 for D3Q19
# (s1 five shear moments, s2 the trace, s3 and s4 three third-order
# combinations each, s7 three fourth-order ones); the d'Humieres basis:
# energy, energy squared, three heat fluxes, five viscous stresses, two
# fourth-order stresses, three antisymmetric third-order moments
GROUPS = {"table1": [("shear", 5), (0, 1), (1, 3), (2, 3), (3, 3)],
          "dhumieres": [(0, 1), (1, 1), (2, 3), ("shear", 5), (3, 2), (4, 3)]}


def _mrt_lat(basis, nu=0.01, cs=0.1, rates=None):
    return oracle.Lattice(oracle.MRT19, 4, 4, 4, nu=nu, cs_smag=cs, basis=BASES[basis],
                          rates=rates)


def _mrt_state(seed, amp=1e-2):
    """One D3Q19 node: an incompressible equilibrium of a moving fluid plus
    noise (so that the strain and the eddy viscosity are non-zero)."""
    rng = np.random.default_rng(seed)
    drho = 0.02 * rng.uniform(-1, 1)
    u = 0.05 * rng.uniform(-1, 1, size=3)
    return oracle.feq_incomp(19, drho, u) + amp * rng.uniform(-1, 1, size=19)


def _jacobian(lat, f):
    return np.stack([lat.collide_jvp(f, np.eye(lat.Q)[j]) for j in range(lat.Q)], axis=1)


@pytest.mark.parametrize("basis", list(BASES))
def test_mrt_jvp_matches_central_difference(basis):
    nu, cs = 0.01, 0.1
    tau0 = 3 * nu + 0.5
    lat = _mrt_lat(basis, nu, cs)
    rng = np.random.default_rng(31)
    for seed in range(6):
        f = _mrt_state(seed)
        _, q = oracle.smagorinsky_tau(f, tau0, cs)
        assert q > 1e-4  # the eddy viscosity is active
        v = rng.standard_normal(19)
        h = 1e-6
        fp, _ = oracle.mrt_collide(f + h * v, tau0, cs, BASES[basis])
        fm, _ = oracle.mrt_collide(f - h * v, tau0, cs, BASES[basis])
        fd = (fp - fm) / (2 * h)
        jv = lat.collide_jvp(f, v)
        assert np.abs(jv - fd).max() <= 1e-8 * np.abs(fd).max()
        # without the strain term of tau the product differs: the LES part
        # is in the linearisation
        jv0 = _mrt_lat(basis, nu, 0.0).collide_jvp(f, v)
        assert np.abs(jv0 - jv).max() > 1e-6 * np.abs(jv).max()


@pytest.mark.parametrize("basis", list(BASES))
def test_mrt_jvp_keeps_mass_and_momentum(basis):
    lat = _mrt_lat(basis)
    e, _, _ = oracle.stencil(19)
    rng = np.random.default_rng(32)
    for seed in range(5):
        f = _mrt_state(seed)
        v = rng.standard_normal(19)
        jv = lat.collide_jvp(f, v)
        assert abs(jv.sum() - v.sum()) <= 1e-13 * np.abs(v).sum()
        assert np.abs(e.T @ jv - e.T @ v).max() <= 1e-13 * np.abs(v).sum()


@pytest.mark.parametrize("basis", list(BASES))
def test_mrt_linear_spectrum_at_rest(basis):
    """At rest the collision is the linear moment relaxation I - M^-1 S M
    (I - P) with P the linear equilibrium of mass and momentum: its
    eigenvalues are 1 four times and 1 - s_k for the other moments, with
    each group's multiplicity, and every non-conserved moment mode (a
    column of M^-1 whose mass and momentum vanish) is an eigenvector."""
    nu = 0.01
    tau0 = 3 * nu + 0.5
    rates = FREE_RATES[basis]
    lat = _mrt_lat(basis, nu, 0.1, rates)
    Jm = _jacobian(lat, np.zeros(19))
    want = [1.0] * 4
    for r, k in GROUPS[basis]:
        want += [1.0 - (1.0 / tau0 if r == "shear" else rates[r])] * k
    assert len(want) == 19
    got = np.sort(np.linalg.eigvals(Jm).real)
    np.testing.assert_allclose(got, np.sort(want), atol=1e-10)
    assert np.abs(np.linalg.eigvals(Jm).imag).max() <= 1e-10
    e, _, _ = oracle.stencil(19)
    Minv = np.linalg.inv(oracle.mrt_basis(BASES[basis]))
    modes = 0
    for k in range(19):
        v = Minv[:, k]
        if abs(v.sum()) > 1e-12 or np.abs(e.T @ v).max() > 1e-12:
            continue  # a mode that carries mass or momentum
        modes += 1
        jv = Jm @ v
        lam = float(jv @ v / (v @ v))
        np.testing.assert_allclose(jv, lam * v, atol=1e-13)
        assert min(abs(lam - x) for x in want[4:]) <= 1e-12
    assert modes == 15


@pytest.mark.parametrize("basis", list(BASES))
def test_mrt_equilibrium_tangent_is_fixed(basis):
    """Incompressible equilibria are fixed points of the MRT collision for
    every (drho, u) (their strain is zero, so is the eddy viscosity's
    argument), so the Jacobian there maps the family's tangent onto itself."""
    lat = _mrt_lat(basis)
    rng = np.random.default_rng(33)
    for _ in range(4):
        drho = 0.02 * rng.uniform(-1, 1)
        u = 0.05 * rng.uniform(-1, 1, size=3)
        d = rng.standard_normal(4)
        h = 1e-5
        t = (oracle.feq_incomp(19, drho + h * d[0], u + h * d[1:]) -
             oracle.feq_incomp(19, drho - h * d[0], u - h * d[1:])) / (2 * h)
        jv = lat.collide_jvp(oracle.feq_incomp(19, drho, u), t)
        assert np.abs(jv - t).max() <= 1e-9 * np.abs(t).max()
