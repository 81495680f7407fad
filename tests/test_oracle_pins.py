"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every check uses a printed
table of the paper, a closed form, an invariant, a textbook reduction or a
published test vector, chosen so that a dropped term, a wrong sign or index
or a transposed operand in the oracle fails at least one of them.
"""
import itertools
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden_sets():
    out = {}
    for line in open(os.path.join(GOLD, "velocity_sets.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, i, ex, ey, ez, num, den = line.split()
        out.setdefault(name, []).append((int(i), int(ex), int(ey), int(ez),
                                         int(num) / int(den)))
    return out


@pytest.mark.parametrize("Q", [19, 27])
def test_velocity_sets_match_paper_tables(Q):
    gold = _golden_sets()["D3Q%d" % Q]
    e, w, opp = oracle.stencil(Q)
    assert len(gold) == Q
    for i, ex, ey, ez, wi in gold:
        assert tuple(e[i]) == (ex, ey, ez)
        assert w[i] == pytest.approx(wi, abs=1e-16)
    for i in range(Q):
        assert tuple(e[opp[i]]) == tuple(-e[i])


@pytest.mark.parametrize("Q", [19, 27])
def test_stencil_isotropy(Q):
    e, w, _ = oracle.stencil(Q)
    e = e.astype(float)
    d = np.eye(3)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.abs(np.einsum("i,ia->a", w, e)).max() < 1e-16
    assert np.allclose(np.einsum("i,ia,ib->ab", w, e, e), d / 3, atol=1e-16)
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, e, e, e)).max() < 1e-16
    four = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
            + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e), four, atol=1e-16)


@pytest.mark.parametrize("Q", [19, 27])
def test_incompressible_equilibrium_moments(Q):
    """Eq. (2): sum f_eq = drho, sum f_eq e = u, sum f_eq e e = drho/3 I + u u."""
    e, w, _ = oracle.stencil(Q)
    rng = np.random.default_rng(1)
    for _ in range(5):
        drho = rng.uniform(-0.05, 0.05)
        u = rng.uniform(-0.1, 0.1, 3)
        feq = oracle.feq_incomp(Q, drho, u)
        assert feq.sum() == pytest.approx(drho, abs=1e-15)
        assert np.allclose(feq @ e, u, atol=1e-15)
        P = np.einsum("i,ia,ib->ab", feq, e, e)
        assert np.allclose(P, drho / 3 * np.eye(3) + np.outer(u, u), atol=1e-15)


# ----------------------------------------------------------------------------
# MRT (Eq. 12, Table 1) and the Smagorinsky closure (Eqs. 16-21)

BASES = [oracle.BASIS_TABLE1, oracle.BASIS_DHUMIERES]


@pytest.mark.parametrize("basis", BASES)
def test_mrt_conserves_mass_and_momentum(basis):
    e, w, _ = oracle.stencil(19)
    rng = np.random.default_rng(2)
    for _ in range(20):
        f = rng.uniform(-0.02, 0.02, 19)
        fs, _ = oracle.mrt_collide(f, 0.52, cs=0.1, basis=basis)
        assert fs.sum() == pytest.approx(f.sum(), abs=1e-16)
        assert np.allclose(fs @ e, f @ e, atol=1e-16)


@pytest.mark.parametrize("basis", BASES)
def test_mrt_equilibrium_is_fixed_point(basis):
    rng = np.random.default_rng(3)
    for _ in range(10):
        feq = oracle.feq_incomp(19, rng.uniform(-0.05, 0.05), rng.uniform(-0.1, 0.1, 3))
        rates = rng.uniform(0.5, 1.9, 5)
        fs, tau = oracle.mrt_collide(feq, 0.7, cs=0.18, basis=basis, rates=rates)
        assert tau == pytest.approx(0.7, abs=1e-14)  # no strain -> tau0
        assert np.allclose(fs, feq, atol=1e-16)


@pytest.mark.parametrize("basis", BASES)
def test_mrt_unit_rates_map_to_equilibrium(basis):
    """All rates 1 (tau0 = 1, no eddy viscosity): f* = f_eq of the input."""
    e, _, _ = oracle.stencil(19)
    rng = np.random.default_rng(4)
    f = rng.uniform(-0.02, 0.02, 19)
    fs, _ = oracle.mrt_collide(f, 1.0, cs=0.0, basis=basis, rates=[1.0] * 5)
    assert np.allclose(fs, oracle.feq_incomp(19, f.sum(), f @ e), atol=1e-16)


@pytest.mark.parametrize("basis", BASES)
def test_mrt_equal_rates_reduce_to_bgk(basis):
    """Every rate = 1/tau, no Smagorinsky: Eq. (12) becomes the BGK update of
    Eq. (1), read as f* = f - (f - f_eq)/tau."""
    e, _, _ = oracle.stencil(19)
    rng = np.random.default_rng(5)
    for tau in (0.55, 0.8, 1.7):
        f = rng.uniform(-0.02, 0.02, 19)
        fs, _ = oracle.mrt_collide(f, tau, cs=0.0, basis=basis, rates=[1 / tau] * 5)
        feq = oracle.feq_incomp(19, f.sum(), f @ e)
        assert np.allclose(fs, f - (f - feq) / tau, atol=1e-16)


def test_dhumieres_basis_is_orthogonal_and_table1_invertible():
    M = oracle.mrt_basis(oracle.BASIS_DHUMIERES)
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-12
    M1 = oracle.mrt_basis(oracle.BASIS_TABLE1)
    assert np.linalg.cond(M1) < 100
    assert np.linalg.matrix_rank(M1) == 19


@pytest.mark.parametrize("cs", [0.0, 0.1, 0.18, 0.5])
def test_smagorinsky_recovers_chapman_enskog_strain(cs):
    """A Chapman-Enskog state f = f_eq - 3 tau w_i (e_i e_i - I/3):S must return
    tau_total = tau0 + 3 C_S^2 |S|, |S| = sqrt(2 S:S): the lattice form of
    nu_T = (C_S dx)^2 |S| (Eq. 16) with nu = (tau - 1/2)/3 (Eq. 13)."""
    e, w, _ = oracle.stencil(19)
    e = e.astype(float)
    rng = np.random.default_rng(6)
    tau0 = 0.51
    for _ in range(10):
        A = rng.normal(size=(3, 3)) * 1e-3
        S = 0.5 * (A + A.T)
        S -= np.trace(S) / 3 * np.eye(3)
        Snorm = np.sqrt(2 * np.sum(S * S))
        tau_t = tau0 + 3 * cs * cs * Snorm
        Qi = np.einsum("ia,ib->iab", e, e) - np.eye(3) / 3
        fneq = -3 * tau_t * w * np.einsum("iab,ab->i", Qi, S)
        drho, u = rng.uniform(-0.01, 0.01), rng.uniform(-0.05, 0.05, 3)
        f = oracle.feq_incomp(19, drho, u) + fneq
        tau, Q = oracle.smagorinsky_tau(f, tau0, cs)
        assert tau == pytest.approx(tau_t, rel=1e-13)
        # the closed form Eq. (20) solves tau^2 - tau0 tau - 9/2 C_S^2 Q = 0
        assert tau * tau - tau0 * tau - 4.5 * cs * cs * Q == pytest.approx(0, abs=1e-16)


# ----------------------------------------------------------------------------
# Central moments (Eq. 15) against the printed Table 2 transformations

def _raw(F, e, idx):
    """mu_{idx} per unit mass in the paper's index notation ('112' = x x y)."""
    a, b, c = idx.count("1"), idx.count("2"), idx.count("3")
    rho = F.sum()
    return float(np.sum(F * e[:, 0] ** a * e[:, 1] ** b * e[:, 2] ** c) / rho)


def _table2(F, e):
    m = lambda s: _raw(F, e, s)  # noqa: E731
    m1, m2, m3 = m("1"), m("2"), m("3")
    T = {}
    T["11"] = m("11") - m1 ** 2
    T["22"] = m("22") - m2 ** 2
    T["33"] = m("33") - m3 ** 2
    T["12"] = m("12") - m1 * m2
    T["13"] = m("13") - m1 * m3
    T["23"] = m("23") - m2 * m3
    T["112"] = m("112") - m("11") * m2 - 2 * m1 * m("12") + 2 * m1 * m1 * m2
    T["122"] = m("122") - m("22") * m1 - 2 * m2 * m("12") + 2 * m1 * m2 * m2
    T["113"] = m("113") - m("11") * m3 - 2 * m1 * m("13") + 2 * m1 * m1 * m3
    T["133"] = m("133") - m("33") * m1 - 2 * m3 * m("13") + 2 * m1 * m3 * m3
    T["223"] = m("223") - m("22") * m3 - 2 * m2 * m("23") + 2 * m2 * m2 * m3
    T["233"] = m("233") - m("33") * m2 - 2 * m3 * m("23") + 2 * m2 * m3 * m3
    # printed with -mu3 mu12 twice; read the second as -mu2 mu13
    T["123"] = (m("123") - m("12") * m3 - m("23") * m1 - m2 * m("13")
                + 2 * m1 * m2 * m3)
    # printed with an extra +4 mu11 mu22 (likewise 1133, 2233); dropped
    T["1122"] = (m("1122") - 2 * m("112") * m2 - 2 * m("122") * m1 + m1 ** 2 * m("22")
                 + m("11") * m2 ** 2 + 4 * m1 * m2 * m("12") - 3 * m1 ** 2 * m2 ** 2)
    T["1133"] = (m("1133") - 2 * m("113") * m3 - 2 * m("133") * m1 + m1 ** 2 * m("33")
                 + m("11") * m3 ** 2 + 4 * m1 * m3 * m("13") - 3 * m1 ** 2 * m3 ** 2)
    T["2233"] = (m("2233") - 2 * m("223") * m3 - 2 * m("233") * m2 + m2 ** 2 * m("33")
                 + m("22") * m3 ** 2 + 4 * m2 * m3 * m("23") - 3 * m2 ** 2 * m3 ** 2)
    T["1233"] = (-3 * m3 ** 2 * m2 * m1 + m("33") * m2 * m1 + 2 * m3 * m("23") * m1
                 - m("233") * m1 + 2 * m3 * m2 * m("13") - m2 * m("133")
                 + m3 ** 2 * m("12") - 2 * m3 * m("123") + m("1233"))
    T["1223"] = (-3 * m2 ** 2 * m3 * m1 + m("22") * m3 * m1 + 2 * m2 * m("23") * m1
                 - m("223") * m1 + 2 * m3 * m2 * m("12") - m3 * m("122")
                 + m2 ** 2 * m("13") - 2 * m2 * m("123") + m("1223"))
    T["1123"] = (-3 * m1 ** 2 * m2 * m3 + m("11") * m2 * m3 + 2 * m3 * m("12") * m1
                 - m("112") * m3 + 2 * m1 * m2 * m("13") - m2 * m("113")
                 + m1 ** 2 * m("23") - 2 * m1 * m("123") + m("1123"))
    T["11223"] = (4 * m3 * m2 ** 2 * m1 ** 2 - 2 * m2 * m("23") * m1 ** 2
                  - m3 * m("22") * m1 ** 2 + m("223") * m1 ** 2 - 2 * m2 ** 2 * m1 * m("13")
                  - 4 * m3 * m2 * m1 * m("12") + 4 * m2 * m1 * m("123")
                  + 2 * m3 * m1 * m("122") - 2 * m1 * m("1223") - m3 * m2 ** 2 * m("11")
                  + m2 ** 2 * m("113") + 2 * m3 * m2 * m("112") - 2 * m2 * m("1123")
                  - m3 * m("1122") + m("11223"))
    T["11233"] = (4 * m3 ** 2 * m2 * m1 ** 2 - m("33") * m2 * m1 ** 2
                  - 2 * m3 * m("23") * m1 ** 2 + m("233") * m1 ** 2
                  - 4 * m3 * m2 * m1 * m("13") + 2 * m2 * m1 * m("133")
                  - 2 * m3 ** 2 * m1 * m("12") + 4 * m3 * m1 * m("123")
                  - 2 * m1 * m("1233") - m3 ** 2 * m2 * m("11") + 2 * m3 * m2 * m("113")
                  - m2 * m("1133") + m3 ** 2 * m("112") - 2 * m3 * m("1123") + m("11233"))
    T["12233"] = (4 * m3 ** 2 * m2 ** 2 * m1 - m("33") * m2 ** 2 * m1
                  - 2 * m3 * m("13") * m2 ** 2 + m("133") * m2 ** 2
                  - 4 * m3 * m2 * m1 * m("23") + 2 * m2 * m1 * m("233")
                  - 2 * m3 ** 2 * m2 * m("12") + 4 * m3 * m2 * m("123")
                  - 2 * m2 * m("1233") - m3 ** 2 * m1 * m("22") + 2 * m3 * m1 * m("223")
                  - m1 * m("2233") + m3 ** 2 * m("122") - 2 * m3 * m("1223") + m("12233"))
    T["112233"] = (-5 * m3 ** 2 * m2 ** 2 * m1 ** 2 + m("33") * m2 ** 2 * m1 ** 2
                   + 4 * m3 * m2 * m("23") * m1 ** 2 - 2 * m2 * m("233") * m1 ** 2
                   + m3 ** 2 * m("22") * m1 ** 2 - 2 * m3 * m("223") * m1 ** 2
                   + m("2233") * m1 ** 2 + 4 * m3 * m2 ** 2 * m1 * m("13")
                   - 2 * m2 ** 2 * m1 * m("133") + 4 * m3 ** 2 * m2 * m1 * m("12")
                   - 8 * m3 * m2 * m1 * m("123") + 4 * m2 * m1 * m("1233")
                   - 2 * m3 ** 2 * m1 * m("122") + 4 * m3 * m1 * m("1223")
                   - 2 * m1 * m("12233") + m3 ** 2 * m2 ** 2 * m("11")
                   - 2 * m3 * m2 ** 2 * m("113") + m2 ** 2 * m("1133")
                   - 2 * m3 * m3 * m2 * m("112") + 4 * m3 * m2 * m("1123")
                   - 2 * m2 * m("11233") + m3 ** 2 * m("1122") - 2 * m3 * m("11223")
                   + m("112233"))
    return T


def test_central_moments_match_table2_transformations():
    e, w, _ = oracle.stencil(27)
    e = e.astype(float)
    rng = np.random.default_rng(7)
    for _ in range(10):
        F = w * (1 + rng.uniform(-0.3, 0.3, 27))
        rho, u, k = oracle.central_moments(F)
        assert rho == pytest.approx(F.sum(), abs=1e-15)
        assert np.allclose(u, (F @ e) / F.sum(), atol=1e-16)
        for idx, val in _table2(F, e).items():
            a, b, c = idx.count("1"), idx.count("2"), idx.count("3")
            assert k[a, b, c] == pytest.approx(val, abs=1e-14), idx


# ----------------------------------------------------------------------------
# FCLB collision

def _product_eq(rho, u):
    """Closed form: rho prod_a phi(e_a; u_a), phi(0)=2/3-u^2,
    phi(+-1)=(1/3+u^2+-u)/2 -- central moments 1, 0, 1/3 per direction."""
    e, _, _ = oracle.stencil(27)
    def phi(c, v):
        return np.where(c == 0, 2 / 3 - v * v, 0.5 * (1 / 3 + v * v + c * v))
    return rho * phi(e[:, 0], u[0]) * phi(e[:, 1], u[1]) * phi(e[:, 2], u[2])


def test_product_equilibrium_closed_form():
    rng = np.random.default_rng(8)
    rho, u = 1.02, rng.uniform(-0.1, 0.1, 3)
    F = oracle.feq_product(rho, u)
    assert np.allclose(F, _product_eq(rho, u), atol=1e-16)
    _, uu, k = oracle.central_moments(F)
    assert np.allclose(uu, u, atol=1e-15)
    expect = np.zeros((3, 3, 3))
    cm = [1.0, 0.0, 1.0 / 3.0]
    for a, b, c in itertools.product(range(3), repeat=3):
        expect[a, b, c] = cm[a] * cm[b] * cm[c]
    assert np.allclose(k, expect, atol=1e-15)


def test_fclb_conserves_mass_and_momentum():
    e, w, _ = oracle.stencil(27)
    rng = np.random.default_rng(9)
    for omega in (0.6, 1.0, 1.5, 1.95):
        f = rng.uniform(-0.01, 0.01, 27)
        fs = oracle.fclb_collide(f, omega)
        assert fs.sum() == pytest.approx(f.sum(), abs=1e-15)
        assert np.allclose(fs @ e, f @ e, atol=1e-15)


def test_fclb_product_equilibrium_is_fixed_point():
    _, w, _ = oracle.stencil(27)
    rng = np.random.default_rng(10)
    for omega in (0.6, 1.2, 1.9):
        rho, u = 1 + rng.uniform(-0.05, 0.05), rng.uniform(-0.1, 0.1, 3)
        f = _product_eq(rho, u) - w
        assert np.allclose(oracle.fclb_collide(f, omega), f, atol=1e-15)


def test_fclb_unit_rate_maps_to_product_equilibrium():
    e, w, _ = oracle.stencil(27)
    rng = np.random.default_rng(11)
    f = rng.uniform(-0.01, 0.01, 27)
    rho = 1 + f.sum()
    u = (f @ e) / rho
    assert np.allclose(oracle.fclb_collide(f, 1.0) + w, _product_eq(rho, u), atol=1e-15)


def test_fclb_post_collision_moments():
    """The relaxed second order: trace 1, deviator scaled by (1 - omega);
    third and fifth order vanish; fourth/sixth are the Table 2 products."""
    _, w, _ = oracle.stencil(27)
    rng = np.random.default_rng(12)
    omega = 1.3
    f = rng.uniform(-0.01, 0.01, 27)
    _, _, k = oracle.central_moments(f + w)
    _, _, ks = oracle.central_moments(oracle.fclb_collide(f, omega) + w)
    dev = np.array([k[2, 0, 0], k[0, 2, 0], k[0, 0, 2]])
    dev -= dev.sum() / 3
    devs = np.array([ks[2, 0, 0], ks[0, 2, 0], ks[0, 0, 2]])
    assert devs.sum() == pytest.approx(1.0, abs=1e-14)
    assert np.allclose(devs - 1 / 3, (1 - omega) * dev, atol=1e-14)
    for ab in [(1, 1, 0), (1, 0, 1), (0, 1, 1)]:
        assert ks[ab] == pytest.approx((1 - omega) * k[ab], abs=1e-14)
    odd = [(a, b, c) for a, b, c in itertools.product(range(3), repeat=3)
           if (a + b + c) in (1, 3, 5)]
    for idx in odd:
        assert abs(ks[idx]) < 1e-14, idx
    assert ks[2, 2, 0] == pytest.approx(ks[2, 0, 0] * ks[0, 2, 0], abs=1e-14)
    assert ks[2, 1, 1] == pytest.approx(ks[2, 0, 0] * ks[0, 1, 1], abs=1e-14)
    assert ks[1, 1, 2] == pytest.approx(ks[0, 0, 2] * ks[1, 1, 0], abs=1e-14)
    assert ks[2, 2, 2] == pytest.approx(ks[2, 0, 0] * ks[0, 2, 0] * ks[0, 0, 2], abs=1e-14)


def _perm(e, R):
    """Population permutation P with (P f)_j = f_i for e_j = R e_i."""
    Q = len(e)
    idx = {tuple(v): i for i, v in enumerate(e)}
    P = np.zeros((Q, Q))
    for i in range(Q):
        P[idx[tuple(R @ e[i])], i] = 1.0
    return P


@pytest.mark.parametrize("model", [oracle.MRT19, oracle.FCLB27])
def test_collisions_commute_with_cube_symmetries(model):
    Q = oracle.q_of(model)
    e, _, _ = oracle.stencil(Q)
    rng = np.random.default_rng(13)
    Rz = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]])
    Mx = np.diag([-1, 1, 1])
    def C(f):
        if model == oracle.MRT19:
            return oracle.mrt_collide(f, 0.53, cs=0.15, basis=oracle.BASIS_DHUMIERES)[0]
        return oracle.fclb_collide(f, 1.4)
    for R in (Rz, Rx, Mx):
        P = _perm(e, R)
        f = rng.uniform(-0.01, 0.01, Q)
        assert np.allclose(C(P @ f), P @ C(f), atol=1e-15)
    if model == oracle.MRT19:
        # the Table 1 basis is symmetric as a set of groups too
        for R in (Rz, Rx, Mx):
            P = _perm(e, R)
            f = rng.uniform(-0.01, 0.01, Q)
            c = lambda g: oracle.mrt_collide(g, 0.53, cs=0.15, basis=oracle.BASIS_TABLE1,  # noqa
                                             rates=[1.1, 1.2, 1.3, 1.4])[0]
            assert np.allclose(c(P @ f), P @ c(f), atol=1e-15)


# ----------------------------------------------------------------------------
# Lattice: streaming, boundary rules, hydrodynamics

def test_splitmix64_published_vector():
    lines = [l.split() for l in open(os.path.join(GOLD, "splitmix64.txt"))
             if l.strip() and not l.startswith("#")]
    seed = int(lines[0][1])
    gamma = 0x9E3779B97F4A7C15
    for k, (val,) in enumerate(lines[1:]):
        assert oracle.splitmix64((seed + k * gamma) & (2 ** 64 - 1)) == int(val)


def test_inlet_uniform_statistics():
    u = np.array([oracle.inlet_uniform(12060389, t, a, b, c)
                  for t in range(4) for a in range(16) for b in range(16) for c in range(3)])
    assert 0.0 <= u.min() and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.03
    assert abs(u.var() - 1 / 12) < 0.01


@pytest.mark.parametrize("model", [oracle.MRT19, oracle.FCLB27])
def test_first_mass_moment_moves_with_momentum(model):
    """Exact streaming law: sum_x x drho(t+1) = sum_x x drho(t) + J(t).
    Pins the direction of streaming (pull from x - e_i) and conservation."""
    Q = oracle.q_of(model)
    n = 12
    lat = oracle.Lattice(model, n, n, n, nu=0.02, cs_smag=0.1)
    rng = np.random.default_rng(14)
    f = np.zeros((Q, n, n, n))
    f[:, 3:9, 3:9, 3:9] = rng.uniform(-0.01, 0.01, (Q, 6, 6, 6))
    e, _, _ = oracle.stencil(Q)
    X = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    pos = [X[2], X[1], X[0]]
    for _ in range(2):
        d0 = f.sum(0)
        J = np.einsum("in,ia->a", f.reshape(Q, -1), e)
        g = lat.run(f, 0, 1)
        d1 = g.sum(0)
        for a in range(3):
            # per-node conservation holds to ~1e-16; 216 nodes at |x| <= 12
            assert np.sum(pos[a] * d1) - np.sum(pos[a] * d0) == pytest.approx(J[a], abs=1e-11)
        assert d1.sum() == pytest.approx(d0.sum(), abs=1e-12)
        f = g


def _shear_decay_nu(model, n, nu, steps, u0=1e-4):
    lat = oracle.Lattice(model, 1, n, 1, nu=nu)
    import synth
    drho, u = synth.shear_wave(1, n, 1, u0)
    f = lat.init_equilibrium(drho, u)
    amps = []
    y = np.arange(n)
    for _ in range(2):
        f = lat.run(f, 0, steps)
        _, uu = lat.macroscopic(f)
        amps.append(2 / n * np.sum(uu[0, 0, :, 0] * np.sin(2 * np.pi * y / n)))
    k = 2 * np.pi / n
    return np.log(amps[0] / amps[1]) / (steps * k * k)


@pytest.mark.parametrize("model", [oracle.MRT19, oracle.FCLB27, oracle.CLB27])
def test_shear_wave_viscosity_converges(model):
    """Shear-wave amplitude decays as exp(-nu k^2 t) with nu = (1/omega-1/2)/3
    (Eq. 13); the lattice error is O(k^2), so it shrinks 4x per refinement."""
    nu = 0.05
    err = []
    for n in (16, 32):
        measured = _shear_decay_nu(model, n, nu, steps=int(0.05 * n * n / nu / 10))
        err.append(abs(measured / nu - 1))
    assert err[1] < 0.01
    assert err[1] < err[0] / 2.5 or err[1] < 1e-4


@pytest.mark.parametrize("model", [oracle.MRT19, oracle.FCLB27])
def test_taylor_green_energy_decay_rate(model):
    """Taylor-Green decay without an eddy viscosity: dE/dt / E -> -6 nu k0^2
    (three shear modes with |k|^2 = 3 k0^2). Measured after the kinetic
    transient of the equilibrium start; the O(k^2) lattice error must shrink
    under refinement."""
    import synth
    u0, nu = 0.01, 0.02
    err = []
    for n in (16, 32):
        lat = oracle.Lattice(model, n, n, n, nu=nu, cs_smag=0.0)
        drho, u = synth.taylor_green(n, u0)
        f = lat.run(lat.init_equilibrium(drho, u), 0, 50)
        E0 = lat.reduce(f)[4]
        f = lat.run(f, 50, 50)
        rate = np.log(lat.reduce(f)[4] / E0) / 50
        k0 = 2 * np.pi / n
        err.append(abs(rate / (-6 * nu * k0 * k0) - 1))
    assert err[1] < 0.04
    assert err[1] < err[0] / 2


def test_smagorinsky_taylor_green_decay_matches_les_dissipation():
    """With an eddy viscosity as large as nu, the measured energy decay equals
    the LES dissipation -sum 2 (nu + C_S^2 |S|) S:S / E (Eqs. 16-17, |S| =
    sqrt(2 S:S)) evaluated with spectral derivatives of the lattice's own
    velocity field. A sqrt(2) or factor-2 slip in Eqs. (18)-(21) moves the
    eddy part by 40-100 %, far outside the 5 % lattice error allowed here."""
    import synth
    n, u0, nu, cs, t0, steps = 32, 0.05, 0.01, 1.0, 60, 20
    lat = oracle.Lattice(oracle.MRT19, n, n, n, nu=nu, cs_smag=cs)
    drho, u = synth.taylor_green(n, u0)
    f = lat.run(lat.init_equilibrium(drho, u), 0, t0)
    k = 2 * np.pi * np.fft.fftfreq(n)

    def les_rate(f, c):
        _, uu = lat.macroscopic(f)
        G = np.zeros((3, 3, n, n, n))
        kk = [k[None, None, :], k[None, :, None], k[:, None, None]]  # x, y, z
        for a in range(3):
            U = np.fft.fftn(uu[a])
            for b in range(3):
                G[a, b] = np.real(np.fft.ifftn(1j * kk[b] * U))
        S = 0.5 * (G + G.transpose(1, 0, 2, 3, 4))
        SS = np.sum(S * S, axis=(0, 1))
        nut = c * c * np.sqrt(2 * SS)
        E = 0.5 * np.sum(uu * uu)
        return -np.sum(2 * (nu + nut) * SS) / E

    E0 = lat.reduce(f)[4]
    g = lat.run(f, t0, steps)
    rate = np.log(lat.reduce(g)[4] / E0) / steps
    predicted = 0.5 * (les_rate(f, cs) + les_rate(g, cs))
    molecular = 0.5 * (les_rate(f, 0.0) + les_rate(g, 0.0))
    assert rate == pytest.approx(predicted, rel=0.05)
    assert rate < 1.5 * molecular  # the eddy part is at least half of the total


@pytest.mark.parametrize("model", [oracle.MRT19, oracle.FCLB27])
def test_couette_flow_with_moving_wall(model):
    """Halfway bounce-back, static wall at y = -1/2, wall moving with u_w at
    y = ny - 1/2: the steady profile is linear, u_x = u_w (y + 1/2) / ny."""
    ny, uw = 8, 0.01
    faces = [oracle.PERIODIC, oracle.PERIODIC, oracle.WALL, oracle.WALL,
             oracle.PERIODIC, oracle.PERIODIC]
    face_u = [[0, 0, 0]] * 6
    face_u = [list(v) for v in face_u]
    face_u[3] = [uw, 0, 0]
    lat = oracle.Lattice(model, 1, ny, 1, nu=1 / 6, faces=faces, face_u=face_u)
    f = np.zeros((lat.Q, 1, ny, 1))
    f = lat.run(f, 0, 4000)
    drho, u = lat.macroscopic(f)
    y = np.arange(ny)
    assert np.allclose(u[0, 0, :, 0], uw * (y + 0.5) / ny, rtol=0, atol=1e-9 * uw)
    assert np.abs(u[1]).max() < 1e-12 and np.abs(drho).max() < 1e-9


@pytest.mark.parametrize("model", [oracle.MRT19, oracle.FCLB27])
def test_inlet_outflow_plug_flow_carries_inlet_flux(model):
    """Velocity inlet at z = -1/2 and zero-gradient outflow, periodic sides:
    the flow settles to a plug carrying the inlet momentum. The inlet term
    6 w_i rho0 (e_i . u_in) with rho0 = 1 fixes the momentum j = rho0 u_in, so
    the compressible model's velocity is j / rho."""
    nz, uin = 16, 0.02
    faces = [oracle.PERIODIC] * 4 + [oracle.INLET, oracle.OUTFLOW]
    iu = np.zeros((3, 2, 2))
    iu[2] = uin
    lat = oracle.Lattice(model, 2, 2, nz, nu=0.1, faces=faces, inlet_u=iu)
    f = lat.run(np.zeros((lat.Q, nz, 2, 2)), 0, 3000)
    drho, u = lat.macroscopic(f)
    rho = 1.0 if model == oracle.MRT19 else 1.0 + drho
    assert np.allclose(rho * u[2], uin, rtol=1e-3)
    assert np.abs(u[0]).max() < 1e-12 and np.abs(u[1]).max() < 1e-12


# Moment polynomials typed here from their published definitions, independent
# of the oracle's tables: d'Humieres et al. (2002) orthogonal D3Q19 basis with
# the name of the rate each row relaxes with ("nu" = the viscous rate 1/tau).
_DH_ROWS = [
    ("rho", lambda x, y, z: 1.0, None),
    ("e", lambda x, y, z: 19 * (x * x + y * y + z * z) - 30, "s_e"),
    ("eps", lambda x, y, z: (21 * (x * x + y * y + z * z) ** 2
                             - 53 * (x * x + y * y + z * z) + 24) / 2, "s_eps"),
    ("jx", lambda x, y, z: x, None),
    ("qx", lambda x, y, z: (5 * (x * x + y * y + z * z) - 9) * x, "s_q"),
    ("jy", lambda x, y, z: y, None),
    ("qy", lambda x, y, z: (5 * (x * x + y * y + z * z) - 9) * y, "s_q"),
    ("jz", lambda x, y, z: z, None),
    ("qz", lambda x, y, z: (5 * (x * x + y * y + z * z) - 9) * z, "s_q"),
    ("pxx", lambda x, y, z: 3 * x * x - (x * x + y * y + z * z), "nu"),
    ("pixx", lambda x, y, z: (3 * (x * x + y * y + z * z) - 5)
     * (3 * x * x - (x * x + y * y + z * z)), "s_pi"),
    ("pww", lambda x, y, z: y * y - z * z, "nu"),
    ("piww", lambda x, y, z: (3 * (x * x + y * y + z * z) - 5) * (y * y - z * z), "s_pi"),
    ("pxy", lambda x, y, z: x * y, "nu"),
    ("pyz", lambda x, y, z: y * z, "nu"),
    ("pxz", lambda x, y, z: x * z, "nu"),
    ("mx", lambda x, y, z: (y * y - z * z) * x, "s_m"),
    ("my", lambda x, y, z: (z * z - x * x) * y, "s_m"),
    ("mz", lambda x, y, z: (x * x - y * y) * z, "s_m"),
]

# Table 1 of the paper: moment groups and their rate names (s1 = the shear
# rate 1/tau; the two fourth-order rows printed with the label s7 relax at s7,
# and the third the same: "for D3Q19 only s1, s2, s3, s4, s7").
_T1_ROWS = [
    (lambda x, y, z: 1.0, None), (lambda x, y, z: x, None), (lambda x, y, z: y, None),
    (lambda x, y, z: z, None),
    (lambda x, y, z: x * y, "s1"), (lambda x, y, z: x * z, "s1"),
    (lambda x, y, z: y * z, "s1"), (lambda x, y, z: x * x - y * y, "s1"),
    (lambda x, y, z: x * x - z * z, "s1"), (lambda x, y, z: x * x + y * y + z * z, "s2"),
    (lambda x, y, z: x * y * y + x * z * z, "s3"), (lambda x, y, z: x * x * y + y * z * z, "s3"),
    (lambda x, y, z: x * x * z + y * y * z, "s3"),
    (lambda x, y, z: x * y * y - x * z * z, "s4"), (lambda x, y, z: x * x * y - y * z * z, "s4"),
    (lambda x, y, z: x * x * z - y * y * z, "s4"),
    (lambda x, y, z: x * x * y * y - 2 * x * x * z * z + y * y * z * z, "s7"),
    (lambda x, y, z: x * x * y * y + x * x * z * z - 2 * y * y * z * z, "s7"),
    (lambda x, y, z: x * x * y * y + x * x * z * z + y * y * z * z, "s7"),
]


def _typed_basis(rows):
    e, _, _ = oracle.stencil(19)
    return np.array([[r[1 if len(r) == 3 else 0](*e[i]) for i in range(19)]
                     for r in rows], dtype=float)


def test_dhumieres_rates_relax_their_named_moments():
    """Perturb the rest state along one published d'Humieres moment (its row
    itself: the basis is orthogonal, so no other moment is excited; the
    perturbation has no mass or momentum, so f_eq stays 0 and the collision
    is linear). With C_S = 0 the named moment must relax by (1 - s_named)
    and every other published moment must stay 0. Distinct rates per group
    (and a viscous rate 1/tau0 different from all of them) make any swap of
    the rate-to-row mapping fail."""
    Mt = _typed_basis(_DH_ROWS)
    G = Mt @ Mt.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-12  # the typed rows are orthogonal
    tau0 = 0.8
    named = {"s_e": 1.11, "s_eps": 1.33, "s_q": 1.55, "s_pi": 1.77, "s_m": 1.91,
             "nu": 1.0 / tau0}
    rates = [named[k] for k in ("s_e", "s_eps", "s_q", "s_pi", "s_m")]
    for k, (name, _, rate) in enumerate(_DH_ROWS):
        if rate is None:
            continue
        f = 1e-3 * Mt[k]
        fs, tau = oracle.mrt_collide(f, tau0, cs=0.0, basis=oracle.BASIS_DHUMIERES,
                                     rates=rates)
        assert abs(tau - tau0) < 1e-15
        m0, m1 = Mt @ f, Mt @ fs
        want = m0.copy()
        want[k] *= 1.0 - named[rate]
        assert np.abs(m1 - want).max() < 1e-15 * np.abs(m0).max() * 10, name


def test_table1_rates_relax_their_named_groups():
    """The same check for the Table 1 groups (not orthogonal: the test
    inverts its own typed basis to excite one moment alone): the perturbed
    moment relaxes by (1 - s) of its group, the other 18 moments stay."""
    Mt = _typed_basis(_T1_ROWS)
    Minv = np.linalg.inv(Mt)
    tau0 = 0.8
    named = {"s1": 1.0 / tau0, "s2": 1.1, "s3": 1.35, "s4": 1.6, "s7": 1.85}
    rates = [named[k] for k in ("s2", "s3", "s4", "s7")]
    for k, (_, rate) in enumerate(_T1_ROWS):
        if rate is None:
            continue
        unit = np.zeros(19)
        unit[k] = 1e-3
        f = Minv @ unit
        fs, _ = oracle.mrt_collide(f, tau0, cs=0.0, basis=oracle.BASIS_TABLE1, rates=rates)
        m1 = Mt @ fs
        want = unit.copy()
        want[k] *= 1.0 - named[rate]
        assert np.abs(m1 - want).max() < 1e-16, (k, rate)
