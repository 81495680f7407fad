"""Pins of the oracle's jet spreading profile (the width of Eq. (23) and the
profile of Eq. (24), Section 3).

* A streamwise velocity linear in the cross-section is reproduced exactly by
  bilinear interpolation: along a ray it is linear, so the crossing radius
  of every ray has a closed form, and the ray-averaged profile is 1 (the
  linear parts cancel over a symmetric set of rays).
* A round Gaussian jet u_m exp(-(r/b)^2): r_e = b sqrt(ln(1/0.368)) on every
  ray, within the bilinear interpolation error; an elliptic one gives the
  two semi-axes as minimum and maximum.
* The same field laid along x, y or z gives the same result.
"""
import numpy as np
import pytest

import oracle

FR = oracle.SPREAD_FRACTION


def _field(fn, npl, nb, na):
    """[3][z][y][x] with the streamwise (z) component fn(p, a, b)."""
    p, b, a = np.meshgrid(np.arange(npl), np.arange(nb), np.arange(na), indexing="ij")
    m = np.zeros((3, npl, nb, na))
    m[2] = fn(p.astype(float), a.astype(float), b.astype(float))
    m[0] = 0.01 * a  # other components are ignored
    return m


def test_linear_section_closed_form():
    na, nb, npl = 21, 17, 3
    c = (10.25, 8.5)
    beta, gamma = -0.004, -0.0025
    alpha = np.array([0.1, 0.11, 0.12])
    m = _field(lambda p, a, b: alpha[p.astype(int)] + beta * a + gamma * b, npl, nb, na)
    ndir, dr, nr = 16, 0.25, 30  # the last section's crossings lie beyond nr samples
    um, re, prof = oracle.jet_profile(m, 2, c, ndir, dr, nr)
    for p in range(npl):
        u0 = alpha[p] + beta * c[0] + gamma * c[1]
        assert abs(um[p] - u0) <= 1e-15
        radii = []
        for j in range(ndir):
            th = 2 * np.pi * j / ndir
            s = beta * np.cos(th) + gamma * np.sin(th)
            if s >= 0:
                continue
            r = (FR - 1.0) * u0 / s
            a, b = c[0] + r * np.cos(th), c[1] + r * np.sin(th)
            # reached only if the samples up to the crossing stay inside
            kmax = int(np.ceil(r / dr))
            ea, eb = c[0] + kmax * dr * np.cos(th), c[1] + kmax * dr * np.sin(th)
            if kmax < nr and 0 <= ea <= na - 1 and 0 <= eb <= nb - 1:
                radii.append(r)
        if not radii:  # no ray reaches the crossing within nr samples
            assert np.all(np.isnan(re[:, p]))
            continue
        np.testing.assert_allclose(re[:, p], [min(radii), max(radii), np.mean(radii)],
                                   rtol=1e-12)
        np.testing.assert_allclose(prof[p], 1.0, atol=1e-12)


@pytest.mark.parametrize("bx,by", [(6.0, 6.0), (8.0, 5.0)])
def test_gaussian_jet_radius(bx, by):
    na = nb = 48
    c = (23.5, 23.5)
    m = _field(lambda p, a, b: (0.05 - 0.01 * p) *
               np.exp(-((a - c[0]) / bx) ** 2 - ((b - c[1]) / by) ** 2), 2, nb, na)
    um, re, prof = oracle.jet_profile(m, 2, c, 64, 0.2, 100)
    k = np.sqrt(np.log(1.0 / FR))
    for p in range(2):
        u0 = 0.05 - 0.01 * p
        assert abs(um[p] - u0) <= 0.02 * u0  # the centre sits between nodes
        assert abs(re[0, p] - k * min(bx, by)) <= 0.02 * k * min(bx, by)
        assert abs(re[1, p] - k * max(bx, by)) <= 0.02 * k * max(bx, by)
        if bx == by:
            # the ray-averaged profile follows the Gaussian
            r = 0.2 * np.arange(100)
            ok = r < 20
            np.testing.assert_allclose(prof[p, ok] * um[p] / u0, np.exp(-(r[ok] / bx) ** 2),
                                       atol=0.02)


def test_axis_permutations_agree():
    rng = np.random.default_rng(3)
    base = rng.uniform(0.0, 0.05, size=(3, 5, 9, 11))  # [3][z][y][x], streamwise z
    c = (5.2, 3.9)
    ref = oracle.jet_profile(base, 2, c, 12, 0.5, 12)
    # x as the jet axis: [3][z][y][x] with x <- old z, y <- old x, z <- old y
    mx = np.zeros((3, 9, 11, 5))
    mx[0] = np.transpose(base[2], (1, 2, 0))
    got = oracle.jet_profile(mx, 0, c, 12, 0.5, 12)
    for g, r in zip(got, ref):
        np.testing.assert_array_equal(g, r)
    # y as the jet axis: x <- old x, z <- old y, y <- old z
    my = np.zeros((3, 9, 5, 11))
    my[1] = np.transpose(base[2], (1, 0, 2))
    got = oracle.jet_profile(my, 1, c, 12, 0.5, 12)
    for g, r in zip(got, ref):
        np.testing.assert_array_equal(g, r)


def test_jet_laws_recover_their_constants():
    """Sections that follow Eqs. (22)-(24) exactly give back k_par, k_perp
    and a zero residual; an offset added to the profile comes back as the
    residual; sections at or upstream of the nozzle exit are ignored."""
    npl, nr, dr = 40, 30, 0.5
    x0, u0, d, kp, kq = 3.0, 0.05, 8.0, 6.104, 0.109
    p = np.arange(npl)
    x = p - x0
    um = np.where(x > 0, u0 * kp * d / np.where(x > 0, x, 1.0), 0.3)
    re = np.zeros((3, npl))
    re[2] = np.where(x > 0, kq * np.maximum(x, 1.0), np.nan)
    prof = np.full((npl, nr), np.nan)
    for q in range(npl):
        if x[q] > 0:
            r = dr * np.arange(nr)
            prof[q] = 0.938 * np.exp(-0.944 * (r / re[2, q]) ** 2)
    k_par, k_perp, res, n = oracle.jet_fit(um, re, prof, dr, x0, u0, d, 0, npl)
    assert abs(k_par - kp) <= 1e-12 * kp and abs(k_perp - kq) <= 1e-12 * kq
    assert res <= 1e-15 and n > 0
    _, _, res2, n2 = oracle.jet_fit(um, re, prof + 0.01, dr, x0, u0, d, 0, npl)
    assert abs(res2 - 0.01) <= 1e-12 and n2 == n
    # a single section, by hand: samples up to 2 r_e
    q = 20
    k_par1, k_perp1, _, n1 = oracle.jet_fit(um, re, prof, dr, x0, u0, d, q, q + 1)
    assert n1 == int(np.floor(2 * re[2, q] / dr)) + 1
    assert abs(k_perp1 - re[2, q] / x[q]) <= 1e-15
