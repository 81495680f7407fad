"""Pins of the oracle's time averages (the jet statistics of Section 3:
mean velocity and the turbulent intensity of Eq. (25)).

Each check fixes its answer independently of the oracle's formula: a
constant sequence has no fluctuation (up to the rounding of its sum); a sequence alternating m + a, m - a
has mean m and rms |a|; a ramp 0, c, ..., (K-1) c has mean c (K-1)/2 and the
population variance c^2 (K^2 - 1)/12 (a sum of squares in closed form); the
turbulent intensity of fields built with a known axis velocity and a known
fluctuation is their ratio.
"""
import numpy as np
import pytest

import oracle

SHAPE = (3, 4, 3, 5)  # [3][nz][ny][nx]


def _field(seed):
    return np.random.default_rng(seed).normal(size=SHAPE)


def test_constant_sequence_has_no_fluctuation():
    u = _field(1)
    mean, rms, _ = oracle.velocity_statistics([u.copy() for _ in range(9)])
    # the only error is the rounding of the running sum (9 terms)
    assert np.allclose(mean, u, rtol=1e-15, atol=0)
    assert np.all(rms <= 1e-15 * np.abs(u))


@pytest.mark.parametrize("K", [2, 10])
def test_two_level_sequence(K):
    m, a = _field(2), _field(3)
    us = [m + a if k % 2 == 0 else m - a for k in range(K)]
    mean, rms, _ = oracle.velocity_statistics(us)
    assert np.allclose(mean, m, rtol=0, atol=1e-14)
    assert np.allclose(rms, np.abs(a), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("K", [1, 7, 40])
def test_ramp_variance_closed_form(K):
    c = _field(4)
    us = [k * c for k in range(K)]
    mean, rms, _ = oracle.velocity_statistics(us)
    assert np.allclose(mean, c * (K - 1) / 2.0, rtol=1e-13, atol=1e-14)
    assert np.allclose(rms ** 2, c ** 2 * (K * K - 1) / 12.0, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("axis,point", [(2, (1, 2)), (0, (2, 1)), (1, (3, 2))])
def test_turbulent_intensity_of_known_fields(axis, point):
    """Streamwise velocity U(s) + a sin(2 pi k / K) at every node of the
    cross-section at streamwise coordinate s (K a multiple of 4: the mean of
    the sine and of its square are 0 and 1/2 exactly), with the amplitude a
    varying over the nodes; Eq. (25) gives a / sqrt(2) / U(s)."""
    nz, ny, nx = SHAPE[1:]
    n3 = (nx, ny, nz)
    rng = np.random.default_rng(5)
    U = 1.0 + rng.random(n3[axis])              # axis velocity per cross-section
    amp = rng.random((nz, ny, nx))               # fluctuation amplitude per node
    shape = [1, 1, 1]
    shape[2 - axis] = -1
    Ufield = np.broadcast_to(U.reshape(shape), (nz, ny, nx))
    K = 8
    us = []
    for k in range(K):
        u = np.zeros(SHAPE)
        u[axis] = Ufield + amp * np.sin(2 * np.pi * k / K)
        u[(axis + 1) % 3] = 0.3 * amp                    # steady cross-flow
        us.append(u)
    mean, rms, ti = oracle.velocity_statistics(us, axis=axis, point=point)
    assert np.allclose(mean[axis], Ufield, rtol=1e-13, atol=1e-14)
    assert np.allclose(rms[axis], amp / np.sqrt(2.0), rtol=1e-12, atol=1e-13)
    assert np.allclose(rms[(axis + 1) % 3], 0.0, atol=1e-14)
    assert np.allclose(ti, amp / np.sqrt(2.0) / Ufield, rtol=1e-12, atol=1e-13)
