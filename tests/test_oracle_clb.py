"""Pins of the oracle's cascaded collision with Gaussian higher-order
equilibria (the CLB the paper starts from before the factorization,
Section 2).

* Mass and momentum are conserved; the product equilibrium (central
  moments of the Gaussian with variance 1/3) is a fixed point.
* At omega = 1 every second-order central moment relaxes to its equilibrium,
  where the factorized equilibria of the FCLB equal the Gaussian ones: the
  two collisions coincide for any state.
* After the collision, the fourth- and sixth-order central moments computed
  here from the populations are those of the Gaussian (1/9, 0, 1/27 per unit
  mass), whatever the state; the FCLB's are not.
* The shear-wave decay rate gives the viscosity of Eq. (13)
  (test_oracle_pins.test_shear_wave_viscosity_converges).
"""
import itertools

import numpy as np
import pytest

import oracle
import synth

E = np.array(oracle.stencil(27)[0])
W = np.array(oracle.stencil(27)[1])


def _central(F):
    rho = F.sum()
    u = (F[:, None] * E).sum(axis=0) / rho
    k = np.zeros((3, 3, 3))
    for a, b, c in itertools.product(range(3), repeat=3):
        k[a, b, c] = (F * (E[:, 0] - u[0]) ** a * (E[:, 1] - u[1]) ** b *
                      (E[:, 2] - u[2]) ** c).sum() / rho
    return rho, u, k


def _states(n=6, seed=4):
    f = synth.random_populations(27, (n, 1, 1), amp=2e-2, seed=seed)
    return [f[:, k, 0, 0] for k in range(n)]


def test_conserves_mass_and_momentum():
    for f in _states():
        g = oracle.clb_collide(f, 1.3)
        assert abs(g.sum() - f.sum()) <= 1e-15
        assert np.abs(((g - f)[:, None] * E).sum(axis=0)).max() <= 1e-15


def test_product_equilibrium_is_fixed_point():
    rng = np.random.default_rng(2)
    for _ in range(4):
        rho, u = 1 + rng.uniform(-0.05, 0.05), rng.uniform(-0.08, 0.08, 3)
        f = oracle.feq_product(rho, u) - W
        np.testing.assert_allclose(oracle.clb_collide(f, 1.7), f, atol=1e-15)


def test_equals_factorized_at_unit_rate():
    for f in _states(seed=9):
        np.testing.assert_allclose(oracle.clb_collide(f, 1.0), oracle.fclb_collide(f, 1.0),
                                   atol=2e-16)


@pytest.mark.parametrize("omega", [0.6, 1.4, 1.9])
def test_higher_central_moments_are_gaussian(omega):
    gauss = {(2, 2, 0): 1 / 9, (2, 0, 2): 1 / 9, (0, 2, 2): 1 / 9, (2, 1, 1): 0.0,
             (1, 2, 1): 0.0, (1, 1, 2): 0.0, (2, 2, 2): 1 / 27}
    for f in _states(seed=11):
        _, _, k = _central(oracle.clb_collide(f, omega) + W)
        for idx, v in gauss.items():
            assert abs(k[idx] - v) <= 1e-14, (idx, k[idx])
        # orders 3 and 5 vanish, as in the FCLB
        for idx in [(2, 1, 0), (1, 1, 1), (2, 2, 1), (0, 1, 2)]:
            assert abs(k[idx]) <= 1e-14
        _, _, kf = _central(oracle.fclb_collide(f, omega) + W)
        assert abs(kf[2, 2, 0] - 1 / 9) > 1e-6
