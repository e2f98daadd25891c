"""Checks of the stored 128^3 oracle spectrum used for the resolution
comparison of the 512^3 decaying-turbulence run (written by
tests/golden/make_resolution_golden.py from oracle/ and inputs only).

The t = 0 column is pinned by what the start is built to be: total energy
k = 3/2 u_rms^2 and the shell spectrum ~ kappa^4 exp(-2 (kappa/k0)^2)
(section V.A's initial condition) with k0 = 8.  The t = 500 column is pinned
by conservation (the mean flow stays zero) and by dissipation (the energy
decays, no shell becomes negative or non-finite).
"""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_resolution128_spectrum.txt")
U_RMS, K0 = 0.04, 8.0


@pytest.fixture(scope="module")
def spec():
    d = np.loadtxt(GOLDEN)
    assert d.shape[1] == 3 and np.array_equal(d[:, 0], np.arange(len(d)))
    return d[:, 1], d[:, 2]


def test_start_energy_is_three_halves_u_rms_squared(spec):
    e0, _ = spec
    assert e0.sum() == pytest.approx(1.5 * U_RMS ** 2, rel=1e-12)


def test_start_follows_the_prescribed_shell_spectrum(spec):
    e0, _ = spec
    kap = np.arange(1, 33, dtype=float)
    shape = kap ** 4 * np.exp(-2.0 * (kap / K0) ** 2)
    ratio = e0[1:33] / shape
    np.testing.assert_allclose(ratio, ratio[7], rtol=1e-9)
    assert int(np.argmax(e0)) == int(K0)


def test_evolved_spectrum_conserves_momentum_and_decays(spec):
    e0, e1 = spec
    assert np.all(np.isfinite(e1)) and np.all(e1 >= 0.0)
    # zero mean flow stays zero: the kappa = 0 shell holds round-off only
    assert e1[0] < 1e-30 * e1.sum()
    assert 0.0 < e1.sum() < e0.sum()
    # the cascade carries energy to the small scales the start left empty
    assert e1[40] > 1e6 * e0[40]
