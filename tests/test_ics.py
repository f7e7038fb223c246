"""Checks of the seeded synthetic inputs (the paper's core-halo cluster
workloads, Abstract; Sec. "Large scale astrophysical results") against
closed forms and tabulated model properties."""
import os

import numpy as np
import pytest
from scipy import stats

import nbody_ics
import oracle
from oracle import OracleConfig

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_king_concentration_table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "king_concentration.txt"))
            if l.strip() and not l.startswith("#")]
    for W0, c in rows:
        prof = nbody_ics.king_profile(float(W0))
        assert abs(np.log10(prof["r_t"]) - float(c)) < 0.02, (W0, c)


def test_plummer_virial_equilibrium(oracle_lib):
    """Henon units: W = -1/2 and T = 1/4 for the model (W = -3 pi/32 G M^2 / a
    for a Plummer sphere of scale a; a = 3 pi / 16)."""
    m = nbody_ics.plummer(16384, 7)
    T, W = oracle.energy(OracleConfig(eps2=0.0), m.m, m.x, m.v)
    assert abs(W + 0.5) < 0.02
    assert abs(T - 0.25) < 0.01
    assert abs(2 * T / abs(W) - 1.0) < 0.05


@pytest.mark.parametrize("W0", [6.0, 7.0])
def test_king_energy_and_profile(oracle_lib, W0):
    m = nbody_ics.king(16384, W0, 8)
    T, W = oracle.energy(OracleConfig(eps2=0.0), m.m, m.x, m.v)
    assert abs(T + W + 0.25) < 0.015
    assert abs(2 * T / abs(W) - 1.0) < 0.05
    # sampled radii follow the model's cumulative mass (scaled to Henon units)
    prof = nbody_ics.king_profile(W0)
    lam = -2.0 * prof["Wpot"] / prof["M_t"] ** 2
    r = np.linalg.norm(m.x, axis=0) / lam
    cdf = lambda q: np.interp(q, prof["r"], prof["M"] / prof["M_t"])
    # recentring shifts radii slightly; the KS test is on the unshifted law
    assert stats.kstest(r, cdf).pvalue > 0.001


def test_centre_of_mass_frame_and_masses():
    for m in (nbody_ics.plummer(1000, 1), nbody_ics.king(1000, 6.0, 2)):
        assert abs(m.m.sum() - 1.0) < 1e-14
        assert np.all(np.abs(m.x @ m.m) < 1e-15)
        assert np.all(np.abs(m.v @ m.m) < 1e-15)


def test_bh_binary_circular():
    base = nbody_ics.plummer(100, 3)
    m = nbody_ics.with_bh_binary(base, 0.01, 0.2)
    r = m.x[:, 0] - m.x[:, 1]
    v = m.v[:, 0] - m.v[:, 1]
    assert abs(np.linalg.norm(r) - 0.2) < 1e-15
    assert abs(np.linalg.norm(v) - np.sqrt(0.02 / 0.2)) < 1e-15
    assert abs(r @ v) < 1e-16
    assert np.all(np.abs(m.x @ m.m) < 1e-15)


def test_seeded_determinism():
    a = nbody_ics.king(512, 7.0, 13)
    b = nbody_ics.king(512, 7.0, 13)
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.v, b.v)
    s1 = nbody_ics.active_subset(1000, 37, 5)
    assert len(np.unique(s1)) == 37 and np.all(np.diff(s1) > 0)
