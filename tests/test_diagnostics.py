"""Host-side black-hole binary diagnostics (orbital elements, Peters'
gravitational-wave luminosity, decay rates, inspiral time) checked against
Kepler orbits of known elements, the oracle's pinned 2.5PN terms and the
consistency of Peters' energy and angular-momentum losses."""
import numpy as np
import pytest
from scipy.integrate import quad

import nbody_ics
import oracle
from paper_1312_1789_amd import diagnostics as dg


def _kepler_state(a, e, M, E):
    """Relative position and velocity at eccentric anomaly E of a Kepler orbit
    with the periastron on +x, tilted about the x axis by 0.4 rad."""
    n = np.sqrt(M / a ** 3)
    Edot = n / (1.0 - e * np.cos(E))
    x = np.array([a * (np.cos(E) - e), a * np.sqrt(1 - e * e) * np.sin(E), 0.0])
    v = np.array([-a * np.sin(E) * Edot, a * np.sqrt(1 - e * e) * np.cos(E) * Edot, 0.0])
    c, s = np.cos(0.4), np.sin(0.4)
    R = np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    return R @ x, R @ v


@pytest.mark.parametrize("a,e,m1,m2", [(1.0, 0.0, 0.5, 0.5), (0.2, 0.3, 0.01, 0.01), (3.0, 0.9, 0.7, 0.1)])
def test_elements_of_kepler_orbits(a, e, m1, m2):
    M = m1 + m2
    for E in (0.0, 1.1, 2.9, 4.4):
        x, v = _kepler_state(a, e, M, E)
        el = dg.orbital_elements(m1, m2, x, v)
        assert el["a"] == pytest.approx(a, rel=1e-13)
        assert el["e"] == pytest.approx(e, abs=1e-13)
        assert el["h"] == pytest.approx(np.sqrt(M * a * (1 - e * e)), rel=1e-13)
    model = nbody_ics.kepler_pair(e, a, m1, m2)
    el = dg.orbital_elements(m1, m2, model.x[:, 0] - model.x[:, 1], model.v[:, 0] - model.v[:, 1])
    assert el["a"] == pytest.approx(a, rel=1e-13) and el["e"] == pytest.approx(e, abs=1e-13)


@pytest.mark.parametrize("e", [0.0, 0.3, 0.7])
def test_luminosity_is_the_orbit_average_of_the_radiation_reaction_power(e):
    """Peters' luminosity equals minus the orbit average of mu v.a over the
    oracle's 2.5PN acceleration on a Kepler orbit."""
    M, nu, a, c = 1.3, 0.2, 0.8, 20.0
    m1 = M * (1 + np.sqrt(1 - 4 * nu)) / 2
    m2 = M - m1
    mu = nu * M
    npts = 4096
    Es = 2 * np.pi * np.arange(npts) / npts
    vals = []
    for E in Es:
        x, v = _kepler_state(a, e, M, E)
        acc, _ = oracle.pn_rel(M, nu, c, 4, x, v)
        vals.append(mu * np.dot(v, acc) * (1 - e * np.cos(E)))
    assert -np.mean(vals) == pytest.approx(dg.peters_luminosity(m1, m2, a, e, c), rel=1e-9)


@pytest.mark.parametrize("e", [0.1, 0.5, 0.8])
def test_decay_rates_follow_from_energy_and_angular_momentum_loss(e):
    """da/dt from the orbital energy -mu M / (2a) losing Peters' luminosity;
    de/dt from that and the angular momentum mu sqrt(M a (1 - e^2)) losing
    (32/5) nu^2 M^(9/2) / (a^(7/2) c^5) (1 + 7/8 e^2) / (1 - e^2)^2 (the
    orbit-averaged torque, pinned in the oracle's tests)."""
    m1, m2, a, c = 0.9, 0.5, 0.7, 9.0
    M = m1 + m2
    nu = m1 * m2 / M ** 2
    mu = nu * M
    L = dg.peters_luminosity(m1, m2, a, e, c)
    dadt_want = -2.0 * a * a / (mu * M) * L
    dJdt = -32.0 / 5.0 * nu ** 2 * M ** 4.5 / (a ** 3.5 * c ** 5) * (1 + 7 / 8 * e * e) / (1 - e * e) ** 2
    J = mu * np.sqrt(M * a * (1 - e * e))
    # dJ/dt = J (da/dt / (2a) - e de/dt / (1 - e^2))
    dedt_want = (dadt_want / (2 * a) - dJdt / J) * (1 - e * e) / e
    dadt, dedt = dg.peters_rates(m1, m2, a, e, c)
    assert dadt == pytest.approx(dadt_want, rel=1e-12)
    assert dedt == pytest.approx(dedt_want, rel=1e-12)


def test_inspiral_time_integrates_the_circular_decay():
    m1, m2, a0, c = 0.01, 0.01, 0.2, 50.0
    T, _ = quad(lambda a: -1.0 / dg.peters_rates(m1, m2, a, 0.0, c)[0], 0.0, a0)
    assert dg.inspiral_time_circular(m1, m2, a0, c) == pytest.approx(T, rel=1e-10)


def test_binary_gw_on_a_cluster_state():
    """The pair at indices 0, 1 of a cluster with a circular black-hole binary
    (separation 0.2, masses 0.01): a = 0.2 and e = 0 for the pair alone."""
    model = nbody_ics.with_bh_binary(nbody_ics.plummer(500, 3), 0.01, 0.2)
    h = {"m": model.m, "x": model.x, "v": model.v}
    out = dg.binary_gw(h, 10.0)
    assert out["a"] == pytest.approx(0.2, rel=1e-12) and out["e"] < 1e-12
    assert out["gw_luminosity"] == pytest.approx(dg.peters_luminosity(0.01, 0.01, 0.2, 0.0, 10.0), rel=1e-9)
    assert out["inspiral_time_circular"] > 0 and out["da_dt"] < 0
    assert "gw_luminosity" not in dg.binary_gw(h, 0.0)
