"""Pins of the oracle's post-Newtonian terms between black holes (the paper's
relativistic corrections for black-hole binaries, Introduction; 1PN, 2PN and 2.5PN
two-body terms in harmonic coordinates) against results the physics fixes:

* 2.5PN, circular orbit: the instantaneous power mu v.a equals the
  quadrupole luminosity -(32/5) nu^2 (M/r)^5 / c^5;
* 2.5PN, eccentric orbits: the orbit averages of mu v.a and of the torque
  mu (x cross a) over a Newtonian Kepler orbit equal Peters' (1964) energy
  and angular-momentum loss rates with their e-dependent enhancements;
* 1PN: the circular-orbit frequency omega^2 = (M/r^3)(1 - (3 - nu) M/(c^2 r)),
  and the periastron advance per orbit 6 pi M / (c^2 a (1 - e^2)) from
  Gauss' perturbation equation integrated over a Kepler orbit;
* 2PN: the circular-orbit frequency to second order,
  omega^2 = (M/r^3)(1 + (nu - 3) g + (6 + 41/4 nu + nu^2) g^2), g = M/(c^2 r)
  (its residual falls as g^3), and the conservation of the 2PN two-body
  energy along orbits of the 1PN + 2PN equations of motion to O(c^-6) (its
  variation falls 64-fold when c doubles; any wrong 2PN coefficient leaves a
  c^-4 variation);
* the jerk, snap and crackle are the time derivatives of the acceleration
  along the two-body motion (central differences of the oracle's own
  acceleration on the integrated two-body path);
* pairwise use conserves momentum and leaves soft particles alone;
* the oracle's own block-step integration of a circular binary shrinks at
  Peters' rate.
"""
import numpy as np
import pytest

import oracle
from oracle import OracleConfig
from oracle.oracle import TICKS_PER_UNIT


def kepler(a, e, M, E):
    """Relative position and velocity on a Newtonian Kepler orbit at eccentric
    anomalies E (orbit in the x-y plane, periastron on +x)."""
    nmean = np.sqrt(M / a ** 3)
    Edot = nmean / (1.0 - e * np.cos(E))
    x = np.stack([a * (np.cos(E) - e), a * np.sqrt(1 - e * e) * np.sin(E), 0 * E])
    v = np.stack([-a * np.sin(E) * Edot, a * np.sqrt(1 - e * e) * np.cos(E) * Edot, 0 * E])
    return x, v


def orbit_average(f, a, e, M, npts=4096):
    """Time average over one orbit of f(x, v): dt = (1 - e cos E) dE / n, so
    <f> = (1/2pi) int f (1 - e cos E) dE (trapezoid rule, periodic)."""
    E = 2 * np.pi * np.arange(npts) / npts
    x, v = kepler(a, e, M, E)
    vals = np.array([f(x[:, k], v[:, k]) for k in range(npts)])
    w = 1.0 - e * np.cos(E)
    return np.mean(vals * w)


@pytest.mark.parametrize("M,nu,r", [(1.0, 0.25, 1.0), (0.02, 0.2, 0.2), (3.0, 0.1, 7.0)])
def test_circular_power_is_quadrupole_luminosity(M, nu, r):
    c = 13.0
    v = np.sqrt(M / r)
    x = np.array([r, 0.0, 0.0])
    vel = np.array([0.0, v, 0.0])
    a, _ = oracle.pn_rel(M, nu, c, 4, x, vel)
    mu = nu * M
    P = mu * np.dot(vel, a)
    want = -32.0 / 5.0 * nu ** 2 * (M / r) ** 5 / c ** 5
    assert P == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("e", [0.0, 0.3, 0.7])
def test_peters_energy_and_angular_momentum_loss(e):
    M, nu, a, c = 1.0, 0.2, 1.0, 20.0
    mu = nu * M

    def power(x, v):
        acc, _ = oracle.pn_rel(M, nu, c, 4, x, v)
        return mu * np.dot(v, acc)

    def torque(x, v):
        acc, _ = oracle.pn_rel(M, nu, c, 4, x, v)
        return mu * (x[0] * acc[1] - x[1] * acc[0])

    dE = orbit_average(power, a, e, M)
    dL = orbit_average(torque, a, e, M)
    e2 = e * e
    dE_want = -32.0 / 5.0 * nu ** 2 * M ** 5 / (a ** 5 * c ** 5) * (1 + 73 / 24 * e2 + 37 / 96 * e2 ** 2) / (1 - e2) ** 3.5
    dL_want = -32.0 / 5.0 * nu ** 2 * M ** 4.5 / (a ** 3.5 * c ** 5) * (1 + 7 / 8 * e2) / (1 - e2) ** 2
    assert dE == pytest.approx(dE_want, rel=1e-9)
    assert dL == pytest.approx(dL_want, rel=1e-9)


@pytest.mark.parametrize("nu", [0.25, 0.09, 0.0])
def test_1pn_circular_frequency(nu):
    """On a circular orbit the 1PN radial term changes the centripetal
    balance to omega^2 r = (M/r^2)(1 + A_1PN): omega^2 = (M/r^3)(1 - (3 - nu)
    M/(c^2 r)); the velocity term vanishes (rdot = 0)."""
    M, r, c = 1.0, 5.0, 30.0
    v = np.sqrt(M / r)
    a, _ = oracle.pn_rel(M, nu, c, 1, [r, 0, 0], [0, v, 0])
    radial = -a[0] / (M / r ** 2)           # A_1PN
    assert radial == pytest.approx(-(3 - nu) * M / (c * c * r), rel=1e-13)
    assert abs(a[1]) < 1e-18


def _circular_omega2(M, nu, c, r, terms):
    """omega^2 of the circular orbit of radius r under Newton + the oracle's
    PN terms: v^2 = r |a(v)| solved by fixed-point iteration (rdot = 0, so
    only the radial A term acts)."""
    v2 = M / r
    for _ in range(60):
        a, _ = oracle.pn_rel(M, nu, c, terms, [r, 0.0, 0.0], [0.0, np.sqrt(v2), 0.0])
        v2_new = r * (M / r ** 2 - a[0])
        if v2_new == v2:
            break
        v2 = v2_new
    return v2 / r ** 2


@pytest.mark.parametrize("nu", [0.25, 0.21, 0.0])
def test_2pn_circular_frequency(nu):
    """The circular-orbit frequency with the 1PN and 2PN terms matches the
    2PN series omega^2 = (M/r^3)(1 + (nu - 3) g + (6 + 41/4 nu + nu^2) g^2),
    g = M/(c^2 r), up to a residual of order g^3 (it falls ~64-fold when c
    doubles); with the 1PN terms alone the residual is of order g^2."""
    M, r = 1.0, 10.0
    res = {}
    for c in (10.0, 20.0):
        g = M / (c * c * r)
        series = M / r ** 3 * (1 + (nu - 3) * g + (6 + 41 / 4 * nu + nu * nu) * g * g)
        res[c] = _circular_omega2(M, nu, c, r, 3) / series - 1.0
        res[c, 1] = _circular_omega2(M, nu, c, r, 1) / series - 1.0
        assert abs(res[c]) <= 100 * g ** 3
    assert 40 < abs(res[10.0] / res[20.0]) < 100
    assert 12 < abs(res[10.0, 1] / res[20.0, 1]) < 20


def _energy_2pn(M, nu, c, x, v):
    """Conserved energy per reduced mass of the 2PN two-body motion in
    harmonic coordinates (Blanchet 2014, Living Rev. Relativ. 17, 2): the
    Newtonian, 1PN and 2PN truncations.  Plain arithmetic and one square
    root, so that it also takes complex arguments (complex-step gradients)."""
    r = np.sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2])
    v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2]
    rd = (x[0] * v[0] + x[1] * v[1] + x[2] * v[2]) / r
    Mr = M / r
    e0 = v2 / 2 - Mr
    e1 = 3 / 8 * v2 ** 2 - 9 / 8 * nu * v2 ** 2 + Mr * (rd ** 2 * nu / 2 + 3 / 2 * v2 + nu * v2 / 2) + Mr ** 2 / 2
    e2 = (5 / 16 * v2 ** 3 - 35 / 16 * nu * v2 ** 3 + 65 / 16 * nu ** 2 * v2 ** 3
          + Mr * (-3 / 8 * rd ** 4 * nu + 9 / 8 * rd ** 4 * nu ** 2 + 1 / 4 * rd ** 2 * nu * v2
                  - 15 / 4 * rd ** 2 * nu ** 2 * v2 + 21 / 8 * v2 ** 2 - 23 / 8 * nu * v2 ** 2
                  - 27 / 8 * nu ** 2 * v2 ** 2)
          + Mr ** 2 * (rd ** 2 / 2 + 69 / 8 * rd ** 2 * nu + 3 / 2 * rd ** 2 * nu ** 2 + 7 / 4 * v2
                       - 55 / 8 * nu * v2 + nu ** 2 * v2 / 2)
          + Mr ** 3 * (-1 / 2 - 15 / 4 * nu))
    return e0, e0 + e1 / c ** 2, e0 + e1 / c ** 2 + e2 / c ** 4


def _energy_variation(M, nu, c, e, steps=16000, orbits=1.5):
    """Largest change of the 1PN and 2PN energies along the 1PN + 2PN
    relative equation of motion (Newton + oracle PN terms) from the
    pericentre of a Kepler orbit of eccentricity e, a = 1: RK4 in the
    Sundman variable s (dt = r ds, so that the steps shrink with r at
    pericentre)."""
    y = np.array([1.0 - e, 0.0, 0.0, 0.0, np.sqrt(M * (1 + e) / (1 - e)), 0.0])
    h = orbits * 2 * np.pi / steps   # ds; one orbit spans about 2 pi in s (a = 1)

    def f(y):
        x, v = y[:3], y[3:]
        r = np.linalg.norm(x)
        pn, _ = oracle.pn_rel(M, nu, c, 3, x, v)
        return r * np.concatenate([v, -M * x / r ** 3 + pn])

    e1, e2 = [], []
    for _ in range(steps):
        k1 = f(y); k2 = f(y + h / 2 * k1); k3 = f(y + h / 2 * k2); k4 = f(y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        _, a1, a2 = _energy_2pn(M, nu, c, y[:3], y[3:])
        e1.append(a1)
        e2.append(a2)
    return np.ptp(e1), np.ptp(e2)


def _energy_rate(M, nu, c, x, v):
    """dE_2PN/dt = grad_x E . v + grad_v E . a at one phase-space point, with
    a = Newton + the oracle's 1PN + 2PN terms; the gradient by complex steps
    (exact to rounding)."""
    pn, _ = oracle.pn_rel(M, nu, c, 3, x, v)
    a = -M * x / np.linalg.norm(x) ** 3 + pn
    rate = 0.0
    for k in range(3):
        dx = np.zeros(3, complex)
        dx[k] = 1e-30j
        rate += _energy_2pn(M, nu, c, x + dx, v.astype(complex))[2].imag / 1e-30 * v[k]
        rate += _energy_2pn(M, nu, c, x.astype(complex), v + dx)[2].imag / 1e-30 * a[k]
    return rate


def test_2pn_energy_rate_is_order_c6():
    """At phase-space points (the identity holds at any point, bound or not)
    the rate of change of the 2PN energy under the 1PN + 2PN equations of
    motion is O(c^-6): doubling c shrinks it ~64-fold at every point.  A
    wrong 2PN coefficient of the acceleration leaves an O(c^-4) rate
    (16-fold).  Two sets: random directions with |v|^2 ~ M/r, and nearly
    radial motion at up to three times that speed, where the terms in powers
    of rdot weigh most."""
    rng = np.random.default_rng(35)
    M = 1.0
    for radial in (False, True):
        ratios = []
        for _ in range(16):
            nu = rng.uniform(0.15, 0.25)
            x = rng.normal(size=3)
            x *= rng.uniform(0.5, 2.0) / np.linalg.norm(x)
            v = rng.normal(size=3) + (8.0 * x / np.linalg.norm(x) if radial else 0.0)
            v *= rng.uniform(0.5, 3.0 if radial else 1.5) * np.sqrt(M / np.linalg.norm(x)) / np.linalg.norm(v)
            r1, r2 = (_energy_rate(M, nu, c, x, v) for c in (80.0, 160.0))
            ratios.append(r1 / r2)
        assert np.all((np.array(ratios) > 55) & (np.array(ratios) < 75)), ratios


@pytest.mark.parametrize("e", [0.5, 0.85])
def test_2pn_energy_conserved_to_order_c6(e):
    """Along orbits of the 1PN + 2PN equations of motion (nu = 1/4, where
    the nu^2 terms weigh most; e = 0.85 makes the rdot^4 terms count) the 2PN
    energy changes only at O(c^-6): doubling c shrinks its variation ~64-fold,
    while the 1PN energy's variation (O(c^-4), the 2PN terms being on)
    shrinks ~16-fold."""
    M, nu = 1.0, 0.25
    c0 = 10.0 if e < 0.7 else 24.0
    d1 = _energy_variation(M, nu, c0, e)
    d2 = _energy_variation(M, nu, 2 * c0, e)
    r1, r2 = d1[0] / d2[0], d1[1] / d2[1]
    assert 12 < r1 < 20, r1
    assert 45 < r2 < 90, r2
    assert d1[1] < 0.05 * d1[0]


@pytest.mark.parametrize("e", [0.2, 0.6])
def test_1pn_periastron_advance(e):
    """Gauss' equation for the argument of periastron, planar orbit:
    d omega/dt = sqrt(p/M)/e (-R cos f + S (1 + r/p) sin f), R and S the
    radial and transverse components of the 1PN acceleration on the Kepler
    orbit; its integral over one period is 6 pi M / (c^2 p)."""
    M, nu, a, c = 1.0, 0.22, 1.0, 50.0
    p = a * (1 - e * e)
    T = 2 * np.pi * np.sqrt(a ** 3 / M)

    def domega(x, v):
        acc, _ = oracle.pn_rel(M, nu, c, 1, x, v)
        r = np.linalg.norm(x)
        nvec = x / r
        tvec = np.array([-nvec[1], nvec[0], 0.0])          # along the motion (counter-clockwise)
        R, S = np.dot(acc, nvec), np.dot(acc, tvec)
        cosf, sinf = x[0] / r, x[1] / r
        return np.sqrt(p / M) / e * (-R * cosf + S * (1 + r / p) * sinf)

    dw = orbit_average(domega, a, e, M) * T
    assert dw == pytest.approx(6 * np.pi * M / (c * c * p), rel=1e-3)   # 1PN order: O(M/(c^2 p)) corrections


def test_jerk_is_time_derivative_along_two_body_motion():
    rng = np.random.default_rng(31)
    for _ in range(5):
        M, nu, c = rng.uniform(0.5, 2.0), rng.uniform(0.05, 0.25), rng.uniform(5.0, 20.0)
        x = rng.normal(size=3)
        v = rng.normal(size=3) * np.sqrt(M / np.linalg.norm(x))
        an = -M * x / np.linalg.norm(x) ** 3
        _, j = oracle.pn_rel(M, nu, c, 7, x, v)
        h = 1e-4
        ap, _ = oracle.pn_rel(M, nu, c, 7, x + v * h + an * h * h / 2, v + an * h)
        am, _ = oracle.pn_rel(M, nu, c, 7, x - v * h + an * h * h / 2, v - an * h)
        fd = (ap - am) / (2 * h)
        np.testing.assert_allclose(j, fd, rtol=1e-6, atol=1e-9 * np.abs(j).max())


def _two_body_path(M, x, v, ts, substeps=200):
    """States (x, v) of the Newtonian two-body motion at the times ts (RK4
    from t = 0 in small steps, forward and backward)."""
    def f(y):
        r = y[:3]
        return np.concatenate([y[3:], -M * r / np.linalg.norm(r) ** 3])
    out = []
    for t in ts:
        y = np.concatenate([x, v]).astype(float)
        h = t / substeps
        for _ in range(substeps):
            k1 = f(y); k2 = f(y + h / 2 * k1); k3 = f(y + h / 2 * k2); k4 = f(y + h * k3)
            y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        out.append((y[:3], y[3:]))
    return out


def test_snap_and_crackle_are_time_derivatives_along_two_body_motion():
    """Second and third derivatives of the oracle's own PN acceleration along
    the integrated two-body path (central differences) equal its snap and
    crackle; its jerk and acceleration agree with the first-derivative route."""
    rng = np.random.default_rng(33)
    for _ in range(4):
        M, nu, c = rng.uniform(0.5, 2.0), rng.uniform(0.05, 0.25), rng.uniform(5.0, 20.0)
        x = rng.normal(size=3)
        v = rng.normal(size=3) * np.sqrt(M / np.linalg.norm(x))
        d = oracle.pn_rel_derivs(M, nu, c, 7, x, v)
        a, j = oracle.pn_rel(M, nu, c, 7, x, v)
        np.testing.assert_array_equal(d[0], a)
        np.testing.assert_array_equal(d[1], j)
        h = 2e-3
        f = {k: oracle.pn_rel(M, nu, c, 7, xs, vs)[0]
             for k, (xs, vs) in zip((-2, -1, 1, 2), _two_body_path(M, x, v, (-2 * h, -h, h, 2 * h)))}
        f[0] = a
        snap = (f[1] - 2 * f[0] + f[-1]) / h ** 2
        crackle = (f[2] - 2 * f[1] + 2 * f[-1] - f[-2]) / (2 * h ** 3)
        scale_s, scale_c = np.abs(d[2]).max(), np.abs(d[3]).max()
        np.testing.assert_allclose(d[2], snap, rtol=0, atol=2e-5 * scale_s)
        np.testing.assert_allclose(d[3], crackle, rtol=0, atol=2e-4 * scale_c)


def test_pairwise_terms_conserve_momentum_and_skip_soft_particles():
    rng = np.random.default_rng(32)
    n = 5
    m = np.array([0.3, 0.1, 1e-3, 1e-3, 1e-3])
    x = rng.normal(size=(3, n))
    v = rng.normal(size=(3, n))
    act = np.arange(n, dtype=np.int32)
    acc = np.zeros((3, n))
    jrk = np.zeros((3, n))
    oracle.pn(OracleConfig(order=4, n_hard=2, c_light=5.0, pn_terms=5), m, x, v, act, acc, jrk)
    np.testing.assert_allclose(m[0] * acc[:, 0] + m[1] * acc[:, 1], 0.0, atol=1e-17)
    np.testing.assert_allclose(m[0] * jrk[:, 0] + m[1] * jrk[:, 1], 0.0, atol=1e-17)
    assert np.all(acc[:, 2:] == 0) and np.all(jrk[:, 2:] == 0)
    a_rel, _ = oracle.pn_rel(m[0] + m[1], m[0] * m[1] / (m[0] + m[1]) ** 2, 5.0, 5, x[:, 0] - x[:, 1], v[:, 0] - v[:, 1])
    np.testing.assert_allclose(acc[:, 0] - acc[:, 1], a_rel, rtol=1e-14)
    off = np.zeros((3, n))
    oracle.pn(OracleConfig(order=4, n_hard=2, c_light=0.0, pn_terms=5), m, x, v, act, off, off.copy())
    assert np.all(off == 0)


def test_three_hard_bodies_conserve_momentum_and_rows_do_not_depend_on_the_active_set():
    """With three hard bodies each row sums the terms of its two pairs: the
    total momentum change still vanishes (each pair's share is m2/M and
    -m1/M of one relative acceleration), and a row computed in a smaller
    active set has the same bits as in the full one."""
    rng = np.random.default_rng(33)
    n = 6
    m = np.array([0.3, 0.1, 0.2, 1e-3, 1e-3, 1e-3])
    x = rng.normal(size=(3, n))
    v = rng.normal(size=(3, n))
    cfg = OracleConfig(order=8, n_hard=3, c_light=4.0, pn_terms=5)
    act = np.arange(n, dtype=np.int32)
    out = [np.zeros((3, n)) for _ in range(4)]
    oracle.pn(cfg, m, x, v, act, *out)
    for o in out:
        scale = np.abs(m[:3] * o[:, :3]).max()
        assert scale > 0
        np.testing.assert_allclose(o[:, :3] @ m[:3], 0.0, atol=1e-14 * scale)
        assert np.all(o[:, 3:] == 0)
    pair01 = [np.zeros((3, n)) for _ in range(4)]
    oracle.pn(OracleConfig(order=8, n_hard=2, c_light=4.0, pn_terms=5), m, x, v, act, *pair01)
    assert np.abs(out[0][:, 0] - pair01[0][:, 0]).max() > 1e-3 * np.abs(pair01[0][:, 0]).max()
    sub = np.array([1], dtype=np.int32)
    one = [np.zeros((3, 1)) for _ in range(4)]
    oracle.pn(cfg, m, x, v, sub, *one)
    for o, f in zip(one, out):
        np.testing.assert_array_equal(o[:, 0], f[:, 1])


def test_oracle_integration_inspiral_at_peters_rate():
    """The oracle's 4th-order block-step integration of a circular binary
    with the 2.5PN terms alone: the semi-major axis from the Newtonian energy
    shrinks at Peters' rate da/dt = -(64/5) nu M^3 / (a^3 c^5)."""
    m = np.array([0.6, 0.4])
    M, nu, a0, c = 1.0, 0.24, 1.0, 8.0
    x = np.array([[0.4 * a0, -0.6 * a0], [0.0, 0.0], [0.0, 0.0]])
    vc = np.sqrt(M / a0)
    v = np.array([[0.0, 0.0], [0.4 * vc, -0.6 * vc], [0.0, 0.0]])
    cfg = OracleConfig(order=4, eps2=0.0, n_hard=2, eta=0.01, eta_start=0.01, k_min=3, k_max=20,
                       c_light=c, pn_terms=4)
    st = oracle.State(m, x, v, 4)
    oracle.init(cfg, st)
    T = 16.0
    oracle.integrate(cfg, st, int(T * TICKS_PER_UNIT))
    r = np.linalg.norm(st.x[:, 0] - st.x[:, 1])
    w = st.v[:, 0] - st.v[:, 1]
    a1 = -M / (2.0 * (0.5 * np.dot(w, w) - M / r))
    rate = (a1 - a0) / T
    want = -64.0 / 5.0 * nu * M ** 3 / (a0 ** 3 * c ** 5)
    assert rate == pytest.approx(want, rel=0.02)
