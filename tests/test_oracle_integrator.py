"""Pins of the oracle's integrator: predictor, Hermite corrector and
interpolation, time-step criterion and block quantisation, and whole block-step
integration (convergence order on the Kepler problem, block invariants,
conservation).

Method (paper: Abstract; Sec. "Codes description"): 4th/6th/8th-order Hermite
integration with individual hierarchical block time steps.  The formulas are
the standard ones (Makino & Aarseth 1992; Nitadori & Makino 2008; Aarseth's
time-step criterion).
"""
import math

import mpmath as mp
import numpy as np
import pytest

import nbody_ics
import oracle
from oracle import OracleConfig
from oracle.oracle import TICK_BITS, TICKS_PER_UNIT

ORDERS = [4, 6, 8]


# --------------------------------------------------------------------------
# predictor

@pytest.mark.parametrize("p", ORDERS)
def test_predictor_exact_on_polynomials(oracle_lib, p):
    """A trajectory that is a polynomial of degree p-1 is predicted exactly
    (position, velocity, and for p >= 6 acceleration, p = 8 jerk)."""
    rng = np.random.default_rng(p)
    n = 5
    coef = rng.uniform(-1, 1, (p, 3, n))       # coef[k] = x^(k)(t0)
    t0 = 3 * (TICKS_PER_UNIT >> 6)
    s = oracle.State(np.ones(n), coef[0], coef[1], p, [coef[k + 2] for k in range(p - 2)],
                     np.full(n, t0, np.int64), np.full(n, 6, np.int32))
    t1 = t0 + 5 * (TICKS_PER_UNIT >> 8)
    dt = (t1 - t0) / TICKS_PER_UNIT
    xp, vp, ap, jp = oracle.predict(OracleConfig(order=p), s, t1)

    def deriv(q):
        return sum(coef[q + k] * dt ** k / math.factorial(k) for k in range(p - q))
    np.testing.assert_allclose(xp, deriv(0), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(vp, deriv(1), rtol=1e-14, atol=1e-15)
    if p >= 6:
        np.testing.assert_allclose(ap, deriv(2), rtol=1e-14, atol=1e-15)
    if p >= 8:
        np.testing.assert_allclose(jp, deriv(3), rtol=1e-14, atol=1e-15)


# --------------------------------------------------------------------------
# interpolation and corrector

def _poly_derivs(c, t, nder):
    """Derivatives 0..nder-1 of sum_k c[k] t^k at t."""
    P = np.polynomial.Polynomial(c)
    out = []
    for _ in range(nder):
        out.append(P(t))
        P = P.deriv()
    return np.array(out)


@pytest.mark.parametrize("p", ORDERS)
def test_interpolation_exact_up_to_degree_p_minus_1(oracle_lib, p):
    q = p // 2
    rng = np.random.default_rng(10 + p)
    h = 0.375
    for _ in range(5):
        c = rng.uniform(-1, 1, p)               # degree p-1
        D0 = _poly_derivs(c, 0.0, q)
        D1 = _poly_derivs(c, h, p)
        H = oracle.hermite_high(p, h, D0, D1[:q])
        np.testing.assert_allclose(H, D1[q:], rtol=1e-11, atol=1e-11)
    # one degree more is no longer reproduced: the formula is pinned exactly
    c = np.zeros(p + 1)
    c[p] = 1.0
    D1 = _poly_derivs(c, h, p)
    H = oracle.hermite_high(p, h, _poly_derivs(c, 0.0, q), D1[:q])
    assert np.max(np.abs(H - D1[q:])) > 1e-3


@pytest.mark.parametrize("p", ORDERS)
def test_interpolation_matches_confluent_vandermonde_solve(oracle_lib, p):
    """Independent construction: solve the 2q x 2q confluent Vandermonde
    system for the interpolant's coefficients about t1, read off a^(q..p-1)."""
    q = p // 2
    rng = np.random.default_rng(20 + p)
    h = 0.6
    D0 = rng.uniform(-1, 1, q)
    D1 = rng.uniform(-1, 1, q)
    # polynomial P(s) = sum_k b_k s^k / k!, s = t - t1; P^(l)(0) = b_l,
    # P^(l)(-h) = sum_{k>=l} b_k (-h)^(k-l) / (k-l)!
    M = np.zeros((p, p))
    rhs = np.zeros(p)
    for l in range(q):
        M[l, l] = 1.0
        rhs[l] = D1[l]
        for k in range(l, p):
            M[q + l, k] = (-h) ** (k - l) / math.factorial(k - l)
        rhs[q + l] = D0[l]
    b = np.linalg.solve(M, rhs)
    np.testing.assert_allclose(oracle.hermite_high(p, h, D0, D1), b[q:], rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("p", ORDERS)
def test_corrector_exactness(oracle_lib, p):
    """The velocity corrector is exact when x(t) is a polynomial of degree
    <= p+1, the position corrector (with the corrected v1) for degree <= p;
    one degree more breaks each (so every coefficient is pinned)."""
    q = p // 2
    rng = np.random.default_rng(30 + p)
    h = 0.5

    def run(c):
        X0 = _poly_derivs(c, 0.0, q + 2)
        X1 = _poly_derivs(c, h, q + 2)
        x1, v1 = oracle.hermite_correct(p, h, X0[0], X0[1], X0[2:], X1[2:])
        return x1 - X1[0], v1 - X1[1]

    for _ in range(4):
        ex, ev = run(rng.uniform(-1, 1, p + 2))        # degree p+1
        assert abs(ev) < 1e-13
        ex, ev = run(rng.uniform(-1, 1, p + 1))        # degree p
        assert abs(ex) < 1e-13 and abs(ev) < 1e-13
    c = np.zeros(p + 3)
    c[p + 2] = 1.0
    assert abs(run(c)[1]) > 1e-6
    c = np.zeros(p + 2)
    c[p + 1] = 1.0
    assert abs(run(c)[0]) > 1e-6


# --------------------------------------------------------------------------
# time step

@pytest.mark.parametrize("p", ORDERS)
def test_dt_crit_circular_orbit(oracle_lib, p):
    """On a circular orbit |a^(k)| = omega^k |a|: Aarseth's criterion gives
    sqrt(eta)/omega and the generalised one eta/omega."""
    w = 1.7
    F = np.array([2.3 * w ** k for k in range(p)])
    eta = 0.02
    want = math.sqrt(eta) / w if p == 4 else eta / w
    assert abs(oracle.dt_crit(p, eta, F) - want) < 1e-14 * want


@pytest.mark.parametrize("p", [6, 8])
def test_dt_crit_order4_form(oracle_lib, p):
    """The order-4 form of the generalised criterion: eta/omega on a circular
    orbit like the full-order one, reads only a .. a^(3) (any value of the
    higher derivatives, even NaN, leaves it unchanged) and so does not
    depend on the scheme's order; a^(3) does change it."""
    w = 1.7
    F = np.array([2.3 * w ** k for k in range(p)])
    eta = 0.1
    assert abs(oracle.dt_crit(p, eta, F, rule=2) - eta / w) < 1e-14 * eta / w
    G = F.copy()
    G[4:] = [np.nan, 1e30, 0.0, 7.0][: p - 4]
    assert oracle.dt_crit(p, eta, G, rule=2) == oracle.dt_crit(p, eta, F, rule=2)
    assert oracle.dt_crit(p, eta, F, rule=2) == oracle.dt_crit(6, eta, F[:6], rule=2)
    H = F.copy()
    H[3] *= 4.0
    assert oracle.dt_crit(p, eta, H, rule=2) < oracle.dt_crit(p, eta, F, rule=2)
    # the full-order criterion does read the higher derivatives (finite
    # values: a NaN would make any comparison pass)
    K = F * np.r_[1, 1, 1, 1, [2.0] * (p - 4)]
    assert np.isfinite(oracle.dt_crit(p, eta, K, rule=1))
    assert oracle.dt_crit(p, eta, K, rule=1) != oracle.dt_crit(p, eta, F, rule=1)


@pytest.mark.parametrize("p,F", [
    # p = 6: A_1 = sqrt(1*1) + 1 = 2, A_4 = sqrt(|a^(3)||a^(5)|) + |a^(4)| = sqrt(4*9) + 10 = 16,
    #        dt = eta (2/16)^(1/3) = eta/2
    (6, [1.0, 1.0, 1.0, 4.0, 10.0, 9.0]),
    # p = 8: A_1 = 2, A_6 = sqrt(|a^(5)||a^(7)|) + |a^(6)| = sqrt(4*100) + 44 = 64,
    #        dt = eta (2/64)^(1/5) = eta/2
    (8, [1.0, 1.0, 1.0, 3.0, 7.0, 4.0, 44.0, 100.0]),
])
def test_dt_crit_full_order_hand_values(oracle_lib, p, F):
    """The generalised criterion of the scheme's order, dt = eta (A_1/A_(p-2))^(1/(p-3))
    with A_k = sqrt(|a^(k-1)||a^(k+1)|) + |a^(k)| (Nitadori & Makino 2008), on
    derivative magnitudes that are not a geometric sequence, so that an index
    or exponent slip changes the value.  At p = 6, A_(p-3) in place of
    A_(p-2) gives eta * 0.654, the exponent 1/(p-4) eta * 0.354, both slips
    eta * 0.528; at p = 8 eta * 0.622, 0.420 and 0.552.  Both cases are built
    to give exactly eta/2 (arithmetic in the parameter list)."""
    eta = 0.1
    got = oracle.dt_crit(p, eta, np.array(F), rule=1)
    assert abs(got - eta / 2) < 1e-15, got
    # the order-4 form on the same input: eta A_1/A_2, A_2 = sqrt(|a^(1)||a^(3)|) + |a^(2)|
    A2 = math.sqrt(F[1] * F[3]) + F[2]
    assert abs(oracle.dt_crit(p, eta, np.array(F), rule=2) - eta * 2.0 / A2) < 1e-15


@pytest.mark.parametrize("eta_start,level", [(0.01, 10), (0.02, 9), (0.003, 12)])
def test_init_first_level_circular_binary(oracle_lib, eta_start, level):
    """The initial step dt0 = eta_start |a|/|jerk|, quantised to the largest
    2^-k <= dt0.  Two equal unsoftened masses 1/2 on a circular orbit of
    separation r = 1/4 have angular frequency w = sqrt(M/r^3) = 8, and for each
    body |jerk| = w |a|, so dt0 = eta_start/8 in closed form:
    0.01/8 = 1.25e-3 lies in [2^-10, 2^-9), 0.02/8 in [2^-9, 2^-8),
    0.003/8 = 3.75e-4 in [2^-12, 2^-11).  The inverted ratio |jerk|/|a| would
    give levels 4, 3 and 6."""
    r, M = 0.25, 1.0
    vrel = math.sqrt(M / r)
    x = np.array([[-r / 2, r / 2], [0.0, 0.0], [0.0, 0.0]])
    v = np.array([[0.0, 0.0], [-vrel / 2, vrel / 2], [0.0, 0.0]])
    for p in ORDERS:
        cfg = OracleConfig(order=p, eps2=0.0, eta=0.1, eta_start=eta_start, k_min=3, k_max=20)
        s = oracle.State(np.array([0.5, 0.5]), x, v, p)
        oracle.init(cfg, s)
        a, j = s.d[0], s.d[1]
        np.testing.assert_allclose(np.linalg.norm(a, axis=0), 0.5 * M / r ** 2 * 1.0, rtol=1e-14)
        np.testing.assert_allclose(np.linalg.norm(j, axis=0), 8.0 * np.linalg.norm(a, axis=0), rtol=1e-14)
        assert list(s.level) == [level, level], (p, s.level)
        assert list(s.t_tick) == [0, 0]
    # the clamp to [k_min, k_max] applies to the first step too
    cfg = OracleConfig(order=4, eps2=0.0, eta=0.01, eta_start=eta_start, k_min=3, k_max=level - 2)
    s = oracle.State(np.array([0.5, 0.5]), x, v, 4)
    oracle.init(cfg, s)
    assert list(s.level) == [level - 2, level - 2]
    cfg = OracleConfig(order=4, eps2=0.0, eta=0.01, eta_start=eta_start, k_min=level + 3, k_max=20)
    s = oracle.State(np.array([0.5, 0.5]), x, v, 4)
    oracle.init(cfg, s)
    assert list(s.level) == [level + 3, level + 3]


def test_dt_crit_aarseth_mixed_magnitudes(oracle_lib):
    F = np.array([1.0, 2.0, 4.0, 16.0])
    # sqrt(eta (1*4 + 2^2) / (2*16 + 4^2)) = sqrt(eta / 6)
    assert abs(oracle.dt_crit(4, 0.06, F) - 0.1) < 1e-16


def _quantise_brute(dtc, k_min, k_max):
    for k in range(k_min, k_max + 1):
        if 2.0 ** -k <= dtc:
            return k
    return k_max


@pytest.mark.parametrize("k_max", [20, 32, 40])
def test_new_level_rules(oracle_lib, k_max):
    """Largest 2^-k <= dt_crit within [k_min, k_max]; at most one doubling,
    only when the end time is a multiple of the doubled step (levels up to
    40: time ticks of 2^-40)."""
    k_min = 3
    rng = np.random.default_rng(40 + k_max)
    for _ in range(3000):
        old = int(rng.integers(k_min, k_max + 1))
        dt_old = 1 << (TICK_BITS - old)
        t1 = int(rng.integers(1, 1 << 10)) * dt_old
        dtc = 2.0 ** rng.uniform(-(k_max + 3), -1)
        want = _quantise_brute(dtc, k_min, k_max)
        if want < old:
            want = old - 1 if (old - 1 >= k_min and t1 % (2 * dt_old) == 0) else old
        assert oracle.new_level(dtc, old, t1, k_min, k_max) == want
    # exact powers of two map to themselves; NaN goes to the smallest step
    assert oracle.new_level(2.0 ** -7, 7, 1 << (TICK_BITS - 7), k_min, k_max) == 7
    assert oracle.new_level(float("nan"), 7, 1 << (TICK_BITS - 7), k_min, k_max) == k_max


# --------------------------------------------------------------------------
# whole integration

def _kepler_state(t, e, a, M, m1, m2, nder):
    """Exact derivatives 0..nder-1 of both bodies' positions at time t."""
    mp.mp.dps = 40

    def rel(tt, c):
        n = mp.sqrt(M / a ** 3)
        E = mp.findroot(lambda E: E - e * mp.sin(E) - n * tt, n * tt)
        return [a * (mp.cos(E) - e), a * mp.sqrt(1 - e * e) * mp.sin(E)][c]
    d = np.zeros((nder, 3))
    for k in range(nder):
        for c in range(2):
            d[k, c] = float(mp.diff(lambda tt: rel(tt, c), mp.mpf(t), k))
    return np.stack([-m2 / M * d, m1 / M * d], axis=2)   # (nder, 3, 2)


@pytest.mark.parametrize("p,ks", [(4, [3, 4, 5, 6]), (6, [2, 3, 4, 5]), (8, [1, 2, 3, 4])])
def test_kepler_local_error_order(oracle_lib, p, ks):
    """One step of size h = 2^-k from the exact state of an e=0.1 Kepler orbit:
    the velocity error falls as h^(p+1) (local order of a p-th order scheme)."""
    m1 = m2 = 0.5
    e, a, M = mp.mpf("0.1"), mp.mpf(1), mp.mpf(1)
    d0 = _kepler_state(0.0, e, a, M, m1, m2, p)
    errs = []
    for k in ks:
        exact = _kepler_state(2.0 ** -k, e, a, M, m1, m2, 2)
        cfg = OracleConfig(order=p, eps2=0.0, eta=1.0, eta_start=1.0, k_min=k, k_max=k)
        s = oracle.State(np.array([m1, m2]), d0[0], d0[1], p, [d0[l + 2] for l in range(p - 2)])
        s.level[:] = k
        oracle.block_step(cfg, s)
        errs.append(float(np.linalg.norm(s.v - exact[1])))
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(abs(sl - (p + 1)) < 0.2 for sl in slopes), (errs, slopes)


@pytest.mark.parametrize("p,ks", [(4, [5, 6, 7]), (6, [4, 5, 6])])
def test_kepler_global_convergence(oracle_lib, p, ks):
    """Shared power-of-two steps on an e=0.3 Kepler orbit over t = 0..3: the
    largest position error at 12 checkpoints falls as dt^p (slope p +- 0.3).
    (At order 8 the asymptotic range lies below double-precision rounding on
    this problem; the local-order test above covers it.)"""
    m1 = m2 = 0.5
    e, a, M = mp.mpf("0.3"), mp.mpf(1), mp.mpf(1)
    cps = [0.25 * i for i in range(1, 13)]
    exact = [_kepler_state(t, e, a, M, m1, m2, 1)[0] for t in cps]
    d0 = _kepler_state(0.0, e, a, M, m1, m2, p)
    errs = []
    for k in ks:
        cfg = OracleConfig(order=p, eps2=0.0, eta=1.0, eta_start=1.0, k_min=k, k_max=k)
        s = oracle.State(np.array([m1, m2]), d0[0], d0[1], p)
        oracle.init(cfg, s)
        err = 0.0
        for t, ex in zip(cps, exact):
            oracle.integrate(cfg, s, int(t * TICKS_PER_UNIT))
            assert np.all(s.t_tick == int(t * TICKS_PER_UNIT))
            err = max(err, float(np.linalg.norm(s.x - ex)))
        errs.append(err)
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(abs(sl - p) < 0.3 for sl in slopes), (errs, slopes)


def _check_block_invariants(cfg, s, t_end):
    n = s.n
    steps_per_particle = np.zeros(n, np.int64)
    sum_act = 0
    t_prev = 0
    while True:
        nxt = s.t_tick + (1 << (TICK_BITS - s.level.astype(np.int64)))
        if nxt.min() > t_end:
            break
        lvl_old = s.level.copy()
        t_old = s.t_tick.copy()
        na, t_next, _ = oracle.block_step(cfg, s)
        assert t_next > t_prev
        t_prev = t_next
        moved = s.t_tick != t_old
        assert moved.sum() == na
        assert np.all(t_old[moved] + (1 << (TICK_BITS - lvl_old[moved].astype(np.int64))) == t_next)
        steps_per_particle += moved
        sum_act += na
        dt = 1 << (TICK_BITS - s.level.astype(np.int64))
        assert np.all(s.t_tick % dt == 0)                     # t_i multiple of dt_i
        assert np.all(s.level >= lvl_old - 1)                 # at most one doubling
        assert np.all((s.level >= cfg.k_min) & (s.level <= cfg.k_max))
    assert np.all(s.t_tick == t_end)                          # synchronised at t_end
    assert steps_per_particle.sum() == sum_act


@pytest.mark.parametrize("p", ORDERS)
def test_block_step_invariants(oracle_lib, p):
    m = nbody_ics.plummer(256, 101)
    cfg = OracleConfig(order=p, eps2=1e-4, eta=0.01 if p == 4 else 0.1, eta_start=0.01, k_min=3, k_max=20)
    s = oracle.State(m.m, m.x, m.v, p)
    oracle.init(cfg, s)
    _check_block_invariants(cfg, s, TICKS_PER_UNIT // 8)


def test_shared_steps_conserve_momentum(oracle_lib):
    """With one shared step size the Hermite corrector conserves linear
    momentum to rounding (the pair terms cancel at both ends of every step)."""
    m = nbody_ics.plummer(256, 102)
    cfg = OracleConfig(order=6, eps2=1e-4, eta=0.1, k_min=9, k_max=9)
    s = oracle.State(m.m, m.x, m.v, 6)
    oracle.init(cfg, s)
    P0 = s.v @ s.m
    oracle.integrate(cfg, s, TICKS_PER_UNIT // 8)
    scale = np.abs(s.v) @ s.m
    assert np.all(np.abs(s.v @ s.m - P0) < 1e-14 * scale.max() * 64)


def test_c1_energy_conservation(oracle_lib):
    """The small parity workload: Plummer N=1024, 4th order, eta=0.01, eps=1e-4,
    t = 0 -> 0.125.  The drift is a sanity bound, not a pinned value."""
    m = nbody_ics.plummer(1024, 11)
    cfg = OracleConfig(order=4, eps2=1e-8, eta=0.01, eta_start=0.01, k_min=3, k_max=20)
    s = oracle.State(m.m, m.x, m.v, 4)
    oracle.init(cfg, s)
    E0 = sum(oracle.energy(cfg, s.m, s.x, s.v))
    st = oracle.integrate(cfg, s, TICKS_PER_UNIT // 8)
    E1 = sum(oracle.energy(cfg, s.m, s.x, s.v))
    assert st["nonfinite"] == 0
    assert abs((E1 - E0) / E0) < 1e-6
    assert abs(E0 + 0.25) < 0.02
