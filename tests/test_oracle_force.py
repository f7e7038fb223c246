"""Pins of the oracle's pairwise force and derivatives (acceleration, jerk,
snap, crackle, potential) against results fixed by mathematics, not by the
oracle's own formula: high-precision numerical differentiation of the
softened force along polynomial trajectories, the Kepler two-body solution,
momentum antisymmetry and rotation / translation symmetry.

The method is direct summation of softened Newtonian gravity with the force
derivatives a high-order Hermite scheme needs (paper: Abstract; Sec. "Codes
description"); the formulas follow Nitadori & Makino (2008).
"""
import mpmath as mp
import numpy as np
import pytest

import oracle
from oracle import OracleConfig


def _rel(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _mp_force_derivs(m, X, V, A, J, S, eps2, n_hard, i):
    """d^k/dt^k at t=0 (k=0..3) of sum_j m_j r_ij / (r_ij^2 + eps_ij^2)^(3/2)
    along x_k(t) = X + V t + A t^2/2 + J t^3/6 + S t^4/24, and the potential,
    evaluated with mpmath at 50 digits."""
    mp.mp.dps = 50
    n = len(m)
    mm = [mp.mpf(float(q)) for q in m]

    def pos(k, c, t):
        return (mp.mpf(float(X[c, k])) + mp.mpf(float(V[c, k])) * t + mp.mpf(float(A[c, k])) * t ** 2 / 2
                + mp.mpf(float(J[c, k])) * t ** 3 / 6 + mp.mpf(float(S[c, k])) * t ** 4 / 24)

    def force_comp(c):
        def F(t):
            s = mp.mpf(0)
            for j in range(n):
                if j == i:
                    continue
                e2 = 0 if (i < n_hard and j < n_hard) else mp.mpf(eps2)
                r = [pos(j, cc, t) - pos(i, cc, t) for cc in range(3)]
                f = r[0] ** 2 + r[1] ** 2 + r[2] ** 2 + e2
                s += mm[j] * r[c] / f ** mp.mpf(1.5)
            return s
        return F

    out = np.zeros((4, 3))
    for c in range(3):
        F = force_comp(c)
        for k in range(4):
            out[k, c] = float(mp.diff(F, 0, k))
    pot = mp.mpf(0)
    for j in range(n):
        if j == i:
            continue
        e2 = 0 if (i < n_hard and j < n_hard) else mp.mpf(eps2)
        r = [pos(j, cc, 0) - pos(i, cc, 0) for cc in range(3)]
        pot -= mm[j] / mp.sqrt(r[0] ** 2 + r[1] ** 2 + r[2] ** 2 + e2)
    return out, float(pot)


@pytest.mark.parametrize("seed", [1, 2])
def test_force_matches_numerical_derivatives(oracle_lib, seed):
    """Brute force on N=6: the four outputs are the successive time
    derivatives of the softened force; pairs among particles 0, 1 are
    unsoftened (n_hard = 2)."""
    rng = np.random.default_rng(seed)
    n = 6
    m = rng.uniform(0.2, 1.0, n)
    X = rng.uniform(-1, 1, (3, n))
    V = rng.uniform(-1, 1, (3, n))
    A = rng.uniform(-1, 1, (3, n))
    J = rng.uniform(-1, 1, (3, n))
    S = rng.uniform(-1, 1, (3, n))
    eps2 = 0.05
    cfg = OracleConfig(order=8, eps2=eps2, n_hard=2)
    out = oracle.force(cfg, m, X, V, A, J)
    for i in range(n):
        ref, pot = _mp_force_derivs(m, X, V, A, J, S, eps2, 2, i)
        for k, key in enumerate(("acc", "jrk", "snp", "crk")):
            assert _rel(out[key][:, i], ref[k]) < 1e-13, (i, key)
        assert abs(out["pot"][i] - pot) < 1e-13 * abs(pot)


def test_lower_orders_ignore_unused_inputs(oracle_lib):
    """Order 4 uses only (x, v); order 6 adds a: the results for the
    derivatives they define do not depend on higher inputs."""
    rng = np.random.default_rng(3)
    n = 16
    m = rng.uniform(0.2, 1.0, n)
    X, V, A, J = (rng.uniform(-1, 1, (3, n)) for _ in range(4))
    o8 = oracle.force(OracleConfig(order=8, eps2=0.01), m, X, V, A, J)
    o6 = oracle.force(OracleConfig(order=6, eps2=0.01), m, X, V, A, None)
    o4 = oracle.force(OracleConfig(order=4, eps2=0.01), m, X, V, None, None)
    np.testing.assert_array_equal(o8["acc"], o4["acc"])
    np.testing.assert_array_equal(o8["jrk"], o4["jrk"])
    np.testing.assert_array_equal(o8["snp"], o6["snp"])


def _kepler_rel(t, e, a, M):
    """Relative position of a Kepler orbit (pericentre at t=0, along +x)."""
    n = mp.sqrt(M / a ** 3)
    Mn = n * t
    E = mp.findroot(lambda E: E - e * mp.sin(E) - Mn, Mn)
    return [a * (mp.cos(E) - e), a * mp.sqrt(1 - e * e) * mp.sin(E)]


def test_kepler_two_body_derivatives(oracle_lib):
    """Unsoftened two-body problem: a_2 = -m_1 r / |r|^3 and the jerk, snap
    and crackle equal the time derivatives of the exact Kepler orbit when the
    inputs are the exact positions, velocities, accelerations and jerks."""
    mp.mp.dps = 40
    m1, m2 = 0.6, 0.4
    M = m1 + m2
    e, a = mp.mpf("0.5"), mp.mpf(1)
    t0 = mp.mpf("0.7")
    d = []
    for k in range(6):
        d.append([float(mp.diff(lambda t, c=c: _kepler_rel(t, e, a, M)[c], t0, k)) for c in range(2)])
    d = np.array([[q[0], q[1], 0.0] for q in d])  # d[k] = r^(k)(t0), 3-vectors
    # particle 1 at -(m2/M) r, particle 2 at +(m1/M) r
    X = np.stack([-m2 / M * d[0], m1 / M * d[0]], axis=1)
    V = np.stack([-m2 / M * d[1], m1 / M * d[1]], axis=1)
    Acc = np.stack([-m2 / M * d[2], m1 / M * d[2]], axis=1)
    Jk = np.stack([-m2 / M * d[3], m1 / M * d[3]], axis=1)
    out = oracle.force(OracleConfig(order=8, eps2=0.0), [m1, m2], X, V, Acc, Jk)
    r = d[0]
    closed = -m1 * r / np.linalg.norm(r) ** 3
    assert _rel(out["acc"][:, 1], closed) < 1e-14
    for k, key in enumerate(("acc", "jrk", "snp", "crk")):
        assert _rel(out[key][:, 1], m1 / M * d[k + 2]) < 1e-12, key
        assert _rel(out[key][:, 0], -m2 / M * d[k + 2]) < 1e-12, key
    assert abs(out["pot"][1] + m1 / np.linalg.norm(r)) < 1e-15


def test_circular_orbit_derivative_magnitudes(oracle_lib):
    """On a circular orbit every derivative rotates with the orbit, so
    |a^(k)| = omega^k |a| exactly."""
    m1 = m2 = 0.5
    sep = 1.0
    w = np.sqrt((m1 + m2) / sep ** 3)
    r = np.array([sep, 0, 0.0])
    rv = np.array([0, sep * w, 0.0])
    ra = -w * w * r
    rj = -w * w * rv
    X = np.stack([-0.5 * r, 0.5 * r], 1)
    V = np.stack([-0.5 * rv, 0.5 * rv], 1)
    A = np.stack([-0.5 * ra, 0.5 * ra], 1)
    J = np.stack([-0.5 * rj, 0.5 * rj], 1)
    out = oracle.force(OracleConfig(order=8, eps2=0.0), [m1, m2], X, V, A, J)
    amag = np.linalg.norm(out["acc"][:, 1])
    for k, key in enumerate(("acc", "jrk", "snp", "crk")):
        assert abs(np.linalg.norm(out[key][:, 1]) - w ** k * amag) < 1e-14, key


def _random_system(n, seed):
    rng = np.random.default_rng(seed)
    m = rng.uniform(0.5, 1.5, n) / n
    X, V, A, J = (rng.normal(size=(3, n)) for _ in range(4))
    return m, X, V, A, J


def test_momentum_antisymmetry(oracle_lib):
    """m_i (term on i from j) = -m_j (term on j from i), so the
    mass-weighted sums of a, jerk, snap and crackle vanish."""
    m, X, V, A, J = _random_system(200, 5)
    out = oracle.force(OracleConfig(order=8, eps2=1e-4, n_hard=3), m, X, V, A, J)
    for key in ("acc", "jrk", "snp", "crk"):
        s = out[key] @ m
        scale = np.abs(out[key]) @ m
        assert np.all(np.abs(s) <= 1e-13 * scale), key


def test_translation_and_rotation(oracle_lib):
    m, X, V, A, J = _random_system(64, 6)
    cfg = OracleConfig(order=8, eps2=1e-3)
    ref = oracle.force(cfg, m, X, V, A, J)
    sh = oracle.force(cfg, m, X + np.array([[0.25], [-0.5], [0.125]]), V + 0.3, A - 0.7, J + 1.1)
    for key in ("acc", "jrk", "snp", "crk", "pot"):
        assert _rel(sh[key], ref[key]) < 1e-12, key
    Q, _ = np.linalg.qr(np.random.default_rng(7).normal(size=(3, 3)))
    rot = oracle.force(cfg, m, Q @ X, Q @ V, Q @ A, Q @ J)
    for key in ("acc", "jrk", "snp", "crk"):
        assert _rel(rot[key], Q @ ref[key]) < 1e-13, key
    assert _rel(rot["pot"], ref["pot"]) < 1e-14


def test_active_subset_matches_full(oracle_lib):
    """The active list only selects rows: same values as the full evaluation."""
    m, X, V, A, J = _random_system(100, 8)
    cfg = OracleConfig(order=8, eps2=1e-3)
    full = oracle.force(cfg, m, X, V, A, J)
    act = np.array([3, 17, 18, 64, 99], np.int32)
    sub = oracle.force(cfg, m, X, V, A, J, act=act)
    for key in ("acc", "jrk", "snp", "crk"):
        np.testing.assert_array_equal(sub[key], full[key][:, act])


def test_potential_consistent_with_energy(oracle_lib):
    """W = 1/2 sum_i m_i pot_i, computed by the separate energy routine."""
    m, X, V, _, _ = _random_system(300, 9)
    cfg = OracleConfig(order=4, eps2=1e-3, n_hard=4)
    out = oracle.force(cfg, m, X, V)
    T, W = oracle.energy(cfg, m, X, V)
    assert abs(0.5 * m @ out["pot"] - W) < 1e-13 * abs(W)
    assert abs(T - 0.5 * np.sum(m * np.sum(V * V, axis=0))) < 1e-14 * T
    # two-body closed form
    T2, W2 = oracle.energy(OracleConfig(eps2=0.01), [0.3, 0.7], [[0, 1.0], [0, 0], [0, 0]], np.zeros((3, 2)))
    assert abs(W2 + 0.3 * 0.7 / np.sqrt(1.01)) < 1e-16 and T2 == 0.0
