"""Shared helpers of the GPU parity tests (inputs, error norms)."""
import sys

import numpy as np

import nbody_ics
import oracle
from oracle import OracleConfig

from paper_1312_1789_amd.abi import TICK_BITS, TICKS_PER_UNIT as TICKS  # noqa: E402

assert TICKS == oracle.oracle.TICKS_PER_UNIT and TICK_BITS == oracle.oracle.TICK_BITS


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(gpu, ref):
    """Per-particle relative error of vectors (3, n) or scalars (n,)."""
    gpu = np.asarray(gpu, float)
    ref = np.asarray(ref, float)
    if ref.ndim == 2:
        return np.linalg.norm(gpu - ref, axis=0) / np.linalg.norm(ref, axis=0)
    return np.abs(gpu - ref) / np.abs(ref)


def err_stats(e):
    e = np.asarray(e)
    return {"rms": float(np.sqrt(np.mean(e * e))), "max": float(e.max()), "p999": float(np.quantile(e, 0.999))}


def cluster_with_bh(n_stars, seed, W0=7.0):
    """King model plus a massive binary at indices 0, 1 (n_hard = 2)."""
    return nbody_ics.with_bh_binary(nbody_ics.king(n_stars, W0, seed), 0.01, 0.2)


def physical_derivs(m, x, v, eps2, n_hard):
    """Acceleration and jerk of the state (oracle, FP64): realistic inputs for
    the j-particle records of a force test."""
    out = oracle.force(OracleConfig(order=4, eps2=eps2, n_hard=n_hard), m, x, v, with_pot=False)
    return out["acc"], out["jrk"]


def random_derivs(n, seed, order):
    return nbody_ics.random_derivs(n, seed, order)


def random_block_state(n, seed, k_min=3, k_max=20):
    """Valid block-step times: t_i a multiple of dt_i = 2^-level_i, all
    t_i <= T and t_i + dt_i > T for T = 3 * 2^-k_min + 2^-5."""
    rng = np.random.default_rng(seed)
    level = rng.integers(k_min, k_max + 1, n).astype(np.int32)
    T = 3 * (TICKS >> k_min) + (TICKS >> 5)
    dt = (1 << (TICK_BITS - level.astype(np.int64)))
    t = (T // dt) * dt
    return t.astype(np.int64), level


def band_free_radii(x, act, seed, k_max=40, min_margin=1e-4):
    """h^2 per active particle in a gap of its sorted squared distances: k
    neighbours (k drawn in 0..k_max, moved up to the next gap at least
    2 min_margin wide in relative terms), h^2 at the geometric middle of the
    gap.  Also returns each sphere's relative distance to the nearest pair."""
    rng = np.random.default_rng(seed)
    h2 = np.zeros(act.size)
    margin = np.zeros(act.size)
    for q, i in enumerate(act):
        d2 = np.sum((x - x[:, i:i + 1]) ** 2, axis=0)
        d2[i] = np.inf
        s = np.sort(d2)
        k = int(rng.integers(0, k_max + 1))
        while True:
            lo = s[k - 1] if k > 0 else s[0] * 0.25
            hi = s[k]
            h2[q] = np.sqrt(lo * hi)
            margin[q] = min(h2[q] / lo - 1.0, 1.0 - h2[q] / hi)
            if margin[q] >= min_margin:
                break
            k += 1
    return h2, margin


def oracle_force(order, eps2, n_hard, m, x, v, a=None, j=None, act=None):
    return oracle.force(OracleConfig(order=order, eps2=eps2, n_hard=n_hard), m, x, v,
                        a if order >= 6 else None, j if order >= 8 else None, act=act)


def oracle_correct(ocfg, os0, act, T, F):
    """Oracle corrector, interpolation and level for the active list, composed
    from the oracle's per-component routines.  Also returns, per active row,
    the rounding scale of each interpolated derivative (sum of |coefficient x
    input|; the interpolation cancels heavily for short steps) and the
    distance of log2(dt_crit) from the nearest integer."""
    p, q = ocfg.order, ocfg.order // 2
    newd = [F["acc"], F["jrk"], F["snp"], F["crk"]]
    x, v = os0.x.copy(), os0.v.copy()
    d = [a.copy() for a in os0.d]
    lv = os0.level.copy()
    scale = np.zeros((p - q, 3, act.size))
    margin = np.zeros(act.size)
    dnorm = np.zeros((p, act.size))
    mats = {}
    for r, i in enumerate(act):
        h = (T - os0.t_tick[i]) / TICKS
        if h not in mats:
            eye = np.eye(2 * q)
            mats[h] = np.stack([oracle.hermite_high(p, h, eye[k, :q], eye[k, q:]) for k in range(2 * q)], axis=1)
        M = mats[h]
        Dall = np.zeros((p, 3))
        for c in range(3):
            D0 = [os0.d[k][c, i] for k in range(q)]
            D1 = [newd[k][c, r] for k in range(q)]
            x[c, i], v[c, i] = oracle.hermite_correct(p, h, os0.x[c, i], os0.v[c, i], D0, D1)
            Dall[:q, c] = D1
            Dall[q:, c] = oracle.hermite_high(p, h, D0, D1)
            scale[:, c, r] = np.abs(M) @ np.abs(np.concatenate([D0, D1]))
        for k in range(p - 2):
            d[k][:, i] = Dall[k]
        dnorm[:, r] = np.linalg.norm(Dall, axis=1)
        dtc = oracle.dt_crit(p, ocfg.eta, dnorm[:, r], ocfg.dt_rule)
        lv[i] = oracle.new_level(dtc, int(os0.level[i]), T, ocfg.k_min, ocfg.k_max)
        margin[r] = abs(np.log2(dtc) - np.round(np.log2(dtc)))
    return x, v, d, lv, scale, margin, dnorm


def compare_corrected(got, want, act, order, rel_force_err, tag, rule=1):
    """x, v to FP64 rounding; interpolated derivatives within their rounding
    scale (amplified by the force difference); levels equal except where
    log2(dt_crit) lies within its own rounding uncertainty of an integer
    (the highest interpolated derivatives cancel heavily for short steps)."""
    x, v, d, lv, scale, margin, dnorm = want
    q = order // 2
    # relative uncertainty of each interpolated |a^(k)| from its rounding
    # scale, carried into log2(dt_crit): the criterion uses a^(p-3..p-1)
    # under a 1/(p-3) power (order 4: a^(2), a^(3) under a square root; the
    # order-4 form at orders 6, 8: a^(1..3), power 1)
    unc = (512 * 2.0 ** -53 + rel_force_err) * np.linalg.norm(scale, axis=1) / np.maximum(dnorm[q:], 1e-300)
    if order == 4:
        ks, root = [2, 3], 2.0
    elif rule == 2:
        ks, root = [1, 2, 3], 1.0
    else:
        ks, root = list(range(order - 3, order)), float(order - 3)
    margin_tol = 4.0 * sum((unc[k - q] for k in ks if k >= q), np.zeros(act.size)) / root / np.log(2.0) + 1e-12
    for name, g, w in [("x", got["x"], x), ("v", got["v"], v)]:
        st = err_stats(rel_err(g[:, act], w[:, act]))
        say("%s order %d %s rms %.2e max %.2e" % (tag, order, name, st["rms"], st["max"]))
        assert st["max"] <= 1e-12
    for k in range(order - 2):
        diff = np.abs(got["d"][k][:, act] - d[k][:, act])
        if k < q:
            bound = 1e-13 * np.abs(d[k][:, act]) + 1e-300 if rel_force_err == 0 else \
                rel_force_err * np.linalg.norm(d[k][:, act], axis=0)
        else:
            bound = (512 * 2.0 ** -53 + rel_force_err) * scale[k - q]
        ratio = float(np.max(diff / np.maximum(bound, 1e-300)))
        say("%s order %d d[%d] max |diff| / bound %.2e" % (tag, order, k, ratio))
        assert ratio <= 1.0, (k, ratio)
    mism = np.nonzero(got["level"][act] != lv[act])[0]
    say("%s order %d level mismatches %d of %d (margins %s, allowed %s)"
        % (tag, order, mism.size, act.size, margin[mism], margin_tol[mism]))
    assert np.all(margin[mism] < margin_tol[mism])
    assert np.all(np.abs(got["level"][act].astype(int) - lv[act].astype(int)) <= 1)
