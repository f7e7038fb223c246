"""Shared helpers of the GPU parity tests (inputs, error norms)."""
import sys

import numpy as np

import nbody_ics
import oracle
from oracle import OracleConfig

TICKS = 1 << 20


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
    """Seeded derivative inputs a^(0..order-3) with magnitudes typical of a
    cluster in Henon units (|a| ~ 1, higher derivatives ~ 10^k)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.normal(size=(3, n)) * 10.0 ** k for k in range(order - 2)]


def oracle_force(order, eps2, n_hard, m, x, v, a=None, j=None, act=None):
    return oracle.force(OracleConfig(order=order, eps2=eps2, n_hard=n_hard), m, x, v,
                        a if order >= 6 else None, j if order >= 8 else None, act=act)
