"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

The paper's workloads are star clusters with a core-halo density structure
(Abstract) and galactic nuclei with massive black holes (Introduction); it
uses no public dataset.  These generators stand in for them:

* ``plummer``  -- Plummer sphere sampled as in Aarseth, Henon & Wielen (1974);
* ``king``     -- King (1966) model of central potential W0 (core-halo);
* ``with_bh_binary`` -- two massive bodies on a circular orbit added to a model.

All models come out in Henon units (G = M = 1, E = -1/4) with equal masses,
centred on the centre of mass.  The energy scaling uses the model's own
(analytic or quadrature) energy, so a sample of N bodies has E = -1/4 up to
sampling noise of order N^-1/2.

This module holds none of the integration arithmetic: no forces, no
predictor or corrector, no time steps.  It only draws initial conditions.
Random numbers come from NumPy's PCG64 seeded per workload.
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import numpy as np
from scipy.integrate import solve_ivp, cumulative_trapezoid
from scipy.special import erf

__all__ = ["plummer", "king", "king_profile", "with_bh_binary", "active_subset", "Model"]


@dataclass
class Model:
    m: np.ndarray   # (n,)
    x: np.ndarray   # (3, n)
    v: np.ndarray   # (3, n)

    @property
    def n(self) -> int:
        return self.m.shape[0]


def _isotropic(rng: np.random.Generator, r: np.ndarray) -> np.ndarray:
    """Vectors of length r with uniformly random directions, shape (3, n)."""
    n = r.shape[0]
    cth = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    sth = np.sqrt(1.0 - cth * cth)
    return np.stack([r * sth * np.cos(phi), r * sth * np.sin(phi), r * cth])


def _recentre(m: np.ndarray, x: np.ndarray, v: np.ndarray):
    M = m.sum()
    x = x - (x @ m / M)[:, None]
    v = v - (v @ m / M)[:, None]
    return x, v


def plummer(n: int, seed: int) -> Model:
    """Plummer sphere in Henon units.

    Radii from the inverted cumulative mass r = (X^(-2/3) - 1)^(-1/2), with X
    uniform on (0, 0.999] (the usual truncation of the infinite model);
    speeds v = q sqrt(2) (1 + r^2)^(-1/4) with q drawn by rejection from
    g(q) = q^2 (1 - q^2)^(7/2); isotropic directions.  Lengths are scaled by
    3 pi / 16 and speeds by sqrt(16 / (3 pi)), which gives E = -1/4 for the
    model with G = M = 1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.uniform(0.0, 1.0, n)
    while True:
        bad = (X <= 0.0) | (X > 0.999)
        if not bad.any():
            break
        X[bad] = rng.uniform(0.0, 1.0, int(bad.sum()))
    r = 1.0 / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        qq = rng.uniform(0.0, 1.0, todo.size)
        yy = rng.uniform(0.0, 0.1, todo.size)
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    vmag = q * np.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    x = _isotropic(rng, r) * (3.0 * np.pi / 16.0)
    v = _isotropic(rng, vmag) * np.sqrt(16.0 / (3.0 * np.pi))
    m = np.full(n, 1.0 / n)
    x, v = _recentre(m, x, v)
    return Model(m, x, v)


def _king_rho(W):
    """King density in units of the central density's normalisation:
    rho(W) proportional to e^W erf(sqrt W) - sqrt(4W/pi) (1 + 2W/3)."""
    W = np.maximum(W, 0.0)
    return np.exp(W) * erf(np.sqrt(W)) - np.sqrt(4.0 * W / np.pi) * (1.0 + 2.0 * W / 3.0)


@lru_cache(maxsize=16)
def king_profile(W0: float, npts: int = 20000):
    """Integrate the King (1966) model: W'' + (2/r) W' = -9 rho(W)/rho(W0),
    W(0) = W0, W'(0) = 0, out to W = 0 (the tidal radius).

    Units: G = 1, sigma = 1, King radius r0 = 1 (so 4 pi G rho0 = 9).
    Returns a dict with r, W, M (enclosed mass), r_t, M_t, and the model's
    potential (Wpot) and kinetic (T) energies."""
    rho0 = float(_king_rho(W0))

    def rhs(r, y):
        W, dW = y
        return [dW, -9.0 * _king_rho(W) / rho0 - 2.0 * dW / r]

    def hit_zero(r, y):
        return y[0]
    hit_zero.terminal = True
    hit_zero.direction = -1
    r_start = 1e-6
    y0 = [W0 - 1.5 * r_start ** 2, -3.0 * r_start]   # series W = W0 - 3/2 r^2 near 0
    sol = solve_ivp(rhs, (r_start, 1e4), y0, events=hit_zero, rtol=1e-11, atol=1e-13,
                    dense_output=True, method="DOP853")
    r_t = float(sol.t_events[0][0])
    r = np.concatenate([[0.0], np.geomspace(r_start, r_t, npts)])
    W = np.concatenate([[W0], sol.sol(r[1:])[0]])
    W[-1] = 0.0
    # enclosed mass from Gauss's law: M(r) = -r^2 W'(r)
    dW = np.concatenate([[0.0], sol.sol(r[1:])[1]])
    M = -r * r * dW
    M[0] = 0.0
    M_t = float(M[-1])
    # potential energy of a spherical system: -int G M(r) / r dM
    # dM/dr = 4 pi r^2 rho = 9 r^2 rho(W)/rho(W0), so M/r dM = 9 M r rho/rho0 dr
    integrand = 9.0 * M * r * _king_rho(W) / rho0
    Wpot = -float(np.trapezoid(integrand, r))
    # virial equilibrium of the isolated truncated model: 2T + W = 0
    T = -0.5 * Wpot
    return {"r": r, "W": W, "M": M, "r_t": r_t, "M_t": M_t, "Wpot": Wpot, "T": T, "rho0": rho0}


def king(n: int, W0: float, seed: int) -> Model:
    """King model of central potential W0 in Henon units.

    Radii are drawn from the model's cumulative mass profile; speeds by
    rejection from the local distribution v^2 (exp(W - v^2/2) - 1),
    0 <= v <= sqrt(2W); isotropic directions.  Then masses are set to 1/n and
    lengths / speeds rescaled with the model's energies so that G = M = 1 and
    E = -1/4 with virial ratio 1/2."""
    prof = king_profile(float(W0))
    rng = np.random.Generator(np.random.PCG64(seed))
    r_grid, M_grid, W_grid = prof["r"], prof["M"], prof["W"]
    cdf = M_grid / M_grid[-1]
    # strictly increasing cdf for inversion
    keep = np.concatenate([[True], np.diff(cdf) > 0])
    u = rng.uniform(0.0, 1.0, n)
    r = np.interp(u, cdf[keep], r_grid[keep])
    W = np.interp(r, r_grid, W_grid)
    # rejection sampling of the speed at each radius
    vesc = np.sqrt(2.0 * np.maximum(W, 0.0))
    vmag = np.zeros(n)
    todo = np.nonzero(W > 0)[0]
    # bound of g(v) = v^2 (e^(W - v^2/2) - 1) on [0, vesc]; with u = v^2/2,
    # g = 2u (e^(W-u) - 1) < 2u e^(W-u) <= 2 e^(W-1), and also g <= 2W (e^W - 1)
    while todo.size:
        Wt = W[todo]
        vt = rng.uniform(0.0, 1.0, todo.size) * vesc[todo]
        gmax = np.minimum(2.0 * np.exp(Wt - 1.0), 2.0 * Wt * np.expm1(Wt))
        y = rng.uniform(0.0, 1.0, todo.size) * gmax
        ok = y < vt * vt * np.expm1(Wt - 0.5 * vt * vt)
        vmag[todo[ok]] = vt[ok]
        todo = todo[~ok]
    x = _isotropic(rng, r)
    v = _isotropic(rng, vmag)
    # Henon scaling from the model energies (G = 1, model mass M_t):
    # W' = Wpot / M_t^2 / lam = -1/2  and  T' = T / M_t * mu^2 = 1/4
    lam = -2.0 * prof["Wpot"] / prof["M_t"] ** 2
    mu = np.sqrt(prof["M_t"] / (4.0 * prof["T"]))
    x = x * lam
    v = v * mu
    m = np.full(n, 1.0 / n)
    x, v = _recentre(m, x, v)
    return Model(m, x, v)


def with_bh_binary(model: Model, m_bh: float = 0.01, sep: float = 0.2) -> Model:
    """Prepend two bodies of mass m_bh at (+-sep/2, 0, 0) with velocities
    (0, +-v/2, 0), v = sqrt(2 m_bh / sep) (the circular relative speed of the
    pair alone), then recentre the whole system.  The two bodies get indices 0
    and 1, so a softening rule that exempts pairs below index 2 leaves their
    mutual force unsoftened."""
    vrel = np.sqrt(2.0 * m_bh / sep)
    xb = np.array([[sep / 2, -sep / 2], [0.0, 0.0], [0.0, 0.0]])
    vb = np.array([[0.0, 0.0], [vrel / 2, -vrel / 2], [0.0, 0.0]])
    m = np.concatenate([[m_bh, m_bh], model.m])
    x = np.concatenate([xb, model.x], axis=1)
    v = np.concatenate([vb, model.v], axis=1)
    x, v = _recentre(m, x, v)
    return Model(m, x, v)


def active_subset(n: int, n_act: int, seed: int) -> np.ndarray:
    """Sorted random subset of n_act distinct indices of [0, n), int32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if n_act >= n:
        return np.arange(n, dtype=np.int32)
    return np.sort(rng.choice(n, size=n_act, replace=False)).astype(np.int32)


def batched_plummer(n_clusters: int = 256, seed: int = 1400) -> list:
    """Independent Plummer clusters for the batched workload: sizes
    round(2^U(10, 16)) from one seeded draw, cluster c drawn with seed
    seed + c."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.round(2.0 ** rng.uniform(10.0, 16.0, n_clusters)).astype(int)
    return [plummer(int(s), seed + c) for c, s in enumerate(sizes)]


def kepler_pair(e: float = 0.5, a: float = 1.0, m1: float = 0.5, m2: float = 0.5) -> Model:
    """Two bodies at the pericentre of a Kepler orbit of eccentricity e and
    semi-major axis a (G = 1), in the centre-of-mass frame."""
    M = m1 + m2
    rp = a * (1.0 - e)
    vp = np.sqrt(M / a * (1.0 + e) / (1.0 - e))
    rel_x = np.array([rp, 0.0, 0.0])
    rel_v = np.array([0.0, vp, 0.0])
    x = np.stack([-m2 / M * rel_x, m1 / M * rel_x], axis=1)
    v = np.stack([-m2 / M * rel_v, m1 / M * rel_v], axis=1)
    return Model(np.array([m1, m2]), x, v)


def random_derivs(n: int, seed: int, order: int) -> list:
    """Seeded stand-ins for the stored acceleration derivatives a^(0..order-3)
    of n particles, (3, n) each, with magnitudes typical of a cluster in Henon
    units (|a| ~ 1, each higher derivative ~ 10 times the previous)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.normal(size=(3, n)) * 10.0 ** k for k in range(order - 2)]
