"""Host-side diagnostics of a black-hole binary in the integrated state (the
paper's galactic nuclei with massive black-hole binaries and their
gravitational-wave emission, Abstract and Introduction): the Newtonian
orbital elements of a pair and Peters' (1964) orbit-averaged
gravitational-wave luminosity, decay rates and inspiral time (G = 1).

These read a state already copied to the host (``Simulation.to_numpy()``);
they are analysis of results, not a step of the block-step path.
"""
from __future__ import annotations

import numpy as np


def orbital_elements(m1: float, m2: float, x_rel, v_rel) -> dict:
    """Semi-major axis a, eccentricity e, specific orbital energy and the
    specific angular momentum of the Newtonian relative orbit of two bodies
    with relative position x_rel = x1 - x2 and velocity v_rel = v1 - v2
    (a < 0 for an unbound pair)."""
    M = float(m1) + float(m2)
    r = np.asarray(x_rel, float).reshape(3)
    w = np.asarray(v_rel, float).reshape(3)
    rn = float(np.linalg.norm(r))
    energy = 0.5 * float(np.dot(w, w)) - M / rn
    h = np.cross(r, w)
    ecc = np.cross(w, h) / M - r / rn          # Laplace-Runge-Lenz vector / M
    return {"a": -M / (2.0 * energy), "e": float(np.linalg.norm(ecc)), "energy": energy,
            "h": float(np.linalg.norm(h))}


def _enhancement_energy(e2: float) -> float:
    return (1.0 + 73.0 / 24.0 * e2 + 37.0 / 96.0 * e2 * e2) / (1.0 - e2) ** 3.5


def peters_luminosity(m1: float, m2: float, a: float, e: float, c: float) -> float:
    """Orbit-averaged gravitational-wave luminosity of a Kepler orbit,
    (32/5) nu^2 M^5 / (a^5 c^5) f(e), f(e) = (1 + 73/24 e^2 + 37/96 e^4) /
    (1 - e^2)^(7/2)."""
    M = m1 + m2
    nu = m1 * m2 / (M * M)
    return 32.0 / 5.0 * nu * nu * M ** 5 / (a ** 5 * c ** 5) * _enhancement_energy(e * e)


def peters_rates(m1: float, m2: float, a: float, e: float, c: float) -> tuple:
    """Orbit-averaged da/dt and de/dt of Peters (1964):
    da/dt = -(64/5) nu M^3 / (a^3 c^5) f(e),
    de/dt = -(304/15) nu M^3 e / (a^4 c^5) (1 + 121/304 e^2) / (1 - e^2)^(5/2)."""
    M = m1 + m2
    nu = m1 * m2 / (M * M)
    e2 = e * e
    dadt = -64.0 / 5.0 * nu * M ** 3 / (a ** 3 * c ** 5) * _enhancement_energy(e2)
    dedt = -304.0 / 15.0 * nu * M ** 3 * e / (a ** 4 * c ** 5) * (1.0 + 121.0 / 304.0 * e2) / (1.0 - e2) ** 2.5
    return dadt, dedt


def inspiral_time_circular(m1: float, m2: float, a: float, c: float) -> float:
    """Time for a circular binary to shrink to a = 0 under Peters' da/dt:
    (5/256) a^4 c^5 / (nu M^3)."""
    M = m1 + m2
    nu = m1 * m2 / (M * M)
    return 5.0 / 256.0 * a ** 4 * c ** 5 / (nu * M ** 3)


def binary_gw(h: dict, c: float, i: int = 0, j: int = 1) -> dict:
    """Diagnostics of the pair (i, j) of a host state dict (m, x, v as from
    Simulation.to_numpy()): its orbital elements and, when c > 0 and the
    pair is bound, Peters' luminosity, decay rates and circular-orbit
    inspiral time."""
    m1, m2 = float(h["m"][i]), float(h["m"][j])
    el = orbital_elements(m1, m2, h["x"][:, i] - h["x"][:, j], h["v"][:, i] - h["v"][:, j])
    out = {"a": float(el["a"]), "e": float(el["e"])}
    if c > 0 and el["a"] > 0 and el["e"] < 1:
        out["gw_luminosity"] = float(peters_luminosity(m1, m2, el["a"], el["e"], c))
        dadt, dedt = peters_rates(m1, m2, el["a"], el["e"], c)
        out["da_dt"] = float(dadt)
        out["de_dt"] = float(dedt)
        out["inspiral_time_circular"] = float(inspiral_time_circular(m1, m2, el["a"], c))
    return out
