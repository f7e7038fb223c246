"""GPU tests of the post-Newtonian terms between hard particles (c_light,
pn_terms; 4th order), against the oracle (its pinned PN terms) and against
the physics the oracle pins fix:

* initial forces and derivatives (orders 4, 6, 8) of a cluster with a
  black-hole binary (c = 2: the 1PN terms are ~2.5% of the binary's mutual
  force), and with a third black hole (three pairs), equal the oracle's;
* whole block steps from the GPU's own state match the oracle's predictor,
  force + PN terms and corrector (FP64: the comparison of the plain step
  tests; MIXED: x, v within 1e-9, 1e-7, the new acceleration within the
  force tolerance, the FP32 pair terms setting the scale);
* a two-body inspiral with the 2.5PN terms shrinks at Peters' rate, and the
  FP64 run ends where the oracle's integration ends;
* an eccentric two-body orbit with the 1PN terms advances its periastron by
  6 pi M / (c^2 a (1 - e^2)) per orbit.
The 2PN terms (pn_terms & 2) take part in the init and step parity cases.
"""
import numpy as np
import pytest

import nbody_ics
import oracle
from helpers import TICK_BITS, TICKS, compare_corrected, oracle_correct, rel_err, say
from oracle import OracleConfig

pytestmark = pytest.mark.gpu


def _sim(m, x, v, precision, c, terms, n_hard=2, eps2=1e-8, eta=0.01, order=4):
    from paper_1312_1789_amd import Simulation
    return Simulation(m, x, v, order=order, precision=precision, eps2=eps2, n_hard=n_hard, eta=eta,
                      eta_start=0.01, c_light=c, pn_terms=terms)


def _ocfg(sim):
    c = sim.cfg
    return OracleConfig(order=c.order, eps2=c.eps2, n_hard=c.n_hard, eta=c.eta, eta_start=c.eta_start,
                        k_min=c.k_min, k_max=c.k_max, dt_rule=sim.dt_rule, c_light=c.c_light, pn_terms=c.pn_terms)


def _bh_model(n_bh):
    """Plummer cluster with a black-hole binary (indices 0, 1; separation 0.2,
    mass 0.01 each) and, for n_bh = 3, a third black hole of the same mass at
    index 2 on a roughly circular orbit about the binary at distance 0.2
    (three pairs of post-Newtonian terms per hard particle row)."""
    model = nbody_ics.with_bh_binary(nbody_ics.plummer(1022, 91), 0.01, 0.2)
    if n_bh == 3:
        m, x, v = model.m.copy(), model.x.copy(), model.v.copy()
        m[2] = 0.01
        x[:, 2] = [0.0, 0.16, 0.12]
        v[:, 2] = np.array([-1.0, 0.0, 0.0]) * np.sqrt(0.02 / 0.2)
        model = nbody_ics.Model(m, x, v)
    return model


# pn_terms: 5 = 1PN + 2.5PN, 7 = 1PN + 2PN + 2.5PN, 2 = 2PN alone
@pytest.mark.parametrize("order,precision,n_bh,terms", [(4, "fp64", 2, 5), (4, "mixed", 2, 5), (6, "fp64", 2, 5),
                                                        (8, "fp64", 2, 5), (8, "mixed", 2, 5), (4, "fp64", 3, 5),
                                                        (6, "fp64", 3, 5), (4, "fp64", 2, 7), (6, "mixed", 2, 7),
                                                        (8, "fp64", 2, 7), (8, "fp64", 3, 2)])
def test_pn_init_and_step_parity(order, precision, n_bh, terms):
    model = _bh_model(n_bh)
    sim = _sim(model.m, model.x, model.v, precision, 2.0, terms, n_hard=n_bh, order=order,
               eta=0.01 if order == 4 else 0.1)
    ocfg = _ocfg(sim)
    sim.init()
    h = sim.to_numpy()
    os_ = oracle.State(model.m, model.x, model.v, order)
    oracle.init(ocfg, os_)
    for k in range(min(order - 2, 4)):
        e = rel_err(h["d"][k], os_.d[k])
        rms = float(np.sqrt(np.mean(e * e)))
        say("pn init p%d %s %d BHs d[%d] rms rel %.2e max %.2e (black holes %.2e)"
            % (order, precision, n_bh, k, rms, e.max(), e[:n_bh].max()))
        assert rms <= 1e-12 and e.max() <= 1e-9 and e[:n_bh].max() <= 1e-12
    assert np.sum(h["level"] != os_.level) <= 2
    plain = oracle.State(model.m, model.x, model.v, order)
    oracle.init(OracleConfig(order=order, eps2=ocfg.eps2, n_hard=n_bh, eta=ocfg.eta, eta_start=ocfg.eta_start),
                plain)
    shift = (np.linalg.norm(os_.d[0][:, :n_bh] - plain.d[0][:, :n_bh], axis=0)
             / np.linalg.norm(plain.d[0][:, :n_bh], axis=0))
    say("pn init: relative change of the black holes' acceleration %.2e" % shift.max())
    assert shift.min() > 1e-3                # the terms are on
    rel_force = 1e-11 if precision == "fp64" else 3e-5
    bh_steps = 0
    for step in range(10):
        h0 = sim.to_numpy()
        os0 = oracle.State(h0["m"], h0["x"], h0["v"], order, [a.copy() for a in h0["d"]], h0["t_tick"].copy(),
                           h0["level"].copy())
        nxt = h0["t_tick"] + (1 << (TICK_BITS - h0["level"].astype(np.int64)))
        T = int(nxt.min())
        act = np.nonzero(nxt == T)[0].astype(np.int32)
        bh_steps += int(np.sum(act < n_bh))
        t_g, na_g = sim.step()
        assert (t_g, na_g) == (T, act.size), step
        xp, vp, ap, jp = oracle.predict(ocfg, os0, T)
        F = oracle.force(ocfg, os0.m, xp, vp, ap if order >= 6 else None, jp if order >= 8 else None, act=act)
        oracle.pn(ocfg, os0.m, xp, vp, act, F["acc"], F["jrk"], F["snp"] if order >= 6 else None,
                  F["crk"] if order >= 8 else None)
        want = oracle_correct(ocfg, os0, act, T, F)
        got = sim.to_numpy()
        if precision == "fp64":
            compare_corrected(got, want, act, order, rel_force, "pn step %d p%d %s" % (step, order, precision),
                              sim.dt_rule)
        else:
            # FP32 pair terms (the PN terms are FP64 in both modes): x, v within
            # what a force difference of ~1e-6 moves them in one step of up to
            # 2^-3 (h |da| for v, h^2 |da| for x), the new acceleration within
            # the force tolerance
            for name, g, w, tol in (("x", got["x"], want[0], 1e-9), ("v", got["v"], want[1], 1e-7)):
                e = rel_err(g[:, act], w[:, act])
                say("pn step %d mixed %s max rel %.2e" % (step, name, e.max()))
                assert e.max() <= tol
            ea = rel_err(got["d"][0][:, act], want[2][0][:, act])
            say("pn step %d mixed acc rms rel %.2e" % (step, np.sqrt(np.mean(ea * ea))))
            assert np.sqrt(np.mean(ea * ea)) <= 2e-6
    assert bh_steps > 0
    sim.close()


def _binary(e, m1=0.6, m2=0.4, a=1.0, apastron=False):
    """Two bodies on a Newtonian orbit of semi-major axis a and eccentricity e,
    at periastron (or apastron) on the x axis, centre of mass at rest at the
    origin."""
    M = m1 + m2
    s = -1.0 if apastron else 1.0
    rp = a * (1 - s * e)
    vp = np.sqrt(M / a * (1 + s * e) / (1 - s * e))
    x = np.array([[m2 / M * rp, -m1 / M * rp], [0.0, 0.0], [0.0, 0.0]])
    v = np.array([[0.0, 0.0], [m2 / M * vp, -m1 / M * vp], [0.0, 0.0]])
    return np.array([m1, m2]), x, v


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pn_two_body_inspiral_peters_rate(precision):
    m, x, v = _binary(0.0)
    M, nu, a0, c, T = 1.0, 0.24, 1.0, 8.0, 16.0
    sim = _sim(m, x, v, precision, c, 4, eps2=0.0)
    sim.init()
    sim.integrate(int(T * TICKS))
    h = sim.to_numpy()
    r = np.linalg.norm(h["x"][:, 0] - h["x"][:, 1])
    w = h["v"][:, 0] - h["v"][:, 1]
    a1 = -M / (2.0 * (0.5 * np.dot(w, w) - M / r))
    rate = (a1 - a0) / T
    want = -64.0 / 5.0 * nu * M ** 3 / (a0 ** 3 * c ** 5)
    say("pn inspiral %s: da/dt %.5e, Peters %.5e" % (precision, rate, want))
    assert rate == pytest.approx(want, rel=0.02 if precision == "fp64" else 0.05)
    if precision == "fp64":
        os_ = oracle.State(m, x, v, 4)
        ocfg = _ocfg(sim)
        oracle.init(ocfg, os_)
        oracle.integrate(ocfg, os_, int(T * TICKS))
        e = np.abs(h["x"] - os_.x).max() / np.abs(os_.x).max()
        say("pn inspiral fp64: GPU vs oracle final positions max rel %.2e" % e)
        assert e <= 1e-7
    sim.close()


def _runge_lenz_angle(x, v, M):
    r = x[:, 0] - x[:, 1]
    w = v[:, 0] - v[:, 1]
    A = np.cross(w, np.cross(r, w)) - M * r / np.linalg.norm(r)
    return np.arctan2(A[1], A[0])


def test_pn_periastron_advance():
    """Ten orbits of an e = 0.5 binary with the 1PN terms, from apastron to
    (close to) apastron: the osculating periastron moves mostly during the
    periastron passages, so whole passages are counted.  The advance is
    6 pi M / (c^2 a (1 - e^2)) per orbit within 1%, and the run ends where
    the oracle's ends."""
    e, c, orbits = 0.5, 20.0, 10
    m, x, v = _binary(e, apastron=True)
    M, a = 1.0, 1.0
    t_end = int(orbits * 2 * np.pi * np.sqrt(a ** 3 / M) * TICKS)
    sim = _sim(m, x, v, "fp64", c, 1, eps2=0.0)
    sim.init()
    w0 = _runge_lenz_angle(x, v, M)
    sim.integrate(t_end)
    h = sim.to_numpy()
    dw = (_runge_lenz_angle(h["x"], h["v"], M) - w0) % (2 * np.pi)
    want = orbits * 6 * np.pi * M / (c * c * a * (1 - e * e))
    os_ = oracle.State(m, x, v, 4)
    ocfg = _ocfg(sim)
    oracle.init(ocfg, os_)
    oracle.integrate(ocfg, os_, t_end)
    dw_o = (_runge_lenz_angle(os_.x, os_.v, M) - w0) % (2 * np.pi)
    say("pn periastron advance over %d orbits: GPU %.6f rad, oracle %.6f, 1PN prediction %.6f"
        % (orbits, dw, dw_o, want))
    assert dw == pytest.approx(want, rel=0.01)
    assert dw == pytest.approx(dw_o, rel=1e-8)
    sim.close()
