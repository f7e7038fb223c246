"""GPU parity of the O(n) / O(n_act) steps of the hot path (scheduler,
predictor, corrector + interpolation + time step, initialisation, energy,
whole block steps) against the CPU oracle on identical inputs.

Integer work (active sets, times, levels) must match exactly; a level may
differ only where the step criterion lies within rounding of a power of two
(checked).  FP64 values: relative error <= 1e-12 per particle (rounding order
differs between the two implementations).
"""
import numpy as np
import pytest
import torch

import nbody_ics
import oracle
from helpers import TICK_BITS, TICKS, compare_corrected, err_stats, oracle_correct, random_block_state, rel_err, say
from oracle import OracleConfig

pytestmark = pytest.mark.gpu


def _sim(model, order, precision="fp64", eps2=1e-8, n_hard=0, eta=None, k_min=3, k_max=20):
    from paper_1312_1789_amd import Simulation
    eta = eta if eta is not None else (0.01 if order == 4 else 0.1)
    return Simulation(model.m, model.x, model.v, order=order, precision=precision, eps2=eps2, n_hard=n_hard,
                      eta=eta, eta_start=0.01, k_min=k_min, k_max=k_max)


def _ocfg(sim):
    c = sim.cfg
    return OracleConfig(order=c.order, eps2=c.eps2, n_hard=c.n_hard, eta=c.eta, eta_start=c.eta_start,
                        k_min=c.k_min, k_max=c.k_max, dt_rule=sim.dt_rule)


def _ostate(h, order):
    return oracle.State(h["m"], h["x"], h["v"], order, [a.copy() for a in h["d"]], h["t_tick"].copy(),
                        h["level"].copy())


def test_schedule_exact():
    # n = 2^20 is the largest system whose compaction blocks find their own
    # offsets (1024 scheduling blocks); 2^20 + 3000 takes the path with a
    # separate one-block scan
    for n, seed in [(1, 1), (1000, 2), (5003, 3), (70000, 4), (1 << 20, 6), ((1 << 20) + 3000, 7)]:
        model = nbody_ics.plummer(max(n, 2), seed)
        sim = _sim(model, 4)
        t, lv = random_block_state(model.n, seed)
        sim.load_state(model.x, model.v, [np.zeros((3, model.n))] * 2, t, lv)
        t_next, act = sim.schedule()
        nxt = t + (1 << (TICK_BITS - lv.astype(np.int64)))
        want_t = int(nxt.min())
        want = np.nonzero(nxt == want_t)[0]
        say("schedule n=%d n_act=%d" % (model.n, want.size))
        assert t_next == want_t
        np.testing.assert_array_equal(act.cpu().numpy(), want)


def test_schedule_block_minima():
    """Crafted states for the per-block (minimum, count at the minimum) pass,
    n = 5003 (five scheduling blocks of 1024, a ragged last one): every
    particle active; one active particle in the ragged block while every
    other block has many particles tied at a larger minimum of its own; the
    global minimum reached in two blocks only, with ties inside a block."""
    n = 5003
    model = nbody_ics.plummer(n, 5)
    sim = _sim(model, 4)
    cases = []
    cases.append((np.zeros(n, np.int64), np.full(n, 5, np.int32)))
    t = np.zeros(n, np.int64)
    lv = np.full(n, 6, np.int32)
    lv[::7] = 8                      # block minima at t = 2^-8, many ties per block
    lv[5002] = 9                     # the global minimum, 2^-9, in the ragged block
    cases.append((t, lv))
    t = np.full(n, TICKS >> 6, np.int64)
    lv = np.full(n, 4, np.int32)
    lv[100:140] = 7                  # block 0: 40 ties at a larger minimum
    lv[[1500, 3100, 3101]] = 9       # the global minimum in blocks 1 and 3
    lv[4200:4300] = 8                # block 4: ties at an intermediate value
    cases.append((t, lv))
    for k, (t, lv) in enumerate(cases):
        sim.load_state(model.x, model.v, [np.zeros((3, n))] * 2, t, lv)
        t_next, act = sim.schedule()
        nxt = t + (1 << (TICK_BITS - lv.astype(np.int64)))
        want_t = int(nxt.min())
        want = np.nonzero(nxt == want_t)[0]
        say("schedule case %d: t_next %d, n_act %d" % (k, want_t, want.size))
        assert t_next == want_t
        np.testing.assert_array_equal(act.cpu().numpy(), want)
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
@pytest.mark.parametrize("order", [4, 6, 8])
def test_predict_parity(order, precision):
    n = 1500
    model = nbody_ics.plummer(n, 31)
    sim = _sim(model, order, precision)
    rng = np.random.default_rng(32)
    d = [rng.normal(size=(3, n)) * 4.0 ** k for k in range(order - 2)]
    t, lv = random_block_state(n, 33)
    sim.load_state(model.x, model.v, d, t, lv)
    T = int((t + (1 << (TICK_BITS - lv.astype(np.int64)))).min())
    sim.predict(T)
    got = {k: v.cpu().numpy() for k, v in sim.predicted().items()}
    os_ = oracle.State(model.m, model.x, model.v, order, d, t, lv)
    xp, vp, ap, jp = oracle.predict(_ocfg(sim), os_, T)
    want = {"xp": xp, "vp": vp, "ap": ap, "jp": jp}
    keys = ["xp", "vp"] + (["ap"] if order >= 6 else []) + (["jp"] if order >= 8 else [])
    for k in keys:
        scale = np.sqrt(np.mean(want[k] ** 2))
        e = np.abs(got[k] - want[k]) / (np.abs(want[k]) + 1e-6 * scale)
        if precision == "fp64" or k in ("xp", "vp") and precision == "mixed":
            tol = 1e-14
        elif precision == "ds" and k in ("xp", "vp"):
            tol = 2.0 ** -44           # hi + lo keeps ~48 bits
        else:
            tol = 2.0 ** -24           # FP32 acceleration / jerk
        say("predict order %d %s %s max rel %.2e" % (order, precision, k, e.max()))
        assert e.max() <= tol, (k, e.max())


@pytest.mark.parametrize("order", [4, 6, 8])
def test_init_parity(order):
    model = nbody_ics.with_bh_binary(nbody_ics.plummer(1998, 41))
    sim = _sim(model, order, n_hard=2)
    sim.init()
    got = sim.to_numpy()
    os_ = oracle.State(model.m, model.x, model.v, order)
    oracle.init(_ocfg(sim), os_)
    for k in range(order - 2):
        if order == 8 and k >= 4:
            assert np.all(got["d"][k] == 0.0)
            continue
        st = err_stats(rel_err(got["d"][k], os_.d[k]))
        say("init order %d d[%d] rms %.2e max %.2e" % (order, k, st["rms"], st["max"]))
        assert st["rms"] <= 1e-12 and st["max"] <= 1e-9
    assert np.all(got["t_tick"] == 0)
    assert np.sum(got["level"] != os_.level) <= 2


@pytest.mark.parametrize("order", [4, 6, 8])
def test_correct_parity(order):
    """Identical old state, identical new forces: corrected state,
    interpolated derivatives and new levels."""
    n = 2000
    model = nbody_ics.plummer(n, 51)
    sim = _sim(model, order)
    sim.init()
    h0 = sim.to_numpy()
    ocfg = _ocfg(sim)
    os0 = _ostate(h0, order)
    nxt = h0["t_tick"] + (1 << (TICK_BITS - h0["level"].astype(np.int64)))
    T = int(nxt.min())
    act = np.nonzero(nxt == T)[0].astype(np.int32)
    xp, vp, ap, jp = oracle.predict(ocfg, os0, T)
    F = oracle.force(ocfg, os0.m, xp, vp, ap if order >= 6 else None, jp if order >= 8 else None, act=act)
    dev = sim.device
    f = {k: torch.as_tensor(np.ascontiguousarray(F[k]), device=dev) for k in ("acc", "jrk", "snp", "crk")}
    sim.correct(torch.as_tensor(act, device=dev), T, f)
    got = sim.to_numpy()
    assert np.all(got["t_tick"][act] == T)
    compare_corrected(got, oracle_correct(ocfg, os0, act, T, F), act, order, 0.0, "correct", sim.dt_rule)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("order", [4, 6, 8])
def test_step_parity(order, precision):
    """Whole block steps, each from the GPU's own previous state: identical
    time and active set (integer work), corrected state within the bound set
    by the force difference of the precision mode."""
    model = nbody_ics.with_bh_binary(nbody_ics.plummer(1022, 61))
    sim = _sim(model, order, precision=precision, n_hard=2)
    sim.init()
    ocfg = _ocfg(sim)
    rel_force = 1e-11 if precision == "fp64" else 3e-5
    for step in range(10):
        h0 = sim.to_numpy()
        os0 = _ostate(h0, order)
        nxt = h0["t_tick"] + (1 << (TICK_BITS - h0["level"].astype(np.int64)))
        T = int(nxt.min())
        act = np.nonzero(nxt == T)[0].astype(np.int32)
        t_g, na_g = sim.step()
        assert (t_g, na_g) == (T, act.size), step
        xp, vp, ap, jp = oracle.predict(ocfg, os0, T)
        F = oracle.force(ocfg, os0.m, xp, vp, ap if order >= 6 else None, jp if order >= 8 else None, act=act)
        got = sim.to_numpy()
        assert np.all(got["t_tick"][act] == T)
        if precision == "fp64":
            compare_corrected(got, oracle_correct(ocfg, os0, act, T, F), act, order, rel_force, "step", sim.dt_rule)
        else:
            # MIXED: the corrected state differs by the force error times h
            want = oracle_correct(ocfg, os0, act, T, F)
            st = err_stats(rel_err(got["v"][:, act] - os0.v[:, act], want[1][:, act] - os0.v[:, act]))
            say("step order %d mixed dv rms %.2e max %.2e" % (order, st["rms"], st["max"]))
            assert st["rms"] <= 2e-5


def test_energy_parity():
    model = nbody_ics.with_bh_binary(nbody_ics.king(4094, 7.0, 71))
    sim = _sim(model, 4, n_hard=2)
    T, W = sim.energy()
    To, Wo = oracle.energy(_ocfg(sim), model.m, model.x, model.v)
    say("energy T %.16e / %.16e  W %.16e / %.16e" % (T, To, W, Wo))
    assert abs(T - To) <= 1e-13 * abs(To)
    assert abs(W - Wo) <= 1e-12 * abs(Wo)


def test_c1_integration_vs_oracle():
    """The small parity workload: Plummer n=1024, 4th order, eta=0.01,
    eps=1e-4, FP64, t = 0 -> 0.125: same block-step sequence at the start,
    energy drift within twice the oracle's, positions close at the end."""
    model = nbody_ics.plummer(1024, 11)
    sim = _sim(model, 4, eta=0.01)
    sim.init()
    E0 = sum(sim.energy())
    os_ = _ostate(sim.to_numpy(), 4)
    ocfg = _ocfg(sim)
    Eo0 = sum(oracle.energy(ocfg, os_.m, os_.x, os_.v))
    t_end = TICKS // 8
    steps = sim.integrate(t_end)
    st = oracle.integrate(ocfg, os_, t_end)
    E1 = sum(sim.energy())
    Eo1 = sum(oracle.energy(ocfg, os_.m, os_.x, os_.v))
    dg, do = abs((E1 - E0) / E0), abs((Eo1 - Eo0) / Eo0)
    got = sim.to_numpy()
    dx = err_stats(np.linalg.norm(got["x"] - os_.x, axis=0))
    say("C1: steps gpu %d oracle %d; |dE/E| gpu %.3e oracle %.3e; |dx| rms %.2e max %.2e; level diffs %d"
        % (steps, st["steps"], dg, do, dx["rms"], dx["max"], int(np.sum(got["level"] != os_.level))))
    assert np.all(got["t_tick"] == t_end)
    assert dg <= 2.0 * do + 1e-12
    assert abs(steps - st["steps"]) <= 0.02 * st["steps"]
    assert dx["rms"] < 1e-8


@pytest.mark.parametrize("order", [6, 8])
def test_mixed_energy_drift_matches_oracle(order):
    """Plummer n=8192, eta=0.1, to t = 1/8 with the default time-step rule of
    each precision: |dE/E| of the MIXED force within twice the oracle's drift
    under the same rule; no particle stuck at the smallest step; FP64 (its own
    rule) against the oracle likewise."""
    model = nbody_ics.plummer(8192, 12)
    t_end = TICKS // 8
    for prec in ("mixed", "fp64"):
        sim = _sim(model, order, precision=prec, eta=0.1)
        sim.init()
        E0 = sum(sim.energy())
        steps = sim.integrate(t_end)
        E1 = sum(sim.energy())
        dg = abs((E1 - E0) / E0)
        got = sim.to_numpy()
        ocfg = _ocfg(sim)
        os_ = oracle.State(model.m, model.x, model.v, order)
        oracle.init(ocfg, os_)
        Eo0 = sum(oracle.energy(ocfg, os_.m, os_.x, os_.v))
        st = oracle.integrate(ocfg, os_, t_end)
        Eo1 = sum(oracle.energy(ocfg, os_.m, os_.x, os_.v))
        do = abs((Eo1 - Eo0) / Eo0)
        say("order %d %s (rule %d): %d steps (oracle %d), |dE/E| %.3e (oracle %.3e), level-20 particles %d, "
            "dt underflows %d" % (order, prec, sim.dt_rule, steps, st["steps"], dg, do,
                                  int(np.sum(got["level"] == 20)), sim.stats().dt_underflow))
        assert np.all(got["t_tick"] == t_end)
        assert sim.stats().dt_underflow == 0
        assert steps <= 1.5 * st["steps"]
        assert dg <= 2.0 * do + (1e-13 if prec == "fp64" else 1e-10)


def test_nonfinite_is_reported():
    from paper_1312_1789_amd import abi
    model = nbody_ics.plummer(512, 81)
    sim = _sim(model, 4)
    sim.init()
    h = sim.to_numpy()
    h["x"][0, 5] = np.nan
    sim.load_state(h["x"], h["v"], h["d"], h["t_tick"], h["level"])
    with pytest.raises(abi.NBodyError) as e:
        for _ in range(200):
            sim.step()
    assert e.value.status == abi.NBODY_E_NONFINITE


def test_run_equals_single_steps():
    """nbody_run to t_end takes exactly the steps nbody_step takes one by one
    (the same kernels and launch shapes: identical bits) and stops before the
    first block time past t_end."""
    model = nbody_ics.plummer(700, 91)
    a = _sim(model, 6, precision="mixed", eta=0.1)
    b = _sim(model, 6, precision="mixed", eta=0.1)
    a.init()
    b.init()
    t_end = TICKS // 64 + 3 * (TICKS >> 16)
    steps_a, t_a = a.run(t_end)
    steps_b, t_b = 0, 0
    while True:
        h = b.to_numpy()
        nxt = int((h["t_tick"] + (1 << (TICK_BITS - h["level"].astype(np.int64)))).min())
        if nxt > t_end:
            break
        t_b, _ = b.step()
        steps_b += 1
    say("run: %d steps to tick %d; single steps %d to tick %d" % (steps_a, t_a, steps_b, t_b))
    assert (steps_a, t_a) == (steps_b, t_b) and steps_a > 10
    ha, hb = a.to_numpy(), b.to_numpy()
    for key in ("x", "v", "t_tick", "level"):
        np.testing.assert_array_equal(ha[key], hb[key])
    assert a.stats().steps == b.stats().steps
    assert a.run(t_end) == (0, 0)


def test_run_reports_nonfinite():
    from paper_1312_1789_amd import abi
    model = nbody_ics.plummer(512, 92)
    sim = _sim(model, 4)
    sim.init()
    h = sim.to_numpy()
    h["v"][1, 7] = np.inf
    sim.load_state(h["x"], h["v"], h["d"], h["t_tick"], h["level"])
    with pytest.raises(abi.NBodyError) as e:
        sim.run(TICKS)
    assert e.value.status == abi.NBODY_E_NONFINITE


def test_c2_size_integration_vs_oracle():
    """C2 at its size: Plummer n = 131072 (seed 12), 6th order, eta = 0.1, the
    order-4 form of the time-step criterion (MIXED's default), t = 0 -> 1/1024
    with the largest step 1/1024 (k_min = 10) so that every particle is
    synchronised there (the oracle's two initial force passes over n^2
    pairs dominate its time).  One oracle run against the GPU in FP64 (the
    same step count to within 1, final positions to 1e-10, |dE/E| within
    twice the oracle's plus 1e-13) and in MIXED (step counts within 5% + 2,
    |dE/E| within twice the oracle's plus 1e-10 for the FP32 force terms).
    Over so short a span the drift is at the rounding level (~1e-14 to
    1e-13): this checks integration parity at size, not the drift of a
    whole time unit (shown against the oracle at n = 8192 over 1/8)."""
    model = nbody_ics.plummer(131072, 12)
    t_end = TICKS // 1024
    ocfg = None
    runs = {}
    from paper_1312_1789_amd import Simulation
    for prec in ("fp64", "mixed"):
        sim = Simulation(model.m, model.x, model.v, order=6, precision=prec, eps2=1e-8, eta=0.1, eta_start=0.01,
                         k_min=10, k_max=20, dt_rule=2)
        sim.init()
        E0 = sum(sim.energy())
        steps = sim.integrate(t_end)
        E1 = sum(sim.energy())
        runs[prec] = (steps, abs((E1 - E0) / E0), sim.to_numpy(), sim.stats().dt_underflow)
        say("C2 size, GPU %s (rule %d): %d steps, |dE/E| %.3e" % (prec, sim.dt_rule, steps, runs[prec][1]))
        ocfg = _ocfg(sim)
        sim.close()
    os_ = oracle.State(model.m, model.x, model.v, 6)
    oracle.init(ocfg, os_)
    Eo0 = sum(oracle.energy(ocfg, os_.m, os_.x, os_.v))
    st = oracle.integrate(ocfg, os_, t_end)
    Eo1 = sum(oracle.energy(ocfg, os_.m, os_.x, os_.v))
    do = abs((Eo1 - Eo0) / Eo0)
    say("C2 size: oracle %d steps, |dE/E| %.3e" % (st["steps"], do))
    for prec, (steps, dg, got, underflow) in runs.items():
        assert np.all(got["t_tick"] == t_end) and underflow == 0
        if prec == "fp64":
            assert abs(steps - st["steps"]) <= 1
            dx = err_stats(rel_err(got["x"], os_.x))
            say("C2 size fp64 final x vs oracle: rms %.2e max %.2e" % (dx["rms"], dx["max"]))
            assert dx["max"] <= 1e-10
            assert dg <= 2.0 * do + 1e-13
        else:
            assert abs(steps - st["steps"]) <= 0.05 * st["steps"] + 2
            assert dg <= 2.0 * do + 1e-10
