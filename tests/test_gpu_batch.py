"""GPU parity of the batched form (many independent clusters per launch
sequence) against the CPU oracle run on each cluster separately.

Integer work (each cluster's next time and active set) must match exactly;
forces and corrected states follow the tolerances of the single-system tests:
FP64 relative error rms <= 1e-12, max <= 1e-9; MIXED / DS forces rms <= 2e-6
(acceleration), 2e-5 (jerk), 2e-4 (snap), 2e-3 (crackle).  The cluster mix
spans several scheduling blocks (2500 and 1030 particles), ragged i-tiles
(257, 700), a single partial tile (64) and a two-body cluster, with the
first two particles of every cluster unsoftened (n_hard = 2).
"""
import numpy as np
import pytest
import torch

import nbody_ics
import oracle
from helpers import TICK_BITS, TICKS, compare_corrected, err_stats, oracle_correct, rel_err, say
from oracle import OracleConfig

pytestmark = pytest.mark.gpu

LOW_TOL = {"acc": 2e-6, "jrk": 2e-5, "snp": 2e-4, "crk": 2e-3}
KEYS = ["acc", "jrk", "snp", "crk"]


def _clusters(seed=900):
    return [nbody_ics.with_bh_binary(nbody_ics.king(2498, 7.0, seed)),
            nbody_ics.plummer(700, seed + 1),
            nbody_ics.plummer(257, seed + 2),
            nbody_ics.kepler_pair(0.3),
            nbody_ics.plummer(1030, seed + 3),
            nbody_ics.plummer(64, seed + 4)]


def _batch(models, order, precision="fp64", eps2=1e-8, n_hard=2, eta=None, k_min=3, k_max=20):
    from paper_1312_1789_amd import Batch
    eta = eta if eta is not None else (0.01 if order == 4 else 0.1)
    return Batch([(m.m, m.x, m.v) for m in models], order=order, precision=precision, eps2=eps2, n_hard=n_hard,
                 eta=eta, eta_start=0.01, k_min=k_min, k_max=k_max)


def _ocfg(B):
    c = B.cfg
    return OracleConfig(order=c.order, eps2=c.eps2, n_hard=c.n_hard, eta=c.eta, eta_start=c.eta_start,
                        k_min=c.k_min, k_max=c.k_max, dt_rule=B.dt_rule)


def _ostate(hc, order):
    return oracle.State(hc["m"], hc["x"], hc["v"], order, [a.copy() for a in hc["d"]], hc["t_tick"].copy(),
                        hc["level"].copy())


def _next(hc):
    nxt = hc["t_tick"] + (1 << (TICK_BITS - hc["level"].astype(np.int64)))
    T = int(nxt.min())
    return T, np.nonzero(nxt == T)[0].astype(np.int32)


@pytest.mark.parametrize("order", [4, 6, 8])
def test_batch_init_parity(order):
    models = _clusters()
    B = _batch(models, order)
    B.init()
    h = B.to_numpy()
    ocfg = _ocfg(B)
    errs = {k: [] for k in range(order - 2)}
    lv_diff = 0
    for c, mdl in enumerate(models):
        hc = B.cluster(h, c)
        os_ = oracle.State(mdl.m, mdl.x, mdl.v, order)
        oracle.init(ocfg, os_)
        for k in range(order - 2):
            if order == 8 and k >= 4:
                assert np.all(hc["d"][k] == 0.0)
                continue
            errs[k].append(rel_err(hc["d"][k], os_.d[k]))
        assert np.all(hc["t_tick"] == 0)
        lv_diff += int(np.sum(hc["level"] != os_.level))
    for k, e in errs.items():
        if not e:
            continue
        st = err_stats(np.concatenate(e))
        say("batch init order %d d[%d] rms %.2e max %.2e" % (order, k, st["rms"], st["max"]))
        assert st["rms"] <= 1e-12 and st["max"] <= 1e-9
    assert lv_diff <= 2


def _force_errors(B, models, h0, aoff, act, f, ocfg, order, errs):
    """Check the active sets exactly; collect per-particle force errors."""
    for c in range(B.nc):
        hc = B.cluster(h0, c)
        T, want = _next(hc)
        got = act[aoff[c]:aoff[c + 1]] - B.off[c]
        np.testing.assert_array_equal(got, want)
        os0 = _ostate(hc, order)
        xp, vp, ap, jp = oracle.predict(ocfg, os0, T)
        F = oracle.force(ocfg, os0.m, xp, vp, ap if order >= 6 else None, jp if order >= 8 else None, act=want,
                         with_pot=False)
        for k, key in enumerate(KEYS[: order // 2]):
            errs[key].append(rel_err(f[k][:, aoff[c]:aoff[c + 1]], F[key]))


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
@pytest.mark.parametrize("order", [4, 6, 8])
def test_batch_force_all_active(order, precision):
    """Every particle on one level (k_min = k_max): each batched step
    evaluates all particles of all clusters."""
    models = _clusters(910)
    B = _batch(models, order, precision, k_min=7, k_max=7)
    B.init()
    ocfg = _ocfg(B)
    errs = {k: [] for k in KEYS}
    for step in range(2):
        h0 = B.to_numpy()
        B.step(1)
        aoff, act, f = B.last_step()
        assert aoff[-1] == B.n
        _force_errors(B, models, h0, aoff, act.cpu().numpy(), f.cpu().numpy(), ocfg, order, errs)
    for key in KEYS[: order // 2]:
        st = err_stats(np.concatenate(errs[key]))
        say("batch force all-active order %d %s %s rms %.2e max %.2e" % (order, precision, key, st["rms"], st["max"]))
        if precision == "fp64":
            assert st["rms"] <= 1e-12 and st["max"] <= 1e-9, (key, st)
        else:
            assert st["rms"] <= LOW_TOL[key] and st["max"] <= 10 * LOW_TOL[key], (key, st)


@pytest.mark.parametrize("shape,precision", [((64, 4), "fp64"), ((256, 4), "fp64"), ((64, 16), "fp64"),
                                             ((256, 1), "fp64"), ((64, 1), "fp64"), ((128, 4), "fp64"),
                                             ((64, 32), "fp64"), ((64, 4), "mixed"), ((128, 32), "mixed")])
@pytest.mark.parametrize("order", [4, 6, 8])
def test_batch_force_block_steps(order, shape, precision):
    """Individual block steps: every cluster at its own time with its own
    (small) active set, j-ranges split into items of equal cost; i-tiles of
    64, 128 and 256 rows (a tile's last active rows spread over lane groups
    of 2 to 64 lanes), 1 to 32 work items aimed for per workgroup."""
    models = _clusters(920)
    B = _batch(models, order, precision)
    B.set_launch(0, shape[1], shape[0])
    assert B.get_launch()[1:] == (shape[1], shape[0])
    B.init()
    ocfg = _ocfg(B)
    errs = {k: [] for k in KEYS}
    n_rows = 0
    for step in range(6):
        h0 = B.to_numpy()
        B.step(1)
        aoff, act, f = B.last_step()
        n_rows += aoff[-1]
        _force_errors(B, models, h0, aoff, act.cpu().numpy(), f.cpu().numpy(), ocfg, order, errs)
    say("batch block steps order %d: %d active rows in 6 steps" % (order, n_rows))
    for key in KEYS[: order // 2]:
        st = err_stats(np.concatenate(errs[key]))
        say("batch force blocks order %d %s %s rms %.2e max %.2e" % (order, precision, key, st["rms"], st["max"]))
        if precision == "fp64":
            assert st["rms"] <= 1e-12 and st["max"] <= 1e-9, (key, st)
        else:
            assert st["rms"] <= LOW_TOL[key] and st["max"] <= 10 * LOW_TOL[key], (key, st)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("order", [4, 6, 8])
def test_batch_step_parity(order, precision):
    """Whole batched steps, each from the GPU's own previous state, checked
    cluster by cluster against the oracle's corrector on the same forces."""
    models = _clusters(930)
    B = _batch(models, order, precision)
    B.init()
    ocfg = _ocfg(B)
    rel_force = 1e-11 if precision == "fp64" else 3e-5
    for step in range(6):
        h0 = B.to_numpy()
        B.step(1)
        got_all = B.to_numpy()
        for c in range(B.nc):
            hc = B.cluster(h0, c)
            T, act = _next(hc)
            os0 = _ostate(hc, order)
            xp, vp, ap, jp = oracle.predict(ocfg, os0, T)
            F = oracle.force(ocfg, os0.m, xp, vp, ap if order >= 6 else None, jp if order >= 8 else None, act=act)
            got = B.cluster(got_all, c)
            assert np.all(got["t_tick"][act] == T), (step, c)
            rest = np.setdiff1d(np.arange(hc["m"].size), act)
            assert np.all(got["t_tick"][rest] == hc["t_tick"][rest])
            want = oracle_correct(ocfg, os0, act, T, F)
            if precision == "fp64":
                compare_corrected(got, want, act, order, rel_force, "batch step c%d" % c, B.dt_rule)
            else:
                st = err_stats(rel_err(got["v"][:, act] - os0.v[:, act], want[1][:, act] - os0.v[:, act]))
                assert st["rms"] <= 2e-5, (step, c, st)
    s = B.stats()
    assert s.steps == 6 and s.nonfinite == 0


def test_batch_graph_replay_matches_eager():
    """A captured batched step replayed k times gives the same state, bit for
    bit, as k eager steps (the persistent kernel's work items are independent
    of which workgroup takes them; split partials are summed in fixed order).
    Every replay is checked, with eager work and synchronisation between."""
    models = _clusters(940)
    A = _batch(models, 6, "mixed")
    G = _batch(models, 6, "mixed")
    A.init()
    G.init()
    G.capture()
    for r in range(5):
        A.step(1)
        G.replay(1)
        ha, hg = A.to_numpy(), G.to_numpy()
        for key in ("x", "v", "t_tick", "level"):
            np.testing.assert_array_equal(ha[key], hg[key], err_msg="replay %d %s" % (r, key))
        for k in range(4):
            np.testing.assert_array_equal(ha["d"][k], hg["d"][k], err_msg="replay %d d[%d]" % (r, k))
        torch.cuda.synchronize()
    G.replay(7)
    A.step(7)
    ha, hg = A.to_numpy(), G.to_numpy()
    np.testing.assert_array_equal(ha["x"], hg["x"])
    np.testing.assert_array_equal(ha["t_tick"], hg["t_tick"])
    assert A.stats().steps == G.stats().steps == 12


def test_batch_energy_parity():
    models = _clusters(950)
    B = _batch(models, 4)
    T, W = B.energy()
    ocfg = _ocfg(B)
    for c, mdl in enumerate(models):
        To, Wo = oracle.energy(ocfg, mdl.m, mdl.x, mdl.v)
        assert abs(T[c] - To) <= 1e-13 * abs(To), c
        assert abs(W[c] - Wo) <= 1e-12 * abs(Wo), c


def test_batch_integrate_to_end_vs_oracle():
    """4th order, FP64, three Plummer clusters to t_end = 1/32 (k_min = 5, so
    every particle lands on t_end): replay until every cluster rests, then
    per-cluster energy drift within twice the oracle's."""
    models = [nbody_ics.plummer(256, 960), nbody_ics.plummer(512, 961), nbody_ics.plummer(300, 962)]
    B = _batch(models, 4, "fp64", eta=0.01, k_min=5, n_hard=0)
    B.init()
    E0 = [t + w for t, w in zip(*B.energy())]
    t_end = TICKS // 32
    B.set_end(t_end)
    B.capture()
    replays = 0
    while True:
        B.replay(32)
        replays += 32
        live, tcur = B.poll()
        if live == 0:
            break
        assert replays < 20000
    E1 = [t + w for t, w in zip(*B.energy())]
    h = B.to_numpy()
    assert np.all(h["t_tick"] == t_end)
    assert tcur == [t_end] * 3
    ocfg = _ocfg(B)
    for c, mdl in enumerate(models):
        os_ = oracle.State(mdl.m, mdl.x, mdl.v, 4)
        oracle.init(ocfg, os_)
        Eo0 = sum(oracle.energy(ocfg, os_.m, os_.x, os_.v))
        oracle.integrate(ocfg, os_, t_end)
        Eo1 = sum(oracle.energy(ocfg, os_.m, os_.x, os_.v))
        dg, do = abs((E1[c] - E0[c]) / E0[c]), abs((Eo1 - Eo0) / Eo0)
        say("batch cluster %d |dE/E| gpu %.3e oracle %.3e" % (c, dg, do))
        assert dg <= 2.0 * do + 1e-12


def test_batch_unsoftened_pairs():
    """eps2 = 0: every pair unsoftened (two Kepler pairs and a small cluster),
    order 8, FP64 initial derivatives against the oracle."""
    models = [nbody_ics.kepler_pair(0.5), nbody_ics.kepler_pair(0.1, 2.0), nbody_ics.plummer(40, 970)]
    B = _batch(models, 8, "fp64", eps2=0.0, n_hard=0)
    B.init()
    h = B.to_numpy()
    ocfg = _ocfg(B)
    for c, mdl in enumerate(models):
        hc = B.cluster(h, c)
        os_ = oracle.State(mdl.m, mdl.x, mdl.v, 8)
        oracle.init(ocfg, os_)
        for k in range(4):
            st = err_stats(rel_err(hc["d"][k], os_.d[k]))
            assert st["max"] <= 1e-9, (c, k, st)


def test_batch_autotune_keeps_parity():
    """The autotuner times every shape on the same step, takes that step and
    leaves a valid shape; the next steps still match the oracle."""
    models = _clusters(980)
    B = _batch(models, 6, "mixed")
    B.init()
    B.autotune(1)
    grid, per_wg, itile = B.get_launch()
    say("autotuned batch shape: grid %d items per workgroup %d i_tile %d" % (grid, per_wg, itile))
    assert grid > 0 and per_wg in (2, 4, 8, 16, 32) and itile in (64, 128, 256)
    assert B.stats().steps == 1   # one real step, after the shapes were timed on it
    ocfg = _ocfg(B)
    errs = {k: [] for k in KEYS}
    for step in range(3):
        h0 = B.to_numpy()
        B.step(1)
        aoff, act, f = B.last_step()
        _force_errors(B, models, h0, aoff, act.cpu().numpy(), f.cpu().numpy(), ocfg, 6, errs)
    for key in KEYS[:3]:
        st = err_stats(np.concatenate(errs[key]))
        say("after autotune %s rms %.2e max %.2e" % (key, st["rms"], st["max"]))
        assert st["max"] <= 50 * LOW_TOL[key]


def test_batch_autotune_takes_plain_steps():
    """The shapes the autotuner times leave no trace: after autotune(k) the
    state equals, bit for bit, that of k plain batched steps with the shape
    in use before the call (the timed force phases overwrite only scratch;
    the counters, cluster times and live count the planning writes are put
    back)."""
    models = _clusters(990)
    A = _batch(models, 6, "mixed")
    A.init()
    A.autotune(2)
    B = _batch(models, 6, "mixed")
    B.init()
    B.step(2)
    ha, hb = A.to_numpy(), B.to_numpy()
    for k in ("x", "v", "t_tick", "level"):
        np.testing.assert_array_equal(ha[k], hb[k])
    for da, db in zip(ha["d"], hb["d"]):
        np.testing.assert_array_equal(da, db)
    sa, sb = A.stats(), B.stats()
    assert (sa.steps, sa.sum_n_act, sa.interactions) == (sb.steps, sb.sum_n_act, sb.interactions)
    la, lb = A.poll(), B.poll()
    assert la[0] == lb[0] and list(la[1]) == list(lb[1])
    A.close()
    B.close()


def test_batch_c4_scale():
    """The batched workload at its configured scale: 256 Plummer clusters,
    N_c = round(2^U(10, 16)) (seed 1400, n = 4.25M), 6th order, MIXED, one
    batched step per captured-graph replay.  First step from the initial
    state: every cluster's next time and active set exactly.  Second, every
    particle on the largest step, so that the step evaluates sum N_c^2 ~
    1.3e11 pair interactions (the plan's item cap and its partial-sum bound
    are reached).  Forces of sampled active rows of the largest, the median
    and the smallest cluster against the oracle, in both steps."""
    models = nbody_ics.batched_plummer(256, 1400)
    sizes = np.array([m.n for m in models])
    say("C4 scale: %d clusters, n %d (min %d, max %d)" % (len(models), sizes.sum(), sizes.min(), sizes.max()))
    B = _batch(models, 6, "mixed", n_hard=0)
    B.init()
    ocfg = _ocfg(B)
    order_ = np.argsort(sizes, kind="stable")
    picks = [int(order_[-1]), int(order_[len(order_) // 2]), int(order_[0])]
    h_init = B.to_numpy()
    for label in ("initial levels", "all active"):
        if label == "all active":
            h = dict(h_init)
            h["level"] = np.full(B.n, 3, np.int32)
            B.load_state(h)
        h0 = B.to_numpy()
        B.capture()
        B.replay(1)
        B.synchronize()
        aoff, act, f = B.last_step()
        act = act.cpu().numpy()
        f = f.cpu().numpy()
        say("C4 step (%s): %d active rows in all" % (label, aoff[-1]))
        for c in range(B.nc):
            _, want = _next(B.cluster(h0, c))
            np.testing.assert_array_equal(act[aoff[c]:aoff[c + 1]] - B.off[c], want)
        if label == "all active":
            assert aoff[-1] == B.n
        errs = {k: [] for k in KEYS[:3]}
        for c in picks:
            hc = B.cluster(h0, c)
            T, want = _next(hc)
            rows = np.arange(want.size) if want.size <= 64 else \
                np.sort(np.random.default_rng(c).choice(want.size, 64, replace=False))
            os0 = _ostate(hc, 6)
            xp, vp, ap, _ = oracle.predict(ocfg, os0, T)
            F = oracle.force(ocfg, os0.m, xp, vp, ap, None, act=want[rows], with_pot=False)
            for k, key in enumerate(KEYS[:3]):
                errs[key].append(rel_err(f[k][:, aoff[c] + rows], F[key]))
            say("  cluster %d (N_c %d): %d active, %d checked" % (c, sizes[c], want.size, rows.size))
        for key in KEYS[:3]:
            st = err_stats(np.concatenate(errs[key]))
            say("  C4 %s %s rms %.2e max %.2e" % (label, key, st["rms"], st["max"]))
            assert st["rms"] <= LOW_TOL[key] and st["max"] <= 10 * LOW_TOL[key], (key, st)
    B.close()
