"""GPU tests of the predictor folded into the wave j-split force kernel
(nbody_predict_force, nbody_set_fusion).

* The fused call equals, bit for bit, the predictor kernel followed by the
  force kernel (same arithmetic, same j order and FP32 chunk boundaries), on
  a random valid block state (every particle at its own time, with its own
  level), for every order and precision, active sets that take every row
  count of the kernel (1, 4 and 16 rows per workgroup, one and two i-tiles),
  one split and several, with the unsoftened black-hole pair.
* The fused forces match the oracle's (its predictor, then its force) within
  the force tolerances.
* Whole integrations with fusion on and off end in identical states.
"""
import numpy as np
import pytest
import torch

import nbody_ics
import oracle
from helpers import TICK_BITS, TICKS, cluster_with_bh, err_stats, oracle_force, physical_derivs, random_block_state, rel_err, say
from oracle import OracleConfig

pytestmark = pytest.mark.gpu

KEYS = {4: ["acc", "jrk"], 6: ["acc", "jrk", "snp"], 8: ["acc", "jrk", "snp", "crk"]}
FP64_TOL = {"rms": 1e-12, "max": 1e-9}
LOW_TOL = {"acc": 2e-6, "jrk": 2e-5, "snp": 2e-4, "crk": 2e-3, "pot": 1e-6}


@pytest.fixture(scope="module")
def block_case():
    """King W0=7 cluster of 2998 stars + BH binary (n = 3000, n_hard = 2),
    physical acceleration and jerk, smaller random higher derivatives, and a
    random block state: particle times multiples of their own steps, levels
    3..20, predicted to the next block time T."""
    model = cluster_with_bh(2998, 71)
    eps2, n_hard = 1e-8, 2
    a, j = physical_derivs(model.m, model.x, model.v, eps2, n_hard)
    rng = np.random.default_rng(72)
    d = [a, j] + [rng.normal(size=(3, model.n)) * 10.0 ** (k + 2) for k in range(4)]
    t, lv = random_block_state(model.n, 73)
    T = int((t + (1 << (TICK_BITS - lv.astype(np.int64)))).min())
    return model, eps2, n_hard, d, t, lv, T


def _sim(case, order, precision):
    from paper_1312_1789_amd import Simulation
    model, eps2, n_hard, d, t, lv, T = case
    sim = Simulation(model.m, model.x, model.v, order=order, precision=precision, eps2=eps2, n_hard=n_hard)
    sim.load_state(model.x, model.v, d[: order - 2], t, lv)
    return sim


def _sets(n):
    return [np.array([0], np.int32), np.array([1, 0], np.int32), np.array([n - 1], np.int32),
            nbody_ics.active_subset(n, 3, 741), nbody_ics.active_subset(n, 4, 742),
            nbody_ics.active_subset(n, 7, 743), nbody_ics.active_subset(n, 16, 744),
            nbody_ics.active_subset(n, 17, 745), nbody_ics.active_subset(n, 32, 746)]


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
@pytest.mark.parametrize("order", [4, 6, 8])
def test_fused_equals_predict_then_force(block_case, order, precision):
    model, eps2, n_hard, d, t, lv, T = block_case
    n = model.n
    sim = _sim(block_case, order, precision)
    for with_pot in (True, False):          # the kernels without the potential are the ones steps use
        keys = KEYS[order] + (["pot"] if with_pot else [])
        for n_split in (0, 1, 7):
            sim.set_launch(1, 64, n_split, 3)
            for act_np in _sets(n):
                act = torch.as_tensor(act_np, device=sim.device)
                sim.set_fusion(True)
                fused = {k: v.clone() for k, v in sim.predict_force(T, act, with_pot=with_pot).items()}
                with pytest.raises(Exception):
                    sim.predicted()            # the fused call wrote no records
                sim.set_fusion(False)
                plain = sim.predict_force(T, act, with_pot=with_pot)
                for k in keys:
                    g = fused[k][..., : act_np.size].cpu().numpy()
                    w = plain[k][..., : act_np.size].cpu().numpy()
                    assert np.array_equal(g, w), (with_pot, n_split, act_np.size, k, float(np.max(np.abs(g - w))))
    say("fused == predict + force: order %d %s, %d sets x 3 splits, with and without the potential"
        % (order, precision, len(_sets(n))))
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
@pytest.mark.parametrize("order", [4, 6, 8])
def test_fused_force_parity(block_case, order, precision):
    """Fused forces against the oracle's predictor and force, errors pooled
    over the active sets."""
    model, eps2, n_hard, d, t, lv, T = block_case
    n = model.n
    sim = _sim(block_case, order, precision)
    ocfg = OracleConfig(order=order, eps2=eps2, n_hard=n_hard)
    os_ = oracle.State(model.m, model.x, model.v, order, [a.copy() for a in d[: order - 2]], t.copy(), lv.copy())
    xp, vp, ap, jp = oracle.predict(ocfg, os_, T)
    errs = {k: [] for k in KEYS[order] + ["pot"]}
    for act_np in _sets(n):
        out = sim.predict_force(T, torch.as_tensor(act_np, device=sim.device))
        ref = oracle_force(order, eps2, n_hard, model.m, xp, vp, ap, jp, act=act_np)
        for k in errs:
            errs[k].append(rel_err(out[k].cpu().numpy()[..., : act_np.size], ref[k]))
    for k, e in errs.items():
        st = err_stats(np.concatenate(e))
        say("   fused %s p%d %-4s rms %.2e max %.2e" % (precision, order, k, st["rms"], st["max"]))
        if precision == "fp64":
            assert st["rms"] <= FP64_TOL["rms"] and st["max"] <= FP64_TOL["max"], (k, st)
        else:
            assert st["rms"] <= LOW_TOL[k] and st["max"] <= 10 * LOW_TOL[k], (k, st)
    sim.close()


@pytest.mark.parametrize("order,precision", [(4, "fp64"), (6, "mixed"), (8, "ds"), (6, "fp64"), (8, "mixed")])
def test_integration_with_and_without_fusion(order, precision):
    """Block steps from t = 0 of a Plummer model with a black-hole binary:
    the states after 400 steps with fusion on and off are bitwise equal, and
    some of the steps had active sets small enough for the fused kernel."""
    from paper_1312_1789_amd import Simulation
    model = nbody_ics.with_bh_binary(nbody_ics.plummer(4094, 75))
    finals, sizes = [], []
    for fuse in (True, False):
        sim = Simulation(model.m, model.x, model.v, order=order, precision=precision, eps2=1e-8, n_hard=2,
                         eta=0.01 if order == 4 else 0.1)
        sim.set_fusion(fuse)
        sim.init()
        acts = []
        for _ in range(400):
            _, na = sim.step()
            acts.append(na)
        finals.append(sim.to_numpy())
        sizes.append(acts)
        sim.close()
    assert sizes[0] == sizes[1]
    small = sum(1 for a in sizes[0] if a <= 32)
    say("order %d %s: %d of 400 steps with n_act <= 32" % (order, precision, small))
    assert small > 0
    for k in ("x", "v", "t_tick", "level"):
        assert np.array_equal(finals[0][k], finals[1][k]), k
    for a, b in zip(finals[0]["d"], finals[1]["d"]):
        assert np.array_equal(a, b)


def test_fused_records_and_validation(block_case):
    """After a fused call the force call on records and the record readout ask
    for a new prediction; after nbody_predict they work again.  Fusion flag
    values other than 0 and 1 are rejected."""
    from paper_1312_1789_amd import abi
    model, eps2, n_hard, d, t, lv, T = block_case
    sim = _sim(block_case, 6, "mixed")
    act = torch.as_tensor(np.array([5, 9], np.int32), device=sim.device)
    sim.predict_force(T, act)
    with pytest.raises(abi.NBodyError) as e:
        sim.force_block(act)
    assert e.value.status == abi.NBODY_E_STATE
    sim.predict(T)
    out = sim.force_block(act)
    assert torch.isfinite(out["acc"]).all()
    with pytest.raises(abi.NBodyError) as e:
        abi.nbody_set_fusion(sim.ctx, 2)
    assert e.value.status == abi.NBODY_E_INVALID
    # an empty active set predicts (records written) and computes nothing
    sim.set_fusion(True)
    sim.predict_force(T, torch.zeros(0, dtype=torch.int32, device=sim.device))
    assert sim.predicted()["xp"].shape == (3, model.n)
    sim.close()
