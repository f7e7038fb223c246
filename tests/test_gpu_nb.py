"""GPU parity of the neighbour-split force (nbody_force_block_nb) against the
oracle's (oracle.force_nb) on identical inputs.

Neighbour radii sit in the middle of gaps of each particle's sorted squared
distances, at least 1e-4 (relative) from every pair, so the neighbour sets
are the same in FP64 and in the FP32 distance of MIXED mode: counts and lists
must match exactly (integer results).  Forces: FP64 relative error per row
rms <= 1e-12, max <= 1e-9; MIXED rms <= 2e-6 (acceleration) and 2e-5 (jerk),
the tolerances of the full force, and max <= 10x those (as for the full
force).
"""
import numpy as np
import pytest
import torch

import nbody_ics
import oracle
from helpers import TICKS, band_free_radii, cluster_with_bh, err_stats, rel_err, say
from oracle import OracleConfig

pytestmark = pytest.mark.gpu

FP64_TOL = {"rms": 1e-12, "max": 1e-9}
LOW_TOL = {"acc": 2e-6, "jrk": 2e-5}
PARTS = ("acc_irr", "jrk_irr", "acc_reg", "jrk_reg")


def _sim(model, precision, eps2, n_hard, order=4):
    from paper_1312_1789_amd import Simulation
    sim = Simulation(model.m, model.x, model.v, order=order, precision=precision, eps2=eps2, n_hard=n_hard)
    n = model.n
    t0 = 5 * (TICKS >> 3)
    d = [np.zeros((3, n))] * (order - 2)
    sim.load_state(model.x, model.v, d, np.full(n, t0, np.int64), np.full(n, 3, np.int32))
    sim.predict(t0)     # zero step: the records are the state itself
    return sim


def _run(sim, act, h2, max_nb):
    out = sim.force_block_nb(torch.as_tensor(act, device=sim.device),
                             torch.as_tensor(h2, dtype=torch.float64, device=sim.device), max_nb)
    return {k: v.cpu().numpy() for k, v in out.items()}


def _compare(got, ref, act_n, max_nb, precision, tag, errs=None):
    np.testing.assert_array_equal(got["nb_count"], ref["nb_count"])
    for q in range(act_n):
        k = min(int(ref["nb_count"][q]), max_nb)
        np.testing.assert_array_equal(got["nb_list"][q, :k], ref["nb_list"][q, :k])
    for key in PARTS:
        with np.errstate(invalid="ignore", divide="ignore"):
            e = rel_err(got[key], ref[key])
        # rows without neighbours have an irregular part of exactly zero on both sides
        assert np.all(got[key][:, ref["nb_count"][:act_n] == 0] == 0) or not key.endswith("irr")
        e = e[np.isfinite(e)]
        if errs is not None:
            errs[key].append(e)
        else:
            _check(e, key, precision, tag)


def _check(e, key, precision, tag):
    st = err_stats(e)
    say("   %s %-6s %-7s rms %.2e max %.2e" % (tag, precision, key, st["rms"], st["max"]))
    if precision == "fp64":
        assert st["rms"] <= FP64_TOL["rms"] and st["max"] <= FP64_TOL["max"], (key, st)
    else:
        assert st["rms"] <= LOW_TOL[key[:3]] and st["max"] <= 10 * LOW_TOL[key[:3]], (key, st)


@pytest.fixture(scope="module")
def nb_case():
    """King W0=7 cluster of 2998 stars + BH binary (n = 3000, n_hard = 2,
    eps = 1e-4); active sets of 1, 2 (the two black holes), 7, 130 (two
    i-tiles) and 1000 rows; up to 60 neighbours per row."""
    model = cluster_with_bh(2998, 81)
    n = model.n
    sets = [np.array([5], np.int32), np.array([0, 1], np.int32), nbody_ics.active_subset(n, 7, 811),
            nbody_ics.active_subset(n, 130, 812), nbody_ics.active_subset(n, 1000, 813)]
    radii = [band_free_radii(model.x, a, 820 + k, k_max=60) for k, a in enumerate(sets)]
    return model, 1e-8, 2, sets, radii


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_nb_parity(nb_case, precision):
    model, eps2, n_hard, sets, radii = nb_case
    sim = _sim(model, precision, eps2, n_hard)
    cfg = OracleConfig(order=4, eps2=eps2, n_hard=n_hard)
    errs = {k: [] for k in PARTS}
    for act, (h2, margin) in zip(sets, radii):
        assert margin.min() >= 1e-4
        ref = oracle.force_nb(cfg, model.m, model.x, model.v, act, h2, 64)
        got = _run(sim, act, h2, 64)
        _compare(got, ref, act.size, 64, precision, "nb", errs)
        say("   %d rows: %d..%d neighbours" % (act.size, ref["nb_count"].min(), ref["nb_count"].max()))
    for key, e in errs.items():
        _check(np.concatenate(e), key, precision, "nb")
    # reruns are bitwise identical
    a1 = _run(sim, sets[4], radii[4][0], 64)
    a2 = _run(sim, sets[4], radii[4][0], 64)
    for key in PARTS + ("nb_count", "nb_list"):
        np.testing.assert_array_equal(a1[key], a2[key])
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_nb_list_cap_and_no_list(nb_case, precision):
    """A cap below the counts keeps the true counts and the first neighbours;
    rows whose list was cut get NaN for the irregular part (it is summed over
    the list), the others the same bits as without a cut; max_nb = 0 gives
    counts and the regular part only.  The regular part does not depend on
    the cap."""
    model, eps2, n_hard, sets, radii = nb_case
    sim = _sim(model, precision, eps2, n_hard)
    act, (h2, _) = sets[3], radii[3]
    full = _run(sim, act, h2, 64)
    capped = _run(sim, act, h2, 3)
    assert full["nb_count"].max() > 3 and full["nb_count"].min() <= 3
    np.testing.assert_array_equal(capped["nb_count"], full["nb_count"])
    for q in range(act.size):
        k = min(3, int(full["nb_count"][q]))
        np.testing.assert_array_equal(capped["nb_list"][q, :k], full["nb_list"][q, :k])
    out = sim.force_block_nb(torch.as_tensor(act, device=sim.device),
                             torch.as_tensor(h2, dtype=torch.float64, device=sim.device), 0)
    none = {k: v.cpu().numpy() for k, v in out.items()}
    np.testing.assert_array_equal(none["nb_count"], full["nb_count"])
    for key in ("acc_reg", "jrk_reg"):
        np.testing.assert_array_equal(capped[key], full[key])
        np.testing.assert_array_equal(none[key], full[key])
    cut = full["nb_count"] > 3
    for key in ("acc_irr", "jrk_irr"):
        assert np.all(np.isnan(capped[key][:, cut]))
        np.testing.assert_array_equal(capped[key][:, ~cut], full[key][:, ~cut])
        some = full["nb_count"] > 0
        assert np.all(np.isnan(none[key][:, some])) and np.all(none[key][:, ~some] == 0)
    sim.close()


def test_nb_one_split_and_scratch_limit():
    """15000 rows of a 20000-particle system with room for 2048 neighbours
    each fit the scratch only as one j-split; 20000 rows with 4096 do not fit
    and are refused.  The one-split case is checked on 200 rows."""
    from paper_1312_1789_amd import abi
    model = nbody_ics.plummer(20000, 83)
    sim = _sim(model, "mixed", 1e-8, 0)
    act = np.arange(15000, dtype=np.int32)
    h2 = np.full(act.size, 1e-4)
    rows = act[:200]
    h2r, margin = band_free_radii(model.x, rows, 84, k_max=30)
    h2[:200] = h2r
    got = _run(sim, act, h2, 2048)
    ref = oracle.force_nb(OracleConfig(order=4, eps2=1e-8), model.m, model.x, model.v, rows, h2r, 2048)
    sub = {k: (v[:, :200] if v.ndim == 2 and k in PARTS else v[:200]) for k, v in got.items()}
    _compare(sub, ref, 200, 2048, "mixed", "one split")
    with pytest.raises(abi.NBodyError) as e:
        sim.force_block_nb(torch.arange(20000, dtype=torch.int32, device=sim.device),
                           torch.full((20000,), 1e-4, dtype=torch.float64, device=sim.device), 4096)
    assert e.value.status == abi.NBODY_E_INVALID
    sim.close()


def test_nb_full_size_sampled():
    """n = 2^20 (Plummer), 1024 active rows with up to 80 neighbours; 48 rows
    checked against the oracle, FP64 and MIXED."""
    n = 1 << 20
    model = nbody_ics.plummer(n, 85)
    act = nbody_ics.active_subset(n, 1024, 86)
    check = np.arange(0, 1024, 22)
    h2 = np.full(act.size, 1e-6)
    h2c, margin = band_free_radii(model.x, act[check], 87, k_max=80)
    h2[check] = h2c
    ref = oracle.force_nb(OracleConfig(order=4, eps2=1e-8), model.m, model.x, model.v, act[check], h2c, 128)
    for precision in ("fp64", "mixed"):
        sim = _sim(model, precision, 1e-8, 0)
        got = _run(sim, act, h2, 128)
        sub = {k: (v[:, check] if k in PARTS else v[check]) for k, v in got.items()}
        _compare(sub, ref, check.size, 128, precision, "2^20")
        sim.close()
        del sim
        torch.cuda.empty_cache()


def test_nb_validation():
    from paper_1312_1789_amd import abi
    model = nbody_ics.plummer(500, 88)
    act = torch.arange(10, dtype=torch.int32, device="cuda:0")
    h2 = torch.full((10,), 0.01, dtype=torch.float64, device="cuda:0")
    for order, precision in ((6, "mixed"), (4, "ds")):
        sim = _sim(model, precision, 1e-8, 0, order=order)
        with pytest.raises(abi.NBodyError) as e:
            sim.force_block_nb(act, h2, 8)
        assert e.value.status == abi.NBODY_E_INVALID
        sim.close()
    from paper_1312_1789_amd import Simulation
    sim = Simulation(model.m, model.x, model.v, order=4, precision="fp64", eps2=1e-8)
    with pytest.raises(abi.NBodyError) as e:
        sim.force_block_nb(act, h2, 8)          # no prediction yet
    assert e.value.status == abi.NBODY_E_STATE
    sim.predict(0)
    with pytest.raises(abi.NBodyError) as e:
        sim.force_block_nb(act, h2, 5000)
    assert e.value.status == abi.NBODY_E_INVALID
    out = sim.force_block_nb(act, h2, 8)
    assert torch.isfinite(out["acc_reg"]).all()
    sim.close()


def test_nb_max_size_sampled():
    """The largest system the C-ABI accepts, n = 2^26 (Plummer): 512 active
    rows, 3 of them with radii in distance gaps checked against the oracle
    (64-bit indexing of the lists and partial sums at full size), FP64 and
    MIXED."""
    n = 1 << 26
    model = nbody_ics.plummer(n, 89)
    act = nbody_ics.active_subset(n, 512, 90)
    check = np.array([0, 255, 511])
    h2 = np.full(act.size, 1e-9)
    h2c, margin = band_free_radii(model.x, act[check], 91, k_max=30)
    h2[check] = h2c
    ref = oracle.force_nb(OracleConfig(order=4, eps2=1e-8), model.m, model.x, model.v, act[check], h2c, 64)
    for precision in ("fp64", "mixed"):
        say("max-size neighbour split %s n=%d" % (precision, n))
        sim = _sim(model, precision, 1e-8, 0)
        got = _run(sim, act, h2, 64)
        sub = {k: (v[:, check] if k in PARTS else v[check]) for k, v in got.items()}
        _compare(sub, ref, check.size, 64, precision, "2^26")
        sim.close()
        del sim
        torch.cuda.empty_cache()
