"""GPU parity of the pairwise force kernels (nbody_predict + nbody_force_block)
against the CPU oracle on identical inputs, element by element.

Tolerances:
* FP64: results differ from the oracle only by summation order and the
  last-bit rounding of rsqrt / FMA contraction: relative error per particle
  rms <= 1e-12, max <= 1e-9 (the max allows for particles whose jerk / snap
  nearly cancel, where the error relative to the small sum grows).
* MIXED and DS: rms relative error <= 2e-6 (acceleration) and <= 2e-5 (jerk),
  the accuracy bar of the mixed-precision scheme; snap and crackle,
  higher derivatives with more cancellation, rms <= 2e-4 / 2e-3; potential
  rms <= 1e-6.  The largest error of any row is bounded at ten times those
  values: FP32 terms carry a relative error of a few 2^-24 each, and a row's
  error relative to its sum grows with how much its terms cancel
  (sum |t_j| / |sum t_j|), which is several times the typical value on the
  rare rows whose jerk, snap or crackle nearly vanish (measured: every
  row's error below 0.4 times the rms bar).
"""
import numpy as np
import pytest
import torch

import nbody_ics
from helpers import TICKS, cluster_with_bh, err_stats, oracle_force, physical_derivs, random_derivs, rel_err, say

pytestmark = pytest.mark.gpu

FP64_TOL = {"rms": 1e-12, "max": 1e-9}
LOW_TOL = {"acc": 2e-6, "jrk": 2e-5, "snp": 2e-4, "crk": 2e-3, "pot": 1e-6}
LOW_MAX = {k: 10.0 * v for k, v in LOW_TOL.items()}
KEYS = {4: ["acc", "jrk"], 6: ["acc", "jrk", "snp"], 8: ["acc", "jrk", "snp", "crk"]}


def _sim(model, order, precision, eps2, n_hard, d, **kw):
    from paper_1312_1789_amd import Simulation
    sim = Simulation(model.m, model.x, model.v, order=order, precision=precision, eps2=eps2, n_hard=n_hard, **kw)
    n = model.n
    t0 = 5 * (TICKS >> 3)
    sim.load_state(model.x, model.v, d[: order - 2], np.full(n, t0, np.int64), np.full(n, 3, np.int32))
    sim.predict(t0)     # zero step: the records are the state itself
    return sim


def _check(out, ref, order, precision, act_n):
    for key in KEYS[order] + ["pot"]:
        e = rel_err(out[key].cpu().numpy()[..., :act_n], ref[key])
        st = err_stats(e)
        say("   %-6s %-4s rms %.2e max %.2e p99.9 %.2e" % (precision, key, st["rms"], st["max"], st["p999"]))
        if precision == "fp64":
            assert st["rms"] <= FP64_TOL["rms"] and st["max"] <= FP64_TOL["max"], (key, st)
        else:
            assert st["rms"] <= LOW_TOL[key] and st["max"] <= LOW_MAX[key], (key, st)


@pytest.fixture(scope="module")
def small_case():
    """King W0=7 cluster of 2998 stars + BH binary: n = 3000 (not a multiple of
    any tile), n_hard = 2, eps = 1e-4, physical a and jerk from the oracle."""
    model = cluster_with_bh(2998, 21)
    eps2, n_hard = 1e-8, 2
    a, j = physical_derivs(model.m, model.x, model.v, eps2, n_hard)
    d = [a, j, np.zeros_like(a), np.zeros_like(a), np.zeros_like(a), np.zeros_like(a)]
    return model, eps2, n_hard, d


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
@pytest.mark.parametrize("order", [4, 6, 8])
def test_force_parity_small(small_case, order, precision):
    model, eps2, n_hard, d = small_case
    n = model.n
    say("force parity order %d %s n=%d" % (order, precision, n))
    sim = _sim(model, order, precision, eps2, n_hard, d)
    acts = {
        "all": np.arange(n, dtype=np.int32),
        "subset1000": nbody_ics.active_subset(n, 1000, 1510),
        "bh": np.array([0], np.int32),
        "last": np.array([n - 1], np.int32),
        "ragged17": nbody_ics.active_subset(n, 17, 1504),
    }
    for name, act in acts.items():
        say("  act=%s n_act=%d" % (name, act.size))
        out = sim.force_block(torch.as_tensor(act, device=sim.device))
        torch.cuda.synchronize()
        ref = oracle_force(order, eps2, n_hard, model.m, model.x, model.v, d[0], d[1], act=act)
        _check(out, ref, order, precision, act.size)


def test_unsorted_active_list_permutes_rows(small_case):
    model, eps2, n_hard, d = small_case
    sim = _sim(model, 6, "fp64", eps2, n_hard, d)
    act = nbody_ics.active_subset(model.n, 300, 1520)
    perm = np.random.default_rng(0).permutation(300)
    a1 = sim.force_block(torch.as_tensor(act, device=sim.device))["acc"].cpu().numpy()
    a2 = sim.force_block(torch.as_tensor(act[perm], device=sim.device))["acc"].cpu().numpy()
    np.testing.assert_array_equal(a1[:, perm], a2)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_launch_shapes_and_determinism(small_case, precision):
    """ni, block and the j path (scalar loads or LDS tiles) do not change any
    bit; reruns are bitwise identical; the split count changes only the
    summation order (in MIXED mode also where the FP32 chunk sums start, so up
    to FP32 rounding)."""
    model, eps2, n_hard, d = small_case
    sim = _sim(model, 6, precision, eps2, n_hard, d)
    act = torch.as_tensor(nbody_ics.active_subset(model.n, 700, 1530), device=sim.device)
    ref = None
    for ni, block, jpath in [(1, 256, 1), (2, 256, 1), (1, 64, 2), (2, 128, 2), (1, 256, 2), (2, 256, 2)]:
        sim.set_launch(ni, block, 5, jpath)
        out = {k: t.cpu().numpy().copy() for k, t in sim.force_block(act).items()}
        if ref is None:
            ref = out
        for k in ("acc", "jrk", "snp", "pot"):
            np.testing.assert_array_equal(out[k], ref[k])
    again = sim.force_block(act)
    np.testing.assert_array_equal(again["acc"].cpu().numpy(), ref["acc"])
    sim.set_launch(1, 256, 1)
    one = sim.force_block(act)["acc"].cpu().numpy()
    assert np.max(rel_err(one, ref["acc"])) < (1e-12 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_split_layouts(precision):
    """Partial sums of launches with more than 32 j-splits are stored
    split-fastest, with fewer row-fastest.  n = 20000 (King W0=7 + black-hole
    binary), order 6, 300 active rows: for requests of 16, 64 and 160 splits
    (16, 53 and 157 after rounding to whole 128-particle chunks: row-fastest,
    then split-fastest with 16 and 64 reduction lanes per output) every
    i-tile shape and j path gives the same bits, and the result matches the
    oracle."""
    model = cluster_with_bh(19998, 23)
    eps2, n_hard = 1e-8, 2
    a, j = physical_derivs(model.m, model.x, model.v, eps2, n_hard)
    d = [a, j, np.zeros_like(a), np.zeros_like(a), np.zeros_like(a), np.zeros_like(a)]
    sim = _sim(model, 6, precision, eps2, n_hard, d)
    act_np = nbody_ics.active_subset(model.n, 300, 1560)
    act = torch.as_tensor(act_np, device=sim.device)
    ref = oracle_force(6, eps2, n_hard, model.m, model.x, model.v, d[0], d[1], act=act_np)
    for n_split in (16, 64, 160):
        first = None
        for ni, block, jpath in [(1, 256, 1), (2, 128, 1), (1, 64, 2), (2, 256, 2)]:
            sim.set_launch(ni, block, n_split, jpath)
            out = {k: t.cpu().numpy().copy() for k, t in sim.force_block(act).items()}
            if first is None:
                first = out
                say("split layouts %s: %d splits" % (precision, n_split))
                _check(sim.force_block(act), ref, 6, precision, act_np.size)
            for k in ("acc", "jrk", "snp", "pot"):
                np.testing.assert_array_equal(out[k], first[k])
    sim.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotuned_launch_keeps_parity(small_case, precision):
    """nbody_autotune fills one row per power-of-two active size with a valid
    shape; force calls then take their shape from the table and still match
    the oracle; a shape set afterwards replaces the table."""
    model, eps2, n_hard, d = small_case
    n = model.n
    sim = _sim(model, 6, precision, eps2, n_hard, d)
    sim.autotune(1024, 1)
    table = sim.tuning()
    say("tuned table (%s): %s" % (precision, [(r[0], r[1], r[2], r[3], r[4], round(r[5], 4)) for r in table]))
    assert [r[0] for r in table] == [1 << k for k in range(11)]
    for na, ni, block, sp, jpath, ms in table:
        assert ni in (1, 2) and block in (64, 128, 256) and jpath in (1, 2, 3) and sp >= 1 and ms > 0
    for k in (1, 17, 300, 2999):
        act = nbody_ics.active_subset(n, k, 1540 + k)
        out = sim.force_block(torch.as_tensor(act, device=sim.device))
        ref = oracle_force(6, eps2, n_hard, model.m, model.x, model.v, d[0], d[1], act=act)
        _check(out, ref, 6, precision, act.size)
    act = torch.as_tensor(nbody_ics.active_subset(n, 700, 1530), device=sim.device)
    sim.set_launch(2, 128, 5, 2)
    a1 = sim.force_block(act)["acc"].cpu().numpy()
    sim.set_launch(1, 64, 5, 1)
    a2 = sim.force_block(act)["acc"].cpu().numpy()
    np.testing.assert_array_equal(a1, a2)


def test_unsoftened_pair_and_empty_call():
    """eps = 0 (every pair unsoftened, self pair excluded by index): the
    two-body closed form; n_act = 0 is a no-op."""
    from paper_1312_1789_amd import Simulation
    m = np.array([0.6, 0.4])
    x = np.array([[0.1, -0.3], [0.2, 0.5], [-0.1, 0.0]])
    v = np.zeros((3, 2))
    sim = Simulation(m, x, v, order=4, precision="fp64", eps2=0.0)
    sim.predict(0)
    out = sim.force_block(torch.arange(2, dtype=torch.int32, device=sim.device))
    r = x[:, 1] - x[:, 0]
    want = 0.4 * r / np.linalg.norm(r) ** 3
    np.testing.assert_allclose(out["acc"].cpu().numpy()[:, 0], want, rtol=1e-14)
    assert abs(out["pot"].cpu().numpy()[0] + 0.4 / np.linalg.norm(r)) < 1e-15
    empty = torch.empty(0, dtype=torch.int32, device=sim.device)
    sim.force_block(empty)


# launch shapes the benchmark fixes for the all-active force at n = 2^20
# (ni, block, n_split, jpath)
BENCH_SHAPE = {"mixed": (2, 256, 16, 2), "fp64": (2, 128, 16, 1)}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_force_full_size_sampled(precision):
    """The headline workload: King W0=7, n = 2^20, 6th order, all particles
    active in one call, in the untuned default launch and in the launch the
    benchmark times (which must run as asked: 16 splits); 256 sampled rows
    are checked against the oracle in both, and the two agree to the
    summation-order difference."""
    n = 1 << 20
    say("full-size force %s n=%d" % (precision, n))
    model = nbody_ics.king(n, 7.0, 13)
    d = random_derivs(n, 1313, 8)
    sim = _sim(model, 6, precision, 1e-8, 0, d)
    act = torch.arange(n, dtype=torch.int32, device=sim.device)
    sample = nbody_ics.active_subset(n, 256, 1520)
    ref = oracle_force(6, 1e-8, 0, model.m, model.x, model.v, d[0], None, act=sample)
    idx = torch.as_tensor(sample.astype(np.int64), device=sim.device)
    outs = []
    for shape in (None, BENCH_SHAPE[precision]):
        if shape is not None:
            sim.set_launch(*shape)
        out = sim.force_block(act, with_pot=False)
        torch.cuda.synchronize()
        used = sim.last_launch()
        say("  launch %s ran as %s" % (shape or "default", used))
        if shape is not None:
            assert used == shape, (used, shape)
        got = {k: t[..., idx] for k, t in out.items() if k != "pot"}
        for key in KEYS[6]:
            st = err_stats(rel_err(got[key].cpu().numpy(), ref[key]))
            say("   %-6s %-4s rms %.2e max %.2e" % (precision, key, st["rms"], st["max"]))
            if precision == "fp64":
                assert st["rms"] <= FP64_TOL["rms"] and st["max"] <= FP64_TOL["max"], (key, st)
            else:
                assert st["rms"] <= LOW_TOL[key] and st["max"] <= LOW_MAX[key], (key, st)
        outs.append(out["acc"].clone())
    diff = float(((outs[0] - outs[1]).norm(dim=0) / outs[1].norm(dim=0)).max())
    say("  default vs benchmark launch: max relative difference %.2e" % diff)
    assert diff <= (1e-12 if precision == "fp64" else 1e-5)
    sim.close()


def test_force_c3_size_sampled():
    """The C3 system at its size and order: King W0=7 with 2^20 stars plus a
    black-hole binary (n = 2^20 + 2, n_hard = 2: the two black holes are
    mutually unsoftened), 8th order, MIXED, all particles active, in the
    default launch and with 16 splits; 254 random rows plus both black holes
    against the oracle (stored derivatives seeded, |a| ~ 1)."""
    model = cluster_with_bh(1 << 20, 13)
    n = model.n
    d = random_derivs(n, 1314, 8)
    sim = _sim(model, 8, "mixed", 1e-8, 2, d)
    act = torch.arange(n, dtype=torch.int32, device=sim.device)
    sample = np.concatenate([np.array([0, 1], np.int32), nbody_ics.active_subset(n - 2, 254, 1521) + 2])
    ref = oracle_force(8, 1e-8, 2, model.m, model.x, model.v, d[0], d[1], act=sample)
    idx = torch.as_tensor(sample.astype(np.int64), device=sim.device)
    for shape in (None, (2, 256, 16, 2)):
        if shape is not None:
            sim.set_launch(*shape)
        out = sim.force_block(act, with_pot=False)
        torch.cuda.synchronize()
        say("C3 force n=%d order 8 mixed, launch %s ran as %s" % (n, shape or "default", sim.last_launch()))
        got = {k: t[..., idx].cpu().numpy() for k, t in out.items() if k != "pot"}
        for key in KEYS[8]:
            e = rel_err(got[key], ref[key])
            st = err_stats(e)
            say("   %-4s rms %.2e max %.2e; black holes %.2e %.2e" % (key, st["rms"], st["max"], e[0], e[1]))
            assert st["rms"] <= LOW_TOL[key] and st["max"] <= LOW_MAX[key], (key, st)
            assert max(e[0], e[1]) <= LOW_TOL[key], key
    sim.close()


def test_last_launch_reports_split_bounds(small_case):
    """A requested split count is lowered to what the partial-sum scratch
    holds (n_act * n_split <= 2^21 rows at this size) and to splits of at
    least 128 j; nbody_get_last_launch reports what ran."""
    model, eps2, n_hard, d = small_case
    n = model.n
    sim = _sim(model, 6, "mixed", eps2, n_hard, d)
    assert sim.last_launch() == (0, 0, 0, 0)
    act = torch.arange(n, dtype=torch.int32, device=sim.device)
    for req in (1, 5, 23, 24, 65535):
        sim.set_launch(2, 128, req, 2)
        sim.force_block(act, with_pot=False)
        sp = min(req, (1 << 21) // n)
        chunk = -(-(-(-n // sp)) // 128) * 128
        want = -(-n // chunk)
        assert sim.last_launch() == (2, 128, want, 2), (req, sim.last_launch(), want)
    sim.set_launch(2, 256, 0, 3)   # the wave j-split kernel ignores ni and block
    sim.force_block(act[:5], with_pot=False)
    got = sim.last_launch()
    assert got[0] == 1 and got[1] == 64 and got[3] == 3 and got[2] >= 1
    sim.close()


def test_force_max_size_sampled():
    """The largest system the C-ABI accepts, n = 2^26 (Plummer, 4th order):
    4096 random active rows through the tiled kernels and 7 through the wave
    j-split kernel, in FP64 and MIXED; 128 and 7 rows checked against the
    oracle (64-bit indexing, split-count and partial-buffer caps at full
    size); the 7 rows again with the predictor inside the kernel, bit for
    bit."""
    n = 1 << 26
    model = nbody_ics.plummer(n, 1717)
    d = random_derivs(n, 1718, 4)
    sample = nbody_ics.active_subset(n, 4096, 1719)
    check = sample[:: 32]
    tiny = nbody_ics.active_subset(n, 7, 1720)
    ref_big = oracle_force(4, 1e-8, 0, model.m, model.x, model.v, act=check)
    ref_tiny = oracle_force(4, 1e-8, 0, model.m, model.x, model.v, act=tiny)
    for precision in ("fp64", "mixed"):
        say("max-size force %s n=%d" % (precision, n))
        sim = _sim(model, 4, precision, 1e-8, 0, d)
        out = sim.force_block(torch.as_tensor(sample, device=sim.device), with_pot=False)
        idx = torch.as_tensor(np.arange(0, sample.size, 32), device=sim.device)
        got = {k: t[..., idx] for k, t in out.items() if k != "pot"}
        for key in ("acc", "jrk"):
            st = err_stats(rel_err(got[key].cpu().numpy(), ref_big[key]))
            say("   %-6s %-4s rms %.2e max %.2e" % (precision, key, st["rms"], st["max"]))
            tol = FP64_TOL["rms"] if precision == "fp64" else LOW_TOL[key]
            assert st["rms"] <= tol and st["max"] <= (FP64_TOL["max"] if precision == "fp64" else LOW_MAX[key]), \
                (key, st)
        tiny_t = torch.as_tensor(tiny, device=sim.device)
        out = sim.force_block(tiny_t, with_pot=False)
        for key in ("acc", "jrk"):
            e = rel_err(out[key].cpu().numpy(), ref_tiny[key])
            say("   %-6s %-4s (7 rows, wave j-split) max %.2e" % (precision, key, float(e.max())))
            assert float(e.max()) <= (FP64_TOL["max"] if precision == "fp64" else 20 * LOW_TOL[key]), key
        # the same rows with the predictor inside the force kernel: the same bits
        fused = sim.predict_force(5 * (TICKS >> 3), tiny_t, with_pot=False)
        for key in ("acc", "jrk"):
            assert torch.equal(fused[key], out[key]), key
        sim.close()
        del sim, out
        torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
@pytest.mark.parametrize("order", [4, 6, 8])
def test_wave_split_kernel_parity(small_case, order, precision):
    """The wave j-split kernel (j path 3: 1, 4 or 16 rows per wave, each row's
    j range spread over 64, 16 or 4 lanes) on small active sets, including
    the black holes (unsoftened pair) and ragged row counts, with one split
    and with many; errors pooled over all rows of all sets."""
    model, eps2, n_hard, d = small_case
    n = model.n
    sim = _sim(model, order, precision, eps2, n_hard, d)
    sets = [np.array([0], np.int32), np.array([1, 0], np.int32), np.array([n - 1], np.int32),
            nbody_ics.active_subset(n, 3, 1561), nbody_ics.active_subset(n, 4, 1562),
            nbody_ics.active_subset(n, 7, 1563), nbody_ics.active_subset(n, 16, 1564),
            nbody_ics.active_subset(n, 17, 1565), nbody_ics.active_subset(n, 64, 1566)]
    errs = {k: [] for k in KEYS[order] + ["pot"]}
    for n_split in (0, 1, 7):
        sim.set_launch(1, 64, n_split, 3)
        for act in sets:
            out = sim.force_block(torch.as_tensor(act, device=sim.device))
            ref = oracle_force(order, eps2, n_hard, model.m, model.x, model.v, d[0], d[1], act=act)
            for key in errs:
                errs[key].append(rel_err(out[key].cpu().numpy()[..., :act.size], ref[key]))
    for key, e in errs.items():
        st = err_stats(np.concatenate(e))
        say("   wave split %s p%d %-4s rms %.2e max %.2e" % (precision, order, key, st["rms"], st["max"]))
        if precision == "fp64":
            assert st["rms"] <= FP64_TOL["rms"] and st["max"] <= FP64_TOL["max"], (key, st)
        else:
            assert st["rms"] <= LOW_TOL[key] and st["max"] <= LOW_MAX[key], (key, st)
    # reruns are bitwise identical
    act = torch.as_tensor(sets[6], device=sim.device)
    a1 = sim.force_block(act)["acc"].cpu().numpy()
    a2 = sim.force_block(act)["acc"].cpu().numpy()
    np.testing.assert_array_equal(a1, a2)
