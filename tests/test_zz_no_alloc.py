"""nbody_predict_force_noalloc (no context, partial sums in a static device
array) against nbody_predict_force on the same inputs: calls in a row, each
on a smaller system than the one before, so that the static scratch still
holds the previous call's partial sums; plus the oracle."""
import numpy as np
import pytest
import torch

import nbody_ics
import oracle
from oracle import OracleConfig
from paper_1312_1789_amd import Simulation, abi

from helpers import TICK_BITS, random_block_state, random_derivs, rel_err, say

pytestmark = pytest.mark.gpu

# (n, n_act, order, precision, n_hard, seed): decreasing sizes; n_act 200 and
# 7 take 16 and 4 rows per workgroup, 1 a whole workgroup per row
CASES = [(6000, 200, 6, "mixed", 0, 41), (1500, 7, 6, "mixed", 0, 42), (900, 1, 8, "fp64", 2, 43)]
TOL = {"fp64": {"acc": 1e-12, "jrk": 1e-12, "snp": 1e-12, "crk": 1e-12, "pot": 1e-12},
       "mixed": {"acc": 2e-6, "jrk": 2e-5, "snp": 2e-4, "crk": 2e-3, "pot": 1e-6}}


def test_noalloc_matches_predict_force():
    for n, n_act, order, prec, n_hard, seed in CASES:
        say("noalloc case: n %d n_act %d order %d %s n_hard %d seed %d" % (n, n_act, order, prec, n_hard, seed))
        model = nbody_ics.plummer(n, seed)
        t_tick, level = random_block_state(n, seed + 1)
        T = int((t_tick + (1 << (TICK_BITS - level.astype(np.int64)))).min())
        d = random_derivs(n, seed + 2, order)
        sim = Simulation(model.m, model.x, model.v, order=order, precision=prec, eps2=1e-8, n_hard=n_hard,
                         eta=0.1)
        sim.load_state(model.x, model.v, d, t_tick, level)
        act_np = nbody_ics.active_subset(n, n_act, seed + 3)
        act = torch.as_tensor(act_np, device=sim.device)
        sim.set_launch(1, 64, 0, 3)   # the fused wave j-split kernel with its default split
        ref = sim.predict_force(T, act)
        out = sim.alloc_forces(n_act)
        for t in out.values():
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        abi.nbody_predict_force_noalloc(sim.cfg, sim.state, T, n_act, act.data_ptr(), out["acc"].data_ptr(),
                                        out["jrk"].data_ptr(), out["snp"].data_ptr(), out["crk"].data_ptr(),
                                        out["pot"].data_ptr(), sim.stream.cuda_stream)
        torch.cuda.synchronize()
        keys = ("acc", "jrk", "snp", "crk")[: order // 2] + ("pot",)
        for key in keys:
            assert torch.equal(out[key], ref[key]), (key, n, n_act)
        # the oracle on the same inputs
        cfg = OracleConfig(order=order, eps2=1e-8, n_hard=n_hard)
        st = oracle.State(model.m, model.x, model.v, order, d, t_tick, level)
        xp, vp, ap, jp = oracle.predict(cfg, st, T)
        r = oracle.force(cfg, model.m, xp, vp, ap, jp, act=act_np)
        for key in keys:
            e = rel_err(out[key].cpu().numpy(), r[key])
            rms = float(np.sqrt(np.mean(e * e)))
            say("  %s rms %.2e max %.2e" % (key, rms, e.max()))
            assert rms <= TOL[prec][key], (key, rms)
        sim.close()


def test_noalloc_rejects_large_active_sets():
    model = nbody_ics.plummer(2000, 44)
    sim = Simulation(model.m, model.x, model.v, order=4, precision="mixed", eps2=1e-8)
    act = torch.arange(1025, dtype=torch.int32, device=sim.device)
    out = sim.alloc_forces(1025)
    with pytest.raises(abi.NBodyError) as e:
        abi.nbody_predict_force_noalloc(sim.cfg, sim.state, 0, 1025, act.data_ptr(), out["acc"].data_ptr(),
                                        out["jrk"].data_ptr())
    assert e.value.status == abi.NBODY_E_INVALID and "1024" in abi.last_error()
    sim.close()
