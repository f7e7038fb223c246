"""Thin Python front end over the C-ABI: device memory and streams come from
PyTorch (ROCm build), every computation from libnbody.so.

    sim = Simulation(m, x, v, order=6, precision="mixed", eps2=1e-8)
    sim.init()
    t, n_act = sim.step()
"""
from __future__ import annotations

import numpy as np
import torch

from . import abi


def _dev(a, dtype, device):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(device)


class Simulation:
    """Particle state, workspace and context on one GPU.

    m (n,), x and v (3, n) are host arrays (copied to the device).  State
    tensors: ``m``, ``x``, ``v`` and ``d[k]`` (k = 0 .. order-3) float64,
    ``t_tick`` int64, ``level`` int32, component-major like the C-ABI."""

    def __init__(self, m, x, v, order: int = 4, precision: str | int = "fp64", eps2: float = 1e-8,
                 n_hard: int = 0, eta: float = 0.01, eta_start: float = 0.01, k_min: int = 3, k_max: int = 20,
                 device: str = "cuda:0", stream: torch.cuda.Stream | None = None, dt_rule: int = 0,
                 c_light: float = 0.0, pn_terms: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the N-body library runs only on the device")
        self.device = torch.device(device)
        self.order = int(order)
        prec = abi.PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        n = int(np.asarray(m).shape[0])
        self.n = n
        self.dt_rule = abi.effective_dt_rule(self.order, prec, dt_rule)
        self.cfg = abi.nbody_config(self.order, prec, n, int(n_hard), float(eps2), float(eta), float(eta_start),
                                    int(k_min), int(k_max), int(dt_rule), float(c_light), int(pn_terms))
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.m = _dev(m, torch.float64, self.device)
        self.x = _dev(np.asarray(x).reshape(3, n), torch.float64, self.device)
        self.v = _dev(np.asarray(v).reshape(3, n), torch.float64, self.device)
        self.d = [torch.zeros((3, n), dtype=torch.float64, device=self.device) for _ in range(self.order - 2)]
        self.t_tick = torch.zeros(n, dtype=torch.int64, device=self.device)
        self.level = torch.zeros(n, dtype=torch.int32, device=self.device)
        nbytes = abi.nbody_workspace_size(self.cfg)
        # 256-byte aligned workspace carved from a byte tensor
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.ctx = abi.nbody_create(self.cfg, self._ws_ptr, nbytes, self.stream.cuda_stream)
        self.state = self._state_struct()

    def _state_struct(self) -> abi.nbody_state:
        ds = [t.data_ptr() for t in self.d] + [None] * (6 - len(self.d))
        return abi.nbody_state(self.m.data_ptr(), self.x.data_ptr(), self.v.data_ptr(),
                               (abi.C.c_void_p * 6)(*ds), self.t_tick.data_ptr(), self.level.data_ptr())

    def close(self):
        if getattr(self, "ctx", 0):
            abi.nbody_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- entry points -------------------------------------------------------
    def set_launch(self, ni: int = 1, block: int = 256, n_split: int = 0, jpath: int = 0):
        abi.nbody_set_launch(self.ctx, ni, block, n_split, jpath)

    def autotune(self, max_n_act: int = 16384, reps: int = 3):
        """Tune the force launch per active size on the last prediction."""
        abi.nbody_autotune(self.ctx, max_n_act, reps)

    def tuning(self):
        return abi.nbody_get_tuning(self.ctx)

    def last_launch(self):
        """(ni, block, n_split, jpath) of the last force kernel run."""
        return abi.nbody_get_last_launch(self.ctx)

    def set_timing(self, enable: bool = True):
        abi.nbody_set_timing(self.ctx, enable)

    def timers(self):
        return abi.nbody_get_timers(self.ctx)

    def init(self):
        abi.nbody_init(self.ctx, self.state)

    def predict(self, t_tick: int):
        abi.nbody_predict(self.ctx, self.state, t_tick)

    def alloc_forces(self, n_act: int):
        z = lambda: torch.empty((3, n_act), dtype=torch.float64, device=self.device)
        return {"acc": z(), "jrk": z(), "snp": z(), "crk": z(),
                "pot": torch.empty(n_act, dtype=torch.float64, device=self.device)}

    def force_block(self, act: torch.Tensor, out: dict | None = None, with_pot: bool = True):
        """Forces on the active indices (int32 device tensor) from the last
        prediction; returns dict of (3, n_act) tensors and pot (n_act,)."""
        n_act = int(act.numel())
        out = out if out is not None else self.alloc_forces(n_act)
        abi.nbody_force_block(self.ctx, n_act, act.data_ptr(), out["acc"].data_ptr(), out["jrk"].data_ptr(),
                              out["snp"].data_ptr(), out["crk"].data_ptr(),
                              out["pot"].data_ptr() if with_pot else 0)
        return out

    def predict_force(self, t_tick: int, act: torch.Tensor, out: dict | None = None, with_pot: bool = True):
        """predict(t_tick) then force_block(act), in one kernel where the launch
        shape allows (the records are then not written)."""
        n_act = int(act.numel())
        out = out if out is not None else self.alloc_forces(n_act)
        abi.nbody_predict_force(self.ctx, self.state, t_tick, n_act, act.data_ptr(), out["acc"].data_ptr(),
                                out["jrk"].data_ptr(), out["snp"].data_ptr(), out["crk"].data_ptr(),
                                out["pot"].data_ptr() if with_pot else 0)
        return out

    def force_block_nb(self, act: torch.Tensor, h2: torch.Tensor, max_nb: int, out: dict | None = None):
        """Forces on the active indices split by neighbour spheres (h2: FP64
        device tensor, one radius squared per row) from the last prediction;
        returns acc_irr, jrk_irr, acc_reg, jrk_reg (3, n_act), nb_count
        (n_act,) and nb_list (n_act, max_nb) (int32; -1 past the written
        entries when out is not given)."""
        n_act = int(act.numel())
        if out is None:
            z = lambda: torch.empty((3, n_act), dtype=torch.float64, device=self.device)
            out = {"acc_irr": z(), "jrk_irr": z(), "acc_reg": z(), "jrk_reg": z(),
                   "nb_count": torch.empty(n_act, dtype=torch.int32, device=self.device),
                   "nb_list": torch.full((n_act, max(max_nb, 1)), -1, dtype=torch.int32, device=self.device)}
        abi.nbody_force_block_nb(self.ctx, n_act, act.data_ptr(), h2.data_ptr(), max_nb, out["acc_irr"].data_ptr(),
                                 out["jrk_irr"].data_ptr(), out["acc_reg"].data_ptr(), out["jrk_reg"].data_ptr(),
                                 out["nb_count"].data_ptr(), out["nb_list"].data_ptr() if max_nb > 0 else 0)
        return out

    def set_fusion(self, enable: bool = True):
        abi.nbody_set_fusion(self.ctx, 1 if enable else 0)

    def correct(self, act: torch.Tensor, t_tick: int, f: dict):
        abi.nbody_correct(self.ctx, self.state, int(act.numel()), act.data_ptr(), t_tick, f["acc"].data_ptr(),
                          f["jrk"].data_ptr(), f["snp"].data_ptr(), f["crk"].data_ptr())

    def predicted(self) -> dict:
        """The last prediction as FP64 device tensors xp, vp, ap, jp (3, n)."""
        z = lambda: torch.zeros((3, self.n), dtype=torch.float64, device=self.device)
        out = {"xp": z(), "vp": z(), "ap": z(), "jp": z()}
        abi.nbody_get_predicted(self.ctx, out["xp"].data_ptr(), out["vp"].data_ptr(), out["ap"].data_ptr(),
                                out["jp"].data_ptr())
        return out

    def schedule(self):
        act = torch.empty(self.n, dtype=torch.int32, device=self.device)
        t, na = abi.nbody_schedule(self.ctx, self.state, act.data_ptr())
        return t, act[:na]

    def step(self):
        return abi.nbody_step(self.ctx, self.state)

    def energy(self):
        return abi.nbody_energy(self.ctx, self.state)

    def stats(self) -> abi.nbody_stats:
        return abi.nbody_get_stats(self.ctx)

    def run(self, t_end_tick: int, max_steps: int = 1 << 62):
        """nbody_run: (steps, time of the last step)."""
        return abi.nbody_run(self.ctx, self.state, t_end_tick, max_steps)

    def integrate(self, t_end_tick: int, max_steps: int = 1 << 62):
        """Block steps until the next one would pass t_end_tick (nbody_run);
        returns the number of steps."""
        steps, _ = abi.nbody_run(self.ctx, self.state, t_end_tick, max_steps)
        return steps

    def to_numpy(self) -> dict:
        torch.cuda.synchronize(self.device)
        return {"m": self.m.cpu().numpy(), "x": self.x.cpu().numpy(), "v": self.v.cpu().numpy(),
                "d": [t.cpu().numpy() for t in self.d], "t_tick": self.t_tick.cpu().numpy(),
                "level": self.level.cpu().numpy()}

    def load_state(self, x, v, d, t_tick, level):
        """Overwrite the device state from host arrays."""
        self.x.copy_(_dev(np.asarray(x).reshape(3, self.n), torch.float64, self.device))
        self.v.copy_(_dev(np.asarray(v).reshape(3, self.n), torch.float64, self.device))
        for k, a in enumerate(d):
            self.d[k].copy_(_dev(np.asarray(a).reshape(3, self.n), torch.float64, self.device))
        self.t_tick.copy_(_dev(t_tick, torch.int64, self.device))
        self.level.copy_(_dev(level, torch.int32, self.device))


class Batch:
    """Many independent clusters advanced together through the batched
    entry points.  ``clusters`` is a list of (m, x, v) host arrays; the
    device state is their concatenation (cluster c owns [off[c], off[c+1])),
    with the same tensors as Simulation.  Runs on its own (default-priority)
    stream so that one batched step can be captured in a HIP graph."""

    def __init__(self, clusters, order: int = 6, precision: str | int = "mixed", eps2: float = 1e-8,
                 n_hard: int = 0, eta: float = 0.1, eta_start: float = 0.01, k_min: int = 3, k_max: int = 20,
                 device: str = "cuda:0", dt_rule: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the N-body library runs only on the device")
        self.device = torch.device(device)
        self.order = int(order)
        prec = abi.PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        sizes = [int(np.asarray(c[0]).shape[0]) for c in clusters]
        self.off = [0] + list(np.cumsum(sizes).astype(int))
        self.nc = len(sizes)
        n = self.off[-1]
        self.n = n
        self.dt_rule = abi.effective_dt_rule(self.order, prec, dt_rule)
        self.cfg = abi.nbody_config(self.order, prec, n, int(n_hard), float(eps2), float(eta), float(eta_start),
                                    int(k_min), int(k_max), int(dt_rule))
        self.stream = torch.cuda.Stream(self.device)
        m = np.concatenate([np.asarray(c[0], dtype=np.float64) for c in clusters])
        x = np.concatenate([np.asarray(c[1], dtype=np.float64).reshape(3, -1) for c in clusters], axis=1)
        v = np.concatenate([np.asarray(c[2], dtype=np.float64).reshape(3, -1) for c in clusters], axis=1)
        self.m = _dev(m, torch.float64, self.device)
        self.x = _dev(x, torch.float64, self.device)
        self.v = _dev(v, torch.float64, self.device)
        self.d = [torch.zeros((3, n), dtype=torch.float64, device=self.device) for _ in range(self.order - 2)]
        self.t_tick = torch.zeros(n, dtype=torch.int64, device=self.device)
        self.level = torch.zeros(n, dtype=torch.int32, device=self.device)
        nbytes = abi.nbody_batch_workspace_size(self.cfg, self.off)
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._ws_ptr = (self._ws.data_ptr() + 255) // 256 * 256
        torch.cuda.synchronize(self.device)   # state tensors written before the batch stream reads them
        self.b = abi.nbody_batch_create(self.cfg, self.off, self._ws_ptr, nbytes, self.stream.cuda_stream)
        ds = [t.data_ptr() for t in self.d] + [None] * (6 - len(self.d))
        self.state = abi.nbody_state(self.m.data_ptr(), self.x.data_ptr(), self.v.data_ptr(),
                                     (abi.C.c_void_p * 6)(*ds), self.t_tick.data_ptr(), self.level.data_ptr())

    def close(self):
        if getattr(self, "b", 0):
            self.stream.synchronize()
            abi.nbody_batch_destroy(self.b)
            self.b = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, force_grid: int = 0, items_per_wg: int = 0, i_tile: int = 0):
        abi.nbody_batch_set_launch(self.b, force_grid, items_per_wg, i_tile)

    def get_launch(self):
        return abi.nbody_batch_get_launch(self.b)

    def autotune(self, steps: int = 4):
        abi.nbody_batch_autotune(self.b, self.state, steps)

    def set_end(self, t_end_tick: int):
        abi.nbody_batch_set_end(self.b, t_end_tick)

    def init(self):
        abi.nbody_batch_init(self.b, self.state)

    def step(self, k: int = 1):
        abi.nbody_batch_step(self.b, self.state, k)

    def capture(self):
        abi.nbody_batch_capture(self.b, self.state)

    def replay(self, k: int = 1):
        abi.nbody_batch_replay(self.b, k)

    def poll(self):
        return abi.nbody_batch_poll(self.b, self.nc)

    def last_step(self):
        """(aoff list, act int32 tensor, forces (order/2, 3, n_act) tensor)."""
        aoff = abi.nbody_batch_last_step(self.b, self.nc)
        na = aoff[-1]
        act = torch.empty(max(na, 1), dtype=torch.int32, device=self.device)
        f = torch.empty((self.order // 2, 3, max(na, 1)), dtype=torch.float64, device=self.device)
        abi.nbody_batch_last_step(self.b, self.nc, act.data_ptr(), f.data_ptr())
        return aoff, act[:na], f[:, :, :na]

    def energy(self):
        return abi.nbody_batch_energy(self.b, self.state, self.nc)

    def stats(self) -> abi.nbody_stats:
        return abi.nbody_batch_get_stats(self.b)

    def synchronize(self):
        self.stream.synchronize()

    def to_numpy(self) -> dict:
        self.stream.synchronize()
        return {"m": self.m.cpu().numpy(), "x": self.x.cpu().numpy(), "v": self.v.cpu().numpy(),
                "d": [t.cpu().numpy() for t in self.d], "t_tick": self.t_tick.cpu().numpy(),
                "level": self.level.cpu().numpy()}

    def load_state(self, h: dict):
        """Overwrite the device state from a to_numpy()-style dict of host arrays."""
        self.stream.synchronize()
        self.x.copy_(_dev(h["x"], torch.float64, self.device))
        self.v.copy_(_dev(h["v"], torch.float64, self.device))
        for k, a in enumerate(h["d"]):
            self.d[k].copy_(_dev(a, torch.float64, self.device))
        self.t_tick.copy_(_dev(h["t_tick"], torch.int64, self.device))
        self.level.copy_(_dev(h["level"], torch.int32, self.device))
        torch.cuda.synchronize(self.device)

    def cluster(self, h: dict, c: int) -> dict:
        """Cluster c's slice of a to_numpy() dict."""
        a, b = self.off[c], self.off[c + 1]
        return {"m": h["m"][a:b], "x": h["x"][:, a:b].copy(), "v": h["v"][:, a:b].copy(),
                "d": [t[:, a:b].copy() for t in h["d"]], "t_tick": h["t_tick"][a:b].copy(),
                "level": h["level"][a:b].copy()}
