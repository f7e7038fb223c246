"""ctypes binding of libnbody.so: the entry points of include/nbody.h under
the same names, with argument marshalling only (every step of the path runs
in the HIP kernels).  Device pointers are plain integers (e.g. a torch
tensor's ``data_ptr()``); the stream is a ``hipStream_t`` integer.

Loading fails loudly when the library has not been built: there is no
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnbody.so")

NBODY_OK = 0
NBODY_E_INVALID = -1
NBODY_E_HIP = -2
NBODY_E_WORKSPACE = -3
NBODY_E_STATE = -4
NBODY_E_UNSUPPORTED = -5
NBODY_E_NONFINITE = -6

#: time is counted in integer ticks of 2^-TICK_BITS time units
TICK_BITS = 40
TICKS_PER_UNIT = 1 << TICK_BITS

NBODY_FP64 = 0
NBODY_MIXED = 1
NBODY_DS = 2
PRECISIONS = {"fp64": NBODY_FP64, "mixed": NBODY_MIXED, "ds": NBODY_DS}


def effective_dt_rule(order: int, precision: int, dt_rule: int = 0) -> int:
    """The time-step rule a configuration runs with (dt_rule 0 resolved as
    the library resolves it)."""
    if dt_rule:
        return int(dt_rule)
    return 2 if (precision != NBODY_FP64 or order == 8) else 1

#: every symbol the header declares
EXPORTS = (
    "nbody_workspace_size", "nbody_create", "nbody_destroy", "nbody_init", "nbody_predict",
    "nbody_force_block", "nbody_predict_force", "nbody_predict_force_noalloc", "nbody_set_fusion", "nbody_force_block_nb", "nbody_correct", "nbody_schedule", "nbody_step", "nbody_run", "nbody_energy",
    "nbody_get_predicted", "nbody_get_stats", "nbody_set_launch", "nbody_set_timing", "nbody_get_timers",
    "nbody_autotune", "nbody_get_tuning", "nbody_get_last_launch",
    "nbody_batch_workspace_size", "nbody_batch_create", "nbody_batch_destroy", "nbody_batch_init",
    "nbody_batch_set_end", "nbody_batch_step", "nbody_batch_capture", "nbody_batch_replay", "nbody_batch_poll",
    "nbody_batch_last_step", "nbody_batch_energy", "nbody_batch_get_stats", "nbody_batch_set_launch",
    "nbody_batch_get_launch", "nbody_batch_autotune",
    "nbody_last_error",
)


class nbody_config(C.Structure):
    _fields_ = [("order", C.c_int32), ("precision", C.c_int32), ("n", C.c_int64), ("n_hard", C.c_int64),
                ("eps2", C.c_double), ("eta", C.c_double), ("eta_start", C.c_double),
                ("k_min", C.c_int32), ("k_max", C.c_int32), ("dt_rule", C.c_int32),
                ("c_light", C.c_double), ("pn_terms", C.c_int32)]


class nbody_state(C.Structure):
    _fields_ = [("m", C.c_void_p), ("x", C.c_void_p), ("v", C.c_void_p), ("d", C.c_void_p * 6),
                ("t_tick", C.c_void_p), ("level", C.c_void_p)]


class nbody_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("sum_n_act", C.c_int64), ("interactions", C.c_double),
                ("dt_underflow", C.c_int64), ("nonfinite", C.c_int64)]


class NBodyError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__("%s failed (%d): %s" % (func, status, msg))
        self.status = status


_lib = None


def lib():
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnbody.so is not built (%s); run paper_1312_1789_amd/build_lib.py" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        I64 = C.c_int64
        sig = {
            "nbody_workspace_size": [C.POINTER(nbody_config), C.POINTER(C.c_size_t)],
            "nbody_create": [C.POINTER(nbody_config), P, C.c_size_t, P, C.POINTER(P)],
            "nbody_destroy": [P],
            "nbody_init": [P, C.POINTER(nbody_state)],
            "nbody_predict": [P, C.POINTER(nbody_state), I64],
            "nbody_force_block": [P, I64, P, P, P, P, P, P],
            "nbody_predict_force": [P, C.POINTER(nbody_state), I64, I64, P, P, P, P, P, P],
            "nbody_predict_force_noalloc": [C.POINTER(nbody_config), C.POINTER(nbody_state), I64, I64, P, P, P, P,
                                            P, P, P],
            "nbody_set_fusion": [P, C.c_int32],
            "nbody_force_block_nb": [P, I64, P, P, C.c_int32, P, P, P, P, P, P],
            "nbody_correct": [P, C.POINTER(nbody_state), I64, P, I64, P, P, P, P],
            "nbody_schedule": [P, C.POINTER(nbody_state), P, C.POINTER(I64), C.POINTER(I64)],
            "nbody_step": [P, C.POINTER(nbody_state), C.POINTER(I64), C.POINTER(I64)],
            "nbody_run": [P, C.POINTER(nbody_state), I64, I64, C.POINTER(I64), C.POINTER(I64)],
            "nbody_energy": [P, C.POINTER(nbody_state), C.POINTER(C.c_double), C.POINTER(C.c_double)],
            "nbody_get_predicted": [P, P, P, P, P],
            "nbody_get_stats": [P, C.POINTER(nbody_stats)],
            "nbody_set_launch": [P, C.c_int32, C.c_int32, C.c_int32, C.c_int32],
            "nbody_set_timing": [P, C.c_int32],
            "nbody_get_timers": [P, C.POINTER(C.c_double), C.POINTER(I64)],
            "nbody_autotune": [P, I64, C.c_int32],
            "nbody_get_tuning": [P, C.c_int32, C.POINTER(I64), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                 C.POINTER(C.c_int32)],
            "nbody_get_last_launch": [P, C.POINTER(C.c_int32)],
            "nbody_batch_workspace_size": [C.POINTER(nbody_config), C.c_int32, C.POINTER(I64), C.POINTER(C.c_size_t)],
            "nbody_batch_create": [C.POINTER(nbody_config), C.c_int32, C.POINTER(I64), P, C.c_size_t, P,
                                   C.POINTER(P)],
            "nbody_batch_destroy": [P],
            "nbody_batch_init": [P, C.POINTER(nbody_state)],
            "nbody_batch_set_end": [P, I64],
            "nbody_batch_step": [P, C.POINTER(nbody_state), I64],
            "nbody_batch_capture": [P, C.POINTER(nbody_state)],
            "nbody_batch_replay": [P, I64],
            "nbody_batch_poll": [P, C.POINTER(I64), C.POINTER(I64)],
            "nbody_batch_last_step": [P, C.POINTER(I64), P, P],
            "nbody_batch_energy": [P, C.POINTER(nbody_state), C.POINTER(C.c_double), C.POINTER(C.c_double)],
            "nbody_batch_get_stats": [P, C.POINTER(nbody_stats)],
            "nbody_batch_set_launch": [P, C.c_int32, C.c_int32, C.c_int32],
            "nbody_batch_get_launch": [P, C.POINTER(C.c_int32)],
            "nbody_batch_autotune": [P, C.POINTER(nbody_state), C.c_int32],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.nbody_last_error.argtypes = []
        L.nbody_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def last_error() -> str:
    return lib().nbody_last_error().decode()


def _check(status: int, func: str) -> int:
    if status != NBODY_OK:
        raise NBodyError(status, func, last_error())
    return status


def nbody_workspace_size(cfg: nbody_config) -> int:
    b = C.c_size_t(0)
    _check(lib().nbody_workspace_size(C.byref(cfg), C.byref(b)), "nbody_workspace_size")
    return int(b.value)


def nbody_create(cfg: nbody_config, workspace: int, nbytes: int, stream: int = 0) -> int:
    out = C.c_void_p(0)
    _check(lib().nbody_create(C.byref(cfg), C.c_void_p(workspace), nbytes, C.c_void_p(stream), C.byref(out)),
           "nbody_create")
    return int(out.value)


def nbody_destroy(ctx: int) -> None:
    _check(lib().nbody_destroy(C.c_void_p(ctx)), "nbody_destroy")


def nbody_init(ctx: int, st: nbody_state) -> None:
    _check(lib().nbody_init(C.c_void_p(ctx), C.byref(st)), "nbody_init")


def nbody_predict(ctx: int, st: nbody_state, t_tick: int) -> None:
    _check(lib().nbody_predict(C.c_void_p(ctx), C.byref(st), int(t_tick)), "nbody_predict")


def nbody_force_block(ctx: int, n_act: int, act_idx: int, acc: int, jrk: int, snp: int = 0, crk: int = 0,
                      pot: int = 0) -> None:
    P = C.c_void_p
    _check(lib().nbody_force_block(P(ctx), int(n_act), P(act_idx), P(acc), P(jrk), P(snp or None),
                                   P(crk or None), P(pot or None)), "nbody_force_block")


def nbody_predict_force(ctx: int, st: nbody_state, t_tick: int, n_act: int, act_idx: int, acc: int, jrk: int,
                        snp: int = 0, crk: int = 0, pot: int = 0) -> None:
    P = C.c_void_p
    _check(lib().nbody_predict_force(P(ctx), C.byref(st), int(t_tick), int(n_act), P(act_idx), P(acc), P(jrk),
                                     P(snp or None), P(crk or None), P(pot or None)), "nbody_predict_force")


def nbody_predict_force_noalloc(cfg: nbody_config, st: nbody_state, t_tick: int, n_act: int, act_idx: int, acc: int,
                                jrk: int, snp: int = 0, crk: int = 0, pot: int = 0, stream: int = 0) -> None:
    P = C.c_void_p
    _check(lib().nbody_predict_force_noalloc(C.byref(cfg), C.byref(st), int(t_tick), int(n_act), P(act_idx), P(acc),
                                             P(jrk), P(snp or None), P(crk or None), P(pot or None),
                                             P(stream or None)), "nbody_predict_force_noalloc")


def nbody_force_block_nb(ctx: int, n_act: int, act_idx: int, h2: int, max_nb: int, acc_irr: int, jrk_irr: int,
                         acc_reg: int, jrk_reg: int, nb_count: int, nb_list: int = 0) -> None:
    P = C.c_void_p
    _check(lib().nbody_force_block_nb(P(ctx), int(n_act), P(act_idx), P(h2), int(max_nb), P(acc_irr), P(jrk_irr),
                                      P(acc_reg), P(jrk_reg), P(nb_count), P(nb_list or None)),
           "nbody_force_block_nb")


def nbody_set_fusion(ctx: int, enable: int) -> None:
    _check(lib().nbody_set_fusion(C.c_void_p(ctx), int(enable)), "nbody_set_fusion")


def nbody_correct(ctx: int, st: nbody_state, n_act: int, act_idx: int, t_tick: int, acc: int, jrk: int,
                  snp: int = 0, crk: int = 0) -> None:
    P = C.c_void_p
    _check(lib().nbody_correct(P(ctx), C.byref(st), int(n_act), P(act_idx), int(t_tick), P(acc), P(jrk),
                               P(snp or None), P(crk or None)), "nbody_correct")


def nbody_schedule(ctx: int, st: nbody_state, act_idx_out: int):
    t = C.c_int64(0)
    na = C.c_int64(0)
    _check(lib().nbody_schedule(C.c_void_p(ctx), C.byref(st), C.c_void_p(act_idx_out), C.byref(t), C.byref(na)),
           "nbody_schedule")
    return int(t.value), int(na.value)


def nbody_step(ctx: int, st: nbody_state):
    """One block step; returns (t_tick, n_act).  Raises NBodyError (status
    NBODY_E_NONFINITE) when a corrected value became non-finite."""
    t = C.c_int64(0)
    na = C.c_int64(0)
    _check(lib().nbody_step(C.c_void_p(ctx), C.byref(st), C.byref(t), C.byref(na)), "nbody_step")
    return int(t.value), int(na.value)


def nbody_run(ctx: int, st: nbody_state, t_end_tick: int, max_steps: int = (1 << 62)):
    """Block steps until the next would pass t_end_tick; returns (steps, t_tick).
    Raises NBodyError (status NBODY_E_NONFINITE) on a non-finite value."""
    n = C.c_int64(0)
    t = C.c_int64(0)
    _check(lib().nbody_run(C.c_void_p(ctx), C.byref(st), int(t_end_tick), int(max_steps), C.byref(n), C.byref(t)),
           "nbody_run")
    return int(n.value), int(t.value)


def nbody_energy(ctx: int, st: nbody_state):
    T = C.c_double(0)
    W = C.c_double(0)
    _check(lib().nbody_energy(C.c_void_p(ctx), C.byref(st), C.byref(T), C.byref(W)), "nbody_energy")
    return float(T.value), float(W.value)


def nbody_get_predicted(ctx: int, xp: int, vp: int, ap: int = 0, jp: int = 0) -> None:
    P = C.c_void_p
    _check(lib().nbody_get_predicted(P(ctx), P(xp), P(vp), P(ap or None), P(jp or None)), "nbody_get_predicted")


def nbody_get_stats(ctx: int) -> nbody_stats:
    s = nbody_stats()
    _check(lib().nbody_get_stats(C.c_void_p(ctx), C.byref(s)), "nbody_get_stats")
    return s


def nbody_set_launch(ctx: int, ni: int, block: int, n_split: int, jpath: int = 0) -> None:
    _check(lib().nbody_set_launch(C.c_void_p(ctx), int(ni), int(block), int(n_split), int(jpath)), "nbody_set_launch")


def nbody_set_timing(ctx: int, enable: bool) -> None:
    _check(lib().nbody_set_timing(C.c_void_p(ctx), 1 if enable else 0), "nbody_set_timing")


def nbody_autotune(ctx: int, max_n_act: int, reps: int = 3) -> None:
    _check(lib().nbody_autotune(C.c_void_p(ctx), int(max_n_act), int(reps)), "nbody_autotune")


def nbody_get_tuning(ctx: int):
    """List of (n_act, ni, block, n_split, jpath, ms) rows of the tuned table."""
    k = 32
    na = (C.c_int64 * k)()
    sh = (C.c_int32 * (4 * k))()
    ms = (C.c_double * k)()
    rows = C.c_int32(0)
    _check(lib().nbody_get_tuning(C.c_void_p(ctx), k, na, sh, ms, C.byref(rows)), "nbody_get_tuning")
    return [(int(na[r]), int(sh[4 * r]), int(sh[4 * r + 1]), int(sh[4 * r + 2]), int(sh[4 * r + 3]), float(ms[r]))
            for r in range(rows.value)]


def nbody_get_last_launch(ctx: int):
    """(ni, block, n_split, jpath) of the last force kernel the context ran."""
    out = (C.c_int32 * 4)()
    _check(lib().nbody_get_last_launch(C.c_void_p(ctx), out), "nbody_get_last_launch")
    return tuple(int(v) for v in out)


PHASES = ("schedule", "host_roundtrip", "predict", "force", "correct")


def nbody_get_timers(ctx: int):
    """(dict phase -> total ms, number of timed steps)."""
    ms = (C.c_double * 5)()
    steps = C.c_int64(0)
    _check(lib().nbody_get_timers(C.c_void_p(ctx), ms, C.byref(steps)), "nbody_get_timers")
    return dict(zip(PHASES, list(ms))), int(steps.value)


# ---- batched form ------------------------------------------------------------
def _offsets(off):
    off = [int(o) for o in off]
    return len(off) - 1, (C.c_int64 * len(off))(*off)


def nbody_batch_workspace_size(cfg: nbody_config, off) -> int:
    nc, arr = _offsets(off)
    b = C.c_size_t(0)
    _check(lib().nbody_batch_workspace_size(C.byref(cfg), nc, arr, C.byref(b)), "nbody_batch_workspace_size")
    return int(b.value)


def nbody_batch_create(cfg: nbody_config, off, workspace: int, nbytes: int, stream: int = 0) -> int:
    nc, arr = _offsets(off)
    out = C.c_void_p(0)
    _check(lib().nbody_batch_create(C.byref(cfg), nc, arr, C.c_void_p(workspace), nbytes, C.c_void_p(stream),
                                    C.byref(out)), "nbody_batch_create")
    return int(out.value)


def nbody_batch_destroy(b: int) -> None:
    _check(lib().nbody_batch_destroy(C.c_void_p(b)), "nbody_batch_destroy")


def nbody_batch_init(b: int, st: nbody_state) -> None:
    _check(lib().nbody_batch_init(C.c_void_p(b), C.byref(st)), "nbody_batch_init")


def nbody_batch_set_end(b: int, t_end_tick: int) -> None:
    _check(lib().nbody_batch_set_end(C.c_void_p(b), int(t_end_tick)), "nbody_batch_set_end")


def nbody_batch_step(b: int, st: nbody_state, k: int = 1) -> None:
    _check(lib().nbody_batch_step(C.c_void_p(b), C.byref(st), int(k)), "nbody_batch_step")


def nbody_batch_capture(b: int, st: nbody_state) -> None:
    _check(lib().nbody_batch_capture(C.c_void_p(b), C.byref(st)), "nbody_batch_capture")


def nbody_batch_replay(b: int, k: int = 1) -> None:
    _check(lib().nbody_batch_replay(C.c_void_p(b), int(k)), "nbody_batch_replay")


def nbody_batch_poll(b: int, n_clusters: int):
    """(clusters that stepped in the last batched step, list of cluster times)."""
    live = C.c_int64(0)
    t = (C.c_int64 * n_clusters)()
    _check(lib().nbody_batch_poll(C.c_void_p(b), C.byref(live), t), "nbody_batch_poll")
    return int(live.value), list(t)


def nbody_batch_last_step(b: int, n_clusters: int, act: int = 0, forces: int = 0):
    """Offsets (n_clusters + 1) of the last step's active lists; fills the
    device buffers act / forces when given."""
    aoff = (C.c_int64 * (n_clusters + 1))()
    _check(lib().nbody_batch_last_step(C.c_void_p(b), aoff, C.c_void_p(act or None), C.c_void_p(forces or None)),
           "nbody_batch_last_step")
    return list(aoff)


def nbody_batch_energy(b: int, st: nbody_state, n_clusters: int):
    T = (C.c_double * n_clusters)()
    W = (C.c_double * n_clusters)()
    _check(lib().nbody_batch_energy(C.c_void_p(b), C.byref(st), T, W), "nbody_batch_energy")
    return list(T), list(W)


def nbody_batch_get_stats(b: int) -> nbody_stats:
    s = nbody_stats()
    _check(lib().nbody_batch_get_stats(C.c_void_p(b), C.byref(s)), "nbody_batch_get_stats")
    return s


def nbody_batch_set_launch(b: int, force_grid: int = 0, items_per_wg: int = 0, i_tile: int = 0) -> None:
    _check(lib().nbody_batch_set_launch(C.c_void_p(b), int(force_grid), int(items_per_wg), int(i_tile)),
           "nbody_batch_set_launch")


def nbody_batch_get_launch(b: int):
    """(force_grid, items_per_wg, i_tile) in use."""
    out = (C.c_int32 * 3)()
    _check(lib().nbody_batch_get_launch(C.c_void_p(b), out), "nbody_batch_get_launch")
    return tuple(out)


def nbody_batch_autotune(b: int, st: nbody_state, steps: int = 4) -> None:
    _check(lib().nbody_batch_autotune(C.c_void_p(b), C.byref(st), int(steps)), "nbody_batch_autotune")
