"""ctypes binding of the C oracle (nbody_oracle.c) with NumPy arrays.

Test infrastructure only.  All arrays are float64, 3-vectors component-major
with shape (3, n); times are int64 ticks of 2^-40 time units; levels int32
(a particle on level k has dt = 2^-k, k <= 40).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
TICK_BITS = 40
TICKS_PER_UNIT = 1 << TICK_BITS


def lib_path() -> str:
    return os.path.join(_BUILD, "liboracle.so")


def build() -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off -fopenmp)."""
    os.makedirs(_BUILD, exist_ok=True)
    out = lib_path()
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(
        ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99",
         "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, out)
    return out


class _Config(C.Structure):
    _fields_ = [("order", C.c_int), ("eps2", C.c_double), ("n_hard", C.c_int64),
                ("eta", C.c_double), ("eta_start", C.c_double),
                ("k_min", C.c_int), ("k_max", C.c_int), ("dt_rule", C.c_int),
                ("c_light", C.c_double), ("pn_terms", C.c_int)]


class _State(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_void_p), ("x", C.c_void_p), ("v", C.c_void_p),
                ("d", C.c_void_p * 6), ("t_tick", C.c_void_p), ("level", C.c_void_p)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path()) or os.path.getmtime(lib_path()) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(lib_path())
        P = C.c_void_p
        lib.oracle_force.argtypes = [C.POINTER(_Config), C.c_int64, P, P, P, P, P, C.c_int64, P,
                                     P, P, P, P, P]
        lib.oracle_predict.argtypes = [C.POINTER(_Config), C.POINTER(_State), C.c_int64, P, P, P, P]
        lib.oracle_pn_rel.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, P, P, P, P]
        lib.oracle_pn_rel.restype = None
        lib.oracle_pn_rel_derivs.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, P, P, P]
        lib.oracle_pn_rel_derivs.restype = None
        lib.oracle_pn.argtypes = [C.POINTER(_Config), C.c_int64, P, P, P, C.c_int64, P, P, P, P, P]
        lib.oracle_force_nb.argtypes = [C.POINTER(_Config), C.c_int64, P, P, P, C.c_int64, P, P, C.c_int32,
                                        P, P, P, P, P, P]
        lib.oracle_hermite_high.argtypes = [C.c_int, C.c_double, P, P, P]
        lib.oracle_hermite_high.restype = None
        lib.oracle_hermite_correct.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, P, P, P, P]
        lib.oracle_hermite_correct.restype = None
        lib.oracle_dt_crit.argtypes = [C.c_int, C.c_double, P, C.c_int]
        lib.oracle_dt_crit.restype = C.c_double
        lib.oracle_new_level.argtypes = [C.c_double, C.c_int, C.c_int64, C.c_int, C.c_int]
        lib.oracle_init.argtypes = [C.POINTER(_Config), C.POINTER(_State)]
        lib.oracle_block_step.argtypes = [C.POINTER(_Config), C.POINTER(_State), P, P]
        lib.oracle_block_step.restype = C.c_int64
        lib.oracle_integrate.argtypes = [C.POINTER(_Config), C.POINTER(_State), C.c_int64, C.c_int64, P, P]
        lib.oracle_energy.argtypes = [C.POINTER(_Config), C.c_int64, P, P, P, P, P]
        lib.oracle_num_threads.argtypes = []
        _lib = lib
    return _lib


@dataclass
class OracleConfig:
    order: int = 4
    eps2: float = 1e-8
    n_hard: int = 0
    eta: float = 0.01
    eta_start: float = 0.01
    k_min: int = 3
    k_max: int = 20
    dt_rule: int = 1    # orders 6, 8: 1 = generalised criterion of the order, 2 = its order-4 form
    c_light: float = 0.0  # > 0: post-Newtonian terms between hard particles
    pn_terms: int = 0     # a sum of 1 = 1PN, 2 = 2PN, 4 = 2.5PN

    def _c(self) -> _Config:
        return _Config(self.order, self.eps2, self.n_hard, self.eta, self.eta_start, self.k_min, self.k_max,
                       self.dt_rule, self.c_light, self.pn_terms)


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


@dataclass
class State:
    """Particle state owned by NumPy: m (n,), x, v (3, n), d list of (3, n)
    arrays a^(0..order-3), t_tick (n,) int64, level (n,) int32."""
    m: np.ndarray
    x: np.ndarray
    v: np.ndarray
    order: int
    d: list = field(default_factory=list)
    t_tick: np.ndarray | None = None
    level: np.ndarray | None = None

    def __post_init__(self):
        n = self.m.shape[0]
        self.m = _f64(self.m)
        self.x = _f64(self.x, (3, n))
        self.v = _f64(self.v, (3, n))
        if not self.d:
            self.d = [np.zeros((3, n)) for _ in range(self.order - 2)]
        else:
            self.d = [_f64(a, (3, n)) for a in self.d]
        if self.t_tick is None:
            self.t_tick = np.zeros(n, np.int64)
        if self.level is None:
            self.level = np.zeros(n, np.int32)
        self.t_tick = np.ascontiguousarray(self.t_tick, np.int64)
        self.level = np.ascontiguousarray(self.level, np.int32)

    @property
    def n(self) -> int:
        return self.m.shape[0]

    def copy(self) -> "State":
        return State(self.m.copy(), self.x.copy(), self.v.copy(), self.order,
                     [a.copy() for a in self.d], self.t_tick.copy(), self.level.copy())

    def _c(self) -> _State:
        ds = (C.c_void_p * 6)(*([a.ctypes.data for a in self.d] + [None] * (6 - len(self.d))))
        return _State(self.n, self.m.ctypes.data, self.x.ctypes.data, self.v.ctypes.data, ds,
                      self.t_tick.ctypes.data, self.level.ctypes.data)


def force(cfg: OracleConfig, m, x, v, a=None, jk=None, act=None, with_pot=True):
    """Direct-sum force and derivatives on the active list.

    Returns dict with acc, jrk, snp, crk (each (3, n_act)) and pot (n_act,)."""
    lib = _load()
    m = _f64(m)
    n = m.shape[0]
    x = _f64(x, (3, n))
    v = _f64(v, (3, n))
    a = np.zeros((3, n)) if a is None else _f64(a, (3, n))
    jk = np.zeros((3, n)) if jk is None else _f64(jk, (3, n))
    act = np.arange(n, dtype=np.int32) if act is None else np.ascontiguousarray(act, np.int32)
    na = act.shape[0]
    out = {k: np.zeros((3, na)) for k in ("acc", "jrk", "snp", "crk")}
    out["pot"] = np.zeros(na)
    c = cfg._c()
    lib.oracle_force(C.byref(c), n, _p(m), _p(x), _p(v), _p(a), _p(jk), na, _p(act),
                     _p(out["acc"]), _p(out["jrk"]), _p(out["snp"]), _p(out["crk"]),
                     _p(out["pot"]) if with_pot else None)
    return out


def force_nb(cfg: OracleConfig, m, x, v, act, h2, max_nb: int):
    """Acceleration and jerk on the active list split by neighbour spheres:
    j != i is a neighbour of active row q when |x_j - x_i|^2 < h2[q].
    Returns dict with acc_irr, jrk_irr (sums over the neighbours), acc_reg,
    jrk_reg (over the others), each (3, n_act); nb_count (n_act,) and nb_list
    (n_act, max_nb), the first min(count, max_nb) entries the neighbours in
    increasing index order (-1 beyond)."""
    lib = _load()
    m = _f64(m)
    n = m.shape[0]
    x = _f64(x, (3, n))
    v = _f64(v, (3, n))
    act = np.ascontiguousarray(act, np.int32)
    na = act.shape[0]
    h2 = _f64(h2, (na,))
    out = {k: np.zeros((3, na)) for k in ("acc_irr", "jrk_irr", "acc_reg", "jrk_reg")}
    out["nb_count"] = np.zeros(na, np.int32)
    out["nb_list"] = np.full((na, max(int(max_nb), 1)), -1, np.int32)
    lib.oracle_force_nb(C.byref(cfg._c()), n, _p(m), _p(x), _p(v), na, _p(act), _p(h2), int(max_nb),
                        _p(out["acc_irr"]), _p(out["jrk_irr"]), _p(out["acc_reg"]), _p(out["jrk_reg"]),
                        _p(out["nb_count"]), _p(out["nb_list"]))
    return out


def pn_rel(M: float, nu: float, c: float, terms: int, x, v):
    """Post-Newtonian part of the two-body relative acceleration (1PN: terms
    & 1, 2PN: terms & 2, 2.5PN: terms & 4) at relative position x and
    velocity v, and its time derivative along the Newtonian two-body motion."""
    lib = _load()
    x = _f64(x, (3,))
    v = _f64(v, (3,))
    a = np.zeros(3)
    j = np.zeros(3)
    lib.oracle_pn_rel(float(M), float(nu), float(c), int(terms), _p(x), _p(v), _p(a), _p(j))
    return a, j


def pn_rel_derivs(M: float, nu: float, c: float, terms: int, x, v) -> np.ndarray:
    """(4, 3): the post-Newtonian part of the two-body relative acceleration
    and its first three time derivatives along the Newtonian two-body motion."""
    lib = _load()
    x = _f64(x, (3,))
    v = _f64(v, (3,))
    out = np.zeros((4, 3))
    lib.oracle_pn_rel_derivs(float(M), float(nu), float(c), int(terms), _p(x), _p(v), _p(out))
    return out


def pn(cfg: OracleConfig, m, x, v, act, acc, jrk, snp=None, crk=None):
    """Adds the post-Newtonian terms of the hard pairs to acc, jrk (and snp,
    crk when given) ((3, n_act) arrays, modified in place) for the active
    list."""
    lib = _load()
    m = _f64(m)
    n = m.shape[0]
    x = _f64(x, (3, n))
    v = _f64(v, (3, n))
    act = np.ascontiguousarray(act, np.int32)
    assert acc.dtype == np.float64 and acc.flags.c_contiguous and jrk.flags.c_contiguous
    for a in (snp, crk):
        assert a is None or (a.dtype == np.float64 and a.flags.c_contiguous)
    lib.oracle_pn(C.byref(cfg._c()), n, _p(m), _p(x), _p(v), act.shape[0], _p(act), _p(acc), _p(jrk), _p(snp),
                  _p(crk))


def predict(cfg: OracleConfig, s: State, t_tick: int):
    lib = _load()
    n = s.n
    xp, vp, ap, jp = (np.zeros((3, n)) for _ in range(4))
    cs = s._c()
    lib.oracle_predict(C.byref(cfg._c()), C.byref(cs), int(t_tick), _p(xp), _p(vp), _p(ap), _p(jp))
    return xp, vp, ap, jp


def hermite_high(p: int, h: float, D0, D1) -> np.ndarray:
    lib = _load()
    D0 = _f64(D0)
    D1 = _f64(D1)
    H = np.zeros(p // 2)
    lib.oracle_hermite_high(p, h, _p(D0), _p(D1), _p(H))
    return H


def hermite_correct(p: int, h: float, x0: float, v0: float, D0, D1):
    lib = _load()
    D0 = _f64(D0)
    D1 = _f64(D1)
    x1 = np.zeros(1)
    v1 = np.zeros(1)
    lib.oracle_hermite_correct(p, h, x0, v0, _p(D0), _p(D1), _p(x1), _p(v1))
    return float(x1[0]), float(v1[0])


def dt_crit(p: int, eta: float, F, rule: int = 1) -> float:
    """Time-step criterion from |a^(k)|, k = 0 .. p-1 (rule: see OracleConfig)."""
    F = _f64(F)
    return float(_load().oracle_dt_crit(p, eta, _p(F), int(rule)))


def new_level(dtc: float, level_old: int, t1_tick: int, k_min: int, k_max: int) -> int:
    return int(_load().oracle_new_level(dtc, level_old, t1_tick, k_min, k_max))


def init(cfg: OracleConfig, s: State) -> State:
    lib = _load()
    cs = s._c()
    if lib.oracle_init(C.byref(cfg._c()), C.byref(cs)) != 0:
        raise MemoryError("oracle_init")
    return s


def block_step(cfg: OracleConfig, s: State):
    """One block step in place.  Returns (n_act, t_next, stats[under, nonfinite])."""
    lib = _load()
    t_next = np.zeros(1, np.int64)
    stats = np.zeros(2, np.int64)
    cs = s._c()
    na = lib.oracle_block_step(C.byref(cfg._c()), C.byref(cs), _p(t_next), _p(stats))
    if na < 0:
        raise MemoryError("oracle_block_step")
    return int(na), int(t_next[0]), stats


def integrate(cfg: OracleConfig, s: State, t_end_tick: int, max_steps: int = 1 << 62):
    """Block-step integration in place to t_end_tick.  Returns dict of counters."""
    lib = _load()
    out = np.zeros(5, np.int64)
    hist = np.zeros(21, np.int64)
    cs = s._c()
    if lib.oracle_integrate(C.byref(cfg._c()), C.byref(cs), int(t_end_tick), int(max_steps),
                            _p(out), _p(hist)) != 0:
        raise MemoryError("oracle_integrate")
    return {"steps": int(out[0]), "sum_nact": int(out[1]), "interactions": int(out[2]),
            "underflow": int(out[3]), "nonfinite": int(out[4]), "nact_hist": hist}


def energy(cfg: OracleConfig, m, x, v):
    """(T, W) kinetic and potential energy, FP64 pairwise."""
    lib = _load()
    m = _f64(m)
    n = m.shape[0]
    x = _f64(x, (3, n))
    v = _f64(v, (3, n))
    T = np.zeros(1)
    W = np.zeros(1)
    lib.oracle_energy(C.byref(cfg._c()), n, _p(m), _p(x), _p(v), _p(T), _p(W))
    return float(T[0]), float(W[0])


def num_threads() -> int:
    return int(_load().oracle_num_threads())
