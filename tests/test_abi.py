"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol include/nbody.h declares, and validates arguments before any
device work."""
import ctypes as C
import os
import re

import pytest

from paper_1312_1789_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "nbody.h")).read()
    return sorted(set(re.findall(r"\b(nbody_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = abi.lib()
    declared = _header_symbols()
    assert set(declared) == set(abi.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def _cfg(**kw):
    base = dict(order=6, precision=abi.NBODY_MIXED, n=1000, n_hard=0, eps2=1e-8, eta=0.1, eta_start=0.01,
                k_min=3, k_max=20, dt_rule=0, c_light=0.0, pn_terms=0)
    base.update(kw)
    return abi.nbody_config(base["order"], base["precision"], base["n"], base["n_hard"], base["eps2"],
                            base["eta"], base["eta_start"], base["k_min"], base["k_max"], base["dt_rule"],
                            base["c_light"], base["pn_terms"])


def test_workspace_size_scales_with_n():
    a = abi.nbody_workspace_size(_cfg(n=1000))
    b = abi.nbody_workspace_size(_cfg(n=100000))
    assert b > a > 0
    # FP64 records are larger than MIXED ones at order 6
    assert abi.nbody_workspace_size(_cfg(precision=abi.NBODY_FP64, n=100000)) > b


@pytest.mark.parametrize("kw", [dict(order=5), dict(order=10), dict(precision=3), dict(n=1), dict(n_hard=2000),
                                dict(eps2=-1.0), dict(eta=0.0), dict(eta_start=-1.0), dict(k_min=5, k_max=4),
                                dict(k_max=41), dict(eps2=float("nan")), dict(dt_rule=3), dict(dt_rule=-1),
                                dict(c_light=-1.0), dict(c_light=float("inf")), dict(pn_terms=8),
                                dict(pn_terms=-1), dict(order=4, n=5000, n_hard=2000, c_light=10.0, pn_terms=1)])
def test_config_validation(kw):
    with pytest.raises(abi.NBodyError) as e:
        abi.nbody_workspace_size(_cfg(**kw))
    assert e.value.status == abi.NBODY_E_INVALID
    assert abi.last_error()


def test_create_rejects_bad_workspace():
    cfg = _cfg()
    n = abi.nbody_workspace_size(cfg)
    with pytest.raises(abi.NBodyError) as e:
        abi.nbody_create(cfg, 0, n)
    assert e.value.status == abi.NBODY_E_WORKSPACE
    with pytest.raises(abi.NBodyError) as e:
        abi.nbody_create(cfg, 256 * 1000 + 8, n)       # misaligned
    assert e.value.status == abi.NBODY_E_WORKSPACE
    with pytest.raises(abi.NBodyError) as e:
        abi.nbody_create(cfg, 256 * 1000, n - 1)       # too small
    assert e.value.status == abi.NBODY_E_WORKSPACE


def test_null_context_is_rejected():
    L = abi.lib()
    assert L.nbody_destroy(None) == abi.NBODY_E_INVALID
    assert L.nbody_step(None, None, None, None) == abi.NBODY_E_INVALID
    assert L.nbody_set_launch(None, 1, 256, 0, 0) == abi.NBODY_E_INVALID
    assert L.nbody_get_predicted(None, None, None, None, None) == abi.NBODY_E_INVALID
    assert L.nbody_autotune(None, 16, 1) == abi.NBODY_E_INVALID
    assert L.nbody_get_tuning(None, 0, None, None, None, None) == abi.NBODY_E_INVALID
    assert L.nbody_set_fusion(None, 1) == abi.NBODY_E_INVALID
    assert L.nbody_force_block_nb(None, 0, None, None, 0, None, None, None, None, None, None) == abi.NBODY_E_INVALID
    assert L.nbody_predict_force(None, None, 0, 0, None, None, None, None, None, None) == abi.NBODY_E_INVALID


def test_batch_workspace_size():
    off = [0, 1000, 3000, 3002]
    a = abi.nbody_batch_workspace_size(_cfg(n=3002), off)
    b = abi.nbody_batch_workspace_size(_cfg(n=6002), off[:-1] + [3002, 6002])
    assert b > a > 0


@pytest.mark.parametrize("off,kw", [
    ([0, 1000, 999], dict(n=999)),           # decreasing offsets
    ([0, 1, 1000], dict(n=1000)),            # a one-particle cluster
    ([1, 500, 1000], dict(n=1000)),          # off[0] != 0
    ([0, 500, 1000], dict(n=1001)),          # last offset != n
    ([0, 500, 1000], dict(n=1000, n_hard=501)),   # n_hard beyond a cluster
    ([0, 500, 1000], dict(n=1000, order=7)),
    ([0], dict(n=1000)),                     # no clusters
])
def test_batch_validation(off, kw):
    with pytest.raises(abi.NBodyError) as e:
        abi.nbody_batch_workspace_size(_cfg(**kw), off)
    assert e.value.status == abi.NBODY_E_INVALID
    assert abi.last_error()


def test_pn_config_accepted_and_refused_in_batches():
    for order in (4, 6, 8):
        assert abi.nbody_workspace_size(_cfg(order=order, n_hard=2, c_light=10.0, pn_terms=5)) > 0
    with pytest.raises(abi.NBodyError) as e:
        abi.nbody_batch_workspace_size(_cfg(order=4, n_hard=2, c_light=10.0, pn_terms=4), [0, 500, 1000])
    assert e.value.status == abi.NBODY_E_UNSUPPORTED


def test_batch_too_uneven_is_unsupported():
    # one cluster of 2^23 and 65534 pairs: 8192 scheduling blocks x 65535 cells
    off = [0, 1 << 23] + [(1 << 23) + 2 * (k + 1) for k in range(65534)]
    with pytest.raises(abi.NBodyError) as e:
        abi.nbody_batch_workspace_size(_cfg(n=off[-1]), off)
    assert e.value.status == abi.NBODY_E_UNSUPPORTED


def test_batch_null_handles_are_rejected():
    L = abi.lib()
    assert L.nbody_batch_destroy(None) == abi.NBODY_E_INVALID
    assert L.nbody_batch_step(None, None, 1) == abi.NBODY_E_INVALID
    assert L.nbody_batch_replay(None, 1) == abi.NBODY_E_INVALID
    assert L.nbody_batch_set_launch(None, 0, 0, 0) == abi.NBODY_E_INVALID
    assert L.nbody_batch_autotune(None, None, 1) == abi.NBODY_E_INVALID
    assert L.nbody_batch_poll(None, None, None) == abi.NBODY_E_INVALID
