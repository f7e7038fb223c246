"""Pins of the oracle's neighbour-split force (Ahmad & Cohen 1973; the scheme
of the paper's second code, NBODY6++GPU, Sec. "Results"): particle j != i is a
neighbour of i when its unsoftened squared distance is below h_i^2; the
acceleration and jerk are summed separately over the neighbours (irregular
part) and the other particles (regular part).

Pinned by routes other than the function itself:
* neighbour sets against a brute-force distance check in numpy, with radii
  placed in the middle of gaps of the sorted distances (no pair near a
  sphere's surface, so the set is the same in any precision);
* each part against the already pinned full-force oracle run on a subsystem:
  particle i with only its neighbours (irregular), or with only the others
  (regular);
* a three-body line configuration in closed form;
* the list-length cap.
"""
import numpy as np

import nbody_ics
import oracle
from helpers import band_free_radii
from oracle import OracleConfig


def _case(n=400, seed=5, n_act=48):
    model = nbody_ics.plummer(n, seed)
    act = nbody_ics.active_subset(n, n_act, seed + 1)
    h2, margin = band_free_radii(model.x, act, seed + 2)
    return model, act, h2, margin


def test_neighbour_sets_match_brute_force():
    model, act, h2, margin = _case()
    assert margin.min() > 1e-6
    out = oracle.force_nb(OracleConfig(order=4, eps2=1e-4), model.m, model.x, model.v, act, h2, 64)
    for q, i in enumerate(act):
        d2 = np.sum((model.x - model.x[:, i:i + 1]) ** 2, axis=0)
        want = np.array([j for j in range(model.n) if j != i and d2[j] < h2[q]], np.int32)
        assert out["nb_count"][q] == want.size
        np.testing.assert_array_equal(out["nb_list"][q, : want.size], want)
        assert np.all(out["nb_list"][q, want.size:] == -1)
    assert out["nb_count"].max() > 10


def test_parts_are_forces_of_subsystems():
    """Irregular part of i = full force on i in the system {i} + neighbours;
    regular part = full force on i in {i} + the others (index order kept, so
    the sums run in the same order)."""
    model, act, h2, margin = _case()
    cfg = OracleConfig(order=4, eps2=1e-4)
    out = oracle.force_nb(cfg, model.m, model.x, model.v, act, h2, 400)
    for q in range(0, act.size, 5):
        i = int(act[q])
        nb = out["nb_list"][q, : out["nb_count"][q]]
        others = np.setdiff1d(np.arange(model.n), np.append(nb, i))
        for part, members in (("irr", nb), ("reg", others)):
            sub = np.sort(np.append(members, i))
            pos = int(np.searchsorted(sub, i))
            full = oracle.force(cfg, model.m[sub], model.x[:, sub], model.v[:, sub], act=np.array([pos]),
                                with_pot=False)
            np.testing.assert_allclose(out["acc_" + part][:, q], full["acc"][:, 0], rtol=1e-14, atol=0)
            np.testing.assert_allclose(out["jrk_" + part][:, q], full["jrk"][:, 0], rtol=1e-14, atol=0)


def test_parts_add_up_to_full_force():
    model, act, h2, margin = _case(n=300, seed=9, n_act=30)
    cfg = OracleConfig(order=4, eps2=1e-4)
    out = oracle.force_nb(cfg, model.m, model.x, model.v, act, h2, 300)
    full = oracle.force(cfg, model.m, model.x, model.v, act=act, with_pot=False)
    for key in ("acc", "jrk"):
        tot = out[key + "_irr"] + out[key + "_reg"]
        err = np.linalg.norm(tot - full[key], axis=0) / np.linalg.norm(full[key], axis=0)
        assert err.max() < 1e-12, (key, err.max())


def test_three_bodies_on_a_line_closed_form():
    """Bodies at x = 0, 1, 3 (masses 1, 2, 5), unsoftened; body 0 with h^2 = 2
    has the neighbour 1.  With r along x and w = v_j - v_0:
    A = m r / r^3, J = m (w / r^3 - 3 (r.w) r / r^5)."""
    m = np.array([1.0, 2.0, 5.0])
    x = np.array([[0.0, 1.0, 3.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    v = np.array([[0.0, 0.5, 0.0], [0.0, 0.0, 0.25], [0.0, 0.0, 0.0]])
    out = oracle.force_nb(OracleConfig(order=4, eps2=0.0), m, x, v, np.array([0]), np.array([2.0]), 4)
    assert out["nb_count"][0] == 1 and out["nb_list"][0, 0] == 1
    np.testing.assert_allclose(out["acc_irr"][:, 0], [2.0, 0.0, 0.0], rtol=1e-15)
    np.testing.assert_allclose(out["jrk_irr"][:, 0], [2.0 * (0.5 - 3.0 * 0.5), 0.0, 0.0], rtol=1e-15)
    np.testing.assert_allclose(out["acc_reg"][:, 0], [5.0 * 3.0 / 27.0, 0.0, 0.0], rtol=1e-15)
    np.testing.assert_allclose(out["jrk_reg"][:, 0], [0.0, 5.0 * 0.25 / 27.0, 0.0], rtol=1e-15, atol=1e-300)


def test_list_cap_keeps_the_true_count():
    model, act, h2, margin = _case(n=300, seed=13, n_act=20)
    cfg = OracleConfig(order=4, eps2=1e-4)
    full = oracle.force_nb(cfg, model.m, model.x, model.v, act, h2, 300)
    capped = oracle.force_nb(cfg, model.m, model.x, model.v, act, h2, 5)
    none = oracle.force_nb(cfg, model.m, model.x, model.v, act, h2, 0)
    np.testing.assert_array_equal(capped["nb_count"], full["nb_count"])
    np.testing.assert_array_equal(none["nb_count"], full["nb_count"])
    for q in range(act.size):
        k = min(5, full["nb_count"][q])
        np.testing.assert_array_equal(capped["nb_list"][q, :k], full["nb_list"][q, :k])
    for key in ("acc_irr", "jrk_irr", "acc_reg", "jrk_reg"):
        np.testing.assert_array_equal(capped[key], full[key])
