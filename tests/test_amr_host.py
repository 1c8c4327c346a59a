"""The library's host steps of hp-adaptation (Alg. hpamr: marking, smooth-pred decisions, mesh
adaptation with 2:1 restoration) against the oracle's decisions and an independent octree
adaptation; no device is used."""
import os

import numpy as np
import pytest

import meshgen
from oracle import estimator as est
from oracle.operator import SIPG

hp = pytest.importorskip("paper_1907_01572_amd")
if not os.path.exists(hp.LIB_PATH):
    pytest.skip("library not built", allow_module_level=True)


def _eta2(n, seed, ties=True):
    rng = np.random.default_rng(seed)
    e = rng.lognormal(0.0, 2.0, n)
    if ties:  # repeated values: the order among equal keys is part of the contract
        e[rng.integers(0, n, n // 4)] = e[0]
    return e


@pytest.mark.parametrize("n", [1, 7, 30, 1000])
def test_mark_matches_oracle(n):
    for seed in range(3):
        e = _eta2(n, seed)
        for frac in (0.0, 0.1, 0.25, 0.5, 1.0):
            assert np.array_equal(hp.amr_mark(e, hp.MARK_FRACTION, frac), est.mark_fraction(e, frac)), (n, frac)
        for fac in (0.25, 1.0, 3.0):
            assert np.array_equal(hp.amr_mark(e, hp.MARK_MEAN, fac), est.mark_mean(e, fac))
    # 0.1 x 30 rounds above 3 in binary: three elements, not four
    assert hp.amr_mark(_eta2(30, 0), hp.MARK_FRACTION, 0.1).sum() == 3


def test_smooth_pred_matches_oracle():
    rng = np.random.default_rng(4)
    n = 500
    for step in range(3):
        e = _eta2(n, 10 + step, ties=False)
        pred = np.where(rng.random(n) < 0.3, np.inf, e * rng.lognormal(0.0, 1.0, n))
        p = rng.integers(1, 9, n)
        marked = rng.random(n) < 0.4
        for gh, gp in ((0.25, 0.1), (10.0, 0.1)):
            a, pr = hp.amr_smooth_pred(e, pred, p, marked, gh, gp)
            ao, pro = est.smooth_pred(e, pred, p, marked, gamma_h=gh, gamma_p=gp)
            assert np.array_equal(a, ao)
            assert np.array_equal(pr, pro)


def _cells(mesh):
    return list(zip(mesh["elem_macro"].tolist(), mesh["elem_level"].tolist(),
                    map(tuple, mesh["elem_anchor"].tolist()), mesh["elem_p"].tolist()))


MESHES = {
    "box_2to1": lambda: meshgen.box_grid((2, 1, 1), 1, 3, refine=[lambda k, c0, c1: k[1] == 1 and c1.max() <= 0.5]),
    "hp_sphere": lambda: meshgen.hp_sphere_cube(level=2, p_lo=1, p_hi=5, seed=2, r_cut=0.6),
    "shell": lambda: meshgen.cubed_sphere_shell(level=1, p=2, r_out=1e3),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_adapt_matches_octree_adaptation(name):
    m = MESHES[name]()
    rng = np.random.default_rng(7)
    for step in range(3):
        E = len(m["elem_p"])
        act = rng.choice([0, 1, 2], size=E, p=[0.8, 0.1, 0.1]).astype(np.int8)
        new, origin = hp.amr_adapt(m, act, max_degree=6)
        ref, origin_ref = meshgen.adapt(m, act, max_p=6)
        assert _cells(new) == _cells(ref)
        assert np.array_equal(origin, origin_ref)
        # every marked cell was refined as asked; the volume of each macro is kept
        for e in np.flatnonzero(act == 1):
            assert all(new["elem_level"][origin == e] > m["elem_level"][e])
        for e in np.flatnonzero(act == 2):
            kids = origin == e
            assert np.all(new["elem_p"][kids] == min(m["elem_p"][e] + 1, max(6, m["elem_p"][e])))
        for mac in range(len(m["macro_kind"])):
            assert np.isclose(np.sum(0.125 ** new["elem_level"][new["elem_macro"] == mac]), 1.0)
        # the oracle builds its mortars on the result (it refuses meshes that are not 2:1)
        SIPG(new, meshgen.problem_config1())
        m = new
        print(name, "step", step, "elements", len(m["elem_p"]), flush=True)


def test_adapt_errors():
    m = MESHES["box_2to1"]()
    E = len(m["elem_p"])
    with pytest.raises(hp.HpdgError) as ei:
        hp.amr_adapt(m, np.full(E, 3, np.int8))
    assert ei.value.code == hp.ERR_INVALID_ARG
    bad = dict(m)
    bad["elem_level"] = m["elem_level"].copy()
    bad["elem_level"][0] += 2  # a cell outside the forest: unmatched faces
    with pytest.raises(hp.HpdgError) as ei:
        hp.amr_adapt(bad, np.zeros(E, np.int8))
    assert ei.value.code == hp.ERR_INVALID_MESH
    with pytest.raises(hp.HpdgError) as ei:
        hp.amr_mark(np.ones(3), hp.MARK_FRACTION, 1.5)
    assert ei.value.code == hp.ERR_INVALID_ARG
