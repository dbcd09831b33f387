"""Pins of the oracle's rarely taken transport branches.

* energy cut (1 keV in the configs; raised here so it fires): a photon below
  the cut deposits its energy in its current touchable and stops, checked
  before every step, strictly below the cut;
* pair conversion: both annihilation photons start at the conversion point
  with m_e c^2, exactly back to back, with isotropic directions;
* zero-length steps: on a stack of foils thinner than the tolerance every
  step is shorter than it, so a track is pushed 100 tolerances along its
  direction after the 10th and the 20th consecutive zero step and killed at
  the 25th; the touchables it visits follow from the foil geometry alone.
"""
import math

import numpy as np
from scipy import stats

import workloads as W

ME = 0.51099895


def _one(pos, d, E):
    return W.primaries.one_per_event(np.atleast_2d(pos).astype(float), np.atleast_2d(d).astype(float),
                                     np.atleast_1d(E).astype(float))


def test_cut_is_strict_and_deposits_where_the_track_is(oracle_lib):
    og = oracle_lib.Geometry(W.geometry.slab("water"))
    ecut = 0.2
    below = math.nextafter(ecut, 0.0)
    prim = _one([[0, 0, -1.0], [0, 0, -1.0]], [[0, 0, 1.0], [0, 0, 1.0]], [below, ecut])
    r = og.transport(prim, seed=0, ecut=ecut, log_cap=64)
    # below the cut at the start: no step at all, the energy stays in the slab
    assert r["log_n"][0] == 0 and r["log_fate"][0] == oracle_lib.FATE_CUTOFF
    assert r["edep_event"][0] == below and r["edep_touchable"][1] >= below
    # exactly at the cut: transported (it takes at least one step; a later scatter may
    # still take it below the cut)
    assert r["log_n"][3] >= 1 and r["log"][3, 0]["step"] > 0
    assert r["counters"]["cutoff"] >= 1


def test_cut_after_compton(oracle_lib):
    """Photons of 0.3 MeV in water with a 0.2 MeV cut: a track ends by the cut
    exactly when a Compton scatter leaves it below 0.2 MeV; that last energy is
    deposited in the touchable of the scatter."""
    og = oracle_lib.Geometry(W.geometry.slab("water", thickness=400.0))
    n = 3000
    rng = np.random.default_rng(3)
    prim = _one(np.tile([0, 0, -150.0], (n, 1)), W.primaries.isotropic(rng, n), np.full(n, 0.3))
    ecut = 0.2
    r = og.transport(prim, seed=5, ecut=ecut, log_cap=256)
    cut = np.nonzero(r["log_fate"] == oracle_lib.FATE_CUTOFF)[0]
    assert len(cut) > 300
    assert r["counters"]["cutoff"] == len(cut)
    for s in range(3 * n):
        k = r["log_n"][s]
        if r["log_fate"][s] == 0 or k == 0:
            continue
        rec = r["log"][s, :k]
        live = rec["energy"][:-1]
        assert np.all(live >= ecut), s  # no step starts below the cut
        if r["log_fate"][s] == oracle_lib.FATE_CUTOFF:
            assert rec["code"][-1] == oracle_lib.LIM_COMPTON and rec["energy"][-1] < ecut
            ev = prim.event[s // 3]
            # event deposit = the logged deposits + the energy left at the cut
            want = rec["edep"].sum() + rec["energy"][-1]
            assert abs(r["edep_event"][ev] - want) <= 1e-12 * want
        elif rec["code"][-1] == oracle_lib.LIM_COMPTON:
            assert rec["energy"][-1] >= ecut  # a scatter that stays above the cut continues
    tot = r["edep_event"] + r["escaped_event"]
    assert np.allclose(tot, prim.energy, rtol=1e-12, atol=0)


def test_pair_photons_back_to_back_isotropic(oracle_lib):
    desc = W.geometry.slab("lead", thickness=200.0)
    og = oracle_lib.Geometry(desc)
    n = 20000
    prim = _one(np.tile([0, 0, -150.0], (n, 1)), np.tile([0, 0, 1.0], (n, 1)), np.full(n, 20.0))
    r = og.transport(prim, seed=0, log_cap=4, want_start=True)
    st = r["start"]
    conv = np.nonzero(r["log_fate"][0::3] == oracle_lib.FATE_PAIR)[0]
    assert len(conv) > 5000
    a, b = st[3 * conv + 1], st[3 * conv + 2]
    # both at the conversion point (the end of the primary's last logged step)
    assert np.array_equal(a[:, :3], b[:, :3])
    assert np.all(a[:, 6] == ME) and np.all(b[:, 6] == ME)
    assert np.array_equal(a[:, 3:6], -b[:, 3:6])
    assert np.allclose(np.linalg.norm(a[:, 3:6], axis=1), 1.0, atol=1e-15)
    # isotropic: cos(theta) uniform on [-1, 1], phi uniform on (-pi, pi]
    assert stats.kstest(a[:, 5], "uniform", args=(-1, 2)).pvalue > 1e-3
    phi = np.arctan2(a[:, 4], a[:, 3])
    assert stats.kstest(phi, "uniform", args=(-math.pi, 2 * math.pi)).pvalue > 1e-3
    # the conversion point lies inside the slab
    assert np.all(np.abs(a[:, 2]) <= 100.0 + 1e-9)


def _foil_path():
    """Touchables a photon along +z visits in the foil stack (world = 0, foil k =
    1 + k): the world step to foil 0; ten zero steps through foils 0-9; a push of
    1e-7 mm from the top of foil 9 into foil 10 + floor(1e-7 / 9e-10) = 121;
    foils 121-130; a second push into foil 131 + 111 = 242; foils 242-246, where
    the 25th zero step kills it."""
    t = 9e-10
    first = 10 + int(1e-7 // t)
    second = first + 10 + int(1e-7 // t)
    foils = list(range(0, 10)) + list(range(first, first + 10)) + list(range(second, second + 5))
    return [0] + [1 + k for k in foils]


def test_zero_steps_push_and_kill(oracle_lib):
    desc = W.geometry.foil_stack()
    og = oracle_lib.Geometry(desc)
    n = 200
    rng = np.random.default_rng(9)
    pos = np.stack([rng.uniform(-5, 5, n), rng.uniform(-5, 5, n), np.full(n, -50.0)], 1)
    prim = _one(pos, np.tile([0, 0, 1.0], (n, 1)), np.full(n, 1.0))
    r = og.transport(prim, seed=0, log_cap=64)
    path = _foil_path()
    assert path[11] == 122 and path[21] == 243  # foils 121 and 242
    c = r["counters"]
    assert c["stuck"] == n and c["pushes"] == 2 * n and c["steps"] == 26 * n
    for i in range(n):
        k = r["log_n"][3 * i]
        rec = r["log"][3 * i, :k]
        assert r["log_fate"][3 * i] == oracle_lib.FATE_STUCK
        assert list(rec["touchable"]) == path, i
        assert rec["code"][0] == 0 and np.all(rec["code"][1:] == oracle_lib.LIM_MOTHER)
        assert np.all(rec["step"][1:] < 1e-9) and rec["step"][0] > 49.0
    # the killed track leaves its energy in the last foil
    assert np.allclose(r["edep_touchable"][path[-1]], n * 1.0)
    assert np.allclose(r["edep_event"], 1.0, rtol=0, atol=0)
