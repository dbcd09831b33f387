"""Pins of the oracle's transport loop: Alg. 1, Beer-Lambert, energy conservation."""
import math

import numpy as np
import pytest
from scipy import stats

import workloads as W

ME = 0.51099895


def _slab_hits(p, d, lo, hi):
    """Ray-slab entry/exit distances for axis-aligned boxes (independent helper)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (lo - p) / d
        t2 = (hi - p) / d
    tn = np.nanmax(np.minimum(t1, t2), axis=-1)
    tf = np.nanmin(np.maximum(t1, t2), axis=-1)
    return tn, tf


def test_alg1_regular_lifetime_one(oracle_lib):
    """Sec. 3.5 Regular setup: Y = 1 for every particle.  Along fixed rays of the
    tiny geometry, T = t_M + (1 - S_M) / mu_{M+1} (Eq. 7) from analytic slab
    intersections and the material attenuation at 1 MeV."""
    desc = W.geometry.tiny()
    g = oracle_lib.Geometry(desc)
    mu = {m: g.mu(i, [1.0])[0].sum() for i, m in enumerate(desc.mat_names)}
    rng = np.random.Generator(np.random.Philox(key=8))
    dirs = W.primaries.isotropic(rng, 400)
    checked = 0
    for d in dirs:
        # segments crossed by the ray from the origin, in order
        segs = []
        for k in range(8):
            c = desc.pv_trans[k]
            tn, tf = _slab_hits(np.zeros(3), d, c - 100, c + 100)
            if tf > max(tn, 0):
                mat = desc.mat_names[desc.lv_mat[desc.pv_lv[k]]]
                segs.append((tn, tf, mu[mat]))
        segs.sort()
        S, T_ref = 0.0, math.inf
        for tn, tf, m in segs:
            if S + (tf - tn) * m >= 1.0:
                T_ref = tn + (1.0 - S) / m
                break
            S += (tf - tn) * m
        T, nb = g.free_path(np.zeros(3), d, 1.0, 1.0)
        if T_ref == math.inf:
            assert T == math.inf
        else:
            assert abs(T - T_ref) <= 1e-12 * T_ref
            checked += 1
    assert checked > 20


def test_alg1_paper_mode_aluminium(oracle_lib):
    """mu = rho * mu_Al (Eq. 9): an aluminium ball of radius R at distance D,
    Y small enough to interact inside -> T = D - R + Y / (rho mu_Al)."""
    desc = W.geometry.spheres(n_per_axis=2, radius=100.0, half=500.0)
    g = oracle_lib.Geometry(desc)
    g.set_paper_mode(True, 0.06146)
    mu = 2.699 * 0.06146 * 0.1  # 1/mm
    c = desc.pv_trans[0]
    d = c / np.linalg.norm(c)
    Y = 0.5
    T, _ = g.free_path(np.zeros(3), d, 1.0, Y)
    assert abs(T - (np.linalg.norm(c) - 100 + Y / mu)) < 1e-11 * T


@pytest.mark.parametrize("name,n", [("tiny", 4000), ("calorimeter", 3000), ("barrel", 1500), ("endcap", 3000)])
def test_energy_conservation_per_event(oracle_lib, name, n):
    geoms, prim, _ = W.WORKLOADS[name](n=n)
    g = oracle_lib.Geometry(geoms[0])
    r = g.transport(prim, seed=0)
    assert r["counters"]["truncated"] == 0
    tot = r["edep_event"] + r["escaped_event"]
    assert np.allclose(tot, prim.energy, rtol=1e-12, atol=0)
    assert abs(r["edep_touchable"].sum() - r["edep_event"].sum()) <= 1e-10 * prim.energy.sum()
    c = r["counters"]
    # every track ends exactly once
    ends = c["pe"] + c["pair"] + c["escaped"] + c["cutoff"] + c["stuck"]
    assert ends == c["tracks"]
    assert c["tracks"] == n + 2 * c["pair"]


def test_beer_lambert_uncollided_fraction(oracle_lib):
    """Eqs. 1-3: the uncollided fraction of a pencil beam through a slab of
    thickness L is exp(-mu L).  Binomial test at 5 sigma."""
    L = 50.0
    desc = W.geometry.slab("water", L)
    g = oracle_lib.Geometry(desc)
    mu = g.mu(desc.mat_names.index("water"), [1.0])[0].sum()
    n = 200_000
    prim = W.primaries.pencil(n, (0.0, 0.0, -900.0), (0, 0, 1), 1.0)
    r = g.transport(prim, seed=3, log_cap=3)
    log = r["log"][0::3]
    # uncollided: world step into the slab, then a mother-limited exit from it
    unc = (log["code"][:, 0] == 0) & (log["touchable"][:, 1] == 1) & (log["code"][:, 1] == -1)
    p = math.exp(-mu * L)
    k = unc.sum()
    assert abs(k - n * p) < 5 * math.sqrt(n * p * (1 - p))
    # first-interaction depth inside the slab: truncated exponential (KS)
    inter = (log["touchable"][:, 1] == 1) & (log["code"][:, 1] < -1)
    depth = log["step"][inter, 1]
    cdf = lambda x: (1 - np.exp(-mu * x)) / (1 - math.exp(-mu * L))
    assert stats.kstest(depth, cdf).pvalue > 1e-3


def test_first_step_hits_daughters_fraction(oracle_lib):
    """Isotropic rays from the centre of the tiny geometry enter a cube with a
    probability computed independently by slab tests on 2e6 rays."""
    rng = np.random.Generator(np.random.Philox(key=77))
    d = W.primaries.isotropic(rng, 2_000_000)
    desc = W.geometry.tiny()
    hit = np.zeros(len(d), bool)
    for k in range(8):
        c = desc.pv_trans[k]
        tn, tf = _slab_hits(np.zeros(3), d, c - 100, c + 100)
        hit |= tf > np.maximum(tn, 0)
    p_ref = hit.mean()
    geoms, prim, _ = W.tiny(n=10_000, seed=0)
    g = oracle_lib.Geometry(geoms[0])
    r = g.transport(prim, log_cap=1)
    first = r["log"]["code"][0::3, 0]
    p = (first >= 0).mean()
    n = len(first)
    assert abs(p - p_ref) < 5 * math.sqrt(p_ref * (1 - p_ref) / n) + 5 * math.sqrt(
        p_ref * (1 - p_ref) / len(d))


def test_log_replays_track(oracle_lib):
    """Per-track logs are self-consistent: steps sum along straight segments,
    energies drop only at Compton steps, deposits match the event tally."""
    geoms, prim, _ = W.calorimeter(n=500)
    g = oracle_lib.Geometry(geoms[0])
    r = g.transport(prim, log_cap=512)
    assert r["log_n"].max() <= 512
    dep = np.zeros(prim.n_events)
    for s in range(3 * prim.n):
        n = r["log_n"][s]
        if n == 0:
            continue
        rec = r["log"][s, :n]
        dep[s // 3] += rec["edep"].sum()
        geo = rec["code"] >= -1
        assert np.all(rec["step"] >= 0)
        assert np.all(rec["edep"][geo] == 0)
    cut = r["edep_event"] - dep  # cutoff and stuck deposits are not logged as steps
    assert np.all(cut >= -1e-12)
    assert np.all(cut < 1e-3 + 1e-12)
