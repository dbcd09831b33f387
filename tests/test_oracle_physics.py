"""Pins of the oracle's photon physics: cross sections, tables, Compton sampling."""
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

import workloads as W

ME = 0.51099895
RE = 2.8179403262e-13  # cm
NA = 6.02214076e23
THOMSON = 8.0 * math.pi / 3.0 * RE * RE


def kn_dsigma_domega(cost, k):
    """Klein-Nishina differential cross section per electron (cm2/sr)."""
    P = 1.0 / (1.0 + k * (1.0 - cost))
    return 0.5 * RE * RE * P * P * (P + 1.0 / P - (1.0 - cost * cost))


def kn_quad(k):
    val, _ = integrate.quad(lambda c: 2 * math.pi * kn_dsigma_domega(c, k), -1.0, 1.0,
                            epsabs=0, epsrel=1e-13, limit=200)
    return val


@pytest.mark.parametrize("E", [1e-3, 1e-2, 0.1, 0.511, 1.0, 10.0, 100.0])
def test_kn_total_matches_quadrature(oracle_lib, E):
    k = E / ME
    got = oracle_lib.sigma_atom(1, E)[1]
    ref = kn_quad(k)
    assert abs(got - ref) <= 1e-10 * ref


def test_kn_thomson_limit(oracle_lib):
    # sigma_KN = sigma_T (1 - 2k + O(k^2)) as k -> 0
    for k in [1e-4, 1e-5]:
        got = oracle_lib.kn_per_electron(k)
        assert abs(got / THOMSON - (1 - 2 * k)) < 10 * k * k


def paper_mu_al():
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")):
        if line.startswith("mu_mass_al_1mev"):
            return float(line.split()[1])
    raise AssertionError


def test_aluminium_attenuation_matches_paper(oracle_lib):
    """Sec. 3.4 quotes mu/rho(Al, 1 MeV) = 0.06146 cm2/g (XCOM).  The oracle's
    model (KN Compton + Z^4/E^3 photoelectric + pair, no coherent scattering
    and no binding) must land within 0.5 % of it."""
    s = oracle_lib.sigma_atom(13, 1.0)
    mu_mass = s.sum() * NA / 26.9815385
    assert abs(mu_mass / paper_mu_al() - 1) < 5e-3


def test_photoelectric_scaling(oracle_lib):
    a = oracle_lib.sigma_atom(82, 0.1)[0]
    assert abs(oracle_lib.sigma_atom(82, 0.2)[0] / a - 1 / 8) < 1e-14
    assert abs(oracle_lib.sigma_atom(41, 0.1)[0] / a - 1 / 16) < 1e-14
    # constant: 4.0e-8 barn MeV^3 Z^4 / E^3
    assert abs(a - 4.0e-32 * 82 ** 4 / 0.1 ** 3) < 1e-12 * a


def test_pair_threshold_and_limits(oracle_lib):
    thr = 2 * ME
    assert oracle_lib.sigma_atom(82, thr * (1 - 1e-12))[2] == 0.0
    assert oracle_lib.sigma_atom(82, 1.0)[2] == 0.0
    assert oracle_lib.sigma_atom(82, 1.1)[2] > 0.0
    alpha = 1 / 137.035999084
    # complete-screening asymptote at very high energy
    Z = 82
    fcs = 28 / 9 * math.log(183 * Z ** (-1 / 3)) - 2 / 27
    hi = oracle_lib.sigma_atom(Z, 1e5)[2]
    assert abs(hi - alpha * RE * RE * Z * Z * fcs) < 1e-12 * hi
    # near threshold: the leading (k-2)^3 term
    k = 2.05
    lo = oracle_lib.sigma_atom(Z, k * ME)[2]
    ref = alpha * RE * RE * Z * Z * (2 * math.pi / 3) * ((k - 2) / k) ** 3
    assert abs(lo - ref) < 1e-12 * ref
    # monotone in energy
    es = np.geomspace(1.03, 100.0, 50)
    s = [oracle_lib.sigma_atom(Z, e)[2] for e in es]
    assert np.all(np.diff(s) > 0)


def test_water_attenuation_is_electron_density_times_kn(oracle_lib):
    """At 1 MeV water attenuation is Compton dominated: n_e sigma_KN(quad)."""
    g = oracle_lib.Geometry(W.geometry.tiny())
    mat = g.desc.mat_names.index("water")
    mu = g.mu(mat, [1.0])[0]
    ne = 1.0 * NA * (0.111894 * 1 / 1.008 + 0.888106 * 8 / 15.999)  # electrons / cm3
    ref_c = ne * kn_quad(1.0 / ME) * 0.1  # 1/mm
    # linear interpolation in ln E over nodes 0.045 apart: error well below 1e-4
    assert abs(mu[1] - ref_c) < 1e-4 * ref_c
    assert mu[2] == 0.0
    assert mu[0] < 1e-3 * mu[1]


def test_tables_interpolate_nodes(oracle_lib):
    g = oracle_lib.Geometry(W.geometry.calorimeter())
    tab, lnE0, dlnE = g.table()
    assert abs(lnE0 - math.log(1e-3)) < 1e-15 and abs(dlnE * 256 - math.log(1e5)) < 1e-13
    nodes = np.exp(lnE0 + dlnE * np.arange(257))
    for m in range(g.desc.n_mats):
        mu = g.mu(m, nodes[1:-1])
        ref = tab[m][:, 1:-1].T.copy()
        ref[nodes[1:-1] < 2 * ME, 2] = 0.0
        assert np.allclose(mu, ref, rtol=1e-12, atol=0)
        # node values equal the per-atom closed forms summed over elements
        for i in [0, 100, 256]:
            E = nodes[i]
            acc = np.zeros(3)
            d = g.desc
            for e in range(d.mat_el_off[m], d.mat_el_off[m + 1]):
                acc += d.mat_density[m] * NA * d.el_wfrac[e] / d.el_A[e] * \
                    oracle_lib.sigma_atom(int(d.el_Z[e]), E)
            assert np.allclose(tab[m][:, i], 0.1 * acc, rtol=1e-12, atol=0)
    # between nodes: bounded by the neighbours (linear in ln E)
    mid = np.sqrt(nodes[:-1] * nodes[1:])
    lead = g.desc.mat_names.index("lead")
    mu = g.mu(lead, mid)
    lo = np.minimum(tab[lead][:, :-1], tab[lead][:, 1:]).T
    hi = np.maximum(tab[lead][:, :-1], tab[lead][:, 1:]).T
    ok = mid >= 2 * ME
    assert np.all(mu[ok] >= lo[ok] * (1 - 1e-12)) and np.all(mu[ok] <= hi[ok] * (1 + 1e-12))


def _kn_cost_pdf_bins(k, edges):
    cdf = [integrate.quad(lambda c: kn_dsigma_domega(c, k), -1.0, e, epsrel=1e-11)[0] for e in edges]
    p = np.diff(cdf)
    return p / p.sum()


@pytest.mark.parametrize("E", [0.05, 1.0, 10.0])
def test_compton_sampler_angular_chi2(oracle_lib, E):
    n = 400_000
    eps, cost, draws = oracle_lib.compton_sample(E, n, seed=11)
    edges = np.linspace(-1, 1, 101)
    obs, _ = np.histogram(cost, bins=edges)
    p = _kn_cost_pdf_bins(E / ME, edges)
    exp = p * n
    chi2 = ((obs - exp) ** 2 / exp).sum()
    pval = stats.chi2.sf(chi2, df=len(obs) - 1)
    assert pval > 1e-3, (chi2, pval)
    # Compton kinematics: E'/E = 1 / (1 + k (1 - cos theta))
    k = E / ME
    assert np.allclose(eps, 1.0 / (1.0 + k * (1.0 - cost)), rtol=1e-12, atol=1e-14)
    assert np.all(draws % 3 == 0) and np.all(draws >= 3)


@pytest.mark.parametrize("E", [0.2, 2.0])
def test_compton_mean_energy_transfer(oracle_lib, E):
    n = 400_000
    eps, _, _ = oracle_lib.compton_sample(E, n, seed=5)
    k = E / ME
    num = integrate.quad(lambda c: kn_dsigma_domega(c, k) * (1 - 1 / (1 + k * (1 - c))), -1, 1,
                         epsrel=1e-11)[0]
    den = integrate.quad(lambda c: kn_dsigma_domega(c, k), -1, 1, epsrel=1e-11)[0]
    ref = num / den
    x = 1 - eps
    assert abs(x.mean() - ref) < 5 * x.std() / np.sqrt(n)


def test_rotation_preserves_angle(oracle_lib):
    rng = np.random.Generator(np.random.Philox(key=3))
    n = 20000
    v = W.primaries.isotropic(rng, n)
    v[:10] = [[0, 0, 1]] * 5 + [[0, 0, -1]] * 5  # the on-axis branch
    cost = rng.uniform(-1, 1, n)
    phi = rng.uniform(0, 2 * math.pi, n)
    w = oracle_lib.rotate(v, cost, phi)
    assert np.allclose(np.linalg.norm(w, axis=1), 1, atol=1e-15)
    assert np.allclose((v * w).sum(1), cost, atol=1e-12)
    # the azimuth about v is uniform: project on a fixed frame
    e1 = np.cross(v[10:], [0.3, 0.5, 0.8])
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(v[10:], e1)
    az = np.arctan2((w[10:] * e2).sum(1), (w[10:] * e1).sum(1))
    assert stats.kstest((az + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-3
