"""Pins of the oracle's Draine (2003) hybrid HG-Rayleigh cloud phase function
(Sect. 3, aerosol scattering), P = P_HG(G) (1 + alpha mu^2) / (1 + alpha
(1 + 2 G^2)/3) with G found from the cloud's asymmetry factor g:

- normalisation, and the mean cosine by quadrature equals g after the
  inversion G(g) (so both the normalisation and the inversion are fixed by
  the definition of the asymmetry factor);
- alpha = 1 is the Cornette-Shanks function; G = 0 with alpha = 1 is Rayleigh;
- the rejection sampler against the CDF by quadrature (KS);
- exact single scattering from a Draine-cloud slab;
- alpha = 0 reduces to the HG path packet by packet.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import oracle as O
from paper_2110_15640_amd import inputs as I


def quad(f):
    v, _ = integrate.quad(f, -1.0, 1.0, epsabs=0.0, epsrel=1e-12, limit=400)
    return v


@pytest.mark.parametrize("alpha", [0.25, 0.5, 1.0])
@pytest.mark.parametrize("g", [-0.5, 0.1, 0.6, 0.9])
def test_normalisation_and_asymmetry_factor(g, alpha):
    G = O.draine_G(g, alpha)
    assert quad(lambda m: O.phase_draine(m, G, alpha)) == pytest.approx(2.0, rel=1e-10)
    assert quad(lambda m: m * O.phase_draine(m, G, alpha)) / 2.0 == pytest.approx(g, rel=1e-9, abs=1e-12)
    assert abs(G) < abs(g) + 1e-15  # the Rayleigh-like factor raises the mean cosine above G's HG value


def test_cornette_shanks_and_rayleigh_limits():
    for G in (0.0, 0.4, -0.3, 0.8):
        for m in (-0.9, -0.2, 0.3, 0.95):
            cs = 1.5 * (1 - G * G) / (2 + G * G) * (1 + m * m) / (1 + G * G - 2 * G * m) ** 1.5
            assert O.phase_draine(m, G, 1.0) == pytest.approx(cs, rel=1e-13)
    for m in (-1.0, -0.4, 0.0, 0.7):
        assert O.phase_draine(m, 0.0, 1.0) == pytest.approx(O.phase_rayleigh(m), rel=1e-14)
    assert O.draine_G(0.37, 0.0) == 0.37


@pytest.mark.parametrize("g,alpha", [(0.6, 0.5), (0.2, 1.0), (-0.4, 0.5)])
def test_sampler_matches_cdf(g, alpha):
    G = O.draine_G(g, alpha)
    rng = np.random.default_rng(11)
    n = 20000
    mu = np.array([O.sample_draine(rng.uniform(size=32), rng.uniform(size=32), G, alpha) for _ in range(n)])
    grid = np.linspace(-1.0, 1.0, 2001)
    pdf = np.array([O.phase_draine(m, G, alpha) for m in grid]) / 2.0
    cdf_t = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(grid))])
    cdf = lambda x: np.interp(x, grid, cdf_t / cdf_t[-1])
    assert stats.kstest(mu, cdf).pvalue > 1e-3


def test_single_scattering_draine_slab():
    """max_events = 1: E = omega P_D(cos)/(4 pi) mu (1 - e^{-tau (1/mu0 + 1/mu)}) / (mu + mu0)."""
    tau, om, mu0, gc, alpha = 0.75, 0.8, 0.6, 0.55, 0.5
    g, t = I.make_homogeneous_slab(tau, om, g_cld=gc)
    obs = []
    for mu, dphi in ((0.9, math.pi), (0.5, 0.0), (0.3, 2.0)):
        s = math.sqrt(1.0 - mu * mu)
        obs.append([s * math.cos(dphi), s * math.sin(dphi), mu])
    n = 80000
    p = O.Params(n_packets=n, mu0=mu0, max_events=1, seed=131, obs_dir=np.array(obs), cloud_phase=2,
                 draine_alpha=alpha)
    r = O.solve_albedo(g, t, p)
    d0 = np.array([math.sqrt(1 - mu0 * mu0), 0.0, -mu0])
    kext = float(t.kappa.ravel()[0]) + float(g.cld_ksca[0])
    tau_e = kext * g.r_edges[-1]
    om_e = float(g.cld_ksca[0]) / kext
    G = O.draine_G(float(np.float32(gc)), alpha)
    for o, ov in enumerate(obs):
        mu = ov[2]
        P = O.phase_draine(float(d0 @ np.array(ov)), G, alpha)
        E = om_e * P / (4 * math.pi) * mu * (1 - math.exp(-tau_e * (1 / mu0 + 1 / mu))) / (mu + mu0)
        within = abs(r.value[0, o] / math.pi - E) <= 4.0 * r.stderr[0, o] / math.pi
        assert within, (o, r.value[0, o] / math.pi, E)


def test_multiple_scattering_differs_from_hg_but_zero_alpha_is_hg():
    g, t = I.make_homogeneous_slab(2.0, 0.9, g_cld=0.5)
    base = dict(n_packets=2000, mu0=0.5, seed=133, obs_dir=np.array([[0.0, 0.6, 0.8]]))
    a = O.solve_albedo(g, t, O.Params(cloud_phase=0, **base), keep_packets=True)
    b = O.solve_albedo(g, t, O.Params(cloud_phase=2, draine_alpha=0.0, **base), keep_packets=True)
    for k in (0, 1):
        np.testing.assert_array_equal(a.extra["packets"][(0, 0)][k], b.extra["packets"][(0, 0)][k])
    c = O.solve_albedo(g, t, O.Params(cloud_phase=2, draine_alpha=0.5, **base), keep_packets=True)
    assert not np.array_equal(a.extra["packets"][(0, 0)][0], c.extra["packets"][(0, 0)][0])
