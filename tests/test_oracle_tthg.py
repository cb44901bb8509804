"""Pins of the oracle's two-term Henyey-Greenstein cloud phase function
(Sect. 3, aerosol scattering; lobes g1 = g, g2 = -g/2, forward weight
a = 1 - g2^2):

- normalisation and mean cosine a g1 + (1 - a) g2 by quadrature;
- the sampler against the closed-form mixture CDF (KS test);
- exact single scattering from a slab of TTHG cloud;
- g = 0 reduces to the isotropic HG path packet by packet.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import oracle as O
from paper_2110_15640_amd import inputs as I


def hg_cdf(mu, g):
    if abs(g) < 1e-12:
        return 0.5 * (mu + 1.0)
    return (1.0 - g * g) / (2.0 * g) * (1.0 / math.sqrt(1.0 + g * g - 2.0 * g * mu) - 1.0 / (1.0 + g))


@pytest.mark.parametrize("g", [0.0, 0.35, 0.85, -0.5])
def test_normalisation_and_mean_cosine(g):
    n, _ = integrate.quad(lambda m: O.phase_tthg(m, g), -1, 1, epsabs=0, epsrel=1e-12)
    c, _ = integrate.quad(lambda m: m * O.phase_tthg(m, g), -1, 1, epsabs=0, epsrel=1e-12)
    a = 1.0 - (g / 2.0) ** 2
    assert n == pytest.approx(2.0, rel=1e-9)
    assert c / 2.0 == pytest.approx(a * g + (1.0 - a) * (-g / 2.0), rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("g", [0.35, 0.85, -0.5])
def test_sampler_matches_mixture_cdf(g):
    rng = np.random.default_rng(7)
    n = 20000
    zl, z = rng.uniform(size=n), rng.uniform(size=n)
    mu = np.array([O.sample_tthg(a, b, g) for a, b in zip(zl, z)])
    a = 1.0 - (g / 2.0) ** 2
    cdf = np.vectorize(lambda m: a * hg_cdf(m, g) + (1.0 - a) * hg_cdf(m, -g / 2.0))
    assert stats.kstest(mu, cdf).pvalue > 1e-3


def test_single_scattering_tthg_slab():
    """max_events = 1, fixed incidence: E = omega P_TTHG(cos)/(4 pi) mu (1 - e^{-tau (1/mu0 + 1/mu)}) / (mu + mu0)."""
    tau, om, mu0, gc = 0.75, 0.8, 0.6, 0.6
    g, t = I.make_homogeneous_slab(tau, om, g_cld=gc)
    obs = []
    for mu, dphi in ((0.9, math.pi), (0.5, 0.0), (0.3, 2.0)):
        s = math.sqrt(1.0 - mu * mu)
        obs.append([s * math.cos(dphi), s * math.sin(dphi), mu])
    n = 80000
    p = O.Params(n_packets=n, mu0=mu0, max_events=1, seed=61, obs_dir=np.array(obs), cloud_phase=1)
    r = O.solve_albedo(g, t, p)
    d0 = np.array([math.sqrt(1 - mu0 * mu0), 0.0, -mu0])
    kext = float(t.kappa.ravel()[0]) + float(g.cld_ksca[0])
    tau_e = kext * g.r_edges[-1]
    om_e = float(g.cld_ksca[0]) / kext
    for o, ov in enumerate(obs):
        mu = ov[2]
        c = float(d0 @ np.array(ov))
        a = 1.0 - (gc / 2.0) ** 2
        hg = lambda cc, gg: (1 - gg * gg) / (1 + gg * gg - 2 * gg * cc) ** 1.5
        P = a * hg(c, gc) + (1 - a) * hg(c, -gc / 2)
        E = om_e * P / (4 * math.pi) * mu * (1 - math.exp(-tau_e * (1 / mu0 + 1 / mu))) / (mu + mu0)
        got, se = r.value[0, o] / math.pi, r.stderr[0, o] / math.pi
        assert abs(got - E) <= 3.0 * se, (o, got, E, se)


def test_zero_asymmetry_reduces_to_isotropic_hg():
    g, t = I.make_homogeneous_slab(2.0, 0.9, g_cld=0.0)
    base = dict(n_packets=2000, mu0=0.5, seed=63, obs_dir=np.array([[0.0, 0.6, 0.8]]))
    a = O.solve_albedo(g, t, O.Params(cloud_phase=0, **base), keep_packets=True)
    b = O.solve_albedo(g, t, O.Params(cloud_phase=1, **base), keep_packets=True)
    np.testing.assert_array_equal(a.extra["packets"][(0, 0)][0], b.extra["packets"][(0, 0)][0])
