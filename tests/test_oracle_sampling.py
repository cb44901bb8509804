"""Pins of the oracle's phase functions, samplers and direction rotation."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import oracle as O


def rayleigh_cdf(mu):
    # integral of (3/8)(1 + x^2) from -1 to mu
    return (mu ** 3 + 3.0 * mu + 4.0) / 8.0


def hg_cdf(mu, g):
    # integral of (1/2)(1-g^2)(1+g^2-2gx)^-3/2 from -1 to mu
    return (1.0 - g * g) / (2.0 * g) * (1.0 / math.sqrt(1.0 + g * g - 2.0 * g * mu) - 1.0 / (1.0 + g))


@pytest.mark.parametrize("fn,args", [(O.phase_rayleigh, ()), (O.phase_hg, (0.0,)), (O.phase_hg, (0.5,)),
                                      (O.phase_hg, (-0.3,)), (O.phase_hg, (0.9,))])
def test_phase_functions_are_normalised(fn, args):
    v, _ = integrate.quad(lambda m: fn(m, *args) / 2.0, -1.0, 1.0, epsabs=1e-13, limit=400)
    assert abs(v - 1.0) < 1e-10


@pytest.mark.parametrize("g", [0.2, 0.5, 0.9, -0.6])
def test_hg_mean_cosine_is_g(g):
    v, _ = integrate.quad(lambda m: m * O.phase_hg(m, g) / 2.0, -1.0, 1.0, epsabs=1e-13, limit=400)
    assert abs(v - g) < 1e-9


def test_rayleigh_sampler_inverts_cdf():
    for z in np.linspace(1e-9, 1 - 1e-9, 1001):
        assert abs(rayleigh_cdf(O.sample_rayleigh(z)) - z) < 1e-13
    assert O.sample_rayleigh(0.5) == pytest.approx(0.0, abs=1e-15)


@pytest.mark.parametrize("g", [0.05, 0.5, 0.9, -0.4])
def test_hg_sampler_inverts_cdf(g):
    for z in np.linspace(1e-9, 1 - 1e-9, 1001):
        assert abs(hg_cdf(O.sample_hg(z, g), g) - z) < 1e-11


def test_hg_small_g_is_isotropic():
    for z in (0.1, 0.37, 0.9):
        assert O.sample_hg(z, 1e-8) == 2.0 * z - 1.0
        assert O.phase_hg(0.3, 1e-8) == 1.0


def test_sampled_moments():
    u = np.array([O.draw_pair(5, 0, p, 1, 1) for p in range(20000)])
    mr = np.array([O.sample_rayleigh(z) for z in u[:, 0]])
    assert abs(mr.mean()) < 3 * math.sqrt(0.4 / len(mr))
    # <mu^4> = 9/35 for Rayleigh, so var(mu^2) = 9/35 - 4/25
    assert abs((mr ** 2).mean() - 0.4) < 3 * math.sqrt((9 / 35 - 4 / 25) / len(mr))
    mh = np.array([O.sample_hg(z, 0.7) for z in u[:, 1]])
    assert abs(mh.mean() - 0.7) < 3 * mh.std() / math.sqrt(len(mh))
    assert stats.kstest(mr, lambda x: rayleigh_cdf(np.clip(x, -1, 1))).pvalue > 1e-3


@pytest.mark.parametrize("d", [[0.0, 0.0, 1.0], [0.0, 0.0, -1.0], [0.6, 0.0, 0.8],
                               [-0.36, 0.48, -0.8], [1.0, 0.0, 0.0], [0.0, 0.999999, 0.0014142]])
def test_rotation_sets_polar_angle(d):
    d = np.array(d) / np.linalg.norm(d)
    for mu in (-0.9, -0.2, 0.0, 0.5, 0.99):
        for psi in (0.0, 1.0, 2.5, 4.0):
            n = O.rotate(d, mu, psi)
            assert abs(np.linalg.norm(n) - 1.0) < 1e-14
            assert abs(float(n @ d) - mu) < 1e-9


def test_rotation_azimuth_is_uniform():
    d = np.array([0.3, -0.4, math.sqrt(1 - 0.25)])
    e1 = np.cross(d, [0.0, 0.0, 1.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    ang = []
    for p in range(3000):
        z = O.draw_pair(1, 0, p, 3, 1)
        n = O.rotate(d, 0.1, 2 * math.pi * z[1])
        ang.append(math.atan2(n @ e2, n @ e1) % (2 * math.pi))
    assert stats.kstest(np.array(ang) / (2 * math.pi), "uniform").pvalue > 1e-3
