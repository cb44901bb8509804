"""Pins of the oracle's Lambert lower boundary (Sect. 3, surface scattering
with a Lambertian reflector of albedo A_s):

- transparent slab: every packet reflects once, so E = A_s mu / pi exactly;
- absorbing, non-scattering slab: E = A_s mu e^{-tau (1/mu0 + 1/mu)} / pi;
- transparent sphere: A_g = 2 A_s / 3 (over the surface disk; the albedo is
  quoted per top-of-atmosphere disk, hence (r_0 / R_TOA)^2) and the Lambert
  phase law (sin a + (pi - a) cos a) / pi;
- scattering layer over the floor (HG and Rayleigh, omega < 1): the
  reflection function from adding-doubling with the floor added;
- conservative layer over a white floor: no weight is lost;
- A_s = 0 is the absorbing boundary packet by packet.
"""
import math

import numpy as np
import pytest

import closed_forms as CF
from oracle import oracle as O
from paper_2110_15640_amd import inputs as I


def within(x, ref, se, k=3.0, floor=0.0):
    assert abs(x - ref) <= k * se + floor, (x, ref, se, (x - ref) / max(se, 1e-300))


def slab_obs(mu, dphi):
    s = math.sqrt(1.0 - mu * mu)
    return [s * math.cos(dphi), s * math.sin(dphi), mu]


@pytest.mark.parametrize("As", [1.0, 0.35])
def test_transparent_slab_is_exact(As):
    g, t = I.make_homogeneous_slab(1e-9, 0.0)
    t.kappa[:] = 0.0
    obs = [slab_obs(0.8, 0.0), slab_obs(0.3, 2.0), slab_obs(0.05, math.pi)]
    r = O.solve_albedo(g, t, O.Params(n_packets=500, mu0=0.45, seed=71, surface_albedo=As,
                                      obs_dir=np.array(obs)), keep_packets=True)
    F, K = r.extra["packets"][(0, 0)]
    for o, ov in enumerate(obs):
        np.testing.assert_allclose(F[:, o], As * ov[2] / math.pi, rtol=1e-14)
    np.testing.assert_allclose(K[:, 1], 1.0 - As, rtol=1e-14, atol=1e-15)  # absorbed by the floor
    np.testing.assert_allclose(K[:, 0], As, rtol=1e-14)  # escaped


def test_absorbing_slab_attenuates_both_ways():
    tau, mu0, As = 0.5, 0.7, 0.8
    g, t = I.make_homogeneous_slab(tau, 0.0)
    obs = [slab_obs(0.9, 0.0), slab_obs(0.4, 1.0)]
    n = 40000
    r = O.solve_albedo(g, t, O.Params(n_packets=n, mu0=mu0, seed=73, surface_albedo=As, obs_dir=np.array(obs)))
    for o, ov in enumerate(obs):
        mu = ov[2]
        E = As * mu * math.exp(-tau * (1 / mu0 + 1 / mu)) / math.pi
        within(r.value[0, o] / math.pi, E, r.stderr[0, o] / math.pi)
    # continuous absorption: the reflected peel is deterministic
    r = O.solve_albedo(g, t, O.Params(n_packets=200, mu0=mu0, seed=73, surface_albedo=As, absorption=1,
                                      obs_dir=np.array(obs)), keep_packets=True)
    F, _ = r.extra["packets"][(0, 0)]
    for o, ov in enumerate(obs):
        mu = ov[2]
        np.testing.assert_allclose(F[:, o], As * mu * math.exp(-tau * (1 / mu0 + 1 / mu)) / math.pi, rtol=1e-12)


def _transparent_sphere():
    g = I.make_sphere(8, 4, 3, seed=75)
    tab = I.CKTable(np.array([0.5]), np.ones(1), np.array([1000.0]), np.array([1.0]),
                    np.zeros((1, 1, 1, 1), np.float32), np.zeros(1))
    return g, tab


def test_transparent_lambert_sphere_phase_law():
    As = 0.6
    g, tab = _transparent_sphere()
    alphas = (0.0, 0.8, 1.9, 2.8)
    r = O.solve_albedo(g, tab, O.Params(n_packets=60000, seed=77, surface_albedo=As, obs_phase=alphas))
    disk = (g.r_edges[0] / g.r_edges[-1]) ** 2
    for o, a in enumerate(alphas):
        want = disk * 2.0 * As / 3.0 * (math.sin(a) + (math.pi - a) * math.cos(a)) / math.pi
        within(r.value[0, o], want, r.stderr[0, o], floor=1e-12)
    assert r.value[0, 0] / disk == pytest.approx(0.4, rel=1e-2)


@pytest.fixture(scope="module")
def dbl_surface():
    return {
        "hg": CF.Doubling(CF.phase_hg(0.5), 0.875, 1.0, n=32, mmax=48, n_double=36, surface_albedo=0.6),
        "ray": CF.Doubling(CF.phase_rayleigh, 0.875, 1.0, n=32, mmax=2, n_double=36, surface_albedo=0.6),
    }


@pytest.mark.parametrize("which", ["hg", "ray"])
def test_scattering_layer_over_floor_by_adding(which, dbl_surface):
    D = dbl_surface[which]
    if which == "ray":
        g, t = I.make_homogeneous_slab(1.0, 0.875, rayleigh=True)
    else:
        g, t = I.make_homogeneous_slab(1.0, 0.875, g_cld=0.5)
    j0 = 22
    mu0 = float(D.mu[j0])
    sel = [(30, math.pi), (22, 0.0), (14, 1.0), (6, 2.5)]
    obs = [slab_obs(float(D.mu[i]), dp) for i, dp in sel]
    r = O.solve_albedo(g, t, O.Params(n_packets=40000, mu0=mu0, seed=79, surface_albedo=0.6, obs_dir=np.array(obs)))
    for o, (i, dp) in enumerate(sel):
        E = float(D.mu[i]) * D.rho_nodes(dp)[i, j0] / math.pi
        within(r.value[0, o] / math.pi, E, r.stderr[0, o] / math.pi, floor=1e-4 * E)
    # the floor adds to the reflection of the bare layer by a visible margin
    bare = CF.Doubling(CF.phase_rayleigh if which == "ray" else CF.phase_hg(0.5), 0.875, 1.0, n=32,
                       mmax=D.mmax, n_double=36)
    i, dp = sel[1]
    assert D.rho_nodes(dp)[i, j0] > 1.2 * bare.rho_nodes(dp)[i, j0]


def test_white_floor_conserves_weight():
    g, t = I.make_homogeneous_slab(2.0, 1.0, g_cld=0.3, nlay=4)
    r = O.solve_albedo(g, t, O.Params(n_packets=3000, seed=81, surface_albedo=1.0, rr_threshold=0.0,
                                      max_events=100000), keep_packets=True)
    F, K = r.extra["packets"][(0, 0)]
    np.testing.assert_allclose(K[:, 0], 1.0, rtol=1e-12)  # every packet escapes with its full weight
    assert np.all(K[:, 1] == 0.0) and np.all(K[:, 2] == 0.0)
    assert K[:, 6].mean() > 2.0  # with many events


def test_zero_albedo_is_the_absorbing_boundary():
    g, t = I.make_homogeneous_slab(1.0, 0.9, g_cld=0.4)
    base = dict(n_packets=2000, mu0=0.5, seed=83, obs_dir=np.array([[0.0, 0.6, 0.8]]))
    a = O.solve_albedo(g, t, O.Params(**base), keep_packets=True)
    b = O.solve_albedo(g, t, O.Params(surface_albedo=0.0, **base), keep_packets=True)
    for k in (0, 1):
        np.testing.assert_array_equal(a.extra["packets"][(0, 0)][k], b.extra["packets"][(0, 0)][k])
