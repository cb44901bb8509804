"""Pins of the oracle's transmission with multiple scattering and stellar
limb darkening (Sect. 5.1 and 5.1.1):

- births: b = R0 + zeta (R_TOA - R0) from the birth event's Philox block 0,
  weight W0 = b; the first peel-off is the chord's direct transmission,
  b e^{-tau(b)} with tau(b) the closed-form shell chord depth;
- with scattering off the depth estimate matches the shell integral;
- single scattering (max_events = 1): the scattered light of a packet has
  expectation b Omega_* Theta(0 deg) tau_sca(b) e^{-tau(b)} (the scattering
  point lies on the chord, so the peel-off continues along it), for Rayleigh
  gas and for an HG cloud;
- weight bookkeeping per packet;
- limb-darkening laws: the disk average int_0^1 I(mu) 2 mu dmu of each law
  against its closed form; the chord weight is the law at the stellar-disk
  zenith cosine and zero off the disk;
- limb-darkened transit depth (raytrace chords, planet off the disk centre)
  and limb-darkened packet weights against 2D quadrature.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import closed_forms as CF
from oracle import oracle as O
from paper_2110_15640_amd import inputs as I

A_ORBIT = 0.05 * 1.495978707e13  # 0.05 au


def within(x, ref, se, k=3.0, floor=0.0):
    assert abs(x - ref) <= k * se + floor, (x, ref, se, (x - ref) / max(se, 1e-300))


def shells(nlay, alpha, omega=0.0, cloud_g=None, seed=91):
    """1D shells of extinction alpha[k]; a fraction omega scatters (Rayleigh
    gas, or an HG cloud of asymmetry cloud_g)."""
    g = I.make_sphere(8, 4, nlay, seed=seed)
    g.rho = np.repeat(np.asarray(alpha, dtype=np.float64), g.nlon * g.nlat)
    if cloud_g is None:
        tab = I.CKTable(np.array([0.5]), np.ones(1), np.array([1000.0]), np.array([1.0]),
                        np.full((1, 1, 1, 1), 1.0 - omega, np.float32), np.array([omega]))
    else:
        tab = I.CKTable(np.array([0.5]), np.ones(1), np.array([1000.0]), np.array([1.0]),
                        np.full((1, 1, 1, 1), 1.0 - omega, np.float32), np.zeros(1))
        g.cld_ksca = np.full(g.ncell, omega, np.float32)
        g.cld_kabs = np.zeros(g.ncell, np.float32)
        g.cld_g = np.full(g.ncell, cloud_g, np.float32)
    return g, tab


def test_births_and_direct_chord_light():
    alpha = 2e-9 * np.exp(-np.arange(10) / 2.0)
    g, tab = shells(10, alpha)
    p = O.Params(n_packets=400, seed=93, scattering=False, r_star=I.R_SUN)
    r = O.solve_transmission_ms(g, tab, p, keep_packets=True)
    v, K = r.extra["packets"][(0, 0)]
    a_ext = np.float32(1.0) * alpha  # kappa = 1 exactly in float32
    for q in range(p.n_packets):
        ua, _ = O.draw_pair(p.seed, 0, q, 0, 0)
        b = g.r0 + ua * (g.r_toa - g.r0)
        assert K[q, 10] == pytest.approx(b, rel=1e-15)
        tau = CF.chord_tau(b, g.r_edges, a_ext)
        assert K[q, 10] - v[q] == pytest.approx(b * math.exp(-tau), rel=1e-9)
        assert v[q] == pytest.approx(b * (1.0 - math.exp(-tau)), rel=1e-9, abs=1e-12 * b)


def test_raytrace_depth_matches_shell_integral():
    alpha = 3e-8 * np.exp(-np.arange(12) / 1.5)
    g, tab = shells(12, alpha, seed=95)
    p = O.Params(n_packets=160000, seed=97, scattering=False, r_star=I.R_SUN)
    r = O.solve_transmission_ms(g, tab, p)
    want = (g.r0 ** 2 + 2.0 * CF.transit_integral(g.r_edges, alpha)) / p.r_star ** 2
    within(r.value[0, 0], want, r.stderr[0, 0])
    # the same depth as the stratified raytrace chords
    k5 = O.solve_transmission(g, tab, O.Params(n_b=256, n_alpha=64, seed=97, r_star=I.R_SUN))
    within(r.value[0, 0] - k5.value[0, 0], 0.0, math.hypot(r.stderr[0, 0], k5.stderr[0, 0]))


@pytest.mark.parametrize("cloud_g", [None, 0.6])
def test_single_scattering_into_the_line_of_sight(cloud_g):
    om = 0.8
    alpha = 4e-9 * np.exp(-np.arange(10) / 2.5)
    g, tab = shells(10, alpha, omega=om, cloud_g=cloud_g, seed=99)
    n = 40000
    p = O.Params(n_packets=n, seed=101, max_events=1, a_orbit=A_ORBIT, r_star=I.R_SUN, rr_threshold=0.0)
    r = O.solve_transmission_ms(g, tab, p, keep_packets=True)
    v, K = r.extra["packets"][(0, 0)]
    b = K[:, 10]
    a_ext = np.asarray(alpha, dtype=np.float64) * float(np.float32(1.0 - om) + om)
    tau = np.array([CF.chord_tau(x, g.r_edges, a_ext) for x in b])
    scat = (b - v) - b * np.exp(-tau)  # light scattered into the line of sight
    P0 = 1.5 if cloud_g is None else (1.0 + cloud_g) / (1.0 - cloud_g) ** 2
    om_e = om / float(np.float32(1.0 - om) + om)
    expect = b * O.omega_star(p) * P0 / (4.0 * math.pi) * om_e * tau * np.exp(-tau)
    d = scat - expect
    within(d.mean(), 0.0, d.std() / math.sqrt(n))
    assert expect.mean() > 20.0 * d.std() / math.sqrt(n)  # the term is resolved


def test_weight_bookkeeping():
    g, tab = shells(6, 5e-9 * np.ones(6), omega=0.95, cloud_g=0.3, seed=103)
    p = O.Params(n_packets=2000, seed=105, a_orbit=A_ORBIT, r_star=I.R_SUN, rr_threshold=0.0)
    r = O.solve_transmission_ms(g, tab, p, keep_packets=True)
    _, K = r.extra["packets"][(0, 0)]
    np.testing.assert_allclose(K[:, :6].sum(axis=1), K[:, 10], rtol=1e-12)
    assert K[:, 6].mean() > 0.5  # packets scatter


LAWS = [  # law, c1, c2, closed-form disk average int_0^1 I(mu) 2 mu dmu
    (1, 0.6, 0.0, 1.0 - 0.6 / 3.0),
    (2, 0.4, 0.25, 1.0 - 0.4 / 3.0 - 0.25 / 6.0),
    (3, 0.3, 0.45, 1.0 - 0.3 / 3.0 - 0.45 / 5.0),
    (4, 0.5, 0.2, 1.0 - 0.5 / 3.0 + 2.0 * 0.2 / 9.0),
    (6, 0.7, 0.8, 1.0 - 0.7 * 0.8 / 2.8),
]


@pytest.mark.parametrize("law,c1,c2,avg", LAWS)
def test_limb_darkening_disk_averages(law, c1, c2, avg):
    got, _ = integrate.quad(lambda m: O.limb_darkening(law, c1, c2, m) * 2.0 * m, 0.0, 1.0,
                            epsabs=0.0, epsrel=1e-12, limit=200)
    assert got == pytest.approx(avg, rel=1e-10)
    assert O.limb_darkening(law, c1, c2, 1.0) == 1.0


def test_exponential_law_and_chord_weight_geometry():
    # exponential law (Claret & Hauschildt): I(1) = 1 - h / (1 - e)
    assert O.limb_darkening(5, 0.3, 0.1, 1.0) == pytest.approx(1.0 - 0.1 / (1.0 - math.e), rel=1e-15)
    assert O.limb_darkening(0, 0.3, 0.1, 0.2) == 1.0
    R = I.R_SUN
    p = O.Params(ld_law=2, ld_c1=0.4, ld_c2=0.25, r_star=R, transit_y=0.3 * R, transit_z=-0.2 * R)
    for y, z in ((0.0, 0.0), (0.1 * R, 0.05 * R), (0.5 * R, 0.6 * R)):
        rr = math.hypot(0.3 * R + y, -0.2 * R + z) / R
        mu = math.sqrt(1.0 - rr * rr)
        assert O.chord_limb_weight(p, y, z) == pytest.approx(1.0 - 0.4 * (1 - mu) - 0.25 * (1 - mu) ** 2, rel=1e-12)
    assert O.chord_limb_weight(p, 0.9 * R, 0.0) == 0.0  # off the stellar disk


def _ld_quad(g, p, f):
    """(1/2pi) int_{R0}^{R_TOA} int_0^{2pi} LD(b, a) f(b) b da db."""
    def inner(b):
        v, _ = integrate.quad(lambda a: O.chord_limb_weight(p, b * math.cos(a), b * math.sin(a)), 0.0, 2 * math.pi,
                              epsabs=0.0, epsrel=1e-11, limit=200)
        return v / (2 * math.pi) * f(b) * b
    tot = 0.0
    for k in range(len(g.r_edges) - 1):
        v, _ = integrate.quad(inner, g.r_edges[k], g.r_edges[k + 1], epsabs=0.0, epsrel=1e-10, limit=200)
        tot += v
    return tot


def test_limb_darkened_transit_depth():
    alpha = 3e-8 * np.exp(-np.arange(8) / 1.5)
    g, tab = shells(8, alpha, seed=107)
    R = I.R_SUN
    p = O.Params(n_b=256, n_alpha=64, seed=109, r_star=R, ld_law=2, ld_c1=0.45, ld_c2=0.2,
                 transit_y=0.55 * R, transit_z=0.3 * R)
    r = O.solve_transmission(g, tab, p)
    I_ld = _ld_quad(g, p, lambda b: 1.0 - math.exp(-CF.chord_tau(b, g.r_edges, alpha)))
    want = (g.r0 ** 2 + 2.0 * I_ld) / R ** 2
    within(r.value[0, 0], want, r.stderr[0, 0])
    plain = O.solve_transmission(g, tab, O.Params(n_b=256, n_alpha=64, seed=109, r_star=R))
    assert r.value[0, 0] < plain.value[0, 0] - 10 * r.stderr[0, 0]  # darkened limb: shallower


def test_limb_darkened_packet_weights():
    g, tab = shells(6, 1e-9 * np.ones(6), omega=0.5, seed=111)
    R = I.R_SUN
    p = O.Params(n_packets=20000, seed=113, r_star=R, a_orbit=A_ORBIT, ld_law=3, ld_c1=0.2, ld_c2=0.5,
                 transit_y=-0.4 * R, transit_z=0.5 * R)
    r = O.solve_transmission_ms(g, tab, p, keep_packets=True)
    _, K = r.extra["packets"][(0, 0)]
    W0 = K[:, 10]
    want = _ld_quad(g, p, lambda b: 1.0) / (g.r_toa - g.r0)
    within(W0.mean(), want, W0.std() / math.sqrt(len(W0)))
    p.transit_y = 2.0 * R  # the planet off the stellar disk: no light in its packets
    r = O.solve_transmission_ms(g, tab, p, keep_packets=True)
    assert np.all(r.extra["packets"][(0, 0)][1][:, 10] == 0.0)
    assert r.value[0, 0] == pytest.approx(g.r0 ** 2 / R ** 2, rel=1e-15)
