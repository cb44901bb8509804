"""Pins of the oracle's observables: transit depth against exact shell sums,
isothermal emission against the projected-area integral, albedo of a thin
spherical shell against the slab value."""
import math

import numpy as np
import pytest

import closed_forms as CF
from oracle import oracle as O
from paper_2110_15640_amd import inputs as I


def within(x, ref, se, k=3.0, floor=0.0):
    assert abs(x - ref) <= k * se + floor, (x, ref, se)


def shell_table(alpha_per_layer, grid):
    """A ck table + grid with extinction alpha_k in layer k (rho = alpha/kappa)."""
    nl = grid.nlay
    k = np.repeat(np.asarray(alpha_per_layer, dtype=np.float64), grid.nlon * grid.nlat)
    grid.rho = k.copy()
    tab = I.CKTable(np.array([1.0]), np.ones(1), np.array([1000.0]), np.array([1.0]),
                    np.ones((1, 1, 1, 1), np.float32), np.zeros(1))
    return tab


@pytest.mark.parametrize("nlon,nlat", [(1, 1), (16, 8)])
def test_chord_optical_depths_are_exact(nlon, nlat):
    g = I.make_sphere(nlon, nlat, 9, seed=21)
    alpha = np.geomspace(1e-6, 1e-9, 9) * np.array([1, 3, 0.5, 2, 1, 4, 0.2, 1, 1])
    tab = shell_table(alpha, g)
    p = O.Params(n_b=16, n_alpha=12, seed=22)
    r = O.solve_transmission(g, tab, p, tau_out=True)
    tau = r.extra["tau"][:, 0]
    for ch in range(p.n_b * p.n_alpha):
        ib = ch // p.n_alpha
        u = O.draw_pair(p.seed, 0, ch, 0, 0)
        b = g.r0 + (ib + u[0]) * (g.r_toa - g.r0) / p.n_b
        assert tau[ch] == pytest.approx(CF.chord_tau(b, g.r_edges, alpha), rel=1e-9)


def test_transit_depth_against_shell_integral():
    g = I.make_sphere(8, 4, 12, seed=23)
    alpha = 3e-8 * np.exp(-np.arange(12) / 1.5)
    tab = shell_table(alpha, g)
    p = O.Params(n_b=256, n_alpha=40, seed=24, r_star=I.R_SUN)
    r = O.solve_transmission(g, tab, p)
    want = (g.r0 ** 2 + 2.0 * CF.transit_integral(g.r_edges, alpha)) / p.r_star ** 2
    within(r.value[0, 0], want, r.stderr[0, 0], floor=1e-12 * want)
    # the stratified estimator is far better than its iid standard error
    assert abs(r.value[0, 0] - want) < 2e-4 * (want - g.r0 ** 2 / p.r_star ** 2)


def test_transit_depth_limits():
    g = I.make_sphere(4, 2, 5, seed=25)
    p = O.Params(n_b=8, n_alpha=8, seed=26, r_star=I.R_SUN)
    tab = shell_table(np.zeros(5), g)
    r = O.solve_transmission(g, tab, p)
    assert r.value[0, 0] == pytest.approx(g.r0 ** 2 / p.r_star ** 2, rel=1e-15)
    tab = shell_table(np.full(5, 1e3), g)
    r = O.solve_transmission(g, tab, p)
    # opaque: (R0^2 + 2 <b (R_TOA - R0)>)/R*^2 with b stratified in b
    assert r.value[0, 0] == pytest.approx(g.r_toa ** 2 / p.r_star ** 2, rel=1e-3)


def test_isothermal_emission_against_disk_integral():
    """Pure absorption, isothermal, no tau cut: F_p = B(T) * A_proj / R_TOA^2
    with A_proj = int (1 - e^-tau(b)) 2 pi b db (surface rays included)."""
    g = I.make_sphere(16, 8, 10, seed=27)
    g.T = np.full(g.ncell, 1300.0, np.float32)
    alpha = 2e-8 * np.exp(-np.arange(10) / 2.0)
    tab = shell_table(alpha, g)
    tab.lam_um = np.array([2.0])
    p = O.Params(n_packets=60000, seed=28, scattering=False, tau_vert_max=1e300, obs_phase=(0.5, 0.13))
    r = O.solve_emission(g, tab, p)
    B = O.planck(2.0e-4, 1300.0)
    want = B * CF.isothermal_disk_integral(g.r_edges, alpha) / g.r_toa ** 2
    for o in range(2):
        within(r.value[0, o], want, r.stderr[0, o])
        assert abs(r.value[0, o] / want - 1) < 1e-2


def test_thin_spherical_shell_albedo_matches_slab():
    """A thin homogeneous shell (dR/R = 1e-4) reflects like the slab: A_g of
    the sphere = (1/2) int S(mu, mu, pi) dmu of the slab (single scattering,
    tau = 0.5, Rayleigh)."""
    tau, om = 0.5, 1.0
    g = I.make_sphere(1, 1, 1, seed=29)
    r0 = g.r0
    g.r_edges = np.array([r0, r0 * (1 + 1e-4)])
    h = g.r_edges[1] - g.r_edges[0]
    g.rho = np.array([1.0])
    tab = I.CKTable(np.array([0.5]), np.ones(1), np.array([1000.0]), np.array([1.0]),
                    np.zeros((1, 1, 1, 1), np.float32), np.array([tau / h]))
    p = O.Params(n_packets=60000, seed=30, max_events=1, obs_phase=(0.0,))
    r = O.solve_albedo(g, tab, p)
    mu, w = CF.gauss01(64)
    S1 = om * 0.75 * 2.0 * (1 - np.exp(-tau * 2 / mu)) / (2 / mu)
    want = 0.5 * float((w * S1).sum())
    within(r.value[0, 0], want, r.stderr[0, 0], floor=2e-3 * want)
