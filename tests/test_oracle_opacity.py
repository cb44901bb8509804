"""Pins of the oracle's opacity gathers, Doppler shift, Planck function and
emission sources."""
import math

import numpy as np
import pytest
from scipy import integrate

import closed_forms as CF
from oracle import oracle as O
from paper_2110_15640_amd import inputs as I


def _grid_with(T, P):
    n = len(T)
    return I.Grid(1, 1, 1, n, np.linspace(0, 1, n + 1), np.array([-1.5707963267948966, 1.5707963267948966]),
                  np.array([-math.pi, math.pi]), np.asarray(T, np.float32), np.asarray(P, np.float32),
                  np.ones(n))


def _table(fn, nT=5, nP=6):
    Tg = np.linspace(600.0, 2600.0, nT)
    Pg = 10.0 ** np.linspace(-4, 2, nP)
    kap = np.array([[fn(t, p) for p in Pg] for t in Tg], dtype=np.float32)[None, None]
    return I.CKTable(np.array([1.0]), np.ones(1), Tg, Pg, kap, np.zeros(1))


def test_ck_gather_reproduces_power_law_in_pressure():
    """ln kappa linear in ln P: bilinear in (T, ln P) on ln kappa is exact at
    tabulated T for any P inside the table, and clamps outside it."""
    tab = _table(lambda t, p: 0.03 * (t / 1000.0) * p ** 0.7)
    Ps = np.array([1e-4, 3.3e-3, 0.05, 0.71, 9.0, 100.0], np.float32)
    T = np.full(len(Ps), 1100.0, np.float32)
    op = O.ck_optics(_grid_with(T, Ps), tab, 0, 0)
    want = 0.03 * 1.1 * Ps.astype(np.float64) ** 0.7
    np.testing.assert_allclose(op.a_abs, want, rtol=2e-7)  # float32 table entries
    op2 = O.ck_optics(_grid_with(np.array([100.0, 9000.0], np.float32), np.array([1e-9, 1e5], np.float32)),
                      tab, 0, 0)
    assert op2.a_abs[0] == pytest.approx(0.03 * 0.6 * 1e-4 ** 0.7, rel=2e-7)
    assert op2.a_abs[1] == pytest.approx(0.03 * 2.6 * 100.0 ** 0.7, rel=2e-7)


def test_ck_gather_is_geometric_between_temperatures():
    tab = _table(lambda t, p: 1e-3 if t < 1500 else 4e-3)
    # half way between T nodes 1100 and 1600: sqrt(1e-3 * 4e-3) = 2e-3
    op = O.ck_optics(_grid_with([1350.0], [1.0]), tab, 0, 0)
    assert op.a_abs[0] == pytest.approx(2e-3, rel=1e-7)


def test_ck_gather_zero_corner_gives_zero_only_with_weight():
    tab = _table(lambda t, p: 0.0 if t > 2000 else 1e-2)
    op = O.ck_optics(_grid_with([1600.0, 2100.0, 1350.0], [1.0, 1.0, 1.0]), tab, 0, 0)
    assert op.a_abs[0] == pytest.approx(1e-2, rel=1e-7)  # at a node: the zero corner has weight 0
    assert op.a_abs[1] == 0.0
    assert op.a_abs[2] == pytest.approx(1e-2, rel=1e-7)


def test_ck_albedo_and_gas_fraction():
    g = _grid_with([1000.0] * 3, [1.0] * 3)
    g.rho = np.array([2.0, 2.0, 2.0])
    g.cld_ksca = np.array([0.0, 3.0, 1.0], np.float32)
    g.cld_kabs = np.array([0.0, 0.0, 1.0], np.float32)
    g.cld_g = np.array([0.0, 0.4, 0.8], np.float32)
    tab = _table(lambda t, p: 1.0)
    tab.k_ray = np.array([1.0])
    op = O.ck_optics(g, tab, 0, 0)
    # cell 0: kabs 1, kray 1 ; cell 1: kabs 1, kray 1, ksca 3 ; cell 2: kabs 1+1, kray 1, ksca 1
    np.testing.assert_allclose(op.a_ext, [4.0, 10.0, 8.0], rtol=1e-7)
    np.testing.assert_allclose(op.omega, [0.5, 0.8, 0.5], rtol=1e-7)
    np.testing.assert_allclose(op.p_gas, [1.0, 0.25, 0.5], rtol=1e-7)
    np.testing.assert_allclose(op.g_cld, [0.0, 0.4, 0.8], rtol=1e-7)


def _paper_vlos(u, v, w, omega, r, colat, lon, colat_v, lon_v):
    """The v_LOS equation of the paper, read with colatitudes for theta and
    theta_v (the only reading under which it is the line-of-sight speed)."""
    t, tv, dp = colat, colat_v, lon - lon_v
    return (u * math.sin(tv) * math.sin(dp)
            + (v * math.cos(t) - w * math.sin(t)) * math.sin(tv) * math.cos(dp)
            - (v * math.sin(t) + w * math.cos(t)) * math.cos(tv)
            + omega * r * math.sin(t) * math.sin(tv) * math.sin(dp))


def test_doppler_shift_matches_paper_component_form():
    g = I.make_sphere(8, 4, 3, seed=7)
    rng = np.random.default_rng(2)
    g.u = rng.normal(0, 3e5, g.ncell).astype(np.float32)
    g.v = rng.normal(0, 2e5, g.ncell).astype(np.float32)
    g.w = rng.normal(0, 1e4, g.ncell).astype(np.float32)
    g.omega_rot = 2.1e-5
    dln = 4.77e-6
    for colat_v, lon_v in [(math.pi / 2, math.pi), (0.7, 0.3), (2.0, -1.2)]:
        o = np.array([math.sin(colat_v) * math.cos(lon_v), math.sin(colat_v) * math.sin(lon_v), math.cos(colat_v)])
        sh = O.doppler_shift(g, o, dln)
        for c in range(0, g.ncell, 5):
            i, j, k = c % g.nlon, (c // g.nlon) % g.nlat, c // (g.nlon * g.nlat)
            r = 0.5 * (g.r_edges[k] + g.r_edges[k + 1])
            lat = 0.5 * (g.lat_edges[j] + g.lat_edges[j + 1])
            lon = 0.5 * (g.lon_edges[i] + g.lon_edges[i + 1])
            vl = _paper_vlos(float(g.u[c]), float(g.v[c]), float(g.w[c]), g.omega_rot, r,
                             math.pi / 2 - lat, lon, colat_v, lon_v)
            want = math.log1p(-vl / 2.99792458e10) / dln
            assert sh[c] == pytest.approx(want, rel=1e-9, abs=1e-9)


def test_uniform_recession_shifts_spectrum_by_whole_indices():
    """A uniform receding speed with ln(1 - v/c) = -3 dlnlam moves every
    cell's opacity three table points to the blue: alpha(n) = alpha0(n - 3)."""
    g = I.make_sphere(8, 4, 3, seed=8)
    gh, tab = I.make_transmission_hires(8, 4, 3, nlam=64, nT=4, nP=4)
    dln = tab.dlnlam
    V = 2.99792458e10 * (1.0 - math.exp(-3.0 * dln))
    latc = 0.5 * (g.lat_edges[:-1] + g.lat_edges[1:])
    lonc = 0.5 * (g.lon_edges[:-1] + g.lon_edges[1:])
    # velocity V along +x (receding from an observer at -x)
    U = np.zeros(g.ncell); Vn = np.zeros(g.ncell); Wr = np.zeros(g.ncell)
    for k in range(g.nlay):
        for j in range(g.nlat):
            for i in range(g.nlon):
                c = (k * g.nlat + j) * g.nlon + i
                th, ph = latc[j], lonc[i]
                U[c] = -V * math.sin(ph)
                Vn[c] = -V * math.sin(th) * math.cos(ph)
                Wr[c] = V * math.cos(th) * math.cos(ph)
    g.u, g.v, g.w = U, Vn, Wr  # float64 winds keep the speed exact enough
    sh = O.doppler_shift(g, np.array([-1.0, 0.0, 0.0]), dln)
    np.testing.assert_allclose(sh, -3.0, atol=1e-6)
    for n in (3, 10, 40, 63):
        # line absorption moves; Rayleigh stays at the rest wavelength
        a = O.hires_optics(g, tab, n, sh).a_abs
        a0 = O.hires_optics(g, tab, n - 3, None).a_abs
        np.testing.assert_allclose(a, a0, rtol=1e-5)
    # no winds: no shift
    np.testing.assert_array_equal(O.hires_optics(g, tab, 5, np.zeros(g.ncell)).a_ext,
                                  O.hires_optics(g, tab, 5, None).a_ext)


def test_planck_stefan_boltzmann_and_wien():
    for T in (300.0, 1200.0, 5800.0):
        v, _ = integrate.quad(lambda l: O.planck(l, T), 1e-6, 1.0, limit=500, epsrel=1e-11,
                              points=[CF.WIEN_B / T])
        assert v == pytest.approx(CF.SIGMA_SB * T ** 4 / math.pi, rel=1e-7)
        lam = np.linspace(0.8, 1.2, 20001) * CF.WIEN_B / T
        peak = lam[np.argmax([O.planck(l, T) for l in lam])]
        assert peak == pytest.approx(CF.WIEN_B / T, rel=1e-4)


def test_emission_sources_cdf_and_weights():
    g, tab, _ = I.make_emission_3d(8, 4, 6, nband=3, ng=2)
    op = O.ck_optics(g, tab, 1, 1)
    src = O.emission_sources(g, op, tab.lam_um[1], 1e300, 0.5)
    assert src.n_emit == g.ncell and src.L_tot == pytest.approx(src.L.sum(), rel=1e-12)
    assert src.cdf[-1] == pytest.approx(1.0, rel=1e-12)
    q = np.diff(np.concatenate([[0.0], src.cdf]))
    np.testing.assert_allclose(src.wbirth * q, src.L / src.L_tot, rtol=1e-9)
    # total volume of the shells
    vol = 4 * math.pi / 3 * (g.r_toa ** 3 - g.r0 ** 3)
    Lhat = src.L / (4 * math.pi * op.a_abs * np.array([O.planck(tab.lam_um[1] * 1e-4, t) for t in g.T]))
    assert Lhat.sum() == pytest.approx(vol, rel=1e-12)


def test_vertical_tau_cut():
    """Homogeneous extinction: a cell emits iff the column optical depth above
    its top face is <= tau_vert."""
    g = I.make_sphere(4, 2, 10, seed=9)
    n = g.ncell
    dr = g.r_edges[1] - g.r_edges[0]
    a = np.full(n, 3.3 / dr)  # 3.3 per layer
    op = O.Optics(a, a.copy(), np.zeros(n), np.ones(n), np.zeros(n))
    src = O.emission_sources(g, op, 2.0, 10.0, 0.5)
    k = np.arange(n) // (g.nlon * g.nlat)
    tau_above = 3.3 * (g.nlay - 1 - k)
    assert np.array_equal(src.L > 0, tau_above <= 10.0 + 1e-9)
    assert src.n_emit == 4 * g.nlon * g.nlat
