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


def _linear_hires_table(nlam=16, a=0.5, b=0.125, p_pow=0.0):
    """kappa(n, T, P) = (a + b n) (P / 1 bar)^p_pow: linear in the wavelength
    index (exact in float32), so the Doppler interpolation is checked alone."""
    Tg = np.array([800.0, 1600.0, 2400.0])
    Pg = np.array([1e-2, 1.0, 100.0])
    kap = ((a + b * np.arange(nlam))[:, None, None] * np.ones(3)[None, :, None] *
           (Pg[None, None, :] ** p_pow)).astype(np.float32)
    return I.HiresTable(1.0, 1e-5, Tg, Pg, kap, np.zeros(nlam))


def test_doppler_interpolation_is_linear_in_kappa_at_fractional_shifts():
    """At lambda_eff between two table wavelengths the oracle interpolates
    kappa linearly in the (fractional) log-uniform index.  With kappa_n =
    a + b n the result must be a + b (n + shift) exactly (to rounding);
    interpolating ln kappa instead would give a geometric mean, off by up to
    ~1e-2 here.  Cells sit on (T, P) nodes, also with a power law in P."""
    g = I.make_sphere(8, 4, 3, seed=11)
    rng = np.random.default_rng(4)
    Tn, Pn = np.array([800.0, 1600.0, 2400.0]), np.array([1e-2, 1.0, 100.0])
    g.T = Tn[rng.integers(0, 3, g.ncell)].astype(np.float32)
    g.P = Pn[rng.integers(0, 3, g.ncell)].astype(np.float32)
    nlam, a, b = 16, 0.5, 0.125
    for p_pow in (0.0, 0.5):
        tab = _linear_hires_table(nlam, a, b, p_pow)
        pfac = g.P.astype(np.float64) ** p_pow
        for frac in (-2.5, -0.3, 0.75, 3.125):
            sh = np.full(g.ncell, frac) + rng.uniform(-0.49, 0.49, g.ncell)
            for n in (4, 7, 11):
                x = n + sh  # stays inside [0, nlam - 1] for these n and shifts
                assert x.min() > 0.0 and x.max() < nlam - 1
                got = O.hires_optics(g, tab, n, sh).a_abs
                # exact to rounding; with the power law the float32 table
                # entries carry ~6e-8 (a ln-kappa interpolation is off by >= 5e-4)
                np.testing.assert_allclose(got, g.rho * (a + b * x) * pfac, rtol=1e-12 if p_pow == 0.0 else 2e-7)
    # a uniform recession of 2.5 table steps gives the fractional shift the
    # same way (observer at -x, speed V along +x)
    dln = _linear_hires_table().dlnlam
    V = 2.99792458e10 * (1.0 - math.exp(-2.5 * dln))
    latc = 0.5 * (g.lat_edges[:-1] + g.lat_edges[1:])
    lonc = 0.5 * (g.lon_edges[:-1] + g.lon_edges[1:])
    kk, jj, ii = np.meshgrid(np.arange(g.nlay), np.arange(g.nlat), np.arange(g.nlon), indexing="ij")
    th, ph = latc[jj.ravel()], lonc[ii.ravel()]
    g.u, g.v, g.w = -V * np.sin(ph), -V * np.sin(th) * np.cos(ph), V * np.cos(th) * np.cos(ph)
    sh = O.doppler_shift(g, np.array([-1.0, 0.0, 0.0]), dln)
    np.testing.assert_allclose(sh, -2.5, atol=1e-6)
    tab = _linear_hires_table()
    np.testing.assert_allclose(O.hires_optics(g, tab, 9, sh).a_abs, g.rho * (a + b * (9 + sh)), rtol=1e-12)


def test_doppler_interpolation_clamps_at_the_table_ends():
    """lambda_eff outside the table takes the end value: kappa_0 below the
    first wavelength, kappa_{nlam-1} above the last."""
    g = I.make_sphere(8, 4, 3, seed=12)
    g.T = np.full(g.ncell, 1600.0, np.float32)
    g.P = np.full(g.ncell, 1.0, np.float32)
    nlam, a, b = 16, 0.5, 0.125
    tab = _linear_hires_table(nlam, a, b)
    rng = np.random.default_rng(5)
    lo = -rng.uniform(0.0, 40.0, g.ncell)
    for n in (0, 1, 2):
        sh = lo - n  # n + shift <= 0
        np.testing.assert_allclose(O.hires_optics(g, tab, n, sh).a_abs, g.rho * a, rtol=1e-12)
    hi = rng.uniform(0.0, 40.0, g.ncell)
    for n in (nlam - 1, nlam - 2, nlam - 5):
        sh = hi + (nlam - 1 - n)  # n + shift >= nlam - 1
        np.testing.assert_allclose(O.hires_optics(g, tab, n, sh).a_abs, g.rho * (a + b * (nlam - 1)), rtol=1e-12)
    # exactly on an end and one step inside: no clamping artefact
    sh = np.zeros(g.ncell)
    np.testing.assert_allclose(O.hires_optics(g, tab, nlam - 1, sh).a_abs, g.rho * (a + b * (nlam - 1)), rtol=1e-12)
    np.testing.assert_allclose(O.hires_optics(g, tab, 0, sh + 0.5).a_abs, g.rho * (a + 0.5 * b), rtol=1e-12)
