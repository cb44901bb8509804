"""Pins of the oracle's contribution functions (per-cell peel-off tallies,
thermal and scattered parts; Sect. "Albedo and emission contribution
functions"):

- single scattering in a layered homogeneous slab: the scattered tally of
  each layer against the closed-form integral of e^{-tau/mu0} e^{-tau/mu}
  over that layer;
- pure-absorption emission on a small spherical grid: the thermal tally of
  every cell that the planet's shadow does not cut against a deterministic
  volume quadrature of (L_c/L_tot) <e^{-tau(r -> observer)}> / 4 pi, with the
  expected Monte Carlo spread from the same quadrature;
- the band functions add up to 1 per observer and reproduce the spectrum;
- images: an isothermal pure-absorption planet against pixel integrals of
  the closed-form B (1 - e^{-tau(b)}), and the orientation of the sky-plane
  axes with a single warm cell.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_2110_15640_amd import inputs as I


def test_single_scattering_layer_tallies():
    """Fixed incidence mu0, max_events = 1, homogeneous slab of 5 layers:
    E_k = omega Theta mu0^-1 / (1/mu0 + 1/mu) [e^{-tau_k s} - e^{-tau_{k+1} s}],
    s = 1/mu0 + 1/mu, per unit incident packet."""
    tau, om, mu0, nlay = 1.5, 0.7, 0.55, 5
    g, t = I.make_homogeneous_slab(tau, om, g_cld=0.0, nlay=nlay)
    mu, dphi = 0.8, 2.0
    s_ = math.sqrt(1 - mu * mu)
    ov = np.array([[s_ * math.cos(dphi), s_ * math.sin(dphi), mu]])
    n = 200_000
    p = O.Params(n_packets=n, mu0=mu0, max_events=1, seed=21, obs_dir=ov)
    r = O.solve_albedo(g, t, p, keep_packets=True, contrib=True)
    cf = r.extra["cf"][0, 0]  # [2][nlay], normalised
    assert np.all(cf[0] == 0.0)  # albedo has no thermal part
    np.testing.assert_allclose(cf.sum(), 1.0, rtol=1e-12)
    # unnormalised tallies per unit packet: cf * E_total
    E_tot = r.value[0, 0] / math.pi
    got = cf[1] * E_tot
    kext = float(t.kappa.ravel()[0]) + float(g.cld_ksca[0])
    om_e = float(g.cld_ksca[0]) / kext
    dtau = kext * (g.r_edges[1] - g.r_edges[0])
    ssum = 1.0 / mu0 + 1.0 / mu
    theta = 1.0 / (4.0 * math.pi)  # isotropic
    # layer k = 0 is the bottom; optical depth from the top to layer k's top face
    for k in range(nlay):
        top = (nlay - 1 - k) * dtau
        want = om_e * theta / mu0 / ssum * (math.exp(-top * ssum) - math.exp(-(top + dtau) * ssum))
        # per-packet f in layer k is a constant times e^{-tau/mu}: binomial-like spread
        fmax = om_e * theta * math.exp(-top / mu)
        se = math.sqrt(max(want * fmax, 1e-300) / n)
        assert abs(got[k] - want) <= 4.5 * se, (k, got[k], want, se)


def _cell_quadrature(grid, op, obs, m=8):
    """<e^{-tau}> and <e^{-2 tau}> over each cell's volume (midpoint rule in
    the volume-uniform coordinates u_r, u_sinlat, u_lon), and whether every
    point and corner of the cell sees the observer (the rule is only accurate
    where the planet's shadow does not cut the cell)."""
    u = (np.arange(m) + 0.5) / m
    nlon, nlat, nlay = grid.nlon, grid.nlat, grid.nlay
    m1 = np.zeros(grid.ncell)
    m2 = np.zeros(grid.ncell)
    visible = np.ones(grid.ncell, dtype=bool)
    for k in range(nlay):
        for j in range(nlat):
            for i in range(nlon):
                c = (k * nlat + j) * nlon + i
                r3a, r3b = grid.r_edges[k] ** 3, grid.r_edges[k + 1] ** 3
                sa, sb = math.sin(grid.lat_edges[j]), math.sin(grid.lat_edges[j + 1])
                la, lb = grid.lon_edges[i], grid.lon_edges[i + 1]
                acc1 = acc2 = 0.0
                for ur, us, ul in np.ndindex(2, 2, 2):  # corners, nudged inside
                    rr = (r3a + (0.001 + 0.998 * ur) * (r3b - r3a)) ** (1.0 / 3.0)
                    sl = sa + (0.001 + 0.998 * us) * (sb - sa)
                    cl = math.sqrt(max(1.0 - sl * sl, 0.0))
                    lo = la + (0.001 + 0.998 * ul) * (lb - la)
                    p = np.array([rr * cl * math.cos(lo), rr * cl * math.sin(lo), rr * sl])
                    visible[c] &= O.trace_segments(grid, p, obs, i, j, k, cap=512)[2] == 1
                for ur in u:
                    rr = (r3a + ur * (r3b - r3a)) ** (1.0 / 3.0)
                    for us in u:
                        sl = sa + us * (sb - sa)
                        cl = math.sqrt(max(1.0 - sl * sl, 0.0))
                        for ul in u:
                            lo = la + ul * (lb - la)
                            p = np.array([rr * cl * math.cos(lo), rr * cl * math.sin(lo), rr * sl])
                            cells, lens, term = O.trace_segments(grid, p, obs, i, j, k, cap=512)
                            tau = float(np.dot(op.a_ext[cells], lens)) if term == 1 else math.inf
                            visible[c] &= term == 1
                            acc1 += math.exp(-tau)
                            acc2 += math.exp(-2.0 * tau)
                m1[c] = acc1 / m ** 3
                m2[c] = acc2 / m ** 3
    return m1, m2, visible


def test_thermal_cell_tallies_against_volume_quadrature():
    grid, table, _ = I.make_emission_3d(6, 4, 4, nband=1, ng=1, config_no=30)
    # uniform density scaled to a radial optical depth of about 3 (each layer
    # about 0.75), so that the midpoint rule resolves e^{-tau} inside a cell
    grid.rho = np.ones(grid.ncell)
    a1 = O.ck_optics(grid, table, 0, 0).a_ext.reshape(grid.nlay, -1).mean(axis=1)
    grid.rho = np.full(grid.ncell, 3.0 / float(np.dot(a1, np.diff(grid.r_edges))))
    obs = O.emission_obs_dirs([0.4])
    n = 400_000
    p = O.Params(n_packets=n, seed=23, scattering=False, obs_phase=(0.4,), tau_vert_max=1e30)
    r = O.solve_emission(grid, table, p, contrib=True)
    cf = r.extra["cf"][0, 0]
    assert np.all(cf[1] == 0.0)  # no scattering: thermal part only
    op = O.ck_optics(grid, table, 0, 0)
    src = O.emission_sources(grid, op, table.lam_um[0], 1e30, 0.5)
    m1, m2, vis = _cell_quadrature(grid, op, obs[0], m=10)
    assert vis.sum() >= grid.ncell // 3
    frac = src.L / src.L_tot
    E = frac * m1 / (4.0 * math.pi)  # expected tally per packet, per cell
    q = np.where(src.wbirth > 0, frac / np.maximum(src.wbirth, 1e-300), 0.0)
    var = (q * src.wbirth ** 2 * m2 / (16 * math.pi ** 2) - E ** 2) / n
    got = cf[0] * (r.value[0, 0] * grid.r_toa ** 2 / src.L_tot)  # back to sum f / N
    se = np.sqrt(np.maximum(var, 0.0))
    bad = vis & (np.abs(got - E) > 4.5 * se + 3e-3 * E)
    assert not bad.any(), (np.argwhere(bad).ravel()[:5], got[bad][:3], E[bad][:3], se[bad][:3])


def test_band_function_sums_and_reproduces_the_spectrum():
    grid, table, ph = I.make_emission_3d(10, 6, 6, nband=2, ng=3, config_no=31)
    table.k_ray = table.k_ray * 300.0
    p = O.Params(n_packets=4000, seed=25, obs_phase=tuple(ph[:2]))
    r = O.solve_emission(grid, table, p, contrib=True)
    cf = r.extra["cf"]
    np.testing.assert_allclose(cf.sum(axis=(2, 3)), 1.0, rtol=1e-12)
    assert np.all(cf >= 0.0) and cf[:, :, 1].sum() > 0.0
    # the unnormalised per-g tallies add up to the packets' peel-off sums
    op = O.ck_optics(grid, table, 1, 2)
    src = O.emission_sources(grid, op, table.lam_um[1], 30.0, 0.5)
    obs = O.emission_obs_dirs(ph[:2])
    t = np.zeros((2, 2, grid.ncell))
    F, _ = O.transport(grid, op, p, 1, obs, sources=src, cf=t)
    np.testing.assert_allclose(t.sum(axis=(1, 2)), F.sum(axis=0), rtol=1e-12)
    # albedo: scattered part only
    ra = O.solve_albedo(grid, table, O.Params(n_packets=3000, seed=26, obs_phase=(0.0, 1.0)), contrib=True)
    assert np.all(ra.extra["cf"][:, :, 0] == 0.0)
    np.testing.assert_allclose(ra.extra["cf"].sum(axis=(2, 3)), 1.0, rtol=1e-12)


# ------------------------------------------------------------------ images
def _iso_grid():
    import closed_forms as CF  # noqa: F401  (shell sums below)
    g = I.make_sphere(16, 8, 10, seed=27)
    g.T = np.full(g.ncell, 1300.0, np.float32)
    alpha = 2e-8 * np.exp(-np.arange(10) / 2.0)
    g.rho = np.repeat(alpha, g.nlon * g.nlat)
    tab = I.CKTable(np.array([2.0]), np.ones(1), np.array([1000.0]), np.array([1.0]),
                    np.ones((1, 1, 1, 1), np.float32), np.zeros(1))
    return g, tab, alpha


def test_isothermal_image_against_pixel_integrals():
    """Pure absorption, isothermal, spherically symmetric extinction: pixel
    (row, col) of the image holds (1/R_TOA^2) int_pixel B (1 - e^{-tau(b)}) dA,
    tau the optical depth of the ray at impact distance b in front of the
    absorbing surface (closed-form shell sums), integrated by sub-sampling."""
    import closed_forms as CF
    g, tab, alpha = _iso_grid()
    npix, nb, nper = 10, 8, 40_000
    B = O.planck(2.0e-4, 1300.0)
    imgs = []
    for q in range(nb):  # independent packet ranges give the pixel spread
        p = O.Params(n_packets=nper, packet0=q * nper, seed=29, scattering=False, tau_vert_max=1e300,
                     obs_phase=(0.13,))
        imgs.append(O.solve_emission(g, tab, p, image_npix=npix).extra["image"][0, 0])
    imgs = np.array(imgs)
    got, se = imgs.mean(axis=0), imgs.std(axis=0, ddof=1) / math.sqrt(nb)
    R, r0 = g.r_toa, g.r_edges[0]
    m = 24
    want = np.zeros((npix, npix))
    w = 2.0 * R / npix
    for row in range(npix):
        for col in range(npix):
            us = -R + (col + (np.arange(m) + 0.5) / m) * w
            vs = -R + (row + (np.arange(m) + 0.5) / m) * w
            acc = 0.0
            for u in us:
                for v in vs:
                    b = math.hypot(u, v)
                    if b >= R:
                        continue
                    t = CF.chord_tau(b, g.r_edges, alpha) if b >= r0 else CF.surface_ray_tau(b, g.r_edges, alpha)
                    acc += 1.0 - math.exp(-t)
            want[row, col] = B * acc / (m * m) * w * w / R ** 2
    # the disk edge cuts some pixels: allow the sub-sampling error there
    edge = np.zeros_like(want, dtype=bool)
    for row in range(npix):
        for col in range(npix):
            cu = np.array([-R + col * w, -R + (col + 1) * w])
            cv = np.array([-R + row * w, -R + (row + 1) * w])
            bmin = math.hypot(max(0.0, abs(cu).min()) if cu[0] * cu[1] > 0 else 0.0,
                              max(0.0, abs(cv).min()) if cv[0] * cv[1] > 0 else 0.0)
            bmax = math.hypot(abs(cu).max(), abs(cv).max())
            edge[row, col] = bmin < R < bmax
    tol = 4.5 * se + np.where(edge, 0.02, 2e-3) * want + 1e-12 * want.max()
    bad = np.abs(got - want) > tol
    assert not bad.any(), (np.argwhere(bad)[:4].tolist(), got[bad][:4], want[bad][:4], se[bad][:4])
    np.testing.assert_allclose(got.sum(), want.sum(), rtol=5e-3)


def test_image_orientation_single_emitting_cell():
    """Only one cell is warm and the atmosphere is optically thin: the image
    falls inside the bounding box of that cell's corners projected on the
    observer's sky-plane axes (rows along e_v, columns along e_h)."""
    g = I.make_sphere(16, 8, 6, seed=41)
    hot = (3 * g.nlat + 6) * g.nlon + 5  # k = 3, j = 6 (northern), i = 5
    g.T = np.full(g.ncell, 30.0, np.float32)
    g.T[hot] = 1500.0
    g.rho = np.full(g.ncell, 1e-12)
    tab = I.CKTable(np.array([2.0]), np.ones(1), np.array([1000.0]), np.array([1.0]),
                    np.ones((1, 1, 1, 1), np.float32), np.zeros(1))
    npix = 32
    phases = (0.37, 0.81)
    p = O.Params(n_packets=20_000, seed=31, scattering=False, tau_vert_max=1e300, obs_phase=phases)
    r = O.solve_emission(g, tab, p, image_npix=npix)
    img = r.extra["image"][0]
    axes = O.image_axes(O.emission_obs_dirs(phases))
    k, j, i = 3, 6, 5
    corners = []
    for rr in g.r_edges[k:k + 2]:
        for la in np.linspace(g.lat_edges[j], g.lat_edges[j + 1], 5):
            for lo in np.linspace(g.lon_edges[i], g.lon_edges[i + 1], 5):
                corners.append([rr * math.cos(la) * math.cos(lo), rr * math.cos(la) * math.sin(lo), rr * math.sin(la)])
    corners = np.array(corners)
    R = g.r_toa
    for o in range(len(phases)):
        eh, ev = axes[o]
        u, v = corners @ eh, corners @ ev
        c0 = int(math.floor((u.min() + R) / (2 * R) * npix)) - 1
        c1 = int(math.floor((u.max() + R) / (2 * R) * npix)) + 1
        r0_ = int(math.floor((v.min() + R) / (2 * R) * npix)) - 1
        r1_ = int(math.floor((v.max() + R) / (2 * R) * npix)) + 1
        inside = img[o, max(r0_, 0):r1_ + 1, max(c0, 0):c1 + 1].sum()
        assert img[o].sum() > 0.0
        assert inside >= (1.0 - 1e-12) * img[o].sum(), (o, inside / img[o].sum())
        np.testing.assert_allclose(img[o].sum(), r.value[0, o], rtol=1e-12)
