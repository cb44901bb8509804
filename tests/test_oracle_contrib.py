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
- the band functions add up to 1 per observer and reproduce the spectrum.
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
