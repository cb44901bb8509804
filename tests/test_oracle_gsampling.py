"""Pins of the oracle's per-packet g-ordinate sampling (Sect. "G-ordinance
biasing"): unbiased, uniform-biased and composite sampling of the
g-ordinate per packet, with weights p(g)/q(g).

- a single g-ordinate reduces every scheme to the fixed-g solve, packet by
  packet;
- the drawn g-ordinates follow q(g);
- single scattering in a homogeneous slab whose absorption depends on g:
  the band albedo equals sum_g w_g of the closed-form single-scattering
  values for every scheme;
- pure-absorption isothermal emission with g-dependent extinction: the band
  flux equals sum_g w_g B (projected emitting area)_g / R_TOA^2 (closed-form
  shell sums) for every scheme.
"""
import math

import numpy as np
import pytest

import closed_forms as CF
from oracle import oracle as O
from paper_2110_15640_amd import inputs as I


def within(x, ref, se, k=3.0):
    assert abs(x - ref) <= k * se, (x, ref, se, (x - ref) / max(se, 1e-300))


@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_single_g_reduces_to_fixed_g_solve(scheme):
    grid, table, ph = I.make_emission_3d(10, 6, 6, nband=2, ng=1, config_no=40)
    table.k_ray = table.k_ray * 100.0
    base = dict(n_packets=3000, seed=41, obs_phase=tuple(ph[:2]))
    a = O.solve_emission(grid, table, O.Params(**base), keep_packets=True)
    b = O.solve_emission(grid, table, O.Params(g_sampling=scheme, **base), keep_packets=True)
    for s in range(2):
        np.testing.assert_array_equal(a.extra["packets"][(s, 0)][0], b.extra["packets"][(s, 0)][0])
    np.testing.assert_allclose(b.value, a.value, rtol=1e-14)
    ra = O.solve_albedo(grid, table, O.Params(**base))
    rb = O.solve_albedo(grid, table, O.Params(g_sampling=scheme, **base))
    np.testing.assert_allclose(rb.value, ra.value, rtol=1e-14)


def _g_table(kabs, weights):
    ng = len(kabs)
    kap = np.asarray(kabs, dtype=np.float32).reshape(1, ng, 1, 1)
    return I.CKTable(np.array([0.5]), np.asarray(weights, dtype=np.float64), np.array([1000.0]), np.array([1.0]),
                     kap, np.zeros(1))


@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_draws_follow_q(scheme):
    grid, _ = I.make_homogeneous_slab(0.5, 0.5, g_cld=0.0)
    w = np.array([0.1, 0.25, 0.4, 0.25])
    table = _g_table([1e-8, 2e-8, 4e-8, 8e-8], w)
    q, wf = O.g_sampling_weights(scheme, w)
    ops = [O.ck_optics(grid, table, 0, g) for g in range(4)]
    n = 40000
    _, _, G = O.transport_gsampled(grid, ops, O.Params(n_packets=n, seed=43, mu0=0.7), 0, None, q, wf)
    cnt = np.bincount(G, minlength=4)
    p = q / q.sum()
    for h in range(4):
        within(cnt[h], n * p[h], math.sqrt(n * p[h] * (1 - p[h])), k=5.0)


@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_single_scattering_band_albedo(scheme):
    """A_band / pi = sum_g w_g omega_g P/(4 pi) mu (1 - e^{-tau_g (1/mu0 + 1/mu)}) / (mu + mu0)."""
    H = 8388608.0
    g, _ = I.make_homogeneous_slab(1.0, 1.0, g_cld=0.0)
    ksca = 0.5 / H
    g.cld_ksca = np.full(1, ksca, np.float32)
    kabs = np.array([0.05, 0.4, 1.5, 6.0]) / H
    w = np.array([0.3, 0.3, 0.25, 0.15])
    table = _g_table(kabs, w)
    mu0 = 0.6
    mu = 0.75
    ov = [math.sqrt(1 - mu * mu), 0.0, mu]
    n = 80000
    p = O.Params(n_packets=n, mu0=mu0, max_events=1, seed=45, obs_dir=np.array([ov]), g_sampling=scheme)
    r = O.solve_albedo(g, table, p)
    want = 0.0
    for h in range(4):
        ke = float(np.float32(kabs[h])) + float(np.float32(ksca))
        om = float(np.float32(ksca)) / ke
        tau = ke * H
        want += w[h] * om / (4 * math.pi) * mu * (1 - math.exp(-tau * (1 / mu0 + 1 / mu))) / (mu + mu0)
    within(r.value[0, 0] / math.pi, want, r.stderr[0, 0] / math.pi)
    assert abs(r.value[0, 0] / math.pi / want - 1.0) < 3e-2


@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_isothermal_band_emission(scheme):
    grid = I.make_sphere(12, 6, 8, seed=47)
    grid.T = np.full(grid.ncell, 1300.0, np.float32)
    alpha = 2e-8 * np.exp(-np.arange(8) / 2.0)
    grid.rho = np.repeat(alpha, grid.nlon * grid.nlat)
    fac = np.array([0.05, 0.3, 1.0, 4.0])
    w = np.array([0.35, 0.3, 0.2, 0.15])
    table = I.CKTable(np.array([2.0]), w, np.array([1000.0]), np.array([1.0]),
                      fac.astype(np.float32).reshape(1, 4, 1, 1), np.zeros(1))
    n = 60000
    p = O.Params(n_packets=n, seed=49, scattering=False, tau_vert_max=1e300, obs_phase=(0.5,), g_sampling=scheme)
    r = O.solve_emission(grid, table, p)
    B = O.planck(2.0e-4, 1300.0)
    want = sum(w[h] * B * CF.isothermal_disk_integral(grid.r_edges, alpha * float(np.float32(fac[h])))
               for h in range(4)) / grid.r_toa ** 2
    within(r.value[0, 0], want, r.stderr[0, 0])
    assert abs(r.value[0, 0] / want - 1.0) < 2e-2
