"""Pins of the oracle's forced interactions (Sect. 4, forced interaction):
forced scattering, path-length stretching and their hybrid, on every
flight or on the first only ("forced first scattering").

- the forced optical depth follows the stated density q on [0, tp] (KS), and
  the weight factor makes it an importance sample of e^{-tau}: its mean is
  1 - e^{-tp} and its mean times tau is int_0^tp tau e^{-tau} dtau;
- exact single scattering from a thin slab: every scheme reproduces the
  closed form, with a smaller error than the unforced run;
- forced scattering keeps every packet's weight exactly (escaped fraction
  booked); every scheme leaves multiple-scattering albedo and emission
  unchanged within errors.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from paper_2110_15640_amd import inputs as I


def within(x, ref, se, k=3.0, floor=1e-13):
    assert abs(x - ref) <= k * se + floor * abs(ref), (x, ref, se, (x - ref) / max(se, 1e-300))


@pytest.mark.parametrize("kind", [1, 2, 3])
@pytest.mark.parametrize("tp", [0.05, 1.3, 9.0])
def test_forced_density_and_weights(kind, tp):
    rng = np.random.default_rng(5 + kind)
    n = 20000
    z, zc = rng.uniform(size=n), rng.uniform(size=n)
    tw = np.array([O.forced_tau(kind, tp, a, b) for a, b in zip(z, zc)])
    tau, w = tw[:, 0], tw[:, 1]
    assert np.all((tau >= 0.0) & (tau <= tp * (1 + 1e-12)))
    lam = 1.0 / (1.0 + tp)
    F1 = lambda t: (1 - np.exp(-t)) / (1 - math.exp(-tp))
    F2 = lambda t: (1 - np.exp(-lam * t)) / (1 - math.exp(-lam * tp))
    cdf = {1: F1, 2: F2, 3: lambda t: 0.5 * F1(t) + 0.5 * F2(t)}[kind]
    assert stats.kstest(tau, cdf).pvalue > 1e-3
    within(w.mean(), 1 - math.exp(-tp), w.std() / math.sqrt(n))
    m1 = 1 - math.exp(-tp) * (1 + tp)  # int_0^tp tau e^{-tau} dtau
    within((w * tau).mean(), m1, (w * tau).std() / math.sqrt(n))
    if kind == 1:
        np.testing.assert_allclose(w, 1 - math.exp(-tp), rtol=1e-14)


@pytest.mark.parametrize("kind,first", [(1, 0), (2, 0), (3, 0), (1, 1), (3, 1)])
def test_thin_slab_single_scattering(kind, first):
    tau, om, mu0 = 0.05, 0.9, 0.6
    g, t = I.make_homogeneous_slab(tau, om, g_cld=0.3)
    mu = 0.8
    ov = [math.sqrt(1 - mu * mu), 0.0, mu]
    n = 20000
    base = dict(n_packets=n, mu0=mu0, max_events=1, seed=151, obs_dir=np.array([ov]))
    plain = O.solve_albedo(g, t, O.Params(**base))
    forced = O.solve_albedo(g, t, O.Params(forced=kind, forced_first=first, **base))
    d0 = np.array([math.sqrt(1 - mu0 * mu0), 0.0, -mu0])
    kext = float(t.kappa.ravel()[0]) + float(g.cld_ksca[0])
    tau_e = kext * g.r_edges[-1]
    om_e = float(g.cld_ksca[0]) / kext
    P = O.phase_hg(float(d0 @ np.array(ov)), float(np.float32(0.3)))
    E = om_e * P / (4 * math.pi) * mu * (1 - math.exp(-tau_e * (1 / mu0 + 1 / mu))) / (mu + mu0)
    within(forced.value[0, 0] / math.pi, E, forced.stderr[0, 0] / math.pi)
    assert forced.stderr[0, 0] < 0.5 * plain.stderr[0, 0]  # forcing pays off in a thin slab


def test_forced_scattering_keeps_weight_exactly():
    g, t = I.make_albedo_slab(nlay=10, nlam=1)
    # without roulette a packet forced on every flight never leaves: the cap ends it
    r = O.solve_albedo(g, t, O.Params(n_packets=2000, seed=153, forced=1, rr_threshold=0.0, max_events=40),
                       keep_packets=True)
    _, K = r.extra["packets"][(0, 0)]
    np.testing.assert_allclose(K[:, :6].sum(axis=1), K[:, 10], rtol=1e-12)
    assert K[:, 8].sum() == 2000 and K[:, 0].min() > 0.0


@pytest.mark.parametrize("kind,first", [(1, 0), (2, 0), (3, 1)])
def test_multiple_scattering_is_unchanged(kind, first):
    g, t = I.make_homogeneous_slab(0.8, 0.95, g_cld=0.5, nlay=3)
    base = dict(n_packets=30000, mu0=0.5, seed=155, obs_dir=np.array([[0.3, 0.0, math.sqrt(0.91)]]))
    a = O.solve_albedo(g, t, O.Params(**base))
    b = O.solve_albedo(g, t, O.Params(forced=kind, forced_first=first, **base))
    within(b.value[0, 0] - a.value[0, 0], 0.0, math.hypot(a.stderr[0, 0], b.stderr[0, 0]))
    grid, tab, ph = I.make_emission_3d(12, 6, 8, nband=1, ng=1, config_no=44)
    tab.k_ray = tab.k_ray * 200.0
    e0 = O.solve_emission(grid, tab, O.Params(n_packets=20000, seed=157, obs_phase=(0.5,)))
    e1 = O.solve_emission(grid, tab, O.Params(n_packets=20000, seed=157, obs_phase=(0.5,), forced=kind,
                                              forced_first=first))
    within(e1.value[0, 0] - e0.value[0, 0], 0.0, math.hypot(e0.stderr[0, 0], e1.stderr[0, 0]))
