"""Pins of the oracle's spherical and slab traversal against closed-form chord
lengths and brute-force point classification along the ray."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2110_15640_amd import inputs as I


def shell_chord(b, ri, ro):
    """Length of a full chord at impact parameter b inside shell [ri, ro]."""
    f = lambda r: math.sqrt(max(r * r - b * b, 0.0))
    return 2.0 * (f(ro) - f(max(ri, b)))


def brute_lengths(grid, p, d, length, n=400000):
    """Path length per cell by classifying midpoints of n equal steps."""
    h = length / n
    s = (np.arange(n) + 0.5) * h
    pts = p[None, :] + s[:, None] * d[None, :]
    r = np.linalg.norm(pts, axis=1)
    lat = np.arctan2(pts[:, 2], np.hypot(pts[:, 0], pts[:, 1]))
    lon = np.arctan2(pts[:, 1], pts[:, 0])
    k = np.searchsorted(grid.r_edges, r, side="right") - 1
    j = np.clip(np.searchsorted(grid.lat_edges, lat, side="right") - 1, 0, grid.nlat - 1)
    i = np.clip(np.searchsorted(grid.lon_edges, lon, side="right") - 1, 0, grid.nlon - 1)
    inside = (k >= 0) & (k < grid.nlay)
    c = (k * grid.nlat + j) * grid.nlon + i
    out = {}
    for cc in c[inside]:
        out[int(cc)] = out.get(int(cc), 0.0) + h
    return out, h


def test_1d_shell_chords_exact():
    g = I.make_sphere(1, 1, 12, seed=3)
    rt, r0 = g.r_toa, g.r0
    for b in np.linspace(r0 * 1.0000001, rt * 0.9999999, 37):
        p = np.array([math.sqrt(rt * rt - b * b), b * 0.6, b * 0.8])
        p[1:] = [0.0, b]
        cells, lens, term = O.trace_segments(g, p, [-1.0, 0.0, 0.0], 0, 0, g.nlay - 1, ef=0)
        assert term == 1
        per = np.zeros(g.nlay)
        for c, L in zip(cells, lens):
            per[c] += L
        for k in range(g.nlay):
            want = shell_chord(b, g.r_edges[k], g.r_edges[k + 1])
            assert abs(per[k] - want) <= 1e-9 * max(want, 1.0) + 1e-6, (b, k)


def _start_cell(g, p):
    lat = math.atan2(p[2], math.hypot(p[0], p[1]))
    lon = math.atan2(p[1], p[0])
    j = min(max(int(np.searchsorted(g.lat_edges, lat, side="right") - 1), 0), g.nlat - 1)
    i = min(max(int(np.searchsorted(g.lon_edges, lon, side="right") - 1), 0), g.nlon - 1)
    k = int(np.searchsorted(g.r_edges, np.linalg.norm(p), side="right") - 1)
    return i, j, k


def test_3d_traversal_matches_brute_force():
    g = I.make_sphere(12, 6, 5, seed=4)
    rng = np.random.default_rng(11)
    rt, r0 = g.r_toa, g.r0
    checked = 0
    for trial in range(60):
        # random interior start point and direction, some near the poles
        r = r0 + (rt - r0) * rng.uniform(0.05, 0.95)
        lat = rng.uniform(-1.5, 1.5) if trial % 3 else math.copysign(1.55, rng.normal())
        lon = rng.uniform(-math.pi, math.pi)
        p = r * np.array([math.cos(lat) * math.cos(lon), math.cos(lat) * math.sin(lon), math.sin(lat)])
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        i, j, k = _start_cell(g, p)
        cells, lens, term = O.trace_segments(g, p, d, i, j, k, ef=-1)
        assert term in (1, 2)
        total = float(lens.sum())
        # ray end point must sit on the outer boundary or on the surface
        end = p + total * d
        assert abs(np.linalg.norm(end) - (rt if term == 1 else r0)) < 1e-6 * rt
        got = {}
        for c, L in zip(cells, lens):
            got[int(c)] = got.get(int(c), 0.0) + float(L)
        want, h = brute_lengths(g, p, d, total)
        for c in set(got) | set(want):
            assert abs(got.get(c, 0.0) - want.get(c, 0.0)) <= 4 * h, (trial, c)
        checked += 1
    assert checked == 60


def test_3d_chord_sums_to_shell_lengths():
    g = I.make_sphere(16, 8, 6, seed=5)
    rt, r0 = g.r_toa, g.r0
    for a in (0.1, 1.3, math.pi / 2 + 1e-3, 2.9, 4.4):
        for b in (r0 * 1.001, 0.37 * r0 + 0.63 * rt, rt * 0.999):
            p = np.array([math.sqrt(rt * rt - b * b), b * math.cos(a), b * math.sin(a)])
            i, j, _ = _start_cell(g, p)
            cells, lens, term = O.trace_segments(g, p, [-1.0, 0.0, 0.0], i, j, g.nlay - 1, ef=0)
            assert term == 1
            per = np.zeros(g.nlay)
            for c, L in zip(cells, lens):
                per[c // (g.nlon * g.nlat)] += L
            for k in range(g.nlay):
                want = shell_chord(b, g.r_edges[k], g.r_edges[k + 1])
                assert abs(per[k] - want) <= 1e-9 * rt


def test_slab_traversal():
    g, _ = I.make_albedo_slab(nlay=7)
    z = g.r_edges
    mu = 0.37
    d = np.array([math.sqrt(1 - mu * mu), 0.0, -mu])
    cells, lens, term = O.trace_segments(g, [0.0, 0.0, z[-1]], d, 0, 0, 6, ef=0)
    assert term == 2 and list(cells) == list(range(6, -1, -1))
    np.testing.assert_allclose(lens, np.diff(z)[::-1] / mu, rtol=1e-14)
    cells, lens, term = O.trace_segments(g, [0.0, 0.0, 0.5 * (z[2] + z[3])], -d, 0, 0, 2, ef=-1)
    assert term == 1 and list(cells) == [2, 3, 4, 5, 6]
    assert lens[0] == pytest.approx((z[3] - 0.5 * (z[2] + z[3])) / mu, rel=1e-14)
