"""The allocation-free solve (mcrt_solve_noalloc) through the C ABI: its
scratch is the library's fixed per-device array, and its results equal those
of the blocking solve of the same request bit for bit, on two calls in a row
(the second smaller, so stale contents of the array from the first call must
not leak into it)."""
import numpy as np
import pytest

from paper_2110_15640_amd import inputs as I

pytestmark = pytest.mark.gpu

KEYS = ("sums", "value", "stderr", "per_g", "counters", "l_tot")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _same(a, b, what):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), (what, k)


def test_noalloc_emission_equals_blocking_solve_twice(torch_dev):
    from paper_2110_15640_amd import mcrt as M
    grid, ck, phases = I.make_emission_3d(32, 16, 20, nband=6, ng=4)
    with M.Context(0) as ctx:
        gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(ck)
        held = ctx.memory_in_use
        # first call: 24 solves x 2e5 packets of 15-double rows (~0.6 GB of
        # rows) -- several launches through the 256 MiB array
        kw1 = dict(n_packets=200_000, obs_phase=list(phases), seed=11, precision=M.MCRT_MIXED)
        print("noalloc: emission 32x16x20, 6 bands x 4 g x 2e5 packets, mixed", flush=True)
        a = ctx.solve_noalloc("emission", gid, oid, ck, **kw1)
        assert ctx.memory_in_use == held
        ref = ctx.solve_emission(gid, oid, ck, **kw1)
        _same(a, ref, "emission call 1")
        # second call: fewer bands, fewer packets, FP64
        kw2 = dict(n_packets=3_000, obs_phase=list(phases[:2]), seed=12, precision=M.MCRT_FP64,
                   spec_idx=[1, 4])
        print("noalloc: emission, 2 bands x 4 g x 3e3 packets, fp64", flush=True)
        b = ctx.solve_noalloc("emission", gid, oid, ck, **kw2)
        ref2 = ctx.solve_emission(gid, oid, ck, **kw2)
        _same(b, ref2, "emission call 2")
        # per-packet g-ordinate sampling: whole bands per launch
        kw3 = dict(n_packets=40_000, obs_phase=list(phases), seed=13, precision=M.MCRT_MIXED, g_sampling=3)
        print("noalloc: emission with composite g sampling", flush=True)
        c = ctx.solve_noalloc("emission", gid, oid, ck, **kw3)
        _same(c, ctx.solve_emission(gid, oid, ck, **kw3), "emission g sampling")
        assert ctx.memory_in_use >= held


def test_noalloc_albedo_equals_blocking_solve_twice(torch_dev):
    from paper_2110_15640_amd import mcrt as M
    slab, ck = I.make_albedo_slab(nlay=50, nlam=10)
    with M.Context(0) as ctx:
        gid, oid = ctx.upload_grid(slab), ctx.upload_opacity(ck)
        kw1 = dict(n_packets=100_000, seed=3)
        print("noalloc: slab albedo, 10 wavelengths x 1e5 packets", flush=True)
        a = ctx.solve_noalloc("albedo", gid, oid, ck, **kw1)
        _same(a, ctx.solve_albedo(gid, oid, ck, **kw1), "albedo call 1")
        kw2 = dict(n_packets=777, seed=4, spec_idx=[2], precision=M.MCRT_MIXED)
        print("noalloc: slab albedo, 1 wavelength x 777 packets, mixed", flush=True)
        b = ctx.solve_noalloc("albedo", gid, oid, ck, **kw2)
        _same(b, ctx.solve_albedo(gid, oid, ck, **kw2), "albedo call 2")


def test_noalloc_rejections(torch_dev):
    from paper_2110_15640_amd import mcrt as M
    slab, ck = I.make_albedo_slab(nlay=10, nlam=2)
    with M.Context(0) as ctx:
        gid, oid = ctx.upload_grid(slab), ctx.upload_opacity(ck)
        print("noalloc: rejections (host checks only, nothing launched)", flush=True)
        # one solve of 3e6 packets needs 3e6 x 12 x 8 B of rows > 256 MiB
        with pytest.raises(M.McrtError) as e:
            ctx.solve_noalloc("albedo", gid, oid, ck, n_packets=3_000_000, spec_idx=[0])
        assert e.value.name == "EINVAL" and "fixed" in str(e.value)
        with pytest.raises(M.McrtError) as e:
            ctx.solve_noalloc("albedo", gid, oid, ck, n_packets=100, graph=1)
        assert e.value.name == "EINVAL"
        L = M.load()
        p = M.default_params()
        p.n_packets = 100
        r = M.Result()
        assert L.mcrt_solve_noalloc(ctx._h, M.MODES["transmission"], gid, oid, p, r) == -1
        # the context still works afterwards
        ok = ctx.solve_noalloc("albedo", gid, oid, ck, n_packets=1000, seed=1)
        _same(ok, ctx.solve_albedo(gid, oid, ck, n_packets=1000, seed=1), "albedo after rejections")
