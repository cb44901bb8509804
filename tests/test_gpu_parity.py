"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs and the same Philox stream.

FP64 per-packet peel-off sums must agree to 1e-9 relative (absolute floor
1e-12 of the largest packet value); solve values and counters to 1e-9.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2110_15640_amd import inputs as I

pytestmark = pytest.mark.gpu

RTOL = 1e-9


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx(torch_dev):
    from paper_2110_15640_amd import mcrt as M
    c = M.Context(0)
    yield c
    c.close()


def dump_buffer(torch, nsolve, n, nout):
    return torch.zeros(nsolve * n * nout, dtype=torch.float64, device="cuda:0")


def check_packets(dump, ref, shape):
    d = dump.cpu().numpy().reshape(shape)
    ns, ng, n, no = shape
    for s in range(ns):
        for g in range(ng):
            F = ref.extra["packets"][(s, g)][0]
            scale = max(float(np.abs(F).max()), 1e-300)
            bad = np.abs(d[s, g] - F) > RTOL * np.abs(F) + 1e-12 * scale
            assert not bad.any(), (s, g, np.argwhere(bad)[:5].tolist(), d[s, g][bad][:3], F[bad][:3])


def check_solve(got, ref, counters=True):
    np.testing.assert_allclose(got["value"], ref.value, rtol=RTOL, atol=1e-300)
    np.testing.assert_allclose(got["per_g"], ref.per_g, rtol=RTOL, atol=1e-300)
    np.testing.assert_allclose(got["sums"], ref.sums, rtol=RTOL, atol=1e-300)
    if counters:
        c_ref = ref.counters
        np.testing.assert_allclose(got["counters"], c_ref, rtol=RTOL, atol=1e-12 * max(c_ref.max(), 1.0))


def test_albedo_slab_parity(ctx, torch_dev):
    _log("albedo slab parity: 10 wavelengths x 3000 packets, uniform-disk incidence")
    grid, table = I.make_albedo_slab()
    n = 3000  # ragged: not a multiple of the 256-lane block
    dump = dump_buffer(torch_dev, 10, n, 1)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    got = ctx.solve_albedo(gid, oid, table, n_packets=n, seed=101, packet_dump=dump)
    ref = O.solve_albedo(grid, table, O.Params(n_packets=n, seed=101), keep_packets=True)
    check_packets(dump, ref, (10, 1, n, 1))
    check_solve(got, ref)
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_albedo_slab_fixed_incidence_and_observers(ctx, torch_dev):
    _log("albedo slab parity: mu0 = 0.42, 3 explicit observers, continuous absorption, clouds")
    grid, table = I.make_albedo_slab(nlay=12, nlam=3)
    grid.cld_ksca = np.linspace(0.0, 2e-3, 12).astype(np.float32)
    grid.cld_kabs = np.full(12, 1e-4, np.float32)
    grid.cld_g = np.linspace(-0.3, 0.8, 12).astype(np.float32)
    obs = np.array([[-0.6, 0.0, 0.8], [0.28, 0.96 * 0.6, 0.96 * 0.8], [0.0, 0.6, 0.8]])
    obs /= np.linalg.norm(obs, axis=1)[:, None]
    n = 2000
    for absorption in (0, 1):
        dump = dump_buffer(torch_dev, 3, n, 3)
        gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
        got = ctx.solve_albedo(gid, oid, table, n_packets=n, seed=7, mu0=0.42, obs_dir=obs,
                               absorption=absorption, packet_dump=dump)
        p = O.Params(n_packets=n, seed=7, mu0=0.42, obs_dir=obs, absorption=absorption)
        ref = O.solve_albedo(grid, table, p, keep_packets=True)
        check_packets(dump, ref, (3, 1, n, 3))
        check_solve(got, ref)
        ctx.free_grid(gid)
        ctx.free_opacity(oid)


def test_albedo_sphere_parity(ctx, torch_dev):
    _log("albedo 3D sphere parity: 16x8x6 grid, 3 bands x 2 g, 3 phases")
    grid = I.make_sphere(16, 8, 6, seed=31)
    _, table, _ = I.make_emission_3d(16, 8, 6, nband=3, ng=2)
    table.k_ray = table.k_ray * 1e3  # make scattering matter
    n = 1500
    dump = dump_buffer(torch_dev, 6, n, 3)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    phases = [0.0, 0.8, 2.2]
    got = ctx.solve_albedo(gid, oid, table, n_packets=n, seed=33, obs_phase=phases, packet_dump=dump,
                           decorrelate=1)
    ref = O.solve_albedo(grid, table, O.Params(n_packets=n, seed=33, obs_phase=phases, decorrelate=True),
                         keep_packets=True)
    check_packets(dump, ref, (3, 2, n, 3))
    check_solve(got, ref)
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_emission_parity_with_clouds(ctx, torch_dev):
    _log("emission 3D parity: 16x8x10 grid with HG clouds, 2 bands x 2 g, 4 phases, roulette")
    grid, table, phases = I.make_emission_3d(16, 8, 10, nband=2, ng=2)
    rng = np.random.default_rng(3)
    grid.cld_ksca = rng.uniform(0, 5e-2, grid.ncell).astype(np.float32)
    grid.cld_kabs = rng.uniform(0, 1e-2, grid.ncell).astype(np.float32)
    grid.cld_g = rng.uniform(-0.5, 0.9, grid.ncell).astype(np.float32)
    n = 1200
    dump = dump_buffer(torch_dev, 4, n, 4)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    got = ctx.solve_emission(gid, oid, table, n_packets=n, seed=41, obs_phase=phases, packet_dump=dump,
                             rr_threshold=0.05, rr_survive=0.3)
    p = O.Params(n_packets=n, seed=41, obs_phase=tuple(phases), rr_threshold=0.05, rr_survive=0.3)
    ref = O.solve_emission(grid, table, p, keep_packets=True)
    check_packets(dump, ref, (2, 2, n, 4))
    check_solve(got, ref)
    np.testing.assert_allclose(got["l_tot"], ref.extra["L_tot"], rtol=1e-12)
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


@pytest.mark.parametrize("shape", [(8, 4, 8), (4, 2, 3), (16, 8, 10)])
def test_emission_birth_cells_every_packet(ctx, torch_dev, shape):
    """Birth cells found through the per-block table of CDF samples: grids of
    exactly 256 cells (the last sample is the last cell), fewer (repeated
    samples) and more, with flat CDF stretches where the tau cut silences
    cells; every packet's row against the oracle."""
    nlon, nlat, nlay = shape
    _log(f"emission birth cells: {nlon}x{nlat}x{nlay} grid, every packet")
    grid, table, phases = I.make_emission_3d(nlon, nlat, nlay, nband=2, ng=1, config_no=31)
    n = 1100  # several blocks of 256 packets, a ragged last one
    dump = dump_buffer(torch_dev, 2, n, 1)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    got = ctx.solve_emission(gid, oid, table, n_packets=n, seed=53, obs_phase=[0.25], packet_dump=dump)
    ref = O.solve_emission(grid, table, O.Params(n_packets=n, seed=53, obs_phase=(0.25,)), keep_packets=True)
    check_packets(dump, ref, (2, 1, n, 1))
    check_solve(got, ref)
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_peel_off_cut_parity(ctx, torch_dev):
    """A low peel-off cut (tau_peel_max = 1.5) drops many peel-offs mid-walk:
    every packet against the oracle, albedo and emission, FP64."""
    _log("peel-off cut parity: tau_peel_max = 1.5, albedo and emission on 12x6x8")
    grid, table, phases = I.make_emission_3d(12, 6, 8, nband=2, ng=1, config_no=30)
    table.k_ray = table.k_ray * 100.0
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    n = 1500
    kw = dict(n_packets=n, seed=47, tau_peel_max=1.5)
    dump = dump_buffer(torch_dev, 2, n, 2)
    got = ctx.solve_emission(gid, oid, table, obs_phase=[0.0, 0.5], packet_dump=dump, **kw)
    ref = O.solve_emission(grid, table, O.Params(obs_phase=(0.0, 0.5), **kw), keep_packets=True)
    check_packets(dump, ref, (2, 1, n, 2))
    check_solve(got, ref)
    dump = dump_buffer(torch_dev, 2, n, 2)
    got = ctx.solve_albedo(gid, oid, table, obs_phase=[0.0, 0.5], packet_dump=dump, **kw)
    ref = O.solve_albedo(grid, table, O.Params(obs_phase=(0.0, 0.5), **kw), keep_packets=True)
    check_packets(dump, ref, (2, 1, n, 2))
    check_solve(got, ref)
    full = ctx.solve_albedo(gid, oid, table, obs_phase=[0.0, 0.5], n_packets=n, seed=47)
    assert np.all(got["value"] <= full["value"]) and np.any(got["value"] < full["value"])
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_emission_no_scattering_and_tau_cut(ctx, torch_dev):
    _log("emission parity: scattering off, tau_vert = 3, bias xi = 0.8")
    grid, table, phases = I.make_emission_3d(12, 6, 8, nband=3, ng=1)
    n = 2500
    dump = dump_buffer(torch_dev, 3, n, 2)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    got = ctx.solve_emission(gid, oid, table, n_packets=n, seed=43, obs_phase=[0.5, 0.25], packet_dump=dump,
                             scattering=0, tau_vert_max=3.0, emis_bias=0.8)
    p = O.Params(n_packets=n, seed=43, obs_phase=(0.5, 0.25), scattering=False, tau_vert_max=3.0, emis_bias=0.8)
    ref = O.solve_emission(grid, table, p, keep_packets=True)
    check_packets(dump, ref, (3, 1, n, 2))
    check_solve(got, ref)
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_emission_hires_doppler_parity(ctx, torch_dev):
    _log("hi-res emission parity: Doppler-shifted lines, 1 observer, 4 wavelengths")
    grid, table = I.make_transmission_hires(12, 6, 8, nlam=300, nT=6, nP=5)
    n = 1500
    spec = [0, 7, 150, 299]
    dump = dump_buffer(torch_dev, 4, n, 1)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    got = ctx.solve_emission(gid, oid, table, n_packets=n, seed=45, obs_phase=[0.4], spec_idx=spec,
                             scattering=0, packet_dump=dump)
    # oracle: per-wavelength Doppler optics for the observer, emission sources, transport
    o = O.emission_obs_dirs([0.4])
    sh = O.doppler_shift(grid, o[0], table.dlnlam)
    d = dump.cpu().numpy().reshape(4, n)
    for q, lam in enumerate(spec):
        op = O.hires_optics(grid, table, lam, sh)
        src = O.emission_sources(grid, op, table.lam_um()[lam], 30.0, 0.5)
        F, K = O.transport(grid, op, O.Params(n_packets=n, seed=45, scattering=False), 1, o, sources=src)
        scale = F.max()
        assert np.all(np.abs(d[q] - F[:, 0]) <= RTOL * np.abs(F[:, 0]) + 1e-12 * scale)
        want = src.L_tot * F[:, 0].sum() / n / grid.r_toa ** 2
        assert got["value"][q, 0] == pytest.approx(want, rel=RTOL)
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_transmission_ck_parity(ctx, torch_dev):
    _log("transmission ck parity: 16x8x9 grid, 3 bands x 2 g, 24 x 30 chords")
    grid, table, _ = I.make_emission_3d(16, 8, 9, nband=3, ng=2)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    kw = dict(n_b=24, n_alpha=30, seed=47, r_star=I.R_SUN)
    got = ctx.solve_transmission(gid, oid, table, **kw)
    ref = O.solve_transmission(grid, table, O.Params(**kw))
    np.testing.assert_allclose(got["value"], ref.value, rtol=1e-12)
    np.testing.assert_allclose(got["per_g"], ref.per_g, rtol=1e-12)
    np.testing.assert_allclose(got["sums"], ref.sums, rtol=RTOL)
    # mixed form: FP32 extinction rows, FP64 optical depths -- within 1e-3
    # (observed ~1e-7) of the FP64 sums and within 3 sigma of its values
    from paper_2110_15640_amd import mcrt as M
    mix = ctx.solve_transmission(gid, oid, table, precision=M.MCRT_MIXED, **kw)
    np.testing.assert_allclose(mix["sums"][..., 0], got["sums"][..., 0], rtol=1e-3)
    assert np.all(np.abs(mix["value"] - got["value"]) <= 3.0 * got["stderr"])
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_transmission_hires_parity_multi_block(ctx, torch_dev):
    _log("transmission hi-res parity: winds + rotation, 150 wavelengths (3 slot blocks), 32 x 20 chords")
    grid, table = I.make_transmission_hires(16, 8, 10, nlam=400, nT=5, nP=6)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    spec = list(range(100, 250))
    kw = dict(n_b=32, n_alpha=20, seed=49, r_star=I.R_SUN)
    got = ctx.solve_transmission(gid, oid, table, spec_idx=spec, **kw)
    ref = O.solve_transmission(grid, table, O.Params(**kw), spec_idx=spec)
    np.testing.assert_allclose(got["sums"], ref.sums, rtol=RTOL)
    np.testing.assert_allclose(got["value"], ref.value, rtol=1e-12)
    from paper_2110_15640_amd import mcrt as M
    mix = ctx.solve_transmission(gid, oid, table, spec_idx=spec, precision=M.MCRT_MIXED, **kw)
    np.testing.assert_allclose(mix["sums"][..., 0], ref.sums[..., 0], rtol=1e-3)
    assert np.all(np.abs(mix["value"] - ref.value) <= 3.0 * got["stderr"])
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_transmission_hires_slot_order_invariance(ctx, torch_dev):
    """A wavelength's extinction row does not depend on which slot holds it:
    consecutive wavelengths share table values between neighbouring lanes,
    shuffled, repeated or sparse ones load their own.  Both precisions,
    bit-identical per wavelength; 150 wavelengths give a ragged last block."""
    _log("transmission hi-res: slot order invariance (consecutive vs shuffled vs sparse wavelengths)")
    from paper_2110_15640_amd import mcrt as M
    grid, table = I.make_transmission_hires(16, 8, 10, nlam=400, nT=5, nP=6)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    kw = dict(n_b=32, n_alpha=20, seed=49, r_star=I.R_SUN)
    base = list(range(100, 250))
    rng = np.random.default_rng(7)
    shuffled = [int(x) for x in rng.permutation(base)]
    # every other wavelength, each twice in a row, then the table's two ends
    sparse = [w for w in base[::2] for _ in range(2)] + [0, 1, table.nlam - 2, table.nlam - 1]
    for prec in (M.MCRT_FP64, M.MCRT_MIXED):
        ref = ctx.solve_transmission(gid, oid, table, spec_idx=base, precision=prec, **kw)
        for other in (shuffled, sparse):
            got = ctx.solve_transmission(gid, oid, table, spec_idx=other, precision=prec, **kw)
            for row, w in enumerate(other):
                if w in base:
                    assert np.array_equal(got["sums"][row], ref["sums"][base.index(w)]), (prec, w)
        ends = ctx.solve_transmission(gid, oid, table, spec_idx=[0, 1, table.nlam - 2, table.nlam - 1],
                                      precision=prec, **kw)
        got = ctx.solve_transmission(gid, oid, table, spec_idx=sparse, precision=prec, **kw)
        assert np.array_equal(got["sums"][-4:], ends["sums"]), prec
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_transmission_hires_single_wavelength_table(ctx, torch_dev):
    """A one-wavelength hi-res table: every Doppler shift clamps to the one
    entry (no neighbour wavelength to interpolate to), in both precisions."""
    _log("transmission hi-res: one-wavelength table, winds + rotation")
    from paper_2110_15640_amd import mcrt as M
    grid, table = I.make_transmission_hires(16, 8, 10, nlam=1, nT=5, nP=6)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    kw = dict(n_b=32, n_alpha=20, seed=51, r_star=I.R_SUN)
    got = ctx.solve_transmission(gid, oid, table, **kw)
    ref = O.solve_transmission(grid, table, O.Params(**kw))
    np.testing.assert_allclose(got["sums"], ref.sums, rtol=RTOL)
    np.testing.assert_allclose(got["value"], ref.value, rtol=1e-12)
    mix = ctx.solve_transmission(gid, oid, table, precision=M.MCRT_MIXED, **kw)
    np.testing.assert_allclose(mix["sums"][..., 0], ref.sums[..., 0], rtol=1e-3)
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_edge_cases(ctx, torch_dev):
    _log("edge cases: one packet, no emitting cells, error codes")
    from paper_2110_15640_amd import mcrt as M
    grid, table, _ = I.make_emission_3d(8, 4, 5, nband=2, ng=1)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    got = ctx.solve_emission(gid, oid, table, n_packets=1, seed=3, obs_phase=[0.5])
    ref = O.solve_emission(grid, table, O.Params(n_packets=1, seed=3, obs_phase=(0.5,)))
    np.testing.assert_allclose(got["value"], ref.value, rtol=RTOL)
    dark = I.CKTable(table.lam_um, table.g_weights, table.T_grid, table.P_grid,
                     np.zeros_like(table.kappa), np.zeros_like(table.k_ray))
    did = ctx.upload_opacity(dark)
    got = ctx.solve_emission(gid, did, dark, n_packets=100, seed=3, obs_phase=[0.5])
    assert np.all(got["value"] == 0.0) and np.all(got["l_tot"] == 0.0)
    with pytest.raises(M.McrtError) as e:
        ctx.solve_emission(gid, oid, table, n_packets=0, obs_phase=[0.5])
    assert e.value.name == "EINVAL"
    with pytest.raises(M.McrtError) as e:
        ctx.solve_emission(gid + 1000, oid, table, n_packets=10, obs_phase=[0.5])
    assert e.value.name == "ENOTFOUND"
    slab, st = I.make_albedo_slab(nlay=4, nlam=1)
    sid = ctx.upload_grid(slab)
    with pytest.raises(M.McrtError) as e:
        ctx.solve_emission(sid, oid, table, n_packets=10, obs_phase=[0.5])
    assert e.value.name == "EINVAL"
    bad = I.make_sphere(4, 2, 3, seed=1)
    bad.rho = bad.rho.copy()
    bad.rho[3] = -1.0
    with pytest.raises(M.McrtError) as e:
        ctx.upload_grid(bad)
    assert e.value.name == "EINVAL"
    bad_t = I.CKTable(table.lam_um, np.array([0.7]), table.T_grid, table.P_grid, table.kappa, table.k_ray)
    with pytest.raises(M.McrtError) as e:
        ctx.upload_opacity(bad_t)
    assert e.value.name == "EINVAL"
    _, t2, _ = I.make_emission_3d(4, 2, 2, nband=2, ng=4, config_no=5)
    unsorted = t2.kappa.copy()
    unsorted[1, 2, 3, 4] = unsorted[1, 3, 3, 4] * 1.5  # g = 2 above g = 3 at one (T, P)
    with pytest.raises(M.McrtError) as e:
        ctx.upload_opacity(I.CKTable(t2.lam_um, t2.g_weights, t2.T_grid, t2.P_grid, unsorted, t2.k_ray))
    assert e.value.name == "EINVAL"
    with pytest.raises(M.McrtError) as e:
        M.Context(0, hbm_budget_bytes=1024).upload_grid(grid)
    assert e.value.name == "EBUDGET"
    for x in (gid, sid):
        ctx.free_grid(x)
    for x in (oid, did):
        ctx.free_opacity(x)


def test_batched_and_launch_shapes_are_bit_identical(ctx, torch_dev):
    _log("determinism: one launch per solve vs one batched launch vs other launch shapes")
    grid, table, phases = I.make_emission_3d(16, 8, 10, nband=3, ng=2)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    base = dict(n_packets=3000, seed=61, obs_phase=phases)
    ref = ctx.solve_emission(gid, oid, table, max_batch=1, **base)
    for kw in (dict(max_batch=0), dict(max_batch=4), dict(tune_ev_threshold=1, tune_blocks_per_cu=1, tune_wave_batch=7),
               dict(tune_ev_threshold=64, tune_wave_batch=1000)):
        got = ctx.solve_emission(gid, oid, table, **base, **kw)
        assert np.array_equal(got["sums"], ref["sums"]), kw
        assert np.array_equal(got["value"], ref["value"]), kw
        assert np.array_equal(got["counters"], ref["counters"]), kw
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


@pytest.mark.parametrize("mode", ["albedo", "emission"])
def test_autotuner_picks_a_candidate_shape_that_keeps_results(ctx, torch_dev, mode):
    """The autotuner returns one of its candidate launch shapes and a trial
    rate, and the solve run with that shape equals the default-shape solve
    bit for bit; it refuses the chord (transmission) path."""
    _log(f"autotuner: {mode}")
    from paper_2110_15640_amd import mcrt as M
    grid, table, phases = I.make_emission_3d(16, 8, 10, nband=3, ng=2)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    fn = ctx.solve_albedo if mode == "albedo" else ctx.solve_emission
    kw = dict(n_packets=20000, seed=67, obs_phase=[0.0, 0.5], precision=M.MCRT_MIXED)
    tuned = ctx.autotune(mode, gid, oid, **kw)
    assert tuned["tune_ev_threshold"] in (20, 24, 28, 32)
    assert tuned["tune_blocks_per_cu"] in (3, 4)
    assert tuned["tune_wave_batch"] in (32, 128)
    assert np.isfinite(tuned["trial_packets_per_s"]) and tuned["trial_packets_per_s"] > 0.0
    tuned.pop("trial_packets_per_s")
    ref = fn(gid, oid, table, **kw)
    got = fn(gid, oid, table, **kw, **tuned)
    assert np.array_equal(got["sums"], ref["sums"])
    assert np.array_equal(got["counters"], ref["counters"])
    with pytest.raises(M.McrtError) as e:
        ctx.autotune("transmission", gid, oid, n_b=16, n_alpha=16)
    assert e.value.name == "EINVAL"
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


@pytest.mark.parametrize("mode", ["albedo", "emission"])
def test_mixed_precision_agrees_with_fp64(ctx, torch_dev, mode):
    """FP32 opacity / phase-function / direction math on the same random
    stream: spectra within 1e-3 relative and 3 sigma of the FP64 ones."""
    _log(f"mixed vs fp64: {mode}")
    from paper_2110_15640_amd import mcrt as M
    grid, table, phases = I.make_emission_3d(24, 12, 20, nband=4, ng=2)
    table.k_ray = table.k_ray * 30.0
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    fn = ctx.solve_albedo if mode == "albedo" else ctx.solve_emission
    ph = [0.0, 0.5] if mode == "albedo" else list(phases)
    kw = dict(n_packets=40000, seed=63, obs_phase=ph)
    a = fn(gid, oid, table, precision=M.MCRT_FP64, **kw)
    b = fn(gid, oid, table, precision=M.MCRT_MIXED, **kw)
    rel = np.abs(b["value"] - a["value"]) / np.abs(a["value"])
    assert rel.max() < 1e-3, rel
    assert np.all(np.abs(b["value"] - a["value"]) <= 3.0 * a["stderr"])
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_multi_grid_batch_equals_single_solves(ctx, torch_dev):
    """Albedo and emission items on grids of uneven size in multi-grid
    persistent launches: every item's result equals its own single solve."""
    _log("multi-grid batch: 5 items on 3 uneven grids vs single solves")
    specs = [(16, 8, 10), (24, 12, 6), (8, 4, 12)]
    gids, tabs = [], []
    for q, (a, b, c) in enumerate(specs):
        grid, table, _ = I.make_emission_3d(a, b, c, nband=4, ng=2, config_no=10 + q)
        table.k_ray = table.k_ray * 50.0
        gids.append(ctx.upload_grid(grid))
        tabs.append((ctx.upload_opacity(table), table))
    items = [dict(mode="emission", gid=gids[0], oid=tabs[0][0], table=tabs[0][1], spec_idx=[0, 3], n_packets=1700),
             dict(mode="albedo", gid=gids[1], oid=tabs[1][0], table=tabs[1][1], spec_idx=[1], n_packets=900),
             dict(mode="emission", gid=gids[2], oid=tabs[2][0], table=tabs[2][1], spec_idx=[2, 1, 0], n_packets=2500),
             dict(mode="albedo", gid=gids[0], oid=tabs[0][0], table=tabs[0][1], spec_idx=[2], n_packets=300),
             dict(mode="emission", gid=gids[1], oid=tabs[1][0], table=tabs[1][1], spec_idx=[3], n_packets=64)]
    common = dict(obs_phase=[0.0, 0.5], seed=71, decorrelate=1)
    for mb in (0, 3):  # one launch, and launches of at most 3 solves
        outs = ctx.solve_batch(items, max_batch=mb, **common)
        for it, got in zip(items, outs):
            fn = ctx.solve_albedo if it["mode"] == "albedo" else ctx.solve_emission
            ref = fn(it["gid"], it["oid"], it["table"], spec_idx=it["spec_idx"], n_packets=it["n_packets"], **common)
            assert np.array_equal(got["sums"], ref["sums"]), (mb, it["mode"])
            assert np.array_equal(got["value"], ref["value"]), (mb, it["mode"])
    for g in gids:
        ctx.free_grid(g)
    for o, _ in tabs:
        ctx.free_opacity(o)


@pytest.mark.parametrize("feature", [dict(surface_albedo=0.3), dict(cloud_phase=1), dict(cloud_phase=2, draine_alpha=0.7),
                                     dict(forced=2, forced_first=1)],
                         ids=["lambert", "tthg", "draine", "forced"])
def test_multi_grid_batch_with_extended_features(ctx, torch_dev, feature):
    """The multi-grid kernel forms with the Lambert floor, two-term HG or
    Draine clouds and forced interactions: every item of a batch on grids of
    uneven size (with clouds) equals its own single solve, in FP64 and in the
    mixed form."""
    _log(f"multi-grid batch with {feature}")
    from paper_2110_15640_amd import mcrt as M
    specs = [(12, 6, 8), (16, 8, 5)]
    gids, tabs = [], []
    rng = np.random.default_rng(41)
    for q, (a, b, c) in enumerate(specs):
        grid, table, _ = I.make_emission_3d(a, b, c, nband=3, ng=2, config_no=20 + q)
        grid.cld_ksca = rng.uniform(0, 2e-2, grid.ncell).astype(np.float32)
        grid.cld_kabs = rng.uniform(0, 2e-3, grid.ncell).astype(np.float32)
        grid.cld_g = rng.uniform(0.0, 0.8, grid.ncell).astype(np.float32)
        table.k_ray = table.k_ray * 50.0
        gids.append(ctx.upload_grid(grid))
        tabs.append((ctx.upload_opacity(table), table))
    items = [dict(mode="emission", gid=gids[0], oid=tabs[0][0], table=tabs[0][1], spec_idx=[0, 2], n_packets=900),
             dict(mode="albedo", gid=gids[1], oid=tabs[1][0], table=tabs[1][1], spec_idx=[1], n_packets=700),
             dict(mode="emission", gid=gids[1], oid=tabs[1][0], table=tabs[1][1], spec_idx=[2], n_packets=1100)]
    for prec in (M.MCRT_FP64, M.MCRT_MIXED):
        common = dict(obs_phase=[0.0, 0.5], seed=79, decorrelate=1, precision=prec, max_events=200, **feature)
        outs = ctx.solve_batch(items, max_batch=0, **common)
        for it, got in zip(items, outs):
            fn = ctx.solve_albedo if it["mode"] == "albedo" else ctx.solve_emission
            ref = fn(it["gid"], it["oid"], it["table"], spec_idx=it["spec_idx"], n_packets=it["n_packets"], **common)
            assert np.array_equal(got["sums"], ref["sums"]), (prec, it["mode"])
            assert np.array_equal(got["counters"], ref["counters"]), (prec, it["mode"])
            assert np.all(np.isfinite(got["value"]))
    for g in gids:
        ctx.free_grid(g)
    for o, _ in tabs:
        ctx.free_opacity(o)


def test_graph_replays_equal_eager(ctx, torch_dev):
    """Recorded solves (params.graph): the first call records the device chain,
    later identical calls replay it; with other eager work and synchronisations
    between the replays, every replay equals the eager solve bit for bit."""
    _log("hipGraph: record + 4 replays (3 batches each) vs the eager solve, eager work in between")
    from paper_2110_15640_amd import mcrt as M
    grid, table, phases = I.make_emission_3d(16, 8, 10, nband=3, ng=2)
    slab, st = I.make_albedo_slab(nlay=8, nlam=2)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    sid, soid = ctx.upload_grid(slab), ctx.upload_opacity(st)
    for prec in (M.MCRT_FP64, M.MCRT_MIXED):
        base = dict(n_packets=2100, seed=65, obs_phase=phases, max_batch=2, precision=prec)
        ref = ctx.solve_emission(gid, oid, table, **base)
        other = ctx.solve_albedo(sid, soid, st, n_packets=500, seed=3)
        for rep in range(5):
            got = ctx.solve_emission(gid, oid, table, graph=1, **base)
            assert np.array_equal(got["sums"], ref["sums"]), (prec, rep)
            assert np.array_equal(got["value"], ref["value"]), (prec, rep)
            assert np.array_equal(got["counters"], ref["counters"]), (prec, rep)
            # eager work on the same stream and scratch between the replays
            o2 = ctx.solve_albedo(sid, soid, st, n_packets=500, seed=3)
            assert np.array_equal(o2["sums"], other["sums"])
            torch_dev.cuda.synchronize()
    # albedo with a packet dump recorded into the graph
    dump = dump_buffer(torch_dev, 2, 900, 1)
    ref = ctx.solve_albedo(sid, soid, st, n_packets=900, seed=5, packet_dump=dump)
    d0 = dump.clone()
    for rep in range(3):
        dump.zero_()
        got = ctx.solve_albedo(sid, soid, st, n_packets=900, seed=5, packet_dump=dump, graph=1)
        assert np.array_equal(got["sums"], ref["sums"]), rep
        assert torch_dev.equal(dump, d0), rep
    for x in (gid, sid):
        ctx.free_grid(x)
    for x in (oid, soid):
        ctx.free_opacity(x)


def test_contribution_functions_and_images_parity(ctx, torch_dev):
    """Per-cell contribution functions (thermal and scattered parts, per band
    and observer) and sky-plane images against the oracle on the same stream;
    albedo and emission, eager and graph-replayed."""
    _log("contribution functions: emission with clouds (16x8x10, 2 bands x 2 g, 3 phases), albedo sphere")
    from paper_2110_15640_amd import mcrt as M
    grid, table, phases = I.make_emission_3d(16, 8, 10, nband=2, ng=2)
    rng = np.random.default_rng(5)
    grid.cld_ksca = rng.uniform(0, 5e-2, grid.ncell).astype(np.float32)
    grid.cld_kabs = rng.uniform(0, 1e-2, grid.ncell).astype(np.float32)
    grid.cld_g = rng.uniform(-0.5, 0.9, grid.ncell).astype(np.float32)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    ph = list(phases[:3])
    ref = O.solve_emission(grid, table, O.Params(n_packets=2500, seed=81, obs_phase=tuple(ph)), contrib=True,
                           image_npix=24)
    for graph in (0, 1, 1):
        got = ctx.solve_emission(gid, oid, table, n_packets=2500, seed=81, obs_phase=ph, contrib=1, graph=graph,
                                 image_npix=24)
        np.testing.assert_allclose(got["cf"], ref.extra["cf"], rtol=1e-9, atol=1e-13)
        im = ref.extra["image"]
        np.testing.assert_allclose(got["image"], im, rtol=1e-9, atol=1e-12 * im.max())
        np.testing.assert_allclose(got["value"], ref.value, rtol=RTOL)
    assert got["cf"][:, :, 1].sum() > 0.0 and got["cf"][:, :, 0].sum() > 0.0
    sph = I.make_sphere(12, 6, 8, seed=33)
    _, t2, _ = I.make_emission_3d(12, 6, 8, nband=2, ng=2)
    t2.k_ray = t2.k_ray * 1e3
    sid, soid = ctx.upload_grid(sph), ctx.upload_opacity(t2)
    got = ctx.solve_albedo(sid, soid, t2, n_packets=3000, seed=83, obs_phase=[0.0, 1.2], contrib=1,
                           precision=M.MCRT_FP64, image_npix=17)
    ref = O.solve_albedo(sph, t2, O.Params(n_packets=3000, seed=83, obs_phase=(0.0, 1.2)), contrib=True,
                         image_npix=17)
    np.testing.assert_allclose(got["cf"], ref.extra["cf"], rtol=1e-9, atol=1e-13)
    im = ref.extra["image"]
    np.testing.assert_allclose(got["image"], im, rtol=1e-9, atol=1e-12 * im.max())
    np.testing.assert_allclose(got["image"].sum(axis=(2, 3)), got["value"], rtol=1e-12)
    assert np.all(got["cf"][:, :, 0] == 0.0)
    # mixed precision: still a normalised function close to the FP64 one
    mix = ctx.solve_albedo(sid, soid, t2, n_packets=3000, seed=83, obs_phase=[0.0, 1.2], contrib=1,
                           precision=M.MCRT_MIXED)
    np.testing.assert_allclose(mix["cf"].sum(axis=(2, 3)), 1.0, rtol=1e-12)
    assert np.abs(mix["cf"] - got["cf"]).max() < 1e-3
    # not available for transmission, served requests or multi-grid batches
    with pytest.raises(M.McrtError) as e:
        ctx.solve_transmission(gid, oid, table, n_b=8, n_alpha=8, contrib=1)
    assert e.value.name == "EINVAL"
    with pytest.raises(M.McrtError) as e:
        ctx.submit("emission", gid, oid, table, n_packets=100, obs_phase=[0.5], contrib=1)
    assert e.value.name == "EINVAL"
    for x in (gid, sid):
        ctx.free_grid(x)
    for x in (oid, soid):
        ctx.free_opacity(x)


@pytest.mark.parametrize("scheme", [1, 2, 3])
def test_g_sampling_parity(ctx, torch_dev, scheme):
    """Per-packet g-ordinate sampling (unbiased, uniform, composite): every
    packet's peel-off sums and the band values against the oracle, albedo and
    emission; one band per launch equals all bands in one launch bit for bit."""
    _log(f"g-ordinate sampling parity, scheme {scheme}: emission 12x6x8 (2 bands x 4 g), albedo sphere")
    grid, table, phases = I.make_emission_3d(12, 6, 8, nband=2, ng=4, config_no=50)
    rng = np.random.default_rng(9)
    grid.cld_ksca = rng.uniform(0, 3e-2, grid.ncell).astype(np.float32)
    grid.cld_kabs = rng.uniform(0, 1e-2, grid.ncell).astype(np.float32)
    grid.cld_g = rng.uniform(-0.4, 0.8, grid.ncell).astype(np.float32)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    n = 2500
    ph = list(phases[:3])
    dump = dump_buffer(torch_dev, 2, n, 3)
    got = ctx.solve_emission(gid, oid, table, n_packets=n, seed=91, obs_phase=ph, g_sampling=scheme,
                             packet_dump=dump, decorrelate=1)
    ref = O.solve_emission(grid, table, O.Params(n_packets=n, seed=91, obs_phase=tuple(ph), g_sampling=scheme,
                                                 decorrelate=True), keep_packets=True)
    d = dump.cpu().numpy().reshape(2, n, 3)
    for s in range(2):
        F = ref.extra["packets"][(s, 0)][0]
        scale = max(float(np.abs(F).max()), 1e-300)
        bad = np.abs(d[s] - F) > RTOL * np.abs(F) + 1e-12 * scale
        assert not bad.any(), (s, np.argwhere(bad)[:5].tolist())
    np.testing.assert_allclose(got["value"], ref.value, rtol=RTOL)
    np.testing.assert_allclose(got["stderr"], ref.stderr, rtol=1e-7)
    np.testing.assert_allclose(got["sums"], ref.sums, rtol=RTOL, atol=1e-300)
    one = ctx.solve_emission(gid, oid, table, n_packets=n, seed=91, obs_phase=ph, g_sampling=scheme,
                             decorrelate=1, max_batch=4)
    assert np.array_equal(one["sums"], got["sums"]) and np.array_equal(one["value"], got["value"])
    _, t2, _ = I.make_emission_3d(12, 6, 8, nband=2, ng=4, config_no=51)
    t2.k_ray = t2.k_ray * 1e3
    sph = I.make_sphere(12, 6, 8, seed=53)
    sid, soid = ctx.upload_grid(sph), ctx.upload_opacity(t2)
    got = ctx.solve_albedo(sid, soid, t2, n_packets=3000, seed=93, obs_phase=[0.0, 0.9], g_sampling=scheme)
    ref = O.solve_albedo(sph, t2, O.Params(n_packets=3000, seed=93, obs_phase=(0.0, 0.9), g_sampling=scheme))
    np.testing.assert_allclose(got["value"], ref.value, rtol=RTOL)
    np.testing.assert_allclose(got["counters"][:, 0], ref.counters[:, 0], rtol=RTOL,
                               atol=1e-12 * max(ref.counters.max(), 1.0))
    with pytest.raises(Exception):
        ctx.solve_transmission(gid, oid, table, n_b=8, n_alpha=8, g_sampling=scheme)
    for x in (gid, sid):
        ctx.free_grid(x)
    for x in (oid, soid):
        ctx.free_opacity(x)


def test_tthg_clouds_parity(ctx, torch_dev):
    """Two-term HG clouds: every packet against the oracle (emission with
    clouds, FP64), the albedo spectrum, and the mixed form within 1e-3 / 3 sigma."""
    _log("two-term HG clouds: emission 16x8x10 with clouds, albedo sphere, mixed vs fp64")
    from paper_2110_15640_amd import mcrt as M
    grid, table, phases = I.make_emission_3d(16, 8, 10, nband=2, ng=2, config_no=60)
    rng = np.random.default_rng(13)
    grid.cld_ksca = rng.uniform(0, 6e-2, grid.ncell).astype(np.float32)
    grid.cld_kabs = rng.uniform(0, 5e-3, grid.ncell).astype(np.float32)
    grid.cld_g = rng.uniform(-0.3, 0.9, grid.ncell).astype(np.float32)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    n = 1500
    dump = dump_buffer(torch_dev, 4, n, 4)
    got = ctx.solve_emission(gid, oid, table, n_packets=n, seed=95, obs_phase=phases, packet_dump=dump, cloud_phase=1)
    ref = O.solve_emission(grid, table, O.Params(n_packets=n, seed=95, obs_phase=tuple(phases), cloud_phase=1),
                           keep_packets=True)
    check_packets(dump, ref, (2, 2, n, 4))
    check_solve(got, ref)
    alb = ctx.solve_albedo(gid, oid, table, n_packets=4000, seed=97, obs_phase=[0.0, 1.1], cloud_phase=1)
    aref = O.solve_albedo(grid, table, O.Params(n_packets=4000, seed=97, obs_phase=(0.0, 1.1), cloud_phase=1))
    np.testing.assert_allclose(alb["value"], aref.value, rtol=RTOL)
    mix = ctx.solve_albedo(gid, oid, table, n_packets=4000, seed=97, obs_phase=[0.0, 1.1], cloud_phase=1,
                           precision=M.MCRT_MIXED)
    assert np.all(np.abs(mix["value"] - alb["value"]) <= np.maximum(3.0 * alb["stderr"], 1e-3 * np.abs(alb["value"])))
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_lambert_floor_parity(ctx, torch_dev):
    """Lambert floor (A_s > 0): every packet against the oracle for a
    scattering slab (three observers and the backscatter form) and for
    emission from a cloudy sphere; counters, contribution functions and
    images of an albedo sphere; a multi-grid batch equals its single solves;
    the mixed form within 1e-3 / 3 sigma."""
    _log("Lambert floor: slab (Rayleigh + HG cloud), emission sphere 16x8x10, albedo sphere CF/images, batch")
    from paper_2110_15640_amd import mcrt as M
    n = 2500
    obs = [[0.6, 0.0, 0.8], [-0.28, 0.4, math.sqrt(1 - 0.28 ** 2 - 0.16)], [0.0, 0.99, math.sqrt(1 - 0.99 ** 2)]]
    for ray in (True, False):
        if ray:
            grid, table = I.make_homogeneous_slab(1.0, 0.875, rayleigh=True, nlay=4)
        else:
            grid, table = I.make_homogeneous_slab(1.0, 0.875, g_cld=0.5, nlay=4)
        gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
        for o in (obs, None):
            kw = dict(n_packets=n, seed=111, mu0=0.55, surface_albedo=0.6)
            no = 3 if o is not None else 1
            dump = dump_buffer(torch_dev, 1, n, no)
            if o is not None:
                got = ctx.solve_albedo(gid, oid, table, obs_dir=o, packet_dump=dump, **kw)
                ref = O.solve_albedo(grid, table, O.Params(obs_dir=np.array(o), **kw), keep_packets=True)
            else:
                got = ctx.solve_albedo(gid, oid, table, packet_dump=dump, **kw)
                ref = O.solve_albedo(grid, table, O.Params(**kw), keep_packets=True)
            check_packets(dump, ref, (1, 1, n, no))
            check_solve(got, ref)
            assert ref.counters[0, 0, 1] > 0.0  # the floor absorbed some weight
        ctx.free_grid(gid)
        ctx.free_opacity(oid)
    # a thin atmosphere (opacities / 1000), so that packets of every kind
    # reach the floor
    grid, table, phases = I.make_emission_3d(16, 8, 10, nband=2, ng=2, config_no=70)
    rng = np.random.default_rng(17)
    grid.cld_ksca = rng.uniform(0, 3e-5, grid.ncell).astype(np.float32)
    grid.cld_kabs = rng.uniform(0, 5e-6, grid.ncell).astype(np.float32)
    grid.cld_g = rng.uniform(-0.3, 0.9, grid.ncell).astype(np.float32)
    table.kappa = (table.kappa * 1e-3).astype(np.float32)
    table.k_ray = table.k_ray * 0.02
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    n = 1500
    dump = dump_buffer(torch_dev, 4, n, 4)
    kw = dict(n_packets=n, seed=113, surface_albedo=0.45)
    got = ctx.solve_emission(gid, oid, table, obs_phase=phases, packet_dump=dump, cloud_phase=1, **kw)
    ref = O.solve_emission(grid, table, O.Params(obs_phase=tuple(phases), cloud_phase=1, **kw), keep_packets=True)
    check_packets(dump, ref, (2, 2, n, 4))
    check_solve(got, ref)
    assert ref.counters[:, :, 1].min() > 0.0  # every solve has floor events
    kw = dict(n_packets=3000, seed=115, surface_albedo=0.7)
    alb = ctx.solve_albedo(gid, oid, table, obs_phase=[0.0, 1.3], contrib=1, image_npix=15, **kw)
    aref = O.solve_albedo(grid, table, O.Params(obs_phase=(0.0, 1.3), **kw), contrib=True, image_npix=15)
    check_solve(alb, aref)
    np.testing.assert_allclose(alb["cf"], aref.extra["cf"], rtol=1e-9, atol=1e-13)
    im = aref.extra["image"]
    np.testing.assert_allclose(alb["image"], im, rtol=1e-9, atol=1e-12 * im.max())
    # the floor cells (k = 0) carry scattered contribution
    assert alb["cf"][:, :, 1, :grid.nlon * grid.nlat].sum() > 0.0
    mix = ctx.solve_albedo(gid, oid, table, obs_phase=[0.0, 1.3], precision=M.MCRT_MIXED, **kw)
    assert np.all(np.abs(mix["value"] - alb["value"]) <= np.maximum(3.0 * alb["stderr"], 1e-3 * np.abs(alb["value"])))
    items = [dict(mode="emission", gid=gid, oid=oid, table=table, spec_idx=[1], n_packets=900),
             dict(mode="albedo", gid=gid, oid=oid, table=table, spec_idx=[0], n_packets=700)]
    common = dict(obs_phase=[0.25, 0.5], seed=117, decorrelate=1, surface_albedo=0.3)
    outs = ctx.solve_batch(items, **common)
    for it, b in zip(items, outs):
        fn = ctx.solve_albedo if it["mode"] == "albedo" else ctx.solve_emission
        one = fn(it["gid"], it["oid"], it["table"], spec_idx=it["spec_idx"], n_packets=it["n_packets"], **common)
        assert np.array_equal(b["sums"], one["sums"]) and np.array_equal(b["counters"], one["counters"])
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_ms_transmission_and_limb_darkening_parity(ctx, torch_dev):
    """Transmission with multiple scattering (packets on the annulus, direct
    chord light plus scattered light over the stellar beam's solid angle):
    every packet's W0 - F against the oracle for a cloudy ck grid, with and
    without stellar limb darkening, and for a hi-res table with winds; the
    mixed form within 1e-3 / 3 sigma; raytrace chords with limb darkening;
    the parameter checks."""
    _log("ms transmission: 16x8x10 ck grid with clouds (LD off / quadratic, offset), hi-res with winds, K5 LD")
    from paper_2110_15640_amd import mcrt as M
    grid, table, _ = I.make_emission_3d(16, 8, 10, nband=2, ng=2, config_no=80)
    rng = np.random.default_rng(19)
    grid.cld_ksca = rng.uniform(0, 2e-2, grid.ncell).astype(np.float32)
    grid.cld_kabs = rng.uniform(0, 2e-3, grid.ncell).astype(np.float32)
    grid.cld_g = rng.uniform(0.2, 0.9, grid.ncell).astype(np.float32)
    table.k_ray = table.k_ray * 50.0
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    R = I.R_SUN
    n = 2000
    ld = dict(ld_law=2, ld_c1=0.45, ld_c2=0.2, transit_y=0.5 * R, transit_z=-0.3 * R)
    for extra in (dict(), ld):
        kw = dict(n_packets=n, seed=121, a_orbit=0.03 * 1.496e13, r_star=R, **extra)
        dump = dump_buffer(torch_dev, 4, n, 1)
        got = ctx.solve_transmission(gid, oid, table, ms_transmission=1, packet_dump=dump, **kw)
        ref = O.solve_transmission_ms(grid, table, O.Params(**kw), keep_packets=True)
        d = dump.cpu().numpy().reshape(2, 2, n)
        for s in range(2):
            for g in range(2):
                v = ref.extra["packets"][(s, g)][0]
                bad = np.abs(d[s, g] - v) > RTOL * np.abs(v) + 1e-12 * np.abs(v).max()
                assert not bad.any(), (extra, s, g, np.argwhere(bad)[:5].ravel().tolist())
        check_solve(got, ref)
        assert ref.counters[:, :, 6].min() > 0.0  # packets scatter
    mix = ctx.solve_transmission(gid, oid, table, ms_transmission=1, precision=M.MCRT_MIXED, **kw)
    assert np.all(np.abs(mix["value"] - got["value"]) <= np.maximum(3.0 * got["stderr"], 1e-3 * got["value"]))
    # raytrace chords with limb darkening
    kc = dict(n_b=24, n_alpha=30, seed=123, r_star=R, **ld)
    got = ctx.solve_transmission(gid, oid, table, **kc)
    ref = O.solve_transmission(grid, table, O.Params(**kc))
    np.testing.assert_allclose(got["sums"], ref.sums, rtol=RTOL)
    np.testing.assert_allclose(got["value"], ref.value, rtol=1e-12)
    for bad in (dict(ms_transmission=1, a_orbit=0.5 * R), dict(ld_law=7), dict(ms_transmission=1, g_sampling=1)):
        with pytest.raises(M.McrtError) as e:
            ctx.solve_transmission(gid, oid, table, n_packets=100, **dict(dict(a_orbit=10 * R), **bad))
        assert e.value.name == "EINVAL"
    ctx.free_grid(gid)
    ctx.free_opacity(oid)
    hg, ht = I.make_transmission_hires(16, 8, 10, nlam=200, nT=5, nP=6)
    ht.k_ray = ht.k_ray * 1e3
    hid, hoid = ctx.upload_grid(hg), ctx.upload_opacity(ht)
    spec = [0, 57, 199]
    kw = dict(n_packets=1500, seed=125, a_orbit=0.03 * 1.496e13, r_star=R)
    dump = dump_buffer(torch_dev, 3, 1500, 1)
    got = ctx.solve_transmission(hid, hoid, ht, ms_transmission=1, spec_idx=spec, packet_dump=dump, **kw)
    ref = O.solve_transmission_ms(hg, ht, O.Params(**kw), spec_idx=spec, keep_packets=True)
    d = dump.cpu().numpy().reshape(3, 1500)
    for s in range(3):
        v = ref.extra["packets"][(s, 0)][0]
        assert np.all(np.abs(d[s] - v) <= RTOL * np.abs(v) + 1e-12 * np.abs(v).max()), s
    check_solve(got, ref)
    ctx.free_grid(hid)
    ctx.free_opacity(hoid)


def test_draine_clouds_parity(ctx, torch_dev):
    """Draine clouds (G from the asymmetry factor in the optics preparation,
    exact rejection sampler): every packet against the oracle (emission with
    clouds, FP64, alpha = 0.5), the albedo spectrum (alpha = 1), a batch equal
    to its single solves, and the mixed form within 1e-3 / 3 sigma."""
    _log("Draine clouds: emission 16x8x10 with clouds, albedo sphere, batch, mixed vs fp64")
    from paper_2110_15640_amd import mcrt as M
    grid, table, phases = I.make_emission_3d(16, 8, 10, nband=2, ng=2, config_no=90)
    rng = np.random.default_rng(23)
    grid.cld_ksca = rng.uniform(0, 6e-2, grid.ncell).astype(np.float32)
    grid.cld_kabs = rng.uniform(0, 5e-3, grid.ncell).astype(np.float32)
    grid.cld_g = rng.uniform(-0.3, 0.95, grid.ncell).astype(np.float32)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    n = 1500
    dump = dump_buffer(torch_dev, 4, n, 4)
    got = ctx.solve_emission(gid, oid, table, n_packets=n, seed=141, obs_phase=phases, packet_dump=dump,
                             cloud_phase=2)
    ref = O.solve_emission(grid, table, O.Params(n_packets=n, seed=141, obs_phase=tuple(phases), cloud_phase=2),
                           keep_packets=True)
    check_packets(dump, ref, (2, 2, n, 4))
    check_solve(got, ref)
    kw = dict(n_packets=4000, seed=143, obs_phase=[0.0, 1.1], cloud_phase=2, draine_alpha=1.0)
    alb = ctx.solve_albedo(gid, oid, table, **kw)
    aref = O.solve_albedo(grid, table, O.Params(**dict(kw, obs_phase=(0.0, 1.1))))
    check_solve(alb, aref)
    mix = ctx.solve_albedo(gid, oid, table, precision=M.MCRT_MIXED, **kw)
    assert np.all(np.abs(mix["value"] - alb["value"]) <= np.maximum(3.0 * alb["stderr"], 1e-3 * np.abs(alb["value"])))
    items = [dict(mode="emission", gid=gid, oid=oid, table=table, spec_idx=[1], n_packets=900),
             dict(mode="albedo", gid=gid, oid=oid, table=table, spec_idx=[0], n_packets=700)]
    common = dict(obs_phase=[0.25, 0.5], seed=145, decorrelate=1, cloud_phase=2)
    outs = ctx.solve_batch(items, **common)
    for it, b in zip(items, outs):
        fn = ctx.solve_albedo if it["mode"] == "albedo" else ctx.solve_emission
        one = fn(it["gid"], it["oid"], it["table"], spec_idx=it["spec_idx"], n_packets=it["n_packets"], **common)
        assert np.array_equal(b["sums"], one["sums"]) and np.array_equal(b["counters"], one["counters"])
    with pytest.raises(M.McrtError) as e:
        ctx.solve_albedo(gid, oid, table, n_packets=10, obs_phase=[0.0], cloud_phase=2, draine_alpha=1.5)
    assert e.value.name == "EINVAL"
    ctx.free_grid(gid)
    ctx.free_opacity(oid)


def test_forced_interactions_parity(ctx, torch_dev):
    """Forced interactions (probe to the grid's edge, forced optical depth,
    weight factor, unscattered fraction booked): every packet against the
    oracle for each scheme on every flight and on the first only (emission
    sphere with clouds, slab albedo, multiple-scattering transmission),
    counters included; the mixed form within 1e-3 / 3 sigma; parameter
    checks."""
    _log("forced interactions: emission sphere 12x6x8 (kinds 1-3, every / first), slab albedo, ms transmission")
    from paper_2110_15640_amd import mcrt as M
    grid, table, phases = I.make_emission_3d(12, 6, 8, nband=1, ng=2, config_no=100)
    rng = np.random.default_rng(29)
    grid.cld_ksca = rng.uniform(0, 2e-2, grid.ncell).astype(np.float32)
    grid.cld_kabs = rng.uniform(0, 2e-3, grid.ncell).astype(np.float32)
    grid.cld_g = rng.uniform(0.0, 0.8, grid.ncell).astype(np.float32)
    table.k_ray = table.k_ray * 100.0
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    n = 1200
    for kind, first in ((1, 0), (2, 0), (3, 0), (1, 1), (3, 1)):
        dump = dump_buffer(torch_dev, 2, n, 2)
        kw = dict(n_packets=n, seed=161 + kind, forced=kind, forced_first=first)
        got = ctx.solve_emission(gid, oid, table, obs_phase=list(phases[:2]), packet_dump=dump, **kw)
        ref = O.solve_emission(grid, table, O.Params(obs_phase=tuple(phases[:2]), **kw), keep_packets=True)
        check_packets(dump, ref, (1, 2, n, 2))
        check_solve(got, ref)
    R = I.R_SUN
    kw = dict(n_packets=n, seed=171, forced=3, a_orbit=0.03 * 1.496e13, r_star=R)
    dump = dump_buffer(torch_dev, 2, n, 1)
    got = ctx.solve_transmission(gid, oid, table, ms_transmission=1, packet_dump=dump, **kw)
    ref = O.solve_transmission_ms(grid, table, O.Params(**kw), keep_packets=True)
    d = dump.cpu().numpy().reshape(2, n)
    for gi in range(2):
        v = ref.extra["packets"][(0, gi)][0]
        assert np.all(np.abs(d[gi] - v) <= RTOL * np.abs(v) + 1e-12 * np.abs(v).max()), gi
    check_solve(got, ref)
    mix = ctx.solve_emission(gid, oid, table, obs_phase=list(phases[:2]), precision=M.MCRT_MIXED,
                             n_packets=4000, seed=173, forced=1)
    f64 = ctx.solve_emission(gid, oid, table, obs_phase=list(phases[:2]), n_packets=4000, seed=173, forced=1)
    assert np.all(np.abs(mix["value"] - f64["value"]) <= np.maximum(3.0 * f64["stderr"], 1e-3 * f64["value"]))
    for bad in (dict(forced=4), dict(forced=1, absorption=M.MCRT_CONTINUOUS), dict(forced=1, surface_albedo=0.3)):
        with pytest.raises(M.McrtError) as e:
            ctx.solve_emission(gid, oid, table, n_packets=10, obs_phase=[0.5], **bad)
        assert e.value.name == "EINVAL"
    ctx.free_grid(gid)
    ctx.free_opacity(oid)
    slab, st = I.make_albedo_slab(nlay=10, nlam=2)
    sid, soid = ctx.upload_grid(slab), ctx.upload_opacity(st)
    n = 2000
    dump = dump_buffer(torch_dev, 2, n, 1)
    kw = dict(n_packets=n, seed=175, forced=2, forced_first=1)
    got = ctx.solve_albedo(sid, soid, st, packet_dump=dump, **kw)
    ref = O.solve_albedo(slab, st, O.Params(**kw), keep_packets=True)
    check_packets(dump, ref, (2, 1, n, 1))
    check_solve(got, ref)
    ctx.free_grid(sid)
    ctx.free_opacity(soid)


def test_maximum_index_grids(ctx, torch_dev):
    """Grids at the index limits of the packed lane state: 2048 longitudes x
    1024 latitudes (4.2e6 cells) and 2048 layers; every packet against the
    oracle for emission and albedo; one longitude, latitude or layer more is
    rejected."""
    _log("maximum index grids: 2048x1024x2 and 1x1x2048, emission + albedo, every packet")
    from paper_2110_15640_amd import mcrt as M
    _, table, _ = I.make_emission_3d(8, 4, 2, nband=2, ng=1, config_no=110)
    oid = ctx.upload_opacity(table)
    n = 400
    for grid, seed in ((I.make_sphere(2048, 1024, 2, seed=111), 181), (I.make_sphere(1, 1, 2048, seed=113), 185)):
        gid = ctx.upload_grid(grid)
        dump = dump_buffer(torch_dev, 2, n, 2)
        got = ctx.solve_emission(gid, oid, table, n_packets=n, seed=seed, obs_phase=[0.5, 0.0], packet_dump=dump)
        ref = O.solve_emission(grid, table, O.Params(n_packets=n, seed=seed, obs_phase=(0.5, 0.0)), keep_packets=True)
        check_packets(dump, ref, (2, 1, n, 2))
        check_solve(got, ref)
        alb = ctx.solve_albedo(gid, oid, table, n_packets=n, seed=seed + 1, obs_phase=[0.0, 1.0])
        aref = O.solve_albedo(grid, table, O.Params(n_packets=n, seed=seed + 1, obs_phase=(0.0, 1.0)))
        check_solve(alb, aref)
        ctx.free_grid(gid)
    for shape in ((2049, 4, 2), (8, 1025, 2), (1, 1, 2049)):
        with pytest.raises(M.McrtError) as e:
            ctx.upload_grid(I.make_sphere(*shape, seed=115))
        assert e.value.name == "EINVAL", shape
    ctx.free_opacity(oid)


def test_uploads_on_a_caller_stream(ctx, torch_dev):
    """Uploads ordered on a caller's stream: a copied grid and table uploaded
    on a side stream, and a borrowed grid whose tensors are filled on that
    stream and checked there without a device-wide synchronisation, give the
    same results bit for bit as uploads on the null stream."""
    _log("uploads on a caller stream (copied and borrowed) vs null-stream uploads")
    torch = torch_dev
    grid, table, phases = I.make_emission_3d(16, 8, 10, nband=2, ng=2, config_no=121)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    s = torch.cuda.Stream()
    sid, soid = ctx.upload_grid(grid, stream=s), ctx.upload_opacity(table, stream=s)
    with torch.cuda.stream(s):
        bid = ctx.upload_grid(grid, borrow=True)  # tensors filled and checked on s
    kw = dict(n_packets=2000, seed=195, obs_phase=list(phases[:2]))
    a = ctx.solve_emission(gid, oid, table, **kw)
    for g2, o2 in ((sid, soid), (bid, oid), (bid, soid)):
        b = ctx.solve_emission(g2, o2, table, **kw)
        assert np.array_equal(a["sums"], b["sums"]) and np.array_equal(a["counters"], b["counters"])
    for g2 in (bid, sid, gid):
        ctx.free_grid(g2)
    ctx.free_opacity(soid)
    ctx.free_opacity(oid)


def test_borrowed_device_grid(ctx, torch_dev):
    """A grid whose per-cell arrays are borrowed device tensors (read in
    place, not counted in the library's memory): bit-identical results to the
    copied grid for emission with clouds and raytrace transmission; borrowed
    host pointers and bad device values are rejected."""
    _log("borrowed device grid: emission + transmission vs copied grid; error checks")
    from paper_2110_15640_amd import mcrt as M
    grid, table, phases = I.make_emission_3d(16, 8, 10, nband=2, ng=2, config_no=120)
    rng = np.random.default_rng(31)
    grid.cld_ksca = rng.uniform(0, 3e-2, grid.ncell).astype(np.float32)
    grid.cld_kabs = rng.uniform(0, 3e-3, grid.ncell).astype(np.float32)
    grid.cld_g = rng.uniform(-0.2, 0.8, grid.ncell).astype(np.float32)
    oid = ctx.upload_opacity(table)
    gid = ctx.upload_grid(grid)
    used = ctx.memory_in_use
    bid = ctx.upload_grid(grid, borrow=True)
    per_cell = grid.ncell * (4 + 4 + 8 + 3 * 4)
    assert ctx.memory_in_use - used < per_cell  # only the edge tables were allocated
    kw = dict(n_packets=3000, seed=191, obs_phase=list(phases[:2]))
    a = ctx.solve_emission(gid, oid, table, **kw)
    b = ctx.solve_emission(bid, oid, table, **kw)
    assert np.array_equal(a["sums"], b["sums"]) and np.array_equal(a["counters"], b["counters"])
    kt = dict(n_b=16, n_alpha=24, seed=193, r_star=I.R_SUN)
    assert np.array_equal(ctx.solve_transmission(gid, oid, table, **kt)["sums"],
                          ctx.solve_transmission(bid, oid, table, **kt)["sums"])
    ctx.free_grid(bid)
    ctx.free_grid(gid)
    # a host pointer passed as borrowed
    T = np.ascontiguousarray(grid.T, dtype=np.float32)
    rho = np.ascontiguousarray(grid.rho, dtype=np.float64)
    r, lat, lon = (np.ascontiguousarray(x, dtype=np.float64) for x in (grid.r_edges, grid.lat_edges, grid.lon_edges))
    d = M.GridDesc(0, grid.nlon, grid.nlat, grid.nlay, r.ctypes.data, lat.ctypes.data, lon.ctypes.data,
                   T.ctypes.data, T.ctypes.data, rho.ctypes.data, None, None, None, None, None, None, 0.0,
                   M.MCRT_BORROW_DEVICE)
    import ctypes
    out = ctypes.c_int32()
    assert M.load().mcrt_grid_upload(ctx._h, ctypes.byref(d), None, ctypes.byref(out)) == -1
    # bad values in borrowed device memory: found by the device check
    bad = I.make_sphere(8, 4, 3, seed=5)
    bad.rho = bad.rho.copy()
    bad.rho[7] = np.nan
    with pytest.raises(M.McrtError) as e:
        ctx.upload_grid(bad, borrow=True)
    assert e.value.name == "EINVAL"
    ctx.free_opacity(oid)


def test_multi_grid_batch_graph_replays(ctx, torch_dev):
    """A multi-grid batch recorded as a hipGraph (params.graph): the first call
    records the whole chain (two launches of solves on three uneven grids),
    later identical calls replay it; with eager work and synchronisations in
    between, every replay equals the eager batch bit for bit."""
    _log("multi-grid batch graph: record + 3 replays (2 launches) vs eager, eager work in between")
    specs = [(16, 8, 10), (24, 12, 6), (8, 4, 12)]
    gids, tabs = [], []
    for q, (a, b, c) in enumerate(specs):
        grid, table, _ = I.make_emission_3d(a, b, c, nband=3, ng=2, config_no=130 + q)
        table.k_ray = table.k_ray * 30.0
        gids.append(ctx.upload_grid(grid))
        tabs.append((ctx.upload_opacity(table), table))
    items = [dict(mode="emission", gid=gids[0], oid=tabs[0][0], table=tabs[0][1], spec_idx=[0, 2], n_packets=1500),
             dict(mode="albedo", gid=gids[1], oid=tabs[1][0], table=tabs[1][1], spec_idx=[1], n_packets=800),
             dict(mode="emission", gid=gids[2], oid=tabs[2][0], table=tabs[2][1], spec_idx=[2, 0], n_packets=1100)]
    common = dict(obs_phase=[0.0, 0.5], seed=197, decorrelate=1, max_batch=5)
    eager = ctx.solve_batch(items, **common)
    for rep in range(4):
        got = ctx.solve_batch(items, graph=1, **common)
        for e, g in zip(eager, got):
            assert np.array_equal(e["sums"], g["sums"]) and np.array_equal(e["counters"], g["counters"]), rep
            assert np.array_equal(e["value"], g["value"]), rep
        # eager work and a synchronisation between replays
        ctx.solve_emission(gids[0], tabs[0][0], tabs[0][1], n_packets=300, seed=rep, obs_phase=[0.25], spec_idx=[1])
        torch_dev.cuda.synchronize()
    for g in gids:
        ctx.free_grid(g)
    for o, _ in tabs:
        ctx.free_opacity(o)
