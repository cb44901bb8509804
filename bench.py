#!/usr/bin/env python3
"""Benchmark: 3D emission phase curve on one MI355X.

Workload (one step = one pass of the whole hot path): a 128 x 64 x 50
lon-lat-radius grid with a day-night temperature contrast, a 100 band x 8 g
correlated-k table, 4 orbital phases and 1e6 packets per (band, g) solve:
for every (band, g) the ck gather, emission sources + CDF, the transport with
peel-off toward all 4 observers and the tally reduction, then the spectra
F_p(band, phase).  Inputs are uploaded (resident in HBM) before timing.

Prints one JSON line with packets/s, the achieved Monte Carlo error (and the
packets needed for 1e-3 relative standard error), the transport kernel's
roofline figure measured live with HIP events, and the FP64 oracle timed on a
bounded sample on this host's cores.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "packets/s at 1e-3 rel. spectral error, plain vs batched; p50/p99 solve latency"
# Algorithmic work of one cell crossing of the transport (the dominant kernel):
# about 80 FP64 flops, 3 square roots and 5 divisions, each root or division
# counted as one operation here (88), plus the 4 B alpha gather of the mixed
# form.  Our own finer count of the spherical traversal is 110 FP64 flops: r.r
# and p.d (10); outer shell C, D, sqrt, root (7); inner shell on inward rays
# (3.5 on average); the entry-face tolerance (2); two latitude cones, each a,
# b, c, discriminant, sqrt, two roots and the nappe checks (2 x 33); two
# longitude half-planes when approached (15); the move (6); the optical-depth
# update (2).  Both fractions are reported.
FLOP_PER_CROSSING = 88.0
FLOP_PER_CROSSING_OWN = 110.0
ALPHA_BYTES_MIXED = 4.0   # per crossing
OMEGA_PGAS_BYTES = 8.0    # per interaction (omega and P_gas, FP32)
CDF_PROBE_BYTES = 8.0     # per probe of the emission CDF (FP64), ceil(log2(ncell)) probes per birth
PEAK_FP64_VECTOR = 78.6  # TFLOP/s, MI355X
PEAK_HBM = 8000.0  # GB/s
# VALU issue peak: a wave64 instruction occupies a 16-lane SIMD for 4 cycles,
# 256 CUs x 4 SIMDs at 2.4 GHz (the same unit counts give 78.6 FP64 TFLOP/s)
PEAK_VALU_WAVE_INSTS = 256 * 4 * 2.4e9 / 4.0  # wave-level VALU instructions per second

# HBM traffic of the transport kernel from two rocprofv3 counter passes
# (FETCH_SIZE, WRITE_SIZE, each scaled by what it reads for a 1 GiB copy) and
# its VALU busy fraction, measured on one launch configuration of this
# workload.  Reported only while the kernel sources hash to `sha` and the run
# matches that configuration (grid, packets per solve, observers, launch
# shape, solves per launch); otherwise null.
def _traffic(fetch_kib, write_kib, copy_fetch_kib, copy_write_kib):
    """HBM bytes from FETCH_SIZE / WRITE_SIZE (KiB per dispatch), each scaled
    by what it reads for a 1 GiB device copy (1,048,576 KiB each way)."""
    return (fetch_kib * 1048576.0 / copy_fetch_kib + write_kib * 1048576.0 / copy_write_kib) * 1024.0


def _busy(active_valu, wave_cycles, waves_per_simd=4):
    """SQ_ACTIVE_INST_VALU per wave cycle times the waves sharing a SIMD: the
    share of SIMD cycles with a VALU instruction in flight (about 1 when the
    SIMDs issue VALU work every cycle; FP64 instructions that occupy a SIMD
    for more than one cycle can take it slightly past 1)."""
    return active_valu / wave_cycles * waves_per_simd


K4_PROFILE = {
    "sha": "672340fea5202d167d0d2aa733b7075f8f01962dfdbd22a013706e8becd4c134",
    "grid": [128, 64, 50], "packets_per_solve": 1000000, "n_obs": 4, "solves_per_launch": 800,
    # per event threshold (4 blocks per compute unit, wave batch 32): bytes, VALU busy and
    # wave-level VALU instructions (SQ_INSTS_VALU) per launch
    "shapes": {
        20: {"bytes_per_launch": _traffic(1.31076e8, 1.18905e8, 524343, 1.04859e6),
             "valu_busy": _busy(1.61723e12, 6.51007e12), "valu_insts": 1.57343e12},
        24: {"bytes_per_launch": _traffic(2.61871e8 / 2, 2.3786e8 / 2, 524343, 1.04859e6),
             "valu_busy": _busy(3.19614e12, 1.28055e13), "valu_insts": 3.1132e12 / 2},
        28: {"bytes_per_launch": _traffic(1.30884e8, 1.18958e8, 524343, 1.04859e6),
             "valu_busy": _busy(1.60599e12, 6.41207e12), "valu_insts": 1.5658e12},
        32: {"bytes_per_launch": _traffic(1.31367e8, 1.18989e8, 524343, 1.04859e6),
             "valu_busy": _busy(1.6346e12, 6.50642e12), "valu_insts": 1.59495e12},
    },
}
# The same for the chord optical-depth kernel of the transmission solve: bytes
# per (chord segment, wavelength) over its launches.
K5_PROFILE = {
    "sha": "0eb2314978dcf52aae2f8960283e4800abb4b033705255706a7519cf7c401028",
    "n_segments": 7861278, "n_lambda": 20000,
    # per precision (1 mixed: FP32 rows; 0 FP64), over 314 launches of 64 wavelengths (20,064)
    "bytes_per_seg_wl": {1: _traffic(1.88063e8, 902880, 524722, 1.04923e6) / (7861278 * 20064),
                         0: _traffic(4.72339e8, 902880, 524722, 1.04923e6) / (7861278 * 20064)},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1, help="untimed full steps of the batched form first")
    ap.add_argument("--bands", type=int, default=100, help="bands solved per step (workload: 100)")
    ap.add_argument("--packets", type=float, default=1e6, help="packets per (band, g) (workload: 1e6)")
    ap.add_argument("--plain-steps", type=int, default=1, help="timed steps of the plain FP64 form (0 = skip)")
    ap.add_argument("--autotune", type=int, default=1, help="pick the persistent launch shape by trial solves")
    ap.add_argument("--ev-threshold", type=int, default=0, help="launch shape when --autotune 0 (0 = library default)")
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--wave-batch", type=int, default=0)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-packets", type=int, default=30000)
    ap.add_argument("--transmission", type=int, default=1, help="also time the hi-res transmission workload")
    ap.add_argument("--gsample", type=int, default=1,
                    help="also run the workload with per-packet g sampling (composite), same packets per band")
    ap.add_argument("--albedo", type=int, default=1, help="also time the 1D albedo workload (plain / batched / graph)")
    ap.add_argument("--batch-scale", type=float, default=0.1,
                    help="packet scale of the 256-request multi-grid batch leg (0 = skip)")
    ap.add_argument("--batch-plain", type=int, default=32,
                    help="time N randomly chosen requests of that batch in the plain FP64 form too (0 = skip)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="duration of the Poisson serving leg (0 = skip)")
    ap.add_argument("--serve-workers", type=int, default=3, help="serving worker threads (requests on the device at once)")
    ap.add_argument("--serve-scale", type=float, default=0.0,
                    help="packet scale of the served requests (0 = calibrate to the offered load)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="run one 1 GiB device copy first (reference kernel for HBM counter scaling)")
    return ap.parse_args()


def kernel_sha(main: str = "transport.hip") -> str:
    """sha256 of a kernel's sources (its file, then the shared headers)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2110_15640_amd", "csrc")
    h = hashlib.sha256()
    for f in (main, "device_common.hpp", "mcrt_internal.hpp"):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def host_cpu() -> dict:
    """CPU model and clock of this host (from /proc/cpuinfo)."""
    model, mhz = None, []
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name") and model is None:
                model = ln.split(":", 1)[1].strip()
            elif ln.startswith("cpu MHz"):
                mhz.append(float(ln.split(":", 1)[1]))
    except OSError:
        pass
    return {"cpu_model": model, "cpu_mhz_mean": float(np.mean(mhz)) if mhz else None,
            "logical_cpus": os.cpu_count()}


def cpu_baseline(grid, table, phases, n_per, log):
    """The FP64 oracle as it stands, on this host's cores: a bounded sample of
    the emission workload (the reported rate), the 1D albedo workload in full
    and a 200-wavelength window of the hi-res transmission workload."""
    from oracle import oracle as O  # test infrastructure: the CPU baseline leg only
    from paper_2110_15640_amd import inputs as I
    bands = list(range(0, table.nband, max(table.nband // 10, 1)))[:10]
    p = O.Params(n_packets=n_per, seed=211015641, obs_phase=tuple(phases))
    t0 = time.perf_counter()
    r = O.solve_emission(grid, table, p, spec_idx=bands)
    dt = time.perf_counter() - t0
    npk = len(bands) * table.ng * n_per
    cross = float(r.counters[:, :, 7].sum())
    cores = int(O.lib().orc_max_threads())
    out = {"value": npk / dt, "unit": "packets/s", "cores": cores, "kind": "oracle",
           "sample": f"{len(bands)} evenly spaced bands x {table.ng} g x {n_per} packets on the full "
                     f"{grid.nlon}x{grid.nlat}x{grid.nlay} grid, 4 phases ({npk} packets, {dt:.1f} s)",
           "crossings_per_s_per_core": cross / dt / cores, **host_cpu()}
    log(f"[bench]   oracle emission sample: {dt:.1f} s")
    slab, ck1 = I.make_albedo_slab()
    t0 = time.perf_counter()
    O.solve_albedo(slab, ck1, O.Params(n_packets=100_000, seed=211015641))
    d1 = time.perf_counter() - t0
    out["albedo_1d_full"] = {"packets": ck1.nband * 100_000, "s": d1, "packets_per_s": ck1.nband * 100_000 / d1}
    log(f"[bench]   oracle 1D albedo in full: {d1:.1f} s")
    hg, hr = I.make_transmission_hires()
    t0 = time.perf_counter()
    O.solve_transmission(hg, hr, O.Params(n_b=256, n_alpha=360, seed=211015643, r_star=I.R_SUN),
                         spec_idx=list(range(200)))
    d3 = time.perf_counter() - t0
    out["transmission_window"] = {"wavelengths": 200, "chords": 256 * 360, "s": d3,
                                  "chord_wavelengths_per_s": 256 * 360 * 200 / d3,
                                  "full_20000_extrapolated_s": d3 * 100.0}
    log(f"[bench]   oracle transmission, 200 wavelengths: {d3:.1f} s")
    return out


def transmission_leg(M, I):
    """3D high-resolution transmission: 128x64x60 grid with winds, 20,000
    wavelengths (1.0-1.1 um), 256 x 360 jittered chords; the Doppler-shifted
    alpha gather and the chord optical depths for every wavelength, in the
    FP32-alpha mixed form (the reported one) and in FP64."""
    import torch
    grid, table = I.make_transmission_hires()
    nch = 256 * 360
    out = {"workload": f"3D hi-res transmission: {grid.nlon}x{grid.nlat}x{grid.nlay} grid, {table.nlam} wavelengths "
                       "1.0-1.1 um, 256 x 360 chords, winds + rotation Doppler"}
    with M.Context(0) as ctx:
        gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
        res = {}
        for name, prec in (("fp64", M.MCRT_FP64), ("mixed", M.MCRT_MIXED)):
            kw = dict(n_b=256, n_alpha=360, seed=211015643, r_star=I.R_SUN, profile=1, precision=prec)
            ctx.solve_transmission(gid, oid, table, spec_idx=list(range(64)), **kw)  # scratch and chords warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.solve_transmission(gid, oid, table, **kw)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            res[name] = r
            # K5: per (segment, wavelength) one alpha gather (4 B mixed, 8 B FP64),
            # plus once per 64-wavelength launch the segment record (cell and length:
            # 8 B mixed, 12 B FP64) and the chord record (offset, impact weight, flag: 20 B)
            nseg, nl, nblk = r["n_segments"], table.nlam, r["kernel_launches"]
            ab = 4.0 if prec == M.MCRT_MIXED else 8.0
            k5_bytes = nseg * nl * ab + nseg * nblk * (ab + 4.0) + nch * nblk * 20.0
            ncell_tr = grid.nlon * grid.nlat * grid.nlay
            k5_gbps = k5_bytes / (r["kernel_ms"] * 1e-3) / 1e9
            P = K5_PROFILE
            same = kernel_sha("kernels.hip") == P["sha"] and nseg == P["n_segments"] and nl == P["n_lambda"]
            out[name] = {"ms": wall * 1e3, "chord_wavelengths_per_s": nch * nl / wall,
                         "chord_tau_kernel_ms": r["kernel_ms"], "chord_tau_launches": nblk, "segments": nseg,
                         # the extinction blocks of one launch are formed while the previous launch's
                         # chords are summed (two streams), so launches overlap: the same bytes over
                         # the whole leg's wall time
                         "chord_tau_bytes_over_leg_GBps": k5_bytes / wall / 1e9,
                         "roofline": {"bound": "hbm", "kernel": f"k_chord_tau<{'float' if ab == 4 else 'double'}>",
                                      "achieved": k5_gbps, "peak": PEAK_HBM, "unit": "GB/s",
                                      "frac": k5_gbps / PEAK_HBM,
                                      "traffic": (P["bytes_per_seg_wl"][prec] * nseg * nl / max(nblk, 1)
                                                  if same else None),
                                      "traffic_unit": "bytes per launch (mean)",
                                      "bytes_per_segment_wavelength": ab,
                                      # one launch's extinction block (cells x 64 wavelengths) is 126 MB in
                                      # FP32, 252 MB in FP64: it stays in the 256 MB Infinity Cache, so the
                                      # gathers can pass the HBM rate (frac > 1); the bytes that do leave
                                      # L2 are the traffic above
                                      "block_MB": ncell_tr * 64 * ab / 1e6}}
        depth = res["mixed"]["value"][:, 0]
        d64 = res["fp64"]["value"][:, 0]
        excess = np.abs(res["mixed"]["sums"][..., 0] - res["fp64"]["sums"][..., 0]) / \
            np.abs(res["fp64"]["sums"][..., 0])
        out.update({"form": "mixed (FP32 alpha rows, FP64 optical depths)",
                    "ms": out["mixed"]["ms"], "chord_wavelengths_per_s": out["mixed"]["chord_wavelengths_per_s"],
                    "roofline": out["mixed"]["roofline"],
                    "depth_min": float(depth.min()), "depth_max": float(depth.max()),
                    "rel_se_median": float(np.median(res["mixed"]["stderr"][:, 0] / depth)),
                    "mixed_vs_fp64_sums_rel_max": float(excess.max()),
                    "mixed_vs_fp64_sigma_max": float((np.abs(depth - d64) / res["fp64"]["stderr"][:, 0]).max())})
    return out


def albedo_leg(M, I, reps=15):
    """1D plane-parallel albedo spectrum (50 layers, 10 wavelengths x 1e5
    packets, uniform-disk incidence): plain FP64 launches per solve, the
    batched FP32-mixed form, and the same batched solve recorded once as a
    hipGraph and replayed.  The three forms are timed call by call in
    interleaved rounds (so drift of clocks or of the host hits them alike)
    and the median call is reported."""
    import torch
    grid, table = I.make_albedo_slab()
    npk = 100_000
    out = {"workload": f"1D albedo: {grid.nlay} layers, {table.nband} wavelengths x {npk} packets"}
    with M.Context(0) as ctx:
        gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
        forms = (("plain_fp64", dict(precision=M.MCRT_FP64, max_batch=1)),
                 ("batched_mixed", dict(precision=M.MCRT_MIXED, max_batch=0)),
                 ("batched_mixed_graph", dict(precision=M.MCRT_MIXED, max_batch=0, graph=1)))
        vals, times = {}, {name: [] for name, _ in forms}
        for name, kw in forms:  # warm up; the graph form records here
            ctx.solve_albedo(gid, oid, table, n_packets=npk, seed=211015641, **kw)
        torch.cuda.synchronize()
        for _ in range(reps):
            for name, kw in forms:
                t0 = time.perf_counter()
                vals[name] = ctx.solve_albedo(gid, oid, table, n_packets=npk, seed=211015641, **kw)
                torch.cuda.synchronize()
                times[name].append(time.perf_counter() - t0)
        for name, _ in forms:
            dt = float(np.median(times[name]))
            out[name] = {"ms": dt * 1e3, "packets_per_s": table.nband * npk / dt,
                         "ms_min": min(times[name]) * 1e3, "ms_max": max(times[name]) * 1e3}
        a, b, c = vals["plain_fp64"], vals["batched_mixed"], vals["batched_mixed_graph"]
        out["graph_equals_eager"] = bool(np.array_equal(b["sums"], c["sums"]))
        out["mixed_vs_fp64_rel_max"] = float((np.abs(b["value"] - a["value"]) / np.abs(a["value"])).max())
        out["A_g_rel_se_median"] = float(np.median(a["stderr"] / a["value"]))
    return out


def batch_leg(M, I, scale, plain, log):
    """256 albedo / emission requests on grids from 32x16x30 to 128x64x60,
    10-500 bands x 8 g each, packets per (band, g) log-uniform 1e4-1e6 times
    `scale`: all of them in one mcrt_solve_batch call (FP32-mixed, multi-grid
    persistent launches) against one FP64 launch per (band, g) solve."""
    import torch
    grids, table, reqs = I.make_batch_mix(packet_scale=scale)
    common = dict(obs_phase=[0.0, 0.5], seed=211015644, profile=1)
    out = {"workload": f"{len(reqs)} albedo/emission requests on grids 32x16x30..128x64x60, 10-500 bands x 8 g, "
                       f"packets per (band, g) log-uniform 1e4-1e6 x {scale:g}, 2 observers"}
    with M.Context(0) as ctx:
        oid = ctx.upload_opacity(table)
        gids = [ctx.upload_grid(g) for g in grids]
        items = [dict(mode=r.mode, gid=gids[r.grid_index], oid=oid, table=table, spec_idx=r.bands,
                      n_packets=r.n_packets) for r in reqs]
        packets = sum(len(r.bands) * table.ng * r.n_packets for r in reqs)
        solves = sum(len(r.bands) * table.ng for r in reqs)
        ctx.solve_batch(items[:2], precision=M.MCRT_MIXED, **common)  # warm kernels and scratch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bo = ctx.solve_batch(items, precision=M.MCRT_MIXED, **common)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        log(f"[bench]   batch: {solves} solves, {packets} packets in {tb:.2f} s")
        out.update({"solves": solves, "packets": packets, "batched_s": tb, "batched_packets_per_s": packets / tb,
                    "batched_transport_launches": int(sum(o["kernel_launches"] for o in bo[:1]))})
        if plain:
            # plain FP64 (one launch per solve) against the batched form on the
            # same randomly chosen subset of requests (the whole set would take
            # several minutes in the plain form)
            pick = np.random.Generator(np.random.PCG64(211015644)).choice(len(items), size=min(plain, len(items)),
                                                                          replace=False)
            sub = [items[q] for q in sorted(pick)]
            psolves = sum(len(it["spec_idx"]) * table.ng for it in sub)
            ppk = sum(len(it["spec_idx"]) * table.ng * it["n_packets"] for it in sub)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bs = ctx.solve_batch(sub, precision=M.MCRT_MIXED, **common)
            torch.cuda.synchronize()
            tbs = time.perf_counter() - t0
            t0 = time.perf_counter()
            po = []
            for q, it in enumerate(sub):
                fn = ctx.solve_albedo if it["mode"] == "albedo" else ctx.solve_emission
                po.append(fn(it["gid"], oid, table, spec_idx=it["spec_idx"], n_packets=it["n_packets"],
                             precision=M.MCRT_FP64, max_batch=1, **common))
                if q % 4 == 3:
                    log(f"[bench]   plain: {q + 1}/{len(sub)} requests")
            torch.cuda.synchronize()
            tp = time.perf_counter() - t0
            log(f"[bench]   subset of {len(sub)} requests ({psolves} solves): plain {tp:.2f} s, batched {tbs:.2f} s")
            d = np.concatenate([(np.abs(b["value"] - a["value"]) / np.maximum(np.abs(a["value"]), 1e-300)).ravel()
                                for a, b in zip(po, bs)])
            z = np.concatenate([(np.abs(b["value"] - a["value"]) / np.maximum(a["stderr"], 1e-300)).ravel()
                                for a, b in zip(po, bs)])
            # the whole set in the plain form, extrapolated from the subset two
            # ways: per solve (launch-bound) and per packet (transport-bound)
            plain_all_per_solve = tp * solves / psolves
            plain_all_per_packet = tp * packets / ppk
            out["subset"] = {"requests": len(sub), "request_indices": [int(q) for q in sorted(pick)],
                             "solves": psolves, "packets": ppk,
                             "plain_s": tp, "plain_packets_per_s": ppk / tp,
                             "batched_s": tbs, "batched_packets_per_s": ppk / tbs, "batched_over_plain": tp / tbs,
                             "mixed_vs_fp64_rel_median": float(np.median(d)),
                             "mixed_vs_fp64_rel_p99": float(np.quantile(d, 0.99)),
                             "mixed_vs_fp64_sigma_max": float(z.max())}
            out["plain_all_extrapolated"] = {
                "per_solve_s": plain_all_per_solve, "per_packet_s": plain_all_per_packet,
                "batched_over_plain_per_solve": plain_all_per_solve / tb,
                "batched_over_plain_per_packet": plain_all_per_packet / tb,
                "formula": "plain_s(subset) x solves(all) / solves(subset); plain_s(subset) x packets(all) / "
                           "packets(subset)"}
        rel = np.concatenate([(o["stderr"] / np.maximum(np.abs(o["value"]), 1e-300)).ravel() for o in bo])
        out["rel_se_median"] = float(np.median(rel))
    return out


def run_form(ctx, M, gid, oid, table, bands, npk, phases, precision, max_batch, steps, warmup, tune):
    kw = dict(n_packets=npk, obs_phase=list(phases), spec_idx=bands, precision=precision, profile=1,
              seed=211015642, max_batch=max_batch, **tune)
    for w in range(warmup):
        r = ctx.solve_emission(gid, oid, table, **kw)
        print(f"[bench]   warmup {w + 1}/{warmup}: {r['elapsed_ms']:.1f} ms device", flush=True)
    import torch
    torch.cuda.synchronize()
    res = []
    t0 = time.perf_counter()
    for s in range(steps):
        res.append(ctx.solve_emission(gid, oid, table, **kw))
        print(f"[bench]   step {s + 1}/{steps}: {res[-1]['elapsed_ms']:.1f} ms device", flush=True)
    torch.cuda.synchronize()
    return res, time.perf_counter() - t0


def summarize(res, wall, steps, pk_step, npk, ng):
    value = pk_step * steps / wall
    r = res[-1]
    rel = (r["stderr"] / np.maximum(r["value"], 1e-300)).ravel()
    need = npk * ng * (rel / 1e-3) ** 2  # packets per band for 1e-3 relative error
    cross = float(sum(x["counters"][:, :, 7].sum() for x in res))
    nint = float(sum(x["counters"][:, :, 6].sum() for x in res))
    kms = float(sum(x["kernel_ms"] for x in res))
    launches = int(sum(x["kernel_launches"] for x in res))
    return value, rel, need, cross, nint, kms, launches


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the path would shard by whole "
              "(band, g) solves across GPUs, each GPU holding the grid and table", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2110_15640_amd import inputs as I
    from paper_2110_15640_amd import mcrt as M

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    grid, table, phases = I.make_emission_3d()
    bands = list(range(a.bands))
    npk = int(a.packets)
    ctx = M.Context(0)
    gid, oid = ctx.upload_grid(grid), ctx.upload_opacity(table)
    pk_step = len(bands) * table.ng * npk
    tune = {}
    if a.copy_calib:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print(f"[bench] workload: {len(bands)} bands x {table.ng} g x {npk} packets, 4 phases", flush=True)
    pres = None
    if a.plain_steps > 0:
        print("[bench] plain form: FP64, one transport launch per (band, g)", flush=True)
        # one untimed band warms the FP64 kernels and the scratch
        ctx.solve_emission(gid, oid, table, n_packets=npk, obs_phase=list(phases), spec_idx=[0],
                           precision=M.MCRT_FP64, max_batch=1)
        pres, pwall = run_form(ctx, M, gid, oid, table, bands, npk, phases, M.MCRT_FP64, 1, a.plain_steps, 0, tune)
        pval, prel, _, pcross, _, pkms, plaunch = summarize(pres, pwall, a.plain_steps, pk_step, npk, table.ng)
    if a.autotune:
        print("[bench] autotuning the persistent launch shape (untimed)", flush=True)
        tuned = ctx.autotune("emission", gid, oid, n_packets=npk, obs_phase=list(phases), spec_idx=bands,
                             precision=M.MCRT_MIXED)
        tune = {k: v for k, v in tuned.items() if k.startswith("tune_")}
    else:
        tune = {"tune_ev_threshold": a.ev_threshold, "tune_blocks_per_cu": a.blocks_per_cu,
                "tune_wave_batch": a.wave_batch}
    print(f"[bench] launch shape: {tune}", flush=True)
    print("[bench] batched form: FP32-mixed, all (band, g) solves in persistent launches", flush=True)
    bres, bwall = run_form(ctx, M, gid, oid, table, bands, npk, phases, M.MCRT_MIXED, 0, a.steps, a.warmup, tune)
    value, rel, need, cross, nint, kms, launches = summarize(bres, bwall, a.steps, pk_step, npk, table.ng)
    ksec = kms * 1e-3
    ach = cross * FLOP_PER_CROSSING / ksec / 1e12
    ach_own = cross * FLOP_PER_CROSSING_OWN / ksec / 1e12
    solves_per_launch = len(bands) * table.ng * a.steps / max(launches, 1)
    # algorithmic HBM bytes of the transport: alpha gathers, omega / P_gas per
    # interaction, emission-CDF probes per birth
    probes = math.ceil(math.log2(grid.ncell))
    k4_bytes = cross * ALPHA_BYTES_MIXED + nint * OMEGA_PGAS_BYTES + pk_step * a.steps * probes * CDF_PROBE_BYTES
    k4_gbps = k4_bytes / ksec / 1e9
    P = K4_PROFILE
    shape = P["shapes"].get(tune.get("tune_ev_threshold")) if (
        tune.get("tune_blocks_per_cu") == 4 and tune.get("tune_wave_batch") == 32) else None
    same_run = (shape is not None and kernel_sha() == P["sha"] and [grid.nlon, grid.nlat, grid.nlay] == P["grid"]
                and npk == P["packets_per_solve"] and len(phases) == P["n_obs"]
                and abs(solves_per_launch - P["solves_per_launch"]) < 1e-9)
    traffic = shape["bytes_per_launch"] if same_run else None
    avg_s = ksec / max(launches, 1)
    out = {
        "metric": METRIC, "value": value, "unit": "packets/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": bwall / a.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"3D emission phase curve: {grid.nlon}x{grid.nlat}x{grid.nlay} lon-lat-radius grid, "
                               f"{len(bands)} bands x {table.ng} g correlated-k (log-normal k), 4 phases, "
                               f"{npk} packets per (band, g)",
                   "form": "batched FP32-mixed persistent", "packets_per_step": pk_step,
                   "crossings_per_step": cross / a.steps},
        "tuned_launch": tune,
        "error": {"rel_se_median": float(np.median(rel)), "rel_se_max": float(rel.max()),
                  "packets_per_band_for_1e-3_median": float(np.median(need)),
                  "packets_per_band_for_1e-3_max": float(need.max()),
                  "seconds_per_band_for_1e-3_median_batched": float(np.median(need)) / value,
                  "seconds_per_band_for_1e-3_max_batched": float(need.max()) / value},
        "roofline": {"bound": "alu", "kernel": "k_transport_persistent<MIXED>", "achieved": ach,
                     "peak": PEAK_FP64_VECTOR, "unit": "TFLOP/s", "frac": ach / PEAK_FP64_VECTOR, "traffic": traffic,
                     "traffic_unit": "bytes per launch", "avg_launch_ms": avg_s * 1e3, "launches": launches,
                     "solves_per_launch": solves_per_launch, "crossings": cross,
                     "flop_per_crossing": FLOP_PER_CROSSING,
                     "flop_per_crossing_own_count": FLOP_PER_CROSSING_OWN,
                     "frac_own_count": ach_own / PEAK_FP64_VECTOR,
                     "hbm_algorithmic_GBps": k4_gbps, "hbm_frac": k4_gbps / PEAK_HBM,
                     "hbm_algorithmic_bytes": k4_bytes,
                     "traffic_GBps": None if traffic is None else traffic / avg_s / 1e9,
                     "valu_busy": shape["valu_busy"] if same_run else None,
                     # the issue roofline: wave-level VALU instructions per second (profiled
                     # count per launch over this run's launch time) against the VALU peak
                     "valu_insts_per_s": shape["valu_insts"] / avg_s if same_run else None,
                     "valu_issue_frac": shape["valu_insts"] / avg_s / PEAK_VALU_WAVE_INSTS if same_run else None},
    }
    if a.gsample:
        print("[bench] per-packet g sampling (composite), same packets per band", flush=True)
        kw = dict(n_packets=npk * table.ng, obs_phase=list(phases), spec_idx=bands, precision=M.MCRT_MIXED,
                  seed=211015642, g_sampling=3, **tune)
        ctx.solve_emission(gid, oid, table, **{**kw, "spec_idx": bands[:1]})  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gr = ctx.solve_emission(gid, oid, table, **kw)
        torch.cuda.synchronize()
        gt = time.perf_counter() - t0
        grel = (gr["stderr"] / np.maximum(gr["value"], 1e-300)).ravel()
        gneed = npk * table.ng * (grel / 1e-3) ** 2
        gdiff = np.abs(gr["value"] - bres[-1]["value"]) / np.sqrt(gr["stderr"] ** 2 + bres[-1]["stderr"] ** 2)
        out["g_sampled"] = {"scheme": "composite", "packets_per_band": npk * table.ng, "ms": gt * 1e3,
                            "packets_per_s": pk_step / gt, "rel_se_median": float(np.median(grel)),
                            "packets_per_band_for_1e-3_median": float(np.median(gneed)),
                            "seconds_per_band_for_1e-3_median": float(np.median(gneed)) / (pk_step / gt),
                            "vs_fixed_g_sigma_max": float(gdiff.max())}
    if pres is not None:
        # spectrum difference of the mixed form from the FP64 form on the same random stream
        dmix = np.abs(bres[-1]["value"] - pres[-1]["value"]) / np.abs(pres[-1]["value"])
        out["plain"] = {"value": pval, "unit": "packets/s", "dtype": "f64", "steps": a.plain_steps,
                        "ms_per_step": pwall / a.plain_steps * 1e3, "launches_per_step": plaunch // a.plain_steps,
                        "kernel_ms_per_step": pkms / a.plain_steps}
        out["batched_over_plain"] = value / pval
        out["error"].update({"seconds_per_band_for_1e-3_median_plain": float(np.median(need)) / pval,
                             "seconds_per_band_for_1e-3_max_plain": float(need.max()) / pval,
                             "mixed_vs_fp64_rel_max": float(dmix.max()),
                             "mixed_vs_fp64_rel_median": float(np.median(dmix))})
    if a.transmission:
        out["transmission"] = transmission_leg(M, I)
    if a.albedo:
        print("[bench] 1D albedo leg: plain vs batched vs graph replay", flush=True)
        out["albedo_1d"] = albedo_leg(M, I)
    if a.batch_scale > 0:
        print(f"[bench] batch leg: 256 multi-grid requests, packet scale {a.batch_scale:g}", flush=True)
        out["batch"] = batch_leg(M, I, a.batch_scale, a.batch_plain, lambda m: print(m, flush=True))
    if a.serve_seconds > 0:
        print(f"[bench] serving leg: Poisson 20 req/s for {a.serve_seconds:.0f} s, then 8 requests of each kind "
              "re-run alone", flush=True)
        from paper_2110_15640_amd import serve as SV
        with M.Context(0) as sctx:
            rep = SV.run_poisson(sctx, rate=20.0, duration=a.serve_seconds, load=0.7, workers=a.serve_workers,
                                 scale=a.serve_scale,
                                 log=lambda m: print(m, flush=True))
        out["serving"] = rep.summary()
    if a.cpu_baseline:
        print("[bench] timing the FP64 oracle on a bounded sample", flush=True)
        out["cpu_baseline"] = cpu_baseline(grid, table, phases, a.cpu_packets, lambda m: print(m, flush=True))
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
