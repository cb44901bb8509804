"""Poisson request stream over the library's serving API (mcrt_submit / poll /
wait): mixed albedo, emission and transmission requests on resident grids and
tables, continuous admission by the HBM budget, p50 / p99 latency.

Request mix (by arrival): 50 % albedo on the 1D column (10 wavelengths),
35 % emission on the 3D grid (10 bands x 8 g, one phase), 15 % hi-res
transmission on the 3D grid with winds (a 200-wavelength window, 256 x 360
chords).  Packet counts are scaled once so that the offered load is a chosen
fraction of the measured service capacity.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Dict, List

import numpy as np

from . import inputs as I
from . import mcrt as M


@dataclass
class Workload:
    kind: str
    mode: str
    gid: int
    oid: int
    table: object
    kw: dict
    packets: int  # packets (or chords x wavelengths) per request


@dataclass
class ServeReport:
    rate: float
    duration: float
    n_requests: int
    load_target: float
    scale: float
    latencies_ms: List[float] = field(default_factory=list)
    kinds: List[str] = field(default_factory=list)
    packets: int = 0           # Monte Carlo packets (albedo and emission requests)
    chord_wavelengths: int = 0  # chords x wavelengths (transmission requests)
    wall: float = 0.0
    service_ms: Dict[str, float] = field(default_factory=dict)
    # per finished request: (start, end) on the device side of admission, in s
    # from the first submit (submit time + queued_ms, submit time + latency_ms)
    spans: List[tuple] = field(default_factory=list)
    alone: dict = field(default_factory=dict)

    def overlap(self) -> dict:
        """Fractions of the busy time (some request running) during which at
        least 2 (and 3) requests were running together."""
        ev = sorted([(a, 1) for a, _ in self.spans] + [(b, -1) for _, b in self.spans])
        busy = two = three = 0.0
        n, last = 0, None
        for t, d in ev:
            if last is not None and n > 0:
                dt = t - last
                busy += dt
                two += dt if n >= 2 else 0.0
                three += dt if n >= 3 else 0.0
            n += d
            last = t
        return {"busy_s": busy, "frac_ge2_running": two / busy if busy > 0 else 0.0,
                "frac_ge3_running": three / busy if busy > 0 else 0.0}

    def summary(self) -> dict:
        lat = np.array(self.latencies_ms)
        out = {"requests": self.n_requests, "rate_per_s": self.rate, "duration_s": self.duration,
               "offered_load": self.load_target, "packet_scale": self.scale,
               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "mean_ms": float(lat.mean()), "packets_per_s": self.packets / self.wall,
               "chord_wavelengths_per_s": self.chord_wavelengths / self.wall,
               "service_ms_alone": self.service_ms, "concurrency": self.overlap()}
        for k in ("albedo", "emission", "transmission"):
            sel = [l for l, kk in zip(self.latencies_ms, self.kinds) if kk == k]
            if sel:
                out[f"p50_ms_{k}"] = float(np.percentile(sel, 50))
                out[f"p99_ms_{k}"] = float(np.percentile(sel, 99))
        if self.alone:
            out["alone_vs_mix"] = self.alone
        return out


def upload_inputs(ctx: M.Context) -> dict:
    """Upload the three grids and tables once; they stay resident."""
    slab, ck1 = I.make_albedo_slab()
    grid, ck, _ = I.make_emission_3d()
    hg, hr = I.make_transmission_hires()
    return dict(albedo=(ctx.upload_grid(slab), ctx.upload_opacity(ck1), ck1),
                emission=(ctx.upload_grid(grid), ctx.upload_opacity(ck), ck),
                transmission=(ctx.upload_grid(hg), ctx.upload_opacity(hr), hr))


def build_workloads(res: dict, scale: float = 1.0, precision: int = M.MCRT_MIXED) -> List[Workload]:
    g1, o1, ck1 = res["albedo"]
    g2, o2, ck = res["emission"]
    g3, o3, hr = res["transmission"]
    n_alb = max(int(1e5 * scale), 64)
    n_em = max(int(1e5 * scale), 64)
    nb = max(int(round(256 * math.sqrt(scale))), 8)
    na = max(int(round(360 * math.sqrt(scale))), 8)
    bands = list(range(0, 100, 10))
    return [
        Workload("albedo", "albedo", g1, o1, ck1, dict(n_packets=n_alb, precision=precision), 10 * n_alb),
        Workload("emission", "emission", g2, o2, ck, dict(n_packets=n_em, obs_phase=[0.5], spec_idx=bands,
                                                          precision=precision), len(bands) * 8 * n_em),
        Workload("transmission", "transmission", g3, o3, hr, dict(n_b=nb, n_alpha=na, spec_idx=list(range(200))),
                 nb * na * 200),
    ]


def service_times(ctx: M.Context, wl: List[Workload], reps: int = 2) -> Dict[str, float]:
    out = {}
    for w in wl:
        best = math.inf
        for _ in range(reps):
            t0 = time.perf_counter()
            ctx.wait(ctx.submit(w.mode, w.gid, w.oid, w.table, **w.kw))
            best = min(best, time.perf_counter() - t0)
        out[w.kind] = best * 1e3
    return out


MIX = (("albedo", 0.50), ("emission", 0.35), ("transmission", 0.15))


def calibrate(ctx: M.Context, rate: float, load: float, precision: int = M.MCRT_MIXED, scale: float = 0.0):
    """Scale packets so that rate * E[service time alone] = load (scale > 0:
    use that packet scale and only measure the service times)."""
    res = upload_inputs(ctx)
    if scale > 0.0:
        wl = build_workloads(res, scale, precision)
        return wl, service_times(ctx, wl), scale
    scale = 1.0
    for _ in range(3):
        wl = build_workloads(res, scale, precision)
        st = service_times(ctx, wl)
        mean_s = sum(p * st[k] for k, p in MIX) / 1e3
        target = load / rate
        new = scale * target / mean_s
        if abs(new / scale - 1.0) < 0.15:
            return wl, st, scale
        scale = new
    wl = build_workloads(res, scale, precision)
    return wl, service_times(ctx, wl), scale


def run_poisson(ctx: M.Context, rate: float = 20.0, duration: float = 60.0, load: float = 0.7, seed: int = 211015645,
                precision: int = M.MCRT_MIXED, workers: int = 3, log=print, rerun_alone: int = 8,
                scale: float = 0.0) -> ServeReport:
    """Poisson arrivals of the mix for `duration` seconds; each request has its
    own transport seed.  Afterwards `rerun_alone` requests of each kind
    (seeded choice) are run again with nothing else on the device and their
    sums compared with the ones they got in the mix."""
    ctx.serve_config(workers)
    wl, st, scale = calibrate(ctx, rate, load, precision, scale)
    by_kind = {w.kind: w for w in wl}
    rng = np.random.Generator(np.random.PCG64(seed))
    t_arr = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        t_arr.append(t)
    kinds = rng.choice([k for k, _ in MIX], size=len(t_arr), p=[p for _, p in MIX])
    rep = ServeReport(rate, duration, len(t_arr), load, scale, service_ms=st)
    pending = {}
    sums = {}
    t0 = time.perf_counter()
    nxt = 0
    last_log = t0
    while nxt < len(t_arr) or pending:
        now = time.perf_counter() - t0
        while nxt < len(t_arr) and t_arr[nxt] <= now:
            w = by_kind[kinds[nxt]]
            tk = ctx.submit(w.mode, w.gid, w.oid, w.table, **{**w.kw, "seed": seed + 1 + nxt})
            pending[tk] = (w, nxt, time.perf_counter() - t0)
            nxt += 1
        done = [tk for tk in pending if ctx.poll(tk)]
        for tk in done:
            w, q, t_sub = pending.pop(tk)
            r = ctx.wait(tk)
            rep.latencies_ms.append(r["latency_ms"])
            rep.kinds.append(w.kind)
            rep.spans.append((t_sub + r["queued_ms"] * 1e-3, t_sub + r["latency_ms"] * 1e-3))
            sums[q] = r["sums"]
            if w.kind == "transmission":
                rep.chord_wavelengths += w.packets
            else:
                rep.packets += w.packets
        if time.perf_counter() - last_log > 10.0:
            last_log = time.perf_counter()
            log(f"[serve] t={now:.0f}s submitted {nxt}/{len(t_arr)} in flight {len(pending)}")
        if not done:
            wait_for = (t_arr[nxt] - (time.perf_counter() - t0)) if nxt < len(t_arr) else 0.002
            time.sleep(min(max(wait_for, 0.0), 0.002))
    rep.wall = time.perf_counter() - t0
    if rerun_alone > 0:
        pick = np.random.Generator(np.random.PCG64(seed + 7))
        same, worst, n = 0, 0.0, 0
        for k, _ in MIX:
            idx = [q for q in range(len(t_arr)) if kinds[q] == k and q in sums]
            for q in pick.choice(idx, size=min(rerun_alone, len(idx)), replace=False):
                w = by_kind[k]
                a = ctx.wait(ctx.submit(w.mode, w.gid, w.oid, w.table, **{**w.kw, "seed": seed + 1 + int(q)}))
                d = np.abs(a["sums"] - sums[q]) / np.maximum(np.abs(sums[q]), 1e-300)
                worst = max(worst, float(d.max()))
                same += int(np.array_equal(a["sums"], sums[q]))
                n += 1
        rep.alone = {"requests": n, "identical": same, "max_rel_diff": worst}
    return rep
