"""Python binding of libmcrt.so (ctypes; argument marshalling only).

Every step of the transport runs in the library's HIP kernels.  The binding
fails loudly when the library has not been built; there is no fallback.
Names follow include/mcrt.h.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcrt.so")

MCRT_SPHERICAL, MCRT_PLANE_PARALLEL = 0, 1
MCRT_SURVIVAL, MCRT_CONTINUOUS = 0, 1
MCRT_FP64, MCRT_MIXED = 0, 1
MCRT_OPAC_CK, MCRT_OPAC_HIRES = 0, 1
NCOUNTERS = 11
COUNTER_NAMES = ["escaped", "surface", "absorbed", "roulette", "capped", "lost",
                 "n_interactions", "n_crossings", "n_capped", "n_lost", "w0"]
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOTFOUND", -5: "EBUDGET",
          -6: "EBUSY", -7: "ECANCELLED"}

MODES = {"albedo": 0, "emission": 1, "transmission": 2}


class McrtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


_vp, _i32, _u64, _i64, _dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double


class GridDesc(ctypes.Structure):
    _fields_ = [("geometry", _i32), ("nlon", _i32), ("nlat", _i32), ("nlay", _i32),
                ("r_edges", _vp), ("lat_edges", _vp), ("lon_edges", _vp),
                ("T", _vp), ("P", _vp), ("rho", _vp), ("u", _vp), ("v", _vp), ("w", _vp),
                ("cld_ksca", _vp), ("cld_kabs", _vp), ("cld_g", _vp), ("omega_rot", _dbl),
                ("flags", _i32)]


MCRT_BORROW_DEVICE = 1


class OpacityDesc(ctypes.Structure):
    _fields_ = [("kind", _i32), ("nspec", _i32), ("ng", _i32), ("nT", _i32), ("nP", _i32),
                ("lam_um", _vp), ("lam_min_um", _dbl), ("dlnlam", _dbl), ("g_weights", _vp),
                ("T_grid", _vp), ("P_grid", _vp), ("kappa", _vp), ("k_ray", _vp)]


class SolveParams(ctypes.Structure):
    _fields_ = [("seed", _u64), ("n_packets", _u64), ("decorrelate", _i32), ("precision", _i32),
                ("n_spec", _i32), ("spec_idx", _vp), ("n_obs", _i32), ("obs_phase", _vp),
                ("obs_dir", _vp), ("scattering", _i32), ("absorption", _i32),
                ("rr_threshold", _dbl), ("rr_survive", _dbl), ("emis_bias", _dbl),
                ("tau_vert_max", _dbl), ("tau_peel_max", _dbl), ("max_events", _i64), ("mu0", _dbl),
                ("n_b", _i32), ("n_alpha", _i32), ("r_star", _dbl), ("stream", _vp),
                ("packet_dump", _vp), ("profile", _i32), ("max_batch", _i32),
                ("tune_ev_threshold", _i32), ("tune_blocks_per_cu", _i32), ("tune_wave_batch", _i32),
                ("graph", _i32), ("contrib", _i32), ("image_npix", _i32),
                ("g_sampling", _i32), ("cloud_phase", _i32),
                ("surface_albedo", ctypes.c_double), ("ms_transmission", _i32), ("ld_law", _i32),
                ("a_orbit", ctypes.c_double), ("ld_c1", ctypes.c_double), ("ld_c2", ctypes.c_double),
                ("transit_y", ctypes.c_double), ("transit_z", ctypes.c_double),
                ("draine_alpha", ctypes.c_double), ("forced", _i32), ("forced_first", _i32)]


class BatchItem(ctypes.Structure):
    _fields_ = [("mode", _i32), ("grid_id", _i32), ("opac_id", _i32), ("n_spec", _i32), ("spec_idx", _vp),
                ("n_packets", _u64)]


class Result(ctypes.Structure):
    _fields_ = [("value", _vp), ("stderr_", _vp), ("per_g", _vp), ("sums", _vp),
                ("counters", _vp), ("l_tot", _vp), ("elapsed_ms", _dbl), ("kernel_ms", _dbl),
                ("kernel_launches", _i64), ("queued_ms", _dbl), ("latency_ms", _dbl), ("cf", _vp),
                ("image", _vp), ("n_segments", _i64)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libmcrt.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    L.mcrt_create.argtypes = [ctypes.c_int, _u64, ctypes.POINTER(_vp)]
    L.mcrt_destroy.argtypes = [_vp]
    L.mcrt_destroy.restype = None
    L.mcrt_last_error.restype = ctypes.c_char_p
    L.mcrt_memory_in_use.argtypes = [_vp]
    L.mcrt_memory_in_use.restype = _u64
    L.mcrt_grid_upload.argtypes = [_vp, ctypes.POINTER(GridDesc), _vp, ctypes.POINTER(_i32)]
    L.mcrt_grid_free.argtypes = [_vp, _i32]
    L.mcrt_opacity_upload.argtypes = [_vp, ctypes.POINTER(OpacityDesc), _vp, ctypes.POINTER(_i32)]
    L.mcrt_opacity_free.argtypes = [_vp, _i32]
    L.mcrt_default_params.argtypes = [ctypes.POINTER(SolveParams)]
    L.mcrt_default_params.restype = None
    for nm in ("mcrt_solve_albedo", "mcrt_solve_emission", "mcrt_solve_transmission"):
        getattr(L, nm).argtypes = [_vp, _i32, _i32, ctypes.POINTER(SolveParams), ctypes.POINTER(Result)]
    L.mcrt_solve_noalloc.argtypes = [_vp, _i32, _i32, _i32, ctypes.POINTER(SolveParams), ctypes.POINTER(Result)]
    L.mcrt_solve_batch.argtypes = [_vp, _i32, ctypes.POINTER(BatchItem), ctypes.POINTER(SolveParams),
                                   ctypes.POINTER(Result)]
    L.mcrt_autotune.argtypes = [_vp, _i32, _i32, _i32, ctypes.POINTER(SolveParams), ctypes.POINTER(_dbl)]
    L.mcrt_serve_config.argtypes = [_vp, _i32]
    L.mcrt_submit.argtypes = [_vp, _i32, _i32, _i32, ctypes.POINTER(SolveParams), ctypes.POINTER(_u64)]
    L.mcrt_poll.argtypes = [_vp, _u64, ctypes.POINTER(_i32)]
    L.mcrt_wait.argtypes = [_vp, _u64, ctypes.POINTER(Result)]
    L.mcrt_cancel.argtypes = [_vp, _u64]
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise McrtError(rc, load().mcrt_last_error().decode())


def _arr(a, dtype):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data


def default_params() -> SolveParams:
    p = SolveParams()
    load().mcrt_default_params(ctypes.byref(p))
    return p


class Context:
    """A library context on one HIP device (owns resident grids and tables)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        L = load()
        h = _vp()
        _check(L.mcrt_create(device, hbm_budget_bytes, ctypes.byref(h)))
        self._h = h
        self.device = device
        self._keep = []
        self._ncell = {}
        self._borrowed = {}  # grid id -> device tensors the library reads in place

    def close(self):
        if getattr(self, "_h", None):
            load().mcrt_destroy(self._h)
            self._h = None
        self._borrowed = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def memory_in_use(self) -> int:
        return int(load().mcrt_memory_in_use(self._h))

    # ---------------------------------------------------------- uploads
    def upload_grid(self, g, borrow: bool = False, stream=None) -> int:
        """g: paper_2110_15640_amd.inputs.Grid (host numpy arrays).  borrow:
        the per-cell arrays are first placed in torch device tensors, which
        the library reads in place (MCRT_BORROW_DEVICE); this context keeps
        them alive until free_grid.  stream: a torch stream (or a raw
        hipStream_t) to upload on; with borrow it defaults to torch's current
        stream, so the library checks the tensors after the copies that
        filled them."""
        arrs = dict(r=_arr(g.r_edges, np.float64), lat=_arr(g.lat_edges, np.float64),
                    lon=_arr(g.lon_edges, np.float64), T=_arr(g.T, np.float32),
                    P=_arr(g.P, np.float32), rho=_arr(g.rho, np.float64),
                    u=_arr(g.u, np.float32), v=_arr(g.v, np.float32), w=_arr(g.w, np.float32),
                    cs=_arr(g.cld_ksca, np.float32), ca=_arr(g.cld_kabs, np.float32),
                    cg=_arr(g.cld_g, np.float32))
        cell = dict(arrs)
        held = None
        if borrow:
            import torch
            dev = torch.device("cuda", self.device)
            held = {k: torch.from_numpy(v).to(dev, non_blocking=False) for k, v in arrs.items()
                    if v is not None and k not in ("r", "lat", "lon")}
            if stream is None:
                stream = torch.cuda.current_stream(dev)
            cell.update(held)

        def ptr(k):
            v = cell[k]
            return None if v is None else (v.data_ptr() if hasattr(v, "data_ptr") else _ptr(v))

        d = GridDesc(g.geometry, g.nlon, g.nlat, g.nlay, _ptr(arrs["r"]), _ptr(arrs["lat"]),
                     _ptr(arrs["lon"]), ptr("T"), ptr("P"), ptr("rho"), ptr("u"), ptr("v"), ptr("w"),
                     ptr("cs"), ptr("ca"), ptr("cg"), float(g.omega_rot), MCRT_BORROW_DEVICE if borrow else 0)
        gid = _i32()
        st = None if stream is None else getattr(stream, "cuda_stream", stream)
        _check(load().mcrt_grid_upload(self._h, ctypes.byref(d), st, ctypes.byref(gid)))
        self._ncell[gid.value] = g.nlon * g.nlat * g.nlay
        if held is not None:
            self._borrowed[gid.value] = held
        return gid.value

    def upload_opacity(self, t, stream=None) -> int:
        """t: inputs.CKTable or inputs.HiresTable; stream as for upload_grid."""
        hires = not hasattr(t, "g_weights")
        kap = _arr(t.kappa, np.float32)
        Tg, Pg, kr = _arr(t.T_grid, np.float64), _arr(t.P_grid, np.float64), _arr(t.k_ray, np.float64)
        if hires:
            d = OpacityDesc(MCRT_OPAC_HIRES, t.nlam, 1, len(Tg), len(Pg), None, float(t.lam_min_um),
                            float(t.dlnlam), None, _ptr(Tg), _ptr(Pg), _ptr(kap), _ptr(kr))
        else:
            lam, gw = _arr(t.lam_um, np.float64), _arr(t.g_weights, np.float64)
            d = OpacityDesc(MCRT_OPAC_CK, t.nband, t.ng, len(Tg), len(Pg), _ptr(lam), 0.0, 0.0, _ptr(gw),
                            _ptr(Tg), _ptr(Pg), _ptr(kap), _ptr(kr))
        oid = _i32()
        st = None if stream is None else getattr(stream, "cuda_stream", stream)
        _check(load().mcrt_opacity_upload(self._h, ctypes.byref(d), st, ctypes.byref(oid)))
        return oid.value

    def free_grid(self, gid: int):
        _check(load().mcrt_grid_free(self._h, gid))
        self._borrowed.pop(gid, None)

    def free_opacity(self, oid: int):
        _check(load().mcrt_opacity_free(self._h, oid))

    # ---------------------------------------------------------- solves
    def _params(self, kw):
        p = default_params()
        keep = []
        spec_idx = kw.pop("spec_idx", None)
        if spec_idx is not None:
            a = _arr(spec_idx, np.int32)
            keep.append(a)
            p.n_spec, p.spec_idx = len(a), a.ctypes.data
        obs_phase = kw.pop("obs_phase", None)
        obs_dir = kw.pop("obs_dir", None)
        if obs_dir is not None:
            a = _arr(obs_dir, np.float64).reshape(-1, 3)
            keep.append(a)
            p.n_obs, p.obs_dir = len(a), a.ctypes.data
        elif obs_phase is not None:
            a = _arr(obs_phase, np.float64).reshape(-1)
            keep.append(a)
            p.n_obs, p.obs_phase = len(a), a.ctypes.data
        stream = kw.pop("stream", None)
        if stream is not None:
            p.stream = getattr(stream, "cuda_stream", stream)
        dump = kw.pop("packet_dump", None)
        if dump is not None:
            p.packet_dump = dump.data_ptr() if hasattr(dump, "data_ptr") else int(dump)
        for k, v in kw.items():
            if not hasattr(p, k):
                raise TypeError(f"unknown solve parameter {k!r}")
            setattr(p, k, v)
        return p, keep

    def _solve(self, fn, gid, oid, n_spec, n_out, ng, kw):
        p, keep = self._params(dict(kw))
        ns = p.n_spec if p.spec_idx else n_spec
        no = n_out(p)
        out = self._alloc(ns, ng, no)
        if p.contrib:
            out["cf"] = np.zeros((ns, no, 2, self._ncell.get(gid, 0)))
        if p.image_npix > 0:
            out["image"] = np.zeros((ns, no, p.image_npix, p.image_npix))
        r = self._result(out)
        _check(fn(self._h, gid, oid, ctypes.byref(p), ctypes.byref(r)))
        self._finish(out, r)
        del keep
        return out

    @staticmethod
    def _shapes(table, mode, p):
        ck = hasattr(table, "g_weights")
        ns_tab = table.nband if ck else table.nlam
        ns = p.n_spec if p.spec_idx else ns_tab
        ng = table.ng if ck else 1
        no = 1 if mode == "transmission" else max(p.n_obs, 1)
        return ns, ng, no

    @staticmethod
    def _alloc(ns, ng, no):
        return dict(value=np.zeros((ns, no)), stderr=np.zeros((ns, no)), per_g=np.zeros((ns, ng, no)),
                    sums=np.zeros((ns, ng, no, 2)), counters=np.zeros((ns, ng, NCOUNTERS)),
                    l_tot=np.zeros((ns, ng)))

    @staticmethod
    def _result(out):
        cf, im = out.get("cf"), out.get("image")
        return Result(out["value"].ctypes.data, out["stderr"].ctypes.data, out["per_g"].ctypes.data,
                      out["sums"].ctypes.data, out["counters"].ctypes.data, out["l_tot"].ctypes.data,
                      0.0, 0.0, 0, 0.0, 0.0, None if cf is None else cf.ctypes.data,
                      None if im is None else im.ctypes.data, 0)

    @staticmethod
    def _finish(out, r):
        out["elapsed_ms"] = r.elapsed_ms
        out["kernel_ms"] = r.kernel_ms
        out["kernel_launches"] = r.kernel_launches
        out["queued_ms"] = r.queued_ms
        out["latency_ms"] = r.latency_ms
        out["n_segments"] = r.n_segments

    def solve_batch(self, items, **kw):
        """items: list of dicts (mode, gid, oid, table, spec_idx, n_packets);
        kw: common parameters.  Returns one result dict per item."""
        p, keep = self._params(dict(kw))
        arr = (BatchItem * len(items))()
        outs, res = [], (Result * len(items))()
        for q, it in enumerate(items):
            t = it["table"]
            spec = it.get("spec_idx")
            sa = None if spec is None else _arr(spec, np.int32)
            keep.append(sa)
            ns = len(sa) if sa is not None else t.nband
            arr[q] = BatchItem(MODES[it["mode"]], it["gid"], it["oid"], 0 if sa is None else len(sa),
                               None if sa is None else sa.ctypes.data, int(it["n_packets"]))
            out = self._alloc(ns, t.ng, max(p.n_obs, 1))
            outs.append(out)
            res[q] = self._result(out)
        _check(load().mcrt_solve_batch(self._h, len(items), arr, ctypes.byref(p), res))
        for q in range(len(items)):
            self._finish(outs[q], res[q])
        del keep
        return outs

    def autotune(self, mode: str, gid: int, oid: int, **kw) -> dict:
        """Pick the persistent launch shape for this request; returns the
        tune_* settings (pass them to the solve) and the trial rate."""
        p, keep = self._params(dict(kw))
        rate = _dbl()
        _check(load().mcrt_autotune(self._h, MODES[mode], gid, oid, ctypes.byref(p), ctypes.byref(rate)))
        del keep
        return dict(tune_ev_threshold=p.tune_ev_threshold, tune_blocks_per_cu=p.tune_blocks_per_cu,
                    tune_wave_batch=p.tune_wave_batch, trial_packets_per_s=rate.value)

    # ---------------------------------------------------------- serving
    def serve_config(self, n_workers: int):
        _check(load().mcrt_serve_config(self._h, n_workers))

    def submit(self, mode: str, gid: int, oid: int, table, **kw) -> int:
        """Queue a solve; returns a ticket.  The result shape is kept with it."""
        p, keep = self._params(dict(kw))
        t = _u64()
        _check(load().mcrt_submit(self._h, MODES[mode], gid, oid, ctypes.byref(p), ctypes.byref(t)))
        self._pending = getattr(self, "_pending", {})
        self._pending[t.value] = self._shapes(table, mode, p)
        return t.value

    def poll(self, ticket: int) -> bool:
        d = _i32()
        _check(load().mcrt_poll(self._h, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int) -> dict:
        ns, ng, no = self._pending.pop(ticket)
        out = self._alloc(ns, ng, no)
        r = self._result(out)
        _check(load().mcrt_wait(self._h, ticket, ctypes.byref(r)))
        self._finish(out, r)
        return out

    def cancel(self, ticket: int):
        _check(load().mcrt_cancel(self._h, ticket))

    def solve_albedo(self, gid, oid, table, **kw):
        return self._solve(load().mcrt_solve_albedo, gid, oid, table.nband,
                           lambda p: max(p.n_obs, 1), table.ng, kw)

    def solve_emission(self, gid, oid, table, **kw):
        ns = table.nband if hasattr(table, "g_weights") else table.nlam
        ng = table.ng if hasattr(table, "g_weights") else 1
        return self._solve(load().mcrt_solve_emission, gid, oid, ns, lambda p: p.n_obs, ng, kw)

    def solve_noalloc(self, mode: str, gid, oid, table, **kw):
        """mcrt_solve_noalloc: an albedo or emission solve whose scratch is the
        library's fixed per-device array (no device allocation in the call)."""
        m = MODES[mode]
        if mode == "albedo":
            return self._solve(lambda h, g, o, p, r: load().mcrt_solve_noalloc(h, m, g, o, p, r), gid, oid,
                               table.nband, lambda p: max(p.n_obs, 1), table.ng, kw)
        ns = table.nband if hasattr(table, "g_weights") else table.nlam
        ng = table.ng if hasattr(table, "g_weights") else 1
        return self._solve(lambda h, g, o, p, r: load().mcrt_solve_noalloc(h, m, g, o, p, r), gid, oid, ns,
                           lambda p: p.n_obs, ng, kw)

    def solve_transmission(self, gid, oid, table, **kw):
        ns = table.nband if hasattr(table, "g_weights") else table.nlam
        ng = table.ng if hasattr(table, "g_weights") else 1
        return self._solve(load().mcrt_solve_transmission, gid, oid, ns, lambda p: 1, ng, kw)
