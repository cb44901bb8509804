"""Python driver of the FP64 CPU oracle (mcrt_oracle.c).

TEST INFRASTRUCTURE ONLY: used by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports this module.

The solve drivers below follow the paper's observables (Sect. 5):
* albedo: the escaping fraction toward the observer per unit incident flux,
  times pi (geometric albedo at zero phase, the A_g equation);
* emission: L_p = (L_tot/N) sum_n F_n, I_p = L_p / (pi R_TOA^2), F_p = pi I_p;
* transmission: <I> = (R_TOA - R0)/N sum (1 - e^-tau) b and
  (R_p/R_star)^2 = (R0^2 + 2 <I>)/R_star^2;
band values are sum_g w_g X_g over fixed-g solves.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcrt_oracle.c")
_LIB = os.path.join(_HERE, "libmcrt_oracle.so")

NK = 11
K_NAMES = ["escaped", "surface", "absorbed", "roulette", "capped", "lost",
           "n_interactions", "n_crossings", "n_capped", "n_lost", "w0"]


def build(force: bool = False) -> str:
    """Compile the oracle (plain FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("geom", ctypes.c_int64), ("nlon", ctypes.c_int64), ("nlat", ctypes.c_int64),
                ("nlay", ctypes.c_int64), ("r", ctypes.c_void_p), ("lat", ctypes.c_void_p),
                ("lon", ctypes.c_void_p)]


class _Params(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_packets", ctypes.c_uint64),
                ("packet0", ctypes.c_uint64), ("mode", ctypes.c_int64),
                ("scattering", ctypes.c_int64), ("absorption", ctypes.c_int64),
                ("tag", ctypes.c_int64), ("max_events", ctypes.c_int64),
                ("max_cross", ctypes.c_int64), ("n_obs", ctypes.c_int64),
                ("rr_threshold", ctypes.c_double), ("rr_survive", ctypes.c_double),
                ("tau_peel_max", ctypes.c_double), ("mu0", ctypes.c_double),
                ("cloud_phase", ctypes.c_int64), ("surface_albedo", ctypes.c_double),
                ("omega_star", ctypes.c_double), ("ld_law", ctypes.c_int64), ("ld_c1", ctypes.c_double),
                ("ld_c2", ctypes.c_double), ("transit_y", ctypes.c_double), ("transit_z", ctypes.c_double),
                ("r_star", ctypes.c_double), ("draine_alpha", ctypes.c_double),
                ("forced", ctypes.c_int64), ("forced_first", ctypes.c_int64)]


class _Optics(ctypes.Structure):
    _fields_ = [("a_ext", ctypes.c_void_p), ("a_abs", ctypes.c_void_p), ("omega", ctypes.c_void_p),
                ("p_gas", ctypes.c_void_p), ("g_cld", ctypes.c_void_p)]


class _Tally(ctypes.Structure):
    _fields_ = [("cf", ctypes.c_void_p), ("img", ctypes.c_void_p), ("npix", ctypes.c_int64),
                ("half", ctypes.c_double), ("axes", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        vp, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_u01.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.orc_u01.restype = dbl
        L.orc_draw_pair.argtypes = [u64, ctypes.c_uint32, u64, ctypes.c_uint32, ctypes.c_uint32, vp]
        for nm in ("orc_phase_rayleigh",):
            getattr(L, nm).argtypes = [dbl]
            getattr(L, nm).restype = dbl
        L.orc_phase_hg.argtypes = [dbl, dbl]
        L.orc_phase_hg.restype = dbl
        L.orc_sample_rayleigh.argtypes = [dbl]
        L.orc_sample_rayleigh.restype = dbl
        L.orc_sample_hg.argtypes = [dbl, dbl]
        L.orc_sample_hg.restype = dbl
        L.orc_phase_tthg.argtypes = [dbl, dbl]
        L.orc_phase_tthg.restype = dbl
        L.orc_sample_tthg.argtypes = [dbl, dbl, dbl]
        L.orc_sample_tthg.restype = dbl
        L.orc_rotate.argtypes = [vp, dbl, dbl]
        L.orc_planck.argtypes = [dbl, dbl]
        L.orc_planck.restype = dbl
        L.orc_trace_segments.argtypes = [ctypes.POINTER(_Grid), vp, vp, i64, i64, i64, i64, i64, vp, vp, vp]
        L.orc_trace_segments.restype = i64
        L.orc_ck_optics.argtypes = [i64, vp, vp, vp, vp, vp, vp, i64, i64, vp, vp, vp, dbl,
                                    vp, vp, vp, vp, vp]
        L.orc_doppler_shift.argtypes = [ctypes.POINTER(_Grid), vp, vp, vp, dbl, vp, dbl, vp]
        L.orc_hires_optics.argtypes = [i64, vp, vp, vp, vp, i64, i64, i64, vp, vp, vp, i64, dbl,
                                       vp, vp, vp, vp, vp]
        L.orc_emission_sources.argtypes = [ctypes.POINTER(_Grid), vp, vp, vp, dbl, dbl, dbl,
                                           vp, vp, vp, vp]
        L.orc_emission_sources.restype = dbl
        L.orc_transport.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Optics),
                                    ctypes.POINTER(_Params), vp, vp, vp, dbl, vp, vp,
                                    ctypes.POINTER(_Tally), i64]
        L.orc_transport.restype = i64
        L.orc_transport_gsampled.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Optics), i64,
                                             ctypes.POINTER(_Params), vp, vp, vp, vp, vp, dbl, vp, vp, vp, i64]
        L.orc_transport_gsampled.restype = i64
        L.orc_transmission.argtypes = [ctypes.POINTER(_Grid), vp, i64, i64, i64, u64, i64, dbl, dbl,
                                       ctypes.POINTER(_Params), vp, vp, i64]
        L.orc_draine_mean_cosine.argtypes = [dbl, dbl]
        L.orc_draine_mean_cosine.restype = dbl
        L.orc_draine_G.argtypes = [dbl, dbl]
        L.orc_draine_G.restype = dbl
        L.orc_phase_draine.argtypes = [dbl, dbl, dbl]
        L.orc_phase_draine.restype = dbl
        L.orc_sample_draine.argtypes = [vp, vp, ctypes.c_int, dbl, dbl]
        L.orc_sample_draine.restype = dbl
        L.orc_forced_tau.argtypes = [i64, dbl, dbl, dbl, vp]
        L.orc_forced_tau.restype = dbl
        L.orc_limb_darkening.argtypes = [i64, dbl, dbl, dbl]
        L.orc_limb_darkening.restype = dbl
        L.orc_chord_limb_weight.argtypes = [i64, dbl, dbl, dbl, dbl, dbl, dbl, dbl]
        L.orc_chord_limb_weight.restype = dbl
        L.orc_max_threads.restype = i64
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


# ---------------------------------------------------------------- primitives
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def u01(a: int, b: int) -> float:
    return lib().orc_u01(a, b)


def draw_pair(seed, tag, packet, event, block):
    out = np.zeros(2)
    lib().orc_draw_pair(seed, tag, packet, event, block, out.ctypes.data)
    return out


def sample_rayleigh(z):
    return lib().orc_sample_rayleigh(float(z))


def sample_hg(z, g):
    return lib().orc_sample_hg(float(z), float(g))


def phase_rayleigh(mu):
    return lib().orc_phase_rayleigh(float(mu))


def phase_hg(mu, g):
    return lib().orc_phase_hg(float(mu), float(g))


def phase_tthg(mu, g):
    return lib().orc_phase_tthg(float(mu), float(g))


def sample_tthg(z_lobe, z, g):
    return lib().orc_sample_tthg(float(z_lobe), float(z), float(g))


def draine_G(g, alpha):
    return lib().orc_draine_G(float(g), float(alpha))


def draine_mean_cosine(G, alpha):
    return lib().orc_draine_mean_cosine(float(G), float(alpha))


def phase_draine(mu, G, alpha):
    return lib().orc_phase_draine(float(mu), float(G), float(alpha))


def sample_draine(za, zacc, G, alpha):
    a, b = _f64(za), _f64(zacc)
    return lib().orc_sample_draine(a.ctypes.data, b.ctypes.data, len(a), float(G), float(alpha))


def forced_tau(kind, tp, zeta, zc):
    """(tau, weight factor) of a forced flight over a path of depth tp."""
    w = np.zeros(1)
    t = lib().orc_forced_tau(int(kind), float(tp), float(zeta), float(zc), w.ctypes.data)
    return t, float(w[0])


def rotate(d, mu, psi):
    v = np.ascontiguousarray(d, dtype=np.float64).copy()
    lib().orc_rotate(v.ctypes.data, float(mu), float(psi))
    return v


def planck(lam_cm, T):
    return lib().orc_planck(float(lam_cm), float(T))


class GridView:
    """Keeps the numpy arrays alive behind the C grid struct."""

    def __init__(self, grid):
        self.grid = grid
        self.r = _f64(grid.r_edges)
        self.lat = _f64(grid.lat_edges)
        self.lon = _f64(grid.lon_edges)
        self.c = _Grid(grid.geometry, grid.nlon, grid.nlat, grid.nlay, self.r.ctypes.data,
                       self.lat.ctypes.data, self.lon.ctypes.data)

    @property
    def max_cross(self):
        g = self.grid
        return 4 * (g.nlay + g.nlat + g.nlon) + 16


def trace_segments(grid, p, d, i, j, k, ef=-1, cap=100000):
    gv = GridView(grid)
    p = _f64(p)
    d = _f64(d)
    cells = np.zeros(cap, dtype=np.int64)
    lens = np.zeros(cap)
    term = np.zeros(1, dtype=np.int64)
    n = lib().orc_trace_segments(ctypes.byref(gv.c), p.ctypes.data, d.ctypes.data, i, j, k, ef,
                                 cap, cells.ctypes.data, lens.ctypes.data, term.ctypes.data)
    return cells[:n], lens[:n], int(term[0])


@dataclass
class Optics:
    a_ext: np.ndarray
    a_abs: np.ndarray
    omega: np.ndarray
    p_gas: np.ndarray
    g_cld: np.ndarray


def ck_optics(grid, table, band: int, g: int) -> Optics:
    n = grid.ncell
    out = [np.zeros(n) for _ in range(5)]
    T, P, rho = _f32(grid.T), _f32(grid.P), _f64(grid.rho)
    cs, ca, cg = _f32(grid.cld_ksca), _f32(grid.cld_kabs), _f32(grid.cld_g)
    Tg, Pg = _f64(table.T_grid), _f64(table.P_grid)
    tab = np.ascontiguousarray(table.kappa[band, g], dtype=np.float32)
    lib().orc_ck_optics(n, _p(T), _p(P), _p(rho), _p(cs), _p(ca), _p(cg), len(Tg), len(Pg),
                        _p(Tg), _p(Pg), _p(tab), float(table.k_ray[band]), *[o.ctypes.data for o in out])
    return Optics(*out)


def doppler_shift(grid, obs_dir, dlnlam) -> np.ndarray:
    gv = GridView(grid)
    o = _f64(obs_dir)
    out = np.zeros(grid.ncell)
    u, v, w = _f32(grid.u), _f32(grid.v), _f32(grid.w)
    lib().orc_doppler_shift(ctypes.byref(gv.c), _p(u), _p(v), _p(w), float(grid.omega_rot),
                            o.ctypes.data, float(dlnlam), out.ctypes.data)
    return out


def hires_optics(grid, table, n: int, shift: Optional[np.ndarray]) -> Optics:
    nc = grid.ncell
    out = [np.zeros(nc) for _ in range(5)]
    T, P, rho = _f32(grid.T), _f32(grid.P), _f64(grid.rho)
    Tg, Pg = _f64(table.T_grid), _f64(table.P_grid)
    tab = np.ascontiguousarray(table.kappa, dtype=np.float32)
    sh = _f64(shift)
    lib().orc_hires_optics(nc, _p(T), _p(P), _p(rho), _p(sh), table.nlam, len(Tg), len(Pg),
                           _p(Tg), _p(Pg), _p(tab), int(n), float(table.k_ray[n]),
                           *[o.ctypes.data for o in out])
    return Optics(*out)


@dataclass
class Sources:
    L: np.ndarray
    cdf: np.ndarray
    wbirth: np.ndarray
    L_tot: float
    n_emit: int


def emission_sources(grid, optics: Optics, lam_um: float, tau_vert: float, xi: float) -> Sources:
    gv = GridView(grid)
    n = grid.ncell
    L, cdf, wb = np.zeros(n), np.zeros(n), np.zeros(n)
    info = np.zeros(1, dtype=np.int64)
    T = _f32(grid.T)
    Ltot = lib().orc_emission_sources(ctypes.byref(gv.c), T.ctypes.data, optics.a_ext.ctypes.data,
                                      optics.a_abs.ctypes.data, float(lam_um) * 1e-4, float(tau_vert),
                                      float(xi), L.ctypes.data, cdf.ctypes.data, wb.ctypes.data,
                                      info.ctypes.data)
    return Sources(L, cdf, wb, Ltot, int(info[0]))


@dataclass
class Params:
    seed: int = 12345
    n_packets: int = 1000
    packet0: int = 0
    scattering: bool = True
    absorption: int = 0  # 0 survival, 1 continuous
    decorrelate: bool = False
    max_events: int = 1_000_000
    rr_threshold: float = 1e-3
    rr_survive: float = 0.1
    tau_peel_max: float = 50.0
    mu0: float = 0.0
    emis_bias: float = 0.5
    tau_vert_max: float = 30.0
    obs_phase: Sequence[float] = (0.0,)
    obs_dir: Optional[np.ndarray] = None
    n_b: int = 256
    n_alpha: int = 360
    r_star: float = 6.957e10
    g_sampling: int = 0  # 0 fixed-g solves; per-packet g: 1 unbiased, 2 uniform, 3 composite
    cloud_phase: int = 0  # 0 Henyey-Greenstein, 1 two-term Henyey-Greenstein, 2 Draine
    draine_alpha: float = 0.5  # alpha of Draine's function
    forced: int = 0  # forced interaction: 0 off, 1 forced scattering, 2 path-length stretching, 3 hybrid
    forced_first: int = 0  # 1: only the first flight of a packet is forced
    surface_albedo: float = 0.0  # 0 absorbing lower boundary; > 0 Lambert surface
    a_orbit: float = 0.0  # star-planet distance [cm] (transmission with scattering)
    ld_law: int = 0  # stellar limb darkening: 0 none, 1 linear, 2 quadratic, 3 sqrt, 4 log, 5 exp, 6 power-2
    ld_c1: float = 0.0
    ld_c2: float = 0.0
    transit_y: float = 0.0  # planet centre on the stellar disk (sky plane) [cm]
    transit_z: float = 0.0
    threads: int = 0


def albedo_obs_dirs(phases):
    """Albedo phase angle a: o = (cos a, sin a, 0) (star at +x)."""
    return np.array([[math.cos(a), math.sin(a), 0.0] for a in phases], dtype=np.float64).reshape(-1, 3)


def emission_obs_dirs(phases):
    """Orbital phase phi: o = (cos l, sin l, 0), l = pi (1 - 2 phi); phi = 0.5
    views the dayside (substellar point at lon = 0)."""
    out = []
    for ph in phases:
        lo = math.pi * (1.0 - 2.0 * ph)
        out.append([math.cos(lo), math.sin(lo), 0.0])
    return np.array(out, dtype=np.float64).reshape(-1, 3)


def image_axes(obs) -> np.ndarray:
    """Sky-plane axes per observer o: vertical e_v = the projection of the
    rotation axis z (x if o is along z), horizontal e_h = e_v x o, so that
    (e_h, e_v, o) is right-handed.  Returns [n_obs, 2, 3]."""
    out = []
    for o in np.asarray(obs, dtype=np.float64).reshape(-1, 3):
        ref = np.array([0.0, 0.0, 1.0])
        v = ref - (ref @ o) * o
        if np.linalg.norm(v) < 1e-12:
            ref = np.array([1.0, 0.0, 0.0])
            v = ref - (ref @ o) * o
        v = v / np.linalg.norm(v)
        h = np.cross(v, o)
        out.append([h, v])
    return np.array(out)


def omega_star(params: Params) -> float:
    """Solid angle pi (R*/a)^2 of the stellar beam at the planet (0 without a_orbit)."""
    return math.pi * (params.r_star / params.a_orbit) ** 2 if params.a_orbit > 0.0 else 0.0


def _params(params: Params, mode: int, tag: int, max_cross: int, nobs: int) -> _Params:
    return _Params(params.seed, params.n_packets, params.packet0, mode, int(bool(params.scattering)),
                   int(params.absorption), tag, params.max_events, max_cross, nobs,
                   params.rr_threshold, params.rr_survive, params.tau_peel_max, params.mu0,
                   int(params.cloud_phase), float(params.surface_albedo), omega_star(params),
                   int(params.ld_law), float(params.ld_c1), float(params.ld_c2), float(params.transit_y),
                   float(params.transit_z), float(params.r_star), float(params.draine_alpha),
                   int(params.forced), int(params.forced_first))


def limb_darkening(law: int, c1: float, c2: float, mu: float) -> float:
    return lib().orc_limb_darkening(int(law), float(c1), float(c2), float(mu))


def chord_limb_weight(params: Params, y: float, z: float) -> float:
    return lib().orc_chord_limb_weight(int(params.ld_law), float(params.ld_c1), float(params.ld_c2),
                                       float(params.transit_y), float(params.transit_z), float(params.r_star),
                                       float(y), float(z))


def transport(grid, optics: Optics, params: Params, mode: int, obs: Optional[np.ndarray],
              sources: Optional[Sources] = None, tag: int = 0, cf: Optional[np.ndarray] = None,
              img: Optional[np.ndarray] = None):
    """Run params.n_packets histories; returns per-packet F [n, nout] and
    counters K [n, NK].  cf: optional float64 array [nout, 2, ncell] to which
    every peel-off f is added at the cell of its event, thermal (emission
    point, index 0) or scattered (interaction, index 1).  img: optional
    float64 array [nout, npix, npix] to which f is added at the pixel of the
    event point on the observer's sky plane (image_axes), rows along e_v and
    columns along e_h, covering [-R_TOA, R_TOA]^2."""
    gv = GridView(grid)
    nobs = 0 if obs is None else len(obs)
    pr = _params(params, mode, tag, gv.max_cross, nobs)
    op = _Optics(optics.a_ext.ctypes.data, optics.a_abs.ctypes.data, optics.omega.ctypes.data,
                 optics.p_gas.ctypes.data, optics.g_cld.ctypes.data)
    nout = 1 if (grid.geometry == 1 and nobs == 0) else nobs
    F = np.zeros((params.n_packets, max(nout, 1)))
    K = np.zeros((params.n_packets, NK))
    o = None if obs is None else _f64(obs)
    cdf = None if sources is None else sources.cdf
    wb = None if sources is None else sources.wbirth
    tl = None
    axes = None
    if cf is not None or img is not None:
        npix = 0
        if cf is not None:
            assert cf.dtype == np.float64 and cf.flags.c_contiguous and cf.shape == (max(nout, 1), 2, grid.ncell)
        if img is not None:
            assert grid.geometry == 0 and obs is not None
            npix = img.shape[1]
            assert img.dtype == np.float64 and img.flags.c_contiguous and img.shape == (nout, npix, npix)
            axes = np.ascontiguousarray(image_axes(obs))
        tl = _Tally(_p(cf), _p(img), npix, float(grid.r_toa), _p(axes))
    lib().orc_transport(ctypes.byref(gv.c), ctypes.byref(op), ctypes.byref(pr), _p(o), _p(cdf), _p(wb),
                        float(grid.r_toa), F.ctypes.data, K.ctypes.data,
                        None if tl is None else ctypes.byref(tl), int(params.threads))
    return F[:, :nout], K


def g_sampling_weights(scheme: int, w, L=None):
    """Sampling weights q(g) (unnormalised) and weight factors p(g)/q(g) of
    per-packet g-ordinate sampling (Sect. "G-ordinance biasing"): p(g) = w_g
    (albedo) or w_g L_g / sum(w L) (emission); scheme 1 samples p itself
    (factor 1), 2 the uniform q = 1/N_g (factor N_g p), 3 the composite
    q = (p + 1/N_g) / 2."""
    w = np.asarray(w, dtype=np.float64)
    ng = len(w)
    raw = w if L is None else w * np.asarray(L, dtype=np.float64)
    tot = float(raw.sum())
    p = raw / tot if tot > 0 else np.zeros(ng)
    if scheme == 1:
        return raw.copy(), np.ones(ng)
    if scheme == 2:
        return np.ones(ng), p * ng
    if scheme == 3:
        q = 0.5 * p + 0.5 / ng
        return q, p / q
    raise ValueError(f"unknown g-sampling scheme {scheme}")


def transport_gsampled(grid, optics_list, params: Params, mode: int, obs, q, wfac, sources_list=None, tag=0):
    """Per-packet g sampling over the g-ordinates of one band; returns F, K
    and the g each packet drew."""
    gv = GridView(grid)
    ng = len(optics_list)
    nobs = 0 if obs is None else len(obs)
    pr = _params(params, mode, tag, gv.max_cross, nobs)
    ops = (_Optics * ng)()
    for h, op in enumerate(optics_list):
        ops[h] = _Optics(op.a_ext.ctypes.data, op.a_abs.ctypes.data, op.omega.ctypes.data,
                         op.p_gas.ctypes.data, op.g_cld.ctypes.data)
    nout = 1 if (grid.geometry == 1 and nobs == 0) else nobs
    F = np.zeros((params.n_packets, max(nout, 1)))
    K = np.zeros((params.n_packets, NK))
    G = np.zeros(params.n_packets, dtype=np.int64)
    o = None if obs is None else _f64(obs)
    qa, wa = _f64(q), _f64(wfac)
    cdfs = wbs = None
    if sources_list is not None:
        cdfs = (ctypes.c_void_p * ng)(*[sv.cdf.ctypes.data for sv in sources_list])
        wbs = (ctypes.c_void_p * ng)(*[sv.wbirth.ctypes.data for sv in sources_list])
    lib().orc_transport_gsampled(ctypes.byref(gv.c), ops, ng, ctypes.byref(pr), _p(o), cdfs, wbs,
                                 qa.ctypes.data, wa.ctypes.data, float(grid.r_toa), F.ctypes.data, K.ctypes.data,
                                 G.ctypes.data, int(params.threads))
    return F[:, :nout], K, G


def _tag(params, spec, g, ng):
    """Key tag of the (spectral point, g) solve: 1 + spec * ng + g with
    decorrelate (spec is the band or table wavelength index), else 0."""
    return (1 + spec * ng + g) if params.decorrelate else 0


@dataclass
class Result:
    value: np.ndarray           # [n_spec, n_obs]
    stderr: np.ndarray          # [n_spec, n_obs]
    per_g: np.ndarray           # [n_spec, n_g, n_obs] value per g-ordinate
    sums: np.ndarray            # [n_spec, n_g, n_obs, 2] (sum F, sum F^2)
    counters: np.ndarray        # [n_spec, n_g, NK]
    extra: dict = field(default_factory=dict)


def _spec_list(table, spec_idx):
    if spec_idx is None:
        return list(range(table.nband))
    return [int(s) for s in spec_idx]


def contribution_function(cf_g, scale_g, w_g):
    """Band contribution function (Sect. "Albedo and emission contribution
    functions"): the per-cell peel-off tallies of every g-ordinate, scaled as
    their spectrum values are and weighted by w_g, divided per observer by
    their sum over cells and both parts (thermal, scattered), so that they
    add up to 1.  cf_g: [ng, nout, 2, ncell]."""
    acc = np.zeros(cf_g.shape[1:])
    for g in range(cf_g.shape[0]):
        acc += w_g[g] * scale_g[g] * cf_g[g]
    tot = acc.sum(axis=(1, 2))
    out = np.zeros_like(acc)
    for o in range(acc.shape[0]):
        if tot[o] > 0.0:
            out[o] = acc[o] / tot[o]
    return out


def band_image(img_g, scale_g, w_g):
    """Band image: the per-pixel peel-off tallies of every g-ordinate, scaled
    as their spectrum values are and weighted by w_g; its pixels add up to the
    band value.  img_g: [ng, nout, npix, npix]."""
    acc = np.zeros(img_g.shape[1:])
    for g in range(img_g.shape[0]):
        acc += w_g[g] * scale_g[g] * img_g[g]
    return acc


def _solve_gsampled(grid, table, params: Params, mode: int, obs, specs, keep_packets):
    """Band values with per-packet g-ordinate sampling: albedo A = pi sum F / N,
    emission F_p = sum_g(w_g L_g) sum F / (N R_TOA^2); the band's sums and
    counters are reported in its g = 0 slot (other slots and per_g stay 0)."""
    ng = table.ng
    nout = 1 if obs is None else len(obs)
    N = params.n_packets
    w = np.asarray(table.g_weights, dtype=np.float64)
    value = np.zeros((len(specs), nout))
    stderr = np.zeros_like(value)
    sums = np.zeros((len(specs), ng, nout, 2))
    cnt = np.zeros((len(specs), ng, NK))
    ltot = np.zeros((len(specs), ng))
    packets = {}
    for si, b in enumerate(specs):
        ops = [ck_optics(grid, table, b, g) for g in range(ng)]
        srcs = None
        if mode == 1:
            srcs = [emission_sources(grid, op, table.lam_um[b], params.tau_vert_max, params.emis_bias) for op in ops]
            ltot[si] = [sv.L_tot for sv in srcs]
            q, wf = g_sampling_weights(params.g_sampling, w, ltot[si])
            scale = float(np.dot(w, ltot[si])) / grid.r_toa ** 2
        else:
            q, wf = g_sampling_weights(params.g_sampling, w)
            scale = math.pi
        tag = (1 + b * ng) if params.decorrelate else 0
        if q.sum() > 0.0:
            F, K, G = transport_gsampled(grid, ops, params, mode, obs, q, wf, sources_list=srcs, tag=tag)
        else:  # nothing emits
            F, K, G = np.zeros((N, nout)), np.zeros((N, NK)), np.zeros(N, dtype=np.int64)
        if keep_packets:
            packets[(si, 0)] = (F, K, G)
        sums[si, 0, :, 0] = F.sum(axis=0)
        sums[si, 0, :, 1] = (F * F).sum(axis=0)
        cnt[si, 0] = K.sum(axis=0)
        mean = sums[si, 0, :, 0] / N
        var = np.maximum(sums[si, 0, :, 1] / N - mean * mean, 0.0) / N
        value[si] = scale * mean
        stderr[si] = scale * np.sqrt(var)
    extra = {"packets": packets}
    if mode == 1:
        extra["L_tot"] = ltot
    return Result(value, stderr, np.zeros((len(specs), ng, nout)), sums, cnt, extra)


def solve_albedo(grid, table, params: Params, spec_idx=None, keep_packets=False, contrib=False,
                 image_npix=0) -> Result:
    specs = _spec_list(table, spec_idx)
    if params.g_sampling:
        obs = None if (grid.geometry == 1 and params.obs_dir is None) else (
            _f64(params.obs_dir) if params.obs_dir is not None else albedo_obs_dirs(params.obs_phase))
        return _solve_gsampled(grid, table, params, 0, obs, specs, keep_packets)
    ng = table.ng
    if grid.geometry == 1:
        obs = None if params.obs_dir is None else _f64(params.obs_dir)
    else:
        obs = _f64(params.obs_dir) if params.obs_dir is not None else albedo_obs_dirs(params.obs_phase)
    nout = 1 if obs is None else len(obs)
    N = params.n_packets
    sums = np.zeros((len(specs), ng, nout, 2))
    cnt = np.zeros((len(specs), ng, NK))
    per_g = np.zeros((len(specs), ng, nout))
    se_g = np.zeros_like(per_g)
    packets = {}
    w = np.asarray(table.g_weights, dtype=np.float64)
    cfs, imgs = [], []
    for si, b in enumerate(specs):
        cf_g = np.zeros((ng, nout, 2, grid.ncell)) if contrib else None
        im_g = np.zeros((ng, nout, image_npix, image_npix)) if image_npix else None
        for g in range(ng):
            op = ck_optics(grid, table, b, g)
            F, K = transport(grid, op, params, 0, obs, tag=_tag(params, b, g, ng),
                             cf=cf_g[g] if contrib else None, img=im_g[g] if image_npix else None)
            if keep_packets:
                packets[(si, g)] = (F, K)
            sums[si, g, :, 0] = F.sum(axis=0)
            sums[si, g, :, 1] = (F * F).sum(axis=0)
            cnt[si, g] = K.sum(axis=0)
            E = sums[si, g, :, 0] / N
            var = np.maximum(sums[si, g, :, 1] / N - E * E, 0.0) / N
            per_g[si, g] = math.pi * E
            se_g[si, g] = math.pi * np.sqrt(var)
        if contrib:
            cfs.append(contribution_function(cf_g, np.full(ng, math.pi / N), w))
        if image_npix:
            imgs.append(band_image(im_g, np.full(ng, math.pi / N), w))
    value = np.einsum("g,sgo->so", w, per_g)
    stderr = np.sqrt(np.einsum("g,sgo->so", w * w, se_g * se_g))
    extra = {"packets": packets}
    if contrib:
        extra["cf"] = np.array(cfs)
    if image_npix:
        extra["image"] = np.array(imgs)
    return Result(value, stderr, per_g, sums, cnt, extra)


def solve_emission(grid, table, params: Params, spec_idx=None, keep_packets=False, contrib=False,
                   image_npix=0) -> Result:
    """Correlated-k emission spectrum F_p(band, phase) [erg/s/cm^2/cm]."""
    specs = _spec_list(table, spec_idx)
    if params.g_sampling:
        obs = _f64(params.obs_dir) if params.obs_dir is not None else emission_obs_dirs(params.obs_phase)
        return _solve_gsampled(grid, table, params, 1, obs, specs, keep_packets)
    ng = table.ng
    obs = _f64(params.obs_dir) if params.obs_dir is not None else emission_obs_dirs(params.obs_phase)
    nout = len(obs)
    N = params.n_packets
    sums = np.zeros((len(specs), ng, nout, 2))
    cnt = np.zeros((len(specs), ng, NK))
    per_g = np.zeros((len(specs), ng, nout))
    se_g = np.zeros_like(per_g)
    ltot = np.zeros((len(specs), ng))
    packets = {}
    rt2 = grid.r_toa ** 2
    w = np.asarray(table.g_weights, dtype=np.float64)
    cfs, imgs = [], []
    for si, b in enumerate(specs):
        cf_g = np.zeros((ng, nout, 2, grid.ncell)) if contrib else None
        im_g = np.zeros((ng, nout, image_npix, image_npix)) if image_npix else None
        for g in range(ng):
            op = ck_optics(grid, table, b, g)
            src = emission_sources(grid, op, table.lam_um[b], params.tau_vert_max, params.emis_bias)
            ltot[si, g] = src.L_tot
            if src.L_tot > 0.0:
                F, K = transport(grid, op, params, 1, obs, sources=src, tag=_tag(params, b, g, ng),
                                 cf=cf_g[g] if contrib else None, img=im_g[g] if image_npix else None)
            else:
                F, K = np.zeros((N, nout)), np.zeros((N, NK))
            if keep_packets:
                packets[(si, g)] = (F, K, src)
            sums[si, g, :, 0] = F.sum(axis=0)
            sums[si, g, :, 1] = (F * F).sum(axis=0)
            cnt[si, g] = K.sum(axis=0)
            mean = sums[si, g, :, 0] / N
            var = np.maximum(sums[si, g, :, 1] / N - mean * mean, 0.0) / N
            # L_p = (L_tot/N) sum F ; I_p = L_p/(pi R_TOA^2) ; F_p = pi I_p
            per_g[si, g] = src.L_tot * mean / rt2
            se_g[si, g] = src.L_tot * np.sqrt(var) / rt2
        if contrib:
            cfs.append(contribution_function(cf_g, ltot[si] / (N * rt2), w))
        if image_npix:
            imgs.append(band_image(im_g, ltot[si] / (N * rt2), w))
    value = np.einsum("g,sgo->so", w, per_g)
    stderr = np.sqrt(np.einsum("g,sgo->so", w * w, se_g * se_g))
    extra = {"packets": packets, "L_tot": ltot}
    if contrib:
        extra["cf"] = np.array(cfs)
    if image_npix:
        extra["image"] = np.array(imgs)
    return Result(value, stderr, per_g, sums, cnt, extra)


def transmission_alpha(grid, table, specs, hires: bool):
    """alpha_ext per spectral point (rows) for the transmission chords."""
    if hires:
        sh = doppler_shift(grid, np.array([-1.0, 0.0, 0.0]), table.dlnlam) if grid.u is not None or \
            grid.omega_rot != 0.0 else None
        return [hires_optics(grid, table, n, sh).a_ext for n in specs], [0] * len(specs)
    rows, gs = [], []
    for b in specs:
        for g in range(table.ng):
            rows.append(ck_optics(grid, table, b, g).a_ext)
            gs.append(g)
    return rows, gs


def solve_transmission(grid, table, params: Params, spec_idx=None, tau_out=False) -> Result:
    """Raytrace transmission with jittered (b, alpha) chords along -x."""
    hires = not hasattr(table, "g_weights")
    if spec_idx is None:
        specs = list(range(table.nlam if hires else table.nband))
    else:
        specs = [int(s) for s in spec_idx]
    rows, _ = transmission_alpha(grid, table, specs, hires)
    alpha = np.ascontiguousarray(np.stack(rows), dtype=np.float64)
    gv = GridView(grid)
    nrow = alpha.shape[0]
    nch = params.n_b * params.n_alpha
    val = np.zeros((nch, nrow))
    tau = np.zeros((nch, nrow)) if tau_out else None
    ld = _params(params, 0, 0, gv.max_cross, 0)
    lib().orc_transmission(ctypes.byref(gv.c), alpha.ctypes.data, nrow, params.n_b, params.n_alpha,
                           params.seed, 0, grid.r0, grid.r_toa, ctypes.byref(ld), val.ctypes.data, _p(tau),
                           int(params.threads))
    s1 = val.sum(axis=0)
    s2 = (val * val).sum(axis=0)
    dr = grid.r_toa - grid.r0
    I = dr * s1 / nch
    var = np.maximum(s2 / nch - (s1 / nch) ** 2, 0.0) / nch
    depth = (grid.r0 ** 2 + 2.0 * I) / params.r_star ** 2
    se = 2.0 * dr * np.sqrt(var) / params.r_star ** 2
    ng = 1 if hires else table.ng
    depth = depth.reshape(len(specs), ng)
    se = se.reshape(len(specs), ng)
    w = np.ones(1) if hires else np.asarray(table.g_weights, dtype=np.float64)
    value = (depth * w[None, :]).sum(axis=1)[:, None]
    stderr = np.sqrt(((se * w[None, :]) ** 2).sum(axis=1))[:, None]
    sums = np.stack([s1, s2], axis=-1).reshape(len(specs), ng, 1, 2)
    return Result(value, stderr, depth[:, :, None], sums, np.zeros((len(specs), ng, NK)),
                  {"tau": tau})


def solve_transmission_ms(grid, table, params: Params, spec_idx=None, keep_packets=False) -> Result:
    """Transmission with multiple scattering (Sect. 5.1).  Packets enter at
    random points of the annulus R0 <= b <= R_TOA with weight W0 = b times
    the stellar limb-darkening fraction of their chord; the first peel-off,
    along the chord, is the directly transmitted light and every later
    peel-off toward the observer (-x), taken over the stellar beam's solid
    angle pi (R*/a)^2, light scattered into the line of sight.  Per packet
    v = W0 - F is the light taken out of the beam, and per g-ordinate
    (R_p/R*)^2 = (R0^2 + 2 (R_TOA - R0) <v>) / R*^2, summed over g with w_g."""
    hires = not hasattr(table, "g_weights")
    if spec_idx is None:
        specs = list(range(table.nlam if hires else table.nband))
    else:
        specs = [int(s) for s in spec_idx]
    ng = 1 if hires else table.ng
    obs = np.array([[-1.0, 0.0, 0.0]])
    sh = None
    if hires and (grid.u is not None or grid.omega_rot != 0.0):
        sh = doppler_shift(grid, obs[0], table.dlnlam)
    N = params.n_packets
    dr = grid.r_toa - grid.r0
    rs2 = params.r_star ** 2
    sums = np.zeros((len(specs), ng, 1, 2))
    cnt = np.zeros((len(specs), ng, NK))
    per_g = np.zeros((len(specs), ng, 1))
    se_g = np.zeros_like(per_g)
    packets = {}
    for si, s in enumerate(specs):
        for g in range(ng):
            op = hires_optics(grid, table, s, sh) if hires else ck_optics(grid, table, s, g)
            F, K = transport(grid, op, params, 2, obs, tag=_tag(params, s, g, ng))
            v = K[:, 10] - F[:, 0]
            if keep_packets:
                packets[(si, g)] = (v, K)
            sums[si, g, 0, 0] = v.sum()
            sums[si, g, 0, 1] = (v * v).sum()
            cnt[si, g] = K.sum(axis=0)
            m = sums[si, g, 0, 0] / N
            var = max(sums[si, g, 0, 1] / N - m * m, 0.0) / N
            per_g[si, g, 0] = (grid.r0 ** 2 + 2.0 * dr * m) / rs2
            se_g[si, g, 0] = 2.0 * dr * math.sqrt(var) / rs2
    w = np.ones(1) if hires else np.asarray(table.g_weights, dtype=np.float64)
    value = np.einsum("g,sgo->so", w, per_g)
    stderr = np.sqrt(np.einsum("g,sgo->so", w * w, se_g * se_g))
    return Result(value, stderr, per_g, sums, cnt, {"packets": packets})
