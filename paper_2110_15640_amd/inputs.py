"""Seeded synthetic inputs shaped like the paper's GCM post-processing runs.

The paper's demonstrations post-process GCM outputs with HELIOS-K/ExoMol
k-tables and line lists (Sect. 7, Table 1, Sect. 9-13); none of those data
are available, so these generators stand in for them with grids and opacity
tables of the same shapes and value distributions:

* ``make_albedo_slab``   -- 1D plane-parallel albedo column (50 layers,
  100 bar to 1e-6 bar, isothermal, H2 Rayleigh + grey absorber, 10
  wavelengths 0.3-1.0 um).
* ``make_emission_3d``   -- 3D hot-Jupiter-like lon-lat-radius grid (128 x
  64 x 50), day-night temperature contrast with noise, a 100 band x 8 g
  correlated-k table (log-normal k), 4 phases.
* ``make_transmission_hires`` -- 128 x 64 x 60 grid with an equatorial jet
  and solid-body rotation, a 20,000 point log-uniform high-resolution
  line-forest table on 1.0-1.1 um.
* ``make_batch_mix``     -- 256 emission/albedo solves on uneven grids.

This module holds input data only: no transport arithmetic.  Both the HIP
library tests and the oracle tests draw their inputs from here.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# CGS constants used to build the synthetic atmospheres.
K_B = 1.380649e-16
M_U = 1.66053906660e-24
R_JUP = 7.1492e9
R_SUN = 6.957e10
GRAV = 1000.0  # cm s^-2
MMW = 2.3
BAR = 1.0e6  # dyn cm^-2
SEED0 = 211015640


@dataclasses.dataclass
class Grid:
    """Atmosphere structure.  geometry: 0 spherical, 1 plane-parallel slab.

    Cells are ordered (k, j, i) with longitude fastest: c = (k*nlat + j)*nlon + i.
    ``r_edges`` are radii [cm] (slab: heights [cm]); ``lat_edges``,
    ``lon_edges`` in radians; T [K] and P [bar] float32, rho [g cm^-3] float64,
    winds u (east), v (north), w (up) in cm/s float32 or None.
    """

    geometry: int
    nlon: int
    nlat: int
    nlay: int
    r_edges: np.ndarray
    lat_edges: np.ndarray
    lon_edges: np.ndarray
    T: np.ndarray
    P: np.ndarray
    rho: np.ndarray
    u: Optional[np.ndarray] = None
    v: Optional[np.ndarray] = None
    w: Optional[np.ndarray] = None
    omega_rot: float = 0.0
    cld_ksca: Optional[np.ndarray] = None
    cld_kabs: Optional[np.ndarray] = None
    cld_g: Optional[np.ndarray] = None

    @property
    def ncell(self) -> int:
        return self.nlon * self.nlat * self.nlay

    @property
    def r0(self) -> float:
        return float(self.r_edges[0])

    @property
    def r_toa(self) -> float:
        return float(self.r_edges[-1])


@dataclasses.dataclass
class CKTable:
    """Pre-mixed correlated-k table kappa[band][g][T][P] (cm^2/g, float32).

    lam_um: band-centre wavelengths [um]; g_weights sum to 1; T_grid [K] and
    P_grid [bar] increasing; k_ray: Rayleigh opacity per band [cm^2/g].
    """

    lam_um: np.ndarray
    g_weights: np.ndarray
    T_grid: np.ndarray
    P_grid: np.ndarray
    kappa: np.ndarray
    k_ray: np.ndarray

    @property
    def nband(self) -> int:
        return int(self.kappa.shape[0])

    @property
    def ng(self) -> int:
        return int(self.kappa.shape[1])


@dataclasses.dataclass
class HiresTable:
    """High-resolution table kappa[lam][T][P] on lam_n = lam_min exp(n dlnlam)."""

    lam_min_um: float
    dlnlam: float
    T_grid: np.ndarray
    P_grid: np.ndarray
    kappa: np.ndarray
    k_ray: np.ndarray

    @property
    def nlam(self) -> int:
        return int(self.kappa.shape[0])

    def lam_um(self) -> np.ndarray:
        return self.lam_min_um * np.exp(np.arange(self.nlam) * self.dlnlam)


def rayleigh_h2(lam_um) -> np.ndarray:
    """H2 Rayleigh opacity [cm^2/g]: sigma = 8.14e-13 l^-4 + 1.28e-6 l^-6 +
    1.61 l^-8 cm^2 (l in Angstrom; Dalgarno & Williams form), per mean
    particle mass mmw*m_u.  An input choice for the synthetic atmospheres."""
    la = np.asarray(lam_um, dtype=np.float64) * 1.0e4
    sigma = 8.14e-13 * la ** -4 + 1.28e-6 * la ** -6 + 1.61 * la ** -8
    return sigma / (MMW * M_U)


def pressure_edges(nlay: int, p_bot: float = 100.0, p_top: float = 1e-6) -> np.ndarray:
    """Log-spaced pressure edges [bar], bottom first."""
    k = np.arange(nlay + 1, dtype=np.float64)
    return p_bot * (p_top / p_bot) ** (k / nlay)


def hydrostatic_heights(p_edges: np.ndarray, t_ref: float = 1200.0) -> np.ndarray:
    """Heights [cm] of isothermal hydrostatic pressure edges (scale height H)."""
    H = K_B * t_ref / (MMW * M_U * GRAV)
    return H * np.log(p_edges[0] / p_edges)


def latlon_edges(nlon: int, nlat: int):
    lon = -math.pi + 2.0 * math.pi * np.arange(nlon + 1) / nlon
    lat = -0.5 * math.pi + math.pi * np.arange(nlat + 1) / nlat
    lon[0], lon[-1] = -math.pi, math.pi
    lat[0], lat[-1] = -0.5 * math.pi, 0.5 * math.pi
    return lat, lon


def gauss_legendre_01(ng: int):
    x, w = np.polynomial.legendre.leggauss(ng)
    return 0.5 * (x + 1.0), 0.5 * w


def _probit(p):
    from scipy.special import ndtri
    return ndtri(p)


# --------------------------------------------------------------------------
# Albedo column (1D plane-parallel)
# --------------------------------------------------------------------------
def make_albedo_slab(nlay: int = 50, nlam: int = 10, lam_lo: float = 0.3, lam_hi: float = 1.0,
                     T: float = 1200.0, k_abs: float = 1e-3):
    """Slab column: mass-conserving layer densities rho_k = dP_k/(g dz_k), so a
    layer's optical depth is kappa dP/g exactly."""
    pe = pressure_edges(nlay)
    z = hydrostatic_heights(pe)
    dz = np.diff(z)
    rho = (pe[:-1] - pe[1:]) * BAR / (GRAV * dz)
    pc = np.sqrt(pe[:-1] * pe[1:])
    lam = np.linspace(lam_lo, lam_hi, nlam)
    grid = Grid(1, 1, 1, nlay, z.astype(np.float64), np.array([-math.pi / 2, math.pi / 2]),
                np.array([-math.pi, math.pi]), np.full(nlay, T, np.float32),
                pc.astype(np.float32), rho.astype(np.float64))
    table = CKTable(lam_um=lam, g_weights=np.ones(1), T_grid=np.array([500.0, 3000.0]),
                    P_grid=np.array([1e-6, 100.0]),
                    kappa=np.full((nlam, 1, 2, 2), k_abs, np.float32),
                    k_ray=rayleigh_h2(lam))
    return grid, table


def make_homogeneous_slab(tau: float, omega: float, g_cld: float = 0.0, rayleigh: bool = False,
                          nlay: int = 1, height: float = 8388608.0):
    """A homogeneous slab of total optical depth tau and albedo omega for the
    closed-form checks (unit density, opacities chosen to give tau; the
    default height 2^23 cm keeps kappa = tau/height exact in float32 for
    power-of-two tau).
    rayleigh=True: gas (Rayleigh) scatterer; else a cloud scatterer with HG g
    (g = 0 is isotropic)."""
    z = np.linspace(0.0, height, nlay + 1)
    rho = np.ones(nlay)
    kext = tau / height
    ksca = omega * kext
    kabs = kext - ksca
    ncell = nlay
    if rayleigh:
        table = CKTable(np.array([0.5]), np.ones(1), np.array([1000.0]), np.array([1.0]),
                        np.full((1, 1, 1, 1), kabs, np.float32), np.array([ksca]))
        grid = Grid(1, 1, 1, nlay, z, np.array([-math.pi / 2, math.pi / 2]),
                    np.array([-math.pi, math.pi]), np.full(ncell, 1000.0, np.float32),
                    np.ones(ncell, np.float32), rho)
    else:
        table = CKTable(np.array([0.5]), np.ones(1), np.array([1000.0]), np.array([1.0]),
                        np.full((1, 1, 1, 1), kabs, np.float32), np.zeros(1))
        grid = Grid(1, 1, 1, nlay, z, np.array([-math.pi / 2, math.pi / 2]),
                    np.array([-math.pi, math.pi]), np.full(ncell, 1000.0, np.float32),
                    np.ones(ncell, np.float32), rho,
                    cld_ksca=np.full(ncell, ksca, np.float32),
                    cld_kabs=np.zeros(ncell, np.float32),
                    cld_g=np.full(ncell, g_cld, np.float32))
    return grid, table


# --------------------------------------------------------------------------
# 3D spherical grids
# --------------------------------------------------------------------------
def _sphere_structure(rng, nlon, nlat, nlay, noise=50.0):
    pe = pressure_edges(nlay)
    r = R_JUP + hydrostatic_heights(pe)
    lat, lon = latlon_edges(nlon, nlat)
    latc = 0.5 * (lat[:-1] + lat[1:])
    lonc = 0.5 * (lon[:-1] + lon[1:])
    day = np.maximum(np.cos(lonc)[None, :] * np.cos(latc)[:, None], 0.0)  # [j, i]
    T = 1000.0 + 800.0 * day[None, :, :] + noise * rng.standard_normal((nlay, nlat, nlon))
    T = np.maximum(T, 100.0)
    pc = np.sqrt(pe[:-1] * pe[1:])
    P = np.broadcast_to(pc[:, None, None], (nlay, nlat, nlon))
    rho = P * BAR * MMW * M_U / (K_B * T)
    return r, lat, lon, T.reshape(-1).astype(np.float32), \
        np.ascontiguousarray(P).reshape(-1).astype(np.float32), rho.reshape(-1).astype(np.float64)


def make_sphere(nlon, nlat, nlay, seed, noise=50.0) -> Grid:
    rng = np.random.Generator(np.random.PCG64(seed))
    r, lat, lon, T, P, rho = _sphere_structure(rng, nlon, nlat, nlay, noise)
    return Grid(0, nlon, nlat, nlay, r, lat, lon, T, P, rho)


def make_ck_table(rng, nband=100, ng=8, nT=20, nP=20, lam_lo=0.3, lam_hi=30.0) -> CKTable:
    edges = lam_lo * (lam_hi / lam_lo) ** (np.arange(nband + 1) / nband)
    lam_c = np.sqrt(edges[:-1] * edges[1:])
    gx, gw = gauss_legendre_01(ng)
    Tg = np.linspace(500.0, 3000.0, nT)
    Pg = 1e-6 * (100.0 / 1e-6) ** (np.arange(nP) / max(nP - 1, 1))
    m_b = rng.normal(math.log(1e-2), 1.5, nband)
    s_b = rng.uniform(0.5, 2.0, nband)
    z_g = _probit(gx)
    lnk = m_b[:, None] + s_b[:, None] * z_g[None, :]
    kap = np.exp(lnk)[:, :, None, None] * (Pg[None, None, None, :] ** 0.5) * \
        (Tg[None, None, :, None] / 1000.0)
    return CKTable(lam_c, gw, Tg, Pg, kap.astype(np.float32), rayleigh_h2(lam_c))


def make_emission_3d(nlon=128, nlat=64, nlay=50, nband=100, ng=8, config_no=2):
    """3D emission phase-curve inputs: grid + ck table + phases."""
    seed = SEED0 + config_no
    rng = np.random.Generator(np.random.PCG64(seed))
    r, lat, lon, T, P, rho = _sphere_structure(rng, nlon, nlat, nlay)
    grid = Grid(0, nlon, nlat, nlay, r, lat, lon, T, P, rho)
    table = make_ck_table(rng, nband=nband, ng=ng)
    phases = np.array([0.0, 0.25, 0.5, 0.75])
    return grid, table, phases


def make_transmission_hires(nlon=128, nlat=64, nlay=60, nlam=20000, lam_lo=1.0, lam_hi=1.1,
                            nT=20, nP=20, u_jet=5.0e5, config_no=3):
    """3D transmission inputs with winds: equatorial jet u = u_jet
    exp(-lat^2 / (2 (15 deg)^2)) and solid-body rotation 2 pi / 3.5 d."""
    seed = SEED0 + config_no
    rng = np.random.Generator(np.random.PCG64(seed))
    r, lat, lon, T, P, rho = _sphere_structure(rng, nlon, nlat, nlay)
    latc = 0.5 * (lat[:-1] + lat[1:])
    jet = u_jet * np.exp(-latc ** 2 / (2.0 * math.radians(15.0) ** 2))
    u = np.broadcast_to(jet[None, :, None], (nlay, nlat, nlon)).reshape(-1).astype(np.float32)
    grid = Grid(0, nlon, nlat, nlay, r, lat, lon, T, P, rho,
                u=np.ascontiguousarray(u), v=np.zeros_like(u), w=np.zeros_like(u),
                omega_rot=2.0 * math.pi / (3.5 * 86400.0))
    dlnlam = math.log(lam_hi / lam_lo) / max(nlam - 1, 1)
    Tg = np.linspace(500.0, 3000.0, nT)
    Pg = 1e-6 * (100.0 / 1e-6) ** (np.arange(nP) / max(nP - 1, 1))
    zn = rng.standard_normal(nlam)
    kap = np.exp(math.log(1e-2) + 2.0 * zn)[:, None, None] * (Pg[None, None, :] ** 0.3) * \
        ((Tg[None, :, None] / 1000.0) ** 0.5)
    lam = lam_lo * np.exp(np.arange(nlam) * dlnlam)
    table = HiresTable(lam_lo, dlnlam, Tg, Pg, kap.astype(np.float32), rayleigh_h2(lam))
    return grid, table


@dataclasses.dataclass
class BatchSolve:
    mode: str  # "albedo" or "emission"
    grid_index: int
    bands: np.ndarray
    n_packets: int


def make_batch_mix(n_solves=256, packet_scale=1.0, config_no=4):
    """Batched mix: grids Nlon = 32 + 16 round(6 s1), Nlat = Nlon/2,
    Nlay = round(30 + 30 s2); 10-500 bands from a 500-band table; packets per
    (band, g) log-uniform 1e4-1e6 (times packet_scale); albedo/emission 50/50."""
    seed = SEED0 + config_no
    rng = np.random.Generator(np.random.PCG64(seed))
    table = make_ck_table(rng, nband=500, ng=8)
    grids: List[Grid] = []
    solves: List[BatchSolve] = []
    for s in range(n_solves):
        s1, s2 = rng.uniform(), rng.uniform()
        nlon = 32 + 16 * int(round(6 * s1))
        nlat = nlon // 2
        nlay = int(round(30 + 30 * s2))
        grids.append(make_sphere(nlon, nlat, nlay, seed * 1000 + s))
        nb = int(rng.integers(10, 501))
        bands = np.sort(rng.choice(500, size=nb, replace=False)).astype(np.int32)
        npk = int(round(10 ** rng.uniform(4, 6) * packet_scale))
        solves.append(BatchSolve("albedo" if rng.uniform() < 0.5 else "emission", s, bands, max(npk, 64)))
    return grids, table, solves


def transmission_strata(n_b=256, n_alpha=360):
    return n_b, n_alpha
