"""Independent reference solutions used to pin the oracle.

None of this code shares anything with the oracle or the HIP library; it
solves the same physics by different, textbook routes:

* Chandrasekhar's H-function for isotropic and separable-kernel scattering
  (Newton solve of the discretised H-equation);
* adding-doubling reflection of a homogeneous plane-parallel layer, per
  azimuthal Fourier mode, for any phase function (isotropic, Rayleigh, HG);
* exact transit chord optical depths for piecewise-constant spherical shells
  and the transmission / isothermal-emission integrals over impact parameter;
* Stefan-Boltzmann and Wien-law values of the Planck function.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

SIGMA_SB = 5.670374419e-5  # erg cm^-2 s^-1 K^-4 (CODATA 2018)
WIEN_B = 0.2897771955      # cm K (CODATA 2018)


def gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


# ----------------------------------------------------------------- H function
def h_function(psi, n=96):
    """Solve H(mu) = 1 + mu H(mu) int_0^1 Psi(mu') H(mu') / (mu + mu') dmu'
    on n Gauss nodes by Newton's method.  Returns (nodes, weights, H, evaluator)
    where evaluator(mu) is the Nystrom extension of the discrete solution."""
    mu, w = gauss01(n)
    ps = psi(mu)
    K = (w * ps)[None, :] / (mu[:, None] + mu[None, :])

    def resid(H):
        return H - 1.0 - mu * H * (K @ H)

    def jac(H):
        J = np.eye(n) - np.diag(mu * (K @ H)) - (mu * H)[:, None] * K
        return J

    H = np.ones(n)
    for _ in range(200):  # damped fixed point to get near the root
        H = 0.5 * H + 0.5 / (1.0 - mu * (K @ H))
    sol = optimize.root(resid, H, jac=jac, method="hybr", tol=1e-14)
    H = sol.x

    def ev(m):
        m = np.atleast_1d(np.asarray(m, dtype=np.float64))
        s = ((w * ps * H)[None, :] / (m[:, None] + mu[None, :])).sum(axis=1)
        return 1.0 / (1.0 - m * s)

    return mu, w, H, ev


def isotropic_semi_infinite(omega=1.0, n=96):
    """Reflection of a semi-infinite isotropic scatterer:
    S(mu, mu0) = omega/... in Chandrasekhar's form S = mu mu0 H H / (mu + mu0)
    (omega is inside Psi = omega/2).  Returns S(mu, mu0) callable."""
    _, _, _, H = h_function(lambda m: np.full_like(m, 0.5 * omega), n)

    def S(m, m0):
        m, m0 = np.broadcast_arrays(np.asarray(m, dtype=np.float64), np.asarray(m0, dtype=np.float64))
        hm = H(m.ravel()).reshape(m.shape)
        h0 = H(m0.ravel()).reshape(m0.shape)
        return omega * m * m0 * hm * h0 / (m + m0)

    return S, H


# ----------------------------------------------------------- adding-doubling
def phase_iso(c):
    return np.ones_like(c)


def phase_rayleigh(c):
    return 0.75 * (1.0 + c * c)


def phase_hg(g):
    def P(c):
        return (1.0 - g * g) / (1.0 + g * g - 2.0 * g * c) ** 1.5
    return P


def _fourier(P, mu, mu0, sign, mmax, nphi):
    phi = (np.arange(nphi) + 0.5) * 2.0 * math.pi / nphi
    s = np.sqrt(1.0 - mu * mu)
    s0 = np.sqrt(1.0 - mu0 * mu0)
    ct = sign * mu[:, None, None] * mu0[None, :, None] + \
        s[:, None, None] * s0[None, :, None] * np.cos(phi)[None, None, :]
    ct = np.clip(ct, -1.0, 1.0)
    Pv = P(ct)
    out = []
    for m in range(mmax + 1):
        out.append((Pv * np.cos(m * phi)[None, None, :]).mean(axis=2))
    return out


class Doubling:
    """Reflection function rho(mu, mu0, dphi) of a homogeneous layer by
    adding-doubling per Fourier mode (accurate for omega < 1; the conservative
    thick limit loses digits to the near-singular (1 - R R) and is pinned by
    the H-function instead).  Convention: reflected intensity for a
    collimated beam of flux pi F at mu0 is I = F mu0 rho; Chandrasekhar's
    S = 4 mu mu0 rho; dphi = pi is the backscatter azimuth.  surface_albedo > 0
    puts a Lambert reflector of that albedo under the layer (adding method)."""

    def __init__(self, P, omega, tau, n=48, mmax=0, nphi=512, n_double=None, surface_albedo=0.0):
        self.mu, self.w = gauss01(n)
        mu, w = self.mu, self.w
        self.mmax = mmax
        if n_double is None:
            n_double = 50  # start from tau / 2^50 (single scattering is then exact to O(d0^2))
        d0 = tau / 2.0 ** n_double
        Pr = _fourier(P, mu, mu, -1.0, mmax, nphi)
        Pt = _fourier(P, mu, mu, +1.0, mmax, nphi)
        Wq = (2.0 * mu * w)[None, :]
        mi, mj = mu[:, None], mu[None, :]
        ref_fac = (1.0 - np.exp(-d0 * (1.0 / mi + 1.0 / mj))) / (mi + mj)
        with np.errstate(divide="ignore", invalid="ignore"):
            tr_fac = (np.exp(-d0 / mj) - np.exp(-d0 / mi)) / (mj - mi)
        diag = np.arange(n)
        tr_fac[diag, diag] = d0 * np.exp(-d0 / mu) / (mu * mu)
        E = np.diag(np.exp(-d0 / mu))
        self.rho = []
        for m in range(mmax + 1):
            R = 0.25 * omega * Pr[m] * ref_fac * Wq
            T = 0.25 * omega * Pt[m] * tr_fac * Wq + E
            for _ in range(n_double):
                X = np.linalg.solve(np.eye(n) - R @ R, np.eye(n))
                Rn = R + T @ X @ R @ T
                Tn = T @ X @ T
                R, T = Rn, Tn
            if m == 0 and surface_albedo > 0.0:
                # add a Lambert floor below the layer: its reflection operator
                # is A_s 2 mu_j w_j in the azimuth-mean mode and zero above;
                # the layer is homogeneous, so it transmits and reflects alike
                # from either side
                Rs = surface_albedo * np.repeat(Wq, n, axis=0)
                R = R + T @ np.linalg.solve(np.eye(n) - Rs @ R, Rs @ T)
            self.rho.append(R / Wq)

    def rho_nodes(self, dphi):
        out = np.zeros_like(self.rho[0])
        for m, r in enumerate(self.rho):
            out += (1.0 if m == 0 else 2.0) * r * math.cos(m * dphi)
        return out

    def S_nodes(self, dphi):
        mu = self.mu
        return 4.0 * mu[:, None] * mu[None, :] * self.rho_nodes(dphi)

    def geometric_albedo(self):
        """A_g = (1/2) int_0^1 S(mu, mu; dphi = pi) dmu (zero-phase disk integral)."""
        S = self.S_nodes(math.pi)
        return 0.5 * float((self.w * np.diag(S)).sum())


# ----------------------------------------------------------------- transits
def _sqrt_diff2(r, b):
    return math.sqrt(max((r - b) * (r + b), 0.0))


def chord_tau(b, r_edges, alpha):
    """Full chord optical depth at impact parameter b through shells with
    constant extinction alpha[k] on [r_k, r_{k+1}] (b above the surface)."""
    t = 0.0
    for k in range(len(alpha)):
        ro, ri = r_edges[k + 1], r_edges[k]
        if ro <= b:
            continue
        t += 2.0 * alpha[k] * (_sqrt_diff2(ro, b) - _sqrt_diff2(max(ri, b), b))
    return t


def surface_ray_tau(b, r_edges, alpha):
    """Optical depth from the top to the surface along a ray with b < R0."""
    t = 0.0
    for k in range(len(alpha)):
        t += alpha[k] * (_sqrt_diff2(r_edges[k + 1], b) - _sqrt_diff2(r_edges[k], b))
    return t


def transit_integral(r_edges, alpha):
    """int_{R0}^{R_TOA} (1 - exp(-tau(b))) b db by adaptive quadrature with
    break points at every shell radius."""
    r = np.asarray(r_edges, dtype=np.float64)
    tot = 0.0
    for k in range(len(r) - 1):
        v, _ = integrate.quad(lambda b: (1.0 - math.exp(-chord_tau(b, r, alpha))) * b,
                              r[k], r[k + 1], epsabs=0.0, epsrel=1e-12, limit=200)
        tot += v
    return tot


def isothermal_disk_integral(r_edges, alpha):
    """int_0^{R_TOA} (1 - exp(-tau_path(b))) 2 pi b db: the projected emitting
    area of an isothermal atmosphere over a non-emitting, absorbing surface."""
    r = np.asarray(r_edges, dtype=np.float64)
    v0, _ = integrate.quad(lambda b: (1.0 - math.exp(-surface_ray_tau(b, r, alpha))) * b,
                           0.0, r[0], epsabs=0.0, epsrel=1e-12, limit=200)
    return 2.0 * math.pi * (v0 + transit_integral(r, alpha))
