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


# ------------------------------------------ invariance (separable kernels)
def _invariance_X(vfun, M, omega, n, X0=None):
    """Solve the Fourier-mode invariance equation of a semi-infinite
    atmosphere whose mode kernel is separable, p^m(mu, mu') = v(mu)^T M v(mu').

    Ambartsumian's principle gives, for each mode m (azimuth convention
    S = sum_m (2 - delta_m0) S^m cos m dphi),
        (1/mu + 1/mu0) S^m = omega [p^m(mu, -mu0) + (1/2) int p^m S^m dmu''/mu''
                                     + (1/2) int S^m p^m dmu'/mu' + (1/4) int int S^m p^m S^m]
    which factors as S^m = eps omega mu mu0 / (mu + mu0) X(mu)^T M X(mu0),
    eps = +-1 the parity of v, with the vector function
        X(mu) = v(mu) + (omega/2) mu int_0^1 [X(mu)^T M X(mu')] v(mu') / (mu + mu') dmu'.
    Solved on n Gauss nodes: damped fixed point, then Newton (hybr).
    Returns (nodes, weights, X at the nodes)."""
    mu, w = gauss01(n)
    V = vfun(mu)
    r = V.shape[1]
    Wm = w[None, :] / (mu[:, None] + mu[None, :])

    def kmat(X):  # K_i with X_i = v_i + K_i X_i
        return 0.5 * omega * mu[:, None, None] * np.einsum("ij,ja,jb->iab", Wm, V, X @ M.T)

    X = V.copy() if X0 is None else X0.copy()
    for _ in range(300):
        K = kmat(X)
        X = 0.5 * X + 0.5 * np.stack([np.linalg.solve(np.eye(r) - K[i], V[i]) for i in range(n)])

    def resid(x):
        Xx = x.reshape(n, r)
        return (Xx - V - np.einsum("iab,ib->ia", kmat(Xx), Xx)).ravel()

    sol = optimize.root(resid, X.ravel(), method="hybr", tol=1e-14)
    X = sol.x.reshape(n, r)
    assert np.abs(resid(sol.x)).max() < 1e-10
    return mu, w, X


class InvarianceMode:
    """S^m(mu, mu0) of one Fourier mode with a separable kernel, solved from
    the invariance equation (see _invariance_X); omega = 1 is reached by
    continuation from omega = 0.9 so that the physical root is followed."""

    def __init__(self, vfun, M, eps, omega, n=96):
        self.vfun, self.M, self.eps, self.omega = vfun, np.asarray(M, dtype=np.float64), eps, omega
        X = None
        path = [o for o in (0.9, 0.99, 0.999, 0.9999) if o < omega] + [omega]
        for o in path:
            self.mu, self.w, X = _invariance_X(vfun, self.M, o, n, X)
        self.X = X

    def X_at(self, m):
        """Nystrom extension of X to arbitrary mu in (0, 1]."""
        m = np.atleast_1d(np.asarray(m, dtype=np.float64))
        V = self.vfun(m)
        Wm = self.w[None, :] / (m[:, None] + self.mu[None, :])
        K = 0.5 * self.omega * m[:, None, None] * np.einsum("ij,ja,jb->iab", Wm, self.vfun(self.mu),
                                                           self.X @ self.M.T)
        r = V.shape[1]
        return np.stack([np.linalg.solve(np.eye(r) - K[i], V[i]) for i in range(len(m))])

    def S(self, m, m0):
        m = np.atleast_1d(np.asarray(m, dtype=np.float64))
        m0 = np.atleast_1d(np.asarray(m0, dtype=np.float64))
        Xa, Xb = self.X_at(m), self.X_at(m0)
        return self.eps * self.omega * (m[:, None] * m0[None, :]) / (m[:, None] + m0[None, :]) * \
            np.einsum("ia,ab,jb->ij", Xa, self.M, Xb)


class RayleighSemiInfinite:
    """Reflection of a semi-infinite atmosphere scattering with the scalar
    Rayleigh phase function (3/4)(1 + cos^2 Theta), from the invariance
    equation of its three Fourier modes:
        p^0 = (3/8)(3 - mu^2 - mu'^2 + 3 mu^2 mu'^2)   (rank 2, even),
        p^1 = (3/4) mu mu' sqrt(1-mu^2) sqrt(1-mu'^2)   (rank 1, odd),
        p^2 = (3/16)(1-mu^2)(1-mu'^2)                    (rank 1, even).
    S(mu, mu0, dphi) = S^0 + 2 S^1 cos dphi + 2 S^2 cos 2 dphi (dphi = pi is
    backscatter); E = S / (4 pi mu0) per incident packet."""

    def __init__(self, omega=1.0, n=96):
        self.modes = [
            InvarianceMode(lambda m: np.stack([np.ones_like(m), m * m], axis=1),
                           0.375 * np.array([[3.0, -1.0], [-1.0, 3.0]]), 1.0, omega, n),
            InvarianceMode(lambda m: (m * np.sqrt(np.maximum(1.0 - m * m, 0.0)))[:, None],
                           np.array([[0.75]]), -1.0, omega, n),
            InvarianceMode(lambda m: (1.0 - m * m)[:, None], np.array([[3.0 / 16.0]]), 1.0, omega, n),
        ]

    def S(self, m, m0, dphi):
        out = self.modes[0].S(m, m0)
        for k in (1, 2):
            out = out + 2.0 * self.modes[k].S(m, m0) * math.cos(k * dphi)
        return out

    def geometric_albedo(self, n=200):
        mu, w = gauss01(n)
        back = np.diag(self.S(mu, mu, math.pi))
        return 0.5 * float((w * back).sum())

    def plane_albedo(self, mu0, n=200):
        """Reflected over incident flux: (1/(2 mu0)) int_0^1 S^0(mu, mu0) dmu."""
        mu, w = gauss01(n)
        return float((w * self.modes[0].S(mu, np.array([mu0]))[:, 0]).sum()) / (2.0 * mu0)
