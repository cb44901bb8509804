// Device building blocks shared by the HIP kernels: the Philox4x32-10 draw
// keyed by (packet, event, block), phase functions and their samplers
// (Sect. 3), direction rotation, the spherical / slab cell traversal
// (Sect. 2) and the opacity-table interpolation (Sect. 7).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mcrt_internal.hpp"

namespace mcrt {
namespace dev {

constexpr double kPi = 3.14159265358979323846;
constexpr double kH = 6.62607015e-27;
constexpr double kC = 2.99792458e10;
constexpr double kKB = 1.380649e-16;

// ---------------------------------------------------------------- RNG
// Philox4x32-10 (Salmon et al. 2011): counter (packet lo, packet hi, event,
// block), key (seed lo, seed hi ^ tag).
struct U2 {
    double a, b;
};

__device__ __forceinline__ U2 draw(uint64_t seed, uint32_t tag, uint64_t packet, uint32_t event,
                                   uint32_t block)
{
    uint32_t c0 = (uint32_t)packet, c1 = (uint32_t)(packet >> 32), c2 = event, c3 = block;
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32) ^ tag;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    U2 u;
    uint64_t ma = ((uint64_t)c0 << 20) | (uint64_t)(c1 >> 12);
    uint64_t mb = ((uint64_t)c2 << 20) | (uint64_t)(c3 >> 12);
    u.a = ((double)ma + 0.5) * (1.0 / 4503599627370496.0);
    u.b = ((double)mb + 0.5) * (1.0 / 4503599627370496.0);
    return u;
}

// ---------------------------------------------------------------- phase functions
__device__ __forceinline__ double p_rayleigh(double mu) { return 0.75 * (1.0 + mu * mu); }

__device__ __forceinline__ double p_hg(double mu, double g)
{
    if (fabs(g) < 1e-6) return 1.0;
    double den = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (den * sqrt(den));
}

// Rayleigh: Cardano root of mu^3 + 3 mu = 2 (4 zeta - 2), the inverse of the
// CDF (mu^3 + 3 mu + 4)/8 of the normalised phase function.
__device__ __forceinline__ double sample_rayleigh(double z)
{
    double q = 4.0 * z - 2.0;
    double u = cbrt(q + sqrt(q * q + 1.0));
    double mu = u - 1.0 / u;
    return fmin(fmax(mu, -1.0), 1.0);
}

__device__ __forceinline__ double sample_hg(double z, double g)
{
    double mu;
    if (fabs(g) < 1e-6) {
        mu = 2.0 * z - 1.0;
    } else {
        double t = (1.0 - g * g) / (1.0 - g + 2.0 * g * z);
        mu = (1.0 + g * g - t * t) / (2.0 * g);
    }
    return fmin(fmax(mu, -1.0), 1.0);
}

__device__ __forceinline__ void rotate_dir(double& dx, double& dy, double& dz, double mu, double psi)
{
    double st = sqrt(fmax(1.0 - mu * mu, 0.0));
    double cp = cos(psi), sp = sin(psi);
    double nx, ny, nz;
    if (fabs(dz) < 0.99999) {
        double t = sqrt(1.0 - dz * dz);
        nx = st * (dx * dz * cp - dy * sp) / t + dx * mu;
        ny = st * (dy * dz * cp + dx * sp) / t + dy * mu;
        nz = -st * cp * t + dz * mu;
    } else {
        double sgn = dz >= 0.0 ? 1.0 : -1.0;
        nx = st * cp;
        ny = st * sp;
        nz = sgn * mu;
    }
    double n = sqrt(nx * nx + ny * ny + nz * nz);
    dx = nx / n;
    dy = ny / n;
    dz = nz / n;
}

// ------------------------------------------------------ Draine phase function
// Draine's hybrid HG-Rayleigh function (Sect. 3, aerosol scattering) is
// P_HG(G) (1 + alpha mu^2) / (1 + alpha (1 + 2 G^2)/3); its mean cosine
// G (1 + alpha (3 + 2 G^2)/5) / (1 + alpha (1 + 2 G^2)/3) rises from -1 to 1
// on [-1, 1], so the G of a cloud with asymmetry factor g is found by
// bisection to the last bit (alpha = 0: HG, G = g).
__host__ __device__ inline double draine_G(double g, double alpha)
{
    if (alpha == 0.0) return g;
    double lo = -1.0, hi = 1.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        const double m = mid * (1.0 + alpha * (3.0 + 2.0 * mid * mid) / 5.0) /
                         (1.0 + alpha * (1.0 + 2.0 * mid * mid) / 3.0);
        if (m < g) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// ------------------------------------------------------ forced interaction
// Optical depth of a forced flight over a path of depth tp (0 < tp < inf)
// from zeta, and the weight factor e^{-tau}/q(tau) of its density q on
// [0, tp]: kind 1 forced scattering q = e^{-tau}/(1 - e^{-tp}); kind 2
// path-length stretching q = l e^{-l tau}/(1 - e^{-l tp}), l = 1/(1 + tp);
// kind 3 their equal mixture, the component picked by zc < 1/2.
__host__ __device__ inline double forced_tau(int kind, double tp, double zeta, double zc, double& wf)
{
    const double pf = -expm1(-tp);
    const double l = 1.0 / (1.0 + tp);
    const double pl = -expm1(-l * tp);
    const bool stretch = kind == 2 || (kind == 3 && !(zc < 0.5));
    const double tau = stretch ? -log1p(-zeta * pl) / l : -log1p(-zeta * pf);
    if (kind == 1) {
        wf = pf;
    } else if (kind == 2) {
        wf = exp(-tau) * pl / (l * exp(-l * tau));
    } else {
        const double q = 0.5 * exp(-tau) / pf + 0.5 * l * exp(-l * tau) / pl;
        wf = exp(-tau) / q;
    }
    return tau;
}

// ------------------------------------------------- stellar limb darkening
// I(mu)/I(1) of the stellar disk at zenith cosine mu (Sect. 5.1.1): laws
// 0 none, 1 linear, 2 quadratic, 3 square-root, 4 logarithmic,
// 5 exponential, 6 power-2; and the weight of the stellar light behind the
// sky-plane point (y, z) of the planet's frame, which lies at (ty + y,
// tz + z) on the stellar disk (zero off the disk).
__host__ __device__ inline double limb_law(int law, double c1, double c2, double mu)
{
    const double x = 1.0 - mu;
    if (law == 1) return 1.0 - c1 * x;
    if (law == 2) return 1.0 - c1 * x - c2 * x * x;
    if (law == 3) return 1.0 - c1 * x - c2 * (1.0 - sqrt(mu));
    if (law == 4) return 1.0 - c1 * x - c2 * (mu > 0.0 ? mu * log(mu) : 0.0);
    if (law == 5) return 1.0 - c1 * x - c2 / (1.0 - exp(mu));
    if (law == 6) return 1.0 - c1 * (1.0 - pow(mu, c2));
    return 1.0;
}

__host__ __device__ inline double limb_weight(const LimbDark& ld, double y, double z)
{
    if (ld.law == 0) return 1.0;
    const double sy = ld.ty + y, sz = ld.tz + z;
    const double q = (sy * sy + sz * sz) / (ld.r_star * ld.r_star);
    return q < 1.0 ? limb_law(ld.law, ld.c1, ld.c2, sqrt(1.0 - q)) : 0.0;
}

// ---------------------------------------------------------------- geometry
enum { F_NONE = -1, F_OUT = 0, F_IN = 1, F_LATLO = 2, F_LATHI = 3, F_LONLO = 4, F_LONHI = 5 };
enum { T_INTERACT = 0, T_ESCAPE = 1, T_SURFACE = 2, T_LOST = 3 };

struct Ray {
    double x, y, z;
    int i, j, k;
    int ef;
};

__host__ __device__ __forceinline__ int find_edge(const double* e, int n, double x)
{
    // largest m in [0, n-1] with e[m] <= x, 0 if none (edges increasing)
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (e[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Distance to the latitude cone (the equatorial plane when tb == 0) of an
// edge with cos^2 = c2, sin^2 = s2; roots below lo ignored; hits must be on
// the nappe whose z has the sign of tb.
__host__ __device__ __forceinline__ double cone_distance(const Ray& p, double dx, double dy, double dz, double tb,
                                                double c2, double s2, double lo)
{
    double best = INFINITY;
    if (tb == 0.0) {
        if (dz != 0.0) {
            double s = -p.z / dz;
            if (s >= lo) best = s;
        }
        return best;
    }
    double a = dz * dz * c2 - (dx * dx + dy * dy) * s2;
    double b = p.z * dz * c2 - (p.x * dx + p.y * dy) * s2;
    double c = p.z * p.z * c2 - (p.x * p.x + p.y * p.y) * s2;
    double r0 = -1.0, r1 = -1.0;
    bool h0 = false, h1 = false;
    if (a == 0.0) {
        if (b != 0.0) {
            r0 = -c / (2.0 * b);
            h0 = true;
        }
    } else {
        double disc = b * b - a * c;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double q = -(b + (b >= 0.0 ? sq : -sq));
            r0 = q / a;
            h0 = true;
            if (q != 0.0) {
                r1 = c / q;
                h1 = true;
            }
        }
    }
    if (h0 && r0 >= lo) {
        double zh = p.z + r0 * dz;
        bool ok = tb > 0.0 ? (zh > 0.0) : (zh < 0.0);
        if (ok && r0 < best) best = r0;
    }
    if (h1 && r1 >= lo) {
        double zh = p.z + r1 * dz;
        bool ok = tb > 0.0 ? (zh > 0.0) : (zh < 0.0);
        if (ok && r1 < best) best = r1;
    }
    return best;
}

// Distance to leave the current cell along d; returns the face (ties in the
// order outer, inner, lat-low, lat-high, lon-low, lon-high).
__host__ __device__ __forceinline__ int exit_distance(const GridDev& g, const Ray& p, double dx, double dy,
                                             double dz, double& s_out)
{
    if (g.geom == 1) {
        if (dz > 0.0) {
            double s = (g.r[p.k + 1] - p.z) / dz;
            s_out = s < 0.0 ? 0.0 : s;
            return F_OUT;
        }
        if (dz < 0.0) {
            double s = (g.r[p.k] - p.z) / dz;
            s_out = s < 0.0 ? 0.0 : s;
            return F_IN;
        }
        s_out = INFINITY;
        return F_NONE;
    }
    double rr = p.x * p.x + p.y * p.y + p.z * p.z;
    double B = p.x * dx + p.y * dy + p.z * dz;
    double best;
    int face;
    {
        double ro = g.r[p.k + 1];
        double C = rr - ro * ro;
        double D = B * B - C;
        if (D < 0.0) D = 0.0;
        double s = (B <= 0.0) ? (-B + sqrt(D)) : (-C / (B + sqrt(D)));
        if (s < 0.0) s = 0.0;
        best = s;
        face = F_OUT;
    }
    if (B < 0.0) {
        double ri = g.r[p.k];
        double C = rr - ri * ri;
        double D = B * B - C;
        if (D >= 0.0) {
            double s = C / (-B + sqrt(D));
            if (s < 0.0) s = 0.0;
            if (s < best) {
                best = s;
                face = F_IN;
            }
        }
    }
    double tol = 1e-9 * sqrt(rr);
    if (p.j > 0) {
        int e = p.j;
        double s = cone_distance(p, dx, dy, dz, g.lat[e], g.lat_c2[e], g.lat_s2[e],
                                 p.ef == F_LATLO ? tol : 0.0);
        if (s < best) {
            best = s;
            face = F_LATLO;
        }
    }
    if (p.j < g.nlat - 1) {
        int e = p.j + 1;
        double s = cone_distance(p, dx, dy, dz, g.lat[e], g.lat_c2[e], g.lat_s2[e],
                                 p.ef == F_LATHI ? tol : 0.0);
        if (s < best) {
            best = s;
            face = F_LATHI;
        }
    }
    if (g.nlon > 1) {
        {
            double sb = g.lon_s[p.i], cb = g.lon_c[p.i];
            double nx = -sb, ny = cb;
            double dn = dx * nx + dy * ny;
            if (dn < 0.0) {
                double s = -(p.x * nx + p.y * ny) / dn;
                if (s < 0.0) s = 0.0;
                double hx = p.x + s * dx, hy = p.y + s * dy;
                if (cb * hx + sb * hy > 0.0 && s < best) {
                    best = s;
                    face = F_LONLO;
                }
            }
        }
        {
            int iu = p.i + 1 == g.nlon ? 0 : p.i + 1;
            double sb = g.lon_s[iu], cb = g.lon_c[iu];
            double nx = -sb, ny = cb;
            double dn = dx * nx + dy * ny;
            if (dn > 0.0) {
                double s = -(p.x * nx + p.y * ny) / dn;
                if (s < 0.0) s = 0.0;
                double hx = p.x + s * dx, hy = p.y + s * dy;
                if (cb * hx + sb * hy > 0.0 && s < best) {
                    best = s;
                    face = F_LONHI;
                }
            }
        }
    }
    s_out = best;
    return face;
}

__host__ __device__ __forceinline__ void advance(const GridDev& g, Ray& p, double dx, double dy, double dz, double s)
{
    if (g.geom == 1) {
        p.z = p.z + s * dz;
    } else {
        p.x = p.x + s * dx;
        p.y = p.y + s * dy;
        p.z = p.z + s * dz;
    }
}

__host__ __device__ __forceinline__ void cross(const GridDev& g, Ray& p, int f)
{
    switch (f) {
    case F_OUT:
        p.k += 1;
        p.ef = F_IN;
        if (g.geom == 1 && p.k <= g.nlay) p.z = g.r[p.k];
        break;
    case F_IN:
        p.k -= 1;
        p.ef = F_OUT;
        if (g.geom == 1 && p.k >= -1) p.z = g.r[p.k + 1];
        break;
    case F_LATLO: p.j -= 1; p.ef = F_LATHI; break;
    case F_LATHI: p.j += 1; p.ef = F_LATLO; break;
    case F_LONLO: p.i = p.i == 0 ? g.nlon - 1 : p.i - 1; p.ef = F_LONHI; break;
    case F_LONHI: p.i = p.i + 1 == g.nlon ? 0 : p.i + 1; p.ef = F_LONLO; break;
    default: break;
    }
}

__host__ __device__ __forceinline__ int cell_of(const GridDev& g, const Ray& p)
{
    return (p.k * g.nlat + p.j) * g.nlon + p.i;
}

__host__ __device__ __forceinline__ void locate_column(const GridDev& g, Ray& p)
{
    double lat = atan2(p.z, sqrt(p.x * p.x + p.y * p.y));
    double lon = atan2(p.y, p.x);
    p.j = find_edge(g.lat, g.nlat, lat);
    p.i = find_edge(g.lon, g.nlon, lon);
}

// ---------------------------------------------------------------- opacity interpolation
struct Bracket {
    int i0, i1;
    double t;
};

__device__ __forceinline__ Bracket bracket(const double* gx, int n, double x)
{
    Bracket b;
    if (n == 1) {
        b.i0 = 0; b.i1 = 0; b.t = 0.0;
        return b;
    }
    if (x <= gx[0]) {
        b.i0 = 0; b.i1 = 1; b.t = 0.0;
        return b;
    }
    if (x >= gx[n - 1]) {
        b.i0 = n - 2; b.i1 = n - 1; b.t = 1.0;
        return b;
    }
    int m = find_edge(gx, n - 1, x);
    b.i0 = m;
    b.i1 = m + 1;
    b.t = (x - gx[m]) / (gx[m + 1] - gx[m]);
    return b;
}

// ln-kappa bilinear in (T, ln P); a -inf (zero kappa) corner with positive
// weight gives zero.  lnk(iT, iP) read through the accessor.
template <typename F>
__device__ __forceinline__ double interp_tp(F lnk, const Bracket& bt, const Bracket& bp)
{
    double t = bt.t, u = bp.t;
    double w0 = (1.0 - t) * (1.0 - u), w1 = (1.0 - t) * u, w2 = t * (1.0 - u), w3 = t * u;
    double acc = 0.0;
    if (w0 > 0.0) { double l = lnk(bt.i0, bp.i0); if (isinf(l)) return 0.0; acc = acc + w0 * l; }
    if (w1 > 0.0) { double l = lnk(bt.i0, bp.i1); if (isinf(l)) return 0.0; acc = acc + w1 * l; }
    if (w2 > 0.0) { double l = lnk(bt.i1, bp.i0); if (isinf(l)) return 0.0; acc = acc + w2 * l; }
    if (w3 > 0.0) { double l = lnk(bt.i1, bp.i1); if (isinf(l)) return 0.0; acc = acc + w3 * l; }
    return exp(acc);
}


// Arithmetic of a crossing.  The exact form rounds every product and sum on
// its own and divides correctly rounded, operation for operation as the FP64
// oracle; the fast form, taken by the FP32-mixed transport, contracts a
// product and a sum into one multiply-add and divides through the hardware
// reciprocal (good to about 5e-8 on gfx950) refined by one Newton step and a
// residual correction: within an ulp of the rounded quotient, and equal to it
// on every one of 2^20 random operands over 30 decades tried on the device.
template <bool FAST>
__host__ __device__ __forceinline__ double wk_mad(double a, double b, double c)
{
    if constexpr (FAST) return fma(a, b, c);
    else return a * b + c;
}

template <bool FAST>
__host__ __device__ __forceinline__ double wk_div(double a, double b)
{
    if constexpr (FAST) {
        double r = __builtin_amdgcn_rcp(b);
        r = fma(r, fma(-b, r, 1.0), r);
        const double qt = a * r;
        return fma(fma(-b, qt, a), r, qt);
    } else {
        return a / b;
    }
}

// Square root of x >= 0 (finite).  The fast form refines the hardware
// reciprocal square root y ~ 1/sqrt(x) by Goldschmidt's iteration (g = x y,
// h = y/2, r = 1/2 - h g, g <- g + g r, h <- h + h r) and one correction
// g <- g + (x - g^2) h, which bring it within an ulp of the rounded root
// (equal to it on 2^20 random operands over 30 decades tried on the device;
// y is good to about 5e-8); without the library's range scaling, which these
// operands (squared lengths of ~1e9 cm and their differences) never need.
template <bool FAST>
__host__ __device__ __forceinline__ double wk_sqrt(double x)
{
    if constexpr (FAST) {
        const double y = __builtin_amdgcn_rsq(x);
        double g = x * y, h = 0.5 * y;
        const double r = fma(-h, g, 0.5);
        g = fma(g, r, g);
        h = fma(h, r, h);
        g = fma(fma(-g, g, x), h, g);
        return x > 0.0 ? g : 0.0;
    } else {
        return sqrt(x);
    }
}

// ---------------------------------------------------------------- walker
// Straight-line walk through the cells from an origin p0 along unit d.  Along
// a straight line every face surface is met at fixed ray parameters t (a
// shell or a cone at most twice, a longitude plane once), so the walk keeps
// the parameters of the current cell's faces and, after a crossing, computes
// only the faces that are new to the cell: one shell, one cone or one plane.
// Positions are never advanced step by step (p(t) = p0 + t d), so there is no
// drift; tie order and entry-face rules are those of exit_distance.
struct Walker {
    double px, py, pz;      // origin
    double dx, dy, dz;      // unit direction
    double t;               // distance walked from the origin
    double B0, C0;          // p0 . d, |p0|^2 (spherical) ; unused for the slab
    double tout, tin;       // outer-face exit / inner-face hit (INFINITY = none)
    double tin_far;         // far root of the inner sphere when tin is set: the
                            // outer face's exit once that sphere is crossed
    double lo1, lo2;        // lower latitude cone roots on its nappe, ascending
    double hi1, hi2;        // upper latitude cone roots
    double tlo, thi;        // lower / upper longitude half-plane hits
    int i, j, k;
    int c;                  // cell index (k * nlat + j) * nlon + i, kept as the walk moves
    int ef;                 // face by which the current cell was entered
};

// The faces of a walk's first cell (wk_start); FAST: the fast arithmetic of
// wk_mad, wk_div and wk_sqrt, otherwise every operation rounded on its own.
template <bool FAST = false>
__host__ __device__ __forceinline__ void wk_shells(const GridDev& g, Walker& w, bool need_out, bool need_in)
{
    if (g.geom == 1) {
        if (need_out) w.tout = w.dz > 0.0 ? fmax(wk_div<FAST>(g.r[w.k + 1] - w.pz, w.dz), w.t) : INFINITY;
        if (need_in) w.tin = w.dz < 0.0 ? fmax(wk_div<FAST>(g.r[w.k] - w.pz, w.dz), w.t) : INFINITY;
        return;
    }
    if (need_out) {
        double R = g.r[w.k + 1];
        double C = wk_mad<FAST>(-R, R, w.C0);
        double D = wk_mad<FAST>(w.B0, w.B0, -C);
        if (D < 0.0) D = 0.0;
        double sq = wk_sqrt<FAST>(D);
        double far = (w.B0 <= 0.0) ? (-w.B0 + sq) : wk_div<FAST>(-C, w.B0 + sq);
        w.tout = fmax(far, w.t);
    }
    if (need_in) {
        w.tin = INFINITY;
        if (w.B0 < 0.0) {
            double R = g.r[w.k];
            double C = wk_mad<FAST>(-R, R, w.C0);
            double D = wk_mad<FAST>(w.B0, w.B0, -C);
            if (D >= 0.0) {
                const double q = -w.B0 + wk_sqrt<FAST>(D);
                double nr = wk_div<FAST>(C, q);
                if (nr >= w.t || C < 0.0) {
                    w.tin = fmax(nr, w.t);
                    w.tin_far = q;
                }
            }
        }
    }
}

// Coefficients of the latitude cone z^2 cos^2(lat) = (x^2 + y^2) sin^2(lat)
// along p0 + t d: a t^2 + 2 b t + c = 0.  The exact form evaluates them as
// written; the fast form (FP32-mixed transport) uses cos^2 + sin^2 = 1 and
// |d| = 1, i.e. a = dz^2 - sin^2, b = pz dz - (p0.d) sin^2,
// c = pz^2 - |p0|^2 sin^2 (three multiply-adds instead of fifteen operations).
template <bool FAST>
__host__ __device__ __forceinline__ void wk_cone_coef(const GridDev& g, const Walker& w, int e, double& a, double& b,
                                                      double& c)
{
    const double s2 = g.lat_s2[e];
    if constexpr (FAST) {
        a = fma(w.dz, w.dz, -s2);
        b = fma(w.pz, w.dz, -(w.B0 * s2));
        c = fma(w.pz, w.pz, -(w.C0 * s2));
    } else {
        const double c2 = g.lat_c2[e];
        a = w.dz * w.dz * c2 - (w.dx * w.dx + w.dy * w.dy) * s2;
        b = w.pz * w.dz * c2 - (w.px * w.dx + w.py * w.dy) * s2;
        c = w.pz * w.pz * c2 - (w.px * w.px + w.py * w.py) * s2;
    }
}

// Roots of the latitude cone of edge e on the nappe of its sign (or the
// equatorial plane), ascending, INFINITY where absent.
template <bool FAST = false>
__host__ __device__ __forceinline__ void wk_cone(const GridDev& g, const Walker& w, int e, double& r1, double& r2)
{
    r1 = INFINITY;
    r2 = INFINITY;
    double tb = g.lat[e];
    if (tb == 0.0) {
        if (w.dz != 0.0) r1 = wk_div<FAST>(-w.pz, w.dz);
        return;
    }
    double a, b, c;
    wk_cone_coef<FAST>(g, w, e, a, b, c);
    double x0 = INFINITY, x1 = INFINITY;
    if (a == 0.0) {
        if (b != 0.0) x0 = wk_div<FAST>(-c, 2.0 * b);
    } else {
        double disc = wk_mad<FAST>(b, b, -(a * c));
        if (disc >= 0.0) {
            double sq = wk_sqrt<FAST>(disc);
            double q = -(b + (b >= 0.0 ? sq : -sq));
            if constexpr (FAST) {  // both roots from one reciprocal, as in wk_cross_end
                if (q != 0.0) {
                    const double inv = wk_div<true>(1.0, a * q);
                    x0 = (q * q) * inv;
                    x1 = (c * a) * inv;
                } else {
                    x0 = 0.0;
                }
            } else {
                x0 = wk_div<FAST>(q, a);
                if (q != 0.0) x1 = wk_div<FAST>(c, q);
            }
        }
    }
    const double z0 = wk_mad<FAST>(x0, w.dz, w.pz), z1 = wk_mad<FAST>(x1, w.dz, w.pz);
    bool ok0 = x0 < INFINITY && (tb > 0.0 ? (z0 > 0.0) : (z0 < 0.0));
    bool ok1 = x1 < INFINITY && (tb > 0.0 ? (z1 > 0.0) : (z1 < 0.0));
    if (!ok0) x0 = INFINITY;
    if (!ok1) x1 = INFINITY;
    r1 = fmin(x0, x1);
    r2 = fmax(x0, x1);
    if (!(r1 < INFINITY)) r2 = INFINITY;
}

// Hit of the longitude half-plane of edge e (upper = the cell's upper face).
template <bool FAST = false>
__host__ __device__ __forceinline__ double wk_plane(const GridDev& g, const Walker& w, int e, bool upper)
{
    double sb = g.lon_s[e], cb = g.lon_c[e];
    double nx = -sb, ny = cb;
    double dn = wk_mad<FAST>(w.dx, nx, w.dy * ny);
    if (upper ? !(dn > 0.0) : !(dn < 0.0)) return INFINITY;
    double th = fmax(wk_div<FAST>(-wk_mad<FAST>(w.px, nx, w.py * ny), dn), w.t);
    double hx = wk_mad<FAST>(th, w.dx, w.px), hy = wk_mad<FAST>(th, w.dy, w.py);
    return (wk_mad<FAST>(cb, hx, sb * hy) > 0.0) ? th : INFINITY;
}

template <bool FAST = false>
__host__ __device__ __forceinline__ void wk_start(const GridDev& g, Walker& w, double px, double py, double pz, double dx,
                                         double dy, double dz, int i, int j, int k, int ef)
{
    w.px = px; w.py = py; w.pz = pz;
    w.dx = dx; w.dy = dy; w.dz = dz;
    w.t = 0.0;
    w.i = i; w.j = j; w.k = k;
    w.c = (k * g.nlat + j) * g.nlon + i;
    w.ef = ef;
    w.B0 = px * dx + py * dy + pz * dz;
    w.C0 = px * px + py * py + pz * pz;
    wk_shells<FAST>(g, w, true, true);
    w.lo1 = w.lo2 = w.hi1 = w.hi2 = INFINITY;
    w.tlo = w.thi = INFINITY;
    if (g.geom == 1) return;
    if (j > 0) wk_cone<FAST>(g, w, j, w.lo1, w.lo2);
    if (j < g.nlat - 1) wk_cone<FAST>(g, w, j + 1, w.hi1, w.hi2);
    if (g.nlon > 1) {
        w.tlo = wk_plane<FAST>(g, w, i, false);
        w.thi = wk_plane<FAST>(g, w, i + 1 == g.nlon ? 0 : i + 1, true);
    }
}

// Next cone root at or after t; roots of the cone just crossed must lie more
// than 1e-9 |p| ahead (the same entry-face tolerance as exit_distance).
__host__ __device__ __forceinline__ double wk_next_root(double r1, double r2, double t, double lo)
{
    if (r1 >= lo) return r1;
    if (r2 >= lo) return r2;
    return INFINITY;
}

// Parameter and face of the next crossing (ties: outer, inner, lat-low,
// lat-high, lon-low, lon-high).
template <bool FAST = false>
__host__ __device__ __forceinline__ int wk_next(const GridDev& g, const Walker& w, double& tf, double r_top = 0.0)
{
    double best = w.tout;
    int face = w.tout < INFINITY ? F_OUT : F_NONE;
    if (w.tin < best) { best = w.tin; face = F_IN; }
    if (g.geom == 1) {
        tf = best;
        return face;
    }
    // entry-face tolerance 1e-9 |p|, with |p| bounded by the cell's outer
    // radius (it only separates a re-found root of the cone just crossed,
    // ~1e-16 |p| away, from genuine ones); the fast form bounds |p| by the
    // top of the grid, r_top (the caller's, no gather per step)
    double lo = w.t;
    if (w.ef == F_LATLO || w.ef == F_LATHI) lo = w.t + 1e-9 * (FAST ? r_top : g.r[w.k + 1]);
    double a = wk_next_root(w.lo1, w.lo2, w.t, w.ef == F_LATLO ? lo : w.t);
    if (a < best) { best = a; face = F_LATLO; }
    double b = wk_next_root(w.hi1, w.hi2, w.t, w.ef == F_LATHI ? lo : w.t);
    if (b < best) { best = b; face = F_LATHI; }
    if (w.tlo < best) { best = w.tlo; face = F_LONLO; }
    if (w.thi < best) { best = w.thi; face = F_LONHI; }
    tf = best;
    return face;
}

// Move to parameter tf on face f, enter the neighbour cell and compute the
// faces that are new to it.  Returns false when the walk left the grid
// (k == nlay: top; k < 0: surface).
//
// Every crossing needs exactly one new surface: the next outer sphere
// (outward), the next inner sphere (inward; the new outer face is the sphere
// just crossed, whose far root was kept with tin), the next cone, or the next
// longitude plane.  All of them are met where A t^2 + 2 B t + C = 0 (planes
// and the equator: the linear B2 t + C = 0), so one branch-free body solves
// that equation for every lane of a wave, whatever face kind it crosses, and
// per-kind selects pick the roots.  The arithmetic of each kind is the same,
// operation for operation, as in wk_shells, wk_cone and wk_plane (in the
// exact form; FAST: see wk_mad and wk_div).
// The grid-table values a crossing reads, loaded by wk_cross_begin so that a
// caller can issue other loads (the extinction gather) before the crossing's
// arithmetic in wk_cross_end waits for them: v1 = the new sphere's radius,
// the cone's latitude or the plane's sin(lon); v2 = the cone's sin^2(lat) or
// the plane's cos(lon); v3 = the cone's cos^2(lat) (exact form only).
struct CrossIn {
    double v1, v2, v3;
    bool inside;
};

// Index update and table loads of a crossing, without branches: every lane
// of a wave runs the same instructions whatever face it crosses (a lane with
// no face, f < 0, keeps its indices and loads in-range entries it ignores).
template <bool FAST = false>
__host__ __device__ __forceinline__ CrossIn wk_cross_begin(const GridDev& g, Walker& w, int f, double tf)
{
    CrossIn x;
    w.t = tf;
    const bool valid = f >= 0;
    const bool shell = valid && f <= F_IN, cone = f == F_LATLO || f == F_LATHI, plane = f == F_LONLO || f == F_LONHI;
    const bool outward = f == F_OUT, down = f == F_LATLO, west = f == F_LONLO;
    const int dk = shell ? (outward ? 1 : -1) : 0;
    const int dj = cone ? (down ? -1 : 1) : 0;
    const bool wrap = west ? (w.i == 0) : (w.i + 1 == g.nlon);
    const int ni = west ? (w.i == 0 ? g.nlon - 1 : w.i - 1) : (w.i + 1 == g.nlon ? 0 : w.i + 1);
    const int di = plane ? (west ? (wrap ? g.nlon - 1 : -1) : (wrap ? 1 - g.nlon : 1)) : 0;
    w.k += dk;
    w.j += dj;
    w.i = plane ? ni : w.i;
    w.c += dk * (g.nlon * g.nlat) + dj * g.nlon + di;
    w.ef = shell ? (outward ? F_IN : F_OUT)
                 : (cone ? (down ? F_LATHI : F_LATLO) : (plane ? (west ? F_LONHI : F_LONLO) : w.ef));
    x.inside = valid && w.k < g.nlay && w.k >= 0;
    const int kr = outward ? w.k + 1 : w.k;
    const int kk = kr < 0 ? 0 : (kr > g.nlay ? g.nlay : kr);
    const int e = down ? w.j : w.j + 1;
    const bool has = down ? w.j > 0 : w.j < g.nlat - 1;
    const int ee = g.lat_base + 3 * ((cone && has) ? e : 0);
    const int ep = g.lon_base + 2 * (west ? w.i : (w.i + 1 == g.nlon ? 0 : w.i + 1));
    const int o1 = shell ? kk : (cone ? ee : ep);
    const int o2 = (cone ? ee : ep) + 1;
    x.v1 = g.faces[o1];
    x.v2 = g.faces[o2];
    x.v3 = FAST ? 0.0 : g.faces[ee + 2];
    return x;
}

template <bool FAST = false>
__host__ __device__ __forceinline__ bool wk_cross_end(const GridDev& g, Walker& w, int f, const CrossIn& x)
{
    if (!x.inside) return false;
    const bool shell = f <= F_IN, cone = f == F_LATLO || f == F_LATHI;
    const bool outward = f == F_OUT, down = f == F_LATLO, west = f == F_LONLO;
    const bool slab = g.geom == 1;
    // the new surface: coefficients of A t^2 + 2 B t + C (A = 0: B2 t + C)
    double A = 0.0, B = 0.0, C = 0.0, B2 = 0.0;
    bool has = true;     // a surface to intersect at all
    bool equator = false;
    double tb = 0.0, sb = 0.0, cb = 0.0;
    if (shell) {
        const double R = x.v1;
        has = outward || slab || w.B0 < 0.0;
        if (slab) {
            B2 = w.dz;
            C = w.pz - R;
        } else {
            A = 1.0;
            B = w.B0;
            C = wk_mad<FAST>(-R, R, w.C0);
        }
    } else if (cone) {
        has = down ? w.j > 0 : w.j < g.nlat - 1;
        tb = x.v1;
        equator = tb == 0.0;
        if (equator) {
            B2 = w.dz;
            C = w.pz;
        } else {
            const double s2 = x.v2;
            if constexpr (FAST) {  // as wk_cone_coef's fast form
                A = fma(w.dz, w.dz, -s2);
                B = fma(w.pz, w.dz, -(w.B0 * s2));
                C = fma(w.pz, w.pz, -(w.C0 * s2));
            } else {
                const double c2 = x.v3;
                A = wk_mad<FAST>(w.dz * w.dz, c2, -(wk_mad<FAST>(w.dx, w.dx, w.dy * w.dy) * s2));
                B = wk_mad<FAST>(w.pz * w.dz, c2, -(wk_mad<FAST>(w.px, w.dx, w.py * w.dy) * s2));
                C = wk_mad<FAST>(w.pz * w.pz, c2, -(wk_mad<FAST>(w.px, w.px, w.py * w.py) * s2));
            }
            B2 = 2.0 * B;
        }
    } else {
        sb = x.v1;
        cb = x.v2;
        const double nx = -sb, ny = cb;
        const double dn = wk_mad<FAST>(w.dx, nx, w.dy * ny);
        has = west ? dn < 0.0 : dn > 0.0;
        B2 = dn;
        C = wk_mad<FAST>(w.px, nx, w.py * ny);
    }
    // one solve for every lane
    const bool quad = A != 0.0;
    const double D = wk_mad<FAST>(B, B, -(A * C));
    const double sq = wk_sqrt<FAST>(fmax(D, 0.0));
    const bool neg = cone ? B >= 0.0 : B > 0.0;  // the sign rule of each kind at B = 0
    const double q = neg ? -(B + sq) : (-B + sq);
    // one division gives the near root q / A of a quadric (a shell has A = 1)
    // or the root -C / B2 of a linear face, whichever the lane has
    double rd, x1q;
    if constexpr (FAST) {
        // both roots of a quadric from one reciprocal, 1/(A q): q/A = q^2/(A q)
        // and C/q = C A/(A q); a linear face's root -C/B2 from 1/B2
        const bool qz = quad && q == 0.0;
        const double den = quad ? (qz ? A : A * q) : B2;
        const double inv = wk_div<true>(1.0, den);
        rd = quad ? (qz ? 0.0 : (q * q) * inv) : -C * inv;
        x1q = (quad && !qz) ? (C * A) * inv : INFINITY;
    } else {
        rd = wk_div<FAST>(quad ? q : -C, quad ? A : B2);
        x1q = (quad && q != 0.0) ? wk_div<FAST>(C, q) : INFINITY;
    }
    const double x0q = rd;
    const double xl = (!quad && B2 != 0.0) ? rd : INFINITY;
    if (shell) {
        if (slab) {
            const double x = fmax(wk_div<FAST>(-C, B2), w.t);  // (R - pz) / dz
            if (outward) {
                w.tout = w.dz > 0.0 ? x : INFINITY;
                w.tin = INFINITY;
            } else {
                w.tout = INFINITY;
                w.tin = w.dz < 0.0 ? x : INFINITY;
            }
            return true;
        }
        if (outward) {  // far root of the next outer sphere; the sphere crossed is behind
            w.tout = fmax(B > 0.0 ? x1q : x0q, w.t);
            w.tin = INFINITY;
        } else {        // outer face: the sphere just crossed; inner face: the next sphere, if hit
            w.tout = fmax(w.tin_far, w.t);
            w.tin = INFINITY;
            if (has && D >= 0.0 && (x1q >= w.t || C < 0.0)) {
                w.tin = fmax(x1q, w.t);
                w.tin_far = q;
            }
        }
        return true;
    }
    if (cone) {
        double r1 = INFINITY, r2 = INFINITY;
        if (has) {
            if (equator) {
                r1 = w.dz != 0.0 ? xl : INFINITY;
            } else {
                double x0 = INFINITY, x1 = INFINITY;
                if (!quad) {
                    x0 = B != 0.0 ? rd : INFINITY;
                } else if (D >= 0.0) {
                    x0 = x0q;
                    x1 = x1q;
                }
                const bool ok0 = x0 < INFINITY && (tb > 0.0 ? (wk_mad<FAST>(x0, w.dz, w.pz) > 0.0)
                                                            : (wk_mad<FAST>(x0, w.dz, w.pz) < 0.0));
                const bool ok1 = x1 < INFINITY && (tb > 0.0 ? (wk_mad<FAST>(x1, w.dz, w.pz) > 0.0)
                                                            : (wk_mad<FAST>(x1, w.dz, w.pz) < 0.0));
                if (!ok0) x0 = INFINITY;
                if (!ok1) x1 = INFINITY;
                r1 = fmin(x0, x1);
                r2 = fmax(x0, x1);
                if (!(r1 < INFINITY)) r2 = INFINITY;
            }
        }
        // the cone crossed becomes the opposite face of the new cell
        const double k1 = down ? w.lo1 : w.hi1, k2 = down ? w.lo2 : w.hi2;
        if (down) {
            w.hi1 = k1; w.hi2 = k2;
            w.lo1 = r1; w.lo2 = r2;
        } else {
            w.lo1 = k1; w.lo2 = k2;
            w.hi1 = r1; w.hi2 = r2;
        }
        return true;
    }
    // longitude half-plane (the one crossed is behind the ray: never met again)
    double th = INFINITY;
    if (has) {
        th = fmax(xl, w.t);
        const double hx = wk_mad<FAST>(th, w.dx, w.px), hy = wk_mad<FAST>(th, w.dy, w.py);
        if (!(wk_mad<FAST>(cb, hx, sb * hy) > 0.0)) th = INFINITY;
    }
    w.tlo = west ? th : INFINITY;
    w.thi = west ? INFINITY : th;
    return true;
}

template <bool FAST = false>
__host__ __device__ __forceinline__ bool wk_cross(const GridDev& g, Walker& w, int f, double tf)
{
    const CrossIn x = wk_cross_begin<FAST>(g, w, f, tf);
    return wk_cross_end<FAST>(g, w, f, x);
}

__host__ __device__ __forceinline__ int wk_cell(const GridDev& /*g*/, const Walker& w) { return w.c; }

}  // namespace dev
}  // namespace mcrt
