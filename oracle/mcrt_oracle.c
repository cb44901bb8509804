/*
 * mcrt_oracle.c -- plain, slow, FP64 CPU oracle of the gCMCRT photon-transport
 * hot path (Lee et al., "3D radiative-transfer for exoplanet atmospheres.
 * gCMCRT: a GPU accelerated MCRT code", arXiv:2110.15640).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or helper with
 * the HIP library.
 *
 * Every function follows the paper's definitions, step by step, in FP64 with
 * no blocking, fusion or reordering:
 *   - photon-packet Monte Carlo with peel-off (Sect. 2, Sect. 4.6 "Next event
 *     estimation", the peel-off fraction equation);
 *   - phase functions and their samplers (Sect. 3: isotropic, Rayleigh, HG
 *     with its inverse-CDF equation; gas/cloud choice by P_gas);
 *   - continuous absorption and survival biasing (Sect. 4.1, 4.4),
 *     Russian roulette (Sect. 4.5), hybrid emission biasing (Sect. 4.3),
 *     the vertical optical-depth cut (Sect. 4.6, tau_vert);
 *   - observables (Sect. 5: transmission equation and its MC estimator,
 *     geometric albedo A_g, cell luminosity L_i, L_p, I_p, F_p);
 *   - Doppler shifted high-resolution opacity (Sect. 7: v_LOS and
 *     lambda_eff equations) and band-centre continuum in ck mode.
 * Where the paper is silent or garbled the reading taken is stated inline
 * (e.g. the Rayleigh inverse CDF, the RNG, the traversal tie order).
 *
 * Pins (tests/test_oracle_*.py) tie it to closed forms: Philox KAT vs
 * rocRAND, sampler CDFs/moments, brute-force geometry, Beer-Lambert,
 * Chandrasekhar H-function reflection, single scattering, transit shell sums,
 * isothermal emission and energy conservation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
static const double ORC_H = 6.62607015e-27;  /* erg s */
static const double ORC_C = 2.99792458e10;   /* cm / s */
static const double ORC_KB = 1.380649e-16;   /* erg / K */

/* ------------------------------------------------------------------------ */
/* Counter-based RNG: Philox4x32-10 (Salmon et al. 2011).  The paper does not
 * name its RNG; a counter-based one keyed by (packet, event, block) makes the
 * packet histories independent of scheduling.                              */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)prod1;
        uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)prod0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 52 random bits from a word pair -> (m + 1/2) 2^-52, exactly in (0,1). */
double orc_u01(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)a << 20) | (uint64_t)(b >> 12);
    return ((double)m + 0.5) * (1.0 / 4503599627370496.0);
}

/* Uniform pair for (packet, event, block) under the solve key. */
static void orc_draw(uint64_t seed, uint32_t tag, uint64_t packet, uint32_t event,
                     uint32_t block, double *ua, double *ub)
{
    uint32_t ctr[4] = {(uint32_t)packet, (uint32_t)(packet >> 32), event, block};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ tag};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    *ua = orc_u01(w[0], w[1]);
    *ub = orc_u01(w[2], w[3]);
}

void orc_draw_pair(uint64_t seed, uint32_t tag, uint64_t packet, uint32_t event,
                   uint32_t block, double out[2])
{
    orc_draw(seed, tag, packet, event, block, &out[0], &out[1]);
}

/* ------------------------------------------------------------------------ */
/* Phase functions (Sect. 3).                                               */
/* ------------------------------------------------------------------------ */
double orc_phase_rayleigh(double mu) { return 0.75 * (1.0 + mu * mu); }

double orc_phase_hg(double mu, double g)
{
    if (fabs(g) < 1e-6) return 1.0;  /* g -> 0: HG is isotropic */
    double den = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (den * sqrt(den));
}

/* Rayleigh cos(theta): exact inverse of F(mu) = (mu^3 + 3 mu + 4)/8.  The
 * printed sampling formula is garbled (it is not a CDF inverse); Cardano's
 * root of mu^3 + 3 mu = 2q with q = 4 zeta - 2 is used instead.             */
double orc_sample_rayleigh(double zeta)
{
    double q = 4.0 * zeta - 2.0;
    double u = cbrt(q + sqrt(q * q + 1.0));
    double mu = u - 1.0 / u;
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    return mu;
}

/* HG cos(theta) by the paper's inverse CDF; isotropic when |g| < 1e-6. */
double orc_sample_hg(double zeta, double g);

/* Two-term HG (Sect. 3, aerosol scattering): a forward lobe g1 = g with
 * weight a = 1 - g2^2 and a backward lobe g2 = -g/2 (the paper's default
 * relation between the lobes and the asymmetry factor). */
static void tthg_lobes(double g, double *g1, double *g2, double *a)
{
    *g1 = g;
    *g2 = -0.5 * g;
    *a = 1.0 - (*g2) * (*g2);
}

double orc_phase_tthg(double mu, double g)
{
    double g1, g2, a;
    tthg_lobes(g, &g1, &g2, &a);
    return a * orc_phase_hg(mu, g1) + (1.0 - a) * orc_phase_hg(mu, g2);
}

/* A lobe is chosen with zeta_lobe < a (forward) and cos(theta) is sampled
 * from that lobe's HG function with zeta. */
double orc_sample_tthg(double zeta_lobe, double zeta, double g)
{
    double g1, g2, a;
    tthg_lobes(g, &g1, &g2, &a);
    return orc_sample_hg(zeta, zeta_lobe < a ? g1 : g2);
}

double orc_sample_hg(double zeta, double g)
{
    double mu;
    if (fabs(g) < 1e-6) {
        mu = 2.0 * zeta - 1.0;
    } else {
        double t = (1.0 - g * g) / (1.0 - g + 2.0 * g * zeta);
        mu = (1.0 + g * g - t * t) / (2.0 * g);
    }
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    return mu;
}

/* Draine's hybrid HG-Rayleigh function (Sect. 3, aerosol scattering):
 * P = (1 - G^2)/(1 + alpha (1 + 2 G^2)/3) (1 + alpha mu^2)/(1 + G^2 - 2 G mu)^{3/2},
 * i.e. P_HG(G) (1 + alpha mu^2) over its normalisation, whose mean cosine
 * is G (1 + alpha (3 + 2 G^2)/5)/(1 + alpha (1 + 2 G^2)/3).               */
double orc_draine_mean_cosine(double G, double alpha)
{
    return G * (1.0 + alpha * (3.0 + 2.0 * G * G) / 5.0) / (1.0 + alpha * (1.0 + 2.0 * G * G) / 3.0);
}

/* G of a cloud whose asymmetry factor is g: the root of mean cosine = g on
 * [-1, 1] by bisection (the mean cosine rises from -1 to 1); alpha = 0 is
 * HG itself (G = g). */
double orc_draine_G(double g, double alpha)
{
    if (alpha == 0.0) return g;
    double lo = -1.0, hi = 1.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (orc_draine_mean_cosine(mid, alpha) < g) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

double orc_phase_draine(double mu, double G, double alpha)
{
    return orc_phase_hg(mu, G) * (1.0 + alpha * mu * mu) / (1.0 + alpha * (1.0 + 2.0 * G * G) / 3.0);
}

/* Exact sampling by rejection from HG(G): candidate k has cos(theta) from
 * HG(G) with za[k] and is accepted when zacc[k] (1 + alpha) < 1 + alpha mu^2
 * (the acceptance probability (1 + alpha mu^2)/(1 + alpha) <= 1 for
 * alpha >= 0); the n-th candidate is taken if none before is accepted.     */
double orc_sample_draine(const double *za, const double *zacc, int n, double G, double alpha)
{
    double mu = 0.0;
    for (int k = 0; k < n; ++k) {
        mu = orc_sample_hg(za[k], G);
        if (zacc[k] * (1.0 + alpha) < 1.0 + alpha * mu * mu) break;
    }
    return mu;
}

/* Forced interaction of a flight whose path to the edge of the grid has
 * optical depth tp (0 < tp < inf) (Sect. 4, forced interaction): tau is
 * drawn with zeta (the flight's block 0, slot a) from a density q on
 * [0, tp] and the packet's weight is multiplied by e^{-tau}/q(tau), while
 * the fraction e^{-tp} that would have left unscattered is booked as
 * escaped.  1: forced scattering, q = e^{-tau}/(1 - e^{-tp}) (the factor is
 * 1 - e^{-tp}); 2: path-length stretching, q = l e^{-l tau}/(1 - e^{-l tp})
 * with l = 1/(1 + tp); 3: hybrid, q the equal mixture of 1 and 2, the
 * component chosen by zc < 1/2.                                            */
double orc_forced_tau(int64_t kind, double tp, double zeta, double zc, double *wfac)
{
    double pf = -expm1(-tp);
    double l = 1.0 / (1.0 + tp);
    double pl = -expm1(-l * tp);
    double tau;
    if (kind == 1 || (kind == 3 && zc < 0.5)) tau = -log1p(-zeta * pf);
    else tau = -log1p(-zeta * pl) / l;
    if (kind == 1) {
        *wfac = pf;
    } else if (kind == 2) {
        *wfac = exp(-tau) * pl / (l * exp(-l * tau));
    } else {
        double q = 0.5 * exp(-tau) / pf + 0.5 * l * exp(-l * tau) / pl;
        *wfac = exp(-tau) / q;
    }
    return tau;
}

/* Candidates drawn for one Draine scattering (the last is taken if none of
 * the others is accepted: probability below (alpha/(1+alpha))^31). */
#define ORC_DRAINE_MAXC 32

/* Rotate unit d by polar cos(theta)=mu about it and azimuth psi. */
void orc_rotate(double d[3], double mu, double psi)
{
    double st = sqrt(fmax(1.0 - mu * mu, 0.0));
    double cp = cos(psi), sp = sin(psi);
    double nx, ny, nz;
    if (fabs(d[2]) < 0.99999) {
        double t = sqrt(1.0 - d[2] * d[2]);
        nx = st * (d[0] * d[2] * cp - d[1] * sp) / t + d[0] * mu;
        ny = st * (d[1] * d[2] * cp + d[0] * sp) / t + d[1] * mu;
        nz = -st * cp * t + d[2] * mu;
    } else {
        double sgn = d[2] >= 0.0 ? 1.0 : -1.0;
        nx = st * cp;
        ny = st * sp;
        nz = sgn * mu;
    }
    double n = sqrt(nx * nx + ny * ny + nz * nz);
    d[0] = nx / n;
    d[1] = ny / n;
    d[2] = nz / n;
}

/* ------------------------------------------------------------------------ */
/* Grid and geometry (Sect. 2: spherical lon-lat-radius cells, sub-grid     */
/* packet motion; also the plane-parallel slab for 1D structures).          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t geom; /* 0 spherical, 1 plane-parallel slab */
    int64_t nlon, nlat, nlay;
    const double *r;   /* nlay+1 radii [cm] (slab: heights z [cm]) */
    const double *lat; /* nlat+1 latitude edges [rad], -pi/2 .. pi/2 */
    const double *lon; /* nlon+1 longitude edges [rad], -pi .. pi */
} orc_grid;

enum { F_NONE = -1, F_OUT = 0, F_IN = 1, F_LATLO = 2, F_LATHI = 3, F_LONLO = 4, F_LONHI = 5 };
enum { T_INTERACT = 0, T_ESCAPE = 1, T_SURFACE = 2, T_LOST = 3, T_CUT = 4 };

static int64_t cell_index(const orc_grid *g, int i, int j, int k)
{
    return ((int64_t)k * g->nlat + j) * g->nlon + i;
}

/* largest index m in [0, n-1] with e[m] <= x (clamped) */
static int edge_find(const double *e, int64_t n, double x)
{
    int m = 0;
    for (int64_t q = 1; q < n; ++q)
        if (e[q] <= x) m = (int)q;
    return m;
}

/* Candidate distance to a latitude cone (or the equatorial plane) of edge
 * latitude tb.  Roots below lo are ignored; the hit must lie on the nappe
 * whose z sign is that of tb.  Returns +inf when there is none.            */
static double cone_distance(const double p[3], const double d[3], double tb, double lo)
{
    double best = INFINITY;
    if (tb == 0.0) {
        if (d[2] != 0.0) {
            double s = -p[2] / d[2];
            if (s >= lo) best = s;
        }
        return best;
    }
    double ct = cos(tb), st = sin(tb);
    double c2 = ct * ct, s2 = st * st;
    double a = d[2] * d[2] * c2 - (d[0] * d[0] + d[1] * d[1]) * s2;
    double b = p[2] * d[2] * c2 - (p[0] * d[0] + p[1] * d[1]) * s2;
    double c = p[2] * p[2] * c2 - (p[0] * p[0] + p[1] * p[1]) * s2;
    double roots[2];
    int nr = 0;
    if (a == 0.0) {
        if (b != 0.0) roots[nr++] = -c / (2.0 * b);
    } else {
        double disc = b * b - a * c;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double q = -(b + (b >= 0.0 ? sq : -sq));
            roots[nr++] = q / a;
            if (q != 0.0) roots[nr++] = c / q;
        }
    }
    for (int m = 0; m < nr; ++m) {
        double s = roots[m];
        if (!(s >= lo)) continue;
        double zh = p[2] + s * d[2];
        int ok = tb > 0.0 ? (zh > 0.0) : (zh < 0.0);
        if (ok && s < best) best = s;
    }
    return best;
}

/* Distance to leave spherical cell (i,j,k) from p along d.  ef = face by
 * which the ray entered (F_NONE at an event point).  Ties resolve in the
 * order outer, inner, lat-low, lat-high, lon-low, lon-high.               */
static int sph_exit(const orc_grid *g, const double p[3], const double d[3],
                    int i, int j, int k, int ef, double *s_out)
{
    double rr = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    double B = p[0] * d[0] + p[1] * d[1] + p[2] * d[2];
    double best = INFINITY;
    int face = F_NONE;

    /* outer shell r_{k+1} */
    {
        double ro = g->r[k + 1];
        double C = rr - ro * ro;
        double D = B * B - C;
        if (D < 0.0) D = 0.0;
        double s = (B <= 0.0) ? (-B + sqrt(D)) : (-C / (B + sqrt(D)));
        if (s < 0.0) s = 0.0;
        if (s < best) { best = s; face = F_OUT; }
    }
    /* inner shell r_k (the planet surface when k == 0) */
    if (B < 0.0) {
        double ri = g->r[k];
        double C = rr - ri * ri;
        double D = B * B - C;
        if (D >= 0.0) {
            double s = C / (-B + sqrt(D));
            if (s < 0.0) s = 0.0;
            if (s < best) { best = s; face = F_IN; }
        }
    }
    /* latitude cones; the poles are not faces */
    double tol = 1e-9 * sqrt(rr);
    if (j > 0) {
        double s = cone_distance(p, d, g->lat[j], ef == F_LATLO ? tol : 0.0);
        if (s < best) { best = s; face = F_LATLO; }
    }
    if (j < g->nlat - 1) {
        double s = cone_distance(p, d, g->lat[j + 1], ef == F_LATHI ? tol : 0.0);
        if (s < best) { best = s; face = F_LATHI; }
    }
    /* longitude half-planes (periodic; edge nlon is edge 0) */
    if (g->nlon > 1) {
        double pb = g->lon[i];
        double nx = -sin(pb), ny = cos(pb);
        double dn = d[0] * nx + d[1] * ny;
        if (dn < 0.0) {
            double s = -(p[0] * nx + p[1] * ny) / dn;
            if (s < 0.0) s = 0.0;
            double hx = p[0] + s * d[0], hy = p[1] + s * d[1];
            if (cos(pb) * hx + sin(pb) * hy > 0.0 && s < best) { best = s; face = F_LONLO; }
        }
        int iu = (int)((i + 1) % g->nlon);
        pb = g->lon[iu];
        nx = -sin(pb);
        ny = cos(pb);
        dn = d[0] * nx + d[1] * ny;
        if (dn > 0.0) {
            double s = -(p[0] * nx + p[1] * ny) / dn;
            if (s < 0.0) s = 0.0;
            double hx = p[0] + s * d[0], hy = p[1] + s * d[1];
            if (cos(pb) * hx + sin(pb) * hy > 0.0 && s < best) { best = s; face = F_LONHI; }
        }
    }
    *s_out = best;
    return face;
}

/* Slab: distance along d to the top or bottom of layer k from height z. */
static int slab_exit(const orc_grid *g, double z, const double d[3], int k, double *s_out)
{
    if (d[2] > 0.0) {
        double s = (g->r[k + 1] - z) / d[2];
        *s_out = s < 0.0 ? 0.0 : s;
        return F_OUT;
    }
    if (d[2] < 0.0) {
        double s = (g->r[k] - z) / d[2];
        *s_out = s < 0.0 ? 0.0 : s;
        return F_IN;
    }
    *s_out = INFINITY;
    return F_NONE;
}

typedef struct {
    double p[3];
    int i, j, k;
    int ef;
} orc_ray;

/* Move across face f: update indices and the entry face of the new cell.
 * In the slab the height snaps onto the crossed edge.                     */
static void cross_face(const orc_grid *g, orc_ray *ry, int f)
{
    switch (f) {
    case F_OUT: ry->k += 1; ry->ef = F_IN; if (g->geom == 1 && ry->k <= g->nlay) ry->p[2] = g->r[ry->k]; break;
    case F_IN: ry->k -= 1; ry->ef = F_OUT; if (g->geom == 1 && ry->k >= -1) ry->p[2] = g->r[ry->k + 1]; break;
    case F_LATLO: ry->j -= 1; ry->ef = F_LATHI; break;
    case F_LATHI: ry->j += 1; ry->ef = F_LATLO; break;
    case F_LONLO: ry->i = (int)((ry->i - 1 + g->nlon) % g->nlon); ry->ef = F_LONHI; break;
    case F_LONHI: ry->i = (int)((ry->i + 1) % g->nlon); ry->ef = F_LONLO; break;
    default: break;
    }
}

static int exit_distance(const orc_grid *g, const orc_ray *ry, const double d[3], double *s)
{
    if (g->geom == 1) return slab_exit(g, ry->p[2], d, ry->k, s);
    return sph_exit(g, ry->p, d, ry->i, ry->j, ry->k, ry->ef, s);
}

static void advance(const orc_grid *g, orc_ray *ry, const double d[3], double s)
{
    if (g->geom == 1) {
        ry->p[2] = ry->p[2] + s * d[2];
    } else {
        ry->p[0] = ry->p[0] + s * d[0];
        ry->p[1] = ry->p[1] + s * d[1];
        ry->p[2] = ry->p[2] + s * d[2];
    }
}

/* Locate the (i,j) column of a spherical position. */
static void locate_column(const orc_grid *g, const double p[3], int *i, int *j)
{
    double lat = atan2(p[2], sqrt(p[0] * p[0] + p[1] * p[1]));
    double lon = atan2(p[1], p[0]);
    *j = edge_find(g->lat, g->nlat, lat);
    *i = edge_find(g->lon, g->nlon, lon);
}

/* Exported for the brute-force geometry pin: trace a ray from p (in cell
 * i,j,k, entry face ef) to the boundary, recording cells and path lengths.
 * Returns the number of segments (<= cap) and the termination code.        */
int64_t orc_trace_segments(const orc_grid *g, const double p0[3], const double d[3],
                           int64_t i, int64_t j, int64_t k, int64_t ef, int64_t cap,
                           int64_t *cells, double *lens, int64_t *term)
{
    orc_ray ry = {{p0[0], p0[1], p0[2]}, (int)i, (int)j, (int)k, (int)ef};
    int64_t n = 0;
    *term = T_LOST;
    while (n < cap) {
        double s;
        int f = exit_distance(g, &ry, d, &s);
        if (f == F_NONE) { *term = T_LOST; return n; }
        cells[n] = cell_index(g, ry.i, ry.j, ry.k);
        lens[n] = s;
        ++n;
        advance(g, &ry, d, s);
        cross_face(g, &ry, f);
        if (ry.k >= g->nlay) { *term = T_ESCAPE; return n; }
        if (ry.k < 0) { *term = T_SURFACE; return n; }
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Opacity gathers.                                                         */
/* ------------------------------------------------------------------------ */

/* Bracket x on an increasing grid: clamped, lower index and weight. */
static void bracket(const double *gx, int64_t n, double x, int *i0, int *i1, double *t)
{
    if (n == 1) { *i0 = 0; *i1 = 0; *t = 0.0; return; }
    if (x <= gx[0]) { *i0 = 0; *i1 = 1; *t = 0.0; return; }
    if (x >= gx[n - 1]) { *i0 = (int)n - 2; *i1 = (int)n - 1; *t = 1.0; return; }
    int m = 0;
    for (int64_t q = 0; q < n - 1; ++q)
        if (gx[q] <= x) m = (int)q;
    *i0 = m;
    *i1 = m + 1;
    *t = (x - gx[m]) / (gx[m + 1] - gx[m]);
}

/* Bilinear interpolation in (T, ln P) on ln kappa (kappa^w product form; a
 * zero kappa at a corner with positive weight gives zero).                 */
static double interp_tp(const float *tab, int64_t nP, int iT0, int iT1, double t,
                        int iP0, int iP1, double u)
{
    double w[4] = {(1.0 - t) * (1.0 - u), (1.0 - t) * u, t * (1.0 - u), t * u};
    int64_t idx[4] = {(int64_t)iT0 * nP + iP0, (int64_t)iT0 * nP + iP1,
                      (int64_t)iT1 * nP + iP0, (int64_t)iT1 * nP + iP1};
    double acc = 0.0;
    for (int q = 0; q < 4; ++q) {
        if (w[q] > 0.0) {
            double kv = (double)tab[idx[q]];
            if (kv <= 0.0) return 0.0;
            acc = acc + w[q] * log(kv);
        }
    }
    return exp(acc);
}

/* Correlated-k gather for one (band, g): per cell alpha_ext [1/cm],
 * alpha_abs, single-scattering albedo omega, gas scattering probability
 * P_gas and cloud asymmetry g.  kappa_abs from the pre-mixed k-table
 * interpolated to the cell (T, P); Rayleigh and cloud terms at the band
 * centre (Sect. 7).  tab points at kappa[band][g][T][P].                  */
void orc_ck_optics(int64_t ncell, const float *T, const float *P, const double *rho,
                   const float *cld_ksca, const float *cld_kabs, const float *cld_g,
                   int64_t nT, int64_t nP, const double *T_grid, const double *P_grid,
                   const float *tab, double k_ray,
                   double *a_ext, double *a_abs, double *omega, double *p_gas, double *g_cld)
{
    double *lnP = (double *)malloc(sizeof(double) * nP);
    for (int64_t q = 0; q < nP; ++q) lnP[q] = log(P_grid[q]);
    for (int64_t c = 0; c < ncell; ++c) {
        int iT0, iT1, iP0, iP1;
        double t, u;
        bracket(T_grid, nT, (double)T[c], &iT0, &iT1, &t);
        bracket(lnP, nP, log((double)P[c]), &iP0, &iP1, &u);
        double kg = interp_tp(tab, nP, iT0, iT1, t, iP0, iP1, u);
        double ks = cld_ksca ? (double)cld_ksca[c] : 0.0;
        double ka = cld_kabs ? (double)cld_kabs[c] : 0.0;
        double kab = kg + ka;
        double ksc = k_ray + ks;
        double kext = kab + ksc;
        a_ext[c] = rho[c] * kext;
        a_abs[c] = rho[c] * kab;
        omega[c] = kext > 0.0 ? ksc / kext : 0.0;
        p_gas[c] = ksc > 0.0 ? k_ray / ksc : 1.0;
        g_cld[c] = cld_g ? (double)cld_g[c] : 0.0;
    }
    free(lnP);
}

/* Line-of-sight velocity of each cell centre toward observer direction o:
 * v_LOS = -(v . o), with v = u e_E + v e_N + w e_r + Omega z x r (the wind and
 * solid-body rotation of the v_LOS equation, written in vector form; positive
 * is receding).  The result is the fractional index shift
 * ln(1 - v_LOS/c)/dlnlam of lambda_eff = lambda_0 (1 - v_LOS/c).            */
void orc_doppler_shift(const orc_grid *g, const float *u, const float *v, const float *w,
                       double omega_rot, const double o[3], double dlnlam, double *shift)
{
    for (int64_t k = 0; k < g->nlay; ++k)
        for (int64_t j = 0; j < g->nlat; ++j)
            for (int64_t i = 0; i < g->nlon; ++i) {
                int64_t c = cell_index(g, (int)i, (int)j, (int)k);
                double rc = 0.5 * (g->r[k] + g->r[k + 1]);
                double th = 0.5 * (g->lat[j] + g->lat[j + 1]);
                double ph = 0.5 * (g->lon[i] + g->lon[i + 1]);
                double eE[3] = {-sin(ph), cos(ph), 0.0};
                double eN[3] = {-sin(th) * cos(ph), -sin(th) * sin(ph), cos(th)};
                double eR[3] = {cos(th) * cos(ph), cos(th) * sin(ph), sin(th)};
                double uu = u ? (double)u[c] : 0.0, vv = v ? (double)v[c] : 0.0, ww = w ? (double)w[c] : 0.0;
                double ue = uu + omega_rot * rc * cos(th);
                double vel[3];
                for (int q = 0; q < 3; ++q) vel[q] = ue * eE[q] + vv * eN[q] + ww * eR[q];
                double vlos = -(vel[0] * o[0] + vel[1] * o[1] + vel[2] * o[2]);
                shift[c] = log1p(-vlos / ORC_C) / dlnlam;
            }
}

/* High-resolution gather at table wavelength index n: kappa interpolated at
 * the Doppler shifted effective wavelength (linear in kappa between the two
 * neighbouring table wavelengths of the log-uniform grid; bilinear (T, ln P)
 * on ln kappa at each), plus Rayleigh at the rest wavelength.  Lines are
 * pure absorbers.  tab is kappa[lam][T][P].                               */
void orc_hires_optics(int64_t ncell, const float *T, const float *P, const double *rho,
                      const double *shift, int64_t nlam, int64_t nT, int64_t nP,
                      const double *T_grid, const double *P_grid, const float *tab,
                      int64_t n, double k_ray,
                      double *a_ext, double *a_abs, double *omega, double *p_gas, double *g_cld)
{
    double *lnP = (double *)malloc(sizeof(double) * nP);
    for (int64_t q = 0; q < nP; ++q) lnP[q] = log(P_grid[q]);
    for (int64_t c = 0; c < ncell; ++c) {
        int iT0, iT1, iP0, iP1;
        double t, uu;
        bracket(T_grid, nT, (double)T[c], &iT0, &iT1, &t);
        bracket(lnP, nP, log((double)P[c]), &iP0, &iP1, &uu);
        double x = (double)n + (shift ? shift[c] : 0.0);
        int64_t n0;
        double fr;
        if (nlam == 1) { n0 = 0; fr = 0.0; }
        else if (x <= 0.0) { n0 = 0; fr = 0.0; }
        else if (x >= (double)(nlam - 1)) { n0 = nlam - 2; fr = 1.0; }
        else { n0 = (int64_t)floor(x); fr = x - (double)n0; }
        double k0 = interp_tp(tab + n0 * nT * nP, nP, iT0, iT1, t, iP0, iP1, uu);
        double kl = k0;
        if (nlam > 1) {
            double k1 = interp_tp(tab + (n0 + 1) * nT * nP, nP, iT0, iT1, t, iP0, iP1, uu);
            kl = (1.0 - fr) * k0 + fr * k1;
        }
        double kext = kl + k_ray;
        a_ext[c] = rho[c] * kext;
        a_abs[c] = rho[c] * kl;
        omega[c] = kext > 0.0 ? k_ray / kext : 0.0;
        p_gas[c] = 1.0;
        g_cld[c] = 0.0;
    }
    free(lnP);
}

/* ------------------------------------------------------------------------ */
/* Emission sources (Sect. 5.3 L_i; Sect. 4.3 hybrid biasing; Sect. 4.6     */
/* vertical tau cut).                                                       */
/* ------------------------------------------------------------------------ */
double orc_planck(double lam_cm, double T)
{
    double x = ORC_H * ORC_C / (lam_cm * ORC_KB * T);
    return 2.0 * ORC_H * ORC_C * ORC_C / pow(lam_cm, 5.0) / expm1(x);
}

/* L_i = 4 pi V_i alpha_abs,i B_lambda(T_i), zero for cells whose column
 * extinction optical depth from the top of the atmosphere down to the cell's
 * top face exceeds tau_vert; q_i = (1 - xi) L_i / L_tot + xi / N_emit over
 * emitting cells; cdf = running sum of q in cell order; wbirth = (L_i/L_tot)
 * / q_i.  Returns L_tot (erg/s/cm).  info[0] = N_emit.                    */
double orc_emission_sources(const orc_grid *g, const float *T, const double *a_ext,
                            const double *a_abs, double lam_cm, double tau_vert, double xi,
                            double *L, double *cdf, double *wbirth, int64_t *info)
{
    int64_t ncell = g->nlon * g->nlat * g->nlay;
    for (int64_t j = 0; j < g->nlat; ++j)
        for (int64_t i = 0; i < g->nlon; ++i) {
            double tau = 0.0;
            for (int64_t k = g->nlay - 1; k >= 0; --k) {
                int64_t c = cell_index(g, (int)i, (int)j, (int)k);
                double vol = (pow(g->r[k + 1], 3.0) - pow(g->r[k], 3.0)) / 3.0 *
                             (sin(g->lat[j + 1]) - sin(g->lat[j])) * (g->lon[i + 1] - g->lon[i]);
                double Li = 4.0 * ORC_PI * vol * a_abs[c] * orc_planck(lam_cm, (double)T[c]);
                L[c] = (tau > tau_vert) ? 0.0 : Li;
                tau = tau + a_ext[c] * (g->r[k + 1] - g->r[k]);
            }
        }
    double Ltot = 0.0;
    int64_t nemit = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        Ltot = Ltot + L[c];
        if (L[c] > 0.0) nemit++;
    }
    double run = 0.0;
    for (int64_t c = 0; c < ncell; ++c) {
        double q = 0.0;
        if (L[c] > 0.0) q = (1.0 - xi) * L[c] / Ltot + xi / (double)nemit;
        run = run + q;
        cdf[c] = run;
        wbirth[c] = (L[c] > 0.0) ? (L[c] / Ltot) / q : 0.0;
    }
    info[0] = nemit;
    return Ltot;
}

/* ------------------------------------------------------------------------ */
/* Stellar limb darkening (Sect. 5.1.1): I(mu)/I(1) on the stellar disk,    */
/* mu the cosine of the zenith angle on the stellar surface.  Laws:         */
/* 0 none, 1 linear, 2 quadratic (Kopal), 3 square-root, 4 logarithmic,     */
/* 5 exponential, 6 power-2.                                                */
/* ------------------------------------------------------------------------ */
double orc_limb_darkening(int64_t law, double c1, double c2, double mu)
{
    double x = 1.0 - mu;
    switch (law) {
    case 1: return 1.0 - c1 * x;
    case 2: return 1.0 - c1 * x - c2 * x * x;
    case 3: return 1.0 - c1 * x - c2 * (1.0 - sqrt(mu));
    case 4: return 1.0 - c1 * x - c2 * (mu > 0.0 ? mu * log(mu) : 0.0);
    case 5: return 1.0 - c1 * x - c2 / (1.0 - exp(mu));
    case 6: return 1.0 - c1 * (1.0 - pow(mu, c2));
    default: return 1.0;
    }
}

/* Weight of the stellar light behind sky-plane point (y, z) of the planet's
 * frame: the point lies at (transit_y + y, transit_z + z) on the stellar
 * disk; off the disk there is no light.                                    */
double orc_chord_limb_weight(int64_t law, double c1, double c2, double ty, double tz, double r_star,
                             double y, double z)
{
    if (law == 0) return 1.0;
    double sy = ty + y, sz = tz + z;
    double q = (sy * sy + sz * sz) / (r_star * r_star);
    if (!(q < 1.0)) return 0.0;
    return orc_limb_darkening(law, c1, c2, sqrt(1.0 - q));
}

/* ------------------------------------------------------------------------ */
/* Transport (Sect. 2, 3, 4).                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t seed;
    uint64_t n_packets;
    uint64_t packet0;     /* first packet id */
    int64_t mode;         /* 0 albedo (spherical disk or slab), 1 emission */
    int64_t scattering;   /* 0: no multiple scattering */
    int64_t absorption;   /* 0 survival biasing, 1 continuous absorption */
    int64_t tag;          /* XORed into the high key word */
    int64_t max_events;
    int64_t max_cross;    /* per ray segment walk */
    int64_t n_obs;        /* slab albedo with n_obs == 0: backscatter */
    double rr_threshold;
    double rr_survive;
    double tau_peel_max;
    double mu0;           /* slab incidence cosine; <= 0: uniform over disk */
    int64_t cloud_phase;  /* 0 Henyey-Greenstein, 1 two-term HG, 2 Draine */
    double surface_albedo; /* 0: absorbing lower boundary; > 0: Lambert surface */
    /* transmission with multiple scattering (mode 2) */
    double omega_star;    /* solid angle pi (R_star / a)^2 of the stellar beam at the planet */
    int64_t ld_law;       /* stellar limb darkening, see orc_limb_darkening */
    double ld_c1, ld_c2;
    double transit_y, transit_z; /* planet centre on the stellar disk (sky plane), cm */
    double r_star;
    double draine_alpha;  /* alpha of Draine's function (cloud_phase 2) */
    int64_t forced;       /* forced interaction: 0 off, 1 forced scattering, 2 path-length
                           * stretching, 3 hybrid (equal mixture of 1 and 2) */
    int64_t forced_first; /* 1: only the packet's first flight is forced */
} orc_params;

typedef struct {
    const double *a_ext, *a_abs, *omega, *p_gas, *g_cld;
} orc_optics;

/* counters per packet */
enum { K_ESC = 0, K_SURF, K_ABS, K_RR, K_CAP, K_LOST, K_NINT, K_NCROSS, K_NCAPPED, K_NLOST, K_W0, NK };

/* Walk a ray through the grid until an interaction at optical depth tau
 * (measured in 'a'), escape, the surface or the crossing cap.  With
 * continuous absorption the weight is reduced by exp(-alpha_abs s) on every
 * path element and the removed weight is added to *absorbed.               */
static int walk_flight(const orc_grid *g, const orc_optics *op, orc_ray *ry, const double d[3],
                       double tau, int cont, double *W, double *absorbed, int64_t max_cross,
                       int64_t *ncross)
{
    int64_t nc = 0;
    for (;;) {
        double s;
        int f = exit_distance(g, ry, d, &s);
        int64_t c = cell_index(g, ry->i, ry->j, ry->k);
        double a = cont ? (op->a_ext[c] - op->a_abs[c]) : op->a_ext[c];
        if (f == F_NONE && !(a > 0.0)) { *ncross += nc; return T_LOST; }
        if (a > 0.0 && tau < a * s) {
            double ds = tau / a;
            if (cont) {
                double wn = *W * exp(-op->a_abs[c] * ds);
                *absorbed = *absorbed + (*W - wn);
                *W = wn;
            }
            advance(g, ry, d, ds);
            ry->ef = F_NONE;
            *ncross += nc;
            return T_INTERACT;
        }
        tau = tau - a * s;
        if (cont) {
            double wn = *W * exp(-op->a_abs[c] * s);
            *absorbed = *absorbed + (*W - wn);
            *W = wn;
        }
        advance(g, ry, d, s);
        cross_face(g, ry, f);
        nc++;
        if (ry->k >= g->nlay) { *ncross += nc; return T_ESCAPE; }
        if (ry->k < 0) { *ncross += nc; return T_SURFACE; }
        if (nc >= max_cross) { *ncross += nc; return T_LOST; }
    }
}

/* Optical depth from an event point to the top of the atmosphere along o.
 * Returns +inf for rays that reach the surface, stall, or exceed tau_cut. */
static double peel_tau(const orc_grid *g, const orc_optics *op, const orc_ray *start,
                       const double o[3], double tau_cut, int64_t max_cross, int64_t *ncross)
{
    if (g->geom == 1 && !(o[2] > 0.0)) return INFINITY;
    orc_ray ry = *start;
    ry.ef = F_NONE;
    double tau = 0.0;
    int64_t nc = 0;
    for (;;) {
        double s;
        int f = exit_distance(g, &ry, o, &s);
        if (f == F_NONE) { *ncross += nc; return INFINITY; }
        int64_t c = cell_index(g, ry.i, ry.j, ry.k);
        tau = tau + op->a_ext[c] * s;
        advance(g, &ry, o, s);
        cross_face(g, &ry, f);
        nc++;
        if (tau > tau_cut) { *ncross += nc; return INFINITY; }
        if (ry.k >= g->nlay) { *ncross += nc; return tau; }
        if (ry.k < 0) { *ncross += nc; return INFINITY; }
        if (nc >= max_cross) { *ncross += nc; return INFINITY; }
    }
}

/* Optical depth along d from the event point to the edge of the grid (the
 * extra ray trace of a forced interaction): *to_surface tells whether the
 * path ends on the planet (or the slab's floor) rather than at the top;
 * infinite when the walk fails or meets the crossing cap.                  */
static double path_tau(const orc_grid *g, const orc_optics *op, const orc_ray *start, const double d[3],
                       int64_t max_cross, int64_t *ncross, int *to_surface)
{
    orc_ray ry = *start;
    ry.ef = F_NONE;
    double tau = 0.0;
    int64_t nc = 0;
    for (;;) {
        double s;
        int f = exit_distance(g, &ry, d, &s);
        if (f == F_NONE) { *ncross += nc; return INFINITY; }
        int64_t c = cell_index(g, ry.i, ry.j, ry.k);
        tau = tau + op->a_ext[c] * s;
        advance(g, &ry, d, s);
        cross_face(g, &ry, f);
        nc++;
        if (ry.k >= g->nlay) { *ncross += nc; *to_surface = 0; return tau; }
        if (ry.k < 0) { *ncross += nc; *to_surface = 1; return tau; }
        if (nc >= max_cross) { *ncross += nc; return INFINITY; }
    }
}

/* Per-event tallies besides the packet's peel-off sums (NULL members are
 * skipped):
 * - contribution functions (Sect. "Albedo and emission contribution
 *   functions"): every peel-off f is also added to the cell of the event that
 *   produced it, split into the thermal part (emission points) and the
 *   scattered part (interactions): cf[(o * 2 + part) * ncell + cell];
 * - images (Sect. 2, images from the peel-offs): f is added to the pixel of
 *   the event point projected on the sky plane of observer o, whose
 *   horizontal and vertical unit vectors are axes[o][0], axes[o][1]; pixels
 *   cover [-half, half]^2: img[(o * npix + row) * npix + column].          */
typedef struct {
    double *cf;
    double *img;
    int64_t npix;
    double half;
    const double *axes;
} orc_tally;

static int64_t pixel_of(double x, double half, int64_t npix)
{
    int64_t q = (int64_t)floor((x + half) / (2.0 * half) * (double)npix);
    return q < 0 ? 0 : (q >= npix ? npix - 1 : q);
}

static void tally_add(const orc_tally *tl, int64_t ncell, int o, int part, int64_t cell, const double p[3],
                      double f)
{
    if (!tl) return;
    if (tl->cf) {
#ifdef _OPENMP
#pragma omp atomic
#endif
        tl->cf[((int64_t)o * 2 + part) * ncell + cell] += f;
    }
    if (tl->img) {
        const double *eh = tl->axes + 6 * o, *ev = eh + 3;
        int64_t col = pixel_of(p[0] * eh[0] + p[1] * eh[1] + p[2] * eh[2], tl->half, tl->npix);
        int64_t row = pixel_of(p[0] * ev[0] + p[1] * ev[1] + p[2] * ev[2], tl->half, tl->npix);
#ifdef _OPENMP
#pragma omp atomic
#endif
        tl->img[((int64_t)o * tl->npix + row) * tl->npix + col] += f;
    }
}

/* One packet history.  F[o] receives its peel-off sum per observer. */
static void run_packet(const orc_grid *g, const orc_optics *op, const orc_params *pr,
                       const double *obs, const double *cdf, const double *wbirth, int64_t ncell,
                       double r_toa, uint64_t pid, double wmul, double *F, double *K, const orc_tally *tl)
{
    uint32_t tag = (uint32_t)pr->tag;
    int nobs = (int)pr->n_obs;
    int slab_back = (g->geom == 1 && nobs == 0);
    int nout = slab_back ? 1 : nobs;
    double oback[3] = {0.0, 0.0, 0.0};
    for (int o = 0; o < nout; ++o) F[o] = 0.0;
    for (int q = 0; q < NK; ++q) K[q] = 0.0;

    orc_ray ry;
    double d[3];
    double W, W0;
    double ua, ub;
    int64_t ncross = 0;

    if (pr->mode == 0) {
        /* albedo: unit-weight packets enter at the top along -x (star at +x) */
        orc_draw(pr->seed, tag, pid, 0, 0, &ua, &ub);
        if (g->geom == 1) {
            double mu0 = pr->mu0 > 0.0 ? pr->mu0 : sqrt(1.0 - ua);
            d[0] = sqrt(fmax(1.0 - mu0 * mu0, 0.0));
            d[1] = 0.0;
            d[2] = -mu0;
            oback[0] = -d[0]; oback[1] = 0.0; oback[2] = mu0;
            ry.p[0] = 0.0; ry.p[1] = 0.0; ry.p[2] = g->r[g->nlay];
            ry.i = 0; ry.j = 0; ry.k = (int)g->nlay - 1; ry.ef = F_OUT;
        } else {
            double rho = r_toa * sqrt(ua);
            double a = 2.0 * ORC_PI * ub;
            double y = rho * cos(a), z = rho * sin(a);
            double x = sqrt(fmax(r_toa * r_toa - y * y - z * z, 0.0));
            ry.p[0] = x; ry.p[1] = y; ry.p[2] = z;
            d[0] = -1.0; d[1] = 0.0; d[2] = 0.0;
            ry.k = (int)g->nlay - 1;
            locate_column(g, ry.p, &ry.i, &ry.j);
            ry.ef = F_OUT;
        }
        W = wmul;
    } else if (pr->mode == 2) {
        /* transmission with multiple scattering (Sect. 5.1): the packet
         * enters at a random point of the annulus R0 <= b <= R_TOA (block 0 of
         * the birth event: slot a gives b uniformly, slot b the angle) with
         * the stellar beam along -x; its weight is b (the factor of the
         * estimator) times the limb-darkening fraction of the stellar light
         * behind its chord.  The first peel-off, along the chord toward the
         * observer, is the directly transmitted light.                     */
        orc_draw(pr->seed, tag, pid, 0, 0, &ua, &ub);
        double r0 = g->r[0];
        double b = r0 + ua * (r_toa - r0);
        double al = 2.0 * ORC_PI * ub;
        ry.p[0] = sqrt(fmax(r_toa * r_toa - b * b, 0.0));
        ry.p[1] = b * cos(al);
        ry.p[2] = b * sin(al);
        d[0] = -1.0; d[1] = 0.0; d[2] = 0.0;
        ry.k = (int)g->nlay - 1;
        locate_column(g, ry.p, &ry.i, &ry.j);
        ry.ef = F_OUT;
        W = b * orc_chord_limb_weight(pr->ld_law, pr->ld_c1, pr->ld_c2, pr->transit_y, pr->transit_z,
                                      pr->r_star, ry.p[1], ry.p[2]);
        for (int o = 0; o < nobs; ++o) {
            double tau = peel_tau(g, op, &ry, obs + 3 * o, pr->tau_peel_max, pr->max_cross, &ncross);
            F[o] = F[o] + W * exp(-tau);
        }
    } else {
        /* emission: cell by the biased CDF, uniform position in the cell's
         * volume, isotropic direction, weight (L_i/L_tot)/q_i              */
        if (!(cdf[ncell - 1] > 0.0)) return; /* nothing emits */
        double u0a, u0b, u1a, u1b, u2a, u2b;
        orc_draw(pr->seed, tag, pid, 0, 0, &u0a, &u0b);
        orc_draw(pr->seed, tag, pid, 0, 1, &u1a, &u1b);
        orc_draw(pr->seed, tag, pid, 0, 2, &u2a, &u2b);
        double target = u0a * cdf[ncell - 1];
        int64_t c = 0;
        while (!(cdf[c] > target)) c++; /* smallest c with cdf[c] > target */
        int i = (int)(c % g->nlon);
        int j = (int)((c / g->nlon) % g->nlat);
        int k = (int)(c / (g->nlon * g->nlat));
        double rk3 = g->r[k] * g->r[k] * g->r[k];
        double rk13 = g->r[k + 1] * g->r[k + 1] * g->r[k + 1];
        double r = cbrt(rk3 + u0b * (rk13 - rk3));
        double sl0 = sin(g->lat[j]), sl1 = sin(g->lat[j + 1]);
        double sl = sl0 + u1a * (sl1 - sl0);
        double cl = sqrt(fmax(1.0 - sl * sl, 0.0));
        double lon = g->lon[i] + u1b * (g->lon[i + 1] - g->lon[i]);
        ry.p[0] = r * cl * cos(lon);
        ry.p[1] = r * cl * sin(lon);
        ry.p[2] = r * sl;
        ry.i = i; ry.j = j; ry.k = k; ry.ef = F_NONE;
        double mu = 2.0 * u2a - 1.0;
        double sp = sqrt(fmax(1.0 - mu * mu, 0.0));
        double psi = 2.0 * ORC_PI * u2b;
        d[0] = sp * cos(psi);
        d[1] = sp * sin(psi);
        d[2] = mu;
        W = wbirth[c] * wmul;
        /* initial peel-off from the emission point */
        for (int o = 0; o < nobs; ++o) {
            double tau = peel_tau(g, op, &ry, obs + 3 * o, pr->tau_peel_max, pr->max_cross, &ncross);
            double f = W * exp(-tau) / (4.0 * ORC_PI);
            F[o] = F[o] + f;
            tally_add(tl, ncell, o, 0, c, ry.p, f);
        }
    }
    W0 = W;
    K[K_W0] = W0;

    if (pr->mode >= 1 && !pr->scattering) {
        K[K_ESC] += W; /* weight leaves with its initial peel-off only */
        K[K_NCROSS] = (double)ncross;
        return;
    }

    int cont = pr->absorption == 1;
    for (uint32_t e = 1;; ++e) {
        double tau, usel;
        orc_draw(pr->seed, tag, pid, e, 0, &ua, &usel);
        tau = -log(ua);
        if (pr->forced != 0 && (pr->forced_first == 0 || e == 1)) {
            /* the extra ray trace: optical depth to the edge of the grid
             * along d; the unscattered fraction is booked where the path ends */
            int to_surf = 0;
            double tp = path_tau(g, op, &ry, d, pr->max_cross, &ncross, &to_surf);
            if (tp > 0.0 && tp < INFINITY) {
                double zc, zd, wf;
                orc_draw(pr->seed, tag, pid, e, 34, &zc, &zd);  /* hybrid component: block 34, slot a */
                tau = orc_forced_tau(pr->forced, tp, ua, zc, &wf);
                if (to_surf) K[K_SURF] += W * exp(-tp);
                else K[K_ESC] += W * exp(-tp);
                W = W * wf;
            }
        }
        int term = walk_flight(g, op, &ry, d, tau, cont, &W, &K[K_ABS], pr->max_cross, &ncross);
        if (term == T_ESCAPE) { K[K_ESC] += W; break; }
        if (term == T_SURFACE && !(pr->surface_albedo > 0.0)) { K[K_SURF] += W; break; }
        if (term == T_LOST) { K[K_LOST] += W; K[K_NLOST] += 1.0; break; }
        K[K_NINT] += 1.0;
        if (term == T_SURFACE) {
            /* Lambert surface (Sect. 3, Lambertian surface scattering): a
             * peel-off f = W A_s max(n.o, 0)/pi e^{-tau} toward every observer,
             * then W <- W A_s and a new direction at cos(theta) = sqrt(zeta)
             * (block 1, slot a) from the outward normal n, azimuth 2 pi zeta'
             * (block 1, slot b).  The packet stays in the lowest layer,
             * entered through its inner face. */
            ry.k = 0;
            ry.ef = F_IN;
            double nrm[3] = {0.0, 0.0, 1.0};
            if (g->geom != 1) {
                double rr = sqrt(ry.p[0] * ry.p[0] + ry.p[1] * ry.p[1] + ry.p[2] * ry.p[2]);
                nrm[0] = ry.p[0] / rr; nrm[1] = ry.p[1] / rr; nrm[2] = ry.p[2] / rr;
            }
            int64_t c = cell_index(g, ry.i, ry.j, 0);
            for (int o = 0; o < nout; ++o) {
                const double *ov = slab_back ? oback : obs + 3 * o;
                double mu = nrm[0] * ov[0] + nrm[1] * ov[1] + nrm[2] * ov[2];
                double f = 0.0;
                if (mu > 0.0) {
                    double t = peel_tau(g, op, &ry, ov, pr->tau_peel_max, pr->max_cross, &ncross);
                    f = W * pr->surface_albedo * (mu / ORC_PI) * exp(-t);
                    if (pr->mode == 2) f = f * pr->omega_star;
                }
                F[o] = F[o] + f;
                tally_add(tl, ncell, o, 1, c, ry.p, f);
            }
            K[K_SURF] += W * (1.0 - pr->surface_albedo);
            W = W * pr->surface_albedo;
            double u1a, u1b;
            orc_draw(pr->seed, tag, pid, e, 1, &u1a, &u1b);
            d[0] = nrm[0]; d[1] = nrm[1]; d[2] = nrm[2];
            orc_rotate(d, sqrt(u1a), 2.0 * ORC_PI * u1b);
        } else {
        /* interaction in cell c */
        int64_t c = cell_index(g, ry.i, ry.j, ry.k);
        double om = op->omega[c], pg = op->p_gas[c], gc = op->g_cld[c];
        double Gd = pr->cloud_phase == 2 ? orc_draine_G(gc, pr->draine_alpha) : 0.0;
        for (int o = 0; o < nout; ++o) {
            const double *ov = slab_back ? oback : obs + 3 * o;
            double mu = d[0] * ov[0] + d[1] * ov[1] + d[2] * ov[2];
            double pc = pr->cloud_phase == 1 ? orc_phase_tthg(mu, gc)
                        : pr->cloud_phase == 2 ? orc_phase_draine(mu, Gd, pr->draine_alpha)
                                               : orc_phase_hg(mu, gc);
            double theta = (pg * orc_phase_rayleigh(mu) + (1.0 - pg) * pc) / (4.0 * ORC_PI);
            double t = peel_tau(g, op, &ry, ov, pr->tau_peel_max, pr->max_cross, &ncross);
            double f = cont ? W * theta * exp(-t) : W * om * theta * exp(-t);
            /* transmission: scattered light per steradian, over the beam's solid angle */
            if (pr->mode == 2) f = f * pr->omega_star;
            F[o] = F[o] + f;
            tally_add(tl, ncell, o, 1, c, ry.p, f);
        }
        if (!cont) {
            K[K_ABS] += W * (1.0 - om);
            W = W * om;
        }
        double u1a, u1b;
        orc_draw(pr->seed, tag, pid, e, 1, &u1a, &u1b);
        double mu;
        if (usel < pg) {
            mu = orc_sample_rayleigh(u1a);
        } else if (pr->cloud_phase == 1) {
            double u2a, u2b;  /* the lobe: block 2, slot b */
            orc_draw(pr->seed, tag, pid, e, 2, &u2a, &u2b);
            mu = orc_sample_tthg(u2b, u1a, gc);
        } else if (pr->cloud_phase == 2) {
            /* Draine: candidate 0 from block 1 slot a, accepted by block 2
             * slot b; candidate k >= 1 from block 2 + k (slots a, b) */
            double za[ORC_DRAINE_MAXC], zc[ORC_DRAINE_MAXC], u2a;
            za[0] = u1a;
            orc_draw(pr->seed, tag, pid, e, 2, &u2a, &zc[0]);
            for (int k = 1; k < ORC_DRAINE_MAXC; ++k) orc_draw(pr->seed, tag, pid, e, (uint32_t)(2 + k), &za[k], &zc[k]);
            mu = orc_sample_draine(za, zc, ORC_DRAINE_MAXC, Gd, pr->draine_alpha);
        } else {
            mu = orc_sample_hg(u1a, gc);
        }
        orc_rotate(d, mu, 2.0 * ORC_PI * u1b);
        }
        if (W < pr->rr_threshold * W0) {
            double u2a, u2b;
            orc_draw(pr->seed, tag, pid, e, 2, &u2a, &u2b);
            if (u2a < pr->rr_survive) {
                double wn = W / pr->rr_survive;
                K[K_RR] -= (wn - W);
                W = wn;
            } else {
                K[K_RR] += W;
                W = 0.0;
                break;
            }
        }
        if ((int64_t)e >= pr->max_events) { K[K_CAP] += W; K[K_NCAPPED] += 1.0; break; }
    }
    K[K_NCROSS] = (double)ncross;
}

/* Run n_packets histories.  F_out[n][nout], K_out[n][NK] per packet (the
 * caller sums them in packet order).  obs: n_obs unit vectors.  tl (may be
 * NULL): per-event tallies, added to.                                      */
int64_t orc_transport(const orc_grid *g, const orc_optics *op, const orc_params *pr,
                      const double *obs, const double *cdf, const double *wbirth, double r_toa,
                      double *F_out, double *K_out, const orc_tally *tl, int64_t nthreads)
{
    int64_t ncell = g->nlon * g->nlat * g->nlay;
    int nout = (g->geom == 1 && pr->n_obs == 0) ? 1 : (int)pr->n_obs;
    int64_t n = (int64_t)pr->n_packets;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads((int)nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t q = 0; q < n; ++q) {
        run_packet(g, op, pr, obs, cdf, wbirth, ncell, r_toa, pr->packet0 + (uint64_t)q, 1.0,
                   F_out + q * nout, K_out + q * NK, tl);
    }
    return nout;
}

/* Per-packet g-ordinate sampling (Sect. "G-ordinance biasing"): one band,
 * ng g-ordinates with their own optics (and emission sources).  Packet pid
 * draws u from block 3, slot a of its birth event and takes the smallest g
 * whose cumulative sampling weight q exceeds u times the total; its history
 * then runs with that g's optics and sources, all weights multiplied by
 * wfac[g] = p(g)/q(g).  q: unnormalised sampling weights [ng]; optics,
 * cdf, wbirth: arrays of ng pointers (cdf/wbirth NULL for albedo).        */
int64_t orc_transport_gsampled(const orc_grid *g, const orc_optics *ops, int64_t ng, const orc_params *pr,
                               const double *obs, const double *const *cdfs, const double *const *wbirths,
                               const double *q, const double *wfac, double r_toa, double *F_out,
                               double *K_out, int64_t *g_out, int64_t nthreads)
{
    int64_t ncell = g->nlon * g->nlat * g->nlay;
    int nout = (g->geom == 1 && pr->n_obs == 0) ? 1 : (int)pr->n_obs;
    int64_t n = (int64_t)pr->n_packets;
    double qtot = 0.0;
    for (int64_t h = 0; h < ng; ++h) qtot = qtot + q[h];
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads((int)nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (int64_t i = 0; i < n; ++i) {
        uint64_t pid = pr->packet0 + (uint64_t)i;
        double ua, ub;
        orc_draw(pr->seed, (uint32_t)pr->tag, pid, 0, 3, &ua, &ub);
        double target = ua * qtot, cum = 0.0;
        int64_t gi = ng - 1;
        for (int64_t h = 0; h < ng; ++h) {
            cum = cum + q[h];
            if (cum > target) { gi = h; break; }
        }
        if (g_out) g_out[i] = gi;
        run_packet(g, &ops[gi], pr, obs, cdfs ? cdfs[gi] : NULL, wbirths ? wbirths[gi] : NULL, ncell, r_toa, pid,
                   wfac[gi], F_out + i * nout, K_out + i * NK, NULL);
    }
    return nout;
}

int64_t orc_num_counters(void) { return NK; }

int64_t orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Transmission (Sect. 5.1): chords along -x through the limb, stratified   */
/* jittered (b, alpha) samples; per chord tau(lambda) = sum alpha s and the */
/* estimator term (1 - exp(-tau)) b.                                        */
/* ------------------------------------------------------------------------ */
/* value[c][s] = (1 - exp(-tau_cs)) b_c for chord c and spectral slot s;
 * alpha is [n_spec][ncell].  tau_out (optional) = tau_cs.                 */
void orc_transmission(const orc_grid *g, const double *alpha, int64_t n_spec, int64_t n_b,
                      int64_t n_alpha, uint64_t seed, int64_t tag, double r0, double r_toa,
                      const orc_params *ld, double *value, double *tau_out, int64_t nthreads)
{
    int64_t nch = n_b * n_alpha;
    int64_t cap = 64 * (g->nlay + g->nlat + g->nlon) + 64;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads((int)nthreads);
#pragma omp parallel
#endif
    {
        int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * cap);
        double *lens = (double *)malloc(sizeof(double) * cap);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t ch = 0; ch < nch; ++ch) {
            int64_t ib = ch / n_alpha, ia = ch % n_alpha;
            double ua, ub;
            orc_draw(seed, (uint32_t)tag, (uint64_t)ch, 0, 0, &ua, &ub);
            double b = r0 + ((double)ib + ua) * (r_toa - r0) / (double)n_b;
            double al = 2.0 * ORC_PI * ((double)ia + ub) / (double)n_alpha;
            double p[3] = {sqrt(fmax(r_toa * r_toa - b * b, 0.0)), b * cos(al), b * sin(al)};
            double d[3] = {-1.0, 0.0, 0.0};
            int i, j;
            locate_column(g, p, &i, &j);
            int64_t term;
            int64_t nseg = orc_trace_segments(g, p, d, i, j, g->nlay - 1, F_OUT, cap, cells, lens, &term);
            double wb = b * orc_chord_limb_weight(ld->ld_law, ld->ld_c1, ld->ld_c2, ld->transit_y,
                                                  ld->transit_z, ld->r_star, p[1], p[2]);
            for (int64_t s = 0; s < n_spec; ++s) {
                double tau = 0.0;
                for (int64_t q = 0; q < nseg; ++q)
                    tau = tau + alpha[s * (g->nlon * g->nlat * g->nlay) + cells[q]] * lens[q];
                if (term != T_ESCAPE) tau = INFINITY;
                value[ch * n_spec + s] = (1.0 - exp(-tau)) * wb;
                if (tau_out) tau_out[ch * n_spec + s] = tau;
            }
        }
        free(cells);
        free(lens);
    }
}
