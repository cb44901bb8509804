// HIP kernels of the photon-transport path for gfx950 (CDNA4, wave64).
//
// K1 ck_optics        correlated-k gather to per-cell extinction, albedo,
//                     gas-scattering probability (Sect. 7, pre-mixed tables
//                     interpolated to the T-p structure; continuum at the band
//                     centre)
// K2 doppler/hires    line-of-sight velocity and Doppler-shifted
//                     high-resolution opacity (Sect. 7, v_LOS and lambda_eff)
// (K3 emission sources and the batched K1/K2 of the transport: prep.hip)
// (K4 transport lives in transport.hip)
// K5 chords           transmission chord geometry and per-wavelength optical
//                     depth (Sect. 5.1)
// K6 reductions       deterministic fixed-order FP64 sums of block partials
//
// All FP64 arithmetic is written in the order of its definition and built
// with -ffp-contract=off so that results equal an independent FP64 CPU
// evaluation up to the last-bit differences of the math library.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "device_common.hpp"
#include "mcrt_internal.hpp"

namespace mcrt {
namespace {
using namespace dev;

// ---------------------------------------------------------------- K1
// R: type of the stored properties (double, or float for the mixed form; the
// arithmetic is FP64 either way and the result is rounded once on store).
template <typename R>
__global__ void __launch_bounds__(256) k_ck_optics(GridDev g, int ncell, const double* __restrict__ lnk_tab,
                                                   int nT, int nP, const double* __restrict__ T_grid,
                                                   const double* __restrict__ lnP_grid, double k_ray,
                                                   OpticsDev<R> out, int ext_stride)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    Bracket bt = bracket(T_grid, nT, (double)g.T[c]);
    Bracket bp = bracket(lnP_grid, nP, log((double)g.P[c]));
    double kg = interp_tp([&](int a, int b) { return lnk_tab[a * nP + b]; }, bt, bp);
    double ks = g.cld_ksca ? (double)g.cld_ksca[c] : 0.0;
    double ka = g.cld_kabs ? (double)g.cld_kabs[c] : 0.0;
    double kab = kg + ka;
    double ksc = k_ray + ks;
    double kext = kab + ksc;
    double rho = g.rho[c];
    out.a_ext[(size_t)c * ext_stride] = (R)(rho * kext);
    if (out.a_abs) {
        out.a_abs[c] = (R)(rho * kab);
        out.omega[c] = (R)(kext > 0.0 ? ksc / kext : 0.0);
        out.p_gas[c] = (R)(ksc > 0.0 ? k_ray / ksc : 1.0);
        out.g_cld[c] = (R)(g.cld_g ? (double)g.cld_g[c] : 0.0);
    }
}

// ---------------------------------------------------------------- K2
__global__ void __launch_bounds__(256) k_doppler_shift(GridDev g, double ox, double oy, double oz,
                                                       double dlnlam, double* __restrict__ shift)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    int ncell = g.nlon * g.nlat * g.nlay;
    if (c >= ncell) return;
    int i = c % g.nlon, j = (c / g.nlon) % g.nlat, k = c / (g.nlon * g.nlat);
    double rc = 0.5 * (g.r[k] + g.r[k + 1]);
    double th = 0.5 * (g.lat[j] + g.lat[j + 1]);
    double ph = 0.5 * (g.lon[i] + g.lon[i + 1]);
    double sth = sin(th), cth = cos(th), sph = sin(ph), cph = cos(ph);
    double eE0 = -sph, eE1 = cph, eE2 = 0.0;
    double eN0 = -sth * cph, eN1 = -sth * sph, eN2 = cth;
    double eR0 = cth * cph, eR1 = cth * sph, eR2 = sth;
    double uu = g.u ? (double)g.u[c] : 0.0, vv = g.v ? (double)g.v[c] : 0.0, ww = g.w ? (double)g.w[c] : 0.0;
    double ue = uu + g.omega_rot * rc * cth;
    double v0 = ue * eE0 + vv * eN0 + ww * eR0;
    double v1 = ue * eE1 + vv * eN1 + ww * eR1;
    double v2 = ue * eE2 + vv * eN2 + ww * eR2;
    double vlos = -(v0 * ox + v1 * oy + v2 * oz);
    shift[c] = log1p(-vlos / kC) / dlnlam;
}

// Bilinear ln-kappa in (T, ln P) from the four corner values l[] (order
// (i0,i0), (i0,i1), (i1,i0), (i1,i1)), already loaded: the same terms in the
// same order as interp_tp, a -inf corner with positive weight giving zero.
// FP64, and FP32 for the mixed form (whose stored extinction is FP32):
// table values, weights, weighted sum and exponential in single precision.
__device__ __forceinline__ double tp_vals(const double* l, const Bracket& bt, const Bracket& bp)
{
    const double t = bt.t, u = bp.t;
    const double w[4] = {(1.0 - t) * (1.0 - u), (1.0 - t) * u, t * (1.0 - u), t * u};
    double acc = 0.0;
    bool zero = false;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (w[q] > 0.0) {
            zero = zero || isinf(l[q]);
            acc = acc + w[q] * l[q];
        }
    return zero ? 0.0 : exp(acc);
}
__device__ __forceinline__ float tp_vals(const float* l, const Bracket& bt, const Bracket& bp)
{
    const float t = (float)bt.t, u = (float)bp.t;
    const float w[4] = {(1.0f - t) * (1.0f - u), (1.0f - t) * u, t * (1.0f - u), t * u};
    float acc = 0.0f;
    bool zero = false;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (w[q] > 0.0f) {
            zero = zero || isinf(l[q]);
            acc = fmaf(w[q], l[q], acc);
        }
    return zero ? 0.0f : __expf(acc);
}

// Table position n + shift split into the lower neighbour n0 and the
// fraction fr, clamped at the table ends.
__device__ __forceinline__ void hires_pos(int nlam, int n, double shift, int& n0, double& fr)
{
    const double x = (double)n + shift;
    if (nlam == 1) { n0 = 0; fr = 0.0; }
    else if (x <= 0.0) { n0 = 0; fr = 0.0; }
    else if (x >= (double)(nlam - 1)) { n0 = nlam - 2; fr = 1.0; }
    else { n0 = (int)floor(x); fr = x - (double)n0; }
}

// kappa at table position n0 + fr from the corner values a[] at n0 and b[]
// at n0 + 1, linear in kappa between the two wavelengths; R = float evaluates
// it in single precision (the fraction comes in FP64).
template <typename R>
__device__ __forceinline__ double hires_combine(const R* a, const R* b, const Bracket& bt, const Bracket& bp,
                                                double fr, int nlam)
{
    const R k0 = tp_vals(a, bt, bp);
    if (nlam == 1) return (double)k0;
    const R k1 = tp_vals(b, bt, bp);
    if constexpr (sizeof(R) == sizeof(float)) {
        const float f = (float)fr;
        return (double)fmaf(f, k1, (1.0f - f) * k0);
    } else {
        return (1.0 - fr) * k0 + fr * k1;
    }
}

// Each cell's (T, ln P) brackets in the opacity table, once per solve.
__global__ void __launch_bounds__(256) k_cell_tp(GridDev g, int ncell, int nT, int nP,
                                                 const double* __restrict__ T_grid,
                                                 const double* __restrict__ lnP_grid, CellTP* __restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const Bracket bt = bracket(T_grid, nT, (double)g.T[c]);
    const Bracket bp = bracket(lnP_grid, nP, log((double)g.P[c]));
    out[c] = CellTP{bt.i0, bt.i1, bp.i0, bp.i1, bt.t, bp.t};
}

constexpr int kAlphaCells = 2;  // cells per thread of the hi-res extinction block

// alpha[c * slot_stride + s] = rho (kappa_shifted(n_s) + k_ray(n_s)), n_s = nlist[s], s < nslot.
// Threads run slot-fastest so a wave reads consecutive wavelengths of the
// [T][P][lambda] table (lnk_tpl, in the extinction's type) and writes a
// contiguous row.
template <typename R>
__global__ void __launch_bounds__(256) k_hires_alpha_block(GridDev g, int ncell, const R* __restrict__ lnk_tpl,
                                                           int nlam, int nP, const CellTP* __restrict__ tp,
                                                           const double* __restrict__ k_ray,
                                                           const double* __restrict__ shift,
                                                           const int* __restrict__ nlist, int nslot,
                                                           int slot_stride, R* __restrict__ alpha)
{
    // thread (cell group, slot), kAlphaCells cells each, in passes whose
    // loads are in flight together: the cells' brackets, shifts and
    // densities; the four table corners at n0 of every cell; then the corners
    // at n0 + 1, which in the FP32 form are the next lane's values at its n0
    // whenever that lane has the same cells and the next table wavelength
    // (consecutive slots of one cell group), and loaded only where it has not
    // (the FP64 form loads them all).  A thread
    // past the end mirrors the last one (so every lane takes part in the
    // exchange) and stores nothing; a cell past the grid's end reads the last
    // cell and is dropped.
    const long long total = (long long)((ncell + kAlphaCells - 1) / kAlphaCells) * nslot;
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = t < total;
    const long long tc = live ? t : total - 1;
    const int grp = (int)(tc / nslot), s = (int)(tc % nslot);
    const int c0 = grp * kAlphaCells;
    const int n = nlist[s];
    const double kr = k_ray[n];
    CellTP q[kAlphaCells];
    double sh[kAlphaCells], rho[kAlphaCells];
#pragma unroll
    for (int u = 0; u < kAlphaCells; ++u) {
        const int c = c0 + u < ncell ? c0 + u : ncell - 1;
        q[u] = tp[c];
        sh[u] = shift ? shift[c] : 0.0;
        rho[u] = g.rho[c];
    }
    const int d = nlam == 1 ? 0 : 1;
    R a[kAlphaCells][4], b[kAlphaCells][4];
    int n0[kAlphaCells];
    double fr[kAlphaCells];
    size_t row[kAlphaCells][4];
#pragma unroll
    for (int u = 0; u < kAlphaCells; ++u) {
        hires_pos(nlam, n, sh[u], n0[u], fr[u]);
        row[u][0] = ((size_t)q[u].ti0 * nP + q[u].pi0) * nlam + n0[u];
        row[u][1] = ((size_t)q[u].ti0 * nP + q[u].pi1) * nlam + n0[u];
        row[u][2] = ((size_t)q[u].ti1 * nP + q[u].pi0) * nlam + n0[u];
        row[u][3] = ((size_t)q[u].ti1 * nP + q[u].pi1) * nlam + n0[u];
#pragma unroll
        for (int k = 0; k < 4; ++k) a[u][k] = lnk_tpl[row[u][k]];
    }
    if constexpr (sizeof(R) == sizeof(float)) {
        const bool last_lane = (threadIdx.x & 63) == 63;
        const int grp_next = __shfl_down(grp, 1);
#pragma unroll
        for (int u = 0; u < kAlphaCells; ++u) {
            const int n0_next = __shfl_down(n0[u], 1);
            const bool take = !last_lane && grp_next == grp && n0_next == n0[u] + d;
#pragma unroll
            for (int k = 0; k < 4; ++k) b[u][k] = __shfl_down(a[u][k], 1);
            if (!take) {
#pragma unroll
                for (int k = 0; k < 4; ++k) b[u][k] = lnk_tpl[row[u][k] + d];
            }
        }
    } else {  // FP64: exchanging the doubles costs more registers than the loads save
#pragma unroll
        for (int u = 0; u < kAlphaCells; ++u)
#pragma unroll
            for (int k = 0; k < 4; ++k) b[u][k] = lnk_tpl[row[u][k] + d];
    }
    if (!live) return;
#pragma unroll
    for (int u = 0; u < kAlphaCells; ++u) {
        const int c = c0 + u;
        if (c >= ncell) break;
        Bracket bt, bp;
        bt.i0 = q[u].ti0; bt.i1 = q[u].ti1; bt.t = q[u].tt;
        bp.i0 = q[u].pi0; bp.i1 = q[u].pi1; bp.t = q[u].pt;
        const double kl = hires_combine<R>(a[u], b[u], bt, bp, fr[u], nlam);
        const double kext = kl + kr;
        alpha[(size_t)c * slot_stride + s] = (R)(rho[u] * kext);
    }
}

// (emission sources for the transport live in prep.hip)

// Serial-per-thread then tree reduction of nblk rows of `width` doubles;
// Neumaier-compensated so the result is nearly independent of blocking.
__global__ void __launch_bounds__(256) k_reduce_rows(const double* __restrict__ part, int nrow, int width,
                                                    double* __restrict__ out)
{
    __shared__ double sh[256];
    __shared__ double shc[256];
    int col = blockIdx.x;
    double s = 0.0, comp = 0.0;
    for (int r = threadIdx.x; r < nrow; r += 256) {
        double x = part[(size_t)r * width + col];
        double t = s + x;
        if (fabs(s) >= fabs(x)) comp = comp + ((s - t) + x);
        else comp = comp + ((x - t) + s);
        s = t;
    }
    sh[threadIdx.x] = s;
    shc[threadIdx.x] = comp;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            double a = sh[threadIdx.x], b = sh[threadIdx.x + st];
            double t = a + b;
            double e = (fabs(a) >= fabs(b)) ? ((a - t) + b) : ((b - t) + a);
            sh[threadIdx.x] = t;
            shc[threadIdx.x] = shc[threadIdx.x] + shc[threadIdx.x + st] + e;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[col] = sh[0] + shc[0];
}

// ------------------------------------------------- borrowed grid checks
// The validation of host grids, done where borrowed device arrays live:
// every cell sets the bits of the checks it fails (atomic OR on one word).
__global__ void __launch_bounds__(256) k_check_cells(const float* __restrict__ T, const float* __restrict__ P,
                                                     const double* __restrict__ rho, const float* __restrict__ u,
                                                     const float* __restrict__ v, const float* __restrict__ w,
                                                     const float* __restrict__ cs, const float* __restrict__ ca,
                                                     const float* __restrict__ cg, size_t n, int* __restrict__ bad)
{
    int f = 0;
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (size_t)gridDim.x * 256) {
        if (!(isfinite(T[c]) && T[c] > 0.0f)) f |= 1;
        if (!(isfinite(P[c]) && P[c] > 0.0f)) f |= 2;
        if (!(isfinite(rho[c]) && rho[c] >= 0.0)) f |= 4;
        if ((u && !isfinite(u[c])) || (v && !isfinite(v[c])) || (w && !isfinite(w[c]))) f |= 8;
        if (cs && !(isfinite(cs[c]) && cs[c] >= 0.0f && isfinite(ca[c]) && ca[c] >= 0.0f)) f |= 16;
        if (cg && !(fabsf(cg[c]) < 1.0f)) f |= 32;
    }
    if (f) atomicOr(bad, f);
}

// ---------------------------------------------------------------- K5 chords
__device__ __forceinline__ void chord_start(const GridDev& g, int ch, int n_b, int n_alpha, uint64_t seed,
                                            uint32_t tag, Ray& p, double& b)
{
    int ib = ch / n_alpha, ia = ch % n_alpha;
    U2 u = draw(seed, tag, (uint64_t)ch, 0, 0);
    double r0 = g.r[0], rt = g.r[g.nlay];
    b = r0 + ((double)ib + u.a) * (rt - r0) / (double)n_b;
    double al = 2.0 * kPi * ((double)ia + u.b) / (double)n_alpha;
    p.x = sqrt(fmax(rt * rt - b * b, 0.0));
    p.y = b * cos(al);
    p.z = b * sin(al);
    p.k = g.nlay - 1;
    locate_column(g, p);
    p.ef = F_OUT;
}

__global__ void __launch_bounds__(256) k_chord_count(GridDev g, int n_b, int n_alpha, uint64_t seed, uint32_t tag,
                                                     int* __restrict__ counts)
{
    int ch = blockIdx.x * blockDim.x + threadIdx.x;
    if (ch >= n_b * n_alpha) return;
    Ray p;
    double b;
    chord_start(g, ch, n_b, n_alpha, seed, tag, p, b);
    int n = 0;
    int cap = 64 * (g.nlay + g.nlat + g.nlon) + 64;
    while (n < cap) {
        double s;
        int f = exit_distance(g, p, -1.0, 0.0, 0.0, s);
        if (f == F_NONE) break;
        ++n;
        advance(g, p, -1.0, 0.0, 0.0, s);
        cross(g, p, f);
        if (p.k >= g.nlay || p.k < 0) break;
    }
    counts[ch] = n;
}

// R: type of the stored segment lengths (FP64, or FP32 in the mixed form).
template <typename R>
__global__ void __launch_bounds__(256) k_chord_fill(GridDev g, int n_b, int n_alpha, uint64_t seed, uint32_t tag,
                                                    const long long* __restrict__ offsets,
                                                    uint32_t* __restrict__ seg_cell, R* __restrict__ seg_len,
                                                    double* __restrict__ chord_b, int* __restrict__ chord_ok,
                                                    LimbDark ld)
{
    int ch = blockIdx.x * blockDim.x + threadIdx.x;
    if (ch >= n_b * n_alpha) return;
    Ray p;
    double b;
    chord_start(g, ch, n_b, n_alpha, seed, tag, p, b);
    // the chord's weight: b times the limb-darkening fraction of the stellar
    // light behind it
    const double wb = b * limb_weight(ld, p.y, p.z);
    long long o = offsets[ch], end = offsets[ch + 1];
    int ok = 0;
    while (o < end) {
        double s;
        int f = exit_distance(g, p, -1.0, 0.0, 0.0, s);
        if (f == F_NONE) break;
        seg_cell[o] = (uint32_t)cell_of(g, p);
        seg_len[o] = (R)s;
        ++o;
        advance(g, p, -1.0, 0.0, 0.0, s);
        cross(g, p, f);
        if (p.k >= g.nlay) { ok = 1; break; }
        if (p.k < 0) break;
    }
    chord_b[ch] = wb;
    chord_ok[ch] = ok;
}

__global__ void __launch_bounds__(256) k_scan_int(const int* __restrict__ in, long long* __restrict__ out, int n)
{
    // single block exclusive scan of ints into 64-bit offsets; out[n] = total
    __shared__ long long sh[256];
    int per = (n + 255) / 256;
    int b0 = threadIdx.x * per;
    long long run = 0;
    for (int q = 0; q < per; ++q)
        if (b0 + q < n) run += in[b0 + q];
    sh[threadIdx.x] = run;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        long long v = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    long long acc = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0;
    for (int q = 0; q < per; ++q) {
        if (b0 + q < n) {
            out[b0 + q] = acc;
            acc += in[b0 + q];
        }
    }
    if (threadIdx.x == 255) out[n] = sh[255];
}

// tau per (chord, slot) = sum over the chord's segments of alpha[cell][slot]
// * length, in segment order; one wave per chord, lanes over slots.
// Each block sums (1 - e^-tau) b and its square over its chords in a fixed
// order into partials[block][slot][2].
constexpr int kChordWaves = 4;
constexpr int kChordsPerWave = 8;
constexpr int kChordUnroll = 16;  // row gathers in flight per wave

// Lane k's value of x, for every lane (k uniform across the wave).
__device__ inline float lane_bcast(float x, int k)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), k));
}
__device__ inline double lane_bcast(double x, int k)
{
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// R: the stored extinction (double, or float in the mixed form: half the
// gathered bytes); tau accumulates in FP64 either way.
// Blocks run consecutive chords (one impact parameter, consecutive limb
// angles), so the blocks resident at a time cross a thin shell of cells whose
// extinction rows the caches hold; a wave walks its chords one after another.
template <typename R>
__global__ void __launch_bounds__(256) k_chord_tau(int nch, const long long* __restrict__ offsets,
                                                   const uint32_t* __restrict__ seg_cell,
                                                   const R* __restrict__ seg_len,
                                                   const double* __restrict__ chord_b,
                                                   const int* __restrict__ chord_ok,
                                                   const R* __restrict__ alpha, int nslot,
                                                   double* __restrict__ partials)
{
    __shared__ double sh1[kChordWaves][64];
    __shared__ double sh2[kChordWaves][64];
    const int blk = (int)blockIdx.x;
    // the wave index is uniform: chord bounds and segment counts then live
    // in scalar registers and the per-segment tests are scalar branches
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    for (int s0 = 0; s0 < nslot; s0 += 64) {
        int s = s0 + lane;
        // every lane gathers (a lane past the last slot reads slot 0 and drops
        // it), so the gathers issue unpredicated
        const R* arow = alpha + (s < nslot ? s : 0);
        double a1 = 0.0, a2 = 0.0;
        for (int m = 0; m < kChordsPerWave; ++m) {
            const int ch = (blk * kChordWaves + wave) * kChordsPerWave + m;
            if (ch >= nch) break;
            long long o0 = offsets[ch], o1 = offsets[ch + 1];
            double tau = 0.0;
            // the chord's segments in chunks of 64: each lane loads one (cell,
            // length) pair (coalesced), then the wave walks the chunk in
            // segment order, sixteen segments at a time: their cell indices
            // are broadcast to scalar registers, all sixteen row gathers are
            // issued, and only then added in segment order.  (A loop over the
            // chunk with a cross-lane shuffle in its body is not unrolled by
            // the compiler, which then keeps one gather in flight per wave.)
            for (long long c0 = o0; c0 < o1; c0 += 64) {
                const int nseg = (int)(o1 - c0 < 64 ? o1 - c0 : 64);
                uint32_t mc = 0;
                R ml = (R)0;
                if (lane < nseg) {
                    mc = seg_cell[c0 + lane];
                    ml = seg_len[c0 + lane];
                }
                for (int k0 = 0; k0 < nseg; k0 += kChordUnroll) {
                    R av[kChordUnroll];
#pragma unroll
                    for (int u = 0; u < kChordUnroll; ++u) {
                        // k0 + u <= 63; lanes past the chunk hold cell 0, whose
                        // row is read and dropped below
                        const uint32_t cell = (uint32_t)__builtin_amdgcn_readlane((int)mc, k0 + u);
                        av[u] = arow[(size_t)cell * nslot];
                    }
#pragma unroll
                    for (int u = 0; u < kChordUnroll; ++u)
                        if (k0 + u < nseg) tau = tau + (double)av[u] * (double)lane_bcast(ml, k0 + u);
                }
            }
            if (!chord_ok[ch]) tau = INFINITY;
            double v = (1.0 - exp(-tau)) * chord_b[ch];
            a1 = a1 + v;
            a2 = a2 + v * v;
        }
        sh1[wave][lane] = a1;
        sh2[wave][lane] = a2;
        __syncthreads();
        if (wave == 0 && s < nslot) {
            double t1 = sh1[0][lane], t2 = sh2[0][lane];
            for (int w = 1; w < kChordWaves; ++w) {
                t1 = t1 + sh1[w][lane];
                t2 = t2 + sh2[w][lane];
            }
            double* row = partials + (size_t)blk * (2 * nslot);
            row[2 * s] = t1;
            row[2 * s + 1] = t2;
        }
        __syncthreads();
    }
}

inline int nblk(long long n, int b) { return (int)((n + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------- launchers
template <typename R>
void launch_ck_optics(const GridDev& g, int ncell, const double* lnk_tab, int nT, int nP, const double* T_grid,
                      const double* lnP_grid, double k_ray, OpticsDev<R> out, int ext_stride,
                      hipStream_t stream)
{
    hipLaunchKernelGGL(k_ck_optics<R>, dim3(nblk(ncell, 256)), dim3(256), 0, stream, g, ncell, lnk_tab, nT, nP,
                       T_grid, lnP_grid, k_ray, out, ext_stride);
}
template void launch_ck_optics<double>(const GridDev&, int, const double*, int, int, const double*, const double*,
                                       double, OpticsDev<double>, int, hipStream_t);
template void launch_ck_optics<float>(const GridDev&, int, const double*, int, int, const double*, const double*,
                                      double, OpticsDev<float>, int, hipStream_t);

void launch_doppler_shift(const GridDev& g, double ox, double oy, double oz, double dlnlam, double* shift,
                          hipStream_t stream)
{
    int ncell = g.nlon * g.nlat * g.nlay;
    hipLaunchKernelGGL(k_doppler_shift, dim3(nblk(ncell, 256)), dim3(256), 0, stream, g, ox, oy, oz, dlnlam, shift);
}

void launch_cell_tp(const GridDev& g, int ncell, int nT, int nP, const double* T_grid, const double* lnP_grid,
                    CellTP* out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_cell_tp, dim3(nblk(ncell, 256)), dim3(256), 0, stream, g, ncell, nT, nP, T_grid, lnP_grid,
                       out);
}

template <typename R>
void launch_hires_alpha_block(const GridDev& g, int ncell, const R* lnk_tpl, int nlam, int nP,
                              const CellTP* tp, const double* k_ray, const double* shift, const int* nlist,
                              int nslot, int slot_stride, R* alpha, hipStream_t stream)
{
    long long n = (long long)((ncell + kAlphaCells - 1) / kAlphaCells) * nslot;
    hipLaunchKernelGGL(k_hires_alpha_block<R>, dim3(nblk(n, 256)), dim3(256), 0, stream, g, ncell, lnk_tpl, nlam,
                       nP, tp, k_ray, shift, nlist, nslot, slot_stride, alpha);
}
template void launch_hires_alpha_block<double>(const GridDev&, int, const double*, int, int, const CellTP*,
                                               const double*, const double*, const int*, int, int, double*,
                                               hipStream_t);
template void launch_hires_alpha_block<float>(const GridDev&, int, const float*, int, int, const CellTP*,
                                              const double*, const double*, const int*, int, int, float*,
                                              hipStream_t);

void launch_reduce_partials(const double* partials, int nblocks, int width, double* out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_reduce_rows, dim3(width), dim3(256), 0, stream, partials, nblocks, width, out);
}

void launch_check_cells(const float* T, const float* P, const double* rho, const float* u, const float* v,
                        const float* w, const float* cs, const float* ca, const float* cg, size_t n, int* bad,
                        hipStream_t stream)
{
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_check_cells, dim3(blocks), dim3(256), 0, stream, T, P, rho, u, v, w, cs, ca, cg, n, bad);
}

void launch_chord_count(const GridDev& g, int n_b, int n_alpha, uint64_t seed, uint32_t tag, int* counts,
                        hipStream_t stream)
{
    int nch = n_b * n_alpha;
    hipLaunchKernelGGL(k_chord_count, dim3(nblk(nch, 256)), dim3(256), 0, stream, g, n_b, n_alpha, seed, tag, counts);
}

void launch_exclusive_scan_int(const int* in, long long* out, int n, long long* /*total_dev*/, hipStream_t stream)
{
    hipLaunchKernelGGL(k_scan_int, dim3(1), dim3(256), 0, stream, in, out, n);
}

template <typename R>
void launch_chord_fill(const GridDev& g, int n_b, int n_alpha, uint64_t seed, uint32_t tag, const long long* offsets,
                       uint32_t* seg_cell, R* seg_len, double* chord_b, int* chord_ok, const LimbDark& ld,
                       hipStream_t stream)
{
    int nch = n_b * n_alpha;
    hipLaunchKernelGGL(k_chord_fill<R>, dim3(nblk(nch, 256)), dim3(256), 0, stream, g, n_b, n_alpha, seed, tag,
                       offsets, seg_cell, seg_len, chord_b, chord_ok, ld);
}
template void launch_chord_fill<double>(const GridDev&, int, int, uint64_t, uint32_t, const long long*, uint32_t*,
                                        double*, double*, int*, const LimbDark&, hipStream_t);
template void launch_chord_fill<float>(const GridDev&, int, int, uint64_t, uint32_t, const long long*, uint32_t*,
                                       float*, double*, int*, const LimbDark&, hipStream_t);

int chord_tau_blocks(int nch) { return nblk(nch, kChordWaves * kChordsPerWave); }

template <typename R>
void launch_chord_tau(int n_b, int n_alpha, const long long* offsets, const uint32_t* seg_cell, const R* seg_len,
                      const double* chord_b, const int* chord_ok, const R* alpha, int nslot, double* partials,
                      int nblocks, hipStream_t stream)
{
    const int nch = n_b * n_alpha;
    hipLaunchKernelGGL(k_chord_tau<R>, dim3(nblocks), dim3(256), 0, stream, nch, offsets, seg_cell, seg_len, chord_b,
                       chord_ok, alpha, nslot, partials);
}
template void launch_chord_tau<double>(int, int, const long long*, const uint32_t*, const double*, const double*,
                                       const int*, const double*, int, double*, int, hipStream_t);
template void launch_chord_tau<float>(int, int, const long long*, const uint32_t*, const float*, const double*,
                                      const int*, const float*, int, double*, int, hipStream_t);

}  // namespace mcrt
