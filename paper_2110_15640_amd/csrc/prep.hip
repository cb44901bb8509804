// Batched preparation of the (spectral point, g) solves of one transport
// launch: every stage is a single launch over all solve slots (blockIdx.y =
// slot), so a batch of hundreds of solves costs a handful of launches.
//   optics  K1/K2: per cell, the ck gather or the Doppler-shifted hi-res gather
//                  (Sect. 7) to alpha_ext, alpha_abs, omega, P_gas, g (FP64, and
//                  FP32 copies for the mixed form);
//   sources K3:    per column, L_i = 4 pi V_i alpha_abs B_lambda(T_i) with the
//                  tau_vert cut (Sect. 5.3, Sect. 4.6); per slot L_tot and
//                  N_emit; hybrid bias q_i (Sect. 4.3), birth weights and the
//                  inclusive FP64 CDF of q.
// The arithmetic per cell and the reduction / scan blocking are those of the
// single-solve kernels, so results do not depend on the batch size.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "device_common.hpp"
#include "mcrt_internal.hpp"

namespace mcrt {
namespace {
using namespace dev;

constexpr int kScanPer = 8;
constexpr int kScanBlock = 256 * kScanPer;

__device__ __forceinline__ double planck_bl(double lam_cm, double T)
{
    double x = kH * kC / (lam_cm * kKB * T);
    return 2.0 * kH * kC * kC / pow(lam_cm, 5.0) / expm1(x);
}

__device__ __forceinline__ double hires_kappa_at(const double* __restrict__ lnk_tpl, int nlam, int nP,
                                                 const Bracket& bt, const Bracket& bp, int n, double shift)
{
    double x = (double)n + shift;
    int n0;
    double fr;
    if (nlam == 1) { n0 = 0; fr = 0.0; }
    else if (x <= 0.0) { n0 = 0; fr = 0.0; }
    else if (x >= (double)(nlam - 1)) { n0 = nlam - 2; fr = 1.0; }
    else { n0 = (int)floor(x); fr = x - (double)n0; }
    double k0 = interp_tp([&](int a, int b) { return lnk_tpl[((size_t)a * nP + b) * nlam + n0]; }, bt, bp);
    if (nlam == 1) return k0;
    double k1 = interp_tp([&](int a, int b) { return lnk_tpl[((size_t)a * nP + b) * nlam + n0 + 1]; }, bt, bp);
    return (1.0 - fr) * k0 + fr * k1;
}

__global__ void __launch_bounds__(256) k_prep_optics(GridDev g, int ncell, const PrepSlot* __restrict__ slots,
                                                     int hires, int nT, int nP, const double* __restrict__ T_grid,
                                                     const double* __restrict__ lnP_grid,
                                                     const double* __restrict__ lnk_tpl, int nlam,
                                                     const double* __restrict__ shift, int draine, double alpha)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const PrepSlot S = slots[blockIdx.y];
    Bracket bt = bracket(T_grid, nT, (double)g.T[c]);
    Bracket bp = bracket(lnP_grid, nP, log((double)g.P[c]));
    const double rho = g.rho[c];
    double ae, aa, om, pg, gc;
    if (!hires) {
        const double* tab = S.lnk;
        double kg = interp_tp([&](int a, int b) { return tab[a * nP + b]; }, bt, bp);
        double ks = g.cld_ksca ? (double)g.cld_ksca[c] : 0.0;
        double ka = g.cld_kabs ? (double)g.cld_kabs[c] : 0.0;
        double kab = kg + ka;
        double ksc = S.k_ray + ks;
        double kext = kab + ksc;
        ae = rho * kext;
        aa = rho * kab;
        om = kext > 0.0 ? ksc / kext : 0.0;
        pg = ksc > 0.0 ? S.k_ray / ksc : 1.0;
        gc = g.cld_g ? (double)g.cld_g[c] : 0.0;
        if (draine) gc = draine_G(gc, alpha);  // Draine clouds carry G in place of g
    } else {
        double kl = hires_kappa_at(lnk_tpl, nlam, nP, bt, bp, S.n, shift ? shift[c] : 0.0);
        double kext = kl + S.k_ray;
        ae = rho * kext;
        aa = rho * kl;
        om = kext > 0.0 ? S.k_ray / kext : 0.0;
        pg = 1.0;
        gc = 0.0;
    }
    double* o = S.opt;
    o[c] = ae;
    o[ncell + c] = aa;
    o[2 * (size_t)ncell + c] = om;
    o[3 * (size_t)ncell + c] = pg;
    o[4 * (size_t)ncell + c] = gc;
    if (S.optf) {
        float* f = S.optf;
        f[c] = (float)ae;
        f[ncell + c] = (float)aa;
        f[2 * (size_t)ncell + c] = (float)om;
        f[3 * (size_t)ncell + c] = (float)pg;
        f[4 * (size_t)ncell + c] = (float)gc;
    }
}

// L per cell into the slot's cdf array (the first stage of the CDF).
__global__ void __launch_bounds__(256) k_prep_L(GridDev g, const PrepSlot* __restrict__ slots, double tau_vert)
{
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= g.nlon * g.nlat) return;
    const PrepSlot S = slots[blockIdx.y];
    const int ncell = g.nlon * g.nlat * g.nlay;
    const double* a_ext = S.opt;
    const double* a_abs = S.opt + ncell;
    double* L = S.cdf;
    const int i = col % g.nlon, j = col / g.nlon;
    double tau = 0.0;
    const double dsl = g.lat_sin[j + 1] - g.lat_sin[j];
    const double dph = g.lon[i + 1] - g.lon[i];
    for (int k = g.nlay - 1; k >= 0; --k) {
        int c = (k * g.nlat + j) * g.nlon + i;
        double vol = g.vol_r[k] * dsl * dph;
        double Li = 4.0 * kPi * vol * a_abs[c] * planck_bl(S.lam_cm, (double)g.T[c]);
        L[c] = (tau > tau_vert) ? 0.0 : Li;
        tau = tau + a_ext[c] * (g.r[k + 1] - g.r[k]);
    }
}

template <int NT>
__device__ __forceinline__ double bsum(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// (sum L, count L > 0) per 256 cells -> part[slot][block][2]
__global__ void __launch_bounds__(256) k_prep_sumL(const PrepSlot* __restrict__ slots, int n, double* __restrict__ part)
{
    __shared__ double sh[256];
    const PrepSlot S = slots[blockIdx.y];
    const int c = blockIdx.x * 256 + threadIdx.x;
    double v = c < n ? S.cdf[c] : 0.0;
    double cnt = (c < n && v > 0.0) ? 1.0 : 0.0;
    double s = bsum<256>(v, sh);
    double m = bsum<256>(cnt, sh);
    if (threadIdx.x == 0) {
        double* p = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 2;
        p[0] = s;
        p[1] = m;
    }
}

// Neumaier-compensated sum of the block partials -> slot stats (L_tot, N_emit).
__global__ void __launch_bounds__(256) k_prep_stats(const PrepSlot* __restrict__ slots, const double* __restrict__ part,
                                                    int nb)
{
    __shared__ double sh[256];
    __shared__ double shc[256];
    const PrepSlot S = slots[blockIdx.y];
    const int col = blockIdx.x;
    double s = 0.0, comp = 0.0;
    for (int r = threadIdx.x; r < nb; r += 256) {
        double x = part[((size_t)blockIdx.y * nb + r) * 2 + col];
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
    if (threadIdx.x == 0) S.stats[col] = sh[0] + shc[0];
}

// q_i into cdf (in place of L), birth weights (L_i/L_tot)/q_i.
__global__ void __launch_bounds__(256) k_prep_bias(const PrepSlot* __restrict__ slots, int n, double xi)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    const PrepSlot S = slots[blockIdx.y];
    const double Ltot = S.stats[0], nemit = S.stats[1];
    const double Lc = S.cdf[c];
    double qc = 0.0;
    if (Lc > 0.0) qc = (1.0 - xi) * Lc / Ltot + xi / nemit;
    S.cdf[c] = qc;
    S.wbirth[c] = (Lc > 0.0) ? (Lc / Ltot) / qc : 0.0;
}

// In-place inclusive scan of cdf per slot: runs of 8 per thread, a
// Hillis-Steele scan over the 256 thread totals, block totals scanned by one
// block per slot, then the block offsets added.
__global__ void __launch_bounds__(256) k_prep_scan_local(const PrepSlot* __restrict__ slots, int n,
                                                         double* __restrict__ blocksum)
{
    __shared__ double sh[256];
    const PrepSlot S = slots[blockIdx.y];
    double* io = S.cdf;
    const int base = blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
    double loc[kScanPer];
    double run = 0.0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        double x = (base + q < n) ? io[base + q] : 0.0;
        run = run + x;
        loc[q] = run;
    }
    sh[threadIdx.x] = run;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        double v = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0.0;
        __syncthreads();
        sh[threadIdx.x] = sh[threadIdx.x] + v;
        __syncthreads();
    }
    double pre = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0.0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q)
        if (base + q < n) io[base + q] = pre + loc[q];
    if (threadIdx.x == 255) blocksum[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = sh[255];
}

__global__ void __launch_bounds__(256) k_prep_scan_blocksums(double* __restrict__ blocksum, int nb)
{
    __shared__ double sh[256];
    double* bs = blocksum + (size_t)blockIdx.y * nb;
    const int per = (nb + 255) / 256;
    const int b0 = threadIdx.x * per;
    double run = 0.0;
    for (int q = 0; q < per; ++q)
        if (b0 + q < nb) run = run + bs[b0 + q];
    sh[threadIdx.x] = run;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        double v = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0.0;
        __syncthreads();
        sh[threadIdx.x] = sh[threadIdx.x] + v;
        __syncthreads();
    }
    double acc = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0.0;
    for (int q = 0; q < per; ++q) {
        if (b0 + q < nb) {
            double x = bs[b0 + q];
            bs[b0 + q] = acc;
            acc = acc + x;
        }
    }
}

__global__ void __launch_bounds__(256) k_prep_scan_add(const PrepSlot* __restrict__ slots, int n,
                                                       const double* __restrict__ blocksum, int nb)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    const int b = c / kScanBlock;
    if (b > 0) {
        double* io = slots[blockIdx.y].cdf;
        io[c] = blocksum[(size_t)blockIdx.y * nb + b] + io[c];
    }
}

inline unsigned nb(long long n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

size_t prep_scratch_doubles(int ncell, int nslots)
{
    return (size_t)nslots * (2 * (size_t)nb(ncell, 256) + nb(ncell, kScanBlock)) + 16;
}

void launch_prep_optics(const GridDev& g, int ncell, const PrepSlot* slots, int nslots, int hires, int nT, int nP,
                        const double* T_grid, const double* lnP_grid, const double* lnk_tpl, int nlam,
                        const double* shift, int draine, double alpha, hipStream_t stream)
{
    hipLaunchKernelGGL(k_prep_optics, dim3(nb(ncell, 256), nslots), dim3(256), 0, stream, g, ncell, slots, hires, nT,
                       nP, T_grid, lnP_grid, lnk_tpl, nlam, shift, draine, alpha);
}

void launch_prep_sources(const GridDev& g, int ncell, const PrepSlot* slots, int nslots, double tau_vert, double xi,
                         double* scratch, hipStream_t stream)
{
    const unsigned ncol = nb(g.nlon * g.nlat, 256), b256 = nb(ncell, 256), bs = nb(ncell, kScanBlock);
    double* lpart = scratch;
    double* bsum = lpart + (size_t)nslots * 2 * b256;
    hipLaunchKernelGGL(k_prep_L, dim3(ncol, nslots), dim3(256), 0, stream, g, slots, tau_vert);
    hipLaunchKernelGGL(k_prep_sumL, dim3(b256, nslots), dim3(256), 0, stream, slots, ncell, lpart);
    hipLaunchKernelGGL(k_prep_stats, dim3(2, nslots), dim3(256), 0, stream, slots, lpart, (int)b256);
    hipLaunchKernelGGL(k_prep_bias, dim3(b256, nslots), dim3(256), 0, stream, slots, ncell, xi);
    hipLaunchKernelGGL(k_prep_scan_local, dim3(bs, nslots), dim3(256), 0, stream, slots, ncell, bsum);
    if (bs > 1) {
        hipLaunchKernelGGL(k_prep_scan_blocksums, dim3(1, nslots), dim3(256), 0, stream, bsum, (int)bs);
        hipLaunchKernelGGL(k_prep_scan_add, dim3(b256, nslots), dim3(256), 0, stream, slots, ncell, bsum, (int)bs);
    }
}

}  // namespace mcrt
