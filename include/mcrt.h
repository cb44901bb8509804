/*
 * mcrt.h -- C ABI of the MI355X photon-transport library (libmcrt.so).
 *
 * The library solves the three observables of the gCMCRT method (Lee et al.
 * 2022, arXiv:2110.15640) by Monte Carlo radiative transfer with peel-off on
 * 3D spherical lon-lat-radius grids (Sect. 2) or 1D plane-parallel slabs:
 *   - geometric albedo spectra and scattered-light phase curves (Sect. 5.2,
 *     the A_g and Phi(phi) equations),
 *   - thermal emission spectra and phase curves (Sect. 5.3, L_i, L_p, I_p,
 *     F_p equations),
 *   - transmission spectra (Sect. 5.1, the (R_p/R_star)^2 equation and its
 *     Monte Carlo estimator),
 * with correlated-k opacities or Doppler-shifted high-resolution opacities
 * (Sect. 7, the v_LOS and lambda_eff equations).  All device work runs in
 * hand-written HIP kernels for gfx950; no torch types cross this boundary.
 *
 * Conventions (CGS): star at +x, rotation axis +z, longitude east-positive in
 * [-pi, pi], latitude in [-pi/2, pi/2].  Cell (i, j, k) = (lon, lat, radius)
 * is stored at c = (k*nlat + j)*nlon + i, k = 0 at the bottom (r = R0).
 *
 * Errors: every int-returning call returns MCRT_OK (0) or a negative code
 * below; mcrt_last_error() then gives a message (thread-local, valid until
 * the next failing call on that thread).  No exception crosses the ABI.
 * Thread safety: one context may be used from several threads; uploads,
 * frees and blocking solves are serialised by the context; submit / poll /
 * wait / cancel are safe to call concurrently.
 */
#ifndef MCRT_H
#define MCRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCRT_OK 0
#define MCRT_EINVAL (-1)     /* bad argument or input data            */
#define MCRT_ENOMEM (-2)     /* device or host allocation failed      */
#define MCRT_EDEVICE (-3)    /* HIP runtime error; context unusable   */
#define MCRT_ENOTFOUND (-4)  /* unknown grid / opacity / ticket id    */
#define MCRT_EBUDGET (-5)    /* would exceed the context's HBM budget */
#define MCRT_EBUSY (-6)      /* object in use by a running solve      */
#define MCRT_ECANCELLED (-7) /* request was cancelled                 */

#define MCRT_SPHERICAL 0
#define MCRT_PLANE_PARALLEL 1

#define MCRT_SURVIVAL 0   /* survival biasing (Sect. 4.4) */
#define MCRT_CONTINUOUS 1 /* continuous absorption (Sect. 4.1) */

#define MCRT_FP64 0  /* all arithmetic in FP64 */
#define MCRT_MIXED 1 /* FP32 opacity, phase function, direction; FP64 roots, tau, tallies */

#define MCRT_OPAC_CK 0
#define MCRT_OPAC_HIRES 1

#define MCRT_MODE_ALBEDO 0
#define MCRT_MODE_EMISSION 1
#define MCRT_MODE_TRANSMISSION 2

/* Number of per-solve counters in mcrt_result.counters, in this order:
 * escaped weight, weight reaching the surface, absorbed weight, net weight
 * removed by Russian roulette, weight of capped packets, weight of lost
 * packets, interactions, cell crossings, capped packets, lost packets,
 * total initial weight. */
#define MCRT_NCOUNTERS 11

typedef struct mcrt_ctx mcrt_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory the context may hold (0 = 90 % of the free memory).  The context
 * owns every device buffer it allocates; mcrt_destroy frees them. */
int mcrt_create(int device, uint64_t hbm_budget_bytes, mcrt_ctx** out);
void mcrt_destroy(mcrt_ctx* ctx);
const char* mcrt_last_error(void);
/* Device memory currently held by the context, in bytes. */
uint64_t mcrt_memory_in_use(const mcrt_ctx* ctx);

/* Atmosphere structure (Sect. 2 "spherical geometry grid"; GCM output in
 * lat-lon form).  All arrays are host memory and are copied before return.
 * r_edges[nlay+1]: radii [cm], strictly increasing, r_edges[0] = R0 (slab:
 * heights [cm]); lat_edges[nlat+1] from -pi/2 to pi/2 and lon_edges[nlon+1]
 * from -pi to pi, strictly increasing (ignored for the slab, where nlat =
 * nlon = 1).  Per cell: T [K] float, P [bar] float, rho [g/cm^3] double,
 * optional winds u (east), v (north), w (up) [cm/s] float (NULL = 0) and
 * optional grey cloud opacities cld_ksca, cld_kabs [cm^2/g] and asymmetry
 * cld_g float (NULL = no cloud).  omega_rot: solid-body rotation [1/s].
 * flags: MCRT_BORROW_DEVICE = the per-cell arrays (T, P, rho, winds,
 * clouds) are DEVICE pointers on the context's device (e.g. torch tensors'
 * data_ptr()) that the library reads in place: nothing is copied or counted
 * against the budget, and the caller keeps them alive and unchanged until
 * mcrt_grid_free; the edge arrays stay host memory.  Their values are checked
 * on the device at upload.
 * Errors: EINVAL for non-monotone or incomplete edges, non-finite values,
 * T <= 0, P <= 0, rho < 0, |g| >= 1, or a borrowed pointer that is not
 * device memory of this device; EBUDGET if the copy would exceed the budget
 * (nothing is allocated then). */
#define MCRT_BORROW_DEVICE 1
typedef struct {
    int32_t geometry;
    int32_t nlon, nlat, nlay;
    const double* r_edges;
    const double* lat_edges;
    const double* lon_edges;
    const float* T;
    const float* P;
    const double* rho;
    const float* u;
    const float* v;
    const float* w;
    const float* cld_ksca;
    const float* cld_kabs;
    const float* cld_g;
    double omega_rot;
    int32_t flags;
} mcrt_grid_desc;

/* stream: hipStream_t (NULL = the null stream) on which the copies and the
 * device check of borrowed arrays run, after the caller's earlier work on
 * it; the call returns when they are done.  When the budget is short and no
 * blocking solve is running, the scratch the blocking solves keep (see
 * params.max_batch) is released first. */
int mcrt_grid_upload(mcrt_ctx* ctx, const mcrt_grid_desc* desc, void* stream, int32_t* grid_id);
int mcrt_grid_free(mcrt_ctx* ctx, int32_t grid_id);

/* Opacity table (Sect. 7).  kind = MCRT_OPAC_CK: pre-mixed k-table
 * kappa[nspec][ng][nT][nP] [cm^2/g] interpolated bilinearly in (T, ln P) on
 * ln kappa and clamped to the table, band-centre wavelengths lam_um[nspec],
 * g_weights[ng] (sum 1).  kind = MCRT_OPAC_HIRES: kappa[nspec][nT][nP] on
 * the log-uniform grid lam_n = lam_min_um exp(n dlnlam), ng = 1.  k_ray
 * [nspec]: Rayleigh opacity [cm^2/g] at each spectral point.  Host arrays,
 * copied.  Errors: EINVAL for kappa < 0 or non-finite, a ck kappa that
 * decreases from one g-ordinate to the next at some (band, T, P) (a
 * k-distribution is sorted), a non-increasing T/P grid, P_grid <= 0,
 * weights not summing to 1 within 1e-9. */
typedef struct {
    int32_t kind;
    int32_t nspec;
    int32_t ng;
    int32_t nT, nP;
    const double* lam_um;
    double lam_min_um;
    double dlnlam;
    const double* g_weights;
    const double* T_grid;
    const double* P_grid;
    const float* kappa;
    const double* k_ray;
} mcrt_opacity_desc;

/* stream: as for mcrt_grid_upload (the re-laid-out table is copied on it and
 * the call returns when the copy is done).  The device holds ln kappa in
 * FP64 ([T][P][lambda] for MCRT_OPAC_HIRES, 8 B per entry) and, for
 * MCRT_OPAC_HIRES, the same values rounded to FP32 (4 B per entry more),
 * which the mixed-precision transmission reads. */
int mcrt_opacity_upload(mcrt_ctx* ctx, const mcrt_opacity_desc* desc, void* stream, int32_t* opac_id);
int mcrt_opacity_free(mcrt_ctx* ctx, int32_t opac_id);

/* Solve parameters.  Fill with mcrt_default_params() first.
 * seed: Philox4x32-10 key; packet n at event e draws block b from counter
 *   (lo32 n, hi32 n, e, b) under key (lo32 seed, hi32 seed ^ tag), tag = 0,
 *   or 1 + spec*ng + g with decorrelate != 0.
 * n_packets: packets per (spectral point, g) solve (albedo, emission).
 * spec_idx[n_spec]: bands (CK) or table wavelength indices (HIRES); NULL =
 *   all.  Every g-ordinate of a band is solved and weighted by g_weights.
 * Observers: obs_phase[n_obs] -- albedo: phase angle a, o = (cos a, sin a, 0);
 *   emission: orbital phase p, o = (cos l, sin l, 0), l = pi (1 - 2 p), so
 *   p = 0.5 views the dayside.  obs_dir[n_obs][3] (unit vectors) overrides.
 *   Slab albedo with n_obs = 0 uses the backscatter direction of each packet.
 *   Transmission always observes along -x.  n_obs <= 8.
 * scattering: 0 = emission peel-off only / no multiple scattering.
 * absorption: MCRT_SURVIVAL or MCRT_CONTINUOUS.
 * rr_threshold, rr_survive: Russian roulette (Sect. 4.5) below
 *   rr_threshold * W0, survival probability rr_survive.
 * emis_bias: hybrid emission bias fraction xi (Sect. 4.3).
 * tau_vert_max: cells whose column optical depth above their top face
 *   exceeds this do not emit (Sect. 4.6).
 * tau_peel_max: peel-off rays stop (f = 0) beyond this optical depth.
 * max_events: interactions per packet before it is stopped and counted.
 * mu0: slab albedo incidence cosine; <= 0 samples the uniform-disk mu0.
 * n_b, n_alpha: transmission strata in impact parameter and limb angle.
 * r_star: stellar radius [cm] for transmission depths.
 * ms_transmission: mcrt_solve_transmission only.  0 = raytrace chords (the
 *   n_b x n_alpha jittered strata, no scattering).  1 = multiple scattering
 *   (Sect. 5.1): n_packets packets per (spectral point, g) enter at random
 *   points of the annulus R0 <= b <= R_TOA (birth event, Philox block 0:
 *   slot a gives b uniformly, slot b the angle) with the stellar beam along
 *   -x and weight W0 = b times the limb-darkening fraction; the first
 *   peel-off, along the chord, is the directly transmitted light, and every
 *   interaction (and Lambert-floor reflection) peels off toward -x the light
 *   it scatters into the line of sight, W omega Theta e^{-tau} per steradian
 *   over the stellar beam's solid angle pi (r_star / a_orbit)^2.  Per packet
 *   the light taken out of the beam, v = W0 - F, is the tallied value (and
 *   the packet dump); per g-ordinate (R_p/R*)^2 = (R0^2 + 2 (R_TOA - R0)
 *   <v>) / R*^2, weighted by w_g.  Needs a_orbit > r_star; obs_*, contrib,
 *   image_npix and g_sampling do not apply (EINVAL for the last three).
 * a_orbit: star-planet distance [cm] (ms_transmission).
 * ld_law, ld_c1, ld_c2: stellar limb darkening of transmission packets and
 *   chords (Sect. 5.1.1): the chord at sky-plane offset (y, z) from the
 *   planet centre lies at (transit_y + y, transit_z + z) on the stellar
 *   disk, mu = sqrt(1 - r^2 / r_star^2), and its weight is multiplied by
 *   I(mu)/I(1): 0 none; 1 linear 1 - c1 (1 - mu); 2 quadratic
 *   1 - c1 (1 - mu) - c2 (1 - mu)^2; 3 square-root 1 - c1 (1 - mu)
 *   - c2 (1 - sqrt(mu)); 4 logarithmic 1 - c1 (1 - mu) - c2 mu ln mu;
 *   5 exponential 1 - c1 (1 - mu) - c2 / (1 - e^mu); 6 power-2
 *   1 - c1 (1 - mu^c2).  Off the stellar disk the weight is 0.  The bulk
 *   disk term R0^2 is not weighted.  Other laws: EINVAL.
 * transit_y, transit_z: planet centre on the stellar disk [cm] (sky plane). 
 * precision: MCRT_FP64 or MCRT_MIXED.  The FP64 form rounds every operation
 *   on its own (no contraction) and divides correctly rounded, so per-packet
 *   results agree with an independent FP64 evaluation to ~1e-12; the mixed
 *   form keeps optical properties, phase functions and directions in FP32 and
 *   computes crossings in FP64 with multiply-adds and a refined-reciprocal
 *   division (spectra within 1e-3 and 3 sigma of the FP64 ones).  Raytrace
 *   transmission in the mixed form stores each cell's extinction per
 *   spectral row in FP32 (evaluated in FP64, rounded once) and accumulates
 *   the chords' optical depths in FP64.
 * stream: hipStream_t to run on (NULL = the context's own stream).
 * packet_dump: optional DEVICE buffer of doubles receiving each packet's
 *   peel-off sum per observer, [solve][packet][observer] with solves ordered
 *   (spec, g); NULL = none.
 * profile: non-zero times every launch of the dominant kernel (transport for
 *   albedo/emission, chord optical depth for transmission) with HIP events on
 *   the solve's stream; see mcrt_result.kernel_ms.
 * max_batch: (spectral point, g) solves per persistent transport launch;
 *   1 = one launch per solve, 0 = as many as fit in half of what the HBM
 *   budget leaves (a blocking solve keeps its scratch for the next one,
 *   until an upload or a served request needs the room while no blocking
 *   solve runs).
 * tune_ev_threshold, tune_blocks_per_cu, tune_wave_batch: launch shape of the
 *   persistent transport (lanes waiting before events are handled, 256-lane
 *   blocks per compute unit -- 1 to 3 select the spill-free register form, 4
 *   or more the 128-register form --, packets a wave takes at once);
 *   0 = default.
 * graph: albedo and emission blocking solves: non-zero records the solve's
 *   device work (preparation, transport and reduction launches and their
 *   host-to-device parameter copies) as a hipGraph on the first call and
 *   replays it on later calls with identical arguments (same ids, parameters,
 *   packet_dump and stream, and the same library scratch buffers).  Results are
 *   identical to the eager path; profile is ignored (kernel_ms then holds the
 *   whole replay).  mcrt_solve_batch records likewise (the whole multi-grid
 *   chain: grid table, per-launch solve tables, preparation, transport and
 *   reduction of every launch).  The library keeps at most 16 graphs and
 *   drops those of a grid or table when it is freed.  Ignored by
 *   transmission and served requests.
 * contrib: mcrt_solve_albedo / mcrt_solve_emission only (EINVAL elsewhere):
 *   non-zero also fills mcrt_result.cf with the contribution functions.
 * image_npix: the same solves on a spherical grid: > 0 also fills
 *   mcrt_result.image with npix x npix images per band and observer
 *   (at most 4096).
 * g_sampling: albedo and emission with a correlated-k table: 0 = one solve
 *   per (band, g) weighted by w_g; 1, 2, 3 = n_packets packets per BAND, each
 *   drawing its g-ordinate (birth event, Philox block 3, slot a) from q(g)
 *   and weighted by p(g)/q(g), p(g) = w_g (albedo) or w_g L_g / sum(w L)
 *   (emission) (Sect. "G-ordinance biasing"): 1 unbiased (q = p), 2 uniform
 *   (q = 1/N_g), 3 composite (q = (p + 1/N_g)/2).  The band's sums, counters
 *   and value appear in its g = 0 slots of sums, counters and per_g; the
 *   packet dump is [band][packet][observer]; the random key's tag with
 *   decorrelate is 1 + band * ng.  Not with contrib, image_npix or
 *   mcrt_solve_batch (EINVAL).
 * cloud_phase: 0 = Henyey-Greenstein clouds; 1 = two-term HG (Sect. 3,
 *   aerosol scattering): forward lobe g1 = g with weight a = 1 - g2^2 and
 *   backward lobe g2 = -g/2, the lobe of a cloud scattering chosen by Philox
 *   block 2, slot b of the event (zeta < a: forward); the peel-off uses the
 *   mixture a P_HG(g1) + (1 - a) P_HG(g2).  2 = Draine's hybrid HG-Rayleigh
 *   function (same section) P_HG(G) (1 + alpha mu^2)/(1 + alpha (1 + 2 G^2)
 *   /3), alpha = draine_alpha, G found from the cloud's asymmetry factor g by
 *   bisection on the mean cosine; sampled exactly by rejection from HG(G):
 *   candidate 0 from block 1, slot a, accepted when block 2, slot b times
 *   (1 + alpha) < 1 + alpha mu^2, candidate k >= 1 from block 2 + k (slots a,
 *   b), the 32nd taken if none before is accepted.  Other values: EINVAL.
 * draine_alpha: in [0, 1] (default 0.5; 1 = Cornette-Shanks); EINVAL
 *   outside.
 * forced: forced interactions (Sect. 4, forced interaction), albedo,
 *   emission and multiple-scattering transmission: before a flight, an extra
 *   ray trace finds the optical depth tp to the edge of the grid along the
 *   packet direction (the top, or the planet / the slab floor); with
 *   0 < tp < inf the flight's tau is drawn with the flight's own zeta (block
 *   0, slot a) from a density q on [0, tp], the weight is multiplied by
 *   e^{-tau}/q(tau) and the fraction W e^{-tp} is booked as escaped (or to
 *   SURF when the path ends on the floor).  0 off; 1 forced scattering,
 *   q = e^{-tau}/(1 - e^{-tp}); 2 path-length stretching,
 *   q = l e^{-l tau}/(1 - e^{-l tp}) with l = 1/(1 + tp); 3 hybrid, the
 *   equal mixture, its component chosen by block 34, slot a < 1/2.  Needs
 *   MCRT_SURVIVAL and surface_albedo = 0 (EINVAL otherwise); the probe's
 *   crossings count in NCROSS.  A packet forced on every flight leaves only
 *   through the roulette or the event cap.
 * forced_first: 1 = only a packet's first flight is forced ("forced first
 *   scattering"); 0 = every flight.
 * surface_albedo: 0 = the lower boundary absorbs every packet that reaches
 *   it; A_s in (0, 1] = a Lambert floor (Sect. 3, surface scattering): a
 *   packet reaching it peels off W A_s max(n.o, 0)/pi e^{-tau} toward each
 *   observer (n: outward normal, the radial direction on a sphere, +z in a
 *   slab), leaves W (1 - A_s) in the SURF counter, keeps W A_s and leaves
 *   at cos(theta) = sqrt(zeta) from n, azimuth 2 pi zeta' (Philox block 1
 *   of the event); it counts as an interaction (NINT) and is subject to the
 *   roulette and the event cap.  Outside [0, 1]: EINVAL. */
typedef struct {
    uint64_t seed;
    uint64_t n_packets;
    int32_t decorrelate;
    int32_t precision;
    int32_t n_spec;
    const int32_t* spec_idx;
    int32_t n_obs;
    const double* obs_phase;
    const double* obs_dir;
    int32_t scattering;
    int32_t absorption;
    double rr_threshold;
    double rr_survive;
    double emis_bias;
    double tau_vert_max;
    double tau_peel_max;
    int64_t max_events;
    double mu0;
    int32_t n_b;
    int32_t n_alpha;
    double r_star;
    void* stream;
    double* packet_dump;
    int32_t profile;
    int32_t max_batch;
    int32_t tune_ev_threshold;
    int32_t tune_blocks_per_cu;
    int32_t tune_wave_batch;
    int32_t graph;
    int32_t contrib;
    int32_t image_npix;
    int32_t g_sampling;
    int32_t cloud_phase;
    double surface_albedo;
    int32_t ms_transmission;
    int32_t ld_law;
    double a_orbit;
    double ld_c1;
    double ld_c2;
    double transit_y;
    double transit_z;
    double draine_alpha;
    int32_t forced;
    int32_t forced_first;
} mcrt_solve_params;

void mcrt_default_params(mcrt_solve_params* p);

/* Results, caller-owned HOST arrays (any optional pointer may be NULL):
 * value[n_spec][n_obs]     band value: A_g(phase) = pi E for albedo, F_p
 *                          [erg/s/cm^2/cm] for emission, (R_p/R_star)^2 for
 *                          transmission (n_obs = 1), summed over g with w_g;
 * stderr_[n_spec][n_obs]   its Monte Carlo standard error (g independent);
 * per_g[n_spec][ng][n_obs] value of each g-ordinate;
 * sums[n_spec][ng][n_obs][2] raw (sum F, sum F^2) over packets;
 * counters[n_spec][ng][MCRT_NCOUNTERS];
 * l_tot[n_spec][ng]        emission: L_tot [erg/s/cm].
 * elapsed_ms receives the device time of the solve; with params.profile,
 * kernel_ms and kernel_launches the summed duration and count of the
 * dominant kernel's launches.  queued_ms and latency_ms are set by
 * mcrt_wait: time from submit to start, and from submit to completion.
 * cf[n_spec][n_obs][2][ncell] (with params.contrib; the contribution
 *   functions of the section on albedo and emission contribution functions):
 *   per band and observer, the share of the band value produced by
 *   peel-offs from events in each cell, [0] thermal (emission points) and
 *   [1] scattered (interactions); each (band, observer) block sums to 1, or is
 *   0 where the value is 0.  Cells are ordered as the grid's.  Tallied with
 *   FP64 atomics, so the last bits vary from run to run.
 * image[n_spec][n_obs][npix][npix] (with params.image_npix = npix): every
 *   peel-off added, scaled as the band value, to the pixel of its event point
 *   on the observer's sky plane; the pixels of a (band, observer) add up to
 *   its value.  Row index along the vertical axis e_v = the rotation axis z
 *   projected on the sky plane (x when the observer looks along z), column
 *   index along e_h = e_v x o; pixels cover [-R_TOA, R_TOA]^2 from the
 *   negative end.  FP64 atomics, as cf.
 * n_segments: transmission: the number of (chord, cell) segments of the
 *   chord geometry (each is read once per spectral row); 0 otherwise. */
typedef struct {
    double* value;
    double* stderr_;
    double* per_g;
    double* sums;
    double* counters;
    double* l_tot;
    double elapsed_ms;
    double kernel_ms;
    int64_t kernel_launches;
    double queued_ms;
    double latency_ms;
    double* cf;
    double* image;
    int64_t n_segments;
} mcrt_result;

/* Blocking solves.  Errors: EINVAL (bad parameters, incompatible grid /
 * opacity, e.g. emission on a slab), ENOTFOUND (ids), EBUDGET (scratch would
 * exceed the budget), EDEVICE (HIP failure; the context is then poisoned). */
int mcrt_solve_albedo(mcrt_ctx* ctx, int32_t grid_id, int32_t opac_id,
                      const mcrt_solve_params* params, mcrt_result* result);
int mcrt_solve_emission(mcrt_ctx* ctx, int32_t grid_id, int32_t opac_id,
                        const mcrt_solve_params* params, mcrt_result* result);
int mcrt_solve_transmission(mcrt_ctx* ctx, int32_t grid_id, int32_t opac_id,
                            const mcrt_solve_params* params, mcrt_result* result);

/* Allocation-free solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  mode = MCRT_MODE_ALBEDO or MCRT_MODE_EMISSION; otherwise the
 * same arguments, results and errors as mcrt_solve_albedo /
 * mcrt_solve_emission, and the same values bit for bit (the batch size does
 * not change a result).  The solve's scratch (optics, emission sources,
 * packet rows, tallies) is carved from one fixed device array of
 * MCRT_NOALLOC_SCRATCH_BYTES (256 MiB) that the library holds on every GPU
 * it runs on until the process ends (its address is looked up when a
 * context is created), so the call itself allocates no device or pinned
 * memory; as many (spectral point, g) solves share a transport launch as fit
 * in it (params.max_batch caps that).  The caller still provides resident
 * grids and tables and the host result arrays.  The array is shared by all
 * contexts on a GPU and keeps the last call's contents (each call clears
 * what must start at zero).  Calls that overlapped on one GPU would race on
 * it, so the library serialises them within a process: a call waits for the
 * previous one, which returns only when its results are copied out (each
 * process holds its own copy of the array).  Errors: EINVAL for
 * another mode, params.graph != 0, or when one launch of a single solve
 * (one band with g-ordinate sampling) needs more than the fixed scratch
 * (e.g. n_packets too large: each packet's row takes (n_obs + 11) * 8 B);
 * otherwise as for the blocking solves. */
#define MCRT_NOALLOC_SCRATCH_BYTES (256ull << 20)
int mcrt_solve_noalloc(mcrt_ctx* ctx, int32_t mode, int32_t grid_id, int32_t opac_id,
                       const mcrt_solve_params* params, mcrt_result* result);

/* Batched solves on grids of uneven size: n_items albedo / emission requests,
 * each with its own (spherical) grid, correlated-k table, spectral points and
 * packet count, share the common params (observers, scattering, absorption,
 * roulette, precision, tuning; params' spec_idx, n_packets and packet_dump
 * are ignored) and must have the same number of observers.  All their
 * (spectral point, g) solves run in as few multi-grid persistent launches as
 * the HBM budget allows.  results[q] is filled as for the single-request solve
 * of item q (elapsed_ms / kernel_ms are those of the whole batch); each result
 * equals the one item q gets alone.  Errors as for the blocking solves. */
typedef struct {
    int32_t mode;
    int32_t grid_id;
    int32_t opac_id;
    int32_t n_spec;
    const int32_t* spec_idx;
    uint64_t n_packets;
} mcrt_batch_item;

int mcrt_solve_batch(mcrt_ctx* ctx, int32_t n_items, const mcrt_batch_item* items,
                     const mcrt_solve_params* params, mcrt_result* results);

/* Autotuner for the persistent transport launch shape: runs short trial
 * solves of this request (up to 4 of its spectral points with its packet
 * count, at most 1e6 each) over event thresholds {20, 24, 28, 32}, blocks per
 * compute unit {3, 4} and wave batches {32, 128}, and writes the fastest into
 * params->tune_* (best_packets_per_s, if not NULL, receives its trial rate:
 * packets of all the trial's (spectral point, g) solves per second).
 * Results of a solve do not depend on these settings.  mode: MCRT_MODE_ALBEDO
 * or MCRT_MODE_EMISSION.  Errors as for the blocking solves. */
int mcrt_autotune(mcrt_ctx* ctx, int32_t mode, int32_t grid_id, int32_t opac_id,
                  mcrt_solve_params* params, double* best_packets_per_s);

/* Serving: asynchronous solves with continuous admission.
 * mcrt_submit copies params (and the arrays they point to; stream and
 * packet_dump are ignored) and queues the request; mode is MCRT_MODE_*.
 * Worker threads, each with its own HIP stream on a hardware queue of its
 * own (so their launches are not serialised behind each other), admit queued requests in
 * arrival order whenever the context's HBM budget covers the request's
 * device scratch (estimated at submit), so requests run concurrently on the
 * device while grids and tables stay resident.  A served request reaches
 * the device as persistent launches of at most 2^23 packets, each taking the
 * device's blocks shared among the requests running when it starts, so the
 * launches of concurrent requests are resident together.  Scratch that
 * blocking solves keep for their next call is released when it stands in
 * the way of a request and no blocking solve runs.  A request whose scratch
 * alone exceeds the budget is rejected at submit with MCRT_EBUDGET; one
 * that no longer fits when no other request is running (the memory went to
 * uploads, or to a blocking solve still running, after it was submitted)
 * fails with MCRT_EBUDGET instead of holding up the queue.
 * mcrt_poll sets *done to 1 once the request finished, failed or was
 * cancelled.  mcrt_wait blocks until then, copies the results into the
 * caller's arrays (shaped as for the blocking solve), forgets the ticket and
 * returns the request's own status (MCRT_ECANCELLED if cancelled).
 * mcrt_cancel removes a queued request (MCRT_EBUSY once it runs).
 * mcrt_serve_config sets the number of workers (1..16, default 3) before the
 * first submit.  The workers allocate their scratch stream-ordered from a
 * memory pool of the context, which keeps up to the budget's worth of freed
 * memory while workers run (trimmed first when a blocking allocation would
 * otherwise take the process past the budget) and is destroyed with the
 * context.  Requests on one context are independent: a result is the
 * same alone and in a mix (the RNG is keyed per request and tallies are
 * reduced in a fixed order). */
int mcrt_serve_config(mcrt_ctx* ctx, int32_t n_workers);
int mcrt_submit(mcrt_ctx* ctx, int32_t mode, int32_t grid_id, int32_t opac_id,
                const mcrt_solve_params* params, uint64_t* ticket);
int mcrt_poll(mcrt_ctx* ctx, uint64_t ticket, int32_t* done);
int mcrt_wait(mcrt_ctx* ctx, uint64_t ticket, mcrt_result* result);
int mcrt_cancel(mcrt_ctx* ctx, uint64_t ticket);

#ifdef __cplusplus
}
#endif
#endif /* MCRT_H */
