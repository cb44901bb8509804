// Internal structures shared by the host runtime (api.cpp) and the HIP
// kernels (kernels.hip).  Device pointers only; plain data.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcrt {

constexpr int kMaxObs = 8;
constexpr int kMaxSolvesPerLaunch = 1 << 20;  // solve index field of the transport's packed lane state
constexpr int kXcds = 8;                      // packet dispensers per launch, one per XCD
constexpr int kNCounters = 11;
enum Counter { K_ESC = 0, K_SURF, K_ABS, K_RR, K_CAP, K_LOST, K_NINT, K_NCROSS, K_NCAPPED, K_NLOST, K_W0 };

// Geometry of one resident grid.  The trigonometric edge tables are computed
// once at upload on the host.
struct GridDev {
    int geom;  // 0 spherical, 1 slab
    int nlon, nlat, nlay;
    int max_cross;
    const double* r;       // [nlay+1]
    const double* lat;     // [nlat+1]
    const double* lat_c2;  // cos^2(lat edge)
    const double* lat_s2;  // sin^2(lat edge)
    const double* lat_sin; // sin(lat edge)
    const double* lon;     // [nlon+1]
    const double* lon_s;   // sin(lon edge) [nlon]
    const double* lon_c;   // cos(lon edge) [nlon]
    const double* vol_r;   // (r_{k+1}^3 - r_k^3)/3 [nlay]
    // the edge values a crossing reads, in one array so that one base and a
    // per-lane offset reach any of them: r[k] at k; (lat, sin^2, cos^2) of
    // latitude edge e at lat_base + 3 e; (sin, cos) of longitude edge e at
    // lon_base + 2 e
    const double* faces;
    int lat_base, lon_base;
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
};

// Per-cell optical properties of one (spectral point, g) solve.
template <typename R>
struct OpticsDev {
    R* a_ext;   // extinction coefficient [1/cm]
    R* a_abs;   // absorption coefficient [1/cm]
    R* omega;   // single-scattering albedo
    R* p_gas;   // probability that a scattering is by gas (Rayleigh)
    R* g_cld;   // cloud HG asymmetry
};

// One (spectral point, g) solve inside a persistent transport launch.
// Optical-property arrays are double (FP64) or float (MIXED).
struct SolveDev {
    const void* a_ext;
    const void* a_abs;
    const void* omega;
    const void* p_gas;
    const void* g_cld;
    const double* cdf;     // emission only
    const double* wbirth;  // emission only
    unsigned long long begin;  // global index of the solve's first packet
    unsigned long long n;      // packets of the solve
    unsigned long long pbase;  // packet id 0 of the random stream (begin, or the band's first packet)
    uint32_t tag;
    int mode;  // 0 albedo, 1 emission
    int grid;  // index into BatchArgs.grids (multi-grid launches)
    // per-event tallies, each scaled by cf_w * (*cf_ltot if set):
    // contribution functions cf[(observer * 2 + part) * ncell + cell] and
    // images img[(observer * npix + row) * npix + column] (null = off)
    double* cf;
    double* img;
    double cf_w;
    const double* cf_ltot;
    // per-packet g-ordinate sampling: on the first solve of a band, the number
    // of g-ordinates (the band's solves follow it) and the scheme
    // (1 unbiased, 2 uniform, 3 composite); 0 = fixed-g solve
    int gs_n;
    int gs_scheme;
    const double* gs_w;    // g-ordinate weights of the table
    const double* ltot;    // emission: L_tot of this solve (written by the preparation)
};

// Stellar limb darkening of transmission chords and packets: law (0 none,
// 1 linear, 2 quadratic, 3 square-root, 4 logarithmic, 5 exponential,
// 6 power-2), its coefficients, the planet centre on the stellar disk (sky
// plane, cm) and the stellar radius.
struct LimbDark {
    int law;
    double c1, c2;
    double ty, tz;
    double r_star;
};

struct BatchArgs {
    const SolveDev* solves;
    int n_solves;
    const GridDev* grids;  // per-solve grids of a multi-grid launch (else unused)
    unsigned long long total;     // packets over all solves
    unsigned long long* counter;  // kXcds packet dispensers (one chunk of the packets each)
    double* rows;                 // [total][row_w]: F per observer, then counters
    int row_w;
    uint64_t seed;
    int scattering;
    int absorption;
    int n_obs;
    int n_out;
    long long max_events;
    double rr_threshold;
    double rr_survive;
    double tau_peel_max;
    double mu0;
    double r_toa;
    double obs[2][3 * kMaxObs];  // observer directions for albedo [0] and emission [1] solves
    int batch;         // packets a wave takes from the dispenser at once
    int ev_threshold;  // waiting lanes that trigger event handling
    int cloud_phase;   // 0 Henyey-Greenstein, 1 two-term Henyey-Greenstein, 2 Draine (g_cld holds G)
    double draine_alpha;
    double surface_albedo;  // 0: the lower boundary absorbs; > 0: Lambert albedo of the floor
    // transmission with multiple scattering: births on the annulus, the birth
    // peel-off is the direct light (no 1/4pi), later peel-offs are scaled by
    // peel_w (the stellar beam's solid angle; 1 otherwise), and a packet's
    // row holds W0 - F
    int trans_ms;
    double peel_w;
    int forced;        // forced interaction: 0 off, 1 forced scattering, 2 path-length stretching, 3 hybrid
    int forced_first;  // 1: only a packet's first flight
    LimbDark ld;
    // images: npix x npix pixels over [-img_half, img_half]^2 of each
    // observer's sky plane, horizontal / vertical unit vectors per observer
    int npix;
    double img_half;
    double img_axes[6 * kMaxObs];
};

// One solve slot of a batched preparation.
struct PrepSlot {
    const double* lnk;  // ck: ln kappa slice [T][P] of (band, g)
    double k_ray;       // Rayleigh opacity at the spectral point
    int n;              // hi-res: table wavelength index
    double lam_cm;      // emission: wavelength of B_lambda
    double* opt;        // FP64 optics: alpha_ext, alpha_abs, omega, P_gas, g (ncell each)
    float* optf;        // FP32 copies (mixed form) or null
    double* cdf;        // emission: L, then q, then the inclusive CDF
    double* wbirth;     // emission: (L_i/L_tot)/q_i
    double* stats;      // emission: (L_tot, N_emit)
};

void launch_prep_optics(const GridDev& g, int ncell, const PrepSlot* slots, int nslots, int hires, int nT,
                        int nP, const double* T_grid, const double* lnP_grid, const double* lnk_tpl, int nlam,
                        const double* shift, int draine, double alpha, hipStream_t stream);
void launch_prep_sources(const GridDev& g, int ncell, const PrepSlot* slots, int nslots, double tau_vert,
                         double xi, double* scratch, hipStream_t stream);
size_t prep_scratch_doubles(int ncell, int nslots);

void launch_transport_persistent(const GridDev& g, const BatchArgs& a, bool mixed, bool multi, int blocks,
                                 int blocks_per_cu, hipStream_t stream);
void launch_reduce_rows(const BatchArgs& a, const SolveDev* solves_host, int n_solves,
                        double* partials, int chunks, double* sums, int sums_w, double* dump,
                        hipStream_t stream);
int reduce_rows_chunks(unsigned long long max_n);
void launch_fill_u64(unsigned long long* p, unsigned long long v, hipStream_t stream);
void launch_init_dispensers(unsigned long long* counters, unsigned long long total, hipStream_t stream);
void launch_fill_f64(double* p, size_t n, double v, hipStream_t stream);
void launch_births(const GridDev& g, const BatchArgs& a, bool multi, hipStream_t stream);

// Launchers (kernels.hip).  All run on `stream`; none synchronises.
// R = double, or float for the mixed transmission form (stored once rounded).
template <typename R>
void launch_ck_optics(const GridDev& g, int ncell, const double* lnk_tab, int nT, int nP,
                      const double* T_grid, const double* lnP_grid, double k_ray,
                      OpticsDev<R> out, int ext_stride, hipStream_t stream);
void launch_doppler_shift(const GridDev& g, double ox, double oy, double oz, double dlnlam,
                          double* shift, hipStream_t stream);
// A cell's place in the opacity table's (T, ln P) grid: bracketing nodes
// and fractions, the same for every wavelength of a transmission solve.
struct CellTP {
    int ti0, ti1, pi0, pi1;
    double tt, pt;
};
void launch_cell_tp(const GridDev& g, int ncell, int nT, int nP, const double* T_grid, const double* lnP_grid,
                    CellTP* out, hipStream_t stream);
// lnk_tpl: the [T][P][lambda] ln-kappa table in the extinction's own type
// (FP64, or its FP32 copy for the mixed form).
template <typename R>
void launch_hires_alpha_block(const GridDev& g, int ncell, const R* lnk_tpl, int nlam, int nP,
                              const CellTP* tp, const double* k_ray, const double* shift, const int* nlist,
                              int nslot, int slot_stride, R* alpha, hipStream_t stream);
void launch_reduce_partials(const double* partials, int nblocks, int width, double* out,
                            hipStream_t stream);
void launch_chord_count(const GridDev& g, int n_b, int n_alpha, uint64_t seed, uint32_t tag,
                        int* counts, hipStream_t stream);
void launch_exclusive_scan_int(const int* in, long long* out, int n, long long* total_dev,
                               hipStream_t stream);
// R = double, or float for the mixed form (segment lengths and extinction rows).
template <typename R>
void launch_chord_fill(const GridDev& g, int n_b, int n_alpha, uint64_t seed, uint32_t tag,
                       const long long* offsets, uint32_t* seg_cell, R* seg_len,
                       double* chord_b, int* chord_ok, const LimbDark& ld, hipStream_t stream);
template <typename R>
void launch_chord_tau(int n_b, int n_alpha, const long long* offsets, const uint32_t* seg_cell,
                      const R* seg_len, const double* chord_b, const int* chord_ok,
                      const R* alpha, int nslot, double* partials, int nblocks,
                      hipStream_t stream);
int chord_tau_blocks(int nch);

}  // namespace mcrt
