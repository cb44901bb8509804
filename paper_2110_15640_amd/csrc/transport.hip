// K4: persistent packet transport with wavefront-level regeneration.
//
// Every lane of a wave64 carries one photon packet (Sect. 2: packets are
// emitted or injected, sample an optical depth, move sub-grid through the
// spherical cells, interact, scatter or are absorbed, and are peeled off
// toward every observer at each emission and interaction, Sect. 4.6).
// Flights and peel-off rays are both walks through the grid, so the
// cell-exit computation runs for all walking lanes together; the rarer
// events (interaction, end of a peel-off, death, birth) are handled only
// when at least ev_threshold lanes wait on one, or when no lane walks.
// Lanes whose packet has terminated take the next packet index from the
// wave's reservoir, refilled from a global dispenser, so the grid drains
// without tail imbalance and many (spectral point, g) solves share a launch.
//
// Per packet the kernel writes one row: the peel-off sums F_o toward each
// observer, then the bookkeeping counters.  A fixed-order reduction over the
// rows forms the tallies, so results are deterministic and identical whether
// a solve runs alone or inside a batch.
//
// Precision: FP64 keeps everything in double.  MIXED gathers float optical
// properties and evaluates phase functions, scattering angles, the direction
// rotation and the peel-off attenuation in float; positions, the directions
// the traversal uses, exit distances, optical depths and tallies stay double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <math.h>
#include <stdint.h>

#include "device_common.hpp"
#include "mcrt_internal.hpp"

namespace mcrt {
namespace {
using namespace dev;

// Lane modes; the walking ones come first: a flight, a peel-off ray, or the
// probe of a forced interaction (the optical depth to the grid's edge along
// the packet direction).
enum { M_FLIGHT = 0, M_PEEL = 1, M_PROBE = 2, M_EVENT = 3, M_DEAD = 4, M_BIRTH = 5, M_IDLE = 6 };
// Observer-field values outside the observer range: the walk that ended was a
// probe, or the next flight's optical depth is already chosen.
constexpr int kProbeDone = 15, kTauSet = 14;
enum { E_INTERACT = 0, E_ESCAPE = 1, E_SURFACE = 2, E_LOST = 3, E_PEEL_DONE = 4 };
// Birth record of a packet, kept in the counter columns of its row until the
// packet dies: position, direction, weight, packed cell (i | j << 11 | k << 21)
// * 8 + (entry face + 1) (-1: nothing emits), then the index of the solve
// whose optics it uses;
// with a Lambert floor, the weight the floor has absorbed so far; with
// forced interactions, the unscattered fractions booked so far to the floor
// (B_SURF) and to escape (B_FESC).
enum { B_X = 0, B_Y, B_Z, B_DX, B_DY, B_DZ, B_W, B_CELL, B_SOLVE, B_SURF, B_FESC };

__host__ __device__ __forceinline__ unsigned long long pack_ijk(int i, int j, int k)
{
    return (unsigned long long)i | ((unsigned long long)j << 11) | ((unsigned long long)k << 21);
}

// Per-lane state that the cell walk does not touch lives in LDS (one slot
// per lane, structure of arrays) so the registers hold only the walking ray;
// small fields are packed into 32-bit words.  The packet's peel-off sums
// accumulate in LDS too and reach memory once, with its whole row.
constexpr int kTPB = 256;
struct ColdLDS {
    double sx[kTPB], sy[kTPB], sz[kTPB];      // event point
    double sdx[kTPB], sdy[kTPB], sdz[kTPB];   // packet direction
    double W0[kTPB], w_rr[kTPB];
    unsigned long long gid[kTPB];
    uint32_t ijk[kTPB];   // event cell: i | j << 11 | k << 21
    uint32_t st[kTPB];    // observer:4 | birth:1 | smode:1 | entry face + 1:3 | capped:1 | lost:1 | surface:1 | solve:20
    uint32_t e[kTPB];
    int nint[kTPB];
};

// A bit field [sh, sh + w) of a packed LDS word, used like an int.
struct Bits {
    uint32_t* p;
    int sh;
    uint32_t m;
    __device__ operator int() const { return (int)((*p >> sh) & m); }
    __device__ Bits& operator=(int v)
    {
        *p = (*p & ~(m << sh)) | (((uint32_t)v & m) << sh);
        return *this;
    }
    __device__ Bits& operator+=(int v) { return *this = (int)*this + v; }
};

struct Lane {
    Walker w;      // the walking ray (flight or peel-off)
    double tau;    // flight: optical depth left; peel-off: accumulated
    double W, w_abs;
    int ncw;       // crossings of the current walk
    int ncross;
    int mode, ev;
    // cold state in LDS, accessed through these references
    ColdLDS* C;
    double* F;     // peel-off sums, F[o * kTPB + t]
    int t;
    __device__ double& sx() { return C->sx[t]; }
    __device__ double& sy() { return C->sy[t]; }
    __device__ double& sz() { return C->sz[t]; }
    __device__ double& sdx() { return C->sdx[t]; }
    __device__ double& sdy() { return C->sdy[t]; }
    __device__ double& sdz() { return C->sdz[t]; }
    __device__ double& W0() { return C->W0[t]; }
    __device__ double& w_rr() { return C->w_rr[t]; }
    __device__ unsigned long long& gid() { return C->gid[t]; }
    __device__ uint32_t& e() { return C->e[t]; }
    __device__ int& nint() { return C->nint[t]; }
    __device__ double& Fo(int o) { return F[o * kTPB + t]; }
    __device__ Bits o() { return Bits{&C->st[t], 0, 0xFu}; }
    __device__ Bits birth() { return Bits{&C->st[t], 4, 0x1u}; }
    __device__ Bits smode() { return Bits{&C->st[t], 5, 0x1u}; }
    __device__ int sef() { return (int)((C->st[t] >> 6) & 0x7u) - 1; }
    __device__ void set_sef(int ef) { Bits{&C->st[t], 6, 0x7u} = ef + 1; }
    __device__ Bits ncapped() { return Bits{&C->st[t], 9, 0x1u}; }
    __device__ Bits nlost() { return Bits{&C->st[t], 10, 0x1u}; }
    __device__ Bits surf() { return Bits{&C->st[t], 11, 0x1u}; }  // the event is a reflection by the floor
    __device__ int solve() { return (int)(C->st[t] >> 12); }
    __device__ void set_solve(int s) { Bits{&C->st[t], 12, 0xFFFFFu} = s; }
    __device__ int si() { return (int)(C->ijk[t] & 0x7FFu); }
    __device__ int sj() { return (int)((C->ijk[t] >> 11) & 0x3FFu); }
    __device__ int sk() { return (int)(C->ijk[t] >> 21); }
    __device__ void set_cell(int i, int j, int k) { C->ijk[t] = (uint32_t)i | ((uint32_t)j << 11) | ((uint32_t)k << 21); }
    __device__ int cell(const GridDev& g) { return (sk() * g.nlat + sj()) * g.nlon + si(); }
};

// floor(total * x / kXcds) without overflow.
__device__ __forceinline__ unsigned long long chunk_edge(unsigned long long total, int x)
{
    return (total / kXcds) * (unsigned long long)x + (total % kXcds) * (unsigned long long)x / kXcds;
}

template <bool MIXED>
__device__ __forceinline__ double ld(const void* p, int c)
{
    // per-cell optical properties live in global memory: load through the
    // global address space (a global, not a flat, load)
    typedef const __attribute__((address_space(1))) float gfloat;
    typedef const __attribute__((address_space(1))) double gdouble;
    if (MIXED) return (double)((gfloat*)p)[c];
    return ((gdouble*)p)[c];
}

// Address of cell c's value in a per-cell array of the precision's type.
template <bool MIXED>
__device__ __forceinline__ const void* cell_addr(const void* p, int c)
{
    return MIXED ? (const void*)((const float*)p + c) : (const void*)((const double*)p + c);
}

// Write the packet's row: its peel-off sums, then the counters; `kind` says
// where its remaining weight went.  EXT (here and below): the kernel form
// with the Lambert floor, Draine clouds, forced interactions and
// multiple-scattering transmission; without it that code is compiled out.
template <bool EXT>
__device__ __forceinline__ void finish_packet(Lane& L, const BatchArgs& A, int kind)
{
    double* row = A.rows + L.gid() * (unsigned long long)A.row_w;
    for (int o = 0; o < A.n_out; ++o) row[o] = (EXT && A.trans_ms) ? L.W0() - L.Fo(o) : L.Fo(o);
    row += A.n_out;
    if (EXT) {
        // weight booked before the end: absorbed by a Lambert floor (which
        // never ends a packet) or the unscattered fractions of forced flights
        const double wsurf = (A.surface_albedo > 0.0 || A.forced) ? row[B_SURF] : 0.0;
        const double wesc = A.forced ? row[B_FESC] : 0.0;
        row[K_ESC] = kind == K_ESC ? wesc + L.W : wesc;
        row[K_SURF] = kind == K_SURF ? wsurf + L.W : wsurf;
    } else {
        row[K_ESC] = kind == K_ESC ? L.W : 0.0;
        row[K_SURF] = kind == K_SURF ? L.W : 0.0;
    }
    row[K_ABS] = L.w_abs;
    row[K_RR] = L.w_rr();
    row[K_CAP] = kind == K_CAP ? L.W : 0.0;
    row[K_LOST] = kind == K_LOST ? L.W : 0.0;
    row[K_NINT] = (double)L.nint();
    row[K_NCROSS] = (double)L.ncross;
    row[K_NCAPPED] = (double)L.ncapped();
    row[K_NLOST] = (double)L.nlost();
    row[K_W0] = L.W0();
    L.mode = M_DEAD;
}

__device__ __forceinline__ void observer(Lane& L, const BatchArgs& A, const double* sobs, double& ox, double& oy,
                                         double& oz)
{
    if (A.n_obs == 0) {  // slab backscatter: minus the incidence direction of the birth record
        const double* b = A.rows + L.gid() * (unsigned long long)A.row_w + A.n_out;
        ox = -b[B_DX];
        oy = 0.0;
        oz = -b[B_DZ];
    } else {
        const double* ob = sobs + L.smode() * (3 * kMaxObs);
        ox = ob[3 * L.o()];
        oy = ob[3 * L.o() + 1];
        oz = ob[3 * L.o() + 2];
    }
}

// Start the lane's next walk from its event point: a flight along the
// packet direction (optical depth drawn from the event's block 0, slot a,
// unless a forced interaction chose it), a peel-off ray toward the current
// observer, or, before a forced flight, the probe along the packet
// direction.  All use one inlined walker start, so a wave starting several
// kinds runs it once.
template <bool MIXED, bool EXT>
__device__ __forceinline__ void start_walk(Lane& L, const GridDev& g, const BatchArgs& A, const double* sobs,
                                           bool flight)
{
    double dx, dy, dz;
    int ef;
    if constexpr (!EXT) {
        if (flight) {
            const SolveDev& S = A.solves[L.solve()];
            U2 u = draw(A.seed, S.tag, L.gid() - S.pbase, L.e(), 0);
            L.tau = -log(u.a);
            dx = L.sdx();
            dy = L.sdy();
            dz = L.sdz();
            ef = L.sef();
        } else {
            observer(L, A, sobs, dx, dy, dz);
            L.tau = 0.0;
            ef = F_NONE;
        }
        wk_start<MIXED>(g, L.w, L.sx(), L.sy(), L.sz(), dx, dy, dz, L.si(), L.sj(), L.sk(), ef);
        L.ncw = 0;
        L.mode = flight ? M_FLIGHT : M_PEEL;
        if (!flight && g.geom == 1 && !(dz > 0.0)) {  // a slab peel-off ray that never reaches the top
            L.tau = INFINITY;
            L.mode = M_EVENT;
            L.ev = E_PEEL_DONE;
        }
    } else {
        int kind = flight ? M_FLIGHT : M_PEEL;
        if (flight && A.forced != 0 && L.o() != kTauSet && (A.forced_first == 0 || L.e() == 1)) kind = M_PROBE;
        if (kind == M_FLIGHT) {
            if (A.forced != 0 && L.o() == kTauSet) {
                L.o() = 0;
            } else {
                const SolveDev& S = A.solves[L.solve()];
                U2 u = draw(A.seed, S.tag, L.gid() - S.pbase, L.e(), 0);
                L.tau = -log(u.a);
            }
            ef = L.sef();
        } else {
            L.tau = 0.0;
            ef = F_NONE;
        }
        if (kind == M_PEEL) {
            observer(L, A, sobs, dx, dy, dz);
        } else {
            dx = L.sdx();
            dy = L.sdy();
            dz = L.sdz();
        }
        if (kind == M_PROBE) L.o() = kProbeDone;
        wk_start<MIXED>(g, L.w, L.sx(), L.sy(), L.sz(), dx, dy, dz, L.si(), L.sj(), L.sk(), ef);
        L.ncw = 0;
        L.mode = kind;
        // a slab peel-off ray that never reaches the top, or a floor peel-off
        // ray below the horizon (the floor's normal is the packet direction then)
        const bool dark = kind == M_PEEL && ((g.geom == 1 && !(dz > 0.0)) ||
                                             (L.surf() && !(L.sdx() * dx + L.sdy() * dy + L.sdz() * dz > 0.0)));
        if (dark) {
            L.tau = INFINITY;
            L.mode = M_EVENT;
            L.ev = E_PEEL_DONE;
        }
    }
}

// One cell of a walk.  Flights and peel-off rays share the exit search, the
// extinction gather and the crossing (a single inlined copy of each, so that
// a wave holding both kinds executes them once); they differ only in how the
// optical depth is used and in when the walk stops.  Every walking lane runs
// the crossing: a lane whose walk ends in this cell (interaction, surface
// hit, end of a peel-off) discards its walker afterwards, so the walker is
// never kept in two versions.
template <bool MIXED, bool EXT>
__device__ __forceinline__ void walk_step(Lane& L, const GridDev& g, const void* aext, const void* aabs,
                                          const BatchArgs& A, double r_top)
{
    double tf;
    const int f = wk_next<MIXED>(g, L.w, tf, r_top);
    const double s = tf - L.w.t;
    const int c = wk_cell(g, L.w);
    const bool flight = L.mode == M_FLIGHT;
    const bool cont = flight && A.absorption == 1;
    // the walk's parameter and cell before the crossing (the walker keeps its
    // origin and direction, so the interaction point follows from them)
    const double t0 = L.w.t;
    const int ei = L.w.i, ej = L.w.j, ek = L.w.k;
    // the grid-table loads of the crossing, then the extinction gather (its
    // address formed first); the crossing's arithmetic waits only for the
    // former, so the gather's latency overlaps it
    const void* pe = cell_addr<MIXED>(aext, c);
    const CrossIn xin = wk_cross_begin<MIXED>(g, L.w, f, tf);
    const double ae = ld<MIXED>(pe, 0);
    const double aa = cont ? ld<MIXED>(aabs, c) : 0.0;
    const bool inside = wk_cross_end<MIXED>(g, L.w, f, xin);
    const double a = cont ? (ae - aa) : ae;
    const bool lost = flight && f == F_NONE && !(a > 0.0);
    const bool hit = flight && !lost && a > 0.0 && L.tau < a * s;
    const bool pend = !flight && f == F_NONE;
    if (flight) {
        if (!lost && !hit) L.tau = wk_mad<MIXED>(-a, s, L.tau);
        if (cont && !lost) {
            const double ds = hit ? wk_div<MIXED>(L.tau, a) : s;
            double wn = L.W * exp(-aa * ds);
            L.w_abs = L.w_abs + (L.W - wn);
            L.W = wn;
        }
    } else if (!pend) {
        L.tau = wk_mad<MIXED>(ae, s, L.tau);
    }
    if (lost || hit || pend) {
        L.ncross += L.ncw;
        L.mode = M_EVENT;
        if (hit) {  // at t0 + tau / a (tau is still the depth left on entering the cell)
            const double ti = t0 + wk_div<MIXED>(L.tau, a);
            L.sx() = wk_mad<MIXED>(ti, L.w.dx, L.w.px);
            L.sy() = wk_mad<MIXED>(ti, L.w.dy, L.w.py);
            L.sz() = wk_mad<MIXED>(ti, L.w.dz, L.w.pz);
            L.set_cell(ei, ej, ek);
            L.set_sef(F_NONE);
        }
        if (pend) L.tau = INFINITY;
        L.ev = lost ? E_LOST : (hit ? E_INTERACT : E_PEEL_DONE);
        return;
    }
    L.ncw++;
    bool done;
    if (flight) {
        done = !inside || L.ncw >= g.max_cross;
        if (done) L.ev = !inside ? (L.w.k >= g.nlay ? E_ESCAPE : E_SURFACE) : E_LOST;
    } else {
        // a probe runs to the edge of the grid, the floor included; a
        // peel-off ray stops beyond tau_peel_max or on the planet
        const bool probe = EXT && L.mode == M_PROBE;
        done = true;
        if (L.tau > (probe ? INFINITY : A.tau_peel_max)) L.tau = INFINITY;
        else if (!inside) { if (L.w.k < 0 && !probe) L.tau = INFINITY; }
        else if (L.ncw >= g.max_cross) L.tau = INFINITY;
        else done = false;
        if (done) L.ev = E_PEEL_DONE;
    }
    if (done) {
        L.ncross += L.ncw;
        L.mode = M_EVENT;
    }
}

// Pending actions of a lane after an event; each is executed at exactly one
// place in the kernel loop so its code (and register demand) appears once.
enum { A_NONE = 0, A_PEEL = 1, A_FLIGHT = 2, A_SCATTER = 3, A_FINISH = 4 };

// Survival weight update, scattering angle, rotation, roulette, event cap.
// A reflection by the Lambert floor takes the same steps: its albedo is A_s,
// its absorbed share goes to the floor, and its polar cosine about the
// normal (held as the packet direction) is sqrt(zeta), block 1, slot a.
template <bool MIXED, bool EXT>
__device__ __forceinline__ int scatter(Lane& L, const GridDev& g, const BatchArgs& A, const SolveDev& S)
{
    const unsigned long long q = L.gid() - S.pbase;
    const bool sf = EXT && L.surf();
    const int c = L.cell(g);
    const double om = sf ? A.surface_albedo : ld<MIXED>(S.omega, c);
    const double pg = sf ? 0.0 : ld<MIXED>(S.p_gas, c), gc = sf ? 0.0 : ld<MIXED>(S.g_cld, c);
    if (sf) {
        double* b = A.rows + L.gid() * (unsigned long long)A.row_w + A.n_out;
        b[B_SURF] = b[B_SURF] + L.W * (1.0 - om);
        L.W = L.W * om;
    } else if (A.absorption != 1) {
        L.w_abs += L.W * (1.0 - om);
        L.W = L.W * om;
    }
    const double usel = draw(A.seed, S.tag, q, L.e(), 0).b;  // scatterer choice of this event
    U2 u1 = draw(A.seed, S.tag, q, L.e(), 1);
    // two-term HG clouds: the forward lobe g with weight 1 - (g/2)^2 or the
    // backward lobe -g/2, chosen by block 2, slot b of the event
    double globe = gc;
    if (A.cloud_phase == 1 && !sf && !(usel < pg)) {
        const double g2 = -0.5 * gc, a = 1.0 - g2 * g2;
        globe = draw(A.seed, S.tag, q, L.e(), 2).b < a ? gc : g2;
    }
    // Draine clouds (g_cld holds G): rejection from HG(G), candidate 0 from
    // block 1, slot a with acceptance block 2, slot b; candidate k >= 1 from
    // block 2 + k; at most 32 candidates
    const bool draine = EXT && A.cloud_phase == 2 && !sf && !(usel < pg);
    if (MIXED) {
        float z = fminf((float)u1.a, 0.99999994f);
        float mu;
        float g32 = (float)globe;
        auto hgs = [g32](float zz) {
            if (fabsf(g32) < 1e-6f) return 2.0f * zz - 1.0f;
            const float t = (1.0f - g32 * g32) / (1.0f - g32 + 2.0f * g32 * zz);
            return (1.0f + g32 * g32 - t * t) / (2.0f * g32);
        };
        if (sf) {
            mu = sqrtf(z);
        } else if ((float)usel < (float)pg) {
            float qq = 4.0f * z - 2.0f;
            float u = cbrtf(qq + sqrtf(qq * qq + 1.0f));
            mu = u - 1.0f / u;
        } else {
            mu = hgs(z);
        }
        if (draine) {
            const float al = (float)A.draine_alpha;
            float zc = (float)draw(A.seed, S.tag, q, L.e(), 2).b;
            for (int k = 1; k < 32 && !(zc * (1.0f + al) < 1.0f + al * mu * mu); ++k) {
                const U2 cd = draw(A.seed, S.tag, q, L.e(), 2 + k);
                mu = hgs(fminf((float)cd.a, 0.99999994f));
                zc = (float)cd.b;
            }
        }
        mu = fminf(fmaxf(mu, -1.0f), 1.0f);
        float st = sqrtf(fmaxf(1.0f - mu * mu, 0.0f));
        float sp, cp;
        __sincosf((float)(2.0 * kPi) * (float)u1.b, &sp, &cp);
        float dx = (float)L.sdx(), dy = (float)L.sdy(), dz = (float)L.sdz();
        float nx, ny, nz;
        if (fabsf(dz) < 0.99999f) {
            float t = sqrtf(1.0f - dz * dz);
            float it = 1.0f / t;
            nx = st * (dx * dz * cp - dy * sp) * it + dx * mu;
            ny = st * (dy * dz * cp + dx * sp) * it + dy * mu;
            nz = -st * cp * t + dz * mu;
        } else {
            float sgn = dz >= 0.0f ? 1.0f : -1.0f;
            nx = st * cp;
            ny = st * sp;
            nz = sgn * mu;
        }
        // renormalised in FP64 (the traversal takes |d| = 1): one refined
        // reciprocal square root and three products
        double ddx = nx, ddy = ny, ddz = nz;
        const double nn = fma(ddx, ddx, fma(ddy, ddy, ddz * ddz));
        double y = __builtin_amdgcn_rsq(nn);
        y = y * fma(-0.5 * nn, y * y, 1.5);
        y = y * fma(-0.5 * nn, y * y, 1.5);
        L.sdx() = ddx * y;
        L.sdy() = ddy * y;
        L.sdz() = ddz * y;
    } else {
        double mu = sf ? sqrt(u1.a) : ((usel < pg) ? sample_rayleigh(u1.a) : sample_hg(u1.a, globe));
        if (draine) {
            const double al = A.draine_alpha;
            double zc = draw(A.seed, S.tag, q, L.e(), 2).b;
            for (int k = 1; k < 32 && !(zc * (1.0 + al) < 1.0 + al * mu * mu); ++k) {
                const U2 cd = draw(A.seed, S.tag, q, L.e(), 2 + k);
                mu = sample_hg(cd.a, globe);
                zc = cd.b;
            }
        }
        rotate_dir(L.sdx(), L.sdy(), L.sdz(), mu, 2.0 * kPi * u1.b);
    }
    if (L.W < A.rr_threshold * L.W0()) {
        U2 u2 = draw(A.seed, S.tag, q, L.e(), 2);
        if (u2.a < A.rr_survive) {
            double wn = L.W / A.rr_survive;
            L.w_rr() -= (wn - L.W);
            L.W = wn;
        } else {
            L.w_rr() += L.W;
            L.W = 0.0;
            L.ev = -1;
            return A_FINISH;
        }
    }
    if ((long long)L.e() >= A.max_events) {
        L.ncapped() += 1;
        L.ev = K_CAP;
        return A_FINISH;
    }
    L.e() += 1;
    return A_FLIGHT;
}

// Pixel of a sky-plane coordinate x on npix pixels over [-half, half].
__device__ __forceinline__ int pixel_of(double x, double half, int npix)
{
    const int q = (int)floor((x + half) / (2.0 * half) * (double)npix);
    return q < 0 ? 0 : (q >= npix ? npix - 1 : q);
}

// Bookkeeping of one event; returns the action that follows.  L.ev carries
// the counter that receives the final weight when the action is A_FINISH.
template <bool MIXED, bool EXT>
__device__ __forceinline__ int handle_event(Lane& L, const GridDev& g, const BatchArgs& A)
{
    const SolveDev& S = A.solves[L.solve()];
    if (EXT && L.ev == E_PEEL_DONE && L.o() == kProbeDone) {
        // forced interaction: with the path's optical depth tp known, the
        // flight's tau comes from a density on [0, tp], the weight takes the
        // factor e^{-tau}/q(tau) and the unscattered fraction W e^{-tp} is
        // booked where the path ends (nothing is forced when tp is 0 or
        // infinite: a walk failure or the crossing cap)
        const double tp = L.tau;
        const unsigned long long q = L.gid() - S.pbase;
        const U2 u = draw(A.seed, S.tag, q, L.e(), 0);
        double tau = -log(u.a);
        if (tp > 0.0 && tp < INFINITY) {
            double wf;
            tau = forced_tau(A.forced, tp, u.a, draw(A.seed, S.tag, q, L.e(), 34).a, wf);
            double* b = A.rows + L.gid() * (unsigned long long)A.row_w + A.n_out;
            const int slot = L.w.k < 0 ? B_SURF : B_FESC;
            b[slot] = b[slot] + L.W * exp(-tp);
            L.W = L.W * wf;
        }
        L.tau = tau;
        L.o() = kTauSet;
        return A_FLIGHT;
    }
    if (L.ev == E_PEEL_DONE) {
        double f;
        // attenuation e^{-tau} in FP32 in the mixed form, as for the scattered peel-offs below
        const double att = MIXED ? (double)(L.tau < INFINITY ? __expf(-(float)L.tau) : 0.0f) : exp(-L.tau);
        if (L.birth()) {  // emission point (isotropic), or a transmission chord's direct light
            f = (EXT && A.trans_ms) ? L.W * att : L.W * att / (4.0 * kPi);
        } else if (EXT && L.surf()) {  // Lambert floor: W A_s max(n.o, 0)/pi e^{-tau}, n held as the direction
            const double mu = L.sdx() * L.w.dx + L.sdy() * L.w.dy + L.sdz() * L.w.dz;
            f = mu > 0.0 ? L.W * A.surface_albedo * (mu / kPi) * att : 0.0;
        } else {
            // normalised mixture of the Rayleigh and cloud phase functions
            // toward the observer, weighted by the gas scattering probability
            const int c = L.cell(g);
            const double om = ld<MIXED>(S.omega, c), pg = ld<MIXED>(S.p_gas, c), gc = ld<MIXED>(S.g_cld, c);
            if (MIXED) {
                float mu = (float)(L.sdx() * L.w.dx + L.sdy() * L.w.dy + L.sdz() * L.w.dz);
                float pgf = (float)pg, gcf = (float)gc;
                float pr = 0.75f * (1.0f + mu * mu);
                auto hgf = [mu](float gg) {
                    if (!(fabsf(gg) >= 1e-6f)) return 1.0f;
                    const float den = 1.0f + gg * gg - 2.0f * gg * mu;
                    return (1.0f - gg * gg) / (den * sqrtf(den));
                };
                float ph;
                if (A.cloud_phase == 1) {
                    const float g2 = -0.5f * gcf, af = 1.0f - g2 * g2;
                    ph = af * hgf(gcf) + (1.0f - af) * hgf(g2);
                } else if (EXT && A.cloud_phase == 2) {  // Draine (gcf is G)
                    const float al = (float)A.draine_alpha;
                    ph = hgf(gcf) * (1.0f + al * mu * mu) / (1.0f + al * (1.0f + 2.0f * gcf * gcf) / 3.0f);
                } else {
                    ph = hgf(gcf);
                }
                float theta = (pgf * pr + (1.0f - pgf) * ph) * (float)(0.25 / kPi);
                float w = A.absorption == 1 ? (float)L.W : (float)(L.W * om);
                f = (double)(w * theta * (float)att);
            } else {
                double mu = L.sdx() * L.w.dx + L.sdy() * L.w.dy + L.sdz() * L.w.dz;
                double pc;
                if (A.cloud_phase == 1) {
                    const double g2 = -0.5 * gc, a = 1.0 - g2 * g2;
                    pc = a * p_hg(mu, gc) + (1.0 - a) * p_hg(mu, g2);
                } else if (EXT && A.cloud_phase == 2) {  // Draine (gc is G)
                    const double al = A.draine_alpha;
                    pc = p_hg(mu, gc) * (1.0 + al * mu * mu) / (1.0 + al * (1.0 + 2.0 * gc * gc) / 3.0);
                } else {
                    pc = p_hg(mu, gc);
                }
                double theta = (pg * p_rayleigh(mu) + (1.0 - pg) * pc) / (4.0 * kPi);
                f = A.absorption == 1 ? L.W * theta * att : L.W * om * theta * att;
            }
        }
        // scattered light of a transmission packet: per steradian, over the
        // stellar beam's solid angle (peel_w = 1 otherwise)
        if (EXT && !L.birth()) f = f * A.peel_w;
        L.Fo(L.o()) += f;
        if ((S.cf || S.img) && f > 0.0) {
            const double sc = f * (S.cf_ltot ? S.cf_w * *S.cf_ltot : S.cf_w);
            if (S.cf) {  // contribution function: the event's cell, thermal or scattered part
                const int ncell = g.nlon * g.nlat * g.nlay;
                const int c = L.cell(g);
                unsafeAtomicAdd(S.cf + ((size_t)L.o() * 2 + (L.birth() ? 0 : 1)) * ncell + c, sc);
            }
            if (S.img) {  // image: the event point on the observer's sky plane
                const double* eh = A.img_axes + 6 * L.o();
                const double u = L.sx() * eh[0] + L.sy() * eh[1] + L.sz() * eh[2];
                const double v = L.sx() * eh[3] + L.sy() * eh[4] + L.sz() * eh[5];
                const int col = pixel_of(u, A.img_half, A.npix), row = pixel_of(v, A.img_half, A.npix);
                unsafeAtomicAdd(S.img + ((size_t)L.o() * A.npix + row) * A.npix + col, sc);
            }
        }
        L.o() += 1;
        if (L.o() < A.n_out) return A_PEEL;
        if (L.birth()) {
            L.birth() = 0;
            if (!A.scattering) {
                L.ev = K_ESC;
                return A_FINISH;
            }
            L.e() = 1;
            return A_FLIGHT;
        }
        return A_SCATTER;
    }
    if (L.ev == E_INTERACT) {
        L.nint() += 1;
        L.o() = 0;
        L.birth() = 0;
        if (EXT) L.surf() = 0;
        return A_PEEL;
    }
    if (EXT && L.ev == E_SURFACE && A.surface_albedo > 0.0) {
        // the floor reflects: an event on the surface of the lowest cell,
        // entered through its inner face; until the reflection the packet
        // direction holds the floor's outward normal (radial on a sphere, +z
        // in a slab)
        L.nint() += 1;
        const double x = L.w.px + L.w.t * L.w.dx, y = L.w.py + L.w.t * L.w.dy;
        const double z = g.geom == 1 ? g.r[0] : L.w.pz + L.w.t * L.w.dz;
        L.sx() = x;
        L.sy() = y;
        L.sz() = z;
        if (g.geom == 1) {
            L.sdx() = 0.0;
            L.sdy() = 0.0;
            L.sdz() = 1.0;
        } else {
            const double rr = sqrt(x * x + y * y + z * z);
            L.sdx() = x / rr;
            L.sdy() = y / rr;
            L.sdz() = z / rr;
        }
        L.set_cell(L.w.i, L.w.j, 0);
        L.set_sef(F_IN);
        L.o() = 0;
        L.birth() = 0;
        L.surf() = 1;
        return A_PEEL;
    }
    if (L.ev == E_LOST) L.nlost() += 1;
    L.ev = L.ev == E_ESCAPE ? K_ESC : (L.ev == E_SURFACE ? K_SURF : K_LOST);
    return A_FINISH;
}

// Index of the solve that owns global packet gid (last solve with begin <= gid).
__device__ __forceinline__ int solve_of(const BatchArgs& A, unsigned long long gid)
{
    int lo = 0, hi = A.n_solves - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (A.solves[mid].begin <= gid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}


// K4a: births of every packet of a batch (albedo: uniform on the top disk or
// the slab's incidence; emission: cell from the biased CDF, uniform position in
// its volume, isotropic direction, weight (L_i/L_tot)/q_i), one thread each.
//
// blk_sv >= 0: the solve every packet of the calling block belongs to (found
// once per block); tab: when that solve is an emission solve with a fixed g,
// 256 samples of its CDF, tab[m] = cdf[(m ncell) >> 8], which narrow the
// search for the birth cell to the range between two samples (same cell as
// the search over the whole CDF: see below).
template <bool MULTI>
__device__ __forceinline__ void birth_record(const GridDev& g1, const BatchArgs& A, unsigned long long gid, double* b,
                                             int blk_sv, const double* tab)
{
    int sv = blk_sv >= 0 ? blk_sv : solve_of(A, gid);
    const GridDev& g = MULTI ? A.grids[A.solves[sv].grid] : g1;
    const double r_toa = g.r[g.nlay];
    const unsigned long long q = gid - A.solves[sv].pbase;
    const uint32_t tag = A.solves[sv].tag;
    double wmul = 1.0;
    if (A.solves[sv].gs_n > 0) {
        // per-packet g-ordinate: p(g) = w_g (albedo) or w_g L_g / sum(w L)
        // (emission); sampled from q(g) (1: p, 2: uniform, 3: (p + 1/N_g)/2)
        // with the smallest g whose cumulative weight exceeds u times the total
        const SolveDev& H = A.solves[sv];
        const int ng = H.gs_n, scheme = H.gs_scheme;
        double ptot = 0.0;
        for (int h = 0; h < ng; ++h) ptot += H.ltot ? H.gs_w[h] * *A.solves[sv + h].ltot : H.gs_w[h];
        if (!(ptot > 0.0)) {  // nothing emits in any g-ordinate
            b[B_W] = 0.0;
            b[B_CELL] = -1.0;
            b[B_SOLVE] = (double)sv;
            return;
        }
        double qtot = 0.0;
        for (int h = 0; h < ng; ++h) {
            const double raw = H.ltot ? H.gs_w[h] * *A.solves[sv + h].ltot : H.gs_w[h];
            qtot += scheme == 1 ? raw : (scheme == 2 ? 1.0 : 0.5 * (raw / ptot) + 0.5 / ng);
        }
        const double target = draw(A.seed, tag, q, 0, 3).a * qtot;
        double cum = 0.0;
        int gi = ng - 1;
        double pg = 0.0, qg = 0.0;
        for (int h = 0; h < ng; ++h) {
            const double raw = H.ltot ? H.gs_w[h] * *A.solves[sv + h].ltot : H.gs_w[h];
            const double qh = scheme == 1 ? raw : (scheme == 2 ? 1.0 : 0.5 * (raw / ptot) + 0.5 / ng);
            cum += qh;
            if (cum > target) {
                gi = h;
                pg = raw / ptot;
                qg = qh;
                break;
            }
            if (h == ng - 1) {
                pg = raw / ptot;
                qg = qh;
            }
        }
        wmul = scheme == 1 ? 1.0 : (scheme == 2 ? pg * ng : pg / qg);
        sv += gi;
    }
    const SolveDev& S = A.solves[sv];
    b[B_SOLVE] = (double)sv;
    if (S.mode == 0) {
        U2 u = draw(A.seed, tag, q, 0, 0);
        if (g.geom == 1) {
            double mu0 = A.mu0 > 0.0 ? A.mu0 : sqrt(1.0 - u.a);
            b[B_X] = 0.0; b[B_Y] = 0.0; b[B_Z] = g.r[g.nlay];
            b[B_DX] = sqrt(fmax(1.0 - mu0 * mu0, 0.0)); b[B_DY] = 0.0; b[B_DZ] = -mu0;
            b[B_CELL] = (double)(((unsigned long long)(g.nlay - 1) << 21) * 8 + (F_OUT + 1));
        } else {
            double rho = r_toa * sqrt(u.a);
            double a = 2.0 * kPi * u.b;
            double y = rho * cos(a), z = rho * sin(a);
            double x = sqrt(fmax(r_toa * r_toa - y * y - z * z, 0.0));
            Ray rs;
            rs.x = x; rs.y = y; rs.z = z;
            locate_column(g, rs);
            b[B_X] = x; b[B_Y] = y; b[B_Z] = z;
            b[B_DX] = -1.0; b[B_DY] = 0.0; b[B_DZ] = 0.0;
            b[B_CELL] = (double)(pack_ijk(rs.i, rs.j, g.nlay - 1) * 8 + (F_OUT + 1));
        }
        b[B_W] = wmul;
        return;
    }
    if (S.mode == 2) {
        // transmission: a random point of the annulus R0 <= bi <= R_TOA, the
        // stellar beam along -x, weight bi times the limb-darkening fraction
        U2 u = draw(A.seed, tag, q, 0, 0);
        const double r0 = g.r[0];
        const double bi = r0 + u.a * (r_toa - r0);
        const double al = 2.0 * kPi * u.b;
        Ray rs;
        rs.x = sqrt(fmax(r_toa * r_toa - bi * bi, 0.0));
        rs.y = bi * cos(al);
        rs.z = bi * sin(al);
        locate_column(g, rs);
        b[B_X] = rs.x; b[B_Y] = rs.y; b[B_Z] = rs.z;
        b[B_DX] = -1.0; b[B_DY] = 0.0; b[B_DZ] = 0.0;
        b[B_CELL] = (double)(pack_ijk(rs.i, rs.j, g.nlay - 1) * 8 + (F_OUT + 1));
        b[B_W] = bi * limb_weight(A.ld, rs.y, rs.z) * wmul;
        return;
    }
    const int ncell = g.nlon * g.nlat * g.nlay;
    const double tot = S.cdf[ncell - 1];
    if (!(tot > 0.0)) {  // nothing emits
        b[B_W] = 0.0;
        b[B_CELL] = -1.0;
        return;
    }
    U2 u0 = draw(A.seed, tag, q, 0, 0);
    U2 u1 = draw(A.seed, tag, q, 0, 1);
    U2 u2 = draw(A.seed, tag, q, 0, 2);
    double target = u0.a * tot;
    int lo = 0, hi = ncell - 1;  // smallest c with cdf[c] > target (else ncell - 1)
    if (tab != nullptr && sv == blk_sv) {
        // m = the first sample above target; the cell lies after sample m - 1
        // (every cdf value up to it is <= target) and at or before sample m
        // (its value is > target); past the last sample, up to ncell - 1
        int a = 0, z = 256;
        while (a < z) {
            const int mid = (a + z) >> 1;
            if (tab[mid] > target) z = mid;
            else a = mid + 1;
        }
        lo = a == 0 ? 0 : (int)(((unsigned long long)(a - 1) * (unsigned)ncell) >> 8) + 1;
        hi = a == 256 ? ncell - 1 : (int)(((unsigned long long)a * (unsigned)ncell) >> 8);
    }
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (S.cdf[mid] > target) hi = mid;
        else lo = mid + 1;
    }
    int c = lo < ncell ? lo : ncell - 1;
    int i = c % g.nlon, j = (c / g.nlon) % g.nlat, k = c / (g.nlon * g.nlat);
    double rk = g.r[k], rk1 = g.r[k + 1];
    double rk3 = rk * rk * rk;
    double rk13 = rk1 * rk1 * rk1;
    double r = cbrt(rk3 + u0.b * (rk13 - rk3));
    double sl0 = g.lat_sin[j], sl1 = g.lat_sin[j + 1];
    double sl = sl0 + u1.a * (sl1 - sl0);
    double cl = sqrt(fmax(1.0 - sl * sl, 0.0));
    double lon = g.lon[i] + u1.b * (g.lon[i + 1] - g.lon[i]);
    b[B_X] = r * cl * cos(lon);
    b[B_Y] = r * cl * sin(lon);
    b[B_Z] = r * sl;
    double mu = 2.0 * u2.a - 1.0;
    double sp = sqrt(fmax(1.0 - mu * mu, 0.0));
    double psi = 2.0 * kPi * u2.b;
    b[B_DX] = sp * cos(psi);
    b[B_DY] = sp * sin(psi);
    b[B_DZ] = mu;
    b[B_W] = S.wbirth[c] * wmul;
    b[B_CELL] = (double)(pack_ijk(i, j, k) * 8 + (F_NONE + 1));
}

// The records of a block's packets are built in LDS and its rows written
// as one contiguous range (peel-off columns as zeros): coalesced stores of
// whole lines instead of 72 B pieces of 120 B rows.  Dynamic LDS: 256 CDF
// samples, then 256 rows of row_w doubles (row_w = n_obs + kNCounters <= 19,
// sized at launch, so a narrow row leaves room for more resident blocks).
template <bool MULTI>
__global__ void __launch_bounds__(256) k_births(GridDev g1, BatchArgs A)
{
    extern __shared__ double births_lds[];
    double* tab = births_lds;
    double* sh = births_lds + 256;
    __shared__ int blk[2];  // the block's solve (-1: several), and whether tab holds its CDF samples
    const int w = A.row_w;
    const unsigned long long r0 = (unsigned long long)blockIdx.x * 256;
    const unsigned long long left = A.total - r0;
    if (threadIdx.x == 0) {
        const int sv = solve_of(A, r0);
        const SolveDev& S = A.solves[sv];
        const unsigned long long last = r0 + (left < 256 ? left : 256) - 1;
        const bool one = r0 >= S.begin && last < S.begin + S.n;
        blk[0] = one ? sv : -1;
        blk[1] = one && S.mode == 1 && S.gs_n == 0;
    }
    __syncthreads();
    const int blk_sv = blk[0];
    const bool use_tab = blk[1] != 0;
    if (use_tab) {
        const SolveDev& S = A.solves[blk_sv];
        const GridDev& g = MULTI ? A.grids[S.grid] : g1;
        const unsigned ncell = (unsigned)(g.nlon * g.nlat * g.nlay);
        tab[threadIdx.x] = S.cdf[((unsigned long long)threadIdx.x * ncell) >> 8];
    }
    double* mine = sh + threadIdx.x * w;
    for (int c = 0; c < w; ++c) mine[c] = 0.0;
    __syncthreads();
    const unsigned long long gid = r0 + threadIdx.x;
    if (gid < A.total) birth_record<MULTI>(g1, A, gid, mine + A.n_out, blk_sv, use_tab ? tab : nullptr);
    __syncthreads();
    const int n = (int)(left < 256 ? left : 256) * w;
    double* dst = A.rows + r0 * (unsigned long long)w;
    for (int x = threadIdx.x; x < n; x += 256) dst[x] = sh[x];
}

// New packet L.gid: load its birth record and return the first action (a
// flight for albedo, the emission-point peel-off, or finish if none emits).
template <bool EXT>
__device__ __forceinline__ int birth(Lane& L, const GridDev& g, const BatchArgs& A)
{
    const double* b = A.rows + L.gid() * (unsigned long long)A.row_w + A.n_out;
    if (EXT) {
        double* bw = A.rows + L.gid() * (unsigned long long)A.row_w + A.n_out;
        if (A.surface_albedo > 0.0 || A.forced) bw[B_SURF] = 0.0;
        if (A.forced) bw[B_FESC] = 0.0;
    }
    const int sv = (int)b[B_SOLVE];
    const SolveDev& S = A.solves[sv];
    L.C->st[L.t] = 0u;
    L.set_solve(sv);
    L.smode() = S.mode == 1;  // the emission observer set; albedo and transmission use the other
    for (int o = 0; o < A.n_out; ++o) L.Fo(o) = 0.0;
    L.w_abs = 0.0;
    L.w_rr() = 0.0;
    L.ncross = 0;
    L.nint() = 0;
    L.e() = 1;
    const double cw = b[B_CELL];
    L.W = b[B_W];
    L.W0() = L.W;
    if (cw < 0.0) {
        L.ev = -1;
        return A_FINISH;
    }
    const unsigned long long cc = (unsigned long long)cw;
    L.C->ijk[L.t] = (uint32_t)(cc >> 3);
    L.set_sef((int)(cc & 7) - 1);
    L.sx() = b[B_X]; L.sy() = b[B_Y]; L.sz() = b[B_Z];
    L.sdx() = b[B_DX]; L.sdy() = b[B_DY]; L.sdz() = b[B_DZ];
    if (S.mode == 0) return A_FLIGHT;
    L.birth() = 1;
    return A_PEEL;
}

// MINB: blocks per CU the register allocation is sized for (4: at most 128
// VGPRs per lane, 16 waves per CU, with some spills; 2: no spills, ~170 VGPRs,
// so up to 3 waves per SIMD = 3 blocks per CU), chosen at launch from the
// requested blocks per CU.
template <bool MIXED, bool MULTI, int MINB, bool EXT>
__global__ void __launch_bounds__(kTPB, MINB) k_transport_persistent(GridDev g1, BatchArgs A)
{
    __shared__ double sobs[2 * 3 * kMaxObs];
    __shared__ ColdLDS cold;
    __shared__ double Fsh[kMaxObs * kTPB];
    if (threadIdx.x < 2 * 3 * kMaxObs) sobs[threadIdx.x] = A.obs[threadIdx.x / (3 * kMaxObs)][threadIdx.x % (3 * kMaxObs)];
    __syncthreads();
    int lgrid = 0;  // grid of the lane's packet (multi-grid launches)
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    unsigned long long res_next = 0, res_end = 0;
    bool exhausted = false;
    Lane L;
    L.C = &cold;
    L.F = Fsh;
    L.t = threadIdx.x;
    L.mode = M_DEAD;
    cold.st[threadIdx.x] = 0u;
    const void* aext = nullptr;
    const void* aabs = nullptr;
    const double r_top1 = MULTI ? 0.0 : g1.r[g1.nlay];  // top of the grid (the fast walk's tolerance scale)
    for (;;) {
        const GridDev& g = MULTI ? A.grids[lgrid] : g1;
        if (L.mode <= M_PROBE) walk_step<MIXED, EXT>(L, g, aext, aabs, A, MULTI ? g.r[g.nlay] : r_top1);
        unsigned long long evm = __ballot(L.mode == M_EVENT);
        unsigned long long walking = __ballot(L.mode <= M_PROBE);
        if (__popcll(evm) < A.ev_threshold && walking != 0) continue;
        int act = A_NONE;
        if (L.mode == M_EVENT) act = handle_event<MIXED, EXT>(L, g, A);
        if (act == A_SCATTER) act = scatter<MIXED, EXT>(L, g, A, A.solves[L.solve()]);
        for (int pass = 0; pass < 2; ++pass) {
            if (act == A_FINISH) {
                finish_packet<EXT>(L, A, L.ev);
                act = A_NONE;
            }
            if (pass == 1) break;
            // regeneration: dead lanes take the next packets of the reservoir
            unsigned long long dead = __ballot(L.mode == M_DEAD);
            while (dead != 0) {
                if (res_next >= res_end) {
                    if (exhausted) break;
                    // the packet range is split into one contiguous chunk per XCD (blocks are
                    // dealt to the XCDs round-robin), so each XCD's L2 holds the optics of
                    // its own solves; a wave whose chunk is drained helps the next ones
                    unsigned long long base = 0, end = 0;
                    if (lane == 0) {
                        const int x0 = (int)(blockIdx.x % kXcds);
                        for (int q = 0; q < kXcds; ++q) {
                            const int x = (x0 + q) % kXcds;
                            const unsigned long long lim = chunk_edge(A.total, x + 1);
                            const unsigned long long b = atomicAdd(A.counter + x, (unsigned long long)A.batch);
                            if (b < lim) {
                                base = b;
                                end = b + (unsigned long long)A.batch < lim ? b + A.batch : lim;
                                break;
                            }
                        }
                    }
                    base = __shfl(base, 0);
                    end = __shfl(end, 0);
                    if (end == 0) {
                        exhausted = true;
                        break;
                    }
                    res_next = base;
                    res_end = end;
                }
                unsigned long long avail = res_end - res_next;
                int cnt = __popcll(dead);
                int take = (unsigned long long)cnt < avail ? cnt : (int)avail;
                int rank = __popcll(dead & below);
                if (L.mode == M_DEAD && rank < take) {
                    L.gid() = res_next + (unsigned long long)rank;
                    L.mode = M_BIRTH;
                }
                res_next += (unsigned long long)take;
                dead = __ballot(L.mode == M_DEAD);
            }
            if (L.mode == M_DEAD && exhausted) L.mode = M_IDLE;
            if (L.mode == M_BIRTH) {
                if (MULTI) lgrid = A.solves[solve_of(A, L.gid())].grid;
                const GridDev& gb = MULTI ? A.grids[lgrid] : g1;
                act = birth<EXT>(L, gb, A);
                const SolveDev& S = A.solves[L.solve()];  // the solve the birth record chose
                aext = S.a_ext;
                aabs = S.a_abs;
            }
        }
        const GridDev& ga = MULTI ? A.grids[lgrid] : g1;
        if (act == A_FLIGHT || act == A_PEEL) start_walk<MIXED, EXT>(L, ga, A, sobs, act == A_FLIGHT);
        if (__ballot(L.mode != M_IDLE) == 0) break;
    }
}

// Fixed-order reduction of the packet rows of every solve: block (chunk, s)
// sums rows [chunk*kChunk, (chunk+1)*kChunk) of solve s into
// partials[s][chunk][2*n_out + kNCounters]; then one block per (s, column)
// sums the chunks.  Optional copy of F to a packet dump.
//
// Thread t of a chunk block owns column t % w of the rows t / w, t / w + R,
// ... (w the row width, R = 256 / w rows per pass), so each pass of the
// block reads R whole rows as one contiguous, coalesced range; the R
// per-thread sums of a column are then added in row-slot order.
constexpr int kChunk = 4096;
constexpr int kRT = 256;

__global__ void __launch_bounds__(kRT) k_rows_partial(BatchArgs A, double* __restrict__ partials, int chunks,
                                                      double* __restrict__ dump)
{
    __shared__ double sh[2 * kRT];
    const int s = blockIdx.y;
    const SolveDev S = A.solves[s];
    const int w = A.row_w;  // n_out peel-off sums + the counters
    const int R = kRT / w;
    const int t = threadIdx.x;
    const int c = t % w, r0 = t / w;
    const unsigned long long q0 = (unsigned long long)blockIdx.x * kChunk;
    const unsigned long long qe = q0 + kChunk < S.n ? q0 + kChunk : S.n;
    const double* rows = A.rows + S.begin * (unsigned long long)w + c;
    double acc = 0.0, acc2 = 0.0;
    if (r0 < R) {
#pragma unroll 4
        for (unsigned long long q = q0 + r0; q < qe; q += R) {
            const double v = rows[q * (unsigned long long)w];
            acc = acc + v;
            acc2 = acc2 + v * v;
            if (dump && c < A.n_out) dump[(S.begin + q) * (unsigned long long)A.n_out + c] = v;
        }
    }
    sh[t] = acc;
    sh[kRT + t] = acc2;
    __syncthreads();
    if (t < w) {
        double tot = 0.0, tot2 = 0.0;
        for (int j = 0; j < R; ++j) {
            tot = tot + sh[t + j * w];
            tot2 = tot2 + sh[kRT + t + j * w];
        }
        const int pw = 2 * A.n_out + kNCounters;
        double* out = partials + ((size_t)s * chunks + blockIdx.x) * pw;
        if (t < A.n_out) {
            out[2 * t] = tot;
            out[2 * t + 1] = tot2;
        } else {
            out[2 * A.n_out + (t - A.n_out)] = tot;
        }
    }
}

__global__ void __launch_bounds__(kRT) k_rows_final(const double* __restrict__ partials, int chunks, int pw,
                                                    double* __restrict__ sums, int sums_w)
{
    __shared__ double sh[kRT];
    __shared__ double shc[kRT];
    const int s = blockIdx.y, col = blockIdx.x;
    double acc = 0.0, comp = 0.0;
    for (int c = threadIdx.x; c < chunks; c += kRT) {
        double x = partials[((size_t)s * chunks + c) * pw + col];
        double t = acc + x;
        comp = comp + (fabs(acc) >= fabs(x) ? ((acc - t) + x) : ((x - t) + acc));
        acc = t;
    }
    sh[threadIdx.x] = acc;
    shc[threadIdx.x] = comp;
    __syncthreads();
    for (int st = kRT / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            double a = sh[threadIdx.x], b = sh[threadIdx.x + st];
            double t = a + b;
            double e = fabs(a) >= fabs(b) ? ((a - t) + b) : ((b - t) + a);
            sh[threadIdx.x] = t;
            shc[threadIdx.x] = shc[threadIdx.x] + shc[threadIdx.x + st] + e;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[(size_t)s * sums_w + col] = sh[0] + shc[0];
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Packet dispensers of a launch: counter x starts at the first packet of
// chunk x = [edge(x), edge(x + 1)), edge(x) = floor(total * x / kXcds).
__global__ void k_init_dispensers(unsigned long long* c, unsigned long long total)
{
    if (blockIdx.x == 0 && threadIdx.x < kXcds) c[threadIdx.x] = chunk_edge(total, (int)threadIdx.x);
}

// Fill n doubles (a kernel, so that recorded graphs hold no memset nodes).
__global__ void __launch_bounds__(256) k_fill_f64(double* __restrict__ p, size_t n, double v)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) p[i] = v;
}

}  // namespace

void launch_births(const GridDev& g, const BatchArgs& a, bool multi, hipStream_t stream)
{
    dim3 grid((unsigned)((a.total + 255) / 256));
    const size_t lds = (size_t)(256 + 256 * a.row_w) * sizeof(double);  // <= 40 KB
    if (multi) hipLaunchKernelGGL(k_births<true>, grid, dim3(256), lds, stream, g, a);
    else hipLaunchKernelGGL(k_births<false>, grid, dim3(256), lds, stream, g, a);
}

void launch_transport_persistent(const GridDev& g, const BatchArgs& a, bool mixed, bool multi, int blocks,
                                 int blocks_per_cu, hipStream_t stream)
{
    const bool wide = blocks_per_cu <= 3;  // up to 256 VGPRs: at most 3 waves per SIMD
    // the extended form only when a launch uses one of its features
    const bool ext = a.surface_albedo > 0.0 || a.cloud_phase == 2 || a.forced != 0 || a.trans_ms != 0;
#define MCRT_K4(MX, MU, EX)                                                                                      \
    if (wide)                                                                                                    \
        hipLaunchKernelGGL((k_transport_persistent<MX, MU, 2, EX>), dim3(blocks), dim3(kTPB), 0, stream, g, a); \
    else                                                                                                         \
        hipLaunchKernelGGL((k_transport_persistent<MX, MU, 4, EX>), dim3(blocks), dim3(kTPB), 0, stream, g, a);
#define MCRT_K4X(MX, MU)              \
    if (ext) { MCRT_K4(MX, MU, true) } \
    else { MCRT_K4(MX, MU, false) }
    if (mixed && multi) { MCRT_K4X(true, true) }
    else if (mixed) { MCRT_K4X(true, false) }
    else if (multi) { MCRT_K4X(false, true) }
    else { MCRT_K4X(false, false) }
#undef MCRT_K4X
#undef MCRT_K4
}

int reduce_rows_chunks(unsigned long long max_n) { return (int)((max_n + kChunk - 1) / kChunk); }

void launch_reduce_rows(const BatchArgs& a, const SolveDev* /*solves_host*/, int n_solves, double* partials,
                        int chunks, double* sums, int sums_w, double* dump, hipStream_t stream)
{
    const int pw = 2 * a.n_out + kNCounters;
    hipLaunchKernelGGL(k_rows_partial, dim3(chunks, n_solves), dim3(kRT), 0, stream, a, partials, chunks, dump);
    hipLaunchKernelGGL(k_rows_final, dim3(pw, n_solves), dim3(kRT), 0, stream, partials, chunks, pw, sums, sums_w);
}

void launch_fill_u64(unsigned long long* p, unsigned long long v, hipStream_t stream)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, stream, p, v);
}

void launch_init_dispensers(unsigned long long* counters, unsigned long long total, hipStream_t stream)
{
    hipLaunchKernelGGL(k_init_dispensers, dim3(1), dim3(64), 0, stream, counters, total);
}

void launch_fill_f64(double* p, size_t n, double v, hipStream_t stream)
{
    if (n == 0) return;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, v);
}

}  // namespace mcrt
