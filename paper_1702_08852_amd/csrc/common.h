// Internal declarations shared by the HIP sources of the dual messenger library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dmwf.h"

namespace dmwf {

// Waves per Legendre workgroup, each on its own m (consecutive m share a CU).
#ifndef DMWF_LEG_WAVES
#define DMWF_LEG_WAVES 2
#endif
constexpr int kLegWaves = DMWF_LEG_WAVES;
// l values per block of the Legendre kernels: recurrences start only at the
// first l of a block (counted from m), and the analysis reduces once per block.
constexpr int kLegB = 16;
// Launch classes of the ring stage (by FFT length; ring.hip), and the side
// streams they run on beside the caller's
constexpr int kRingClasses = 5;
constexpr int kRingSide = 3;
// Padding (entries) after the per-(l,m) tables so that look-ahead reads of
// the recurrence coefficients stay inside the allocation.
constexpr int kTablePad = 64;
// A term lambda_lm with |lambda_lm| below 2^kSkipLog2 is treated as zero:
// the recurrence starts at the first l where the magnitude reaches it.
constexpr int kSkipLog2 = -100;
// Sentinel start index for (m, ring) pairs that never reach the threshold.
constexpr int kNever = 0x3fffffff;

enum ProfClass {
    PROF_SEED = 0,
    PROF_LEG_ANA,
    PROF_LEG_SYN,
    PROF_DIAG,
    PROF_RING_ITER,
    PROF_RING_SYN,
    PROF_RING_ANA,
    PROF_REDUCE,
    PROF_MISC,
    PROF_COUNT
};

struct ProfEvent {
    int cls;
    hipEvent_t start, stop;
};

// Device-side description of the ring grid, one entry per ring pair q:
// q < 2N-1 pairs north ring q+1 with south ring 4N-1-q (1-based ring numbers),
// q = 2N-1 is the equator alone.
struct RingGeom {
    const double* x;          // cos(theta) of the north ring
    const double* sint;       // sin(theta)
    const int* nph;           // pixels in each ring of the pair
    const double* phi0pi;     // phi of the first pixel divided by pi
    const long long* start_n; // first pixel of the north ring
    const long long* start_s; // first pixel of the south ring, -1 for the equator
};

// Device-side control of the solve loop.  The host enqueues iterations in
// batches; after each iteration a one-block kernel sums the Cauchy partials,
// takes the level decision of the cooling schedule and, once the solve has
// stopped, sets `done`, after which every iteration kernel returns at once.
struct DevLevel {
    double xi, mu, xi_over_sigma, eps;
    int ell, ell_next;  // l_iter of this level and of the next (the last: its own)
    int replay;         // iterations to run on this level when replaying, else 0
    int pad;
};
struct DevCtrl {
    int done;    // nonzero: the solve has stopped
    int status;  // 0 converged, 1 iteration cap reached, 2 NaN Cauchy ratio
    int level, it_level, total, nlev, max_iter, replay;
    double xi, mu, xi_over_sigma, ratio;
    double alpha;  // min N over unmasked pixels of this map
    int reduced;      // reduced-precision plan: 1 while the Legendre contractions
                      // of this map run on the matrix cores, 0 once they run in FP64
    int it_reduced;   // iterations run with the reduced contractions
    double eps_reduced;  // on the last level, below this ratio the map switches to FP64
    double best;      // smallest ratio seen on the last level in reduced precision
    int stall;        // iterations since `best` last improved by 1%
    int pad;
};
// Most cooling levels one solve may have (the per-level m-bound table is
// kMaxLevels x ring pairs ints of workspace).
constexpr int kMaxLevels = 1024;

// Workspace layout (byte offsets from the workspace base).  The per-map
// regions hold one slice per map of the plan, map k at offset + k * stride.
struct WsLayout {
    size_t spec;       // complex [nq][lp][2] per map: ring Fourier coefficients F_m / G_m
    size_t part;       // complex [nchunk_ana][n_alm + pad] per map: analysis partial sums
    size_t ap;         // complex [n_alm + pad] per map: g-scaled a_lm for the synthesis
    size_t aux;        // complex [n_alm + pad] per map: second a_lm-sized buffer
    size_t cpart;      // double  [nmaps][nq][2]: Cauchy partial sums per ring pair
    size_t mhi;        // int     [nmaps][nq]: per ring pair, the largest m carried at l_iter
    size_t ells;       // int     [3][nmaps]: l_iter, analysis band, input flags per map
    size_t mdbl;       // double  [nmaps][4]: Cauchy sums (2), max N^-1, spare
    size_t bmax;       // double  [nmaps][kCheckBlocks]: block maxima of N^-1
    size_t scal;       // shared scalars: a band-limit int, residual block sums
    size_t ctrl;       // DevCtrl [nmaps]
    size_t levels;     // DevLevel [nmaps][kMaxLevels]
    size_t lev_iters;  // int [nmaps][kMaxLevels]: iterations run per level
    size_t mhi_tab;    // int [nmaps][kMaxLevels][nq]: m bound of every ring pair per level
    size_t total;
    // per-map strides in elements of each region's type
    long long spec_map, part_map, alm_map;
};

// Blocks of the per-map input screening reduction.
constexpr int kCheckBlocks = 1024;

// The maps of one Legendre launch.
struct LegMaps {
    int nm;               // maps in the launch
    const int* ell;       // band limit of map k at ell[k * ell_stride] (device)
    int ell_stride;       // 0: one band limit for every map
    const DevCtrl* ctrl;  // per-map control blocks, or NULL; a stopped map is skipped
    int sel = 0;          // with ctrl: 0 every map, 1 the maps whose contraction runs
                          // in FP64, 2 those on the matrix cores (DevCtrl::reduced)
};

}  // namespace dmwf

struct dmwf_plan {
    int nside, lmax, nmaps, nq, nrings, device;
    // Legendre contraction: DMWF_FP64 (VALU), DMWF_FP32_GEMM or DMWF_BF16X3_GEMM
    // (matrix cores; the recurrence stays FP64)
    int prec = DMWF_FP64;
    long long npix, nalm;
    int nchunk_ana;  // analysis ring chunks (partial-sum rows per map)
    // Legendre tiles, set by default and by dmwf_autotune.  Synthesis: ring
    // pairs per lane (1 or 2) and maps per wave (1, 2, 4 or 8; the recurrence
    // is computed once for all of them).  Analysis: ring pairs per lane (4 or
    // 8; nchunk_ana follows) and maps per wave (1 or 2).
    int syn_k = 2, syn_mb = 1, ana_mb = 1, ana_k = 8;
    int ana_k_min = 8;  // smallest analysis tile the partial-sum buffer holds
    int lp;        // m-row length of the ring-major F/G buffer, lmax+1 rounded up to 4
    double omega;  // 4 pi / Npix
    // device tables
    double* d_x = nullptr;
    double* d_sint = nullptr;
    int* d_nph = nullptr;
    double* d_phi0pi = nullptr;
    long long* d_start_n = nullptr;
    long long* d_start_s = nullptr;
    double* d_A = nullptr;  // recurrence multipliers A_lm, m-major, + pad
    double* d_g = nullptr;  // scale g_lm with lambda_lm = g_lm mu_lm, + pad
    int* d_ls = nullptr;    // [(lmax+1)][nq] first significant l
    int* d_lsmin = nullptr; // [nq][(lmax+1)] min over m' >= m of d_ls (non-decreasing in m)
    int* d_mhi_full = nullptr; // [nq] largest m with d_lsmin <= lmax, or -1
    double* d_s0 = nullptr; // mu at ls-1
    double* d_s1 = nullptr; // mu at ls
    std::vector<int> h_ls;  // host copy of d_ls, made by dmwf_legendre_work
    // ring FFT tables (see ring.hip)
    int* d_ring_M = nullptr;           // per q: FFT length (n, or the Bluestein length)
    int* d_ring_blue = nullptr;        // per q: 1 if the ring length is not a power of two
    long long* d_ring_coff = nullptr;  // per q: offset into the chirp table
    long long* d_ring_boff = nullptr;  // per q: offset into the filter-spectrum table
    double2* d_chirp = nullptr;        // e^{i pi t^2 / n}, t < n, per Bluestein ring
    double2* d_bspec = nullptr;        // FFT_M of the chirp filter, per Bluestein ring
    int* d_ring_class = nullptr;       // q lists of the launch classes, concatenated
    int class_off[dmwf::kRingClasses + 1] = {};
    // side streams (default priority) on which the smaller launch classes run
    // concurrently with the largest, forked from and joined to the caller's
    // stream with events
    hipStream_t ring_side[dmwf::kRingSide] = {};
    hipEvent_t ring_fork = nullptr;
    hipEvent_t ring_join[dmwf::kRingSide] = {};
    dmwf::WsLayout ws;
    // pinned host copy of the control block, read after each batch of the
    // solve loop (two batches in flight)
    dmwf::DevCtrl* h_ctrl = nullptr;
    hipEvent_t batch_ev[2] = {nullptr, nullptr};
    // stream (default priority) on which the solve loop captures its iteration
    hipStream_t cap_stream = nullptr;
    // profiling
    int prof = 0;  // 0 off, 1 every launch, 2 the Legendre analysis launches only
    std::vector<dmwf::ProfEvent> events;
    std::vector<hipEvent_t> event_pool;  // recorded events are returned here on read
    dmwf::RingGeom geom() const {
        return {d_x, d_sint, d_nph, d_phi0pi, d_start_n, d_start_s};
    }
};

namespace dmwf {

void set_error(const std::string& msg);

// Check a HIP call; on failure record the message and return DMWF_ERR_HIP.
#define DMWF_HIP(call)                                                          \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess) {                                                 \
            ::dmwf::set_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
            return DMWF_ERR_HIP;                                                \
        }                                                                       \
    } while (0)

inline hipEvent_t pool_event(dmwf_plan* p) {
    hipEvent_t e = nullptr;
    if (!p->event_pool.empty()) {
        e = p->event_pool.back();
        p->event_pool.pop_back();
    } else {
        (void)hipEventCreate(&e);
    }
    return e;
}

// Bracket a launch with profiling events (recorded on the launch stream) when enabled.
struct ProfScope {
    dmwf_plan* p;
    hipStream_t s;
    int cls;
    hipEvent_t a = nullptr, b = nullptr;
    bool on;
    ProfScope(dmwf_plan* p_, hipStream_t s_, int c_)
        : p(p_), s(s_), cls(c_), on(p_->prof == 1 || (p_->prof == 2 && c_ == PROF_LEG_ANA)) {
        if (on) {
            a = pool_event(p);
            b = pool_event(p);
            (void)hipEventRecord(a, s);
        }
    }
    ~ProfScope() {
        if (on) {
            (void)hipEventRecord(b, s);
            p->events.push_back({cls, a, b});
        }
    }
};

// Largest m <= ell whose suffix-minimum recurrence start row[m] is <= ell, or
// -1 if none: beyond it every lambda_lm of the ring pair lies past the band
// limit.  row = lsmin of one ring pair, non-decreasing in m (binary search).
__device__ inline int m_bound(const int* row, int ell, int lmax) {
    int hi = ell < lmax ? ell : lmax;
    if (hi < 0 || row[0] > ell) return -1;
    int lo = 0;  // row[lo] <= ell
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row[mid] <= ell) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__host__ __device__ inline long long alm_base(int m, int lmax) {
    // slot of (l, m) is alm_base(m) + l
    return (long long)m * (2LL * lmax + 1 - m) / 2;
}

// ---- launchers (ring.hip, legendre.hip, api.hip) ----
dmwf_status launch_seeds(dmwf_plan* p, hipStream_t s);
// Legendre stages over the maps of lm.  ap, spec and part point at map 0's
// slice; the per-map strides are the workspace's.
dmwf_status launch_leg_syn(dmwf_plan* p, const double2* ap, double2* spec, const LegMaps& lm,
                           int mb, hipStream_t s);
dmwf_status launch_leg_ana(dmwf_plan* p, const double2* spec, double2* part, const LegMaps& lm,
                           int mb, hipStream_t s);
// The same two stages with the contraction on the matrix cores in the plan's
// reduced precision (legendre_mx.hip); every map of lm, or with lm.ctrl the
// maps lm.sel selects.
dmwf_status launch_leg_syn_mx(dmwf_plan* p, const double2* ap, double2* spec, const LegMaps& lm,
                              hipStream_t s);
dmwf_status launch_leg_ana_mx(dmwf_plan* p, const double2* spec, double2* part, const LegMaps& lm,
                              hipStream_t s);

// Ring stage modes.  SYN: F -> map.  ANA*: a pixel map -> G, the map being
// map_in (ANA), d on unmasked pixels (ANA_FIRST), w (d - map_in) (ANA_RESID),
// w d (ANA_WD) or c (d - map_in) with the pixel-step coefficient c at the
// control block's current xi (ANA_CRES).
// ITER: F -> s (Cauchy sums, s_map updated) -> r = c (d - s) -> G.
// SYN_WRES: F -> s (not stored) -> r = w (d - s) -> G.
enum RingMode {
    RING_SYN = 0,
    RING_ANA,
    RING_ANA_FIRST,
    RING_ANA_RESID,
    RING_ANA_WD,
    RING_ANA_CRES,
    RING_ITER,
    RING_SYN_WRES
};
struct RingIO {
    double* map_out;        // RING_SYN: synthesised map
    const double* map_in;   // RING_ANA: map to analyse
    const double* d;        // data
    const double* w;        // N^-1
    double* s_map;          // RING_ITER: s_prev in, s out
    double* cpart;          // RING_ITER: Cauchy partials [maps][nq][2]
    double xi, alpha;       // pixel step coefficients when ctrl is NULL
    int first;              // RING_ITER: s_prev taken as 0
    // Per-map control blocks or NULL.  RING_ITER inside the solve loop takes
    // xi, alpha and the m bounds of the current and next level from them, and
    // nothing runs for a map whose solve has stopped; RING_ANA_CRES takes
    // each map's current xi and alpha.
    const DevCtrl* ctrl;
    const int* mhi_tab;     // [maps][kMaxLevels][nq]
    long long pix_map;      // doubles between consecutive maps' pixel arrays
};
// The maps of one ring launch (grid.y).  ell_syn bounds the m of F used by
// the synthesis, ell_ana the m of G written by the analysis (device ints, map
// k at k * ell_stride); mhi_syn / mhi_ana are the per-ring-pair bounds for the
// same band limits (map k at k * mhi_stride; beyond them every lambda_lm is
// skipped, so F is zero and G is never read).
struct RingMaps {
    int nm;
    const int* ell_syn;
    const int* ell_ana;
    int ell_stride;
    const int* mhi_syn;
    const int* mhi_ana;
    int mhi_stride;
};
dmwf_status launch_ring(dmwf_plan* p, RingMode mode, double2* spec, const RingMaps& rm,
                        const RingIO& io, hipStream_t s);
// Ring transform tables and launch classes; called by dmwf_plan_create.
dmwf_status build_ring_tables(dmwf_plan* p);
void free_ring_tables(dmwf_plan* p);

}  // namespace dmwf
