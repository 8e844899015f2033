// C ABI of the dual messenger Wiener filter library: plans, workspace, the
// transform entry points, one iteration, and the host-driven solve loop of
// the paper's Algorithm 2 (cooling of xi, Cauchy stopping rule per level).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace dmwf {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
__global__ void k_set_int(int* p, int v) { *p = v; }

// Level set-up of one iteration call in a single launch: every block finds
// l_iter = max{l : C_l > mu} itself; block 0 stores it and sets the analysis
// band of the ring stage to lmax; each thread then finds the m bound of one
// ring pair (largest m <= l_iter whose suffix-minimum start is <= l_iter).
__global__ void k_level(const double* __restrict__ cl, int lmax, double mu,
                        const int* __restrict__ lsmin, int nq, int* ell_out, int* ell_ana_out,
                        int* __restrict__ mhi) {
    __shared__ int w[4];
    int best = -1;
    for (int l = threadIdx.x; l <= lmax; l += blockDim.x)
        if (cl[l] - mu > 0.0) best = l;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) best = max(best, __shfl_xor(best, o));
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = best;
    __syncthreads();
    int ell = w[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) ell = max(ell, w[i]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *ell_out = ell;
        *ell_ana_out = lmax;
    }
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    mhi[q] = m_bound(lsmin + (size_t)q * (lmax + 1), ell, lmax);
}

// a'_lm = g_lm a_lm (synthesis input), Im a_l0 dropped.  grid (l blocks, m,
// map); map k reads alm + k * alm_map and writes ap + k * ap_map.
__global__ void k_prep_syn(const double2* __restrict__ alm, long long alm_map,
                           const double* __restrict__ g, double2* __restrict__ ap,
                           long long ap_map, int lmax) {
    const int m = blockIdx.y;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > lmax) return;
    const long long i = alm_base(m, lmax) + l;
    alm += blockIdx.z * alm_map;
    ap += blockIdx.z * ap_map;
    double2 v = alm[i];
    if (m == 0) v.y = 0.0;
    ap[i] = make_double2(g[i] * v.x, g[i] * v.y);
}

// Harmonic step of the iteration (residual form):
//   b = Omega g_lm sum_chunks part,  a <- f_l (a + b),  a' = g_lm a,
//   f_l = S_bar_l / (S_bar_l + xi/sigma),  S_bar_l = max(C_l - mu, 0).
// Slots with l > l_iter are set to zero without reading the partial sums.
// grid (l blocks, m, map).  With ctrl (the solve loop) mu and xi / sigma are
// the map's current level's, and nothing runs once its solve has stopped.
struct DiagArgs {
    double2* a;             // state of map 0; map k at a + k * a_map
    long long a_map;
    double2* ap;            // g-scaled copy, map k at ap + k * ap_map
    long long ap_map;
    const double2* part;    // partials: chunk c of map k at part + k * part_map + c * stride
    long long part_map;
    size_t stride;
    int nchunk;
    const double* g;
    const double* cl;       // C_l of map k at cl + k * (lmax + 1)
    double mu, xi_over_sigma, omega;
    const int* ell;         // l_iter of map k at ell[k * ell_stride]
    int ell_stride;
    int lmax;
    const DevCtrl* ctrl;
};

__global__ void k_diag(DiagArgs d) {
    const int k = blockIdx.z;
    double mu = d.mu, xi_over_sigma = d.xi_over_sigma;
    if (d.ctrl) {
        const DevCtrl* c = d.ctrl + k;
        if (c->done) return;
        mu = c->mu;
        xi_over_sigma = c->xi_over_sigma;
    }
    const int m = blockIdx.y;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    const int lmax = d.lmax;
    if (l > lmax) return;
    const int ell = d.ell[k * d.ell_stride];
    const long long i = alm_base(m, lmax) + l;
    double2* a = d.a + k * d.a_map;
    const double2* part = d.part + k * d.part_map;
    const double* cl = d.cl + (long long)k * (lmax + 1);
    double2 out = make_double2(0.0, 0.0);
    if (l <= ell) {
        double sr = 0.0, si = 0.0;
        for (int c = 0; c < d.nchunk; ++c) {
            const double2 v = part[c * d.stride + i];
            sr += v.x;
            si += v.y;
        }
        const double sc = d.omega * d.g[i];
        double sbar = cl[l] - mu;
        sbar = sbar > 0.0 ? sbar : 0.0;
        const double f = sbar / (sbar + xi_over_sigma);
        const double2 ai = a[i];
        out = make_double2(f * (ai.x + sc * sr), f * (ai.y + sc * si));
        if (m == 0) out.y = 0.0;
    }
    a[i] = out;
    d.ap[k * d.ap_map + i] = make_double2(d.g[i] * out.x, d.g[i] * out.y);
}

// out_lm = scale g_lm sum_chunks part (the adjoint), all l.  grid (l blocks,
// m, map): map k sums part + k * part_map into out + k * out_map.
__global__ void k_adj_final(const double2* __restrict__ part, long long part_map, int nchunk,
                            size_t stride, const double* __restrict__ g,
                            double2* __restrict__ out, long long out_map, double scale,
                            int lmax) {
    const int m = blockIdx.y;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > lmax) return;
    part += blockIdx.z * part_map;
    out += blockIdx.z * out_map;
    const long long i = alm_base(m, lmax) + l;
    double sr = 0.0, si = 0.0;
    for (int c = 0; c < nchunk; ++c) {
        const double2 v = part[c * stride + i];
        sr += v.x;
        si += v.y;
    }
    const double sc = scale * g[i];
    out[i] = make_double2(sc * sr, m == 0 ? 0.0 : sc * si);
}

// m bound of ring pair q at the l_iter of every level: mhi_tab[k][q], for
// the levels of map blockIdx.y (its table at mhi_tab + map * kMaxLevels * nq).
__global__ void k_level_tab(const int* __restrict__ lsmin, int nq, int lmax,
                            const DevLevel* __restrict__ levels, const DevCtrl* __restrict__ ctrl,
                            int* __restrict__ mhi_tab) {
    const int map = blockIdx.y;
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i >= (long long)ctrl[map].nlev * nq) return;
    levels += (size_t)map * kMaxLevels;
    mhi_tab += (size_t)map * kMaxLevels * nq;
    const int k = (int)(i / nq), q = (int)(i % nq);
    mhi_tab[i] = m_bound(lsmin + (size_t)q * (lmax + 1), levels[k].ell, lmax);
}

__device__ void ctrl_enter_level(DevCtrl* c, const DevLevel* levels, int k, int* ell_out,
                                 int* ell_ana_out) {
    c->level = k;
    c->it_level = 0;
    c->xi = levels[k].xi;
    c->mu = levels[k].mu;
    c->xi_over_sigma = levels[k].xi_over_sigma;
    *ell_out = levels[k].ell;
    *ell_ana_out = levels[k].ell_next;
}

// Pointers of map k in the solve loop's per-map device state.
struct CtrlMaps {
    DevCtrl* ctrl;          // [maps]
    const DevLevel* levels; // [maps][kMaxLevels]
    int* lev_iters;         // [maps][kMaxLevels]
    int* ell;               // [maps] l_iter
    int* ell_ana;           // [maps] analysis band of the ring stage
};

// One block per map: the control block (uploaded with nlev, max_iter, replay
// and alpha set) enters level 0.
__global__ void k_ctrl_init(CtrlMaps cm) {
    const int k = blockIdx.x;
    DevCtrl* c = cm.ctrl + k;
    const DevLevel* lv = cm.levels + (size_t)k * kMaxLevels;
    int* its = cm.lev_iters + (size_t)k * kMaxLevels;
    for (int i = threadIdx.x; i < c->nlev; i += blockDim.x) its[i] = 0;
    if (threadIdx.x == 0) ctrl_enter_level(c, lv, 0, cm.ell + k, cm.ell_ana + k);
}

// After each iteration of the solve loop (one block per map): the map's
// Cauchy sums over the ring pairs in a fixed order, the ratio
// ||s_i - s_{i-1}|| / ||s_i||, and the schedule's decision: stay on the
// level, move to the next one (a level's tolerance met, or its replayed count
// reached), or stop (the last level met its tolerance, the iteration cap, or
// a NaN ratio).
__global__ void k_control(const double* __restrict__ cpart_all, int n, CtrlMaps cm,
                          double* out2_all) {
    __shared__ double sa[256], sb[256];
    const int map = blockIdx.x;
    DevCtrl* c = cm.ctrl + map;
    if (c->done) return;
    const double* cpart = cpart_all + (size_t)map * 2 * n;
    const DevLevel* levels = cm.levels + (size_t)map * kMaxLevels;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        a += cpart[2 * i];
        b += cpart[2 * i + 1];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sa[threadIdx.x] += sa[threadIdx.x + st];
            sb[threadIdx.x] += sb[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double num = sa[0], den = sb[0];
    double* out2 = out2_all + (size_t)map * 4;
    out2[0] = num;
    out2[1] = den;
    const double ratio = den > 0.0 ? sqrt(num / den) : (num == 0.0 ? 0.0 : INFINITY);
    c->ratio = ratio;
    c->it_level += 1;
    c->total += 1;
    const int k = c->level;
    cm.lev_iters[(size_t)map * kMaxLevels + k] = c->it_level;
    if (isnan(ratio)) {
        c->status = 2;
        c->done = 1;
        return;
    }
    bool advance = c->replay ? c->it_level >= levels[k].replay : ratio < levels[k].eps;
    if (c->reduced) {
        c->it_reduced += 1;
        // Reduced-precision contractions run the coarse levels and the last
        // level down to eps_reduced (or until the ratio stops improving: 64
        // iterations without a 1% gain); the last level then continues in
        // FP64 and only an FP64 iteration can end the solve.  Replayed solves
        // stay reduced throughout.
        if (k + 1 >= c->nlev && !c->replay) {
            if (ratio < 0.99 * c->best) {
                c->best = ratio;
                c->stall = 0;
            } else {
                c->stall += 1;
            }
            if (ratio < c->eps_reduced || c->stall >= 64) c->reduced = 0;
            advance = false;
        }
    }
    // the last level met: converged, even on the capped iteration; else the
    // cap stops the map, also on an iteration that would move to the next
    // level (the host enqueues no iteration beyond the cap)
    if (advance && k + 1 >= c->nlev) {
        c->status = 0;
        c->done = 1;
    } else if (c->total >= c->max_iter) {
        c->status = 1;
        c->done = 1;
    } else if (advance) {
        ctrl_enter_level(c, levels, k + 1, cm.ell + map, cm.ell_ana + map);
    }
}

__global__ void k_zero2(double2* p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

__global__ void k_set_ints(int* p, int n, int v) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

// Sum per-ring-pair pairs (num, den) into out[2] (one block, fixed order).
__global__ void k_sum_pairs(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double sa[256], sb[256];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        a += part[2 * i];
        b += part[2 * i + 1];
    }
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sa[threadIdx.x] += sa[threadIdx.x + s];
            sb[threadIdx.x] += sb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sa[0];
        out[1] = sb[0];
    }
}

// Input screening, grid (kCheckBlocks, map): flags[map] |= 1 non-finite d,
// 2 negative or non-finite N^-1, 4 negative or non-finite C_l.  Per-block
// max of N^-1 into bmax[map][block].
__global__ void k_check(const double* __restrict__ d, const double* __restrict__ w, long long n,
                        const double* __restrict__ cl, int L, int* flags, double* bmax) {
    __shared__ double sm[256];
    const int map = blockIdx.y;
    d += map * n;
    w += map * n;
    cl += (long long)map * L;
    int f = 0;
    double mx = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double dv = d[i], wv = w[i];
        if (!isfinite(dv)) f |= 1;
        if (!isfinite(wv) || wv < 0.0) f |= 2;
        else mx = fmax(mx, wv);
    }
    if (blockIdx.x == 0) {
        for (int l = threadIdx.x; l < L; l += blockDim.x)
            if (!isfinite(cl[l]) || cl[l] < 0.0) f |= 4;
    }
    if (f) atomicOr(flags + map, f);
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) bmax[(size_t)map * gridDim.x + blockIdx.x] = sm[0];
}

// One block per map: out[map * out_map] = max over the map's block maxima.
__global__ void k_max_final(const double* __restrict__ bmax, int n, double* out, int out_map) {
    __shared__ double sm[256];
    bmax += (size_t)blockIdx.x * n;
    double mx = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) mx = fmax(mx, bmax[i]);
    sm[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)blockIdx.x * out_map] = sm[0];
}

// Residual of the whitened Wiener filter equation (paper Appendix C form):
//   res = C^-1/2 a - C^1/2 b1,  y = C^1/2 b2   (b1 = Y^H W (d - Y a), b2 = Y^H W d)
// over C_l > 0; per-block sums of |res|^2 and |y|^2 with m > 0 counted twice.
__global__ void k_resid_norms(const double2* __restrict__ a, const double2* __restrict__ b1,
                              const double2* __restrict__ b2, const double* __restrict__ cl,
                              int lmax, double* __restrict__ bsum) {
    __shared__ double sa[256], sb[256];
    const int m = blockIdx.y;
    const int l = m + blockIdx.x * blockDim.x + threadIdx.x;
    double r2 = 0.0, y2 = 0.0;
    if (l <= lmax && cl[l] > 0.0) {
        const long long i = alm_base(m, lmax) + l;
        const double c = cl[l], sq = sqrt(c), isq = 1.0 / sq;
        const double2 av = a[i], g1 = b1[i], g2 = b2[i];
        const double wt = m == 0 ? 1.0 : 2.0;
        const double rx = isq * av.x - sq * g1.x;
        const double ry = m == 0 ? 0.0 : isq * av.y - sq * g1.y;
        const double yx = sq * g2.x, yy = m == 0 ? 0.0 : sq * g2.y;
        r2 = wt * (rx * rx + ry * ry);
        y2 = wt * (yx * yx + yy * yy);
    }
    sa[threadIdx.x] = r2;
    sb[threadIdx.x] = y2;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sa[threadIdx.x] += sa[threadIdx.x + s];
            sb[threadIdx.x] += sb[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        bsum[2 * b] = sa[0];
        bsum[2 * b + 1] = sb[0];
    }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
// The Legendre stages in the plan's precision.  Reduced-precision plans run
// the matrix-core kernels; inside the solve loop (lm.ctrl set) each map runs
// in the precision its control block names, so both kernels are launched and
// each takes its own maps.
dmwf_status leg_syn(dmwf_plan* p, const double2* ap, double2* spec, LegMaps lm, hipStream_t s) {
    if (p->prec == DMWF_FP64) return launch_leg_syn(p, ap, spec, lm, p->syn_mb, s);
    if (!lm.ctrl) return launch_leg_syn_mx(p, ap, spec, lm, s);
    lm.sel = 1;
    const dmwf_status st = launch_leg_syn(p, ap, spec, lm, p->syn_mb, s);
    if (st != DMWF_OK) return st;
    lm.sel = 2;
    return launch_leg_syn_mx(p, ap, spec, lm, s);
}

dmwf_status leg_ana(dmwf_plan* p, const double2* spec, double2* part, LegMaps lm, hipStream_t s) {
    if (p->prec == DMWF_FP64) return launch_leg_ana(p, spec, part, lm, p->ana_mb, s);
    if (!lm.ctrl) return launch_leg_ana_mx(p, spec, part, lm, s);
    lm.sel = 1;
    const dmwf_status st = launch_leg_ana(p, spec, part, lm, p->ana_mb, s);
    if (st != DMWF_OK) return st;
    lm.sel = 2;
    return launch_leg_ana_mx(p, spec, part, lm, s);
}

struct Ws {
    char* base;
    int nmaps;
    WsLayout off;
    double2* spec(int k) const {
        return reinterpret_cast<double2*>(base + off.spec) + k * off.spec_map;
    }
    double2* part(int k) const {
        return reinterpret_cast<double2*>(base + off.part) + k * off.part_map;
    }
    double2* ap(int k) const { return reinterpret_cast<double2*>(base + off.ap) + k * off.alm_map; }
    double2* aux(int k) const {
        return reinterpret_cast<double2*>(base + off.aux) + k * off.alm_map;
    }
    double* cpart(int k, int nq) const {
        return reinterpret_cast<double*>(base + off.cpart) + (size_t)k * 2 * nq;
    }
    int* mhi(int k, int nq) const { return reinterpret_cast<int*>(base + off.mhi) + (size_t)k * nq; }
    int* ell(int k) const { return reinterpret_cast<int*>(base + off.ells) + k; }
    int* ell_ana(int k) const { return reinterpret_cast<int*>(base + off.ells) + nmaps + k; }
    int* flags(int k) const { return reinterpret_cast<int*>(base + off.ells) + 2 * nmaps + k; }
    double* mdbl(int k) const { return reinterpret_cast<double*>(base + off.mdbl) + 4 * k; }
    double* bmax() const { return reinterpret_cast<double*>(base + off.bmax); }
    int* ell_full() const { return reinterpret_cast<int*>(base + off.scal); }
    double* out2() const { return reinterpret_cast<double*>(base + off.scal + 16); }
    double* scal_d() const { return reinterpret_cast<double*>(base + off.scal + 64); }
    DevCtrl* ctrl(int k) const { return reinterpret_cast<DevCtrl*>(base + off.ctrl) + k; }
    DevLevel* levels(int k) const {
        return reinterpret_cast<DevLevel*>(base + off.levels) + (size_t)k * kMaxLevels;
    }
    int* lev_iters(int k) const {
        return reinterpret_cast<int*>(base + off.lev_iters) + (size_t)k * kMaxLevels;
    }
    int* mhi_tab() const { return reinterpret_cast<int*>(base + off.mhi_tab); }
    CtrlMaps cmaps(int k0 = 0) const {
        return {ctrl(k0), levels(k0), lev_iters(k0), ell(k0), ell_ana(k0)};
    }
};

dmwf_status check_ws(const dmwf_plan* p, void* ws, size_t bytes, Ws* out) {
    if (ws == nullptr || bytes < p->ws.total || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) {
        set_error("workspace is missing, too small or not 256-byte aligned");
        return DMWF_ERR_WORKSPACE;
    }
    out->base = static_cast<char*>(ws);
    out->nmaps = p->nmaps;
    out->off = p->ws;
    return DMWF_OK;
}

dim3 alm_grid(int lmax, int bs, int nm = 1) {
    return dim3((lmax + 1 + bs - 1) / bs, lmax + 1, nm);
}

size_t scal_bytes(const dmwf_plan* p) {
    // ints + 2 doubles + residual block sums
    const size_t nres = 2 * (size_t)((p->lmax + 1 + 255) / 256) * (p->lmax + 1);
    return 64 + sizeof(double) * (8 + nres);
}

// Maps of a launch with one band limit for all (the shared int set to lmax).
RingMaps ring_full(const dmwf_plan* p, const Ws& W, int nm) {
    return RingMaps{nm, W.ell_full(), W.ell_full(), 0, p->d_mhi_full, p->d_mhi_full, 0};
}

// Fixed device scratch of dmwf_alm2map_static: a file-scope array that every
// GPU the library runs on holds until the process ends.  Host code never
// passes its name to a kernel (in host code the name is a host-side stand-in);
// it uses the device address that hipGetSymbolAddress returns for the device,
// looked up once per device when a plan is created there.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
__device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Called by dmwf_plan_create with the plan's device current.
dmwf_status static_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) {
        set_error("device index beyond the library's table of scratch addresses");
        return DMWF_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return DMWF_OK;
    void* ptr = nullptr;
    DMWF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
        set_error("hipGetSymbolAddress returned NULL for the static scratch");
        return DMWF_ERR_HIP;
    }
    g_scratch_ptr[device] = ptr;
    return DMWF_OK;
}

void* static_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

// Bytes of the static scratch dmwf_alm2map_static needs for a plan: the band
// limit int, the g-scaled a_lm and the F rows of every map, in the
// workspace's per-map strides.
size_t static_alm2map_bytes(const dmwf_plan* p) {
    const size_t nm = (size_t)p->nmaps;
    return 256 + align256(nm * p->ws.alm_map * sizeof(double2)) +
           nm * p->ws.spec_map * sizeof(double2);
}

}  // namespace
}  // namespace dmwf

using namespace dmwf;

extern "C" {

const char* dmwf_status_string(dmwf_status s) {
    switch (s) {
        case DMWF_OK: return "ok";
        case DMWF_ERR_INVALID_ARG: return "invalid argument";
        case DMWF_ERR_WORKSPACE: return "workspace too small or misaligned";
        case DMWF_ERR_HIP: return "HIP runtime error";
        case DMWF_ERR_NOT_CONVERGED: return "not converged within max_iter";
        case DMWF_ERR_NONFINITE: return "non-finite or negative input, or non-finite Cauchy ratio";
        case DMWF_ERR_UNSUPPORTED: return "unsupported";
        case DMWF_ERR_OOM: return "device allocation failed";
    }
    return "unknown status";
}

const char* dmwf_last_error(void) { return g_last_error.c_str(); }

void dmwf_plan_destroy(dmwf_plan* p) {
    if (!p) return;
    for (auto& e : p->events) {
        (void)hipEventDestroy(e.start);
        (void)hipEventDestroy(e.stop);
    }
    for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
    free_ring_tables(p);
    if (p->h_ctrl) (void)hipHostFree(p->h_ctrl);
    for (hipEvent_t e : p->batch_ev)
        if (e) (void)hipEventDestroy(e);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    void* bufs[] = {p->d_x, p->d_sint, p->d_nph, p->d_phi0pi, p->d_start_n, p->d_start_s,
                    p->d_A, p->d_g,    p->d_ls,  p->d_s0,     p->d_s1, p->d_lsmin,
                    p->d_mhi_full};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

dmwf_status dmwf_plan_create(const dmwf_plan_desc* desc, dmwf_plan** out) {
    if (!out) {
        set_error("out is NULL");
        return DMWF_ERR_INVALID_ARG;
    }
    *out = nullptr;
    if (!desc) {
        set_error("desc is NULL");
        return DMWF_ERR_INVALID_ARG;
    }
    const int N = desc->nside;
    if (N < 1 || N > 8192 || (N & (N - 1)) != 0) {
        set_error("nside must be a power of two in [1, 8192]");
        return DMWF_ERR_INVALID_ARG;
    }
    if (desc->lmax < 0 || desc->lmax > 3 * N - 1) {
        set_error("lmax must be in [0, 3 nside - 1]");
        return DMWF_ERR_INVALID_ARG;
    }
    if (desc->nmaps < 1 || desc->nmaps > 65535) {
        set_error("nmaps must be in [1, 65535] (the maps of a launch are a grid dimension)");
        return DMWF_ERR_INVALID_ARG;
    }
    if (desc->precision != DMWF_FP64 && desc->precision != DMWF_FP32_GEMM &&
        desc->precision != DMWF_BF16X3_GEMM) {
        set_error("precision must be DMWF_FP64, DMWF_FP32_GEMM or DMWF_BF16X3_GEMM");
        return DMWF_ERR_INVALID_ARG;
    }
    if (N > 1024) {
        set_error("nside > 1024 needs ring FFTs longer than one workgroup's LDS; not implemented");
        return DMWF_ERR_UNSUPPORTED;
    }
    dmwf_plan* p = new dmwf_plan();
    p->nside = N;
    p->lmax = desc->lmax;
    p->nmaps = desc->nmaps;
    p->prec = desc->precision;
    p->nq = 2 * N;
    p->nrings = 4 * N - 1;
    p->npix = 12LL * N * N;
    p->nalm = (long long)(p->lmax + 1) * (p->lmax + 2) / 2;
    p->omega = 4.0 * kPi / (double)p->npix;
    // analysis tile: 8 ring pairs per lane, 4 where a wave of 8 would leave
    // lanes idle (at most 256 ring pairs); the partial-sum buffer holds the
    // chunks of the smallest tile the autotuner may pick
    p->ana_k = p->nq <= 256 ? 4 : 8;
    p->ana_k_min = p->nq <= 512 ? 4 : 8;
    p->nchunk_ana = (p->nq + 64 * p->ana_k - 1) / (64 * p->ana_k);
    p->lp = (p->lmax + 1 + 3) & ~3;
    if (hipGetDevice(&p->device) != hipSuccess) {
        set_error("hipGetDevice failed");
        delete p;
        return DMWF_ERR_HIP;
    }

    // ---- ring pair geometry (HEALPix RING scheme) ----
    const int nq = p->nq;
    std::vector<double> x(nq), st(nq), phi0pi(nq);
    std::vector<int> nph(nq);
    std::vector<long long> sn(nq), ss(nq);
    const long double LN = N;
    for (int q = 0; q < nq; ++q) {
        const long long r = q + 1;  // north ring, 1-based; r = 2N is the equator
        long double z, s;
        if (r < N) {
            const long double u = (long double)r * r / (3.0L * LN * LN);  // 1 - z
            z = 1.0L - u;
            s = sqrtl(u * (2.0L - u));
            nph[q] = (int)(4 * r);
            phi0pi[q] = (double)(1.0L / (4.0L * r));
            sn[q] = 2 * r * (r - 1);
            ss[q] = p->npix - 2 * r * (r + 1);
        } else {
            z = 4.0L / 3.0L - 2.0L * r / (3.0L * LN);
            s = sqrtl((1.0L - z) * (1.0L + z));
            nph[q] = 4 * N;
            const int shift = (int)((r - N + 1) % 2);
            phi0pi[q] = shift ? (double)(1.0L / (4.0L * LN)) : 0.0;
            sn[q] = 2LL * N * (N - 1) + 4LL * N * (r - N);
            const long long rs = 4LL * N - r;
            ss[q] = (r == 2LL * N) ? -1 : 2LL * N * (N - 1) + 4LL * N * (rs - N);
        }
        x[q] = (double)z;
        st[q] = (double)s;
    }

    // ---- recurrence tables: lambda_lm = g_lm mu_lm, mu_l = A_l x mu_{l-1} - mu_{l-2} ----
    const int L = p->lmax;
    const size_t ntab = (size_t)p->nalm + kTablePad;
    std::vector<double> A(ntab, 0.0), G(ntab, 0.0);
    for (int m = 0; m <= L; ++m) {
        const long long b = alm_base(m, L);
        long double gm2 = 1.0L, gm1 = 1.0L, am1 = 0.0L;  // g_{l-2}, g_{l-1}, a_{l-1}
        G[b + m] = 1.0;
        A[b + m] = 0.0;
        for (int l = m + 1; l <= L; ++l) {
            const long double dl = l, dm = m;
            const long double al = sqrtl((4.0L * dl * dl - 1.0L) / (dl * dl - dm * dm));
            long double gl;
            if (l == m + 1) {
                gl = 1.0L;
            } else {
                gl = gm2 * al / am1;
            }
            A[b + l] = (double)(al * gm1 / gl);
            G[b + l] = (double)gl;
            gm2 = gm1;
            gm1 = gl;
            am1 = al;
        }
    }

    auto fail = [&](dmwf_status st_) {
        dmwf_plan_destroy(p);
        return st_;
    };
    auto up = [&](void** dst, const void* src, size_t bytes) -> bool {
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up((void**)&p->d_x, x.data(), nq * sizeof(double)) ||
        !up((void**)&p->d_sint, st.data(), nq * sizeof(double)) ||
        !up((void**)&p->d_nph, nph.data(), nq * sizeof(int)) ||
        !up((void**)&p->d_phi0pi, phi0pi.data(), nq * sizeof(double)) ||
        !up((void**)&p->d_start_n, sn.data(), nq * sizeof(long long)) ||
        !up((void**)&p->d_start_s, ss.data(), nq * sizeof(long long)) ||
        !up((void**)&p->d_A, A.data(), ntab * sizeof(double)) ||
        !up((void**)&p->d_g, G.data(), ntab * sizeof(double))) {
        set_error("allocation or upload of plan tables failed");
        return fail(DMWF_ERR_OOM);
    }
    const size_t nseed = (size_t)(L + 1) * nq;
    if (hipMalloc(&p->d_ls, nseed * sizeof(int)) != hipSuccess ||
        hipMalloc(&p->d_lsmin, nseed * sizeof(int)) != hipSuccess ||
        hipMalloc(&p->d_mhi_full, nq * sizeof(int)) != hipSuccess ||
        hipMalloc(&p->d_s0, nseed * sizeof(double)) != hipSuccess ||
        hipMalloc(&p->d_s1, nseed * sizeof(double)) != hipSuccess) {
        set_error("allocation of recurrence start tables failed");
        return fail(DMWF_ERR_OOM);
    }
    dmwf_status s = launch_seeds(p, nullptr);
    if (s != DMWF_OK) return fail(s);
    s = build_ring_tables(p);
    if (s != DMWF_OK) return fail(s);

    // ---- workspace layout: per-map slices of every per-map region ----
    WsLayout& w = p->ws;
    const size_t nm = (size_t)p->nmaps;
    w.spec_map = (long long)p->lp * nq * 2;
    w.part_map = (long long)((nq + 64 * p->ana_k_min - 1) / (64 * p->ana_k_min)) * ntab;
    w.alm_map = (long long)ntab;
    size_t off = 0;
    w.spec = off;
    off = align256(off + nm * w.spec_map * sizeof(double2));
    w.part = off;
    off = align256(off + nm * w.part_map * sizeof(double2));
    w.ap = off;
    off = align256(off + nm * w.alm_map * sizeof(double2));
    w.aux = off;
    off = align256(off + nm * w.alm_map * sizeof(double2));
    w.cpart = off;
    off = align256(off + nm * nq * 2 * sizeof(double));
    w.mhi = off;
    off = align256(off + nm * nq * sizeof(int));
    w.ells = off;
    off = align256(off + 3 * nm * sizeof(int));
    w.mdbl = off;
    off = align256(off + 4 * nm * sizeof(double));
    w.bmax = off;
    off = align256(off + nm * kCheckBlocks * sizeof(double));
    w.scal = off;
    off = align256(off + scal_bytes(p));
    w.ctrl = off;
    off = align256(off + nm * sizeof(DevCtrl));
    w.levels = off;
    off = align256(off + nm * kMaxLevels * sizeof(DevLevel));
    w.lev_iters = off;
    off = align256(off + nm * kMaxLevels * sizeof(int));
    w.mhi_tab = off;
    off = align256(off + nm * kMaxLevels * nq * sizeof(int));
    w.total = off;
    if (hipHostMalloc((void**)&p->h_ctrl, 2 * nm * sizeof(DevCtrl), hipHostMallocDefault) !=
            hipSuccess ||
        hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->batch_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->batch_ev[1], hipEventDisableTiming) != hipSuccess) {
        set_error("allocation of the solve-loop host buffer failed");
        return fail(DMWF_ERR_OOM);
    }
    // maps per wave of the Legendre kernels until dmwf_autotune measures
    // better: the synthesis shares its recurrence across up to four maps, the
    // analysis (whose lane reduction and registers grow with the maps) across two
    p->syn_mb = p->nmaps >= 4 ? 4 : (p->nmaps >= 2 ? 2 : 1);
    p->ana_mb = p->nmaps >= 2 ? 2 : 1;
    // device address of the static scratch of dmwf_alm2map_static on this device
    s = static_scratch_setup(p->device);
    if (s != DMWF_OK) return fail(s);
    *out = p;
    return DMWF_OK;
}

dmwf_status dmwf_workspace_bytes(const dmwf_plan* p, size_t* bytes) {
    if (!p || !bytes) {
        set_error("NULL argument");
        return DMWF_ERR_INVALID_ARG;
    }
    *bytes = p->ws.total;
    return DMWF_OK;
}

dmwf_status dmwf_profile_enable(dmwf_plan* p, int enable) {
    if (!p) return DMWF_ERR_INVALID_ARG;
    if (enable < 0 || enable > 2) return DMWF_ERR_INVALID_ARG;
    p->prof = enable;
    return DMWF_OK;
}

dmwf_status dmwf_profile_read(dmwf_plan* p, int* n_classes, const char** names, long* counts,
                              double* total_ms) {
    static const char* kNames[PROF_COUNT] = {"seeds", "legendre_analysis", "legendre_synthesis",
                                             "harmonic_diag", "ring_iter", "ring_synthesis",
                                             "ring_analysis", "reduce", "misc"};
    if (!p || !n_classes) return DMWF_ERR_INVALID_ARG;
    *n_classes = PROF_COUNT;
    for (int i = 0; i < PROF_COUNT; ++i) {
        if (names) names[i] = kNames[i];
        if (counts) counts[i] = 0;
        if (total_ms) total_ms[i] = 0.0;
    }
    for (auto& e : p->events) {
        DMWF_HIP(hipEventSynchronize(e.stop));
        float ms = 0.0f;
        DMWF_HIP(hipEventElapsedTime(&ms, e.start, e.stop));
        if (counts) counts[e.cls] += 1;
        if (total_ms) total_ms[e.cls] += ms;
        p->event_pool.push_back(e.start);
        p->event_pool.push_back(e.stop);
    }
    p->events.clear();
    return DMWF_OK;
}

// ---------------------------------------------------------------------------
// transforms
// ---------------------------------------------------------------------------
dmwf_status dmwf_alm2map(dmwf_plan* p, const double* alm, double* map, void* ws, size_t ws_bytes,
                         void* stream) {
    if (!p || !alm || !map) {
        set_error("NULL argument");
        return DMWF_ERR_INVALID_ARG;
    }
    Ws W;
    dmwf_status st = check_ws(p, ws, ws_bytes, &W);
    if (st != DMWF_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nm = p->nmaps;
    {
        ProfScope ps(p, s, PROF_MISC);
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, W.ell_full(), p->lmax);
        hipLaunchKernelGGL(k_prep_syn, alm_grid(p->lmax, 256, nm), dim3(256), 0, s,
                           reinterpret_cast<const double2*>(alm), p->nalm, p->d_g, W.ap(0),
                           p->ws.alm_map, p->lmax);
    }
    DMWF_HIP(hipGetLastError());
    st = leg_syn(p, W.ap(0), W.spec(0), LegMaps{nm, W.ell_full(), 0, nullptr}, s);
    if (st != DMWF_OK) return st;
    RingIO io{};
    io.map_out = map;
    io.pix_map = p->npix;
    return launch_ring(p, RING_SYN, W.spec(0), ring_full(p, W, nm), io, s);
}

dmwf_status dmwf_alm2map_static(dmwf_plan* p, const double* alm, double* map, void* stream) {
    if (!p || !alm || !map) {
        set_error("NULL argument");
        return DMWF_ERR_INVALID_ARG;
    }
    const size_t need = static_alm2map_bytes(p);
    if (need > kStaticScratchBytes) {
        set_error("dmwf_alm2map_static: the plan needs " + std::to_string(need) +
                  " bytes of scratch, the static scratch holds " +
                  std::to_string(kStaticScratchBytes) + "; use dmwf_alm2map with a workspace");
        return DMWF_ERR_WORKSPACE;
    }
    char* base = static_cast<char*>(static_scratch(p->device));
    if (!base) {
        set_error("static scratch address unknown for the plan's device");
        return DMWF_ERR_HIP;
    }
    int* ell = reinterpret_cast<int*>(base);
    double2* ap = reinterpret_cast<double2*>(base + 256);
    double2* spec = reinterpret_cast<double2*>(
        base + 256 + align256((size_t)p->nmaps * p->ws.alm_map * sizeof(double2)));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nm = p->nmaps;
    // no timing events here: recording them may create events
    const int prof = p->prof;
    p->prof = 0;
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, ell, p->lmax);
    hipLaunchKernelGGL(k_prep_syn, alm_grid(p->lmax, 256, nm), dim3(256), 0, s,
                       reinterpret_cast<const double2*>(alm), p->nalm, p->d_g, ap, p->ws.alm_map,
                       p->lmax);
    dmwf_status st = DMWF_OK;
    if (hipGetLastError() != hipSuccess) {
        set_error("launch failed in dmwf_alm2map_static");
        st = DMWF_ERR_HIP;
    }
    if (st == DMWF_OK) st = leg_syn(p, ap, spec, LegMaps{nm, ell, 0, nullptr}, s);
    if (st == DMWF_OK) {
        RingIO io{};
        io.map_out = map;
        io.pix_map = p->npix;
        st = launch_ring(p, RING_SYN, spec,
                         RingMaps{nm, ell, ell, 0, p->d_mhi_full, p->d_mhi_full, 0}, io, s);
    }
    p->prof = prof;
    return st;
}

dmwf_status dmwf_adjoint(dmwf_plan* p, const double* map, double* alm, int scale_by_pixel_area,
                         void* ws, size_t ws_bytes, void* stream) {
    if (!p || !alm || !map) {
        set_error("NULL argument");
        return DMWF_ERR_INVALID_ARG;
    }
    Ws W;
    dmwf_status st = check_ws(p, ws, ws_bytes, &W);
    if (st != DMWF_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nm = p->nmaps;
    {
        ProfScope ps(p, s, PROF_MISC);
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, W.ell_full(), p->lmax);
    }
    RingIO io{};
    io.map_in = map;
    io.pix_map = p->npix;
    st = launch_ring(p, RING_ANA, W.spec(0), ring_full(p, W, nm), io, s);
    if (st != DMWF_OK) return st;
    st = leg_ana(p, W.spec(0), W.part(0), LegMaps{nm, W.ell_full(), 0, nullptr}, s);
    if (st != DMWF_OK) return st;
    {
        ProfScope ps(p, s, PROF_DIAG);
        hipLaunchKernelGGL(k_adj_final, alm_grid(p->lmax, 256, nm), dim3(256), 0, s, W.part(0),
                           p->ws.part_map, p->nchunk_ana, (size_t)p->nalm + kTablePad, p->d_g,
                           reinterpret_cast<double2*>(alm), p->nalm,
                           scale_by_pixel_area ? p->omega : 1.0, p->lmax);
    }
    DMWF_HIP(hipGetLastError());
    return DMWF_OK;
}

dmwf_status dmwf_set_tiles(dmwf_plan* p, int syn_k, int syn_mb, int ana_k, int ana_mb) {
    if (!p || (syn_k != 1 && syn_k != 2) ||
        (syn_mb != 1 && syn_mb != 2 && syn_mb != 4 && syn_mb != 8) ||
        (ana_k != 4 && ana_k != 8) || ana_k < p->ana_k_min || (ana_mb != 1 && ana_mb != 2)) {
        set_error("tiles: synthesis ring pairs per lane 1 or 2, maps per wave 1, 2, 4 or 8; "
                  "analysis ring pairs per lane 4 (nside <= 256) or 8, maps per wave 1 or 2");
        return DMWF_ERR_INVALID_ARG;
    }
    p->syn_k = syn_k;
    p->syn_mb = syn_mb;
    p->ana_k = ana_k;
    p->ana_mb = ana_mb;
    p->nchunk_ana = (p->nq + 64 * ana_k - 1) / (64 * ana_k);
    return DMWF_OK;
}

dmwf_status dmwf_set_pipeline(dmwf_plan* p, int groups) {
    if (!p || groups < 0 || groups > 8) {
        set_error("pipeline groups: 0 to 8");
        return DMWF_ERR_INVALID_ARG;
    }
    if (groups >= 2) {
        // Not built: the pipelined iteration was removed after its first
        // solve ended the process with a host segmentation fault whose cause
        // was not found.
        set_error("the pipelined iteration is switched off (not built)");
        return DMWF_ERR_UNSUPPORTED;
    }
    return DMWF_OK;
}

int dmwf_pipeline_groups(const dmwf_plan* p) { return p ? 0 : -1; }

// Time every Legendre tile on the plan's own shape (all maps, full band; the
// instruction stream does not depend on the values) and keep the fastest.
dmwf_status dmwf_autotune(dmwf_plan* p, void* ws, size_t ws_bytes, void* stream, int* choice,
                          float* ms_out) {
    if (!p) {
        set_error("NULL argument");
        return DMWF_ERR_INVALID_ARG;
    }
    Ws W;
    dmwf_status st = check_ws(p, ws, ws_bytes, &W);
    if (st != DMWF_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nm = p->nmaps;
    const int prof = p->prof;
    p->prof = 0;
    hipLaunchKernelGGL(k_zero2, dim3(256), dim3(256), 0, s, W.ap(0), (long long)nm * p->ws.alm_map);
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, W.ell_full(), p->lmax);
    DMWF_HIP(hipGetLastError());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    DMWF_HIP(hipEventCreate(&e0));
    DMWF_HIP(hipEventCreate(&e1));
    const LegMaps lm{nm, W.ell_full(), 0, nullptr};
    float best = 1e30f;
    int bk = p->syn_k, bmb = p->syn_mb, idx = 0;
    if (ms_out)
        for (int i = 8; i < 12; ++i) ms_out[i] = -1.0f;
    dmwf_status res = DMWF_OK;
    for (int k = 1; k <= 2 && res == DMWF_OK; ++k) {
        for (int mb = 1; mb <= 8 && res == DMWF_OK; mb *= 2, ++idx) {
            if (mb > nm && mb > 1) {
                if (ms_out) ms_out[idx] = -1.0f;
                continue;
            }
            p->syn_k = k;
            const int reps = 3;
            res = launch_leg_syn(p, W.ap(0), W.spec(0), lm, mb, s);  // warm-up
            if (res != DMWF_OK) break;
            if (hipEventRecord(e0, s) != hipSuccess) res = DMWF_ERR_HIP;
            for (int r = 0; r < reps && res == DMWF_OK; ++r)
                res = launch_leg_syn(p, W.ap(0), W.spec(0), lm, mb, s);
            float ms = 0.0f;
            if (res == DMWF_OK && (hipEventRecord(e1, s) != hipSuccess ||
                                   hipEventSynchronize(e1) != hipSuccess ||
                                   hipEventElapsedTime(&ms, e0, e1) != hipSuccess)) {
                set_error("event timing failed during autotuning");
                res = DMWF_ERR_HIP;
            }
            ms /= reps;
            if (ms_out) ms_out[idx] = ms;
            if (res == DMWF_OK && ms < best) {
                best = ms;
                bk = k;
                bmb = mb;
            }
        }
    }
    p->syn_k = bk;
    p->syn_mb = bmb;
    // analysis: ring pairs per lane 8, and 4 where the buffers allow it;
    // one or two maps per wave
    float abest = 1e30f;
    int ak = p->ana_k, amb = p->ana_mb;
    for (int t = 0; t < 4 && res == DMWF_OK; ++t) {
        const int k = t < 2 ? 4 : 8, mb = 1 + (t & 1);
        if (k < p->ana_k_min || mb > nm) continue;
        p->ana_k = k;
        p->nchunk_ana = (p->nq + 64 * k - 1) / (64 * k);
        const int reps = 3;
        res = launch_leg_ana(p, W.spec(0), W.part(0), lm, mb, s);
        if (res != DMWF_OK) break;
        if (hipEventRecord(e0, s) != hipSuccess) res = DMWF_ERR_HIP;
        for (int r = 0; r < reps && res == DMWF_OK; ++r)
            res = launch_leg_ana(p, W.spec(0), W.part(0), lm, mb, s);
        float ms = 0.0f;
        if (res == DMWF_OK && (hipEventRecord(e1, s) != hipSuccess ||
                               hipEventSynchronize(e1) != hipSuccess ||
                               hipEventElapsedTime(&ms, e0, e1) != hipSuccess)) {
            set_error("event timing failed during autotuning");
            res = DMWF_ERR_HIP;
        }
        ms /= reps;
        if (ms_out) ms_out[8 + t] = ms;
        if (res == DMWF_OK && ms < abest) {
            abest = ms;
            ak = k;
            amb = mb;
        }
    }
    p->ana_k = ak;
    p->ana_mb = amb;
    p->nchunk_ana = (p->nq + 64 * ak - 1) / (64 * ak);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->prof = prof;
    if (choice) {
        choice[0] = bk;
        choice[1] = bmb;
        choice[2] = ak;
        choice[3] = amb;
    }
    return res;
}

}  // extern "C"

namespace dmwf {
namespace {

// The iteration body shared by dmwf_dm_iterate (map 0, host parameters) and
// the solve loop (a group of nm maps from map k0, parameters from the per-map
// control blocks): harmonic step from the residual spectrum in the
// workspace, synthesis, pixel step.  cl, d, w, a and s_map point at map k0's
// slices.  The solve loop ends the iteration with each map's level decision;
// dmwf_dm_iterate sums the Cauchy partials into cauchy_out.
// The iteration's first launch, the Legendre analysis of the residual spectrum.
dmwf_status iterate_ana(dmwf_plan* p, const Ws& W, int k0, int nm, DevCtrl* ctrl, hipStream_t s) {
    return leg_ana(p, W.spec(k0), W.part(k0), LegMaps{nm, W.ell(k0), 1, ctrl}, s);
}

// The rest of the iteration after the analysis.
dmwf_status iterate_rest(dmwf_plan* p, const Ws& W, int k0, int nm, double xi, double alpha,
                         double mu, const double* cl, const double* d, const double* w,
                         double2* a, double* s_map, int first_pix, const int* mhi_ana,
                         double* cauchy_out, DevCtrl* ctrl, hipStream_t s) {
    const LegMaps lm{nm, W.ell(k0), 1, ctrl};
    dmwf_status st;
    {
        ProfScope ps(p, s, PROF_DIAG);
        DiagArgs da{a,       p->nalm, W.ap(k0), p->ws.alm_map, W.part(k0), p->ws.part_map,
                    (size_t)p->nalm + kTablePad, p->nchunk_ana, p->d_g, cl, mu, xi * p->omega,
                    p->omega, W.ell(k0), 1, p->lmax, ctrl};
        hipLaunchKernelGGL(k_diag, alm_grid(p->lmax, 256, nm), dim3(256), 0, s, da);
    }
    DMWF_HIP(hipGetLastError());
    RingIO io{};
    io.d = d;
    io.w = w;
    io.s_map = s_map;
    io.cpart = W.cpart(k0, p->nq);
    io.xi = xi;
    io.alpha = alpha;
    io.first = first_pix;
    io.ctrl = ctrl;
    io.mhi_tab = W.mhi_tab() + (size_t)k0 * kMaxLevels * p->nq;
    io.pix_map = p->npix;
    const RingMaps rm{nm, W.ell(k0), W.ell_ana(k0), 1, W.mhi(k0, p->nq), mhi_ana, 0};
    st = leg_syn(p, W.ap(k0), W.spec(k0), lm, s);
    if (st != DMWF_OK) return st;
    st = launch_ring(p, RING_ITER, W.spec(k0), rm, io, s);
    if (st != DMWF_OK) return st;
    {
        ProfScope ps(p, s, PROF_REDUCE);
        if (ctrl)
            hipLaunchKernelGGL(k_control, dim3(nm), dim3(256), 0, s, W.cpart(k0, p->nq), p->nq,
                               W.cmaps(k0), W.mdbl(k0));
        else
            hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(256), 0, s, W.cpart(k0, p->nq), p->nq,
                               cauchy_out);
    }
    DMWF_HIP(hipGetLastError());
    return DMWF_OK;
}

dmwf_status iterate_body(dmwf_plan* p, const Ws& W, int k0, int nm, double xi, double alpha,
                         double mu, const double* cl, const double* d, const double* w,
                         double2* a, double* s_map, int first_pix, const int* mhi_ana,
                         double* cauchy_out, DevCtrl* ctrl, hipStream_t s) {
    dmwf_status st = iterate_ana(p, W, k0, nm, ctrl, s);
    if (st != DMWF_OK) return st;
    return iterate_rest(p, W, k0, nm, xi, alpha, mu, cl, d, w, a, s_map, first_pix, mhi_ana,
                        cauchy_out, ctrl, s);
}

// ||A x - y|| / ||y|| of one map (its C_l, d, N^-1, a); the workspace slices
// of map 0 serve as scratch.
dmwf_status residual_map(dmwf_plan* p, const Ws& W, const double* cl, const double* d,
                         const double* w, const double2* a, double* host_out, hipStream_t s) {
    // b1 = Y^H W (d - Y a) into ap (after its use as synthesis input), b2 = Y^H W d into aux
    {
        ProfScope ps(p, s, PROF_MISC);
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, W.ell_full(), p->lmax);
        hipLaunchKernelGGL(k_prep_syn, alm_grid(p->lmax, 256), dim3(256), 0, s, a, 0LL, p->d_g,
                           W.ap(0), 0LL, p->lmax);
    }
    DMWF_HIP(hipGetLastError());
    const LegMaps lm{1, W.ell_full(), 0, nullptr};
    dmwf_status st = launch_leg_syn(p, W.ap(0), W.spec(0), lm, 1, s);
    if (st != DMWF_OK) return st;
    RingIO io{};
    io.d = d;
    io.w = w;
    st = launch_ring(p, RING_SYN_WRES, W.spec(0), ring_full(p, W, 1), io, s);
    if (st != DMWF_OK) return st;
    st = launch_leg_ana(p, W.spec(0), W.part(0), lm, 1, s);
    if (st != DMWF_OK) return st;
    const size_t stride = (size_t)p->nalm + kTablePad;
    hipLaunchKernelGGL(k_adj_final, alm_grid(p->lmax, 256), dim3(256), 0, s, W.part(0), 0LL,
                       p->nchunk_ana, stride, p->d_g, W.ap(0), 0LL, 1.0, p->lmax);
    st = launch_ring(p, RING_ANA_WD, W.spec(0), ring_full(p, W, 1), io, s);
    if (st != DMWF_OK) return st;
    st = launch_leg_ana(p, W.spec(0), W.part(0), lm, 1, s);
    if (st != DMWF_OK) return st;
    hipLaunchKernelGGL(k_adj_final, alm_grid(p->lmax, 256), dim3(256), 0, s, W.part(0), 0LL,
                       p->nchunk_ana, stride, p->d_g, W.aux(0), 0LL, 1.0, p->lmax);
    const dim3 gr = alm_grid(p->lmax, 256);
    double* bsum = W.scal_d();
    hipLaunchKernelGGL(k_resid_norms, gr, dim3(256), 0, s, a, W.ap(0), W.aux(0), cl, p->lmax,
                       bsum);
    const int nb = (int)(gr.x * gr.y);
    hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(256), 0, s, bsum, nb, W.out2());
    DMWF_HIP(hipGetLastError());
    double h[2];
    DMWF_HIP(hipMemcpyAsync(h, W.out2(), sizeof(h), hipMemcpyDeviceToHost, s));
    DMWF_HIP(hipStreamSynchronize(s));
    *host_out = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : (h[0] == 0.0 ? 0.0 : INFINITY);
    return DMWF_OK;
}

}  // namespace
}  // namespace dmwf

extern "C" {

dmwf_status dmwf_dm_iterate(dmwf_plan* p, double xi, double alpha, const double* cl,
                            const double* d, const double* ninv, double* alm_state, double* s_map,
                            double* cauchy2, int first, void* ws, size_t ws_bytes, void* stream) {
    if (!p || !cl || !d || !ninv || !alm_state || !s_map || !cauchy2) {
        set_error("NULL argument");
        return DMWF_ERR_INVALID_ARG;
    }
    if (!(alpha > 0.0) || !(xi >= alpha) || !std::isfinite(xi)) {
        set_error("need 0 < alpha <= xi < inf");
        return DMWF_ERR_INVALID_ARG;
    }
    Ws W;
    dmwf_status st = check_ws(p, ws, ws_bytes, &W);
    if (st != DMWF_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const double mu = (xi - alpha) / (1.0 / p->omega);
    {
        // l_iter, the m bounds at l_iter, and the analysis band of the ring
        // stage set to lmax: the residual spectrum left for the next call
        // covers every m, so a later call at a smaller xi (larger l_iter)
        // finds it complete
        ProfScope ps(p, s, PROF_MISC);
        hipLaunchKernelGGL(k_level, dim3((p->nq + 255) / 256), dim3(256), 0, s, cl, p->lmax, mu,
                           p->d_lsmin, p->nq, W.ell(0), W.ell_ana(0), W.mhi(0, p->nq));
    }
    DMWF_HIP(hipGetLastError());
    if (first) {
        RingIO io{};
        io.d = d;
        io.w = ninv;
        const RingMaps rm{1, W.ell_ana(0), W.ell_ana(0), 0, p->d_mhi_full, p->d_mhi_full, 0};
        st = launch_ring(p, RING_ANA_FIRST, W.spec(0), rm, io, s);
        if (st != DMWF_OK) return st;
    }
    return iterate_body(p, W, 0, 1, xi, alpha, mu, cl, d, ninv,
                        reinterpret_cast<double2*>(alm_state), s_map, first ? 1 : 0,
                        p->d_mhi_full, cauchy2, nullptr, s);
}

dmwf_status dmwf_wf_residual(dmwf_plan* p, const double* cl, const double* d, const double* ninv,
                             const double* alm, double* host_out, void* ws, size_t ws_bytes,
                             void* stream) {
    if (!p || !cl || !d || !ninv || !alm || !host_out) {
        set_error("NULL argument");
        return DMWF_ERR_INVALID_ARG;
    }
    Ws W;
    dmwf_status st = check_ws(p, ws, ws_bytes, &W);
    if (st != DMWF_OK) return st;
    for (int k = 0; k < p->nmaps; ++k) {
        st = residual_map(p, W, cl + (size_t)k * (p->lmax + 1), d + (size_t)k * p->npix,
                          ninv + (size_t)k * p->npix,
                          reinterpret_cast<const double2*>(alm) + (size_t)k * p->nalm,
                          host_out + k, static_cast<hipStream_t>(stream));
        if (st != DMWF_OK) return st;
    }
    return DMWF_OK;
}

}  // extern "C"

namespace dmwf {
namespace {

// One plan's share of a solve: its inputs and outputs, its workspace, and the
// host copies of its schedule.
struct SolveJob {
    dmwf_plan* p;
    const double* cl;
    const double* d;
    const double* ninv;
    double2* a;
    double* map;
    dmwf_stats* stats;
    Ws W;
    std::vector<double> alpha;
    std::vector<std::vector<DevLevel>> lv;
    int first_pix = 0;
};

dmwf_status check_schedule(const dmwf_schedule* sc) {
    const double beta = sc->beta > 0.0 ? sc->beta : 0.75;
    if (!(beta < 1.0) || !(sc->eps_final > 0.0) || !(sc->eps_coarse > 0.0) || sc->max_iter < 1 ||
        (sc->replay_iters && sc->n_replay < 1)) {
        set_error("schedule: need 0 < beta < 1, eps > 0, max_iter >= 1");
        return DMWF_ERR_INVALID_ARG;
    }
    return DMWF_OK;
}

// a0 (screening, alpha), a1 (every map's level schedule), the device control
// blocks and the start residual of one plan; synchronizes the stream once.
dmwf_status solve_setup(SolveJob& J, const dmwf_schedule* sc, hipStream_t s) {
    dmwf_plan* p = J.p;
    const Ws& W = J.W;
    const int nm = p->nmaps;
    const int L = p->lmax;
    const double sigma = 1.0 / p->omega;
    const double beta = sc->beta > 0.0 ? sc->beta : 0.75;
    // the reduced contractions hand the last level over to FP64 below this ratio
    const double eps_red = sc->eps_reduced > 0.0 ? sc->eps_reduced : sc->eps_final;
    if (J.stats)
        for (int k = 0; k < nm; ++k)
            if (J.stats[k].cap_levels < 0) {
                set_error("stats.cap_levels < 0");
                return DMWF_ERR_INVALID_ARG;
            }

    // a0: screen the inputs and find alpha = 1 / max N^-1, every map at once
    {
        ProfScope ps(p, s, PROF_MISC);
        hipLaunchKernelGGL(k_set_ints, dim3(1), dim3(64), 0, s, W.flags(0), nm, 0);
        hipLaunchKernelGGL(k_check, dim3(kCheckBlocks, nm), dim3(256), 0, s, J.d, J.ninv,
                           p->npix, J.cl, L + 1, W.flags(0), W.bmax());
        hipLaunchKernelGGL(k_max_final, dim3(nm), dim3(256), 0, s, W.bmax(), kCheckBlocks,
                           W.mdbl(0) + 2, 4);
    }
    DMWF_HIP(hipGetLastError());
    std::vector<int> flags(nm);
    std::vector<double> md(4 * (size_t)nm);
    std::vector<double> hcl((size_t)nm * (L + 1));
    DMWF_HIP(hipMemcpyAsync(flags.data(), W.flags(0), nm * sizeof(int), hipMemcpyDeviceToHost, s));
    DMWF_HIP(hipMemcpyAsync(md.data(), W.mdbl(0), md.size() * sizeof(double),
                            hipMemcpyDeviceToHost, s));
    DMWF_HIP(hipMemcpyAsync(hcl.data(), J.cl, hcl.size() * sizeof(double),
                            hipMemcpyDeviceToHost, s));
    DMWF_HIP(hipStreamSynchronize(s));
    J.alpha.assign(nm, 0.0);
    for (int k = 0; k < nm; ++k) {
        if (flags[k]) {
            set_error("non-finite or negative values in d, N^-1 or C_l of map " +
                      std::to_string(k));
            return DMWF_ERR_NONFINITE;
        }
        const double wmax = md[4 * k + 2];
        if (!(wmax > 0.0)) {
            set_error("every pixel of map " + std::to_string(k) + " is masked (N^-1 = 0)");
            return DMWF_ERR_INVALID_ARG;
        }
        J.alpha[k] = 1.0 / wmax;
    }

    // a1: the level schedule of every map
    J.lv.assign(nm, {});
    for (int k = 0; k < nm; ++k) {
        const double* cl = hcl.data() + (size_t)k * (L + 1);
        double clmax = 0.0;
        for (int l = 0; l <= L; ++l) clmax = std::max(clmax, cl[l]);
        std::vector<double> xis;
        if (sc->start_final) {
            xis.push_back(J.alpha[k]);
        } else {
            const double mu0 = sc->mu0 < 0.0 ? beta * clmax : sc->mu0;
            double xi = J.alpha[k] + sigma * mu0;
            while (xi > J.alpha[k] && (int)xis.size() <= kMaxLevels) {
                xis.push_back(xi);
                xi = beta * xi;
            }
            xis.push_back(J.alpha[k]);
        }
        const int nl = (int)xis.size();
        if (nl > kMaxLevels) {
            set_error("the schedule of map " + std::to_string(k) + " has more than " +
                      std::to_string(kMaxLevels) + " levels");
            return DMWF_ERR_INVALID_ARG;
        }
        if (sc->replay_iters && sc->n_replay != nl) {
            set_error("replay_iters has " + std::to_string(sc->n_replay) + " levels, the schedule of map " +
                      std::to_string(k) + " has " + std::to_string(nl));
            return DMWF_ERR_INVALID_ARG;
        }
        J.lv[k].resize(nl);
        for (int i = 0; i < nl; ++i) {
            const double xi = xis[i], mu = (xi - J.alpha[k]) / sigma;
            int ell = -1;
            for (int l = 0; l <= L; ++l)
                if (cl[l] - mu > 0.0) ell = l;
            J.lv[k][i] = DevLevel{xi,  mu, xi * p->omega, xi <= J.alpha[k] ? sc->eps_final : sc->eps_coarse,
                                  ell, 0,  sc->replay_iters ? sc->replay_iters[i] : 0, 0};
        }
        for (int i = 0; i < nl; ++i) J.lv[k][i].ell_next = J.lv[k][std::min(i + 1, nl - 1)].ell;
    }

    // a1 / a6 on the device: the level tables and control blocks go to the
    // workspace, then every map enters its level 0
    std::vector<DevCtrl> c0(nm);
    int nl_max = 1;
    for (int k = 0; k < nm; ++k) {
        DevCtrl c{};
        c.nlev = (int)J.lv[k].size();
        c.max_iter = sc->max_iter;
        c.replay = sc->replay_iters ? 1 : 0;
        c.alpha = J.alpha[k];
        c.reduced = p->prec != DMWF_FP64 ? 1 : 0;
        c.eps_reduced = eps_red;
        c.best = INFINITY;
        c0[k] = c;
        nl_max = std::max(nl_max, c.nlev);
        DMWF_HIP(hipMemcpyAsync(W.levels(k), J.lv[k].data(), J.lv[k].size() * sizeof(DevLevel),
                                hipMemcpyHostToDevice, s));
    }
    DMWF_HIP(hipMemcpyAsync(W.ctrl(0), c0.data(), nm * sizeof(DevCtrl), hipMemcpyHostToDevice, s));
    {
        ProfScope ps(p, s, PROF_MISC);
        const long long nt = (long long)nl_max * p->nq;
        hipLaunchKernelGGL(k_ctrl_init, dim3(nm), dim3(64), 0, s, W.cmaps());
        hipLaunchKernelGGL(k_level_tab, dim3((unsigned)((nt + 255) / 256), nm), dim3(256), 0, s,
                           p->d_lsmin, p->nq, L, W.levels(0), W.ctrl(0), W.mhi_tab());
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, W.ell_full(), L);
    }
    DMWF_HIP(hipGetLastError());

    // start: r = d on unmasked pixels (cold), or r = c (d - Y a0) at the xi of
    // the first level (warm: alpha with start_final, else the cooling's xi_0)
    const RingMaps full = ring_full(p, W, nm);
    dmwf_status st;
    if (sc->start_final || sc->warm_start) {
        {
            ProfScope ps(p, s, PROF_MISC);
            hipLaunchKernelGGL(k_prep_syn, alm_grid(L, 256, nm), dim3(256), 0, s, J.a, p->nalm,
                               p->d_g, W.ap(0), p->ws.alm_map, L);
        }
        st = leg_syn(p, W.ap(0), W.spec(0), LegMaps{nm, W.ell_full(), 0, nullptr}, s);
        if (st != DMWF_OK) return st;
        RingIO io{};
        io.map_out = J.map;
        io.pix_map = p->npix;
        st = launch_ring(p, RING_SYN, W.spec(0), full, io, s);
        if (st != DMWF_OK) return st;
        io = RingIO{};
        io.map_in = J.map;
        io.d = J.d;
        io.w = J.ninv;
        io.ctrl = W.ctrl(0);
        io.pix_map = p->npix;
        st = launch_ring(p, RING_ANA_CRES, W.spec(0), full, io, s);
        if (st != DMWF_OK) return st;
        J.first_pix = 0;
    } else {
        {
            ProfScope ps(p, s, PROF_MISC);
            hipLaunchKernelGGL(k_zero2, dim3(256), dim3(256), 0, s, J.a, (long long)nm * p->nalm);
        }
        RingIO io{};
        io.d = J.d;
        io.w = J.ninv;
        io.pix_map = p->npix;
        st = launch_ring(p, RING_ANA_FIRST, W.spec(0), full, io, s);
        if (st != DMWF_OK) return st;
        J.first_pix = 1;
    }
    DMWF_HIP(hipGetLastError());
    return DMWF_OK;
}

// Every plan's iterations until every map of every plan has stopped.  After
// each iteration k_control takes each map's decision.  The host enqueues
// iterations in growing batches with two batches in flight and reads the
// control blocks once per batch, so the GPU never waits for the host;
// iterations enqueued after a map's stop do nothing for that map.  Every
// iteration after the first is the same sequence of launches with the same
// arguments: one HIP graph holds it for every plan (the plans one after
// another; the ring stage's side-stream fork and join become graph branches)
// and is replayed, which takes the per-launch host cost off the loop.  Timing
// events are not recorded by graph replays: with every launch timed
// (profiling level 1 on some plan) the iterations are launched one by one;
// with the analysis timed (level 2) it is launched between its events and
// the rest of the iteration is replayed from the graph.
dmwf_status solve_loop(std::vector<SolveJob>& jobs, const dmwf_schedule* sc, hipStream_t s,
                       std::vector<const DevCtrl*>& fin) {
    bool any_prof1 = false;
    for (auto& J : jobs) any_prof1 |= J.p->prof == 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    struct GraphGuard {
        hipGraph_t* g;
        hipGraphExec_t* e;
        hipStream_t s;
        ~GraphGuard() {
            if (*e) {
                (void)hipStreamSynchronize(s);  // no replay still in flight
                (void)hipGraphExecDestroy(*e);
            }
            if (*g) (void)hipGraphDestroy(*g);
        }
    } guard{&graph, &gexec, s};
    auto body = [&](SolveJob& J, hipStream_t st_) {
        dmwf_plan* p = J.p;
        return iterate_body(p, J.W, 0, p->nmaps, 0.0, 0.0, 0.0, J.cl, J.d, J.ninv, J.a, J.map,
                            J.first_pix, nullptr, nullptr, J.W.ctrl(0), st_);
    };
    auto one_iteration = [&]() -> dmwf_status {
        bool first = false;
        for (auto& J : jobs) first |= J.first_pix != 0;
        if (first || any_prof1) {
            for (auto& J : jobs) {
                dmwf_status e = body(J, s);
                J.first_pix = 0;
                if (e != DMWF_OK) return e;
            }
            return DMWF_OK;
        }
        if (!gexec) {
            // captured on the first plan's own stream (the caller's may be the
            // null stream, which cannot be captured), replayed on the caller's
            hipStream_t cs = jobs[0].p->cap_stream;
            DMWF_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            dmwf_status e = DMWF_OK;
            for (auto& J : jobs) {
                dmwf_plan* p = J.p;
                e = p->prof == 2
                        ? iterate_rest(p, J.W, 0, p->nmaps, 0.0, 0.0, 0.0, J.cl, J.d, J.ninv, J.a,
                                       J.map, 0, nullptr, nullptr, J.W.ctrl(0), cs)
                        : body(J, cs);
                if (e != DMWF_OK) break;
            }
            const hipError_t ce = hipStreamEndCapture(cs, &graph);
            if (e != DMWF_OK) return e;
            DMWF_HIP(ce);
            DMWF_HIP(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
        }
        for (auto& J : jobs)
            if (J.p->prof == 2) {
                dmwf_status e = iterate_ana(J.p, J.W, 0, J.p->nmaps, J.W.ctrl(0), s);
                if (e != DMWF_OK) return e;
            }
        DMWF_HIP(hipGraphLaunch(gexec, s));
        return DMWF_OK;
    };
    hipEvent_t* bev = jobs[0].p->batch_ev;
    auto enqueue = [&](int nit, int slot) -> dmwf_status {
        for (int i = 0; i < nit; ++i) {
            dmwf_status e = one_iteration();
            if (e != DMWF_OK) return e;
        }
        for (auto& J : jobs) {
            const int nm = J.p->nmaps;
            DMWF_HIP(hipMemcpyAsync(J.p->h_ctrl + (size_t)slot * nm, J.W.ctrl(0),
                                    nm * sizeof(DevCtrl), hipMemcpyDeviceToHost, s));
        }
        DMWF_HIP(hipEventRecord(bev[slot], s));
        return DMWF_OK;
    };
    auto all_done = [&](int slot) {
        for (auto& J : jobs) {
            const int nm = J.p->nmaps;
            for (int k = 0; k < nm; ++k)
                if (!J.p->h_ctrl[(size_t)slot * nm + k].done) return false;
        }
        return true;
    };
    // never more iterations than the cap allows, nor (replaying) than the
    // replayed counts add up to: a replayed solve enqueues exactly its
    // iterations
    long long budget = sc->max_iter;
    if (sc->replay_iters) {
        long long sum = 0;
        for (int i = 0; i < sc->n_replay; ++i) sum += std::max(1, sc->replay_iters[i]);
        budget = std::min(budget, sum);
    }
    long long launched = 0;
    int batch = 4, cur = 0;
    int nb = (int)std::min<long long>(batch, budget);
    dmwf_status st = enqueue(nb, cur);
    if (st != DMWF_OK) return st;
    launched += nb;
    bool whole[2] = {launched >= budget, false};  // snapshot taken after the whole budget
    while (true) {
        batch = std::min(2 * batch, 64);
        nb = (int)std::min<long long>(batch, budget - launched);
        st = enqueue(nb, cur ^ 1);
        if (st != DMWF_OK) return st;
        launched += nb;
        whole[cur ^ 1] = launched >= budget;
        DMWF_HIP(hipEventSynchronize(bev[cur]));
        if (all_done(cur)) {
            DMWF_HIP(hipEventSynchronize(bev[cur ^ 1]));
            cur ^= 1;
            break;
        }
        if (whole[cur]) {
            // every map stops within the budget (the cap, or the replayed
            // counts); a snapshot after it with a map still running is a
            // control failure, reported instead of waiting forever
            set_error("solve loop: a map did not stop within its iteration budget");
            return DMWF_ERR_HIP;
        }
        cur ^= 1;
    }
    fin.clear();
    for (auto& J : jobs) fin.push_back(J.p->h_ctrl + (size_t)cur * J.p->nmaps);
    return DMWF_OK;
}

// Statuses and statistics of one plan's maps after the loop.
dmwf_status solve_finish(SolveJob& J, const dmwf_schedule* sc, const DevCtrl* fin, hipStream_t s,
                         dmwf_status* result) {
    dmwf_plan* p = J.p;
    const int nm = p->nmaps;
    for (int k = 0; k < nm; ++k) {
        if (fin[k].status == 2) {
            set_error("Cauchy ratio of map " + std::to_string(k) + " is NaN");
            return DMWF_ERR_NONFINITE;
        }
        if (fin[k].status == 1) *result = DMWF_ERR_NOT_CONVERGED;
    }
    if (!J.stats) return DMWF_OK;
    const int L = p->lmax;
    for (int k = 0; k < nm; ++k) {
        dmwf_stats& S = J.stats[k];
        const int nlev = fin[k].level + 1;
        std::vector<int> its(J.lv[k].size(), 0);
        DMWF_HIP(hipMemcpy(its.data(), J.W.lev_iters(k), its.size() * sizeof(int),
                           hipMemcpyDeviceToHost));
        for (int i = 0; i < nlev && i < S.cap_levels; ++i) {
            if (S.iters_per_level) S.iters_per_level[i] = its[i];
            if (S.xi_per_level) S.xi_per_level[i] = J.lv[k][i].xi;
            if (S.lmax_per_level) S.lmax_per_level[i] = J.lv[k][i].ell;
        }
        S.n_levels = nlev;
        S.n_iter = fin[k].total;
        S.iters_reduced = fin[k].it_reduced;
        S.alpha = J.alpha[k];
        S.final_cauchy = fin[k].ratio;
        S.wf_residual = -1.0;
        if (sc->want_residual) {
            double res = 0.0;
            dmwf_status st = residual_map(p, J.W, J.cl + (size_t)k * (L + 1),
                                          J.d + (size_t)k * p->npix, J.ninv + (size_t)k * p->npix,
                                          J.a + (size_t)k * p->nalm, &res, s);
            if (st != DMWF_OK) return st;
            S.wf_residual = res;
        }
    }
    return DMWF_OK;
}

dmwf_status solve_jobs(std::vector<SolveJob>& jobs, const dmwf_schedule* sc, hipStream_t s) {
    for (auto& J : jobs) {
        dmwf_status st = solve_setup(J, sc, s);
        if (st != DMWF_OK) return st;
    }
    std::vector<const DevCtrl*> fin;
    dmwf_status st = solve_loop(jobs, sc, s, fin);
    if (st != DMWF_OK) return st;
    dmwf_status result = DMWF_OK;
    for (size_t i = 0; i < jobs.size(); ++i) {
        st = solve_finish(jobs[i], sc, fin[i], s, &result);
        if (st != DMWF_OK) return st;
    }
    return result;
}

}  // namespace
}  // namespace dmwf

extern "C" {

dmwf_status dmwf_solve(dmwf_plan* p, const double* cl_all, const double* d_all,
                       const double* ninv_all, const dmwf_schedule* sc, double* alm_all,
                       double* map_all, dmwf_stats* stats, void* ws, size_t ws_bytes,
                       void* stream) {
    if (!p || !cl_all || !d_all || !ninv_all || !sc || !alm_all || !map_all) {
        set_error("NULL argument");
        return DMWF_ERR_INVALID_ARG;
    }
    dmwf_status st = check_schedule(sc);
    if (st != DMWF_OK) return st;
    std::vector<SolveJob> jobs(1);
    SolveJob& J = jobs[0];
    J.p = p;
    J.cl = cl_all;
    J.d = d_all;
    J.ninv = ninv_all;
    J.a = reinterpret_cast<double2*>(alm_all);
    J.map = map_all;
    J.stats = stats;
    st = check_ws(p, ws, ws_bytes, &J.W);
    if (st != DMWF_OK) return st;
    return solve_jobs(jobs, sc, static_cast<hipStream_t>(stream));
}

dmwf_status dmwf_solve_plans(int nplans, dmwf_plan* const* plans, const double* const* cl,
                             const double* const* d, const double* const* ninv,
                             const dmwf_schedule* sc, double* const* alm_out,
                             double* const* map_out, dmwf_stats* const* stats, void* const* ws,
                             const size_t* ws_bytes, void* stream) {
    if (nplans < 1 || nplans > 64 || !plans || !cl || !d || !ninv || !sc || !alm_out ||
        !map_out || !ws || !ws_bytes) {
        set_error("NULL argument, or nplans outside 1..64");
        return DMWF_ERR_INVALID_ARG;
    }
    dmwf_status st = check_schedule(sc);
    if (st != DMWF_OK) return st;
    std::vector<SolveJob> jobs(nplans);
    for (int i = 0; i < nplans; ++i) {
        if (!plans[i] || !cl[i] || !d[i] || !ninv[i] || !alm_out[i] || !map_out[i]) {
            set_error("NULL argument for plan " + std::to_string(i));
            return DMWF_ERR_INVALID_ARG;
        }
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i] || ws[j] == ws[i]) {
                set_error("plans " + std::to_string(j) + " and " + std::to_string(i) +
                          " share a plan or a workspace");
                return DMWF_ERR_INVALID_ARG;
            }
        SolveJob& J = jobs[i];
        J.p = plans[i];
        J.cl = cl[i];
        J.d = d[i];
        J.ninv = ninv[i];
        J.a = reinterpret_cast<double2*>(alm_out[i]);
        J.map = map_out[i];
        J.stats = stats ? stats[i] : nullptr;
        st = check_ws(plans[i], ws[i], ws_bytes[i], &J.W);
        if (st != DMWF_OK) return st;
    }
    return solve_jobs(jobs, sc, static_cast<hipStream_t>(stream));
}

}  // extern "C"
