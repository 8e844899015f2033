// Ring stage of the transform pair: the phi part of F / F^-1 on each HEALPix
// ring, fused with the pixel-space half of the dual messenger iteration.
//
// One workgroup per ring pair: the north ring and its south mirror share the
// pixel count n and the first-pixel angle phi0 = pi c, so both are carried by
// one complex transform z = (north) + i (south).  With phi_j = phi0 + 2 pi j/n:
//
//   synthesis  s_j = sum_{|m| <= l} F_m e^{i m phi_j} = sum_k H_k w^{jk},
//              H_k = sum_{m = k mod n} F_m e^{i m phi0}   (aliasing fold, F_{-m} = conj F_m)
//   analysis   G_m = e^{-i m phi0} R_{m mod n},  R_k = sum_j r_j w^{-jk},  w = e^{2 pi i/n}.
//
// The length-n DFTs are Stockham FFTs whose data stay in registers: each
// thread holds E = 8 elements (stride M / 8) and computes one radix-8
// butterfly per pass with twiddles formed in registers; between passes the
// outputs go through LDS (padded against bank conflicts), and a last pass of
// radix 4 or 2 takes the remaining bits.  Ring lengths that are not powers of
// two (polar rings, n = 4i), and rings shorter than 16 pixels, use Bluestein's
// chirp-z identity jk = (j^2 + k^2 - (k-j)^2)/2, which turns the DFT into a
// cyclic convolution of length M >= 2n-1 (a power of two, at least 16) with
// the chirp c_t = e^{i pi t^2/n}; the spectrum of the chirp filter is a plan
// table.
//
// In RING_ITER mode the workgroup also performs the pixel step of the paper's
// Algorithm 2 in residual form: it reads s_prev, writes s, accumulates the
// Cauchy sums sum (s - s_prev)^2 and sum s^2, forms r = c (d - s) with
// c = xi w / (1 + (xi - alpha) w) (messenger step with N_bar = N - alpha)
// and analyses r into G, overwriting F in place.
//
// Workgroups are launched in five classes by FFT length (M <= 512, 1024,
// 2048, 4096, 8192), so that small rings neither reserve the LDS of the
// largest nor leave threads of a larger class's workgroup idle; within a
// class the ring pairs are ordered so that consecutive pairs land on the same
// XCD and share its L2 for the neighbouring F/G lines.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace dmwf {
namespace {

enum PixSource { PIX_MAP = 0, PIX_FIRST = 1, PIX_WRES = 2, PIX_WD = 3, PIX_CRES = 4 };

struct RingArgs {
    RingGeom g;
    int nq, lmax, lp;
    double2* spec;
    long long spec_map;
    int mode;
    int pix;
    RingIO io;
    RingMaps rm;
    const int* qlist;
    const int* Mq;
    const int* blue;
    const long long* coff;
    const long long* boff;
    const double2* chirp;
    const double2* bspec;
};

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }

// Workgroup barrier that orders LDS only.  Global stores issued before it may
// still be in flight: no thread of a workgroup reads global memory that
// another thread of the same workgroup wrote (the F row of a ring pair is
// read, and waited for, long before its G row is written over it).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS layout: logical element e lives at e + e/16 (one pad slot per 16) so
// that sixteen lanes touching sixteen consecutive butterflies' outputs of the
// first pass fall in distinct banks.
__device__ __forceinline__ int pad(int e) { return e + (e >> 4); }

constexpr int ilog2(int r) { return r <= 1 ? 0 : 1 + ilog2(r >> 1); }
constexpr int bitrev(int i, int bits) { return bits == 0 ? 0 : ((i & 1) << (bits - 1)) | bitrev(i >> 1, bits - 1); }

// cos and sin of k pi / 8, k = 0..7
__device__ constexpr double kC8[8] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                                      0.38268343236508977173, 0.0, -0.38268343236508977173,
                                      -0.70710678118654752440, -0.92387953251128675613};
__device__ constexpr double kS8[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440,
                                      0.92387953251128675613, 1.0, 0.92387953251128675613,
                                      0.70710678118654752440, 0.38268343236508977173};

// Element i of the bit-reversal permutation of v (all indices compile-time).
template <int R, int I>
__device__ __forceinline__ void bitrev_swap(double2 (&v)[R]) {
    if constexpr (I < R) {
        constexpr int J = bitrev(I, ilog2(R));
        if constexpr (I < J) {
            const double2 t = v[I];
            v[I] = v[J];
            v[J] = t;
        }
        bitrev_swap<R, I + 1>(v);
    }
}

// One radix-2 DIT stage combining length-H sub-transforms, butterfly (B, K).
template <int R, int H, int B, int K>
__device__ __forceinline__ void dit_butterflies(double2 (&v)[R]) {
    if constexpr (B < R) {
        if constexpr (K < H) {
            constexpr int idx = K * (8 / H);  // e^{-i pi K / H}
            const double2 x1 = v[B + K];
            double2 x2 = v[B + K + H];
            if constexpr (idx == 4) x2 = make_double2(x2.y, -x2.x);  // times -i
            else if constexpr (idx != 0) x2 = cmul(make_double2(kC8[idx], -kS8[idx]), x2);
            v[B + K] = cadd(x1, x2);
            v[B + K + H] = csub(x1, x2);
            dit_butterflies<R, H, B, K + 1>(v);
        } else {
            dit_butterflies<R, H, B + 2 * H, 0>(v);
        }
    }
}

template <int R, int H>
__device__ __forceinline__ void dit_stages(double2 (&v)[R]) {
    if constexpr (H < R) {
        dit_butterflies<R, H, 0, 0>(v);
        dit_stages<R, 2 * H>(v);
    }
}

// Radix-R DFT in registers, natural order in and out: V_t = sum_r v_r e^{-2 pi i r t / R}.
template <int R>
__device__ __forceinline__ void dft_small(double2 (&v)[R]) {
    bitrev_swap<R, 0>(v);
    dit_stages<R, 1>(v);
}

// ---------------------------------------------------------------------------
// FFT on the owner layout.  For a transform of length M (every ring FFT has
// M >= 16: rings shorter than 16 pixels go through Bluestein at M = 16) with
// E elements per thread (E = 16 or 8), thread t < S = M / E holds elements
// t + e S, e = 0..E-1, in x[e].  A Stockham pass of radix R at stride Ns lets
// butterfly j read elements j + r M / R and write output t to
// (j / Ns) Ns R + (j mod Ns) + t Ns.  In the owner layout a thread's
// butterflies j = t + i S (i < E / R) read exactly its own elements, so each
// pass starts from registers; the outputs go through LDS to the next pass,
// except after the last pass, whose outputs land on the owner layout again.
// A transform therefore stores and loads LDS once per pass boundary, and
// whatever runs before and after it (the fold, the filter product, the pixel
// step) works on registers.
// ---------------------------------------------------------------------------

// Radix-R butterflies of one pass at stride Ns on the owner registers: the
// thread's butterfly i (j = tid + i S) takes x[i + r B] as input r and leaves
// its output t in x[i + t B], B = E / R.  Radix E has one butterfly per
// thread; a smaller radix is only ever the last pass (Ns R = M).  TW: the
// pass has twiddles (every pass but the first, Ns > 1).
template <int E, int R, bool TW>
__device__ __forceinline__ void pass_regs(double2 (&x)[E], int M, int Ns, int tid, int S,
                                          const double2* __restrict__ tw) {
    constexpr int B = E / R;
    // Twiddle base of the thread's first butterfly, w = e^{-2 pi i k / (Ns R)}
    // = omega_M^t with k = j mod Ns, from the two-level root table.  In the
    // last pass t = j, so butterfly i's base is this one times
    // omega_M^{i S} = e^{-2 pi i i / E}.
    double2 base = make_double2(1.0, 0.0);
    if constexpr (TW) {
        const int t = R == E ? (tid & (Ns - 1)) * (M / (Ns * E)) : tid;
        base = cmul(tw[t & 63], tw[64 + (t >> 6)]);
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = x[i + r * B];
        if constexpr (TW) {
            // powers w^r one product at a time (at most R - 1 roundings)
            const int ci = i * (16 / E);  // e^{-2 pi i i / E} = e^{-i pi ci / 8}
            const double2 w1 = i == 0 ? base : cmul(base, make_double2(kC8[ci], -kS8[ci]));
            double2 w = w1;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                v[r] = cmul(w, v[r]);
                if (r + 1 < R) w = cmul(w, w1);
            }
        }
        dft_small<R>(v);
#pragma unroll
        for (int r = 0; r < R; ++r) x[i + r * B] = v[r];
    }
}

// Outputs of a radix-E pass at stride Ns to LDS in Stockham order, then the
// owner layout back for the next pass.
template <int E>
__device__ __forceinline__ void exchange(double2 (&x)[E], double2* buf, int Ns, int tid, int S,
                                         bool act) {
    if (act) {
        const int o = (tid & ~(Ns - 1)) * E + (tid & (Ns - 1));
#pragma unroll
        for (int t = 0; t < E; ++t) buf[pad(o + t * Ns)] = x[t];
    }
    lds_barrier();
    if (act) {
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = buf[pad(tid + e * S)];
    }
    lds_barrier();
}

// Forward DFT of length M = 2^logM on the owner layout: radix-E passes
// while log2 E or more bits remain, then one pass of the remaining radix.
// MFIX > 0 fixes M at compile time (one code path per launch class), MFIX = 0
// takes it at run time.  Every thread of the workgroup calls it (it holds
// barriers).
template <int E, int MFIX>
__device__ __forceinline__ void fft_owner(double2 (&x)[E], double2* buf, int M, int logM, int tid,
                                          const double2* __restrict__ tw) {
    constexpr int LE = ilog2(E);
    // opaque copy of the thread index: keeps the passes' LDS addresses from
    // being hoisted out of the caller's loop into long-lived registers
    asm volatile("" : "+v"(tid));
    const int lm = MFIX > 0 ? ilog2(MFIX) : logM;
    const int S = M / E;
    const bool act = tid < S;
    const int nmain = lm / LE;
    const int L = lm - nmain * LE;
    // first pass (radix E, no twiddles), then radix-E passes at Ns = E, E^2,
    // ..., then the last pass of radix 2^L when L > 0
    if (act) pass_regs<E, E, false>(x, M, 1, tid, S, tw);
    if (nmain > 1 || L != 0) exchange<E>(x, buf, 1, tid, S, act);
    int Ns = E;
#pragma unroll 1
    for (int p = 1; p < nmain; ++p) {
        if (act) pass_regs<E, E, true>(x, M, Ns, tid, S, tw);
        if (p < nmain - 1 || L != 0) exchange<E>(x, buf, Ns, tid, S, act);
        Ns *= E;
    }
    if (act) {
        if constexpr (E == 16) {
            if (L == 3) pass_regs<E, 8, true>(x, M, Ns, tid, S, tw);
            else if (L == 2) pass_regs<E, 4, true>(x, M, Ns, tid, S, tw);
            else if (L == 1) pass_regs<E, 2, true>(x, M, Ns, tid, S, tw);
        } else {
            if (L == 2) pass_regs<E, 4, true>(x, M, Ns, tid, S, tw);
            else if (L == 1) pass_regs<E, 2, true>(x, M, Ns, tid, S, tw);
        }
    }
}

// Roots of unity omega_M^t = e^{-2 pi i t / M} for t < M / 2 as the product
// tw[t mod 64] tw[64 + t / 64]: 128 entries (2 KB of LDS) per workgroup,
// written before the workgroup's first FFT (callers place a barrier between).
template <int NT>
__device__ __forceinline__ void root_table(double2* tw, int M, int tid) {
    for (int i = tid; i < 128; i += NT) {
        const int e = i < 64 ? i : (i - 64) * 64;
        double sn, cs;
        sincospi(-2.0 * e / M, &sn, &cs);
        tw[i] = make_double2(cs, sn);
    }
}

// Middle step of Bluestein's algorithm on the owner layout: x = FFT_M(a) on
// entry; leaves conj(x B) / M, whose forward FFT is conj(M conv), conv = a (*) b
// the cyclic convolution of length M (B = FFT_M(b) from the plan, loaded into
// the owner layout by load_owner before the FFT that precedes this step).
template <int E>
__device__ __forceinline__ void load_owner(double2 (&v)[E], const double2* __restrict__ src,
                                           int tid, int S) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = src[tid + e * S];
}
template <int E>
__device__ __forceinline__ void filter_regs(double2 (&x)[E], int M, const double2 (&b)[E]) {
    const double inv = 1.0 / M;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const double2 v = cmul(x[e], b[e]);
        x[e] = make_double2(v.x * inv, -v.y * inv);
    }
}

// Sum of (u, v) over the workgroup, returned in thread 0.
template <int NT>
__device__ __forceinline__ double2 block_sum2(double u, double v, double2* scratch) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        u += __shfl_xor(u, o);
        v += __shfl_xor(v, o);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) scratch[w] = make_double2(u, v);
    lds_barrier();
    double2 t = make_double2(0.0, 0.0);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) t = cadd(t, scratch[i]);
    }
    return t;
}

// Contribution of mode m of the F row to the DFT input Z = H^N + i H^S:
// +m feeds bin kp with zp, -m feeds bin km with zm (F_{-m} = conj F_m).
struct FoldTerm {
    double2 zp, zm;
    int kp, km;
};

__device__ __forceinline__ FoldTerm fold_term(double2 fn, double2 fs, int m, int n, double c,
                                              bool eq) {
    double sn, cs;
    sincospi(m * c, &sn, &cs);
    const double2 ph = make_double2(cs, sn);
    if (m == 0) {
        fn.y = 0.0;
        fs.y = 0.0;
    }
    if (eq) fs = make_double2(0.0, 0.0);
    const double2 en = cmul(fn, ph), es = cmul(fs, ph);
    FoldTerm f;
    f.zp = make_double2(en.x - es.y, en.y + es.x);
    f.zm = make_double2(en.x + es.y, es.x - en.y);
    f.kp = m % n;
    f.km = f.kp == 0 ? 0 : n - f.kp;
    return f;
}

// Bin m of the analysed ring pair, G^N_m and G^S_m, from Z_k and Z_{n-k}
// (k = m mod n), both already divided by the chirp for Bluestein rings.
__device__ __forceinline__ void unfold_store(double2 zk, double2 zc, int m, double c, bool eq,
                                             double2* g) {
    const double2 czc = conj2(zc);
    const double2 rN = make_double2(0.5 * (zk.x + czc.x), 0.5 * (zk.y + czc.y));
    const double2 dS = csub(zk, czc);  // R^S = -i dS / 2
    const double2 rS = make_double2(0.5 * dS.y, -0.5 * dS.x);
    double sn, cs;
    sincospi(m * c, &sn, &cs);
    const double2 ph = make_double2(cs, -sn);
    double2 gN = cmul(rN, ph), gS = eq ? make_double2(0.0, 0.0) : cmul(rS, ph);
    if (m == 0) {
        gN.y = 0.0;
        gS.y = 0.0;
    }
    g[0] = gN;
    g[1] = gS;
}

// One workgroup per ring pair.  NT threads, E FFT elements per thread in the
// owner layout, J of them pixels (n <= J S), MFIX the FFT length of the class
// (0: run time).  d and N^-1 of the first PJ elements are loaded before the
// last synthesis FFT.  At most 128 VGPRs (four waves per SIMD): the LDS of
// the classes allows 16 waves per CU, and the registers must not allow fewer.
template <int NT, int E, int J, int MFIX>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_ring_fft(RingArgs a) {
    extern __shared__ double2 buf[];
    __shared__ double2 red[NT / 64];
    __shared__ double2 tw[128];
    // grid.y is the map: every per-map array is offset to its slice here
    const int map = blockIdx.y;
    const DevCtrl* ctrl = a.io.ctrl ? a.io.ctrl + map : nullptr;
    if (ctrl && ctrl->done) return;
    const long long po = map * a.io.pix_map;
    const double* dd = a.io.d + po;
    const double* ww = a.io.w + po;
    const double* min_ = a.io.map_in + po;
    double* mout = a.io.map_out + po;
    double* smap = a.io.s_map + po;
    double2* spec = a.spec + map * a.spec_map;
    const int q = a.qlist[blockIdx.x];
    const int n = a.g.nph[q];
    const int M = MFIX > 0 ? MFIX : a.Mq[q];
    const int logM = 31 - __clz(M);
    const bool blue = a.blue[q] != 0;
    const double2* ch = a.chirp + a.coff[q];
    const double2* B = a.bspec + a.boff[q];
    const double c = a.g.phi0pi[q];
    const bool eq = (q == a.nq - 1);
    const long long st0 = a.g.start_n[q], st1 = a.g.start_s[q];
    int msyn, mana;
    if (ctrl && a.mode == RING_ITER) {
        // m bounds of the current level (synthesis) and of the next (analysis)
        const int* tab = a.io.mhi_tab + (size_t)map * kMaxLevels * a.nq;
        const int lev = ctrl->level, nxt = min(lev + 1, ctrl->nlev - 1);
        msyn = tab[(size_t)lev * a.nq + q];
        mana = tab[(size_t)nxt * a.nq + q];
    } else {
        msyn = a.rm.mhi_syn[map * a.rm.mhi_stride + q];
        mana = a.rm.mhi_ana[map * a.rm.mhi_stride + q];
    }
    const int ell = min(a.rm.ell_syn[map * a.rm.ell_stride], msyn);
    const int ella = min(a.rm.ell_ana[map * a.rm.ell_stride], mana);
    // pixel step coefficients: the map's own in the solve loop (the warm
    // start's residual takes the xi of the level the solve starts on)
    const double xi_ = ctrl ? ctrl->xi : a.io.xi;
    const double alpha_ = ctrl ? ctrl->alpha : a.io.alpha;
    const int tid = threadIdx.x;
    // owner layout: stride S, E elements per thread, threads tid < S active
    const int S = M / E;
    const bool act = tid < S;
    // modes per thread and batch in the fold
    constexpr int FB = NT >= 512 ? 4 : 6;
    constexpr bool CHR = J <= 4;
    constexpr int PJ = J < 4 ? J : 4;

    double2 x[E];
    const bool syn = (a.mode == RING_SYN || a.mode == RING_ITER || a.mode == RING_SYN_WRES);
    // Chirp of a Bluestein ring at the thread's elements (k < n <= J S): with
    // CHR held in registers for its four uses (fold input, pixel output,
    // pixel input, analysis output), else loaded at each use.
    double2 chr[CHR ? J : 1];
    if constexpr (CHR) {
#pragma unroll
        for (int e = 0; e < J; ++e) {
            const int k = tid + e * S;
            chr[e] = blue && act && k < n ? ch[k] : make_double2(1.0, 0.0);
        }
    }
    auto chirp = [&](int e) -> double2 {
        if constexpr (CHR) return chr[e < J ? e : 0];
        else return ch[tid + e * S];
    };
    root_table<NT>(tw, M, tid);  // read after the barriers of the input stage
    if (syn) {
        // Fold F into the DFT input x_k = conj(Z_k) [times conj(c_k)],
        // Z_k = H^N_k + i H^S_k, H_k = sum over m = k mod n of F_m e^{i m phi0}.
        // The row of F is read once, coalesced, and scattered to the bins in
        // LDS: m feeds bin m mod n, and -m feeds bin -m mod n.  Bins collide
        // when 2 ell > n (summed with LDS atomics on zeroed bins); at
        // 2 ell = n only m = n/2 meets -m, which one thread handles alone.
        const double2* Fq = spec + (size_t)q * a.lp * 2;
        const bool alias = 2 * ell > n;
        if (alias) {
            for (int k = tid; k < n; k += NT) buf[pad(k)] = make_double2(0.0, 0.0);
            lds_barrier();
        }
        for (int m0 = tid; m0 <= ell; m0 += FB * NT) {
            // loads for FB modes first: at lmax = 2 nside one batch covers
            // the row, so the fold waits on memory once
            double2 fnv[FB], fsv[FB];
#pragma unroll
            for (int u = 0; u < FB; ++u) {
                const int m = m0 + u * NT;
                fnv[u] = fsv[u] = make_double2(0.0, 0.0);
                if (m <= ell) {
                    fnv[u] = Fq[2 * m];
                    fsv[u] = Fq[2 * m + 1];
                }
            }
#pragma unroll
            for (int u = 0; u < FB; ++u) {
                const int m = m0 + u * NT;
                if (m > ell) continue;
                const FoldTerm f = fold_term(fnv[u], fsv[u], m, n, c, eq);
                if (alias) {
                    atomicAdd(&buf[pad(f.kp)].x, f.zp.x);
                    atomicAdd(&buf[pad(f.kp)].y, f.zp.y);
                    if (m > 0) {
                        atomicAdd(&buf[pad(f.km)].x, f.zm.x);
                        atomicAdd(&buf[pad(f.km)].y, f.zm.y);
                    }
                } else if (m > 0 && f.km == f.kp) {
                    buf[pad(f.kp)] = cadd(f.zp, f.zm);
                } else {
                    buf[pad(f.kp)] = f.zp;
                    if (m > 0) buf[pad(f.km)] = f.zm;
                }
            }
        }
        lds_barrier();
        // owner layout: conj, and the chirp of Bluestein rings; bins no mode
        // reached (n <= k, or ell < k < n - ell without aliasing) are zero
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = tid + e * S;
            double2 v = make_double2(0.0, 0.0);
            if (act && k < n && (alias || k <= ell || k >= n - ell)) {
                v = conj2(buf[pad(k)]);
                if (blue && e < J) v = cmul(v, conj2(chirp(e)));
            }
            x[e] = v;
        }
        lds_barrier();

        // Each DFT is one FFT, or two around the filter product for Bluestein
        // rings.  Memory that a later step needs is loaded before the FFT
        // that precedes it, so that its latency hides behind the FFT: the
        // filter spectrum, and d and N^-1 of the pixel step's first elements.
        double pd[4 * PJ];
        if (blue) {
            double2 bq[E];
            if (act) load_owner<E>(bq, B, tid, S);
            fft_owner<E, MFIX>(x, buf, M, logM, tid, tw);
            if (act) filter_regs<E>(x, M, bq);
        }
#pragma unroll
        for (int e = 0; e < PJ; ++e) {
            const int j = tid + e * S;
            double* v = pd + 4 * e;
            v[0] = v[1] = v[2] = v[3] = 0.0;
            if (act && j < n && a.mode != RING_SYN) {
                v[0] = dd[st0 + j];
                v[1] = ww[st0 + j];
                if (!eq) {
                    v[2] = dd[st1 + j];
                    v[3] = ww[st1 + j];
                }
            }
        }
        fft_owner<E, MFIX>(x, buf, M, logM, tid, tw);
        // y_j = IDFT(Z)_j: blue: c_j x_j; else conj(x_j).  s^N = Re y, s^S = Im y.
        // Pixel data are loaded for JH of the thread's elements first, then
        // combined and stored, so the loads of one pixel never wait on the
        // store of another.  The residual r replaces y in the register as
        // the analysis input z_j = r^N_j + i r^S_j [times conj(c_j)], and
        // zero beyond n (the padding of Bluestein rings).
        double num = 0.0, den = 0.0;
        constexpr int JH = 4;
#pragma unroll
        for (int e0 = 0; e0 < E; e0 += JH) {
            double yN[JH], yS[JH], dN[JH], dS[JH], wN[JH], wS[JH], pN[JH], pS[JH];
#pragma unroll
            for (int u = 0; u < JH; ++u) {
                const int e = e0 + u;
                const int j = tid + e * S;
                yN[u] = yS[u] = dN[u] = dS[u] = wN[u] = wS[u] = pN[u] = pS[u] = 0.0;
                if (e < J && act && j < n) {
                    const double2 y = blue ? cmul(chirp(e), x[e]) : conj2(x[e]);
                    yN[u] = y.x;
                    yS[u] = y.y;
                    if (e < PJ) {
                        const double* v = pd + 4 * (e < PJ ? e : 0);
                        dN[u] = v[0];
                        wN[u] = v[1];
                        dS[u] = v[2];
                        wS[u] = v[3];
                        if (a.mode == RING_ITER && !a.io.first) {
                            pN[u] = smap[st0 + j];
                            if (!eq) pS[u] = smap[st1 + j];
                        }
                    } else if (a.mode != RING_SYN) {
                        dN[u] = dd[st0 + j];
                        wN[u] = ww[st0 + j];
                        if (!eq) {
                            dS[u] = dd[st1 + j];
                            wS[u] = ww[st1 + j];
                        }
                        if (a.mode == RING_ITER && !a.io.first) {
                            pN[u] = smap[st0 + j];
                            if (!eq) pS[u] = smap[st1 + j];
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < JH; ++u) {
                const int e = e0 + u;
                const int j = tid + e * S;
                double2 z = make_double2(0.0, 0.0);
                if (e < J && act && j < n) {
                    double rn = 0.0, rs = 0.0;
                    if (a.mode == RING_SYN) {
                        mout[st0 + j] = yN[u];
                        if (!eq) mout[st1 + j] = yS[u];
                    } else if (a.mode == RING_SYN_WRES) {
                        rn = wN[u] * (dN[u] - yN[u]);
                        rs = eq ? 0.0 : wS[u] * (dS[u] - yS[u]);
                    } else {
                        const double xi = xi_, xa = xi_ - alpha_;
                        double ds = yN[u] - pN[u];
                        num = fma(ds, ds, num);
                        den = fma(yN[u], yN[u], den);
                        smap[st0 + j] = yN[u];
                        rn = xi * wN[u] / fma(xa, wN[u], 1.0) * (dN[u] - yN[u]);
                        if (!eq) {
                            ds = yS[u] - pS[u];
                            num = fma(ds, ds, num);
                            den = fma(yS[u], yS[u], den);
                            smap[st1 + j] = yS[u];
                            rs = xi * wS[u] / fma(xa, wS[u], 1.0) * (dS[u] - yS[u]);
                        }
                    }
                    z = make_double2(rn, rs);
                    if (blue) z = cmul(z, conj2(chirp(e)));
                }
                x[e] = z;
            }
        }
        if (a.mode == RING_ITER) {
            // red[] is written once per launch: no barrier needed before it
            const double2 t = block_sum2<NT>(num, den, red);
            if (tid == 0) {
                double* cp = a.io.cpart + (size_t)map * 2 * a.nq;
                cp[2 * q] = t.x;
                cp[2 * q + 1] = t.y;
            }
        }
        if (a.mode == RING_SYN) return;
    } else {
        // analysis only: the input z_j = r^N_j + i r^S_j [times conj(c_j)]
        // comes from the pixels, zero beyond n
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int j = tid + e * S;
            double2 z = make_double2(0.0, 0.0);
            if (e < J && act && j < n) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (h == 1 && eq) break;
                    const long long p = (h == 0 ? st0 : st1) + j;
                    double v;
                    switch (a.pix) {
                        case PIX_FIRST: v = ww[p] > 0.0 ? dd[p] : 0.0; break;
                        case PIX_WRES: v = ww[p] * (dd[p] - min_[p]); break;
                        case PIX_WD: v = ww[p] * dd[p]; break;
                        case PIX_CRES: {
                            const double w = ww[p];
                            const double cc = xi_ * w / fma(xi_ - alpha_, w, 1.0);
                            v = cc * (dd[p] - min_[p]);
                            break;
                        }
                        default: v = min_[p]; break;
                    }
                    if (h == 0) z.x = v;
                    else z.y = v;
                }
                if (blue) z = cmul(z, conj2(chirp(e)));
            }
            x[e] = z;
        }
        lds_barrier();  // the root table
    }

    if (blue) {
        double2 bq[E];
        if (act) load_owner<E>(bq, B, tid, S);
        fft_owner<E, MFIX>(x, buf, M, logM, tid, tw);
        if (act) filter_regs<E>(x, M, bq);
    }
    fft_owner<E, MFIX>(x, buf, M, logM, tid, tw);
    // Z_k = DFT(z)_k [divided by the chirp] to LDS; split the two real rings
    // and unfold to m
    if (act) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = tid + e * S;
            if (k < n) buf[pad(k)] = blue ? conj2(cmul(chirp(e), x[e])) : x[e];
        }
    }
    lds_barrier();
    for (int m = tid; m <= ella; m += NT) {
        const int k = m % n;
        const int kc = k == 0 ? 0 : n - k;
        unfold_store(buf[pad(k)], buf[pad(kc)], m, c, eq, spec + ((size_t)q * a.lp + m) * 2);
    }
}

// Spectrum of the chirp filter b_t = c_t (0 <= t < n), c_{M-t} (M-n < t < M),
// else 0, for every Bluestein ring pair (plan time).
template <int NT>
__global__ __launch_bounds__(NT) void k_chirp_spectrum(const int* __restrict__ qlist,
                                                       const int* __restrict__ nph,
                                                       const int* __restrict__ Mq,
                                                       const long long* __restrict__ coff,
                                                       const long long* __restrict__ boff,
                                                       const double2* __restrict__ chirp,
                                                       double2* __restrict__ bspec) {
    extern __shared__ double2 buf[];
    __shared__ double2 tw[128];
    const int q = qlist[blockIdx.x];
    const int n = nph[q], M = Mq[q];
    const int logM = 31 - __clz(M);
    const int S = M >> 4;
    const int tid = threadIdx.x;
    const double2* ch = chirp + coff[q];
    double2 x[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const int t = tid + e * S;
        double2 v = make_double2(0.0, 0.0);
        if (tid < S) {
            if (t < n) v = ch[t];
            else if (M - t < n) v = ch[M - t];
        }
        x[e] = v;
    }
    root_table<NT>(tw, M, tid);
    lds_barrier();
    fft_owner<16, 0>(x, buf, M, logM, tid, tw);
    if (tid < S) {
#pragma unroll
        for (int e = 0; e < 16; ++e) bspec[boff[q] + tid + e * S] = x[e];
    }
}

int ring_class(int M) {
    return M <= 512 ? 0 : (M == 1024 ? 1 : (M == 2048 ? 2 : (M == 4096 ? 3 : 4)));
}

// Launch shape per class: threads and FFT elements per thread (one radix-E
// butterfly per thread and pass at the largest length of the class); the FFT
// length is fixed at compile time except in the class of short rings
// (M <= 512, one wave).  Eight
// elements per thread (four passes at M = 4096) measured faster than sixteen
// (three passes): half the registers, so twice the waves per CU.
constexpr int kClassE[kRingClasses] = {8, 8, 8, 8, 8};
constexpr int kClassMaxM[kRingClasses] = {512, 1024, 2048, 4096, 8192};

template <int C>
void launch_one(dim3 grid, size_t lds, hipStream_t s, const RingArgs& a) {
    constexpr int E = kClassE[C], NT = kClassMaxM[C] / E;
    // the Bluestein class has n <= M / 2: half the elements are pixels
    constexpr int J = C == kRingClasses - 1 ? E / 2 : E;
    constexpr int MF = C == 0 ? 0 : kClassMaxM[C];
    hipLaunchKernelGGL((k_ring_fft<NT, E, J, MF>), grid, dim3(NT), lds, s, a);
}

void launch_class(int cls, dim3 grid, size_t lds, hipStream_t s, const RingArgs& a) {
    switch (cls) {
        case 0: launch_one<0>(grid, lds, s, a); break;
        case 1: launch_one<1>(grid, lds, s, a); break;
        case 2: launch_one<2>(grid, lds, s, a); break;
        case 3: launch_one<3>(grid, lds, s, a); break;
        default: launch_one<4>(grid, lds, s, a); break;
    }
}

size_t class_lds(int c) { return (size_t)(kClassMaxM[c] + kClassMaxM[c] / 16) * sizeof(double2); }

// Length n of ring pair q's rings and the FFT length M (n, or the Bluestein
// length for n not a power of two or shorter than 16, at least 16).
void ring_lengths(const dmwf_plan* p, int q, int* n_out, int* M_out, bool* blue_out) {
    const int r = q + 1;
    const int n = r < p->nside ? 4 * r : 4 * p->nside;
    const bool b = (n & (n - 1)) != 0 || n < 16;
    int M = n;
    if (b) {
        M = 16;
        while (M < 2 * n - 1) M <<= 1;
    }
    *n_out = n;
    *M_out = M;
    *blue_out = b;
}

// Appends the ring pairs of L to all in XCD-aware order: block b runs on XCD
// b mod 8, and consecutive blocks of one XCD take consecutive ring pairs.
void append_xcd_order(const std::vector<int>& L, std::vector<int>& all) {
    const int nb = (int)L.size();
    int start[9] = {0};
    for (int x = 0; x < 8; ++x) start[x + 1] = start[x] + nb / 8 + (x < nb % 8 ? 1 : 0);
    for (int b = 0; b < nb; ++b) all.push_back(L[start[b % 8] + b / 8]);
}

}  // namespace

void free_ring_tables(dmwf_plan* p) {
    void* bufs[] = {p->d_ring_M, p->d_ring_blue, p->d_ring_coff, p->d_ring_boff, p->d_chirp,
                    p->d_bspec,  p->d_ring_class};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (int i = 0; i < kRingSide; ++i) {
        if (p->ring_side[i]) (void)hipStreamDestroy(p->ring_side[i]);
        if (p->ring_join[i]) (void)hipEventDestroy(p->ring_join[i]);
    }
    if (p->ring_fork) (void)hipEventDestroy(p->ring_fork);
}

dmwf_status build_ring_tables(dmwf_plan* p) {
    const int nq = p->nq;
    std::vector<int> nph(nq), Mq(nq), blue(nq);
    std::vector<long long> coff(nq, 0), boff(nq, 0);
    long long csum = 0, bsum = 0;
    for (int q = 0; q < nq; ++q) {
        int n, M;
        bool b;
        ring_lengths(p, q, &n, &M, &b);
        nph[q] = n;
        if (M > 8192) {
            set_error("ring FFT longer than 8192 points (nside > 1024) is not implemented");
            return DMWF_ERR_UNSUPPORTED;
        }
        Mq[q] = M;
        blue[q] = b;
        if (b) {
            coff[q] = csum;
            boff[q] = bsum;
            csum += n;
            bsum += M;
        }
    }
    const long double pi = 3.141592653589793238462643383279502884L;
    // chirps e^{i pi t^2 / n} with t^2 reduced mod 2n exactly
    std::vector<double2> C(std::max<long long>(csum, 1));
    for (int q = 0; q < nq; ++q) {
        if (!blue[q]) continue;
        const long long n = nph[q];
        for (long long t = 0; t < n; ++t) {
            const long long rr = (t * t) % (2 * n);
            const long double ang = pi * rr / n;
            C[coff[q] + t] = make_double2((double)cosl(ang), (double)sinl(ang));
        }
    }
    // launch classes in XCD-aware order
    std::vector<int> lists[kRingClasses];
    for (int q = 0; q < nq; ++q) lists[ring_class(Mq[q])].push_back(q);
    std::vector<int> all;
    for (int c = 0; c < kRingClasses; ++c) {
        p->class_off[c] = (int)all.size();
        append_xcd_order(lists[c], all);
    }
    p->class_off[kRingClasses] = (int)all.size();
    for (int i = 0; i < kRingSide; ++i) {
        DMWF_HIP(hipStreamCreateWithFlags(&p->ring_side[i], hipStreamNonBlocking));
        DMWF_HIP(hipEventCreateWithFlags(&p->ring_join[i], hipEventDisableTiming));
    }
    DMWF_HIP(hipEventCreateWithFlags(&p->ring_fork, hipEventDisableTiming));

    auto up = [&](void** dst, const void* src, size_t bytes) -> bool {
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up((void**)&p->d_ring_M, Mq.data(), nq * sizeof(int)) ||
        !up((void**)&p->d_ring_blue, blue.data(), nq * sizeof(int)) ||
        !up((void**)&p->d_ring_coff, coff.data(), nq * sizeof(long long)) ||
        !up((void**)&p->d_ring_boff, boff.data(), nq * sizeof(long long)) ||
        !up((void**)&p->d_chirp, C.data(), C.size() * sizeof(double2)) ||
        !up((void**)&p->d_ring_class, all.data(), all.size() * sizeof(int)) ||
        hipMalloc((void**)&p->d_bspec, std::max<long long>(bsum, 1) * sizeof(double2)) != hipSuccess) {
        set_error("allocation or upload of ring FFT tables failed");
        return DMWF_ERR_OOM;
    }
    // filter spectra, one class at a time
    std::vector<int> bl[kRingClasses];
    for (int q = 0; q < nq; ++q)
        if (blue[q]) bl[ring_class(Mq[q])].push_back(q);
    for (int c = 0; c < kRingClasses; ++c) {
        if (bl[c].empty()) continue;
        int* dq = nullptr;
        if (!up((void**)&dq, bl[c].data(), bl[c].size() * sizeof(int))) {
            set_error("allocation of ring list failed");
            return DMWF_ERR_OOM;
        }
        const size_t lds = class_lds(c);
        hipLaunchKernelGGL((k_chirp_spectrum<512>), dim3(bl[c].size()), dim3(512), lds, nullptr, dq,
                           p->d_nph, p->d_ring_M, p->d_ring_coff, p->d_ring_boff, p->d_chirp,
                           p->d_bspec);
        DMWF_HIP(hipGetLastError());
        DMWF_HIP(hipDeviceSynchronize());
        DMWF_HIP(hipFree(dq));
    }
    return DMWF_OK;
}

dmwf_status launch_ring(dmwf_plan* p, RingMode mode, double2* spec, const RingMaps& rm,
                        const RingIO& io, hipStream_t s) {
    const int* off = p->class_off;
    const int* qlists = p->d_ring_class;
    RingArgs a;
    a.g = p->geom();
    a.nq = p->nq;
    a.lmax = p->lmax;
    a.lp = p->lp;
    a.spec = spec;
    a.spec_map = p->ws.spec_map;
    a.io = io;
    a.rm = rm;
    a.Mq = p->d_ring_M;
    a.blue = p->d_ring_blue;
    a.coff = p->d_ring_coff;
    a.boff = p->d_ring_boff;
    a.chirp = p->d_chirp;
    a.bspec = p->d_bspec;
    int cls = PROF_RING_ANA;
    a.pix = PIX_MAP;
    a.mode = RING_ANA;
    switch (mode) {
        case RING_SYN: a.mode = RING_SYN; cls = PROF_RING_SYN; break;
        case RING_ITER: a.mode = RING_ITER; cls = PROF_RING_ITER; break;
        case RING_SYN_WRES: a.mode = RING_SYN_WRES; cls = PROF_RING_ITER; break;
        case RING_ANA: break;
        case RING_ANA_FIRST: a.pix = PIX_FIRST; break;
        case RING_ANA_RESID: a.pix = PIX_WRES; break;
        case RING_ANA_WD: a.pix = PIX_WD; break;
        case RING_ANA_CRES: a.pix = PIX_CRES; break;
    }
    // The largest non-empty class runs on the caller's stream, the next ones
    // on side streams forked from it, and the caller's stream then waits for
    // every side stream.  At most kRingSide side streams: further (smaller)
    // classes follow the last one on its stream, so that the classes of a
    // launch never need more than four queues.
    ProfScope ps(p, s, cls);
    DMWF_HIP(hipEventRecord(p->ring_fork, s));
    int rank = 0;
    for (int c = kRingClasses - 1; c >= 0; --c) {
        const int nb = off[c + 1] - off[c];
        if (nb == 0) continue;
        const int side = rank == 0 ? -1 : std::min(rank - 1, kRingSide - 1);
        ++rank;
        hipStream_t sc = s;
        if (side >= 0) {
            sc = p->ring_side[side];
            DMWF_HIP(hipStreamWaitEvent(sc, p->ring_fork, 0));
        }
        a.qlist = qlists + off[c];
        launch_class(c, dim3(nb, rm.nm), class_lds(c), sc, a);
        DMWF_HIP(hipGetLastError());
        if (side >= 0) {
            DMWF_HIP(hipEventRecord(p->ring_join[side], sc));
            DMWF_HIP(hipStreamWaitEvent(s, p->ring_join[side], 0));
        }
    }
    return DMWF_OK;
}

}  // namespace dmwf
