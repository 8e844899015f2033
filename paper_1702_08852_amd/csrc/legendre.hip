// Legendre stage of the spherical harmonic transform pair on the HEALPix
// ring grid (the m-by-m part of the paper's basis change F / F^-1, Algorithm 2,
// moved to the sphere).
//
// For every m and every ring pair q (north ring at x = cos(theta), south ring
// at -x):
//   synthesis  F_m(north) = E + O,  F_m(south) = E - O,
//              E = sum_{l-m even} lambda_lm(x) a_lm,  O = sum_{l-m odd} lambda_lm(x) a_lm
//   analysis   b_lm = sum_q lambda_lm(x_q) [G_m(north_q) + (-1)^{l-m} G_m(south_q)]
//
// lambda_lm = g_lm mu_lm where mu obeys the two-term-cost recurrence
//   mu_l = (A_l x) mu_{l-1} - mu_{l-2},
// so one recurrence step is a multiply and an FMA.  The synthesis input is
// pre-scaled (a'_lm = g_lm a_lm) and the analysis output is post-scaled by
// g_lm, both outside these kernels.
//
// Near the poles lambda_lm underflows for l well below the turning point.  The
// plan stores, per (m, q), the first l with |lambda_lm| >= 2^-100 and the
// values mu_{l-1}, mu_l there, computed with exponent rescaling; the kernels
// start each ring at that l and treat the terms before it as zero.
//
// Mapping: one wave per (m, chunk of 64*K ring pairs, group of MB maps);
// lane = ring pair, each lane carries K ring pairs spaced 64 apart.  The
// recurrence runs in l inside a lane and is shared by the wave's MB maps
// (only the contraction FMAs are per map), so the synthesis sum over l needs
// no communication; the analysis sum over rings is reduced across lanes
// through LDS once per block of 16 l.  K and MB are per-plan tiles.
#include <algorithm>
#include <climits>

#include "legendre_dev.h"

namespace dmwf {
namespace {



// lambda_mm(x_q) for m = 0..lmax as mant * 2^expo: lambda_00 = 1/sqrt(4 pi),
// lambda_mm = -sqrt((2m+1)/(2m)) sin(theta) lambda_{m-1,m-1}.  The mantissa is
// renormalised by 2^256 whenever it drops below 2^-256.
__global__ void k_seed_mm(int lmax, int nq, const double* __restrict__ sint,
                          double* __restrict__ mant, int* __restrict__ expo) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const double st = sint[q];
    double v = 0.28209479177387814347403972578039;  // 1/sqrt(4 pi)
    int e = 0;
    mant[q] = v;
    expo[q] = 0;
    for (int m = 1; m <= lmax; ++m) {
        v *= -st * sqrt((2.0 * m + 1.0) / (2.0 * m));
        if (fabs(v) < 0x1p-256) {
            v = ldexp(v, 256);
            e -= 256;
        }
        mant[(size_t)m * nq + q] = v;
        expo[(size_t)m * nq + q] = e;
    }
}

// Walk the recurrence up from l = m until |lambda_lm| >= 2^kSkipLog2 at some
// l = ls.  The Legendre kernels start a ring at the first l of the 16-l block
// (counted from m) that holds ls, ls_a = m + 16 floor((ls - m) / 16), so that
// starts only happen at block boundaries; record ls_a and the pair (p2, p1)
// from which the recurrence's first step there yields mu_{ls_a}:
// (mu_{ls_a - 2}, mu_{ls_a - 1}), or (-mu_m, 0) when ls_a = m (A_m = 0).
// The terms between ls_a and ls are below the threshold but kept: each step
// grows |lambda| by at most about sqrt(2 lmax) there, so 15 steps back stay
// far inside the FP64 range.  kNever if ls is not reached by lmax.
__global__ void k_seed_up(int lmax, int nq, const double* __restrict__ xs,
                          const double* __restrict__ A, const double* __restrict__ g,
                          const double* __restrict__ mant, const int* __restrict__ expo,
                          int* __restrict__ ls_out, double* __restrict__ s0_out,
                          double* __restrict__ s1_out) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (q >= nq) return;
    const size_t o = (size_t)m * nq + q;
    const double x = xs[q];
    const long long base = alm_base(m, lmax);
    const double thr = ldexp(1.0, kSkipLog2);
    double cur = mant[o], prev = 0.0;
    int e = expo[o];
    // state at the start of the current block: (p2, p1) scaled by 2^se
    double sp2 = -cur, sp1 = 0.0;
    int se = e, la = m;
    bool hit = ldexp(fabs(g[base + m] * cur), e) >= thr;
    for (int l = m + 1; !hit && l <= lmax; ++l) {
        if (((l - m) % kLegB) == 0) {
            sp2 = prev;
            sp1 = cur;
            se = e;
            la = l;
        }
        const double nx = fma(A[base + l] * x, cur, -prev);
        prev = cur;
        cur = nx;
        if (fabs(cur) > 0x1p256) {
            cur = ldexp(cur, -256);
            prev = ldexp(prev, -256);
            e += 256;
        }
        hit = ldexp(fabs(g[base + l] * cur), e) >= thr;
    }
    if (!hit) {
        ls_out[o] = kNever;
        s0_out[o] = 0.0;
        s1_out[o] = 0.0;
    } else {
        ls_out[o] = la;
        s0_out[o] = ldexp(sp2, se);
        s1_out[o] = ldexp(sp1, se);
    }
}

// Suffix minimum over m of the recurrence start, stored per ring pair:
// lsmin[q][m] = min_{m' >= m} ls[m'][q].  Non-decreasing in m by construction.
__global__ void k_lsmin(int lmax, int nq, const int* __restrict__ ls, int* __restrict__ lsmin) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    int run = kNever;
    for (int m = lmax; m >= 0; --m) {
        run = min(run, ls[(size_t)m * nq + q]);
        lsmin[(size_t)q * (lmax + 1) + m] = run;
    }
}

// mhi[q] = m_bound of ring pair q at band limit ell (every m above it has
// every start beyond ell, so its lambda_lm are all skipped).
__global__ void k_mhi(int lmax, int nq, const int* __restrict__ lsmin, int ell,
                      int* __restrict__ mhi) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    mhi[q] = m_bound(lsmin + (size_t)q * (lmax + 1), ell, lmax);
}


// ---------------------------------------------------------------------------
// synthesis
// ---------------------------------------------------------------------------

// The analysis takes its coefficient row through LDS, kChunk l at a time per
// wave: each lane fetches one l of the next chunk with a vector load while
// the current chunk is consumed, and the loop reads the values back as
// wave-uniform broadcasts.  (Scalar loads issued per block stall every block
// on their latency: the scalar counter only supports waiting for all
// outstanding loads, so they cannot be issued ahead.)  The synthesis keeps
// scalar loads: its workgroups of one m-group share an XCD, so the rows are
// L2 hits, and it measured faster than LDS staging there.
constexpr int kChunk = 64;




// One even/odd pair of recurrence steps (l even offset from m, l+1 odd) for
// the K rings of a lane, contracted with the coefficients of MB maps: the
// recurrence is shared, only the FMAs of the sums are per map.
template <int K, int MB>
__device__ __forceinline__ void syn_pair(int l, bool odd_live, const double* __restrict__ A,
                                         const double2* const (&ap)[MB], const double (&x)[K],
                                         double (&p1)[K], double (&p2)[K], double (&er)[MB][K],
                                         double (&ei)[MB][K], double (&orr)[MB][K],
                                         double (&oi)[MB][K]) {
    const double Ae = A[l], Ao = A[l + 1];
    double2 ce[MB], co[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        ce[i] = ap[i][l];
        co[i] = ap[i][l + 1];
        if (!odd_live) co[i] = make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const double ue = fma(Ae * x[t], p1[t], -p2[t]);
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            er[i][t] = fma(ue, ce[i].x, er[i][t]);
            ei[i][t] = fma(ue, ce[i].y, ei[i][t]);
        }
        const double uo = fma(Ao * x[t], ue, -p1[t]);
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            orr[i][t] = fma(uo, co[i].x, orr[i][t]);
            oi[i][t] = fma(uo, co[i].y, oi[i][t]);
        }
        p2[t] = ue;
        p1[t] = uo;
    }
}



template <int K, int MB>
__global__ __launch_bounds__(64 * kLegWaves) void k_leg_syn(SynArgs a) {
    // The waves of a workgroup take consecutive m of the same ring chunk; their
    // results meet in LDS and leave as whole segments of the ring-major rows
    // of F, one map after the other.
    __shared__ double2 stage[K][64][kLegWaves][2];
    const int mg = blockIdx.y * MB;
    int ellm[MB];
    const int ell = group_ells<MB>(mg, a.nm, a.ell, a.ell_stride, a.ctrl, a.sel, ellm);
    if (ell < 0) return;
    const int w = threadIdx.x >> 6;
    // wave-uniform; readfirstlane lets the compiler use scalar loads for the
    // per-(l, m) coefficients
    const LegTile tile = leg_tile(a.nchunk);
    const int m = __builtin_amdgcn_readfirstlane(tile.group * kLegWaves + w);
    if (tile.group * kLegWaves > ell) return;  // whole workgroup above the band limit
    const bool live = m <= ell;
    const int lane = threadIdx.x & 63;
    const int nq = a.nq;
    const int q0 = tile.chunk * (64 * K) + lane;
    const size_t mo = (size_t)m * nq;
    double x[K], p1[K], p2[K], s0[K], s1[K];
    double er[MB][K], ei[MB][K], orr[MB][K], oi[MB][K];
    int ls[K];
    int lo = kNever, hi = -1;
    // all loads first, from clamped (valid) addresses, then the masks: one
    // memory round trip for the whole prologue
    const size_t mc = live ? mo : 0;
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const int qc = min(q0 + 64 * t, nq - 1);
        x[t] = a.x[qc];
        ls[t] = a.ls[mc + qc];
        s0[t] = a.s0[mc + qc];
        s1[t] = a.s1[mc + qc];
    }
#pragma unroll
    for (int t = 0; t < K; ++t) {
        int l0 = (live && q0 + 64 * t < nq) ? ls[t] : kNever;
        if (l0 > ell) l0 = kNever;
        ls[t] = l0;
        const bool act = l0 != kNever;
        if (!act) s0[t] = s1[t] = 0.0;
        lo = min(lo, l0);
        if (act) hi = max(hi, l0);
        p1[t] = p2[t] = 0.0;
#pragma unroll
        for (int i = 0; i < MB; ++i) er[i][t] = ei[i][t] = orr[i][t] = oi[i][t] = 0.0;
    }
    // uniform across the wave after the reduction; say so, so that the
    // loop bounds below live in scalar registers
    lo = __builtin_amdgcn_readfirstlane(wave_min(lo));
    hi = __builtin_amdgcn_readfirstlane(wave_max(hi));
    if (lo <= ell) {
        const long long base = alm_base(m, a.lmax);
        const double* A = a.A + base;
        // maps past the end of the batch read the last map's row; their sums
        // are not stored.  A map whose band limit is below the group's reads
        // zeros beyond it (the harmonic step stores them).
        const double2* ap[MB];
#pragma unroll
        for (int i = 0; i < MB; ++i)
            ap[i] = a.ap + (long long)min(mg + i, a.nm - 1) * a.ap_map + base;
        // every start is the first l of a 16-l block counted from m.  The
        // coefficients of PAIRS even/odd pairs are fetched together: all of a
        // block's for one map, fewer for several maps, so that they fit the
        // scalar registers (measured best: 4 pairs for 2 and 4 maps, 2 for 8)
        constexpr int PAIRS = MB >= 8 ? 2 : (MB >= 2 ? 4 : kLegB / 2);
        int l = lo;
        for (; l + kLegB - 1 <= ell; l += kLegB) {
            if (l <= hi) inject<K>(l, ls, s0, s1, p1, p2);
#pragma unroll 1
            for (int j0 = 0; j0 < kLegB / 2; j0 += PAIRS) {
#pragma unroll
                for (int j = 0; j < PAIRS; ++j)
                    syn_pair<K, MB>(l + 2 * (j0 + j), true, A, ap, x, p1, p2, er, ei, orr, oi);
            }
        }
        if (l <= ell) {
            if (l <= hi) inject<K>(l, ls, s0, s1, p1, p2);
            for (; l <= ell; l += 2)
                syn_pair<K, MB>(l, l + 1 <= ell, A, ap, x, p1, p2, er, ei, orr, oi);
        }
    }
    constexpr int kSlots = kLegWaves * 2;
    const int m0 = tile.group * kLegWaves;
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        if (i > 0) __syncthreads();  // the previous map's rows have left the stage
#pragma unroll
        for (int t = 0; t < K; ++t) {
            stage[t][lane][w][0] = make_double2(er[i][t] + orr[i][t], ei[i][t] + oi[i][t]);
            stage[t][lane][w][1] = make_double2(er[i][t] - orr[i][t], ei[i][t] - oi[i][t]);
        }
        __syncthreads();
        const int ei_ = ellm[i];
        double2* spec = a.spec + (long long)(mg + i) * a.spec_map;
        for (int idx = threadIdx.x; idx < K * 64 * kSlots; idx += 64 * kLegWaves) {
            const int slot = idx % kSlots, rr = idx / kSlots;
            const int q = tile.chunk * (64 * K) + rr;
            const int mm = m0 + (slot >> 1);
            if (q < nq && mm <= ei_)
                spec[((size_t)q * a.lp + mm) * 2 + (slot & 1)] = stage[rr >> 6][rr & 63][slot >> 1][slot & 1];
        }
    }
}

// ---------------------------------------------------------------------------
// analysis
// ---------------------------------------------------------------------------

// Cross-lane sums through the lane-swap instructions (no LDS).  xsum32(a, b):
// lanes 0..31 return a_i + a_{i+32}, lanes 32..63 return b_{i-32} + b_i.
__device__ __forceinline__ double xsum32(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false,
                                                     false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false,
                                                     false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// Sums of a over the four lanes i, i ^ 16, i ^ 32, i ^ 48 (lanes 0..15 and
// 32..47) and of b likewise (lanes 16..31 and 48..63), one value per lane: the
// row swap pairs a's rows with b's, so both sums share every instruction.
__device__ __forceinline__ double xsum_rows2(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false,
                                                     false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false,
                                                     false);
    const double c = __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
    return xsum32(c, c);
}

// Row of the analysis reduction buffer: 64 lanes' values with one pad slot
// after lane 31, so that the upper half starts 4 banks after the lower and
// rows are 8 banks apart (66 double2 = 264 dwords).
constexpr int kRedRow = 66;

// Eight even/odd pairs (16 l) of the lane's K rings for MB maps, A_l staged
// at CA[i0..].  Pair j of map i leaves through red[j][i][.]: lanes 0..31 hold
// the even l0 + 2j summed over lanes i and i+32, lanes 32..63 the odd
// l0 + 2j + 1.
// Slots t < T0 hold rings that have not started yet (all their starts lie
// beyond this block): their terms are zero and their state stays (0, 0), so
// they are skipped.
template <int K, int MB, int T0>
__device__ __forceinline__ void ana_block(const double* CA, int i0,
                                          const double (&x)[K], double (&p1)[K], double (&p2)[K],
                                          const double (&gpr)[MB][K], const double (&gpi)[MB][K],
                                          const double (&gmr)[MB][K], const double (&gmi)[MB][K],
                                          double2 (*red)[MB][kRedRow], int lane) {
#pragma unroll
    for (int j = 0; j < kLegB / 2; ++j) {
        const double2 AA = *reinterpret_cast<const double2*>(CA + i0 + 2 * j);
        const double Ae = AA.x, Ao = AA.y;
        double er[MB], ei[MB], orr[MB], oi[MB];
#pragma unroll
        for (int i = 0; i < MB; ++i) er[i] = ei[i] = orr[i] = oi[i] = 0.0;
#pragma unroll
        for (int t = T0; t < K; ++t) {
            const double ue = fma(Ae * x[t], p1[t], -p2[t]);
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                er[i] = fma(ue, gpr[i][t], er[i]);
                ei[i] = fma(ue, gpi[i][t], ei[i]);
            }
            const double uo = fma(Ao * x[t], ue, -p1[t]);
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                orr[i] = fma(uo, gmr[i][t], orr[i]);
                oi[i] = fma(uo, gmi[i][t], oi[i]);
            }
            p2[t] = ue;
            p1[t] = uo;
        }
#pragma unroll
        for (int i = 0; i < MB; ++i)
            red[j][i][lane + (lane >> 5)] = make_double2(xsum32(er[i], orr[i]), xsum32(ei[i], oi[i]));
    }
}

// ana_block over the slots t0..K-1, t0 wave-uniform.
template <int K, int MB, int T = 0>
__device__ __forceinline__ void ana_block_from(int t0, const double* CA, int i0,
                                               const double (&x)[K], double (&p1)[K],
                                               double (&p2)[K], const double (&gpr)[MB][K],
                                               const double (&gpi)[MB][K],
                                               const double (&gmr)[MB][K],
                                               const double (&gmi)[MB][K],
                                               double2 (*red)[MB][kRedRow], int lane) {
    if constexpr (T < K - 1) {
        if (t0 > T) {
            ana_block_from<K, MB, T + 1>(t0, CA, i0, x, p1, p2, gpr, gpi, gmr, gmi, red, lane);
            return;
        }
    }
    ana_block<K, MB, T>(CA, i0, x, p1, p2, gpr, gpi, gmr, gmi, red, lane);
}

template <int K, int MB>
__global__ __launch_bounds__(64 * kLegWaves) void k_leg_ana(AnaArgs a) {
    __shared__ double2 red_all[kLegWaves][kLegB / 2][MB][kRedRow];
    __shared__ double coef[kLegWaves][2][kChunk];  // per wave: two chunks of A
    const int mg = blockIdx.y * MB;
    int ellm[MB];
    const int ell = group_ells<MB>(mg, a.nm, a.ell, a.ell_stride, a.ctrl, a.sel, ellm);
    const int w = threadIdx.x >> 6;
    const LegTile tile = leg_tile((a.nq + 64 * K - 1) / (64 * K));
    const int m = __builtin_amdgcn_readfirstlane(tile.group * kLegWaves + w);
    if (m > ell) return;
    double2 (*red)[MB][kRedRow] = red_all[w];
    const int lane = threadIdx.x & 63;
    const int nq = a.nq;
    const int q0 = tile.chunk * (64 * K) + lane;
    const size_t mo = (size_t)m * nq;
    double x[K], p1[K], p2[K], s0[K], s1[K];
    double gpr[MB][K], gpi[MB][K], gmr[MB][K], gmi[MB][K];
    int ls[K];
    int lo = kNever, hi = -1;
    // all loads first, from clamped (valid) addresses, then the masks: one
    // memory round trip for the whole prologue.  G of a map is used only for
    // rings whose start lies within that map's band limit: the ring stage
    // wrote it there, and may not have elsewhere.
    double2 gn[MB][K], gs[MB][K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const int qc = min(q0 + 64 * t, nq - 1);
        x[t] = a.x[qc];
        ls[t] = a.ls[mo + qc];
        s0[t] = a.s0[mo + qc];
        s1[t] = a.s1[mo + qc];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            const double2* g = a.spec + (long long)min(mg + i, a.nm - 1) * a.spec_map +
                               ((size_t)qc * a.lp + m) * 2;
            gn[i][t] = g[0];
            gs[i][t] = g[1];
        }
    }
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const int lr = q0 + 64 * t < nq ? ls[t] : kNever;
        const int l0 = lr > ell ? kNever : lr;
        ls[t] = l0;
        const bool act = l0 != kNever;
        if (!act) s0[t] = s1[t] = 0.0;
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            if (!(act && lr <= ellm[i])) gn[i][t] = gs[i][t] = make_double2(0.0, 0.0);
            gpr[i][t] = gn[i][t].x + gs[i][t].x;
            gpi[i][t] = gn[i][t].y + gs[i][t].y;
            gmr[i][t] = gn[i][t].x - gs[i][t].x;
            gmi[i][t] = gn[i][t].y - gs[i][t].y;
        }
        lo = min(lo, l0);
        if (act) hi = max(hi, l0);
        p1[t] = p2[t] = 0.0;
    }
    // uniform across the wave after the reduction; say so, so that the
    // loop bounds below live in scalar registers
    lo = __builtin_amdgcn_readfirstlane(wave_min(lo));
    hi = __builtin_amdgcn_readfirstlane(wave_max(hi));
    int slot_lo[K];
#pragma unroll
    for (int t = 0; t < K; ++t) slot_lo[t] = __builtin_amdgcn_readfirstlane(wave_min(ls[t]));
    const long long base = alm_base(m, a.lmax);
    double2* out[MB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
        out[i] = a.part + (long long)(mg + i) * a.part_map + tile.chunk * a.part_stride + base;
    if (lo > ell) {
#pragma unroll
        for (int i = 0; i < MB; ++i)
            if (ellm[i] >= 0)
                for (int l = m + lane; l <= ell; l += 64) out[i][l] = make_double2(0.0, 0.0);
        return;
    }
    const double* A = a.A + base;
    // every start is the first l of a 16-l block counted from m
    const int L0 = lo;
#pragma unroll
    for (int i = 0; i < MB; ++i)
        if (ellm[i] >= 0)
            for (int l = m + lane; l < L0; l += 64) out[i][l] = make_double2(0.0, 0.0);
    // lane sums eight of the 32 half-sums of l0 + rb: row rb >> 1, half rb & 1,
    // part rp = lane >> 4; the four parts then combine across lanes 16 apart
    const int rb = lane & 15, rp = lane >> 4;
    const int rcol = (rb & 1) * 33 + rp * 8;
    double (*cf)[kChunk] = coef[w];
    // A_l for l = c + lane; ana_block runs whole blocks, so rows are read up
    // to l_iter + 16 (inside the table padding) and zero beyond
    auto fetch = [&](int c) {
        const int l = c + lane;
        return l <= ell + kLegB ? A[l] : 0.0;
    };
    double na = fetch(L0);
    cf[0][lane] = na;
    wave_lds_sync();
    int cur = 0;
    for (int cb = L0; cb <= ell; cb += kChunk) {
        na = fetch(cb + kChunk);  // next chunk, in flight meanwhile
        const int cend = min(cb + kChunk - 1, ell);
        for (int l0 = cb; l0 <= cend; l0 += kLegB) {
            if (l0 <= hi) inject<K>(l0, ls, s0, s1, p1, p2);
            // first slot with a started ring (uniform); the slots are ordered
            // from the pole towards the equator, where rings start earliest
            int t0 = K;
#pragma unroll
            for (int t = K - 1; t >= 0; --t)
                if (slot_lo[t] <= l0) t0 = t;
            ana_block_from<K, MB>(t0, cf[cur], l0 - cb, x, p1, p2, gpr, gpi, gmr, gmi, red, lane);
            wave_lds_sync();
            double sr[MB], si[MB];
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                double2 v = red[rb >> 1][i][rcol];
                sr[i] = v.x;
                si[i] = v.y;
#pragma unroll
                for (int u = 1; u < 8; ++u) {
                    v = red[rb >> 1][i][rcol + u];
                    sr[i] += v.x;
                    si[i] += v.y;
                }
            }
            wave_lds_sync();
            // lanes 0..15 end with the real part of row rb, lanes 16..31 with
            // the imaginary part, each stored as one double
#pragma unroll
            for (int i = 0; i < MB; ++i) {
                const double v = xsum_rows2(sr[i], si[i]);
                if (rp < 2 && l0 + rb <= ell && ellm[i] >= 0)
                    reinterpret_cast<double*>(out[i] + l0 + rb)[rp] = v;
            }
        }
        cf[cur ^ 1][lane] = na;
        wave_lds_sync();
        cur ^= 1;
    }
}

}  // namespace

dmwf_status launch_seeds(dmwf_plan* p, hipStream_t s) {
    const size_t cnt = (size_t)(p->lmax + 1) * p->nq;
    double* mant = nullptr;
    int* expo = nullptr;
    DMWF_HIP(hipMalloc(&mant, cnt * sizeof(double)));
    DMWF_HIP(hipMalloc(&expo, cnt * sizeof(int)));
    {
        ProfScope ps(p, s, PROF_SEED);
        hipLaunchKernelGGL(k_seed_mm, dim3((p->nq + 63) / 64), dim3(64), 0, s, p->lmax, p->nq,
                           p->d_sint, mant, expo);
        hipLaunchKernelGGL(k_seed_up, dim3((p->nq + 63) / 64, p->lmax + 1), dim3(64), 0, s,
                           p->lmax, p->nq, p->d_x, p->d_A, p->d_g, mant, expo, p->d_ls, p->d_s0,
                           p->d_s1);
    }
    hipLaunchKernelGGL(k_lsmin, dim3((p->nq + 63) / 64), dim3(64), 0, s, p->lmax, p->nq, p->d_ls,
                       p->d_lsmin);
    hipLaunchKernelGGL(k_mhi, dim3((p->nq + 63) / 64), dim3(64), 0, s, p->lmax, p->nq, p->d_lsmin,
                       p->lmax, p->d_mhi_full);
    DMWF_HIP(hipGetLastError());
    DMWF_HIP(hipStreamSynchronize(s));
    DMWF_HIP(hipFree(mant));
    DMWF_HIP(hipFree(expo));
    return DMWF_OK;
}

int pick_mb(int want, int nm, int cap) {
    int mb = 1;
    while (mb * 2 <= want && mb * 2 <= nm && mb * 2 <= cap) mb *= 2;
    return mb;
}

int leg_groups8(const dmwf_plan* p) {
    // m-groups of kLegWaves consecutive m, rounded up to whole XCD rounds
    return ((p->lmax + kLegWaves) / kLegWaves + 7) / 8 * 8;
}

dmwf_status launch_leg_syn(dmwf_plan* p, const double2* ap, double2* spec, const LegMaps& lm,
                           int mb_want, hipStream_t s) {
    const int k = p->syn_k == 1 ? 1 : 2;
    const int nchunk = (p->nq + 64 * k - 1) / (64 * k);
    SynArgs a{p->d_x,       p->d_ls,    p->d_s0,        p->d_s1,  p->d_A,
              ap,           p->ws.alm_map, spec,        p->ws.spec_map,
              lm.ell,       lm.ell_stride, lm.ctrl,     lm.sel,   p->lmax,
              p->nq,        p->lp,      lm.nm,          nchunk};
    ProfScope ps(p, s, PROF_LEG_SYN);
    const int mb = pick_mb(mb_want, lm.nm, 8);
    const dim3 grid(nchunk * leg_groups8(p), (lm.nm + mb - 1) / mb);
    const dim3 block(64 * kLegWaves);
#define DMWF_SYN(K, MB) hipLaunchKernelGGL((k_leg_syn<K, MB>), grid, block, 0, s, a)
    if (k == 1) {
        switch (mb) {
            case 8: DMWF_SYN(1, 8); break;
            case 4: DMWF_SYN(1, 4); break;
            case 2: DMWF_SYN(1, 2); break;
            default: DMWF_SYN(1, 1); break;
        }
    } else {
        switch (mb) {
            case 8: DMWF_SYN(2, 8); break;
            case 4: DMWF_SYN(2, 4); break;
            case 2: DMWF_SYN(2, 2); break;
            default: DMWF_SYN(2, 1); break;
        }
    }
#undef DMWF_SYN
    DMWF_HIP(hipGetLastError());
    return DMWF_OK;
}

dmwf_status launch_leg_ana(dmwf_plan* p, const double2* spec, double2* part, const LegMaps& lm,
                           int mb_want, hipStream_t s) {
    AnaArgs a{p->d_x,   p->d_ls,        p->d_s0,  p->d_s1, p->d_A,
              spec,     p->ws.spec_map, part,     (size_t)p->nalm + kTablePad,
              p->ws.part_map, lm.ell,   lm.ell_stride, lm.ctrl, lm.sel,
              p->lmax,  p->nq,          p->lp,    lm.nm};
    ProfScope ps(p, s, PROF_LEG_ANA);
    const int mb = pick_mb(mb_want, lm.nm, 2);
    const dim3 grid(p->nchunk_ana * leg_groups8(p), (lm.nm + mb - 1) / mb);
    const dim3 block(64 * kLegWaves);
    if (p->ana_k == 4) {
        if (mb == 2) hipLaunchKernelGGL((k_leg_ana<4, 2>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_leg_ana<4, 1>), grid, block, 0, s, a);
    } else {
        if (mb == 2) hipLaunchKernelGGL((k_leg_ana<8, 2>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_leg_ana<8, 1>), grid, block, 0, s, a);
    }
    DMWF_HIP(hipGetLastError());
    return DMWF_OK;
}

}  // namespace dmwf

extern "C" dmwf_status dmwf_legendre_work(dmwf_plan* p, int ell, long long* out) {
    using namespace dmwf;
    if (!p || !out || ell < 0 || ell > p->lmax) {
        set_error("legendre_work: NULL argument or ell outside 0..lmax");
        return DMWF_ERR_INVALID_ARG;
    }
    const int nq = p->nq, L = p->lmax;
    if (p->h_ls.empty()) {
        p->h_ls.resize((size_t)(L + 1) * nq);
        DMWF_HIP(hipMemcpy(p->h_ls.data(), p->d_ls, p->h_ls.size() * sizeof(int),
                           hipMemcpyDeviceToHost));
    }
    const int* ls = p->h_ls.data();
    long long full = (long long)nq * (ell + 1) * (ell + 2) / 2, useful = 0, syn = 0, ana = 0;
    const int ks = p->syn_k == 1 ? 1 : 2, ka = p->ana_k;
    for (int m = 0; m <= ell; ++m) {
        const int* row = ls + (size_t)m * nq;
        for (int q = 0; q < nq; ++q)
            if (row[q] <= ell) useful += ell - row[q] + 1;
        // synthesis: each wave runs its K x 64 ring pairs from the smallest start
        // in whole 16-l blocks while they fit, then in pairs
        for (int q0 = 0; q0 < nq; q0 += 64 * ks) {
            int lo = kNever;
            for (int q = q0; q < std::min(nq, q0 + 64 * ks); ++q) lo = std::min(lo, row[q]);
            if (lo > ell) continue;
            const int span = ell - lo + 1;
            const int steps = span / kLegB * kLegB + (span % kLegB + 1) / 2 * 2;
            syn += 64LL * ks * steps;
        }
        // analysis: per 16-l block, the slots from the first one holding a
        // started ring (slot t = ring pairs q0 + 64 t + lane)
        for (int q0 = 0; q0 < nq; q0 += 64 * ka) {
            int slo[16];
            int lo = kNever;
            for (int t = 0; t < ka; ++t) {
                slo[t] = kNever;
                for (int j = 0; j < 64; ++j) {
                    const int q = q0 + 64 * t + j;
                    if (q < nq && row[q] <= ell) slo[t] = std::min(slo[t], row[q]);
                }
                lo = std::min(lo, slo[t]);
            }
            if (lo > ell) continue;
            for (int l0 = lo; l0 <= ell; l0 += kLegB) {
                int t0 = ka;
                for (int t = ka - 1; t >= 0; --t)
                    if (slo[t] <= l0) t0 = t;
                ana += 64LL * kLegB * (ka - t0);
            }
        }
    }
    out[0] = full;
    out[1] = useful;
    out[2] = syn;
    out[3] = ana;
    return DMWF_OK;
}
