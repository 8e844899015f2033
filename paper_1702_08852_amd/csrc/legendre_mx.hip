// Legendre stage with the contractions on the matrix cores: the reduced-
// precision forms of the transform pair (DMWF_FP32_GEMM, DMWF_BF16X3_GEMM).
//
// What is computed is the same as in legendre.hip (synthesis F_m(q) = E + O /
// E - O, analysis b_lm = sum_q lambda_lm(x_q) G^{+-}_m(q)); the recurrence
// mu_l = (A_l x) mu_{l-1} - mu_{l-2} with its starts and polar skipping stays
// FP64 in the vector ALUs.  Only the products with the data and their sums
// move to the matrix cores, which take mu_l rounded to FP32 (or split into
// two BF16 parts) and accumulate in FP32.
//
// Synthesis: a GEMM (rings x l) . (l x columns), columns = (re, im) of each
// map.  The 4x4x1 outer-product form (16 blocks of 4 lanes) takes one value
// per lane, so each lane feeds its own ring's mu_l at the current l with no
// transposition; the coefficients come through LDS.  Even and odd l - m go
// to separate accumulators (E and O).
//
// Analysis: a GEMM (l x rings) . (rings x columns), contracted over rings.
// The 16x16 forms contract over values held by different lanes, so each wave
// writes its rings' mu for a 32-l superblock into an LDS tile (16 rows of
// even and 16 of odd l - m) and reads it back in the operand layout.  The
// G^+ (even rows) and G^- (odd rows) operands stay in registers; the
// workgroup's waves (one m, different rings) reduce their FP32 tiles through
// LDS in FP64 once per superblock and write the partial sums of the chunk.
#include "legendre_dev.h"

namespace dmwf {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
// four BF16 values (bit patterns), the operand type of the *_bf16_1k forms
typedef short bf4 __attribute__((ext_vector_type(4)));

// FP32 value split into two BF16 parts: hi = v truncated to BF16, lo = the
// remainder v - hi (exact in FP32) rounded to nearest BF16, so that
// |v - hi - lo| <= 2^-17 |v| with no bias.
struct Split {
    short hi, lo;
};
__device__ __forceinline__ Split split_bf16(float v) {
    const unsigned u = __float_as_uint(v) & 0xffff0000u;
    const unsigned r = __float_as_uint(v - __uint_as_float(u));
    const unsigned rn = (r + 0x7fffu + ((r >> 16) & 1u)) >> 16;  // round half to even
    return {(short)(u >> 16), (short)rn};
}

// ---------------------------------------------------------------------------
// synthesis
// ---------------------------------------------------------------------------
// l per coefficient chunk staged in LDS
constexpr int kSynCL = 32;

// v_mfma_f32_4x4x1f32: block b = lanes 4b..4b+3; lane 4b+j, register i
// accumulates (lane 4b+i's A) x (lane 4b+j's B).  A = the lane's ring's mu_l,
// B = coefficient of column j; columns of map pair p: (map 2p re, map 2p im,
// map 2p+1 re, map 2p+1 im).  So lane 4b+j ends with column j of the four
// rings of lanes 4b..4b+3.
//
// BF16X3 form: v_mfma_f32_4x4x4bf16_1k, the same blocks with four products
// per lane summed: four consecutive l of one parity (l, l+2, l+4, l+6) in one
// instruction, three instructions (hi hi, hi lo, lo hi) per group.
template <int K, int MB, int P>
__global__ __launch_bounds__(64 * kLegWaves) void k_leg_syn_mx(SynArgs a) {
    constexpr int NP = (MB + 1) / 2;  // map pairs: four MFMA columns each
    __shared__ double2 stage[K][64][kLegWaves][2];
    // per wave, two chunks: coefficient of (l, column j, pair p) as FP32, and
    // the recurrence multipliers A_l of the chunk (read back as broadcasts, so
    // the loop waits on LDS only, never on scalar loads)
    __shared__ float coef[kLegWaves][2][kSynCL][4][NP];
    __shared__ __align__(16) double coefA[kLegWaves][2][kSynCL + 8];
    const int mg = blockIdx.y * MB;
    int ellm[MB];
    const int ell = group_ells<MB>(mg, a.nm, a.ell, a.ell_stride, a.ctrl, a.sel, ellm);
    if (ell < 0) return;
    const int w = threadIdx.x >> 6;
    const LegTile tile = leg_tile(a.nchunk);
    const int m = __builtin_amdgcn_readfirstlane(tile.group * kLegWaves + w);
    if (tile.group * kLegWaves > ell) return;  // whole workgroup above the band limit
    const bool live = m <= ell;
    const int lane = threadIdx.x & 63;
    const int jc = lane & 3;
    const int nq = a.nq;
    const int q0 = tile.chunk * (64 * K) + lane;
    const size_t mo = (size_t)m * nq;
    double x[K], p1[K], p2[K], s0[K], s1[K];
    int ls[K];
    f4 ce[K][NP], co[K][NP];
    int lo = kNever, hi = -1;
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
        for (int p = 0; p < NP; ++p) ce[t][p] = co[t][p] = f4{0.f, 0.f, 0.f, 0.f};
    }
    lo = __builtin_amdgcn_readfirstlane(wave_min(lo));
    hi = __builtin_amdgcn_readfirstlane(wave_max(hi));
    if (lo <= ell) {
        const long long base = alm_base(m, a.lmax);
        const double* A = a.A + base;
        float (*cf)[kSynCL][4][NP] = coef[w];
        double (*cA)[kSynCL + 8] = coefA[w];
        // the next chunk's coefficients in registers while the current one is
        // consumed: entry e = (map e / kSynCL, l e % kSynCL), zero beyond l_iter
        constexpr int FE = (kSynCL * MB + 63) / 64;
        double2 nv[FE];
        double na = 0.0;  // A_l of the next chunk, l = c + lane (lanes < kSynCL + 8)
        auto fetch = [&](int c) {
            // whole 16-l blocks run past l_iter (their coefficients are zero):
            // the multipliers are read up to the block end, inside the table's
            // padding
            na = lane < kSynCL + 8 && c + lane <= ell + kLegB ? A[c + lane] : 0.0;
#pragma unroll
            for (int u = 0; u < FE; ++u) {
                const int e = lane + 64 * u;
                const int mi = e / kSynCL, l = c + e % kSynCL;
                nv[u] = make_double2(0.0, 0.0);
                if (e < kSynCL * MB && l <= ell)
                    nv[u] = a.ap[(long long)min(mg + mi, a.nm - 1) * a.ap_map + base + l];
            }
        };
        auto put = [&](int b) {
            if (lane < kSynCL + 8) cA[b][lane] = na;
#pragma unroll
            for (int u = 0; u < FE; ++u) {
                const int e = lane + 64 * u;
                if (e < kSynCL * MB) {
                    const int mi = e / kSynCL, li = e % kSynCL;
                    cf[b][li][2 * (mi & 1)][mi >> 1] = (float)nv[u].x;
                    cf[b][li][2 * (mi & 1) + 1][mi >> 1] = (float)nv[u].y;
                }
            }
            if constexpr (MB & 1) {  // one map: the second map of the pair is absent
                for (int li = lane; li < kSynCL; li += 64) cf[b][li][2][NP - 1] = cf[b][li][3][NP - 1] = 0.f;
            }
        };
        fetch(lo);
        put(0);
        wave_lds_sync();
        int cur = 0;
        for (int cb = lo; cb <= ell; cb += kSynCL) {
            fetch(cb + kSynCL);
            const int cend = min(cb + kSynCL - 1, ell);
            for (int l0 = cb; l0 <= cend; l0 += kLegB) {
                if (l0 <= hi) inject<K>(l0, ls, s0, s1, p1, p2);
                if constexpr (P == DMWF_FP32_GEMM) {
                    // whole blocks: the coefficients beyond l_iter are zero, and
                    // the recurrence tables are padded past the last row
#pragma unroll
                    for (int jj = 0; jj < kLegB / 2; ++jj) {
                        const int l = l0 + 2 * jj;
                        const double2 AA = *reinterpret_cast<const double2*>(&cA[cur][l - cb]);
                        const double Ae = AA.x, Ao = AA.y;
                        float be[NP], bo[NP];
#pragma unroll
                        for (int p = 0; p < NP; ++p) {
                            be[p] = cf[cur][l - cb][jc][p];
                            bo[p] = cf[cur][l + 1 - cb][jc][p];
                        }
#pragma unroll
                        for (int t = 0; t < K; ++t) {
                            const double ue = fma(Ae * x[t], p1[t], -p2[t]);
                            const float fe = (float)ue;
#pragma unroll
                            for (int p = 0; p < NP; ++p)
                                ce[t][p] = __builtin_amdgcn_mfma_f32_4x4x1f32(fe, be[p], ce[t][p], 0, 0, 0);
                            const double uo = fma(Ao * x[t], ue, -p1[t]);
                            const float fo = (float)uo;
#pragma unroll
                            for (int p = 0; p < NP; ++p)
                                co[t][p] = __builtin_amdgcn_mfma_f32_4x4x1f32(fo, bo[p], co[t][p], 0, 0, 0);
                            p2[t] = ue;
                            p1[t] = uo;
                        }
                    }
                } else {
                    // two groups of four pairs per 16-l block; coefficients
                    // beyond l_iter are zero, so whole groups run
#pragma unroll
                    for (int g = 0; g < 2; ++g) {
                        const int lg = l0 + 8 * g;
                        if (lg > ell) break;
                        const double* Ag = &cA[cur][lg - cb];
                        bf4 bhe[NP], ble[NP], bho[NP], blo[NP];
#pragma unroll
                        for (int p = 0; p < NP; ++p) {
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const Split se = split_bf16(cf[cur][lg + 2 * u - cb][jc][p]);
                                const Split so = split_bf16(cf[cur][lg + 2 * u + 1 - cb][jc][p]);
                                bhe[p][u] = se.hi;
                                ble[p][u] = se.lo;
                                bho[p][u] = so.hi;
                                blo[p][u] = so.lo;
                            }
                        }
#pragma unroll
                        for (int t = 0; t < K; ++t) {
                            bf4 ahe, ale, aho, alo;
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const double ue = fma(Ag[2 * u] * x[t], p1[t], -p2[t]);
                                const double uo = fma(Ag[2 * u + 1] * x[t], ue, -p1[t]);
                                p2[t] = ue;
                                p1[t] = uo;
                                const Split se = split_bf16((float)ue), so = split_bf16((float)uo);
                                ahe[u] = se.hi;
                                ale[u] = se.lo;
                                aho[u] = so.hi;
                                alo[u] = so.lo;
                            }
#pragma unroll
                            for (int p = 0; p < NP; ++p) {
                                ce[t][p] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ahe, bhe[p], ce[t][p], 0, 0, 0);
                                ce[t][p] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ahe, ble[p], ce[t][p], 0, 0, 0);
                                ce[t][p] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ale, bhe[p], ce[t][p], 0, 0, 0);
                                co[t][p] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(aho, bho[p], co[t][p], 0, 0, 0);
                                co[t][p] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(aho, blo[p], co[t][p], 0, 0, 0);
                                co[t][p] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(alo, bho[p], co[t][p], 0, 0, 0);
                            }
                        }
                    }
                }
            }
            put(cur ^ 1);
            wave_lds_sync();
            cur ^= 1;
        }
    }
    // E + O (north) and E - O (south) of each map through the stage buffer,
    // then whole row segments of F, one map after the other
    constexpr int kSlots = kLegWaves * 2;
    const int m0 = tile.group * kLegWaves;
    double* stg = reinterpret_cast<double*>(&stage[0][0][0][0]);
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        if (i > 0) __syncthreads();
        const int j0 = 2 * (i & 1);
        if (jc == j0 || jc == j0 + 1) {
#pragma unroll
            for (int t = 0; t < K; ++t) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rl = (lane & ~3) + r;
                    const double e = ce[t][i >> 1][r], o = co[t][i >> 1][r];
                    const size_t at = ((size_t)(t * 64 + rl) * kLegWaves + w) * 4 + (jc & 1);
                    stg[at] = e + o;
                    stg[at + 2] = e - o;
                }
            }
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
constexpr int kAnaW = 4;      // waves per workgroup (one m, different rings)
constexpr int kAnaNM = 8;     // maps per workgroup: 16 columns (re, im)
constexpr int kTileRow = 68;  // floats per tile row: 64 rings + pad (4 r + k distinct banks)

// FP32: v_mfma_f32_16x16x4f32.  Lane i gives A[row i % 16][k i / 16] and
// B[k i / 16][col i % 16]; lane i, register r holds C[4 (i / 16) + r][i % 16].
// Rows = 16 l of one parity, k = 4 rings, columns = maps' re / im.
// BF16X3: v_mfma_f32_16x16x16bf16_1k, lane i gives A[row i % 16][k 4 (i / 16)
// + u] and B[k 4 (i / 16) + u][col i % 16], u = 0..3: 16 rings per instruction.
template <int K, int P>
__global__ __launch_bounds__(64 * kAnaW) void k_leg_ana_mx(AnaArgs a) {
    constexpr int NG = P == DMWF_FP32_GEMM ? 16 : 4;  // ring groups per 64-ring slot
    __shared__ float tile[kAnaW][2][16][kTileRow];
    __shared__ float red[kAnaW][2][16][17];
    __shared__ __align__(16) double coefA[2][32];
    __shared__ int wlohi[kAnaW][2];
    const int mg = blockIdx.y * kAnaNM;
    int ellm[kAnaNM];
    const int ell = group_ells<kAnaNM>(mg, a.nm, a.ell, a.ell_stride, a.ctrl, a.sel, ellm);
    const int nchunk = (a.nq + 64 * K * kAnaW - 1) / (64 * K * kAnaW);
    const LegTile tl = leg_tile(nchunk);
    const int m = tl.group;
    if (m > ell) return;  // the whole workgroup
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nq = a.nq;
    const int qw = tl.chunk * (64 * K * kAnaW) + w * (64 * K);  // first ring pair of the wave
    const size_t mo = (size_t)m * nq;
    double x[K], p1[K], p2[K], s0[K], s1[K];
    int ls[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const int qc = min(qw + 64 * t + lane, nq - 1);
        x[t] = a.x[qc];
        ls[t] = a.ls[mo + qc];
        s0[t] = a.s0[mo + qc];
        s1[t] = a.s1[mo + qc];
    }
    // B operands: G^+ (even rows) and G^- (odd rows) of ring qw + 64 t + ring
    // group offset, column c = lane % 16 (map c / 2, re or im); zero where the
    // ring pair does not exist, or starts beyond that map's band limit
    const int c = lane & 15, mi = c >> 1;
    int em = -1;
#pragma unroll
    for (int i = 0; i < kAnaNM; ++i)
        if (mi == i) em = ellm[i];
    const double* gb = reinterpret_cast<const double*>(
        a.spec + (long long)min(mg + mi, a.nm - 1) * a.spec_map);
    constexpr int BV = P == DMWF_FP32_GEMM ? 1 : 4;  // ring values per lane per group
    float gpv[K][NG][BV], gmv[K][NG][BV];
#pragma unroll
    for (int t = 0; t < K; ++t) {
#pragma unroll
        for (int g = 0; g < NG; ++g) {
#pragma unroll
            for (int u = 0; u < BV; ++u) {
                const int q = qw + 64 * t + (P == DMWF_FP32_GEMM ? 4 * g + (lane >> 4)
                                                                 : 16 * g + 4 * (lane >> 4) + u);
                const int qc = min(q, nq - 1);
                const double* gq = gb + ((size_t)qc * a.lp + m) * 4;
                const double gn = gq[c & 1], gs = gq[2 + (c & 1)];
                const int lr = a.ls[mo + qc];
                const bool on = q < nq && lr <= em;
                gpv[t][g][u] = on ? (float)(gn + gs) : 0.f;
                gmv[t][g][u] = on ? (float)(gn - gs) : 0.f;
            }
        }
    }
    int lo = kNever, hi = -1;
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const int lr = qw + 64 * t + lane < nq ? ls[t] : kNever;
        const int l0 = lr > ell ? kNever : lr;
        ls[t] = l0;
        const bool act = l0 != kNever;
        if (!act) s0[t] = s1[t] = 0.0;
        lo = min(lo, l0);
        if (act) hi = max(hi, l0);
        p1[t] = p2[t] = 0.0;
    }
    int slot_lo[K];
#pragma unroll
    for (int t = 0; t < K; ++t) slot_lo[t] = __builtin_amdgcn_readfirstlane(wave_min(ls[t]));
    lo = wave_min(lo);
    hi = wave_max(hi);
    if (lane == 0) {
        wlohi[w][0] = lo;
        wlohi[w][1] = hi;
    }
    __syncthreads();
    lo = wlohi[0][0];
    hi = wlohi[0][1];
#pragma unroll
    for (int i = 1; i < kAnaW; ++i) {
        lo = min(lo, wlohi[i][0]);
        hi = max(hi, wlohi[i][1]);
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    hi = __builtin_amdgcn_readfirstlane(hi);
    const long long base = alm_base(m, a.lmax);
    double2* part = a.part + tl.chunk * a.part_stride + base;
    // superblocks of 32 l counted from m; zeros below the first
    const int S0 = lo > ell ? ell + 1 : m + ((lo - m) >> 5) * 32;
    for (int e = threadIdx.x; e < kAnaNM * (S0 - m); e += 64 * kAnaW) {
        const int i = e / (S0 - m), l = m + e % (S0 - m);
        int ei = -1;
#pragma unroll
        for (int u = 0; u < kAnaNM; ++u)
            if (i == u) ei = ellm[u];
        if (ei >= 0) part[(long long)(mg + i) * a.part_map + l] = make_double2(0.0, 0.0);
    }
    if (S0 > ell) return;
    const double* A = a.A + base;
    if (threadIdx.x < 32) coefA[0][threadIdx.x] = S0 + (int)threadIdx.x <= ell ? A[S0 + threadIdx.x] : 0.0;
    __syncthreads();
    int cur = 0;
    float (*tw)[16][kTileRow] = tile[w];
    const int ar = lane & 15, ak = lane >> 4;
    for (int sb = S0; sb <= ell; sb += 32) {
        double na = 0.0;
        if (threadIdx.x < 32 && sb + 32 + (int)threadIdx.x <= ell) na = A[sb + 32 + threadIdx.x];
        f4 cE = {0.f, 0.f, 0.f, 0.f}, cO = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < K; ++t) {
            if (slot_lo[t] > sb + 31) continue;  // no ring of the slot has started
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int lb = sb + 16 * h;
                if (ls[t] == lb) {
                    p2[t] = s0[t];
                    p1[t] = s1[t];
                }
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) {
                    const double2 AA = *reinterpret_cast<const double2*>(&coefA[cur][16 * h + 2 * jj]);
                    const double ue = fma(AA.x * x[t], p1[t], -p2[t]);
                    const double uo = fma(AA.y * x[t], ue, -p1[t]);
                    p2[t] = ue;
                    p1[t] = uo;
                    tw[0][8 * h + jj][lane] = (float)ue;
                    tw[1][8 * h + jj][lane] = (float)uo;
                }
            }
            wave_lds_sync();
            if constexpr (P == DMWF_FP32_GEMM) {
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const float aE = tw[0][ar][4 * g + ak], aO = tw[1][ar][4 * g + ak];
                    cE = __builtin_amdgcn_mfma_f32_16x16x4f32(aE, gpv[t][g][0], cE, 0, 0, 0);
                    cO = __builtin_amdgcn_mfma_f32_16x16x4f32(aO, gmv[t][g][0], cO, 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    bf4 ahE, alE, ahO, alO, bhP, blP, bhM, blM;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const Split e = split_bf16(tw[0][ar][16 * g + 4 * ak + u]);
                        const Split o = split_bf16(tw[1][ar][16 * g + 4 * ak + u]);
                        const Split gp = split_bf16(gpv[t][g][u]), gm = split_bf16(gmv[t][g][u]);
                        ahE[u] = e.hi;
                        alE[u] = e.lo;
                        ahO[u] = o.hi;
                        alO[u] = o.lo;
                        bhP[u] = gp.hi;
                        blP[u] = gp.lo;
                        bhM[u] = gm.hi;
                        blM[u] = gm.lo;
                    }
                    cE = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahE, bhP, cE, 0, 0, 0);
                    cE = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahE, blP, cE, 0, 0, 0);
                    cE = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alE, bhP, cE, 0, 0, 0);
                    cO = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahO, bhM, cO, 0, 0, 0);
                    cO = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahO, blM, cO, 0, 0, 0);
                    cO = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alO, bhM, cO, 0, 0, 0);
                }
            }
            wave_lds_sync();
        }
        // the waves' tiles summed in FP64; row r of parity h is l = sb + 2 r + h
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            red[w][0][4 * ak + r][ar] = cE[r];
            red[w][1][4 * ak + r][ar] = cO[r];
        }
        if (threadIdx.x < 32) coefA[cur ^ 1][threadIdx.x] = na;
        __syncthreads();
        for (int e = threadIdx.x; e < 2 * 16 * 16; e += 64 * kAnaW) {
            const int par = e >> 8, row = (e >> 4) & 15, col = e & 15;
            double v = 0.0;
#pragma unroll
            for (int u = 0; u < kAnaW; ++u) v += (double)red[u][par][row][col];
            const int l = sb + 2 * row + par, i = col >> 1;
            int ei = -1;
#pragma unroll
            for (int u = 0; u < kAnaNM; ++u)
                if (i == u) ei = ellm[u];
            if (l <= ell && ei >= 0)
                reinterpret_cast<double*>(part + (long long)(mg + i) * a.part_map + l)[col & 1] = v;
        }
        __syncthreads();
        cur ^= 1;
    }
}

}  // namespace

dmwf_status launch_leg_syn_mx(dmwf_plan* p, const double2* ap, double2* spec, const LegMaps& lm,
                              hipStream_t s) {
    const int k = p->syn_k == 1 ? 1 : 2;
    const int nchunk = (p->nq + 64 * k - 1) / (64 * k);
    SynArgs a{p->d_x,  p->d_ls,  p->d_s0,      p->d_s1,    p->d_A,  ap,      p->ws.alm_map,
              spec,    p->ws.spec_map, lm.ell, lm.ell_stride, lm.ctrl, lm.sel, p->lmax,
              p->nq,   p->lp,    lm.nm,        nchunk};
    ProfScope ps(p, s, PROF_LEG_SYN);
    const int mb = pick_mb(8, lm.nm, 8);
    const dim3 grid(nchunk * leg_groups8(p), (lm.nm + mb - 1) / mb);
    const dim3 block(64 * kLegWaves);
#define DMWF_SYNMX(K, MB, P) hipLaunchKernelGGL((k_leg_syn_mx<K, MB, P>), grid, block, 0, s, a)
#define DMWF_SYNMX_P(K, MB)                                                   \
    do {                                                                      \
        if (p->prec == DMWF_BF16X3_GEMM) DMWF_SYNMX(K, MB, DMWF_BF16X3_GEMM); \
        else DMWF_SYNMX(K, MB, DMWF_FP32_GEMM);                               \
    } while (0)
    if (k == 1) {
        switch (mb) {
            case 8: DMWF_SYNMX_P(1, 8); break;
            case 4: DMWF_SYNMX_P(1, 4); break;
            case 2: DMWF_SYNMX_P(1, 2); break;
            default: DMWF_SYNMX_P(1, 1); break;
        }
    } else {
        switch (mb) {
            case 8: DMWF_SYNMX_P(2, 8); break;
            case 4: DMWF_SYNMX_P(2, 4); break;
            case 2: DMWF_SYNMX_P(2, 2); break;
            default: DMWF_SYNMX_P(2, 1); break;
        }
    }
#undef DMWF_SYNMX_P
#undef DMWF_SYNMX
    DMWF_HIP(hipGetLastError());
    return DMWF_OK;
}

dmwf_status launch_leg_ana_mx(dmwf_plan* p, const double2* spec, double2* part, const LegMaps& lm,
                              hipStream_t s) {
    // the workgroup's rings (64 K kAnaW) are the FP64 analysis's chunk, so the
    // partial sums keep their layout
    const int k = p->ana_k / kAnaW;
    AnaArgs a{p->d_x,   p->d_ls,        p->d_s0,  p->d_s1, p->d_A,
              spec,     p->ws.spec_map, part,     (size_t)p->nalm + kTablePad,
              p->ws.part_map, lm.ell,   lm.ell_stride, lm.ctrl, lm.sel,
              p->lmax,  p->nq,          p->lp,    lm.nm};
    ProfScope ps(p, s, PROF_LEG_ANA);
    const int groups = (p->lmax + 1 + 7) / 8 * 8;
    const dim3 grid(p->nchunk_ana * groups, (lm.nm + kAnaNM - 1) / kAnaNM);
    const dim3 block(64 * kAnaW);
    if (p->prec == DMWF_BF16X3_GEMM) {
        if (k == 1) hipLaunchKernelGGL((k_leg_ana_mx<1, DMWF_BF16X3_GEMM>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_leg_ana_mx<2, DMWF_BF16X3_GEMM>), grid, block, 0, s, a);
    } else {
        if (k == 1) hipLaunchKernelGGL((k_leg_ana_mx<1, DMWF_FP32_GEMM>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_leg_ana_mx<2, DMWF_FP32_GEMM>), grid, block, 0, s, a);
    }
    DMWF_HIP(hipGetLastError());
    return DMWF_OK;
}

}  // namespace dmwf
