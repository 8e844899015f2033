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
// The length-n DFTs run in LDS: an in-place radix-2 decimation-in-time FFT on
// bit-reversed input with up to three stages fused per pass in registers.
// Ring lengths that are not powers of two (polar rings, n = 4i) use
// Bluestein's chirp-z identity jk = (j^2 + k^2 - (k-j)^2)/2, which turns the
// DFT into a cyclic convolution of length M >= 2n-1 (a power of two) with the
// chirp c_t = e^{i pi t^2/n}; the spectrum of the chirp filter is a plan table.
//
// In RING_ITER mode the workgroup also performs the pixel step of the paper's
// Algorithm 2 in residual form: it reads s_prev, writes s, accumulates the
// Cauchy sums sum (s - s_prev)^2 and sum s^2, forms r = c (d - s) with
// c = xi w / (1 + (xi - alpha) w) (messenger step with N_bar = N - alpha)
// and analyses r into G, overwriting F in place.
//
// Workgroups are launched in four classes by FFT length (LDS size) so that
// small rings do not reserve the LDS of the largest; within a class the ring
// pairs are ordered so that consecutive pairs land on the same XCD and share
// its L2 for the neighbouring F/G lines.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace dmwf {
namespace {

enum PixSource { PIX_MAP = 0, PIX_FIRST = 1, PIX_WRES = 2, PIX_WD = 3, PIX_CRES = 4 };

struct RingArgs {
    RingGeom g;
    int nq, lmax;
    const int* ell_syn;
    const int* ell_ana;
    double2* spec;
    int mode;
    int pix;
    RingIO io;
    const int* qlist;
    const int* Mq;
    const int* blue;
    const long long* coff;
    const long long* boff;
    const double2* W;
    int wlog;
    const double2* chirp;
    const double2* bspec;
};

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }

__device__ __forceinline__ int brev(int k, int logM) {
    return logM ? (int)(__brev((unsigned)k) >> (32 - logM)) : 0;
}

// R fused radix-2 DIT stages starting at sub-transform length 2^s.
template <int R>
__device__ __forceinline__ void fft_pass(double2* __restrict__ buf, int M, int s,
                                         const double2* __restrict__ W, int wlog, int tid, int nt) {
    constexpr int P = 1 << R;
    const int L = 1 << s;
    const int nb = M >> R;
    for (int b = tid; b < nb; b += nt) {
        const int j = b & (L - 1);
        const int base = ((b >> s) << (s + R)) + j;
        double2 v[P];
#pragma unroll
        for (int t = 0; t < P; ++t) v[t] = buf[base + t * L];
#pragma unroll
        for (int st = 0; st < R; ++st) {
            const int half = 1 << st;
#pragma unroll
            for (int t = 0; t < P; ++t) {
                if (t & half) continue;
                const int jj = j + (t & (half - 1)) * L;
                const double2 tw = W[jj << (wlog - s - st - 1)];
                const double2 x2 = cmul(tw, v[t + half]);
                v[t + half] = csub(v[t], x2);
                v[t] = cadd(v[t], x2);
            }
        }
#pragma unroll
        for (int t = 0; t < P; ++t) buf[base + t * L] = v[t];
    }
}

// Forward DFT in place: bit-reversed input, natural-order output.
__device__ void fft(double2* buf, int M, int logM, const double2* W, int wlog, int tid, int nt) {
    int s = 0;
    while (s < logM) {
        const int r = min(3, logM - s);
        if (r == 3) fft_pass<3>(buf, M, s, W, wlog, tid, nt);
        else if (r == 2) fft_pass<2>(buf, M, s, W, wlog, tid, nt);
        else fft_pass<1>(buf, M, s, W, wlog, tid, nt);
        __syncthreads();
        s += r;
    }
}

// buf holds a (bit-reversed, zero-padded).  Leaves buf_k = conj(conv_k) in
// natural order, conv = a (*) b cyclic of length M, so the length-n forward
// DFT of the chirped input is X_k = conj(c_k buf_k).
__device__ void bluestein(double2* buf, int M, int logM, const double2* __restrict__ B,
                          const double2* W, int wlog, int tid, int nt) {
    fft(buf, M, logM, W, wlog, tid, nt);
    const double inv = 1.0 / M;
    for (int k = tid; k < M; k += nt) {
        const int kr = brev(k, logM);
        if (k <= kr) {
            const double2 ak = cmul(buf[k], B[k]);
            const double2 akr = cmul(buf[kr], B[kr]);
            buf[kr] = make_double2(ak.x * inv, -ak.y * inv);
            buf[k] = make_double2(akr.x * inv, -akr.y * inv);
        }
    }
    __syncthreads();
    fft(buf, M, logM, W, wlog, tid, nt);
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* scratch) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) t += scratch[i];
    }
    return t;
}

template <int NT, int J>
__global__ __launch_bounds__(NT) void k_ring_fft(RingArgs a) {
    extern __shared__ double2 buf[];
    __shared__ double red[NT / 64];
    const int q = a.qlist[blockIdx.x];
    const int n = a.g.nph[q];
    const int M = a.Mq[q];
    const int logM = 31 - __clz(M);
    const bool blue = a.blue[q] != 0;
    const double2* ch = a.chirp + a.coff[q];
    const double2* B = a.bspec + a.boff[q];
    const double c = a.g.phi0pi[q];
    const bool eq = (q == a.nq - 1);
    const long long st0 = a.g.start_n[q], st1 = a.g.start_s[q];
    const int ell = *a.ell_syn;
    const int ella = *a.ell_ana;
    const int tid = threadIdx.x;
    const size_t nq = a.nq;
    double rn[J], rs[J];

    const bool syn = (a.mode == RING_SYN || a.mode == RING_ITER || a.mode == RING_SYN_WRES);
    if (syn) {
        // x_k = conj(Z_k) [times conj(c_k)], Z_k = H^N_k + i H^S_k, at bit-reversed slots
        for (int k = tid; k < M; k += NT) {
            double2 v = make_double2(0.0, 0.0);
            if (k < n) {
                double2 hn = make_double2(0.0, 0.0), hs = make_double2(0.0, 0.0);
                for (int pass = 0; pass < 2; ++pass) {
                    // pass 0: m = k + t n (m >= 0); pass 1: m = -k mod n + t n, conjugated (-m)
                    int m = pass == 0 ? k : (k == 0 ? n : n - k);
                    for (; m <= ell; m += n) {
                        double sn, cs;
                        sincospi(m * c, &sn, &cs);
                        const double2 ph = make_double2(cs, sn);
                        double2 fn = a.spec[((size_t)m * nq + q) * 2 + 0];
                        double2 fs = a.spec[((size_t)m * nq + q) * 2 + 1];
                        if (m == 0) {
                            fn.y = 0.0;
                            fs.y = 0.0;
                        }
                        double2 en = cmul(fn, ph), es = cmul(fs, ph);
                        if (pass == 1) {
                            en = conj2(en);
                            es = conj2(es);
                        }
                        hn = cadd(hn, en);
                        hs = cadd(hs, es);
                    }
                }
                if (eq) hs = make_double2(0.0, 0.0);
                // conj(Z) = conj(hn + i hs)
                v = make_double2(hn.x - hs.y, -(hn.y + hs.x));
                if (blue) v = cmul(v, conj2(ch[k]));
            }
            buf[brev(k, logM)] = v;
        }
        __syncthreads();
        if (blue) bluestein(buf, M, logM, B, a.W, a.wlog, tid, NT);
        else fft(buf, M, logM, a.W, a.wlog, tid, NT);
        // y_j = IDFT(Z)_j: blue: c_j buf_j; else conj(buf_j).  s^N = Re y, s^S = Im y.
        double num = 0.0, den = 0.0;
#pragma unroll
        for (int t = 0; t < J; ++t) {
            const int j = tid + t * NT;
            rn[t] = 0.0;
            rs[t] = 0.0;
            if (j >= n) continue;
            const double2 y = blue ? cmul(ch[j], buf[j]) : conj2(buf[j]);
            for (int h = 0; h < (eq ? 1 : 2); ++h) {
                const double s = h == 0 ? y.x : y.y;
                const long long p = (h == 0 ? st0 : st1) + j;
                double r = 0.0;
                if (a.mode == RING_SYN) {
                    a.io.map_out[p] = s;
                } else if (a.mode == RING_SYN_WRES) {
                    r = a.io.w[p] * (a.io.d[p] - s);
                } else {
                    const double sp = a.io.first ? 0.0 : a.io.s_map[p];
                    const double ds = s - sp;
                    num = fma(ds, ds, num);
                    den = fma(s, s, den);
                    a.io.s_map[p] = s;
                    const double w = a.io.w[p];
                    const double cc = a.io.xi * w / fma(a.io.xi - a.io.alpha, w, 1.0);
                    r = cc * (a.io.d[p] - s);
                }
                if (h == 0) rn[t] = r;
                else rs[t] = r;
            }
        }
        if (a.mode == RING_ITER) {
            const double tn = block_sum<NT>(num, red);
            const double td = block_sum<NT>(den, red);
            if (tid == 0) {
                a.io.cpart[2 * q] = tn;
                a.io.cpart[2 * q + 1] = td;
            }
        }
        if (a.mode == RING_SYN) return;
    } else {
#pragma unroll
        for (int t = 0; t < J; ++t) {
            const int j = tid + t * NT;
            rn[t] = 0.0;
            rs[t] = 0.0;
            if (j >= n) continue;
            for (int h = 0; h < (eq ? 1 : 2); ++h) {
                const long long p = (h == 0 ? st0 : st1) + j;
                double v;
                switch (a.pix) {
                    case PIX_FIRST: v = a.io.w[p] > 0.0 ? a.io.d[p] : 0.0; break;
                    case PIX_WRES: v = a.io.w[p] * (a.io.d[p] - a.io.map_in[p]); break;
                    case PIX_WD: v = a.io.w[p] * a.io.d[p]; break;
                    case PIX_CRES: {
                        const double w = a.io.w[p];
                        const double cc = a.io.xi * w / fma(a.io.xi - a.io.alpha, w, 1.0);
                        v = cc * (a.io.d[p] - a.io.map_in[p]);
                        break;
                    }
                    default: v = a.io.map_in[p]; break;
                }
                if (h == 0) rn[t] = v;
                else rs[t] = v;
            }
        }
    }
    __syncthreads();
    // analysis input z_j = r^N_j + i r^S_j [times conj(c_j)] at bit-reversed slots
#pragma unroll
    for (int t = 0; t < J; ++t) {
        const int j = tid + t * NT;
        if (j < n) {
            double2 z = make_double2(rn[t], rs[t]);
            if (blue) z = cmul(z, conj2(ch[j]));
            buf[brev(j, logM)] = z;
        }
    }
    for (int j = n + tid; j < M; j += NT) buf[brev(j, logM)] = make_double2(0.0, 0.0);
    __syncthreads();
    if (blue) bluestein(buf, M, logM, B, a.W, a.wlog, tid, NT);
    else fft(buf, M, logM, a.W, a.wlog, tid, NT);
    // Z_k = DFT(z)_k; split the two real rings and unfold to m
    for (int m = tid; m <= ella; m += NT) {
        const int k = m % n;
        const int kc = k == 0 ? 0 : n - k;
        double2 zk = buf[k], zc = buf[kc];
        if (blue) {
            zk = conj2(cmul(ch[k], zk));
            zc = conj2(cmul(ch[kc], zc));
        }
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
        a.spec[((size_t)m * nq + q) * 2 + 0] = gN;
        a.spec[((size_t)m * nq + q) * 2 + 1] = gS;
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
                                                       double2* __restrict__ bspec,
                                                       const double2* __restrict__ W, int wlog) {
    extern __shared__ double2 buf[];
    const int q = qlist[blockIdx.x];
    const int n = nph[q], M = Mq[q];
    const int logM = 31 - __clz(M);
    const double2* ch = chirp + coff[q];
    for (int t = threadIdx.x; t < M; t += NT) {
        double2 v = make_double2(0.0, 0.0);
        if (t < n) v = ch[t];
        else if (M - t < n) v = ch[M - t];
        buf[brev(t, logM)] = v;
    }
    __syncthreads();
    fft(buf, M, logM, W, wlog, threadIdx.x, NT);
    for (int k = threadIdx.x; k < M; k += NT) bspec[boff[q] + k] = buf[k];
}

int ring_class(int M) { return M <= 1024 ? 0 : (M == 2048 ? 1 : (M == 4096 ? 2 : 3)); }

void launch_class(int cls, dim3 grid, size_t lds, hipStream_t s, const RingArgs& a) {
    switch (cls) {
        case 0: hipLaunchKernelGGL((k_ring_fft<256, 4>), grid, dim3(256), lds, s, a); break;
        case 1: hipLaunchKernelGGL((k_ring_fft<256, 8>), grid, dim3(256), lds, s, a); break;
        case 2: hipLaunchKernelGGL((k_ring_fft<512, 8>), grid, dim3(512), lds, s, a); break;
        default: hipLaunchKernelGGL((k_ring_fft<512, 8>), grid, dim3(512), lds, s, a); break;
    }
}

const int kClassMaxM[kRingClasses] = {1024, 2048, 4096, 8192};

}  // namespace

void free_ring_tables(dmwf_plan* p) {
    void* bufs[] = {p->d_ring_M, p->d_ring_blue, p->d_ring_coff, p->d_ring_boff, p->d_twiddle,
                    p->d_chirp,  p->d_bspec,     p->d_ring_class};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
}

dmwf_status build_ring_tables(dmwf_plan* p) {
    const int nq = p->nq;
    std::vector<int> nph(nq), Mq(nq), blue(nq);
    std::vector<long long> coff(nq, 0), boff(nq, 0);
    const int N = p->nside;
    long long csum = 0, bsum = 0;
    int Mmax = 4;
    for (int q = 0; q < nq; ++q) {
        const int r = q + 1;
        const int n = r < N ? 4 * r : 4 * N;
        nph[q] = n;
        const bool b = (n & (n - 1)) != 0;
        int M = n;
        if (b) {
            M = 1;
            while (M < 2 * n - 1) M <<= 1;
        }
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
        Mmax = std::max(Mmax, M);
    }
    // twiddles e^{-2 pi i t / Mmax}
    int wlog = 0;
    while ((1 << wlog) < Mmax) ++wlog;
    std::vector<double2> W(Mmax / 2);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int t = 0; t < Mmax / 2; ++t) {
        const long double ang = -2.0L * pi * t / Mmax;
        W[t] = make_double2((double)cosl(ang), (double)sinl(ang));
    }
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
    // launch classes in XCD-aware order: block b runs on XCD b mod 8 and
    // consecutive blocks of one XCD take consecutive ring pairs
    std::vector<int> lists[kRingClasses];
    for (int q = 0; q < nq; ++q) lists[ring_class(Mq[q])].push_back(q);
    std::vector<int> all;
    for (int c = 0; c < kRingClasses; ++c) {
        p->class_off[c] = (int)all.size();
        const std::vector<int>& L = lists[c];
        const int nb = (int)L.size();
        int start[9] = {0};
        for (int x = 0; x < 8; ++x) start[x + 1] = start[x] + nb / 8 + (x < nb % 8 ? 1 : 0);
        for (int b = 0; b < nb; ++b) all.push_back(L[start[b % 8] + b / 8]);
    }
    p->class_off[kRingClasses] = (int)all.size();

    auto up = [&](void** dst, const void* src, size_t bytes) -> bool {
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up((void**)&p->d_ring_M, Mq.data(), nq * sizeof(int)) ||
        !up((void**)&p->d_ring_blue, blue.data(), nq * sizeof(int)) ||
        !up((void**)&p->d_ring_coff, coff.data(), nq * sizeof(long long)) ||
        !up((void**)&p->d_ring_boff, boff.data(), nq * sizeof(long long)) ||
        !up((void**)&p->d_twiddle, W.data(), W.size() * sizeof(double2)) ||
        !up((void**)&p->d_chirp, C.data(), C.size() * sizeof(double2)) ||
        !up((void**)&p->d_ring_class, all.data(), all.size() * sizeof(int)) ||
        hipMalloc((void**)&p->d_bspec, std::max<long long>(bsum, 1) * sizeof(double2)) != hipSuccess) {
        set_error("allocation or upload of ring FFT tables failed");
        return DMWF_ERR_OOM;
    }
    p->twiddle_log = wlog;
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
        const size_t lds = (size_t)kClassMaxM[c] * sizeof(double2);
        hipLaunchKernelGGL((k_chirp_spectrum<256>), dim3(bl[c].size()), dim3(256), lds, nullptr, dq,
                           p->d_nph, p->d_ring_M, p->d_ring_coff, p->d_ring_boff, p->d_chirp,
                           p->d_bspec, p->d_twiddle, wlog);
        DMWF_HIP(hipGetLastError());
        DMWF_HIP(hipDeviceSynchronize());
        DMWF_HIP(hipFree(dq));
    }
    return DMWF_OK;
}

dmwf_status launch_ring(dmwf_plan* p, RingMode mode, double2* spec, const int* ell_syn,
                        const int* ell_ana, const RingIO& io, hipStream_t s) {
    RingArgs a;
    a.g = p->geom();
    a.nq = p->nq;
    a.lmax = p->lmax;
    a.ell_syn = ell_syn;
    a.ell_ana = ell_ana;
    a.spec = spec;
    a.io = io;
    a.Mq = p->d_ring_M;
    a.blue = p->d_ring_blue;
    a.coff = p->d_ring_coff;
    a.boff = p->d_ring_boff;
    a.W = p->d_twiddle;
    a.wlog = p->twiddle_log;
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
    // largest classes first
    for (int c = kRingClasses - 1; c >= 0; --c) {
        const int nb = p->class_off[c + 1] - p->class_off[c];
        if (nb == 0) continue;
        a.qlist = p->d_ring_class + p->class_off[c];
        ProfScope ps(p, s, cls);
        launch_class(c, dim3(nb), (size_t)kClassMaxM[c] * sizeof(double2), s, a);
        DMWF_HIP(hipGetLastError());
    }
    return DMWF_OK;
}

}  // namespace dmwf
