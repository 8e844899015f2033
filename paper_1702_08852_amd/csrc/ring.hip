// Ring stage of the transform pair: the phi part of F / F^-1 on each HEALPix
// ring, fused with the pixel-space half of the dual messenger iteration.
//
// One workgroup per ring pair (north ring and its south mirror share the pixel
// count n and the first-pixel angle phi0).  With phi_j = phi0 + 2 pi j / n:
//   synthesis  s_j = Re F_0 + 2 Re sum_{m=1..l_iter} F_m e^{i m phi0} w^{(m j) mod n}
//   analysis   G_m = e^{-i m phi0} sum_j r_j conj(w^{(m j) mod n}),   w = e^{2 pi i / n}
// evaluated as direct sums against a table of the n-th roots of unity held in
// LDS (exact index reduction, no accumulated phase error).
//
// In RING_ITER mode the workgroup also performs the pixel step of paper
// Algorithm 2 in residual form: it reads s_prev, writes s, accumulates the
// Cauchy sums sum (s - s_prev)^2 and sum s^2, forms r = c (d - s) with
// c = xi w / (1 + (xi - alpha) w) (the messenger step with N_bar = N - alpha)
// and analyses r into G in place of F.
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
};

__device__ __forceinline__ double block_sum(double v, double* scratch) {
    // 256 threads
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += scratch[i];
    }
    return t;
}

__global__ __launch_bounds__(256) void k_ring_direct(RingArgs a) {
    extern __shared__ double smem[];
    __shared__ double red[8];
    const int q = blockIdx.x;
    const int n = a.g.nph[q];
    const double c = a.g.phi0pi[q];
    const bool eq = (q == a.nq - 1);
    const int nh = eq ? 1 : 2;
    const long long st0 = a.g.start_n[q], st1 = a.g.start_s[q];
    const int ell = *a.ell_syn;
    const int ella = *a.ell_ana;
    const int L1 = a.lmax + 1;
    double2* tw = reinterpret_cast<double2*>(smem);  // [n]
    double2* E = tw + n;                              // [2][L1]
    double* r = reinterpret_cast<double*>(E + 2 * L1);  // [2][n]
    const int tid = threadIdx.x, nt = blockDim.x;

    for (int t = tid; t < n; t += nt) {
        double sn, cs;
        sincospi(2.0 * t / n, &sn, &cs);
        tw[t] = make_double2(cs, sn);
    }
    const bool syn = (a.mode == RING_SYN || a.mode == RING_ITER || a.mode == RING_SYN_WRES);
    if (syn && ell < 0 && tid == 0) {
        E[0] = make_double2(0.0, 0.0);
        E[L1] = make_double2(0.0, 0.0);
    }
    if (syn) {
        for (int m = tid; m <= ell; m += nt) {
            double sn, cs;
            sincospi(m * c, &sn, &cs);
            for (int h = 0; h < nh; ++h) {
                double2 F = a.spec[((size_t)m * a.nq + q) * 2 + h];
                if (m == 0) F.y = 0.0;
                E[h * L1 + m] = make_double2(F.x * cs - F.y * sn, F.x * sn + F.y * cs);
            }
        }
    }
    __syncthreads();

    double num = 0.0, den = 0.0;
    if (syn) {
        for (int j = tid; j < n; j += nt) {
            for (int h = 0; h < nh; ++h) {
                const double2* Eh = E + h * L1;
                double acc = 0.0;
                int t = 0;
                for (int m = 1; m <= ell; ++m) {
                    t += j;
                    if (t >= n) t -= n;
                    const double2 e = Eh[m], w = tw[t];
                    acc = fma(e.x, w.x, fma(-e.y, w.y, acc));
                }
                const double s = fma(2.0, acc, Eh[0].x);
                const long long p = (h == 0 ? st0 : st1) + j;
                if (a.mode == RING_SYN) {
                    a.io.map_out[p] = s;
                } else if (a.mode == RING_SYN_WRES) {
                    r[h * n + j] = a.io.w[p] * (a.io.d[p] - s);
                } else {
                    const double sp = a.io.first ? 0.0 : a.io.s_map[p];
                    const double ds = s - sp;
                    num = fma(ds, ds, num);
                    den = fma(s, s, den);
                    a.io.s_map[p] = s;
                    const double w = a.io.w[p];
                    const double cc = a.io.xi * w / fma(a.io.xi - a.io.alpha, w, 1.0);
                    r[h * n + j] = cc * (a.io.d[p] - s);
                }
            }
        }
    } else {
        for (int j = tid; j < n; j += nt) {
            for (int h = 0; h < nh; ++h) {
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
                r[h * n + j] = v;
            }
        }
    }
    if (a.mode == RING_ITER) {
        const double tn = block_sum(num, red);
        const double td = block_sum(den, red);
        if (tid == 0) {
            a.io.cpart[2 * q] = tn;
            a.io.cpart[2 * q + 1] = td;
        }
    }
    __syncthreads();
    if (a.mode == RING_SYN) return;

    for (int m = tid; m <= ella; m += nt) {
        const int mr = m % n;
        double sn, cs;
        sincospi(m * c, &sn, &cs);
        for (int h = 0; h < 2; ++h) {
            double2 G = make_double2(0.0, 0.0);
            if (h < nh) {
                const double* rh = r + h * n;
                double re = 0.0, im = 0.0;
                int t = 0;
                for (int j = 0; j < n; ++j) {
                    const double v = rh[j];
                    const double2 w = tw[t];
                    re = fma(v, w.x, re);
                    im = fma(-v, w.y, im);
                    t += mr;
                    if (t >= n) t -= n;
                }
                // times e^{-i m phi0}
                G = make_double2(re * cs + im * sn, im * cs - re * sn);
                if (m == 0) G.y = 0.0;
            }
            a.spec[((size_t)m * a.nq + q) * 2 + h] = G;
        }
    }
}

}  // namespace

size_t ring_lds_bytes(const dmwf_plan* p) {
    const size_t n = 4 * (size_t)p->nside;
    return n * sizeof(double2) + 2 * (size_t)(p->lmax + 1) * sizeof(double2) + 2 * n * sizeof(double);
}

dmwf_status launch_ring(dmwf_plan* p, RingMode mode, double2* spec, const int* ell_syn,
                        const int* ell_ana, const RingIO& io, hipStream_t s) {
    const size_t lds = ring_lds_bytes(p);
    if (lds + 64 > 160 * 1024) {
        set_error("ring stage: direct ring transform needs more LDS than a workgroup has");
        return DMWF_ERR_UNSUPPORTED;
    }
    RingArgs a;
    a.g = p->geom();
    a.nq = p->nq;
    a.lmax = p->lmax;
    a.ell_syn = ell_syn;
    a.ell_ana = ell_ana;
    a.spec = spec;
    a.io = io;
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
    ProfScope ps(p, s, cls);
    hipLaunchKernelGGL(k_ring_direct, dim3(p->nq), dim3(256), lds, s, a);
    DMWF_HIP(hipGetLastError());
    return DMWF_OK;
}

}  // namespace dmwf
