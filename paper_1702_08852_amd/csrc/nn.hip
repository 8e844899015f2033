// Learned warm start of the solve: a small harmonic-space network, trained and
// run by the kernels of this file.
//
// The paper's solver starts every solve from s = 0 (Algorithm 2's
// initialisation); a warm start replaces that zero by an estimate of the
// Wiener filter a_lm.  The estimate comes from a per-mode network shared by all
// (l, m): three fully connected layers (F -> 128 -> 128 -> 2, ReLU after the
// first two) in FP32, applied to features of one mode,
//
//   x_0..17  the masked-data coefficients d_{l+k, m}, k = -4..4 (re, im),
//            whitened by sqrt(C_l + N_w) (zero outside m <= l + k <= lmax)
//   x_18     Wiener ratio C_l / (C_l + N_w)
//   x_19     m / (l + 1)
//   x_20     unmasked sky fraction
//   x_21     log10(N_w / C_l) / 10
//   x_22,23  zero
//
// with d_lm = Omega Y^H (d on unmasked pixels) and N_w = Omega / mean(N^-1
// over unmasked pixels) the white-noise level of the map in harmonic units
// (the noise-weight spectrum taken flat).  The output y is the Wiener filter
// coefficient in prior units: a_lm = sqrt(C_l) (y_0 + i y_1).  The window
// along l at fixed m lets the network see the coupling of neighbouring l that
// an azimuthally symmetric cut (the galactic band) induces.
//
// Training: mean squared error over a batch, plain backpropagation, Adam.
// Every product of the layers is a tiled FP32 GEMM (one kernel with strides,
// so that transposed operands need no copies); the weight gradients reduce
// over the batch in split-K partials summed in a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"

struct dmwf_nn {
    int max_batch;
    int device;
    float* params = nullptr;  // flat: W1 [F][H], b1 [H], W2 [H][H], b2 [H], W3 [H][O], b3 [O]
    float* grads = nullptr;
    float* m1 = nullptr;      // Adam first moment
    float* m2 = nullptr;      // Adam second moment
    long long step = 0;
    float* h1 = nullptr;      // [max_batch][H] activations of layer 1
    float* h2 = nullptr;      // [max_batch][H]
    float* y = nullptr;       // [max_batch][O]
    float* g3 = nullptr;      // [max_batch][O] dLoss/dy
    float* g2 = nullptr;      // [max_batch][H] dLoss/d(pre-activation 2)
    float* g1 = nullptr;      // [max_batch][H]
    float* part = nullptr;    // split-K partials of the weight gradients
    float* lpart = nullptr;   // per-block partial sums of the loss
    float* xbuf = nullptr;    // [max_batch][F] features (warm start)
    float* ones = nullptr;    // one 1.0f (the batch sum as a GEMM with a stride-0 operand)
};

namespace dmwf {
namespace nn {

constexpr int F = 24, H = 128, O = 2;
constexpr int kW1 = 0, kB1 = kW1 + F * H, kW2 = kB1 + H, kB2 = kW2 + H * H, kW3 = kB2 + H,
              kB3 = kW3 + H * O, kParams = kB3 + O;
constexpr int kWin = 4;          // the l window: l - 4 .. l + 4
constexpr int kSplit = 32;       // split-K partials of a weight gradient
constexpr int kLossBlocks = 256;

namespace {

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------
// The m of an a_lm slot: the largest m whose first slot, base(m) + m =
// m (2 lmax + 3 - m) / 2, is <= s (a root of the quadratic, then corrected).
__device__ __forceinline__ long long first_slot(int m, int lmax) { return alm_base(m, lmax) + m; }
__device__ __forceinline__ int m_of_slot(long long s, int lmax) {
    const double b = 2.0 * lmax + 3.0;
    int m = (int)floor((b - sqrt(fmax(b * b - 8.0 * (double)s, 0.0))) * 0.5);
    m = max(0, min(m, lmax));
    while (m > 0 && first_slot(m, lmax) > s) --m;
    while (m < lmax && first_slot(m + 1, lmax) <= s) ++m;
    return m;
}

struct FeatArgs {
    int lmax;
    const double2* dlm;   // masked-data coefficients of one map
    const double* cl;
    double nw, fsky;
    const int* slots;     // alm slots of the rows, or NULL: row i is slot s0 + i
    long long s0;
    int n;
    const double2* target;  // Wiener filter a_lm (training) or NULL
    float* x;             // [n][F]
    float* t;             // [n][O] or NULL
};

__global__ void k_features(FeatArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const long long s = a.slots ? a.slots[i] : a.s0 + i;
    const int m = m_of_slot(s, a.lmax);
    const int l = (int)(s - alm_base(m, a.lmax));  // slot = base(m) + l
    float* xr = a.x + (size_t)i * F;
    const double c = a.cl[l];
    const bool ok = l >= 2 && c > 0.0;
    if (!ok) {
        for (int f = 0; f < F; ++f) xr[f] = 0.f;
        if (a.t) a.t[2 * i] = a.t[2 * i + 1] = 0.f;
        return;
    }
    const double iw = 1.0 / sqrt(c + a.nw);
    const long long base = alm_base(m, a.lmax);
    for (int k = -kWin; k <= kWin; ++k) {
        const int lk = l + k;
        double re = 0.0, im = 0.0;
        if (lk >= m && lk <= a.lmax) {
            const double2 v = a.dlm[base + lk];
            re = v.x * iw;
            im = m == 0 ? 0.0 : v.y * iw;
        }
        xr[2 * (k + kWin)] = (float)re;
        xr[2 * (k + kWin) + 1] = (float)im;
    }
    xr[18] = (float)(c / (c + a.nw));
    xr[19] = (float)((double)m / (l + 1.0));
    xr[20] = (float)a.fsky;
    xr[21] = (float)(log10(a.nw / c) / 10.0);
    xr[22] = xr[23] = 0.f;
    if (a.t) {
        const double2 v = a.target[s];
        const double sc = 1.0 / sqrt(c);
        a.t[2 * i] = (float)(v.x * sc);
        a.t[2 * i + 1] = (float)(m == 0 ? 0.0 : v.y * sc);
    }
}

// a_lm = sqrt(C_l) (y_0 + i y_1) on every slot; zero where l < 2 or C_l = 0
__global__ void k_unwhiten(int lmax, const double* cl, const float* y, long long s0, int n,
                           double2* alm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long s = s0 + i;
    const int m = m_of_slot(s, lmax);
    const int l = (int)(s - alm_base(m, lmax));
    const double c = cl[l];
    double2 v = make_double2(0.0, 0.0);
    if (l >= 2 && c > 0.0) {
        const double sc = sqrt(c);
        v = make_double2(sc * y[2 * i], m == 0 ? 0.0 : sc * y[2 * i + 1]);
    }
    alm[s] = v;
}

// ---------------------------------------------------------------------------
// GEMM: C = A B with strided operands, 64 x 64 tiles, 16 k per step, 256
// threads of 4 x 4 outputs.  blockIdx.z takes the k range [z kc, (z+1) kc).
// ---------------------------------------------------------------------------
enum Epi { EPI_STORE = 0, EPI_BIAS, EPI_BIAS_RELU, EPI_RELU_MASK };

struct GemmArgs {
    int M, N, K, kc;
    const float* A;
    long long a_i, a_k;
    const float* B;
    long long b_k, b_j;
    float* C;
    long long c_i, c_z;   // C(i, j) at C + z c_z + i c_i + j
    const float* bias;    // EPI_BIAS*: bias[j]
    const float* R;       // EPI_RELU_MASK: C(i, j) *= (R[i r_i + j] > 0)
    long long r_i;
};

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ float As[16][68];
    __shared__ float Bs[16][68];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int kb = blockIdx.z * g.kc, ke = min(g.K, kb + g.kc);
    float acc[4][4] = {};
    for (int k0 = kb; k0 < ke; k0 += 16) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = threadIdx.x + 256 * u;  // 0..1023
            const int r = e >> 4, kk = e & 15;    // A tile: row r, k kk
            const int gi = i0 + r, gk = k0 + kk;
            As[kk][r] = (gi < g.M && gk < ke) ? g.A[gi * g.a_i + gk * g.a_k] : 0.f;
            const int kr = e >> 6, cj = e & 63;   // B tile: k kr, column cj
            const int bk = k0 + kr, bj = j0 + cj;
            Bs[kr][cj] = (bk < ke && bj < g.N) ? g.B[bk * g.b_k + bj * g.b_j] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                av[u] = As[kk][ty * 4 + u];
                bv[u] = Bs[kk][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fmaf(av[u], bv[v], acc[u][v]);
        }
        __syncthreads();
    }
    float* C = g.C + blockIdx.z * g.c_z;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = i0 + ty * 4 + u;
        if (i >= g.M) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = j0 + tx * 4 + v;
            if (j >= g.N) continue;
            float r = acc[u][v];
            if (EPI == EPI_BIAS || EPI == EPI_BIAS_RELU) r += g.bias[j];
            if (EPI == EPI_BIAS_RELU) r = fmaxf(r, 0.f);
            if (EPI == EPI_RELU_MASK && !(g.R[i * g.r_i + j] > 0.f)) r = 0.f;
            C[i * g.c_i + j] = r;
        }
    }
}

// out[e] = sum over z of part[z][e], z in order
__global__ void k_sum_parts(const float* part, int nz, int n, float* out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float s = 0.f;
    for (int z = 0; z < nz; ++z) s += part[(size_t)z * n + e];
    out[e] = s;
}

// g3 = 2 (y - t) / n, per-block sums of (y - t)^2
__global__ void k_mse(const float* y, const float* t, int n, float* g3, float* lpart) {
    __shared__ float sh[256];
    float acc = 0.f;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * O; e += gridDim.x * blockDim.x) {
        const float d = y[e] - t[e];
        g3[e] = 2.f * d / n;
        acc = fmaf(d, d, acc);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = sh[0];
}

__global__ void k_loss_final(const float* lpart, int nb, int n, float* loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += lpart[b];
    *loss = (float)(s / n);
}

// Adam (Kingma & Ba 2015) with bias-corrected moments
__global__ void k_adam(float* p, const float* g, float* m1, float* m2, int n, float lr, float c1,
                       float c2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gv = g[e];
    const float a = b1 * m1[e] + (1.f - b1) * gv;
    const float b = b2 * m2[e] + (1.f - b2) * gv * gv;
    m1[e] = a;
    m2[e] = b;
    p[e] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// sum of N^-1 and count over unmasked pixels, per block (double, fixed order)
__global__ void k_wstats(const double* w, long long n, double* part) {
    __shared__ double sw[256], sc[256];
    double a = 0.0, c = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double v = w[i];
        if (v > 0.0) {
            a += v;
            c += 1.0;
        }
    }
    sw[threadIdx.x] = a;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sw[threadIdx.x] += sw[threadIdx.x + st];
            sc[threadIdx.x] += sc[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sw[0];
        part[2 * blockIdx.x + 1] = sc[0];
    }
}

__global__ void k_fill(float* p, int n, float v) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

template <int EPI>
dmwf_status gemm(const GemmArgs& g, int splits, hipStream_t s) {
    const dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, splits);
    hipLaunchKernelGGL((k_gemm<EPI>), grid, dim3(256), 0, s, g);
    DMWF_HIP(hipGetLastError());
    return DMWF_OK;
}

// Layer products of a batch of n rows of x.
dmwf_status forward(dmwf_nn* net, const float* x, int n, float* y, hipStream_t s) {
    const float* P = net->params;
    GemmArgs g{};
    // h1 = relu(x W1 + b1)
    g = GemmArgs{n, H, F, F, x, F, 1, P + kW1, H, 1, net->h1, H, 0, P + kB1, nullptr, 0};
    dmwf_status st = gemm<EPI_BIAS_RELU>(g, 1, s);
    if (st != DMWF_OK) return st;
    g = GemmArgs{n, H, H, H, net->h1, H, 1, P + kW2, H, 1, net->h2, H, 0, P + kB2, nullptr, 0};
    st = gemm<EPI_BIAS_RELU>(g, 1, s);
    if (st != DMWF_OK) return st;
    g = GemmArgs{n, O, H, H, net->h2, H, 1, P + kW3, O, 1, y, O, 0, P + kB3, nullptr, 0};
    return gemm<EPI_BIAS>(g, 1, s);
}

// dW = A^T G summed over the batch (A [n][kin], G [n][nout]) into out
// [kin][nout], and db = 1^T G into outb [nout], both through split-K partials.
dmwf_status weight_grad(dmwf_nn* net, const float* A, int kin, const float* G, int nout, int n,
                        float* out, float* outb, hipStream_t s) {
    const int kc = ((n + kSplit - 1) / kSplit + 15) / 16 * 16;
    const int nz = (n + kc - 1) / kc;
    GemmArgs g{kin, nout, n, kc, A, 1, kin, G, nout, 1, net->part, nout,
               (long long)kin * nout, nullptr, nullptr, 0};
    dmwf_status st = gemm<EPI_STORE>(g, nz, s);
    if (st != DMWF_OK) return st;
    hipLaunchKernelGGL(k_sum_parts, dim3((kin * nout + 255) / 256), dim3(256), 0, s, net->part, nz,
                       kin * nout, out);
    g = GemmArgs{1, nout, n, kc, net->ones, 0, 0, G, nout, 1, net->part, nout, nout, nullptr,
                 nullptr, 0};
    st = gemm<EPI_STORE>(g, nz, s);
    if (st != DMWF_OK) return st;
    hipLaunchKernelGGL(k_sum_parts, dim3((nout + 255) / 256), dim3(256), 0, s, net->part, nz, nout,
                       outb);
    DMWF_HIP(hipGetLastError());
    return DMWF_OK;
}

// Gradient of the mean squared error over the batch into net->grads, loss into *loss.
dmwf_status gradient(dmwf_nn* net, const float* x, const float* t, int n, float* loss,
                     hipStream_t s) {
    dmwf_status st = forward(net, x, n, net->y, s);
    if (st != DMWF_OK) return st;
    hipLaunchKernelGGL(k_mse, dim3(kLossBlocks), dim3(256), 0, s, net->y, t, n, net->g3,
                       net->lpart);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, net->lpart, kLossBlocks, n, loss);
    DMWF_HIP(hipGetLastError());
    float* G = net->grads;
    const float* P = net->params;
    // layer 3: dW3 = h2^T g3, db3 = sum g3; g2 = (g3 W3^T) masked by h2 > 0
    st = weight_grad(net, net->h2, H, net->g3, O, n, G + kW3, G + kB3, s);
    if (st != DMWF_OK) return st;
    GemmArgs g{n, H, O, O, net->g3, O, 1, P + kW3, 1, O, net->g2, H, 0, nullptr, net->h2, H};
    st = gemm<EPI_RELU_MASK>(g, 1, s);
    if (st != DMWF_OK) return st;
    // layer 2
    st = weight_grad(net, net->h1, H, net->g2, H, n, G + kW2, G + kB2, s);
    if (st != DMWF_OK) return st;
    g = GemmArgs{n, H, H, H, net->g2, H, 1, P + kW2, 1, H, net->g1, H, 0, nullptr, net->h1, H};
    st = gemm<EPI_RELU_MASK>(g, 1, s);
    if (st != DMWF_OK) return st;
    // layer 1
    return weight_grad(net, x, F, net->g1, H, n, G + kW1, G + kB1, s);
}

}  // namespace
}  // namespace nn
}  // namespace dmwf

using namespace dmwf;

extern "C" {

int dmwf_nn_param_count(void) { return nn::kParams; }

void dmwf_nn_destroy(dmwf_nn* net) {
    if (!net) return;
    float* bufs[] = {net->params, net->grads, net->m1, net->m2, net->h1, net->h2, net->y,
                     net->g3, net->g2, net->g1, net->part, net->lpart, net->xbuf, net->ones};
    for (float* b : bufs)
        if (b) (void)hipFree(b);
    delete net;
}

dmwf_status dmwf_nn_create(int max_batch, dmwf_nn** out) {
    if (!out) {
        set_error("out is NULL");
        return DMWF_ERR_INVALID_ARG;
    }
    *out = nullptr;
    if (max_batch < 1 || max_batch > (1 << 22)) {
        set_error("max_batch must be in [1, 2^22]");
        return DMWF_ERR_INVALID_ARG;
    }
    dmwf_nn* net = new dmwf_nn();
    net->max_batch = max_batch;
    if (hipGetDevice(&net->device) != hipSuccess) {
        delete net;
        set_error("hipGetDevice failed");
        return DMWF_ERR_HIP;
    }
    const size_t B = max_batch;
    const size_t nsplit = (size_t)nn::kSplit * nn::H * nn::H;
    struct {
        float** p;
        size_t n;
    } allocs[] = {{&net->params, nn::kParams}, {&net->grads, nn::kParams}, {&net->m1, nn::kParams},
                  {&net->m2, nn::kParams},     {&net->h1, B * nn::H},       {&net->h2, B * nn::H},
                  {&net->y, B * nn::O},        {&net->g3, B * nn::O},       {&net->g2, B * nn::H},
                  {&net->g1, B * nn::H},       {&net->part, nsplit},        {&net->lpart, nn::kLossBlocks},
                  {&net->xbuf, B * nn::F},     {&net->ones, 1}};
    for (auto& a : allocs) {
        if (hipMalloc((void**)a.p, a.n * sizeof(float)) != hipSuccess) {
            dmwf_nn_destroy(net);
            set_error("allocation of the network's buffers failed");
            return DMWF_ERR_OOM;
        }
    }
    hipLaunchKernelGGL(nn::k_fill, dim3((nn::kParams + 255) / 256), dim3(256), 0, nullptr,
                       net->params, nn::kParams, 0.f);
    hipLaunchKernelGGL(nn::k_fill, dim3((nn::kParams + 255) / 256), dim3(256), 0, nullptr, net->m1,
                       nn::kParams, 0.f);
    hipLaunchKernelGGL(nn::k_fill, dim3((nn::kParams + 255) / 256), dim3(256), 0, nullptr, net->m2,
                       nn::kParams, 0.f);
    hipLaunchKernelGGL(nn::k_fill, dim3(1), dim3(64), 0, nullptr, net->ones, 1, 1.f);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        dmwf_nn_destroy(net);
        set_error("initialisation of the network's buffers failed");
        return DMWF_ERR_HIP;
    }
    *out = net;
    return DMWF_OK;
}

dmwf_status dmwf_nn_get_params(dmwf_nn* net, float* dev_out, void* stream) {
    if (!net || !dev_out) {
        set_error("NULL argument");
        return DMWF_ERR_INVALID_ARG;
    }
    DMWF_HIP(hipMemcpyAsync(dev_out, net->params, nn::kParams * sizeof(float),
                            hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
    return DMWF_OK;
}

dmwf_status dmwf_nn_set_params(dmwf_nn* net, const float* dev_in, void* stream) {
    if (!net || !dev_in) {
        set_error("NULL argument");
        return DMWF_ERR_INVALID_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    DMWF_HIP(hipMemcpyAsync(net->params, dev_in, nn::kParams * sizeof(float),
                            hipMemcpyDeviceToDevice, s));
    // a new start: the optimizer state is reset
    hipLaunchKernelGGL(nn::k_fill, dim3((nn::kParams + 255) / 256), dim3(256), 0, s, net->m1,
                       nn::kParams, 0.f);
    hipLaunchKernelGGL(nn::k_fill, dim3((nn::kParams + 255) / 256), dim3(256), 0, s, net->m2,
                       nn::kParams, 0.f);
    DMWF_HIP(hipGetLastError());
    net->step = 0;
    return DMWF_OK;
}

dmwf_status dmwf_nn_features(int lmax, const double* dev_dlm, const double* dev_cl, double noise_w,
                             double fsky, const int* dev_slots, int n, const double* dev_target,
                             float* dev_x, float* dev_t, void* stream) {
    if (lmax < 0 || !dev_dlm || !dev_cl || !dev_x || n < 0 || (dev_target && !dev_t) ||
        !(noise_w > 0.0) || !(fsky > 0.0 && fsky <= 1.0)) {
        set_error("features: need lmax >= 0, noise_w > 0, 0 < fsky <= 1, outputs for targets");
        return DMWF_ERR_INVALID_ARG;
    }
    if (!dev_slots && (long long)n > (long long)(lmax + 1) * (lmax + 2) / 2) {
        set_error("features: more rows than a_lm slots");
        return DMWF_ERR_INVALID_ARG;
    }
    if (n == 0) return DMWF_OK;
    nn::FeatArgs a{lmax, reinterpret_cast<const double2*>(dev_dlm), dev_cl, noise_w, fsky,
                   dev_slots, 0, n, reinterpret_cast<const double2*>(dev_target), dev_x, dev_t};
    hipLaunchKernelGGL(nn::k_features, dim3((n + 255) / 256), dim3(256), 0,
                       static_cast<hipStream_t>(stream), a);
    DMWF_HIP(hipGetLastError());
    return DMWF_OK;
}

dmwf_status dmwf_nn_forward(dmwf_nn* net, const float* dev_x, int n, float* dev_y, void* stream) {
    if (!net || !dev_x || !dev_y || n < 0 || n > net->max_batch) {
        set_error("forward: NULL argument or batch outside 0..max_batch");
        return DMWF_ERR_INVALID_ARG;
    }
    if (n == 0) return DMWF_OK;
    return nn::forward(net, dev_x, n, dev_y, static_cast<hipStream_t>(stream));
}

dmwf_status dmwf_nn_gradient(dmwf_nn* net, const float* dev_x, const float* dev_t, int n,
                             float* dev_grad, float* dev_loss, void* stream) {
    if (!net || !dev_x || !dev_t || !dev_grad || !dev_loss || n < 1 || n > net->max_batch) {
        set_error("gradient: NULL argument or batch outside 1..max_batch");
        return DMWF_ERR_INVALID_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    dmwf_status st = nn::gradient(net, dev_x, dev_t, n, dev_loss, s);
    if (st != DMWF_OK) return st;
    DMWF_HIP(hipMemcpyAsync(dev_grad, net->grads, nn::kParams * sizeof(float),
                            hipMemcpyDeviceToDevice, s));
    return DMWF_OK;
}

dmwf_status dmwf_nn_train_step(dmwf_nn* net, const float* dev_x, const float* dev_t, int n,
                               float lr, float* dev_loss, void* stream) {
    if (!net || !dev_x || !dev_t || !dev_loss || n < 1 || n > net->max_batch || !(lr > 0.f)) {
        set_error("train_step: NULL argument, batch outside 1..max_batch or lr <= 0");
        return DMWF_ERR_INVALID_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    dmwf_status st = nn::gradient(net, dev_x, dev_t, n, dev_loss, s);
    if (st != DMWF_OK) return st;
    net->step += 1;
    const float c1 = 1.f - powf(0.9f, (float)net->step);
    const float c2 = 1.f - powf(0.999f, (float)net->step);
    hipLaunchKernelGGL(nn::k_adam, dim3((nn::kParams + 255) / 256), dim3(256), 0, s, net->params,
                       net->grads, net->m1, net->m2, nn::kParams, lr, c1, c2);
    DMWF_HIP(hipGetLastError());
    return DMWF_OK;
}

dmwf_status dmwf_nn_noise_stats(const double* dev_ninv, long long npix, double* noise_w,
                                double* fsky, void* stream) {
    if (!dev_ninv || npix < 1 || !noise_w || !fsky) {
        set_error("noise_stats: NULL argument or npix < 1");
        return DMWF_ERR_INVALID_ARG;
    }
    const long long npix_ = npix;
    const int nb = 256;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* part = nullptr;
    DMWF_HIP(hipMallocAsync((void**)&part, 2 * nb * sizeof(double), s));
    hipLaunchKernelGGL(nn::k_wstats, dim3(nb), dim3(256), 0, s, dev_ninv, npix_, part);
    std::vector<double> h(2 * nb);
    const hipError_t e1 = hipMemcpyAsync(h.data(), part, h.size() * sizeof(double),
                                         hipMemcpyDeviceToHost, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFreeAsync(part, s);
    DMWF_HIP(e1);
    DMWF_HIP(e2);
    double sw = 0.0, sc = 0.0;
    for (int b = 0; b < nb; ++b) {
        sw += h[2 * b];
        sc += h[2 * b + 1];
    }
    if (!(sc > 0.0)) {
        set_error("noise_stats: every pixel is masked");
        return DMWF_ERR_INVALID_ARG;
    }
    const double omega = 4.0 * 3.14159265358979323846 / (double)npix_;
    *noise_w = omega / (sw / sc);
    *fsky = sc / (double)npix_;
    return DMWF_OK;
}

dmwf_status dmwf_nn_warm_start(dmwf_nn* net, int lmax, const double* dev_dlm,
                               const double* dev_cl, double noise_w, double fsky,
                               double* dev_alm_out, void* stream) {
    if (!net || !dev_dlm || !dev_cl || !dev_alm_out || lmax < 0) {
        set_error("warm_start: NULL argument or lmax < 0");
        return DMWF_ERR_INVALID_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long long nalm = (long long)(lmax + 1) * (lmax + 2) / 2;
    double2* out = reinterpret_cast<double2*>(dev_alm_out);
    for (long long s0 = 0; s0 < nalm; s0 += net->max_batch) {
        const int n = (int)std::min<long long>(net->max_batch, nalm - s0);
        nn::FeatArgs a{lmax, reinterpret_cast<const double2*>(dev_dlm), dev_cl, noise_w, fsky,
                       nullptr, s0, n, nullptr, net->xbuf, nullptr};
        hipLaunchKernelGGL(nn::k_features, dim3((n + 255) / 256), dim3(256), 0, s, a);
        DMWF_HIP(hipGetLastError());
        dmwf_status st = nn::forward(net, net->xbuf, n, net->y, s);
        if (st != DMWF_OK) return st;
        hipLaunchKernelGGL(nn::k_unwhiten, dim3((n + 255) / 256), dim3(256), 0, s, lmax, dev_cl,
                           net->y, s0, n, out);
        DMWF_HIP(hipGetLastError());
    }
    return DMWF_OK;
}

}  // extern "C"
