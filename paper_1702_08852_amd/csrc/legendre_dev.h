// Device helpers and launch arguments shared by the Legendre kernels of the
// FP64 path (legendre.hip) and of the reduced-precision matrix-core path
// (legendre_mx.hip).
#pragma once

#include "common.h"

namespace dmwf {

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// Workgroup b of a 1-D grid runs on XCD b mod 8 (round-robin dispatch).  Give
// each XCD whole m-groups, all ring chunks of a group together, so that the
// group's coefficient rows are fetched into a single L2; groups in order of
// decreasing work (increasing m) within every XCD.
struct LegTile {
    int chunk, group;
};
__device__ __forceinline__ LegTile leg_tile(int nchunk) {
    const int b = blockIdx.x, xcd = b & 7, slot = b >> 3;
    return {slot % nchunk, (slot / nchunk) * 8 + xcd};
}

// Orders this wave's LDS writes before its later LDS reads (and reads before
// later writes); the other waves of the workgroup use their own LDS region.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Rings whose recurrence starts at block l take their seed pair; the others
// either run already or still hold (0, 0) and contribute nothing.
template <int K>
__device__ __forceinline__ void inject(int l, const int (&ls)[K], const double (&s0)[K],
                                       const double (&s1)[K], double (&p1)[K], double (&p2)[K]) {
#pragma unroll
    for (int t = 0; t < K; ++t)
        if (ls[t] == l) {
            p2[t] = s0[t];
            p1[t] = s1[t];
        }
}

// Band limits of the MB maps of this workgroup's map group: -1 for a map past
// the end of the batch, whose solve has stopped, or (sel = 1 / 2, solve loop
// of a reduced-precision plan) whose contraction currently runs in the other
// precision (sel 1: this launch takes the FP64 maps, sel 2 the reduced ones).
// Returns their maximum.
template <int MB>
__device__ __forceinline__ int group_ells(int mg, int nm, const int* ell, int ell_stride,
                                          const DevCtrl* ctrl, int sel, int (&ellm)[MB]) {
    int e = -1;
#pragma unroll
    for (int i = 0; i < MB; ++i) {
        const int k = mg + i;
        int v = -1;
        bool on = k < nm;
        if (on && ctrl) {
            const DevCtrl& c = ctrl[k];
            on = !c.done && !(sel == 1 && c.reduced) && !(sel == 2 && !c.reduced);
        }
        if (on) v = ell[k * ell_stride];
        ellm[i] = v;
        e = max(e, v);
    }
    return e;
}

struct SynArgs {
    const double* x;
    const int* ls;
    const double* s0;
    const double* s1;
    const double* A;
    const double2* ap;       // pre-scaled a_lm of map 0; map k at ap + k * ap_map
    long long ap_map;
    double2* spec;           // F rows of map 0; map k at spec + k * spec_map
    long long spec_map;
    const int* ell;          // band limit of map k at ell[k * ell_stride]
    int ell_stride;
    const DevCtrl* ctrl;     // per-map control blocks (solve loop) or NULL
    int sel;                 // which maps of the solve loop this launch takes (group_ells)
    int lmax, nq, lp, nm;
    int nchunk;              // ring chunks of 64 K ring pairs
};

struct AnaArgs {
    const double* x;
    const int* ls;
    const double* s0;
    const double* s1;
    const double* A;
    const double2* spec;     // G rows of map 0; map k at spec + k * spec_map
    long long spec_map;
    double2* part;           // partial sums of map 0, chunk c at part + c * part_stride;
    size_t part_stride;      // map k at part + k * part_map
    long long part_map;
    const int* ell;          // band limit of map k at ell[k * ell_stride]
    int ell_stride;
    const DevCtrl* ctrl;     // per-map control blocks (solve loop) or NULL
    int sel;                 // which maps of the solve loop this launch takes (group_ells)
    int lmax, nq, lp, nm;
};

// Host side: largest power-of-two maps-per-wave count <= want, <= nm and
// <= cap; m-groups of kLegWaves consecutive m rounded up to whole XCD rounds.
int pick_mb(int want, int nm, int cap);
int leg_groups8(const dmwf_plan* p);

}  // namespace dmwf
