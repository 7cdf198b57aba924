// The per-lane arithmetic of the 1D NLM line pass (eq. 1dNLM with PatchLift
// distances, Sec. 2.1-2.2) that every line kernel shares: the plain pass
// (snlm_device.hpp), the divergence-carrying pass (snlm_sure.hpp) and the pass
// from stored recursive-Gaussian distances (snlm_iir.hpp).  One definition
// keeps their rounding identical, so that the outputs y of the three agree
// bitwise where they compute the same thing.
//
// A lane holds a window xs of scaled samples a x(v) of its line; window index
// m is position c0 - XO + m, where c0 is the first centre of the current
// chunk of kChunk centres.  For offset s, the lifted diagonal is
//   D_s(v) = (a x(v) - a x(v+s))^2                  (eq. lift, difference form)
// and the patch distance of the pair (u, u+s) its window sum over the patch
//   box:   R_s(u) = sum_{k=-K..K} D_s(u+k), carried along u as eq. recursion
//          R_s(u) = R_s(u-1) + D_s(u+K) - D_s(u-K-1);
//   gauss: R_s(u) = sum_k g(k) D_s(u+k), an exact (2K+1)-tap FIR.
// The weight is w = exp2(-R) = exp(-d2 / h^2) (a^2 = log2(e) / h^2).
#pragma once

#include <hip/hip_runtime.h>

namespace snlm {

constexpr int kChunk = 16;  // centres per chunk; also the block-restart period

// Direct window sum of the lifted diagonal of offset s at centre index i
// (window index i + XO + k for tap k): the block-restart value.
template <int K, int XO, int NX>
__device__ __forceinline__ float box_init(const float (&xs)[NX], int i, int s) {
    float r = 0.0f;
#pragma unroll
    for (int k = -K; k <= K; ++k) {
        const float dd = xs[i + XO + k] - xs[i + XO + k + s];
        r = (k == -K) ? dd * dd : __builtin_fmaf(dd, dd, r);
    }
    return r;
}

// One step of eq. recursion to centre index i: the lifted sample D_s(u+K)
// enters the window, D_s(u-K-1) leaves it (XO = K + 1).
template <int K, int NX>
__device__ __forceinline__ void box_slide(const float (&xs)[NX], float& R, int i, int s) {
    const float de = xs[i + 2 * K + 1] - xs[i + 2 * K + 1 + s];
    const float dl = xs[i] - xs[i + s];
    R = __builtin_fmaf(-dl, dl, __builtin_fmaf(de, de, R));
}

// The same step with Kahan compensation Rc of the running sum.
template <int K, int NX>
__device__ __forceinline__ void box_slide_kahan(const float (&xs)[NX], float& R, float& Rc, int i, int s) {
    const float de = xs[i + 2 * K + 1] - xs[i + 2 * K + 1 + s];
    const float dl = xs[i] - xs[i + s];
    const float t = __builtin_fmaf(de, de, -(dl * dl));
    const float y = t - Rc;
    const float sum = R + y;
    Rc = (sum - R) - y;
    R = sum;
}

// Lifted diagonal of offset s, Dv[m] = D_s(c0 - K + m), for m in [m0, ND)
// (Gaussian kernel; ND = kChunk + 2K).
template <int NX, int ND>
__device__ __forceinline__ void lift_diag(const float (&xs)[NX], float (&Dv)[ND], int s, int m0) {
#pragma unroll
    for (int m = 0; m < ND; ++m) {
        if (m < m0) continue;
        const float dd = xs[m + 1] - xs[m + 1 + s];
        Dv[m] = dd * dd;
    }
}

// Gaussian FIR of the lifted diagonal at centre index i.
template <int K, int ND>
__device__ __forceinline__ float gauss_d2(const float (&Dv)[ND], const float (&g)[K + 1], int i) {
    float r = Dv[i + K];
#pragma unroll
    for (int k = 1; k <= K; ++k) r = __builtin_fmaf(g[k], Dv[i + K - k] + Dv[i + K + k], r);
    return r;
}

// Weight of a pair from its patch distance R (R >= 0 up to rounding).
__device__ __forceinline__ float pair_weight(float r) { return __builtin_amdgcn_exp2f(-__builtin_fabsf(r)); }

// Both centres of the pair (i, i+s) of weight w take the other's sample (the
// band symmetry of Sec. 2.1: w(i, i+s) = w(i+s, i)); own = false adds only
// the partner side (centre i+s), for pairs whose centre i lies before the
// segment.  P, Q hold the centres c0 .. c0+NP-1; xs[i + XO] is centre i.
template <int XO, int NX, int NP>
__device__ __forceinline__ void accumulate_pair(const float (&xs)[NX], float (&P)[NP], float (&Q)[NP], int i, int s,
                                                float w, bool own) {
    if (own) {
        P[i] = __builtin_fmaf(w, xs[i + XO + s], P[i]);
        Q[i] += w;
    }
    P[i + s] = __builtin_fmaf(w, xs[i + XO], P[i + s]);
    Q[i + s] += w;
}

// Moves the window on by one chunk: xs takes the next kChunk samples nx
// (scaled by alpha), the S trailing accumulators move to the front, and the
// new centres start with their s = 0 term (P = a x, Q = 1).
template <int S, int XO, int NX, int NP>
__device__ __forceinline__ void advance_chunk(float (&xs)[NX], float (&P)[NP], float (&Q)[NP], const float (&nx)[kChunk],
                                              float alpha) {
#pragma unroll
    for (int j = 0; j < NX - kChunk; ++j) xs[j] = xs[j + kChunk];
#pragma unroll
    for (int t = 0; t < kChunk; ++t) xs[NX - kChunk + t] = alpha * nx[t];
#pragma unroll
    for (int i = 0; i < S; ++i) {
        P[i] = P[i + kChunk];
        Q[i] = Q[i + kChunk];
    }
#pragma unroll
    for (int i = S; i < NP; ++i) {
        P[i] = xs[i + XO];
        Q[i] = 1.0f;
    }
}

// y = (P / Q) / a for the chunk's centres.
template <int NP>
__device__ __forceinline__ void normalise(const float (&P)[NP], const float (&Q)[NP], float inv_alpha,
                                          float (&y)[kChunk]) {
#pragma unroll
    for (int i = 0; i < kChunk; ++i) y[i] = (P[i] * __builtin_amdgcn_rcpf(Q[i])) * inv_alpha;
}

}  // namespace snlm
