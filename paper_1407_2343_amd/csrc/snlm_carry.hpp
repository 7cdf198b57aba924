// Segment-start states of whole-line running sums (plain or Kahan).
//
// Without block restarts, the window sum R_s(u) of eq. recursion at a position
// depends on every step since the start of the line.  To filter such a line in
// independent segments, this kernel runs, for one offset s per wave, exactly
// the recursion the whole-line pass runs (same scaled samples, same fused
// multiply-adds in the same order, Kahan compensation included) and records
// its state where each later segment's pre-chunk would otherwise start it
// afresh.  Segments that start from these states give bitwise the whole-line
// result.  The offset is a run-time value: each lane keeps a window of its
// line's scaled samples in registers (the next chunk of 16 in flight while a
// chunk's steps run; rows, contiguous in memory, come through the LDS tile of
// the line kernels with 16-byte loads), and once per chunk copies the window
// shifted by s (a branch on s, the same for every lane, to a copy with
// compile-time indices), so the 16 steps of a chunk read registers only.
#pragma once

#include "snlm_device.hpp"

namespace snlm {

struct CarryArgs {
    PassDesc pass;  // the pass to be cut (nseg > 1, restart = 0)
    float* carry;   // out: layout of PassDesc::carry
    int32_t S;      // search half-width of the pass
};

// ys[i] = xs[i + s] for i < NW, for the run-time s in [SF, kMaxS].
template <int NW, int SF>
__device__ __forceinline__ void carry_shift(const float* xs, float* ys, int s) {
    if (s == SF) {
#pragma unroll
        for (int i = 0; i < NW; ++i) ys[i] = xs[i + SF];
    } else if constexpr (SF < kMaxS) {
        carry_shift<NW, SF + 1>(xs, ys, s);
    }
}

template <int K, bool KAHAN>
__global__ __launch_bounds__(kLanes) void snlm_carry_kernel(CarryArgs a) {
    constexpr int C = kChunk;
    constexpr int NW = C + 2 * K + 1;   // a chunk's own samples: u-K-1 .. u+C+K-1
    constexpr int NX = NW + kMaxS;      // and their partners up to s = kMaxS further
    const PassDesc& d = a.pass;
    const int S = a.S;
    const int group = blockIdx.x % d.ngroups;
    const int s = blockIdx.x / d.ngroups + 1;
    const int lane = threadIdx.x & (kLanes - 1);
    const int line0 = group * kLanes;
    const bool active = line0 + lane < d.nlines;
    // input tile only (rows of a row pass: contiguous, 16-byte aligned)
    __shared__ __attribute__((aligned(16))) float tiles[kTileIn];
    const LineIO io = make_io<true>(d, line0, lane, tiles);
    const int line = min(line0 + lane, d.nlines - 1);
    const int R0 = (C - S) % C;  // where each segment's pre-chunk starts its sums
    const long kahan_off = (long)(d.nseg - 1) * S * d.nlines;
    const float alpha = d.alpha;
    float R = 0.0f, Rc = 0.0f;

    // The window of the chunk of steps u .. u+C-1: xs[i] = a x(u - K - 1 + i),
    // ys[i] = xs[i + s].  The first chunk starts one past the first fresh
    // window sum, at u0 = R0 - C (the first pre-chunk).
    const int u0 = R0 - C;
    int u = u0 + 1;
    float xs[NX], ys[NW];
    io.template load<NX>(u - K - 1, xs);
#pragma unroll
    for (int i = 0; i < NX; ++i) xs[i] = alpha * xs[i];
    carry_shift<NW, 1>(xs, ys, s);
    // fresh window sum at u0, as box_init: x(u0 + k) sits at index k + K
#pragma unroll
    for (int k = -K; k <= K; ++k) {
        const float dd = xs[k + K] - ys[k + K];
        R = (k == -K) ? dd * dd : __builtin_fmaf(dd, dd, R);
    }
    // slides R(u) = R(u-1) + D(u+K) - D(u-K-1), 16 at a time, without a
    // branch (each step's state kept), then the state a later segment needs
    int rec = 0;  // next segment start: (rec + 1) * seg_len, recorded at u = start - C + R0
    auto steps = [&]() {
        const int target = (rec + 1) * d.seg_len - C + R0;
        float Rv[C], Cv[KAHAN ? C : 1];
#pragma unroll
        for (int t = 0; t < C; ++t) {
            const float de = xs[t + 2 * K + 1] - ys[t + 2 * K + 1];  // D(u + t + K)
            const float dl = xs[t] - ys[t];                          // D(u + t - K - 1)
            if constexpr (KAHAN) {
                const float tt = __builtin_fmaf(de, de, -(dl * dl));
                const float y = tt - Rc;
                const float sum = R + y;
                Rc = (sum - R) - y;
                R = sum;
                Cv[t] = Rc;
            } else {
                R = __builtin_fmaf(-dl, dl, __builtin_fmaf(de, de, R));
            }
            Rv[t] = R;
        }
        if (u + C > target) {  // a chunk holds at most one target (seg_len >= C)
            const int k = target - u;  // the same for every lane
            if (k >= 0) {
                float r = Rv[0], rc = Cv[0];
#pragma unroll
                for (int t = 1; t < C; ++t)
                    if (k == t) {
                        r = Rv[t];
                        if constexpr (KAHAN) rc = Cv[t];
                    }
                if (active) {
                    const long at = ((long)rec * S + (s - 1)) * d.nlines + line;
                    a.carry[at] = r;
                    if constexpr (KAHAN) a.carry[at + kahan_off] = rc;
                }
            }
            ++rec;
        }
    };
    // The chunk after the window in flight while a chunk's steps run.
    float nx[C];
    int issued = u - K - 1 + NX;
    io.issue_chunk(issued, nx);
    for (;;) {
        steps();
        // the chunk in flight lands (waited for also at the end: no tile load
        // may still be writing LDS when the wave ends)
        io.finish_chunk(issued, nx, 0);
        if (rec >= d.nseg - 1) break;
        // next chunk: the window moves by C samples, the landed chunk enters
        // it, and the one after goes in flight
#pragma unroll
        for (int i = 0; i < NX - C; ++i) xs[i] = xs[i + C];
#pragma unroll
        for (int t = 0; t < C; ++t) xs[NX - C + t] = alpha * nx[t];
        issued += C;
        io.issue_chunk(issued, nx);
        u += C;
        carry_shift<NW, 1>(xs, ys, s);
    }
}

}  // namespace snlm
