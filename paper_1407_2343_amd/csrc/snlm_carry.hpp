// Segment-start states of whole-line running sums (plain or Kahan).
//
// Without block restarts, the window sum R_s(u) of eq. recursion at a position
// depends on every step since the start of the line.  To filter such a line in
// independent segments, this kernel runs, for one offset s per wave, exactly
// the recursion the whole-line pass runs (same scaled samples, same fused
// multiply-adds in the same order, Kahan compensation included) and records
// its state where each later segment's pre-chunk would otherwise start it
// afresh.  Segments that start from these states give bitwise the whole-line
// result.  The offset is a run-time value: each lane streams its line's
// samples (four chunks of 16 in flight) into an LDS ring of the recent scaled
// samples and reads the four it needs per step (positions u+K, u+K+s, u-K-1,
// u-K-1+s) from there.
#pragma once

#include "snlm_device.hpp"

namespace snlm {

struct CarryArgs {
    PassDesc pass;  // the pass to be cut (nseg > 1, restart = 0)
    float* carry;   // out: layout of PassDesc::carry
    int32_t S;      // search half-width of the pass
};

template <int K, bool KAHAN>
__global__ __launch_bounds__(kLanes) void snlm_carry_kernel(CarryArgs a) {
    constexpr int C = kChunk;
    constexpr int NPF = 4;     // chunks of samples in flight ahead of the recursion
    constexpr int RING = 128;  // samples of the line kept per lane (needs 2C + 2K + S + 1)
    __shared__ float ring[RING * kLanes];  // ring[(position mod RING) * 64 + lane]
    const PassDesc& d = a.pass;
    const int S = a.S;
    const int group = blockIdx.x % d.ngroups;
    const int s = blockIdx.x / d.ngroups + 1;
    const int lane = threadIdx.x & (kLanes - 1);
    const int line0 = group * kLanes;
    const bool active = line0 + lane < d.nlines;
    const LineIO io = make_io<false>(d, line0, lane, nullptr);
    const int line = min(line0 + lane, d.nlines - 1);
    const int R0 = (C - S) % C;  // where each segment's pre-chunk starts its sums
    const long kahan_off = (long)(d.nseg - 1) * S * d.nlines;
    const float alpha = d.alpha;
    float R = 0.0f, Rc = 0.0f;
    auto xs = [&](int p) -> float { return ring[(p & (RING - 1)) * kLanes + lane]; };

    // Samples stream through NPF register buffers into the ring.
    float vb[NPF][C];
    int issued = R0 - C - K - 1;  // next position to load
    int taken = issued;           // positions below this are in the ring
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
        io.template load<C>(issued, vb[q]);
        issued += C;
    }
    auto take = [&](int q) {
#pragma unroll
        for (int t = 0; t < C; ++t) ring[((taken + t) & (RING - 1)) * kLanes + lane] = alpha * vb[q][t];
        taken += C;
        io.template load<C>(issued, vb[q]);
        issued += C;
    };

    // fresh window sum at u0 = R0 - C (the first pre-chunk), as box_init: its
    // samples u0-K .. u0+K+s lie in the first three chunks (2K + s <= 32)
    const int u0 = R0 - C;
    take(0);
    take(1);
    take(2);
#pragma unroll
    for (int k = -K; k <= K; ++k) {
        const float dd = xs(u0 + k) - xs(u0 + k + s);
        R = (k == -K) ? dd * dd : __builtin_fmaf(dd, dd, R);
    }
    // slides for u = u0 + 1 .. : R(u) = R(u-1) + D(u+K) - D(u-K-1), 16 at a time
    int rec = 0;  // next segment start: (rec + 1) * seg_len, recorded at u = start - C + R0
    int u = u0 + 1;
    auto steps = [&]() {
        const int target = (rec + 1) * d.seg_len - C + R0;
#pragma unroll
        for (int t = 0; t < C; ++t) {
            const float de = xs(u + t + K) - xs(u + t + K + s);
            const float dl = xs(u + t - K - 1) - xs(u + t - K - 1 + s);
            if constexpr (KAHAN) {
                const float tt = __builtin_fmaf(de, de, -(dl * dl));
                const float y = tt - Rc;
                const float sum = R + y;
                Rc = (sum - R) - y;
                R = sum;
            } else {
                R = __builtin_fmaf(-dl, dl, __builtin_fmaf(de, de, R));
            }
            if (u + t == target && active) {
                const long at = ((long)rec * S + (s - 1)) * d.nlines + line;
                a.carry[at] = R;
                if constexpr (KAHAN) a.carry[at + kahan_off] = Rc;
            }
        }
        if (u + C > target) ++rec;  // a chunk holds at most one target (seg_len >= C)
        u += C;
    };
    while (rec < d.nseg - 1) {
#pragma unroll
        for (int q = 0; q < NPF; ++q) {
            // buffers are taken in issue order: 3, 0, 1, 2, 3, ...
            take((q + 3) % NPF);
            if (rec < d.nseg - 1 && u + C - 1 + K + s < taken) steps();
        }
    }
}

}  // namespace snlm
