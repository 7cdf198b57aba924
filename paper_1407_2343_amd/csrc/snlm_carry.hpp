// Segment-start states of whole-line running sums (plain or Kahan).
//
// Without block restarts, the window sum R_s(u) of eq. recursion at a position
// depends on every step since the start of the line.  To filter such a line in
// independent segments, this kernel runs, for one offset s per wave, exactly
// the recursion the whole-line pass runs (same scaled samples, same fused
// multiply-adds in the same order, Kahan compensation included) and records
// its state where each later segment's pre-chunk would otherwise start it
// afresh.  Segments that start from these states give bitwise the whole-line
// result.  The offset is a run-time value: the entering and leaving lifted
// samples come from four streams of the line (positions u+K, u+K+s, u-K-1,
// u-K-1+s), each read 16 samples at a time.
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

    // fresh window sum at u0 = R0 - C (the first pre-chunk), as box_init
    {
        const int u0 = R0 - C;
        float xa[2 * K + 1], xb[2 * K + 1];
        io.template load<2 * K + 1>(u0 - K, xa);
        io.template load<2 * K + 1>(u0 - K + s, xb);
#pragma unroll
        for (int k = 0; k <= 2 * K; ++k) {
            const float dd = alpha * xa[k] - alpha * xb[k];
            R = (k == 0) ? dd * dd : __builtin_fmaf(dd, dd, R);
        }
    }
    // slides for u = u0 + 1 .. : R(u) = R(u-1) + D(u+K) - D(u-K-1)
    int rec = 0;  // next segment start: (rec + 1) * seg_len, recorded at u = start - C + R0
    int u = R0 - C + 1;
    while (rec < d.nseg - 1) {
        float ea[C], eb[C], la[C], lb[C];
        io.template load<C>(u + K, ea);
        io.template load<C>(u + K + s, eb);
        io.template load<C>(u - K - 1, la);
        io.template load<C>(u - K - 1 + s, lb);
        const int target = (rec + 1) * d.seg_len - C + R0;
#pragma unroll
        for (int t = 0; t < C; ++t) {
            const float de = alpha * ea[t] - alpha * eb[t];
            const float dl = alpha * la[t] - alpha * lb[t];
            if constexpr (KAHAN) {
                const float tt = __builtin_fmaf(de, de, -(dl * dl));
                const float y = tt - Rc;
                const float sum = R + y;
                Rc = (sum - R) - y;
                R = sum;
            } else {
                R = __builtin_fmaf(-dl, dl, __builtin_fmaf(de, de, R));
            }
            if (u + t == target) {
                if (active) {
                    const long at = ((long)rec * S + (s - 1)) * d.nlines + line;
                    a.carry[at] = R;
                    if constexpr (KAHAN) a.carry[at + kahan_off] = Rc;
                }
            }
        }
        if (u + C > target) ++rec;  // a chunk holds at most one target (seg_len >= C)
        u += C;
    }
}

}  // namespace snlm
