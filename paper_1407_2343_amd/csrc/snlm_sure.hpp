// Divergence-carrying line pass for the SURE-optimal combination of the two
// separable orders (Sec. 3.1: Alg. 3, eq. div, eqs. partialrc / partialcr).
//
// Along with the 1D NLM output y(i) of a line, the pass computes
//   dout(i) = din(i) * dy(i)/dx(i),
//   dy(i)/dx(i) = 1/Q + (2 / (h^2 Q)) (T + sum_j w (x(j) - y(i))^2),
//   T = sum_{|j-i|<=K} w g(i-j) (x(j) - y(i)) (x(2i-j) - x(i)),
// which is eq. div regrouped: the printed form's sum of w x(j)^2 minus Q y^2 is
// the weighted spread of x(j) around y(i), and its four T accumulators expand
// the same product.  The kernel accumulates both around the centre sample
// instead, so that FP32 does not cancel:
//   M  = sum_j w (x(j) - x(i))^2
//   U1 = sum_{|j-i|<=K} w g (x(j) - x(i)) (x(2i-j) - x(i))
//   U2 = sum_{|j-i|<=K} w g (x(2i-j) - x(i))
// and at the output, with dx = y(i) - x(i):
//   sum_j w (x(j) - y)^2 = M - Q dx^2,      T = U1 - dx U2.
// Every term is carried on the scaled samples xs = a x (a^2 = log2(e) / h^2),
// so 2 / h^2 becomes 2 ln 2.  Each unordered pair (i, i+s) contributes to both
// of its centres, as in the plain pass; the y(i) it produces is bitwise the
// plain pass's.
#pragma once

#include "snlm_device.hpp"

namespace snlm {

constexpr float kTwoLn2 = 1.3862943611198906f;

struct DivArgs {
    PassDesc pass;        // samples in and out, as for a plain pass
    const float* din;     // divergence carried in; nullptr: 1
    float* dout;          // divergence out
    uint32_t din_bytes, dout_bytes;
    int32_t d_line;       // element stride between lines of both divergence buffers
    int32_t d_pos;        // element stride between samples
};

// The divergence carried in, one chunk of a lane's line at a time.  Row
// passes (samples contiguous, 16-byte aligned) read a whole chunk with four
// 16-byte loads per lane instead of sixteen 4-byte ones.
struct DivIn {
    __amdgpu_buffer_rsrc_t r;
    int32_t base_b, pos_b;
    bool has, vec;

    __device__ __forceinline__ float load(int p) const {
        if (!has) return 1.0f;
        return as_float(__builtin_amdgcn_raw_buffer_load_b32(r, base_b + p * pos_b, 0, 0));
    }
    // positions past the line's end read its last sample (never stored)
    __device__ __forceinline__ void load_chunk(int c0, int n, float* dv) const {
        if (!has) {
#pragma unroll
            for (int i = 0; i < kChunk; ++i) dv[i] = 1.0f;
        } else if (vec && c0 + kChunk <= n) {
#pragma unroll
            for (int q = 0; q < kChunk / 4; ++q) {
                const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, base_b + (c0 + 4 * q) * 4, 0, 0);
#pragma unroll
                for (int e = 0; e < 4; ++e) dv[4 * q + e] = as_float(w[e]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < kChunk; ++i) dv[i] = load(min(c0 + i, n - 1));
        }
    }
};

// io: samples in and y out; dio: the same lines' divergence out (io with the
// divergence buffer as its output; row passes stage it through the same LDS
// output tile as y).
template <int S, int K, bool GAUSS>
__device__ __forceinline__ void run_segment_div(const PassDesc& d, const LineIO& io, const LineIO& dio,
                                                const DivIn& din, int seg_a, int seg_b) {
    constexpr int C = kChunk;
    constexpr int NX = C + S + 2 * K + 1;  // x window: positions c0-K-1 .. c0+C+S+K-1
    constexpr int NP = C + S;              // centres c0 .. c0+C+S-1
    constexpr int ND = C + 2 * K;          // lifted samples of one diagonal (Gaussian)
    constexpr int R0 = (C - S) % C;        // restart offset within a chunk
    constexpr int XO = K + 1;              // x index of centre c0
    constexpr int KU = K < S ? K : S;      // offsets whose pairs enter T (|j - i| <= K)
    constexpr int NU = C + KU;             // centres c0 .. c0+C+KU-1 for U1, U2
    static_assert(S >= 1 && S <= kMaxS && K >= 0 && K <= kMaxK, "parameter range");

    const float alpha = d.alpha;
    const float inv_alpha = d.inv_alpha;
    float xs[NX], P[NP], Q[NP], M[NP], U1[NU], U2[NU], nx[C];
    float R[S];
    float Dv[GAUSS ? ND : 1];
    float g[K + 1];
#pragma unroll
    for (int k = 0; k <= K; ++k) g[k] = d.taps[k];

    // The pre-chunk's window and the first chunk's loads, as in the plain pass.
    int c0 = seg_a - C;
    if (io.stage_in) {
        if (io.template window_staged<NX>(c0 - K - 1)) {
            io.template start_window<NX>(c0 - K - 1);
            const bool tile_loads = io.chunk_staged(seg_a + S + K);
            io.issue_chunk(seg_a + S + K, nx);
            io.template finish_window<NX>(c0 - K - 1, xs, tile_loads);
        } else {
            io.template load<NX>(c0 - K - 1, xs);
            io.issue_chunk(seg_a + S + K, nx);
        }
    } else {
        io.issue_chunk(seg_a + S + K, nx);
        io.template load<NX>(c0 - K - 1, xs);
    }
#pragma unroll
    for (int j = 0; j < NX; ++j) xs[j] = alpha * xs[j];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        P[i] = xs[i + XO];
        Q[i] = 1.0f;
        M[i] = 0.0f;
    }
#pragma unroll
    for (int i = 0; i < NU; ++i) {
        U1[i] = 0.0f;
        U2[i] = 0.0f;
    }

    // Pair (i, i+s) of weight w: its partner terms for centre i+s, and, when
    // centre_i, its terms for centre i.
    auto pair = [&](int i, int s, float w, bool centre_i) {
        accumulate_pair<XO>(xs, P, Q, i, s, w, centre_i);  // y: as the plain pass
        const float xi = xs[i + XO];
        const float xj = xs[i + s + XO];
        const float dc = xi - xj;  // x(i) - x(i+s)
        const float wd2 = w * (dc * dc);
        if (centre_i) M[i] += wd2;
        M[i + s] += wd2;
        if (s <= KU) {
            const float wg = GAUSS ? w * g[s] : w;
            if (centre_i) {
                const float t1 = wg * (xs[i - s + XO] - xi);  // w g (x(i-s) - x(i))
                U1[i] = __builtin_fmaf(t1, -dc, U1[i]);       // times x(i+s) - x(i)
                U2[i] += t1;
            }
            const float t2 = wg * (xs[i + 2 * s + XO] - xj);  // w g (x(i+2s) - x(i+s))
            U1[i + s] = __builtin_fmaf(t2, dc, U1[i + s]);    // times x(i) - x(i+s)
            U2[i + s] += t2;
        }
    };

    // ---- pre-chunk: pairs (u, u+s) with u in [seg_a - s, seg_a) ----
#pragma unroll
    for (int s = 1; s <= S; ++s) {
        const int si = s - 1;
        if constexpr (GAUSS) lift_diag(xs, Dv, s, C - s);
#pragma unroll
        for (int i = R0; i < C; ++i) {
            float r;
            if constexpr (GAUSS) {
                if (i < C - s) continue;
                r = gauss_d2<K>(Dv, g, i);
            } else {
                if (i == R0)
                    R[si] = box_init<K, XO>(xs, i, s);
                else
                    box_slide<K>(xs, R[si], i, s);
                if (i < C - s) continue;
                r = R[si];
            }
            pair(i, s, pair_weight(r), false);
        }
    }

    // ---- main chunks ----
    int stores_last = 0;  // staged stores issued after the pending chunk's loads
    for (c0 = seg_a;; c0 += C) {
        io.finish_chunk(c0 + S + K, nx, stores_last);
        advance_chunk<S, XO>(xs, P, Q, nx, alpha);
#pragma unroll
        for (int i = 0; i < S; ++i) M[i] = M[i + C];
#pragma unroll
        for (int i = S; i < NP; ++i) M[i] = 0.0f;
#pragma unroll
        for (int i = 0; i < KU; ++i) {
            U1[i] = U1[i + C];
            U2[i] = U2[i + C];
        }
#pragma unroll
        for (int i = KU; i < NU; ++i) {
            U1[i] = 0.0f;
            U2[i] = 0.0f;
        }
        const bool has_next = c0 + C < seg_b;
        // (column passes fetch the next chunk unconditionally, as the plain pass)
        if (has_next || !io.stage_in) io.issue_chunk(c0 + C + S + K, nx);
        float dv[C];
        din.load_chunk(c0, d.n, dv);

#pragma unroll
        for (int s = 1; s <= S; ++s) {
            const int si = s - 1;
            if constexpr (GAUSS) lift_diag(xs, Dv, s, 0);
#pragma unroll
            for (int i = 0; i < C; ++i) {
                float r;
                if constexpr (GAUSS) {
                    r = gauss_d2<K>(Dv, g, i);
                } else {
                    if (i == R0)
                        R[si] = box_init<K, XO>(xs, i, s);  // block restart
                    else
                        box_slide<K>(xs, R[si], i, s);
                    r = R[si];
                }
                pair(i, s, pair_weight(r), true);
            }
        }

        float y[C], dd[C];
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const float rq = __builtin_amdgcn_rcpf(Q[i]);
            const float ys = P[i] * rq;
            y[i] = ys * inv_alpha;
            const float dx = ys - xs[i + XO];
            const float spread = __builtin_fmaf(-(Q[i] * dx), dx, M[i]);
            const float t = __builtin_fmaf(-dx, U2[i], U1[i]);
            dd[i] = dv[i] * (__builtin_fmaf(kTwoLn2, t + spread, 1.0f) * rq);
        }
        // Lanes past the last line repeat its work: their stores write the
        // same bits to the same addresses, as in the plain pass.
        if (!has_next) {
            io.store_chunk(c0, seg_b, y);
            dio.store_chunk(c0, seg_b, dd);
            break;
        }
        const bool y_staged = io.store_full(c0, y);
        const bool d_staged = dio.store_full(c0, dd);
        stores_last = y_staged && d_staged ? 8 : 0;
    }
}

// S = 0: y = x and dy/dx = 1.
__device__ __forceinline__ void run_copy_div(const LineIO& io, const LineIO& dio, const DivIn& din, int seg_a,
                                             int seg_b) {
    for (int p = seg_a; p < seg_b; ++p) {
        float v[1];
        io.template load<1>(p, v);
        const float dv = din.load(p);
        io.store(p, v[0]);
        dio.store(p, dv);
    }
}

// One workgroup (one wave) per (line group, segment), as the direct plain
// pass.  ROWS: lines contiguous in memory; samples in, y out and the
// divergence out go through the LDS tiles of the plain row kernel.
template <int S, int K, bool GAUSS, bool ROWS>
__global__ __launch_bounds__(kLanes) void snlm_div_kernel(DivArgs a) {
    __shared__ __attribute__((aligned(16))) float tiles[ROWS ? row_lds_floats(kChunk + S + 2 * K + 1) : 1];
    const PassDesc& d = a.pass;
    const int t = blockIdx.x;
    const int group = t % d.ngroups;
    const int seg_a = (t / d.ngroups) * d.seg_len;
    const int seg_b = min(seg_a + d.seg_len, d.n);
    const int lane = threadIdx.x & (kLanes - 1);
    const int line0 = group * kLanes;
    const LineIO io = make_io<ROWS>(d, line0, lane, tiles);
    const int line = min(line0 + lane, d.nlines - 1);
    LineIO dio = io;
    dio.rout = make_rsrc(a.dout, a.dout_bytes);
    dio.out_base_b = line * a.d_line * 4;
    dio.out_pos_b = a.d_pos * 4;
    dio.out_line = a.d_line;
    dio.out_bytes = a.dout_bytes;
    dio.stage_out = ROWS && a.d_pos == 1 && (a.d_line & 3) == 0 && ((uintptr_t)a.dout & 15) == 0;
    DivIn din;
    din.r = make_rsrc(a.din, a.din ? a.din_bytes : 0u);
    din.base_b = line * a.d_line * 4;
    din.pos_b = a.d_pos * 4;
    din.has = a.din != nullptr;
    din.vec = ROWS && a.d_pos == 1 && (a.d_line & 3) == 0 && ((uintptr_t)a.din & 15) == 0;
    if constexpr (S == 0)
        run_copy_div(io, dio, din, seg_a, seg_b);
    else
        run_segment_div<S, K, GAUSS>(d, io, dio, din, seg_a, seg_b);
}

}  // namespace snlm
