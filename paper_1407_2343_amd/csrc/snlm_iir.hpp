// Gaussian patch kernel by a recursive (IIR) filter: the third-order recursive
// Gaussian of Young & van Vliet (1995), to which Sec. 2.2 refers for the
// Gaussian case of eq. convn.  Its cost per sample does not depend on the
// patch width, so patches far wider than the exact FIR's 2K+1 <= 17 taps are
// affordable; it approximates the untruncated Gaussian exp(-k^2 / (2 beta^2)).
//
// Per offset s and line, the lifted diagonal D_s(v) = (a x(v) - a x(v+s))^2 of
// the reflected line is filtered by the causal recursion
//     w(v) = B D(v) + a1 w(v-1) + a2 w(v-2) + a3 w(v-3)
// forward over v in [-L, n + L) (its three past outputs starting as D(-L)),
// then by the same recursion backward over w (its three future outputs
// starting as w(n + L - 1)); sqrt(2 pi) beta times the result at u is the
// distance between the patches at u and u+s.  One pass runs three kernels
// (four for lines that are contiguous in memory, which first make a
// transposed copy of their input with snlm_iir_transpose_kernel and read
// that instead):
//   snlm_iir_fwd_kernel   w(v) for v in [-S, n + L), in segments
//   snlm_iir_bwd_kernel   the distances for u in [-S, n), in segments
//   snlm_iir_nlm_kernel<S, ROWS>  the 1D NLM of eq. 1dNLM with the weights
//       exp2(-d) of the stored distances, with the pairing, accumulation
//       order and pre-chunk of the lifted pass (results do not depend on its
//       segment length).
// A segment of either recursion starts W samples before its first output
// (forward) or after its last (backward), from the steady state of the value
// found there, or at the line's own start where that comes first.  The
// recursion forgets its start like rho^t, rho the largest pole modulus, and W
// is chosen with rho^W <= 1e-12, so segments reproduce the whole-line
// recursion far below FP32 resolution.  Segment lengths depend on the job
// only, never on the device.
//
// The recursion's state and coefficients are FP64: for wide kernels the poles
// approach 1 and B ~ 1.6 / (0.42 q^3) is small, so FP32 rounding of the
// coefficients alone would move the DC gain by ~1e-7 / B (0.2% at beta = 20)
// and every step's rounding would be amplified up to 1 / B times.  FP64 FMAs
// issue at the FP32 rate on this chip.  Lifted samples and stored values are
// FP32.
//
// Buffers (line fastest: every access of a wave is one 256-byte row):
//   w[((s - 1) * nvw + v + S) * nlines + line],     v in [-S, n + L), nvw = n + L + S
//   dist[((s - 1) * nvd + u + S) * nlines + line],  u in [-S, n),     nvd = n + S
#pragma once

#include "snlm_device.hpp"

namespace snlm {

struct IirArgs {
    PassDesc pass;         // the pass whose distances are wanted (input addressing, n, alpha)
    float* w;              // forward output
    float* dist;           // distances
    uint32_t w_bytes, dist_bytes;
    int32_t S;             // search half-width (offsets 1..S)
    int32_t L;             // the recursion runs L samples beyond each end of the line
    int32_t W;             // warm-up of a segment that does not start at the line's start
    int32_t seg;           // outputs per segment (both recursions)
    int32_t nseg_f, nseg_b;  // segments per (line, s): forward over [-S, n + L), backward over [-S, n)
    int32_t pad0;
    double B, a1, a2, a3;  // recursion coefficients (a_k = b_k / b0)
    double scale;          // sqrt(2 pi) beta: unit gain -> the Gaussian's mass
};

struct IirNlmArgs {
    PassDesc pass;        // samples in (a row pass: the transposed copy) and out
    const float* dist;    // distances written by snlm_iir_bwd_kernel for this pass
    uint32_t dist_bytes;
    int32_t nv;           // n + S
};

// Element (s, v) of a w or dist buffer for one lane's line.
struct DistIO {
    __amdgpu_buffer_rsrc_t r;
    int32_t base_b;  // line * 4
    int32_t pos_b;   // nlines * 4
    int32_t row_b;   // nv * nlines * 4 (one offset s)
    int32_t S;

    // The line's part of the offset goes in the per-lane offset register, the
    // (wave-uniform) offset and position part in the scalar one.
    __device__ __forceinline__ int uoff(int s, int u) const { return (s - 1) * row_b + (u + S) * pos_b; }
    __device__ __forceinline__ float load(int s, int u) const {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, base_b, uoff(s, u), 0));
    }
    __device__ __forceinline__ void store(int s, int u, float v) const {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, base_b, uoff(s, u), 0);
    }
};

__device__ __forceinline__ DistIO make_dist_io(const float* buf, uint32_t bytes, int line, int nlines, int nv, int S) {
    DistIO o;
    o.r = make_rsrc(buf, bytes);
    o.base_b = line * 4;
    o.pos_b = nlines * 4;
    o.row_b = nv * nlines * 4;
    o.S = S;
    return o;
}

// Workgroup t: group t % ngroups, segment k = (t / ngroups) % nseg, offset
// s = t / (ngroups * nseg) + 1 (waves of one group and offset run side by
// side and share the line's samples in L2).
struct IirWave {
    int group, k, s, lane, line, line0;
    bool active;
};

__device__ __forceinline__ IirWave iir_wave(const PassDesc& d, int nseg) {
    IirWave o;
    const int t = blockIdx.x;
    o.group = t % d.ngroups;
    o.k = (t / d.ngroups) % nseg;
    o.s = t / (d.ngroups * nseg) + 1;
    o.lane = threadIdx.x & (kLanes - 1);
    o.line0 = o.group * kLanes;
    o.active = o.line0 + o.lane < d.nlines;
    o.line = min(o.line0 + o.lane, d.nlines - 1);
    return o;
}

// Forward recursion of one segment: outputs w(v) for v in [a, b), a = -S + k
// seg, b = min(a + seg, n + L); the recursion starts at vs = max(a - W, -L)
// (W a multiple of 16, so away from the line's start every 16-step block is
// either all warm-up or all output).  Each lane streams its line's scaled
// samples through NPF register buffers (16 samples each, issued NPF chunks
// ahead) into an LDS ring of two chunks: chunk c (positions vs + 16c ..)
// lands in slots (16c mod 32) .. + 15, and the chunk in slots 0..15 is also
// copied to slots 32..47, so a block's 16 + s <= 32 samples sit at
// consecutive slots.  A block at v0 reads chunks v0 and v0 + 16; the chunk at
// v0 + 32 replaces chunk v0 once the block is done.
// Lanes past the last line repeat the last line's work and store its values
// to its addresses (the same bits), so no store needs a lane mask.
template <int NPF>
__global__ __launch_bounds__(kLanes) void snlm_iir_fwd_kernel(IirArgs a) {
    constexpr int C = kChunk;
    constexpr int RING = 32;  // slots of distinct positions: [v0, v0 + 32) in use
    static_assert(NPF >= 3, "two chunks are taken before the first step, the third in the loop");
    __shared__ float ring[(RING + C) * kLanes];  // ring[slot * 64 + lane]
    const PassDesc& d = a.pass;
    const IirWave wv = iir_wave(d, a.nseg_f);
    const int s = wv.s, lane = wv.lane;
    const LineIO io = make_io<false>(d, wv.line0, lane, nullptr);
    const DistIO wio = make_dist_io(a.w, a.w_bytes, wv.line, d.nlines, d.n + a.L + a.S, a.S);
    const float alpha = d.alpha;
    const double B = a.B, a1 = a.a1, a2 = a.a2, a3 = a.a3;
    const int L = a.L, n = d.n;
    const int out_a = -a.S + wv.k * a.seg;
    const int out_b = min(out_a + a.seg, n + L);
    const int vs = max(out_a - a.W, -L);

    // 16 samples from position p: plain offsets inside the line, reflected
    // ones near its ends
    auto load16 = [&](int p, float* v) {
        if (p >= 0 && p + C <= n && !io.f16) {
            const int base = p * io.in_pos_b;
#pragma unroll
            for (int t = 0; t < C; ++t)
                v[t] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(io.rin, io.in_base_b,
                                                                                     base + t * io.in_pos_b, 0));
        } else {
            io.template load<C>(p, v);
        }
    };
    float vb[NPF][C];
    int issued = vs;  // next position to load
    int taken = vs;   // positions below this are in the ring
#pragma unroll
    for (int q = 0; q < NPF; ++q) {
        load16(issued, vb[q]);
        issued += C;
    }
    auto take = [&](int q) {
        const int slot = (taken - vs) & (RING - 1);
#pragma unroll
        for (int t = 0; t < C; ++t) ring[(slot + t) * kLanes + lane] = alpha * vb[q][t];
        if (slot == 0) {
#pragma unroll
            for (int t = 0; t < C; ++t) ring[(RING + t) * kLanes + lane] = alpha * vb[q][t];
        }
        taken += C;
        load16(issued, vb[q]);
        issued += C;
    };
    take(0);
    take(1);  // chunks vs and vs + 16
    int v0 = vs;
    const float dd0 = ring[lane] - ring[s * kLanes + lane];
    double w1 = (double)(dd0 * dd0), w2 = w1, w3 = w1;
    auto fwd16 = [&]() {
        const int b = (v0 - vs) & (RING - 1);  // 0 or 16
        const float* rx = ring + b * kLanes + lane;
        const float* ry = rx + s * kLanes;
        const bool all_out = v0 >= out_a && v0 + C <= out_b;
        const bool none_out = v0 + C <= out_a || v0 >= out_b;
        const int off0 = wio.uoff(s, v0);
#pragma unroll
        for (int t = 0; t < C; ++t) {
            const float dd = rx[t * kLanes] - ry[t * kLanes];
            const double w = __builtin_fma(a1, w1, __builtin_fma(a2, w2, __builtin_fma(a3, w3, B * (double)(dd * dd))));
            w3 = w2;
            w2 = w1;
            w1 = w;
            if (all_out || (!none_out && v0 + t >= out_a && v0 + t < out_b))
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, (float)w), wio.r, wio.base_b,
                                                      off0 + t * wio.pos_b, 0);
        }
        v0 += C;
    };
    while (v0 < out_b) {
#pragma unroll
        for (int q = 0; q < NPF; ++q) {
            if (v0 < out_b) {
                fwd16();
                // buffers are taken in issue order: 2, 3, .., NPF-1, 0, 1, 2, ...
                take((q + 2) % NPF);  // the chunk at the new v0 + 16
            }
        }
    }
}

// Backward recursion of one segment: distances for u in [a, b), a = -S + k
// seg, b = min(a + seg, n); the recursion starts at min(b - 1 + W, n + L - 1)
// and reads w back C positions at a time through NB register buffers, so
// that NB - 1 chunks stay in flight while one is filtered (the kernel is
// bound by the bytes in flight: its grid gives only a few waves per SIMD).
// Stores as in the forward kernel (no lane masks).
template <int C>
__global__ __launch_bounds__(kLanes) void snlm_iir_bwd_kernel(IirArgs a) {
    constexpr int NB = 4;
    const PassDesc& d = a.pass;
    const IirWave wv = iir_wave(d, a.nseg_b);
    const int s = wv.s;
    const int S = a.S;
    const DistIO wio = make_dist_io(a.w, a.w_bytes, wv.line, d.nlines, d.n + a.L + S, S);
    const DistIO dio = make_dist_io(a.dist, a.dist_bytes, wv.line, d.nlines, d.n + S, S);
    const double B = a.B, a1 = a.a1, a2 = a.a2, a3 = a.a3;
    const double scale = a.scale;
    const int out_a = -S + wv.k * a.seg;
    const int out_b = min(out_a + a.seg, d.n);
    const int vtop = min(out_b - 1 + a.W, d.n + a.L - 1);
    double y1 = (double)wio.load(s, vtop), y2 = y1, y3 = y1;
    // w at top, top - 1, .., top - C + 1 (positions below out_a, never used,
    // read out_a's).  No branches around the loads or the stores below: the
    // compiler then counts them and waits only for the chunk it filters.
    auto load16 = [&](int top, float* dst) {
#pragma unroll
        for (int t = 0; t < C; ++t) dst[t] = wio.load(s, max(top - t, out_a));
    };
    float buf[NB][C];
#pragma unroll
    for (int q = 0; q < NB; ++q) load16(vtop - q * C, buf[q]);
    int top = vtop;
    bool more = true;
    while (more) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            if (!more) break;
            const int off0 = dio.uoff(s, top);
#pragma unroll
            for (int t = 0; t < C; ++t) {
                const double y =
                    __builtin_fma(a1, y1, __builtin_fma(a2, y2, __builtin_fma(a3, y3, B * (double)buf[q][t])));
                y3 = y2;
                y2 = y1;
                y1 = y;
                // positions outside [out_a, out_b) go past the buffer's
                // extent (its size as the uniform offset: line * 4 + size
                // stays below 2^32 as both are below 2^31), where the bounds
                // check drops the store
                const int so = (top - t >= out_a && top - t < out_b) ? off0 - t * dio.pos_b : (int)a.dist_bytes;
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, (float)(scale * y)), dio.r,
                                                      dio.base_b, so, 0);
            }
            more = top - C >= out_a;
            if (more) load16(top - NB * C, buf[q]);  // the chunk NB positions on
            top -= C;
        }
    }
}

// Transposed FP32 copy of a pass's input for the forward recursion of a pass
// whose lines are contiguous in memory: xt[p * nlines + line] = x(line, p).
// Reading lines across lanes touches one cache line per lane and sample; the
// copy lets every offset's forward wave read 64 lines' sample p as one
// 256-byte row.  Workgroup (four waves): 64 lines x 64 positions through an
// LDS tile (odd row stride: no bank conflicts either way).
struct IirTransposeArgs {
    PassDesc pass;
    float* xt;
    uint32_t xt_bytes;
};

template <int NPOS>
__global__ __launch_bounds__(4 * kLanes) void snlm_iir_transpose_kernel(IirTransposeArgs a) {
    static_assert(NPOS == kLanes, "one position per lane");
    __shared__ float tile[kLanes * (kLanes + 1)];
    const PassDesc& d = a.pass;
    const int lane = threadIdx.x & (kLanes - 1);
    const int wq = threadIdx.x / kLanes;  // wave q of 4: lines (and then positions) 16 q .. 16 q + 15
    const int line0 = blockIdx.x * kLanes;
    const int p0 = blockIdx.y * NPOS;
    const int p = min(p0 + lane, d.n - 1);
    // 16 lines' loads in flight per wave, then their LDS writes
    auto rows16 = [&](auto load) {
        float v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const LineIO io = make_io<false>(d, min(line0 + 16 * wq + i, d.nlines - 1), 0, nullptr);
            v[i] = load(io.rin, io.in_base_b + p * io.in_pos_b);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) tile[(16 * wq + i) * (kLanes + 1) + lane] = v[i];
    };
    if (d.in_f16)
        rows16([](__amdgpu_buffer_rsrc_t r, int off) {
            return (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
        });
    else
        rows16([](__amdgpu_buffer_rsrc_t r, int off) {
            return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
        });
    __syncthreads();
    const __amdgpu_buffer_rsrc_t r = make_rsrc(a.xt, a.xt_bytes);
    const int line = line0 + lane;
#pragma unroll
    for (int i = 16 * wq; i < 16 * wq + 16; ++i) {
        if (p0 + i < d.n && line < d.nlines)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, tile[lane * (kLanes + 1) + i]), r,
                                                  ((p0 + i) * d.nlines + line) * 4, 0, 0);
    }
}

// Samples [seg_a, seg_b) of one line from stored distances (seg_a a multiple
// of kChunk).  As run_segment with K = 0 for the samples: the window holds
// positions c0 .. c0 + C + S - 1, and pair (u, u+s) takes d = dist(s, u).
template <int S>
__device__ __forceinline__ void run_segment_dist(const PassDesc& d, const LineIO& io, const DistIO& dio,
                                                 int seg_a, int seg_b) {
    constexpr int C = kChunk;
    constexpr int NX = C + S;
    constexpr int NP = C + S;
    static_assert(S >= 1 && S <= kMaxS, "parameter range");
    const float alpha = d.alpha;
    const float inv_alpha = d.inv_alpha;
    const int nlast = d.n - 1;
    float xs[NX], P[NP], Q[NP], nx[C];

    int c0 = seg_a - C;
    io.template load<NX>(c0, xs);
#pragma unroll
    for (int j = 0; j < NX; ++j) xs[j] = alpha * xs[j];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        P[i] = xs[i];
        Q[i] = 1.0f;
    }
    io.issue_chunk(seg_a + S, nx);

    // ---- pre-chunk: pairs (u, u+s) with u in [seg_a - s, seg_a) ----
#pragma unroll
    for (int s = 1; s <= S; ++s) {
        __builtin_amdgcn_sched_barrier(0);
        float r[C];
#pragma unroll
        for (int i = C - s; i < C; ++i) r[i] = dio.load(s, c0 + i);
#pragma unroll
        for (int i = C - s; i < C; ++i)
            accumulate_pair<0>(xs, P, Q, i, s, __builtin_amdgcn_exp2f(-r[i]), false);
    }

    // distances of offset s for the chunk at c: positions past the line's end
    // (pairs whose both centres are past it) read the last stored one
    auto row = [&](int s, int c, float* dst) {
#pragma unroll
        for (int i = 0; i < C; ++i) dst[i] = dio.load(s, min(c + i, nlast));
    };
    float rc[C], rn[C];
    row(1, seg_a, rc);
    bool staged_store_last = false;  // the previous chunk ended with 4 tile stores
    for (c0 = seg_a;; c0 += C) {
        io.finish_chunk(c0 + S, nx, staged_store_last);
        advance_chunk<S, 0>(xs, P, Q, nx, alpha);
        const bool has_next = c0 + C < seg_b;
        if (has_next) io.issue_chunk(c0 + C + S, nx);
#pragma unroll
        for (int s = 1; s <= S; ++s) {
            // one offset at a time (bounds the loads in flight, and so the
            // registers); the next offset's distances (or the next chunk's
            // first) load while this offset's pairs are accumulated
            __builtin_amdgcn_sched_barrier(0);
            if (s < S)
                row(s + 1, c0, rn);
            else if (has_next)
                row(1, c0 + C, rn);
            // (the distance as stored: a recursive-filter value can be
            // slightly negative, and is not clamped)
#pragma unroll
            for (int i = 0; i < C; ++i) accumulate_pair<0>(xs, P, Q, i, s, __builtin_amdgcn_exp2f(-rc[i]), true);
            if (s < S || has_next) {
#pragma unroll
                for (int i = 0; i < C; ++i) rc[i] = rn[i];
            }
            // Complete this offset's sums here: otherwise the compiler sinks
            // every offset's arithmetic below the last loads and keeps all
            // S * 16 distances live at once.
#pragma unroll
            for (int i = 0; i + 3 < NP; i += 4)
                asm volatile("" ::"v"(P[i]), "v"(P[i + 1]), "v"(P[i + 2]), "v"(P[i + 3]), "v"(Q[i]), "v"(Q[i + 1]),
                             "v"(Q[i + 2]), "v"(Q[i + 3]));
        }
        float y[C];
        normalise(P, Q, inv_alpha, y);
        staged_store_last = io.store_chunk(c0, seg_b, y);
        if (!has_next) break;
    }
}

// Grid: ngroups * nseg workgroups of one wave, as the direct lifted pass.
// ROWS: the variant for lines contiguous in memory (the LDS transpose tile for
// the outputs, as the lifted pass's row variant; its samples come from the
// transposed copy, which every lane reads coalesced, so the input tile stays
// unused).
template <int S, bool ROWS>
__global__ __launch_bounds__(kLanes) void snlm_iir_nlm_kernel(IirNlmArgs a) {
    __shared__ __attribute__((aligned(16))) float tiles[ROWS ? kTileIn + kTileOut : 1];
    const PassDesc& d = a.pass;
    const int t = blockIdx.x;
    const int group = t % d.ngroups;
    const int seg_a = (t / d.ngroups) * d.seg_len;
    const int seg_b = min(seg_a + d.seg_len, d.n);
    const int lane = threadIdx.x & (kLanes - 1);
    const int line0 = group * kLanes;
    const LineIO io = make_io<ROWS>(d, line0, lane, tiles);
    const int line = min(line0 + lane, d.nlines - 1);
    const DistIO dio = make_dist_io(a.dist, a.dist_bytes, line, d.nlines, a.nv, S);
    run_segment_dist<S>(d, io, dio, seg_a, seg_b);
}

}  // namespace snlm
