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
// distance between the patches at u and u+s, and exp2 of minus it the weight
// of the pair (u, u+s) in eq. 1dNLM.
//
// Positions are grouped in blocks of 16: block j holds [16 j, 16 j + 16);
// blocks -1 .. jhi = (n + L - 1) / 16 cover everything a pass needs.  One pass
// runs two kernels (three for lines that are contiguous in memory, which
// first make a transposed copy of their input with snlm_iir_transpose_kernel
// and read that instead):
//   snlm_iir_fwd_kernel<S>  one workgroup of S waves per (64 lines, segment),
//       wave s runs the forward recursion of offset s from a sample ring the
//       waves share, and stores only its state (w'(p-1), w'(p-2), w'(p-3)) in
//       FP64 at the start p = max(16 j, -L) of every block: 24 bytes per 16
//       samples instead of the 64 of the values themselves.
//   snlm_iir_nlm_kernel<S>  one workgroup of S waves per (64 lines, segment
//       of outputs); wave s owns offset s.  It walks the segment's blocks
//       from the top down: each wave recomputes its block of w from the
//       stored state (the same operations as the forward kernel, so the same
//       values), runs the backward recursion over it and writes the block's
//       weights to LDS; then all waves gather the outputs of the block above,
//       whose pairs are now all weighted: y(p) = (x(p) + sum_s [w(p, p+s)
//       x(p+s) + w(p-s, p) x(p-s)]) / (1 + sum_s [w(p, p+s) + w(p-s, p)]).
//       Neither w nor the distances ever reach memory; one exp per pair.
// A segment of either recursion starts W samples before its first output
// (forward) or after its last (backward), from the steady state of the value
// found there, or at the line's own start where that comes first.  The
// recursion forgets its start like rho^t, rho the largest pole modulus, and W
// is chosen with rho^W <= 1e-12, so segments reproduce the whole-line
// recursion far below FP32 resolution.  Segment lengths depend on the job
// only, never on the device.
//
// Both recursions run on scaled values, w' = w / B forward and y'' = y / B^2
// backward: w'(v) = D(v) + a1 w'(v-1) + a2 w'(v-2) + a3 w'(v-3), y''(v) =
// w'(v) + a1 y''(v+1) + ..., the same filter without a multiply by B per step
// (the steady states become D / B and w' / B, the distance sqrt(2 pi) beta B^2
// y'').  The state and coefficients are FP64: for wide kernels the poles
// approach 1 and B ~ 1.6 / (0.42 q^3) is small, so FP32 rounding of the
// coefficients alone would move the DC gain by ~1e-7 / B (0.2% at beta = 20)
// and every step's rounding would be amplified up to 1 / B times.  FP64 FMAs
// issue at half the FP32 rate on this chip.  Lifted samples, distances and
// weights are FP32.
//
// Stored states (line fastest: every access of a wave is one 512-byte row):
//   ck[(((s - 1) * nblk + j + 1) * 3 + k) * nlines + line],  k = 0, 1, 2 for
//   w'(p-1), w'(p-2), w'(p-3);  j in [-1, nblk - 2]
#pragma once

#include "snlm_device.hpp"

namespace snlm {

struct IirArgs {
    PassDesc pass;         // samples in (a row pass: the transposed copy), n, alpha, outputs
    double* ck;            // forward states at block starts
    uint32_t ck_bytes;
    int32_t S;             // search half-width (offsets 1..S)
    int32_t L;             // the recursion runs L samples beyond each end of the line
    int32_t W;             // warm-up of a segment that does not start at the line's start (multiple of 16)
    int32_t nblk;          // blocks per (offset, line): -1 .. nblk - 2
    int32_t fwd_blocks;    // blocks per forward segment
    int32_t nseg_f;        // forward segments per (line group, offset)
    int32_t seg;           // outputs per segment of the NLM kernel (multiple of 16)
    int32_t pad0;
    double inv_B, a1, a2, a3;  // 1 / B and the recursion coefficients a_k = b_k / b0
    double scale;              // sqrt(2 pi) beta B^2: the distance from y''
};

typedef unsigned int iir_u32x2 __attribute__((ext_vector_type(2)));

// The stored states of one lane's line: the line's part of the offset goes in
// the per-lane offset register, the (wave-uniform) offset / block / word part
// in the scalar one.
struct CkIO {
    __amdgpu_buffer_rsrc_t r;
    int32_t base_b;  // line * 8
    int32_t row_b;   // nlines * 8
    int32_t nblk;

    __device__ __forceinline__ int off(int s, int j, int k) const { return (((s - 1) * nblk + j + 1) * 3 + k) * row_b; }
    __device__ __forceinline__ double load(int s, int j, int k) const {
        const iir_u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, base_b, off(s, j, k), 0);
        return __builtin_bit_cast(double, v);
    }
    // a store that, unless keep, goes past the buffer's extent (its size as
    // the uniform offset: line * 8 + size stays below 2^32 as both are below
    // 2^31), where the bounds check drops it
    __device__ __forceinline__ void store_or_drop(int s, int j, int k, double x, bool keep, uint32_t bytes) const {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(iir_u32x2, x), r, base_b,
                                              keep ? off(s, j, k) : (int)bytes, 0);
    }
};

__device__ __forceinline__ CkIO make_ck_io(const double* buf, uint32_t bytes, int line, int nlines, int nblk) {
    CkIO o;
    o.r = make_rsrc(buf, bytes);
    o.base_b = line * 8;
    o.row_b = nlines * 8;
    o.nblk = nblk;
    return o;
}

// One step of the scaled recursion (forward over D, or backward over w'):
// the newest state word enters last, so only one FMA waits for the previous
// step.
__device__ __forceinline__ double iir_step(double a1, double a2, double a3, double in, double w1, double w2,
                                           double w3) {
    return __builtin_fma(a1, w1, __builtin_fma(a2, w2, __builtin_fma(a3, w3, in)));
}

// The lifted input of the forward recursion from two scaled samples.
__device__ __forceinline__ double iir_lift(float xa, float xb) {
    const float dd = xa - xb;
    return (double)(dd * dd);
}

// Forward recursion of one segment, blocks [ja, jb) with ja = -1 + k
// fwd_blocks, for all S offsets: workgroup (group, segment) of S waves, wave
// q owns offset s = q + 1 and stores its state at the start of each block of
// the segment.  The recursion starts at vs = max(16 ja - W, -L) and runs in
// steps of 16 from g0 = vs rounded down to a multiple of 16 (positions below
// vs are skipped), so that every group of 16 steps begins at a block start.
// The waves share one LDS ring of the line's scaled samples: chunk c
// (positions g0 + 16 c ..) sits at slots 16 c mod 64 (slots 64..79 repeat
// 0..15), loaded once for all offsets, positions t = q, q + S, .. of a chunk
// by wave q, two steps ahead through registers.  Step i writes chunk i + 2
// (over chunk i - 2, last read in step i - 2), reads chunks i and i + 1, and
// ends with a barrier; every wave runs the same steps.
// Lanes past the last line repeat the last line's work and store its values
// to its addresses (the same bits), so no store needs a lane mask.
template <int S, bool F16>
__global__ __launch_bounds__(kLanes* S) void snlm_iir_fwd_kernel(IirArgs a) {
    constexpr int C = kChunk;
    constexpr int NR = (C + S - 1) / S;  // ring positions per wave and chunk
    static_assert(S >= 1 && S <= kMaxS, "parameter range");
    __shared__ float ring[80 * kLanes];  // ring[slot * 64 + lane]
    const PassDesc& d = a.pass;
    const int group = blockIdx.x % d.ngroups;
    const int k = blockIdx.x / d.ngroups;
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int lane = threadIdx.x & (kLanes - 1);
    const int s = q + 1;
    const int line0 = group * kLanes;
    const int line = min(line0 + lane, d.nlines - 1);
    const LineIO io = make_io<false>(d, line0, lane, nullptr);
    const CkIO ck = make_ck_io(a.ck, a.ck_bytes, line, d.nlines, a.nblk);
    const float alpha = d.alpha;
    const double a1 = a.a1, a2 = a.a2, a3 = a.a3;
    const int n = d.n;
    const int ja = -1 + k * a.fwd_blocks;
    const int jb = min(ja + a.fwd_blocks, a.nblk - 1);
    const int vs = max(C * ja - a.W, -a.L);
    const int g0 = vs & ~(C - 1);

    // this wave's share of chunk c, as the loaded bits
    auto load_part = [&](int c, unsigned* xn) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (q + S * r >= C) continue;
            const int p = g0 + C * c + q + S * r;
            const int so = ((unsigned)p < (unsigned)n ? p : refl(p, n)) * io.in_pos_b;
            if constexpr (F16)
                xn[r] = __builtin_amdgcn_raw_buffer_load_b16(io.rin, io.in_base_b, so, 0);
            else
                xn[r] = __builtin_amdgcn_raw_buffer_load_b32(io.rin, io.in_base_b, so, 0);
        }
    };
    auto put_part = [&](int c, const unsigned* xn) {
        const int slot = (C * c) & 63;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int t = q + S * r;
            if (t >= C) continue;
            const float x = F16 ? (float)__builtin_bit_cast(_Float16, (unsigned short)xn[r]) : __builtin_bit_cast(float, xn[r]);
            ring[(slot + t) * kLanes + lane] = alpha * x;
            if (slot == 0) ring[(64 + t) * kLanes + lane] = alpha * x;
        }
    };
    unsigned xa[NR], xb[NR];
    load_part(0, xa);
    load_part(1, xb);
    put_part(0, xa);
    put_part(1, xb);
    load_part(2, xa);
    load_part(3, xb);
    __syncthreads();
    const int i0 = vs - g0;
    const double d0 = iir_lift(ring[i0 * kLanes + lane], ring[(i0 + s) * kLanes + lane]) * a.inv_B;
    double w1 = d0, w2 = d0, w3 = d0;  // the steady state of D(vs)
    const int jg0 = g0 >> 4;
    const int m = jb - jg0;  // group starts whose state the segment stores: 0 .. m - 1
    // group i: store the state at its start (block jg0 + i, when it is one of
    // the segment's; the others go past the buffer, where the bounds check
    // drops them), put chunk i + 2 into the ring and load chunk i + 4, run
    // the 16 steps (positions below vs skipped), barrier
    auto group_step = [&](int i, unsigned* xr_regs) {
        const int j = jg0 + i;
        const bool mine = j >= ja && j < jb;
        const int jc = min(max(j, ja), jb - 1);
        ck.store_or_drop(s, jc, 0, w1, mine, a.ck_bytes);
        ck.store_or_drop(s, jc, 1, w2, mine, a.ck_bytes);
        ck.store_or_drop(s, jc, 2, w3, mine, a.ck_bytes);
        put_part(i + 2, xr_regs);
        load_part(i + 4, xr_regs);
        const float* rx = ring + ((C * i) & 63) * kLanes + lane;
        const float* ry = rx + s * kLanes;
        const int skip = max(vs - (g0 + C * i), 0);
#pragma unroll
        for (int t = 0; t < C; ++t) {
            if (t < skip) continue;
            const double w = iir_step(a1, a2, a3, iir_lift(rx[t * kLanes], ry[t * kLanes]), w1, w2, w3);
            w3 = w2;
            w2 = w1;
            w1 = w;
        }
        __syncthreads();
    };
    // groups 0 .. m - 2 run; the state at the start of group m - 1 is the
    // last one stored (two groups per iteration: the register buffers
    // alternate)
    int i = 0;
    for (; i + 1 < m - 1; i += 2) {
        group_step(i, xa);
        group_step(i + 1, xb);
    }
    if (i < m - 1) {
        group_step(i, xa);
        ++i;
    }
    const int j = jg0 + i;
    const bool mine = j >= ja && j < jb;
    const int jc = min(max(j, ja), jb - 1);
    ck.store_or_drop(s, jc, 0, w1, mine, a.ck_bytes);
    ck.store_or_drop(s, jc, 1, w2, mine, a.ck_bytes);
    ck.store_or_drop(s, jc, 2, w3, mine, a.ck_bytes);
}

// LDS of the NLM kernel: the sample ring (96 slots of 64 lanes: positions
// mod 64, slots 64..95 repeating 0..31) and the weights of S offsets for two
// blocks (positions mod 32).
constexpr int kIirXSlots = 96;

// Workgroup t: group t % ngroups, segment t / ngroups of seg outputs [a0, b0).
// Wave q owns offset s = q + 1.  Blocks jbot = a0 / 16 - 1 (weights of the
// pairs that reach into the segment from below) .. jw = (b0 - 1) / 16 carry
// weights; the backward recursion starts at vtop = min(16 (jw + 1) + W - 1,
// n + L - 1), W samples above the segment's top block (or at the line's
// end), so the blocks up to jt = vtop / 16 are its warm-up.  Step j (from jt
// down to jbot):
//   1. the stored state of block j - 1 starts loading; the samples of block
//      j - 1 (loaded during the previous step, positions t = q, q + S, .. of
//      the block by wave q) go into the ring, and those of block j - 2 start
//      loading;
//   2. each wave recomputes w' over block j from its stored state, then runs
//      the backward recursion down the block and (j <= jw) writes the weights
//      exp2(-sqrt(2 pi) beta B^2 y'') of its offset to LDS;
//   3. barrier; the waves gather the outputs of block j + 1 (when it lies in
//      the segment): positions t = q, q + S, .. of the block go to wave q;
//   4. barrier (the next step overwrites the weights of block j + 1 and the
//      samples of block j + 3).
// Step j reads samples of blocks j .. j + 2 (positions up to 16 j + 47 from
// ring slot 16 j mod 64, hence the 32 repeated slots) and weights of blocks
// j and j + 1.  Every wave runs the same steps, so the barriers match.
template <int S>
__global__ __launch_bounds__(kLanes* S) void snlm_iir_nlm_kernel(IirArgs a) {
    constexpr int C = kChunk;
    constexpr int NR = (C + S - 1) / S;  // ring positions per wave and block
    static_assert(S >= 1 && S <= kMaxS, "parameter range");
    __shared__ float xr[kIirXSlots * kLanes];     // a x(v) at slot (v mod 64) * 64 + lane
    __shared__ float wt[S * 2 * C * kLanes];      // w(u, u+s) at ((s - 1) * 32 + u mod 32) * 64 + lane
    const PassDesc& d = a.pass;
    const int group = blockIdx.x % d.ngroups;
    const int kseg = blockIdx.x / d.ngroups;
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int lane = threadIdx.x & (kLanes - 1);
    const int s = q + 1;
    const int line0 = group * kLanes;
    const int line = min(line0 + lane, d.nlines - 1);
    const LineIO io = make_io<false>(d, line0, lane, nullptr);
    const CkIO ck = make_ck_io(a.ck, a.ck_bytes, line, d.nlines, a.nblk);
    const float alpha = d.alpha, inv_alpha = d.inv_alpha;
    const double a1 = a.a1, a2 = a.a2, a3 = a.a3, scale = a.scale;
    const int n = d.n, L = a.L;
    const int a0 = kseg * a.seg;
    const int b0 = min(a0 + a.seg, n);
    const int jw = (b0 - 1) >> 4;
    const int jbot = (a0 >> 4) - 1;
    const int vtop = min(C * (jw + 1) + a.W - 1, n + L - 1);
    const int jt = vtop >> 4;

    // this wave's share of a block's samples: positions q + S r, kept as the
    // loaded bits (FP16 samples convert when they enter the ring, so no load
    // is waited for before then)
    unsigned xn[NR];
    auto load_part = [&](int j) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int p = C * j + q + S * r;
            if (q + S * r < C) {
                int vo = io.in_base_b, so = p * io.in_pos_b;
                if (p < 0 || p >= n) {
                    vo += refl(p, n) * io.in_pos_b;
                    so = 0;
                }
                xn[r] = io.f16 ? (unsigned)__builtin_amdgcn_raw_buffer_load_b16(io.rin, vo, so, 0)
                               : __builtin_amdgcn_raw_buffer_load_b32(io.rin, vo, so, 0);
            }
        }
    };
    auto put_part = [&](int j) {
        const int slot = (C * j) & 63;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int t = q + S * r;
            if (t < C) {
                const float x = io.f16 ? (float)__builtin_bit_cast(_Float16, (unsigned short)xn[r])
                                       : __builtin_bit_cast(float, xn[r]);
                xr[(slot + t) * kLanes + lane] = alpha * x;
                if (slot < 32) xr[(64 + slot + t) * kLanes + lane] = alpha * x;
            }
        }
    };
    load_part(jt + 1);
    put_part(jt + 1);
    load_part(jt);
    put_part(jt);
    load_part(jt - 1);
    double c0 = ck.load(s, jt, 0), c1 = ck.load(s, jt, 1), c2 = ck.load(s, jt, 2);
    double y1 = 0.0, y2 = 0.0, y3 = 0.0;  // backward state
    float* wq = wt + (q * 2 * C) * kLanes + lane;
    __syncthreads();

    for (int j = jt; j >= jbot; --j) {
        const int base = C * j;
        const int t_lo = max(0, -L - base);
        const int t_hi = min(C - 1, vtop - base);
        const bool full = t_lo == 0 && t_hi == C - 1;
        const int xb = base & 63;  // ring slot of position base
        float* wblk = wq + (base & 31) * kLanes;  // this offset's weight of position base
        // ---- 1. state and samples in flight
        double w1 = c0, w2 = c1, w3 = c2;
        if (j > jbot) {
            c0 = ck.load(s, j - 1, 0);
            c1 = ck.load(s, j - 1, 1);
            c2 = ck.load(s, j - 1, 2);
            put_part(j - 1);  // its slots held block j + 3, last read by the previous step's gather
            if (j - 1 > jbot) load_part(j - 2);
        }
        // ---- 2. w' over the block, then backward
        const float* rx = xr + xb * kLanes + lane;  // a x(base + t) at rx[t * 64]
        const float* ry = rx + s * kLanes;          // a x(base + t + s)
        double wv[C];
        if (full) {
#pragma unroll
            for (int t = 0; t < C; ++t) {
                const double w = iir_step(a1, a2, a3, iir_lift(rx[t * kLanes], ry[t * kLanes]), w1, w2, w3);
                w3 = w2;
                w2 = w1;
                w1 = w;
                wv[t] = w;
            }
            if (j == jt) y1 = y2 = y3 = wv[C - 1] * a.inv_B;  // the steady state of w'(vtop)
            if (j <= jw) {
#pragma unroll
                for (int t = C - 1; t >= 0; --t) {
                    const double y = iir_step(a1, a2, a3, wv[t], y1, y2, y3);
                    y3 = y2;
                    y2 = y1;
                    y1 = y;
                    wblk[t * kLanes] = __builtin_amdgcn_exp2f(-(float)(scale * y));
                }
            } else {
#pragma unroll
                for (int t = C - 1; t >= 0; --t) {
                    const double y = iir_step(a1, a2, a3, wv[t], y1, y2, y3);
                    y3 = y2;
                    y2 = y1;
                    y1 = y;
                }
            }
        } else {
            // a block cut by the line's run-in or by the recursion's start
#pragma unroll
            for (int t = 0; t < C; ++t) {
                wv[t] = 0.0;
                if (t < t_lo || t > t_hi) continue;
                const double w = iir_step(a1, a2, a3, iir_lift(rx[t * kLanes], ry[t * kLanes]), w1, w2, w3);
                w3 = w2;
                w2 = w1;
                w1 = w;
                wv[t] = w;
            }
#pragma unroll
            for (int t = C - 1; t >= 0; --t) {
                if (t < t_lo || t > t_hi) continue;
                if (j == jt && t == t_hi) y1 = y2 = y3 = wv[t] * a.inv_B;
                const double y = iir_step(a1, a2, a3, wv[t], y1, y2, y3);
                y3 = y2;
                y2 = y1;
                y1 = y;
                if (j <= jw) wblk[t * kLanes] = __builtin_amdgcn_exp2f(-(float)(scale * y));
            }
        }
        __syncthreads();
        // ---- 3. outputs of block j + 1: this wave's positions together (a
        // position past the block's end repeats its last one, unstored), so
        // their LDS reads overlap
        if (j + 1 <= jw) {
            const float* xg = xr + (xb + C) * kLanes + lane;  // a x(16 (j + 1) + t) at xg[t * 64]
            float P[NR], Q[NR];
            int tt[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                tt[r] = min(q + S * r, C - 1);
                P[r] = xg[tt[r] * kLanes];
                Q[r] = 1.0f;
            }
#pragma unroll
            for (int o = 1; o <= S; ++o) {
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const int p = base + C + tt[r];
                    const float* xp = xg + tt[r] * kLanes;
                    const float wr = wt[((o - 1) * 2 * C + (p & 31)) * kLanes + lane];        // pair (p, p + o)
                    const float wl = wt[((o - 1) * 2 * C + ((p - o) & 31)) * kLanes + lane];  // pair (p - o, p)
                    P[r] = __builtin_fmaf(wr, xp[o * kLanes], P[r]);
                    P[r] = __builtin_fmaf(wl, xp[-o * kLanes], P[r]);
                    Q[r] += wr;
                    Q[r] += wl;
                }
            }
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int t = q + S * r;
                const int p = base + C + t;
                if (t < C && p < b0) io.store(p, (P[r] * __builtin_amdgcn_rcpf(Q[r])) * inv_alpha);
            }
        }
        __syncthreads();
    }
}

// Transposed FP32 copy of a pass's input for the recursions of a pass whose
// lines are contiguous in memory: xt[p * nlines + line] = x(line, p).  Reading
// lines across lanes touches one cache line per lane and sample; the copy
// lets every wave read 64 lines' sample p as one 256-byte row.  Workgroup
// (four waves): 64 lines x 64 positions through an LDS tile (odd row stride:
// no bank conflicts either way).
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

}  // namespace snlm
