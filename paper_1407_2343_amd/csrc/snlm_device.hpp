// Device side of the separable PatchLift non-local means library (gfx950).
//
// One pass of separable NLM (Sec. 3) filters a set of independent lines (the
// rows or the columns of an image) with the 1D NLM of eq. 1dNLM.  Here one
// lane owns one line and walks a segment of it serially, in chunks of kChunk
// samples; a wave therefore filters 64 adjacent lines at once, with no
// cross-lane traffic at all.  For the column pass the 64 lanes read 64
// adjacent columns (coalesced); for the row pass each lane reads its own row.
//
// Per lane, per offset s = 1..S and centre u of the chunk, the pair (u, u+s) is
// visited once (the band symmetry of Sec. 2.1: w(u,u+s) = w(u+s,u)):
//   lift     D_s(v) = (a x(v) - a x(v+s))^2, a = sqrt(log2 e)/h (difference form
//            of eqs. tensor/convn/lift; no cancellation of the tensor form)
//   window   box:   R_s(u) = sum_{k=-K..K} D_s(u+k), carried as the recursion of
//                   eq. recursion: R_s(u) = R_s(u-1) + D_s(u+K) - D_s(u-K-1),
//                   re-initialised directly at line-relative positions
//                   u = -S (mod kChunk) ("block restart"), or never ("plain"),
//                   or carried with Kahan compensation ("kahan");
//            gauss: R_s(u) = sum_k g(k) D_s(u+k), an exact (2K+1)-tap FIR.
//   weight   w = exp2(-R_s(u)) = exp(-d2/h^2)            (eq. 1dNLM)
//   average  P(u) += w x(u+s), Q(u) += w, P(u+s) += w x(u), Q(u+s) += w
//            (P, Q start at x(u), 1: the s = 0 term), y(u) = P(u)/Q(u).
//
// Lines are extended by half-sample symmetric reflection.  A segment
// [a, b) of a line (a a multiple of kChunk) needs the pairs (u, u+s) with
// u in [a-S, a) for its first centres; those are computed in a "pre-chunk"
// that repeats, operation for operation, what the previous chunk would have
// done for them.  Every output therefore has bit-identical arithmetic however
// a line is split into segments (plain launch, batched launch, any tuned
// segment length).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "snlm_lift.hpp"

namespace snlm {

constexpr int kMaxS = 16;   // search half-width limit (S <= kChunk)
constexpr int kMaxK = 8;    // patch half-width limit
constexpr int kLanes = 64;  // lines per wave
constexpr uint32_t kRsrcWord3 = 0x00020000u;  // raw buffer, 32-bit data, gfx9 family

// One pass over the lines of one image.
struct PassDesc {
    const void* in;        // line data (FP32, or FP16 when in_f16)
    float* out;            // FP32 output
    uint32_t in_bytes;     // extent of the input buffer (bounds for buffer ops)
    uint32_t out_bytes;    // extent of the output buffer
    int32_t nlines;        // number of lines
    int32_t n;             // samples per line
    int32_t in_line;       // element stride between lines (input)
    int32_t in_pos;        // element stride between samples of a line (input)
    int32_t out_line;      // element stride between lines (output)
    int32_t out_pos;       // element stride between samples (output)
    int32_t in_f16;        // input stored as FP16
    int32_t restart;       // 1: block-restarted running sums (box only)
    int32_t seg_len;       // samples per segment (multiple of kChunk)
    int32_t nseg;          // segments per line = ceil(n / seg_len)
    int32_t ngroups;       // groups of 64 lines = ceil(nlines / 64)
    int32_t split;         // 0: line l starts at l * in_line; else at (l / split) * in_outer
                           // + (l % split) * in_line (and likewise for the output)
    int32_t in_outer;      // element stride between blocks of `split` lines (input)
    int32_t out_outer;     // element stride between blocks of `split` lines (output)
    float alpha;           // lift scale a = sqrt(log2 e) / h  (2^-64 when h = inf)
    float inv_alpha;       // 1 / a
    float taps[kMaxK + 1]; // Gaussian taps g(0..K) (g(0) = 1)
    int32_t pad0;
    // Whole-line running sums (plain or Kahan) cut into segments: the state of
    // each offset's recursion at the start of every segment after the first,
    // carry[((seg - 1) * S + s - 1) * nlines + line] (Kahan: the compensations
    // follow, (nseg - 1) * S * nlines further on).  nullptr otherwise.
    const float* carry;
};

// A batch: jobs, each with two passes, and a flat list of tiles.  A tile is
// the samples [a, b) of the 64 lines of one group of one pass of one job (a
// a multiple of kChunk).  Tiles of every first pass come before tiles of any
// second pass.
struct BatchJob {
    PassDesc pass[2];
    int32_t tiles[2];      // number of tiles of each pass of this job
};

// Tile t belongs to the first pass when t < BatchHeader::ntiles_first.
struct BatchTile {
    uint32_t job;
    int32_t group;
    int32_t a, b;
};

struct BatchHeader {
    int32_t njobs;
    int32_t ntiles_first;  // tiles of all first passes
    int32_t ntiles;        // all tiles
    uint32_t spin_limit;   // bound on dependency polls before giving up
};

// Kernel arguments.
// * direct (hdr == nullptr): grid = ngroups * nseg workgroups of one wave;
//   workgroup t filters segment t / ngroups of group t % ngroups.
// * static batch (worker_first != nullptr): workgroup k filters the tiles
//   worker_first[k] .. worker_first[k+1] - 1 in order (the host cuts the work
//   of the launch into equal shares, one per workgroup).
// * claimed batch: persistent workgroups claim tiles [tile_lo, tile_hi) with
//   an atomic counter; with wait, second-pass tiles wait for their job's
//   first-pass tiles (per-job counters).
struct KernelArgs {
    PassDesc direct;
    const BatchHeader* hdr;
    const BatchJob* jobs;
    const BatchTile* tiles;
    const uint32_t* worker_first;
    uint32_t* counters;        // [1 + j] finished first-pass tiles of job j
    uint32_t* claim;           // claim counter of this launch
    uint32_t* status;          // set non-zero when a dependency wait gives up
    int32_t tile_lo, tile_hi;  // tiles [lo, hi) handled by this launch (claimed mode)
    int32_t wait;              // second-pass tiles wait for their job's first pass
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                             (int)kRsrcWord3);
}

// Half-sample symmetric reflection into [0, n) (period 2n).  The position is
// the same for every lane of a wave, so this runs on the scalar unit.
__device__ __forceinline__ int refl(int p, int n) {
    while ((unsigned)p >= (unsigned)n) p = p < 0 ? -1 - p : 2 * n - 1 - p;
    return p;
}

constexpr int kStage = kChunk + 1;   // LDS row stride of the output tile (odd: no bank conflicts)
constexpr int kRowF32 = 20;          // input tile: floats per line (16 + up to 3 of alignment)
constexpr int kRowF16 = 24;          // input tile: halves per line (16 + up to 7 of alignment)
constexpr int kVecF32 = 5;           // 16-byte loads per lane for an FP32 input tile
constexpr int kVecF16 = 3;           // 16-byte loads per lane for an FP16 input tile
constexpr int kTileIn = kLanes * kRowF32;   // floats of LDS for the input tile
constexpr int kTileOut = kLanes * kStage;   // floats of LDS for the output tile
// 16-byte vectors per line that hold COUNT consecutive FP32 samples starting
// anywhere in the first vector.
constexpr int win_vectors(int count) { return (count + 6) / 4; }
// LDS floats of a row kernel: the chunk tiles, then a region for the
// pre-chunk's sample window of COUNT samples per line (so that the first
// chunk's loads can fly while the window is read).
constexpr int row_lds_floats(int count) { return kTileIn + kTileOut + kLanes * 4 * win_vectors(count); }
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Reinterprets a 32-bit word as a float.  Vector elements must pass through a
// scalar first: __builtin_bit_cast applied to an element expression of an
// ext_vector_type reads element 0 whatever the index.
__device__ __forceinline__ float as_float(unsigned u) { return __builtin_bit_cast(float, u); }

// Loads and stores of one lane's line.  Chunks of kChunk samples of lines that
// are contiguous in memory (the row pass) go through an LDS transpose tile:
// the wave fetches its 64 lines with 4-element vector loads from 4-element
// aligned addresses (each line's first sample may sit anywhere inside its
// first vector), and writes results back the same way, instead of every lane
// touching its own cache line with each 4-byte access.
struct LineIO {
    __amdgpu_buffer_rsrc_t rin, rout;
    int32_t in_base_b;   // byte offset of this lane's line (input)
    int32_t out_base_b;  // byte offset of this lane's line (output)
    int32_t in_pos_b;    // byte stride between samples (input)
    int32_t out_pos_b;   // byte stride between samples (output)
    int32_t in_line;     // element stride between lines (input)
    int32_t out_line;    // element stride between lines (output)
    int32_t line0;       // first line of this wave
    int32_t nlines;
    int32_t lane;
    int32_t n;
    uint32_t out_bytes;  // extent of the output buffer
    bool f16;
    bool stage_in;       // lines contiguous in the input: use the LDS tile
    bool stage_out;      // lines contiguous and 16-byte aligned in the output
    float* tile_in;      // input tile (kTileIn floats of LDS)
    float* tile_out;     // output tile (kTileOut floats of LDS)
    float* tile_win;     // pre-chunk window region (row kernels)

    // count samples starting at position p (reflected), into v[0..count)
    // (the lane's line start is the per-lane offset, the position the
    // wave-uniform one; samples inside the line need no reflection)
    // sample at per-lane byte offset vo plus uniform byte offset so
    __device__ __forceinline__ float load_at(int vo, int so) const {
        if (f16) {
            const unsigned short bits = __builtin_amdgcn_raw_buffer_load_b16(rin, vo, so, 0);
            return (float)__builtin_bit_cast(_Float16, bits);
        }
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rin, vo, so, 0));
    }
    template <int COUNT>
    __device__ __forceinline__ void load(int p, float* v) const {
        if (p >= 0 && p + COUNT <= n) {
#pragma unroll
            for (int t = 0; t < COUNT; ++t) v[t] = load_at(in_base_b, (p + t) * in_pos_b);
        } else {
#pragma unroll
            for (int t = 0; t < COUNT; ++t) v[t] = load_at(in_base_b + refl(p + t, n) * in_pos_b, 0);
        }
    }

    // The pre-chunk's sample window: COUNT samples from position p into v.
    // Rows inside the line go through the LDS window region with 16-byte
    // loads along each row, instead of COUNT per-lane loads that touch a
    // cache line per lane each.  start_window issues the loads;
    // finish_window waits for them (the first chunk's five tile loads,
    // issued in between, may still fly) and reads them out.
    template <int COUNT>
    __device__ __forceinline__ bool window_staged(int p) const {
        return stage_in && !f16 && p >= 0 && p + COUNT <= n;
    }
    template <int COUNT>
    __device__ __forceinline__ void start_window(int p) const {
        constexpr int V = win_vectors(COUNT);
        typedef __attribute__((address_space(3))) void* lds_ptr;
        // load j = lane + 64 r covers line j / V, vector j % V of that line,
        // and lands at LDS byte 16 j of the window region
#pragma unroll
        for (int r = 0; r < V; ++r) {
            const int j = lane + 64 * r;
            const int line = min(line0 + j / V, nlines - 1);
            const int e = ((line * in_line + p) & ~3) + 4 * (j % V);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rin, (lds_ptr)(tile_win + 256 * r), 16, e * 4, 0, 0, 0);
        }
    }
    template <int COUNT>
    __device__ __forceinline__ void finish_window(int p, float* v, bool five_loads_after) const {
        constexpr int V = win_vectors(COUNT);
        if (five_loads_after)
            __builtin_amdgcn_s_waitcnt(0x0F75);  // vmcnt(5): the first chunk's tile loads may fly
        else
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        __syncthreads();
        const int line = min(line0 + lane, nlines - 1);
        const int m = (line * in_line + p) & 3;
#pragma unroll
        for (int t = 0; t < COUNT; ++t) v[t] = tile_win[lane * 4 * V + m + t];
    }

    // Whether the chunk of samples [p, p + kChunk) goes through the LDS tile.
    __device__ __forceinline__ bool chunk_staged(int p) const {
        return stage_in && p >= 0 && p + kChunk <= n;
    }

    // First half of a chunk load: start the global loads.  Unstaged: into v.
    // Staged: 16-byte loads that write LDS directly (no registers in flight).
    // The tile holds 64 lines of kRowF32 floats (or kRowF16 halves) starting
    // at each line's aligned element (line * in_line + p) & ~3 (& ~7 for FP16);
    // load j = lane + 64 r covers line j / V, vector j % V of that line, and
    // lands at LDS byte 16 j.  Reads past a line's end stay inside the buffer
    // or return 0 (buffer bounds) and are never used.
    __device__ __forceinline__ void issue_chunk(int p, float* v) const {
        if (!chunk_staged(p)) {
            load<kChunk>(p, v);
            return;
        }
        typedef __attribute__((address_space(3))) void* lds_ptr;
        if (f16) {
#pragma unroll
            for (int r = 0; r < kVecF16; ++r) {
                const int j = lane + 64 * r;
                const int line = min(line0 + j / 3, nlines - 1);
                const int e = ((line * in_line + p) & ~7) + 8 * (j % 3);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rin, (lds_ptr)(tile_in + 256 * r), 16, e * 2, 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int r = 0; r < kVecF32; ++r) {
                const int j = lane + 64 * r;
                const int line = min(line0 + j / 5, nlines - 1);
                const int e = ((line * in_line + p) & ~3) + 4 * (j % 5);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rin, (lds_ptr)(tile_in + 256 * r), 16, e * 4, 0, 0, 0);
            }
        }
    }

    // Second half: for a staged chunk, wait for the loads and read this lane's
    // own samples p .. p + kChunk - 1 out of the tile.
    // stores_after: vector stores issued since the chunk's loads, 0, 4 (one
    // staged output tile) or 8 (two); the loads complete in order before
    // them, so they need not be waited for.
    __device__ __forceinline__ void finish_chunk(int p, float* v, int stores_after) const {
        if (!chunk_staged(p)) return;
        if (stores_after >= 8)
            __builtin_amdgcn_s_waitcnt(0x0F78);  // vmcnt(8): loads landed, the 8 stores may fly
        else if (stores_after >= 4)
            __builtin_amdgcn_s_waitcnt(0x0F74);  // vmcnt(4): loads landed, the 4 stores may fly
        else
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        __syncthreads();
        const int line = min(line0 + lane, nlines - 1);
        if (f16) {
            const int m = (line * in_line + p) & 7;
            const _Float16* th = reinterpret_cast<const _Float16*>(tile_in);
#pragma unroll
            for (int t = 0; t < kChunk; ++t) v[t] = (float)th[lane * kRowF16 + m + t];
        } else {
            const int m = (line * in_line + p) & 3;
#pragma unroll
            for (int t = 0; t < kChunk; ++t) v[t] = tile_in[lane * kRowF32 + m + t];
        }
        __syncthreads();
    }

    __device__ __forceinline__ void store(int p, float v) const {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rout, out_base_b, p * out_pos_b, 0);
    }

    // Stores this lane's outputs y[0..kChunk) at positions c0.. (only those
    // below end).  Lanes past the last line repeat the last line's work, so
    // their stores write that line's values to its addresses (the same bits)
    // and need no lane mask.
    // stage_out requires every line start and c0 to be 4-element aligned, so
    // the 16-byte stores below are aligned; tile rows past the last line go
    // past the buffer's extent (its size as the offset), where the bounds
    // check drops them.
    // Returns true when the chunk went out as the 4 tile stores.
    // store_full: the same for a chunk that lies wholly before end.
    __device__ __forceinline__ bool store_full(int c0, const float* y) const {
        if (stage_out) return store_staged(c0, y);
#pragma unroll
        for (int i = 0; i < kChunk; ++i) store(c0 + i, y[i]);
        return false;
    }
    __device__ __forceinline__ bool store_chunk(int c0, int end, const float* y) const {
        if (c0 + kChunk <= end) return store_full(c0, y);
#pragma unroll
        for (int i = 0; i < kChunk; ++i)
            if (c0 + i < end) store(c0 + i, y[i]);
        return false;
    }
    __device__ __forceinline__ bool store_staged(int c0, const float* y) const {
#pragma unroll
        for (int i = 0; i < kChunk; ++i) tile_out[lane * kStage + i] = y[i];
        __syncthreads();
        const int col = (lane & 3) * 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = (lane >> 2) + 16 * r;
            u32x4 w;
#pragma unroll
            for (int e = 0; e < 4; ++e) w[e] = __builtin_bit_cast(unsigned, tile_out[row * kStage + col + e]);
            const int off = line0 + row < nlines ? ((line0 + row) * out_line + c0 + col) * 4 : (int)out_bytes;
            __builtin_amdgcn_raw_buffer_store_b128(w, rout, off, 0, 0);
        }
        __syncthreads();
        return true;
    }
};

// Filters samples [seg_a, seg_b) of one line.  seg_a is a multiple of kChunk.
// RESTART (box only): the running sums restart at the block positions (the
// default, "block"); otherwise they run over the whole segment ("plain", or
// "kahan" with KAHAN), starting from d.carry where a scan provided states.
template <int S, int K, bool GAUSS, bool KAHAN, bool RESTART>
__device__ __forceinline__ void run_segment(const PassDesc& d, const LineIO& io, int seg_a, int seg_b) {
    constexpr int C = kChunk;
    constexpr int NX = C + S + 2 * K + 1;  // x window: positions c0-K-1 .. c0+C+S+K-1
    constexpr int NP = C + S;              // accumulators: centres c0 .. c0+C+S-1
    constexpr int ND = C + 2 * K;          // lifted samples of one diagonal (Gaussian)
    constexpr int R0 = (C - S) % C;        // restart offset within a chunk
    constexpr int XO = K + 1;              // x index of centre c0
    static_assert(S >= 1 && S <= kMaxS && K >= 0 && K <= kMaxK, "parameter range");
    static_assert(!(GAUSS && (KAHAN || RESTART)) && !(KAHAN && RESTART), "variant");

    // Everything runs on the scaled samples xs = a x: the lift then needs no
    // multiply, and the average of scaled samples is unscaled once per output
    // (y = (P / Q) / a).
    const float alpha = d.alpha;
    const float inv_alpha = d.inv_alpha;
    float xs[NX], P[NP], Q[NP], nx[C];  // nx: the next chunk's samples
    float R[S];
    float Rc[KAHAN ? S : 1];
    float Dv[GAUSS ? ND : 1];
    float g[K + 1];
#pragma unroll
    for (int k = 0; k <= K; ++k) g[k] = d.taps[k];

    // ---- window for the pre-chunk at c0 = seg_a - C ----
    // Column passes: the first chunk's loads go out first; the pre-chunk
    // waits for the window's, so the loop finds them complete and its own
    // wait at the top counts only the previous iteration's loads.  Row
    // passes: the window's loads into its LDS region go out first, the first
    // chunk's tile loads behind them.
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
    }

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
                if (i == R0) {
                    if (!RESTART && d.carry != nullptr && seg_a > 0) {
                        // the whole-line recursion's state here (snlm_carry_kernel)
                        const int line = min(io.line0 + io.lane, io.nlines - 1);
                        const long at = ((long)(seg_a / d.seg_len - 1) * S + si) * io.nlines + line;
                        R[si] = d.carry[at];
                        if constexpr (KAHAN) Rc[si] = d.carry[at + (long)(d.nseg - 1) * S * io.nlines];
                    } else {
                        R[si] = box_init<K, XO>(xs, i, s);
                        if constexpr (KAHAN) Rc[si] = 0.0f;
                    }
                } else if constexpr (KAHAN) {
                    box_slide_kahan<K>(xs, R[si], Rc[si], i, s);
                } else {
                    box_slide<K>(xs, R[si], i, s);
                }
                if (i < C - s) continue;
                r = R[si];
            }
            accumulate_pair<XO>(xs, P, Q, i, s, pair_weight(r), false);
        }
    }

    // ---- main chunks ----
    bool staged_store_last = false;  // the previous chunk ended with 4 tile stores
    for (c0 = seg_a;; c0 += C) {
        io.finish_chunk(c0 + S + K, nx, staged_store_last ? 4 : 0);
        advance_chunk<S, XO>(xs, P, Q, nx, alpha);
        const bool has_next = c0 + C < seg_b;
        // Column passes fetch the next chunk unconditionally (a chunk past the
        // segment is read and dropped), so that every iteration issues the same
        // loads and stores and the loop waits only for the loads; row passes
        // fill the LDS tile, which nothing may still be writing at a tile's end.
        if (has_next || !io.stage_in) io.issue_chunk(c0 + C + S + K, nx);

#pragma unroll
        for (int s = 1; s <= S; ++s) {
            const int si = s - 1;
            // Let the scheduler interleave two offsets at a time (two
            // independent running-sum chains), but not more: that bounds the
            // live registers (and so raises occupancy).
            if (s % 2 == 1) __builtin_amdgcn_sched_barrier(0);
            if constexpr (GAUSS) lift_diag(xs, Dv, s, 0);
#pragma unroll
            for (int i = 0; i < C; ++i) {
                float r;
                if constexpr (GAUSS) {
                    r = gauss_d2<K>(Dv, g, i);
                } else {
                    if (RESTART && i == R0)
                        R[si] = box_init<K, XO>(xs, i, s);  // block restart
                    else if constexpr (KAHAN)
                        box_slide_kahan<K>(xs, R[si], Rc[si], i, s);
                    else
                        box_slide<K>(xs, R[si], i, s);
                    r = R[si];
                }
                accumulate_pair<XO>(xs, P, Q, i, s, pair_weight(r), true);
            }
        }

        float y[C];
        normalise(P, Q, inv_alpha, y);
        // Materialise all outputs before the (partly masked) stores, so that
        // the compiler does not sink the last accumulations into the store
        // branches and split the chunk into small blocks.
#pragma unroll
        for (int i = 0; i < C; i += 4)
            asm volatile("" ::"v"(y[i]), "v"(y[i + 1]), "v"(y[i + 2]), "v"(y[i + 3]));
        if (!has_next) {
            io.store_chunk(c0, seg_b, y);
            break;
        }
        // (the loop continues only after a whole chunk's stores, so every
        // iteration issues the same memory operations)
        staged_store_last = io.store_full(c0, y);
    }
}

// Copy / convert pass for S = 0 (the 1D NLM is then the identity).
__device__ __forceinline__ void run_copy(const LineIO& io, int seg_a, int seg_b) {
    for (int p = seg_a; p < seg_b; ++p) {
        float v[1];
        io.template load<1>(p, v);
        io.store(p, v[0]);
    }
}

// ROWS: the kernel variant for passes whose lines are contiguous in memory
// (it carries the LDS transpose tiles); column-pass variants compile the
// tiles out and so keep fewer registers live.
template <bool ROWS>
__device__ __forceinline__ LineIO make_io(const PassDesc& d, int line0, int lane, float* tiles) {
    LineIO io;
    const int line = min(line0 + lane, d.nlines - 1);
    io.rin = make_rsrc(d.in, d.in_bytes);
    io.rout = make_rsrc(d.out, d.out_bytes);
    const int esz = d.in_f16 ? 2 : 4;
    int lin = line * d.in_line, lout = line * d.out_line;
    if (d.split) {  // lines in blocks (a volume's y or z lines)
        const int hi = line / d.split, lo = line - hi * d.split;
        lin = hi * d.in_outer + lo * d.in_line;
        lout = hi * d.out_outer + lo * d.out_line;
    }
    io.in_base_b = lin * esz;
    io.in_pos_b = d.in_pos * esz;
    io.in_line = d.in_line;
    io.out_base_b = lout * 4;
    io.out_pos_b = d.out_pos * 4;
    io.out_line = d.out_line;
    io.line0 = line0;
    io.nlines = d.nlines;
    io.lane = lane;
    io.n = d.n;
    io.out_bytes = d.out_bytes;
    io.f16 = d.in_f16 != 0;
    io.stage_in = ROWS && d.split == 0 && d.in_pos == 1 && ((uintptr_t)d.in & 15) == 0;
    io.stage_out = ROWS && d.split == 0 && d.out_pos == 1 && (d.out_line & 3) == 0 &&
                   ((uintptr_t)d.out & 15) == 0;
    io.tile_in = tiles;
    io.tile_out = tiles + kTileIn;
    io.tile_win = tiles + kTileIn + kTileOut;
    return io;
}

template <int S, int K, bool GAUSS, bool KAHAN, bool RESTART, bool ROWS>
__device__ __forceinline__ void run_tile(const PassDesc& d, int group, int a, int b, float* tiles) {
    const int lane = threadIdx.x & (kLanes - 1);
    const int line0 = group * kLanes;
    const LineIO io = make_io<ROWS>(d, line0, lane, tiles);
    if constexpr (S == 0) {
        run_copy(io, a, b);
    } else {
        run_segment<S, K, GAUSS, KAHAN, RESTART>(d, io, a, b);
    }
}

// Loads a table entry the whole wave agrees on (a batch's header, tiles and
// pass descriptors, which no kernel writes) with scalar loads: read through
// the constant address space, a wave-uniform address becomes s_load
// instructions into scalar registers instead of per-lane loads.
template <typename T>
__device__ __forceinline__ T load_uniform(const T* src) {
    static_assert(sizeof(T) % 4 == 0, "word-sized");
    typedef __attribute__((address_space(4))) const uint32_t* const_words;
    const_words w = (const_words)(src);
    T v;
    uint32_t* o = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) o[i] = w[i];
    return v;
}

// One kernel per (S, K, kernel, running-sum variant, row/column variant).
// Workgroup = one wave.
template <int S, int K, bool GAUSS, bool KAHAN, bool RESTART, bool ROWS>
__global__ __launch_bounds__(kLanes) void snlm_kernel(KernelArgs args) {
    const bool batch = args.hdr != nullptr;
    BatchHeader hdr = {0, 0, 0, 0u};
    if (batch) hdr = load_uniform(args.hdr);
    __shared__ uint32_t claimed;
    __shared__ __attribute__((aligned(16))) float tiles[ROWS ? row_lds_floats(kChunk + S + 2 * K + 1) : 1];
    const bool stat = batch && args.worker_first != nullptr;
    uint32_t t_next = 0, t_end = 0;
    if (stat) {
        t_next = load_uniform(&args.worker_first[blockIdx.x]);
        t_end = load_uniform(&args.worker_first[blockIdx.x + 1]);
    }
    for (int iter = 0;; ++iter) {
        PassDesc d;
        int group, a, b, job = 0, pass = 0;
        if (!batch) {
            if (iter > 0) break;
            d = args.direct;
            const int t = blockIdx.x;
            group = t % d.ngroups;
            a = (t / d.ngroups) * d.seg_len;
            b = min(a + d.seg_len, d.n);
        } else {
            uint32_t t;
            if (stat) {
                if (t_next >= t_end) break;
                t = t_next++;
            } else {
                if (threadIdx.x == 0) claimed = atomicAdd(args.claim, 1u);
                __syncthreads();
                t = __builtin_amdgcn_readfirstlane(claimed) + (uint32_t)args.tile_lo;
                __syncthreads();
                if (t >= (uint32_t)args.tile_hi) break;
            }
            const BatchTile bt = load_uniform(&args.tiles[t]);
            job = (int)bt.job;
            pass = t < (uint32_t)hdr.ntiles_first ? 0 : 1;
            group = bt.group;
            a = bt.a;
            b = bt.b;
            if (pass == 1 && args.wait) {
                // Wait until every first-pass tile of this job has been written:
                // poll with relaxed device-scope loads (no cache invalidation per
                // poll), then one acquire fence before reading the intermediate.
                const uint32_t need = __builtin_amdgcn_readfirstlane(args.jobs[job].tiles[0]);
                uint32_t polls = 0;
                bool ok = true;
                while (__hip_atomic_load(&args.counters[1 + job], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) < need) {
                    if (++polls > hdr.spin_limit) {
                        ok = false;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(4);
                }
                if (!ok) {
                    if (threadIdx.x == 0) atomicOr(args.status, 1u);
                    break;
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            d = load_uniform(&args.jobs[job].pass[pass]);
        }
        run_tile<S, K, GAUSS, KAHAN, RESTART, ROWS>(d, group, a, b, tiles);
        if (batch && pass == 0 && args.wait) {
            // publish this tile's intermediate rows (one release per tile)
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_fetch_add(&args.counters[1 + job], 1u, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace snlm
