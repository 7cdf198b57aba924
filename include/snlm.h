/*
 * snlm.h -- separable PatchLift non-local means on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libsnlm.so.  All pointers named "device" are device (HBM) addresses,
 * typically the data pointers of PyTorch tensors; the caller owns them.  The
 * library owns only its context (streams, events, graphs, small job tables,
 * pinned staging memory and the serving thread).
 *
 * What is computed (Ghosh & Chaudhury, "Fast Separable Non-Local Means"):
 *
 *   1D NLM (Sec. 2, eq. 1dNLM), on every line of a pass:
 *       y(i) = sum_{j=i-S..i+S} w(i,j) x(j) / sum_j w(i,j),
 *       w(i,j) = exp(-d2(i,j) / h^2),
 *       d2(i,j) = sum_{k=-K..K} g(k) (x(i+k) - x(j+k))^2     (eq. distanceSquared)
 *   with g = box (1) or Gaussian exp(-k^2/(2 beta^2)) (Sec. 2), the line
 *   extended by half-sample symmetric reflection (x1 x0 | x0 x1 ... ), and the
 *   distances obtained by lifting each offset-s diagonal (x(t)-x(t+s))^2 and
 *   summing it over the patch with running (prefix-difference) sums
 *   (PatchLift, Sec. 2.1-2.2, eqs. lift and recursion; Prop. 1, Cor. 1).
 *
 *   Separable NLM (Sec. 3): SNLM_ROW_COL filters every row, then every column
 *   of the row-filtered image (the RC pipeline); SNLM_COL_ROW does columns
 *   first (CR).  The same S, K, h are used for both passes.
 *
 * Arithmetic is FP32 (inputs FP32 or FP16, outputs FP32).  Against an FP64
 * evaluation of the same formulas the maximum absolute error is below 1e-3 on
 * the [0, 255] scale for the block-restarted running sums (the default).
 *
 * Status codes: 0 = SNLM_OK, > 0 = SNLM_PENDING (snlm_poll only), < 0 = error.
 * No C++ exception crosses this interface.
 */
#ifndef SNLM_H
#define SNLM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SNLM_OK = 0,
    SNLM_PENDING = 1,      /* snlm_poll: the job is still in flight */
    SNLM_EINVAL = -1,      /* invalid argument (see each call) */
    SNLM_ENOMEM = -2,      /* the job can never fit the arena / table capacity */
    SNLM_EDEVICE = -3,     /* a HIP runtime error or a device-side failure */
    SNLM_ENOTICKET = -4,   /* unknown or already collected ticket */
    SNLM_ECLOSED = -5,     /* the context is shutting down */
    SNLM_EBUSY = -6        /* a direct call while served jobs hold the arena */
};

/* Patch kernels g of eq. distanceSquared.
 *   SNLM_BOX        g = 1 on [-K, K], window sums by the recursion of eq. recursion
 *   SNLM_GAUSS      g(k) = exp(-k^2 / (2 beta^2)) on [-K, K], an exact FIR
 *   SNLM_GAUSS_IIR  the untruncated Gaussian of width beta approximated by the
 *                   third-order recursive filter of Young & van Vliet (1995),
 *                   the recursive Gaussian Sec. 2.2 points to: each lifted
 *                   diagonal D_s(v) = (x(v) - x(v+s))^2 of the reflected line is
 *                   filtered forward then backward, starting L = ceil(6 beta) +
 *                   S + 3 samples beyond each end with the steady state of its
 *                   first input, and scaled by sqrt(2 pi) beta (g(0) = 1):
 *                     q  = 0.98711 beta - 0.96330 (beta >= 2.5),
 *                          3.97156 - 4.14554 sqrt(1 - 0.26891 beta) otherwise
 *                     b0 = 1.57825 + 2.44413 q + 1.4281 q^2 + 0.422205 q^3
 *                     b1 = 2.44413 q + 2.85619 q^2 + 1.26661 q^3
 *                     b2 = -(1.4281 q^2 + 1.26661 q^3),  b3 = 0.422205 q^3
 *                     w(v) = B D(v) + (b1 w(v-1) + b2 w(v-2) + b3 w(v-3)) / b0,
 *                     B = 1 - (b1 + b2 + b3) / b0
 *                   The weight is exp(-d / h^2) of the filtered value d (which
 *                   can be slightly negative where the response's lobes
 *                   reach).  Cost per sample is independent of beta; K only
 *                   sets the default beta = K / 2.  0.5 <= beta <= 256.  Runs
 *                   in snlm_denoise, snlm_denoise_ex and snlm_denoise3d (other
 *                   entry points return SNLM_EINVAL); each pass keeps the
 *                   forward recursion's FP64 state at every 16th position,
 *                   3 S ((n + L - 1) / 16 + 2) values per line, and for a
 *                   pass along rows an FP32 transposed copy of its input, in
 *                   a library-owned device buffer (grown on demand, held
 *                   until snlm_destroy) whose two regions must each stay
 *                   below 2 GiB. */
typedef enum { SNLM_BOX = 0, SNLM_GAUSS = 1, SNLM_GAUSS_IIR = 2 } snlm_kernel;
typedef enum { SNLM_ROW_COL = 0, SNLM_COL_ROW = 1 } snlm_order;
typedef enum { SNLM_F32 = 0, SNLM_F16 = 1 } snlm_dtype;

/* How the box-kernel window sums along each lifted diagonal are carried
 * (eq. recursion).  The Gaussian kernel uses an exact (2K+1)-tap FIR per
 * diagonal and ignores this field. */
typedef enum {
    SNLM_SUM_BLOCK = 0,  /* recursion re-initialised every 16 samples at fixed
                            line-relative positions (default; fastest, and
                            results do not depend on how lines are tiled) */
    SNLM_SUM_KAHAN = 1,  /* recursion over the whole line, Kahan-compensated */
    SNLM_SUM_PLAIN = 2   /* recursion over the whole line, plain FP32 */
} snlm_sum;
/* With KAHAN or PLAIN, snlm_denoise_ex still cuts lines into segments: a scan
 * first replays each offset's whole-line recursion and records its state at
 * every segment start (a library-owned device buffer), so the result is
 * bitwise the same as one segment per line.  Batched and served jobs with
 * these modes keep one segment per line. */

/* Limits of the compiled kernels.  S <= 16: a lane walks its line in chunks
 * of 16 samples, and a segment's first chunk takes the pairs reaching into it
 * from the one chunk before it (every offset s must fit in that chunk); the
 * running sums restart every 16 samples.  K <= 8 bounds the registers of the
 * sample window. */
#define SNLM_MAX_S 16
#define SNLM_MAX_K 8

typedef struct snlm_ctx snlm_ctx;

/* One denoising job.
 *   img      device pointer, H x W, row pitch ld_in elements, FP32 or FP16
 *   out      device pointer, H x W FP32, row pitch ld_out elements; must not
 *            overlap img
 *   S        search half-width, 0..SNLM_MAX_S (S = 0 returns the input)
 *   K        patch half-width, 0..SNLM_MAX_K
 *   h        smoothing parameter, > 0; +INFINITY gives w = 1 (moving average)
 *   beta     Gaussian width; <= 0 selects K/2
 *   seg_len  samples per line segment of one wave (a multiple of 16), or 0 to
 *            let the library choose.  Results do not depend on it. */
typedef struct {
    const void *img;
    float *out;
    int H, W, ld_in, ld_out;
    snlm_dtype dtype;
    int S, K;
    float h;
    float beta;
    snlm_kernel kernel;
    snlm_order order;
    snlm_sum sum;
    int seg_len;
} snlm_job;

/* Creates a context on HIP device `device`.
 *   stream       the caller's hipStream_t (NULL = legacy default stream);
 *                every call is ordered after work already queued on it, and
 *                work queued on it afterwards runs after the call's kernels
 *   arena        caller-owned device buffer for the FP32 intermediates
 *                (snlm_workspace_bytes per image); may be NULL only with
 *                arena_bytes = 0, which then rejects every job (SNLM_ENOMEM)
 * Returns SNLM_OK and *ctx, SNLM_EINVAL for a NULL ctx or a bad device,
 * SNLM_EDEVICE if the HIP runtime fails. */
int snlm_create(snlm_ctx **ctx, int device, void *stream, void *arena, size_t arena_bytes);

/* Waits for all work of the context (including served jobs), stops the
 * serving thread and releases library-owned resources.  Never frees caller
 * memory.  NULL is accepted. */
int snlm_destroy(snlm_ctx *ctx);

/* Arena bytes one job of a direct call needs for its FP32 intermediate image
 * (H x Wp, Wp = W rounded up to 16), rounded up to 256 bytes. */
size_t snlm_workspace_bytes(int H, int W, snlm_dtype dtype);

/* Arena bytes one served job holds while in flight: its staged input (H x W
 * of the job's dtype), its FP32 intermediate (H x Wp, Wp = W rounded up to
 * 16) and its FP32 output slot (H x W), each rounded up to 256 bytes. */
size_t snlm_serving_bytes(int H, int W, snlm_dtype dtype);

/* Arena use.  Direct calls (snlm_denoise*, snlm_enqueue_*, snlm_denoise_sure,
 * snlm_denoise_full, snlm_denoise3d, the autotuners) place their workspace at
 * the start of the arena; served jobs take slots anywhere in it.  The two may
 * not overlap in time: a direct call made while any served job is pending or
 * in flight returns SNLM_EBUSY, and served jobs start only after the caller's
 * stream has passed their submit, so after earlier direct calls' kernels.
 * Direct calls and submits from different threads on one context are not
 * supported. */

/* Separable NLM of one FP32 image with contiguous rows (ld = W).
 * Synchronous: returns when out holds the result (the work runs on the
 * context stream, after work already queued there).
 * Errors: SNLM_EINVAL (NULL pointers, H or W < 1, S or K out of range, h not
 * > 0, unknown kernel/order, out overlapping img), SNLM_ENOMEM (arena smaller
 * than snlm_workspace_bytes), SNLM_EBUSY, SNLM_EDEVICE. */
int snlm_denoise(snlm_ctx *ctx, const void *img, float *out, int H, int W, int S, int K,
                 float h, int kernel, int order);

/* As snlm_denoise with every option of snlm_job.  Synchronous. */
int snlm_denoise_ex(snlm_ctx *ctx, const snlm_job *job);

/* As snlm_denoise_ex, but returns once the work is enqueued on the context
 * stream (ordered like any other work on it; snlm_sync or a stream
 * synchronisation gives completion).  For callers that order work on their own
 * stream. */
int snlm_enqueue_ex(snlm_ctx *ctx, const snlm_job *job);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * two passes as snlm_enqueue_ex, enqueued on `stream` (a hipStream_t of the
 * current device; NULL = legacy default stream), with no context and no
 * arena.  The FP32 intermediate lives in a file-scope device array of
 * SNLM_STATIC_SCRATCH_BYTES that each GPU the library runs on holds until the
 * process ends; the call makes no hipMalloc, hipFree or other allocating call
 * (the array's device address is looked up once per device, at snlm_create or
 * at the first call).  Every call on one GPU shares that array: calls whose
 * kernels overlap in time on one GPU (different streams, or other threads)
 * race and give wrong results; order them.  Results are bitwise those of
 * snlm_enqueue_ex.  Box jobs with plain or Kahan sums run one segment per line.
 * Errors: SNLM_EINVAL (as snlm_denoise_ex, and for SNLM_GAUSS_IIR, which needs
 * library buffers), SNLM_ENOMEM (H x Wp x 4 bytes, Wp = W rounded up to 16,
 * above SNLM_STATIC_SCRATCH_BYTES), SNLM_EDEVICE (HIP runtime errors).  There
 * is no context, so there is no snlm_last_error detail. */
#define SNLM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int snlm_enqueue_static(const snlm_job *job, void *stream);

/* Many images in two persistent launches per (S, K, kernel, order) class,
 * captured once in a HIP graph (first-pass launch + second-pass launch)
 * and replayed.  The line groups of every image of a pass
 * are cut at 16-sample boundaries into one equal share of work per persistent
 * workgroup (jobs with seg_len > 0, and box jobs with plain or Kahan sums,
 * keep their segments whole).  The arena must hold the sum of the jobs'
 * snlm_workspace_bytes.  Synchronous.  Results are bitwise
 * identical to snlm_denoise_ex of each job.  Errors as snlm_denoise_ex, plus
 * SNLM_EINVAL for n < 1 and SNLM_ENOMEM when the jobs do not fit the arena
 * together.  With the environment variable SNLM_BATCH_MODE=fused at context
 * creation, a single launch per class instead claims tiles with an atomic
 * counter, second-pass tiles waiting for the first-pass tiles of their image. */
int snlm_denoise_batch(snlm_ctx *ctx, const snlm_job *jobs, int n);

/* As snlm_denoise_batch, but returns once enqueued on the context stream.  A
 * batch identical to the previous one (same jobs, arena and tuning) only
 * replays the captured graphs. */
int snlm_enqueue_batch(snlm_ctx *ctx, const snlm_job *jobs, int n);

/* SURE-optimal combination of the two orders (Sec. 3.1, Alg. 3 and Alg. 4):
 * out = theta1 f_rc + theta2 f_cr, where f_rc / f_cr are the row_col / col_row
 * separable NLM of img, and theta solves the 2x2 system of eqs. A and bb built
 * from image sums and the chained 1D divergences (eq. div; eqs. partialrc and
 * partialcr), with sigma the noise level of eq. noise.  job->order is ignored;
 * box jobs must use SNLM_SUM_BLOCK.  When f_rc and f_cr are proportional
 * (singular system, e.g. h = +inf) theta1 = theta2 = (b1 + b2) / sum(A).
 * The arena must hold snlm_sure_workspace_bytes(H, W); after the call it holds
 * (snlm_sure_layout byte offsets): [0] scratch, [1] scratch, [2] f_cr, [3] the
 * divergence of f_rc, [4] the divergence of f_cr (each H x Wp FP32, Wp = W
 * rounded up to 16), [6] theta1, theta2 and the seven sums (doubles: sum f_rc^2,
 * sum f_rc f_cr, sum f_cr^2, sum f f_rc, sum f f_cr, sum div_rc, sum div_cr).
 * Enqueued on the context stream; when theta (2 doubles) or stats (7 doubles)
 * are non-NULL host pointers the call waits for the result and copies it out.
 * Errors: as snlm_denoise_ex, plus SNLM_EINVAL for sigma < 0 or not finite,
 * and SNLM_ENOMEM when the arena is too small. */
int snlm_denoise_sure(snlm_ctx *ctx, const snlm_job *job, float sigma, double *theta, double *stats);

/* Bilateral post-processing of eq. BF (Sec. 3.2):
 *   out(i) = sum_j w(j) g(in(i-j) - in(i)) in(i-j) / sum_j w(j) g(in(i-j) - in(i)),
 *   w(j) = exp(-|j|^2 / (2 sigma_s^2)),  g(t) = exp(-t^2 / (2 sigma_r^2)),
 * over the integer offsets j of [-3 sigma_s, 3 sigma_s]^2, the image extended
 * by half-sample symmetric reflection.  in, out: device FP32 H x W with row
 * pitches ld_in, ld_out (elements); out must not overlap in.  sigma_r = +inf
 * gives a normalised Gaussian blur.  Enqueued on the context stream.
 * Errors: SNLM_EINVAL for NULL pointers, H or W < 1, pitches < W, overlap,
 * sigma_s not in (0, 3) (the support radius floor(3 sigma_s) is at most 8),
 * sigma_r not > 0. */
int snlm_bilateral(snlm_ctx *ctx, const float *in, int ld_in, float *out, int ld_out, int H, int W,
                   float sigma_s, float sigma_r);

/* The bilateral parameters the paper's rules give for noise level sigma
 * (Sec. 4.1): sigma_s = 2.5e-6 s^3 - 3.4e-4 s^2 + 0.021 s + 0.46 and
 * sigma_r = 2.8e-4 s^3 - 0.088 s^2 + 8 s - 24.  Either pointer may be NULL. */
void snlm_bilateral_params(float sigma, float *sigma_s, float *sigma_r);

/* SNLM[f] of Sec. 3.2: the SURE-optimal combination of the two orders
 * (snlm_denoise_sure) followed by the bilateral filter with the parameters of
 * snlm_bilateral_params(sigma), written to job->out.  The arena must hold
 * snlm_full_workspace_bytes(H, W): the snlm_sure_layout regions, then the
 * combined image (H x Wp FP32) at byte offset snlm_sure_workspace_bytes(H, W).
 * theta / stats as for snlm_denoise_sure.  Errors: as snlm_denoise_sure, plus
 * SNLM_EINVAL when the rules give parameters snlm_bilateral rejects. */
int snlm_denoise_full(snlm_ctx *ctx, const snlm_job *job, float sigma, double *theta, double *stats);

/* Arena bytes snlm_denoise_full needs (0 for H or W < 1). */
size_t snlm_full_workspace_bytes(int H, int W);

/* Separable NLM of a volume (the extension to volumes noted in the paper's
 * conclusion): the 1D NLM (eq. 1dNLM, same S, K, h, patch kernel, reflection
 * and block-restarted sums as the 2D passes) along axes[0], then axes[1], then
 * axes[2] of the previous pass's output, with 0 = x (the contiguous axis),
 * 1 = y, 2 = z.  img: D x H x W, element (z, y, x) at (z H + y) ld_in + x,
 * FP32 or FP16 per dtype; out: FP32, element at (z H + y) ld_out + x.  The
 * arena must hold snlm_workspace3d_bytes(D, H, W) (two FP32 intermediate
 * volumes).  Enqueued on the context stream.  Errors: SNLM_EINVAL for NULL
 * pointers, D, H or W < 1, pitches < W, axes not a permutation of 0, 1, 2, the
 * parameter checks of snlm_denoise, out overlapping img, or a volume over
 * 2 GiB; SNLM_ENOMEM for a small arena; SNLM_EDEVICE. */
int snlm_denoise3d(snlm_ctx *ctx, const void *img, int ld_in, snlm_dtype dtype, float *out, int ld_out,
                   int D, int H, int W, int S, int K, float h, int kernel, const int *axes);

/* Arena bytes snlm_denoise3d needs (0 for D, H or W < 1). */
size_t snlm_workspace3d_bytes(int D, int H, int W);

/* Arena bytes snlm_denoise_sure needs (0 for H or W < 1). */
size_t snlm_sure_workspace_bytes(int H, int W);

/* Byte offsets of the snlm_denoise_sure workspace regions: offsets[0..4] the
 * five H x Wp FP32 planes, [5] partial sums, [6] result doubles, [7] total.
 * SNLM_EINVAL for H or W < 1 or offsets NULL. */
int snlm_sure_layout(int H, int W, size_t *offsets);

/* Waits for everything enqueued on the context stream by this library and
 * reports device-side failures of batched launches (SNLM_EDEVICE). */
int snlm_sync(snlm_ctx *ctx);

/* Serving.  Submits a job to the context's scheduler and returns at once with
 * a ticket.  An event recorded on the context stream at the call orders the
 * job after work already queued there (img may be written by a kernel still
 * running on that stream).  Whenever one of its library streams is free,
 * the scheduler forms a round from the kernel class (S, K, kernel, order) of
 * the oldest queued job: the queued jobs of that class, in arrival order,
 * while their snlm_serving_bytes fit what the arena has left (the HBM budget
 * bounds every byte a served job touches on the device); jobs of other
 * classes keep their places.  A round overlaps on the device with rounds
 * already running on the other streams: one launch copies every input into
 * its arena slot, the two batched persistent launches (grids sized to the
 * round's work) compute into the arena output slots, one launch copies the
 * outputs to each job->out.  img and out must stay valid until snlm_poll
 * returns non-PENDING.
 * Errors: SNLM_EINVAL, SNLM_ENOMEM (the job can never fit the arena),
 * SNLM_ECLOSED, SNLM_EDEVICE. */
int snlm_submit(snlm_ctx *ctx, const snlm_job *job, uint64_t *ticket);

/* Submits jobs[0..n) in order from the calling thread, job i at arrival_us[i]
 * microseconds (host monotonic clock) after the call (all at once when
 * arrival_us is NULL), waiting between arrivals; tickets[i] receives each
 * ticket.  Returns when the last job is submitted, or at the first error
 * (jobs before it stay submitted).  A request driver that does not depend on
 * the caller's language runtime. */
int snlm_submit_many(snlm_ctx *ctx, const snlm_job *jobs, int n, const double *arrival_us,
                     uint64_t *tickets);

/* Device-side latency of a finished served job: milliseconds between its
 * submit event on the context stream and the end of its round (outputs
 * copied), both timestamps taken by the GPU.  -1 if the round failed.
 * SNLM_ENOTICKET if unknown; call before the final snlm_poll. */
int snlm_job_device_ms(snlm_ctx *ctx, uint64_t ticket, double *ms);

/* Scheduler statistics of the context since its creation: rounds launched,
 * the served jobs they carried, and the host time (microseconds) the
 * scheduler thread spent planning and enqueueing them.  NULL outputs are
 * skipped.  Errors: SNLM_EINVAL for a NULL context. */
int snlm_serving_stats(snlm_ctx *ctx, uint64_t *rounds, uint64_t *jobs, double *host_us);

/* SNLM_PENDING while the job runs; then its final status once (SNLM_OK or an
 * error), after which the ticket is forgotten (SNLM_ENOTICKET). */
int snlm_poll(snlm_ctx *ctx, uint64_t ticket);

/* Timestamps of a finished served job, in microseconds of the host monotonic
 * clock: submit, admission, completion observed.  SNLM_ENOTICKET if unknown.
 * Must be called before the final snlm_poll of the ticket. */
int snlm_job_times(snlm_ctx *ctx, uint64_t ticket, double *t_submit, double *t_admit,
                   double *t_done);

/* Host-side validation of a job (no device access).  SNLM_OK or SNLM_EINVAL,
 * with the reason in *why (static string) when why is not NULL. */
int snlm_validate(const snlm_job *job, const char **why);

/* Selects the segment length for jobs of this shape class by timing
 * candidates on the context stream with the given job (whose buffers are used
 * as scratch input/output), and remembers it for later jobs with seg_len = 0
 * of the same (S, K, kernel, size class).  *best receives the choice. */
int snlm_autotune(snlm_ctx *ctx, const snlm_job *probe, int *best);

/* Selects the number of persistent waves per SIMD (1..4, within the kernel's
 * occupancy) of batched launches for the kernel classes of these jobs, timing
 * each candidate on the jobs themselves (their outputs are overwritten), and
 * remembers it for later batches of the same classes (untuned classes run two
 * waves per SIMD, or fewer where the kernel's occupancy is lower).  Results do
 * not depend on the choice.  *best receives it. */
int snlm_autotune_batch(snlm_ctx *ctx, const snlm_job *jobs, int n, int *best);

/* Saves / loads the autotuner's choices as a small JSON file. */
int snlm_autotune_save(snlm_ctx *ctx, const char *path);
int snlm_autotune_load(snlm_ctx *ctx, const char *path);

/* Segment length the library would use for this job (after validation). */
int snlm_plan_seg_len(snlm_ctx *ctx, const snlm_job *job, int pass);

/* Kernel timing for measurement.  enable = 1 clears and starts recording HIP
 * events on the stream of each persistent batched launch (immediately around
 * the graph replay of its persistent kernels) and of each direct
 * pass launch; enable = 0 stops, waits for the recorded events and returns the
 * summed device time of batched launches in *batch_ms (count in *batch_n) and
 * of direct pass launches in *direct_ms (count in *direct_n).  For the
 * recursive Gaussian kernel a pass's events bracket all of its launches (the
 * transposed copy of a row pass's input, the forward recursion, and the
 * backward recursion with the NLM).  Pointers may be NULL. */
int snlm_timing(snlm_ctx *ctx, int enable, double *batch_ms, int *batch_n, double *direct_ms,
                int *direct_n);

const char *snlm_strerror(int status);
const char *snlm_last_error(snlm_ctx *ctx);
const char *snlm_version(void);

/* Measurement helper behind the roofline figures (not part of denoising):
 * how many clock cycles one SIMD of the current device takes per pair body
 * of the line kernels (one lifted difference, two fused multiply-adds of the
 * running window sum, the weight, two fused multiply-adds and two adds of
 * the accumulation), with waves_per_simd (1, 2 or 4) waves resident on every
 * SIMD, each running eight independent copies of the body.
 *   mode 0  the body with the weight replaced by the window sum (FP32 only)
 *   mode 1  the body with the weight w = exp2(-|R|) (v_exp_f32)
 *   mode 2  v_exp_f32 alone (clk_per_pair is then cycles per exp per SIMD)
 * *clk_per_pair: per SIMD, the cycles from its first wave's start to its
 * last wave's end over the pair bodies its waves ran (iters x 8 each); the
 * median over SIMDs.  *clock_ghz (optional): the shader clock, shader-clock
 * cycles over constant-clock time summed over the waves.  Allocates and frees
 * two small device buffers.  Errors: SNLM_EINVAL for arguments out of range,
 * SNLM_EDEVICE for HIP failures. */
int snlm_issue_rate(int mode, int waves_per_simd, int iters, double *clk_per_pair, double *clock_ghz);

#ifdef __cplusplus
}
#endif

#endif /* SNLM_H */
