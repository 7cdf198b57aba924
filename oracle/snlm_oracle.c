/*
 * FP64 oracle for separable non-local means (Ghosh & Chaudhury, "Fast Separable
 * Non-Local Means").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
 * this file; it exists so that tests, the smoke check and the CPU baseline of
 * the benchmark can compare the GPU library against a plain, slow, obviously
 * correct computation.  It shares no code, header, table or helper with the GPU
 * library.
 *
 * What it computes (all in double precision, 0-based indices):
 *
 *   patch distance  (Sec. 2, eq. distanceSquared)
 *       d2(i,j) = sum_{k=-K..K} g(k) * (x_e(i+k) - x_e(j+k))^2
 *   patch kernel    (Sec. 2, definition of g_beta under eq. distanceSquared)
 *       box: g(k) = 1 ;  gauss: g(k) = exp(-k^2 / (2 beta^2)), g(0) = 1
 *   1D NLM          (Sec. 2, eq. 1dNLM)
 *       y(i) = sum_{j=i-S..i+S} w(i,j) x_e(j) / sum_{j=i-S..i+S} w(i,j),
 *       w(i,j) = exp(-d2(i,j) / h^2)
 *   separable NLM   (Sec. 3, the RC and CR pipelines)
 *       row_col: filter every row, then every column of the row-filtered image
 *       col_row: filter every column, then every row of the column-filtered image
 *
 * Readings where the paper is silent:
 *   - x_e is the line extended by half-sample symmetric reflection
 *     (... x1 x0 | x0 x1 ... x_{N-1} | x_{N-1} x_{N-2} ...), applied to patch
 *     taps and to the search window alike, with period 2N so that lines shorter
 *     than the reach S+K are handled.  Sec. 2 only notes that the signal is
 *     assumed extended beyond its ends.
 *   - h = +inf gives w = 1 everywhere.  w(i,i) = 1 for every h > 0, and any pair
 *     with d2 = 0 has w = 1 (exp(-0/h^2) = 1), written out explicitly so that a
 *     tiny h whose square underflows does not turn 0/0 into NaN.
 *   - For the Gaussian kernel beta defaults to K/2 (the caller passes beta).
 *
 * Distances are computed literally from their definition (no lifting, no
 * running sums), so the cost is O(N S K) per line.  Threads, when asked for,
 * split independent lines; they never change the arithmetic of a pixel.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_BOX 0
#define ORACLE_GAUSS 1
#define ORACLE_GAUSS_IIR 2
#define ORACLE_ROW_COL 0
#define ORACLE_COL_ROW 1

/* Half-sample symmetric reflection of index t into [0, n), period 2n. */
static long refl(long t, long n) {
    long p = 2 * n;
    long m = t % p;
    if (m < 0) m += p;
    return m < n ? m : p - 1 - m;
}

/* Patch kernel tap g(k) (Sec. 2). */
static double tap(int k, int kernel, double beta) {
    if (kernel == ORACLE_BOX || k == 0) return 1.0;
    return exp(-((double)k * (double)k) / (2.0 * beta * beta));
}

/* Weighted squared distance between the patches centred at i and j of the
 * extended line (eq. distanceSquared). */
static double patch_d2(const double *x, long n, long stride, long i, long j, int K,
                       int kernel, double beta) {
    double d2 = 0.0;
    for (int k = -K; k <= K; ++k) {
        double a = x[refl(i + k, n) * stride];
        double b = x[refl(j + k, n) * stride];
        d2 += tap(k, kernel, beta) * (a - b) * (a - b);
    }
    return d2;
}

/* One output sample of the 1D NLM of a strided line (eq. 1dNLM). */
static double nlm1d_at(const double *x, long n, long stride, long i, int S, int K,
                       double h, int kernel, double beta) {
    double P = 0.0, Q = 0.0;
    for (long j = i - S; j <= i + S; ++j) {
        double d2 = patch_d2(x, n, stride, i, j, K, kernel, beta);
        double w;
        if (d2 == 0.0)
            w = 1.0;
        else
            w = exp(-d2 / (h * h));
        P += w * x[refl(j, n) * stride];
        Q += w;
    }
    return P / Q;
}

static int bad_args(long n, int S, int K, double h, int kernel, double beta) {
    if (n < 1 || S < 0 || K < 0) return 1;
    if (!(h > 0.0)) return 1; /* rejects NaN too */
    if (kernel != ORACLE_BOX && kernel != ORACLE_GAUSS && kernel != ORACLE_GAUSS_IIR) return 1;
    if (kernel == ORACLE_GAUSS && K > 0 && !(beta > 0.0)) return 1;
    if (kernel == ORACLE_GAUSS_IIR && !(beta >= 0.5)) return 1;
    return 0;
}

static int nlm1d_iir(const double *x, long n, long stride, int S, double h, double beta, double *y,
                     long ystride);

/* Patch distance d2(i, j) of a contiguous line, i and j any integers (the line
 * is extended by reflection). */
double snlm_oracle_patch_d2(const double *x, long n, long i, long j, int K, int kernel,
                            double beta) {
    if (!x || n < 1 || K < 0) return NAN;
    if (kernel != ORACLE_BOX && kernel != ORACLE_GAUSS) return NAN;
    return patch_d2(x, n, 1, i, j, K, kernel, beta);
}

/* 1D NLM of a whole line: y[i*ystride] for i in [0, n). */
int snlm_oracle_nlm1d(const double *x, long n, long stride, int S, int K, double h,
                      int kernel, double beta, double *y, long ystride) {
    if (!x || !y || bad_args(n, S, K, h, kernel, beta)) return -1;
    if (kernel == ORACLE_GAUSS_IIR) return nlm1d_iir(x, n, stride, S, h, beta, y, ystride);
    for (long i = 0; i < n; ++i)
        y[i * ystride] = nlm1d_at(x, n, stride, i, S, K, h, kernel, beta);
    return 0;
}

/* Filter every row (rows=1) or every column (rows=0) of an H x W image with
 * row pitch ld (elements), writing an H x W image with pitch ldo. */
static void filter_lines(const double *in, long H, long W, long ld, int rows, int S,
                         int K, double h, int kernel, double beta, double *out,
                         long ldo, int nthreads) {
    long nlines = rows ? H : W;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
#endif
    for (long l = 0; l < nlines; ++l) {
        if (rows)
            snlm_oracle_nlm1d(in + l * ld, W, 1, S, K, h, kernel, beta, out + l * ldo, 1);
        else
            snlm_oracle_nlm1d(in + l, H, ld, S, K, h, kernel, beta, out + l, ldo);
    }
    (void)nthreads;
}

/* Separable NLM of an H x W image (Sec. 3).  order: 0 = row_col, 1 = col_row.
 * out has pitch W.  Returns 0, or -1 on bad arguments / allocation failure. */
int snlm_oracle_snlm(const double *f, long H, long W, long ld, int S, int K, double h,
                     int kernel, double beta, int order, double *out, int nthreads) {
    if (!f || !out || H < 1 || W < 1 || ld < W) return -1;
    if (bad_args(H, S, K, h, kernel, beta) || bad_args(W, S, K, h, kernel, beta)) return -1;
    if (order != ORACLE_ROW_COL && order != ORACLE_COL_ROW) return -1;
    double *mid = (double *)malloc(sizeof(double) * (size_t)H * (size_t)W);
    if (!mid) return -1;
    int first_rows = (order == ORACLE_ROW_COL);
    filter_lines(f, H, W, ld, first_rows, S, K, h, kernel, beta, mid, W, nthreads);
    filter_lines(mid, H, W, W, !first_rows, S, K, h, kernel, beta, out, W, nthreads);
    free(mid);
    return 0;
}

/* One output pixel (r, c) of the separable NLM, computed from the input alone:
 * the second pass at (r, c) needs the first-pass output along line r or c at
 * the reflected positions within reach S+K, and each of those is one sample of
 * a first-pass 1D NLM.  Used to check large images at sampled pixels. */
double snlm_oracle_pixel(const double *f, long H, long W, long ld, int S, int K,
                         double h, int kernel, double beta, int order, long r, long c) {
    if (!f || H < 1 || W < 1 || ld < W || r < 0 || r >= H || c < 0 || c >= W) return NAN;
    if (bad_args(H, S, K, h, kernel, beta) || bad_args(W, S, K, h, kernel, beta)) return NAN;
    if (kernel == ORACLE_GAUSS_IIR) return NAN; /* its distances are not local */
    int reach = S + K;
    if (order == ORACLE_ROW_COL) {
        /* second pass runs along column c; first pass along rows at column c */
        double *col = (double *)malloc(sizeof(double) * (size_t)H);
        if (!col) return NAN;
        for (long t = 0; t < H; ++t) col[t] = NAN;
        for (long m = r - reach; m <= r + reach; ++m) {
            long rr = refl(m, H);
            if (isnan(col[rr]))
                col[rr] = nlm1d_at(f + rr * ld, W, 1, c, S, K, h, kernel, beta);
        }
        double v = nlm1d_at(col, H, 1, r, S, K, h, kernel, beta);
        free(col);
        return v;
    } else if (order == ORACLE_COL_ROW) {
        double *row = (double *)malloc(sizeof(double) * (size_t)W);
        if (!row) return NAN;
        for (long t = 0; t < W; ++t) row[t] = NAN;
        for (long m = c - reach; m <= c + reach; ++m) {
            long cc = refl(m, W);
            if (isnan(row[cc]))
                row[cc] = nlm1d_at(f + cc, H, ld, r, S, K, h, kernel, beta);
        }
        double v = nlm1d_at(row, W, 1, c, S, K, h, kernel, beta);
        free(row);
        return v;
    }
    return NAN;
}

/* ------------------------------------------------------------------------
 * Recursive Gaussian patch kernel (Sec. 2.2 refers to recursive Gaussian
 * filters for the Gaussian case): the lifted diagonal D_s is smoothed by the
 * third-order recursive Gaussian of Young & van Vliet (1995), width beta,
 * forward then backward, and scaled by sqrt(2 pi) beta so that it stands for
 * the untruncated sum_k exp(-k^2 / (2 beta^2)) D_s(u + k) (g(0) = 1, as the
 * exact kernel).  Its cost does not depend on the patch width.
 *   q  = 0.98711 beta - 0.96330                      (beta >= 2.5)
 *      = 3.97156 - 4.14554 sqrt(1 - 0.26891 beta)    (0.5 <= beta < 2.5)
 *   b0 = 1.57825 + 2.44413 q + 1.4281 q^2 + 0.422205 q^3
 *   b1 = 2.44413 q + 2.85619 q^2 + 1.26661 q^3
 *   b2 = -(1.4281 q^2 + 1.26661 q^3),  b3 = 0.422205 q^3
 *   B  = 1 - (b1 + b2 + b3) / b0
 *   forward   w(v) = B D(v) + (b1 w(v-1) + b2 w(v-2) + b3 w(v-3)) / b0
 *   backward  y(v) = B w(v) + (b1 y(v+1) + b2 y(v+2) + b3 y(v+3)) / b0
 * Reading (the paper gives no details): D_s(v) = (x_e(v) - x_e(v+s))^2 over
 * the reflected line for v in [-L, n + L), L = ceil(6 beta) + S + 3; the
 * forward pass starts at -L with its three past outputs equal to D_s(-L), the
 * backward pass at n + L - 1 with its three future outputs equal to
 * w(n + L - 1) (the steady states of constant input).  beta >= 0.5.
 * ------------------------------------------------------------------------ */
static void yvv_coeffs(double beta, double *B, double *b) {
    double q = beta >= 2.5 ? 0.98711 * beta - 0.96330 : 3.97156 - 4.14554 * sqrt(1.0 - 0.26891 * beta);
    double q2 = q * q, q3 = q2 * q;
    b[0] = 1.57825 + 2.44413 * q + 1.4281 * q2 + 0.422205 * q3;
    b[1] = 2.44413 * q + 2.85619 * q2 + 1.26661 * q3;
    b[2] = -(1.4281 * q2 + 1.26661 * q3);
    b[3] = 0.422205 * q3;
    *B = 1.0 - (b[1] + b[2] + b[3]) / b[0];
}

/* The recursive Gaussian of a finite sequence (forward then backward, the
 * steady-state starts above), without the sqrt(2 pi) beta scale. */
void snlm_oracle_yvv(const double *in, long n, double beta, double *out) {
    double B, b[4];
    yvv_coeffs(beta, &B, b);
    double w1 = in[0], w2 = in[0], w3 = in[0];
    for (long v = 0; v < n; ++v) {
        double w = B * in[v] + (b[1] * w1 + b[2] * w2 + b[3] * w3) / b[0];
        out[v] = w;
        w3 = w2;
        w2 = w1;
        w1 = w;
    }
    double y1 = out[n - 1], y2 = out[n - 1], y3 = out[n - 1];
    for (long v = n - 1; v >= 0; --v) {
        double y = B * out[v] + (b[1] * y1 + b[2] * y2 + b[3] * y3) / b[0];
        out[v] = y;
        y3 = y2;
        y2 = y1;
        y1 = y;
    }
}

/* Recursive-Gaussian patch distances of one strided line: d2[(s - 1) * (n + S)
 * + (u + S)] = d2 between the patches at u and u + s, u in [-S, n). */
static int iir_distances(const double *x, long n, long stride, int S, double beta, double *d2) {
    long L = (long)ceil(6.0 * beta) + S + 3;
    long m = n + 2 * L;
    double *D = (double *)malloc(sizeof(double) * (size_t)m);
    if (!D) return -1;
    const double scale = sqrt(2.0 * M_PI) * beta;
    for (int s = 1; s <= S; ++s) {
        for (long v = -L; v < n + L; ++v) {
            double a = x[refl(v, n) * stride] - x[refl(v + s, n) * stride];
            D[v + L] = a * a;
        }
        snlm_oracle_yvv(D, m, beta, D);
        for (long u = -S; u < n; ++u) d2[(size_t)(s - 1) * (n + S) + (u + S)] = scale * D[u + L];
    }
    free(D);
    return 0;
}

/* The recursive-Gaussian distances of a contiguous line, laid out as above
 * (S rows of n + S values). */
int snlm_oracle_iir_d2(const double *x, long n, int S, double beta, double *d2) {
    if (!x || !d2 || n < 1 || S < 1 || !(beta >= 0.5)) return -1;
    return iir_distances(x, n, 1, S, beta, d2);
}

/* 1D NLM (eq. 1dNLM) with the recursive-Gaussian patch distances. */
static int nlm1d_iir(const double *x, long n, long stride, int S, double h, double beta, double *y,
                     long ystride) {
    double *d2 = (double *)malloc(sizeof(double) * (size_t)(S > 0 ? S : 1) * (size_t)(n + S));
    if (!d2) return -1;
    if (S > 0 && iir_distances(x, n, stride, S, beta, d2)) {
        free(d2);
        return -1;
    }
    for (long i = 0; i < n; ++i) {
        double P = 0.0, Q = 0.0;
        for (long j = i - S; j <= i + S; ++j) {
            double w = 1.0;
            if (j != i) {
                long lo = j < i ? j : i, s = j < i ? i - j : j - i;
                double d = d2[(size_t)(s - 1) * (n + S) + (lo + S)];
                w = (d == 0.0) ? 1.0 : exp(-d / (h * h));
            }
            P += w * x[refl(j, n) * stride];
            Q += w;
        }
        y[i * ystride] = P / Q;
    }
    free(d2);
    return 0;
}

/* ------------------------------------------------------------------------
 * SURE-optimal combination of the two orders (Sec. 3.1, Alg. 3 and Alg. 4).
 *
 *   1D NLM with its divergence (eq. div, derived in the Appendix): along with
 *   y(i) = sum_j w_ij x(j) / W_i, W_i = sum_j w_ij (eq. 1dNLM), the derivative
 *   dy(i)/dx(i) by the quotient rule of the Appendix (eq. derivfrac),
 *     dy(i)/dx(i) = (w_ii + sum_j (x(j) - y(i)) dw_ij/dx(i)) / W_i,   w_ii = 1,
 *   where the chain rule through eq. distanceSquared gives (g(0) = 1)
 *     dw_ij/dx(i) = (2 w_ij / h^2) [ (x(j) - x(i))
 *                                    + g(i-j) (x(2i-j) - x(i)) if |i-j| <= K ]
 *   (the second term: the tap k = i - j of the patch at j sits on x(i)).
 *   Expanding the sum gives eq. div term by term; Alg. 3 accumulates the
 *   same quantities in one pass.  dout(i) = din(i) dy(i)/dx(i).  For h = +inf,
 *   or h^2 = 0, the limit 1/W_i is used.  The formula is the paper's, i.e. it
 *   treats x(j), j != i, as independent of x(i) even where the reflection at a
 *   line end maps j onto i.
 *
 *   Alg. 4: delta = 1; rows then columns carry (f_r, delta_r) -> (f_rc,
 *   delta_rc); columns then rows carry (f_c, delta_c) -> (f_cr, delta_cr); the
 *   chained deltas are the divergences of eqs. partialrc / partialcr.  Then
 *     A = [sum f_rc^2, sum f_rc f_cr; sum f_rc f_cr, sum f_cr^2]      (eq. A)
 *     b = [sum f f_rc - sigma^2 sum delta_rc, sum f f_cr - sigma^2 sum delta_cr]
 *                                                                      (eq. bb)
 *   theta solves A theta = b, and the output is theta1 f_rc + theta2 f_cr
 *   (eq. snlm).  When A is singular (f_rc proportional to f_cr, e.g. h = inf)
 *   the minimum-norm minimiser theta1 = theta2 = (b1 + b2) / (sum of A) is used.
 * ------------------------------------------------------------------------ */
static void nlm1d_div_at(const double *x, long n, long stride, long i, int S, int K,
                         double h, int kernel, double beta, double *yi, double *divi) {
    const double xi = x[refl(i, n) * stride];
    const double h2 = h * h;
    double wt[2 * S + 1];
    double P = 0.0, W = 0.0;
    for (long j = i - S; j <= i + S; ++j) {
        double d2 = patch_d2(x, n, stride, i, j, K, kernel, beta);
        double w = (d2 == 0.0) ? 1.0 : exp(-d2 / h2);
        wt[j - (i - S)] = w;
        P += w * x[refl(j, n) * stride];
        W += w;
    }
    const double y = P / W;
    *yi = y;
    if (isinf(h) || h2 == 0.0) {
        *divi = 1.0 / W;
        return;
    }
    double acc = 0.0; /* sum_j (x(j) - y) dw_ij/dx(i) */
    for (long j = i - S; j <= i + S; ++j) {
        const double xj = x[refl(j, n) * stride];
        double dd = xj - xi; /* the bracket of dw_ij/dx(i) */
        if (labs(i - j) <= K) dd += tap((int)(i - j), kernel, beta) * (x[refl(2 * i - j, n) * stride] - xi);
        const double dw = 2.0 * wt[j - (i - S)] / h2 * dd;
        acc += (xj - y) * dw;
    }
    *divi = (1.0 + acc) / W;
}

/* 1D NLM with divergence of a strided line: y and dout = din * dy(i)/dx(i). */
int snlm_oracle_nlm1d_div(const double *x, long n, long stride, int S, int K, double h,
                          int kernel, double beta, const double *din, long dstride, double *y,
                          long ystride, double *dout, long ostride) {
    if (!x || !y || !dout || bad_args(n, S, K, h, kernel, beta)) return -1;
    if (kernel == ORACLE_GAUSS_IIR) return -1;
    for (long i = 0; i < n; ++i) {
        double yi, di;
        nlm1d_div_at(x, n, stride, i, S, K, h, kernel, beta, &yi, &di);
        y[i * ystride] = yi;
        dout[i * ostride] = (din ? din[i * dstride] : 1.0) * di;
    }
    return 0;
}

/* One pass of Alg. 4 over every row (rows=1) or column: (in, din) -> (out, dout),
 * all H x W with pitch W except in (pitch ld). */
static void div_lines(const double *in, long ld, const double *din, long H, long W, int rows,
                      int S, int K, double h, int kernel, double beta, double *out,
                      double *dout, int nthreads) {
    long nlines = rows ? H : W;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
#endif
    for (long l = 0; l < nlines; ++l) {
        if (rows)
            snlm_oracle_nlm1d_div(in + l * ld, W, 1, S, K, h, kernel, beta, din ? din + l * W : 0,
                                  1, out + l * W, 1, dout + l * W, 1);
        else
            snlm_oracle_nlm1d_div(in + l, H, ld, S, K, h, kernel, beta, din ? din + l : 0, W,
                                  out + l, W, dout + l, W);
    }
    (void)nthreads;
}

/* SNLM with the SURE-optimal combination (Alg. 4).  Outputs (pitch W, any may
 * not be NULL): f_rc, f_cr, their chained divergences d_rc, d_cr, the combined
 * image out, theta[2], and stats[7] = {sum f_rc^2, sum f_rc f_cr, sum f_cr^2,
 * sum f f_rc, sum f f_cr, sum d_rc, sum d_cr}. */
int snlm_oracle_sure(const double *f, long H, long W, long ld, int S, int K, double h,
                     int kernel, double beta, double sigma, double *f_rc, double *f_cr,
                     double *d_rc, double *d_cr, double *out, double *theta, double *stats,
                     int nthreads) {
    if (!f || !f_rc || !f_cr || !d_rc || !d_cr || !out || !theta || !stats) return -1;
    if (H < 1 || W < 1 || ld < W || !(sigma >= 0.0)) return -1;
    if (bad_args(H, S, K, h, kernel, beta) || bad_args(W, S, K, h, kernel, beta)) return -1;
    if (kernel == ORACLE_GAUSS_IIR) return -1;
    size_t npx = (size_t)H * (size_t)W;
    double *mid = (double *)malloc(sizeof(double) * npx);
    double *dmid = (double *)malloc(sizeof(double) * npx);
    if (!mid || !dmid) {
        free(mid);
        free(dmid);
        return -1;
    }
    div_lines(f, ld, 0, H, W, 1, S, K, h, kernel, beta, mid, dmid, nthreads);
    div_lines(mid, W, dmid, H, W, 0, S, K, h, kernel, beta, f_rc, d_rc, nthreads);
    div_lines(f, ld, 0, H, W, 0, S, K, h, kernel, beta, mid, dmid, nthreads);
    div_lines(mid, W, dmid, H, W, 1, S, K, h, kernel, beta, f_cr, d_cr, nthreads);
    free(mid);
    free(dmid);
    double a11 = 0, a12 = 0, a22 = 0, c1 = 0, c2 = 0, s1 = 0, s2 = 0;
    for (long r = 0; r < H; ++r)
        for (long c = 0; c < W; ++c) {
            size_t i = (size_t)r * W + c;
            double x = f[r * ld + c];
            a11 += f_rc[i] * f_rc[i];
            a12 += f_rc[i] * f_cr[i];
            a22 += f_cr[i] * f_cr[i];
            c1 += x * f_rc[i];
            c2 += x * f_cr[i];
            s1 += d_rc[i];
            s2 += d_cr[i];
        }
    double sg2 = sigma * sigma;
    double b1 = c1 - sg2 * s1, b2 = c2 - sg2 * s2;
    double det = a11 * a22 - a12 * a12;
    if (det > 1e-12 * a11 * a22) {
        theta[0] = (a22 * b1 - a12 * b2) / det;
        theta[1] = (a11 * b2 - a12 * b1) / det;
    } else {
        double t = (b1 + b2) / (a11 + 2.0 * a12 + a22);
        theta[0] = t;
        theta[1] = t;
    }
    for (size_t i = 0; i < npx; ++i) out[i] = theta[0] * f_rc[i] + theta[1] * f_cr[i];
    stats[0] = a11;
    stats[1] = a12;
    stats[2] = a22;
    stats[3] = c1;
    stats[4] = c2;
    stats[5] = s1;
    stats[6] = s2;
    return 0;
}

/* ------------------------------------------------------------------------
 * Separable NLM of a volume (the extension to volumes noted in the
 * conclusion): the 1D NLM of eq. 1dNLM along each axis in turn, axes[k] in
 * {0 = x (contiguous), 1 = y, 2 = z}, each pass on the previous output.
 * f and out are D x H x W with element (z, y, x) at (z H + y) W + x.
 * ------------------------------------------------------------------------ */
int snlm_oracle_snlm3d(const double *f, long D, long H, long W, int S, int K, double h,
                       int kernel, double beta, const int *axes, double *out, int nthreads) {
    if (!f || !out || !axes || D < 1 || H < 1 || W < 1) return -1;
    if (bad_args(W, S, K, h, kernel, beta)) return -1;
    int seen[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) {
        if (axes[k] < 0 || axes[k] > 2 || seen[axes[k]]) return -1;
        seen[axes[k]] = 1;
    }
    size_t npx = (size_t)D * H * W;
    double *a = (double *)malloc(sizeof(double) * npx);
    double *b = (double *)malloc(sizeof(double) * npx);
    if (!a || !b) {
        free(a);
        free(b);
        return -1;
    }
    memcpy(a, f, sizeof(double) * npx);
    for (int k = 0; k < 3; ++k) {
        int ax = axes[k];
        long n = ax == 0 ? W : (ax == 1 ? H : D);
        long stride = ax == 0 ? 1 : (ax == 1 ? W : H * W);
        long nlines = (long)(npx / (size_t)n);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
#endif
        for (long l = 0; l < nlines; ++l) {
            long base;
            if (ax == 0)
                base = l * W;                             /* line (z, y) */
            else if (ax == 1)
                base = (l / W) * H * W + (l % W);         /* line (z, x) */
            else
                base = l;                                 /* line (y, x) */
            snlm_oracle_nlm1d(a + base, n, stride, S, K, h, kernel, beta, b + base, stride);
        }
        double *t = a;
        a = b;
        b = t;
    }
    memcpy(out, a, sizeof(double) * npx);
    free(a);
    free(b);
    (void)nthreads;
    return 0;
}

/* ------------------------------------------------------------------------
 * Bilateral post-processing (Sec. 3.2, eq. BF) and its parameter rules
 * (Sec. 4.1):
 *   out(i) = sum_j w(j) g(f(i-j) - f(i)) f(i-j) / sum_j w(j) g(f(i-j) - f(i))
 *   w(j) = exp(-|j|^2 / (2 sigma_s^2)),  g(t) = exp(-t^2 / (2 sigma_r^2)),
 *   j over the integer offsets of [-3 sigma_s, 3 sigma_s]^2, i.e. |j1|, |j2| <=
 *   floor(3 sigma_s);  the image is extended by the same half-sample symmetric
 *   reflection as the NLM passes (the paper does not say).  sigma_r = +inf
 *   gives g = 1 (a normalised Gaussian blur).
 *   sigma_s = 2.5e-6 s^3 - 3.4e-4 s^2 + 0.021 s + 0.46,
 *   sigma_r = 2.8e-4 s^3 - 0.088 s^2 + 8 s - 24,   s the noise level.
 * ------------------------------------------------------------------------ */
void snlm_oracle_bf_params(double sigma, double *sigma_s, double *sigma_r) {
    double s2 = sigma * sigma, s3 = s2 * sigma;
    if (sigma_s) *sigma_s = 2.5e-6 * s3 - 3.4e-4 * s2 + 0.021 * sigma + 0.46;
    if (sigma_r) *sigma_r = 2.8e-4 * s3 - 0.088 * s2 + 8.0 * sigma - 24.0;
}

int snlm_oracle_bilateral(const double *f, long H, long W, long ld, double sigma_s,
                          double sigma_r, double *out, int nthreads) {
    if (!f || !out || H < 1 || W < 1 || ld < W) return -1;
    if (!(sigma_s > 0.0) || !(sigma_r > 0.0)) return -1;
    long R = (long)floor(3.0 * sigma_s);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
#endif
    for (long r = 0; r < H; ++r) {
        for (long c = 0; c < W; ++c) {
            double v = f[r * ld + c];
            double num = 0.0, den = 0.0;
            for (long dy = -R; dy <= R; ++dy)
                for (long dx = -R; dx <= R; ++dx) {
                    double u = f[refl(r - dy, H) * ld + refl(c - dx, W)];
                    double ws = exp(-(double)(dy * dy + dx * dx) / (2.0 * sigma_s * sigma_s));
                    double g = isinf(sigma_r) ? 1.0
                                              : exp(-(u - v) * (u - v) / (2.0 * sigma_r * sigma_r));
                    num += ws * g * u;
                    den += ws * g;
                }
            out[r * W + c] = num / den;
        }
    }
    (void)nthreads;
    return 0;
}

/* Number of threads an OpenMP region would use (1 without OpenMP). */
int snlm_oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
