/*
 * CPU oracle for single-scan min-sum LDPC decoding -- TEST INFRASTRUCTURE.
 *
 * This file is the plain, slow reference that the GPU decoder is checked
 * against.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the decoder library never links or calls it, and
 * the two share no code.
 *
 * Source: X. Huang, "Single-Scan Min-Sum Algorithms for Fast Decoding of LDPC
 * Codes", ITW 2006.  Three decoders are written out separately, each in the
 * paper's order of steps and without any blocking or reordering:
 *
 *   two_scan     Sec. III: horizontal scan Eq.(1), vertical scan Eq.(2), the
 *                posterior sum and hard decision, the stop rule; NMS/OMS
 *                modifications of Sec. III.
 *   single_scan  Sec. IV, Eq.(3): L^(0)=0; per iteration Z_n reset to Z^(0)_n,
 *                each L_mn recomputed from Z^(k-1)_{n'} - L^(k-1)_{mn'}, and
 *                Z_n accumulated in the same pass.
 *   one_bit      Sec. V: per check only A_m, B_m, n~_m and per-edge signs s_mn
 *                are kept; L^(k-1) is rebuilt through f(A,B,n,n~), and the new
 *                A, B, n~, s come from Eqs.(4),(5) with the normalised/offset
 *                forms at the end of Sec. V.
 *
 * Every check update is the literal exclusion form (a min and a sign product
 * over N(m)\n for every n), not the min1/min2 shortcut, so the oracle does not
 * rely on the observation it is used to test.
 *
 * Arithmetic variants
 *   _int : b-bit fixed point (the paper's b = 6..8 bit messages, Sec. V; the
 *          plain entry points are 6-bit, the _ex ones take b = 6, 7 or 8).
 *          With Q = 2^(b-1) - 1 (31, 63, 127): inputs are int8 in [-Q, Q];
 *          every variable-to-check value (two-scan Z_mn, single-scan
 *          Z_n - L_mn) is saturated to +-Q; accumulators are not.
 *          Normalisation/offset: |L| = max(((m*a8 + 128) >> 8) - b, 0) with
 *          a8 = round(256*alpha), b = round(beta/step) (round half away).
 *          The _ex entry points also take a schedule of one (alpha_k, beta_k)
 *          pair per iteration k (Sec. III indexes both by the iteration):
 *          iteration k uses row min(k, n_sched) - 1, each converted as above.
 *   _f32, _f64 : IEEE binary32 / binary64, no saturation; |L| =
 *          max(alpha*m - beta, 0) with the product rounded before the
 *          subtraction (build with -ffp-contract=off).
 *
 * Readings where the paper is silent or garbled (listed in the design notes):
 *   - Eq.(3) subtracts L_mn' from Z_{n'} (the printed Z_n is an index slip).
 *   - Z_n is double-buffered: iteration k reads Z^(k-1) throughout (flooding).
 *   - sgn(x) = -1 iff x < 0.
 *   - OMS acts on magnitudes: sgn(L) max(|L| - beta, 0); NMS and OMS combine
 *     as max(alpha*|L| - beta, 0).
 *   - In the 1-bit form the normalisation is applied to the emitted L (before
 *     Z_n += L), which is what makes it equal to normalised min-sum.
 *   - argmax ties in the 1-bit form go to the lowest position in the row.
 *   - The stop test runs after each iteration k >= 1; max_iter = 0 returns the
 *     channel decisions.  Hard decision: x_n = 0 iff Z_n > 0.
 *
 * Return value of every decoder: 0 on success, -1 on an invalid argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_QMAX6 31 /* Q of the 6-bit entry points */

/* ------------------------------------------------------------------------ */
/* shared helpers of the oracle itself                                       */
/* ------------------------------------------------------------------------ */

/* Transposed index: for each variable n, the edges (CSR positions) of M(n) in
 * ascending check order. */
typedef struct {
    int *ptr; /* N+1 */
    int *edge; /* E */
} orc_cols;

static int orc_cols_build(int M, int N, const int *row_ptr, const int *col_idx, orc_cols *c)
{
    int E = row_ptr[M];
    c->ptr = (int *)calloc((size_t)N + 1, sizeof(int));
    c->edge = (int *)malloc(sizeof(int) * (size_t)(E > 0 ? E : 1));
    int *fill = (int *)calloc((size_t)N + 1, sizeof(int));
    if (!c->ptr || !c->edge || !fill) { free(c->ptr); free(c->edge); free(fill); return -1; }
    for (int e = 0; e < E; ++e) c->ptr[col_idx[e] + 1]++;
    for (int n = 0; n < N; ++n) c->ptr[n + 1] += c->ptr[n];
    for (int m = 0; m < M; ++m)
        for (int e = row_ptr[m]; e < row_ptr[m + 1]; ++e) {
            int n = col_idx[e];
            c->edge[c->ptr[n] + fill[n]++] = e;
        }
    free(fill);
    return 0;
}

static void orc_cols_free(orc_cols *c) { free(c->ptr); free(c->edge); }

static int orc_check_code(int M, int N, const int *row_ptr, const int *col_idx)
{
    if (M < 0 || N < 0 || !row_ptr) return -1;
    if (row_ptr[0] != 0) return -1;
    for (int m = 0; m < M; ++m) {
        if (row_ptr[m + 1] - row_ptr[m] < 2) return -1;
        for (int e = row_ptr[m]; e < row_ptr[m + 1]; ++e)
            if (col_idx[e] < 0 || col_idx[e] >= N) return -1;
    }
    return 0;
}

/* Syndrome test of hard decisions x (0/1): 1 iff H x^T = 0. */
static int orc_syndrome_ok(int M, const int *row_ptr, const int *col_idx, const uint8_t *x)
{
    for (int m = 0; m < M; ++m) {
        int p = 0;
        for (int e = row_ptr[m]; e < row_ptr[m + 1]; ++e) p ^= x[col_idx[e]];
        if (p) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* 6-bit fixed point                                                         */
/* ------------------------------------------------------------------------ */

static int sat_q(int v, int Q) { return v > Q ? Q : (v < -Q ? -Q : v); }
static int iabs_(int v) { return v < 0 ? -v : v; }

/* Normalised/offset magnitude (Sec. III NMS and OMS in fixed point). */
static int norm_q(int mag, int a8, int b)
{
    int v = ((mag * a8 + 128) >> 8) - b;
    return v > 0 ? v : 0;
}

/* Literal check update, Eq.(1)/(3): for each position j of a row with inputs
 * t[0..d-1], L[j] = prod_{i!=j} sgn(t[i]) * norm(min_{i!=j} |t[i]|). */
static void row_update_q(int d, const int *t, int a8, int b, int *L)
{
    for (int j = 0; j < d; ++j) {
        int sign = 1, mn = -1;
        for (int i = 0; i < d; ++i) {
            if (i == j) continue;
            if (t[i] < 0) sign = -sign;
            if (mn < 0 || iabs_(t[i]) < mn) mn = iabs_(t[i]);
        }
        L[j] = sign * norm_q(mn, a8, b);
    }
}

static int params_q(double alpha, double beta, double step, int *a8, int *b)
{
    if (!(alpha > 0.0 && alpha <= 1.0) || !(beta >= 0.0) || !(step > 0.0)) return -1;
    *a8 = (int)lround(alpha * 256.0);
    /* an offset of 255 steps already exceeds every b-bit magnitude (b <= 8),
     * so every larger beta gives the same all-zero messages; the cap keeps
     * the conversion in range */
    *b = (int)lround(fmin(beta / step, 255.0));
    return 0;
}

/* Fixed-point pairs of iterations 1..max_iter: the constant (alpha, beta)
 * when sched is NULL, else row min(k, n_sched) - 1 of sched [n_sched][2]. */
static int schedule_q(int max_iter, const double *sched, int n_sched, double alpha, double beta,
                      double step, int *a8k, int *bk)
{
    for (int k = 1; k <= max_iter; ++k) {
        const int r = (k < n_sched ? k : n_sched) - 1;
        if (sched ? params_q(sched[2 * r], sched[2 * r + 1], step, &a8k[k], &bk[k])
                  : params_q(alpha, beta, step, &a8k[k], &bk[k]))
            return -1;
    }
    return 0;
}

static int qmax_of(int qbits) { return qbits >= 6 && qbits <= 8 ? (1 << (qbits - 1)) - 1 : -1; }

static int input_q_ok(long n, const int8_t *llr, int Q)
{
    for (long i = 0; i < n; ++i)
        if (llr[i] < -Q || llr[i] > Q) return 0;
    return 1;
}

/* Finish one frame: outputs and trace are written by the callers; this only
 * computes hard decisions from posteriors. */
static void decide_q(int N, const int *Z, uint8_t *x)
{
    for (int n = 0; n < N; ++n) x[n] = Z[n] > 0 ? 0 : 1;
}

int oracle_two_scan_int(int M, int N, const int *row_ptr, const int *col_idx,
                        int n_frames, const int8_t *llr, int max_iter,
                        double alpha, double beta, int early_stop, double step,
                        float *post_out, uint8_t *hard_out, int32_t *iters_out,
                        uint8_t *ok_out, int32_t *trace_L, int32_t *trace_Z,
                        int32_t *trace_Zmn)
{
    int a8, b;
    if (orc_check_code(M, N, row_ptr, col_idx) || n_frames < 0 || max_iter < 0 ||
        params_q(alpha, beta, step, &a8, &b) || !input_q_ok((long)n_frames * N, llr, ORC_QMAX6))
        return -1;
    const int E = row_ptr[M];
    orc_cols cols;
    if (orc_cols_build(M, N, row_ptr, col_idx, &cols)) return -1;
    int *Z0 = (int *)malloc(sizeof(int) * ((size_t)N + 1));
    int *Zn = (int *)malloc(sizeof(int) * ((size_t)N + 1));
    int *Zmn = (int *)malloc(sizeof(int) * ((size_t)E + 1));
    int *L = (int *)malloc(sizeof(int) * ((size_t)E + 1));
    int *t = (int *)malloc(sizeof(int) * ((size_t)N + 1));
    int *Lr = (int *)malloc(sizeof(int) * ((size_t)N + 1));
    uint8_t *x = (uint8_t *)malloc((size_t)N + 1);
    for (int f = 0; f < n_frames; ++f) {
        const int8_t *in = llr + (size_t)f * N;
        for (int n = 0; n < N; ++n) Z0[n] = in[n];
        /* Initialisation: Z^(0)_mn = Z^(0)_n for m in M(n). */
        for (int e = 0; e < E; ++e) Zmn[e] = Z0[col_idx[e]];
        for (int n = 0; n < N; ++n) Zn[n] = Z0[n];
        decide_q(N, Zn, x);
        int k = 0;
        for (k = 1; k <= max_iter; ++k) {
            /* Horizontal scan, Eq.(1) with NMS/OMS. */
            for (int m = 0; m < M; ++m) {
                int d = row_ptr[m + 1] - row_ptr[m];
                for (int j = 0; j < d; ++j) t[j] = Zmn[row_ptr[m] + j];
                row_update_q(d, t, a8, b, Lr);
                for (int j = 0; j < d; ++j) L[row_ptr[m] + j] = Lr[j];
            }
            /* Vertical scan, Eq.(2) (each exclusion sum written out), and the
             * posterior of the decoding step. */
            for (int n = 0; n < N; ++n) {
                int s = Z0[n];
                for (int i = cols.ptr[n]; i < cols.ptr[n + 1]; ++i) s += L[cols.edge[i]];
                Zn[n] = s;
                for (int i = cols.ptr[n]; i < cols.ptr[n + 1]; ++i) {
                    int v = Z0[n];
                    for (int i2 = cols.ptr[n]; i2 < cols.ptr[n + 1]; ++i2)
                        if (i2 != i) v += L[cols.edge[i2]];
                    Zmn[cols.edge[i]] = sat_q(v, ORC_QMAX6);
                }
            }
            decide_q(N, Zn, x);
            if (trace_L) memcpy(trace_L + ((size_t)f * max_iter + (k - 1)) * E, L, sizeof(int) * E);
            if (trace_Z) memcpy(trace_Z + ((size_t)f * max_iter + (k - 1)) * N, Zn, sizeof(int) * N);
            if (trace_Zmn) memcpy(trace_Zmn + ((size_t)f * max_iter + (k - 1)) * E, Zmn, sizeof(int) * E);
            if (early_stop && orc_syndrome_ok(M, row_ptr, col_idx, x)) break;
        }
        if (k > max_iter) k = max_iter;
        for (int n = 0; n < N; ++n) {
            if (post_out) post_out[(size_t)f * N + n] = (float)(Zn[n] * step);
            if (hard_out) hard_out[(size_t)f * N + n] = x[n];
        }
        if (iters_out) iters_out[f] = k;
        if (ok_out) ok_out[f] = (uint8_t)orc_syndrome_ok(M, row_ptr, col_idx, x);
    }
    free(Z0); free(Zn); free(Zmn); free(L); free(t); free(Lr); free(x);
    orc_cols_free(&cols);
    return 0;
}

int oracle_single_scan_int_ex(int M, int N, const int *row_ptr, const int *col_idx,
                              int n_frames, const int8_t *llr, int max_iter,
                              const double *sched, int n_sched, double alpha, double beta,
                              int qbits, int early_stop, double step,
                              float *post_out, uint8_t *hard_out, int32_t *iters_out,
                              uint8_t *ok_out, int32_t *trace_L, int32_t *trace_Z)
{
    const int Q = qmax_of(qbits);
    if (orc_check_code(M, N, row_ptr, col_idx) || n_frames < 0 || max_iter < 0 || Q < 0 ||
        (sched && n_sched < 1) || !input_q_ok((long)n_frames * N, llr, Q))
        return -1;
    int *a8k = (int *)malloc(sizeof(int) * ((size_t)max_iter + 1));
    int *bk = (int *)malloc(sizeof(int) * ((size_t)max_iter + 1));
    if (schedule_q(max_iter, sched, n_sched, alpha, beta, step, a8k, bk)) {
        free(a8k); free(bk);
        return -1;
    }
    const int E = row_ptr[M];
    int *Z0 = (int *)malloc(sizeof(int) * ((size_t)N + 1));
    int *Zold = (int *)malloc(sizeof(int) * ((size_t)N + 1));
    int *Znew = (int *)malloc(sizeof(int) * ((size_t)N + 1));
    int *L = (int *)malloc(sizeof(int) * ((size_t)E + 1));
    int *t = (int *)malloc(sizeof(int) * ((size_t)N + 1));
    int *Lr = (int *)malloc(sizeof(int) * ((size_t)N + 1));
    uint8_t *x = (uint8_t *)malloc((size_t)N + 1);
    for (int f = 0; f < n_frames; ++f) {
        const int8_t *in = llr + (size_t)f * N;
        for (int n = 0; n < N; ++n) Z0[n] = in[n];
        /* Initialisation: L^(0)_mn = 0, and Z^(0)_n is the previous posterior. */
        for (int e = 0; e < E; ++e) L[e] = 0;
        for (int n = 0; n < N; ++n) Zold[n] = Z0[n];
        decide_q(N, Zold, x);
        int k = 0;
        for (k = 1; k <= max_iter; ++k) {
            for (int n = 0; n < N; ++n) Znew[n] = Z0[n];            /* Z^(k)_n = Z^(0)_n */
            for (int m = 0; m < M; ++m) {
                int d = row_ptr[m + 1] - row_ptr[m];
                const int *cn = col_idx + row_ptr[m];
                for (int j = 0; j < d; ++j)                          /* Z^(k-1)_n' - L^(k-1)_mn' */
                    t[j] = sat_q(Zold[cn[j]] - L[row_ptr[m] + j], Q);
                row_update_q(d, t, a8k[k], bk[k], Lr);               /* Eq.(3) */
                for (int j = 0; j < d; ++j) {
                    L[row_ptr[m] + j] = Lr[j];
                    Znew[cn[j]] += Lr[j];                            /* Z^(k)_n += L^(k)_mn */
                }
            }
            decide_q(N, Znew, x);
            for (int n = 0; n < N; ++n) Zold[n] = Znew[n];
            if (trace_L) memcpy(trace_L + ((size_t)f * max_iter + (k - 1)) * E, L, sizeof(int) * E);
            if (trace_Z) memcpy(trace_Z + ((size_t)f * max_iter + (k - 1)) * N, Zold, sizeof(int) * N);
            if (early_stop && orc_syndrome_ok(M, row_ptr, col_idx, x)) break;
        }
        if (k > max_iter) k = max_iter;
        for (int n = 0; n < N; ++n) {
            if (post_out) post_out[(size_t)f * N + n] = (float)(Zold[n] * step);
            if (hard_out) hard_out[(size_t)f * N + n] = x[n];
        }
        if (iters_out) iters_out[f] = k;
        if (ok_out) ok_out[f] = (uint8_t)orc_syndrome_ok(M, row_ptr, col_idx, x);
    }
    free(Z0); free(Zold); free(Znew); free(L); free(t); free(Lr); free(x); free(a8k); free(bk);
    return 0;
}

int oracle_single_scan_int(int M, int N, const int *row_ptr, const int *col_idx,
                           int n_frames, const int8_t *llr, int max_iter,
                           double alpha, double beta, int early_stop, double step,
                           float *post_out, uint8_t *hard_out, int32_t *iters_out,
                           uint8_t *ok_out, int32_t *trace_L, int32_t *trace_Z)
{
    return oracle_single_scan_int_ex(M, N, row_ptr, col_idx, n_frames, llr, max_iter, NULL, 0, alpha, beta, 6,
                                     early_stop, step, post_out, hard_out, iters_out, ok_out, trace_L, trace_Z);
}

/* Sec. V compression of one row's messages L[0..d-1]:
 * A = min |L|, B = max |L|, idx = argmax |L| (lowest position on ties),
 * s[j] = 1 iff L[j] < 0. */
void oracle_compress_row_int(int d, const int32_t *L, int32_t *A, int32_t *B,
                             int32_t *idx, uint8_t *s)
{
    int a = -1, bb = -1, ix = 0;
    for (int j = 0; j < d; ++j) {
        int v = iabs_(L[j]);
        if (a < 0 || v < a) a = v;
        if (v > bb) { bb = v; ix = j; }
        s[j] = L[j] < 0 ? 1 : 0;
    }
    *A = a; *B = bb; *idx = ix;
}

/* L_mn = s_mn * f(A, B, n, n~), with f = B at n = n~ and A elsewhere. */
void oracle_expand_row_int(int d, int32_t A, int32_t B, int32_t idx, const uint8_t *s,
                           int32_t *L)
{
    for (int j = 0; j < d; ++j) {
        int f = (j == idx) ? B : A;
        L[j] = s[j] ? -f : f;
    }
}

/* Literal check update of one row, exported for the row-level pins. */
void oracle_row_update_int(int d, const int32_t *t, double alpha, double beta,
                           double step, int32_t *L)
{
    int a8 = 256, b = 0;
    params_q(alpha, beta, step, &a8, &b);
    row_update_q(d, t, a8, b, L);
}

int oracle_one_bit_int_ex(int M, int N, const int *row_ptr, const int *col_idx,
                          int n_frames, const int8_t *llr, int max_iter,
                          const double *sched, int n_sched, double alpha, double beta,
                          int qbits, int early_stop, double step,
                          float *post_out, uint8_t *hard_out, int32_t *iters_out,
                          uint8_t *ok_out, int32_t *trace_L, int32_t *trace_Z,
                          int32_t *state_out /* [F][M][3] = A, B, n~ after the last iteration; nullable */,
                          uint8_t *sign_out /* [F][E]; nullable */)
{
    const int Q = qmax_of(qbits);
    if (orc_check_code(M, N, row_ptr, col_idx) || n_frames < 0 || max_iter < 0 || Q < 0 ||
        (sched && n_sched < 1) || !input_q_ok((long)n_frames * N, llr, Q))
        return -1;
    int *a8k = (int *)malloc(sizeof(int) * ((size_t)max_iter + 1));
    int *bk = (int *)malloc(sizeof(int) * ((size_t)max_iter + 1));
    if (schedule_q(max_iter, sched, n_sched, alpha, beta, step, a8k, bk)) {
        free(a8k); free(bk);
        return -1;
    }
    const int E = row_ptr[M];
    int *Z0 = (int *)malloc(sizeof(int) * ((size_t)N + 1));
    int *Zold = (int *)malloc(sizeof(int) * ((size_t)N + 1));
    int *Znew = (int *)malloc(sizeof(int) * ((size_t)N + 1));
    int32_t *A = (int32_t *)malloc(sizeof(int32_t) * ((size_t)M + 1));
    int32_t *B = (int32_t *)malloc(sizeof(int32_t) * ((size_t)M + 1));
    int32_t *nt = (int32_t *)malloc(sizeof(int32_t) * ((size_t)M + 1));
    uint8_t *s = (uint8_t *)malloc((size_t)E + 1);
    int32_t *Lold = (int32_t *)malloc(sizeof(int32_t) * ((size_t)N + 1));
    int32_t *Lnew = (int32_t *)malloc(sizeof(int32_t) * ((size_t)N + 1));
    int *t = (int *)malloc(sizeof(int) * ((size_t)N + 1));
    int32_t *Lall = trace_L ? (int32_t *)malloc(sizeof(int32_t) * ((size_t)E + 1)) : NULL;
    uint8_t *x = (uint8_t *)malloc((size_t)N + 1);
    for (int f = 0; f < n_frames; ++f) {
        const int8_t *in = llr + (size_t)f * N;
        for (int n = 0; n < N; ++n) Z0[n] = in[n];
        /* Initialisation: A = B = n~ = 0, s = 0 (so L^(0) = 0). */
        for (int m = 0; m < M; ++m) { A[m] = 0; B[m] = 0; nt[m] = 0; }
        for (int e = 0; e < E; ++e) s[e] = 0;
        for (int n = 0; n < N; ++n) Zold[n] = Z0[n];
        decide_q(N, Zold, x);
        int k = 0;
        for (k = 1; k <= max_iter; ++k) {
            for (int n = 0; n < N; ++n) Znew[n] = Z0[n];
            for (int m = 0; m < M; ++m) {
                int d = row_ptr[m + 1] - row_ptr[m];
                const int *cn = col_idx + row_ptr[m];
                oracle_expand_row_int(d, A[m], B[m], nt[m], s + row_ptr[m], Lold);  /* L^(k-1) */
                for (int j = 0; j < d; ++j) t[j] = sat_q(Zold[cn[j]] - Lold[j], Q);
                row_update_q(d, t, a8k[k], bk[k], Lnew);                            /* L^(k), normalised */
                for (int j = 0; j < d; ++j) Znew[cn[j]] += Lnew[j];                 /* Z += L */
                oracle_compress_row_int(d, Lnew, &A[m], &B[m], &nt[m], s + row_ptr[m]); /* Eqs.(4),(5) */
                if (Lall) for (int j = 0; j < d; ++j) Lall[row_ptr[m] + j] = Lnew[j];
            }
            decide_q(N, Znew, x);
            for (int n = 0; n < N; ++n) Zold[n] = Znew[n];
            if (trace_L) memcpy(trace_L + ((size_t)f * max_iter + (k - 1)) * E, Lall, sizeof(int32_t) * E);
            if (trace_Z) memcpy(trace_Z + ((size_t)f * max_iter + (k - 1)) * N, Zold, sizeof(int) * N);
            if (early_stop && orc_syndrome_ok(M, row_ptr, col_idx, x)) break;
        }
        if (k > max_iter) k = max_iter;
        for (int n = 0; n < N; ++n) {
            if (post_out) post_out[(size_t)f * N + n] = (float)(Zold[n] * step);
            if (hard_out) hard_out[(size_t)f * N + n] = x[n];
        }
        if (iters_out) iters_out[f] = k;
        if (ok_out) ok_out[f] = (uint8_t)orc_syndrome_ok(M, row_ptr, col_idx, x);
        if (state_out)
            for (int m = 0; m < M; ++m) {
                state_out[((size_t)f * M + m) * 3 + 0] = A[m];
                state_out[((size_t)f * M + m) * 3 + 1] = B[m];
                state_out[((size_t)f * M + m) * 3 + 2] = nt[m];
            }
        if (sign_out) memcpy(sign_out + (size_t)f * E, s, (size_t)E);
    }
    free(Z0); free(Zold); free(Znew); free(A); free(B); free(nt); free(s);
    free(Lold); free(Lnew); free(t); free(Lall); free(x); free(a8k); free(bk);
    return 0;
}

int oracle_one_bit_int(int M, int N, const int *row_ptr, const int *col_idx,
                       int n_frames, const int8_t *llr, int max_iter,
                       double alpha, double beta, int early_stop, double step,
                       float *post_out, uint8_t *hard_out, int32_t *iters_out,
                       uint8_t *ok_out, int32_t *trace_L, int32_t *trace_Z,
                       int32_t *state_out, uint8_t *sign_out)
{
    return oracle_one_bit_int_ex(M, N, row_ptr, col_idx, n_frames, llr, max_iter, NULL, 0, alpha, beta, 6,
                                 early_stop, step, post_out, hard_out, iters_out, ok_out, trace_L, trace_Z,
                                 state_out, sign_out);
}

/* ------------------------------------------------------------------------ */
/* IEEE floating point: binary32 and binary64 instantiations                */
/* ------------------------------------------------------------------------ */
#define REAL float
#define SFX(name) name##_f32
#include "oracle_float.inc"
#undef REAL
#undef SFX

#define REAL double
#define SFX(name) name##_f64
#include "oracle_float.inc"
#undef REAL
#undef SFX
