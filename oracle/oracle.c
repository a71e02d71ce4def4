/*
 * oracle.c -- plain CPU reference for the lower-bound iteration of
 * Heineman, Miller, Reichman, Salls, Sarkozy, Soiffer, "Improved Lower Bounds
 * on the Expected Length of Longest Common Subsequences" (arXiv 2407.10925).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU library
 * never links, loads or calls it; the two share no source, header or table.
 *
 * Everything is single-threaded FP64, written to be checked against the
 * paper by eye, with no blocking, fusion or reordering:
 *
 *   - a head-string tuple A = (a_1..a_d), a_j in Sigma^l, is kept decoded as
 *     symbol arrays; the vector index is an independent mixed-radix encoder
 *     (position-major, string 1 first, the heads most significant), which for
 *     sigma = 2 and d = 2 is the interleaved pair of Sec. 3.2 ("Indexing");
 *   - F_z follows Algorithm 1 ("Calculating F_z"): the strings whose head is
 *     not z drop their head and take one appended symbol each, every appended
 *     tuple in Sigma^|N| is visited, and the lag-|N| vector is averaged;
 *   - F(A) = b(A) + max_z F_z(A) is eq. (4) (which merges the all-match
 *     inequality (2) and the branch inequality (3));
 *   - the driver follows Algorithm 2 ("The Feasible Triplet Algorithm"): a
 *     ring of d+1 vectors, R = max_j (v_d - v_{d-1})[j], then
 *     W = v_d + dR - F(v_d + (d-1)R, ..., v_d), E = max(0, max W), keep
 *     (u, r, eps) when R - E >= r - eps, and the bound d (r - eps) of eq. (6);
 *   - the optimal certificate of a single table u is the largest r for which
 *     (u, r, 0) satisfies the feasibility inequality of the lemma of Sec. 2.1:
 *     r* = min_A max_z (b(A) + mean_z(u) - u[A]) / |N_z|, bound d r*
 *     (derived below, at or_certify_optimal);
 *   - W_n(a_1..a_d) of Sec. 2.1 is evaluated exactly by enumerating every
 *     random tail and running the textbook LCS dynamic programme.
 *
 * Readings of points the paper leaves open:
 *   - F_z with N empty (z equal to the common head of an all-match tuple)
 *     would read a vector "v_0" that Algorithm 1 does not receive; that branch
 *     is skipped, so the all-match value is exactly 1 + the mean of eq. (2).
 *   - Argument k of F is the vector k steps back (lag k); a branch moving |N|
 *     strings reads lag |N| (Algorithm 1 reads v_|N|).
 *   - The sum over the sigma^|N| appended tuples is taken as a pairwise
 *     (balanced binary) tree over the tuples in lexicographic order, c_1 most
 *     significant; the mean is that sum divided by sigma^|N|.  Division by a
 *     power of two is exact, so for sigma in {2,4} this is the exact mean of
 *     the rounded sum.  For sigma = 2 the leaves are the tuples t with
 *     c_1 = 0, in lexicographic order, each followed by its complement
 *     (00, 11, 01, 10 for |N| = 2).  Complementing every appended symbol
 *     maps each pair to itself, and for |N| = 2 so does exchanging the two
 *     moved strings, so the tree only sees the two operands of some
 *     additions swapped: F then keeps the complement symmetry of eq. (10)
 *     and, for d = 2, the exchange of the two strings bit for bit.  For
 *     sigma = 4 and two moved strings the sixteen leaves (c_1 c_2) are, in
 *     order, the pairs {ab, ba} with a xor b = 1 (01 10 23 32), = 2
 *     (02 20 13 31), = 3 (03 30 12 21), then {aa, ~a~a} (00 33 11 22), ~ the
 *     complement of a symbol (xor 3): every relabelling c -> c xor m and the
 *     exchange of the two moved strings map pairs to pairs and each group of
 *     four to a group of four, so the tree keeps both symmetries bit for bit.
 *   - The certificate is made rigorous by directed rounding: the arguments
 *     v_d + (d-k)R and every step of F are rounded toward -inf, W and E
 *     toward +inf, and the reported bound d (R - E) toward -inf.  The C
 *     rounding mode is switched with fesetround and the file is compiled with
 *     -frounding-math -ffp-contract=off.  gcc does not promise to keep
 *     floating-point operations on the right side of a mode switch, so single
 *     operations go through rnd_add / rnd_mul (operands and result held in
 *     volatile objects between the switches) and F itself is evaluated by a
 *     call that is never inlined.
 */
#include <fenv.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_D 16
#define OR_MAX_H 40

typedef struct {
    int sigma, d, h;
    uint64_t n_entries; /* sigma^(d*h) */
} or_shape;

/* ------------------------------------------------------------------ */
/* tuple <-> index                                                     */
/* ------------------------------------------------------------------ */

static int shape_init(or_shape *s, int sigma, int d, int h)
{
    if (sigma < 2 || d < 1 || d > OR_MAX_D || h < 1 || h > OR_MAX_H) return -1;
    s->sigma = sigma; s->d = d; s->h = h;
    double approx = pow((double)sigma, (double)d * h);
    if (approx > 18446744073709551615.0) return -1;
    uint64_t n = 1;
    for (int i = 0; i < d * h; ++i) n *= (uint64_t)sigma;
    s->n_entries = n;
    return 0;
}

/* sym[j*h + p] = symbol p (p = 0 is the head) of string j.  The digits of the
 * index, most significant first, are a_1[0], a_2[0], ..., a_d[0], a_1[1], ... */
static void decode(const or_shape *s, uint64_t idx, int *sym)
{
    for (int p = s->h - 1; p >= 0; --p)
        for (int j = s->d - 1; j >= 0; --j) {
            sym[j * s->h + p] = (int)(idx % (uint64_t)s->sigma);
            idx /= (uint64_t)s->sigma;
        }
}

static uint64_t encode(const or_shape *s, const int *sym)
{
    uint64_t idx = 0;
    for (int p = 0; p < s->h; ++p)
        for (int j = 0; j < s->d; ++j)
            idx = idx * (uint64_t)s->sigma + (uint64_t)sym[j * s->h + p];
    return idx;
}

static uint64_t ipow(int base, int e)
{
    uint64_t r = 1;
    for (int i = 0; i < e; ++i) r *= (uint64_t)base;
    return r;
}

/* balanced binary tree over x[0..n) (left half first) */
static double pairwise_sum(const double *x, uint64_t n)
{
    if (n == 1) return x[0];
    uint64_t m = n / 2;
    return pairwise_sum(x, m) + pairwise_sum(x + m, n - m);
}

/* ------------------------------------------------------------------ */
/* F_z and F at one coordinate (Algorithm 1, eq. (4))                  */
/* ------------------------------------------------------------------ */

/* Reads of lag k go through lag_value(k, index).  shift[k] is added to every
 * value read from lag k before it is averaged (no shift for the plain
 * iteration, (d-k)R for the certificate's F(v_d + (d-1)R, ..., v_d)). */
typedef struct {
    const void *const *lag;   /* lag[k] for k = 1..d; lag[0] unused */
    int f32;                  /* lag tables hold floats (read as exact doubles) */
    const double *shift;      /* shift[k] for k = 1..d, or NULL */
    const double *delta;      /* delta[k] added to the mean of a branch moving
                                 k >= 2 strings (the two-array step), or NULL */
} or_args;

static double lag_value(const or_args *a, int k, uint64_t idx)
{
    double v = a->f32 ? (double)((const float *)a->lag[k])[idx] : ((const double *)a->lag[k])[idx];
    if (a->shift) v = v + a->shift[k];
    return v;
}

/* F_z(lag_1..lag_d, A) of Algorithm 1; returns 0 and sets *skip when N is
 * empty (see the reading above). */
static double F_z(const or_shape *s, const or_args *a, const int *sym, int z,
                  double *buf, int *work, int *skip)
{
    int N[OR_MAX_D], k = 0;
    for (int j = 0; j < s->d; ++j)
        if (sym[j * s->h] != z) N[k++] = j;
    if (k == 0) { *skip = 1; return 0.0; }
    *skip = 0;
    uint64_t count = ipow(s->sigma, k);
    for (uint64_t t = 0; t < count; ++t) {
        /* (c_1..c_k): lexicographic, c_1 the most significant digit of t */
        memcpy(work, sym, sizeof(int) * (size_t)(s->d * s->h));
        uint64_t rest = t;
        for (int i = k - 1; i >= 0; --i) {
            int c = (int)(rest % (uint64_t)s->sigma);
            rest /= (uint64_t)s->sigma;
            int j = N[i];
            /* string j drops its head and ends with the appended symbol c */
            for (int p = 0; p + 1 < s->h; ++p) work[j * s->h + p] = sym[j * s->h + p + 1];
            work[j * s->h + s->h - 1] = c;
        }
        buf[t] = lag_value(a, k, encode(s, work));
    }
    if (s->sigma == 2 && count > 2) {
        /* complement-paired leaf order: t, ~t for t = 0 .. count/2 - 1 */
        double *leaves = buf + count;  /* the scratch holds 2 sigma^d values */
        for (uint64_t j = 0; j < count; ++j) {
            uint64_t t = j >> 1;
            leaves[j] = buf[(j & 1) ? count - 1 - t : t];
        }
        return pairwise_sum(leaves, count) / (double)count;
    }
    if (s->sigma == 4 && count == 16) {
        /* exchange- and relabel-invariant order of the tuples 4 c_1 + c_2 */
        static const int order16[16] = {1, 4, 11, 14, 2, 8, 7, 13, 3, 12, 6, 9, 0, 15, 5, 10};
        double *leaves = buf + count;
        for (int j = 0; j < 16; ++j) leaves[j] = buf[order16[j]];
        return pairwise_sum(leaves, count) / (double)count;
    }
    return pairwise_sum(buf, count) / (double)count;
}

/* F(...)[A] = b(A) + max_z F_z(..., A), eq. (4) */
static double F_at(const or_shape *s, const or_args *a, uint64_t idx,
                   double *buf, int *sym, int *work)
{
    decode(s, idx, sym);
    int all_match = 1;
    for (int j = 1; j < s->d; ++j)
        if (sym[j * s->h] != sym[0]) all_match = 0;
    double best = -INFINITY;
    for (int z = 0; z < s->sigma; ++z) {
        int skip;
        double v = F_z(s, a, sym, z, buf, work, &skip);
        if (skip) continue;
        if (a->delta) {
            int k = 0;
            for (int j = 0; j < s->d; ++j)
                if (sym[j * s->h] != z) ++k;
            if (k >= 2) v = v + a->delta[k];
        }
        if (v > best) best = v;
    }
    return all_match ? 1.0 + best : best;
}

/* a + b and a * b under rounding `mode`: the operands are read and the result
 * written through volatile objects between the two switches, so the operation
 * cannot be moved outside them. */
static double rnd_add(double a, double b, int mode)
{
    volatile double x = a, y = b;
    fesetround(mode);
    volatile double r = x + y;
    fesetround(FE_TONEAREST);
    return r;
}

static double rnd_mul(double a, double b, int mode)
{
    volatile double x = a, y = b;
    fesetround(mode);
    volatile double r = x * y;
    fesetround(FE_TONEAREST);
    return r;
}

/* F at one coordinate with every step rounded toward -inf */
static __attribute__((noinline)) double F_at_noinline(const or_shape *s, const or_args *a,
                                                      uint64_t idx, double *buf, int *sym,
                                                      int *work)
{
    return F_at(s, a, idx, buf, sym, work);
}

static double F_at_down(const or_shape *s, const or_args *a, uint64_t idx, double *buf,
                        int *sym, int *work)
{
    fesetround(FE_DOWNWARD);
    volatile double f = F_at_noinline(s, a, idx, buf, sym, work);
    fesetround(FE_TONEAREST);
    return f;
}

/* scratch for one F evaluation */
typedef struct { double *buf; int *sym; int *work; } or_scratch;

static int scratch_alloc(const or_shape *s, or_scratch *w)
{
    w->buf = (double *)malloc(2 * sizeof(double) * ipow(s->sigma, s->d));
    w->sym = (int *)malloc(sizeof(int) * (size_t)(s->d * s->h));
    w->work = (int *)malloc(sizeof(int) * (size_t)(s->d * s->h));
    return (w->buf && w->sym && w->work) ? 0 : -1;
}

static void scratch_free(or_scratch *w)
{
    free(w->buf); free(w->sym); free(w->work);
}

/* ------------------------------------------------------------------ */
/* exported: shape, codec                                              */
/* ------------------------------------------------------------------ */

uint64_t or_num_entries(int sigma, int d, int h)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h)) return 0;
    return s.n_entries;
}

int or_decode(int sigma, int d, int h, uint64_t idx, int *sym)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h) || idx >= s.n_entries) return -1;
    decode(&s, idx, sym);
    return 0;
}

uint64_t or_encode(int sigma, int d, int h, const int *sym)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h)) return UINT64_MAX;
    return encode(&s, sym);
}

/* ------------------------------------------------------------------ */
/* exported: one sweep v_new = F(lag_1, ..., lag_d)                     */
/* ------------------------------------------------------------------ */

/* lags[k-1] = vector k steps back, k = 1..d.  Writes every coordinate of out. */
int or_sweep(int sigma, int d, int h, const double *const *lags, double *out)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h)) return -1;
    const void *lag[OR_MAX_D + 1];
    lag[0] = NULL;
    for (int k = 1; k <= d; ++k) lag[k] = lags[k - 1];
    or_args a = {lag, 0, NULL};
    or_scratch w;
    if (scratch_alloc(&s, &w)) { scratch_free(&w); return -2; }
    for (uint64_t i = 0; i < s.n_entries; ++i) out[i] = F_at(&s, &a, i, w.buf, w.sym, w.work);
    scratch_free(&w);
    return 0;
}

/* Same as or_sweep, for a list of coordinates only (sampled checks). */
static int sweep_at(int sigma, int d, int h, const void *const *lags, int f32,
                    const uint64_t *idx, uint64_t count, double *out)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h)) return -1;
    const void *lag[OR_MAX_D + 1];
    lag[0] = NULL;
    for (int k = 1; k <= d; ++k) lag[k] = lags[k - 1];
    or_args a = {lag, f32, NULL};
    or_scratch w;
    if (scratch_alloc(&s, &w)) { scratch_free(&w); return -2; }
    for (uint64_t i = 0; i < count; ++i) {
        if (idx[i] >= s.n_entries) { scratch_free(&w); return -1; }
        out[i] = F_at(&s, &a, idx[i], w.buf, w.sym, w.work);
    }
    scratch_free(&w);
    return 0;
}

int or_sweep_at(int sigma, int d, int h, const double *const *lags,
                const uint64_t *idx, uint64_t count, double *out)
{
    return sweep_at(sigma, d, h, (const void *const *)lags, 0, idx, count, out);
}

/* float tables, every value read as the double it represents exactly */
int or_sweep_at_f32(int sigma, int d, int h, const float *const *lags,
                    const uint64_t *idx, uint64_t count, double *out)
{
    return sweep_at(sigma, d, h, (const void *const *)lags, 1, idx, count, out);
}

/* ------------------------------------------------------------------ */
/* exported: the certificate of one iterate (Algorithm 2, eq. (6))     */
/* ------------------------------------------------------------------ */

typedef struct {
    double R;      /* max_j (u - prev)[j], round to nearest                    */
    double maxW;   /* max_j W[j], W = u + dR - F(u+(d-1)R, ..., u), rounded up  */
    double E;      /* max(0, maxW)                                             */
    double bound;  /* d (R - E), rounded down; meaningful when R - E >= 0       */
    double rho;    /* R - E, rounded down                                      */
    uint64_t argmax_W;   /* a coordinate where W attains maxW (lowest index)   */
    uint64_t nonfinite;  /* number of coordinates where u, prev or W is not finite */
} or_cert;

/* W[A] for a given R, with the rounding directions stated above.  Must be
 * called with the rounding mode at FE_TONEAREST; restores it. */
static double W_at(const or_shape *s, const void *u, int f32, double R, uint64_t idx,
                   const void *const *lag, const double *shift, or_scratch *w)
{
    or_args a = {lag, f32, shift};
    double f_lo = F_at_down(s, &a, idx, w->buf, w->sym, w->work);
    double dR = rnd_mul((double)s->d, R, FE_UPWARD);
    double uA = f32 ? (double)((const float *)u)[idx] : ((const double *)u)[idx];
    return rnd_add(rnd_add(uA, dR, FE_UPWARD), -f_lo, FE_UPWARD);
}

/* The d shifted arguments v_d + (d-k)R, rounded down.  Each lag reads u and
 * adds shift[k] = (d-k)R; that product is formed with rounding toward -inf
 * so the shifted argument never exceeds its exact value. */
static void make_shift(const or_shape *s, double R, double *shift)
{
    for (int k = 1; k <= s->d; ++k) shift[k] = rnd_mul((double)(s->d - k), R, FE_DOWNWARD);
}

int or_certify(int sigma, int d, int h, const double *u, const double *prev, or_cert *out)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h)) return -1;
    or_cert c;
    memset(&c, 0, sizeof c);
    /* R = max_j (v_d - v_{d-1})[j] */
    double R = -INFINITY;
    for (uint64_t i = 0; i < s.n_entries; ++i) {
        double diff = u[i] - prev[i];
        if (!isfinite(u[i]) || !isfinite(prev[i])) c.nonfinite++;
        if (diff > R) R = diff;
    }
    c.R = R;
    double shift[OR_MAX_D + 1];
    make_shift(&s, R, shift);
    const void *lag[OR_MAX_D + 1];
    lag[0] = NULL;
    for (int k = 1; k <= d; ++k) lag[k] = u;
    or_scratch w;
    if (scratch_alloc(&s, &w)) { scratch_free(&w); return -2; }
    double maxW = -INFINITY;
    uint64_t arg = 0;
    for (uint64_t i = 0; i < s.n_entries; ++i) {
        double Wv = W_at(&s, u, 0, R, i, lag, shift, &w);
        if (!isfinite(Wv)) c.nonfinite++;
        if (Wv > maxW) { maxW = Wv; arg = i; }
    }
    scratch_free(&w);
    c.maxW = maxW;
    c.argmax_W = arg;
    c.E = maxW > 0.0 ? maxW : 0.0;
    c.rho = rnd_add(c.R, -c.E, FE_DOWNWARD);
    c.bound = rnd_mul((double)d, c.rho, FE_DOWNWARD);
    *out = c;
    return 0;
}

/* W at a list of coordinates for a given R (sampled checks at sizes where a
 * whole-table pass is too slow). */
static int certify_W_at(int sigma, int d, int h, const void *u, int f32, double R,
                        const uint64_t *idx, uint64_t count, double *out)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h)) return -1;
    double shift[OR_MAX_D + 1];
    make_shift(&s, R, shift);
    const void *lag[OR_MAX_D + 1];
    lag[0] = NULL;
    for (int k = 1; k <= d; ++k) lag[k] = u;
    or_scratch w;
    if (scratch_alloc(&s, &w)) { scratch_free(&w); return -2; }
    for (uint64_t i = 0; i < count; ++i) {
        if (idx[i] >= s.n_entries) { scratch_free(&w); return -1; }
        out[i] = W_at(&s, u, f32, R, idx[i], lag, shift, &w);
    }
    scratch_free(&w);
    return 0;
}

int or_certify_W_at(int sigma, int d, int h, const double *u, double R,
                    const uint64_t *idx, uint64_t count, double *out)
{
    return certify_W_at(sigma, d, h, u, 0, R, idx, count, out);
}

int or_certify_W_at_f32(int sigma, int d, int h, const float *u, double R,
                        const uint64_t *idx, uint64_t count, double *out)
{
    return certify_W_at(sigma, d, h, u, 1, R, idx, count, out);
}

/* ------------------------------------------------------------------ */
/* exported: the largest r of a feasible triplet (u, r, 0)              */
/* ------------------------------------------------------------------ */

/*
 * The lemma of Sec. 2.1 accepts any triplet (u, r, eps) with 0 <= eps <= r and
 * F(u + (d-1)r, ..., u + r, u) >= u + (d r - eps) 1; Algorithm 2 fixes r to
 * the largest step of the last sweep and then finds eps.  For a fixed u the
 * best certificate is instead the largest r with eps = 0.  Branch z of
 * coordinate A moves k_z = |N_z| strings and so reads argument k_z, which is
 * u + (d - k_z) r; every argument moves by the same r, so that branch
 * contributes b(A) + mean_z(u) + (d - k_z) r to F (eq. (4)).  The inequality
 * at A with eps = 0 therefore holds iff some branch has
 *     c_z(A) = b(A) + mean_z(u) - u[A] >= k_z r,
 * and the largest r for which it holds at every A is
 *     r* = min_A max_z c_z(A) / k_z,
 * with bound d r* by eq. (6) (a triplet needs r* >= 0).
 *
 * Rounding: every mean, the 1 + of an all-match tuple and the subtraction of
 * u[A] are rounded toward -inf, so each computed c_z is at most its exact
 * value; the division by k_z is a multiply by 1/k_z, exact for powers of two,
 * otherwise by 1/k_z rounded down (c_z >= 0) or up (c_z < 0), the product
 * rounded toward -inf.  Every q_z is then at most c_z / k_z, the computed r
 * at most r*, and (u, r, 0) is a feasible triplet for the table given.
 * Branches whose mean is NaN never win the max over z (which starts from
 * -inf), as in F; a zero ratio is taken as +0, so the max over z does not
 * depend on the order the branches are visited in (the sign of a zero r
 * means nothing for the bound).
 */

/* a / b under rounding `mode` (see rnd_add) */
static double rnd_div(double a, double b, int mode)
{
    volatile double x = a, y = b;
    fesetround(mode);
    volatile double r = x / y;
    fesetround(FE_TONEAREST);
    return r;
}

/* inv_lo[k] <= 1/k <= inv_hi[k] for k = 1..d (equal, and exact, for powers of two) */
static void make_inverses(const or_shape *s, double *inv_lo, double *inv_hi)
{
    for (int k = 1; k <= s->d; ++k) {
        inv_lo[k] = rnd_div(1.0, (double)k, FE_DOWNWARD);
        inv_hi[k] = rnd_div(1.0, (double)k, FE_UPWARD);
    }
}

/* max_z c_z(A) / k_z at one coordinate.  Every operation here runs in the
 * rounding mode of the caller (FE_DOWNWARD); the call is never inlined, so no
 * operation can move across the caller's mode switches. */
static __attribute__((noinline)) double opt_ratio_core(const or_shape *s, const or_args *a,
                                                        uint64_t idx, double uA,
                                                        const double *inv_lo,
                                                        const double *inv_hi, double *buf,
                                                        int *sym, int *work)
{
    decode(s, idx, sym);
    int all_match = 1;
    for (int j = 1; j < s->d; ++j)
        if (sym[j * s->h] != sym[0]) all_match = 0;
    double best = -INFINITY;
    for (int z = 0; z < s->sigma; ++z) {
        int skip;
        double m = F_z(s, a, sym, z, buf, work, &skip);
        if (skip) continue;
        int k = 0;
        for (int j = 0; j < s->d; ++j)
            if (sym[j * s->h] != z) ++k;
        double c = (all_match ? 1.0 + m : m) - uA;
        double q = c >= 0.0 ? c * inv_lo[k] : c * inv_hi[k];
        if (q == 0.0) q = 0.0;  /* +0 for either zero: the max is then the same in any order */
        if (q > best) best = q;
    }
    return best;
}

static double opt_ratio_at(const or_shape *s, const or_args *a, uint64_t idx, double uA,
                           const double *inv_lo, const double *inv_hi, double *buf, int *sym,
                           int *work)
{
    fesetround(FE_DOWNWARD);
    volatile double q = opt_ratio_core(s, a, idx, uA, inv_lo, inv_hi, buf, sym, work);
    fesetround(FE_TONEAREST);
    return q;
}

typedef struct {
    double r;          /* min_A max_z c_z(A) / k_z, rounded down as above        */
    double bound;      /* d r, rounded down                                      */
    uint64_t argmin;   /* lowest coordinate attaining r                          */
    uint64_t nonfinite;/* coordinates whose ratio is not finite                  */
} or_cert_opt;

static int certify_optimal(int sigma, int d, int h, const void *u, int f32, or_cert_opt *out)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h)) return -1;
    const void *lag[OR_MAX_D + 1];
    lag[0] = NULL;
    for (int k = 1; k <= d; ++k) lag[k] = u;
    or_args a = {lag, f32, NULL};
    double inv_lo[OR_MAX_D + 1], inv_hi[OR_MAX_D + 1];
    make_inverses(&s, inv_lo, inv_hi);
    or_scratch w;
    if (scratch_alloc(&s, &w)) { scratch_free(&w); return -2; }
    or_cert_opt c;
    memset(&c, 0, sizeof c);
    c.r = INFINITY;
    for (uint64_t i = 0; i < s.n_entries; ++i) {
        double uA = f32 ? (double)((const float *)u)[i] : ((const double *)u)[i];
        double q = opt_ratio_at(&s, &a, i, uA, inv_lo, inv_hi, w.buf, w.sym, w.work);
        if (!isfinite(q)) c.nonfinite++;
        if (q < c.r) { c.r = q; c.argmin = i; }
    }
    scratch_free(&w);
    c.bound = rnd_mul((double)d, c.r, FE_DOWNWARD);
    *out = c;
    return 0;
}

int or_certify_optimal(int sigma, int d, int h, const double *u, or_cert_opt *out)
{
    return certify_optimal(sigma, d, h, u, 0, out);
}

int or_certify_optimal_f32(int sigma, int d, int h, const float *u, or_cert_opt *out)
{
    return certify_optimal(sigma, d, h, u, 1, out);
}

/* max_z c_z(A) / k_z at a list of coordinates (sampled checks) */
static int optimal_ratio_at(int sigma, int d, int h, const void *u, int f32,
                            const uint64_t *idx, uint64_t count, double *out)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h)) return -1;
    const void *lag[OR_MAX_D + 1];
    lag[0] = NULL;
    for (int k = 1; k <= d; ++k) lag[k] = u;
    or_args a = {lag, f32, NULL};
    double inv_lo[OR_MAX_D + 1], inv_hi[OR_MAX_D + 1];
    make_inverses(&s, inv_lo, inv_hi);
    or_scratch w;
    if (scratch_alloc(&s, &w)) { scratch_free(&w); return -2; }
    for (uint64_t i = 0; i < count; ++i) {
        if (idx[i] >= s.n_entries) { scratch_free(&w); return -1; }
        double uA = f32 ? (double)((const float *)u)[idx[i]] : ((const double *)u)[idx[i]];
        out[i] = opt_ratio_at(&s, &a, idx[i], uA, inv_lo, inv_hi, w.buf, w.sym, w.work);
    }
    scratch_free(&w);
    return 0;
}

int or_optimal_ratio_at(int sigma, int d, int h, const double *u, const uint64_t *idx,
                        uint64_t count, double *out)
{
    return optimal_ratio_at(sigma, d, h, u, 0, idx, count, out);
}

int or_optimal_ratio_at_f32(int sigma, int d, int h, const float *u, const uint64_t *idx,
                            uint64_t count, double *out)
{
    return optimal_ratio_at(sigma, d, h, u, 1, idx, count, out);
}

/* ------------------------------------------------------------------ */
/* exported: the two-array iteration                                   */
/* ------------------------------------------------------------------ */

/*
 * Sec. 3.3 remarks that the recurrence can be run on two arrays instead of a
 * ring, without saying how.  The reading taken here keeps one table u and a
 * rate R: the d arguments of F are u and the earlier tables as the iteration
 * would have them if every coordinate had grown by R per step,
 *     u_new = F(u, u - R, .., u - (d-1) R),
 * which (translation invariance, property 2 of the lemma) is the ring's step
 * whenever v_{n-k} = v_n - k R; at the ring's limit every coordinate grows by
 * the same r, so the two iterations share their fixed points.  Of the two
 * stored arrays one is u, the other receives u_new.  The shift is applied to
 * each branch mean: a branch moving k >= 2 strings gives mean_z(u) + delta_k,
 * delta_k = -(k-1) R (a branch moving one string reads u itself).
 *
 * R of the next step is the mean growth over a fixed sample of coordinates:
 * c_i = (i * 0x9E3779B97F4A7C15 mod 2^64) mod (n / sigma), i = 0 .. 4095
 * (coordinates whose string 1 starts with symbol 0; a multiplicative hash
 * spreads them over the table), R = (pairwise sum over i of
 * (u_new - u)[c_i]) / 4096.  The iteration, its certificates and its limit
 * do not depend on how R is chosen beyond the speed of convergence (every
 * table gives a rigorous certificate); this choice costs one small pass.
 */
#define OR_SAMPLE 4096

static uint64_t sample_coordinate(const or_shape *s, uint64_t i)
{
    return (i * 0x9E3779B97F4A7C15ull) % (s->n_entries / (uint64_t)s->sigma);
}

/* u_new = F(u, u - R, .., u - (d-1) R) at every coordinate */
int or_two_array_step(int sigma, int d, int h, const double *u, double R, double *out)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h)) return -1;
    const void *lag[OR_MAX_D + 1];
    double delta[OR_MAX_D + 1];
    lag[0] = NULL;
    delta[0] = delta[1] = 0.0;
    for (int k = 1; k <= d; ++k) lag[k] = u;
    for (int k = 2; k <= d; ++k) delta[k] = -((double)(k - 1) * R);
    or_args a = {lag, 0, NULL, delta};
    or_scratch w;
    if (scratch_alloc(&s, &w)) { scratch_free(&w); return -2; }
    for (uint64_t i = 0; i < s.n_entries; ++i) out[i] = F_at(&s, &a, i, w.buf, w.sym, w.work);
    scratch_free(&w);
    return 0;
}

/* the same step at a list of coordinates only (sampled checks) */
int or_two_array_step_at(int sigma, int d, int h, const double *u, double R,
                         const uint64_t *idx, uint64_t count, double *out)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h)) return -1;
    const void *lag[OR_MAX_D + 1];
    double delta[OR_MAX_D + 1];
    lag[0] = NULL;
    delta[0] = delta[1] = 0.0;
    for (int k = 1; k <= d; ++k) lag[k] = u;
    for (int k = 2; k <= d; ++k) delta[k] = -((double)(k - 1) * R);
    or_args a = {lag, 0, NULL, delta};
    or_scratch w;
    if (scratch_alloc(&s, &w)) { scratch_free(&w); return -2; }
    for (uint64_t i = 0; i < count; ++i) {
        if (idx[i] >= s.n_entries) { scratch_free(&w); return -1; }
        out[i] = F_at(&s, &a, idx[i], w.buf, w.sym, w.work);
    }
    scratch_free(&w);
    return 0;
}

/* the rate of the next step: mean of u_new - u over the sample */
int or_sample_growth(int sigma, int d, int h, const double *u_new, const double *u, double *R)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h)) return -1;
    double *diff = (double *)malloc(sizeof(double) * OR_SAMPLE);
    if (!diff) return -2;
    for (uint64_t i = 0; i < OR_SAMPLE; ++i) {
        uint64_t c = sample_coordinate(&s, i);
        diff[i] = u_new[c] - u[c];
    }
    *R = pairwise_sum(diff, OR_SAMPLE) / (double)OR_SAMPLE;
    free(diff);
    return 0;
}

/* the sample's coordinates (for tests) */
int or_sample_coordinates(int sigma, int d, int h, uint64_t *out)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h)) return -1;
    for (uint64_t i = 0; i < OR_SAMPLE; ++i) out[i] = sample_coordinate(&s, i);
    return 0;
}

/* R = max_j (u - prev)[j] of Algorithm 2 alone (round to nearest), for
 * whole tables too large for or_certify; the float variant reads exact
 * doubles.  *arg = lowest index attaining it. */
int or_max_diff(const double *u, const double *prev, uint64_t n, double *R, uint64_t *arg)
{
    double best = -INFINITY;
    uint64_t at = 0;
    for (uint64_t i = 0; i < n; ++i) {
        double diff = u[i] - prev[i];
        if (diff > best) { best = diff; at = i; }
    }
    *R = best;
    *arg = at;
    return 0;
}

int or_max_diff_f32(const float *u, const float *prev, uint64_t n, double *R, uint64_t *arg)
{
    double best = -INFINITY;
    uint64_t at = 0;
    for (uint64_t i = 0; i < n; ++i) {
        double diff = (double)u[i] - (double)prev[i];
        if (diff > best) { best = diff; at = i; }
    }
    *R = best;
    *arg = at;
    return 0;
}

/* ------------------------------------------------------------------ */
/* exported: the Feasible Triplet driver (Algorithm 2)                 */
/* ------------------------------------------------------------------ */

/*
 * Runs n_sweeps applications of F from the all-zero ring (the first sweep
 * produces v_d from v_{d-1} = ... = v_0 = 0).  Every `cadence` sweeps the
 * newest vector is certified and the best triplet is kept with the rule
 * R - E >= r - eps (a later iterate wins ties).  Algorithm 2 certifies after
 * every sweep, which is cadence = 1.
 *
 * hist (optional, 4 doubles per certified sweep): sweep number, R, E, bound.
 * best (4 doubles): sweep number, r, eps, bound; all zero when nothing beat
 * the initial triplet (v_0, 0, 0).
 * final_ring (optional, d tables of N doubles): lag 1 .. lag d at the end.
 */
int or_feasible_triplet(int sigma, int d, int h, int64_t n_sweeps, int64_t cadence,
                        double *hist, double *best, double *final_ring)
{
    or_shape s;
    if (shape_init(&s, sigma, d, h) || n_sweeps < 0 || cadence < 1) return -1;
    uint64_t N = s.n_entries;
    double **ring = (double **)calloc((size_t)d + 1, sizeof(double *));
    if (!ring) return -2;
    for (int i = 0; i <= d; ++i) {
        ring[i] = (double *)calloc(N, sizeof(double));
        if (!ring[i]) {
            for (int k = 0; k < i; ++k) free(ring[k]);
            free(ring);
            return -2;
        }
    }
    /* ring[0] is the newest vector (lag 1), ring[d] the slot to overwrite */
    double r_best = 0.0, eps_best = 0.0, bound_best = 0.0, sweep_best = 0.0;
    int64_t nh = 0;
    int rc = 0;
    for (int64_t t = 1; t <= n_sweeps; ++t) {
        const double *lags[OR_MAX_D];
        for (int k = 1; k <= d; ++k) lags[k - 1] = ring[k - 1];
        rc = or_sweep(sigma, d, h, lags, ring[d]);
        if (rc) break;
        /* shift the rows: the new vector becomes lag 1 */
        double *newest = ring[d];
        for (int k = d; k > 0; --k) ring[k] = ring[k - 1];
        ring[0] = newest;
        if (t % cadence == 0) {
            or_cert c;
            rc = or_certify(sigma, d, h, ring[0], ring[1], &c);
            if (rc) break;
            if (hist) {
                hist[4 * nh + 0] = (double)t;
                hist[4 * nh + 1] = c.R;
                hist[4 * nh + 2] = c.E;
                hist[4 * nh + 3] = c.bound;
            }
            nh++;
            /* keep (u, r, eps) <- (v_d, R, E) when R - E >= r - eps */
            double cur = rnd_add(c.R, -c.E, FE_DOWNWARD);
            double old = rnd_add(r_best, -eps_best, FE_DOWNWARD);
            if (c.nonfinite == 0 && cur >= old) {
                r_best = c.R; eps_best = c.E; bound_best = c.bound; sweep_best = (double)t;
            }
        }
    }
    if (best) {
        best[0] = sweep_best; best[1] = r_best; best[2] = eps_best; best[3] = bound_best;
    }
    if (final_ring && rc == 0)
        for (int k = 0; k < d; ++k) memcpy(final_ring + (uint64_t)k * N, ring[k], N * sizeof(double));
    for (int i = 0; i <= d; ++i) free(ring[i]);
    free(ring);
    return rc;
}

/* ------------------------------------------------------------------ */
/* exported: W_n(a_1..a_d) by exhaustive enumeration (Sec. 2.1)         */
/* ------------------------------------------------------------------ */

/*
 * W_n(a_1..a_d) = E[ max_{i_1+...+i_d = n} L(a_1 x_1[..i_1], ..., a_d x_d[..i_d]) ]
 * with x_j uniform in Sigma^n.  Only the first n symbols of each x_j can be
 * used, so the expectation is an exact average over sigma^(d n) tails.
 * Returns the integer sum over all tails (the expectation is
 * *sum / sigma^(d n)).  L is the textbook d-string LCS recurrence over
 * prefix lengths.  heads[j*h + p] = a_j[p].
 */
int or_brute_W(int sigma, int d, int h, int n, const int *heads, uint64_t *sum)
{
    if (sigma < 2 || d < 1 || d > 4 || h < 0 || n < 0) return -1;
    int len = h + n;                 /* full string length */
    int side = len + 1;              /* prefix lengths 0..len */
    uint64_t cells = 1;
    for (int j = 0; j < d; ++j) cells *= (uint64_t)side;
    if (cells > (1u << 26)) return -1;
    double tails_d = pow((double)sigma, (double)d * n);
    if (tails_d > 1e9) return -1;
    uint64_t tails = ipow(sigma, d * n);
    int *str = (int *)malloc(sizeof(int) * (size_t)(d * (len > 0 ? len : 1)));
    uint32_t *L = (uint32_t *)malloc(sizeof(uint32_t) * cells);
    if (!str || !L) { free(str); free(L); return -2; }
    uint64_t stride[4];
    stride[d - 1] = 1;
    for (int j = d - 2; j >= 0; --j) stride[j] = stride[j + 1] * (uint64_t)side;
    uint64_t total = 0;
    for (uint64_t t = 0; t < tails; ++t) {
        /* string j = a_j followed by x_j (digits of t, string 1 first) */
        uint64_t rest = t;
        for (int j = d - 1; j >= 0; --j) {
            for (int p = 0; p < h; ++p) str[j * len + p] = heads[j * h + p];
            for (int p = len - 1; p >= h; --p) {
                str[j * len + p] = (int)(rest % (uint64_t)sigma);
                rest /= (uint64_t)sigma;
            }
        }
        /* L over prefix-length vectors q, lexicographic order */
        for (uint64_t cell = 0; cell < cells; ++cell) {
            int q[4];
            uint64_t r2 = cell;
            int any_zero = 0;
            for (int j = 0; j < d; ++j) {
                q[j] = (int)(r2 / stride[j]);
                r2 %= stride[j];
                if (q[j] == 0) any_zero = 1;
            }
            if (any_zero) { L[cell] = 0; continue; }
            int same = 1;
            int c0 = str[0 * len + q[0] - 1];
            for (int j = 1; j < d; ++j)
                if (str[j * len + q[j] - 1] != c0) same = 0;
            if (same) {
                uint64_t back = cell;
                for (int j = 0; j < d; ++j) back -= stride[j];
                L[cell] = L[back] + 1;
            } else {
                uint32_t m = 0;
                for (int j = 0; j < d; ++j) {
                    uint32_t v = L[cell - stride[j]];
                    if (v > m) m = v;
                }
                L[cell] = m;
            }
        }
        /* max over i_1 + ... + i_d = n of L(h + i_1, ..., h + i_d) */
        uint32_t best = 0;
        uint64_t splits = ipow(n + 1, d);
        for (uint64_t sp = 0; sp < splits; ++sp) {
            uint64_t r3 = sp;
            int sumi = 0;
            uint64_t cell = 0;
            for (int j = 0; j < d; ++j) {
                int i = (int)(r3 % (uint64_t)(n + 1));
                r3 /= (uint64_t)(n + 1);
                sumi += i;
                cell += (uint64_t)(h + i) * stride[j];
            }
            if (sumi != n) continue;
            if (L[cell] > best) best = L[cell];
        }
        total += best;
    }
    free(str);
    free(L);
    *sum = total;
    return 0;
}
