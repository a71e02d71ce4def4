/*
 * lcsb.h -- C ABI of the gfx950 library for the lower-bound iteration of
 * Heineman, Miller, Reichman, Salls, Sarkozy, Soiffer, "Improved Lower Bounds
 * on the Expected Length of Longest Common Subsequences" (arXiv 2407.10925).
 *
 * The library sweeps the table v over all sigma^(d*l) tuples of head strings
 * with the recurrence F of Sec. 2.1 (eqs. (2)-(4), Algorithm 1) and certifies
 * an iterate with the feasible-triplet step of Algorithm 2, giving the bound
 * gamma_{sigma,d} >= d (r - eps) of eq. (6).
 *
 * Conventions shared by every entry point:
 *   - Every function returns an int status: LCSB_OK (0) or a negative code.
 *     On error lcsb_last_error() returns a message (thread-local, valid until
 *     the next call on the same thread).  No function throws or aborts.
 *   - Device pointers are HIP device addresses on the device that is current
 *     when the function is called; the caller owns every buffer and stream it
 *     passes and keeps them alive until lcsb_destroy.  The library allocates
 *     no device memory: the caller (typically PyTorch) allocates the ring and
 *     the workspace whose sizes lcsb_query reports.
 *   - Work is enqueued on the stream given to lcsb_bind and is asynchronous,
 *     except where a function says it synchronises.
 *   - After an LCSB_EHIP error the context is poisoned: every later call on it
 *     except lcsb_destroy returns LCSB_ESTATE.
 *
 * Table layout.  A tuple A = (a_1..a_d), a_j = a_j[1] .. a_j[l] over the
 * alphabet {0..sigma-1}, sigma = 2^beta, has the index whose bits, most
 * significant first, are the beta-bit symbols a_1[1], a_2[1], .., a_d[1],
 * a_1[2], .., a_d[l] (position-major, string 1 first, heads on top).  For
 * sigma = d = 2 this is the interleaved pair of Sec. 3.2.
 *
 * Folded storage.  Relabelling every symbol c -> c xor m leaves LCS lengths
 * unchanged (for sigma = 2 this is the complement symmetry of Sec. 3.3,
 * eq. (10)), and so every iterate: v[i] = v[i xor (m rep)], rep the index with
 * symbol 1 at every position.  A table buffer therefore holds only the
 * n / sigma indices whose string-1 head is 0, which are the lowest n / sigma
 * indices: entry i is the value at index i for i < n / sigma (8-byte doubles
 * for LCSB_F64, 4-byte floats for LCSB_F32), and index i with string-1 head
 * m holds the value of entry i xor (m rep).  With the branch sums taken in
 * the order stated at lcsb_iterate, every sweep and certificate on the folded
 * table is bit-identical to the same computation on the full table.
 *
 * Packed storage (LCSB_ITER_TWO_ARRAY_PACKED, sigma = d = 2, l >= 2).  A table
 * of a ring symmetric under exchanging the two strings as well is constant on
 * each orbit of a tuple (a, b) under the complement and the exchange, and a
 * packed table holds one entry per orbit: packed_entries = 4^(l-1) + 2^l
 * entries, about half of the folded table.  With c = a xor b (kept by both
 * maps; the complement sends a to ~a, the exchange a to a xor c), the orbit's
 * representative has a_1 = 0 and, for c'' = c if c_1 = 0 else ~c and p the
 * first position j >= 2 with c''_j = 1, a_p = 0.  Its code has 2l - 2 bits,
 * from the top: c_1, c_2, then a_j, c_j for j = 3..l, where the a bit of
 * position p holds a_2 instead (for p = 2 every position its own).  Orbits
 * with c'' = 0 (b = a or b = ~a) take the codes 4^(l-1) + c_1 2^(l-1) +
 * (a_2 .. a_l read as a binary number, a_2 most significant).  Entry k of a
 * packed table is the value of every tuple whose code is k; codes below
 * 4^(l-1) whose c'' is 0 belong to no tuple and hold no value.
 */
#ifndef LCSB_H
#define LCSB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LCSB_OK            0
#define LCSB_EINVAL       (-1) /* bad argument (null pointer, size, range)   */
#define LCSB_ENOMEM       (-2) /* host allocation of the context failed      */
#define LCSB_EHIP         (-3) /* a HIP runtime call or launch failed        */
#define LCSB_ESTATE       (-4) /* call out of order, or context poisoned     */
#define LCSB_EUNSUPPORTED (-5) /* (sigma, d, dtype) has no GPU kernel here   */
#define LCSB_ENONFINITE   (-6) /* the certified table holds a NaN or inf     */
#define LCSB_ECKPT        (-7) /* checkpoint file missing, foreign or corrupt */

/* element types of the ring tables */
#define LCSB_F64 0
#define LCSB_F32 1

typedef struct lcsb_ctx lcsb_ctx;

/* One certificate (Algorithm 2 for a single iterate, eq. (6)).
 * With u the newest table and prev the one before it:
 *   R     = max_j (u - prev)[j]                         (round to nearest)
 *   W[A]  = u[A] + dR - F(u + (d-1)R, u + (d-2)R, .., u)[A]
 *   maxW  = max_A W[A], every W rounded toward +inf (F's arguments and every
 *           step of F toward -inf)
 *   E     = max(0, maxW)
 *   rho   = R - E, rounded toward -inf
 *   bound = d * rho, rounded toward -inf: a rigorous lower bound on
 *           gamma_{sigma,d} whenever rho >= 0 (the feasible-triplet lemma,
 *           Sec. 2.1), for whatever table u was certified. */
typedef struct {
    double bound;
    double R;
    double E;
    double maxW;
    double rho;
    int64_t sweep;      /* sweeps applied before this certificate            */
    uint64_t argmax_W;  /* lowest index where W attains maxW                 */
    uint64_t nonfinite; /* stored coordinates where u, prev or W is not finite */
    int64_t kind;       /* LCSB_CERT_FEASIBLE (this struct's formulas) or
                           LCSB_CERT_OPTIMAL (see lcsb_certify_optimal)       */
} lcsb_cert;

#define LCSB_CERT_FEASIBLE 0 /* Algorithm 2: R from the last step, then E     */
#define LCSB_CERT_OPTIMAL  1 /* the largest r with E = 0 for the table        */

/* iterations a context can run */
#define LCSB_ITER_RING      0 /* Algorithm 2: a ring of d + 1 tables            */
#define LCSB_ITER_TWO_ARRAY 1 /* two tables and a rate (lcsb_create_iter)       */
#define LCSB_ITER_TWO_ARRAY_PACKED 2 /* the same on packed tables (lcsb_create_iter) */

/* Create a context for (sigma, d, l = h) and a table element type running
 * the ring iteration of Algorithm 2.  GPU kernels exist for (sigma, d) in
 * {(2,2), (4,2), (2,3)} and both element types; other pairs give
 * LCSB_EUNSUPPORTED.  h >= 1 and sigma^(d h) <= 2^36 (else LCSB_EINVAL; at
 * 2^36 indices one FP32 table of the stored half is 128 GiB, so only the
 * two-array iteration in FP32 fits one 288 GB GPU there).  *out receives a
 * host object owned by the library. */
int lcsb_create(int sigma, int d, int h, int dtype, lcsb_ctx **out);

/* As lcsb_create, choosing the iteration.  LCSB_ITER_TWO_ARRAY is this
 * library's reading of the remark of Sec. 3.3 that the recurrence runs on
 * two arrays: the context keeps the newest table u (lag 1), the table before
 * it (lag 2) and a rate R, and one sweep is
 *     u_new = F(u, u - R, .., u - (d-1) R)                 (eq. (4))
 * with the shift added to each branch mean (a branch moving k >= 2 strings
 * gives mean_z(u) - (k-1) R; in LCSB_F64 that sum is rounded to nearest, in
 * LCSB_F32 the FP32 offset mechanism of lcsb_iterate carries it).  R of the
 * next sweep is the mean of u_new - u over the fixed sample of 4096 stored
 * coordinates c_i = (i * 0x9E3779B97F4A7C15 mod 2^64) mod (n / sigma), as a
 * balanced binary tree over i in order, divided by 4096 (FP32: plus the
 * difference of the two offsets).  At the limit every coordinate grows by the
 * same r, so the two iterations share their fixed points and certified
 * bounds; the two-array one needs 2 tables instead of d + 1 (nbuf = 2) and
 * every certificate works on it unchanged (Algorithm 2's with prev = lag 2).
 * lcsb_load_ring, lcsb_lag, lcsb_save and lcsb_load then handle 2 tables.
 * LCSB_ITER_TWO_ARRAY_PACKED runs the same iteration, bit for bit, on packed
 * tables (see packed storage; sigma = d = 2 and l >= 2, else
 * LCSB_EUNSUPPORTED), so that an FP64 pair of tables at l = 18 (2^36 tuples)
 * takes 2 x 128 GiB: it starts from lcsb_init_zero or lcsb_load, certifies
 * with lcsb_certify_optimal (lcsb_certify, lcsb_load_ring and
 * lcsb_init_seed_mlp give LCSB_EUNSUPPORTED), lcsb_lag returns packed tables,
 * and lcsb_upcast takes a packed FP32 context to a packed FP64 one.  Its
 * certificates report the lowest stored index of the minimising orbit, as
 * on the folded table. */
int lcsb_create_iter(int sigma, int d, int h, int dtype, int iteration, lcsb_ctx **out);

/* Sizes the caller must allocate: nbuf = d + 1 ring tables (2 for the
 * two-array iteration) of bytes_per_buf
 * bytes each (entries = sigma^(d h - 1) stored elements, see folded storage;
 * packed_entries for packed tables),
 * and one device workspace of workspace_bytes bytes, 256-byte aligned.  Any
 * output pointer may be NULL. */
int lcsb_query(const lcsb_ctx *ctx, int *nbuf, uint64_t *entries,
               uint64_t *bytes_per_buf, uint64_t *workspace_bytes);

/* Attach caller-owned device memory and a HIP stream (hipStream_t passed as
 * void*, NULL for the null stream).  dev_bufs holds nbuf table pointers, each
 * at least bytes_per_buf bytes and 256-byte aligned.  May be called again to
 * rebind; the ring contents are then undefined until an init call. */
int lcsb_bind(lcsb_ctx *ctx, void *const *dev_bufs, int nbuf, void *dev_workspace,
              void *hip_stream);

/* Set every table to zero and forget the best certificate: the starting
 * ring v_0 = .. = v_{d-1} = 0 of Algorithm 2 (first row of its pseudo-code)
 * and the initial triplet (v_0, 0, 0). */
int lcsb_init_zero(lcsb_ctx *ctx);

/* Set lag k (k = 1..d; 1..2 for the two-array iteration, which then takes
 * its rate from the two tables) to the caller's device table src[k-1]: the ring's
 * element type, aligned to it, at least `entries` elements (a full table of
 * sigma^(d h) values may be passed), not aliasing a ring buffer.  Its first
 * `entries` values are copied: every other index takes the value of its image
 * with string-1 head 0, so the loaded ring is the symmetric table that agrees
 * with src at the stored indices.  offsets (host, d doubles, may be NULL =
 * all zero) are the values the FP32 tables are relative to (true value =
 * offset + stored value); ignored for LCSB_F64.  Resets the sweep count and
 * the best certificate.  For sigma = 2 (d = 2 or 3, l >= 2) it then checks
 * whether the ring is symmetric under exchanging strings 1 and 2 (see
 * lcsb_swap_symmetric; one read of the ring, synchronises the stream). */
int lcsb_load_ring(lcsb_ctx *ctx, const void *const *src, int nsrc, const double *offsets);

/* Apply k >= 0 sweeps v_new = F(lag 1, .., lag d) of eq. (4) on the bound
 * stream; the new table becomes lag 1.  In LCSB_F64 every value is computed
 * in FP64, round to nearest, summing the sigma^k appended tuples by a
 * balanced binary tree in lexicographic order (appended symbol of the first
 * advanced string most significant; for sigma = 2 each tuple starting with 0
 * followed by its complement: 00, 11, 01, 10) and multiplying by sigma^-k.  In
 * LCSB_F32 the same is done in FP32 relative to lag 1's offset, and the new
 * table is shifted so that its entry 0 is exactly 0 (translation invariance,
 * property 2 of the lemma); the FP64 offsets stay on the device. */
int lcsb_iterate(lcsb_ctx *ctx, int64_t k);

/* Certify the newest table (see lcsb_cert).  Synchronises the stream.  When
 * nonfinite == 0 and cur.rho >= best.rho, the best certificate is replaced
 * (Algorithm 2's keep rule; a later iterate wins ties).  Either output
 * pointer may be NULL.  Returns LCSB_ENONFINITE (after filling the outputs)
 * when a non-finite value was met; the best certificate is then unchanged.
 * Right after an init call it certifies the initial ring (lag 1 against
 * lag 2). */
int lcsb_certify(lcsb_ctx *ctx, lcsb_cert *cur, lcsb_cert *best);

/* The largest-r certificate of the newest table u (not in Algorithm 2,
 * which fixes r to the largest step of the last sweep; derived from the
 * feasible-triplet lemma of Sec. 2.1).  For a fixed u the lemma's inequality
 * with eps = 0, F(u + (d-1)r, .., u + r, u) >= u + d r, holds at coordinate A
 * iff some branch z (moving k_z strings, so reading u + (d - k_z) r) has
 *     c_z(A) = b(A) + mean_z(u)[A] - u[A] >= k_z r        (eq. (4)),
 * so the largest such r is r* = min_A max_z c_z(A) / k_z, and (u, r*, 0) is a
 * feasible triplet giving gamma_{sigma,d} >= d r* (eq. (6)) when r* >= 0.
 * Every mean, the 1 + of an all-match tuple and the subtraction of u[A] are
 * rounded toward -inf, c_z / k_z is a multiply by 1/k_z (exact for k = 1, 2;
 * 1/3 rounded down for c >= 0, up for c < 0) rounded toward -inf, so the
 * computed r is at most r* and the certificate is rigorous; a zero ratio is
 * +0.  One pass over u (no previous table, no R pass).  Fills lcsb_cert with
 * kind = LCSB_CERT_OPTIMAL, R = rho = r, E = 0, bound = d r rounded toward
 * -inf, maxW = 0 (W <= 0 at R = r by construction; not evaluated), argmax_W =
 * the lowest index where the ratio attains r, nonfinite = stored coordinates
 * whose ratio is not finite.  Keep rule, synchronisation and errors as
 * lcsb_certify (the best certificate is shared by both kinds: the larger
 * rho = R - E wins). */
int lcsb_certify_optimal(lcsb_ctx *ctx, lcsb_cert *cur, lcsb_cert *best);

/* For callers that cannot allocate device memory or bind a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the largest-r certificate of lcsb_certify_optimal for a
 * caller's table, with no context.  u: the stored entries of a folded table
 * of (sigma, d, l = h) (n / sigma values, LCSB_F64 or LCSB_F32, 16-byte
 * aligned; see "Folded storage").  exchange_symmetric: 1 only if the table is
 * symmetric bit for bit under exchanging strings 1 and 2 (then only the lower
 * stored index of each exchanged pair is read, as for a lazily written table
 * of an exchange-symmetric ring); 0 reads every entry.  dev_out (device, 4
 * doubles): r, d r rounded toward -inf, and, as the bit patterns of uint64,
 * the lowest index where the ratio attains r and the count of stored
 * coordinates whose ratio is not finite.  Enqueued on `stream` (hipStream_t
 * as void*); nothing is read back and nothing synchronises.  Allocates
 * nothing: its scratch is a fixed 385 KiB device array (reduction partials and
 * scalars, enough for every size up to sigma^(d h) = 2^36, larger sizes give
 * LCSB_EINVAL) that each GPU the library runs on holds until the process
 * ends; every call on one GPU shares it, so calls that overlap on one GPU
 * race. */
int lcsb_certify_optimal_noalloc(int sigma, int d, int h, int dtype, const void *u,
                                 int exchange_symmetric, double *dev_out, void *stream);

/* Branch-mean tables (folded tables, l >= 3: sigma = 2 with d = 2 or 3 and
 * sigma = 4 with d = 2, ring or two-array iteration.  Eq. (3)
 * and Algorithm 1: a branch that advances some strings reads the mean of the
 * entries that differ in those strings' appended symbols).  sigma = d = 2,
 * for a stored group prefix P < n/8 (entries 4P .. 4P+3):
 *   Ma[2P + b] = (T[4P + b] + T[4P + 2 + b]) * 1/2,
 *   Mab[P]     = ((T[4P] + T[4P+3]) + (T[4P+1] + T[4P+2])) * 1/4;
 * sigma = 2, d = 3, for the aligned group of eight (appended bits s1 s2 s3):
 *   M1 (over s1), M3 (over s3), M12 (over s1 s2), M23 (over s2 s3) and M123
 *   (all eight, complement-paired tree);
 * sigma = 4, for the aligned group of sixteen (member 4 a + b):
 *   M4a[4P + b] = ((T[16P+b] + T[16P+4+b]) + (T[16P+8+b] + T[16P+12+b])) * 1/4,
 *   M4ab[P]     = the sixteen members summed pair by pair ({ab, ba} grouped
 *                 by a xor b, then {aa, ~a~a}) * 1/16;
 * in each case the means the entry-reading sweep forms (same operations, same
 * order).  On tables symmetric in the two strings (lcsb_swap_symmetric; the
 * zero start) a sweep then reads one mean per branch instead of its entries
 * (a mean over string 2's symbols is the one over string 1's at the
 * exchanged tuple; means over both strings are kept at the lower prefix of
 * each exchanged pair of groups), with the same table bit for bit.  Each
 * sweep writes its table's means and, on the last d sweeps of an
 * lcsb_iterate call, its entries, so every lag a caller or a certificate sees
 * is complete; the two-array rate reads the new table's values at its 4096
 * sample coordinates, which are computed from the same means with the
 * sweep's operations.  Other tables sweep from the entries.
 *
 * lcsb_query_means: bytes of one mean buffer (the parts in the order above,
 * then the 4096 sample values, each 256-byte aligned; about 3/4 of a table
 * buffer for sigma = d = 2, 7/4 for d = 3, 5/16 for sigma = 4).
 * LCSB_EUNSUPPORTED for other shapes, packed tables and l < 3.  lcsb_bind_means (after lcsb_bind): nbuf = the ring's buffer count
 * of caller-owned device buffers, 256-byte aligned, distinct from the ring
 * buffers and the workspace, kept until unbound or the context is destroyed;
 * bufs = NULL with nbuf = 0 unbinds.  The means are derived from the entries
 * before the first sweep that needs them (after lcsb_init_zero, lcsb_load_ring,
 * lcsb_load, lcsb_upcast, lcsb_init_seed_mlp or lcsb_lag). */
int lcsb_query_means(const lcsb_ctx *ctx, uint64_t *bytes_per_buf);
int lcsb_bind_means(lcsb_ctx *ctx, void *const *bufs, int nbuf);

/* Device address of lag k (1..d; 1..2 for the two-array iteration) and, for LCSB_F32, the FP64 offset its
 * values are relative to (read from the device; synchronises).  The pointer
 * stays valid until the next lcsb_iterate, lcsb_load_ring or lcsb_bind.  On
 * an exchange-symmetric ring (lcsb_swap_symmetric) sweeps write only one
 * entry of each exchanged pair; this call first completes the table on the
 * stream (one kernel over the table), so every stored entry can be read.
 * The caller may write through the pointer (as lcsb_load_ring does, in
 * place): with branch-mean buffers bound, the next lcsb_iterate derives the
 * lags' means from their entries again. */
int lcsb_lag(lcsb_ctx *ctx, int k, void **dev_ptr, double *offset);

/* Copy lag k (as for lcsb_lag) to host memory: the `entries` stored values
 * (lcsb_query; packed contexts: their packed_entries codes) in the ring's
 * element type (as_f64 = 0; host_dst holds entries elements of 8 or 4 bytes),
 * or as FP64 true values (as_f64 = 1; host_dst holds entries doubles; an
 * FP32 table is widened exactly and its offset added in round-to-nearest).
 * Synchronises; host_dst is caller memory of any kind (pageable is fine). */
int lcsb_read_table(const lcsb_ctx *ctx, int k, void *host_dst, int as_f64);

/* sigma = 2, d = 2 or 3, l >= 2: *symmetric = 1 when every lag table is
 * known to be symmetric, bit for bit, under exchanging strings 1 and 2 (after
 * lcsb_init_zero, lcsb_init_seed_mlp, a load_ring or load of such a ring, an
 * upcast of such a ring, and every sweep of such a ring: F keeps the
 * symmetry exactly, the sums being taken in the order stated at
 * lcsb_iterate).  lcsb_iterate and lcsb_certify then compute one tuple of
 * each exchanged pair, and a sweep writes only the entry of the pair with the
 * lower stored index (lcsb_lag and lcsb_save complete the table before it is
 * read), which halves the bytes they move; otherwise (and for every other
 * shape) *symmetric = 0 and every tuple is computed and written.  The
 * results are the same bits either way. */
int lcsb_swap_symmetric(const lcsb_ctx *ctx, int *symmetric);

/* Number of sweeps applied since the last init, and the best certificate. */
int lcsb_status(const lcsb_ctx *ctx, int64_t *sweeps, lcsb_cert *best);

/* Two-array iteration only: the rate R the next sweep uses (see
 * lcsb_create_iter; absolute, offsets included).  Synchronises.  LCSB_EINVAL
 * for a ring context. */
int lcsb_rate(const lcsb_ctx *ctx, double *rate);

/* Stop rule and certificate cadence of a run (Algorithm 2's loop with its
 * certificate taken every `cadence` sweeps instead of every sweep). */
typedef struct {
    int64_t cadence;     /* sweeps between certificates, > 0                  */
    int64_t first;       /* sweeps before the first certificate; 0 = cadence  */
    int64_t max_sweeps;  /* no new period once this many sweeps have run in
                            this call (the last period may pass it), >= 0     */
    double target;       /* stop once best.bound >= target; NaN = no target    */
    double stop_delta;   /* stop once two consecutive certificates differ by
                            less than this, the newer is >= best and the best
                            bound is positive; 0 = off                        */
    double min_gain;     /* stop once a positive best bound gained less than
                            this over one period (an FP32 run at its error
                            floor); 0 = off                                   */
    int64_t certificate; /* LCSB_CERT_FEASIBLE (lcsb_certify) or
                            LCSB_CERT_OPTIMAL (lcsb_certify_optimal)          */
    const char *log_path;/* NULL, or a file that gets one JSON line appended
                            per certificate: sweep, kind, R, E, maxW, rho,
                            bound, best_bound, nonfinite, seconds since the
                            call began (LCSB_EINVAL if it cannot be opened)  */
} lcsb_run_policy;

#define LCSB_STOP_MAX_SWEEPS 0  /* max_sweeps reached                          */
#define LCSB_STOP_TARGET     1  /* best.bound >= target (possibly at entry)    */
#define LCSB_STOP_CONVERGED  2  /* consecutive certificates within stop_delta  */
#define LCSB_STOP_FLOOR      3  /* best bound gained less than min_gain        */

/* Sweep and certify under policy p until one of its stop conditions holds
 * (checked after each certificate in the order target, converged, floor,
 * then the sweep limit).  If the best bound already meets the target, no
 * sweep is run.  Outputs (each may be NULL): the last certificate (the best
 * one if none was taken), the best certificate, the number of certificates
 * taken and the LCSB_STOP_* reason.  Errors are those of lcsb_iterate and
 * lcsb_certify (an LCSB_ENONFINITE certificate ends the run with that code,
 * after filling the outputs). */
int lcsb_run(lcsb_ctx *ctx, const lcsb_run_policy *p, lcsb_cert *cur, lcsb_cert *best,
             int64_t *certificates, int *stop);

/* Copy the ring of an LCSB_F32 context into an LCSB_F64 context of the same
 * (sigma, d, h) as FP64 values offset + stored value (the switch from FP32
 * sweeps to an FP64 polish).  The sweep count and best certificate move with
 * it.  Enqueued on dst's stream after synchronising src's.  The two rings are
 * either disjoint, or src was bound to dst's own buffers slot for slot (each
 * FP32 table in the first half of its FP64 buffer): then every table is
 * widened in place and src's tables are consumed, so one FP64 ring of memory
 * serves both precisions.  Any other sharing of buffers, or a shared
 * workspace, gives LCSB_EINVAL. */
int lcsb_upcast(const lcsb_ctx *src_f32, lcsb_ctx *dst_f64);

/* Write the ring to `path`: the stored entries of lag 1 .. d (1 .. 2 for the
 * two-array iteration, whose rate is recomputed from them on load), the FP32
 * offsets, the sweep count and the best certificate, with a hash of every
 * table and of the header.  The file is written as `path`.part and renamed
 * over `path` once complete, so an interrupted save leaves an earlier
 * checkpoint at `path` intact.  Synchronises the stream; stages through a
 * 64 MiB pinned host buffer it allocates and frees.  LCSB_ECKPT on a file
 * error. */
int lcsb_save(const lcsb_ctx *ctx, const char *path);

/* Restore a ring written by lcsb_save for the same (sigma, d, l, dtype) into
 * a bound context: afterwards iterate and certify continue bit for bit as
 * the saved context would have.  The header (magic, version, shape, its hash
 * and the file size) is checked before anything is written; a foreign,
 * truncated or corrupt file gives LCSB_ECKPT.  A table hash mismatch is only
 * found while the ring is being overwritten: the context is then left bound
 * but not initialised (iterate and certify return LCSB_ESTATE until an init
 * call or a good load).  Checks the exchange symmetry as lcsb_load_ring
 * does.  Synchronises the stream. */
int lcsb_load(lcsb_ctx *ctx, const char *path);

/* ------------------------------------------------------------------------
 * Learned warm start for sigma = d = 2 (not part of the paper's method: the
 * limit of Algorithm 2's iteration does not depend on the starting ring, so
 * a better start only shortens the run; the certificate decides the result).
 *
 * Network: 32 inputs -> 256 -> 256 -> 256 -> 1, ReLU, every matrix product
 * with BF16 operands and FP32 accumulation (gfx950 MFMA).  Parameters are one
 * FP32 master vector of LCSB_MLP_NPARAMS floats, matrices output-major:
 *   W1[256][32] b1[256] W2[256][256] b2[256] W3[256][256] b3[256] w4[256] b4[1]
 * plus a BF16 copy (uint16 bit patterns, same layout, round to nearest even)
 * used as the matrix operands.  Inputs of a table index at window length h
 * (8 <= h <= 16): the symbols of strings a and b at positions 1..8 and
 * h-7..h, slot 2j = a, slot 2j+1 = b, symbol s -> 2s - 1.  Activations are
 * rounded to BF16 after each ReLU.
 * All pointers are device pointers; work is enqueued on `stream` (hipStream_t
 * as void*, NULL = null stream).  `batch` is a positive multiple of 256.
 * ------------------------------------------------------------------------ */
#define LCSB_MLP_INPUTS 32
#define LCSB_MLP_WIDTH 256
#define LCSB_MLP_NPARAMS 140289

/* Bytes of the training workspace for `batch` samples (the stored BF16
 * activations and encoded inputs, two BF16 gradient buffers, the transposed
 * hidden weights, and the per-split partial sums of the weight gradients). */
int lcsb_mlp_workspace(int64_t batch, uint64_t *bytes);

/* Seeded initialisation: every weight of a layer with fan-in k uniform in
 * (-sqrt(6/k), sqrt(6/k)) (He initialisation for ReLU networks), drawn from
 * SplitMix64 at counter seed * 2^32 + i + 1 for parameter i; biases 0. */
int lcsb_mlp_init(float *params, uint64_t seed, void *stream);

/* wbf16[i] = BF16 rounding of params[i] for every parameter. */
int lcsb_mlp_to_bf16(const float *params, uint16_t *wbf16, void *stream);

/* Draw `batch` table indices uniformly (SplitMix64 of Steele, Lea and Flood,
 * counter seed * 2^32 + j + 1, top 2h bits) from a folded sigma = d = 2 table
 * of window length h (FP64 or FP32 per dtype, 4^h / 2 stored entries) and
 * gather the normalised targets target[j] = v[idx[j]] - v[0] (as FP32), an
 * index with string-1 head 1 read at its complement. */
int lcsb_mlp_sample(const void *table, int dtype, int h, uint64_t seed, int64_t batch,
                    uint64_t *idx, float *target, void *stream);

/* y[j] = network(idx[j]) at window length h.  If ws is non-null (a training
 * workspace for this batch) the BF16 activations are kept there for
 * lcsb_mlp_backward. */
int lcsb_mlp_forward(const float *params, const uint16_t *wbf16, const uint64_t *idx, int h,
                     int64_t batch, void *ws, float *y, void *stream);

/* Mean squared error: dy[j] = 2 (y[j] - target[j]) / batch, *loss (device
 * double) = mean of (y - target)^2. */
int lcsb_mlp_loss(const float *y, const float *target, int64_t batch, float *dy, double *loss,
                  void *stream);

/* Gradient of the loss with respect to every parameter (FP32, layout as the
 * parameters), from dy and the activations a preceding lcsb_mlp_forward left
 * in ws for the same idx, h and batch.  The BF16 rounding of the weights and
 * activations passes gradients unchanged; every upstream gradient is rounded
 * to BF16 before it meets a weight matrix.  Deterministic: every sum runs in
 * a fixed order. */
int lcsb_mlp_backward(const uint16_t *wbf16, const uint64_t *idx, int h, const float *dy,
                      int64_t batch, void *ws, float *grad, void *stream);

/* One Adam step (Kingma and Ba, 2015) on the FP32 master parameters with FP32
 * moments m and v, step number t >= 1; refreshes the BF16 copy. */
int lcsb_mlp_adam(float *params, uint16_t *wbf16, const float *grad, float *m, float *v,
                  float lr, float beta1, float beta2, float eps, int64_t t, void *stream);

/* Fill the ring of a sigma = d = 2 context (8 <= h <= 16) from the network.
 * The network is evaluated once per orbit of the group generated by
 * exchanging the two strings and complementing both (Sec. 3.3: the converged
 * table is invariant under both), at one member u = network(i) of the orbit,
 * and lag 2 = u, lag 1 = u + rate are written at every member (so the ring
 * is symmetric, as the sweeps require).  (4^h + 2^(h+1)) / 4 evaluations.
 * FP32 offsets are set to 0.  Resets the sweep count and the best
 * certificate, like the other init calls. */
int lcsb_init_seed_mlp(lcsb_ctx *ctx, const float *params, const uint16_t *wbf16, double rate);

/* Release the context (never the caller's buffers or stream). NULL is ok. */
int lcsb_destroy(lcsb_ctx *ctx);

/* Message for the last failed call on this thread ("" if none). */
const char *lcsb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LCSB_H */
