// Host side of the C ABI declared in include/lcsb.h: argument checks, the
// ring of d+1 tables (Algorithm 2 keeps v_{n-d} .. v_n), launches on the
// caller's stream, and the keep-best rule of Algorithm 2.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <cstddef>
#include <new>
#include <string>

#include "internal.h"
#include "rounding.h"

using namespace lcsb;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

enum State { kCreated = 0, kBound = 1, kReady = 2, kPoisoned = 3 };

}  // namespace

struct lcsb_ctx {
    Geometry g;
    int dtype;
    int nbuf;
    void *buf[4];
    unsigned char *ws;
    hipStream_t stream;
    int state;
    int head;        // ring slot holding lag 1
    int64_t sweeps;  // sweeps since the last init
    lcsb_cert best;
    int swap_sym;    // sigma = d = 2, l >= 2: lag 1 .. d symmetric in the two strings
    int lazy[4];     // per slot: only the lower index of each exchanged pair written
    int two_array;   // LCSB_ITER_TWO_ARRAY(_PACKED): tables u (lag 1) and the one before (lag 2), rate R
    int lags;        // tables the context keeps: d for the ring, 2 for the two-array iteration
    int packed;      // LCSB_ITER_TWO_ARRAY_PACKED: one entry per exchange orbit (packed_index)
    uint64_t entries;  // entries per table: g.ns, or packed_entries(h)
    // branch-mean tables (lcsb_bind_means): per slot the parts at part_off
    // (d = 2: Ma, Mab, the table's values at the two-array rate's sample;
    // d = 3: M1, M3, M12, M23, M123, the sample)
    void *means_buf[4];
    uint64_t part_off[6];
    int means_ok[4];    // the slot's means are those of its table
    int entries_ok[4];  // the slot's entries hold its table (a branch-mean sweep may skip them)
    int samples_ok[4];  // the slot's sample values are its table's
};

namespace {

int slot_of_lag(const lcsb_ctx *c, int k) { return ((c->head - (k - 1)) % c->nbuf + c->nbuf) % c->nbuf; }

size_t elem_size(int dtype) { return dtype == LCSB_F32 ? 4 : 8; }

int hip_fail(lcsb_ctx *c, hipError_t e, const char *what)
{
    if (c) c->state = kPoisoned;
    return fail(LCSB_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int need_ready(const lcsb_ctx *c)
{
    if (!c) return fail(LCSB_EINVAL, "null context");
    if (c->state == kPoisoned) return fail(LCSB_ESTATE, "context poisoned by an earlier HIP error");
    if (c->state != kReady) return fail(LCSB_ESTATE, "context not initialised (bind, then init)");
    return LCSB_OK;
}

// the exchange-folded kernels apply to sigma = 2 with d = 2 or 3 and to
// sigma = 4 with d = 2, at l >= 2
bool swap_shape(const lcsb_ctx *c)
{
    if (c->g.h < 2) return false;
    return (c->g.sigma == 2 && (c->g.d == 2 || c->g.d == 3)) || (c->g.sigma == 4 && c->g.d == 2);
}

// Every slot's entries were just (re)written from outside the branch-mean
// sweep: complete, and no slot's means describe them.
void clear_lazy(lcsb_ctx *c)
{
    for (int k = 0; k < 4; ++k) {
        c->lazy[k] = 0;
        c->means_ok[k] = 0;
        c->entries_ok[k] = 1;
        c->samples_ok[k] = 0;
    }
}

// Folded tables of l >= 3 symmetric in the two strings sweep from the
// branch-mean tables once they are bound: sigma = 2 with d = 2 or 3 and
// sigma = 4 with d = 2, rings and two arrays
bool means_shape(const lcsb_ctx *c)
{
    if (c->packed || c->g.h < 3) return false;
    if (c->g.sigma == 4) return c->g.d == 2;
    return c->g.sigma == 2 && (c->g.d == 2 || c->g.d == 3);
}
bool means_path(const lcsb_ctx *c) { return c->means_buf[0] && c->swap_sym && means_shape(c); }

uint64_t round256(uint64_t b) { return (b + 255) & ~(uint64_t)255; }
// byte offsets of the parts of a mean buffer; returns the buffer's size
uint64_t means_layout(const lcsb_ctx *c, uint64_t *off)
{
    const uint64_t es = elem_size(c->dtype), ns = c->g.ns;
    // entries per part: d = 2 Ma ns/2, Mab ns/4; d = 3 M1, M3 ns/2, M12, M23
    // ns/4, M123 ns/8; sigma = 4 M4a ns/4, M4ab ns/16
    const uint64_t d2[2] = {ns / 2, ns / 4}, d3[5] = {ns / 2, ns / 2, ns / 4, ns / 4, ns / 8},
                   s4[2] = {ns / 4, ns / 16};
    const uint64_t *cnt = c->g.sigma == 4 ? s4 : c->g.d == 2 ? d2 : d3;
    const int parts = c->g.d == 2 ? 2 : 5;
    uint64_t at = 0;
    for (int k = 0; k < parts; ++k) {
        off[k] = at;
        at = round256(at + cnt[k] * es);
    }
    off[parts] = at;  // the sample values
    return at + kRateSample * es;
}

void *slot_part(const lcsb_ctx *c, int slot, int part)
{
    return static_cast<unsigned char *>(c->means_buf[slot]) + c->part_off[part];
}
void *slot_ma(const lcsb_ctx *c, int slot) { return slot_part(c, slot, 0); }
void *slot_mab(const lcsb_ctx *c, int slot) { return slot_part(c, slot, 1); }
void *slot_smp(const lcsb_ctx *c, int slot) { return slot_part(c, slot, c->g.d == 2 ? 2 : 5); }

// Complete the exchanged entries of a lazily written slot (stream order).
int materialize(lcsb_ctx *c, int slot)
{
    if (!c->lazy[slot]) return LCSB_OK;
    hipError_t e = launch_materialize_swap(c->g, c->dtype, c->buf[slot], c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "materialize");
    c->lazy[slot] = 0;
    return LCSB_OK;
}

// Set c->swap_sym by checking lag 1 .. d on the device (synchronises).
// Packed tables hold one value per exchange orbit: symmetric by construction.
int refresh_swap(lcsb_ctx *c)
{
    c->swap_sym = c->packed;
    clear_lazy(c);
    if (c->packed || !swap_shape(c)) return LCSB_OK;
    uint32_t *flag = reinterpret_cast<uint32_t *>(c->ws + Ws::kAsym);
    hipError_t e;
    if ((e = launch_fill_zero(flag, 4, c->stream)) != hipSuccess) return hip_fail(c, e, "fill");
    for (int k = 1; k <= c->lags; ++k)
        if ((e = launch_check_swap(c->g, c->dtype, c->buf[slot_of_lag(c, k)], flag, c->stream)) !=
            hipSuccess)
            return hip_fail(c, e, "symmetry check");
    uint32_t host = 1;
    if ((e = hipMemcpyAsync(&host, flag, 4, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
        return hip_fail(c, e, "symmetry copy");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "symmetry sync");
    c->swap_sym = host == 0;
    return LCSB_OK;
}

// Two-array iteration: the rate of the next step from lag 1 and lag 2 (stream order).
int refresh_rate(lcsb_ctx *c)
{
    if (!c->two_array) return LCSB_OK;
    const int s1 = slot_of_lag(c, 1), s2 = slot_of_lag(c, 2);
    hipError_t e = launch_two_array_rate(c->g, c->dtype, c->buf[s1], c->buf[s2], s1, s2,
                                         c->swap_sym, c->packed, c->ws, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "rate");
    return LCSB_OK;
}

lcsb_cert initial_best()
{
    lcsb_cert b;
    memset(&b, 0, sizeof b);
    return b;  // (u, r, eps) = (v_0, 0, 0): rho = 0, bound = 0
}

}  // namespace

extern "C" {

const char *lcsb_last_error(void) { return g_err.c_str(); }

int lcsb_create(int sigma, int d, int h, int dtype, lcsb_ctx **out)
{
    return lcsb_create_iter(sigma, d, h, dtype, LCSB_ITER_RING, out);
}

int lcsb_create_iter(int sigma, int d, int h, int dtype, int iteration, lcsb_ctx **out)
{
    if (!out) return fail(LCSB_EINVAL, "out is null");
    *out = nullptr;
    if (dtype != LCSB_F64 && dtype != LCSB_F32) return fail(LCSB_EINVAL, "dtype %d", dtype);
    if (iteration != LCSB_ITER_RING && iteration != LCSB_ITER_TWO_ARRAY &&
        iteration != LCSB_ITER_TWO_ARRAY_PACKED)
        return fail(LCSB_EINVAL, "iteration %d", iteration);
    if (sigma < 2 || d < 1 || h < 1) return fail(LCSB_EINVAL, "sigma=%d d=%d h=%d", sigma, d, h);
    const bool ok = (sigma == 2 && d == 2) || (sigma == 4 && d == 2) || (sigma == 2 && d == 3);
    if (!ok) return fail(LCSB_EUNSUPPORTED, "no GPU kernel for sigma=%d d=%d", sigma, d);
    const int beta = sigma == 2 ? 1 : 2;
    const int bits = beta * d * h;
    if (bits > 36) return fail(LCSB_EINVAL, "sigma^(d h) = 2^%d exceeds 2^36", bits);
    if (iteration == LCSB_ITER_TWO_ARRAY_PACKED && (sigma != 2 || d != 2 || h < 2))
        return fail(LCSB_EUNSUPPORTED, "packed tables need sigma = d = 2 and l >= 2");
    lcsb_ctx *c = new (std::nothrow) lcsb_ctx;
    if (!c) return fail(LCSB_ENOMEM, "context allocation failed");
    memset(c, 0, sizeof *c);
    c->g.sigma = sigma;
    c->g.d = d;
    c->g.h = h;
    c->g.beta = beta;
    c->g.slot = beta * d;
    c->g.n = 1ull << bits;
    c->g.ns = c->g.n >> beta;
    c->dtype = dtype;
    c->two_array = iteration != LCSB_ITER_RING;
    c->packed = iteration == LCSB_ITER_TWO_ARRAY_PACKED;
    c->entries = c->packed ? packed_entries(h) : c->g.ns;
    c->nbuf = c->two_array ? 2 : d + 1;
    c->lags = c->two_array ? 2 : d;
    c->state = kCreated;
    c->best = initial_best();
    *out = c;
    return LCSB_OK;
}

int lcsb_query(const lcsb_ctx *c, int *nbuf, uint64_t *entries, uint64_t *bytes_per_buf,
               uint64_t *workspace_bytes)
{
    if (!c) return fail(LCSB_EINVAL, "null context");
    if (nbuf) *nbuf = c->nbuf;
    if (entries) *entries = c->entries;
    if (bytes_per_buf) *bytes_per_buf = c->entries * elem_size(c->dtype);
    if (workspace_bytes) *workspace_bytes = Ws::kBytes;
    return LCSB_OK;
}

int lcsb_bind(lcsb_ctx *c, void *const *bufs, int nbuf, void *ws, void *stream)
{
    if (!c) return fail(LCSB_EINVAL, "null context");
    if (c->state == kPoisoned) return fail(LCSB_ESTATE, "context poisoned by an earlier HIP error");
    if (!bufs || nbuf != c->nbuf) return fail(LCSB_EINVAL, "need %d ring buffers", c->nbuf);
    if (!ws || ((uintptr_t)ws & 255)) return fail(LCSB_EINVAL, "workspace null or not 256-byte aligned");
    for (int k = 0; k < nbuf; ++k) {
        if (!bufs[k] || ((uintptr_t)bufs[k] & 255))
            return fail(LCSB_EINVAL, "ring buffer %d null or not 256-byte aligned", k);
        for (int j = 0; j < k; ++j)
            if (bufs[j] == bufs[k]) return fail(LCSB_EINVAL, "ring buffers %d and %d alias", j, k);
    }
    for (int k = 0; k < nbuf; ++k) c->buf[k] = bufs[k];
    c->ws = static_cast<unsigned char *>(ws);
    c->stream = static_cast<hipStream_t>(stream);
    c->state = kBound;
    c->head = 0;
    c->sweeps = 0;
    c->best = initial_best();
    c->swap_sym = 0;
    clear_lazy(c);
    return LCSB_OK;
}

int lcsb_query_means(const lcsb_ctx *c, uint64_t *bytes_per_buf)
{
    if (!c) return fail(LCSB_EINVAL, "null context");
    if (!means_shape(c))
        return fail(LCSB_EUNSUPPORTED, "branch-mean tables serve folded sigma = 2 tables of l >= 3 "
                                       "(d = 2: ring or two arrays; d = 3: ring)");
    uint64_t off[6];
    if (bytes_per_buf) *bytes_per_buf = means_layout(c, off);
    return LCSB_OK;
}

int lcsb_bind_means(lcsb_ctx *c, void *const *bufs, int nbuf)
{
    if (!c) return fail(LCSB_EINVAL, "null context");
    if (c->state == kPoisoned) return fail(LCSB_ESTATE, "context poisoned by an earlier HIP error");
    if (c->state < kBound) return fail(LCSB_ESTATE, "bind the ring buffers first");
    int rc = lcsb_query_means(c, nullptr);
    if (rc) return rc;
    if (!bufs && nbuf == 0) {  // unbind: sweep from the entries again
        for (int k = 0; k < 4; ++k) {
            c->means_buf[k] = nullptr;
            c->means_ok[k] = c->samples_ok[k] = 0;
        }
        return LCSB_OK;
    }
    if (!bufs || nbuf != c->nbuf) return fail(LCSB_EINVAL, "need %d mean buffers", c->nbuf);
    for (int k = 0; k < nbuf; ++k) {
        if (!bufs[k] || ((uintptr_t)bufs[k] & 255))
            return fail(LCSB_EINVAL, "mean buffer %d null or not 256-byte aligned", k);
        for (int j = 0; j < c->nbuf; ++j)
            if (bufs[k] == c->buf[j] || (j < k && bufs[j] == bufs[k]))
                return fail(LCSB_EINVAL, "mean buffer %d aliases another buffer", k);
        if (bufs[k] == c->ws) return fail(LCSB_EINVAL, "mean buffer %d is the workspace", k);
    }
    for (int k = 0; k < nbuf; ++k) {
        c->means_buf[k] = bufs[k];
        c->means_ok[k] = c->samples_ok[k] = 0;
    }
    means_layout(c, c->part_off);
    return LCSB_OK;
}

int lcsb_init_zero(lcsb_ctx *c)
{
    if (!c) return fail(LCSB_EINVAL, "null context");
    if (c->state == kPoisoned) return fail(LCSB_ESTATE, "context poisoned by an earlier HIP error");
    if (c->state < kBound) return fail(LCSB_ESTATE, "bind before init");
    const uint64_t bytes = c->entries * elem_size(c->dtype);
    hipError_t e;
    for (int k = 0; k < c->nbuf; ++k)
        if ((e = launch_fill_zero(c->buf[k], bytes, c->stream)) != hipSuccess)
            return hip_fail(c, e, "fill");
    if ((e = launch_fill_zero(c->ws, Ws::kBytes, c->stream)) != hipSuccess)
        return hip_fail(c, e, "fill workspace");
    c->head = 0;
    c->sweeps = 0;
    c->best = initial_best();
    c->swap_sym = c->packed || swap_shape(c);
    clear_lazy(c);
    int rc = refresh_rate(c);
    if (rc) return rc;
    c->state = kReady;
    return LCSB_OK;
}

int lcsb_load_ring(lcsb_ctx *c, const void *const *src, int nsrc, const double *offsets)
{
    if (!c) return fail(LCSB_EINVAL, "null context");
    if (c->state == kPoisoned) return fail(LCSB_ESTATE, "context poisoned by an earlier HIP error");
    if (c->state < kBound) return fail(LCSB_ESTATE, "bind before load");
    if (c->packed) return fail(LCSB_EUNSUPPORTED, "packed contexts start from zero or a checkpoint");
    if (!src || nsrc != c->lags) return fail(LCSB_EINVAL, "need %d source tables", c->lags);
    for (int k = 0; k < nsrc; ++k) {
        if (!src[k] || ((uintptr_t)src[k] & (elem_size(c->dtype) - 1)))
            return fail(LCSB_EINVAL, "source %d null or not aligned to its element", k);
        for (int j = 0; j < c->nbuf; ++j)
            if (src[k] == c->buf[j]) return fail(LCSB_EINVAL, "source %d aliases a ring buffer", k);
    }
    hipError_t e;
    if ((e = launch_fill_zero(c->ws, Ws::kBytes, c->stream)) != hipSuccess)
        return hip_fail(c, e, "fill workspace");
    c->head = 0;
    for (int k = 1; k <= c->lags; ++k) {
        const int slot = slot_of_lag(c, k);
        if ((e = launch_copy(src[k - 1], c->buf[slot], c->g.ns * elem_size(c->dtype), c->stream)) !=
            hipSuccess)
            return hip_fail(c, e, "copy");
        if (c->dtype == LCSB_F32) {
            double o = offsets ? offsets[k - 1] : 0.0;
            double *dev = reinterpret_cast<double *>(c->ws + Ws::kOffsets) + slot;
            if ((e = launch_fill_f64(dev, 1, o, c->stream)) != hipSuccess)
                return hip_fail(c, e, "offset");
        }
    }
    c->sweeps = 0;
    c->best = initial_best();
    int rc = refresh_swap(c);
    if (rc) return rc;
    if ((rc = refresh_rate(c))) return rc;
    c->state = kReady;
    return LCSB_OK;
}

int lcsb_iterate(lcsb_ctx *c, int64_t k)
{
    int rc = need_ready(c);
    if (rc) return rc;
    if (k < 0) return fail(LCSB_EINVAL, "negative sweep count");
    if (means_path(c) && k > 0) {
        // the means of the lags the sweep reads (lags 1 .. d of the ring; u,
        // lag 1, of the two-array iteration), derived from their entries where stale
        for (int j = 1; j <= (c->two_array ? 1 : c->g.d); ++j) {
            const int slot = slot_of_lag(c, j);
            if (c->means_ok[slot]) continue;
            if (!c->entries_ok[slot]) return fail(LCSB_ESTATE, "lag %d has neither entries nor means", j);
            hipError_t e =
                c->g.sigma == 4
                    ? launch_derive_means4(c->g, c->dtype, c->buf[slot], c->lazy[slot],
                                           slot_ma(c, slot), slot_mab(c, slot), c->stream)
                : c->g.d == 2
                    ? launch_derive_means(c->g, c->dtype, c->buf[slot], c->lazy[slot],
                                          slot_ma(c, slot), slot_mab(c, slot), c->stream)
                    : launch_derive_means3(c->g, c->dtype, c->buf[slot], c->lazy[slot],
                                           slot_part(c, slot, 0), slot_part(c, slot, 1),
                                           slot_part(c, slot, 2), slot_part(c, slot, 3),
                                           slot_part(c, slot, 4), c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "derive means");
            c->means_ok[slot] = 1;
        }
        for (int64_t t = 0; t < k && c->g.d == 3; ++t) {
            Means3Launch a;
            // two arrays: every lag is u, lags 2 and 3 read relative to offsets
            // slots kSlotLag2/3 (u - R, u - 2R, set by the rate pass)
            const int r1 = slot_of_lag(c, 1), r2 = c->two_array ? r1 : slot_of_lag(c, 2),
                      r3 = c->two_array ? r1 : slot_of_lag(c, 3);
            a.m1 = slot_part(c, r1, 0);
            a.m3 = slot_part(c, r1, 1);
            a.m12 = slot_part(c, r2, 2);
            a.m23 = slot_part(c, r2, 3);
            a.m123 = slot_part(c, r3, 4);
            a.snew = (c->head + 1) % c->nbuf;
            const bool entries = t >= k - c->g.d;
            a.out = entries ? c->buf[a.snew] : nullptr;
            a.n1 = slot_part(c, a.snew, 0);
            a.n3 = slot_part(c, a.snew, 1);
            a.n12 = slot_part(c, a.snew, 2);
            a.n23 = slot_part(c, a.snew, 3);
            a.n123 = slot_part(c, a.snew, 4);
            a.offsets = reinterpret_cast<double *>(c->ws + Ws::kOffsets);
            a.s1 = c->two_array && c->dtype != LCSB_F32 ? Ws::kSlotZero : r1;
            a.s2 = c->two_array ? Ws::kSlotLag2 : r2;
            a.s3 = c->two_array ? Ws::kSlotLag3 : r3;
            a.shift = c->two_array;
            hipError_t e = launch_sweep_means3(c->g, c->dtype, a, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "sweep launch");
            if (c->two_array) {  // the next rate from sample values, as for d = 2
                if ((e = launch_means_samples3(c->g, c->dtype, a, slot_smp(c, a.snew), c->stream)) !=
                    hipSuccess)
                    return hip_fail(c, e, "sample values");
                if (!c->samples_ok[r1] && !c->entries_ok[r1])
                    return fail(LCSB_ESTATE, "the old table has neither entries nor sample values");
                e = launch_two_array_rate(c->g, c->dtype, c->buf[a.snew], c->buf[r1], a.snew, r1,
                                          c->swap_sym, 0, c->ws, c->stream, slot_smp(c, a.snew),
                                          c->samples_ok[r1] ? slot_smp(c, r1) : nullptr);
                if (e != hipSuccess) return hip_fail(c, e, "rate");
                c->samples_ok[a.snew] = 1;
            }
            c->lazy[a.snew] = 1;
            c->means_ok[a.snew] = 1;
            c->entries_ok[a.snew] = entries;
            c->head = a.snew;
            c->sweeps++;
        }
        for (int64_t t = 0; t < k && c->g.d == 2; ++t) {
            MeansLaunch a;
            const int r1 = slot_of_lag(c, 1), r2 = c->two_array ? r1 : slot_of_lag(c, 2);
            a.ma1 = slot_ma(c, r1);
            a.mab2 = slot_mab(c, r2);
            // offsets: the ring's lags are read relative to lag 1; the
            // two-array lag 2 is u - R (slot kSlotLag2, set by the rate pass)
            a.s1 = c->two_array && c->dtype != LCSB_F32 ? Ws::kSlotZero : r1;
            a.s2 = c->two_array ? Ws::kSlotLag2 : r2;
            a.shift = c->two_array;
            a.snew = (c->head + 1) % c->nbuf;
            // the entries of the last d tables: what a certificate or a caller reads
            const bool entries = t >= k - c->g.d;
            a.out = entries ? c->buf[a.snew] : nullptr;
            a.ma_new = slot_ma(c, a.snew);
            a.mab_new = slot_mab(c, a.snew);
            a.offsets = reinterpret_cast<double *>(c->ws + Ws::kOffsets);
            hipError_t e = c->g.sigma == 4 ? launch_sweep_means4(c->g, c->dtype, a, c->stream)
                                           : launch_sweep_means(c->g, c->dtype, a, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "sweep launch");
            if (c->two_array) {
                // the rate of the next step from the new table's sample values
                // (computed as the sweep computed them) and the old table's
                if ((e = launch_means_samples(c->g, c->dtype, a, slot_smp(c, a.snew), c->stream)) !=
                    hipSuccess)
                    return hip_fail(c, e, "sample values");
                if (!c->samples_ok[r1] && !c->entries_ok[r1])
                    return fail(LCSB_ESTATE, "the old table has neither entries nor sample values");
                e = launch_two_array_rate(c->g, c->dtype, c->buf[a.snew], c->buf[r1], a.snew, r1,
                                          c->swap_sym, 0, c->ws, c->stream, slot_smp(c, a.snew),
                                          c->samples_ok[r1] ? slot_smp(c, r1) : nullptr);
                if (e != hipSuccess) return hip_fail(c, e, "rate");
                c->samples_ok[a.snew] = 1;
            }
            c->lazy[a.snew] = 1;
            c->means_ok[a.snew] = 1;
            c->entries_ok[a.snew] = entries;
            c->head = a.snew;
            c->sweeps++;
        }
        return LCSB_OK;
    }
    for (int64_t t = 0; t < k; ++t) {
        SweepLaunch a;
        memset(&a, 0, sizeof a);
        if (c->two_array) {
            // every argument is u; lag k is read relative to offsets slot
            // kSlotLag2/3, which the rate pass set to u's offset - (k-1) R (FP32)
            // or -(k-1) R against the zero slot (FP64)
            for (int j = 0; j < c->g.d; ++j) a.lag[j] = c->buf[c->head];
            a.lag_slot[0] = c->dtype == LCSB_F32 ? c->head : Ws::kSlotZero;
            a.lag_slot[1] = Ws::kSlotLag2;
            a.lag_slot[2] = Ws::kSlotLag3;
            a.shift = 1;
        } else {
            for (int j = 1; j <= c->g.d; ++j) {
                a.lag_slot[j - 1] = slot_of_lag(c, j);
                a.lag[j - 1] = c->buf[a.lag_slot[j - 1]];
            }
        }
        a.new_slot = (c->head + 1) % c->nbuf;
        a.out = c->buf[a.new_slot];
        a.offsets = reinterpret_cast<double *>(c->ws + Ws::kOffsets);
        a.swap_sym = c->swap_sym;
        a.packed = c->packed;
        hipError_t e = launch_sweep(c->g, c->dtype, a, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "sweep launch");
        c->lazy[a.new_slot] = c->swap_sym && !c->packed;
        c->means_ok[a.new_slot] = 0;
        c->entries_ok[a.new_slot] = 1;
        c->samples_ok[a.new_slot] = 0;
        c->head = a.new_slot;
        c->sweeps++;
        if ((rc = refresh_rate(c))) return rc;
    }
    return LCSB_OK;
}

int lcsb_certify(lcsb_ctx *c, lcsb_cert *cur, lcsb_cert *best)
{
    int rc = need_ready(c);
    if (rc) return rc;
    if (c->packed)
        return fail(LCSB_EUNSUPPORTED, "packed contexts certify with lcsb_certify_optimal");
    const int su = slot_of_lag(c, 1), sp = slot_of_lag(c, 2);
    hipError_t e = launch_certify(c->g, c->dtype, c->buf[su], c->buf[sp], su, sp, c->swap_sym,
                                  c->ws, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "certify launch");
    unsigned char host[Ws::kScalarBytes];
    if ((e = hipMemcpyAsync(host, c->ws, Ws::kScalarBytes, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
        return hip_fail(c, e, "certify copy");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "certify sync");
    double sc[Ws::kScalarBytes / 8];
    memcpy(sc, host, sizeof sc);
    lcsb_cert k;
    memset(&k, 0, sizeof k);
    k.R = sc[Ws::kR / 8];
    k.maxW = sc[Ws::kMaxW / 8];
    uint64_t u64[Ws::kScalarBytes / 8];
    memcpy(u64, host, sizeof u64);
    k.argmax_W = u64[Ws::kArgmax / 8];
    k.nonfinite = u64[Ws::kNonfinite / 8] + u64[Ws::kNonfiniteR / 8];
    k.kind = LCSB_CERT_FEASIBLE;
    k.E = k.maxW > 0.0 ? k.maxW : 0.0;
    k.rho = add_rd(k.R, -k.E);
    k.bound = mul_rd((double)c->g.d, k.rho);
    k.sweep = c->sweeps;
    // keep (u, r, eps) <- (v_d, R, E) when R - E >= r - eps (Algorithm 2)
    if (k.nonfinite == 0 && k.rho >= c->best.rho) c->best = k;
    if (cur) *cur = k;
    if (best) *best = c->best;
    if (k.nonfinite) return fail(LCSB_ENONFINITE, "%llu non-finite values in the certified tables",
                                 (unsigned long long)k.nonfinite);
    return LCSB_OK;
}

int lcsb_certify_optimal(lcsb_ctx *c, lcsb_cert *cur, lcsb_cert *best)
{
    int rc = need_ready(c);
    if (rc) return rc;
    const int su = slot_of_lag(c, 1);
    hipError_t e = c->packed ? launch_certify_optimal_packed(c->g, c->dtype, c->buf[su], c->ws,
                                                             c->stream)
                             : launch_certify_optimal(c->g, c->dtype, c->buf[su], c->swap_sym,
                                                      c->ws, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "certify launch");
    unsigned char host[Ws::kScalarBytes];
    if ((e = hipMemcpyAsync(host, c->ws, Ws::kScalarBytes, hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
        return hip_fail(c, e, "certify copy");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "certify sync");
    double r;
    uint64_t arg, nonfinite;
    memcpy(&r, host + Ws::kOptR, 8);
    memcpy(&arg, host + Ws::kOptArg, 8);
    memcpy(&nonfinite, host + Ws::kOptNonfinite, 8);
    lcsb_cert k;
    memset(&k, 0, sizeof k);
    k.kind = LCSB_CERT_OPTIMAL;
    k.R = r;
    k.rho = r;  // E = 0, maxW = 0
    k.bound = mul_rd((double)c->g.d, r);
    k.argmax_W = arg;
    k.nonfinite = nonfinite;
    k.sweep = c->sweeps;
    // the keep rule of Algorithm 2 on rho = r - eps
    if (k.nonfinite == 0 && k.rho >= c->best.rho) c->best = k;
    if (cur) *cur = k;
    if (best) *best = c->best;
    if (k.nonfinite) return fail(LCSB_ENONFINITE, "%llu non-finite ratios in the certified table",
                                 (unsigned long long)k.nonfinite);
    return LCSB_OK;
}

int lcsb_certify_optimal_noalloc(int sigma, int d, int h, int dtype, const void *u,
                                 int exchange_symmetric, double *dev_out, void *stream)
{
    std::string err;
    const int rc = certify_optimal_noalloc(sigma, d, h, dtype, u, exchange_symmetric, dev_out,
                                           stream, &err);
    if (rc) return fail(rc, "%s", err.c_str());
    return LCSB_OK;
}

namespace {
// lag k's stored entries (completed when lazily written) and offset
int lag_pointer(const lcsb_ctx *c, int k, void **dev_ptr, double *offset)
{
    int rc = need_ready(c);
    if (rc) return rc;
    if (k < 1 || k > c->lags) return fail(LCSB_EINVAL, "lag %d outside 1..%d", k, c->lags);
    const int slot = slot_of_lag(c, k);
    // the caller may read any stored entry: complete a lazily written table
    // (its values do not change, so the context stays logically const)
    if ((rc = materialize(const_cast<lcsb_ctx *>(c), slot))) return rc;
    if (dev_ptr) *dev_ptr = c->buf[slot];
    if (offset) {
        *offset = 0.0;
        if (c->dtype == LCSB_F32) {
            hipError_t e = hipMemcpyAsync(offset, c->ws + Ws::kOffsets + 8 * slot, 8,
                                          hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) return fail(LCSB_EHIP, "offset read: %s", hipGetErrorString(e));
        }
    }
    return LCSB_OK;
}
}  // namespace

int lcsb_lag(lcsb_ctx *c, int k, void **dev_ptr, double *offset)
{
    int rc = lag_pointer(c, k, dev_ptr, offset);
    if (rc) return rc;
    // the caller may write through the pointer: no branch-mean table or
    // sample value is trusted until it is derived again from the entries
    for (int j = 0; j < 4; ++j) c->means_ok[j] = c->samples_ok[j] = 0;
    return LCSB_OK;
}

int lcsb_read_table(const lcsb_ctx *c, int k, void *host_dst, int as_f64)
{
    void *dev = nullptr;
    double off = 0.0;
    int rc = lag_pointer(c, k, &dev, &off);
    if (rc) return rc;
    if (!host_dst) return fail(LCSB_EINVAL, "null host buffer");
    if (as_f64 != 0 && as_f64 != 1) return fail(LCSB_EINVAL, "as_f64 must be 0 or 1");
    const size_t es = elem_size(c->dtype);
    const uint64_t bytes = c->entries * es;
    hipError_t e = hipMemcpyAsync(host_dst, dev, bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(LCSB_EHIP, "table read: %s", hipGetErrorString(e));
    if (as_f64 && c->dtype == LCSB_F32) {
        // widen in place from the top down: element j's 8 bytes overlap only
        // float elements j' >= j, which are already widened
        float *f = static_cast<float *>(host_dst);
        double *dd = static_cast<double *>(host_dst);
        for (uint64_t j = c->entries; j-- > 0;) {
            const float v = f[j];
            dd[j] = off + (double)v;
        }
    }
    return LCSB_OK;
}

int lcsb_swap_symmetric(const lcsb_ctx *c, int *symmetric)
{
    int rc = need_ready(c);
    if (rc) return rc;
    if (!symmetric) return fail(LCSB_EINVAL, "null output");
    *symmetric = c->swap_sym;
    return LCSB_OK;
}

int lcsb_rate(const lcsb_ctx *c, double *rate)
{
    int rc = need_ready(c);
    if (rc) return rc;
    if (!rate) return fail(LCSB_EINVAL, "null output");
    if (!c->two_array) return fail(LCSB_EINVAL, "the ring iteration keeps no rate");
    hipError_t e = hipMemcpyAsync(rate, c->ws + Ws::kRate, 8, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(LCSB_EHIP, "rate read: %s", hipGetErrorString(e));
    return LCSB_OK;
}

int lcsb_status(const lcsb_ctx *c, int64_t *sweeps, lcsb_cert *best)
{
    if (!c) return fail(LCSB_EINVAL, "null context");
    if (sweeps) *sweeps = c->sweeps;
    if (best) *best = c->best;
    return LCSB_OK;
}

int lcsb_run(lcsb_ctx *c, const lcsb_run_policy *p, lcsb_cert *cur_out, lcsb_cert *best_out,
             int64_t *certificates, int *stop)
{
    int rc = need_ready(c);
    if (rc) return rc;
    if (!p) return fail(LCSB_EINVAL, "policy is null");
    if (p->cadence <= 0 || p->first < 0 || p->max_sweeps < 0 || !(p->stop_delta >= 0.0) ||
        !(p->min_gain >= 0.0) ||
        (p->certificate != LCSB_CERT_FEASIBLE && p->certificate != LCSB_CERT_OPTIMAL))
        return fail(LCSB_EINVAL, "policy: cadence > 0, first >= 0, max_sweeps >= 0, "
                                 "stop_delta >= 0, min_gain >= 0 and a known certificate "
                                 "kind required");
    FILE *log = nullptr;
    if (p->log_path && !(log = fopen(p->log_path, "a")))
        return fail(LCSB_EINVAL, "cannot open the certificate log %s", p->log_path);
    struct Closer {
        FILE *f;
        ~Closer() { if (f) fclose(f); }
    } closer{log};
    timespec t_start;
    clock_gettime(CLOCK_MONOTONIC, &t_start);
    const bool use_target = !isnan(p->target);
    int64_t certs = 0;
    int why = LCSB_STOP_MAX_SWEEPS;
    lcsb_cert cur = c->best, best = c->best;
    if (use_target && best.bound >= p->target) {
        why = LCSB_STOP_TARGET;
    } else {
        const int64_t start = c->sweeps;
        int64_t step = p->first > 0 ? p->first : p->cadence;
        bool have_prev = false;
        double prev = 0.0, best_prev = 0.0;
        while (c->sweeps - start < p->max_sweeps) {
            if ((rc = lcsb_iterate(c, step)) != LCSB_OK) return rc;
            step = p->cadence;
            rc = p->certificate == LCSB_CERT_OPTIMAL ? lcsb_certify_optimal(c, &cur, &best)
                                                     : lcsb_certify(c, &cur, &best);
            ++certs;
            if (log) {
                timespec t;
                clock_gettime(CLOCK_MONOTONIC, &t);
                const double secs = (double)(t.tv_sec - t_start.tv_sec) +
                                    1e-9 * (double)(t.tv_nsec - t_start.tv_nsec);
                fprintf(log,
                        "{\"sweep\": %lld, \"kind\": \"%s\", \"R\": %.17g, \"E\": %.17g, "
                        "\"maxW\": %.17g, \"rho\": %.17g, \"bound\": %.17g, "
                        "\"best_bound\": %.17g, \"nonfinite\": %llu, \"seconds\": %.6f}\n",
                        (long long)cur.sweep, cur.kind == LCSB_CERT_OPTIMAL ? "optimal" : "feasible",
                        cur.R, cur.E, cur.maxW, cur.rho, cur.bound, best.bound,
                        (unsigned long long)cur.nonfinite, secs);
                fflush(log);
            }
            if (rc != LCSB_OK) {
                if (cur_out) *cur_out = cur;
                if (best_out) *best_out = best;
                if (certificates) *certificates = certs;
                return rc;
            }
            if (use_target && best.bound >= p->target) { why = LCSB_STOP_TARGET; break; }
            if (p->stop_delta > 0.0 && have_prev && fabs(cur.bound - prev) < p->stop_delta &&
                cur.bound >= best.bound && best.bound > 0.0) { why = LCSB_STOP_CONVERGED; break; }
            if (p->min_gain > 0.0 && have_prev && best.bound > 0.0 &&
                best.bound - best_prev < p->min_gain) { why = LCSB_STOP_FLOOR; break; }
            prev = cur.bound;
            best_prev = best.bound;
            have_prev = true;
        }
    }
    if (cur_out) *cur_out = cur;
    if (best_out) *best_out = best;
    if (certificates) *certificates = certs;
    if (stop) *stop = why;
    return LCSB_OK;
}

int lcsb_upcast(const lcsb_ctx *src, lcsb_ctx *dst)
{
    int rc = need_ready(src);
    if (rc) return rc;
    if (!dst) return fail(LCSB_EINVAL, "null destination");
    if (dst->state == kPoisoned) return fail(LCSB_ESTATE, "destination poisoned");
    if (dst->state < kBound) return fail(LCSB_ESTATE, "bind the destination first");
    if (src->dtype != LCSB_F32 || dst->dtype != LCSB_F64)
        return fail(LCSB_EINVAL, "upcast goes from an FP32 to an FP64 context");
    if (src->g.sigma != dst->g.sigma || src->g.d != dst->g.d || src->g.h != dst->g.h)
        return fail(LCSB_EINVAL, "shape mismatch");
    if (src->two_array != dst->two_array || src->packed != dst->packed)
        return fail(LCSB_EINVAL, "the two contexts run different iterations");
    // every destination slot is either the source slot's own buffer (widened
    // in place) or no source slot's buffer
    const bool inplace = dst->buf[0] == src->buf[0];
    for (int j = 0; j < dst->nbuf; ++j)
        for (int k = 0; k < src->nbuf; ++k)
            if ((dst->buf[j] == src->buf[k]) != (inplace && j == k))
                return fail(LCSB_EINVAL, "destination buffers must be the source's, slot for slot, "
                                         "or none of them");
    if (dst->ws == src->ws) return fail(LCSB_EINVAL, "the two contexts share a workspace");
    hipError_t e = hipStreamSynchronize(src->stream);
    if (e != hipSuccess) return fail(LCSB_EHIP, "source sync: %s", hipGetErrorString(e));
    if ((e = launch_fill_zero(dst->ws, Ws::kBytes, dst->stream)) != hipSuccess)
        return hip_fail(dst, e, "fill workspace");
    dst->head = src->head;
    Geometry gt = src->g;  // the element-wise passes run over every entry of a table
    gt.ns = src->entries;
    for (int k = 1; k <= src->lags; ++k) {
        const int slot = slot_of_lag(src, k);
        const double *off = reinterpret_cast<const double *>(src->ws + Ws::kOffsets) + slot;
        e = inplace ? launch_upcast_inplace(gt, dst->buf[slot], off, dst->stream)
                    : launch_upcast(gt, static_cast<const float *>(src->buf[slot]), off,
                                    static_cast<double *>(dst->buf[slot]), dst->stream);
        if (e != hipSuccess) return hip_fail(dst, e, "upcast");
    }
    dst->sweeps = src->sweeps;
    dst->best = src->best;
    dst->swap_sym = src->swap_sym;
    for (int k = 0; k < 4; ++k) {
        dst->lazy[k] = src->lazy[k];  // same slots, converted as stored
        dst->means_ok[k] = 0;
        dst->entries_ok[k] = 1;
        dst->samples_ok[k] = 0;
    }
    if ((rc = refresh_rate(dst))) return rc;
    dst->state = kReady;
    return LCSB_OK;
}

// ------------------------------------------------------------------ warm start
static int check_batch(int64_t batch)
{
    if (batch <= 0 || batch % 256 || batch > (int64_t)1 << 26)
        return fail(LCSB_EINVAL, "batch %lld must be a positive multiple of 256 up to 2^26",
                    (long long)batch);
    return LCSB_OK;
}

static int check_h(int h)
{
    if (h < 8 || h > 16) return fail(LCSB_EINVAL, "window length %d outside 8..16", h);
    return LCSB_OK;
}

static int launch_status(hipError_t e, const char *what)
{
    if (e != hipSuccess) return fail(LCSB_EHIP, "%s: %s", what, hipGetErrorString(e));
    return LCSB_OK;
}

int lcsb_mlp_workspace(int64_t batch, uint64_t *bytes)
{
    int rc = check_batch(batch);
    if (rc) return rc;
    if (!bytes) return fail(LCSB_EINVAL, "bytes is null");
    *bytes = mlp_ws_layout(batch).bytes;
    return LCSB_OK;
}

int lcsb_mlp_init(float *params, uint64_t seed, void *stream)
{
    if (!params) return fail(LCSB_EINVAL, "null pointer");
    return launch_status(launch_mlp_init(params, seed, static_cast<hipStream_t>(stream)), "init");
}

int lcsb_mlp_to_bf16(const float *params, uint16_t *wbf16, void *stream)
{
    if (!params || !wbf16) return fail(LCSB_EINVAL, "null pointer");
    return launch_status(launch_to_bf16(params, wbf16, static_cast<hipStream_t>(stream)), "to_bf16");
}

int lcsb_mlp_sample(const void *table, int dtype, int h, uint64_t seed, int64_t batch,
                    uint64_t *idx, float *target, void *stream)
{
    int rc = check_batch(batch);
    if (rc) return rc;
    if (!table || !idx || !target) return fail(LCSB_EINVAL, "null pointer");
    if (dtype != LCSB_F32 && dtype != LCSB_F64) return fail(LCSB_EINVAL, "dtype %d", dtype);
    if (h < 1 || h > 16) return fail(LCSB_EINVAL, "window length %d outside 1..16", h);
    return launch_status(launch_mlp_sample(table, dtype, 2 * h, seed, batch, idx, target,
                                           static_cast<hipStream_t>(stream)), "sample");
}

int lcsb_mlp_forward(const float *params, const uint16_t *wbf16, const uint64_t *idx, int h,
                     int64_t batch, void *ws, float *y, void *stream)
{
    int rc = check_batch(batch);
    if (rc || (rc = check_h(h))) return rc;
    if (!params || !wbf16 || !idx || !y) return fail(LCSB_EINVAL, "null pointer");
    if (ws && ((uintptr_t)ws & 255)) return fail(LCSB_EINVAL, "workspace not 256-byte aligned");
    uint16_t *act = ws ? reinterpret_cast<uint16_t *>(static_cast<unsigned char *>(ws) +
                                                      mlp_ws_layout(batch).act)
                       : nullptr;
    return launch_status(launch_mlp_forward(wbf16, params, idx, h, batch, y, act,
                                            static_cast<hipStream_t>(stream)), "forward");
}

int lcsb_mlp_loss(const float *y, const float *target, int64_t batch, float *dy, double *loss,
                  void *stream)
{
    int rc = check_batch(batch);
    if (rc) return rc;
    if (!y || !target || !dy || !loss) return fail(LCSB_EINVAL, "null pointer");
    return launch_status(launch_mlp_mse(y, target, batch, dy, loss, static_cast<hipStream_t>(stream)),
                         "loss");
}

int lcsb_mlp_backward(const uint16_t *wbf16, const uint64_t *idx, int h, const float *dy,
                      int64_t batch, void *ws, float *grad, void *stream)
{
    int rc = check_batch(batch);
    if (rc || (rc = check_h(h))) return rc;
    if (!wbf16 || !idx || !dy || !ws || !grad) return fail(LCSB_EINVAL, "null pointer");
    if ((uintptr_t)ws & 255) return fail(LCSB_EINVAL, "workspace not 256-byte aligned");
    const MlpWs L = mlp_ws_layout(batch);
    return launch_status(launch_mlp_backward(wbf16, dy, batch, static_cast<unsigned char *>(ws), L,
                                             idx, h, grad, static_cast<hipStream_t>(stream)),
                         "backward");
}

int lcsb_mlp_adam(float *params, uint16_t *wbf16, const float *grad, float *m, float *v,
                  float lr, float beta1, float beta2, float eps, int64_t t, void *stream)
{
    if (!params || !wbf16 || !grad || !m || !v) return fail(LCSB_EINVAL, "null pointer");
    if (t < 1) return fail(LCSB_EINVAL, "Adam step number starts at 1");
    return launch_status(launch_mlp_adam(params, wbf16, grad, m, v, lr, beta1, beta2, eps, t,
                                         static_cast<hipStream_t>(stream)), "adam");
}

int lcsb_init_seed_mlp(lcsb_ctx *c, const float *params, const uint16_t *wbf16, double rate)
{
    if (!c) return fail(LCSB_EINVAL, "null context");
    if (c->state == kPoisoned) return fail(LCSB_ESTATE, "context poisoned by an earlier HIP error");
    if (c->state < kBound) return fail(LCSB_ESTATE, "bind before init");
    if (c->g.sigma != 2 || c->g.d != 2) return fail(LCSB_EUNSUPPORTED, "the network is for sigma = d = 2");
    if (c->packed) return fail(LCSB_EUNSUPPORTED, "packed contexts start from zero or a checkpoint");
    int rc = check_h(c->g.h);
    if (rc) return rc;
    if (!params || !wbf16) return fail(LCSB_EINVAL, "null pointer");
    hipError_t e;
    if ((e = launch_fill_zero(c->ws, Ws::kBytes, c->stream)) != hipSuccess)
        return hip_fail(c, e, "fill workspace");
    c->head = 0;
    const int s1 = slot_of_lag(c, 1), s2 = slot_of_lag(c, 2);
    if ((e = launch_mlp_seed(c->g, c->dtype, wbf16, params, c->buf[s1], c->buf[s2], rate,
                             c->stream)) != hipSuccess)
        return hip_fail(c, e, "seed");
    c->sweeps = 0;
    c->best = initial_best();
    c->swap_sym = c->g.d == 2 && swap_shape(c);  // one value per exchange orbit, written to every member
    clear_lazy(c);
    if ((rc = refresh_rate(c))) return rc;
    c->state = kReady;
    return LCSB_OK;
}

// ------------------------------------------------------------------ checkpoint
// File: a fixed header (every field little-endian, as on the host), then the
// stored entries of lag 1 .. lag d.  The header carries a hash of each table
// and a hash of itself; a file whose sizes or hashes do not match is refused.
namespace {

constexpr char kCkptMagic[8] = {'L', 'C', 'S', 'B', 'R', 'I', 'N', 'G'};
constexpr uint32_t kCkptVersion = 2;
constexpr size_t kStageBytes = size_t(64) << 20;  // pinned staging buffer

struct CkptHeader {
    char magic[8];
    uint32_t version;
    int32_t sigma, d, h, dtype;
    int32_t iteration;  // LCSB_ITER_*
    uint64_t stored;
    int64_t sweeps;
    double bound, R, E, maxW, rho;
    int64_t best_sweep;
    uint64_t argmax_W, nonfinite;
    int64_t best_kind;
    double offsets[3];
    uint64_t table_hash[3];
    uint64_t header_hash;  // of every byte before this field
};

// 64-bit hash of a byte stream, 8-byte words (a zero-padded tail word);
// streaming: feed consecutive chunks whose sizes are multiples of 8.
struct Hash64 {
    uint64_t h = 0x243F6A8885A308D3ull;
    void feed(const unsigned char *p, size_t bytes)
    {
        for (size_t i = 0; i < bytes; i += 8) {
            uint64_t w = 0;
            memcpy(&w, p + i, bytes - i < 8 ? bytes - i : 8);
            h ^= w;
            h *= 0x9E3779B97F4A7C15ull;
            h ^= h >> 29;
        }
    }
};

uint64_t header_hash(const CkptHeader &hd)
{
    Hash64 hs;
    hs.feed(reinterpret_cast<const unsigned char *>(&hd), offsetof(CkptHeader, header_hash));
    return hs.h;
}

struct File {
    FILE *f = nullptr;
    ~File() { if (f) fclose(f); }
};

// Pinned staging buffer; copies from or to it run on `stream`, which is
// drained before the buffer is freed (also on every early return).
struct Pinned {
    void *p = nullptr;
    hipStream_t stream = nullptr;
    ~Pinned()
    {
        if (!p) return;
        (void)hipStreamSynchronize(stream);
        (void)hipHostFree(p);
    }
};

}  // namespace

int lcsb_save(const lcsb_ctx *c, const char *path)
{
    int rc = need_ready(c);
    if (rc) return rc;
    if (!path) return fail(LCSB_EINVAL, "path is null");
    const size_t es = elem_size(c->dtype);
    const uint64_t tbytes = c->entries * es;
    CkptHeader hd;
    memset(&hd, 0, sizeof hd);
    memcpy(hd.magic, kCkptMagic, 8);
    hd.version = kCkptVersion;
    hd.sigma = c->g.sigma; hd.d = c->g.d; hd.h = c->g.h; hd.dtype = c->dtype;
    hd.stored = c->entries;
    hd.sweeps = c->sweeps;
    hd.bound = c->best.bound; hd.R = c->best.R; hd.E = c->best.E; hd.maxW = c->best.maxW;
    hd.rho = c->best.rho; hd.best_sweep = c->best.sweep;
    hd.argmax_W = c->best.argmax_W; hd.nonfinite = c->best.nonfinite;
    hd.best_kind = c->best.kind;
    hd.iteration = c->packed ? LCSB_ITER_TWO_ARRAY_PACKED
                             : c->two_array ? LCSB_ITER_TWO_ARRAY : LCSB_ITER_RING;
    for (int k = 1; k <= c->lags; ++k)  // the file holds complete tables
        if ((rc = materialize(const_cast<lcsb_ctx *>(c), slot_of_lag(c, k)))) return rc;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(LCSB_EHIP, "sync: %s", hipGetErrorString(e));
    if (c->dtype == LCSB_F32) {
        for (int k = 1; k <= c->lags; ++k) {
            e = hipMemcpy(&hd.offsets[k - 1], c->ws + Ws::kOffsets + 8 * slot_of_lag(c, k), 8,
                          hipMemcpyDeviceToHost);
            if (e != hipSuccess) return fail(LCSB_EHIP, "offset read: %s", hipGetErrorString(e));
        }
    }
    // written beside the target and renamed over it once complete, so a run
    // killed while saving keeps its previous checkpoint
    const std::string part = std::string(path) + ".part";
    File out;
    out.f = fopen(part.c_str(), "wb");
    if (!out.f) return fail(LCSB_ECKPT, "cannot create %s", part.c_str());
    if (fwrite(&hd, sizeof hd, 1, out.f) != 1) return fail(LCSB_ECKPT, "write failed: %s", path);
    Pinned stage;
    stage.stream = c->stream;
    if ((e = hipHostMalloc(&stage.p, kStageBytes, hipHostMallocDefault)) != hipSuccess)
        return fail(LCSB_EHIP, "pinned staging buffer: %s", hipGetErrorString(e));
    for (int k = 1; k <= c->lags; ++k) {
        const unsigned char *src = static_cast<const unsigned char *>(c->buf[slot_of_lag(c, k)]);
        Hash64 hs;
        for (uint64_t at = 0; at < tbytes; at += kStageBytes) {
            const size_t n = (size_t)std::min<uint64_t>(kStageBytes, tbytes - at);
            e = hipMemcpyAsync(stage.p, src + at, n, hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) return fail(LCSB_EHIP, "table read: %s", hipGetErrorString(e));
            hs.feed(static_cast<const unsigned char *>(stage.p), n);
            if (fwrite(stage.p, 1, n, out.f) != n) return fail(LCSB_ECKPT, "write failed: %s", path);
        }
        hd.table_hash[k - 1] = hs.h;
    }
    hd.header_hash = header_hash(hd);
    if (fseek(out.f, 0, SEEK_SET) != 0 || fwrite(&hd, sizeof hd, 1, out.f) != 1)
        return fail(LCSB_ECKPT, "header rewrite failed: %s", path);
    const int closed = fclose(out.f);
    out.f = nullptr;
    if (closed != 0) return fail(LCSB_ECKPT, "close failed: %s", part.c_str());
    if (rename(part.c_str(), path) != 0) return fail(LCSB_ECKPT, "cannot rename %s to %s", part.c_str(), path);
    return LCSB_OK;
}

int lcsb_load(lcsb_ctx *c, const char *path)
{
    if (!c) return fail(LCSB_EINVAL, "null context");
    if (c->state == kPoisoned) return fail(LCSB_ESTATE, "context poisoned by an earlier HIP error");
    if (c->state < kBound) return fail(LCSB_ESTATE, "bind before load");
    if (!path) return fail(LCSB_EINVAL, "path is null");
    File in;
    in.f = fopen(path, "rb");
    if (!in.f) return fail(LCSB_ECKPT, "cannot open %s", path);
    CkptHeader hd;
    if (fread(&hd, sizeof hd, 1, in.f) != 1) return fail(LCSB_ECKPT, "%s: short header", path);
    if (memcmp(hd.magic, kCkptMagic, 8) != 0 || hd.version != kCkptVersion)
        return fail(LCSB_ECKPT, "%s: not a ring checkpoint of this version", path);
    if (hd.header_hash != header_hash(hd)) return fail(LCSB_ECKPT, "%s: header hash mismatch", path);
    const int iteration = c->packed ? LCSB_ITER_TWO_ARRAY_PACKED
                          : c->two_array ? LCSB_ITER_TWO_ARRAY : LCSB_ITER_RING;
    if (hd.sigma != c->g.sigma || hd.d != c->g.d || hd.h != c->g.h || hd.dtype != c->dtype ||
        hd.stored != c->entries || hd.iteration != iteration)
        return fail(LCSB_ECKPT, "%s: holds sigma=%d d=%d l=%d dtype=%d iteration=%d, the context "
                                "is sigma=%d d=%d l=%d dtype=%d iteration=%d", path, hd.sigma,
                    hd.d, hd.h, hd.dtype, hd.iteration, c->g.sigma, c->g.d, c->g.h, c->dtype,
                    iteration);
    const size_t es = elem_size(c->dtype);
    const uint64_t tbytes = c->entries * es;
    if (fseek(in.f, 0, SEEK_END) != 0) return fail(LCSB_ECKPT, "%s: cannot seek", path);
    const long long size = ftell(in.f);
    if (size < 0 || (uint64_t)size != sizeof hd + (uint64_t)c->lags * tbytes)
        return fail(LCSB_ECKPT, "%s: %lld bytes, expected %llu", path, size,
                    (unsigned long long)(sizeof hd + (uint64_t)c->lags * tbytes));
    if (fseek(in.f, (long)sizeof hd, SEEK_SET) != 0) return fail(LCSB_ECKPT, "%s: cannot seek", path);
    // from here the ring is being overwritten: not ready until every hash checks
    c->state = kBound;
    hipError_t e;
    Pinned stage;
    stage.stream = c->stream;
    if ((e = hipHostMalloc(&stage.p, kStageBytes, hipHostMallocDefault)) != hipSuccess)
        return fail(LCSB_EHIP, "pinned staging buffer: %s", hipGetErrorString(e));
    if ((e = launch_fill_zero(c->ws, Ws::kBytes, c->stream)) != hipSuccess)
        return hip_fail(c, e, "fill workspace");
    c->head = 0;
    for (int k = 1; k <= c->lags; ++k) {
        unsigned char *dst = static_cast<unsigned char *>(c->buf[slot_of_lag(c, k)]);
        Hash64 hs;
        for (uint64_t at = 0; at < tbytes; at += kStageBytes) {
            const size_t n = (size_t)std::min<uint64_t>(kStageBytes, tbytes - at);
            // the previous chunk's copy must finish before the buffer is refilled
            if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "sync");
            if (fread(stage.p, 1, n, in.f) != n) return fail(LCSB_ECKPT, "%s: short read", path);
            hs.feed(static_cast<const unsigned char *>(stage.p), n);
            if ((e = hipMemcpyAsync(dst + at, stage.p, n, hipMemcpyHostToDevice, c->stream)) !=
                hipSuccess)
                return hip_fail(c, e, "table write");
        }
        if (hs.h != hd.table_hash[k - 1])
            return fail(LCSB_ECKPT, "%s: lag %d hash mismatch (corrupt checkpoint)", path, k);
        if (c->dtype == LCSB_F32) {
            double *dev = reinterpret_cast<double *>(c->ws + Ws::kOffsets) + slot_of_lag(c, k);
            if ((e = launch_fill_f64(dev, 1, hd.offsets[k - 1], c->stream)) != hipSuccess)
                return hip_fail(c, e, "offset");
        }
    }
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "sync");
    c->sweeps = hd.sweeps;
    c->best = initial_best();
    c->best.bound = hd.bound; c->best.R = hd.R; c->best.E = hd.E; c->best.maxW = hd.maxW;
    c->best.rho = hd.rho; c->best.sweep = hd.best_sweep;
    c->best.argmax_W = hd.argmax_W; c->best.nonfinite = hd.nonfinite;
    c->best.kind = hd.best_kind;
    int rc = refresh_swap(c);
    if (rc) return rc;
    if ((rc = refresh_rate(c))) return rc;
    c->state = kReady;
    return LCSB_OK;
}

int lcsb_destroy(lcsb_ctx *c)
{
    delete c;
    return LCSB_OK;
}

}  // extern "C"
