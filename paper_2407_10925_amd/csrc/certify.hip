// Certificate of one iterate: the R, W and E steps of Algorithm 2 (Sec. 2.1)
// with directed rounding so that the bound d (R - E) of eq. (6) is rigorous
// for the table it is given.
//
//   pass 1: R = max_j (u - prev)[j]                 (round to nearest)
//   final : shift_k = (d-k) R rounded down, dR rounded up
//   pass 2: W[A] = (u[A] + dR) - F(u + shift_1, .., u + shift_d)[A]
//           with F rounded down step by step (each shifted argument, every
//           add of the pairwise tree, the scaling by sigma^-k, the 1 +) and
//           both outer operations rounded up; maxW and its lowest index.
//           The W pass runs with the wave's FP rounding mode set to toward
//           -inf, so every directed operation is one hardware instruction;
//           a round-up sum is the negation of the round-down sum of the
//           negated operands.  IEEE-754 fixes each directed result
//           uniquely, so this equals the error-free-transform evaluation
//           bit for bit.
//
// Tables are stored folded (the indices with string-1 head 0; every other
// index holds the value of its image under the symbol relabelling, Sec. 3.3).
// Both passes evaluate every stored coordinate.  The coordinate i xor (m rep)
// reads the images of the values coordinate i reads, in an order that only
// swaps operands of commutative additions and of the max, so its W equals W[i]
// bit for bit in every rounding mode: the max over stored coordinates is the
// max over all coordinates, and its lowest index is a stored one.  FP32 tables
// are certified as their exact FP64 values: the certificate is translation
// invariant, so the FP64 offset of an FP32 table does not enter W; it enters
// only R.
#include <math.h>

#include <type_traits>

#include "internal.h"
#include "rounding.h"

namespace lcsb {
namespace {

__device__ __forceinline__ void merge_max_idx(double &v, uint64_t &i, double ov, uint64_t oi)
{
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
}

// workgroup reduction of (max value, lowest index, count); result in thread 0
__device__ void block_reduce(double &v, uint64_t &i, uint64_t &c)
{
    for (int o = 32; o > 0; o >>= 1) {
        double ov = __shfl_xor(v, o);
        uint64_t oi = __shfl_xor(i, o);
        uint64_t oc = __shfl_xor(c, o);
        merge_max_idx(v, i, ov, oi);
        c += oc;
    }
    __shared__ double sv[kBlock / 64];
    __shared__ uint64_t si[kBlock / 64], sc[kBlock / 64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) { sv[w] = v; si[w] = i; sc[w] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlock / 64; ++k) {
            merge_max_idx(v, i, sv[k], si[k]);
            c += sc[k];
        }
    }
}

// Fold the per-workgroup partials (max value, lowest index, count) of a pass
// into this thread's running result: thread k takes partials k, k + 256, ..,
// eight loads in flight at a time (up to 16384 partials: one load after the
// other made this final pass 56 us).
__device__ __forceinline__ void merge_partials(const unsigned char *__restrict__ ws, int nparts,
                                               double &best, uint64_t &arg, uint64_t &nonfinite)
{
    const double *pv = reinterpret_cast<const double *>(ws + Ws::kPartVal);
    const uint64_t *pi = reinterpret_cast<const uint64_t *>(ws + Ws::kPartIdx);
    const uint64_t *pc = reinterpret_cast<const uint64_t *>(ws + Ws::kPartCnt);
    constexpr int kBatch = 8;
    for (int k0 = threadIdx.x; k0 < nparts; k0 += kBatch * kBlock) {
        double v[kBatch];
        uint64_t i[kBatch], c[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const int k = k0 + j * kBlock;
            const bool in = k < nparts;
            v[j] = in ? pv[k] : -INFINITY;
            i[j] = in ? pi[k] : 0;
            c[j] = in ? pc[k] : 0;
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            merge_max_idx(best, arg, v[j], i[j]);
            nonfinite += c[j];
        }
    }
}

// n = stored entries.  SWAP_D (2 or 3: sigma = 2 with d = SWAP_D; 4: sigma =
// 4, d = 2; both tables symmetric in strings 1 and 2): u - prev is equal at a
// stored entry and at its exchanged twin (exchange_twin, exchange_twin4), so
// only the lower of the two is read, counted twice unless it is its own twin.
// A thread takes aligned groups of G entries (the groups of twin_group,
// twin_group8, twin_group16): a group is entirely lower (read as a vector,
// every member counted twice), entirely upper (not read) or its own twin
// (member by member).  The maximum is exact in any order; only its value
// leaves the pass (the index carried beside it is the lowest one).
// 16 bytes: four floats or two doubles
template <typename T>
__device__ __forceinline__ void ld16(const T *p, T *v)
{
    if constexpr (std::is_same<T, float>::value) {
        const float4 q = *reinterpret_cast<const float4 *>(p);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
        const double2 q = *reinterpret_cast<const double2 *>(p);
        v[0] = q.x; v[1] = q.y;
    }
}

template <typename T, int SWAP_D>
__global__ __launch_bounds__(kBlock) void cert_r(const T *__restrict__ u,
                                                const T *__restrict__ prev, uint64_t n,
                                                unsigned char *__restrict__ ws)
{
    constexpr int G = SWAP_D == 3 ? 8 : SWAP_D == 4 ? 16 : 4;
    constexpr int V = 16 / sizeof(T);  // elements per 16-byte load
    double best = -INFINITY;
    uint64_t arg = 0, nonfinite = 0;
    auto twin_of = [&](uint64_t j) {
        return SWAP_D == 4 ? exchange_twin4(j, 4 * n) : exchange_twin(j, 2 * n, SWAP_D);
    };
    auto take = [&](uint64_t j, double a, double b, uint64_t mult) {
        if (!isfinite(a) || !isfinite(b)) nonfinite += mult;
        const double diff = a - b;
        if (diff > best) { best = diff; arg = j; }
    };
    const uint64_t stride = (uint64_t)gridDim.x * kBlock, ng = n / G;
    const uint64_t t0 = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    for (uint64_t q = t0; q < ng; q += stride) {
        const uint64_t base = q * G;
        int kind = 0;  // 0 lower (or no symmetry), 1 upper, 2 its own twin
        if constexpr (SWAP_D == 2) {
            const int m = twin_group(base, 2 * n).mode;
            kind = m == 0 ? 0 : m <= 2 ? 1 : 2;
        } else if constexpr (SWAP_D == 3) {
            const int m = twin_group8(base, 2 * n).mode;
            kind = m == 0 ? 0 : m <= 2 ? 1 : 2;
        } else if constexpr (SWAP_D == 4) {
            kind = twin_group16(base, 4 * n).kind;
        }
        if (kind == 1) continue;
        T a[G], b[G];
#pragma unroll
        for (int k = 0; k < G; k += V) {
            ld16(u + base + k, a + k);
            ld16(prev + base + k, b + k);
        }
#pragma unroll
        for (int v = 0; v < G; ++v) {
            const uint64_t j = base + v;
            uint64_t mult = SWAP_D != 0 ? 2 : 1;
            if (SWAP_D != 0 && kind == 2) {
                const uint64_t js = twin_of(j);
                if (js < j) continue;
                mult = js == j ? 1 : 2;
            }
            take(j, (double)a[v], (double)b[v], mult);
        }
    }
    // entries after the last whole group (tables of fewer than G entries)
    const uint64_t j = ng * G + t0;
    if (j < n) {
        uint64_t mult = 1;
        bool use = true;
        if constexpr (SWAP_D != 0) {
            const uint64_t js = twin_of(j);
            use = js >= j;
            mult = js == j ? 1 : 2;
        }
        if (use) take(j, (double)u[j], (double)prev[j], mult);
    }
    block_reduce(best, arg, nonfinite);
    if (threadIdx.x == 0) {
        reinterpret_cast<double *>(ws + Ws::kPartVal)[blockIdx.x] = best;
        reinterpret_cast<uint64_t *>(ws + Ws::kPartIdx)[blockIdx.x] = arg;
        reinterpret_cast<uint64_t *>(ws + Ws::kPartCnt)[blockIdx.x] = nonfinite;
    }
}

// Reduce the pass-1 partials; derive the shifts.  One workgroup.
__global__ __launch_bounds__(kBlock) void cert_r_final(unsigned char *__restrict__ ws,
                                                      int nparts, int d, int f32, int u_slot,
                                                      int prev_slot)
{
    double best = -INFINITY;
    uint64_t arg = 0, nonfinite = 0;
    merge_partials(ws, nparts, best, arg, nonfinite);
    block_reduce(best, arg, nonfinite);
    if (threadIdx.x == 0) {
        double R = best;
        if (f32) {
            const double *off = reinterpret_cast<const double *>(ws + Ws::kOffsets);
            R = R + (off[u_slot] - off[prev_slot]);
        }
        double *sc = reinterpret_cast<double *>(ws);
        sc[Ws::kR / 8] = R;
        sc[Ws::kDRup / 8] = mul_ru((double)d, R);
        for (int k = 0; k < 4; ++k) sc[Ws::kShift / 8 + k] = mul_rd((double)(d - k), R);
        reinterpret_cast<uint64_t *>(ws)[Ws::kNonfiniteR / 8] = nonfinite;
    }
}

// ------------------------------------------------------------------ W pass
// One thread per x (the non-head positions) evaluates W at every head slot
// of x, reading the all-advance group of x once and each branch group as a
// vector.  Per coordinate the arithmetic is exactly the one stated above
// (identical to evaluating each coordinate on its own).

// Four consecutive values as doubles.  FP32 groups are read non-temporally:
// the pass visits each address from four streams at far-apart times, so
// nothing it loads is found again in the caches (5% faster at l = 16; FP64
// keeps ordinary loads, which non-temporal ones slowed down in the sweep).
template <typename T>
__device__ __forceinline__ void ld4(const T *p, double *v)
{
    if constexpr (std::is_same<T, float>::value) {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = __builtin_nontemporal_load(p + k);
    } else {
        const double2 a = reinterpret_cast<const double2 *>(p)[0];
        const double2 b = reinterpret_cast<const double2 *>(p)[1];
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
}

// Set this wave's FP rounding mode (MODE.FP_ROUND, single and double
// fields) to toward -inf.  The wave keeps the mode until it ends; a new
// wave starts from the kernel descriptor's mode.  The returned zero is
// opaque to the compiler: every load of the pass adds it to its base, so no
// arithmetic on loaded data can be scheduled ahead of the switch.  Within
// such a pass the code must not negate a product (the compiler may rewrite
// -(a b) as a (-b), which is equal only under round-to-nearest); sums,
// differences, negated sums, max and the exact FP32 -> FP64 widening are
// safe.
__device__ __forceinline__ uint64_t round_toward_neg_inf()
{
    uint64_t z = 0;
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 0, 4), 10\n\ts_nop 3" : "+s"(z));
    return z;
}

// 2^-j for j = 1..4, hidden from the compiler so that the scaling stays a
// multiply (rounded by the mode) rather than a rewrite into ldexp.
struct Scales {
    double q[5];
    __device__ __forceinline__ Scales()
    {
        q[0] = 1.0; q[1] = 0.5; q[2] = 0.25; q[3] = 0.125; q[4] = 0.0625;
#pragma unroll
        for (int j = 1; j <= 4; ++j) asm volatile("" : "+s"(q[j]));
    }
};

// In round-toward-minus-infinity mode: mean over CNT values of (v + shift),
// every add rounded down, the pairwise tree in the given order, the exact
// power-of-two scaling rounded down.  Callers pass sigma = 2 groups in the
// complement-paired leaf order of the sweep (t, ~t for t = 0, 1, ..).
template <int CNT>
__device__ __forceinline__ double mean_rd(double *v, double shift, double scale)
{
#pragma unroll
    for (int t = 0; t < CNT; ++t) v[t] = v[t] + shift;
#pragma unroll
    for (int step = 1; step < CNT; step <<= 1)
#pragma unroll
        for (int t = 0; t < CNT; t += 2 * step) v[t] = v[t] + v[t + step];
    return v[0] * scale;
}

// F's max over branch means starts from -inf (a NaN branch never wins, every
// branch NaN gives -inf): the first value of each max chain goes through this.
__device__ __forceinline__ double first(double v) { return v > -INFINITY ? v : -INFINITY; }

// Two evaluations share the coordinate walk below.
//
// WEval (Algorithm 2): F on the shifted arguments u + (d-k)R, then
// W = u + dR - F at every coordinate and its max.
//
// OptEval (the largest r of a feasible triplet (u, r, 0), from the lemma of
// Sec. 2.1 with eps = 0): every argument of F is u (no shift); branch z of
// coordinate A, moving k_z strings, gives c_z = b(A) + mean_z - u[A] and the
// ratio q_z = c_z / k_z; the coordinate's value is the max over its branches
// and r the min over coordinates.  All in round-toward-minus-infinity mode:
// the mean, the 1 +, the subtraction and the scaling by 1/k_z (exact for
// k = 1, 2; for k = 3 a multiply by 1/3 rounded down when c >= 0, up when
// c < 0), so every q_z is at most the exact c_z / k_z.  A zero ratio is +0,
// so the max does not depend on the order of the branches.  Coordinates
// arrive in any order: keep the min, lowest index on ties.

struct WEval {
    double shift[4];  // (d-k)R rounded down, k = 0..3
    double dR_up;
    double w = -INFINITY;
    uint64_t arg = 0, nonfinite = 0;

    template <int CNT>
    __device__ __forceinline__ double mean(double *v, int k, double scale) const
    {
        return mean_rd<CNT>(v, shift[k], scale);
    }
    // W = RU(RU(u_i + dR_up) - f_lo) = -RD(RD(-u_i - dR_up) + f_lo); `mult`:
    // how many coordinates of equal W this evaluation stands for
    __device__ __forceinline__ void put(double u_i, double f_lo, uint64_t i, int mult)
    {
        const double t = (-u_i) - dR_up;
        const double w_i = -(t + f_lo);
        if (!isfinite(w_i)) nonfinite += (uint64_t)mult;
        if (w_i > w || (w_i == w && i < arg)) { w = w_i; arg = i; }
    }
    // all-match coordinate: F = 1 + mean over all d moved strings
    __device__ __forceinline__ void match(double u_i, double m_all, uint64_t i, int mult)
    {
        put(u_i, 1.0 + first(m_all), i, mult);
    }
    // mismatched coordinate with branch means m[j] moving k[j] strings, in z order
    template <int NB>
    __device__ __forceinline__ void mismatch(double u_i, const double *m, const int *, uint64_t i,
                                             int mult)
    {
        double f = first(m[0]);
#pragma unroll
        for (int j = 1; j < NB; ++j) f = m[j] > f ? m[j] : f;
        put(u_i, f, i, mult);
    }
    // block result: the value whose max the final pass takes
    __device__ __forceinline__ double result() const { return w; }
};

struct OptEval {
    double half, inv3_lo, inv3_hi;  // 1/2; 1/3 rounded down and up (opaque to the compiler)
    double r = INFINITY;
    uint64_t arg = 0, nonfinite = 0;

    __device__ __forceinline__ OptEval(double h, double lo, double hi) : half(h), inv3_lo(lo), inv3_hi(hi)
    {
        asm volatile("" : "+s"(half));
        asm volatile("" : "+s"(inv3_lo));
        asm volatile("" : "+s"(inv3_hi));
    }
    template <int CNT>
    __device__ __forceinline__ double mean(double *v, int, double scale) const
    {
#pragma unroll
        for (int step = 1; step < CNT; step <<= 1)
#pragma unroll
            for (int t = 0; t < CNT; t += 2 * step) v[t] = v[t] + v[t + step];
        return v[0] * scale;
    }
    __device__ __forceinline__ double ratio(double c, int k) const
    {
        double q = k == 1 ? c : k == 2 ? c * half : (c >= 0.0 ? c * inv3_lo : c * inv3_hi);
        return q == 0.0 ? 0.0 : q;
    }
    __device__ __forceinline__ void put(double q, uint64_t i, int mult)
    {
        if (!isfinite(q)) nonfinite += (uint64_t)mult;
        if (q < r || (q == r && i < arg)) { r = q; arg = i; }
    }
    // whether put(q, ...) could change the state: a candidate above the
    // current r that is finite leaves it as it is, whatever its index
    __device__ __forceinline__ bool may_take(double q) const { return !(q > r) || !isfinite(q); }
    template <int D>
    __device__ __forceinline__ double match_q(double u_i, double m_all) const
    {
        return first(ratio((1.0 + m_all) - u_i, D));
    }
    template <int NB>
    __device__ __forceinline__ double mismatch_q(double u_i, const double *m, const int *k) const
    {
        double f = first(ratio(m[0] - u_i, k[0]));
#pragma unroll
        for (int j = 1; j < NB; ++j) {
            const double q = ratio(m[j] - u_i, k[j]);
            f = q > f ? q : f;
        }
        return f;
    }
    template <int D>
    __device__ __forceinline__ void match_d(double u_i, double m_all, uint64_t i, int mult)
    {
        put(match_q<D>(u_i, m_all), i, mult);
    }
    template <int NB>
    __device__ __forceinline__ void mismatch(double u_i, const double *m, const int *k, uint64_t i,
                                             int mult)
    {
        put(mismatch_q<NB>(u_i, m, k), i, mult);
    }
    // the final pass takes a max: hand it -r (exact; lowest index kept on ties)
    __device__ __forceinline__ double result() const { return -r; }
};

// the all-match call of either evaluation (d strings move)
template <int D>
__device__ __forceinline__ void eval_match(WEval &ev, double u_i, double m_all, uint64_t i, int mult)
{
    ev.match(u_i, m_all, i, mult);
}
template <int D>
__device__ __forceinline__ void eval_match(OptEval &ev, double u_i, double m_all, uint64_t i,
                                           int mult)
{
    ev.template match_d<D>(u_i, m_all, i, mult);
}

// sigma = d = 2: thread t < n/8 evaluates the stored coordinates 0/0|t,
// 0/0|xc, 0/1|t, 0/1|xc (xc = n/4-1-t, the complement of t).  The lag-2 group
// of xc is the image of the one of t; the advance-a pair of 0/1|xc is read in
// the image group at the other parity (see the sweep).
// SWAP (a table symmetric under exchanging the strings): the value is then
// equal, bit for bit, at exchanged tuples (the trees are exchange-invariant),
// so only the lower of the threads t and p (St or ~St, as in the sweep)
// evaluates, each value standing for two coordinates unless p = t.  The
// lowest index of each pair is t, ~St, 0/1|t and 0/1|St; the table is kept
// lazily (TwinGroup), so u is read there and every group through its lower
// members.
template <typename T, bool SWAP, class Ev>
__device__ __forceinline__ void w_s2d2(const T *__restrict__ u, uint64_t n, uint64_t t,
                                      const Scales &sc, Ev &ev)
{
    const uint64_t nq = n >> 2, xc = nq - 1 - t;
    uint64_t rep_xc = xc, rep_mis1 = nq + xc;
    int mult = 1;
    if constexpr (SWAP) {
        const uint64_t mq = nq - 1, aq = 0xAAAAAAAAAAAAAAAAull & mq;
        const uint64_t st = ((t & aq) >> 1) | ((t & ~aq & mq) << 1);
        const uint64_t p = (t & (nq >> 2)) ? st ^ mq : st;
        if (p < t) return;
        mult = p == t ? 1 : 2;
        rep_xc = mq - st;
        rep_mis1 = nq + st;
    }
    const uint64_t am = 0xAAAAAAAAAAAAAAAAull & (n - 1), bm = ~am & (n - 1);
    // the group at `base` in member order (through its lower members if SWAP)
    auto group = [&](uint64_t base, double *e) {
        if constexpr (SWAP) {
            const TwinGroup tg = twin_group(base, n);
            double q[4];
            ld4(u + tg.read, q);
            twin_values(q, tg.mode, e);
        } else {
            ld4(u + base, e);
        }
    };
    double q4[4];
    group(4 * t, q4);
    double g[4] = {q4[0], q4[3], q4[1], q4[2]};
    const double m_all = ev.template mean<4>(g, 2, sc.q[2]);
    eval_match<2>(ev, (double)u[t], m_all, t, mult);
    eval_match<2>(ev, (double)u[rep_xc], m_all, rep_xc, mult);
    constexpr int ks[2] = {1, 1};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const uint64_t i = nq + (c ? xc : t);
        const uint64_t sb = (i & am) | ((i << 2) & bm);
        const uint64_t sa = ((i << 2) & am) | (i & bm);
        double q[4], pb[2], pa[2];
        group(sb & ~(uint64_t)3, q);
        const bool hi = (sb & 2) != 0;
        pb[0] = hi ? q[2] : q[0]; pb[1] = hi ? q[3] : q[1];
        const uint64_t grp = sa & ~(uint64_t)3;
        group(c ? (n - 4) - grp : grp, q);
        const bool odd = ((sa & 1) ^ (uint64_t)c) != 0;
        pa[0] = odd ? q[1] : q[0]; pa[1] = odd ? q[3] : q[2];
        // branches in z order: z = 0 advances b, z = 1 advances a
        const double m[2] = {ev.template mean<2>(pb, 1, sc.q[1]), ev.template mean<2>(pa, 1, sc.q[1])};
        const uint64_t at = c ? rep_mis1 : i;  // i itself unless SWAP
        ev.template mismatch<2>((double)u[at], m, ks, at, mult);
    }
}

// sigma = 4, d = 2: thread t < n/64 evaluates the stored coordinates
// (0, b1)|x_m, x_m = t xor (m rep), m, b1 = 0..3.  Branches of a mismatched
// pair: advance b (stored directly), advance a (the image of the advance-a
// group of (0, b1 xor m)|t), advance both (the image of t's group, shared
// with the all-match value).
// SWAP (a table symmetric in the two strings): as in the sweep, only the
// lower of t and its twin thread p evaluates; each coordinate is read and
// reported at the lower index of its exchanged pair and counts for both
// unless p = t; groups are read through their lower members (Twin16).
template <typename T, bool SWAP, class Ev>
__device__ __forceinline__ void w_s4d2(const T *__restrict__ u, uint64_t n, int h, uint64_t t,
                                      const Scales &sc, Ev &ev)
{
    const int top = 4 * (h - 1);
    const uint64_t am = 0xCCCCCCCCCCCCCCCCull & (n - 1), bm = ~am & (n - 1);
    const uint64_t rep = ((n >> 4) - 1) / 3;
    uint64_t p = t;
    int sx = 0, mult = 1;
    if constexpr (SWAP) {
        sx = (int)((t >> (top - 4)) & 3);
        p = exchange4(t, n >> 4) ^ ((uint64_t)sx * rep);
        if (p < t) return;
        mult = p == t ? 1 : 2;
    }
    double q16[16];
    if constexpr (SWAP) {
        const Twin16 tw = twin_group16(16 * t, n);
        if (tw.kind == 2) {
#pragma unroll
            for (int v = 0; v < 16; ++v) q16[v] = (double)u[member16(16 * t, tw, v)];
        } else {  // the tree is invariant under the twin's member permutation
#pragma unroll
            for (int k = 0; k < 16; k += 4) ld4(u + tw.read + k, q16 + k);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; k += 4) ld4(u + 16 * t + k, q16 + k);
    }
    // leaves in the sweep's order (tree16): pairs {ab, ba} by a xor b, {aa, ~a~a}
    double g[16] = {q16[1], q16[4], q16[11], q16[14], q16[2], q16[8], q16[7], q16[13],
                    q16[3], q16[12], q16[6], q16[9], q16[0], q16[15], q16[5], q16[10]};
    const double m_both = ev.template mean<16>(g, 2, sc.q[4]);
    double ma[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const uint64_t i = ((uint64_t)v << top) | t;
        const uint64_t sa = ((i << 4) & am) | (i & bm);
        double q[4];
        if constexpr (SWAP) {
            const uint64_t gb = sa & ~(uint64_t)15;
            const int o = (int)(sa & 15);
            const Twin16 tw = twin_group16(gb, n);
#pragma unroll
            for (int k = 0; k < 4; ++k) q[k] = (double)u[member16(gb, tw, o + 4 * k)];
        } else {
            q[0] = u[sa]; q[1] = u[sa + 4]; q[2] = u[sa + 8]; q[3] = u[sa + 12];
        }
        ma[v] = ev.template mean<4>(q, 1, sc.q[2]);
    }
    constexpr int ks[3] = {1, 1, 2};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const uint64_t x = t ^ ((uint64_t)m * rep);
        const uint64_t sb = (x & am) | ((x << 4) & bm);
        double q[4];
        if constexpr (SWAP) {
            const uint64_t gb = sb & ~(uint64_t)15;
            const int o = (int)(sb & 15);
            const Twin16 tw = twin_group16(gb, n);
#pragma unroll
            for (int k = 0; k < 4; ++k) q[k] = (double)u[member16(gb, tw, o + k)];
        } else {
            ld4(u + sb, q);
        }
        const double mb = ev.template mean<4>(q, 1, sc.q[2]);
        // the lower index of the exchanged pair of coordinate (b1 << top) | x
        auto at = [&](int b1) {
            const uint64_t xt = p ^ ((uint64_t)(m ^ b1 ^ sx) * rep);
            return ((uint64_t)b1 << top) | (SWAP && xt < x ? xt : x);
        };
        eval_match<2>(ev, (double)u[at(0)], m_both, at(0), mult);
#pragma unroll
        for (int b1 = 1; b1 < 4; ++b1) {
            // z = 0 advances b, z = b1 advances a, the other two advance both
            const double mz[3] = {mb, ma[b1 ^ m], m_both};
            ev.template mismatch<3>((double)u[at(b1)], mz, ks, at(b1), mult);
        }
    }
}

// sigma = 2, d = 3: thread t < n/16 evaluates the stored head triples 000 ..
// 011 of x = t and of its complement xc.  A mismatched triple has two
// branches: the strings with head 1 advance (z = 0) and the strings with head
// 0 advance (z = 1); k = |N| selects the lag and shift.  A branch that moves
// string 1 of xc reads every value at the image of its index.
template <int SET, bool SWAP, typename T, class Ev>
__device__ __forceinline__ double branch23(const T *__restrict__ u, uint64_t n, uint64_t i,
                                           int img, const Scales &sc, const Ev &ev)
{
    // SET: bit 2 = string 1, bit 1 = string 2, bit 0 = string 3
    constexpr int K = __builtin_popcount(SET);
    const uint64_t r3 = (n - 1) / 7;
    const uint64_t sm = ((SET & 4) ? r3 << 2 : 0) | ((SET & 2) ? r3 << 1 : 0) | ((SET & 1) ? r3 : 0);
    const uint64_t base = (i & ~sm) | ((i << 3) & sm & (n - 1));
    double lx[K == 1 ? 2 : 4];
    int k = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c)  // appended tuples in lexicographic order of the moved strings
        if ((c & ~SET) == 0) {
            const uint64_t e = base | (uint64_t)c;
            uint64_t at = img ? (n - 1) - e : e;
            if constexpr (SWAP) {  // the lower member of its exchanged pair
                const uint64_t tw = exchange_twin(at, n, 3);
                at = tw < at ? tw : at;
            }
            lx[k++] = (double)u[at];
        }
    if constexpr (K == 1) return ev.template mean<2>(lx, 1, sc.q[1]);
    double v[4] = {lx[0], lx[3], lx[1], lx[2]};  // complement-paired leaves
    return ev.template mean<4>(v, 2, sc.q[2]);
}

// SWAP (a table symmetric in strings 1 and 2): as for d = 2, only the lower of
// the threads t and p (Et or ~Et, as in the sweep) evaluates; every value is
// read, and reported, at the lower index of its exchanged pair, and counts
// for both coordinates unless p = t.
template <typename T, bool SWAP, class Ev>
__device__ __forceinline__ void w_s2d3(const T *__restrict__ u, uint64_t n, int h, uint64_t t,
                                      const Scales &sc, Ev &ev)
{
    const int top = 3 * (h - 1);
    const uint64_t mx = (n >> 3) - 1, xc = mx - t;
    int mult = 1;
    if constexpr (SWAP) {
        const uint64_t et = exchange12(t, n >> 3);
        const uint64_t p = (t & (mx + 1) >> 2) ? et ^ mx : et;
        if (p < t) return;
        mult = p == t ? 1 : 2;
    }
    auto lower = [&](uint64_t j) {
        if constexpr (SWAP) {
            const uint64_t tw = exchange_twin(j, n, 3);
            return tw < j ? tw : j;
        } else {
            return j;
        }
    };
    double q8[8];
    if constexpr (SWAP) {
        const TwinGroup tg = twin_group8(8 * t, n);
        double r8[8];
        ld4(u + tg.read, r8);
        ld4(u + tg.read + 4, r8 + 4);
        twin_values8(r8, tg.mode, q8);
    } else {
        ld4(u + 8 * t, q8);
        ld4(u + 8 * t + 4, q8 + 4);
    }
    double g[8] = {q8[0], q8[7], q8[1], q8[6], q8[2], q8[5], q8[3], q8[4]};
    const double m_all = ev.template mean<8>(g, 3, sc.q[3]);
    eval_match<3>(ev, (double)u[lower(t)], m_all, lower(t), mult);
    eval_match<3>(ev, (double)u[lower(xc)], m_all, lower(xc), mult);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const uint64_t x = c ? xc : t;
#define LCSB_HEAD(H)                                                                             \
        {                                                                                        \
            const uint64_t i = ((uint64_t)(H) << top) | x;                                       \
            /* z order: z = 0 moves the strings with head 1, z = 1 those with head 0 */         \
            const double m[2] = {                                                                \
                branch23<(H), SWAP, T>(u, n, i, ((H) & 4) ? c : 0, sc, ev),                     \
                branch23<(~(H)) & 7, SWAP, T>(u, n, i, ((~(H)) & 4) ? c : 0, sc, ev)};          \
            constexpr int ks[2] = {__builtin_popcount(H), __builtin_popcount((~(H)) & 7)};      \
            const uint64_t at = lower(i);                                                        \
            ev.template mismatch<2>((double)u[at], m, ks, at, mult);                             \
        }
        LCSB_HEAD(1) LCSB_HEAD(2) LCSB_HEAD(3)
#undef LCSB_HEAD
    }
}

// the evaluation a kernel runs: W (Algorithm 2) reads its scalars from the
// workspace; the largest-r certificate takes 1/2 and 1/3 rounded both ways
template <bool OPT>
using EvalOf = typename std::conditional<OPT, OptEval, WEval>::type;

__device__ __forceinline__ WEval make_eval(const double *sc_ws, const double *, std::false_type)
{
    WEval ev;
    ev.dR_up = sc_ws[Ws::kDRup / 8];
#pragma unroll
    for (int k = 0; k < 4; ++k) ev.shift[k] = sc_ws[Ws::kShift / 8 + k];  // (d-k)R, rounded down
    return ev;
}
__device__ __forceinline__ OptEval make_eval(const double *, const double *inv, std::true_type)
{
    return OptEval(0.5, inv[0], inv[1]);
}

template <class Ev>
__device__ __forceinline__ void store_block(const Ev &ev, unsigned char *__restrict__ ws)
{
    double v = ev.result();
    uint64_t arg = ev.arg, nonfinite = ev.nonfinite;
    block_reduce(v, arg, nonfinite);
    if (threadIdx.x == 0) {
        reinterpret_cast<double *>(ws + Ws::kPartVal)[blockIdx.x] = v;
        reinterpret_cast<uint64_t *>(ws + Ws::kPartIdx)[blockIdx.x] = arg;
        reinterpret_cast<uint64_t *>(ws + Ws::kPartCnt)[blockIdx.x] = nonfinite;
    }
}

// inv3 (OPT only): 1/3 rounded down and up, for the all-match ratio of d = 3
template <int SIGMA, int D, typename T, bool SWAP, bool OPT>
__global__ __launch_bounds__(kBlock) void cert_w(const T *__restrict__ u_arg, uint64_t n, int h,
                                                unsigned char *__restrict__ ws, double inv3_lo,
                                                double inv3_hi)
{
    constexpr int BITS = (SIGMA == 2 ? 1 : 2) * (D + 1);  // head slot and string-1 symbol 2
    const uint64_t z = round_toward_neg_inf();
    const T *__restrict__ u = u_arg + z;
    const double *sc_ws = reinterpret_cast<const double *>(ws + z);
    const double inv[2] = {inv3_lo, inv3_hi};
    auto ev = make_eval(sc_ws, inv, std::integral_constant<bool, OPT>());
    const Scales sc;
    const uint64_t nt = n >> BITS;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x; t < nt; t += stride) {
        if constexpr (SIGMA == 2 && D == 2) w_s2d2<T, SWAP>(u, n, t, sc, ev);
        else if constexpr (SIGMA == 4) w_s4d2<T, SWAP>(u, n, h, t, sc, ev);
        else w_s2d3<T, SWAP>(u, n, h, t, sc, ev);
    }
    store_block(ev, ws);
}

// Exchange-packed tables (sigma = d = 2, packed_index): one thread per code
// evaluates its orbit's representative tuple exactly as w_s2d2 evaluates
// that coordinate (the same values in the same trees); the ratio stands for
// every coordinate of the orbit, the index kept is the orbit's lowest stored
// index (the representative or its exchanged twin) and `mult` counts the
// stored coordinates of the orbit (1 or 2).
template <typename T>
__device__ __forceinline__ void packed_group_rd(const T *__restrict__ u, uint64_t gbase, int h,
                                                double *e)
{
    const PackedGroup pg = packed_group(gbase, h);
    if (pg.regular) {
        double q[4];
        ld4(u + pg.base, q);
#pragma unroll
        for (int k = 0; k < 4; ++k) asm volatile("" : "+v"(q[k]));
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int at = packed_member(pg, v);
            e[v] = at == 0 ? q[0] : at == 1 ? q[1] : at == 2 ? q[2] : q[3];
        }
    } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) e[v] = (double)u[packed_index(gbase + (uint64_t)v, h)];
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void cert_opt_packed(const T *__restrict__ u_arg, int h,
                                                         unsigned char *__restrict__ ws)
{
    const uint64_t z = round_toward_neg_inf();
    const T *__restrict__ u = u_arg + z;
    OptEval ev(0.5, 0.0, 0.0);  // d = 2: no division by 3
    const Scales sc;
    const uint64_t n = 1ull << (2 * h), nq = n >> 2, ncodes = packed_entries(h);
    const uint64_t am = 0xAAAAAAAAAAAAAAAAull & (n - 1), bm = ~am & (n - 1);
    constexpr int ks[2] = {1, 1};
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x; k < ncodes; k += stride) {
        const uint64_t i = packed_tuple(k, h);
        if (i == kNoOrbit) continue;
        // a coordinate's reported index (the lower stored member of its
        // exchanged pair) and its multiplicity only matter where put can use
        // them, so they are computed there
        const auto take = [&](double q, uint64_t tuple) {
            if (!ev.may_take(q)) return;
            const uint64_t tw = exchange_twin(tuple, n, 2);
            ev.put(q, tw < tuple ? tw : tuple, tw == tuple ? 1 : 2);
        };
        const double u_i = (double)u[k];
        if (i < nq) {  // head 0/0
            // 0/0|x and 0/0|~x share their group mean (image groups): the
            // lower of the two codes evaluates both coordinates
            const uint64_t ic = i ^ (nq - 1), kc = packed_index(ic, h);
            if (kc < k) continue;
            double q4[4];
            packed_group_rd(u, (i << 2) & (n - 1), h, q4);
            double g[4] = {q4[0], q4[3], q4[1], q4[2]};
            const double m_all = ev.template mean<4>(g, 2, sc.q[2]);
            take(ev.template match_q<2>(u_i, m_all), i);
            if (kc != k) {
                const double q = ev.template match_q<2>((double)u[kc], m_all);
                if (ev.may_take(q)) take(q, packed_tuple(kc, h));
            }
        } else {       // head 0/1: z = 0 advances b, z = 1 advances a
            const uint64_t sb = (i & am) | ((i << 2) & bm);
            const uint64_t sa = ((i << 2) & am) | (i & bm);
            double q[4], pb[2], pa[2];
            packed_group_rd(u, sb & ~(uint64_t)3, h, q);
            const bool hi = (sb & 2) != 0;
            pb[0] = hi ? q[2] : q[0]; pb[1] = hi ? q[3] : q[1];
            packed_group_rd(u, sa & ~(uint64_t)3, h, q);
            const bool odd = (sa & 1) != 0;
            pa[0] = odd ? q[1] : q[0]; pa[1] = odd ? q[3] : q[2];
            const double m[2] = {ev.template mean<2>(pb, 1, sc.q[1]),
                                 ev.template mean<2>(pa, 1, sc.q[1])};
            take(ev.template mismatch_q<2>(u_i, m, ks), i);
        }
    }
    store_block(ev, ws);
}

// l = 1: each branch appends its symbols in the head slot, so its tuples
// straddle the stored half and every value is read at the image of its
// index.  One workgroup; thread j evaluates stored coordinate j.  Templates on
// (sigma, d) and the moved set M keep every array in registers.
template <int SIGMA, int D>
struct L1 {
    static constexpr int kBeta = SIGMA == 2 ? 1 : 2;
    static constexpr int kN = 1 << (kBeta * D);
    static constexpr int kNs = kN >> kBeta;
    static constexpr int kRep = (kN - 1) / (SIGMA - 1);
    static __device__ __forceinline__ int image(int i) { return i ^ ((i >> (kBeta * (D - 1))) * kRep); }
    template <int M>  // head with the moved strings' symbols replaced by tuple c
    static __device__ __forceinline__ int successor(int head, int c)
    {
#pragma unroll
        for (int s = D - 1; s >= 0; --s) {
            if (!((M >> s) & 1)) continue;
            const int sh = kBeta * (D - 1 - s);
            head = (head & ~((SIGMA - 1) << sh)) | ((c & (SIGMA - 1)) << sh);
            c >>= kBeta;
        }
        return head;
    }
    template <int CNT>  // appended tuple at leaf j of the branch tree (as the sweep's)
    static __device__ __forceinline__ int leaf(int j)
    {
        constexpr int order16[16] = {1, 4, 11, 14, 2, 8, 7, 13, 3, 12, 6, 9, 0, 15, 5, 10};
        if (SIGMA == 4) return CNT == 16 ? order16[j] : j;
        return (j & 1) ? CNT - 1 - (j >> 1) : j >> 1;
    }
};

// In round-toward-minus-infinity mode: the branch mean of moved set `moved`
// (searched from M up), as the evaluation's mean
template <typename T, int SIGMA, int D, int M, class Ev>
__device__ __forceinline__ double l1_branch_rd(const T *__restrict__ u, const Ev &ev,
                                               const Scales &sc, int head, int moved)
{
    using G = L1<SIGMA, D>;
    if constexpr (M >= (1 << D)) {
        return 0.0;
    } else {
        if (moved != M) return l1_branch_rd<T, SIGMA, D, M + 1>(u, ev, sc, head, moved);
        constexpr int K = __builtin_popcount(M), CNT = 1 << (G::kBeta * K);
        double v[CNT];
#pragma unroll
        for (int c = 0; c < CNT; ++c)
            v[c] = (double)u[G::image(G::template successor<M>(head, G::template leaf<CNT>(c)))];
        return ev.template mean<CNT>(v, K, sc.q[G::kBeta * K]);
    }
}

template <typename T, int SIGMA, int D, bool OPT>
__global__ __launch_bounds__(kBlock) void cert_w_l1(const T *__restrict__ u_arg,
                                                   unsigned char *__restrict__ ws, double inv3_lo,
                                                   double inv3_hi)
{
    using G = L1<SIGMA, D>;
    const uint64_t z = round_toward_neg_inf();
    const T *__restrict__ u = u_arg + z;
    const double *sc_ws = reinterpret_cast<const double *>(ws + z);
    const double inv[2] = {inv3_lo, inv3_hi};
    auto ev = make_eval(sc_ws, inv, std::integral_constant<bool, OPT>());
    const Scales sc;
    const int j = threadIdx.x;
    if (j < G::kNs) {
        int sym[D];
        bool same = true;
#pragma unroll
        for (int s = 0; s < D; ++s) {
            sym[s] = (j >> (G::kBeta * (D - 1 - s))) & (SIGMA - 1);
            same = same && sym[s] == sym[0];
        }
        if (same) {
            const double m = l1_branch_rd<T, SIGMA, D, 1>(u, ev, sc, j, (1 << D) - 1);
            eval_match<D>(ev, (double)u[j], m, (uint64_t)j, 1);
        } else {
            double m[SIGMA];
            int ks[SIGMA];
#pragma unroll
            for (int zz = 0; zz < SIGMA; ++zz) {
                int moved = 0;
#pragma unroll
                for (int s = 0; s < D; ++s)
                    if (sym[s] != zz) moved |= 1 << s;
                m[zz] = l1_branch_rd<T, SIGMA, D, 1>(u, ev, sc, j, moved);
                ks[zz] = __builtin_popcount(moved);
            }
            ev.template mismatch<SIGMA>((double)u[j], m, ks, (uint64_t)j, 1);
        }
    }
    double v = ev.result();
    uint64_t arg = ev.arg, nonfinite = ev.nonfinite;
    block_reduce(v, arg, nonfinite);
    if (threadIdx.x == 0) {
        reinterpret_cast<double *>(ws + Ws::kPartVal)[0] = v;
        reinterpret_cast<uint64_t *>(ws + Ws::kPartIdx)[0] = arg;
        reinterpret_cast<uint64_t *>(ws + Ws::kPartCnt)[0] = nonfinite;
    }
}

// Reduce the W pass partials (max W, lowest index), or for the largest-r
// certificate the partials of -q (so r = -max, lowest index kept).
template <bool OPT>
__global__ __launch_bounds__(kBlock) void cert_w_final(unsigned char *__restrict__ ws, int nparts)
{
    double best = -INFINITY;
    uint64_t arg = 0, nonfinite = 0;
    merge_partials(ws, nparts, best, arg, nonfinite);
    block_reduce(best, arg, nonfinite);
    if (threadIdx.x == 0) {
        double *sc = reinterpret_cast<double *>(ws);
        uint64_t *su = reinterpret_cast<uint64_t *>(ws);
        if constexpr (OPT) {
            sc[Ws::kOptR / 8] = -best;
            su[Ws::kOptArg / 8] = arg;
            su[Ws::kOptNonfinite / 8] = nonfinite;
        } else {
            sc[Ws::kMaxW / 8] = best;
            su[Ws::kArgmax / 8] = arg;
            su[Ws::kNonfinite / 8] = nonfinite;
        }
    }
}

// Workgroups of a grid-stride pass over n work items: at most 16384 for FP32
// tables, 4096 for FP64 ones (measured on the largest-r pass: 16384 is 6%
// faster than 4096 at l = 16 FP32 and 8% at (2, 3, 10), but 7% slower at
// l = 14 FP64, where the extra partials cost more than they hide).
int reduce_blocks(uint64_t n, int dtype)
{
    const uint64_t cap = dtype == LCSB_F32 ? (uint64_t)kMaxReduceBlocks : 4096;
    uint64_t b = (n + kBlock - 1) / kBlock;
    return (int)(b < cap ? b : cap);
}

template <typename T, bool OPT>
hipError_t launch_w(const Geometry &g, const T *u, int swap_sym, unsigned char *ws, int nbw,
                    hipStream_t s)
{
    double lo = 0.0, hi = 0.0;
    inverse_bounds(3.0, &lo, &hi);
    if (g.h == 1 && g.sigma == 2 && g.d == 2)
        cert_w_l1<T, 2, 2, OPT><<<1, kBlock, 0, s>>>(u, ws, lo, hi);
    else if (g.h == 1 && g.sigma == 4 && g.d == 2)
        cert_w_l1<T, 4, 2, OPT><<<1, kBlock, 0, s>>>(u, ws, lo, hi);
    else if (g.h == 1 && g.sigma == 2 && g.d == 3)
        cert_w_l1<T, 2, 3, OPT><<<1, kBlock, 0, s>>>(u, ws, lo, hi);
    else if (g.h == 1)
        return hipErrorInvalidValue;
    else if (g.sigma == 2 && g.d == 2 && swap_sym)
        cert_w<2, 2, T, true, OPT><<<nbw, kBlock, 0, s>>>(u, g.n, g.h, ws, lo, hi);
    else if (g.sigma == 2 && g.d == 2)
        cert_w<2, 2, T, false, OPT><<<nbw, kBlock, 0, s>>>(u, g.n, g.h, ws, lo, hi);
    else if (g.sigma == 4 && g.d == 2 && swap_sym)
        cert_w<4, 2, T, true, OPT><<<nbw, kBlock, 0, s>>>(u, g.n, g.h, ws, lo, hi);
    else if (g.sigma == 4 && g.d == 2)
        cert_w<4, 2, T, false, OPT><<<nbw, kBlock, 0, s>>>(u, g.n, g.h, ws, lo, hi);
    else if (g.sigma == 2 && g.d == 3 && swap_sym)
        cert_w<2, 3, T, true, OPT><<<nbw, kBlock, 0, s>>>(u, g.n, g.h, ws, lo, hi);
    else if (g.sigma == 2 && g.d == 3)
        cert_w<2, 3, T, false, OPT><<<nbw, kBlock, 0, s>>>(u, g.n, g.h, ws, lo, hi);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T>
hipError_t certify_typed(const Geometry &g, const void *u, const void *prev, int u_slot,
                         int prev_slot, int swap_sym, unsigned char *ws, hipStream_t s)
{
    const int nb = reduce_blocks(g.ns, std::is_same<T, float>::value ? LCSB_F32 : LCSB_F64);
    const T *uu = static_cast<const T *>(u), *pp = static_cast<const T *>(prev);
    if (swap_sym && g.sigma == 2 && g.d == 2 && g.h >= 2)
        cert_r<T, 2><<<nb, kBlock, 0, s>>>(uu, pp, g.ns, ws);
    else if (swap_sym && g.sigma == 2 && g.d == 3 && g.h >= 2)
        cert_r<T, 3><<<nb, kBlock, 0, s>>>(uu, pp, g.ns, ws);
    else if (swap_sym && g.sigma == 4 && g.d == 2 && g.h >= 2)
        cert_r<T, 4><<<nb, kBlock, 0, s>>>(uu, pp, g.ns, ws);
    else
        cert_r<T, 0><<<nb, kBlock, 0, s>>>(uu, pp, g.ns, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    cert_r_final<<<1, kBlock, 0, s>>>(ws, nb, g.d, std::is_same<T, float>::value ? 1 : 0,
                                      u_slot, prev_slot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // one thread per x with string-1 symbol 0 at position 2 (one workgroup at l = 1)
    const int nbw = g.h == 1 ? 1 : reduce_blocks(g.n >> (g.slot + g.beta),
                                                 std::is_same<T, float>::value ? LCSB_F32 : LCSB_F64);
    if ((e = launch_w<T, false>(g, static_cast<const T *>(u), swap_sym, ws, nbw, s)) !=
        hipSuccess)
        return e;
    cert_w_final<false><<<1, kBlock, 0, s>>>(ws, nbw);
    return hipGetLastError();
}

// The largest-r certificate: one pass over u, then its final reduction.
template <typename T>
hipError_t certify_optimal_typed(const Geometry &g, const void *u, int swap_sym,
                                 unsigned char *ws, hipStream_t s)
{
    const int nbw = g.h == 1 ? 1 : reduce_blocks(g.n >> (g.slot + g.beta),
                                                 std::is_same<T, float>::value ? LCSB_F32 : LCSB_F64);
    hipError_t e;
    if ((e = launch_w<T, true>(g, static_cast<const T *>(u), swap_sym, ws, nbw, s)) !=
        hipSuccess)
        return e;
    cert_w_final<true><<<1, kBlock, 0, s>>>(ws, nbw);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_certify_optimal_packed(const Geometry &g, int dtype, const void *u,
                                         unsigned char *ws, hipStream_t s)
{
    if (g.sigma != 2 || g.d != 2 || g.h < 2) return hipErrorInvalidValue;
    const int nb = reduce_blocks(packed_entries(g.h), dtype);
    if (dtype == LCSB_F32)
        cert_opt_packed<float><<<nb, kBlock, 0, s>>>(static_cast<const float *>(u), g.h, ws);
    else
        cert_opt_packed<double><<<nb, kBlock, 0, s>>>(static_cast<const double *>(u), g.h, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    cert_w_final<true><<<1, kBlock, 0, s>>>(ws, nb);
    return hipGetLastError();
}

hipError_t launch_certify_optimal(const Geometry &g, int dtype, const void *u, int swap_sym,
                                  unsigned char *ws, hipStream_t s)
{
    return dtype == LCSB_F32 ? certify_optimal_typed<float>(g, u, swap_sym, ws, s)
                             : certify_optimal_typed<double>(g, u, swap_sym, ws, s);
}

namespace {

// The largest-r result of a finished pass into caller memory: out[0] = r,
// out[1] = d r rounded toward -inf, out[2] = the lowest minimising index and
// out[3] = the count of non-finite ratios (the two integers as the bit
// patterns of uint64).  One thread, after cert_w_final<true>.
__global__ void cert_opt_out(const unsigned char *__restrict__ ws, int d, double *__restrict__ out)
{
    const double r = reinterpret_cast<const double *>(ws)[Ws::kOptR / 8];
    out[0] = r;
    out[1] = mul_rd((double)d, r);
    reinterpret_cast<uint64_t *>(out)[2] = reinterpret_cast<const uint64_t *>(ws)[Ws::kOptArg / 8];
    reinterpret_cast<uint64_t *>(out)[3] =
        reinterpret_cast<const uint64_t *>(ws)[Ws::kOptNonfinite / 8];
}

}  // namespace

hipError_t launch_certify_optimal_out(const Geometry &g, int dtype, const void *u, int swap_sym,
                                      unsigned char *ws, double *out, hipStream_t s)
{
    hipError_t e = launch_certify_optimal(g, dtype, u, swap_sym, ws, s);
    if (e != hipSuccess) return e;
    cert_opt_out<<<1, 1, 0, s>>>(ws, g.d, out);
    return hipGetLastError();
}

hipError_t launch_certify(const Geometry &g, int dtype, const void *u, const void *prev,
                          int u_slot, int prev_slot, int swap_sym, unsigned char *ws,
                          hipStream_t s)
{
    return dtype == LCSB_F32
               ? certify_typed<float>(g, u, prev, u_slot, prev_slot, swap_sym, ws, s)
               : certify_typed<double>(g, u, prev, u_slot, prev_slot, swap_sym, ws, s);
}

}  // namespace lcsb
