// One sweep v_new = F(lag 1, .., lag d) of eq. (4) (Sec. 2.1), gfx950.
//
// Layout: index bits, most significant first, are the beta-bit symbols of
// position 1 (string 1 .. string d), then position 2, .. position l.  The
// top "slot" (d*beta bits) holds the heads; x below denotes the remaining
// (l-1) slots.  Advancing a set N of strings (Algorithm 1) shifts their
// symbol fields up one slot and appends the new symbols in the lowest slot,
// so every branch reads sigma^|N| entries of one aligned sigma^d group.
//
// Folded storage (Sec. 3.3): relabelling every symbol c -> c xor m leaves
// the table unchanged (the complement of eq. (10) for sigma = 2), so a table
// stores only the ns = n / sigma indices whose string-1 head is 0 -- the
// lowest ns indices -- and index i is read at its image i xor (m rep), m the
// string-1 head of i, rep the index with symbol 1 everywhere.  For l >= 2 the
// image of an aligned group is an aligned group whose members are permuted
// by the same xor (reversed, for sigma = 2).  Every branch sum is a balanced
// tree over its members in order, and a xor of the member indices only swaps
// the two operands of some of its additions, so a branch read through the
// image gives the same bits as on the unfolded table.
//
// Work split (l >= 2): one thread per x whose string-1 symbol at position 2
// is 0, which also computes the x' = x xor (m rep) of the other m (the
// complement of x for sigma = 2): the all-advance lag-d group of x' is the
// image of the one of x and is read once for both.  Per sweep each stored
// lag table is then read at most twice and the output written once.
//
// Arithmetic (bit-exact with the FP64 reference): each branch sums its
// sigma^k values with a balanced binary tree over the appended tuples in
// lexicographic order (first advanced string most significant); for sigma = 2
// the leaves are the tuples t starting with 0, each followed by its complement
// ~t (00, 11, 01, 10), so that complementing the symbols, and for two moved
// strings exchanging them, maps every pair to itself; for sigma = 4 and two
// moved strings they are the pairs {ab, ba} grouped by a xor b, then
// {aa, ~a~a} (tree16).  It multiplies by
// the exact power of two sigma^-k, takes the max over branches, and adds 1 to
// all-match tuples.  FP32 tables store values relative to a per-slot FP64
// offset: a branch reading lag k adds delta_k = offset(lag k) - offset(lag 1)
// and the result is shifted by the value y0 of entry 0 (all strings 0..0, an
// all-match tuple) so entry 0 of every new table is exactly 0.
#include <type_traits>

#include "internal.h"

namespace lcsb {
namespace {

template <typename T>
__device__ __forceinline__ T tree4(T a, T b, T c, T d) { return (a + b) + (c + d); }

// sigma = 2 groups, members in lexicographic order of the appended bits:
// complement-paired trees
template <typename T>
__device__ __forceinline__ T pair4(T m0, T m1, T m2, T m3) { return (m0 + m3) + (m1 + m2); }

template <typename T>
__device__ __forceinline__ T pair8(const T *g)
{
    return ((g[0] + g[7]) + (g[1] + g[6])) + ((g[2] + g[5]) + (g[3] + g[4]));
}

// sigma = 4 all-advance group (member 4 c1 + c2): pairs {ab, ba} grouped by
// a xor b, then {aa, ~a~a}, so that the exchange of the two strings and every
// relabelling c -> c xor m only swap operands
template <typename T>
__device__ __forceinline__ T tree16(const T *g)
{
    return (((g[1] + g[4]) + (g[11] + g[14])) + ((g[2] + g[8]) + (g[7] + g[13]))) +
           (((g[3] + g[12]) + (g[6] + g[9])) + ((g[0] + g[15]) + (g[5] + g[10])));
}

template <typename T>
__device__ __forceinline__ T vmax(T best, T cand) { return cand > best ? cand : best; }

// One thread per x: the grid is one-dimensional up to 2^32 threads and
// two-dimensional beyond (a dimension holds fewer than 2^32 work-items), rows
// of blockIdx.y following each other.
__device__ __forceinline__ uint64_t thread_index()
{
    return ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * kBlock + threadIdx.x;
}

// F takes the max over the branch means starting from -inf, so a NaN branch
// never wins and a tuple whose every branch is NaN gets -inf: the first value
// of every max chain goes through this (a no-op on every other value).
template <typename T>
__device__ __forceinline__ T first(T v) { return v > -(T)INFINITY ? v : -(T)INFINITY; }

// The new table is not read again until the next sweep, after 2-3 more
// tables have streamed through the caches: write it non-temporally.
template <typename T>
__device__ __forceinline__ void put(T *p, T v) { __builtin_nontemporal_store(v, p); }

// contiguous aligned stores, loads
template <typename T>
__device__ __forceinline__ void store4(T *p, const T *g)
{
    using V = T __attribute__((ext_vector_type(4)));
    V v;
    v.x = g[0];
    v.y = g[1];
    v.z = g[2];
    v.w = g[3];
    *reinterpret_cast<V *>(p) = v;
}
// contiguous aligned loads
__device__ __forceinline__ void load2(const double *p, double &a, double &b)
{
    double2 v = *reinterpret_cast<const double2 *>(p);
    a = v.x; b = v.y;
}
__device__ __forceinline__ void load2(const float *p, float &a, float &b)
{
    float2 v = *reinterpret_cast<const float2 *>(p);
    a = v.x; b = v.y;
}
__device__ __forceinline__ void load4(const double *p, double *g)
{
    double2 u = reinterpret_cast<const double2 *>(p)[0];
    double2 v = reinterpret_cast<const double2 *>(p)[1];
    g[0] = u.x; g[1] = u.y; g[2] = v.x; g[3] = v.y;
}
__device__ __forceinline__ void load4(const float *p, float *g)
{
    float4 v = *reinterpret_cast<const float4 *>(p);
    g[0] = v.x; g[1] = v.y; g[2] = v.z; g[3] = v.w;
}
template <typename T>
__device__ __forceinline__ void load8(const T *p, T *g)
{
    load4(p, g);
    load4(p + 4, g + 4);
}
// Non-temporal variants, for the sigma = d = 2 kernel, whose lag bytes are
// never read again from the caches (lag 2 once, lag 1 twice at far-apart
// times).  Measured on folded tables: non-temporal reads of both lags make
// the FP32 sweep 4.5% faster, of lag 2 only the FP64 sweep 1.4-5% faster
// (non-temporal lag-1 reads slow FP64 down).  The sigma = 4 kernel and the
// branch reads of the d = 3 kernel share groups between lanes through L2 and
// keep ordinary loads (non-temporal ones made sigma = 4 6-35% slower).
template <bool NT, typename T>
__device__ __forceinline__ void stream2(const T *p, T &a, T &b)
{
    if constexpr (NT) {
        a = __builtin_nontemporal_load(p);
        b = __builtin_nontemporal_load(p + 1);
    } else {
        load2(p, a, b);
    }
}
template <bool NT, typename T>
__device__ __forceinline__ void stream4(const T *p, T *g)
{
    if constexpr (NT) {
#pragma unroll
        for (int k = 0; k < 4; ++k) g[k] = __builtin_nontemporal_load(p + k);
    } else {
        load4(p, g);
    }
}

// an adjacent pair as one 8-byte (FP32) or 16-byte (FP64) access, p aligned
// to the pair's size
template <typename T>
using Pair2 = T __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ void pair_load(const T *p, T &a, T &b)
{
    const Pair2<T> v = __builtin_nontemporal_load(reinterpret_cast<const Pair2<T> *>(p));
    a = v.x;
    b = v.y;
}
template <typename T>
__device__ __forceinline__ void pair_put(T *p, T a, T b)
{
    Pair2<T> v;
    v.x = a;
    v.y = b;
    __builtin_nontemporal_store(v, reinterpret_cast<Pair2<T> *>(p));
}

constexpr uint64_t kAlt2 = 0xAAAAAAAAAAAAAAAAull;  // high bit of every 2-bit slot
constexpr uint64_t kAlt4Hi = 0xCCCCCCCCCCCCCCCCull; // high 2-bit field of every nibble

// ---------------------------------------------------------------- sigma = 2, d = 2
// Slot = (a bit, b bit); stored heads 0/0 (all-match) and 0/1.
//   0/0|x : 1 + mean(lag2[4x .. 4x+3])                         (eq. (2))
//   0/1|x : max( mean lag1[sb], lag1[sb+1]   (advance b, z = 0),
//                mean lag1[sa], lag1[sa+2] ) (advance a, z = 1) (Alg. 1)
// Thread t < n/8 computes x = t and its complement xc = n/4-1-t.  The lag-2
// group of xc is the image of the one of t, so 0/0|t and 0/0|xc share their
// value.  Advance b keeps a (head 0) and reads the stored half directly;
// advance a reads head a_2, 0 for t and 1 for xc, whose pair sa, sa+2 is then
// read in the image group n-4-(sa & ~3) at the other parity.
//
// SWAP (a ring symmetric under exchanging the two strings, bit for bit: the
// zero start, the network seed and every sweep of such a ring): with S the
// exchange of the a and b bits of every slot of x, 0/0|x and 0/0|Sx are
// exchanged tuples, and so are 0/1|x and 0/1|~Sx (exchange, then complement
// to bring the head back to 0/1).  The branch trees are exchange-invariant,
// so a thread's four values also belong at St, ~St (0/0) and ~St, St (0/1).
// Of the two threads t and p = St or ~St (whichever has a_2 = 0) only the
// lower one runs.  Tables are kept lazily (TwinGroup): the thread writes the
// lower index of each of its four exchanged pairs (t and ~St at 0/0, t and St
// at 0/1) and reads every group through its lower members, so a sweep reads
// half of the groups and writes half of the stored table.
template <typename T, bool SWAP, bool SHIFT>
__global__ __launch_bounds__(kBlock) void sweep_s2d2(const T *__restrict__ lag1,
                                                    const T *__restrict__ lag2,
                                                    T *__restrict__ out, uint64_t n,
                                                    double *__restrict__ off, int s1, int s2,
                                                    int snew)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    constexpr bool kShift = kF32 || SHIFT;  // lag 2 carries delta_2
    const uint64_t nq = n >> 2;
    const uint64_t t = thread_index();
    T d2 = 0, y0 = 0;
    if constexpr (!kF32 && SHIFT) d2 = off[s2] - off[s1];
    if constexpr (kF32) {
        const double o1 = off[s1];
        d2 = (float)(off[s2] - o1);
        T e[4];
        if constexpr (SWAP) {
            const TwinGroup tg = twin_group(0, n);
            T q[4] = {lag2[tg.read], lag2[tg.read + 1], lag2[tg.read + 2], lag2[tg.read + 3]};
            twin_values(q, tg.mode, e);
        } else {
            e[0] = lag2[0]; e[1] = lag2[1]; e[2] = lag2[2]; e[3] = lag2[3];
        }
        y0 = 1.0f + first(pair4(e[0], e[1], e[2], e[3]) * 0.25f + d2);
        if (t == 0) off[snew] = o1 + (double)y0;
    }
    if (t >= (n >> 3)) return;
    const uint64_t xc = nq - 1 - t;
    uint64_t st = 0;
    if constexpr (SWAP) {
        const uint64_t mq = nq - 1, am = kAlt2 & mq;
        st = ((t & am) >> 1) | ((t & ~am & mq) << 1);
        const uint64_t p = (t & (nq >> 2)) ? st ^ mq : st;  // b_2 = 1: ~St has a_2 = 0
        if (p < t) return;
    }

    T g[4];
    if constexpr (SWAP) {
        const TwinGroup tg = twin_group(4 * t, n);
        T q[4];
        stream4<true>(lag2 + tg.read, q);
        twin_values(q, tg.mode, g);
    } else {
        stream4<true>(lag2 + 4 * t, g);
    }
    T m2 = pair4(g[0], g[1], g[2], g[3]) * (T)0.25;
    if constexpr (kShift) m2 = m2 + d2;
    const T match = (T)1 + first(m2);

    const uint64_t am = kAlt2 & (n - 1), bm = ~kAlt2 & (n - 1);
    T mis[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const uint64_t i = nq + (c ? xc : t);
        const uint64_t sb = (i & am) | ((i << 2) & bm);
        const uint64_t sa = ((i << 2) & am) | (i & bm);
        T b0, b1;
        if constexpr (SWAP) {
            // the advance-b pair is the low or high half of its group
            const TwinGroup tg = twin_group(sb & ~(uint64_t)3, n);
            T q[4], e[4];
            stream4<kF32>(lag1 + tg.read, q);
            twin_values(q, tg.mode, e);
            const bool hi = (sb & 2) != 0;
            b0 = hi ? e[2] : e[0];
            b1 = hi ? e[3] : e[1];
        } else {
            stream2<kF32>(lag1 + sb, b0, b1);
        }
        const T mb = (b0 + b1) * (T)0.5;
        // the advance-a pair is the even or odd half of an aligned group that
        // the neighbouring thread (t ^ 1) also reads: one vector load serves both
        T q[4];
        const uint64_t grp = sa & ~(uint64_t)3, gbase = c ? (n - 4) - grp : grp;
        if constexpr (SWAP) {
            const TwinGroup tg = twin_group(gbase, n);
            T r[4];
            stream4<kF32>(lag1 + tg.read, r);
            twin_values(r, tg.mode, q);
        } else {
            stream4<kF32>(lag1 + gbase, q);
        }
        const bool odd = ((sa & 1) ^ (uint64_t)c) != 0;
        const T ma = ((odd ? q[1] : q[0]) + (odd ? q[3] : q[2])) * (T)0.5;
        mis[c] = vmax(first(mb), ma);
    }

    const T vm = kF32 ? (T)(match - y0) : match;
    const T v0 = kF32 ? (T)(mis[0] - y0) : mis[0];
    const T v1 = kF32 ? (T)(mis[1] - y0) : mis[1];
    if constexpr (SWAP) {  // the lower index of each exchanged pair
        put(out + t, vm);
        put(out + (nq - 1 - st), vm);
        put(out + nq + t, v0);
        put(out + nq + st, v1);
    } else {
        put(out + t, vm);
        put(out + xc, vm);
        put(out + nq + t, v0);
        put(out + nq + xc, v1);
    }
}

// ---------------------------------------------------------------- sigma = d = 2 from branch means
// The values of sweep_s2d2<T, true, SHIFT> (rings symmetric in the two
// strings) from the branch-mean tables of the lags (ma_index, mab_index)
// instead of their entries: an all-match tuple reads one all-advance mean of
// lag 2, a mismatched one an advance-a and an advance-b mean of lag 1 (the
// latter at the exchanged tuple).  Every mean is the one the entry-reading
// kernel forms, so the values agree bit for bit, and a branch reads one
// value instead of two or four.  The kernel writes the new table's means, and
// its entries when `out` is given.
//
// Thread j < n/32 owns the tails t = 4j + v, v = (a_l, b_l) = 0..3 (a_2 = 0),
// and computes 0/0|t and 0/0|~t (one value: an all-match tuple drops both
// heads), 0/1|t and 0/1|~t: every member of the four aligned groups with
// prefixes j and ~j at heads 0/0 and 0/1, so each group mean it writes comes
// from its own registers.  The exchanged quad p (Sj, or ~Sj when b_2 = 1)
// computes the same values; only the lower of j and p runs (p = j: the quad
// is its own twin), and it also writes the means of p's groups: their
// advance-a means are its own groups' advance-b means, their all-advance means
// its own (Mab only at the lower prefix of each exchanged pair of groups:
// the readers are lower quads).  Within a thread the four advance-a means of one head lie at
// offsets {0, 1, 4, 5} from the v = 0 one, the four advance-b means at
// {0, 4, 1, 5}, descending when b_2 = 1: two loads of adjacent pairs each.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(kBlock) void sweep_s2d2_means(const T *__restrict__ ma1,
                                                          const T *__restrict__ mab2,
                                                          T *__restrict__ out,
                                                          T *__restrict__ ma_new,
                                                          T *__restrict__ mab_new, uint64_t n,
                                                          double *__restrict__ off, int s1,
                                                          int s2, int snew)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    constexpr bool kShift = kF32 || SHIFT;  // lag 2 carries delta_2
    const uint64_t nq = n >> 2, n16 = n >> 4;
    const uint64_t j = thread_index();
    T d2 = 0, y0 = 0;
    if constexpr (!kF32 && SHIFT) d2 = off[s2] - off[s1];
    if constexpr (kF32) {
        const double o1 = off[s1];
        d2 = (float)(off[s2] - o1);
        y0 = 1.0f + first(mab2[0] + d2);
        if (j == 0) off[snew] = o1 + (double)y0;
    }
    if (j >= (n >> 5)) return;
    const uint64_t mq = n16 - 1, qa = kAlt2 & mq;
    const uint64_t sj = ((j & qa) >> 1) | ((j & ~qa & mq) << 1);
    const bool b2 = (j & (n16 >> 2)) != 0;
    const uint64_t pj = b2 ? sj ^ mq : sj;
    if (pj < j) return;

    // all-match: the lag-2 all-advance means of t = 4j .. 4j + 3.  Mab holds
    // the lower prefix of each exchanged pair (the twin of 4j + v is
    // 4p + perm(v)); in a quad that is its own twin the upper members are
    // taken from their partners in the same load.
    T g[4];
    stream4<true>(mab2 + 4 * j, g);
    if (pj == j) {
#pragma unroll
        for (int v = 1; v < 4; ++v) {
            const int sv = ((v & 1) << 1) | (v >> 1), pv = b2 ? 3 - sv : sv;
            if (pv < v) g[v] = g[pv];
        }
    }
    T a[4], b[4], c[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        T m2 = g[v];
        if constexpr (kShift) m2 = m2 + d2;
        a[v] = (T)1 + first(m2);
    }
    // mismatched: 0/1|t (cc = 0) and 0/1|~t (cc = 1)
    const uint64_t am = kAlt2 & (n - 1), bm = ~kAlt2 & (n - 1);
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
        const uint64_t i0 = nq + (cc ? nq - 1 - 4 * j : 4 * j);  // the v = 0 tuple
        const uint64_t sa0 = ((i0 << 2) & am) | (i0 & bm);
        const uint64_t sb0 = (i0 & am) | ((i0 << 2) & bm);
        const uint64_t ia = ma_index(sa0, n);
        const uint64_t ib = ma_index(exchange_twin(sb0, n, 2), n);
        T ma[4], mb[4], p0, p1, q0, q1;
        pair_load(ma1 + ia, p0, p1);
        pair_load(ma1 + ia + 4, q0, q1);
        ma[0] = p0; ma[1] = p1; ma[2] = q0; ma[3] = q1;
        // descending where the exchange complements symbols of t itself:
        // the exchanged tuple of 0/1|t has string-1 head b_2 (complemented
        // when 1); that of 0/1|~t has ~b_2 and its symbols are already
        // complemented (uncomplemented when ~b_2 = 1)
        const bool desc = b2;
        pair_load(ma1 + (desc ? ib - 5 : ib), p0, p1);
        pair_load(ma1 + (desc ? ib - 1 : ib + 4), q0, q1);
        mb[0] = desc ? q1 : p0;
        mb[1] = desc ? p1 : q0;
        mb[2] = desc ? q0 : p1;
        mb[3] = desc ? p0 : q1;
#pragma unroll
        for (int v = 0; v < 4; ++v) (cc ? c : b)[v] = vmax(first(mb[v]), ma[v]);
    }
    if constexpr (kF32) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            a[v] = (T)(a[v] - y0);
            b[v] = (T)(b[v] - y0);
            c[v] = (T)(c[v] - y0);
        }
    }

    if (out) {  // entries at the lower index of each exchanged pair, as sweep_s2d2
        // 0/0|t at t; 0/0|~t at ~St = 4(~Sj) + 3 - S(v); 0/1|t at t; 0/1|~t at St = 4Sj + S(v)
        put(out + 4 * j, a[0]); put(out + 4 * j + 1, a[1]);
        put(out + 4 * j + 2, a[2]); put(out + 4 * j + 3, a[3]);
        const uint64_t nsj = 4 * (mq - sj);
        put(out + nsj, a[3]); put(out + nsj + 1, a[1]);
        put(out + nsj + 2, a[2]); put(out + nsj + 3, a[0]);
        put(out + nq + 4 * j, b[0]); put(out + nq + 4 * j + 1, b[1]);
        put(out + nq + 4 * j + 2, b[2]); put(out + nq + 4 * j + 3, b[3]);
        const uint64_t psj = nq + 4 * sj;
        put(out + psj, c[0]); put(out + psj + 1, c[2]);
        put(out + psj + 2, c[1]); put(out + psj + 3, c[3]);
    }

    // the four groups: prefixes j and ~j (= mq - j) at heads 0/0 and 0/1,
    // members in order v; the ~j groups hold the ~t values reversed
    const T half = (T)0.5, quarter = (T)0.25;
    const T mall0 = pair4(a[0], a[1], a[2], a[3]) * quarter;  // both 0/0 groups
    const T mall1 = pair4(b[0], b[1], b[2], b[3]) * quarter;
    const T mall2 = pair4(c[0], c[1], c[2], c[3]) * quarter;
    const uint64_t P[4] = {j, mq - j, n16 + j, n16 + mq - j};
    const T m[4][4] = {{a[0], a[1], a[2], a[3]},
                       {a[3], a[2], a[1], a[0]},
                       {b[0], b[1], b[2], b[3]},
                       {c[3], c[2], c[1], c[0]}};
    const T mall[4] = {mall0, mall0, mall1, mall2};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint64_t g4 = 4 * P[k];
        pair_put(ma_new + 2 * P[k], (m[k][0] + m[k][2]) * half, (m[k][1] + m[k][3]) * half);
        // Mab at the lower prefix of the group and its exchanged twin (half
        // of these stores scatter: ordinary FP64 stores, which the L2 merges,
        // are 4-10% faster; non-temporal ones stay faster in FP32)
        const uint64_t tw = mab_index(exchange_twin(g4, n, 2), n);
        if constexpr (kF32) put(mab_new + (tw < P[k] ? tw : P[k]), mall[k]);
        else mab_new[tw < P[k] ? tw : P[k]] = mall[k];
        if (pj != j) {
            // the exchanged quad's group: its advance-a means are this group's
            // advance-b means over b_l for a_l = 0 and 1, one adjacent pair,
            // reversed where the exchange complements
            const uint64_t x0 = ma_index(exchange_twin(g4, n, 2), n);
            const T mb0 = (m[k][0] + m[k][1]) * half, mb1 = (m[k][2] + m[k][3]) * half;
            if (x0 & 1) pair_put(ma_new + (x0 - 1), mb1, mb0);
            else pair_put(ma_new + x0, mb0, mb1);
        }
    }
}

// The new table's values at the two-array rate's sample coordinates (each
// at the lower index of its exchanged pair, where the sweep stores it), in
// sample order: what sweep_s2d2_means computes there, from the same means
// with the same operations (the sweep writes these entries only on the last
// sweeps of a call; the rate pass reads them from here instead).
template <typename T, bool SHIFT>
__global__ __launch_bounds__(kBlock) void means_samples(const T *__restrict__ ma1,
                                                       const T *__restrict__ mab2,
                                                       T *__restrict__ smp, uint64_t n,
                                                       const double *__restrict__ off, int s1,
                                                       int s2)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    constexpr bool kShift = kF32 || SHIFT;
    T d2 = 0, y0 = 0;
    if constexpr (!kF32 && SHIFT) d2 = off[s2] - off[s1];
    if constexpr (kF32) {
        d2 = (float)(off[s2] - off[s1]);
        y0 = 1.0f + first(mab2[0] + d2);
    }
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (uint64_t)kRateSample) return;
    const uint64_t nq = n >> 2;
    uint64_t c = (i * kRateSampleMul) & ((n >> 1) - 1);
    const uint64_t tw = exchange_twin(c, n, 2);
    c = tw < c ? tw : c;
    T v;
    if (!(c & nq)) {  // 0/0|x: the all-advance mean of x's group, at its kept prefix
        const uint64_t P = mab_index(4 * c, n);
        const uint64_t pt = mab_index(exchange_twin(4 * P, n, 2), n);
        T m2 = mab2[pt < P ? pt : P];
        if constexpr (kShift) m2 = m2 + d2;
        v = (T)1 + first(m2);
    } else {          // 0/1|x: advance b, then advance a
        const uint64_t am = kAlt2 & (n - 1), bm = ~kAlt2 & (n - 1);
        const uint64_t sa = ((c << 2) & am) | (c & bm), sb = (c & am) | ((c << 2) & bm);
        v = vmax(first(ma1[ma_index(exchange_twin(sb, n, 2), n)]), ma1[ma_index(sa, n)]);
    }
    smp[i] = kF32 ? (T)(v - y0) : v;
}

// Ma and Mab of a stored table, one thread per group prefix P < n/8
template <typename T>
__global__ __launch_bounds__(kBlock) void derive_means(const T *__restrict__ tab, int lazy,
                                                      T *__restrict__ ma, T *__restrict__ mab,
                                                      uint64_t n)
{
    const uint64_t P = thread_index();
    if (P >= (n >> 3)) return;
    T e[4];
    if (lazy) {
        const TwinGroup tg = twin_group(4 * P, n);
        T q[4];
        load4(tab + tg.read, q);
        twin_values(q, tg.mode, e);
    } else {
        load4(tab + 4 * P, e);
    }
    ma[2 * P] = (e[0] + e[2]) * (T)0.5;
    ma[2 * P + 1] = (e[1] + e[3]) * (T)0.5;
    mab[P] = pair4(e[0], e[1], e[2], e[3]) * (T)0.25;
}

// ---------------------------------------------------------------- sigma = 4, d = 2
// Slot = (a: 2 bits, b: 2 bits); stored heads (0, b1), b1 = 0..3.
// Branches of (0, b1), b1 != 0: z = 0 advances b (lag 1), z = b1 advances a
// (lag 1), the two other z advance both (lag 2, the same group as the
// all-match tuple).  Thread t < n/64 owns x = t (string-1 symbol 0 at
// position 2) and its images x_m = x xor (m rep), m = 0..3:
//   - advance both: the lag-2 group of x_m is the image of the one of x;
//   - advance b keeps string 1 (head 0): stored directly;
//   - advance a of (0, b1)|x_m reads string-1 head m; its image is the
//     advance-a group of (0, b1 xor m)|x, so four means ma[v] serve all
//     twelve mismatched tuples.
//
// SWAP (a ring symmetric in the two strings, bit for bit): exchanging the
// strings and relabelling by the new string-1 head maps (0, b1)|x_m to
// (0, b1)|p_(m xor b1 xor s), p = exchange4(t) relabelled by s, the string-2
// symbol of t at position 2.  Threads t and p compute the same sixteen
// values, so only the lower runs; it stores each value at the lower index of
// its exchanged pair and reads every group through its lower members
// (Twin16): the all-advance tree is invariant under the twin's member
// permutation, so an own or twin group is summed as loaded.  Where the four
// members a branch needs are contiguous (advance b in an own group, advance a
// in a twin group, one row of it) they are one vector load (6.8% faster in
// FP32, 11.6% in FP64 than a load per member).
template <typename T, bool SWAP, bool SHIFT>
__global__ __launch_bounds__(kBlock) void sweep_s4d2(const T *__restrict__ lag1,
                                                    const T *__restrict__ lag2,
                                                    T *__restrict__ out, uint64_t n, int h,
                                                    double *__restrict__ off, int s1, int s2,
                                                    int snew)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    constexpr bool kShift = kF32 || SHIFT;  // lag 2 carries delta_2
    const uint64_t t = thread_index();
    const int top = 4 * (h - 1);
    T d2 = 0, y0 = 0;
    if constexpr (!kF32 && SHIFT) d2 = off[s2] - off[s1];
    if constexpr (kF32) {
        const double o1 = off[s1];
        d2 = (float)(off[s2] - o1);
        T g0[16];
        if constexpr (SWAP) {
            const Twin16 tw = twin_group16(0, n);  // its own twin: read the lower members
#pragma unroll
            for (int v = 0; v < 16; ++v) g0[v] = lag2[member16(0, tw, v)];
        } else {
            for (int k = 0; k < 16; k += 4) load4(lag2 + k, g0 + k);
        }
        y0 = 1.0f + first(tree16(g0) * 0.0625f + d2);
        if (t == 0) off[snew] = o1 + (double)y0;
    }
    if (t >= (n >> 6)) return;
    const uint64_t rep = ((n >> 4) - 1) / 3;  // symbol 1 at every position of x
    uint64_t p = t;
    int sx = 0;
    if constexpr (SWAP) {
        sx = (int)((t >> (top - 4)) & 3);
        p = exchange4(t, n >> 4) ^ ((uint64_t)sx * rep);
        if (p < t) return;
    }

    T g[16];
    if constexpr (SWAP) {
        const Twin16 tw = twin_group16(16 * t, n);
        if (tw.kind == 2) {
#pragma unroll
            for (int v = 0; v < 16; ++v) g[v] = lag2[member16(16 * t, tw, v)];
        } else {
#pragma unroll
            for (int k = 0; k < 16; k += 4) load4(lag2 + tw.read + k, g + k);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 16; k += 4) load4(lag2 + 16 * t + k, g + k);
    }
    T both = tree16(g) * (T)0.0625;
    if constexpr (kShift) both = both + d2;
    const T match = (T)1 + first(both);

    const uint64_t am = kAlt4Hi & (n - 1), bm = ~kAlt4Hi & (n - 1);
    T ma[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const uint64_t i = ((uint64_t)v << top) | t;
        const uint64_t sa = ((i << 4) & am) | (i & bm);
        if constexpr (SWAP) {
            const uint64_t gb = sa & ~(uint64_t)15;
            const int o = (int)(sa & 15);  // < 4: members o + 4k
            const Twin16 tw = twin_group16(gb, n);
            T q[4];
            if (tw.kind == 1) {  // member o + 4k at 4 (o ^ m) + (k ^ m) of the twin: one row
                T r[4];
                load4(lag1 + tw.read + 4 * (o ^ tw.m), r);
#pragma unroll
                for (int k = 0; k < 4; ++k) asm volatile("" : "+v"(r[k]));
                const bool s1 = tw.m & 1, s2 = tw.m & 2;
                const T a0 = s1 ? r[1] : r[0], a1 = s1 ? r[0] : r[1];
                const T a2 = s1 ? r[3] : r[2], a3 = s1 ? r[2] : r[3];
                q[0] = s2 ? a2 : a0;
                q[1] = s2 ? a3 : a1;
                q[2] = s2 ? a0 : a2;
                q[3] = s2 ? a1 : a3;
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) q[k] = lag1[member16(gb, tw, o + 4 * k)];
            }
            ma[v] = tree4(q[0], q[1], q[2], q[3]) * (T)0.25;
        } else {
            ma[v] = tree4(lag1[sa], lag1[sa + 4], lag1[sa + 8], lag1[sa + 12]) * (T)0.25;
        }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const uint64_t x = t ^ ((uint64_t)m * rep);
        const uint64_t sb = (x & am) | ((x << 4) & bm);
        T bv[4];
        if constexpr (SWAP) {
            const uint64_t gb = sb & ~(uint64_t)15;
            const int o = (int)(sb & 15);
            const Twin16 tw = twin_group16(gb, n);
            if (tw.kind == 0) {  // own group: members o .. o + 3 in place
                load4(lag1 + sb, bv);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) bv[k] = lag1[member16(gb, tw, o + k)];
            }
        } else {
            load4(lag1 + sb, bv);
        }
        const T mb = tree4(bv[0], bv[1], bv[2], bv[3]) * (T)0.25;
        // the lower index of each output's exchanged pair (b1 << top) | p_(m ^ b1 ^ s).
        // A wave's stores at its twin's side fill 64-byte halves of lines
        // whose other halves the neighbouring wave writes: in FP32 they are
        // ordinary stores, which the L2 merges (WRITE_SIZE 2.33 -> 2.18 GB at
        // l = 8, the same time); FP64 keeps non-temporal ones (3% faster).
        auto st = [&](int b1, T v) {
            const uint64_t xt = p ^ ((uint64_t)(m ^ b1 ^ sx) * rep);
            if (SWAP && xt < x) {
                if constexpr (kF32) out[((uint64_t)b1 << top) | xt] = v;
                else put(out + (((uint64_t)b1 << top) | xt), v);
            } else {
                put(out + (((uint64_t)b1 << top) | x), v);
            }
        };
        st(0, kF32 ? (T)(match - y0) : match);
#pragma unroll
        for (int b1 = 1; b1 < 4; ++b1) {
            T best = first(mb);                              // z = 0
#pragma unroll
            for (int z = 1; z < 4; ++z) best = vmax(best, z == b1 ? ma[b1 ^ m] : both);
            st(b1, kF32 ? (T)(best - y0) : best);
        }
    }
}

// ---------------------------------------------------------------- sigma = 4, d = 2 from branch means
// The values of sweep_s4d2<T, true, SHIFT> from the lags' branch means
// (m4a_index, m4ab_index): the thread's four advance-a means of lag 1 (M4a),
// its four advance-b means (M4a at the exchanged tuples) and its all-advance
// mean of lag 2 (M4ab at the lower prefix of its exchanged pair) instead of
// 16 + 16 + 16 entries; each mean is the entry sweep's own (tree4 over the
// appended symbol, which relabelling and exchange only permute by xor; the
// sixteen-member tree, invariant under the twin permutations).
//
// The sixteen threads of a hexadecet (t = 16J + w) hold every member of
// sixteen aligned groups (heads (0, b1), images m: member u = w xor 5m); a
// pass through LDS gives each lane one whole group, whose four advance-a
// means, four advance-a means of the exchanged group (this one's advance-b
// means) and sixteen-member tree it forms in registers.  Hexadecets are
// exchange-folded whole: the lower of a hexadecet and its exchanged one runs.
template <typename I>
struct S4Idx {
    I mask, rep, A, B;
    int hs;  // the string-1 head's shift
    __device__ S4Idx(uint64_t n, int h)
        : mask((I)(n - 1)), rep((I)((n - 1) / 3)), A((I)(kAlt4Hi & (n - 1))),
          B((I)(~kAlt4Hi & (n - 1))), hs(4 * h - 2)
    {
    }
    __device__ __forceinline__ I fold(I s) const { return s ^ (((s >> hs) & 3) * rep); }
    __device__ __forceinline__ I exch(I x) const { return ((x & A) >> 2) | ((x & B) << 2); }
    __device__ __forceinline__ I twin(I j) const { return fold(exch(j)); }
    __device__ __forceinline__ I ma(I s) const { s = fold(s); return ((s >> 4) << 2) | (s & 3); }
    __device__ __forceinline__ I mab(I s) const { return fold(s) >> 4; }
};

template <typename T, bool SHIFT, typename I>
__global__ __launch_bounds__(kBlock) void sweep_s4d2_means(const T *__restrict__ ma1,
                                                          const T *__restrict__ mab2,
                                                          T *__restrict__ out,
                                                          T *__restrict__ na,
                                                          T *__restrict__ nab, uint64_t n, int h,
                                                          double *__restrict__ off, int s1,
                                                          int s2, int snew)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    constexpr bool kShift = kF32 || SHIFT;
    const uint64_t t64 = thread_index();
    const int top = 4 * (h - 1);
    T d2 = 0, y0 = 0;
    if constexpr (!kF32 && SHIFT) d2 = off[s2] - off[s1];
    if constexpr (kF32) {
        const double o1 = off[s1];
        d2 = (float)(off[s2] - o1);
        y0 = 1.0f + first(mab2[0] + d2);
        if (t64 == 0) off[snew] = o1 + (double)y0;
    }
    constexpr int kStride = 17, kHex = 16 * kStride;
    __shared__ T lds[(kBlock / 16) * kHex];
    if (t64 >= (n >> 6)) return;
    const S4Idx<I> ix(n, h);
    const I t = (I)t64, rep = (I)(((n >> 4) - 1) / 3), repJ = (I)(((n >> 8) - 1) / 3);
    const I J = t >> 4;
    const int w = (int)(t & 15);
    const I sx = (t >> (top - 4)) & 3;  // string-2 symbol at position 2 (string 1's is 0)
    const I pJ = (ix.exch(t & ~(I)15) ^ (sx * rep)) >> 4;
    if (pJ < J) return;
    const bool self = pJ == J;

    // reads: the all-advance mean of t's group, the advance-a means of
    // (0, v)|t, the advance-b means of the images
    T both;
    {
        const I tw = ix.mab(ix.twin(16 * t));
        both = mab2[tw < t ? tw : t];
        if constexpr (kShift) both = both + d2;
    }
    const T match = (T)1 + first(both);
    T ma[4], mb[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const I i = ((I)v << top) | t, sa = ((i << 4) & ix.A) | (i & ix.B);
        ma[v] = ma1[ix.ma(sa)];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const I x = t ^ ((I)m * rep), sb = (x & ix.A) | ((x << 4) & ix.B);
        mb[m] = ma1[ix.ma(ix.twin(sb))];
    }
    T val[4][4];  // [m][b1]
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        val[m][0] = match;
#pragma unroll
        for (int b1 = 1; b1 < 4; ++b1) {
            T best = first(mb[m]);  // z = 0
#pragma unroll
            for (int z = 1; z < 4; ++z) best = vmax(best, z == b1 ? ma[b1 ^ m] : both);
            val[m][b1] = best;
        }
    }
    if constexpr (kF32) {
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int b1 = 0; b1 < 4; ++b1) val[m][b1] = (T)(val[m][b1] - y0);
    }
    if (out) {  // entries at the lower index of each exchanged pair, as sweep_s4d2
        const I p = ix.exch(t) ^ (sx * rep);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const I x = t ^ ((I)m * rep);
#pragma unroll
            for (int b1 = 0; b1 < 4; ++b1) {
                const I xt = p ^ (((I)m ^ (I)b1 ^ sx) * rep);
                put(out + (((I)b1 << top) | (xt < x ? xt : x)), val[m][b1]);
            }
        }
    }

    // means: the hexadecet's sixteen groups (b1, m), prefix P = (0, b1)|(J xor
    // m rep), lane w holding member u = w xor 5m of each, pass through LDS
    // (members padded to 17 values: the writes of one group and the reads of
    // one member across the groups fall in distinct banks) so that lane w
    // holds every member of group (w >> 2, w & 3); the hexadecet lies in one
    // wave, which orders its own LDS accesses
    T *hx = lds + (threadIdx.x >> 4) * kHex;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int b1 = 0; b1 < 4; ++b1) hx[(4 * b1 + m) * kStride + (w ^ (5 * m))] = val[m][b1];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    T e[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) e[u] = hx[w * kStride + u];
    const int gm = w & 3;
    const I P = ((I)(w >> 2) << (top - 4)) | (J ^ ((I)gm * repJ));
    const T quarter = (T)0.25;
    T own[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) own[b] = tree4(e[b], e[4 + b], e[8 + b], e[12 + b]) * quarter;
    store4(na + 4 * P, own);
    const I tw = ix.twin(16 * P);  // member 0 of the exchanged group
    {
        const I at = ix.mab(tw);
        nab[at < P ? at : P] = tree16(e) * (T)0.0625;
    }
    if (!self) {
        // the exchanged group's advance-a means: member 4 c1 + c2 sits there
        // at a = c2 xor m', b = c1 xor m' (m' its relabelling), so its mean
        // for b is this group's mean over c2 at c1 = b xor m'
        const I at = ix.ma(tw);
        const int r = (int)(at & 3);
        T q[4];
#pragma unroll
        for (int c1 = 0; c1 < 4; ++c1)
            q[c1] = tree4(e[4 * c1], e[4 * c1 + 1], e[4 * c1 + 2], e[4 * c1 + 3]) * quarter;
        const bool r1 = r & 1, r2 = r & 2;
        const T a0 = r1 ? q[1] : q[0], a1 = r1 ? q[0] : q[1];
        const T a2 = r1 ? q[3] : q[2], a3 = r1 ? q[2] : q[3];
        T tv[4] = {r2 ? a2 : a0, r2 ? a3 : a1, r2 ? a0 : a2, r2 ? a1 : a3};
        store4(na + (at & ~(I)3), tv);
    }
}

// M4a and M4ab of a stored table, one thread per group prefix P < n/64
template <typename T>
__global__ __launch_bounds__(kBlock) void derive_means4(const T *__restrict__ tab, int lazy,
                                                       T *__restrict__ ma, T *__restrict__ mab,
                                                       uint64_t n)
{
    const uint64_t P = thread_index();
    if (P >= (n >> 6)) return;
    T e[16];
    if (lazy) {
        const Twin16 tw = twin_group16(16 * P, n);
#pragma unroll
        for (int v = 0; v < 16; ++v) e[v] = tab[member16(16 * P, tw, v)];
    } else {
#pragma unroll
        for (int k = 0; k < 16; k += 4) load4(tab + 16 * P + k, e + k);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) ma[4 * P + b] = tree4(e[b], e[4 + b], e[8 + b], e[12 + b]) * (T)0.25;
    mab[P] = tree16(e) * (T)0.0625;
}

// The new table's values at the two-array rate's sample coordinates (each at
// the lower index of its exchanged pair), in sample order: what
// sweep_s4d2_means computes for that tuple (the thread owning tail x is
// t = x with string 1's symbol at position 2 relabelled to 0, x its image m),
// from the same means with the same operations.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(kBlock) void means_samples4(const T *__restrict__ ma1,
                                                        const T *__restrict__ mab2,
                                                        T *__restrict__ smp, uint64_t n, int h,
                                                        const double *__restrict__ off, int s1,
                                                        int s2)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    constexpr bool kShift = kF32 || SHIFT;
    T d2 = 0, y0 = 0;
    if constexpr (!kF32 && SHIFT) d2 = off[s2] - off[s1];
    if constexpr (kF32) {
        d2 = (float)(off[s2] - off[s1]);
        y0 = 1.0f + first(mab2[0] + d2);
    }
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (uint64_t)kRateSample) return;
    const int top = 4 * (h - 1);
    uint64_t c = (i * kRateSampleMul) & ((n >> 2) - 1);
    const uint64_t tw = exchange_twin4(c, n);
    c = tw < c ? tw : c;
    const int b1 = (int)((c >> top) & 3);
    const uint64_t x = c & ((1ull << top) - 1), rep = ((n >> 4) - 1) / 3;
    const int m = (int)((x >> (top - 2)) & 3);
    const uint64_t t = x ^ ((uint64_t)m * rep);
    T both;
    {
        const uint64_t at = m4ab_index(exchange_twin4(16 * t, n), n);
        both = mab2[at < t ? at : t];
        if constexpr (kShift) both = both + d2;
    }
    T v;
    if (b1 == 0) {
        v = (T)1 + first(both);
    } else {
        const uint64_t am = kAlt4Hi & (n - 1), bm = ~kAlt4Hi & (n - 1);
        const uint64_t sb = (x & am) | ((x << 4) & bm);
        const T mb = ma1[m4a_index(exchange_twin4(sb, n), n)];
        const uint64_t iv = ((uint64_t)(b1 ^ m) << top) | t, sa = ((iv << 4) & am) | (iv & bm);
        const T ma = ma1[m4a_index(sa, n)];
        T best = first(mb);  // z = 0
#pragma unroll
        for (int z = 1; z < 4; ++z) best = vmax(best, z == b1 ? ma : both);
        v = best;
    }
    smp[i] = kF32 ? (T)(v - y0) : v;
}

// ---------------------------------------------------------------- sigma = 2, d = 3
// Slot = (s1, s2, s3) bits; stored heads 000 (all-match), 001, 010, 011.
// Each mismatched tuple has one branch moving the single string whose head
// differs (lag 1) and one moving the other two (lag 2):  001: z=0 -> {3},
// z=1 -> {1,2};  010: z=0 -> {2}, z=1 -> {1,3};  011: z=0 -> {2,3},
// z=1 -> {1}.  Thread t < n/16 computes x = t and its complement xc; a
// branch that moves string 1 reads head s1_2, which is 1 for xc, and then
// reads the image group, whose members are the reversed originals.
//
// SWAP (a ring symmetric in strings 1 and 2, bit for bit): with E the
// exchange of the s1 and s2 bits of every slot of x, 000|x and 001|x are
// exchanged with 000|Ex and 001|Ex, and 010|x with 011|~Ex (the exchange,
// then the complement that brings string 1's head back to 0).  Thread t and
// the thread p of its twin (Et when s2_2 = 0, ~Et otherwise) compute the same
// eight values, so only the lower runs; it stores each value at the lower
// index of its exchanged pair (exchange_twin), reads the all-advance group
// through its lower members (TwinGroup, eight members) and every branch value
// at the lower index of its pair (one load each: measured 1.2-1.4x faster
// than loading twin groups and permuting them), so a sweep reads half of the
// groups and writes half of the table.
template <typename T, bool SWAP, bool SHIFT>
__global__ __launch_bounds__(kBlock) void sweep_s2d3(const T *__restrict__ lag1,
                                                    const T *__restrict__ lag2,
                                                    const T *__restrict__ lag3,
                                                    T *__restrict__ out, uint64_t n, int h,
                                                    double *__restrict__ off, int s1, int s2,
                                                    int s3, int snew)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    constexpr bool kShift = kF32 || SHIFT;  // lags 2 and 3 carry delta_2, delta_3
    const uint64_t t = thread_index();
    const int top = 3 * (h - 1);
    T d2 = 0, d3 = 0, y0 = 0;
    if constexpr (!kF32 && SHIFT) {
        d2 = off[s2] - off[s1];
        d3 = off[s3] - off[s1];
    }
    if constexpr (kF32) {
        const double o1 = off[s1];
        d2 = (float)(off[s2] - o1);
        d3 = (float)(off[s3] - o1);
        T g0[8];
        if constexpr (SWAP) {
            const TwinGroup tg = twin_group8(0, n);
            T q[8];
            load8(lag3 + tg.read, q);
            twin_values8(q, tg.mode, g0);
        } else {
            load8(lag3, g0);
        }
        y0 = 1.0f + first(pair8(g0) * 0.125f + d3);
        if (t == 0) off[snew] = o1 + (double)y0;
    }
    if (t >= (n >> 4)) return;
    const uint64_t mx = (n >> 3) - 1, xc = mx - t;
    if constexpr (SWAP) {
        const uint64_t et = exchange12(t, n >> 3);
        const uint64_t p = (t & (mx + 1) >> 2) ? et ^ mx : et;  // s2_2 = 1: ~Et has s1_2 = 0
        if (p < t) return;
    }

    T g[8];
    if constexpr (SWAP) {
        const TwinGroup tg = twin_group8(8 * t, n);
        T q[8];
        stream4<kF32>(lag3 + tg.read, q);
        stream4<kF32>(lag3 + tg.read + 4, q + 4);
        twin_values8(q, tg.mode, g);
    } else {
        stream4<kF32>(lag3 + 8 * t, g);  // read once: non-temporal in FP32 (4.8% faster)
        stream4<kF32>(lag3 + 8 * t + 4, g + 4);
    }
    T all3 = pair8(g) * (T)0.125;
    if constexpr (kShift) all3 = all3 + d3;
    const T match = (T)1 + first(all3);

    const uint64_t mask = n - 1;
    const uint64_t r3 = mask / 7;  // 001 in every slot
    const uint64_t S1 = r3 << 2, S2 = r3 << 1, S3 = r3;
    auto base = [&](uint64_t i, uint64_t sm) { return (i & ~sm) | ((i << 3) & sm & mask); };
    // the aligned 8-group holding entry e, or its image
    auto group = [&](const T *tab, uint64_t e, int img, T *q) {
        const uint64_t grp = e & ~(uint64_t)7;
        load8(tab + (img ? (mask - 7) - grp : grp), q);
    };

    // SWAP: the value of (unfolded) index e, or of its image if img, read at
    // the lower index of its exchanged pair
    auto mem = [&](const T *tab, uint64_t e, int img) {
        const uint64_t at = img ? mask - e : e, tw = exchange_twin(at, n, 3);
        return tab[tw < at ? tw : at];
    };

#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const uint64_t x = c ? xc : t;
        T val[4];
        val[0] = match;
        {   // 001: lag 1 entries b1, b1 + 1; lag 2 entries b2 + 0, 2, 4, 6
            const uint64_t i = ((uint64_t)1 << top) | x;
            const uint64_t b1 = base(i, S3), b2 = base(i, S1 | S2);
            T p0, p1, k2;
            if constexpr (SWAP) {
                p0 = mem(lag1, b1, 0);
                p1 = mem(lag1, b1 + 1, 0);
                k2 = pair4(mem(lag2, b2, c), mem(lag2, b2 + 2, c), mem(lag2, b2 + 4, c),
                           mem(lag2, b2 + 6, c)) * (T)0.25;
            } else {
                load2(lag1 + b1, p0, p1);
                T q[8];
                group(lag2, b2, c, q);
                const int o = (int)(b2 & 1) ^ c;
                k2 = pair4(q[o], q[o + 2], q[o + 4], q[o + 6]) * (T)0.25;
            }
            const T k1 = (p0 + p1) * (T)0.5;
            if constexpr (kShift) k2 = k2 + d2;
            val[1] = vmax(first(k1), k2);
        }
        {   // 010: lag 1 entries b1, b1 + 2; lag 2 entries b2 + 0, 1, 4, 5
            const uint64_t i = ((uint64_t)2 << top) | x;
            const uint64_t b1 = base(i, S2), b2 = base(i, S1 | S3);
            T k1, k2;
            if constexpr (SWAP) {
                k1 = (mem(lag1, b1, 0) + mem(lag1, b1 + 2, 0)) * (T)0.5;
                k2 = pair4(mem(lag2, b2, c), mem(lag2, b2 + 1, c), mem(lag2, b2 + 4, c),
                           mem(lag2, b2 + 5, c)) * (T)0.25;
            } else {
                T e[8];
                group(lag1, b1, 0, e);
                const int o = (int)(b1 & 7);
                k1 = (e[o] + e[o + 2]) * (T)0.5;
                T q[8];
                group(lag2, b2, c, q);
                const int o2 = c ? 2 - (int)(b2 & 7) : (int)(b2 & 7);
                k2 = pair4(q[o2], q[o2 + 1], q[o2 + 4], q[o2 + 5]) * (T)0.25;
            }
            if constexpr (kShift) k2 = k2 + d2;
            val[2] = vmax(first(k1), k2);
        }
        {   // 011: lag 2 entries b2 + 0..3; lag 1 entries b1, b1 + 4
            const uint64_t i = ((uint64_t)3 << top) | x;
            const uint64_t b2 = base(i, S2 | S3), b1 = base(i, S1);
            T k1, k2;
            if constexpr (SWAP) {
                k2 = pair4(mem(lag2, b2, 0), mem(lag2, b2 + 1, 0), mem(lag2, b2 + 2, 0),
                           mem(lag2, b2 + 3, 0)) * (T)0.25;
                k1 = (mem(lag1, b1, c) + mem(lag1, b1 + 4, c)) * (T)0.5;
            } else {
                T q[4];
                load4(lag2 + b2, q);
                k2 = pair4(q[0], q[1], q[2], q[3]) * (T)0.25;
                T e[8];
                group(lag1, b1, c, e);
                const int o = c ? 3 - (int)(b1 & 7) : (int)(b1 & 7);
                k1 = (e[o] + e[o + 4]) * (T)0.5;
            }
            if constexpr (kShift) k2 = k2 + d2;
            val[3] = vmax(first(k2), k1);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            uint64_t j = ((uint64_t)r << top) | x;
            if constexpr (SWAP) {  // the lower index of the exchanged pair
                const uint64_t jj = exchange_twin(j, n, 3);
                j = jj < j ? jj : j;
            }
            put(out + j, kF32 ? (T)(val[r] - y0) : val[r]);
        }
    }
}

// ---------------------------------------------------------------- sigma = 2, d = 3 from branch means
// The values of sweep_s2d3<T, true, SHIFT> (rings symmetric in strings 1 and
// 2) from the lags' branch-mean tables (m1_index .. m123_index): the all-match
// tuple reads lag 3's M123, 001 lag 1's M3 and lag 2's M12, 010 the string-2
// mean of lag 1 (M1 at the exchanged tuple) and the (s1 s3) mean of lag 2
// (M23 at the exchanged tuple), 011 lag 2's M23 and lag 1's M1; M3, M12 and
// M123 are read at the lower index of each exchanged pair.  Each mean is the
// entry sweep's own, so the tables agree bit for bit.
//
// Thread t < n/16 computes the tuples of tail t and of its complement, as
// sweep_s2d3 does; the eight threads of an octet (t = 8j + v) hold every
// member of eight aligned groups (heads 000 .. 011, tails 8j + v and their
// complements, member v or 7 - v), which exchange their values by lane
// shuffles (q[k] = the value of member u xor k) and each write the means
// whose first member they hold, in the entry sweep's order of operations.
// Octets are exchange-folded whole: the lower of octet j and its exchanged
// octet runs (both members when they are one), and it also writes the
// exchanged octet's M1 (its string-2 means) and M23 (its (s1 s3) means).
// Index arithmetic in I (32 bits when every index of the table fits, which
// halves the integer work the kernel is bound by, else 64); mask = n - 1.
template <typename I>
struct D3Idx {
    I mask, half, r3;
    __device__ D3Idx(uint64_t n) : mask((I)(n - 1)), half((I)(n >> 1)), r3((I)((n - 1) / 7)) {}
    // strings 1 and 2 exchanged in every slot, complemented when that puts a
    // 1 at string 1's head (exchange_twin for d = 3)
    __device__ __forceinline__ I twin(I j) const
    {
        const I x = (j & r3) | ((j & (r3 << 2)) >> 1) | ((j & (r3 << 1)) << 1);
        return (x & half) ? x ^ mask : x;
    }
    __device__ __forceinline__ I fold(I s) const { return (s & half) ? s ^ mask : s; }
    __device__ __forceinline__ I m1(I s) const { s = fold(s); return ((s >> 3) << 2) | (s & 3); }
    __device__ __forceinline__ I m3(I s) const { return fold(s) >> 1; }
    __device__ __forceinline__ I m12(I s) const { s = fold(s); return ((s >> 3) << 1) | (s & 1); }
    __device__ __forceinline__ I m23(I s) const { s = fold(s); return ((s >> 3) << 1) | ((s >> 2) & 1); }
    __device__ __forceinline__ I m123(I s) const { return fold(s) >> 3; }
    // the strings in sm advanced: their bits move up one slot, 0 appended
    __device__ __forceinline__ I base(I i, I sm) const { return (i & ~sm) | ((i << 3) & sm & mask); }
};

template <typename T, bool SHIFT, typename I>
__global__ __launch_bounds__(kBlock) void sweep_s2d3_means(
    const T *__restrict__ m1a, const T *__restrict__ m3a, const T *__restrict__ m12b,
    const T *__restrict__ m23b, const T *__restrict__ m123c, T *__restrict__ out,
    T *__restrict__ n1, T *__restrict__ n3, T *__restrict__ n12, T *__restrict__ n23,
    T *__restrict__ n123, uint64_t n, int h, double *__restrict__ off, int s1, int s2, int s3,
    int snew)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    constexpr bool kShift = kF32 || SHIFT;
    const uint64_t t64 = thread_index();
    const int top = 3 * (h - 1);
    T d2 = 0, d3 = 0, y0 = 0;
    if constexpr (!kF32 && SHIFT) {
        d2 = off[s2] - off[s1];
        d3 = off[s3] - off[s1];
    }
    if constexpr (kF32) {
        const double o1 = off[s1];
        d2 = (float)(off[s2] - o1);
        d3 = (float)(off[s3] - o1);
        y0 = 1.0f + first(m123c[0] + d3);
        if (t64 == 0) off[snew] = o1 + (double)y0;
    }
    if (t64 >= (n >> 4)) return;
    const D3Idx<I> ix(n);
    const I t = (I)t64, mx = (I)((n >> 3) - 1), j = t >> 3;
    const int v = (int)(t & 7);
    // whole octets: the exchanged tail of 8j is 8 Ej, or 8 ~Ej + 7 when s2_2 = 1
    const I t0 = t & ~(I)7, sb = (mx + 1) >> 2, r3t = mx / 7;
    const I e0 = (t0 & r3t) | ((t0 & (r3t << 2)) >> 1) | ((t0 & (r3t << 1)) << 1);
    const I pj = ((t & sb) ? e0 ^ mx : e0) >> 3;
    if (pj < j) return;
    const bool self = pj == j;

    // reads
    T val[2][4];
    {
        const I tw = ix.m123(ix.twin(8 * t));
        T all3 = m123c[tw < t ? tw : t];
        if constexpr (kShift) all3 = all3 + d3;
        val[0][0] = val[1][0] = (T)1 + first(all3);
    }
    const I S3 = ix.r3, S2 = S3 << 1, S1 = S3 << 2;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const I x = c ? mx - t : t;
        {   // 001: string 3 (lag 1), strings 1 and 2 (lag 2)
            const I i = ((I)1 << top) | x, b1 = ix.base(i, S3), b2 = ix.base(i, S1 | S2);
            const I a3 = ix.m3(b1), a3t = ix.m3(ix.twin(b1));
            const I a12 = ix.m12(b2), a12t = ix.m12(ix.twin(b2));
            const T k1 = m3a[a3t < a3 ? a3t : a3];
            T k2 = m12b[a12t < a12 ? a12t : a12];
            if constexpr (kShift) k2 = k2 + d2;
            val[c][1] = vmax(first(k1), k2);
        }
        {   // 010: string 2 (lag 1), strings 1 and 3 (lag 2), at the exchanged tuples
            const I i = ((I)2 << top) | x, b1 = ix.base(i, S2), b2 = ix.base(i, S1 | S3);
            const T k1 = m1a[ix.m1(ix.twin(b1))];
            T k2 = m23b[ix.m23(ix.twin(b2))];
            if constexpr (kShift) k2 = k2 + d2;
            val[c][2] = vmax(first(k1), k2);
        }
        {   // 011: strings 2 and 3 (lag 2), string 1 (lag 1)
            const I i = ((I)3 << top) | x, b2 = ix.base(i, S2 | S3), b1 = ix.base(i, S1);
            T k2 = m23b[ix.m23(b2)];
            const T k1 = m1a[ix.m1(b1)];
            if constexpr (kShift) k2 = k2 + d2;
            val[c][3] = vmax(first(k2), k1);
        }
    }
    if constexpr (kF32) {
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) val[c][r] = (T)(val[c][r] - y0);
    }

    // writes: for head r and tail x (t, or its complement: prefix P = j or
    // ~j, member u = v or 7 - v), the entry at the lower index of its
    // exchanged pair when asked, and the group means this lane begins, from
    // q[k] = the value of member u xor k
    const T half = (T)0.5, quarter = (T)0.25, eighth = (T)0.125;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        T q[8];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            // the 000 groups of j and ~j hold the same lane values: one exchange
            if (!(r == 0 && c == 1)) {
                q[0] = val[c][r];
#pragma unroll
                for (int k = 1; k < 8; ++k) q[k] = __shfl_xor(q[0], k);
            }
            const int u = c ? 7 - v : v;
            const I jj = ((I)r << top) | (c ? mx - t : t);  // = 8P + u
            const I P = jj >> 3, tw = ix.twin(jj);
            if (out) put(out + (tw < jj ? tw : jj), val[c][r]);
            if (!(u & 4)) put(n1 + (4 * P + (I)(u & 3)), (q[0] + q[4]) * half);
            if (!(u & 1)) {
                const I own = 4 * P + (I)(u >> 1), twi = ix.m3(tw);
                put(n3 + (twi < own ? twi : own), (q[0] + q[1]) * half);
            }
            if (!(u & 6)) {
                const I own = 2 * P + (I)(u & 1), twi = ix.m12(tw);
                put(n12 + (twi < own ? twi : own), ((q[0] + q[6]) + (q[2] + q[4])) * quarter);
            }
            if (!(u & 3)) put(n23 + (2 * P + (I)(u >> 2)), ((q[0] + q[3]) + (q[1] + q[2])) * quarter);
            if (u == 0) {
                const I twi = ix.m123(tw);
                put(n123 + (twi < P ? twi : P),
                    (((q[0] + q[7]) + (q[1] + q[6])) + ((q[2] + q[5]) + (q[3] + q[4]))) * eighth);
            }
            if (!self) {  // the exchanged octet's string-2 and (s1 s3) means
                if (!(u & 2)) put(n1 + ix.m1(tw), (q[0] + q[2]) * half);
                if (!(u & 5)) put(n23 + ix.m23(tw), ((q[0] + q[5]) + (q[1] + q[4])) * quarter);
            }
        }
    }
}

// The new table's values at the two-array rate's sample coordinates (each at
// the lower index of its exchanged pair), in sample order: what
// sweep_s2d3_means computes for head r and tail x (the all-match tuple from
// the group at the folded prefix of x), from the same means with the same
// operations.
template <typename T, bool SHIFT>
__global__ __launch_bounds__(kBlock) void means_samples3(
    const T *__restrict__ m1a, const T *__restrict__ m3a, const T *__restrict__ m12b,
    const T *__restrict__ m23b, const T *__restrict__ m123c, T *__restrict__ smp, uint64_t n,
    int h, const double *__restrict__ off, int s1, int s2, int s3)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    constexpr bool kShift = kF32 || SHIFT;
    T d2 = 0, d3 = 0, y0 = 0;
    if constexpr (!kF32 && SHIFT) {
        d2 = off[s2] - off[s1];
        d3 = off[s3] - off[s1];
    }
    if constexpr (kF32) {
        const double o1 = off[s1];
        d2 = (float)(off[s2] - o1);
        d3 = (float)(off[s3] - o1);
        y0 = 1.0f + first(m123c[0] + d3);
    }
    const uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= (uint64_t)kRateSample) return;
    const D3Idx<uint64_t> ix(n);
    const int top = 3 * (h - 1);
    uint64_t c = (k * kRateSampleMul) & ((n >> 1) - 1);
    const uint64_t tw = ix.twin(c);
    c = tw < c ? tw : c;
    const int r = (int)((c >> top) & 3);
    const uint64_t x = c & ((1ull << top) - 1), mx = (n >> 3) - 1;
    const uint64_t S3 = ix.r3, S2 = S3 << 1, S1 = S3 << 2;
    const uint64_t i = ((uint64_t)r << top) | x;
    T v;
    if (r == 0) {
        const uint64_t t = x < (n >> 4) ? x : mx - x;
        const uint64_t at = ix.m123(ix.twin(8 * t));
        T all3 = m123c[at < t ? at : t];
        if constexpr (kShift) all3 = all3 + d3;
        v = (T)1 + first(all3);
    } else if (r == 1) {  // string 3 (lag 1), strings 1 and 2 (lag 2)
        const uint64_t b1 = ix.base(i, S3), b2 = ix.base(i, S1 | S2);
        const uint64_t a3 = ix.m3(b1), a3t = ix.m3(ix.twin(b1));
        const uint64_t a12 = ix.m12(b2), a12t = ix.m12(ix.twin(b2));
        const T k1 = m3a[a3t < a3 ? a3t : a3];
        T k2 = m12b[a12t < a12 ? a12t : a12];
        if constexpr (kShift) k2 = k2 + d2;
        v = vmax(first(k1), k2);
    } else if (r == 2) {  // string 2 (lag 1), strings 1 and 3 (lag 2), at the exchanged tuples
        const uint64_t b1 = ix.base(i, S2), b2 = ix.base(i, S1 | S3);
        const T k1 = m1a[ix.m1(ix.twin(b1))];
        T k2 = m23b[ix.m23(ix.twin(b2))];
        if constexpr (kShift) k2 = k2 + d2;
        v = vmax(first(k1), k2);
    } else {  // strings 2 and 3 (lag 2), string 1 (lag 1)
        const uint64_t b2 = ix.base(i, S2 | S3), b1 = ix.base(i, S1);
        T k2 = m23b[ix.m23(b2)];
        const T k1 = m1a[ix.m1(b1)];
        if constexpr (kShift) k2 = k2 + d2;
        v = vmax(first(k2), k1);
    }
    smp[k] = kF32 ? (T)(v - y0) : v;
}

// the five means of a stored table, one thread per group prefix P < n/16
template <typename T>
__global__ __launch_bounds__(kBlock) void derive_means3(const T *__restrict__ tab, int lazy,
                                                       T *__restrict__ m1, T *__restrict__ m3,
                                                       T *__restrict__ m12, T *__restrict__ m23,
                                                       T *__restrict__ m123, uint64_t n)
{
    const uint64_t P = thread_index();
    if (P >= (n >> 4)) return;
    T e[8];
    if (lazy) {
        const TwinGroup tg = twin_group8(8 * P, n);
        T q[8];
        load8(tab + tg.read, q);
        twin_values8(q, tg.mode, e);
    } else {
        load8(tab + 8 * P, e);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        m1[4 * P + k] = (e[k] + e[k + 4]) * (T)0.5;
        m3[4 * P + k] = (e[2 * k] + e[2 * k + 1]) * (T)0.5;
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        m12[2 * P + b] = pair4(e[b], e[2 + b], e[4 + b], e[6 + b]) * (T)0.25;
        m23[2 * P + b] = pair4(e[4 * b], e[4 * b + 1], e[4 * b + 2], e[4 * b + 3]) * (T)0.25;
    }
    m123[P] = pair8(e) * (T)0.125;
}

// ---------------------------------------------------------------- l = 1
// Every tuple is its head slot and each branch appends its symbols in that
// slot, so a branch group straddles the stored half: every value is read at
// the image of its index.  One workgroup; thread j computes stored entry j.
// Templates on (sigma, d) and the moved set M keep every array in registers.
template <int SIGMA, int D>
struct L1 {
    static constexpr int kBeta = SIGMA == 2 ? 1 : 2;
    static constexpr int kN = 1 << (kBeta * D);
    static constexpr int kNs = kN >> kBeta;
    static constexpr int kRep = (kN - 1) / (SIGMA - 1);
    static __device__ __forceinline__ int image(int i) { return i ^ ((i >> (kBeta * (D - 1))) * kRep); }
    // head with the symbols of the strings in M replaced by appended tuple c
    // (lexicographic, first moved string most significant)
    template <int M>
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
    // appended tuple at leaf j of the branch tree over CNT tuples
    template <int CNT>
    static __device__ __forceinline__ int leaf(int j)
    {
        constexpr int order16[16] = {1, 4, 11, 14, 2, 8, 7, 13, 3, 12, 6, 9, 0, 15, 5, 10};
        if (SIGMA == 4) return CNT == 16 ? order16[j] : j;
        return (j & 1) ? CNT - 1 - (j >> 1) : j >> 1;
    }
};

template <typename T, int CNT>
__device__ __forceinline__ T tree_pow2(T *v)  // the balanced tree over CNT = 2^k values
{
#pragma unroll
    for (int step = 1; step < CNT; step <<= 1)
#pragma unroll
        for (int k = 0; k < CNT; k += 2 * step) v[k] = v[k] + v[k + step];
    return v[0];
}

// mean of lag |M| over the successors of `head` for moved set M, FP32 tables
// shifted by delta_|M|; the mean of the set `moved` when M reaches it
template <typename T, int SIGMA, int D, int M, bool SHIFT>
__device__ __forceinline__ T l1_branch(const T *const *lag, const T *delta, int head, int moved)
{
    using G = L1<SIGMA, D>;
    if constexpr (M >= (1 << D)) {
        return (T)0;
    } else {
        if (moved != M) return l1_branch<T, SIGMA, D, M + 1, SHIFT>(lag, delta, head, moved);
        constexpr int K = __builtin_popcount(M), CNT = 1 << (G::kBeta * K);
        T v[CNT];
#pragma unroll
        for (int c = 0; c < CNT; ++c)
            v[c] = lag[K - 1][G::image(G::template successor<M>(head, G::template leaf<CNT>(c)))];
        T m = tree_pow2<T, CNT>(v) * ((T)1 / (T)CNT);
        if ((std::is_same<T, float>::value || SHIFT) && K >= 2) m = m + delta[K - 1];
        return m;
    }
}

template <typename T, int SIGMA, int D, bool SHIFT>
__device__ __forceinline__ T l1_value(const T *const *lag, const T *delta, int head)
{
    constexpr int kBeta = L1<SIGMA, D>::kBeta;
    int sym[D];
    bool same = true;
#pragma unroll
    for (int s = 0; s < D; ++s) {
        sym[s] = (head >> (kBeta * (D - 1 - s))) & (SIGMA - 1);
        same = same && sym[s] == sym[0];
    }
    if (same)
        return (T)1 + first(l1_branch<T, SIGMA, D, 1, SHIFT>(lag, delta, head, (1 << D) - 1));
    T best = 0;
#pragma unroll
    for (int z = 0; z < SIGMA; ++z) {
        int moved = 0;
#pragma unroll
        for (int s = 0; s < D; ++s)
            if (sym[s] != z) moved |= 1 << s;
        const T m = l1_branch<T, SIGMA, D, 1, SHIFT>(lag, delta, head, moved);
        best = z == 0 ? first(m) : vmax(best, m);
    }
    return best;
}

template <typename T, int SIGMA, int D, bool SHIFT>
__global__ __launch_bounds__(kBlock) void sweep_l1(const T *__restrict__ lag1,
                                                  const T *__restrict__ lag2,
                                                  const T *__restrict__ lag3,
                                                  T *__restrict__ out,
                                                  double *__restrict__ off, int s1, int s2,
                                                  int s3, int snew)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    const T *lag[3] = {lag1, lag2, lag3};
    T delta[3] = {0, 0, 0};
    double o1 = 0.0;
    if constexpr (kF32) {
        o1 = off[s1];
        delta[1] = (float)(off[s2] - o1);
        if (D == 3) delta[2] = (float)(off[s3] - o1);
    } else if constexpr (SHIFT) {
        delta[1] = off[s2] - off[s1];
        if (D == 3) delta[2] = off[s3] - off[s1];
    }
    const T y0 = kF32 ? l1_value<T, SIGMA, D, SHIFT>(lag, delta, 0) : (T)0;
    const int j = threadIdx.x;
    if (kF32 && j == 0) off[snew] = o1 + (double)y0;
    if (j < L1<SIGMA, D>::kNs) {
        const T v = l1_value<T, SIGMA, D, SHIFT>(lag, delta, j);
        out[j] = kF32 ? (T)(v - y0) : v;
    }
}

// ---------------------------------------------------------------- packed tables
// sigma = d = 2 on exchange-packed tables (packed_index): one thread per code
// k computes the value of its orbit's representative tuple, as sweep_s2d2
// computes it (the same values in the same trees: every branch tree is
// invariant under the complement and the exchange, so a group read through
// its orbit's codes gives the bits of the unpacked table), and stores it at
// k.  An aligned group of four whose pivot lies above the last position is
// four consecutive codes (one vector load, members permuted); other groups
// are read member by member.  Codes that belong to no orbit are not written.
template <typename T>
__device__ __forceinline__ void packed_group_values(const T *__restrict__ tab, uint64_t gbase,
                                                    int h, T *e)
{
    const PackedGroup pg = packed_group(gbase, h);
    if (pg.regular) {
        T q[4];
        load4(tab + pg.base, q);
#pragma unroll
        for (int k = 0; k < 4; ++k) asm volatile("" : "+v"(q[k]));
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int at = packed_member(pg, v);
            e[v] = at == 0 ? q[0] : at == 1 ? q[1] : at == 2 ? q[2] : q[3];
        }
    } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) e[v] = tab[packed_index(gbase + (uint64_t)v, h)];
    }
}

template <typename T, bool SHIFT>
__global__ __launch_bounds__(kBlock) void sweep_s2d2_packed(const T *__restrict__ lag1,
                                                           const T *__restrict__ lag2,
                                                           T *__restrict__ out, int h,
                                                           double *__restrict__ off, int s1,
                                                           int s2, int snew)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    constexpr bool kShift = kF32 || SHIFT;  // lag 2 carries delta_2
    const uint64_t n = 1ull << (2 * h), nq = n >> 2;
    const uint64_t k = thread_index();
    T d2 = 0, y0 = 0;
    if constexpr (!kF32 && SHIFT) d2 = off[s2] - off[s1];
    if constexpr (kF32) {
        const double o1 = off[s1];
        d2 = (float)(off[s2] - o1);
        const T e0 = lag2[packed_zero_group(0, h)], e1 = lag2[packed_zero_group(1, h)];
        const T e3 = lag2[packed_zero_group(3, h)];
        y0 = 1.0f + first(pair4(e0, e1, e1, e3) * 0.25f + d2);
        if (k == 0) off[snew] = o1 + (double)y0;
    }
    if (k >= packed_entries(h)) return;
    const uint64_t i = packed_tuple(k, h);
    if (i == kNoOrbit) return;
    T v;
    if (i < nq) {  // head 0/0
        // 0/0|x and 0/0|~x read image groups, so their values are equal:
        // the lower of the two codes computes both
        const uint64_t kc = packed_index(i ^ (nq - 1), h);
        if (kc < k) return;
        T g[4];
        packed_group_values(lag2, (i << 2) & (n - 1), h, g);
        T m2 = pair4(g[0], g[1], g[2], g[3]) * (T)0.25;
        if constexpr (kShift) m2 = m2 + d2;
        v = (T)1 + first(m2);
        if (kc != k) put(out + kc, kF32 ? (T)(v - y0) : v);
    } else {       // head 0/1: advance b (z = 0) and advance a (z = 1) read lag 1
        const uint64_t am = kAlt2 & (n - 1), bm = ~kAlt2 & (n - 1);
        const uint64_t sb = (i & am) | ((i << 2) & bm);
        const uint64_t sa = ((i << 2) & am) | (i & bm);
        T q[4];
        packed_group_values(lag1, sb & ~(uint64_t)3, h, q);
        const bool hi = (sb & 2) != 0;
        const T mb = ((hi ? q[2] : q[0]) + (hi ? q[3] : q[1])) * (T)0.5;
        packed_group_values(lag1, sa & ~(uint64_t)3, h, q);
        const bool odd = (sa & 1) != 0;
        const T ma = ((odd ? q[1] : q[0]) + (odd ? q[3] : q[2])) * (T)0.5;
        v = vmax(first(mb), ma);
    }
    put(out + k, kF32 ? (T)(v - y0) : v);
}

// a grid of `threads` threads of kBlock (two-dimensional past 2^32 threads)
dim3 sweep_grid(uint64_t threads)
{
    const uint64_t blocks = (threads + kBlock - 1) / kBlock;
    constexpr uint64_t kRow = 1ull << 16;  // blocks per grid row when one row is not enough
    if (blocks * kBlock >= (1ull << 32)) return dim3((unsigned)kRow, (unsigned)((blocks + kRow - 1) / kRow));
    return dim3((unsigned)blocks);
}

template <typename T, bool SHIFT>
hipError_t launch_typed(const Geometry &g, const SweepLaunch &a, hipStream_t s)
{
    const T *l1 = static_cast<const T *>(a.lag[0]);
    const T *l2 = static_cast<const T *>(a.lag[1]);
    const T *l3 = g.d == 3 ? static_cast<const T *>(a.lag[2]) : nullptr;
    T *out = static_cast<T *>(a.out);
    const int s1 = a.lag_slot[0], s2 = a.lag_slot[1], s3 = g.d == 3 ? a.lag_slot[2] : 0;
    if (g.h == 1) {
        if (g.sigma == 2 && g.d == 2)
            sweep_l1<T, 2, 2, SHIFT><<<1, kBlock, 0, s>>>(l1, l2, l3, out, a.offsets, s1, s2, s3,
                                                          a.new_slot);
        else if (g.sigma == 4 && g.d == 2)
            sweep_l1<T, 4, 2, SHIFT><<<1, kBlock, 0, s>>>(l1, l2, l3, out, a.offsets, s1, s2, s3,
                                                          a.new_slot);
        else if (g.sigma == 2 && g.d == 3)
            sweep_l1<T, 2, 3, SHIFT><<<1, kBlock, 0, s>>>(l1, l2, l3, out, a.offsets, s1, s2, s3,
                                                          a.new_slot);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    const dim3 block(kBlock);
    if (a.packed) {
        if (g.sigma != 2 || g.d != 2) return hipErrorInvalidValue;
        sweep_s2d2_packed<T, SHIFT><<<sweep_grid(packed_entries(g.h)), block, 0, s>>>(
            l1, l2, out, g.h, a.offsets, s1, s2, a.new_slot);
        return hipGetLastError();
    }
    // one thread per x with string-1 symbol 0 at position 2
    const dim3 grid = sweep_grid(g.n >> (g.slot + g.beta));
    if (g.sigma == 2 && g.d == 2) {
        if (a.swap_sym)
            sweep_s2d2<T, true, SHIFT><<<grid, block, 0, s>>>(l1, l2, out, g.n, a.offsets, s1, s2,
                                                              a.new_slot);
        else
            sweep_s2d2<T, false, SHIFT><<<grid, block, 0, s>>>(l1, l2, out, g.n, a.offsets, s1,
                                                               s2, a.new_slot);
    } else if (g.sigma == 4 && g.d == 2) {
        if (a.swap_sym)
            sweep_s4d2<T, true, SHIFT><<<grid, block, 0, s>>>(l1, l2, out, g.n, g.h, a.offsets,
                                                              s1, s2, a.new_slot);
        else
            sweep_s4d2<T, false, SHIFT><<<grid, block, 0, s>>>(l1, l2, out, g.n, g.h, a.offsets,
                                                               s1, s2, a.new_slot);
    } else if (g.sigma == 2 && g.d == 3) {
        if (a.swap_sym)
            sweep_s2d3<T, true, SHIFT><<<grid, block, 0, s>>>(l1, l2, l3, out, g.n, g.h,
                                                              a.offsets, s1, s2, s3, a.new_slot);
        else
            sweep_s2d3<T, false, SHIFT><<<grid, block, 0, s>>>(l1, l2, l3, out, g.n, g.h,
                                                               a.offsets, s1, s2, s3, a.new_slot);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

template <typename T, bool SHIFT>
hipError_t means_typed(const Geometry &g, const MeansLaunch &a, void *samples, hipStream_t s)
{
    if (samples)
        means_samples<T, SHIFT><<<kRateSample / kBlock, dim3(kBlock), 0, s>>>(
            static_cast<const T *>(a.ma1), static_cast<const T *>(a.mab2),
            static_cast<T *>(samples), g.n, a.offsets, a.s1, a.s2);
    else
        sweep_s2d2_means<T, SHIFT><<<sweep_grid(g.n >> 5), dim3(kBlock), 0, s>>>(
            static_cast<const T *>(a.ma1), static_cast<const T *>(a.mab2),
            static_cast<T *>(a.out), static_cast<T *>(a.ma_new), static_cast<T *>(a.mab_new), g.n,
            a.offsets, a.s1, a.s2, a.snew);
    return hipGetLastError();
}

hipError_t means_dispatch(const Geometry &g, int dtype, const MeansLaunch &a, void *samples,
                          hipStream_t s)
{
    if (g.sigma != 2 || g.d != 2 || g.h < 3) return hipErrorInvalidValue;
    if (dtype == LCSB_F32) return means_typed<float, false>(g, a, samples, s);
    return a.shift ? means_typed<double, true>(g, a, samples, s)
                   : means_typed<double, false>(g, a, samples, s);
}

hipError_t launch_sweep_means(const Geometry &g, int dtype, const MeansLaunch &a, hipStream_t s)
{
    return means_dispatch(g, dtype, a, nullptr, s);
}

template <typename T, bool SHIFT>
hipError_t samples4_typed(const Geometry &g, const MeansLaunch &a, void *samples, hipStream_t s)
{
    means_samples4<T, SHIFT><<<kRateSample / kBlock, dim3(kBlock), 0, s>>>(
        static_cast<const T *>(a.ma1), static_cast<const T *>(a.mab2), static_cast<T *>(samples),
        g.n, g.h, a.offsets, a.s1, a.s2);
    return hipGetLastError();
}

hipError_t launch_means_samples(const Geometry &g, int dtype, const MeansLaunch &a, void *samples,
                                hipStream_t s)
{
    if (!samples) return hipErrorInvalidValue;
    if (g.sigma == 4) {
        if (g.d != 2 || g.h < 3) return hipErrorInvalidValue;
        if (dtype == LCSB_F32) return samples4_typed<float, false>(g, a, samples, s);
        return a.shift ? samples4_typed<double, true>(g, a, samples, s)
                       : samples4_typed<double, false>(g, a, samples, s);
    }
    return means_dispatch(g, dtype, a, samples, s);
}

hipError_t launch_derive_means(const Geometry &g, int dtype, const void *table, int lazy,
                               void *ma, void *mab, hipStream_t s)
{
    if (g.sigma != 2 || g.d != 2 || g.h < 3) return hipErrorInvalidValue;
    const dim3 grid = sweep_grid(g.n >> 3);
    if (dtype == LCSB_F32)
        derive_means<float><<<grid, dim3(kBlock), 0, s>>>(static_cast<const float *>(table), lazy,
                                                          static_cast<float *>(ma),
                                                          static_cast<float *>(mab), g.n);
    else
        derive_means<double><<<grid, dim3(kBlock), 0, s>>>(static_cast<const double *>(table),
                                                           lazy, static_cast<double *>(ma),
                                                           static_cast<double *>(mab), g.n);
    return hipGetLastError();
}

template <typename T, bool SHIFT, typename I>
hipError_t means3_typed(const Geometry &g, const Means3Launch &a, hipStream_t s)
{
    sweep_s2d3_means<T, SHIFT, I><<<sweep_grid(g.n >> 4), dim3(kBlock), 0, s>>>(
        static_cast<const T *>(a.m1), static_cast<const T *>(a.m3), static_cast<const T *>(a.m12),
        static_cast<const T *>(a.m23), static_cast<const T *>(a.m123), static_cast<T *>(a.out),
        static_cast<T *>(a.n1), static_cast<T *>(a.n3), static_cast<T *>(a.n12),
        static_cast<T *>(a.n23), static_cast<T *>(a.n123), g.n, g.h, a.offsets, a.s1, a.s2, a.s3,
        a.snew);
    return hipGetLastError();
}

hipError_t launch_sweep_means3(const Geometry &g, int dtype, const Means3Launch &a, hipStream_t s)
{
    if (g.sigma != 2 || g.d != 3 || g.h < 3) return hipErrorInvalidValue;
    if (g.n <= (1ull << 31)) {  // every index, and 8 t, in 32 bits
        if (dtype == LCSB_F32) return means3_typed<float, false, uint32_t>(g, a, s);
        return a.shift ? means3_typed<double, true, uint32_t>(g, a, s)
                       : means3_typed<double, false, uint32_t>(g, a, s);
    }
    if (dtype == LCSB_F32) return means3_typed<float, false, uint64_t>(g, a, s);
    return a.shift ? means3_typed<double, true, uint64_t>(g, a, s)
                   : means3_typed<double, false, uint64_t>(g, a, s);
}

template <typename T, bool SHIFT>
hipError_t samples3_typed(const Geometry &g, const Means3Launch &a, void *samples, hipStream_t s)
{
    means_samples3<T, SHIFT><<<kRateSample / kBlock, dim3(kBlock), 0, s>>>(
        static_cast<const T *>(a.m1), static_cast<const T *>(a.m3), static_cast<const T *>(a.m12),
        static_cast<const T *>(a.m23), static_cast<const T *>(a.m123), static_cast<T *>(samples),
        g.n, g.h, a.offsets, a.s1, a.s2, a.s3);
    return hipGetLastError();
}

hipError_t launch_means_samples3(const Geometry &g, int dtype, const Means3Launch &a,
                                 void *samples, hipStream_t s)
{
    if (!samples || g.sigma != 2 || g.d != 3 || g.h < 3) return hipErrorInvalidValue;
    if (dtype == LCSB_F32) return samples3_typed<float, false>(g, a, samples, s);
    return a.shift ? samples3_typed<double, true>(g, a, samples, s)
                   : samples3_typed<double, false>(g, a, samples, s);
}

hipError_t launch_derive_means3(const Geometry &g, int dtype, const void *table, int lazy, void *m1,
                                void *m3, void *m12, void *m23, void *m123, hipStream_t s)
{
    if (g.sigma != 2 || g.d != 3 || g.h < 3) return hipErrorInvalidValue;
    const dim3 grid = sweep_grid(g.n >> 4);
    if (dtype == LCSB_F32)
        derive_means3<float><<<grid, dim3(kBlock), 0, s>>>(
            static_cast<const float *>(table), lazy, static_cast<float *>(m1),
            static_cast<float *>(m3), static_cast<float *>(m12), static_cast<float *>(m23),
            static_cast<float *>(m123), g.n);
    else
        derive_means3<double><<<grid, dim3(kBlock), 0, s>>>(
            static_cast<const double *>(table), lazy, static_cast<double *>(m1),
            static_cast<double *>(m3), static_cast<double *>(m12), static_cast<double *>(m23),
            static_cast<double *>(m123), g.n);
    return hipGetLastError();
}

template <typename T, bool SHIFT, typename I>
hipError_t means4_typed(const Geometry &g, const MeansLaunch &a, hipStream_t s)
{
    sweep_s4d2_means<T, SHIFT, I><<<sweep_grid(g.n >> 6), dim3(kBlock), 0, s>>>(
        static_cast<const T *>(a.ma1), static_cast<const T *>(a.mab2), static_cast<T *>(a.out),
        static_cast<T *>(a.ma_new), static_cast<T *>(a.mab_new), g.n, g.h, a.offsets, a.s1, a.s2,
        a.snew);
    return hipGetLastError();
}

hipError_t launch_sweep_means4(const Geometry &g, int dtype, const MeansLaunch &a, hipStream_t s)
{
    if (g.sigma != 4 || g.d != 2 || g.h < 3) return hipErrorInvalidValue;
    if (g.n <= (1ull << 32)) {  // every index in 32 bits
        if (dtype == LCSB_F32) return means4_typed<float, false, uint32_t>(g, a, s);
        return a.shift ? means4_typed<double, true, uint32_t>(g, a, s)
                       : means4_typed<double, false, uint32_t>(g, a, s);
    }
    if (dtype == LCSB_F32) return means4_typed<float, false, uint64_t>(g, a, s);
    return a.shift ? means4_typed<double, true, uint64_t>(g, a, s)
                   : means4_typed<double, false, uint64_t>(g, a, s);
}

hipError_t launch_derive_means4(const Geometry &g, int dtype, const void *table, int lazy, void *ma,
                                void *mab, hipStream_t s)
{
    if (g.sigma != 4 || g.d != 2 || g.h < 3) return hipErrorInvalidValue;
    const dim3 grid = sweep_grid(g.n >> 6);
    if (dtype == LCSB_F32)
        derive_means4<float><<<grid, dim3(kBlock), 0, s>>>(static_cast<const float *>(table), lazy,
                                                           static_cast<float *>(ma),
                                                           static_cast<float *>(mab), g.n);
    else
        derive_means4<double><<<grid, dim3(kBlock), 0, s>>>(static_cast<const double *>(table),
                                                            lazy, static_cast<double *>(ma),
                                                            static_cast<double *>(mab), g.n);
    return hipGetLastError();
}

hipError_t launch_sweep(const Geometry &g, int dtype, const SweepLaunch &a, hipStream_t s)
{
    // FP32 tables always read lag k shifted by delta_k (their offsets); FP64
    // ones only in the two-array iteration
    if (dtype == LCSB_F32) return launch_typed<float, false>(g, a, s);
    return a.shift ? launch_typed<double, true>(g, a, s) : launch_typed<double, false>(g, a, s);
}

}  // namespace lcsb
