// One sweep v_new = F(lag 1, .., lag d) of eq. (4) (Sec. 2.1), gfx950.
//
// Layout: index bits, most significant first, are the beta-bit symbols of
// position 1 (string 1 .. string d), then position 2, .. position l.  The
// top "slot" (d*beta bits) holds the heads; x below denotes the remaining
// (l-1) slots.  Advancing a set N of strings (Algorithm 1) shifts their
// symbol fields up one slot and appends the new symbols in the lowest slot,
// so every branch reads sigma^|N| entries of one aligned sigma^d group.
//
// Work split: one thread per x.  The thread evaluates the tuples whose
// string-1 head is 0 (one per orbit of the symbol relabelling c -> c xor m,
// the complement symmetry of Sec. 3.3 for sigma = 2) and stores each value
// at all sigma members of its orbit.  Over the grid every lag table is read
// once and the output written once: (d+1) * sizeof(T) bytes per entry for
// d = 2 (one lag-2 group shared by all heads, the lag-1 branch groups of the
// representatives, sigma writes per value).
//
// Arithmetic (bit-exact with the FP64 reference): each branch sums its
// sigma^k values with a balanced binary tree in lexicographic order of the
// appended symbols (first advanced string most significant), multiplies by
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

template <typename T>
__device__ __forceinline__ T tree8(const T *g)
{
    return tree4(g[0], g[1], g[2], g[3]) + tree4(g[4], g[5], g[6], g[7]);
}

template <typename T>
__device__ __forceinline__ T tree16(const T *g) { return tree8(g) + tree8(g + 8); }

template <typename T>
__device__ __forceinline__ T vmax(T best, T cand) { return cand > best ? cand : best; }

// The new table is not read again until the next sweep, after 2-3 more
// tables have streamed through the caches: write it non-temporally.
template <typename T>
__device__ __forceinline__ void put(T *p, T v) { __builtin_nontemporal_store(v, p); }

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
// Streaming variants for the sigma = d = 2 kernel, whose lag bytes are each
// read once per sweep: FP64 reads are non-temporal there (1.8% faster at
// l = 16; FP32 unchanged).  The other kernels share groups between
// representatives through L2 and keep ordinary loads (non-temporal reads
// made their FP64 sweeps 15-55% slower).
__device__ __forceinline__ void stream2(const double *p, double &a, double &b)
{
    a = __builtin_nontemporal_load(p);
    b = __builtin_nontemporal_load(p + 1);
}
__device__ __forceinline__ void stream4(const double *p, double *g)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = __builtin_nontemporal_load(p + k);
}
__device__ __forceinline__ void stream2(const float *p, float &a, float &b) { load2(p, a, b); }
__device__ __forceinline__ void load4(const float *p, float *g)
{
    float4 v = *reinterpret_cast<const float4 *>(p);
    g[0] = v.x; g[1] = v.y; g[2] = v.z; g[3] = v.w;
}
__device__ __forceinline__ void stream4(const float *p, float *g) { load4(p, g); }

constexpr uint64_t kAlt2 = 0xAAAAAAAAAAAAAAAAull;  // high bit of every 2-bit slot
constexpr uint64_t kAlt4Hi = 0xCCCCCCCCCCCCCCCCull; // high 2-bit field of every nibble

// ---------------------------------------------------------------- sigma = 2, d = 2
// Slot = (a bit, b bit).  Representatives: 0/0|x (all-match) and 0/1|x.
//   0/0|x : 1 + mean(lag2[4x .. 4x+3])                         (eq. (2))
//   0/1|x : max( mean lag1[sb], lag1[sb+1]   (advance b, z = 0),
//                mean lag1[sa], lag1[sa+2] ) (advance a, z = 1) (Alg. 1)
// Orbit partner of index i under the complement is n-1-i (eq. (10)).
template <typename T>
__global__ __launch_bounds__(kBlock) void sweep_s2d2(const T *__restrict__ lag1,
                                                    const T *__restrict__ lag2,
                                                    T *__restrict__ out, uint64_t n,
                                                    double *__restrict__ off, int s1, int s2,
                                                    int snew)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    const uint64_t nq = n >> 2;
    const uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    T d2 = 0, y0 = 0;
    if constexpr (kF32) {
        const double o1 = off[s1];
        d2 = (float)(off[s2] - o1);
        y0 = 1.0f + (tree4(lag2[0], lag2[1], lag2[2], lag2[3]) * 0.25f + d2);
        if (x == 0) off[snew] = o1 + (double)y0;
    }
    if (x >= nq) return;

    T g[4];
    stream4(lag2 + 4 * x, g);
    T m2 = tree4(g[0], g[1], g[2], g[3]) * (T)0.25;
    if constexpr (kF32) m2 = m2 + d2;
    const T match = (T)1 + m2;

    const uint64_t am = kAlt2 & (n - 1), bm = ~kAlt2 & (n - 1);
    const uint64_t i = nq + x;
    const uint64_t sb = (i & am) | ((i << 2) & bm);
    const uint64_t sa = ((i << 2) & am) | (i & bm);
    T b0, b1;
    stream2(lag1 + sb, b0, b1);
    const T mb = (b0 + b1) * (T)0.5;
    // the advance-a pair sa, sa+2 is the even or odd half of the aligned
    // group sa & ~3, which the neighbouring thread (x ^ 1) also reads: one
    // vector load of the group serves both
    T q[4];
    stream4(lag1 + (sa & ~(uint64_t)3), q);
    const T ma = ((sa & 1) ? (q[1] + q[3]) : (q[0] + q[2])) * (T)0.5;
    const T mis = vmax(mb, ma);

    if constexpr (kF32) {
        put(out + x, match - y0);
        put(out + (n - 1 - x), match - y0);
        put(out + i, mis - y0);
        put(out + (n - 1 - i), mis - y0);
    } else {
        put(out + x, match);
        put(out + (n - 1 - x), match);
        put(out + i, mis);
        put(out + (n - 1 - i), mis);
    }
}

// ---------------------------------------------------------------- sigma = 4, d = 2
// Slot = (a: 2 bits, b: 2 bits).  Representatives (0, b1)|x, b1 = 0..3.
// Branches of (0, b1), b1 != 0: z = 0 advances b (lag 1), z = b1 advances a
// (lag 1), the two other z advance both (lag 2, the same group as the
// all-match representative).  Orbit: xor every 2-bit symbol with m.
template <typename T>
__global__ __launch_bounds__(kBlock) void sweep_s4d2(const T *__restrict__ lag1,
                                                    const T *__restrict__ lag2,
                                                    T *__restrict__ out, uint64_t n, int h,
                                                    double *__restrict__ off, int s1, int s2,
                                                    int snew)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    const uint64_t ng = n >> 4;
    const uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const int top = 4 * (h - 1);
    T d2 = 0, y0 = 0;
    if constexpr (kF32) {
        const double o1 = off[s1];
        d2 = (float)(off[s2] - o1);
        T g0[16];
        for (int t = 0; t < 16; t += 4) load4(lag2 + t, g0 + t);
        y0 = 1.0f + (tree16(g0) * 0.0625f + d2);
        if (x == 0) off[snew] = o1 + (double)y0;
    }
    if (x >= ng) return;

    T g[16];
#pragma unroll
    for (int t = 0; t < 16; t += 4) load4(lag2 + 16 * x + t, g + t);
    T both = tree16(g) * (T)0.0625;
    if constexpr (kF32) both = both + d2;

    const uint64_t am = kAlt4Hi & (n - 1), bm = ~kAlt4Hi & (n - 1);
    const uint64_t sb = (x & am) | ((x << 4) & bm);
    T bv[4];
    load4(lag1 + sb, bv);
    const T mb = tree4(bv[0], bv[1], bv[2], bv[3]) * (T)0.25;
    const uint64_t sa0 = ((x << 4) & am) | (x & bm);

    T val[4];
    val[0] = (T)1 + both;
#pragma unroll
    for (int b1 = 1; b1 < 4; ++b1) {
        const uint64_t sa = sa0 | ((uint64_t)b1 << top);
        const T ma = tree4(lag1[sa], lag1[sa + 4], lag1[sa + 8], lag1[sa + 12]) * (T)0.25;
        T best = mb;                                     // z = 0
#pragma unroll
        for (int z = 1; z < 4; ++z) best = vmax(best, z == b1 ? ma : both);
        val[b1] = best;
    }
    const uint64_t rep = (n - 1) / 3;  // 01 in every 2-bit field
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint64_t i = ((uint64_t)r << top) | x;
        const T v = kF32 ? (T)(val[r] - y0) : val[r];
#pragma unroll
        for (int m = 0; m < 4; ++m) put(out + (i ^ ((uint64_t)m * rep)), v);
    }
}

// ---------------------------------------------------------------- sigma = 2, d = 3
// Slot = (s1, s2, s3) bits.  Representatives 000|x (all-match), 001|x,
// 010|x, 011|x.  Each mismatch representative has one branch moving the
// single string whose head differs (lag 1) and one moving the other two
// (lag 2):  001: z=0 -> {3}, z=1 -> {1,2};  010: z=0 -> {2}, z=1 -> {1,3};
// 011: z=0 -> {2,3}, z=1 -> {1}.  Orbit partner: n-1-i.
template <typename T>
__global__ __launch_bounds__(kBlock) void sweep_s2d3(const T *__restrict__ lag1,
                                                    const T *__restrict__ lag2,
                                                    const T *__restrict__ lag3,
                                                    T *__restrict__ out, uint64_t n, int h,
                                                    double *__restrict__ off, int s1, int s2,
                                                    int s3, int snew)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    const uint64_t ng = n >> 3;
    const uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const int top = 3 * (h - 1);
    T d2 = 0, d3 = 0, y0 = 0;
    if constexpr (kF32) {
        const double o1 = off[s1];
        d2 = (float)(off[s2] - o1);
        d3 = (float)(off[s3] - o1);
        T g0[8];
        load4(lag3, g0);
        load4(lag3 + 4, g0 + 4);
        y0 = 1.0f + (tree8(g0) * 0.125f + d3);
        if (x == 0) off[snew] = o1 + (double)y0;
    }
    if (x >= ng) return;

    T g[8];
    load4(lag3 + 8 * x, g);
    load4(lag3 + 8 * x + 4, g + 4);
    T all3 = tree8(g) * (T)0.125;
    if constexpr (kF32) all3 = all3 + d3;

    const uint64_t mask = n - 1;
    const uint64_t r3 = mask / 7;  // 001 in every slot
    const uint64_t S1 = r3 << 2, S2 = r3 << 1, S3 = r3;
    auto base = [&](uint64_t i, uint64_t sm) { return (i & ~sm) | ((i << 3) & sm & mask); };

    T val[4];
    val[0] = (T)1 + all3;
    {   // 001
        const uint64_t i = ((uint64_t)1 << top) | x;
        const uint64_t b1 = base(i, S3), b2 = base(i, S1 | S2);
        T p0, p1;
        load2(lag1 + b1, p0, p1);
        const T k1 = (p0 + p1) * (T)0.5;
        // entries b2 + 0, 2, 4, 6: the even or odd half of the aligned group
        // b2 & ~7, whose other half another thread of the wave reads
        T q[8];
        load4(lag2 + (b2 & ~(uint64_t)7), q);
        load4(lag2 + (b2 & ~(uint64_t)7) + 4, q + 4);
        const int o = (int)(b2 & 1);
        T k2 = tree4(q[o], q[o + 2], q[o + 4], q[o + 6]) * (T)0.25;
        if constexpr (kF32) k2 = k2 + d2;
        val[1] = vmax(k1, k2);
    }
    {   // 010
        const uint64_t i = ((uint64_t)2 << top) | x;
        const uint64_t b1 = base(i, S2), b2 = base(i, S1 | S3);
        T e[8];  // entries b1, b1 + 2 from their aligned group
        load4(lag1 + (b1 & ~(uint64_t)7), e);
        load4(lag1 + (b1 & ~(uint64_t)7) + 4, e + 4);
        const int o = (int)(b1 & 7);
        const T k1 = (e[o] + e[o + 2]) * (T)0.5;
        T q0, q1, q2, q3;
        load2(lag2 + b2, q0, q1);
        load2(lag2 + b2 + 4, q2, q3);
        T k2 = tree4(q0, q1, q2, q3) * (T)0.25;
        if constexpr (kF32) k2 = k2 + d2;
        val[2] = vmax(k1, k2);
    }
    {   // 011
        const uint64_t i = ((uint64_t)3 << top) | x;
        const uint64_t b2 = base(i, S2 | S3), b1 = base(i, S1);
        T q[4];
        load4(lag2 + b2, q);
        T k2 = tree4(q[0], q[1], q[2], q[3]) * (T)0.25;
        if constexpr (kF32) k2 = k2 + d2;
        T e[8];  // entries b1, b1 + 4 from their aligned group
        load4(lag1 + (b1 & ~(uint64_t)7), e);
        load4(lag1 + (b1 & ~(uint64_t)7) + 4, e + 4);
        const int o = (int)(b1 & 7);
        const T k1 = (e[o] + e[o + 4]) * (T)0.5;
        val[3] = vmax(k2, k1);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint64_t i = ((uint64_t)r << top) | x;
        const T v = kF32 ? (T)(val[r] - y0) : val[r];
        put(out + i, v);
        put(out + (mask - i), v);
    }
}

template <typename T>
hipError_t launch_typed(const Geometry &g, const SweepLaunch &a, hipStream_t s)
{
    const T *l1 = static_cast<const T *>(a.lag[0]);
    const T *l2 = static_cast<const T *>(a.lag[1]);
    T *out = static_cast<T *>(a.out);
    const uint64_t groups = g.n >> g.slot;  // one thread per x
    const uint64_t blocks = (groups + kBlock - 1) / kBlock;
    if (blocks > 0x7fffffffull) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)blocks), block(kBlock);
    if (g.sigma == 2 && g.d == 2) {
        sweep_s2d2<T><<<grid, block, 0, s>>>(l1, l2, out, g.n, a.offsets, a.lag_slot[0],
                                              a.lag_slot[1], a.new_slot);
    } else if (g.sigma == 4 && g.d == 2) {
        sweep_s4d2<T><<<grid, block, 0, s>>>(l1, l2, out, g.n, g.h, a.offsets, a.lag_slot[0],
                                              a.lag_slot[1], a.new_slot);
    } else if (g.sigma == 2 && g.d == 3) {
        const T *l3 = static_cast<const T *>(a.lag[2]);
        sweep_s2d3<T><<<grid, block, 0, s>>>(l1, l2, l3, out, g.n, g.h, a.offsets,
                                              a.lag_slot[0], a.lag_slot[1], a.lag_slot[2],
                                              a.new_slot);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep(const Geometry &g, int dtype, const SweepLaunch &a, hipStream_t s)
{
    return dtype == LCSB_F32 ? launch_typed<float>(g, a, s) : launch_typed<double>(g, a, s);
}

}  // namespace lcsb
