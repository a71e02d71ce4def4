// Declarations shared by the library's translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "lcsb.h"

namespace lcsb {

constexpr int kBlock = 256;          // threads per workgroup (4 wavefronts)
constexpr int kMaxReduceBlocks = 16384;

// Device workspace layout (byte offsets).  The caller allocates
// kWorkspaceBytes; the library clears the parts it uses.
struct Ws {
    // scalars written by the certificate kernels
    static constexpr size_t kR = 0;          // double: R (offset-corrected)
    static constexpr size_t kDRup = 8;       // double: d*R rounded up
    static constexpr size_t kShift = 16;     // double[4]: (d-k)R rounded down, k = 0..3
    static constexpr size_t kMaxW = 48;      // double
    static constexpr size_t kArgmax = 56;    // uint64
    static constexpr size_t kNonfinite = 64; // uint64: W pass
    static constexpr size_t kNonfiniteR = 72;// uint64: R pass (u, prev)
    // the largest-r certificate
    static constexpr size_t kOptR = 80;          // double: min over coordinates of max_z c_z / k_z
    static constexpr size_t kOptArg = 88;        // uint64: lowest index attaining it
    static constexpr size_t kOptNonfinite = 96;  // uint64: coordinates whose ratio is not finite
    static constexpr size_t kScalarBytes = 104;
    static constexpr size_t kRate = 112;     // double: R of the two-array iteration
    static constexpr size_t kAsym = 128;     // uint32: set when a table is not exchange-symmetric
    // FP64 offsets of the FP32 tables, one per ring slot (0 .. 3); slots 4 and
    // 5 hold the values lag 2 and lag 3 are read relative to in the two-array
    // iteration (FP32: offset of u - (k-1) R; FP64: -(k-1) R), slot 6 is
    // always zero (the reference of FP64 tables)
    static constexpr size_t kOffsets = 256;  // double[8]
    static constexpr int kSlotLag2 = 4, kSlotLag3 = 5, kSlotZero = 6;
    // per-workgroup partials of the reductions
    static constexpr size_t kPartVal = 512;                                  // double[kMaxReduceBlocks]
    static constexpr size_t kPartIdx = kPartVal + 8 * kMaxReduceBlocks;      // uint64[kMaxReduceBlocks]
    static constexpr size_t kPartCnt = kPartIdx + 8 * kMaxReduceBlocks;      // uint64[kMaxReduceBlocks]
    static constexpr size_t kBytes = kPartCnt + 8 * kMaxReduceBlocks;
};

struct Geometry {
    int sigma, d, h, beta, slot;  // slot = bits per position = d * beta
    uint64_t n;                   // sigma^(d h) indices
    uint64_t ns;                  // n / sigma stored entries: the string-1 head is 0
};

// One sweep: reads lag 1..d (ring slots lag_slot[0..d-1]), writes slot new_slot.
struct SweepLaunch {
    const void *lag[3];
    void *out;
    int lag_slot[3];
    int new_slot;
    double *offsets;  // device, per slot (FP32 only)
    int swap_sym;     // sigma = 2, d = 2 or 3: the lag tables are symmetric in strings 1 and 2
                      // (read lazily, see TwinGroup; the new table is written lazily)
    int shift;        // FP64 only: lag k is read as its values + (offsets[lag_slot[k-1]] -
                      // offsets[lag_slot[0]]) (the two-array iteration); FP32 always is
    int packed;       // sigma = d = 2: the tables are exchange-packed (packed_index), h >= 2
};

hipError_t launch_sweep(const Geometry &g, int dtype, const SweepLaunch &a, hipStream_t s);

// Branch-mean tables of a folded sigma = d = 2 table T that is symmetric in
// the two strings (n = 4^l, stored tuples s < n/2, l >= 3).  For a stored
// group prefix P < n/8 (the tuples 4P .. 4P + 3 share all but their last
// slot (a_l, b_l)):
//   Ma[2P + b] = (T[4P + b] + T[4P + 2 + b]) * 1/2   the mean over a_l: what
//                an advance-a branch reads (eq. (3) with string 1 moved)
//   Mab[P]     = ((T[4P] + T[4P+3]) + (T[4P+1] + T[4P+2])) * 1/4
//                the all-advance mean, in the complement-paired tree
// Both are the means the entry-reading sweep forms, so a sweep that reads
// them computes the same bits.  The advance-b mean over b_l of s is the
// advance-a mean of the exchanged tuple; a tuple with string-1 head 1 is read
// at its complement (the last b bit flips, a two-term sum does not care).
__host__ __device__ inline uint64_t ma_index(uint64_t s, uint64_t n)
{
    if (s & (n >> 1)) s ^= n - 1;
    return ((s >> 2) << 1) | (s & 1);
}
__host__ __device__ inline uint64_t mab_index(uint64_t s, uint64_t n)
{
    if (s & (n >> 1)) s ^= n - 1;
    return s >> 2;
}

// sigma = 2, d = 3 (slot bits s1 s2 s3, s1 most significant; stored tuples
// s < n/2, n = 8^l).  For a stored group prefix P < n/16 (entries 8P .. 8P+7,
// member u = the last slot) the branch means, each the entry sweep's own:
//   M1[4P + (u & 3)]   mean over s1 of members u, u + 4      (moves string 1)
//   M3[4P + (u >> 1)]  mean over s3 of members u, u + 1      (string 3)
//   M12[2P + s3]       pair tree over (s1 s2) of 8P + s3 + {0, 2, 4, 6}  (strings 1, 2)
//   M23[2P + s1]       pair tree over (s2 s3) of 8P + 4 s1 + {0, 1, 2, 3} (strings 2, 3)
//   M123[P]            the eight-member pair tree                 (all three)
// On a table symmetric in strings 1 and 2 the string-2 mean is M1 at the
// exchanged tuple and the (s1 s3) mean is M23 at the exchanged tuple; M3, M12
// and M123 are exchange-symmetric and kept at the lower index of each
// exchanged pair.  An index with string-1 head 1 is read at its complement.
__host__ __device__ inline uint64_t d3_fold(uint64_t s, uint64_t n) { return (s & (n >> 1)) ? s ^ (n - 1) : s; }
__host__ __device__ inline uint64_t m1_index(uint64_t s, uint64_t n)
{
    s = d3_fold(s, n);
    return ((s >> 3) << 2) | (s & 3);
}
__host__ __device__ inline uint64_t m3_index(uint64_t s, uint64_t n) { return d3_fold(s, n) >> 1; }
__host__ __device__ inline uint64_t m12_index(uint64_t s, uint64_t n)
{
    s = d3_fold(s, n);
    return ((s >> 3) << 1) | (s & 1);
}
__host__ __device__ inline uint64_t m23_index(uint64_t s, uint64_t n)
{
    s = d3_fold(s, n);
    return ((s >> 3) << 1) | ((s >> 2) & 1);
}
__host__ __device__ inline uint64_t m123_index(uint64_t s, uint64_t n) { return d3_fold(s, n) >> 3; }

// sigma = 4, d = 2 (slot = a: 2 bits high, b: 2 bits low; stored tuples have
// string-1 head 0, n = 16^l).  For a stored group prefix P < n/64 (entries
// 16P .. 16P+15, member u = 4 a_l + b_l):
//   M4a[4P + b]  tree4 over a_l of members 4a + b      (advance a)
//   M4ab[P]      the sixteen-member tree of the group    (advance both)
// The advance-b mean (over b_l) is M4a at the exchanged tuple; M4ab is
// exchange-symmetric and kept at the lower prefix of each exchanged pair.
// An index whose string-1 head is m is read at its relabelling by m.
__host__ __device__ inline uint64_t s4_fold(uint64_t s, uint64_t n)
{
    const uint64_t m = (s >> (63 - __builtin_clzll(n) - 2)) & 3;
    return s ^ (m * ((n - 1) / 3));
}
__host__ __device__ inline uint64_t m4a_index(uint64_t s, uint64_t n)
{
    s = s4_fold(s, n);
    return ((s >> 4) << 2) | (s & 3);
}
__host__ __device__ inline uint64_t m4ab_index(uint64_t s, uint64_t n) { return s4_fold(s, n) >> 4; }

struct MeansLaunch {
    const void *ma1;   // Ma of lag 1
    const void *mab2;  // Mab of lag 2
    void *out;         // the new table's entries, or null: not written this sweep
    void *ma_new, *mab_new;
    double *offsets;   // device, per slot (FP32)
    int s1, s2, snew;  // offset slots of lag 1, lag 2 and the new table
    int shift;         // FP64: lag 2 read with delta = offsets[s2] - offsets[s1] (two arrays)
};
// Entries of lag 1 and lag 2 are not read.  FP32 tables (and their means)
// are relative to their slot's offset, as in launch_sweep.
hipError_t launch_sweep_means(const Geometry &g, int dtype, const MeansLaunch &a, hipStream_t s);
// The values the sweep of `a` writes at the 4096 coordinates the two-array
// rate samples (the lower index of each sampled coordinate's exchanged
// pair), in sample order, computed from the same means with the same
// arithmetic; launched after that sweep, before the rate pass
hipError_t launch_means_samples(const Geometry &g, int dtype, const MeansLaunch &a, void *samples,
                                hipStream_t s);
// Ma and Mab of a stored table (lazy: only the lower index of each exchanged
// pair holds a value, see TwinGroup)
hipError_t launch_derive_means(const Geometry &g, int dtype, const void *table, int lazy,
                               void *ma, void *mab, hipStream_t s);

// The same for sigma = 2, d = 3 (m1_index .. m123_index): lag 1's M1 and M3,
// lag 2's M12 and M23, lag 3's M123 read; the new table's five written
struct Means3Launch {
    const void *m1, *m3, *m12, *m23, *m123;
    void *out;  // the new table's entries, or null
    void *n1, *n3, *n12, *n23, *n123;
    double *offsets;
    int s1, s2, s3, snew;
    int shift;  // FP64: lags 2 and 3 read with their offset differences (two arrays)
};
hipError_t launch_sweep_means3(const Geometry &g, int dtype, const Means3Launch &a, hipStream_t s);
// the two-array rate's sample values of the table launch_sweep_means3 computes
// from the same means (in sample order, kRateSample values)
hipError_t launch_means_samples3(const Geometry &g, int dtype, const Means3Launch &a,
                                 void *samples, hipStream_t s);
// sigma = 4, d = 2 (m4a_index, m4ab_index): lag 1's M4a and lag 2's M4ab
// read, the new table's written (MeansLaunch: ma = M4a, mab = M4ab)
hipError_t launch_sweep_means4(const Geometry &g, int dtype, const MeansLaunch &a, hipStream_t s);
hipError_t launch_derive_means4(const Geometry &g, int dtype, const void *table, int lazy, void *ma,
                                void *mab, hipStream_t s);
hipError_t launch_derive_means3(const Geometry &g, int dtype, const void *table, int lazy, void *m1,
                                void *m3, void *m12, void *m23, void *m123, hipStream_t s);

// Certificate passes (see lcsb_cert); results land in the workspace scalars.
// swap_sym: as in SweepLaunch (the W pass then evaluates one coordinate per
// exchange pair)
hipError_t launch_certify(const Geometry &g, int dtype, const void *u, const void *prev,
                          int u_slot, int prev_slot, int swap_sym, unsigned char *ws,
                          hipStream_t s);

// The largest-r certificate of u (kOptR, kOptArg, kOptNonfinite).
hipError_t launch_certify_optimal(const Geometry &g, int dtype, const void *u, int swap_sym,
                                  unsigned char *ws, hipStream_t s);

// The same for an exchange-packed sigma = d = 2 table (packed_index), l >= 2
hipError_t launch_certify_optimal_packed(const Geometry &g, int dtype, const void *u,
                                         unsigned char *ws, hipStream_t s);

// The same, its result written to out (4 doubles: r, d r rounded down, and
// the lowest minimising index and the non-finite count as uint64 bits)
hipError_t launch_certify_optimal_out(const Geometry &g, int dtype, const void *u, int swap_sym,
                                      unsigned char *ws, double *out, hipStream_t s);

// lcsb_certify_optimal_noalloc without the error-message plumbing (csrc/noalloc.hip)
int certify_optimal_noalloc(int sigma, int d, int h, int dtype, const void *u,
                            int exchange_symmetric, double *dev_out, void *stream,
                            std::string *err);

// The two-array iteration: R = mean over the fixed sample of nw - old, and the
// offsets slots kSlotLag2/3 for the next sweep (csrc/two_array.hip)
// packed: the two tables are exchange-packed (sigma = d = 2)
// nw_smp / old_smp (optional): the tables' values at the sample, in sample
// order (launch_means_samples), read instead of the tables
hipError_t launch_two_array_rate(const Geometry &g, int dtype, const void *nw, const void *old,
                                 int s_new, int s_old, int swap_sym, int packed,
                                 unsigned char *ws, hipStream_t s, const void *nw_smp = nullptr,
                                 const void *old_smp = nullptr);
constexpr int kRateSample = 4096;  // coordinates of the two-array rate
constexpr uint64_t kRateSampleMul = 0x9E3779B97F4A7C15ull;

// Utilities
hipError_t launch_fill_zero(void *p, uint64_t bytes, hipStream_t s);
hipError_t launch_fill_f64(double *p, uint64_t count, double v, hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, uint64_t bytes, hipStream_t s);
// sigma = 2 with d = 2 or 3, or sigma = 4 with d = 2, l >= 2: set *flag
// (device) to 1 unless every stored entry equals, bit for bit, the stored
// entry of its tuple with strings 1 and 2 exchanged
hipError_t launch_check_swap(const Geometry &g, int dtype, const void *table, uint32_t *flag,
                             hipStream_t s);
// a lazily written table (see TwinGroup): set every upper entry to its lower twin
hipError_t launch_materialize_swap(const Geometry &g, int dtype, void *table, hipStream_t s);
hipError_t launch_upcast(const Geometry &g, const float *src, const double *offset_dev,
                         double *dst, hipStream_t s);
// the FP32 table in the first half of an FP64-sized buffer, widened in place
hipError_t launch_upcast_inplace(const Geometry &g, void *buf, const double *offset_dev,
                                 hipStream_t s);

// sigma = d = 2 rings symmetric in the two strings are written lazily: of the
// exchanged pair {j, J(j)} of stored entries (J swaps the a and b bits of
// every slot, then complements when that makes the string-1 head 1) only the
// lower index is kept.  An aligned group of four shares its prefix, so it is
// entirely lower (read as is), entirely upper (read at its twin group, member
// v at position perm(v): perm swaps 1 and 2 for heads 0/0 and 0 and 3 for
// heads 0/1), or its own twin (each upper member read at its lower partner).
struct TwinGroup {
    uint64_t read;  // base of the group to load
    int mode;       // 0 own, 1 twin (0/0), 2 twin (0/1), 3 self (0/0), 4 self (0/1)
};

__host__ __device__ inline TwinGroup twin_group(uint64_t base, uint64_t n)
{
    const uint64_t full = n - 1, am = 0xAAAAAAAAAAAAAAAAull & full;
    const uint64_t x = ((base & am) >> 1) | ((base & ~am & full) << 1);
    const bool h01 = (x & (n >> 1)) != 0;  // the exchange moved a head 1 to string 1
    const uint64_t jb = h01 ? x ^ (full & ~(uint64_t)3) : x;
    if (jb > base) return {base, 0};
    if (jb < base) return {jb, h01 ? 2 : 1};
    return {base, h01 ? 4 : 3};
}

// the group's four values, in its own member order, from the loaded q
template <typename T>
__device__ __forceinline__ void twin_values(const T *q, int mode, T *g)
{
    g[0] = mode == 2 ? q[3] : q[0];
    g[1] = mode == 1 ? q[2] : q[1];
    g[2] = (mode == 1 || mode == 3) ? q[1] : q[2];
    g[3] = (mode == 2 || mode == 4) ? q[0] : q[3];
}

// The same for sigma = 2, d = 3 with strings 1 and 2 exchanged: J swaps the
// string-1 and string-2 bits of every 3-bit slot, then complements when that
// makes the string-1 head 1.  Groups are aligned runs of eight (the last
// slot, members c1 c2 c3); a twin group holds member v at PE[v] (c1 and c2
// swapped) or, when J complements, at 7 - PE[v].
__host__ __device__ inline uint64_t exchange12(uint64_t x, uint64_t n)
{
    const uint64_t r3 = (n - 1) / 7;  // bit 0 of every slot
    return (x & r3) | ((x & (r3 << 2)) >> 1) | ((x & (r3 << 1)) << 1);
}

// J for d = 2 (bits of each 2-bit slot swapped) or d = 3 (exchange12), folded
__host__ __device__ inline uint64_t exchange_twin(uint64_t j, uint64_t n, int d)
{
    uint64_t x;
    if (d == 2) {
        const uint64_t am = 0xAAAAAAAAAAAAAAAAull & (n - 1);
        x = ((j & am) >> 1) | ((j & ~am & (n - 1)) << 1);
    } else {
        x = exchange12(j, n);
    }
    return (x & (n >> 1)) ? x ^ (n - 1) : x;
}

__host__ __device__ inline TwinGroup twin_group8(uint64_t base, uint64_t n)
{
    const uint64_t x = exchange12(base, n);
    const bool h1 = (x & (n >> 1)) != 0;
    const uint64_t jb = h1 ? x ^ ((n - 1) & ~(uint64_t)7) : x;
    if (jb > base) return {base, 0};
    if (jb < base) return {jb, h1 ? 2 : 1};
    return {base, h1 ? 4 : 3};
}

// the group's eight values, in its own member order, from the loaded q:
// mode 1 q[PE[v]], 2 q[7 - PE[v]], 3 q[min(v, PE[v])], 4 q[min(v, 7 - PE[v])],
// PE = {0, 1, 4, 5, 2, 3, 6, 7}
template <typename T>
__device__ __forceinline__ void twin_values8(const T *qm, int mode, T *g)
{
    // the values as registers: otherwise the compiler may turn the selects
    // below into one load from a private copy of q at a computed offset
    T q[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        q[v] = qm[v];
        asm volatile("" : "+v"(q[v]));
    }
    g[0] = mode == 2 ? q[7] : q[0];
    g[1] = mode == 2 ? q[6] : q[1];
    g[2] = (mode == 1) ? q[4] : mode == 2 ? q[3] : q[2];
    g[3] = (mode == 1) ? q[5] : mode == 2 ? q[2] : mode == 4 ? q[2] : q[3];
    g[4] = (mode == 1 || mode == 3) ? q[2] : mode == 2 ? q[5] : q[4];
    g[5] = (mode == 1 || mode == 3) ? q[3] : (mode == 2 || mode == 4) ? q[4] : q[5];
    g[6] = mode == 2 ? q[1] : mode == 4 ? q[1] : q[6];
    g[7] = (mode == 2 || mode == 4) ? q[0] : q[7];
}

// sigma = 4, d = 2 with the two strings exchanged: exchange4 swaps the a and
// b symbols (2-bit fields) of every 4-bit slot, and J relabels the result by
// its string-1 head so that it is a stored index.  An aligned group of
// sixteen (the last slot, member v = 4 c1 + c2) is its own (kind 0), lies at
// its twin group with member v at perm16(v, m) (kind 1, m the relabelling),
// or is its own twin (kind 2: member v read at min(v, perm16(v, m))).
__host__ __device__ inline uint64_t exchange4(uint64_t x, uint64_t n)
{
    const uint64_t a = 0xCCCCCCCCCCCCCCCCull & (n - 1), b = 0x3333333333333333ull & (n - 1);
    return ((x & a) >> 2) | ((x & b) << 2);
}

__host__ __device__ inline uint64_t exchange_twin4(uint64_t j, uint64_t n)
{
    const uint64_t x = exchange4(j, n);
    const uint64_t m = (x >> (__builtin_ctzll(n) - 2)) & 3;  // string-1 head of x
    return x ^ (m * ((n - 1) / 3));
}

struct Twin16 {
    uint64_t read;  // base of the twin group (kind 1), else the group's own
    int m;          // relabelling of the twin
    int kind;       // 0 own, 1 twin, 2 self
};

__host__ __device__ inline Twin16 twin_group16(uint64_t base, uint64_t n)
{
    const uint64_t x = exchange4(base, n);
    const int m = (int)((x >> (__builtin_ctzll(n) - 2)) & 3);
    const uint64_t jb = (x ^ ((uint64_t)m * ((n - 1) / 3))) & ~(uint64_t)15;
    if (jb > base) return {base, m, 0};
    if (jb < base) return {jb, m, 1};
    return {base, m, 2};
}

__host__ __device__ inline int perm16(int v, int m) { return 4 * ((v & 3) ^ m) + ((v >> 2) ^ m); }

// stored position holding member v of the group at `base` (tw = its twin)
__host__ __device__ inline uint64_t member16(uint64_t base, const Twin16 &tw, int v)
{
    if (tw.kind == 0) return base + (uint64_t)v;
    const int pv = perm16(v, tw.m);
    if (tw.kind == 1) return tw.read + (uint64_t)pv;
    return base + (uint64_t)(pv < v ? pv : v);
}

// ---------------------------------------------------------------- packed tables
// Exchange-packed storage for sigma = d = 2: one entry per orbit of the tuple
// (a, b) under complementing both strings and exchanging them (a table of an
// exchange-symmetric ring is constant on each orbit).  With c = a xor b, which
// both maps keep, the complement sends a to ~a and the exchange a to a xor c,
// so an orbit is a coset of {0, c, 1..1, ~c} among the a strings.  Its
// representative has a_1 = 0 and, with c'' = c (c_1 = 0) or ~c (c_1 = 1) and
// p the first position j >= 2 where c''_j = 1, a_p = 0.  Code, 2l - 2 bits
// from the top: c_1, c_2, then (a_j, c_j) for j = 3..l, where the a bit of
// position p holds a_2 instead (for p = 2 every position holds its own).
// The orbits with c'' = 0 (b = a or b = ~a) have no p: they take the codes
// n/4 + c_1 2^(l-1) + (a_2 .. a_l).  Codes below n/4 whose c'' is 0 belong to
// no orbit and are never read or written.  The last position's pair is the
// code's lowest two bits, so the four tuples that append one symbol to each
// string (an aligned group of four standard indices) sit at four
// consecutive codes whenever p < l.
//
// In the index arithmetic below, q is a standard index with the string-2
// bit of every position replaced by c_j = a_j xor b_j (a_j at the odd bit
// 2(l-j)+1, c_j at the even bit 2(l-j)).

__host__ __device__ inline uint64_t packed_entries(int h)
{
    return (1ull << (2 * h - 2)) + (1ull << h);
}

constexpr uint64_t kNoOrbit = ~0ull;  // packed_tuple of a code that belongs to no orbit

// packed_index of member v of the aligned group at index 0 (every position
// 0/0 but the last, which is (a_l, b_l) = (v >> 1, v & 1)): 0/0 and 1/1 leave
// c = 0, degenerate orbits with a_2..a_l = 0 and 1; 0/1 and 1/0 are exchange
// twins whose pivot is the last position, the code of the tuple with b_l = 1
__host__ __device__ inline uint64_t packed_zero_group(int v, int h)
{
    const uint64_t nq = 1ull << (2 * h - 2);
    return v == 0 ? nq : v == 3 ? nq + 1 : 1;
}

// (a_2 .. a_l) of q as an (l-1)-bit number (a_1 ignored)
__host__ __device__ inline uint64_t packed_odd_bits(uint64_t q, int h)
{
    uint64_t x = (q >> 1) & 0x5555555555555555ull & ((1ull << (2 * h - 2)) - 1);
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    return x;
}

// the inverse: bit j of x to the odd bit 2j + 1
__host__ __device__ inline uint64_t packed_spread_odd(uint64_t x)
{
    x &= 0x00000000FFFFFFFFull;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x << 1;
}

// the code of standard index i (any of the 4^l tuples)
__host__ __device__ inline uint64_t packed_index(uint64_t i, int h)
{
    const uint64_t n = 1ull << (2 * h), A = 0xAAAAAAAAAAAAAAAAull & (n - 1), B = A >> 1;
    uint64_t q = (i & A) | ((i ^ (i >> 1)) & B);
    if (q >> (2 * h - 1)) q ^= A;                     // complement: a_1 = 0
    const uint64_t c1 = (q >> (2 * h - 2)) & 1;
    const uint64_t cc = (q & B) ^ (c1 ? B : 0);       // c'' (its top bit is 0)
    if (cc == 0) return (n >> 2) + (c1 << (h - 1)) + packed_odd_bits(q, h);
    const int pos = 63 - __builtin_clzll(cc);         // the even bit of c''_p
    if ((q >> (pos + 1)) & 1) q ^= cc << 1;           // exchange: a_p = 0
    if (pos < 2 * h - 4) q |= ((q >> (2 * h - 3)) & 1) << (pos + 1);  // a_2 into p's slot
    return (c1 << (2 * h - 3)) | (q & ((1ull << (2 * h - 3)) - 1));
}

// the representative's standard index (a_1 = 0, so a stored index) of code
// k, or kNoOrbit
__host__ __device__ inline uint64_t packed_tuple(uint64_t k, int h)
{
    const uint64_t n = 1ull << (2 * h), A = 0xAAAAAAAAAAAAAAAAull & (n - 1), B = A >> 1;
    const uint64_t nq = n >> 2;
    uint64_t q;
    if (k >= nq) {
        const uint64_t r = k - nq, c1 = (r >> (h - 1)) & 1;
        q = packed_spread_odd(r & ((1ull << (h - 1)) - 1)) | (c1 ? B : 0);
    } else {
        const uint64_t c1 = k >> (2 * h - 3);
        q = (c1 << (2 * h - 2)) | (k & ((1ull << (2 * h - 3)) - 1));
        const uint64_t cc = (q & B) ^ (c1 ? B : 0);
        if (cc == 0) return kNoOrbit;
        const int pos = 63 - __builtin_clzll(cc);
        if (pos < 2 * h - 4) {
            const uint64_t a2 = (q >> (pos + 1)) & 1;
            q = (q & ~(1ull << (pos + 1))) | (a2 << (2 * h - 3));
        }
    }
    const uint64_t a = q & A;
    return a | ((a >> 1) ^ (q & B));
}

// Where the aligned group of four standard indices at gbase (low two bits 0)
// lives: when the group's pivot lies above the last position (regular) its
// member v = 2 alpha + beta is at code base + ((alpha ^ u0 ^ (u1 & g)) << 1 | g),
// g = alpha ^ beta; otherwise each member is looked up on its own.
struct PackedGroup {
    uint64_t base;
    int u0, u1;
    bool regular;
};

__host__ __device__ inline PackedGroup packed_group(uint64_t gbase, int h)
{
    const uint64_t n = 1ull << (2 * h), A = 0xAAAAAAAAAAAAAAAAull & (n - 1), B = A >> 1;
    uint64_t q = (gbase & A) | ((gbase ^ (gbase >> 1)) & B);
    const int comp = (int)((q >> (2 * h - 1)) & 1);
    if (comp) q ^= A;
    const uint64_t c1 = (q >> (2 * h - 2)) & 1;
    const uint64_t cc = ((q & B) ^ (c1 ? B : 0)) & ~(uint64_t)3;  // c'' above the last position
    if (cc == 0) return {0, 0, 0, false};
    const int pos = 63 - __builtin_clzll(cc);
    const int flip = (int)((q >> (pos + 1)) & 1);
    if (flip) q ^= (cc | (c1 ? 1 : 0)) << 1;  // a xor c'' (c''_l of member 0 = c1)
    if (pos < 2 * h - 4) q |= ((q >> (2 * h - 3)) & 1) << (pos + 1);
    const uint64_t code0 = (c1 << (2 * h - 3)) | (q & ((1ull << (2 * h - 3)) - 1));
    return {code0 & ~(uint64_t)3, comp ^ (flip & (int)c1), flip, true};
}

__host__ __device__ inline int packed_member(const PackedGroup &pg, int v)
{
    const int alpha = v >> 1, g = (v >> 1) ^ (v & 1);
    return ((alpha ^ pg.u0 ^ (pg.u1 & g)) << 1) | g;
}

// Learned warm start (csrc/mlp.hip)
struct MlpWs {  // byte offsets inside the caller's training workspace
    size_t act, X, dZ, T1, WT, part, bytes;
    int splits;
};
MlpWs mlp_ws_layout(int64_t batch);
hipError_t launch_mlp_forward(const uint16_t *wb, const float *pf, const uint64_t *idx, int h,
                              int64_t count, float *y, uint16_t *act, hipStream_t s);
hipError_t launch_mlp_seed(const Geometry &g, int dtype, const uint16_t *wb, const float *pf,
                           void *lag1, void *lag2, double rate, hipStream_t s);
hipError_t launch_mlp_backward(const uint16_t *wb, const float *dy, int64_t count,
                               unsigned char *ws, const MlpWs &L, const uint64_t *idx, int h,
                               float *grad, hipStream_t s);
hipError_t launch_mlp_mse(const float *y, const float *t, int64_t count, float *dy, double *loss,
                          hipStream_t s);
hipError_t launch_mlp_adam(float *p, uint16_t *wb, const float *g, float *m, float *v, float lr,
                           float b1, float b2, float eps, int64_t t, hipStream_t s);
hipError_t launch_to_bf16(const float *p, uint16_t *wb, hipStream_t s);
hipError_t launch_mlp_init(float *p, uint64_t seed, hipStream_t s);
hipError_t launch_mlp_sample(const void *table, int dtype, int bits, uint64_t seed, int64_t count,
                             uint64_t *idx, float *target, hipStream_t s);

}  // namespace lcsb
