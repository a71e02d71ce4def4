// Host-side check of the library's exchange-fold index arithmetic
// (paper_2407_10925_amd/csrc/internal.h): every grouped fast path the
// kernels take agrees, entry by entry, with the plain rule "a stored entry
// stands for itself and its exchanged twin, and the lower index of the two
// holds the value".  Exits non-zero on the first disagreement.
#include "internal.h"

#include <cstdio>

using namespace lcsb;

static long bad = 0;
#define EXPECT(c, ...)                                  \
    do {                                                \
        if (!(c) && bad++ < 8) {                        \
            printf("FAIL %s:%d: ", __FILE__, __LINE__); \
            printf(__VA_ARGS__);                        \
            printf("\n");                               \
        }                                               \
    } while (0)

static uint64_t lower(uint64_t j, uint64_t tw) { return tw < j ? tw : j; }

// Group bases to visit: every one (step 0), or `count` of them spread by a
// multiplicative hash plus the first and last groups of the stored range
// (large l, where the stored range passes 2^31 and 2^32).
struct Bases {
    uint64_t ns, G, count;
    uint64_t size() const { return count ? count + 2 : ns / G; }
    uint64_t operator[](uint64_t k) const
    {
        if (!count) return k * G;
        if (k == count) return 0;
        if (k == count + 1) return ns - G;
        return ((k * 0x9E3779B97F4A7C15ull) % (ns / G)) * G;
    }
};

// d = 2 (sigma = 2) and d = 3: a TwinGroup's mode and member mapping
template <int D>
static void groups(int h, uint64_t count = 0)
{
    const int G = D == 2 ? 4 : 8;
    const uint64_t n = 1ull << (D * h), ns = n / 2;
    const Bases bases{ns, (uint64_t)G, count};
    for (uint64_t k = 0; k < bases.size(); ++k) {
        const uint64_t base = bases[k];
        const TwinGroup tg = D == 2 ? twin_group(base, n) : twin_group8(base, n);
        for (int v = 0; v < G; ++v) {
            const uint64_t j = base + v, js = exchange_twin(j, n, D);
            EXPECT(js < ns, "d=%d h=%d j=%llu: twin not stored", D, h, (unsigned long long)j);
            EXPECT(exchange_twin(js, n, D) == j, "d=%d h=%d j=%llu: not an involution", D, h,
                   (unsigned long long)j);
            if (tg.mode == 0) EXPECT(js > j, "d=%d own group holds an upper entry", D);
            if (tg.mode == 1 || tg.mode == 2) {
                EXPECT(js < j, "d=%d twin group holds a lower entry", D);
                EXPECT(js >= tg.read && js < tg.read + G, "d=%d twin outside the twin group", D);
            }
            if (tg.mode >= 3) EXPECT(js >= base && js < base + G, "d=%d self group leaves itself", D);
        }
        if (D == 3) {  // the member lookup the folded d = 3 kernels use
            for (int v = 0; v < 8; ++v) {
                const uint64_t j = base + v;
                const int pe = (v & 1) | ((v & 2) << 1) | ((v & 4) >> 1);
                const int at = tg.mode == 0 ? v
                             : tg.mode == 1 ? pe
                             : tg.mode == 2 ? 7 - pe
                             : tg.mode == 3 ? (v < pe ? v : pe)
                                            : (v < 7 - pe ? v : 7 - pe);
                EXPECT(tg.read + at == lower(j, exchange_twin(j, n, 3)), "d=3 h=%d member %d", h, v);
            }
        }
    }
}

// sigma = 4, d = 2: Twin16 and member16, the vector-load addresses of the
// folded sweep, and the grouped R pass
static void sigma4(int h, uint64_t count = 0)
{
    const uint64_t n = 1ull << (4 * h), ns = n / 4;
    const Bases bases{ns, 16, count};
    for (uint64_t k = 0; k < bases.size(); ++k) {
        const uint64_t base = bases[k];
        const Twin16 tw = twin_group16(base, n);
        for (int v = 0; v < 16; ++v) {
            const uint64_t j = base + v, js = exchange_twin4(j, n);
            EXPECT(js < ns && exchange_twin4(js, n) == j, "sigma=4 h=%d: twin not a stored involution", h);
            EXPECT(member16(base, tw, v) == lower(j, js), "sigma=4 h=%d member %d", h, v);
            if (tw.kind == 0) EXPECT(js > j, "sigma=4 own group holds an upper entry");
            if (tw.kind == 1) EXPECT(js < j, "sigma=4 twin group holds a lower entry");
        }
        for (int o = 0; o < 4; ++o) {
            // advance a: members o + 4k of a twin group are one row of it
            if (tw.kind == 1)
                for (int k = 0; k < 4; ++k)
                    EXPECT(member16(base, tw, o + 4 * k) ==
                               tw.read + 4 * (uint64_t)(o ^ tw.m) + (uint64_t)(k ^ tw.m),
                           "sigma=4 advance-a row");
            // advance b: members 4o .. 4o + 3 of an own group are in place
            if (tw.kind == 0)
                for (int k = 0; k < 4; ++k)
                    EXPECT(member16(base, tw, 4 * o + k) == base + 4 * (uint64_t)o + k, "sigma=4 advance-b run");
        }
    }
}

// Exchange-packed tables (sigma = d = 2): every tuple's code is below
// packed_entries, the code's representative lies in the tuple's orbit
// {i, ~i, E i, ~E i} with a_1 = 0 and has the same code, every code that
// belongs to an orbit is the code of its representative, distinct orbits get
// distinct codes, and a regular group's member positions agree with the
// per-tuple code.  `count` > 0: that many hashed groups (plus the first and
// last) instead of all, and no distinctness count.
static uint64_t exchange2(uint64_t i, uint64_t n)
{
    const uint64_t am = 0xAAAAAAAAAAAAAAAAull & (n - 1);
    return ((i & am) >> 1) | ((i & ~am & (n - 1)) << 1);
}

static void packed(int h, uint64_t count = 0)
{
    const uint64_t n = 1ull << (2 * h), ne = packed_entries(h);
    const Bases bases{n, 4, count};
    for (uint64_t k = 0; k < bases.size(); ++k) {
        const uint64_t gb = bases[k];
        const PackedGroup pg = packed_group(gb, h);
        for (int v = 0; v < 4; ++v) {
            const uint64_t i = gb + v, code = packed_index(i, h);
            EXPECT(code < ne, "h=%d i=%llu: code out of range", h, (unsigned long long)i);
            const uint64_t t = packed_tuple(code, h);
            const uint64_t e = exchange2(i, n);
            const bool in_orbit = t == i || t == (i ^ (n - 1)) || t == e || t == (e ^ (n - 1));
            EXPECT(t != kNoOrbit && in_orbit, "h=%d i=%llu: representative %llu not in the orbit",
                   h, (unsigned long long)i, (unsigned long long)t);
            EXPECT(t < n / 2, "h=%d: representative not stored", h);
            EXPECT(packed_index(t, h) == code, "h=%d i=%llu: representative's code differs", h,
                   (unsigned long long)i);
            if (pg.regular)
                EXPECT(pg.base + (uint64_t)packed_member(pg, v) == code,
                       "h=%d group %llu member %d: regular position differs", h,
                       (unsigned long long)gb, v);
        }
    }
    for (int v = 0; v < 4; ++v)
        EXPECT(packed_zero_group(v, h) == packed_index((uint64_t)v, h),
               "h=%d: zero group member %d", h, v);
    if (count) return;
    uint64_t valid = 0;
    for (uint64_t code = 0; code < ne; ++code) {
        const uint64_t t = packed_tuple(code, h);
        if (t == kNoOrbit) continue;
        ++valid;
        EXPECT(packed_index(t, h) == code, "h=%d code %llu: not the code of its representative",
               h, (unsigned long long)code);
    }
    // orbits: (n + fixed points of E + fixed points of ~E) / 4, E and ~E
    // each fixing 2^l tuples (b = a, b = ~a), the complement none
    EXPECT(valid == (n + 2 * (1ull << h)) / 4, "h=%d: %llu codes in use, expected %llu", h,
           (unsigned long long)valid, (unsigned long long)((n + 2 * (1ull << h)) / 4));
}

int main()
{
    for (int h = 2; h <= 10; ++h) packed(h);
    for (int h = 11; h <= 18; ++h) packed(h, 1u << 18);
    for (int h = 2; h <= 10; ++h) groups<2>(h);
    for (int h = 2; h <= 7; ++h) groups<3>(h);
    for (int h = 2; h <= 5; ++h) sigma4(h);
    // sampled groups at the sizes the benchmarks and the l = 17 runs use
    // (stored ranges up to 2^33 entries)
    for (int h = 11; h <= 17; ++h) groups<2>(h, 1u << 18);
    for (int h = 8; h <= 12; ++h) groups<3>(h, 1u << 18);
    for (int h = 6; h <= 9; ++h) sigma4(h, 1u << 18);
    printf("%s (%ld disagreements)\n", bad ? "FAIL" : "ok", bad);
    return bad != 0;
}
