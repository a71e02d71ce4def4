// Host-side check of the library's exchange-fold index arithmetic
// (paper_2407_10925_amd/csrc/internal.h): every grouped fast path the
// kernels take agrees, entry by entry, with the plain rule "a stored entry
// stands for itself and its exchanged twin, and the lower index of the two
// holds the value".  Exits non-zero on the first disagreement.
#include "internal.h"

#include <cstdio>
#include <vector>

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

// Branch-mean tables (sigma = d = 2, rings symmetric in the two strings):
// on a table that gives every orbit of the complement and the exchange one
// pseudo-random integer (an all-match tuple one for its tail's orbit, as a
// sweep's output has; so every mean below is exact), the means the
// branch-mean sweep reads (its v = 0 index plus the fixed offsets {0, 1, 4,
// 5} and {0, 4, 1, 5}, descending where stated) equal the means the
// entry-reading sweep forms, every index it reads or writes is in range, the
// entries and means it writes (its own groups' and the exchanged quad's)
// equal their definitions, and, over all quads, the writes cover Ma and every
// Mab entry a sweep reads (the lower prefix of each exchanged pair).  `count` > 0: that many hashed quads (plus the first and last).
static double orbit_value(uint64_t s, uint64_t n)
{
    // all-match heads: the value depends only on the tail (in its orbit)
    const bool match = ((s >> 1) ^ s) & (n >> 2) ? false : true;
    if (match) s &= (n >> 2) - 1;  // the tail, flagged apart below
    const uint64_t m = match ? (n >> 2) - 1 : n - 1;
    const uint64_t am = 0xAAAAAAAAAAAAAAAAull & m;
    const uint64_t e = ((s & am) >> 1) | ((s & ~am & m) << 1), c = s ^ m, ec = e ^ m;
    uint64_t r = s < c ? s : c;
    r = r < e ? r : e;
    r = r < ec ? r : ec;
    if (match) r |= 1ull << 62;
    uint64_t z = (r + 0x9E3779B97F4A7C15ull) * 0xBF58476D1CE4E5B9ull;
    z ^= z >> 29;
    return (double)(z & 0xFFFF);
}

static void means(int h, uint64_t count = 0)
{
    const uint64_t n = 1ull << (2 * h), nq = n / 4, n16 = n / 16, mq = n16 - 1;
    const uint64_t alt = 0xAAAAAAAAAAAAAAAAull;
    const uint64_t am = alt & (n - 1), bm = ~alt & (n - 1), qa = alt & mq;
    auto T = [&](uint64_t s) { return orbit_value(s, n); };
    auto ma_def = [&](uint64_t k) {
        const uint64_t P = k >> 1, b = k & 1;
        return (T(4 * P + b) + T(4 * P + 2 + b)) * 0.5;
    };
    auto mab_def = [&](uint64_t P) {
        return ((T(4 * P) + T(4 * P + 3)) + (T(4 * P + 1) + T(4 * P + 2))) * 0.25;
    };
    std::vector<char> wa(count ? 0 : n / 4), wab(count ? 0 : n / 8);
    std::vector<uint64_t> need_ab;
    const uint64_t quads = n >> 5;
    const uint64_t visits = count ? count + 2 : quads;
    for (uint64_t k = 0; k < visits; ++k) {
        const uint64_t j = !count ? k : k == count ? 0 : k == count + 1 ? quads - 1
                                                   : (k * 0x9E3779B97F4A7C15ull) % quads;
        const uint64_t sj = ((j & qa) >> 1) | ((j & ~qa & mq) << 1);
        const bool b2 = (j & (n16 >> 2)) != 0;
        const uint64_t pj = b2 ? sj ^ mq : sj;
        if (pj < j) continue;
        // reads
        double a[4], b[4], c[4];
        for (int v = 0; v < 4; ++v) {
            const uint64_t t = 4 * j + (uint64_t)v;
            EXPECT(t < n / 8, "h=%d: all-advance mean index %llu out of range", h, (unsigned long long)t);
            // Mab is kept at the lower prefix of each exchanged pair: t is
            // lower, or (a quad that is its own twin) its partner lies in the
            // same quad at perm(v) < v
            const uint64_t tw = mab_index(exchange_twin(4 * t, n, 2), n);
            const int sv = ((v & 1) << 1) | (v >> 1), pv = b2 ? 3 - sv : sv;
            EXPECT(tw >= t || (pj == j && tw == 4 * j + (uint64_t)pv && pv < v),
                   "h=%d j=%llu v=%d: all-advance mean not at a kept prefix", h, (unsigned long long)j, v);
            if (!count) need_ab.push_back(tw < t ? tw : t);
            const double want = ((T(4 * t) + T(4 * t + 3)) + (T(4 * t + 1) + T(4 * t + 2))) * 0.25;
            EXPECT(mab_def(t) == want, "h=%d t=%llu: all-advance mean", h, (unsigned long long)t);
            a[v] = T(t);
        }
        for (int cc = 0; cc < 2; ++cc) {
            const uint64_t i0 = nq + (cc ? nq - 1 - 4 * j : 4 * j);
            const uint64_t ia = ma_index(((i0 << 2) & am) | (i0 & bm), n);
            const uint64_t ib = ma_index(exchange_twin((i0 & am) | ((i0 << 2) & bm), n, 2), n);
            const bool desc = b2;
            // the pair loads start at even indices (8- and 16-byte aligned)
            EXPECT(ia % 2 == 0 && ib % 2 == (desc ? 1u : 0u), "h=%d j=%llu cc=%d: pair alignment", h,
                   (unsigned long long)j, cc);
            static const int offa[4] = {0, 1, 4, 5}, offb[4] = {0, 4, 1, 5};
            for (int v = 0; v < 4; ++v) {
                const uint64_t t = 4 * j + (uint64_t)v, i = nq + (cc ? nq - 1 - t : t);
                const uint64_t sa = ((i << 2) & am) | (i & bm), sb = (i & am) | ((i << 2) & bm);
                const uint64_t xa = ma_index(sa, n), xb = ma_index(exchange_twin(sb, n, 2), n);
                EXPECT(xa < n / 4 && xb < n / 4, "h=%d j=%llu: mean index out of range", h,
                       (unsigned long long)j);
                EXPECT(xa == ia + offa[v], "h=%d j=%llu cc=%d v=%d: advance-a offset",
                       h, (unsigned long long)j, cc, v);
                EXPECT(xb == (desc ? ib - offb[v] : ib + offb[v]), "h=%d j=%llu cc=%d v=%d: advance-b offset",
                       h, (unsigned long long)j, cc, v);
                EXPECT(ma_def(xa) == (T(sa) + T(sa + 2)) * 0.5, "h=%d i=%llu: advance-a mean", h,
                       (unsigned long long)i);
                EXPECT(ma_def(xb) == (T(sb) + T(sb + 1)) * 0.5, "h=%d i=%llu: advance-b mean", h,
                       (unsigned long long)i);
                (cc ? c : b)[v] = T(i);
            }
        }
        // entry writes (positions the kernel stores when asked)
        static const int pos_nsj[4] = {3, 1, 2, 0}, pos_psj[4] = {0, 2, 1, 3};
        for (int v = 0; v < 4; ++v) {
            const uint64_t t = 4 * j + (uint64_t)v;
            EXPECT(T(t) == a[v] && T(nq + t) == b[v], "h=%d: own entry", h);
            EXPECT(T(4 * (mq - sj) + (uint64_t)pos_nsj[v]) == a[v], "h=%d j=%llu v=%d: 0/0 twin entry", h,
                   (unsigned long long)j, v);
            EXPECT(T(nq + 4 * sj + (uint64_t)pos_psj[v]) == c[v], "h=%d j=%llu v=%d: 0/1 twin entry", h,
                   (unsigned long long)j, v);
        }
        // mean writes
        const uint64_t P[4] = {j, mq - j, n16 + j, n16 + mq - j};
        const double m[4][4] = {{a[0], a[1], a[2], a[3]}, {a[3], a[2], a[1], a[0]},
                                {b[0], b[1], b[2], b[3]}, {c[3], c[2], c[1], c[0]}};
        for (int g = 0; g < 4; ++g) {
            const double mall = ((m[g][0] + m[g][3]) + (m[g][1] + m[g][2])) * 0.25;
            for (int x = 0; x < 4; ++x)
                EXPECT(T(4 * P[g] + (uint64_t)x) == m[g][x], "h=%d j=%llu: group %d member %d", h,
                       (unsigned long long)j, g, x);
            const uint64_t twp = mab_index(exchange_twin(4 * P[g], n, 2), n);
            uint64_t wi[6] = {2 * P[g], 2 * P[g] + 1, twp < P[g] ? twp : P[g], 0, 0, 0};
            double wv[6] = {(m[g][0] + m[g][2]) * 0.5, (m[g][1] + m[g][3]) * 0.5, mall, 0, 0, 0};
            int nw = 3;
            if (pj != j) {
                wi[3] = ma_index(exchange_twin(4 * P[g], n, 2), n);
                wi[4] = ma_index(exchange_twin(4 * P[g] + 2, n, 2), n);
                // one aligned pair: ascending from an even index, else descending
                EXPECT(wi[4] == (wi[3] & 1 ? wi[3] - 1 : wi[3] + 1), "h=%d j=%llu group %d: twin pair", h,
                       (unsigned long long)j, g);
                wv[3] = (m[g][0] + m[g][1]) * 0.5;
                wv[4] = (m[g][2] + m[g][3]) * 0.5;
                nw = 5;
            }
            for (int w = 0; w < nw; ++w) {
                const bool isab = w == 2;
                EXPECT(wi[w] < (isab ? n / 8 : n / 4), "h=%d: mean write out of range", h);
                if (wi[w] >= (isab ? n / 8 : n / 4)) continue;
                EXPECT((isab ? mab_def(wi[w]) : ma_def(wi[w])) == wv[w],
                       "h=%d j=%llu group %d write %d: value differs from the definition", h,
                       (unsigned long long)j, g, w);
                if (!count) (isab ? wab : wa)[wi[w]] = 1;
            }
        }
    }
    if (count) return;
    uint64_t miss = 0;
    for (char f : wa) miss += !f;
    EXPECT(miss == 0, "h=%d: %llu advance-a means never written", h, (unsigned long long)miss);
    miss = 0;
    for (uint64_t P : need_ab) miss += !wab[P];
    EXPECT(miss == 0, "h=%d: %llu all-advance means read but never written", h, (unsigned long long)miss);
}

// Branch-mean tables for sigma = 2, d = 3 (m1_index .. m123_index): on a
// table that gives every orbit of the complement and the exchange of strings
// 1 and 2 one pseudo-random integer (an all-match tuple one for its tail's
// orbit), emulate the octets of eight lanes of the branch-mean sweep (lane v
// of octet j holds tail t = 8j + v and its complement; member u = v, or 7 - v
// for the complement's groups; partners by lane xor): every mean a lane
// writes equals its definition, the exchange-folded tables (M3, M12, M123)
// are written at the lower index of each exchanged pair, M1 and M23 in full
// (the exchanged octet's through its string-2 and (s1 s3) means), every read
// (with the lower-index redirect where folded) finds the mean the entry
// sweep forms, and every index read is written.
static double orbit_value3(uint64_t s, uint64_t n)
{
    const int h = __builtin_ctzll(n) / 3;
    const uint64_t head = s >> (3 * (h - 1));
    const bool match = head == 0 || head == 7;
    if (match) s &= (n >> 3) - 1;
    const uint64_t m = match ? (n >> 3) - 1 : n - 1;
    const uint64_t e = exchange12(s, m + 1), c = s ^ m, ec = e ^ m;
    uint64_t r = s < c ? s : c;
    r = r < e ? r : e;
    r = r < ec ? r : ec;
    if (match) r |= 1ull << 62;
    uint64_t z = (r + 0x9E3779B97F4A7C15ull) * 0xBF58476D1CE4E5B9ull;
    z ^= z >> 29;
    return (double)(z & 0xFFFF);
}

static void means3(int h, uint64_t count = 0)
{
    const uint64_t n = 1ull << (3 * h), mx = (n >> 3) - 1, s2bit = (mx + 1) >> 2;
    const int top = 3 * (h - 1);
    const uint64_t mask = n - 1, r3 = mask / 7, S1 = r3 << 2, S2 = r3 << 1, S3 = r3;
    auto T = [&](uint64_t s) { return orbit_value3(s, n); };
    auto base = [&](uint64_t i, uint64_t sm) { return (i & ~sm) | ((i << 3) & sm & mask); };
    auto p4 = [](double a, double b, double c, double d) { return ((a + d) + (b + c)) * 0.25; };
    auto p8 = [&](uint64_t g) {
        return (((T(g) + T(g + 7)) + (T(g + 1) + T(g + 6))) + ((T(g + 2) + T(g + 5)) + (T(g + 3) + T(g + 4)))) * 0.125;
    };
    auto m1_def = [&](uint64_t k) { const uint64_t P = k >> 2, r = k & 3; return (T(8 * P + r) + T(8 * P + 4 + r)) * 0.5; };
    auto m3_def = [&](uint64_t k) { const uint64_t P = k >> 2, q = k & 3; return (T(8 * P + 2 * q) + T(8 * P + 2 * q + 1)) * 0.5; };
    auto m12_def = [&](uint64_t k) { const uint64_t g = 8 * (k >> 1) + (k & 1); return p4(T(g), T(g + 2), T(g + 4), T(g + 6)); };
    auto m23_def = [&](uint64_t k) { const uint64_t g = 8 * (k >> 1) + 4 * (k & 1); return p4(T(g), T(g + 1), T(g + 2), T(g + 3)); };
    auto lower = [](uint64_t a, uint64_t b) { return a < b ? a : b; };
    const uint64_t octets = n >> 7;
    std::vector<char> w1(count ? 0 : n / 4), w3(count ? 0 : n / 4), w12(count ? 0 : n / 8),
        w23(count ? 0 : n / 8), w123(count ? 0 : n / 16);
    std::vector<uint64_t> need3, need12, need123;
    const uint64_t visits = count ? count + 2 : octets;
    for (uint64_t k = 0; k < visits; ++k) {
        const uint64_t j = !count ? k : k == count ? 0 : k == count + 1 ? octets - 1
                                                   : (k * 0x9E3779B97F4A7C15ull) % octets;
        const uint64_t e0 = exchange12(8 * j, n >> 3);
        const uint64_t pj = ((8 * j) & s2bit ? e0 ^ mx : e0) >> 3;
        if (pj < j) continue;
        // lane values: [head r][c][v]
        double lv[4][2][8];
        for (int v = 0; v < 8; ++v) {
            const uint64_t t = 8 * j + (uint64_t)v;
            for (int c = 0; c < 2; ++c)
                for (int r = 0; r < 4; ++r) lv[r][c][v] = T(((uint64_t)r << top) | (c ? mx - t : t));
            // reads
            const uint64_t g = 8 * t;
            const uint64_t r123 = lower(m123_index(g, n), m123_index(exchange_twin(g, n, 3), n));
            EXPECT(r123 < n / 16 && m123_index(g, n) == t, "d=3 h=%d: match read", h);
            EXPECT(p8(8 * r123) == p8(g), "d=3 h=%d t=%llu: all-advance mean", h, (unsigned long long)t);
            if (!count) need123.push_back(r123);
            for (int c = 0; c < 2; ++c) {
                const uint64_t x = c ? mx - t : t;
                {   // 001
                    const uint64_t i = (1ull << top) | x, b1 = base(i, S3), b2 = base(i, S1 | S2);
                    const uint64_t a3 = lower(m3_index(b1, n), m3_index(exchange_twin(b1, n, 3), n));
                    const uint64_t a12 = lower(m12_index(b2, n), m12_index(exchange_twin(b2, n, 3), n));
                    EXPECT(a3 < n / 4 && a12 < n / 8, "d=3 h=%d: 001 read out of range", h);
                    EXPECT(m3_def(a3) == (T(b1) + T(b1 + 1)) * 0.5, "d=3 h=%d x=%llu: 001 string-3 mean", h,
                           (unsigned long long)x);
                    EXPECT(m12_def(a12) == p4(T(b2), T(b2 + 2), T(b2 + 4), T(b2 + 6)),
                           "d=3 h=%d x=%llu: 001 strings-1,2 mean", h, (unsigned long long)x);
                    if (!count) { need3.push_back(a3); need12.push_back(a12); }
                }
                {   // 010
                    const uint64_t i = (2ull << top) | x, b1 = base(i, S2), b2 = base(i, S1 | S3);
                    const uint64_t a1 = m1_index(exchange_twin(b1, n, 3), n);
                    const uint64_t a23 = m23_index(exchange_twin(b2, n, 3), n);
                    EXPECT(a1 < n / 4 && a23 < n / 8, "d=3 h=%d: 010 read out of range", h);
                    EXPECT(m1_def(a1) == (T(b1) + T(b1 + 2)) * 0.5, "d=3 h=%d x=%llu: 010 string-2 mean", h,
                           (unsigned long long)x);
                    EXPECT(m23_def(a23) == p4(T(b2), T(b2 + 1), T(b2 + 4), T(b2 + 5)),
                           "d=3 h=%d x=%llu: 010 strings-1,3 mean", h, (unsigned long long)x);
                }
                {   // 011
                    const uint64_t i = (3ull << top) | x, b2 = base(i, S2 | S3), b1 = base(i, S1);
                    const uint64_t a23 = m23_index(b2, n), a1 = m1_index(b1, n);
                    EXPECT(a1 < n / 4 && a23 < n / 8, "d=3 h=%d: 011 read out of range", h);
                    EXPECT(m23_def(a23) == p4(T(b2), T(b2 + 1), T(b2 + 2), T(b2 + 3)),
                           "d=3 h=%d x=%llu: 011 strings-2,3 mean", h, (unsigned long long)x);
                    EXPECT(m1_def(a1) == (T(b1) + T(b1 + 4)) * 0.5, "d=3 h=%d x=%llu: 011 string-1 mean", h,
                           (unsigned long long)x);
                }
            }
        }
        // writes: the eight groups of the octet, as the lanes form them
        const uint64_t jc = (mx >> 3) - j;
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 2; ++c) {
                const uint64_t P = ((uint64_t)r << (top - 3)) | (c ? jc : j);
                double m[8];
                for (int u = 0; u < 8; ++u) m[u] = lv[r][c][c ? 7 - u : u];
                for (int u = 0; u < 8; ++u)
                    EXPECT(T(8 * P + (uint64_t)u) == m[u], "d=3 h=%d: group %llu member %d", h,
                           (unsigned long long)P, u);
                auto put = [&](std::vector<char> &w, uint64_t idx, uint64_t size, double val, double def,
                               const char *what) {
                    EXPECT(idx < size, "d=3 h=%d: %s write out of range", h, what);
                    if (idx >= size) return;
                    EXPECT(val == def, "d=3 h=%d P=%llu: %s write differs from its definition", h,
                           (unsigned long long)P, what);
                    if (!count) w[idx] = 1;
                };
                for (int q = 0; q < 4; ++q) {
                    const uint64_t i1 = 4 * P + (uint64_t)q;
                    put(w1, i1, n / 4, (m[q] + m[q + 4]) * 0.5, m1_def(i1), "M1");
                    const uint64_t i3 = lower(4 * P + (uint64_t)q, m3_index(exchange_twin(8 * P + 2 * q, n, 3), n));
                    put(w3, i3, n / 4, (m[2 * q] + m[2 * q + 1]) * 0.5, m3_def(i3), "M3");
                }
                for (int b = 0; b < 2; ++b) {
                    const uint64_t i12 = lower(2 * P + (uint64_t)b, m12_index(exchange_twin(8 * P + b, n, 3), n));
                    put(w12, i12, n / 8, p4(m[b], m[2 + b], m[4 + b], m[6 + b]), m12_def(i12), "M12");
                    put(w23, 2 * P + (uint64_t)b, n / 8, p4(m[4 * b], m[4 * b + 1], m[4 * b + 2], m[4 * b + 3]),
                        m23_def(2 * P + (uint64_t)b), "M23");
                }
                const double all = (((m[0] + m[7]) + (m[1] + m[6])) + ((m[2] + m[5]) + (m[3] + m[4]))) * 0.125;
                const uint64_t i123 = lower(P, m123_index(exchange_twin(8 * P, n, 3), n));
                put(w123, i123, n / 16, all, p8(8 * i123), "M123");
                if (pj != j) {  // the exchanged octet's M1 and M23
                    for (int u : {0, 1, 4, 5}) {
                        const uint64_t i1 = m1_index(exchange_twin(8 * P + (uint64_t)u, n, 3), n);
                        EXPECT(i1 == m1_index(exchange_twin(8 * P + (uint64_t)(u ^ 2), n, 3), n),
                               "d=3 h=%d: string-2 pair splits", h);
                        put(w1, i1, n / 4, (m[u] + m[u ^ 2]) * 0.5, m1_def(i1), "twin M1");
                    }
                    for (int s2 = 0; s2 < 2; ++s2) {
                        const int u0 = 2 * s2;
                        const uint64_t i23 = m23_index(exchange_twin(8 * P + (uint64_t)u0, n, 3), n);
                        put(w23, i23, n / 8, p4(m[u0], m[u0 + 1], m[u0 + 4], m[u0 + 5]), m23_def(i23),
                            "twin M23");
                    }
                }
            }
    }
    if (count) return;
    uint64_t miss = 0;
    for (char f : w1) miss += !f;
    for (char f : w23) miss += !f;
    EXPECT(miss == 0, "d=3 h=%d: %llu M1/M23 entries never written", h, (unsigned long long)miss);
    miss = 0;
    for (uint64_t i : need3) miss += !w3[i];
    for (uint64_t i : need12) miss += !w12[i];
    for (uint64_t i : need123) miss += !w123[i];
    EXPECT(miss == 0, "d=3 h=%d: %llu folded means read but never written", h, (unsigned long long)miss);
}

// Branch-mean tables for sigma = 4 (m4a_index, m4ab_index): on a table that
// gives every orbit of the relabellings and the exchange one pseudo-random
// integer (an all-match tuple one for its tail's orbit), emulate the
// sixteen lanes of a hexadecet (lane w of hexadecet J holds tail t = 16J + w
// and its images t xor m rep; group (b1, m) has member u = w xor 5m in lane
// w): the advance-a means (tree4 over a_l, partners at lane distances 4 and
// 8), the exchanged hexadecet's advance-a means from this one's advance-b
// means (distances 1 and 2), and the sixteen-member tree in four levels of
// lane pairs (distances 5, 10 or 15; 10 or 5; 3; 2) equal their
// definitions; reads find the entry sweep's means; every index read is
// written.
static uint64_t relabel4(uint64_t s, uint64_t n, uint64_t m) { return s ^ (m * ((n - 1) / 3)); }

static double orbit_value4(uint64_t s, uint64_t n)
{
    const int h = __builtin_ctzll(n) / 4;
    const uint64_t head = s >> (4 * (h - 1));
    const bool match = (head >> 2) == (head & 3);
    uint64_t m = n;
    if (match) {
        s &= (n >> 4) - 1;
        m = n >> 4;
    }
    uint64_t r = ~0ull;
    for (int e = 0; e < 2; ++e) {
        const uint64_t x = e ? exchange4(s, m) : s;
        for (uint64_t k = 0; k < 4; ++k) {
            const uint64_t y = relabel4(x, m, k);
            r = y < r ? y : r;
        }
    }
    if (match) r |= 1ull << 62;
    uint64_t z = (r + 0x9E3779B97F4A7C15ull) * 0xBF58476D1CE4E5B9ull;
    z ^= z >> 29;
    return (double)(z & 0xFFFF);
}

static void means4(int h, uint64_t count = 0)
{
    const uint64_t n = 1ull << (4 * h), nt = n >> 4;  // tails
    const int top = 4 * (h - 1);
    const uint64_t rep = (nt - 1) / 3, am = 0xCCCCCCCCCCCCCCCCull & (n - 1), bm = ~am & (n - 1);
    auto T = [&](uint64_t s) { return orbit_value4(s, n); };
    auto tree4 = [](double a, double b, double c, double d) { return ((a + b) + (c + d)) * 0.25; };
    auto tree16 = [&](const double *g) {
        return ((((g[1] + g[4]) + (g[11] + g[14])) + ((g[2] + g[8]) + (g[7] + g[13]))) +
                (((g[3] + g[12]) + (g[6] + g[9])) + ((g[0] + g[15]) + (g[5] + g[10])))) * 0.0625;
    };
    auto ma_def = [&](uint64_t k) {
        const uint64_t g = 16 * (k >> 2) + (k & 3);
        return tree4(T(g), T(g + 4), T(g + 8), T(g + 12));
    };
    auto mab_def = [&](uint64_t P) {
        double g[16];
        for (int u = 0; u < 16; ++u) g[u] = T(16 * P + (uint64_t)u);
        return tree16(g);
    };
    auto lower = [](uint64_t a, uint64_t b) { return a < b ? a : b; };
    const uint64_t hexes = n >> 10;  // J < n/1024: tails with a_2 = 0, in sixteens
    std::vector<char> wa(count ? 0 : n / 16), wab(count ? 0 : n / 64);
    std::vector<uint64_t> need_ab;
    const uint64_t visits = count ? count + 2 : hexes;
    for (uint64_t k = 0; k < visits; ++k) {
        const uint64_t J = !count ? k : k == count ? 0 : k == count + 1 ? hexes - 1
                                                   : (k * 0x9E3779B97F4A7C15ull) % hexes;
        const uint64_t t0 = 16 * J;
        const uint64_t sx0 = (t0 >> (top - 4)) & 3;
        const uint64_t pJ = (exchange4(t0, nt) ^ (sx0 * rep)) >> 4;
        if (pJ < J) continue;
        const bool self = pJ == J;
        double lv[16][4][4];  // [lane w][m][b1]
        for (int w = 0; w < 16; ++w) {
            const uint64_t t = t0 + (uint64_t)w;
            // reads
            {
                const uint64_t tw = m4ab_index(exchange_twin4(16 * t, n), n), at = lower(t, tw);
                EXPECT(at < n / 64, "s4 h=%d: all-advance read out of range", h);
                EXPECT(mab_def(at) == mab_def(t), "s4 h=%d t=%llu: all-advance mean", h, (unsigned long long)t);
                if (!count) need_ab.push_back(at);
            }
            for (int v = 0; v < 4; ++v) {
                const uint64_t i = ((uint64_t)v << top) | t, sa = ((i << 4) & am) | (i & bm);
                const uint64_t ia = m4a_index(sa, n);
                EXPECT(ia < n / 16, "s4 h=%d: advance-a read out of range", h);
                EXPECT(ma_def(ia) == tree4(T(sa), T(sa + 4), T(sa + 8), T(sa + 12)),
                       "s4 h=%d i=%llu: advance-a mean", h, (unsigned long long)i);
            }
            for (uint64_t m = 0; m < 4; ++m) {
                const uint64_t x = t ^ (m * rep), sb = (x & am) | ((x << 4) & bm);
                const uint64_t ib = m4a_index(exchange_twin4(sb, n), n);
                EXPECT(ib < n / 16, "s4 h=%d: advance-b read out of range", h);
                EXPECT(ma_def(ib) == tree4(T(sb), T(sb + 1), T(sb + 2), T(sb + 3)),
                       "s4 h=%d x=%llu: advance-b mean", h, (unsigned long long)x);
                for (int b1 = 0; b1 < 4; ++b1) lv[w][m][b1] = T(((uint64_t)b1 << top) | x);
            }
        }
        // writes, as the lanes form them
        for (int b1 = 0; b1 < 4; ++b1)
            for (uint64_t m = 0; m < 4; ++m) {
                const uint64_t P = ((uint64_t)b1 << (top - 4)) | (J ^ (m * ((nt >> 4) - 1) / 3));
                double val[16];  // by lane
                for (int w = 0; w < 16; ++w) val[w] = lv[w][m][b1];
                for (int w = 0; w < 16; ++w) {
                    const int u = w ^ (int)(5 * m);
                    EXPECT(T(16 * P + (uint64_t)u) == val[w], "s4 h=%d: group %llu member %d", h,
                           (unsigned long long)P, u);
                }
                auto sh = [&](const double *a, int w, int d) { return a[w ^ d]; };
                double L1[16], L2[16], L3[16], L4[16], p1[16];
                for (int w = 0; w < 16; ++w) {
                    const int u = w ^ (int)(5 * m);
                    const int d1 = (u == 1 || u == 4 || u == 11 || u == 14) ? 5
                                 : (u == 2 || u == 8 || u == 7 || u == 13) ? 10 : 15;
                    L1[w] = val[w] + sh(val, w, d1);
                    p1[w] = val[w] + sh(val, w, 4);
                }
                for (int w = 0; w < 16; ++w) {
                    const int u = w ^ (int)(5 * m);
                    const int d2 = (u == 1 || u == 4 || u == 11 || u == 14) ? 10 : 5;
                    L2[w] = L1[w] + sh(L1, w, d2);
                }
                for (int w = 0; w < 16; ++w) L3[w] = L2[w] + sh(L2, w, 3);
                for (int w = 0; w < 16; ++w) L4[w] = L3[w] + sh(L3, w, 2);
                for (int w = 0; w < 16; ++w) {
                    const int u = w ^ (int)(5 * m);
                    const uint64_t tw = exchange_twin4(16 * P + (uint64_t)u, n);
                    if (!(u & 12)) {  // own advance-a mean
                        const uint64_t idx = 4 * P + (uint64_t)(u & 3);
                        const double a = (p1[w] + sh(p1, w, 8)) * 0.25;
                        EXPECT(idx < n / 16 && a == ma_def(idx), "s4 h=%d P=%llu: M4a", h, (unsigned long long)P);
                        if (!count) wa[idx] = 1;
                    }
                    if (u == 1) {
                        const uint64_t at = lower(P, m4ab_index(tw, n));
                        const double a = L4[w] * 0.0625;
                        EXPECT(at < n / 64 && a == mab_def(at), "s4 h=%d P=%llu: M4ab", h, (unsigned long long)P);
                        if (!count) wab[at] = 1;
                    }
                    if (!self && !(u & 3)) {  // the exchanged hexadecet's advance-a mean
                        const double q1 = val[w] + sh(val, w, 1), q2 = sh(val, w, 2) + sh(val, w, 3);
                        const double b = (q1 + q2) * 0.25;
                        const uint64_t idx = m4a_index(tw, n);
                        EXPECT(idx < n / 16 && b == ma_def(idx), "s4 h=%d P=%llu: twin M4a", h,
                               (unsigned long long)P);
                        if (!count) wa[idx] = 1;
                    }
                }
            }
    }
    if (count) return;
    uint64_t miss = 0;
    for (char f : wa) miss += !f;
    EXPECT(miss == 0, "s4 h=%d: %llu advance-a means never written", h, (unsigned long long)miss);
    miss = 0;
    for (uint64_t P : need_ab) miss += !wab[P];
    EXPECT(miss == 0, "s4 h=%d: %llu all-advance means read but never written", h, (unsigned long long)miss);
}

int main()
{
    for (int h = 3; h <= 4; ++h) means4(h);
    for (int h = 5; h <= 8; ++h) means4(h, 1u << 10);
    for (int h = 3; h <= 6; ++h) means3(h);
    for (int h = 7; h <= 12; ++h) means3(h, 1u << 12);
    for (int h = 3; h <= 10; ++h) means(h);
    for (int h = 11; h <= 18; ++h) means(h, 1u << 16);
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
