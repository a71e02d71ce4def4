// Learned warm start: a 32 -> 256 -> 256 -> 256 -> 1 ReLU network that maps
// a tuple of two binary head strings to a guess of the normalised converged
// table value, trained on converged tables at smaller window length and used
// once to fill the FP32 ring before the iteration of Algorithm 2 starts (the
// limit of that iteration does not depend on where it starts).
//
// Every matrix product runs on the gfx950 matrix cores as
// v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 accumulation.  Parameters
// live as one FP32 master vector (layout below) plus its BF16 rounding
// (round to nearest, ties to even); biases are added in FP32 (as the
// accumulators' initial value) and the activation handed to the next layer
// is the BF16 rounding of its ReLU.
//
// Parameter layout (floats), matrices output-major ([out][in]):
//   W1[256][32] b1[256] W2[256][256] b2[256] W3[256][256] b3[256] w4[256] b4[1]
//
// Inputs (32): window positions P(l) = (1..8, l-7..l); slot 2j holds string
// a at P_j, slot 2j+1 string b, symbol s -> 2s - 1.  At l = 16 these are
// the index bits in order.
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace lcsb {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int kIn = 32, kW = 256;
constexpr int oW1 = 0, ob1 = oW1 + kW * kIn, oW2 = ob1 + kW, ob2 = oW2 + kW * kW;
constexpr int oW3 = ob2 + kW, ob3 = oW3 + kW * kW, ow4 = ob3 + kW, ob4 = ow4 + kW;
constexpr int kNParams = ob4 + 1;
static_assert(kNParams == LCSB_MLP_NPARAMS, "parameter count");

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 load8(const uint16_t *p)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(p));
}

// window position (1-based) feeding input pair j
__device__ __forceinline__ int pos_of(int j, int h) { return j < 8 ? j + 1 : h - 15 + j; }

// input slot value for index i at window length h
__device__ __forceinline__ float input_at(uint64_t i, int h, int slot)
{
    const int p = pos_of(slot >> 1, h);
    const int bit = 2 * (h - p) + ((slot & 1) ? 0 : 1);
    return ((i >> bit) & 1) ? 1.0f : -1.0f;
}

// ------------------------------------------------------------------ seed orbits
// The converged table is invariant under exchanging the two strings and under
// complementing both (Sec. 3.3), so the seed evaluates the network once per
// orbit of the group these generate and writes the value to the members the
// folded table stores (string-1 head 0: the representative and one of the
// two members with the strings exchanged).
// With c = a xor b, both maps fix c and act on a as a -> a xor {0, c, 1..1,
// ~c}: an orbit is a coset of the span of 1..1 and c' (c or ~c, whichever
// has head 0).  Its unique member with a zero bit at both pivots (a's head
// and the highest set bit of c') is the representative.  For c in {0, 1..1}
// the span is one-dimensional and only a's head is fixed.  Orbit number t:
//   t <  2^(2l-2):    t's bits are, from the lowest, x0 x1 c0 c1, then the
//                     other l-4 bits of x, then the other l-2 bits of c; a =
//                     x with a zero inserted at c's pivot (head bit 0); for
//                     c in {0, 1..1}, a = x (the half of a with bit l-2
//                     clear).  Sixteen consecutive t thus hold every value of
//                     the last two symbols of both strings and, unless the
//                     pivot is among those two positions, write one aligned
//                     16-entry window of each stored member;
//   t >= 2^(2l-2):    the other half for c = 0, then for c = 1..1.
// Count (2^l + 2) 2^(l-2) = 4^l / 4 + 2^(l-1).
__device__ __forceinline__ uint32_t spread16(uint32_t x)  // bit k -> bit 2k
{
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

__device__ __forceinline__ uint64_t orbit_rep_index(uint64_t t, int h)
{
    const int lo = h - 2;
    const uint32_t all = (1u << h) - 1u;
    uint32_t a, c;
    if (t < (1ull << (2 * h - 2))) {
        const uint32_t tt = (uint32_t)t;
        const uint32_t x = (tt & 3u) | (((tt >> 4) & ((1u << (h - 4)) - 1u)) << 2);
        c = ((tt >> 2) & 3u) | ((tt >> h) << 2);
        const uint32_t cp = (c >> (h - 1)) ? (c ^ all) : c;
        if (cp == 0u) {
            a = x;
        } else {
            const int j = 31 - __builtin_clz(cp);
            a = ((x >> j) << (j + 1)) | (x & ((1u << j) - 1u));
        }
    } else {
        const uint32_t u = (uint32_t)(t - (1ull << (2 * h - 2)));
        c = (u >> lo) == 0u ? 0u : all;
        a = (u & ((1u << lo) - 1u)) | (1u << lo);
    }
    const uint32_t b = a ^ c;
    return ((uint64_t)spread16(a) << 1) | spread16(b);  // string a in the odd bits
}

__device__ __forceinline__ uint64_t swap_strings(uint64_t i)
{
    const uint64_t ev = 0x5555555555555555ull;
    return ((i >> 1) & ev) | ((i & ev) << 1);
}

// ------------------------------------------------------------------ fused forward
// One wave owns 32 samples (two 16-sample MFMA column blocks).  A layer is
// computed transposed, Y^T = W X^T: the weight tile is the A operand (rows =
// output features) and the activations are the B operand (columns =
// samples).  The MFMA result layout (lane group g holds rows 4g .. 4g+3 of
// a 16-row output tile for one sample) becomes the next layer's B operand
// (lane group g holds k = 8g .. 8g+7 of a 32-wide k block) without moving
// data, because output tile f is made of the weight rows
//   perm_row(f, i) = 32 (f/2) + 8 (i/4) + 4 (f%2) + i%4,   i = 0..15,
// so tiles 2kb and 2kb+1 give lane group g the eight consecutive features
// 32kb + 8g .. 32kb + 8g + 7: input feature 32kb + 8g + t of the next layer
// sits in slot t.  Activations never leave the registers.  Layers
// 2 and 3 stream their weights through LDS in 16-row tiles (8 KB), consumed
// kStep per workgroup barrier and shared by the workgroup's waves.
constexpr int kFwdWaves = 8;
constexpr int kFwdBlocks = 2;                          // 16-sample MFMA column blocks per wave
constexpr int kFwdThreads = 64 * kFwdWaves;
constexpr int kFwdSamples = 16 * kFwdBlocks * kFwdWaves;  // per workgroup batch

__device__ __forceinline__ int feat_of(int kb, int g, int t) { return 32 * kb + 8 * g + t; }

// weight row (output feature) computed in row i of output tile f
__device__ __forceinline__ int perm_row(int f, int i)
{
    return 32 * (f >> 1) + 8 * (i >> 2) + 4 * (f & 1) + (i & 3);
}

enum : int { kSrcIdx = 0, kSrcOrbits = 1 };

struct FwdArgs {
    const uint16_t *wb;      // BF16 parameters
    const float *pf;         // FP32 parameters (biases)
    const uint64_t *idx;     // explicit sample indices (kSrcIdx)
    uint64_t count;          // samples
    int h;                   // window length of the indices
    float *y;                // predictions (or null)
    uint16_t *act;           // if non-null: H1, H2, H3 as BF16 [3][count][256] for backward
    void *lag1, *lag2;       // seed targets (kSrcOrbits)
    uint64_t n;              // indices of the unfolded table (kSrcOrbits)
    double rate;             // lag 1 = u + rate, lag 2 = u
};

// H_layer[s][feature] = the BF16 activations of the wave's samples (backward).
// Words act[kb][b][0..3] of a lane hold features 32 kb + 8 g .. 32 kb + 8 g + 7
// of its sample in memory order, so each k block is one 16-byte store.
__device__ __forceinline__ void store_act(const FwdArgs &a, int layer, uint64_t s0, int r, int g,
                                          const bool (&valid)[kFwdBlocks],
                                          const uint32_t (&act)[8][kFwdBlocks][4])
{
    uint16_t *H = a.act + (size_t)layer * a.count * kW;
#pragma unroll
    for (int b = 0; b < kFwdBlocks; ++b) {
        if (!valid[b]) continue;
        uint16_t *row = H + (s0 + 16 * b + r) * kW + 8 * g;
#pragma unroll
        for (int kb = 0; kb < 8; ++kb)
            *reinterpret_cast<u32x4 *>(row + 32 * kb) =
                u32x4{act[kb][b][0], act[kb][b][1], act[kb][b][2], act[kb][b][3]};
    }
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// two floats -> BF16 pair (round to nearest even; one v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pack2(float lo, float hi)
{
    typedef float float2v __attribute__((ext_vector_type(2)));
    const bf16x2 v = __builtin_convertvector(float2v{lo, hi}, bf16x2);
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ bf16x8 as_bf8(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3)
{
    u32x4 v = {w0, w1, w2, w3};
    return __builtin_bit_cast(bf16x8, v);
}

// Activations of one wave: act[kb][b][w] = BF16 pair (2w, 2w+1) of k-block
// kb, sample block b (slots as described above).  An output tile f fills
// words (f&1)*2 and (f&1)*2+1 of k-block f/2.
//
// Everything a lane reads at a lane-dependent address lives in LDS (W1, the
// biases, w4, the streamed W2/W3 tiles), so those reads use immediate
// offsets.  W2 and W3 do not fit in LDS together, so their 16-row tiles flow
// through a ring of kRing slots as one endless stream (W2 tiles 0..15, W3
// tiles 0..15, W2 again for the next batch, ...) loaded kRing - kStep tiles
// ahead by direct global-to-LDS loads.  The stream position of tile f is
// congruent to f modulo kRing, so slot indices are compile-time constants.
constexpr int kRing = 8;   // ring slots (one 8 KB tile each); divides 16
constexpr int kStep = 2;   // tiles consumed per workgroup barrier; divides kRing
constexpr int kPf = 4;     // k blocks a wave's fragment requests run ahead of its products
static_assert(16 % kRing == 0 && kRing % kStep == 0 && kRing / kStep >= 2, "ring shape");

// The ring slots are separate LDS objects so the compiler's wait insertion
// can tell a read of one slot from the loads still landing in the others.
__shared__ uint16_t ring0[16 * kW], ring1[16 * kW], ring2[16 * kW], ring3[16 * kW];
__shared__ uint16_t ring4[16 * kW], ring5[16 * kW], ring6[16 * kW], ring7[16 * kW];
__shared__ uint16_t ring8[16 * kW], ring9[16 * kW], ring10[16 * kW], ring11[16 * kW];
__shared__ uint16_t ring12[16 * kW], ring13[16 * kW], ring14[16 * kW], ring15[16 * kW];

__device__ __forceinline__ uint16_t *ring_slot(int k)
{
    switch (k % kRing) {
    case 0: return ring0;
    case 1: return ring1;
    case 2: return ring2;
    case 3: return ring3;
    case 4: return ring4;
    case 5: return ring5;
    case 6: return ring6;
    case 7: return ring7;
    case 8: return ring8;
    case 9: return ring9;
    case 10: return ring10;
    case 11: return ring11;
    case 12: return ring12;
    case 13: return ring13;
    case 14: return ring14;
    default: return ring15;
    }
}

constexpr int kW1Stride = kIn + 8;  // padded LDS row of W1 (80 bytes)

// LDS element offset of W1 row `row`.  The eight lanes of a layer-1 fragment
// read that LDS serves together take rows b + {0..3, 8..11} at the same
// 16-byte chunk; with the 80-byte stride alone rows r and r + 8 share banks,
// so every block of 8 rows starts 64 bytes further on (rows stay disjoint)
// and the eight chunks fall in distinct bank groups.
__device__ __forceinline__ int w1_off(int row) { return row * kW1Stride + 32 * (row >> 3); }
// w1_off(perm_row(f, r)) + 8 g split into a lane part and a per-tile constant
// (perm_row(f, r) >> 3 = 4 (f >> 1) + (r >> 2)), so the unrolled tile loop
// reads at one base register plus immediate offsets.
__device__ __forceinline__ int w1_lane(int r, int g)
{
    return (8 * (r >> 2) + (r & 3)) * kW1Stride + 32 * (r >> 2) + 8 * g;
}
__host__ __device__ constexpr int w1_tile(int f)
{
    return (32 * (f >> 1) + 4 * (f & 1)) * kW1Stride + 128 * (f >> 1);
}

struct FwdSmem {
    uint16_t w1[kW * kW1Stride + 32 * (kW / 8 - 1)];  // W1, rows padded and skewed (w1_off)
    float bias[3][kW];              // b1, b2, b3
    uint16_t w4[kW];                // BF16 w4
};

typedef short short2v __attribute__((ext_vector_type(2)));

// ReLU of two BF16 values packed in a word: a BF16 number and its int16 bit
// pattern have the same sign, so an elementwise int16 max with 0 does it
// (-0 becomes +0).  BF16 rounding keeps the sign, so ReLU after rounding
// equals rounding after ReLU.
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t w)
{
    const short2v v = __builtin_elementwise_max(__builtin_bit_cast(short2v, w), short2v{0, 0});
    return __builtin_bit_cast(uint32_t, v);
}

// the four FP32 biases of output rows perm_row(f, 4g .. 4g+3): the initial
// accumulator of an output tile, so the matrix cores add the bias
__device__ __forceinline__ floatx4 bias4(const float *b, int f, int g)
{
    return *reinterpret_cast<const floatx4 *>(b + perm_row(f, 4 * g));
}

// Tile (layer, f) = weight rows perm_row(f, 0..15) of W2 (layer 0) or W3
// (layer 1), stored chunk-major: the 16-byte chunk c (k = 8c .. 8c+7) of
// tile row i sits at byte 16 (16 c + i).  The workgroup's threads move the
// 512 chunks straight from global memory into the ring slot (gfx950
// buffer_load_dwordx4 with the lds bit: no registers, counted by vmcnt),
// kTileOps per thread; chunk q lands at byte 16 q, so it is chunk q/16 of
// row q%16.  A fragment read (lane (i, g)
// needs chunk 4 kb + g of row i) is then the 1 KB at byte 16 lane + 1024 kb:
// contiguous across the 64 lanes (no bank conflicts) and one base address
// plus immediate offsets for every k block and slot.  The buffer form (not
// global_load_lds) matters: the compiler treats the global form as a flat
// access that may touch LDS and then waits for every outstanding LDS read
// before each use of one, which serialises the fragment pipeline below.
// The descriptor's record count bounds the loads to the parameter vector.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t weight_rsrc(const uint16_t *wb)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(wb), (short)0,
                                             (int)(kNParams * sizeof(uint16_t)), 0x00020000);
}

constexpr int kTileChunks = 16 * kW / 8;                  // 16-byte chunks per tile (512)
constexpr int kTileOps = kTileChunks / kFwdThreads;         // loads per thread (and wave) per tile
static_assert(kTileChunks % kFwdThreads == 0, "whole chunks per thread");

__device__ __forceinline__ void issue_tile(__amdgpu_buffer_rsrc_t rs, int layer, int f,
                                           uint16_t *slot)
{
#pragma unroll
    for (int k = 0; k < kTileOps; ++k) {
        const int q = threadIdx.x + k * kFwdThreads, row = q & 15, c = q >> 4;
        const int byte = 2 * ((layer ? oW3 : oW2) + perm_row(f, row) * kW + c * 8);
        uint16_t *dst = slot + (q & ~63) * 8;  // the wave's 1 KB; lane i lands at +16 i
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)dst,
                                                 16, byte, 0, 0, 0);
    }
}

// Workgroup barrier without a memory fence: a fence would make every wave
// wait for all of its loads still landing in the ring.  Callers wait for the
// loads they need (wait_vmcnt) before it; the "memory" clobber keeps the
// compiler from moving LDS accesses across it.
__device__ __forceinline__ void ring_barrier() { asm volatile("s_barrier" ::: "memory"); }

// s_waitcnt vmcnt(n), expcnt and lgkmcnt left free (n < 16)
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 16, "vmcnt field");
    __builtin_amdgcn_s_waitcnt(0xF70 | N);
}

// s_waitcnt vmcnt(n) lgkmcnt(0): also every LDS read of this wave is done, so
// after the following barrier no wave still reads the slot about to be
// refilled (the compiler may move the reads' consumers past the barrier).
template <int N>
__device__ __forceinline__ void wait_vmcnt_lds()
{
    static_assert(N >= 0 && N < 16, "vmcnt field");
    __builtin_amdgcn_s_waitcnt(0x070 | N);
}

template <int SRC, bool STORE, typename T>
__global__ __launch_bounds__(kFwdThreads) void mlp_fwd(FwdArgs a)
{
    constexpr int NB = kFwdBlocks;
    __shared__ FwdSmem sm;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    const uint64_t nbatch = (a.count + kFwdSamples - 1) / kFwdSamples;

    // resident parameters (once per workgroup)
    for (int q = threadIdx.x; q < kW * kIn / 8; q += kFwdThreads)  // 16-byte chunks
        *reinterpret_cast<u32x4 *>(sm.w1 + w1_off(q >> 2) + (q & 3) * 8) =
            reinterpret_cast<const u32x4 *>(a.wb + oW1)[q];
    for (int q = threadIdx.x; q < kW; q += kFwdThreads) {
        sm.bias[0][q] = a.pf[ob1 + q];
        sm.bias[1][q] = a.pf[ob2 + q];
        sm.bias[2][q] = a.pf[ob3 + q];
        sm.w4[q] = a.wb[ow4 + q];
    }
    const float b4 = a.pf[ob4];
    const __amdgpu_buffer_rsrc_t wrs = weight_rsrc(a.wb);
    wait_vmcnt<0>();
#pragma unroll
    for (int f = 0; f < kRing - kStep; ++f) issue_tile(wrs, 0, f, ring_slot(f));
    __syncthreads();

    // the four input pairs of this lane: window positions of pairs 4g .. 4g+3
    int shift[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) shift[q] = 2 * (a.h - pos_of(4 * g + q, a.h));

    for (uint64_t batch = blockIdx.x; batch < nbatch; batch += gridDim.x) {
        const uint64_t s0 = batch * kFwdSamples + (uint64_t)wave * (16 * NB);
        uint64_t sidx[NB];
        bool valid[NB];
        bf16x8 x[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const uint64_t s = s0 + 16 * b + r;
            valid[b] = s < a.count;
            const uint64_t sc = valid[b] ? s : 0;
            sidx[b] = SRC == kSrcIdx ? a.idx[sc] : orbit_rep_index(sc, a.h);
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t ab = (uint32_t)(sidx[b] >> shift[q]) & 3u;  // (a bit, b bit)
                w[q] = pack2((ab & 2u) ? 1.0f : -1.0f, (ab & 1u) ? 1.0f : -1.0f);
            }
            x[b] = as_bf8(w[0], w[1], w[2], w[3]);
        }

        // layer 1 (K = 32: one MFMA per output tile, started from the bias)
        uint32_t act[8][NB][4];
        const uint16_t *w1l = sm.w1 + w1_lane(r, g);
#pragma unroll
        for (int f = 0; f < 16; ++f) {
            const bf16x8 wf = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(w1l + w1_tile(f)));
            const floatx4 b0 = bias4(sm.bias[0], f, g);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const floatx4 acc = mfma(wf, x[b], b0);
                act[f >> 1][b][(f & 1) * 2 + 0] = relu_bf16x2(pack2(acc[0], acc[1]));
                act[f >> 1][b][(f & 1) * 2 + 1] = relu_bf16x2(pack2(acc[2], acc[3]));
            }
        }

        // layers 2 and 3: kStep tiles per workgroup barrier, the ring's
        // remaining kRing - kStep tiles in flight
        uint32_t hid[8][NB][4];
#pragma unroll
        for (int layer = 0; layer < 2; ++layer) {
            uint32_t (&in)[8][NB][4] = layer ? hid : act;
            uint32_t (&out)[8][NB][4] = layer ? act : hid;
            if constexpr (STORE) {
                store_act(a, layer, s0, r, g, valid, in);
                wait_vmcnt<0>();  // keep vmcnt counting tile loads only
                __builtin_amdgcn_sched_barrier(0);
            }
            const float *bias_v = sm.bias[1 + layer];
#pragma unroll
            for (int p = 0; p < 16 / kStep; ++p) {
                // this wave's part of step p's tiles has landed (the tiles of
                // the following kRing/kStep - 2 steps may be in flight).  The
                // first step of a batch waits for everything: the previous
                // batch's output stores are counted by vmcnt too.
                if (p == 0 && layer == 0) wait_vmcnt_lds<0>();
                else wait_vmcnt_lds<(kRing - 2 * kStep) * kTileOps>();
                ring_barrier();  // every wave's part has landed; step p-1's slots are free
#pragma unroll
                for (int t = 0; t < kStep; ++t) {
                    const int fn = kStep * p + kRing - kStep + t;  // next tiles of the stream
                    issue_tile(wrs, fn < 16 ? layer : layer ^ 1, fn & 15, ring_slot(fn));
                }
                // Weight fragments are requested kPf k blocks ahead of the
                // products that use them (LDS answers in order, so a product
                // waits only for its own fragment); the scheduling barriers
                // keep the compiler from pulling the requests back next to
                // their uses.  The activation-storing variant keeps one block
                // fewer in flight to stay within its registers.
                constexpr int PF = STORE ? kPf - 1 : kPf;
                const uint16_t *slot[kStep];
#pragma unroll
                for (int t = 0; t < kStep; ++t) slot[t] = ring_slot(kStep * p + t) + lane * 8;
                u32x4 wf[8][kStep];
#pragma unroll
                for (int kb = 0; kb < PF; ++kb)
#pragma unroll
                    for (int t = 0; t < kStep; ++t)
                        wf[kb][t] = *reinterpret_cast<const u32x4 *>(slot[t] + kb * 512);
                floatx4 acc[kStep][NB];
#pragma unroll
                for (int t = 0; t < kStep; ++t) {
                    const floatx4 bt = bias4(bias_v, kStep * p + t, g);
#pragma unroll
                    for (int b = 0; b < NB; ++b) acc[t][b] = bt;
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int kb = 0; kb < 8; ++kb) {
#pragma unroll
                    for (int t = 0; t < kStep; ++t)
#pragma unroll
                        for (int b = 0; b < NB; ++b)
                            acc[t][b] = mfma(__builtin_bit_cast(bf16x8, wf[kb][t]),
                                             as_bf8(in[kb][b][0], in[kb][b][1], in[kb][b][2],
                                                    in[kb][b][3]), acc[t][b]);
                    if (kb + PF < 8) {
#pragma unroll
                        for (int t = 0; t < kStep; ++t)
                            wf[kb + PF][t] = *reinterpret_cast<const u32x4 *>(slot[t] + (kb + PF) * 512);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
                // output tile f = kStep p + t fills words (f & 1) * 2 .. +1 of
                // k block f / 2 of the next layer's activations
#pragma unroll
                for (int t = 0; t < kStep; ++t) {
                    const int f = kStep * p + t;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        out[f >> 1][b][(f & 1) * 2 + 0] = relu_bf16x2(pack2(acc[t][b][0], acc[t][b][1]));
                        out[f >> 1][b][(f & 1) * 2 + 1] = relu_bf16x2(pack2(acc[t][b][2], acc[t][b][3]));
                    }
                }
            }
        }
        if constexpr (STORE) store_act(a, 2, s0, r, g, valid, act);

        // layer 4: y = w4 . h3 + b4 on the matrix cores: every row of the A
        // operand is w4, the accumulator starts at b4, so each lane ends with
        // y of its sample column in all four rows
        float part[NB];
        {
            floatx4 acc4[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) acc4[b] = floatx4{b4, b4, b4, b4};
#pragma unroll
            for (int kb = 0; kb < 8; ++kb) {
                const bf16x8 w4f = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const u32x4 *>(sm.w4 + feat_of(kb, g, 0)));
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    acc4[b] = mfma(w4f, as_bf8(act[kb][b][0], act[kb][b][1], act[kb][b][2],
                                               act[kb][b][3]), acc4[b]);
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) part[b] = acc4[b][0];
        }
        if (g == 0) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (!valid[b]) continue;
                const float u = part[b];
                const uint64_t s = s0 + 16 * b + r;
                if (a.y) a.y[s] = u;
                if constexpr (SRC == kSrcOrbits) {
                    T *l1 = static_cast<T *>(a.lag1);
                    T *l2 = static_cast<T *>(a.lag2);
                    // the stored members: i and whichever of j, ~j has string-1 head 0
                    const uint64_t i = sidx[b], j = swap_strings(i);
                    const uint64_t js = (j & (a.n >> 1)) ? j ^ (a.n - 1) : j;
                    const T v2 = (T)u;
                    const T v1 = (T)((double)u + a.rate);
                    l2[i] = v2;
                    l2[js] = v2;
                    l1[i] = v1;
                    l1[js] = v1;
                }
            }
        }
        if constexpr (STORE) wait_vmcnt<0>();  // the next batch stores activations first
    }
    wait_vmcnt<0>();  // no load into LDS outlives the workgroup
}

// ------------------------------------------------------------------ backward GEMMs
// Weight gradient of one layer: G[m][n] = sum over samples s of A[s][m] B[s][n]
// (A = dZ of the layer, B = its input; both sample-major BF16 with row
// lengths lda, ldb), for the workgroup's 128 x TN output tile, over the
// 32-sample steps [z per, (z+1) per) of split z = blockIdx.z.  Each step
// stages both operands through LDS transposed (feature-major rows of 32
// samples, padded to 40 elements so the 16 rows of a fragment read fall in
// distinct banks), so a lane's MFMA fragment (8 samples of one feature) is
// one 16-byte read.  Split z writes its partial G to part + z (M N + M) and,
// in the workgroups of output column 0, the bias-gradient partial
// (sum over its samples of A[s][m]) right after it: a fixed-order reduction
// over z then yields the weight and bias gradients, which sit next to each
// other in the parameter layout.
constexpr int kWgRow = 40;

template <int TN>
__global__ __launch_bounds__(256) void wgrad(const uint16_t *__restrict__ A, int lda,
                                             const uint16_t *__restrict__ Bm, int ldb, int ksteps,
                                             int per, int M, int N, float *__restrict__ part)
{
    constexpr int WM = TN == 128 ? 64 : 32, WN = TN == 128 ? 64 : 32;
    constexpr int WAVES_N = TN / WN;  // 2 x 2 waves of 64 x 64, or 4 x 1 waves of 32 x 32
    constexpr int FM = WM / 16, FN = WN / 16;
    __shared__ uint32_t sa[128 * kWgRow / 2];  // A^T: 128 features x 32 samples (+ padding)
    __shared__ uint32_t sb[TN * kWgRow / 2];   // B^T: TN features x 32 samples (+ padding)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    const int wm = wave / WAVES_N, wn = wave % WAVES_N;
    const int m0 = blockIdx.x * 128, n0 = blockIdx.y * TN;
    const int kbeg = blockIdx.z * per, kend = min(ksteps, kbeg + per);
    // staging: thread q moves features 8c .. 8c+7 of samples 2p, 2p+1 (two
    // 16-byte loads) into eight 32-bit LDS words (row 8c + t, samples 2p, 2p+1)
    const int p = threadIdx.x & 15, c = threadIdx.x >> 4;  // c < 16
    constexpr int CB = TN / 8;                              // chunks of a B row
    floatx4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = floatx4{0, 0, 0, 0};
    float bsum = 0.0f;  // bias partial of row threadIdx.x / 2, samples 16 (threadIdx.x & 1) ..
    u32x4 ra[2], rb[2];
    auto fetch = [&](int ks) {
        const size_t s = (size_t)ks * 32 + 2 * p;
        ra[0] = *reinterpret_cast<const u32x4 *>(A + s * lda + m0 + 8 * c);
        ra[1] = *reinterpret_cast<const u32x4 *>(A + (s + 1) * lda + m0 + 8 * c);
        if (c < CB) {
            rb[0] = *reinterpret_cast<const u32x4 *>(Bm + s * ldb + n0 + 8 * c);
            rb[1] = *reinterpret_cast<const u32x4 *>(Bm + (s + 1) * ldb + n0 + 8 * c);
        }
    };
    if (kbeg < kend) fetch(kbeg);
    for (int ks = kbeg; ks < kend; ++ks) {
        __syncthreads();  // every wave is done with the previous step's tiles
#pragma unroll
        for (int t = 0; t < 8; ++t) {  // word t/2 of a chunk holds features 2(t/2), 2(t/2)+1
            const int sh = (t & 1) * 16, w = t >> 1;
            sa[(8 * c + t) * (kWgRow / 2) + p] = (ra[0][w] >> sh & 0xFFFFu) | ((ra[1][w] >> sh) << 16);
            if (c < CB)
                sb[(8 * c + t) * (kWgRow / 2) + p] = (rb[0][w] >> sh & 0xFFFFu) | ((rb[1][w] >> sh) << 16);
        }
        __syncthreads();
        if (ks + 1 < kend) fetch(ks + 1);  // in flight during the products
        if (blockIdx.y == 0) {
            const uint32_t *row = sa + (threadIdx.x >> 1) * (kWgRow / 2) + 8 * (threadIdx.x & 1);
#pragma unroll
            for (int j = 0; j < 8; ++j) bsum += bf2f((uint16_t)(row[j] & 0xFFFFu)) + bf2f((uint16_t)(row[j] >> 16));
        }
        const uint16_t *ta = reinterpret_cast<const uint16_t *>(sa);
        const uint16_t *tb = reinterpret_cast<const uint16_t *>(sb);
        bf16x8 fa[FM], fb[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) fa[i] = load8(ta + (wm * WM + 16 * i + r) * kWgRow + 8 * g);
#pragma unroll
        for (int j = 0; j < FN; ++j) fb[j] = load8(tb + (wn * WN + 16 * j + r) * kWgRow + 8 * g);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = mfma(fa[i], fb[j], acc[i][j]);
    }
    float *P = part + (size_t)blockIdx.z * ((size_t)M * N + M);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                P[(size_t)(m0 + wm * WM + 16 * i + 4 * g + q) * N + n0 + wn * WN + 16 * j + r] = acc[i][j][q];
    if (blockIdx.y == 0) {
        bsum += __shfl_xor(bsum, 1);  // the two halves of a row, low half first
        if ((threadIdx.x & 1) == 0) P[(size_t)M * N + m0 + (threadIdx.x >> 1)] = bsum;
    }
}

// out[e] = sum over z = 0 .. nz-1, in order, of part[z][e]; count % 4 == 0
__global__ __launch_bounds__(256) void reduce_parts(const float *__restrict__ part, int nz,
                                                    size_t count, float *__restrict__ out)
{
    const size_t e = ((size_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (e >= count) return;
    floatx4 s = {0, 0, 0, 0};
#pragma unroll 8
    for (int z = 0; z < nz; ++z) s += *reinterpret_cast<const floatx4 *>(part + (size_t)z * count + e);
    *reinterpret_cast<floatx4 *>(out + e) = s;
}

// Data gradient through one layer, computed transposed so each lane ends
// with four consecutive features of one sample: C[i][s] = sum over o of
// WT[i][o] dZ[s][o] (WT = W^T, 256 x 256; dZ sample-major), then
// Zp[s][i] = bf16(C[i][s]) where the layer input Hp[s][i] > 0, else 0.
// Tile 128 i x 128 s per workgroup, 64 x 64 per wave; operands straight
// from global memory (W^T stays in the caches).
__global__ __launch_bounds__(256) void dgrad(const uint16_t *__restrict__ WT,
                                             const uint16_t *__restrict__ dZ,
                                             const uint16_t *__restrict__ Hp,
                                             uint16_t *__restrict__ Zp)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    const int i0 = blockIdx.x * 128 + (wave & 1) * 64;
    const size_t s0 = (size_t)blockIdx.y * 128 + (wave >> 1) * 64;
    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kW; k += 32) {
        bf16x8 fa[4], fb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) fa[i] = load8(WT + (size_t)(i0 + 16 * i + r) * kW + k + 8 * g);
#pragma unroll
        for (int j = 0; j < 4; ++j) fb[j] = load8(dZ + (s0 + 16 * j + r) * kW + k + 8 * g);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma(fa[i], fb[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const size_t at = (s0 + 16 * j + r) * kW + i0 + 16 * i + 4 * g;
            const u32x2 h = *reinterpret_cast<const u32x2 *>(Hp + at);
            uint32_t w[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint32_t z = pack2(acc[i][j][2 * q], acc[i][j][2 * q + 1]);
                const uint32_t keep = ((h[q] & 0x8000u) == 0u && (h[q] & 0x7FFFu) != 0u ? 0x0000FFFFu : 0u) |
                                      ((h[q] & 0x80000000u) == 0u && (h[q] & 0x7FFF0000u) != 0u ? 0xFFFF0000u : 0u);
                w[q] = z & keep;
            }
            *reinterpret_cast<u32x2 *>(Zp + at) = u32x2{w[0], w[1]};
        }
}

// ------------------------------------------------------------------ elementwise
__global__ __launch_bounds__(256) void encode_x(const uint64_t *__restrict__ idx, int h,
                                                uint64_t count, uint16_t *__restrict__ X)
{
    const uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= count * kIn) return;
    const uint64_t s = e / kIn;
    X[e] = f2bf(input_at(idx[s], h, (int)(e % kIn)));
}

// T[c][r] = S[r][c] for a rows x cols BF16 matrix
__global__ __launch_bounds__(256) void transpose_bf16(const uint16_t *__restrict__ S,
                                                      uint16_t *__restrict__ T, int rows, int cols)
{
    __shared__ uint16_t tile[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int k = ty; k < 32; k += 8) tile[k][tx] = S[(size_t)(r0 + k) * cols + c0 + tx];
    __syncthreads();
    for (int k = ty; k < 32; k += 8) T[(size_t)(c0 + k) * rows + r0 + tx] = tile[tx][k];
}

// dZ3[s][o] = bf16(dy[s] * w4[o]) where H3[s][o] > 0, else 0 (the output layer's
// weight gradient sum_s dy[s] H3[s][o] is column_sums with weights dy)
__global__ __launch_bounds__(256) void head_backward(const float *__restrict__ dy,
                                                     const uint16_t *__restrict__ H3,
                                                     const uint16_t *__restrict__ wb, int count,
                                                     uint16_t *__restrict__ dZ3)
{
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)count * kW) return;
    const int o = (int)(e % kW);
    const size_t s = e / kW;
    const float h = bf2f(H3[e]);
    dZ3[e] = f2bf(h > 0.0f ? dy[s] * bf2f(wb[ow4 + o]) : 0.0f);
}


// part[k][c] = sum over the rows of chunk k (rows k*per .. k*per+per-1) of
// w[r] * M[r][c] in row order (w = null means 1), M BF16 rows x 256;
// reduce_columns then adds the chunks in a fixed order (deterministic).
__global__ __launch_bounds__(256) void column_sums_part(const uint16_t *__restrict__ M,
                                                        const float *__restrict__ w, int rows,
                                                        int per, float *__restrict__ part)
{
    const int c = threadIdx.x, k = blockIdx.x;
    const int r0 = k * per, r1 = min(rows, r0 + per);
    float s = 0.0f;
#pragma unroll 8
    for (int r = r0; r < r1; ++r) s += (w ? w[r] : 1.0f) * bf2f(M[(size_t)r * kW + c]);  // in order
    part[(size_t)k * kW + c] = s;
}

// out[e] = sum over z of part[z][e] (count outputs, nz parts), one wave per
// output: lane j adds parts j, j+64, ... in order, then a butterfly over the
// lanes (a fixed order)
__global__ __launch_bounds__(256) void reduce_columns(const float *__restrict__ part, int nz,
                                                      int count, float *__restrict__ out)
{
    const int e = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (e >= count) return;
    float s = 0.0f;
    for (int z = lane; z < nz; z += 64) s += part[(size_t)z * count + e];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) out[e] = s;
}

// Sums over one workgroup of WAVES waves in a fixed order: each thread's
// strided terms in index order, then a butterfly over the wave, then the
// waves in order (deterministic, and no serial loop over all partials).
template <int WAVES, typename A>
__device__ __forceinline__ A workgroup_sum(A s)
{
    __shared__ A part[WAVES];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    A t = part[0];
#pragma unroll
    for (int w = 1; w < WAVES; ++w) t += part[w];
    return t;
}

// One workgroup of 1024 threads; count % 4 == 0
__global__ __launch_bounds__(1024) void sum_vector(const float *__restrict__ v, int count,
                                                   float *__restrict__ out)
{
    float s = 0.0f;
#pragma unroll 4
    for (int k = 4 * threadIdx.x; k < count; k += 4 * 1024) {
        const floatx4 q = *reinterpret_cast<const floatx4 *>(v + k);
        s += ((q[0] + q[1]) + q[2]) + q[3];
    }
    s = workgroup_sum<16>(s);
    if (threadIdx.x == 0) *out = s;
}

// One workgroup of 1024 threads; count % 4 == 0
__global__ __launch_bounds__(1024) void mse_kernel(const float *__restrict__ y,
                                                   const float *__restrict__ t, int count,
                                                   float *__restrict__ dy, double *__restrict__ loss)
{
    double s = 0.0;
    const float scale = 2.0f / (float)count;
#pragma unroll 4
    for (int k = 4 * threadIdx.x; k < count; k += 4 * 1024) {
        const floatx4 a = *reinterpret_cast<const floatx4 *>(y + k);
        const floatx4 b = *reinterpret_cast<const floatx4 *>(t + k);
        floatx4 d;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float r = a[q] - b[q];
            d[q] = scale * r;
            s += (double)r * r;
        }
        *reinterpret_cast<floatx4 *>(dy + k) = d;
    }
    s = workgroup_sum<16>(s);
    if (threadIdx.x == 0) *loss = s / count;
}

__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ p, uint16_t *__restrict__ wb,
                                                   const float *__restrict__ g, float *__restrict__ m,
                                                   float *__restrict__ v, float lr, float b1, float b2,
                                                   float eps, float c1, float c2)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= kNParams) return;
    const float ge = g[e];
    const float me = b1 * m[e] + (1.0f - b1) * ge;
    const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float pe = p[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
    p[e] = pe;
    wb[e] = f2bf(pe);
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float *__restrict__ p,
                                                      uint16_t *__restrict__ wb, int count)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < count) wb[e] = f2bf(p[e]);
}

// SplitMix64 (Steele, Lea, Flood 2014): the mix of state (seed 2^32 + j + 1) * golden
__device__ __forceinline__ uint64_t splitmix(uint64_t seed, uint64_t j)
{
    uint64_t z = ((seed << 32) + j + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// He-uniform initialisation: weights of a layer with fan-in k uniform in
// (-sqrt(6/k), sqrt(6/k)) from SplitMix64 at counter e, biases 0.
__global__ __launch_bounds__(256) void init_kernel(float *__restrict__ p, uint64_t seed)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= kNParams) return;
    int fan = 0;
    if (e < ob1) fan = kIn;
    else if (e >= oW2 && e < ob2) fan = kW;
    else if (e >= oW3 && e < ob3) fan = kW;
    else if (e >= ow4 && e < ob4) fan = kW;
    if (!fan) { p[e] = 0.0f; return; }
    const double u = (double)(splitmix(seed, (uint64_t)e) >> 11) * 0x1.0p-53;  // [0, 1)
    p[e] = (float)((2.0 * u - 1.0) * sqrt(6.0 / fan));
}

template <typename T>
__global__ __launch_bounds__(256) void sample_kernel(const T *__restrict__ table, int bits,
                                                     uint64_t seed, int count,
                                                     uint64_t *__restrict__ idx,
                                                     float *__restrict__ target)
{
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= count) return;
    const uint64_t i = splitmix(seed, (uint64_t)s) >> (64 - bits);
    idx[s] = i;
    // the table stores the indices with string-1 head 0; i reads its complement otherwise
    const uint64_t is = ((i >> (bits - 1)) & 1) ? i ^ ((1ull << bits) - 1) : i;
    target[s] = (float)((double)table[is] - (double)table[0]);
}

}  // namespace

// ------------------------------------------------------------------ launchers
MlpWs mlp_ws_layout(int64_t batch)
{
    MlpWs w;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o += (bytes + 255) & ~size_t(255); return at; };
    const size_t B = (size_t)batch;
    w.act = take(3 * B * kW * 2);
    w.X = take(B * kIn * 2);
    w.dZ = take(B * kW * 2);
    w.T1 = take(B * kW * 2);            // the other dZ of the ping-pong
    w.WT = take((size_t)2 * kW * kW * 2);
    // batch splits of the weight gradients: enough workgroups for the chip
    w.splits = (int)std::min<int64_t>(64, std::max<int64_t>(1, batch / 256));
    w.part = take((size_t)w.splits * (kW * kW + kW) * 4);
    w.bytes = o;
    return w;
}

hipError_t launch_mlp_forward(const uint16_t *wb, const float *pf, const uint64_t *idx, int h,
                              int64_t count, float *y, uint16_t *act, hipStream_t s)
{
    FwdArgs a{};
    a.wb = wb; a.pf = pf; a.idx = idx; a.count = (uint64_t)count; a.h = h; a.y = y; a.act = act;
    const uint64_t nb = ((uint64_t)count + kFwdSamples - 1) / kFwdSamples;
    const unsigned grid = (unsigned)std::min<uint64_t>(nb, 256ull * 8);
    if (act)
        mlp_fwd<kSrcIdx, true, float><<<grid, kFwdThreads, 0, s>>>(a);
    else
        mlp_fwd<kSrcIdx, false, float><<<grid, kFwdThreads, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_mlp_seed(const Geometry &g, int dtype, const uint16_t *wb, const float *pf,
                           void *lag1, void *lag2, double rate, hipStream_t s)
{
    FwdArgs a{};
    a.wb = wb; a.pf = pf; a.h = g.h; a.lag1 = lag1; a.lag2 = lag2;
    a.count = ((1ull << g.h) + 2) << (g.h - 2);  // orbits of exchange and complement
    a.n = g.n; a.rate = rate;
    const uint64_t nb = (a.count + kFwdSamples - 1) / kFwdSamples;
    const unsigned grid = (unsigned)std::min<uint64_t>(nb, 256ull * 8);
    if (dtype == LCSB_F32)
        mlp_fwd<kSrcOrbits, false, float><<<grid, kFwdThreads, 0, s>>>(a);
    else
        mlp_fwd<kSrcOrbits, false, double><<<grid, kFwdThreads, 0, s>>>(a);
    return hipGetLastError();
}

static hipError_t column_sums(const uint16_t *M, const float *w, int rows, float *part, float *out,
                              hipStream_t s)
{
    const int chunks = std::min(256, (rows + 63) / 64), per = (rows + chunks - 1) / chunks;
    column_sums_part<<<chunks, 256, 0, s>>>(M, w, rows, per, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    reduce_columns<<<kW / 4, 256, 0, s>>>(part, chunks, kW, out);
    return hipGetLastError();
}

static hipError_t weight_grad(const uint16_t *A, const uint16_t *Bm, int ldb, int B, int splits,
                              float *part, float *out, hipStream_t s)
{
    const int ksteps = B / 32, per = (ksteps + splits - 1) / splits;
    const int used = (ksteps + per - 1) / per;
    const int N = ldb;
    if (N == kW)
        wgrad<128><<<dim3(kW / 128, kW / 128, used), 256, 0, s>>>(A, kW, Bm, ldb, ksteps, per, kW, N, part);
    else
        wgrad<32><<<dim3(kW / 128, 1, used), 256, 0, s>>>(A, kW, Bm, ldb, ksteps, per, kW, N, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t count = (size_t)kW * N + kW;  // weights, then the biases that follow them
    reduce_parts<<<(unsigned)((count / 4 + 255) / 256), 256, 0, s>>>(part, used, count, out);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(const uint16_t *wb, const float *dy, int64_t count,
                               unsigned char *ws, const MlpWs &L, const uint64_t *idx, int h,
                               float *grad, hipStream_t s)
{
    const int B = (int)count;
    uint16_t *H1 = reinterpret_cast<uint16_t *>(ws + L.act);
    uint16_t *H2 = H1 + (size_t)B * kW;
    uint16_t *H3 = H2 + (size_t)B * kW;
    uint16_t *X = reinterpret_cast<uint16_t *>(ws + L.X);
    uint16_t *dZa = reinterpret_cast<uint16_t *>(ws + L.dZ);
    uint16_t *dZb = reinterpret_cast<uint16_t *>(ws + L.T1);
    uint16_t *WT = reinterpret_cast<uint16_t *>(ws + L.WT);
    float *part = reinterpret_cast<float *>(ws + L.part);
    const unsigned ew = (unsigned)(((size_t)B * kW + 255) / 256);
    hipError_t e;
#define LCSB_TRY(x) do { if ((e = (x)) != hipSuccess) return e; } while (0)
    // layer 4: gw4 = sum_s dy[s] H3[s][:], gb4 = sum_s dy[s]; dZ3
    LCSB_TRY(column_sums(H3, dy, B, part, grad + ow4, s));
    sum_vector<<<1, 1024, 0, s>>>(dy, B, grad + ob4);
    LCSB_TRY(hipGetLastError());
    head_backward<<<ew, 256, 0, s>>>(dy, H3, wb, B, dZa);
    LCSB_TRY(hipGetLastError());
    transpose_bf16<<<dim3(kW / 32, kW / 32), 256, 0, s>>>(wb + oW3, WT, kW, kW);
    LCSB_TRY(hipGetLastError());
    transpose_bf16<<<dim3(kW / 32, kW / 32), 256, 0, s>>>(wb + oW2, WT + kW * kW, kW, kW);
    LCSB_TRY(hipGetLastError());
    // layer 3: gW3, gb3 from dZ3 and H2; dZ2 = relu'(H2) (dZ3 W3)
    LCSB_TRY(weight_grad(dZa, H2, kW, B, L.splits, part, grad + oW3, s));
    dgrad<<<dim3(kW / 128, B / 128), 256, 0, s>>>(WT, dZa, H2, dZb);
    LCSB_TRY(hipGetLastError());
    // layer 2: gW2, gb2 from dZ2 and H1; dZ1 = relu'(H1) (dZ2 W2)
    LCSB_TRY(weight_grad(dZb, H1, kW, B, L.splits, part, grad + oW2, s));
    dgrad<<<dim3(kW / 128, B / 128), 256, 0, s>>>(WT + kW * kW, dZb, H1, dZa);
    LCSB_TRY(hipGetLastError());
    // layer 1: gW1, gb1 from dZ1 and the encoded inputs
    encode_x<<<(unsigned)(((size_t)B * kIn + 255) / 256), 256, 0, s>>>(idx, h, (uint64_t)B, X);
    LCSB_TRY(hipGetLastError());
    LCSB_TRY(weight_grad(dZa, X, kIn, B, L.splits, part, grad + oW1, s));
#undef LCSB_TRY
    return hipSuccess;
}

hipError_t launch_mlp_mse(const float *y, const float *t, int64_t count, float *dy, double *loss,
                          hipStream_t s)
{
    mse_kernel<<<1, 1024, 0, s>>>(y, t, (int)count, dy, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *p, uint16_t *wb, const float *g, float *m, float *v, float lr,
                           float b1, float b2, float eps, int64_t t, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)t);
    const float c2 = 1.0f - powf(b2, (float)t);
    adam_kernel<<<(kNParams + 255) / 256, 256, 0, s>>>(p, wb, g, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *p, uint16_t *wb, hipStream_t s)
{
    to_bf16_kernel<<<(kNParams + 255) / 256, 256, 0, s>>>(p, wb, kNParams);
    return hipGetLastError();
}

hipError_t launch_mlp_init(float *p, uint64_t seed, hipStream_t s)
{
    init_kernel<<<(kNParams + 255) / 256, 256, 0, s>>>(p, seed);
    return hipGetLastError();
}

hipError_t launch_mlp_sample(const void *table, int dtype, int bits, uint64_t seed, int64_t count,
                             uint64_t *idx, float *target, hipStream_t s)
{
    const unsigned grid = (unsigned)((count + 255) / 256);
    if (dtype == LCSB_F32)
        sample_kernel<float><<<grid, 256, 0, s>>>(static_cast<const float *>(table), bits, seed,
                                                  (int)count, idx, target);
    else
        sample_kernel<double><<<grid, 256, 0, s>>>(static_cast<const double *>(table), bits, seed,
                                                   (int)count, idx, target);
    return hipGetLastError();
}

}  // namespace lcsb
