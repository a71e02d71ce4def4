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
//
// Unlike the sweep, this evaluates every coordinate and assumes no symmetry
// of u, so the certificate holds for any table.  FP32 tables are certified as
// their exact FP64 values: the certificate is translation invariant, so the
// FP64 offset of an FP32 table does not enter W; it enters only R.
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

template <typename T>
__global__ __launch_bounds__(kBlock) void cert_r(const T *__restrict__ u,
                                                const T *__restrict__ prev, uint64_t n,
                                                unsigned char *__restrict__ ws)
{
    double best = -INFINITY;
    uint64_t arg = 0, nonfinite = 0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += stride) {
        const double a = (double)u[j], b = (double)prev[j];
        if (!isfinite(a) || !isfinite(b)) ++nonfinite;
        const double diff = a - b;
        if (diff > best) { best = diff; arg = j; }
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
    for (int k = threadIdx.x; k < nparts; k += kBlock) {
        merge_max_idx(best, arg, reinterpret_cast<const double *>(ws + Ws::kPartVal)[k],
                      reinterpret_cast<const uint64_t *>(ws + Ws::kPartIdx)[k]);
        nonfinite += reinterpret_cast<const uint64_t *>(ws + Ws::kPartCnt)[k];
    }
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

// Offset, inside the lowest slot, of the t-th appended tuple of the strings
// in SET: lexicographic order, the smallest string index most significant.
template <int SIGMA, int D, int SET>
__device__ __forceinline__ constexpr uint64_t tuple_offset(int t)
{
    constexpr int BETA = SIGMA == 2 ? 1 : 2;
    uint64_t o = 0;
    int rest = t;
    for (int j = D - 1; j >= 0; --j)
        if ((SET >> j) & 1) {
            o |= (uint64_t)(rest & (SIGMA - 1)) << (BETA * (D - 1 - j));
            rest >>= BETA;
        }
    return o;
}

// Mean over the branch advancing the strings in SET (Algorithm 1), every
// operation rounded toward -inf; reads u + (d-k)R with k = |SET|.
// smask[j] = the symbol field of string j replicated over every position.
template <int SIGMA, int D, int SET, typename T>
__device__ __forceinline__ double branch_mean_rd(const T *__restrict__ u, uint64_t i, uint64_t n,
                                                 const uint64_t *smask, const double *shift)
{
    constexpr int BETA = SIGMA == 2 ? 1 : 2;
    constexpr int SLOT = BETA * D;
    constexpr int K = __builtin_popcount(SET);
    constexpr int CNT = 1 << (BETA * K);
    uint64_t sm = 0;
#pragma unroll
    for (int j = 0; j < D; ++j)
        if ((SET >> j) & 1) sm |= smask[j];
    const uint64_t base = (i & ~sm) | ((i << SLOT) & sm & (n - 1));
    double v[CNT];
#pragma unroll
    for (int t = 0; t < CNT; ++t)
        v[t] = add_rd((double)u[base | tuple_offset<SIGMA, D, SET>(t)], shift[K]);
#pragma unroll
    for (int step = 1; step < CNT; step <<= 1)
#pragma unroll
        for (int t = 0; t < CNT; t += 2 * step) v[t] = add_rd(v[t], v[t + step]);
    return scale_pow2_rd(v[0], BETA * K);
}

// max over the branch sets that occur (bit SET of `occurs`); order-free (max)
template <int SIGMA, int D, int SET, typename T>
__device__ __forceinline__ void max_branches(const T *__restrict__ u, uint64_t i, uint64_t n,
                                             uint32_t occurs, const uint64_t *smask,
                                             const double *shift, double &best)
{
    if constexpr (SET > 0) {
        if ((occurs >> SET) & 1u) {
            const double m = branch_mean_rd<SIGMA, D, SET, T>(u, i, n, smask, shift);
            if (m > best) best = m;
        }
        max_branches<SIGMA, D, SET - 1, T>(u, i, n, occurs, smask, shift, best);
    }
}

// W[i] = (u[i] + dR) - F(u + shift_1, .., u + shift_d)[i]: F rounded down,
// the two outer operations rounded up.
template <int SIGMA, int D, typename T>
__device__ double w_at(const T *__restrict__ u, uint64_t i, uint64_t n, int h,
                       const uint64_t *smask, const double *shift, double dR_up)
{
    constexpr int BETA = SIGMA == 2 ? 1 : 2;
    constexpr int SLOT = BETA * D;
    const int top = SLOT * (h - 1);
    int hs[D];
#pragma unroll
    for (int j = 0; j < D; ++j) hs[j] = (int)((i >> (top + BETA * (D - 1 - j))) & (SIGMA - 1));
    bool all_match = true;
#pragma unroll
    for (int j = 1; j < D; ++j) all_match = all_match && hs[j] == hs[0];
    // N_z = strings whose head is not z; the empty set (z = common head) is skipped
    uint32_t occurs = 0;
#pragma unroll
    for (int z = 0; z < SIGMA; ++z) {
        uint32_t set = 0;
#pragma unroll
        for (int j = 0; j < D; ++j)
            if (hs[j] != z) set |= 1u << j;
        occurs |= 1u << set;
    }
    occurs &= ~1u;
    double best = -INFINITY;
    max_branches<SIGMA, D, (1 << D) - 1, T>(u, i, n, occurs, smask, shift, best);
    const double f_lo = all_match ? add_rd(1.0, best) : best;
    return add_ru(add_ru((double)u[i], dR_up), -f_lo);
}

template <int SIGMA, int D, typename T>
__global__ __launch_bounds__(kBlock) void cert_w(const T *__restrict__ u, uint64_t n, int h,
                                                unsigned char *__restrict__ ws)
{
    constexpr int BETA = SIGMA == 2 ? 1 : 2;
    constexpr int SLOT = BETA * D;
    const double *sc = reinterpret_cast<const double *>(ws);
    const double dR_up = sc[Ws::kDRup / 8];
    double shift[D + 1];
#pragma unroll
    for (int k = 0; k <= D; ++k) shift[k] = sc[Ws::kShift / 8 + k];  // (d-k)R, rounded down
    uint64_t rep = (n - 1) / ((1ull << SLOT) - 1);  // 1 in the lowest bit of every slot
    uint64_t smask[D];
#pragma unroll
    for (int j = 0; j < D; ++j) smask[j] = (rep * (((1ull << BETA) - 1))) << (BETA * (D - 1 - j));

    double best = -INFINITY;
    uint64_t arg = 0, nonfinite = 0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += stride) {
        const double w = w_at<SIGMA, D, T>(u, j, n, h, smask, shift, dR_up);
        if (!isfinite(w)) ++nonfinite;
        if (w > best) { best = w; arg = j; }
    }
    block_reduce(best, arg, nonfinite);
    if (threadIdx.x == 0) {
        reinterpret_cast<double *>(ws + Ws::kPartVal)[blockIdx.x] = best;
        reinterpret_cast<uint64_t *>(ws + Ws::kPartIdx)[blockIdx.x] = arg;
        reinterpret_cast<uint64_t *>(ws + Ws::kPartCnt)[blockIdx.x] = nonfinite;
    }
}

__global__ __launch_bounds__(kBlock) void cert_w_final(unsigned char *__restrict__ ws, int nparts)
{
    double best = -INFINITY;
    uint64_t arg = 0, nonfinite = 0;
    for (int k = threadIdx.x; k < nparts; k += kBlock) {
        merge_max_idx(best, arg, reinterpret_cast<const double *>(ws + Ws::kPartVal)[k],
                      reinterpret_cast<const uint64_t *>(ws + Ws::kPartIdx)[k]);
        nonfinite += reinterpret_cast<const uint64_t *>(ws + Ws::kPartCnt)[k];
    }
    block_reduce(best, arg, nonfinite);
    if (threadIdx.x == 0) {
        reinterpret_cast<double *>(ws)[Ws::kMaxW / 8] = best;
        reinterpret_cast<uint64_t *>(ws)[Ws::kArgmax / 8] = arg;
        reinterpret_cast<uint64_t *>(ws)[Ws::kNonfinite / 8] = nonfinite;
    }
}

int reduce_blocks(uint64_t n)
{
    uint64_t b = (n + kBlock - 1) / kBlock;
    return (int)(b < (uint64_t)kMaxReduceBlocks ? b : (uint64_t)kMaxReduceBlocks);
}

template <typename T>
hipError_t launch_w(const Geometry &g, const T *u, unsigned char *ws, int nb, hipStream_t s)
{
    if (g.sigma == 2 && g.d == 2)
        cert_w<2, 2, T><<<nb, kBlock, 0, s>>>(u, g.n, g.h, ws);
    else if (g.sigma == 4 && g.d == 2)
        cert_w<4, 2, T><<<nb, kBlock, 0, s>>>(u, g.n, g.h, ws);
    else if (g.sigma == 2 && g.d == 3)
        cert_w<2, 3, T><<<nb, kBlock, 0, s>>>(u, g.n, g.h, ws);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T>
hipError_t certify_typed(const Geometry &g, const void *u, const void *prev, int u_slot,
                         int prev_slot, unsigned char *ws, hipStream_t s)
{
    const int nb = reduce_blocks(g.n);
    cert_r<T><<<nb, kBlock, 0, s>>>(static_cast<const T *>(u), static_cast<const T *>(prev),
                                     g.n, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    cert_r_final<<<1, kBlock, 0, s>>>(ws, nb, g.d, std::is_same<T, float>::value ? 1 : 0,
                                      u_slot, prev_slot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_w<T>(g, static_cast<const T *>(u), ws, nb, s)) != hipSuccess) return e;
    cert_w_final<<<1, kBlock, 0, s>>>(ws, nb);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_certify(const Geometry &g, int dtype, const void *u, const void *prev,
                          int u_slot, int prev_slot, unsigned char *ws, hipStream_t s)
{
    return dtype == LCSB_F32 ? certify_typed<float>(g, u, prev, u_slot, prev_slot, ws, s)
                             : certify_typed<double>(g, u, prev, u_slot, prev_slot, ws, s);
}

}  // namespace lcsb
