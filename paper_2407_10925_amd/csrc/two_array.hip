// The rate of the two-array iteration (a reading of the remark of Sec. 3.3
// that the recurrence runs on two arrays): one table u and a rate R, the
// step u_new = F(u, u - R, .., u - (d-1) R) with the shift added to each
// branch mean (the sweep kernels' delta_k).  R of the next step is the mean
// growth over a fixed sample of 4096 coordinates of the stored half,
// c_i = (i * 0x9E3779B97F4A7C15 mod 2^64) mod (n / sigma), summed as one
// balanced binary tree over i in order; this pass also sets the per-lag
// offsets the next sweep reads.  One workgroup: thread t holds leaves
// 16t .. 16t+15, whose balanced tree is a subtree of the whole one, and the
// 256 partial sums are combined pairwise up the tree (wave shuffles, then
// the four waves).
#include <type_traits>

#include "internal.h"

namespace lcsb {
namespace {

constexpr int kSample = kRateSample;
constexpr uint64_t kSampleMul = kRateSampleMul;
static_assert(kSample == 16 * kBlock, "sixteen leaves per thread");

// swap (0, 2, 3: sigma = 2 with d = swap; 4: sigma = 4, d = 2): a lazily
// written exchange-symmetric table, read at the lower index of each pair;
// packed_h > 0: exchange-packed tables of l = packed_h, read at the code of
// each coordinate (packed_index)
template <typename T>
__global__ __launch_bounds__(kBlock) void rate_kernel(const T *__restrict__ nw,
                                                     const T *__restrict__ old, uint64_t n,
                                                     uint64_t ns, int swap, int packed_h,
                                                     double *__restrict__ off, int s_new,
                                                     int s_old, double *__restrict__ rate,
                                                     const T *__restrict__ nw_smp,
                                                     const T *__restrict__ old_smp)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    double v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint64_t i = 16 * (uint64_t)threadIdx.x + (uint64_t)j;
        uint64_t c = (i * kSampleMul) & (ns - 1);  // ns is a power of two
        if (packed_h) {
            c = packed_index(c, packed_h);
        } else if (swap) {
            const uint64_t tw = swap == 4 ? exchange_twin4(c, n) : exchange_twin(c, n, swap);
            c = tw < c ? tw : c;
        }
        v[j] = (double)(nw_smp ? nw_smp[i] : nw[c]) - (double)(old_smp ? old_smp[i] : old[c]);
    }
#pragma unroll
    for (int step = 1; step < 16; step <<= 1)
#pragma unroll
        for (int k = 0; k < 16; k += 2 * step) v[k] = v[k] + v[k + step];
    double p = v[0];
    // lane L ends each level holding the tree over partials L .. L + 2 width - 1
    // (only the lanes that are multiples of the width are used above it)
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double q = __shfl_down(p, o);
        p = p + q;
    }
    __shared__ double wsum[kBlock / 64];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        static_assert(kBlock / 64 == 4, "four waves");
        const double sum = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
        double R = sum / (double)kSample;
        double base = 0.0;
        if constexpr (kF32) {  // true values are offset + stored value
            R = R + (off[s_new] - off[s_old]);
            base = off[s_new];
            off[Ws::kSlotLag2] = base - R;
            off[Ws::kSlotLag3] = base - 2.0 * R;
        } else {  // FP64 tables carry no offset: the sweep reads delta_k = -(k-1) R
            off[Ws::kSlotLag2] = -R;
            off[Ws::kSlotLag3] = -(2.0 * R);
        }
        *rate = R;
    }
}

}  // namespace

hipError_t launch_two_array_rate(const Geometry &g, int dtype, const void *nw, const void *old,
                                 int s_new, int s_old, int swap_sym, int packed,
                                 unsigned char *ws, hipStream_t s, const void *nw_smp,
                                 const void *old_smp)
{
    const int packed_h = packed ? g.h : 0;
    int swap = 0;
    if (swap_sym) swap = g.sigma == 4 ? 4 : g.d;
    double *off = reinterpret_cast<double *>(ws + Ws::kOffsets);
    double *rate = reinterpret_cast<double *>(ws + Ws::kRate);
    if (dtype == LCSB_F32)
        rate_kernel<float><<<1, kBlock, 0, s>>>(static_cast<const float *>(nw),
                                                static_cast<const float *>(old), g.n, g.ns, swap,
                                                packed_h, off, s_new, s_old, rate,
                                                static_cast<const float *>(nw_smp),
                                                static_cast<const float *>(old_smp));
    else
        rate_kernel<double><<<1, kBlock, 0, s>>>(static_cast<const double *>(nw),
                                                 static_cast<const double *>(old), g.n, g.ns, swap,
                                                 packed_h, off, s_new, s_old, rate,
                                                 static_cast<const double *>(nw_smp),
                                                 static_cast<const double *>(old_smp));
    return hipGetLastError();
}

}  // namespace lcsb
