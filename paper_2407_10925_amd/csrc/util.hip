// Small device kernels around the sweep: clearing, copying a ring in,
// FP32 -> FP64 conversion for the FP64 polish, and the exchange-symmetry check
// and completion of sigma = d = 2 tables.  Fill kernels stand in for hipMemsetAsync so that the calls
// stay valid inside captured HIP graphs.
#include "internal.h"

namespace lcsb {
namespace {

__global__ __launch_bounds__(kBlock) void fill_u32(uint32_t *__restrict__ p, uint64_t words,
                                                   uint32_t v)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t quads = words >> 2;
    uint4 q = make_uint4(v, v, v, v);
    for (uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < quads; j += stride)
        reinterpret_cast<uint4 *>(p)[j] = q;
    for (uint64_t j = (quads << 2) + (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < words;
         j += stride)
        p[j] = v;
}

__global__ __launch_bounds__(kBlock) void fill_f64_kernel(double *__restrict__ p, uint64_t count,
                                                          double v)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < count; j += stride) p[j] = v;
}

// dst[0 .. words) = src[0 .. words); 16-byte vectors when both are aligned
__global__ __launch_bounds__(kBlock) void copy_u32(const uint32_t *__restrict__ src,
                                                   uint32_t *__restrict__ dst, uint64_t words,
                                                   int vec)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t quads = vec ? words >> 2 : 0;
    for (uint64_t j = (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < quads; j += stride)
        reinterpret_cast<uint4 *>(dst)[j] = reinterpret_cast<const uint4 *>(src)[j];
    for (uint64_t j = (quads << 2) + (uint64_t)blockIdx.x * kBlock + threadIdx.x; j < words;
         j += stride)
        dst[j] = src[j];
}

__global__ __launch_bounds__(kBlock) void upcast_kernel(const float *__restrict__ src,
                                                        const double *__restrict__ offset,
                                                        double *__restrict__ dst, uint64_t n)
{
    const double o = *offset;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        dst[i] = o + (double)src[i];
}

// In-place widening, one range [lo, hi) of a table whose FP32 values sit in
// the first half of its FP64 buffer: reads bytes [4 lo, 4 hi), writes bytes
// [8 lo, 8 hi).  For lo = hi / 2 the two ranges are disjoint, and every byte
// written was read by an earlier range (larger indices go first), so ranges
// launched from the top down never read a widened value.  No restrict: the
// two pointers alias.
__global__ __launch_bounds__(kBlock) void upcast_range(const float *src, const double *offset,
                                                       double *dst, uint64_t lo, uint64_t hi)
{
    const double o = *offset;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = lo + (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < hi; i += stride) {
        const float v = src[i];
        dst[i] = o + (double)v;
    }
}

// the stored index of the exchanged twin of stored index i: D = 2 or 3 for
// sigma = 2 (d = D), 4 for sigma = 4, d = 2
template <int D>
__device__ __forceinline__ uint64_t twin_of(uint64_t i, uint64_t n)
{
    if constexpr (D == 4) return exchange_twin4(i, n);
    else return exchange_twin(i, n, D);
}

// raise *flag if a stored entry differs, bit for bit, from the stored entry
// of its tuple with strings 1 and 2 exchanged
template <typename W, int D>
__global__ __launch_bounds__(kBlock) void check_swap_kernel(const W *__restrict__ v, uint64_t n,
                                                            uint32_t *__restrict__ flag)
{
    const uint64_t ns = D == 4 ? n >> 2 : n >> 1;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    bool bad = false;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < ns; i += stride)
        bad = bad || v[i] != v[twin_of<D>(i, n)];
    if (bad) *flag = 1u;
}

// a lazily written table: every stored entry that is the upper index of its
// exchanged pair takes the value of the lower one (reads only lower entries,
// writes only upper ones)
template <typename W, int D>
__global__ __launch_bounds__(kBlock) void materialize_swap_kernel(W *__restrict__ v, uint64_t n)
{
    const uint64_t ns = D == 4 ? n >> 2 : n >> 1;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < ns; i += stride) {
        const uint64_t js = twin_of<D>(i, n);
        if (js < i) v[i] = v[js];
    }
}

// the D of twin_of for a shape, or 0 when no exchange fold applies
int swap_kind(const Geometry &g)
{
    if (g.h < 2 || (g.d != 2 && g.d != 3)) return 0;
    if (g.sigma == 2) return g.d;
    return g.sigma == 4 && g.d == 2 ? 4 : 0;
}


unsigned grid_for(uint64_t work)
{
    uint64_t b = (work + kBlock - 1) / kBlock;
    const uint64_t cap = 256ull * 64;  // 64 workgroups per CU on 256 CUs, grid-stride beyond
    if (b > cap) b = cap;
    return (unsigned)(b ? b : 1);
}

}  // namespace

hipError_t launch_check_swap(const Geometry &g, int dtype, const void *table, uint32_t *flag,
                             hipStream_t s)
{
    const int kind = swap_kind(g);
    const unsigned grid = grid_for(g.ns);
    const uint32_t *t32 = static_cast<const uint32_t *>(table);
    const uint64_t *t64 = static_cast<const uint64_t *>(table);
    const bool f32 = dtype == LCSB_F32;
    switch (kind) {
    case 2:
        if (f32) check_swap_kernel<uint32_t, 2><<<grid, kBlock, 0, s>>>(t32, g.n, flag);
        else check_swap_kernel<uint64_t, 2><<<grid, kBlock, 0, s>>>(t64, g.n, flag);
        break;
    case 3:
        if (f32) check_swap_kernel<uint32_t, 3><<<grid, kBlock, 0, s>>>(t32, g.n, flag);
        else check_swap_kernel<uint64_t, 3><<<grid, kBlock, 0, s>>>(t64, g.n, flag);
        break;
    case 4:
        if (f32) check_swap_kernel<uint32_t, 4><<<grid, kBlock, 0, s>>>(t32, g.n, flag);
        else check_swap_kernel<uint64_t, 4><<<grid, kBlock, 0, s>>>(t64, g.n, flag);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_materialize_swap(const Geometry &g, int dtype, void *table, hipStream_t s)
{
    const int kind = swap_kind(g);
    const unsigned grid = grid_for(g.ns);
    uint32_t *t32 = static_cast<uint32_t *>(table);
    uint64_t *t64 = static_cast<uint64_t *>(table);
    const bool f32 = dtype == LCSB_F32;
    switch (kind) {
    case 2:
        if (f32) materialize_swap_kernel<uint32_t, 2><<<grid, kBlock, 0, s>>>(t32, g.n);
        else materialize_swap_kernel<uint64_t, 2><<<grid, kBlock, 0, s>>>(t64, g.n);
        break;
    case 3:
        if (f32) materialize_swap_kernel<uint32_t, 3><<<grid, kBlock, 0, s>>>(t32, g.n);
        else materialize_swap_kernel<uint64_t, 3><<<grid, kBlock, 0, s>>>(t64, g.n);
        break;
    case 4:
        if (f32) materialize_swap_kernel<uint32_t, 4><<<grid, kBlock, 0, s>>>(t32, g.n);
        else materialize_swap_kernel<uint64_t, 4><<<grid, kBlock, 0, s>>>(t64, g.n);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, uint64_t bytes, hipStream_t s)
{
    if (bytes % 4) return hipErrorInvalidValue;
    const uint64_t words = bytes / 4;
    fill_u32<<<grid_for(words / 4), kBlock, 0, s>>>(static_cast<uint32_t *>(p), words, 0u);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, uint64_t count, double v, hipStream_t s)
{
    fill_f64_kernel<<<grid_for(count), kBlock, 0, s>>>(p, count, v);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, uint64_t bytes, hipStream_t s)
{
    if (bytes % 4 || ((uintptr_t)src & 3) || ((uintptr_t)dst & 3)) return hipErrorInvalidValue;
    const uint64_t words = bytes / 4;
    const int vec = (((uintptr_t)src | (uintptr_t)dst) & 15) == 0;
    copy_u32<<<grid_for(vec ? words / 4 : words), kBlock, 0, s>>>(
        static_cast<const uint32_t *>(src), static_cast<uint32_t *>(dst), words, vec);
    return hipGetLastError();
}

hipError_t launch_upcast(const Geometry &g, const float *src, const double *offset_dev,
                         double *dst, hipStream_t s)
{
    upcast_kernel<<<grid_for(g.ns), kBlock, 0, s>>>(src, offset_dev, dst, g.ns);
    return hipGetLastError();
}

hipError_t launch_upcast_inplace(const Geometry &g, void *buf, const double *offset_dev,
                                 hipStream_t s)
{
    const float *src = static_cast<const float *>(buf);
    double *dst = static_cast<double *>(buf);
    for (uint64_t hi = g.ns; hi > 0;) {
        const uint64_t lo = hi / 2;
        upcast_range<<<grid_for(hi - lo), kBlock, 0, s>>>(src, offset_dev, dst, lo, hi);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hi = lo;
    }
    return hipSuccess;
}

}  // namespace lcsb
