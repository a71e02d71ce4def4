// Small device kernels around the sweep: clearing, loading a ring with the
// symbol-relabelling symmetry enforced, and FP32 -> FP64 conversion for the
// FP64 polish.  Fill kernels stand in for hipMemsetAsync so that the calls
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

// dst[i] = src[representative of i]: the representative has string-1 head 0
// and is reached by xor-ing every symbol with the string-1 head of i.
template <typename T>
__global__ __launch_bounds__(kBlock) void project_copy(const T *__restrict__ src,
                                                       T *__restrict__ dst, uint64_t n,
                                                       int head_shift, uint64_t sym_mask,
                                                       uint64_t sym_rep)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const uint64_t m = (i >> head_shift) & sym_mask;
        dst[i] = src[i ^ (m * sym_rep)];
    }
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

unsigned grid_for(uint64_t work)
{
    uint64_t b = (work + kBlock - 1) / kBlock;
    const uint64_t cap = 256ull * 64;  // 64 workgroups per CU on 256 CUs, grid-stride beyond
    if (b > cap) b = cap;
    return (unsigned)(b ? b : 1);
}

}  // namespace

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

hipError_t launch_project_copy(const Geometry &g, int dtype, const void *src, void *dst,
                               hipStream_t s)
{
    const int head_shift = g.slot * (g.h - 1) + g.beta * (g.d - 1);
    const uint64_t sym_mask = (uint64_t)g.sigma - 1;
    const uint64_t sym_rep = (g.n - 1) / sym_mask;  // 1 in the lowest bit of every symbol
    if (dtype == LCSB_F32)
        project_copy<float><<<grid_for(g.n), kBlock, 0, s>>>(
            static_cast<const float *>(src), static_cast<float *>(dst), g.n, head_shift,
            sym_mask, sym_rep);
    else
        project_copy<double><<<grid_for(g.n), kBlock, 0, s>>>(
            static_cast<const double *>(src), static_cast<double *>(dst), g.n, head_shift,
            sym_mask, sym_rep);
    return hipGetLastError();
}

hipError_t launch_upcast(const Geometry &g, const float *src, const double *offset_dev,
                         double *dst, hipStream_t s)
{
    upcast_kernel<<<grid_for(g.n), kBlock, 0, s>>>(src, offset_dev, dst, g.n);
    return hipGetLastError();
}

}  // namespace lcsb
