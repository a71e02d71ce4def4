// The allocation-free certificate: lcsb_certify_optimal_noalloc (include/lcsb.h)
// runs the largest-r pass with its scratch (reduction partials and scalars)
// in a file-scope device array instead of a context's bound workspace, and
// writes its result to caller device memory, so it allocates nothing and
// never waits on the host.
//
// Each device holds its own copy of `scratch` at its own address: the host
// looks that address up once per device (hipGetSymbolAddress, with the
// device current) and passes it to the kernels; the array's name in host
// code is only a host-side stand-in.  Every call on one device shares the
// array, so calls that overlap on one device race.
#include <mutex>
#include <string>

#include "internal.h"

namespace lcsb {
namespace {

constexpr size_t kScratchBytes = Ws::kBytes;  // fixed: at most kMaxReduceBlocks partials
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices];

// this device's address of `scratch` (looked up on its first use here)
hipError_t scratch_address(void **ptr)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

int certify_optimal_noalloc(int sigma, int d, int h, int dtype, const void *u,
                            int exchange_symmetric, double *dev_out, void *stream,
                            std::string *err)
{
    const bool ok = (sigma == 2 && d == 2) || (sigma == 4 && d == 2) || (sigma == 2 && d == 3);
    if (!ok) { *err = "no GPU kernel for this (sigma, d)"; return LCSB_EUNSUPPORTED; }
    if (dtype != LCSB_F64 && dtype != LCSB_F32) { *err = "dtype"; return LCSB_EINVAL; }
    const int beta = sigma == 2 ? 1 : 2;
    if (h < 1 || beta * d * h > 36) { *err = "need h >= 1 and sigma^(d h) <= 2^36"; return LCSB_EINVAL; }
    if (!u || !dev_out) { *err = "null table or output"; return LCSB_EINVAL; }
    if ((uintptr_t)u & 15) { *err = "table not 16-byte aligned"; return LCSB_EINVAL; }
    Geometry g;
    g.sigma = sigma;
    g.d = d;
    g.h = h;
    g.beta = beta;
    g.slot = beta * d;
    g.n = 1ull << (beta * d * h);
    g.ns = g.n >> beta;
    // the folded kernels need l >= 2 and one of their shapes (all three are)
    const int swap = exchange_symmetric && h >= 2;
    void *ws = nullptr;
    hipError_t e = scratch_address(&ws);
    if (e == hipSuccess)
        e = launch_certify_optimal_out(g, dtype, u, swap, static_cast<unsigned char *>(ws), dev_out,
                                       static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        *err = std::string("certificate launch: ") + hipGetErrorString(e);
        return LCSB_EHIP;
    }
    return LCSB_OK;
}

}  // namespace lcsb
