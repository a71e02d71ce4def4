// Declarations shared by the library's translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lcsb.h"

namespace lcsb {

constexpr int kBlock = 256;          // threads per workgroup (4 wavefronts)
constexpr int kMaxReduceBlocks = 4096;

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
    static constexpr size_t kScalarBytes = 80;
    static constexpr size_t kAsym = 128;     // uint32: set when a table is not exchange-symmetric
    // FP64 offsets of the FP32 tables, one per ring slot
    static constexpr size_t kOffsets = 256;  // double[8]
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
    int swap_sym;     // sigma = d = 2: the lag tables are symmetric under exchanging the strings
};

hipError_t launch_sweep(const Geometry &g, int dtype, const SweepLaunch &a, hipStream_t s);

// Certificate passes (see lcsb_cert); results land in the workspace scalars.
// swap_sym: as in SweepLaunch (the W pass then evaluates one coordinate per
// exchange pair)
hipError_t launch_certify(const Geometry &g, int dtype, const void *u, const void *prev,
                          int u_slot, int prev_slot, int swap_sym, unsigned char *ws,
                          hipStream_t s);

// Utilities
hipError_t launch_fill_zero(void *p, uint64_t bytes, hipStream_t s);
hipError_t launch_fill_f64(double *p, uint64_t count, double v, hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, uint64_t bytes, hipStream_t s);
// sigma = d = 2, l >= 2: set *flag (device) to 1 unless every stored entry
// equals, bit for bit, the stored entry of its string-exchanged tuple
hipError_t launch_check_swap(const Geometry &g, int dtype, const void *table, uint32_t *flag,
                             hipStream_t s);
hipError_t launch_upcast(const Geometry &g, const float *src, const double *offset_dev,
                         double *dst, hipStream_t s);
// the FP32 table in the first half of an FP64-sized buffer, widened in place
hipError_t launch_upcast_inplace(const Geometry &g, void *buf, const double *offset_dev,
                                 hipStream_t s);

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
