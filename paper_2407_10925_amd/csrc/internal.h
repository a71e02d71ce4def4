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
                      // (read lazily, see TwinGroup; the new table is written lazily)
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
