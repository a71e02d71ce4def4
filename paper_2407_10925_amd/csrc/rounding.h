// Directed rounding for the scalar steps of the certificate (the host's
// E, R - E and d (R - E); the device's d R and (d - k) R), built from
// round-to-nearest operations with error-free transforms: Knuth's TwoSum
// for sums and the FMA-based TwoProduct for products (Ogita, Rump, Oishi,
// "Accurate sum and dot product", SIAM J. Sci. Comput. 26(6), 2005).  The
// certificate's per-entry pass uses the GPU's rounding mode instead.  IEEE-754 defines the
// directed-rounding result uniquely, so these agree bit for bit with any
// correct implementation (the CPU's rounding-mode switch included) as long
// as no intermediate overflows; the certificate's values are far from that.
//
// The whole library is compiled with -ffp-contract=off so that the compiler
// never fuses the multiply-adds these rely on.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lcsb {

__host__ __device__ inline uint64_t bits_of(double x) { return __builtin_bit_cast(uint64_t, x); }
__host__ __device__ inline double from_bits(uint64_t b) { return __builtin_bit_cast(double, b); }

// largest double strictly below x (x itself for NaN and -inf)
__host__ __device__ inline double next_down(double x)
{
    if (x != x) return x;
    if (x == 0.0) return from_bits(0x8000000000000001ull);  // -min subnormal
    uint64_t b = bits_of(x);
    if (b == 0xfff0000000000000ull) return x;                // -inf
    return from_bits(x > 0.0 ? b - 1 : b + 1);
}

// smallest double strictly above x (x itself for NaN and +inf)
__host__ __device__ inline double next_up(double x)
{
    if (x != x) return x;
    if (x == 0.0) return from_bits(0x0000000000000001ull);  // +min subnormal
    uint64_t b = bits_of(x);
    if (b == 0x7ff0000000000000ull) return x;                // +inf
    return from_bits(x > 0.0 ? b + 1 : b - 1);
}

// exact error of s = fl(a + b): a + b = s + err (TwoSum)
__host__ __device__ inline double two_sum_err(double a, double b, double s)
{
    double bb = s - a;
    return (a - (s - bb)) + (b - bb);
}

__host__ __device__ inline double add_rd(double a, double b)
{
    double s = a + b;
    double e = two_sum_err(a, b, s);
    return e < 0.0 ? next_down(s) : s;
}

__host__ __device__ inline double mul_rd(double a, double b)
{
    double p = a * b;
    double e = __builtin_fma(a, b, -p);
    return e < 0.0 ? next_down(p) : p;
}

__host__ __device__ inline double mul_ru(double a, double b)
{
    double p = a * b;
    double e = __builtin_fma(a, b, -p);
    return e > 0.0 ? next_up(p) : p;
}

// lo <= 1/k <= hi with lo, hi adjacent doubles (or both exact): q = fl(1/k),
// and the sign of the exactly representable residual q k - 1 (one FMA)
// says on which side of 1/k the rounded quotient fell.
__host__ __device__ inline void inverse_bounds(double k, double *lo, double *hi)
{
    const double q = 1.0 / k;
    const double e = __builtin_fma(q, k, -1.0);
    *lo = e > 0.0 ? next_down(q) : q;
    *hi = e < 0.0 ? next_up(q) : q;
}

}  // namespace lcsb
