// exact.hpp -- order-independent exact sums of floating-point contributions (used by the
// numeric assembly and the load vector).
#pragma once

#include "common.hpp"

namespace pf {

// Exact, order-independent accumulation: every contribution is first rounded onto a fixed
// grid, a power of two chosen per sum (a CSR slot, an entry of the load vector) from that
// sum's largest contribution (found in a first pass, before any add), after which sums of
// up to 64 grid values are exact in the accumulator type, so adds in any order give the
// same bits.  The rounding error of a sum is at most 2^-bits times its largest contribution.
//   FP32 contributions: grid 2^-24 of the sum's maximum's power of two (|x| < 2^E quantizes
//   to an integer below 2^24, exact in FP32 and int32), two's-complement int32 accumulator:
//   at most 64 contributions per sum keep every partial sum below 2^30.  The grid error of
//   a sum is at most (contributions) x 2^-25 of its largest contribution's power of two,
//   i.e. below 2^-18 relative even with 64 contributions, under the FP32 tolerance; the
//   final conversion rounds once.
//   FP64 contributions: grid 2^-56, two's-complement int64 accumulator.
// Only the maximum's exponent matters, so maxima are kept as the high 32 bits of |x|.
template <typename T>
struct Exact;
template <>
struct Exact<float> {
    using acc = unsigned int;  // two's-complement int32 sums (LDS integer atomics wrap)
    static constexpr int bits = 24;
    __device__ static uint32_t mag(float x) { return __float_as_uint(fabsf(x)); }
    // shift = bits - E with max < 2^E (clamped so that 2^shift stays a normal float)
    __device__ static int shift(uint32_t m) {
        int sh = bits - (static_cast<int>((m >> 23) & 255) - 126);
        return sh > 126 ? 126 : sh;
    }
    __device__ static acc quant(float x, int sh) {
        return static_cast<acc>(static_cast<int>(rintf(ldexpf(x, sh))));
    }
    __device__ static float back(acc a, int sh) { return ldexpf(static_cast<float>(static_cast<int>(a)), -sh); }
};
template <>
struct Exact<double> {
    using acc = unsigned long long;
    static constexpr int bits = 56;
    __device__ static uint32_t mag(double x) {
        return static_cast<uint32_t>(static_cast<unsigned long long>(__double_as_longlong(fabs(x))) >> 32);
    }
    __device__ static int shift(uint32_t m) {
        int E = static_cast<int>((m >> 20) & 2047) - 1022;
        E = E < -960 ? -960 : (E > 960 ? 960 : E);  // keep 2^shift and 2^-shift normal
        return bits - E;
    }
    __device__ static acc quant(double x, int sh) {
        return static_cast<unsigned long long>(static_cast<long long>(rint(ldexp(x, sh))));
    }
    __device__ static double back(acc a, int sh) { return ldexp(static_cast<double>(static_cast<long long>(a)), -sh); }
};

}  // namespace pf
