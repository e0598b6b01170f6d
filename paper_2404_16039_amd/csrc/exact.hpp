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

// FP32 contributions of one CSR row, summed exactly as 64-bit integers: the grid is 2^(e-44)
// with e the exponent of the row's largest |contribution| (found in a first pass), so every
// contribution rounds onto it as an integer below 2^45 in magnitude and sums of up to 256 of
// them stay below 2^53 -- exact, in any order of the adds.  The rounding to the grid is done
// by one FP64 add of 3 * 2^51 (the value is then an integer in the low bits of the double);
// subtracting that constant's bit pattern (whose low 32 bits are zero) leaves the integer in
// two's complement.  A contribution's grid error is at most 2^-45 of the row maximum's power
// of two, far below the FP32 result's own rounding, which happens once, in back().  Maxima are
// kept as the bits of |x| (ordered as unsigned integers for non-negative floats); the value
// POISON marks a row that received a non-finite contribution.
struct RowGrid32 {
    static constexpr uint32_t POISON = 0xffffffffu;
    static constexpr uint32_t SKIP = 0xfffffffeu;  // a row left to another kernel (no stores)
    __device__ static uint32_t mag(float x) { return __float_as_uint(fabsf(x)); }
    // 44 - e for a normal maximum; a zero or subnormal maximum takes e = -127 (every
    // contribution is then below 2^-126 and scales below 2^44)
    __device__ static int shift(uint32_t m) { return 171 - static_cast<int>((m >> 23) & 255); }
    __device__ static uint64_t quant(float x, int sh) {
        const double d = static_cast<double>(__builtin_amdgcn_ldexpf(x, sh)) + 6755399441055744.0;
        return static_cast<uint64_t>(__double_as_longlong(d)) - 0x4338000000000000ull;
    }
    __device__ static float back(uint64_t a, int sh) {
        return static_cast<float>(ldexp(static_cast<double>(static_cast<int64_t>(a)), -sh));
    }
};

// Per-slot grid of the long-row kernels (a slot there may receive thousands of contributions):
// FP64 contributions are rounded onto 2^(e + 1 - (62 - HB)), e the exponent of the slot's
// largest one and HB = (bit length of the entry count) + 1 bits of headroom, and summed as
// 64-bit integers: exact, so the order of the adds does not matter, and no sum of at most the
// entry count of them can overflow.  Each contribution's rounding error is at most 2^(HB - 62)
// of the largest one's power of two (for 1000 entries, 2^-51).  POISON marks a slot that got
// a non-finite contribution.
struct LongGrid {
    static constexpr uint32_t POISON = 0xffffffffu;
    static __device__ __forceinline__ uint32_t mag(double x) {  // the high word of |x|: ordered
        return __builtin_isfinite(x) ? static_cast<uint32_t>(static_cast<uint64_t>(__double_as_longlong(fabs(x))) >> 32)
                                     : POISON;
    }
    static __device__ __forceinline__ int headroom(int entries) { return 33 - __clz(entries | 1); }
    static __device__ __forceinline__ int shift(uint32_t m, int hb) {
        const int e = static_cast<int>((m >> 20) & 0x7ff);  // |x| < 2^(e - 1022)
        return (62 - hb) - (e - 1022);
    }
    static __device__ __forceinline__ unsigned long long quant(double x, int sh) {
        return static_cast<unsigned long long>(__double2ll_rn(ldexp(x, sh)));
    }
    static __device__ __forceinline__ double back(unsigned long long a, int sh) {
        return ldexp(static_cast<double>(static_cast<long long>(a)), -sh);
    }
};

}  // namespace pf
