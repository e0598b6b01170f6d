// common.hpp -- shared host and device helpers of libpagefem (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/pagefem.h"

namespace pf {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------------
// host: error reporting
// ------------------------------------------------------------------------------------
void set_error(const std::string& msg);
pf_status fail(pf_status st, const std::string& msg);

#define PF_HIP_TRY(expr)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::pf::fail(PF_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline pf_status launch_check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(PF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return PF_OK;
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------------------------------
// dynamic LDS carved into consecutive arrays
// ------------------------------------------------------------------------------------
// A kernel that carves its dynamic LDS (16-byte aligned base) into arrays of types
// T0, T1, ... with run-time counts starts array k at sum_{j<k} n_j sizeof(Tj).  That offset
// is a multiple of alignof(Tk) for every count when each earlier element size is: the
// condition checked here, at compile time, for every carve-out (a 64-bit LDS atomic on a
// misaligned address faults the wave).
template <typename... Ts>
constexpr bool lds_carve_aligned() {
    constexpr size_t sz[] = {sizeof(Ts)...};
    constexpr size_t al[] = {alignof(Ts)...};
    for (size_t k = 0; k < sizeof...(Ts); ++k) {
        if (al[k] > 16) return false;
        for (size_t j = 0; j < k; ++j)
            if (sz[j] % al[k] != 0) return false;
    }
    return true;
}

// ------------------------------------------------------------------------------------
// device: error-free transformations and compensated small determinants
// ------------------------------------------------------------------------------------
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// a*d - b*c with Kahan's FMA scheme: the rounding error of b*c is recovered exactly by an
// FMA and added back, so the result is within 2 ulp of the exact value (Jeannerod,
// Louvet, Muller, Math. Comp. 2013), whatever the cancellation.
template <typename T>
__device__ __forceinline__ T det2(T a, T b, T c, T d) {
    T w = b * c;
    T e = fmaT(-b, c, w);   // w - b*c, exact
    T f = fmaT(a, d, -w);   // a*d - w, one rounding
    return f + e;
}

// Knuth's TwoSum: s + err = a + b exactly
template <typename T>
__device__ __forceinline__ T two_sum(T a, T b, T& err) {
    T s = a + b;
    T bb = s - a;
    err = (a - (s - bb)) + (b - bb);
    return s;
}

// Compensated dot product of length N (Ogita, Rump, Oishi 2005, Dot2): as accurate as if
// computed in twice the working precision and rounded once.  Also returns sum |x_i y_i|.
template <typename T, int N>
__device__ __forceinline__ T dot_comp(const T* x, const T* y, T& abs_sum) {
    T p = x[0] * y[0];
    T s = fmaT(x[0], y[0], -p);
    abs_sum = fabs(p);
#pragma unroll
    for (int i = 1; i < N; ++i) {
        T h = x[i] * y[i];
        T q = fmaT(x[i], y[i], -h);
        T err;
        p = two_sum(p, h, err);
        s += q + err;
        abs_sum += fabs(h);
    }
    return p + s;
}

// double-word number hi + lo (unevaluated sum), |lo| <= ulp(hi)/2 after normalisation
template <typename T>
struct DW {
    T hi, lo;
};

template <typename T>
__device__ __forceinline__ DW<T> two_prod(T a, T b) {
    const T p = a * b;
    return DW<T>{p, fmaT(a, b, -p)};
}

// a*d - b*c as a double-word value; the error is O(u^2 (|ad| + |bc|)), so the value is
// effectively exact for every later rounding to working precision
template <typename T>
__device__ __forceinline__ DW<T> dw_det2(T a, T b, T c, T d) {
    const DW<T> p = two_prod(a, d), q = two_prod(b, c);
    T e;
    const T s = two_sum(p.hi, -q.hi, e);
    const T lo = e + (p.lo - q.lo);
    T e2;
    const T hi = two_sum(s, lo, e2);
    return DW<T>{hi, e2};
}

// sum_i x_i * y_i with double-word y_i, compensated (Dot2-style): the result carries an
// error of about u |result| + O(u^2) sum |x_i y_i|.  abs_sum = sum |x_i y_i.hi|.
template <typename T, int N>
__device__ __forceinline__ DW<T> dot_dw(const T* x, const DW<T>* y, T& abs_sum) {
    DW<T> p = two_prod(x[0], y[0].hi);
    T s = p.hi;
    T err = fmaT(x[0], y[0].lo, p.lo);
    abs_sum = fabs(p.hi);
#pragma unroll
    for (int i = 1; i < N; ++i) {
        p = two_prod(x[i], y[i].hi);
        T e;
        s = two_sum(s, p.hi, e);
        err += e + fmaT(x[i], y[i].lo, p.lo);
        abs_sum += fabs(p.hi);
    }
    T e2;
    const T hi = two_sum(s, err, e2);
    return DW<T>{hi, e2};
}

template <typename T>
__device__ __forceinline__ bool finiteT(T v) {
    return __builtin_isfinite(v);
}

// counters layout (see pagefem.h): [0] routed, [1] singular, [2] bad index
__device__ __forceinline__ void count_add(int64_t* d_counters, int which, int64_t v) {
    if (d_counters && v) atomicAdd(reinterpret_cast<unsigned long long*>(d_counters + which),
                                   static_cast<unsigned long long>(v));
}

// wave-level sum of an integer flag, one atomic per wave
__device__ __forceinline__ void count_wave(int64_t* d_counters, int which, bool pred) {
    if (!d_counters) return;
    unsigned long long m = __ballot(pred);
    if (m && (__lane_id() == __ffsll(static_cast<long long>(m)) - 1))
        atomicAdd(reinterpret_cast<unsigned long long*>(d_counters + which),
                  static_cast<unsigned long long>(__popcll(m)));
}

// Per-workgroup counts of W integer tallies (v[k], one value per thread): each wave sums
// its lanes, the block's waves meet in LDS, and thread 0 either stores the block's W sums at
// bcnt[W * blockIdx.x + k] (a launch of k_sum_counts adds them to the counters afterwards:
// no two workgroups write one word) or, with no bcnt, adds each nonzero sum to
// d_counters[which[k]].  Every thread of the block must call it (one barrier).  Many
// workgroups adding to the one counter address serialise on it: on meshes that route one
// element in fifty that cost ten times the kernel itself.
template <int W, int NT>
__device__ __forceinline__ void block_counts(int64_t* d_counters, int32_t* bcnt, const int (&which)[W],
                                             const int (&v)[W]) {
    static_assert(NT % 64 == 0 && NT <= 1024, "whole waves");
    if (!d_counters) return;  // uniform across the block
    __shared__ int32_t wsum[NT / 64][W];
    const int lane = static_cast<int>(threadIdx.x & 63), wv = static_cast<int>(threadIdx.x >> 6);
#pragma unroll
    for (int k = 0; k < W; ++k) {
        int x = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) wsum[wv][k] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
            int32_t x = 0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) x += wsum[w][k];
            if (bcnt) bcnt[static_cast<int64_t>(W) * blockIdx.x + k] = x;
            else if (x) count_add(d_counters, which[k], x);
        }
    }
}

// d_counters[w_k] += the sum over blocks b < nb of c[W b + k]: 1024 blocks' counts per
// workgroup (four independent loads per thread and tally), one atomic per workgroup and tally
constexpr int SUM_COUNTS_PER_BLOCK = 1024;
template <int W>
__global__ __launch_bounds__(256) void k_sum_counts(const int32_t* __restrict__ c, int64_t nb, int64_t* d_counters,
                                                    int w0, int w1, int w2) {
    __shared__ int64_t part[4][W];
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * SUM_COUNTS_PER_BLOCK + threadIdx.x;
    int64_t acc[W];
#pragma unroll
    for (int k = 0; k < W; ++k) acc[k] = 0;
    int32_t x[4][W];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int k = 0; k < W; ++k) x[j][k] = b0 + 256 * j < nb ? c[(b0 + 256 * j) * W + k] : 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        int64_t a = static_cast<int64_t>(x[0][k]) + x[1][k] + x[2][k] + x[3][k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o);
        acc[k] = a;
    }
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < W; ++k) part[threadIdx.x >> 6][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int wk[3] = {w0, w1, w2};
#pragma unroll
        for (int k = 0; k < W; ++k) count_add(d_counters, wk[k], part[0][k] + part[1][k] + part[2][k] + part[3][k]);
    }
}

constexpr uint8_t FLAG_SINGULAR = 1;
constexpr uint8_t FLAG_ROUTED = 2;
constexpr uint8_t FLAG_BADINDEX = 4;

struct Fallback {
    double tau_abs;
    double tau_cond;
    int enable;
};

inline Fallback make_fallback(const pf_fallback* fb) {
    if (!fb) return Fallback{0.0, 1e6, 1};
    return Fallback{fb->tau_abs, fb->tau_cond, fb->enable};
}

}  // namespace pf
