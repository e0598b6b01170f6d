// page_ops.hip -- page-wise det, inverse, transpose, products, scaling and bilinear forms
// over batches of 1x1..4x4 matrices (section 2.2 page-wise maps, section 2.3 determinants
// and inverses, section 2.4 library).
//
// One page per lane.  Pages in the paper's contiguous layout (column-major pages stored
// one after another) are staged through LDS by the whole workgroup with 16-byte vector
// loads, so global traffic is fully coalesced although one page is 16..128 bytes; any
// other stride pattern (structure-of-arrays, broadcast pages, views) is read per lane with
// its strides.  A transposed operand is the same storage read with row and column strides
// swapped, so no kernel needs a transpose flag.
#include "smallmat.hpp"

namespace pf {

constexpr int BS = 256;  // pages per workgroup (4 waves)

struct PageArg {        // device view of one operand
    int64_t sr, sc, sp;  // element strides: row, column, page (0 = broadcast)
};

// -------------------------------------------------------------------------------------
// staging of contiguous page tiles through LDS
// -------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void tile_load(const T* __restrict__ g, int64_t first, int64_t count, int P,
                                          T* lds) {
    const int64_t npg = (count - first < BS) ? (count - first) : BS;
    const int nel = static_cast<int>(npg) * P;
    const T* src = g + first * P;
    constexpr int VEC = 16 / sizeof(T);
    const int nvec = nel / VEC;
    const u32x4* s4 = reinterpret_cast<const u32x4*>(src);
    u32x4* d4 = reinterpret_cast<u32x4*>(lds);
    for (int i = threadIdx.x; i < nvec; i += BS) d4[i] = __builtin_nontemporal_load(s4 + i);
    for (int i = nvec * VEC + threadIdx.x; i < nel; i += BS) lds[i] = src[i];
}

template <typename T>
__device__ __forceinline__ void tile_store(T* __restrict__ g, int64_t first, int64_t count, int P,
                                           const T* lds) {
    const int64_t npg = (count - first < BS) ? (count - first) : BS;
    const int nel = static_cast<int>(npg) * P;
    T* dst = g + first * P;
    constexpr int VEC = 16 / sizeof(T);
    const int nvec = nel / VEC;
    const u32x4* s4 = reinterpret_cast<const u32x4*>(lds);
    u32x4* d4 = reinterpret_cast<u32x4*>(dst);
    for (int i = threadIdx.x; i < nvec; i += BS) __builtin_nontemporal_store(s4[i], d4 + i);
    for (int i = nvec * VEC + threadIdx.x; i < nel; i += BS) dst[i] = lds[i];
}

template <typename T, int R, int C>
__device__ __forceinline__ void read_page(const T* __restrict__ p, int64_t sr, int64_t sc, T* out) {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) out[r + c * R] = p[r * sr + c * sc];
}

template <typename T, int R, int C>
__device__ __forceinline__ void write_page(T* __restrict__ p, int64_t sr, int64_t sc, const T* v) {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int r = 0; r < R; ++r) p[r * sr + c * sc] = v[r + c * R];
}

// load operand page k (rows R x cols C) either from an LDS tile or from global memory
template <typename T, int R, int C, bool STAGED>
__device__ __forceinline__ void load_op(const T* __restrict__ g, const PageArg& d, int64_t k, const T* lds,
                                        T* out) {
    if (STAGED && d.sp != 0)
        read_page<T, R, C>(lds + threadIdx.x * (R * C), d.sr, d.sc, out);
    else
        read_page<T, R, C>(g + k * d.sp, d.sr, d.sc, out);
}

// -------------------------------------------------------------------------------------
// determinant and inverse with FP64 routing for FP32 pages
// -------------------------------------------------------------------------------------
template <typename T, int N>
__device__ __forceinline__ bool page_det_routed(const T* m, const Fallback& fb, T& det) {
    T c0[N], absterms;
    det_first_row<T, N>(m, c0, det, absterms);
    if constexpr (sizeof(T) == 4) {
        if (should_route(det, absterms, fb)) {
            double md[N * N], c0d[N], dd, ad;
#pragma unroll
            for (int q = 0; q < N * N; ++q) md[q] = static_cast<double>(m[q]);
            det_first_row<double, N>(md, c0d, dd, ad);
            det = static_cast<T>(dd);
            return true;
        }
    }
    return false;
}

template <typename T, int N, bool STAGED>
__global__ __launch_bounds__(BS) void k_page_det(const T* __restrict__ a, PageArg da, int64_t count,
                                                 T* __restrict__ det, Fallback fb, uint8_t* __restrict__ flags,
                                                 int64_t* d_counters) {
    __shared__ __align__(16) T lds[STAGED ? BS * N * N : 1];
    const int64_t first = static_cast<int64_t>(blockIdx.x) * BS;
    const int64_t k = first + threadIdx.x;
    if (STAGED && da.sp != 0) {
        tile_load(a, first, count, N * N, lds);
        __syncthreads();
    }
    bool routed = false, sing = false;
    if (k < count) {
        T m[N * N], d;
        load_op<T, N, N, STAGED>(a, da, k, lds, m);
        routed = page_det_routed<T, N>(m, fb, d);
        sing = (d == T(0));
        det[k] = d;
        if (flags) flags[k] = (sing ? FLAG_SINGULAR : 0) | (routed ? FLAG_ROUTED : 0);
    }
    count_wave(d_counters, 0, routed);
    count_wave(d_counters, 1, sing);
}

template <typename T, int N, bool STAGED>
__global__ __launch_bounds__(BS) void k_page_inv(const T* __restrict__ a, PageArg da, int64_t count,
                                                 T* __restrict__ x, PageArg dx, T* __restrict__ det, Fallback fb,
                                                 uint8_t* __restrict__ flags, int64_t* d_counters) {
    __shared__ __align__(16) T lds[STAGED ? BS * N * N : 1];
    const int64_t first = static_cast<int64_t>(blockIdx.x) * BS;
    const int64_t k = first + threadIdx.x;
    if (STAGED && da.sp != 0) {
        tile_load(a, first, count, N * N, lds);
        __syncthreads();
    }
    bool routed = false, sing = false;
    T out[N * N];
    if (k < count) {
        T m[N * N], c0[N], d, absterms;
        load_op<T, N, N, STAGED>(a, da, k, lds, m);
        det_first_row<T, N>(m, c0, d, absterms);
        if constexpr (sizeof(T) == 4) routed = should_route(d, absterms, fb);
        if (routed) {
            double md[N * N], adj[N * N], c0d[N], dd, ad;
#pragma unroll
            for (int q = 0; q < N * N; ++q) md[q] = static_cast<double>(m[q]);
            det_first_row<double, N>(md, c0d, dd, ad);
            adjugate<double, N>(md, adj);
#pragma unroll
            for (int q = 0; q < N * N; ++q) out[q] = static_cast<T>(adj[q] / dd);
            d = static_cast<T>(dd);
            sing = (dd == 0.0);
        } else {
            T adj[N * N];
            adjugate<T, N>(m, adj);
#pragma unroll
            for (int q = 0; q < N * N; ++q) out[q] = adj[q] / d;
            sing = (d == T(0));
        }
        if (det) det[k] = d;
        if (flags) flags[k] = (sing ? FLAG_SINGULAR : 0) | (routed ? FLAG_ROUTED : 0);
    }
    if (STAGED && dx.sp != 0) {
        __syncthreads();  // the input tile has been consumed
        if (k < count) write_page<T, N, N>(lds + threadIdx.x * (N * N), dx.sr, dx.sc, out);
        __syncthreads();
        tile_store(x, first, count, N * N, lds);
    } else if (k < count) {
        write_page<T, N, N>(x + k * dx.sp, dx.sr, dx.sc, out);
    }
    count_wave(d_counters, 0, routed);
    count_wave(d_counters, 1, sing);
}

// -------------------------------------------------------------------------------------
// transpose, scale (runtime shapes up to 4x4; pure data movement / one multiply)
// -------------------------------------------------------------------------------------
template <typename T, bool STAGED>
__global__ __launch_bounds__(BS) void k_page_transpose(const T* __restrict__ a, PageArg da, int rows, int cols,
                                                       int64_t count, T* __restrict__ t, PageArg dt) {
    __shared__ __align__(16) T lds[STAGED ? BS * 16 : 1];
    const int64_t first = static_cast<int64_t>(blockIdx.x) * BS;
    const int64_t k = first + threadIdx.x;
    const int P = rows * cols;
    T v[16];
    if (STAGED) {
        tile_load(a, first, count, P, lds);
        __syncthreads();
    }
    if (k < count) {
        const T* src = STAGED ? lds + threadIdx.x * P : a + k * da.sp;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r < rows && c < cols) v[r + c * 4] = src[r * da.sr + c * da.sc];
    }
    if (STAGED) {
        __syncthreads();
        if (k < count) {
            T* dst = lds + threadIdx.x * P;
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (r < rows && c < cols) dst[c * dt.sr + r * dt.sc] = v[r + c * 4];
        }
        __syncthreads();
        tile_store(t, first, count, P, lds);
    } else if (k < count) {
        T* dst = t + k * dt.sp;
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r < rows && c < cols) dst[c * dt.sr + r * dt.sc] = v[r + c * 4];
    }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_page_scale(const T* __restrict__ s, int64_t ss, const T* __restrict__ a,
                                                   PageArg da, int rows, int cols, int64_t count, T* __restrict__ c,
                                                   PageArg dc) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * BS + threadIdx.x;
    if (k >= count) return;
    const T f = s[k * ss];
    const T* src = a + k * da.sp;
    T* dst = c + k * dc.sp;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (r < rows && cc < cols) dst[r * dc.sr + cc * dc.sc] = f * src[r * da.sr + cc * da.sc];
}

// -------------------------------------------------------------------------------------
// products C = op(A) op(B); op() is folded into the strides on the host
// -------------------------------------------------------------------------------------
template <typename T, int M, int K, int N, bool STAGED>
__global__ __launch_bounds__(BS) void k_page_mtimes(const T* __restrict__ a, PageArg da, const T* __restrict__ b,
                                                    PageArg db, int64_t count, T* __restrict__ c, PageArg dc) {
    constexpr int PA = M * K, PB = K * N, PC = M * N;
    constexpr int PMAX = (PA > PB ? (PA > PC ? PA : PC) : (PB > PC ? PB : PC));
    __shared__ __align__(16) T lds[STAGED ? BS * PMAX : 1];
    const int64_t first = static_cast<int64_t>(blockIdx.x) * BS;
    const int64_t k = first + threadIdx.x;
    T A[PA], B[PB], C[PC];
    if (STAGED && da.sp != 0) {
        tile_load(a, first, count, PA, lds);
        __syncthreads();
        if (k < count) read_page<T, M, K>(lds + threadIdx.x * PA, da.sr, da.sc, A);
        __syncthreads();
    } else if (k < count) {
        read_page<T, M, K>(a + k * da.sp, da.sr, da.sc, A);
    }
    if (STAGED && db.sp != 0) {
        tile_load(b, first, count, PB, lds);
        __syncthreads();
        if (k < count) read_page<T, K, N>(lds + threadIdx.x * PB, db.sr, db.sc, B);
        __syncthreads();
    } else if (k < count) {
        read_page<T, K, N>(b + k * db.sp, db.sr, db.sc, B);
    }
    if (k < count) {
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int i = 0; i < M; ++i) {
                T acc = A[i] * B[j * K];
#pragma unroll
                for (int p = 1; p < K; ++p) acc = fmaT(A[i + p * M], B[p + j * K], acc);
                C[i + j * M] = acc;
            }
    }
    if (STAGED && dc.sp != 0) {
        if (k < count) write_page<T, M, N>(lds + threadIdx.x * PC, dc.sr, dc.sc, C);
        __syncthreads();
        tile_store(c, first, count, PC, lds);
    } else if (k < count) {
        write_page<T, M, N>(c + k * dc.sp, dc.sr, dc.sc, C);
    }
}

// any shape with m, k, n <= 4 (used for the rectangular instances such as 3x4 * 4x3)
template <typename T>
__global__ __launch_bounds__(BS) void k_page_mtimes_any(const T* __restrict__ a, PageArg da, const T* __restrict__ b,
                                                        PageArg db, int m, int kk, int n, int64_t count,
                                                        T* __restrict__ c, PageArg dc) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * BS + threadIdx.x;
    if (k >= count) return;
    const T* pa = a + k * da.sp;
    const T* pb = b + k * db.sp;
    T* pc = c + k * dc.sp;
    T A[16], B[16];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            A[r + q * 4] = (r < m && q < kk) ? pa[r * da.sr + q * da.sc] : T(0);
            B[r + q * 4] = (r < kk && q < n) ? pb[r * db.sr + q * db.sc] : T(0);
        }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (i < m && j < n) {
                T acc = A[i] * B[j * 4];
#pragma unroll
                for (int p = 1; p < 4; ++p)
                    if (p < kk) acc = fmaT(A[i + p * 4], B[p + j * 4], acc);
                pc[i * dc.sr + j * dc.sc] = acc;
            }
}

template <typename T, int N>
__global__ __launch_bounds__(BS) void k_page_bilinear(const T* __restrict__ u, PageArg du, const T* __restrict__ a,
                                                      PageArg da, const T* __restrict__ v, PageArg dv, int64_t count,
                                                      T* __restrict__ q) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * BS + threadIdx.x;
    if (k >= count) return;
    T U[N], V[N], A[N * N];
    read_page<T, N, 1>(u + k * du.sp, du.sr, du.sc, U);
    read_page<T, N, 1>(v + k * dv.sp, dv.sr, dv.sc, V);
    read_page<T, N, N>(a + k * da.sp, da.sr, da.sc, A);
    T acc = T(0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        T av = A[i] * V[0];
#pragma unroll
        for (int j = 1; j < N; ++j) av = fmaT(A[i + j * N], V[j], av);
        acc = fmaT(U[i], av, acc);
    }
    q[k] = acc;
}

// =====================================================================================
// host side
// =====================================================================================
namespace {

pf_status check_pages(const pf_pages* d, const void* p, const char* name, bool allow_bcast = true) {
    if (!d) return fail(PF_EINVAL, std::string(name) + ": null descriptor");
    if (d->rows < 1 || d->rows > 4 || d->cols < 1 || d->cols > 4)
        return fail(PF_EORDER, std::string(name) + ": page shape must be 1..4 x 1..4");
    if (d->count < 0) return fail(PF_EINVAL, std::string(name) + ": negative count");
    if (d->count > 0 && !p) return fail(PF_EINVAL, std::string(name) + ": null data pointer");
    if (d->s_page < 0 || d->s_row < 0 || d->s_col < 0)
        return fail(PF_EINVAL, std::string(name) + ": negative stride");
    if (!allow_bcast && d->s_page == 0 && d->count > 1)
        return fail(PF_EINVAL, std::string(name) + ": output pages cannot be broadcast");
    return PF_OK;
}

// page stored contiguously (either column- or row-major inside, pages back to back) and
// 16-byte aligned: eligible for LDS staging
bool contiguous(const pf_pages* d, const void* p) {
    const int64_t P = static_cast<int64_t>(d->rows) * d->cols;
    if (d->s_page != P) return false;
    bool cm = (d->s_row == 1 && d->s_col == d->rows) || (d->cols == 1 && d->s_row == 1);
    bool rm = (d->s_col == 1 && d->s_row == d->cols) || (d->rows == 1 && d->s_col == 1);
    if (!(cm || rm)) return false;
    return (reinterpret_cast<uintptr_t>(p) % 16) == 0;
}

PageArg arg_of(const pf_pages* d, bool trans = false) {
    PageArg a;
    a.sr = trans ? d->s_col : d->s_row;
    a.sc = trans ? d->s_row : d->s_col;
    a.sp = d->s_page;
    return a;
}

unsigned grid_of(int64_t count) { return static_cast<unsigned>(ceil_div(count, BS)); }

template <typename T, int N>
pf_status launch_det(const pf_pages* A, const void* a, void* det, Fallback fb, uint8_t* flags, int64_t* ctr,
                     hipStream_t s) {
    const bool st = A->s_page != 0 && contiguous(A, a);
    PageArg da = arg_of(A);
    if (st)
        hipLaunchKernelGGL((k_page_det<T, N, true>), dim3(grid_of(A->count)), dim3(BS), 0, s,
                           static_cast<const T*>(a), da, A->count, static_cast<T*>(det), fb, flags, ctr);
    else
        hipLaunchKernelGGL((k_page_det<T, N, false>), dim3(grid_of(A->count)), dim3(BS), 0, s,
                           static_cast<const T*>(a), da, A->count, static_cast<T*>(det), fb, flags, ctr);
    return launch_check("pf_page_det");
}

template <typename T, int N>
pf_status launch_inv(const pf_pages* A, const void* a, const pf_pages* X, void* x, void* det, Fallback fb,
                     uint8_t* flags, int64_t* ctr, hipStream_t s) {
    const bool st = A->s_page != 0 && contiguous(A, a) && contiguous(X, x);
    PageArg da = arg_of(A), dx = arg_of(X);
    if (st)
        hipLaunchKernelGGL((k_page_inv<T, N, true>), dim3(grid_of(A->count)), dim3(BS), 0, s,
                           static_cast<const T*>(a), da, A->count, static_cast<T*>(x), dx, static_cast<T*>(det),
                           fb, flags, ctr);
    else
        hipLaunchKernelGGL((k_page_inv<T, N, false>), dim3(grid_of(A->count)), dim3(BS), 0, s,
                           static_cast<const T*>(a), da, A->count, static_cast<T*>(x), dx, static_cast<T*>(det),
                           fb, flags, ctr);
    return launch_check("pf_page_inv");
}

template <typename T, int M, int K, int N>
pf_status launch_mt(const T* a, PageArg da, const T* b, PageArg db, int64_t count, T* c, PageArg dc, bool st,
                    hipStream_t s) {
    if (st)
        hipLaunchKernelGGL((k_page_mtimes<T, M, K, N, true>), dim3(grid_of(count)), dim3(BS), 0, s, a, da, b, db,
                           count, c, dc);
    else
        hipLaunchKernelGGL((k_page_mtimes<T, M, K, N, false>), dim3(grid_of(count)), dim3(BS), 0, s, a, da, b, db,
                           count, c, dc);
    return launch_check("pf_page_mtimes");
}

template <typename T>
pf_status mtimes_typed(const pf_pages* A, const void* a, int transA, const pf_pages* B, const void* b, int transB,
                       const pf_pages* Cd, void* c, hipStream_t s) {
    const int m = transA ? A->cols : A->rows, k = transA ? A->rows : A->cols;
    const int k2 = transB ? B->cols : B->rows, n = transB ? B->rows : B->cols;
    if (k != k2 || Cd->rows != m || Cd->cols != n)
        return fail(PF_EORDER, "pf_page_mtimes: inner or output dimensions do not match");
    const int64_t count = Cd->count;
    if ((A->s_page != 0 && A->count != count) || (B->s_page != 0 && B->count != count))
        return fail(PF_EINVAL, "pf_page_mtimes: operand counts differ from the output count");
    if (count == 0) return PF_OK;
    PageArg da = arg_of(A, transA), db = arg_of(B, transB), dc = arg_of(Cd);
    const T* pa = static_cast<const T*>(a);
    const T* pb = static_cast<const T*>(b);
    T* pc = static_cast<T*>(c);
    const bool st = (A->s_page == 0 || contiguous(A, a)) && (B->s_page == 0 || contiguous(B, b)) &&
                    contiguous(Cd, c) && !(A->s_page == 0 && B->s_page == 0);
    if (m == k && k == n) {
        if (m == 2) return launch_mt<T, 2, 2, 2>(pa, da, pb, db, count, pc, dc, st, s);
        if (m == 3) return launch_mt<T, 3, 3, 3>(pa, da, pb, db, count, pc, dc, st, s);
        if (m == 4) return launch_mt<T, 4, 4, 4>(pa, da, pb, db, count, pc, dc, st, s);
    }
    if (m == k && n == 1) {
        if (m == 2) return launch_mt<T, 2, 2, 1>(pa, da, pb, db, count, pc, dc, st, s);
        if (m == 3) return launch_mt<T, 3, 3, 1>(pa, da, pb, db, count, pc, dc, st, s);
        if (m == 4) return launch_mt<T, 4, 4, 1>(pa, da, pb, db, count, pc, dc, st, s);
    }
    hipLaunchKernelGGL((k_page_mtimes_any<T>), dim3(grid_of(count)), dim3(BS), 0, s, pa, da, pb, db, m, k, n, count,
                       pc, dc);
    return launch_check("pf_page_mtimes");
}

}  // namespace
}  // namespace pf

using namespace pf;

extern "C" {

pf_status pf_page_det(pf_dtype dtype, const pf_pages* A, const void* a, void* det, const pf_fallback* fb,
                      uint8_t* flags, int64_t* d_counters, void* stream) {
    pf_status st = check_pages(A, a, "A");
    if (st) return st;
    if (A->rows != A->cols) return fail(PF_EORDER, "pf_page_det: pages must be square");
    if (A->count == 0) return PF_OK;
    if (!det) return fail(PF_EINVAL, "pf_page_det: null det");
    Fallback f = make_fallback(fb);
    hipStream_t s = as_stream(stream);
    const int n = A->rows;
    if (dtype == PF_F32) {
        switch (n) {
            case 1: return launch_det<float, 1>(A, a, det, f, flags, d_counters, s);
            case 2: return launch_det<float, 2>(A, a, det, f, flags, d_counters, s);
            case 3: return launch_det<float, 3>(A, a, det, f, flags, d_counters, s);
            default: return launch_det<float, 4>(A, a, det, f, flags, d_counters, s);
        }
    } else if (dtype == PF_F64) {
        switch (n) {
            case 1: return launch_det<double, 1>(A, a, det, f, flags, d_counters, s);
            case 2: return launch_det<double, 2>(A, a, det, f, flags, d_counters, s);
            case 3: return launch_det<double, 3>(A, a, det, f, flags, d_counters, s);
            default: return launch_det<double, 4>(A, a, det, f, flags, d_counters, s);
        }
    }
    return fail(PF_EDTYPE, "pf_page_det: dtype must be PF_F32 or PF_F64");
}

pf_status pf_page_inv(pf_dtype dtype, const pf_pages* A, const void* a, const pf_pages* X, void* x, void* det,
                      const pf_fallback* fb, uint8_t* flags, int64_t* d_counters, void* stream) {
    pf_status st = check_pages(A, a, "A");
    if (st) return st;
    if ((st = check_pages(X, x, "X", false))) return st;
    if (A->rows != A->cols || X->rows != A->rows || X->cols != A->cols)
        return fail(PF_EORDER, "pf_page_inv: A and X must be square pages of the same order");
    if (X->count != A->count) return fail(PF_EINVAL, "pf_page_inv: A and X counts differ");
    if (A->count == 0) return PF_OK;
    Fallback f = make_fallback(fb);
    hipStream_t s = as_stream(stream);
    const int n = A->rows;
    if (dtype == PF_F32) {
        switch (n) {
            case 1: return launch_inv<float, 1>(A, a, X, x, det, f, flags, d_counters, s);
            case 2: return launch_inv<float, 2>(A, a, X, x, det, f, flags, d_counters, s);
            case 3: return launch_inv<float, 3>(A, a, X, x, det, f, flags, d_counters, s);
            default: return launch_inv<float, 4>(A, a, X, x, det, f, flags, d_counters, s);
        }
    } else if (dtype == PF_F64) {
        switch (n) {
            case 1: return launch_inv<double, 1>(A, a, X, x, det, f, flags, d_counters, s);
            case 2: return launch_inv<double, 2>(A, a, X, x, det, f, flags, d_counters, s);
            case 3: return launch_inv<double, 3>(A, a, X, x, det, f, flags, d_counters, s);
            default: return launch_inv<double, 4>(A, a, X, x, det, f, flags, d_counters, s);
        }
    }
    return fail(PF_EDTYPE, "pf_page_inv: dtype must be PF_F32 or PF_F64");
}

pf_status pf_page_transpose(pf_dtype dtype, const pf_pages* A, const void* a, const pf_pages* T, void* t,
                            void* stream) {
    pf_status st = check_pages(A, a, "A");
    if (st) return st;
    if ((st = check_pages(T, t, "T", false))) return st;
    if (T->rows != A->cols || T->cols != A->rows) return fail(PF_EORDER, "pf_page_transpose: T must be cols x rows");
    if (T->count != A->count) return fail(PF_EINVAL, "pf_page_transpose: counts differ");
    if (A->count == 0) return PF_OK;
    hipStream_t s = as_stream(stream);
    const bool stg = A->s_page != 0 && contiguous(A, a) && contiguous(T, t);
    PageArg da = arg_of(A), dt = arg_of(T);
    unsigned g = grid_of(A->count);
    if (dtype == PF_F32) {
        if (stg)
            hipLaunchKernelGGL((k_page_transpose<float, true>), dim3(g), dim3(BS), 0, s, (const float*)a, da, A->rows,
                               A->cols, A->count, (float*)t, dt);
        else
            hipLaunchKernelGGL((k_page_transpose<float, false>), dim3(g), dim3(BS), 0, s, (const float*)a, da, A->rows,
                               A->cols, A->count, (float*)t, dt);
    } else if (dtype == PF_F64) {
        if (stg)
            hipLaunchKernelGGL((k_page_transpose<double, true>), dim3(g), dim3(BS), 0, s, (const double*)a, da,
                               A->rows, A->cols, A->count, (double*)t, dt);
        else
            hipLaunchKernelGGL((k_page_transpose<double, false>), dim3(g), dim3(BS), 0, s, (const double*)a, da,
                               A->rows, A->cols, A->count, (double*)t, dt);
    } else {
        return fail(PF_EDTYPE, "pf_page_transpose: bad dtype");
    }
    return launch_check("pf_page_transpose");
}

pf_status pf_page_mtimes(pf_dtype dtype, const pf_pages* A, const void* a, int transA, const pf_pages* B,
                         const void* b, int transB, const pf_pages* C, void* c, void* stream) {
    pf_status st = check_pages(A, a, "A");
    if (st) return st;
    if ((st = check_pages(B, b, "B"))) return st;
    if ((st = check_pages(C, c, "C", false))) return st;
    hipStream_t s = as_stream(stream);
    if (dtype == PF_F32) return mtimes_typed<float>(A, a, transA, B, b, transB, C, c, s);
    if (dtype == PF_F64) return mtimes_typed<double>(A, a, transA, B, b, transB, C, c, s);
    return fail(PF_EDTYPE, "pf_page_mtimes: bad dtype");
}

pf_status pf_page_mv(pf_dtype dtype, const pf_pages* A, const void* a, int transA, const pf_pages* X,
                     const void* x, const pf_pages* Y, void* y, void* stream) {
    if (!X || !Y) return fail(PF_EINVAL, "pf_page_mv: null descriptor");
    if (X->cols != 1 || Y->cols != 1) return fail(PF_EORDER, "pf_page_mv: x and y must be n x 1 pages");
    return pf_page_mtimes(dtype, A, a, transA, X, x, 0, Y, y, stream);
}

pf_status pf_page_scale(pf_dtype dtype, const void* sv, int64_t s_stride, const pf_pages* A, const void* a,
                        const pf_pages* C, void* c, void* stream) {
    pf_status st = check_pages(A, a, "A");
    if (st) return st;
    if ((st = check_pages(C, c, "C", false))) return st;
    if (C->rows != A->rows || C->cols != A->cols) return fail(PF_EORDER, "pf_page_scale: shapes differ");
    if (A->s_page != 0 && A->count != C->count) return fail(PF_EINVAL, "pf_page_scale: counts differ");
    if (s_stride < 0) return fail(PF_EINVAL, "pf_page_scale: negative scalar stride");
    if (C->count == 0) return PF_OK;
    if (!sv) return fail(PF_EINVAL, "pf_page_scale: null scalars");
    hipStream_t s = as_stream(stream);
    PageArg da = arg_of(A), dc = arg_of(C);
    unsigned g = grid_of(C->count);
    if (dtype == PF_F32)
        hipLaunchKernelGGL((k_page_scale<float>), dim3(g), dim3(BS), 0, s, (const float*)sv, s_stride,
                           (const float*)a, da, A->rows, A->cols, C->count, (float*)c, dc);
    else if (dtype == PF_F64)
        hipLaunchKernelGGL((k_page_scale<double>), dim3(g), dim3(BS), 0, s, (const double*)sv, s_stride,
                           (const double*)a, da, A->rows, A->cols, C->count, (double*)c, dc);
    else
        return fail(PF_EDTYPE, "pf_page_scale: bad dtype");
    return launch_check("pf_page_scale");
}

pf_status pf_page_bilinear(pf_dtype dtype, const pf_pages* U, const void* u, const pf_pages* A, const void* a,
                           const pf_pages* V, const void* v, void* q, void* stream) {
    pf_status st = check_pages(A, a, "A");
    if (st) return st;
    if ((st = check_pages(U, u, "U"))) return st;
    if ((st = check_pages(V, v, "V"))) return st;
    const int n = A->rows;
    if (A->cols != n || U->rows != n || V->rows != n || U->cols != 1 || V->cols != 1)
        return fail(PF_EORDER, "pf_page_bilinear: A must be n x n and u, v n x 1");
    int64_t count = A->s_page != 0 ? A->count : (U->s_page != 0 ? U->count : V->count);
    if ((A->s_page != 0 && A->count != count) || (U->s_page != 0 && U->count != count) ||
        (V->s_page != 0 && V->count != count))
        return fail(PF_EINVAL, "pf_page_bilinear: counts differ");
    if (count == 0) return PF_OK;
    if (!q) return fail(PF_EINVAL, "pf_page_bilinear: null output");
    hipStream_t s = as_stream(stream);
    PageArg du = arg_of(U), da = arg_of(A), dv = arg_of(V);
    unsigned g = grid_of(count);
#define PF_BIL(T, N)                                                                                      \
    hipLaunchKernelGGL((k_page_bilinear<T, N>), dim3(g), dim3(BS), 0, s, (const T*)u, du, (const T*)a, da, \
                       (const T*)v, dv, count, (T*)q)
    if (dtype == PF_F32) {
        if (n == 1) PF_BIL(float, 1); else if (n == 2) PF_BIL(float, 2); else if (n == 3) PF_BIL(float, 3);
        else PF_BIL(float, 4);
    } else if (dtype == PF_F64) {
        if (n == 1) PF_BIL(double, 1); else if (n == 2) PF_BIL(double, 2); else if (n == 3) PF_BIL(double, 3);
        else PF_BIL(double, 4);
    } else {
        return fail(PF_EDTYPE, "pf_page_bilinear: bad dtype");
    }
#undef PF_BIL
    return launch_check("pf_page_bilinear");
}

}  // extern "C"
