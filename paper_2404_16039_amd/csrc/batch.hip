// batch.hip -- mixed-order batch plans: the page-wise inverse with determinant (section
// 2.3) and the page-wise product (section 2.2) over many groups of pages of orders 1..4, in ONE
// persistent launch replayed from a HIP graph.
//
// Work list.  Each group is cut into tiles of `tile` chunks; a chunk is one page per lane
// (lanes per matrix = 1) or floor(64 / lanes) pages per wave (lanes = n or n*n).  Tiles of
// all groups are numbered consecutively; workgroup b takes tiles b, b + grid, b + 2 grid, ...
// and finds a tile's group by binary search over the groups' first tile numbers (scalar
// loads of a few KB of descriptors).
//
// Lane mappings of one chunk:
//   lanes = 1    a lane holds its whole page: determinant by first-row expansion with
//                double-word cofactors, full adjugate (as pf_page_inv), product by FMA chains.
//   lanes = n    lane k of a page produces column k of inv(A) and of A*B.  It reads A with
//                its rows rotated by k (row i of the copy = row (i+k) mod n of A): the
//                first-row cofactors of the rotated copy over its determinant are exactly
//                column k of inv(A) (the sign of the rotation cancels), so every lane runs
//                the same compensated first-row expansion on a different copy.
//   lanes = n*n  lane (r, k) produces entry (r, k) of both results: its copy has the rows
//                rotated by k and the columns by r, and the copy's first cofactor over the
//                copy's determinant is entry (r, k) of inv(A) (both signs cancel again).
// The page's lane with k = 0 holds the unrotated page; its routing decision (FP32 plans)
// is broadcast to the page's other lanes, so a page is routed as by pf_page_inv.
// Staging: the chunk's A (then B) bytes are copied into LDS with 16-byte loads, placed so
// that 16-byte units of global memory land on 16-byte units of LDS; lanes then read their
// pages from LDS.  Unstaged, lanes read their pages from global memory directly.
#include "smallmat.hpp"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

namespace pf {

struct PlanGroup {  // device descriptor of one group (80 bytes)
    const void* a;
    const void* b;
    void* x;
    void* c;
    void* det;
    int64_t count;
    int64_t tile0;  // number of the group's first tile
    int32_t order, ops;
    int32_t lanes, staged;
    int32_t chunks;  // chunks per tile
    int32_t ppc;     // pages per chunk
};

struct PlanPhase {  // the tiles of one order: groups [g_lo, g_hi), tiles [t_lo, t_hi)
    int64_t t_lo, t_hi;
    int32_t g_lo, g_hi;
    int32_t lanes, staged;
};

struct PlanHeader {
    int64_t ntiles;
    int64_t* counters;
    Fallback fb;
    int32_t ngroups;
    int32_t pad;
    PlanPhase phase[5];  // indexed by the order
};

constexpr size_t PLAN_GROUPS_OFFSET = 256;
static_assert(sizeof(PlanHeader) <= PLAN_GROUPS_OFFSET, "work-list header");

// ------------------------------------------------------------------------------ staging
// Copy nel elements from src into lds[lead ...], lead = (address of src mod 16) / sizeof(T),
// so that the 16-byte units of src map onto 16-byte aligned LDS addresses.  Returns lead.
template <typename T, int BS>
__device__ __forceinline__ int stage_in(const T* __restrict__ src, int nel, T* lds) {
    constexpr int VEC = 16 / sizeof(T);
    const int lead = static_cast<int>((reinterpret_cast<uintptr_t>(src) & 15) / sizeof(T));
    const int head = lead ? min(VEC - lead, nel) : 0;
    const int nvec = (nel - head) / VEC;
    const int tail0 = head + nvec * VEC;
    const u32x4* s4 = reinterpret_cast<const u32x4*>(src + head);
    u32x4* d4 = reinterpret_cast<u32x4*>(lds + lead + head);
    for (int i = threadIdx.x; i < nvec; i += BS) d4[i] = __builtin_nontemporal_load(s4 + i);
    if (static_cast<int>(threadIdx.x) < head) lds[lead + threadIdx.x] = src[threadIdx.x];
    for (int i = tail0 + static_cast<int>(threadIdx.x); i < nel; i += BS) lds[lead + i] = src[i];
    return lead;
}

template <typename T>
__device__ __forceinline__ int lead_of(const T* p) {
    return static_cast<int>((reinterpret_cast<uintptr_t>(p) & 15) / sizeof(T));
}

// inverse of stage_in: lds[lead ...] (lead = lead_of(dst)) to dst[0, nel)
template <typename T, int BS>
__device__ __forceinline__ void stage_out(T* __restrict__ dst, int nel, const T* lds) {
    constexpr int VEC = 16 / sizeof(T);
    const int lead = lead_of(dst);
    const int head = lead ? min(VEC - lead, nel) : 0;
    const int nvec = (nel - head) / VEC;
    const int tail0 = head + nvec * VEC;
    const u32x4* s4 = reinterpret_cast<const u32x4*>(lds + lead + head);
    u32x4* d4 = reinterpret_cast<u32x4*>(dst + head);
    for (int i = threadIdx.x; i < nvec; i += BS) __builtin_nontemporal_store(s4[i], d4 + i);
    if (static_cast<int>(threadIdx.x) < head) dst[threadIdx.x] = lds[lead + threadIdx.x];
    for (int i = tail0 + static_cast<int>(threadIdx.x); i < nel; i += BS) dst[i] = lds[lead + i];
}

// one page of NN elements from global memory; 16-byte loads when `vec` (page and base
// 16-byte aligned)
template <typename T, int NN>
__device__ __forceinline__ void load_page_g(const T* __restrict__ p, bool vec, T* out) {
    constexpr int BYTES = NN * static_cast<int>(sizeof(T));
    if constexpr (BYTES % 16 == 0) {
        if (vec) {
            const u32x4* s = reinterpret_cast<const u32x4*>(p);
#pragma unroll
            for (int q = 0; q < BYTES / 16; ++q) {
                const u32x4 v = __builtin_nontemporal_load(s + q);
                __builtin_memcpy(out + q * (16 / sizeof(T)), &v, 16);
            }
            return;
        }
    }
#pragma unroll
    for (int e = 0; e < NN; ++e) out[e] = p[e];
}

template <typename T, int NN>
__device__ __forceinline__ void store_page_g(T* __restrict__ p, bool vec, const T* v) {
    constexpr int BYTES = NN * static_cast<int>(sizeof(T));
    if constexpr (BYTES % 16 == 0) {
        if (vec) {
            u32x4* d = reinterpret_cast<u32x4*>(p);
#pragma unroll
            for (int q = 0; q < BYTES / 16; ++q) {
                u32x4 w;
                __builtin_memcpy(&w, v + q * (16 / sizeof(T)), 16);
                __builtin_nontemporal_store(w, d + q);
            }
            return;
        }
    }
#pragma unroll
    for (int e = 0; e < NN; ++e) p[e] = v[e];
}

template <typename T, int NN>
__device__ __forceinline__ bool vec_ok(const void* base) {
    return ((NN * sizeof(T)) % 16 == 0) && ((reinterpret_cast<uintptr_t>(base) & 15) == 0);
}

// product C = A B of column-major N x N pages, FMA chain in ascending inner index
template <typename T, int N>
__device__ __forceinline__ T prod_entry(const T* A, int ai, int as, const T* Bk) {
    T acc = A[ai] * Bk[0];
#pragma unroll
    for (int m = 1; m < N; ++m) acc = fmaT(A[ai + m * as], Bk[m], acc);
    return acc;
}

// Plain FP64 first-row cofactors, determinant and adjugate of an FP32 page that the
// routing predicate sends to FP64.  FP64 carries 29 bits more than the FP32 result needs,
// so no compensation is used here (this keeps the path light on registers).
#define M_(r, c) a[(r) + (c) * N]
template <int N>
__device__ __forceinline__ void first_row_f64(const double* a, double* c0, double& det) {
    if constexpr (N == 1) {
        c0[0] = 1.0;
    } else if constexpr (N == 2) {
        c0[0] = M_(1, 1);
        c0[1] = -M_(1, 0);
    } else if constexpr (N == 3) {
        c0[0] = fmaT(M_(1, 1), M_(2, 2), -M_(1, 2) * M_(2, 1));
        c0[1] = fmaT(M_(1, 2), M_(2, 0), -M_(1, 0) * M_(2, 2));
        c0[2] = fmaT(M_(1, 0), M_(2, 1), -M_(1, 1) * M_(2, 0));
    } else {
        const double q0 = fmaT(M_(2, 0), M_(3, 1), -M_(2, 1) * M_(3, 0));
        const double q1 = fmaT(M_(2, 0), M_(3, 2), -M_(2, 2) * M_(3, 0));
        const double q2 = fmaT(M_(2, 0), M_(3, 3), -M_(2, 3) * M_(3, 0));
        const double q3 = fmaT(M_(2, 1), M_(3, 2), -M_(2, 2) * M_(3, 1));
        const double q4 = fmaT(M_(2, 1), M_(3, 3), -M_(2, 3) * M_(3, 1));
        const double q5 = fmaT(M_(2, 2), M_(3, 3), -M_(2, 3) * M_(3, 2));
        c0[0] = fmaT(M_(1, 1), q5, fmaT(-M_(1, 2), q4, M_(1, 3) * q3));
        c0[1] = fmaT(-M_(1, 0), q5, fmaT(M_(1, 2), q2, -M_(1, 3) * q1));
        c0[2] = fmaT(M_(1, 0), q4, fmaT(-M_(1, 1), q2, M_(1, 3) * q0));
        c0[3] = fmaT(-M_(1, 0), q3, fmaT(M_(1, 1), q1, -M_(1, 2) * q0));
    }
    double s = M_(0, 0) * c0[0];
#pragma unroll
    for (int j = 1; j < N; ++j) s = fmaT(M_(0, j), c0[j], s);
    det = s;
}
#undef M_

// inverse of an FP32 page in plain FP64: column k of inv(A) is the first-row cofactors of
// A with its rows rotated by k, over that copy's determinant
template <int N>
__device__ __forceinline__ void inv_f64(const float* A, float* X, float& det) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
        double m[N * N], c0[N], d;
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int i = 0; i < N; ++i) m[i + j * N] = static_cast<double>(A[(i + k) % N + j * N]);
        first_row_f64<N>(m, c0, d);
#pragma unroll
        for (int r = 0; r < N; ++r) X[r + k * N] = static_cast<float>(c0[r] / d);
        if (k == 0) det = static_cast<float>(d);
    }
}

// ----------------------------------------------------------------------- lanes = 1 chunk
template <typename T, int N, int BS, bool STAGED>
__device__ __forceinline__ void chunk_l1(const PlanGroup& g, int64_t p0, int np, const Fallback& fb, T* lds,
                                         int& nrouted, int& nsing) {
    constexpr int NN = N * N;
    const int i = threadIdx.x;
    const bool active = i < np;
    const bool inv = g.ops & PF_OP_INV, mt = g.ops & PF_OP_MTIMES;
    const T* ga = static_cast<const T*>(g.a) + p0 * NN;
    const T* gb = static_cast<const T*>(g.b) + p0 * NN;
    T* gx = static_cast<T*>(g.x) + p0 * NN;
    T* gc = static_cast<T*>(g.c) + p0 * NN;
    T A[NN], B[NN];
#pragma unroll
    for (int e = 0; e < NN; ++e) A[e] = B[e] = T(0);
    if (STAGED) {
        const int lead = stage_in<T, BS>(ga, np * NN, lds);
        __syncthreads();
        if (active) {
#pragma unroll
            for (int e = 0; e < NN; ++e) A[e] = lds[lead + i * NN + e];
        }
        if (mt) {
            __syncthreads();
            const int lb = stage_in<T, BS>(gb, np * NN, lds);
            __syncthreads();
            if (active) {
#pragma unroll
                for (int e = 0; e < NN; ++e) B[e] = lds[lb + i * NN + e];
            }
        }
    } else if (active) {
        load_page_g<T, NN>(ga + i * NN, vec_ok<T, NN>(g.a), A);
        if (mt) load_page_g<T, NN>(gb + i * NN, vec_ok<T, NN>(g.b), B);
    }
    // product first: B and C leave registers before the inverse needs its temporaries
    if (mt) {
        T Cm[NN];
#pragma unroll
        for (int k = 0; k < N; ++k)
#pragma unroll
            for (int r = 0; r < N; ++r) Cm[r + k * N] = prod_entry<T, N>(A, r, N, B + k * N);
        if (STAGED) {
            __syncthreads();  // every lane has read its inputs
            const int lc = lead_of(gc);
            if (active) {
#pragma unroll
                for (int e = 0; e < NN; ++e) lds[lc + i * NN + e] = Cm[e];
            }
            __syncthreads();
            stage_out<T, BS>(gc, np * NN, lds);
        } else if (active) {
            store_page_g<T, NN>(gc + i * NN, vec_ok<T, NN>(g.c), Cm);
        }
    }
    if (inv) {
        T X[NN], d = T(0);
        if (active) {
            T c0[N], absterms;
            det_first_row<T, N>(A, c0, d, absterms);
            bool routed = false;
            if constexpr (sizeof(T) == 4) routed = should_route(d, absterms, fb);
            if (routed) {
                if constexpr (sizeof(T) == 4) inv_f64<N>(A, X, d);
                ++nrouted;
            } else {
                T adj[NN];
                adjugate<T, N>(A, adj);
#pragma unroll
                for (int q = 0; q < NN; ++q) X[q] = adj[q] / d;
            }
            nsing += (d == T(0));
            if (g.det) static_cast<T*>(g.det)[p0 + i] = d;
        }
        if (STAGED) {
            __syncthreads();
            const int lx = lead_of(gx);
            if (active) {
#pragma unroll
                for (int e = 0; e < NN; ++e) lds[lx + i * NN + e] = X[e];
            }
            __syncthreads();
            stage_out<T, BS>(gx, np * NN, lds);
        } else if (active) {
            store_page_g<T, NN>(gx + i * NN, vec_ok<T, NN>(g.x), X);
        }
    }
    if (STAGED) __syncthreads();  // the staging buffer is free for the next chunk
}

// ------------------------------------------------------------------ lanes = n chunk
// staged or direct base of page `pl` of the chunk starting at page p0
template <typename T, int NN, int BS, bool STAGED>
__device__ __forceinline__ const T* chunk_base(const T* g, int np, int pl, T* lds) {
    if (STAGED) {
        const int lead = stage_in<T, BS>(g, np * NN, lds);
        __syncthreads();
        return lds + lead + pl * NN;
    }
    return g + pl * NN;
}

template <typename T, int N, int BS, bool STAGED>
__device__ __forceinline__ void chunk_col(const PlanGroup& g, int64_t p0, int np, const Fallback& fb, T* lds,
                                          int& nrouted, int& nsing) {
    constexpr int NN = N * N, PW = 64 / N;
    const int wave = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int pl = wave * PW + ln / N;  // page of the lane within the chunk
    const int k = ln % N;               // column of inv(A) and A*B produced by the lane
    const bool active = (ln < PW * N) && (pl < np);
    const bool inv = g.ops & PF_OP_INV, mt = g.ops & PF_OP_MTIMES;
    int rot[N];  // row i of the lane's copy of A = row rot[i] of A
#pragma unroll
    for (int i = 0; i < N; ++i) rot[i] = (i + k) % N;
    T Ar[NN], Bk[N];
#pragma unroll
    for (int e = 0; e < NN; ++e) Ar[e] = T(0);
#pragma unroll
    for (int m = 0; m < N; ++m) Bk[m] = T(0);
    const T* pa = chunk_base<T, NN, BS, STAGED>(static_cast<const T*>(g.a) + p0 * NN, np, pl, lds);
    if (active) {
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int i = 0; i < N; ++i) Ar[i + j * N] = pa[rot[i] + j * N];
    }
    if (mt) {
        if (STAGED) __syncthreads();
        const T* pb = chunk_base<T, NN, BS, STAGED>(static_cast<const T*>(g.b) + p0 * NN, np, pl, lds);
        if (active) {
#pragma unroll
            for (int m = 0; m < N; ++m) Bk[m] = pb[m + k * N];
        }
    }
    if (STAGED) __syncthreads();  // staging buffer free for the next chunk

    const int64_t page = p0 + pl;
    if (inv) {
        T c0[N], d, absterms;
        det_first_row<T, N>(Ar, c0, d, absterms);
        int route = 0;
        if constexpr (sizeof(T) == 4) route = active && should_route(d, absterms, fb);
        route = __shfl(route, (ln / N) * N, 64);  // the decision of the page's unrotated lane
        T xs[N];
        if (route) {
            double md[NN], c0d[N], dd;
#pragma unroll
            for (int e = 0; e < NN; ++e) md[e] = static_cast<double>(Ar[e]);
            first_row_f64<N>(md, c0d, dd);
#pragma unroll
            for (int i = 0; i < N; ++i) xs[i] = static_cast<T>(c0d[i] / dd);
            d = static_cast<T>(dd);
        } else {
#pragma unroll
            for (int i = 0; i < N; ++i) xs[i] = c0[i] / d;
        }
        if (active) {
            T* px = static_cast<T*>(g.x) + page * NN + k * N;
#pragma unroll
            for (int i = 0; i < N; ++i) px[i] = xs[i];
            if (k == 0) {  // the unrotated lane: determinant, counts
                if (g.det) static_cast<T*>(g.det)[page] = d;
                nrouted += route;
                nsing += (d == T(0));
            }
        }
    }
    if (mt && active) {
        // row i of the lane's copy gives row rot[i] of column k of A*B
        T* pc = static_cast<T*>(g.c) + page * NN + k * N;
#pragma unroll
        for (int i = 0; i < N; ++i) pc[rot[i]] = prod_entry<T, N>(Ar, i, N, Bk);
    }
}

// ---------------------------------------------------------------- lanes = n*n chunk
// Lane (r, k) produces entry (r, k) of inv(A) and of A*B.  Every lane evaluates det(A)
// (compensated first-row expansion of the page as stored, so the routing decision is the
// same in all lanes of a page) and the determinant of the minor without row k and column
// r, read with its rows and columns in cyclic order from k+1 and r+1; in that order
// inv(A)(r, k) = (-1)^((k+r)(n-1)) det(minor) / det(A).
template <typename T, int N, int BS, bool STAGED>
__device__ __forceinline__ void chunk_entry(const PlanGroup& g, int64_t p0, int np, const Fallback& fb, T* lds,
                                            int& nrouted, int& nsing) {
    constexpr int NN = N * N, PW = 64 / NN, M = N - 1;
    const int wave = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int pl = wave * PW + ln / NN;
    const int q = ln % NN;
    const int r = q % N, k = q / N;
    const bool active = (ln < PW * NN) && (pl < np);
    const bool inv = g.ops & PF_OP_INV, mt = g.ops & PF_OP_MTIMES;
    T A[NN], mn[M * M > 0 ? M * M : 1], arow[N], Bk[N];
#pragma unroll
    for (int e = 0; e < NN; ++e) A[e] = T(0);
#pragma unroll
    for (int e = 0; e < M * M; ++e) mn[e] = T(0);
#pragma unroll
    for (int m = 0; m < N; ++m) arow[m] = Bk[m] = T(0);
    const T* pa = chunk_base<T, NN, BS, STAGED>(static_cast<const T*>(g.a) + p0 * NN, np, pl, lds);
    if (active) {
        if (inv) {
#pragma unroll
            for (int e = 0; e < NN; ++e) A[e] = pa[e];
#pragma unroll
            for (int j = 0; j < M; ++j)
#pragma unroll
                for (int i = 0; i < M; ++i) mn[i + j * M] = pa[(k + 1 + i) % N + ((r + 1 + j) % N) * N];
        }
        if (mt) {
#pragma unroll
            for (int m = 0; m < N; ++m) arow[m] = pa[r + m * N];
        }
    }
    if (mt) {
        if (STAGED) __syncthreads();
        const T* pb = chunk_base<T, NN, BS, STAGED>(static_cast<const T*>(g.b) + p0 * NN, np, pl, lds);
        if (active) {
#pragma unroll
            for (int m = 0; m < N; ++m) Bk[m] = pb[m + k * N];
        }
    }
    if (STAGED) __syncthreads();

    const int64_t page = p0 + pl;
    if (inv && active) {
        T c0[N], d, absterms;
        det_first_row<T, N>(A, c0, d, absterms);
        const bool neg = ((k + r) * M) & 1;
        bool route = false;
        if constexpr (sizeof(T) == 4) route = should_route(d, absterms, fb);
        T x;
        if (route) {
            double ad[NN], c0d[N], dd, md[M * M > 0 ? M * M : 1], cm[M > 0 ? M : 1], dm = 1.0;
#pragma unroll
            for (int e = 0; e < NN; ++e) ad[e] = static_cast<double>(A[e]);
            first_row_f64<N>(ad, c0d, dd);
            if constexpr (M > 0) {
#pragma unroll
                for (int e = 0; e < M * M; ++e) md[e] = static_cast<double>(mn[e]);
                first_row_f64<M>(md, cm, dm);
            }
            x = static_cast<T>((neg ? -dm : dm) / dd);
            d = static_cast<T>(dd);
        } else {
            T dm = T(1);
            if constexpr (M > 0) {
                T cm[M], am;
                det_first_row<T, M>(mn, cm, dm, am);
            }
            x = (neg ? -dm : dm) / d;
        }
        static_cast<T*>(g.x)[page * NN + r + k * N] = x;
        if (q == 0) {
            if (g.det) static_cast<T*>(g.det)[page] = d;
            nrouted += route;
            nsing += (d == T(0));
        }
    }
    if (mt && active) static_cast<T*>(g.c)[page * NN + r + k * N] = prod_entry<T, N>(arow, 0, 1, Bk);
}

// All tiles of one order under one lane mapping: the mapping is fixed for the loop, so each
// loop body is compiled on its own and the kernel's register budget is that of the largest
// body, not of all of them together.
template <typename T, int N, int L, bool STAGED, int BS>
__device__ __forceinline__ void phase_loop(const PlanGroup* __restrict__ grp, const PlanPhase& ph, const Fallback& fb,
                                           T* lds, int& nr, int& ns) {
    const int64_t G = gridDim.x;
    int64_t t = ph.t_lo + (static_cast<int64_t>(blockIdx.x) - ph.t_lo % G + G) % G;  // first tile of this block
    for (; t < ph.t_hi; t += G) {
        int lo = ph.g_lo, hi = ph.g_hi - 1;  // last group whose first tile is <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (grp[mid].tile0 <= t) lo = mid;
            else hi = mid - 1;
        }
        const PlanGroup g = grp[lo];
        const int64_t first = (t - g.tile0) * g.chunks * g.ppc;
        for (int ch = 0; ch < g.chunks; ++ch) {
            const int64_t p0 = first + static_cast<int64_t>(ch) * g.ppc;
            if (p0 >= g.count) break;
            const int np = static_cast<int>(min(static_cast<int64_t>(g.ppc), g.count - p0));
            if constexpr (L == 1) chunk_l1<T, N, BS, STAGED>(g, p0, np, fb, lds, nr, ns);
            else if constexpr (L == N) chunk_col<T, N, BS, STAGED>(g, p0, np, fb, lds, nr, ns);
            else chunk_entry<T, N, BS, STAGED>(g, p0, np, fb, lds, nr, ns);
        }
    }
}

template <typename T, int N, int BS>
__device__ __forceinline__ void phase(const PlanGroup* __restrict__ grp, const PlanPhase& ph, const Fallback& fb,
                                      T* lds, int& nr, int& ns) {
    if (ph.t_hi <= ph.t_lo) return;
    if constexpr (N == 1) {
        if (ph.staged) phase_loop<T, 1, 1, true, BS>(grp, ph, fb, lds, nr, ns);
        else phase_loop<T, 1, 1, false, BS>(grp, ph, fb, lds, nr, ns);
    } else {
        if (ph.lanes == 1) {
            if (ph.staged) phase_loop<T, N, 1, true, BS>(grp, ph, fb, lds, nr, ns);
            else phase_loop<T, N, 1, false, BS>(grp, ph, fb, lds, nr, ns);
        } else if (ph.lanes == N) {
            if (ph.staged) phase_loop<T, N, N, true, BS>(grp, ph, fb, lds, nr, ns);
            else phase_loop<T, N, N, false, BS>(grp, ph, fb, lds, nr, ns);
        } else {
            if (ph.staged) phase_loop<T, N, N * N, true, BS>(grp, ph, fb, lds, nr, ns);
            else phase_loop<T, N, N * N, false, BS>(grp, ph, fb, lds, nr, ns);
        }
    }
}

// Persistent kernel: the groups are sorted by order, so the tiles of each order form one
// consecutive range (a phase); workgroup b takes the tiles numbered b mod grid of every
// phase in turn, with no barrier between phases.
template <typename T, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_plan(const uint8_t* __restrict__ wl) {
    constexpr int BS = WAVES * 64;
    extern __shared__ __align__(16) unsigned char plan_lds[];
    T* lds = reinterpret_cast<T*>(plan_lds);
    static_assert(lds_carve_aligned<T>(), "plan LDS: one naturally aligned array");
    const PlanHeader* hdr = reinterpret_cast<const PlanHeader*>(wl);
    const PlanGroup* grp = reinterpret_cast<const PlanGroup*>(wl + PLAN_GROUPS_OFFSET);
    const Fallback fb = hdr->fb;
    int nr = 0, ns = 0;
    phase<T, 1, BS>(grp, hdr->phase[1], fb, lds, nr, ns);
    phase<T, 2, BS>(grp, hdr->phase[2], fb, lds, nr, ns);
    phase<T, 3, BS>(grp, hdr->phase[3], fb, lds, nr, ns);
    phase<T, 4, BS>(grp, hdr->phase[4], fb, lds, nr, ns);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        nr += __shfl_xor(nr, o, 64);
        ns += __shfl_xor(ns, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        count_add(hdr->counters, 0, nr);
        count_add(hdr->counters, 1, ns);
    }
}

}  // namespace pf

// ================================================================================= host
using namespace pf;

struct pf_plan {
    pf_dtype dtype = PF_F32;
    Fallback fb{};
    int32_t max_groups = 0;
    int device = 0, num_cus = 0;
    size_t max_lds = 0;
    std::string arch;
    pf_schedule sched{};
    std::vector<pf_group> groups;
    uint8_t* h_wl = nullptr;  // pinned
    uint8_t* d_wl = nullptr;
    size_t wl_bytes = 0;
    int64_t ntiles = 0;
    // graph
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_waves = 0, graph_grid = 0, graph_lds = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};

namespace {

using KernelFn = void (*)(const uint8_t*);

KernelFn kernel_of(pf_dtype dt, int waves) {
    if (dt == PF_F32) {
        switch (waves) {
            case 1: return k_plan<float, 1>;
            case 2: return k_plan<float, 2>;
            case 4: return k_plan<float, 4>;
            case 8: return k_plan<float, 8>;
        }
    } else {
        switch (waves) {
            case 1: return k_plan<double, 1>;
            case 2: return k_plan<double, 2>;
            case 4: return k_plan<double, 4>;
            case 8: return k_plan<double, 8>;
        }
    }
    return nullptr;
}

size_t elem_size(pf_dtype dt) { return dt == PF_F32 ? 4 : 8; }

int pages_per_chunk(int order, const pf_order_schedule& s, int waves) {
    return s.lanes == 1 ? waves * 64 : waves * (64 / s.lanes);
}

// LDS bytes of one workgroup: the largest staged chunk of any order (+16 bytes of lead)
int lds_bytes_of(const pf_schedule& s, pf_dtype dt) {
    size_t m = 0;
    for (int n = 1; n <= 4; ++n) {
        const pf_order_schedule& o = s.order[n];
        if (!o.staged) continue;
        const size_t b = static_cast<size_t>(pages_per_chunk(n, o, s.waves)) * n * n * elem_size(dt) + 16;
        m = std::max(m, b);
    }
    return static_cast<int>(m);
}

pf_schedule default_schedule() {
    pf_schedule s{};
    s.waves = 4;
    for (int n = 0; n <= 4; ++n) s.order[n] = pf_order_schedule{1, 1, 1};
    return s;
}

pf_status check_schedule(const pf_plan* p, const pf_schedule& s) {
    if (s.waves != 1 && s.waves != 2 && s.waves != 4 && s.waves != 8)
        return fail(PF_EINVAL, "pf_plan: waves must be 1, 2, 4 or 8");
    for (int n = 1; n <= 4; ++n) {
        const pf_order_schedule& o = s.order[n];
        if (o.lanes != 1 && o.lanes != n && o.lanes != n * n)
            return fail(PF_EINVAL, "pf_plan: lanes of order " + std::to_string(n) + " must be 1, n or n*n");
        if (o.staged != 0 && o.staged != 1) return fail(PF_EINVAL, "pf_plan: staged must be 0 or 1");
        if (o.tile < 1 || o.tile > 16) return fail(PF_EINVAL, "pf_plan: tile must be 1..16");
    }
    if (static_cast<size_t>(lds_bytes_of(s, p->dtype)) > p->max_lds)
        return fail(PF_EINVAL, "pf_plan: staging buffer exceeds the LDS of one workgroup");
    return PF_OK;
}

// write the work list of `gs` (a subset of the plan's groups) under schedule `s`: groups
// with pages, sorted by order (stable), and the tile range of each order
void build_worklist(pf_plan* p, const std::vector<pf_group>& gs, const pf_schedule& s) {
    PlanHeader* h = reinterpret_cast<PlanHeader*>(p->h_wl);
    PlanGroup* dg = reinterpret_cast<PlanGroup*>(p->h_wl + PLAN_GROUPS_OFFSET);
    int ng = 0;
    int64_t tiles = 0;
    for (int n = 1; n <= 4; ++n) {
        const pf_order_schedule& o = s.order[n];
        const int lanes = n == 1 ? 1 : o.lanes;
        PlanPhase ph{};
        ph.t_lo = tiles;
        ph.g_lo = ng;
        ph.lanes = lanes;
        ph.staged = o.staged;
        for (const pf_group& g : gs) {
            if (g.count <= 0 || g.order != n) continue;
            PlanGroup d{};
            d.a = g.a;
            d.b = g.b;
            d.x = g.x;
            d.c = g.c;
            d.det = g.det;
            d.count = g.count;
            d.order = g.order;
            d.ops = g.ops;
            d.lanes = lanes;
            d.staged = o.staged;
            d.chunks = o.tile;
            d.ppc = pages_per_chunk(n, pf_order_schedule{lanes, o.staged, o.tile}, s.waves);
            d.tile0 = tiles;
            tiles += ceil_div(g.count, static_cast<int64_t>(d.ppc) * d.chunks);
            dg[ng++] = d;
        }
        ph.t_hi = tiles;
        ph.g_hi = ng;
        h->phase[n] = ph;
    }
    h->ntiles = tiles;
    h->ngroups = ng;
    h->fb = p->fb;
    p->ntiles = tiles;
}

pf_status wait_idle(pf_plan* p) {
    if (p->pending) {
        PF_HIP_TRY(hipEventSynchronize(p->done));
        p->pending = false;
    }
    return PF_OK;
}

pf_status grid_of(pf_plan* p, const pf_schedule& s, int& grid, int& lds) {
    lds = lds_bytes_of(s, p->dtype);
    const int bs = s.waves * 64;
    int occ = 0;
    PF_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(kernel_of(p->dtype, s.waves)),
                                                            bs, static_cast<size_t>(lds)));
    if (occ < 1) occ = 1;
    grid = p->num_cus * occ;
    return PF_OK;
}

pf_status set_counters(pf_plan* p, int64_t* d_counters) {
    PlanHeader* h = reinterpret_cast<PlanHeader*>(p->h_wl);
    if (h->counters != d_counters) {
        pf_status st = wait_idle(p);
        if (st != PF_OK) return st;
        h->counters = d_counters;
    }
    return PF_OK;
}

pf_status launch_eager(pf_plan* p, const pf_schedule& s, hipStream_t stream) {
    int grid, lds;
    pf_status st = grid_of(p, s, grid, lds);
    if (st != PF_OK) return st;
    PF_HIP_TRY(hipMemcpyAsync(p->d_wl, p->h_wl, p->wl_bytes, hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(kernel_of(p->dtype, s.waves), dim3(grid), dim3(s.waves * 64), lds, stream, p->d_wl);
    st = launch_check("k_plan");
    if (st != PF_OK) return st;
    PF_HIP_TRY(hipEventRecord(p->done, stream));
    p->pending = true;
    return PF_OK;
}

void drop_graph(pf_plan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->graph_waves = 0;
}

pf_status capture(pf_plan* p) {
    drop_graph(p);
    int grid, lds;
    pf_status st = grid_of(p, p->sched, grid, lds);
    if (st != PF_OK) return st;
    PF_HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = hipMemcpyAsync(p->d_wl, p->h_wl, p->wl_bytes, hipMemcpyHostToDevice, p->cap);
    hipLaunchKernelGGL(kernel_of(p->dtype, p->sched.waves), dim3(grid), dim3(p->sched.waves * 64), lds, p->cap,
                       p->d_wl);
    hipError_t e2 = hipGetLastError();
    hipGraph_t g = nullptr;
    hipError_t e3 = hipStreamEndCapture(p->cap, &g);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        const hipError_t e = e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3);
        return fail(PF_EHIP, std::string("pf_plan: graph capture: ") + hipGetErrorString(e));
    }
    p->graph = g;
    PF_HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    p->graph_waves = p->sched.waves;
    p->graph_grid = grid;
    p->graph_lds = lds;
    return PF_OK;
}

// ------------------------------------------------------------------ tuner and its cache
const char* dtype_name(pf_dtype dt) { return dt == PF_F32 ? "f32" : "f64"; }

int bucket_of(int64_t pages) {
    int b = 0;
    while (b < 62 && (int64_t(1) << (b + 1)) <= pages) ++b;
    return b;
}

using Cache = std::map<std::string, std::map<std::string, long long>>;

// The cache file is one flat JSON object: {"key": {"field": integer, ...}, ...}.
bool read_cache(const char* path, Cache& c) {
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t i = 0;
    auto skip = [&]() {
        while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t' || s[i] == ','))
            ++i;
    };
    auto str = [&](std::string& out) -> bool {
        skip();
        if (i >= s.size() || s[i] != '"') return false;
        const size_t j = s.find('"', i + 1);
        if (j == std::string::npos) return false;
        out = s.substr(i + 1, j - i - 1);
        i = j + 1;
        skip();
        if (i >= s.size() || s[i] != ':') return false;
        ++i;
        return true;
    };
    skip();
    if (i >= s.size() || s[i] != '{') return false;
    ++i;
    for (;;) {
        skip();
        if (i < s.size() && s[i] == '}') return true;
        std::string key;
        if (!str(key)) return false;
        skip();
        if (i >= s.size() || s[i] != '{') return false;
        ++i;
        std::map<std::string, long long> fields;
        for (;;) {
            skip();
            if (i < s.size() && s[i] == '}') {
                ++i;
                break;
            }
            std::string name;
            if (!str(name)) return false;
            skip();
            size_t used = 0;
            long long v = 0;
            try {
                v = std::stoll(s.substr(i, 24), &used);
            } catch (...) {
                return false;
            }
            i += used;
            fields[name] = v;
        }
        c[key] = fields;
    }
}

bool write_cache(const char* path, const Cache& c) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "{\n";
        size_t k = 0;
        for (const auto& kv : c) {
            f << "  \"" << kv.first << "\": {";
            size_t j = 0;
            for (const auto& fv : kv.second) f << (j++ ? ", " : "") << "\"" << fv.first << "\": " << fv.second;
            f << "}" << (++k < c.size() ? ",\n" : "\n");
        }
        f << "}\n";
    }
    return std::rename(tmp.c_str(), path) == 0;
}

// median time (ms) of the plan's kernel on the groups `gs` under schedule `s`
pf_status time_schedule(pf_plan* p, const std::vector<pf_group>& gs, const pf_schedule& s, hipStream_t stream,
                        float& ms) {
    pf_status st = wait_idle(p);
    if (st != PF_OK) return st;
    build_worklist(p, gs, s);
    hipEvent_t e0, e1;
    PF_HIP_TRY(hipEventCreate(&e0));
    PF_HIP_TRY(hipEventCreate(&e1));
    std::vector<float> t;
    for (int rep = 0; rep < 7 && st == PF_OK; ++rep) {
        if (rep >= 2) (void)hipEventRecord(e0, stream);
        st = launch_eager(p, s, stream);
        if (st != PF_OK) break;
        if (rep >= 2) {
            (void)hipEventRecord(e1, stream);
            (void)hipEventSynchronize(e1);
            float x = 0;
            (void)hipEventElapsedTime(&x, e0, e1);
            t.push_back(x);
        }
    }
    (void)hipStreamSynchronize(stream);
    p->pending = false;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PF_OK) return st;
    std::sort(t.begin(), t.end());
    ms = t[t.size() / 2];
    return PF_OK;
}

std::string key_waves(const pf_plan* p, int64_t total) {
    return p->arch + "|" + dtype_name(p->dtype) + "|waves|b" + std::to_string(bucket_of(total));
}

std::string key_order(const pf_plan* p, int waves, int n, int64_t pages) {
    return p->arch + "|" + dtype_name(p->dtype) + "|w" + std::to_string(waves) + "|n" + std::to_string(n) + "|b" +
           std::to_string(bucket_of(pages));
}

pf_status tune(pf_plan* p, hipStream_t stream, pf_schedule& best) {
    const pf_schedule def = default_schedule();
    float t_def = 0;
    pf_status st = time_schedule(p, p->groups, def, stream, t_def);
    if (st != PF_OK) return st;
    // 1. waves per workgroup under the default per-order schedule
    pf_schedule s = def;
    float tb = t_def;
    for (int w : {1, 2, 8}) {
        pf_schedule c = def;
        c.waves = w;
        if (check_schedule(p, c) != PF_OK) continue;
        float t = 0;
        st = time_schedule(p, p->groups, c, stream, t);
        if (st != PF_OK) return st;
        if (t < tb) {
            tb = t;
            s = c;
        }
    }
    // 2. per order: lanes x staging x tile, timed on that order's groups alone
    for (int n = 1; n <= 4; ++n) {
        std::vector<pf_group> sub;
        for (const pf_group& g : p->groups)
            if (g.order == n && g.count > 0) sub.push_back(g);
        if (sub.empty()) continue;
        pf_order_schedule bo = s.order[n];
        float bt = 0;
        st = time_schedule(p, sub, s, stream, bt);
        if (st != PF_OK) return st;
        const int lanes_opts[3] = {1, n, n * n};
        for (int li = 0; li < (n == 1 ? 1 : 3); ++li) {
            if (li == 2 && n == 1) continue;
            for (int staged = 0; staged <= 1; ++staged)
                for (int tile : {1, 2, 4}) {
                    pf_schedule c = s;
                    c.order[n] = pf_order_schedule{lanes_opts[li], staged, tile};
                    if (check_schedule(p, c) != PF_OK) continue;
                    float t = 0;
                    st = time_schedule(p, sub, c, stream, t);
                    if (st != PF_OK) return st;
                    if (t < bt) {
                        bt = t;
                        bo = c.order[n];
                    }
                }
        }
        s.order[n] = bo;
    }
    // 3. keep the tuned schedule only if it beats the default on the whole batch
    float ts = 0;
    st = time_schedule(p, p->groups, s, stream, ts);
    if (st != PF_OK) return st;
    best = ts < t_def ? s : def;
    return PF_OK;
}

}  // namespace

extern "C" {

pf_status pf_plan_create(pf_dtype dtype, int32_t max_groups, const pf_fallback* fb, pf_plan** out) {
    if (!out) return fail(PF_EINVAL, "pf_plan_create: out is NULL");
    *out = nullptr;
    if (dtype != PF_F32 && dtype != PF_F64) return fail(PF_EDTYPE, "pf_plan_create: dtype");
    if (max_groups < 1 || max_groups > (1 << 20)) return fail(PF_EINVAL, "pf_plan_create: max_groups must be 1..2^20");
    pf_plan* p = new (std::nothrow) pf_plan();
    if (!p) return fail(PF_ENOMEM, "pf_plan_create: host allocation");
    p->dtype = dtype;
    p->fb = make_fallback(fb);
    p->max_groups = max_groups;
    p->sched = default_schedule();
    p->wl_bytes = PLAN_GROUPS_OFFSET + sizeof(PlanGroup) * static_cast<size_t>(max_groups);
    hipError_t e = hipGetDevice(&p->device);
    hipDeviceProp_t prop;
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, p->device);
    if (e == hipSuccess) {
        p->num_cus = prop.multiProcessorCount;
        p->max_lds = prop.sharedMemPerBlock;
        p->arch = prop.gcnArchName;
        const size_t colon = p->arch.find(':');
        if (colon != std::string::npos) p->arch = p->arch.substr(0, colon);
    }
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&p->h_wl), p->wl_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&p->d_wl), p->wl_bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        pf_plan_destroy(p);
        return fail(e == hipErrorOutOfMemory ? PF_ENOMEM : PF_EHIP,
                    std::string("pf_plan_create: ") + hipGetErrorString(e));
    }
    std::memset(p->h_wl, 0, p->wl_bytes);
    build_worklist(p, p->groups, p->sched);
    *out = p;
    return PF_OK;
}

pf_status pf_plan_set_groups(pf_plan* p, const pf_group* groups, int32_t ngroups) {
    if (!p) return fail(PF_EINVAL, "pf_plan_set_groups: plan is NULL");
    if (ngroups < 0 || ngroups > p->max_groups || (ngroups > 0 && !groups))
        return fail(PF_EINVAL, "pf_plan_set_groups: ngroups must be 0..max_groups with a group array");
    const size_t es = elem_size(p->dtype);
    for (int32_t i = 0; i < ngroups; ++i) {
        const pf_group& g = groups[i];
        const std::string w = "pf_plan_set_groups: group " + std::to_string(i) + ": ";
        if (g.order < 1 || g.order > 4) return fail(PF_EORDER, w + "order must be 1..4");
        if (g.ops < 1 || g.ops > 3) return fail(PF_EINVAL, w + "ops must be PF_OP_INV and/or PF_OP_MTIMES");
        if (g.count < 0 || g.count > (int64_t(1) << 40)) return fail(PF_EINVAL, w + "count out of range");
        if (g.count == 0) continue;
        auto bad = [&](const void* q) { return !q || (reinterpret_cast<uintptr_t>(q) % es) != 0; };
        if (bad(g.a)) return fail(PF_EINVAL, w + "a is NULL or misaligned");
        if ((g.ops & PF_OP_INV) && bad(g.x)) return fail(PF_EINVAL, w + "x is NULL or misaligned");
        if ((g.ops & PF_OP_INV) && g.det && bad(g.det)) return fail(PF_EINVAL, w + "det is misaligned");
        if ((g.ops & PF_OP_MTIMES) && (bad(g.b) || bad(g.c)))
            return fail(PF_EINVAL, w + "b or c is NULL or misaligned");
    }
    pf_status st = wait_idle(p);
    if (st != PF_OK) return st;
    p->groups.assign(groups, groups + ngroups);
    build_worklist(p, p->groups, p->sched);
    return PF_OK;
}

pf_status pf_plan_get_schedule(const pf_plan* p, pf_schedule* out) {
    if (!p || !out) return fail(PF_EINVAL, "pf_plan_get_schedule: NULL argument");
    *out = p->sched;
    return PF_OK;
}

pf_status pf_plan_set_schedule(pf_plan* p, const pf_schedule* s) {
    if (!p || !s) return fail(PF_EINVAL, "pf_plan_set_schedule: NULL argument");
    pf_schedule c = *s;
    c.order[0] = pf_order_schedule{1, 1, 1};
    pf_status st = check_schedule(p, c);
    if (st != PF_OK) return st;
    st = wait_idle(p);
    if (st != PF_OK) return st;
    p->sched = c;
    build_worklist(p, p->groups, p->sched);
    return PF_OK;
}

pf_status pf_plan_tune(pf_plan* p, const char* cache_path, int32_t mode, void* stream) {
    if (!p) return fail(PF_EINVAL, "pf_plan_tune: plan is NULL");
    if (mode != PF_TUNE_CACHED && mode != PF_TUNE_FORCE && mode != PF_TUNE_DEFAULT)
        return fail(PF_EINVAL, "pf_plan_tune: mode");
    const hipStream_t s = as_stream(stream);
    pf_schedule chosen = default_schedule();
    pf_status st0 = wait_idle(p);
    if (st0 != PF_OK) return st0;
    // tuning runs never add to the caller's counters
    PlanHeader* hdr = reinterpret_cast<PlanHeader*>(p->h_wl);
    int64_t* const user_counters = hdr->counters;
    hdr->counters = nullptr;
    if (mode != PF_TUNE_DEFAULT) {
        int64_t per_order[5] = {0, 0, 0, 0, 0}, total = 0;
        for (const pf_group& g : p->groups) {
            per_order[g.order] += g.count;
            total += g.count;
        }
        Cache cache;
        if (cache_path) read_cache(cache_path, cache);
        bool hit = mode == PF_TUNE_CACHED && total > 0;
        pf_schedule c = default_schedule();
        if (hit) {
            auto it = cache.find(key_waves(p, total));
            if (it == cache.end()) hit = false;
            else c.waves = static_cast<int32_t>(it->second["waves"]);
            for (int n = 1; n <= 4 && hit; ++n) {
                if (!per_order[n]) continue;
                auto jt = cache.find(key_order(p, c.waves, n, per_order[n]));
                if (jt == cache.end()) {
                    hit = false;
                    break;
                }
                c.order[n] = pf_order_schedule{static_cast<int32_t>(jt->second["lanes"]),
                                               static_cast<int32_t>(jt->second["staged"]),
                                               static_cast<int32_t>(jt->second["tile"])};
            }
            if (hit && check_schedule(p, c) != PF_OK) hit = false;  // stale or foreign entry
        }
        if (hit) {
            chosen = c;
        } else if (total > 0) {
            pf_status st = tune(p, s, chosen);
            if (st != PF_OK) {
                build_worklist(p, p->groups, p->sched);
                hdr->counters = user_counters;
                return st;
            }
            if (cache_path) {
                cache[key_waves(p, total)] = {{"waves", chosen.waves}};
                for (int n = 1; n <= 4; ++n)
                    if (per_order[n])
                        cache[key_order(p, chosen.waves, n, per_order[n])] = {
                            {"lanes", chosen.order[n].lanes}, {"staged", chosen.order[n].staged},
                            {"tile", chosen.order[n].tile}};
                if (!write_cache(cache_path, cache)) {
                    hdr->counters = user_counters;
                    return fail(PF_EINVAL, std::string("pf_plan_tune: cannot write ") + cache_path);
                }
            }
        }
    }
    pf_status st = wait_idle(p);
    hdr->counters = user_counters;
    if (st != PF_OK) return st;
    p->sched = chosen;
    build_worklist(p, p->groups, p->sched);
    return PF_OK;
}

pf_status pf_plan_run(pf_plan* p, int64_t* d_counters, void* stream) {
    if (!p) return fail(PF_EINVAL, "pf_plan_run: plan is NULL");
    pf_status st = set_counters(p, d_counters);
    if (st != PF_OK) return st;
    int grid, lds;
    st = grid_of(p, p->sched, grid, lds);
    if (st != PF_OK) return st;
    if (!p->exec || p->graph_waves != p->sched.waves || p->graph_grid != grid || p->graph_lds != lds) {
        st = wait_idle(p);
        if (st == PF_OK) st = capture(p);
        if (st != PF_OK) return st;
    }
    PF_HIP_TRY(hipGraphLaunch(p->exec, as_stream(stream)));
    PF_HIP_TRY(hipEventRecord(p->done, as_stream(stream)));
    p->pending = true;
    return PF_OK;
}

pf_status pf_plan_launch(pf_plan* p, int64_t* d_counters, void* stream) {
    if (!p) return fail(PF_EINVAL, "pf_plan_launch: plan is NULL");
    pf_status st = set_counters(p, d_counters);
    if (st != PF_OK) return st;
    return launch_eager(p, p->sched, as_stream(stream));
}

pf_status pf_plan_info(const pf_plan* p, int64_t* ntiles, int32_t* grid, int32_t* lds_bytes) {
    if (!p) return fail(PF_EINVAL, "pf_plan_info: plan is NULL");
    int g = 0, l = 0;
    pf_status st = grid_of(const_cast<pf_plan*>(p), p->sched, g, l);
    if (st != PF_OK) return st;
    if (ntiles) *ntiles = p->ntiles;
    if (grid) *grid = g;
    if (lds_bytes) *lds_bytes = l;
    return PF_OK;
}

void pf_plan_destroy(pf_plan* p) {
    if (!p) return;
    if (p->pending && p->done) (void)hipEventSynchronize(p->done);
    drop_graph(p);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->done) (void)hipEventDestroy(p->done);
    if (p->d_wl) (void)hipFree(p->d_wl);
    if (p->h_wl) (void)hipHostFree(p->h_wl);
    delete p;
}

}  // extern "C"
