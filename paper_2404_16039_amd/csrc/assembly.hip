// assembly.hip -- COO -> CSR assembly of the P1 stiffness and mass matrices, i.e. the
// sparse(X3D(:), Y3D(:), K3D(:), nn, nn) call of the section 3.5 listings, without ever
// materialising the 16 (row, col, value) triples per element.
//
// Symbolic phase (integer-exact, cached in a pf_csr handle):
//   1. count the elements around every node (node -> element adjacency, a transpose of
//      `elems` by counting sort), scan the counts, scatter (element, local index) pairs;
//   2. per node (one lane per row): sort its adjacency list ascending by element id, and
//      merge the element node lists into the sorted set of distinct neighbours (LDS lists
//      interleaved across lanes, so every lane's dynamic index hits its own bank);
//   3. scan the row lengths into row_ptr, write col_idx.
// Numeric phase (one lane per row, deterministic):
//   each lane walks its node's sorted adjacency, recomputes each element's P1 geometry in
//   registers (FP32 with compensated cofactors, FP64 for routed elements), and adds row a
//   of K_e and M_e into the row's slots, found by binary search in the row's column list.
//   A workgroup owns a contiguous block of rows, hence a contiguous window of the CSR
//   arrays: columns are staged into LDS and the accumulated values leave LDS with fully
//   coalesced stores.  Every slot is summed in ascending element order, so the result is
//   bitwise reproducible and independent of scheduling.
#include "p1elem.hpp"

#include <algorithm>
#include <new>
#include <vector>

struct pf_csr {
    int dim = 0, nlb = 0;
    int64_t nn = 0, ne = 0, nnz = 0;
    int max_window = 0;       // largest CSR window of one numeric workgroup
    int32_t* adj_ptr = nullptr;
    int32_t* adj = nullptr;   // (element << 2) | local index, sorted per node
    int32_t* row_ptr = nullptr;
    int32_t* col_idx = nullptr;
    int32_t* cnt = nullptr;   // per-node counts / cursors / row lengths
    int64_t* bsum = nullptr;  // scan workspace
    int64_t* info = nullptr;  // [0] error bits, [1] adjacency total, [2] nnz, [3] max window
    int64_t cap_adj_ptr = 0, cap_row_ptr = 0, cap_cnt = 0, cap_adj = 0, cap_nnz = 0, cap_bsum = 0, cap_info = 0;
    bool built = false;
};

namespace pf {

constexpr int SBS = 256;         // threads per block in the flat symbolic kernels
constexpr int SCAN_ITEMS = 8;    // items per thread in the scan
constexpr int SCAN_TILE = SBS * SCAN_ITEMS;
constexpr int RBS = 128;         // rows per block in the row kernels
constexpr int MAXADJ = 64;       // elements per node
constexpr int MAXROW = 64;       // nonzeros per row
constexpr int NBS = 128;         // rows per block in the numeric kernel
constexpr size_t LDS_BYTES = 65536;  // largest window staged in LDS (else the global path)

constexpr int64_t ERR_INDEX = 1, ERR_ADJ = 2, ERR_ROW = 4;

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------- scan
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t& total) {
    __shared__ int64_t wsum[SBS / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < SBS / 64; ++q) {
        if (q < w) off += wsum[q];
        tot += wsum[q];
    }
    __syncthreads();
    total = tot;
    return off + x - v;
}

__global__ __launch_bounds__(SBS) void k_scan_reduce(const int32_t* __restrict__ in, int64_t n,
                                                     int64_t* __restrict__ bsum) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE;
    int64_t s = 0;
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        const int64_t i = base + q * SBS + threadIdx.x;
        if (i < n) s += in[i];
    }
    int64_t tot;
    block_exclusive_scan(s, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SBS) void k_scan_top(int64_t* __restrict__ bsum, int64_t nb, int64_t* __restrict__ total_out) {
    int64_t carry = 0;
    for (int64_t c = 0; c < nb; c += SBS) {
        const int64_t i = c + threadIdx.x;
        const int64_t v = (i < nb) ? bsum[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan(v, tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(SBS) void k_scan_apply(const int32_t* __restrict__ in, int64_t n,
                                                    const int64_t* __restrict__ bsum, int32_t* __restrict__ out) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE + static_cast<int64_t>(threadIdx.x) * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        v[q] = (base + q < n) ? in[base + q] : 0;
        s += v[q];
    }
    int64_t tot;
    int64_t run = bsum[blockIdx.x] + block_exclusive_scan(s, tot);
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        if (base + q < n) out[base + q] = static_cast<int32_t>(run);
        run += v[q];
    }
    if (base < n && base + SCAN_ITEMS >= n) out[n] = static_cast<int32_t>(run);  // the tile holding the last item
}

// ---------------------------------------------------------------------------- adjacency
__global__ __launch_bounds__(SBS) void k_count(const int32_t* __restrict__ elems, int64_t m, int64_t nn,
                                               int32_t* __restrict__ cnt, int64_t* __restrict__ info) {
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * SBS + threadIdx.x; t < m;
         t += static_cast<int64_t>(gridDim.x) * SBS) {
        const int32_t node = elems[t];
        if (node < 0 || node >= nn)
            atomicOr(reinterpret_cast<unsigned long long*>(info), static_cast<unsigned long long>(ERR_INDEX));
        else
            atomicAdd(cnt + node, 1);
    }
}

__global__ __launch_bounds__(SBS) void k_scatter(const int32_t* __restrict__ elems, int64_t m, int nlb, int64_t nn,
                                                 const int32_t* __restrict__ adj_ptr, int32_t* __restrict__ cursor,
                                                 int32_t* __restrict__ adj) {
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * SBS + threadIdx.x; t < m;
         t += static_cast<int64_t>(gridDim.x) * SBS) {
        const int32_t node = elems[t];
        if (node < 0 || node >= nn) continue;
        const int64_t e = t / nlb;
        const int a = static_cast<int>(t - e * nlb);
        const int32_t pos = adj_ptr[node] + atomicAdd(cursor + node, 1);
        adj[pos] = static_cast<int32_t>((e << 2) | a);
    }
}

// insert `v` into the interleaved sorted list lst[0..n) (stride RBS); returns false when full
__device__ __forceinline__ bool insert_unique(int32_t* lst, int& n, int32_t v, int cap) {
    int p = 0;
    while (p < n && lst[p * RBS] < v) ++p;
    if (p < n && lst[p * RBS] == v) return true;
    if (n >= cap) return false;
    for (int q = n; q > p; --q) lst[q * RBS] = lst[(q - 1) * RBS];
    lst[p * RBS] = v;
    ++n;
    return true;
}

// sort each node's adjacency and count its distinct neighbours (row length)
__global__ __launch_bounds__(RBS) void k_rows(int64_t nn, int nlb, const int32_t* __restrict__ elems,
                                              const int32_t* __restrict__ adj_ptr, int32_t* __restrict__ adj,
                                              int32_t* __restrict__ rowlen, int64_t* __restrict__ info) {
    __shared__ int32_t lds[MAXADJ * RBS];
    int32_t* lst = lds + threadIdx.x;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * RBS + threadIdx.x;
    if (i >= nn) return;
    const int32_t b = adj_ptr[i];
    const int L = adj_ptr[i + 1] - b;
    if (L > MAXADJ) {
        atomicOr(reinterpret_cast<unsigned long long*>(info), static_cast<unsigned long long>(ERR_ADJ));
        rowlen[i] = 0;
        return;
    }
    for (int j = 0; j < L; ++j) {  // insertion sort (lists are short)
        const int32_t v = adj[b + j];
        int p = j;
        while (p > 0 && lst[(p - 1) * RBS] > v) {
            lst[p * RBS] = lst[(p - 1) * RBS];
            --p;
        }
        lst[p * RBS] = v;
    }
    for (int j = 0; j < L; ++j) adj[b + j] = lst[j * RBS];
    int n = 0;
    bool ok = true;
    for (int j = 0; j < L && ok; ++j) {
        const int64_t e = adj[b + j] >> 2;
        for (int q = 0; q < nlb && ok; ++q) ok = insert_unique(lst, n, elems[e * nlb + q], MAXROW);
    }
    if (!ok) atomicOr(reinterpret_cast<unsigned long long*>(info), static_cast<unsigned long long>(ERR_ROW));
    rowlen[i] = ok ? n : 0;
}

__global__ __launch_bounds__(RBS) void k_cols(int64_t nn, int nlb, const int32_t* __restrict__ elems,
                                              const int32_t* __restrict__ adj_ptr, const int32_t* __restrict__ adj,
                                              const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_idx) {
    __shared__ int32_t lds[MAXROW * RBS];
    int32_t* lst = lds + threadIdx.x;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * RBS + threadIdx.x;
    if (i >= nn) return;
    const int32_t b = adj_ptr[i];
    const int L = adj_ptr[i + 1] - b;
    int n = 0;
    for (int j = 0; j < L; ++j) {
        const int64_t e = adj[b + j] >> 2;
        for (int q = 0; q < nlb; ++q) insert_unique(lst, n, elems[e * nlb + q], MAXROW);
    }
    const int32_t o = row_ptr[i];
    for (int j = 0; j < n; ++j) col_idx[o + j] = lst[j * RBS];
}

__global__ void k_window_max(int64_t nn, const int32_t* __restrict__ row_ptr, int64_t nblk, int64_t* __restrict__ info) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    const int64_t r0 = b * NBS;
    const int64_t r1 = (r0 + NBS < nn) ? r0 + NBS : nn;
    const int64_t w = row_ptr[r1] - row_ptr[r0];
    atomicMax(reinterpret_cast<unsigned long long*>(info + 3), static_cast<unsigned long long>(w));
}

// ---------------------------------------------------------------------------- numeric
__device__ __forceinline__ int find_col(const int32_t* __restrict__ cols, int len, int32_t v) {
    int lo = 0, hi = len;  // first position with cols[p] >= v
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cols[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return (lo < len && cols[lo] == v) ? lo : -1;
}

// Row a of K_e and M_e (coefficients and FP64 routing included), computed in precision C.
template <int DIM, typename C>
__device__ __forceinline__ void elem_row(const P1Geom<DIM, C>& g, int a, C ck, C cm, C (&krow)[DIM + 1], C& moff) {
    const C adet = fabs(g.det);
    const C kf = ck / (static_cast<C>(fact_dim<DIM>()) * adet);
    C ca[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        C v = g.c[0][i];
#pragma unroll
        for (int j = 1; j <= DIM; ++j) v = (a == j) ? g.c[j][i] : v;
        ca[i] = v;
    }
#pragma unroll
    for (int b = 0; b <= DIM; ++b) {
        C s = ca[0] * g.c[b][0];
#pragma unroll
        for (int i = 1; i < DIM; ++i) s = fmaT(ca[i], g.c[b][i], s);
        krow[b] = kf * s;
    }
    moff = cm * (adet / static_cast<C>(fact_dim<DIM>())) / static_cast<C>((DIM + 1) * (DIM + 2));
}

template <int DIM, typename T, bool LDS>
__global__ __launch_bounds__(NBS) void k_numeric(int64_t nn, const double* __restrict__ coords,
                                                 const int32_t* __restrict__ elems, const int32_t* __restrict__ adj_ptr,
                                                 const int32_t* __restrict__ adj, const int32_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ col_idx, const T* __restrict__ cK,
                                                 const T* __restrict__ cM, T* __restrict__ valsK, T* __restrict__ valsM,
                                                 Fallback fb, int64_t* d_counters) {
    constexpr int NLB = DIM + 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * NBS;
    const int64_t r1 = (r0 + NBS < nn) ? r0 + NBS : nn;
    const int32_t w0 = row_ptr[r0];
    const int W = row_ptr[r1] - w0;
    T* accK;
    T* accM;
    const int32_t* cols;
    if constexpr (LDS) {
        accK = reinterpret_cast<T*>(smem);
        accM = accK + W;
        int32_t* c = reinterpret_cast<int32_t*>(accM + W);
        for (int w = threadIdx.x; w < W; w += NBS) {
            c[w] = col_idx[w0 + w];
            accK[w] = T(0);
            accM[w] = T(0);
        }
        cols = c;
        __syncthreads();
    } else {
        accK = valsK + w0;
        accM = valsM ? valsM + w0 : nullptr;
        cols = col_idx + w0;
        for (int w = threadIdx.x; w < W; w += NBS) {
            accK[w] = T(0);
            if (accM) accM[w] = T(0);
        }
        __syncthreads();
    }
    const int64_t i = r0 + threadIdx.x;
    int64_t bad = 0;
    if (i < r1) {
        const int s0 = row_ptr[i] - w0;
        const int len = row_ptr[i + 1] - row_ptr[i];
        const int32_t* rc = cols + s0;
        const int diag = find_col(rc, len, static_cast<int32_t>(i));
        const int32_t t1 = adj_ptr[i + 1];
        for (int32_t t = adj_ptr[i]; t < t1; ++t) {
            const int32_t v = adj[t];
            const int64_t e = v >> 2;
            const int a = v & 3;
            int nd[NLB];
            load_nodes<DIM>(elems, e, nd);
            double ev[DIM][DIM];
            if (!p1_edges<DIM>(coords, nn, nd, ev) || diag < 0) {
                ++bad;
                continue;
            }
            T krow[NLB], moff;
            const T ck = cK ? cK[e] : T(1);
            const T cm = cM ? cM[e] : T(1);
            if constexpr (sizeof(T) == 4) {
                P1Geom<DIM, float> g;
                p1_geom<DIM, float>(ev, g);
                if (should_route(g.det, g.absterms, fb)) {
                    P1Geom<DIM, double> gd;
                    p1_geom<DIM, double>(ev, gd);
                    double kr[NLB], mo;
                    elem_row<DIM, double>(gd, a, ck, cm, kr, mo);
#pragma unroll
                    for (int b = 0; b < NLB; ++b) krow[b] = static_cast<T>(kr[b]);
                    moff = static_cast<T>(mo);
                    if (a == 0) count_add(d_counters, 0, 1);
                } else {
                    elem_row<DIM, float>(g, a, ck, cm, krow, moff);
                }
            } else {
                P1Geom<DIM, double> g;
                p1_geom<DIM, double>(ev, g);
                elem_row<DIM, double>(g, a, ck, cm, krow, moff);
            }
#pragma unroll
            for (int b = 0; b < NLB; ++b) {
                const int slot = (b == a) ? diag : find_col(rc, len, nd[b]);
                if (slot < 0) {
                    ++bad;
                    continue;
                }
                accK[s0 + slot] += krow[b];
                if (LDS || accM) accM[s0 + slot] += (b == a) ? moff + moff : moff;
            }
        }
    }
    if (bad) count_add(d_counters, 2, bad);
    if constexpr (LDS) {
        __syncthreads();
        for (int w = threadIdx.x; w < W; w += NBS) {
            valsK[w0 + w] = accK[w];
            if (valsM) valsM[w0 + w] = accM[w];
        }
    }
}

// ---------------------------------------------------------------------------- host
namespace {

template <typename P>
pf_status grow(P*& p, int64_t& cap, int64_t need) {
    if (need <= cap && p) return PF_OK;
    if (p) {
        PF_HIP_TRY(hipFree(p));
        p = nullptr;
    }
    cap = 0;
    const size_t bytes = sizeof(P) * static_cast<size_t>(need > 0 ? need : 1);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), bytes);
    if (e != hipSuccess) return fail(PF_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    cap = need;
    return PF_OK;
}

unsigned flat_grid(int64_t n) {
    int64_t g = ceil_div(n, SBS);
    if (g > 65536) g = 65536;
    return static_cast<unsigned>(g < 1 ? 1 : g);
}

pf_status scan(const int32_t* in, int64_t n, int32_t* out, int64_t* bsum, int64_t* total, hipStream_t s) {
    const int64_t nb = ceil_div(n, SCAN_TILE);
    if (nb > 0) hipLaunchKernelGGL(k_scan_reduce, dim3(static_cast<unsigned>(nb)), dim3(SBS), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SBS), 0, s, bsum, nb, total);
    if (nb > 0) hipLaunchKernelGGL(k_scan_apply, dim3(static_cast<unsigned>(nb)), dim3(SBS), 0, s, in, n, bsum, out);
    else hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, out, int64_t(1), 0);
    return launch_check("scan");
}

}  // namespace
}  // namespace pf

using namespace pf;

extern "C" {

pf_status pf_csr_create(pf_csr** out) {
    if (!out) return fail(PF_EINVAL, "pf_csr_create: null output");
    *out = new (std::nothrow) pf_csr();
    if (!*out) return fail(PF_ENOMEM, "pf_csr_create: out of host memory");
    return PF_OK;
}

void pf_csr_destroy(pf_csr* c) {
    if (!c) return;
    (void)hipFree(c->adj_ptr);
    (void)hipFree(c->adj);
    (void)hipFree(c->row_ptr);
    (void)hipFree(c->col_idx);
    (void)hipFree(c->cnt);
    (void)hipFree(c->bsum);
    (void)hipFree(c->info);
    delete c;
}

pf_status pf_csr_symbolic(pf_csr* c, int dim, int64_t nn, int64_t ne, const int32_t* elems, void* stream) {
    if (!c) return fail(PF_EINVAL, "pf_csr_symbolic: null handle");
    if (dim != 2 && dim != 3) return fail(PF_EORDER, "pf_csr_symbolic: dim must be 2 or 3");
    if (nn < 0 || ne < 0) return fail(PF_EINVAL, "pf_csr_symbolic: negative size");
    const int nlb = dim + 1;
    if (nn >= INT32_MAX || ne * nlb >= INT32_MAX || ne >= (int64_t(1) << 29))
        return fail(PF_ELIMIT, "pf_csr_symbolic: mesh too large for 32-bit indices");
    if (ne > 0 && !elems) return fail(PF_EINVAL, "pf_csr_symbolic: null elems");
    hipStream_t s = as_stream(stream);
    c->built = false;
    const int64_t m = ne * nlb;
    pf_status st;
    if ((st = grow(c->adj_ptr, c->cap_adj_ptr, nn + 1))) return st;
    if ((st = grow(c->row_ptr, c->cap_row_ptr, nn + 1))) return st;
    if ((st = grow(c->cnt, c->cap_cnt, nn + 1))) return st;
    if ((st = grow(c->adj, c->cap_adj, m))) return st;
    const int64_t nb = std::max<int64_t>(ceil_div(nn + 1, SCAN_TILE), 1);
    if ((st = grow(c->bsum, c->cap_bsum, nb))) return st;
    if ((st = grow(c->info, c->cap_info, 4))) return st;
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, s, c->info, int64_t(4), int64_t(0));
    if (nn > 0) hipLaunchKernelGGL(k_fill_i32, dim3(flat_grid(nn)), dim3(SBS), 0, s, c->cnt, nn, 0);
    if (m > 0) hipLaunchKernelGGL(k_count, dim3(flat_grid(m)), dim3(SBS), 0, s, elems, m, nn, c->cnt, c->info);
    if ((st = scan(c->cnt, nn, c->adj_ptr, c->bsum, c->info + 1, s))) return st;
    if (nn > 0) hipLaunchKernelGGL(k_fill_i32, dim3(flat_grid(nn)), dim3(SBS), 0, s, c->cnt, nn, 0);
    if (m > 0)
        hipLaunchKernelGGL(k_scatter, dim3(flat_grid(m)), dim3(SBS), 0, s, elems, m, nlb, nn, c->adj_ptr, c->cnt,
                           c->adj);
    if (nn > 0)
        hipLaunchKernelGGL(k_rows, dim3(static_cast<unsigned>(ceil_div(nn, RBS))), dim3(RBS), 0, s, nn, nlb, elems,
                           c->adj_ptr, c->adj, c->cnt, c->info);
    if ((st = scan(c->cnt, nn, c->row_ptr, c->bsum, c->info + 2, s))) return st;
    const int64_t nblk = ceil_div(nn, NBS);
    if (nblk > 0)
        hipLaunchKernelGGL(k_window_max, dim3(static_cast<unsigned>(ceil_div(nblk, 256))), dim3(256), 0, s, nn,
                           c->row_ptr, nblk, c->info);
    if ((st = launch_check("pf_csr_symbolic"))) return st;
    int64_t info[4];
    PF_HIP_TRY(hipMemcpyAsync(info, c->info, sizeof(info), hipMemcpyDeviceToHost, s));
    PF_HIP_TRY(hipStreamSynchronize(s));
    if (info[0] & ERR_INDEX) return fail(PF_EINDEX, "pf_csr_symbolic: node index out of range in elems");
    if (info[0] & ERR_ADJ) return fail(PF_ELIMIT, "pf_csr_symbolic: a node belongs to more than 64 elements");
    if (info[0] & ERR_ROW) return fail(PF_ELIMIT, "pf_csr_symbolic: a row has more than 64 nonzeros");
    if (info[2] >= INT32_MAX) return fail(PF_ELIMIT, "pf_csr_symbolic: nnz must be < 2^31");
    const int64_t nnz = info[2];
    if ((st = grow(c->col_idx, c->cap_nnz, nnz))) return st;
    if (nn > 0)
        hipLaunchKernelGGL(k_cols, dim3(static_cast<unsigned>(ceil_div(nn, RBS))), dim3(RBS), 0, s, nn, nlb, elems,
                           c->adj_ptr, c->adj, c->row_ptr, c->col_idx);
    if ((st = launch_check("pf_csr_symbolic cols"))) return st;
    c->dim = dim;
    c->nlb = nlb;
    c->nn = nn;
    c->ne = ne;
    c->nnz = nnz;
    c->max_window = static_cast<int>(info[3]);
    c->built = true;
    return PF_OK;
}

pf_status pf_csr_info(const pf_csr* c, int64_t* nn, int64_t* nnz, const int32_t** row_ptr, const int32_t** col_idx) {
    if (!c) return fail(PF_EINVAL, "pf_csr_info: null handle");
    if (!c->built) return fail(PF_ESTATE, "pf_csr_info: structure not built");
    if (nn) *nn = c->nn;
    if (nnz) *nnz = c->nnz;
    if (row_ptr) *row_ptr = c->row_ptr;
    if (col_idx) *col_idx = c->col_idx;
    return PF_OK;
}

pf_status pf_assemble(const pf_csr* c, pf_dtype prec, const double* coords, const int32_t* elems, const void* cK,
                      const void* cM, void* valsK, void* valsM, const pf_fallback* fb, int64_t* d_counters,
                      void* stream) {
    if (!c) return fail(PF_EINVAL, "pf_assemble: null handle");
    if (!c->built) return fail(PF_ESTATE, "pf_assemble: structure not built");
    if (c->nn == 0 || c->nnz == 0) return PF_OK;
    if (!coords || !elems || !valsK) return fail(PF_EINVAL, "pf_assemble: null coords, elems or valsK");
    if (prec != PF_F32 && prec != PF_F64) return fail(PF_EDTYPE, "pf_assemble: prec must be PF_F32 or PF_F64");
    hipStream_t s = as_stream(stream);
    Fallback f = make_fallback(fb);
    const size_t tsz = prec == PF_F64 ? 8 : 4;
    const size_t need = static_cast<size_t>(c->max_window) * (4 + 2 * tsz);
    const bool lds = need <= LDS_BYTES;
    const size_t shm = lds ? need : 0;
    const unsigned g = static_cast<unsigned>(ceil_div(c->nn, NBS));
#define PF_NUM(DIM, T, L)                                                                                       \
    hipLaunchKernelGGL((k_numeric<DIM, T, L>), dim3(g), dim3(NBS), shm, s, c->nn, coords, elems, c->adj_ptr,     \
                       c->adj, c->row_ptr, c->col_idx, static_cast<const T*>(cK), static_cast<const T*>(cM),     \
                       static_cast<T*>(valsK), static_cast<T*>(valsM), f, d_counters)
    if (prec == PF_F32) {
        if (c->dim == 3) { if (lds) PF_NUM(3, float, true); else PF_NUM(3, float, false); }
        else { if (lds) PF_NUM(2, float, true); else PF_NUM(2, float, false); }
    } else {
        if (c->dim == 3) { if (lds) PF_NUM(3, double, true); else PF_NUM(3, double, false); }
        else { if (lds) PF_NUM(2, double, true); else PF_NUM(2, double, false); }
    }
#undef PF_NUM
    return launch_check("pf_assemble");
}

}  // extern "C"
