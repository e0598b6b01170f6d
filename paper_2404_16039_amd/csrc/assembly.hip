// assembly.hip -- COO -> CSR assembly of the P1 stiffness and mass matrices, i.e. the
// sparse(X3D(:), Y3D(:), K3D(:), nn, nn) call of the section 3.5 listings, without ever
// materialising the 16 (row, col, value) triples per element.
//
// Symbolic phase (integer-exact, kept in a pf_csr handle):
//   1. node -> element adjacency by counting sort: per-tile LDS hash aggregation of the
//      (element, local node) entries, one global atomic per (tile, node), a scan, and a
//      scatter into reserved ranges;
//   2. row lengths: per node, the number of distinct nodes of its elements (per-lane LDS
//      hash tables, interleaved across lanes so dynamic indices stay conflict-free);
//   3. scan into row_ptr; then per node: sort the adjacency by element id, write the
//      sorted distinct neighbours (col_idx), and pack for every adjacency entry the row
//      positions ("slots") of the element's other nodes.
// Numeric phase (deterministic; see k_numeric): a block owns a contiguous range of rows,
// hence a contiguous window of the CSR arrays.  Node coordinates are staged in LDS as the
// FP64 difference vector of every window slot (column node minus row node, rounded once),
// each adjacency entry recomputes its element's row of K_e and M_e from three of those
// vectors, and every slot sums its contributions in ascending element order before one
// coalesced store.  The result is bitwise reproducible and independent of scheduling.
#include "p1elem.hpp"

#include <algorithm>
#include <new>
#include <vector>

struct pf_csr {
    int dim = 0, nlb = 0;
    int64_t nn = 0, ne = 0, nnz = 0;
    int wmax_big = 0, emax_big = 0;      // largest window / adjacency range of a 32-row block
    int wmax_small = 0, emax_small = 0;  // ... of an 8-row block
    int32_t* adj_ptr = nullptr;
    int32_t* adj = nullptr;   // (element << 2) | local index, sorted per node
    uint32_t* pk = nullptr;   // per adjacency entry: local index and slots of the other nodes
    int32_t* row_ptr = nullptr;
    int32_t* col_idx = nullptr;
    int32_t* cnt = nullptr;   // per-node counts / cursors / row lengths
    int64_t* bsum = nullptr;  // scan workspace
    int64_t* info = nullptr;  // [0] error bits, [1] adjacency total, [2] nnz, [3..6] block stats
    int64_t cap_adj_ptr = 0, cap_row_ptr = 0, cap_cnt = 0, cap_adj = 0, cap_pk = 0, cap_nnz = 0, cap_bsum = 0,
            cap_info = 0;
    bool built = false;
};

namespace pf {

constexpr int SBS = 256;         // threads per block in the flat symbolic kernels
constexpr int SCAN_ITEMS = 8;    // items per thread in the scan
constexpr int SCAN_TILE = SBS * SCAN_ITEMS;
constexpr size_t LDS_BYTES = 65536;  // dynamic LDS budget of one numeric block

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
// Node -> element adjacency by counting sort.  Each block aggregates a tile of AG_TILE
// (element, local node) entries in an LDS hash table keyed by node id, so a node that
// appears several times in the tile (neighbouring elements share nodes) costs one global
// atomic per tile instead of one per entry.
constexpr int AG_BS = 256;
constexpr int AG_ITEMS = 16;
constexpr int AG_TILE = AG_BS * AG_ITEMS;
constexpr int AG_HASH = 2 * AG_TILE;  // load factor <= 1/2, probing always ends

__device__ __forceinline__ int ag_hash(int32_t node) {
    return static_cast<int>((static_cast<uint32_t>(node) * 2654435761u) >> (32 - 13)) & (AG_HASH - 1);
}

// insert `node` (or find it) in the block's table; returns its slot
__device__ __forceinline__ int ag_insert(int32_t* keys, int32_t node) {
    int h = ag_hash(node);
    while (true) {
        const int32_t k = atomicCAS(keys + h, -1, node);
        if (k == -1 || k == node) return h;
        h = (h + 1) & (AG_HASH - 1);
    }
}

__global__ __launch_bounds__(AG_BS) void k_count(const int32_t* __restrict__ elems, int64_t m, int64_t nn,
                                                 int32_t* __restrict__ cnt, int64_t* __restrict__ info) {
    __shared__ int32_t keys[AG_HASH];
    __shared__ int32_t vals[AG_HASH];
    for (int h = threadIdx.x; h < AG_HASH; h += AG_BS) {
        keys[h] = -1;
        vals[h] = 0;
    }
    __syncthreads();
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * AG_TILE;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < AG_ITEMS; ++q) {
        const int64_t t = t0 + q * AG_BS + threadIdx.x;
        if (t < m) {
            const int32_t node = elems[t];
            if (node < 0 || node >= nn) bad = true;
            else atomicAdd(vals + ag_insert(keys, node), 1);
        }
    }
    if (bad) atomicOr(reinterpret_cast<unsigned long long*>(info), static_cast<unsigned long long>(ERR_INDEX));
    __syncthreads();
    for (int h = threadIdx.x; h < AG_HASH; h += AG_BS)
        if (keys[h] >= 0) atomicAdd(cnt + keys[h], vals[h]);
}

// Scatter (element << 2 | local index) into each node's list.  One global atomic per
// (tile, node) reserves the tile's range; entries take positions inside it through LDS
// atomics.  The order inside a list is fixed later (k_cols sorts every list).
__global__ __launch_bounds__(AG_BS) void k_scatter(const int32_t* __restrict__ elems, int64_t m, int nlb, int64_t nn,
                                                   const int32_t* __restrict__ adj_ptr, int32_t* __restrict__ cursor,
                                                   int32_t* __restrict__ adj) {
    __shared__ int32_t keys[AG_HASH];
    __shared__ int32_t vals[AG_HASH];
    for (int h = threadIdx.x; h < AG_HASH; h += AG_BS) {
        keys[h] = -1;
        vals[h] = 0;
    }
    __syncthreads();
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * AG_TILE;
    int slot[AG_ITEMS];
#pragma unroll
    for (int q = 0; q < AG_ITEMS; ++q) {
        const int64_t t = t0 + q * AG_BS + threadIdx.x;
        slot[q] = -1;
        if (t < m) {
            const int32_t node = elems[t];
            if (node >= 0 && node < nn) {
                slot[q] = ag_insert(keys, node);
                atomicAdd(vals + slot[q], 1);
            }
        }
    }
    __syncthreads();
    for (int h = threadIdx.x; h < AG_HASH; h += AG_BS) {
        const int32_t node = keys[h];
        if (node >= 0) vals[h] = adj_ptr[node] + atomicAdd(cursor + node, vals[h]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < AG_ITEMS; ++q) {
        if (slot[q] >= 0) {
            const int64_t t = t0 + q * AG_BS + threadIdx.x;
            const int64_t e = t / nlb;
            const int a = static_cast<int>(t - e * nlb);
            adj[atomicAdd(vals + slot[q], 1)] = static_cast<int32_t>((e << 2) | a);
        }
    }
}

// ---------------------------------------------------------------------------- row pattern
constexpr int RBS = 64;        // rows (= lanes) per block in the row kernels
constexpr int MAXADJ = 64;     // elements per node
constexpr int MAXROW = 64;     // nonzeros per row
constexpr int RHASH = 128;     // per-lane hash table of the distinct neighbours

// gather the node lists of up to 4 adjacency entries at once (independent loads in flight)
template <int NLB>
__device__ __forceinline__ void gather4(const int32_t* __restrict__ elems, const int32_t* __restrict__ keys, int j,
                                        int L, int (&nd)[4][4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (j + q < L) {
            const int64_t e = keys[j + q] >> 2;
            if constexpr (NLB == 4) {
                int n4[4];
                load_nodes<3>(elems, e, n4);
#pragma unroll
                for (int k = 0; k < 4; ++k) nd[q][k] = n4[k];
            } else {
                int n3[3];
                load_nodes<2>(elems, e, n3);
#pragma unroll
                for (int k = 0; k < 3; ++k) nd[q][k] = n3[k];
            }
        }
    }
}

// number of distinct neighbours of every node (row lengths), through a per-lane open-
// addressing table in LDS (interleaved across lanes, so each lane's probes hit its bank)
template <int NLB>
__global__ __launch_bounds__(RBS) void k_rows(int64_t nn, const int32_t* __restrict__ elems,
                                              const int32_t* __restrict__ adj_ptr, const int32_t* __restrict__ adj,
                                              int32_t* __restrict__ rowlen, int64_t* __restrict__ info) {
    __shared__ int32_t lds[RHASH * RBS];
    int32_t* tab = lds + threadIdx.x;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * RBS + threadIdx.x;
    if (i >= nn) return;
    const int32_t b = adj_ptr[i];
    const int L = adj_ptr[i + 1] - b;
    if (L > MAXADJ) {
        atomicOr(reinterpret_cast<unsigned long long*>(info), static_cast<unsigned long long>(ERR_ADJ));
        rowlen[i] = 0;
        return;
    }
#pragma unroll 8
    for (int h = 0; h < RHASH; ++h) tab[h * RBS] = -1;
    int n = 0;
    for (int j = 0; j < L; j += 4) {
        int nd[4][4];
        gather4<NLB>(elems, adj + b, j, L, nd);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (j + q >= L) break;
#pragma unroll
            for (int k = 0; k < NLB; ++k) {
                const int32_t v = nd[q][k];
                int h = static_cast<int>((static_cast<uint32_t>(v) * 2654435761u) >> 25);
                while (true) {
                    const int32_t cur = tab[h * RBS];
                    if (cur == v) break;
                    if (cur == -1) {
                        tab[h * RBS] = v;
                        ++n;
                        break;
                    }
                    h = (h + 1) & (RHASH - 1);
                }
            }
        }
        if (n > MAXROW) break;
    }
    if (n > MAXROW) {
        atomicOr(reinterpret_cast<unsigned long long*>(info), static_cast<unsigned long long>(ERR_ROW));
        n = 0;
    }
    rowlen[i] = n;
}

// Per node: sort its adjacency ascending by element (deterministic summation order), build
// the sorted distinct neighbour list (col_idx), and pack for every adjacency entry its local
// index a and the row positions ("slots") of the element's other nodes, in local order:
// bits 0-1 a, bits 2+8k .. 9+8k slot of the k-th other node.
template <int NLB>
__global__ __launch_bounds__(RBS) void k_cols(int64_t nn, const int32_t* __restrict__ elems,
                                              const int32_t* __restrict__ adj_ptr, int32_t* __restrict__ adj,
                                              const int32_t* __restrict__ row_ptr, int32_t* __restrict__ col_idx,
                                              uint32_t* __restrict__ pk) {
    __shared__ int32_t lds[MAXROW * RBS];
    int32_t* lst = lds + threadIdx.x;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * RBS + threadIdx.x;
    if (i >= nn) return;
    const int32_t b = adj_ptr[i];
    const int L = adj_ptr[i + 1] - b;
    // 1. insertion sort of the adjacency keys (L <= MAXADJ, checked by k_rows)
    for (int j = 0; j < L; ++j) {
        const int32_t v = adj[b + j];
        int p = j;
        while (p > 0 && lst[(p - 1) * RBS] > v) {
            lst[p * RBS] = lst[(p - 1) * RBS];
            --p;
        }
        lst[p * RBS] = v;
    }
    for (int j = 0; j < L; ++j) adj[b + j] = lst[j * RBS];
    // 2. sorted distinct neighbours (at most MAXROW, checked by k_rows)
    int n = 0;
    for (int j = 0; j < L; j += 4) {
        int nd[4][4];
        gather4<NLB>(elems, adj + b, j, L, nd);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (j + q >= L) break;
#pragma unroll
            for (int k = 0; k < NLB; ++k) {
                const int32_t v = nd[q][k];
                int p = 0;
                while (p < n && lst[p * RBS] < v) ++p;
                if (p < n && lst[p * RBS] == v) continue;
                for (int r = n; r > p; --r) lst[r * RBS] = lst[(r - 1) * RBS];
                lst[p * RBS] = v;
                ++n;
            }
        }
    }
    const int32_t o = row_ptr[i];
    for (int j = 0; j < n; ++j) col_idx[o + j] = lst[j * RBS];
    // 3. packed slots of every entry
    for (int j = 0; j < L; j += 4) {
        int nd[4][4];
        gather4<NLB>(elems, adj + b, j, L, nd);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (j + q >= L) break;
            const int a = adj[b + j + q] & 3;
            uint32_t word = static_cast<uint32_t>(a);
            int k2 = 0;
#pragma unroll
            for (int k = 0; k < NLB; ++k) {
                if (k == a) continue;
                const int32_t v = nd[q][k];
                int lo = 0, hi = n;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (lst[mid * RBS] < v) lo = mid + 1;
                    else hi = mid;
                }
                word |= static_cast<uint32_t>(lo) << (2 + 8 * k2);
                ++k2;
            }
            pk[b + j + q] = word;
        }
    }
}

// ---------------------------------------------------------------------------- numeric
constexpr int NR_BIG = 32;   // rows per block of the numeric kernel
constexpr int NR_SMALL = 8;  // ... when the big blocks' windows do not fit in LDS
constexpr int NBT = 256;     // threads per block of the numeric kernel

// largest CSR window and adjacency range of one numeric block of `nr` rows, into info[slot],
// info[slot + 1]
__global__ void k_block_stats(int64_t nn, int nr, const int32_t* __restrict__ row_ptr,
                              const int32_t* __restrict__ adj_ptr, int64_t nblk, int64_t* __restrict__ info, int slot) {
    const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (b >= nblk) return;
    const int64_t r0 = b * nr;
    const int64_t r1 = (r0 + nr < nn) ? r0 + nr : nn;
    atomicMax(reinterpret_cast<unsigned long long*>(info + slot),
              static_cast<unsigned long long>(row_ptr[r1] - row_ptr[r0]));
    atomicMax(reinterpret_cast<unsigned long long*>(info + slot + 1),
              static_cast<unsigned long long>(adj_ptr[r1] - adj_ptr[r0]));
}

template <int DIM, typename T>
constexpr size_t numeric_lds_bytes(int nr, int wmax, int emax) {
    return static_cast<size_t>(DIM * wmax + (DIM + 2) * emax) * sizeof(T) + static_cast<size_t>(emax) * 4 +
           static_cast<size_t>(2 * (nr + 1)) * 4 + static_cast<size_t>(wmax);
}

// Row of K_e and M_e for the element's node that is the origin of the edge vectors (local
// vertex 0 of the geometry): k[b] = cK |T| grad phi_0 . grad phi_b, mo = cM |T| / ((d+1)(d+2)).
template <int DIM, typename C>
__device__ __forceinline__ void origin_row(const P1Geom<DIM, C>& g, C ck, C cm, C (&k)[DIM + 1], C& mo) {
    const C adet = fabs(g.det);
    const C kf = ck / (static_cast<C>(fact_dim<DIM>()) * adet);
#pragma unroll
    for (int b = 0; b <= DIM; ++b) {
        C s = g.c[0][0] * g.c[b][0];
#pragma unroll
        for (int q = 1; q < DIM; ++q) s = fmaT(g.c[0][q], g.c[b][q], s);
        k[b] = kf * s;
    }
    mo = cm * (adet / static_cast<C>(fact_dim<DIM>())) / static_cast<C>((DIM + 1) * (DIM + 2));
}

__device__ __forceinline__ int upper_pos(const int32_t* v, int n, int32_t x) {
    // last index r in [0, n) with v[r] <= x (v ascending, v[0] <= x)
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (v[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Numeric assembly, NR rows per block:
//   phase 0  every CSR slot of the block's window gets the edge vector from its row's node to
//            its column's node (FP64 difference, rounded to T) in LDS;
//   phase 1  every adjacency entry (row node = element vertex a) computes, from three edge
//            vectors read from LDS, its element's row a of K_e and M_e (routed elements are
//            recomputed from the FP64 coordinates), into an LDS stage;
//   phase 2  every slot sums its row's stage in ascending element order and stores once.
template <int DIM, typename T, bool COEF, int NR>
__global__ __launch_bounds__(NBT) void k_numeric(int64_t nn, const double* __restrict__ coords,
                                                 const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                                                 const int32_t* __restrict__ adj_ptr, const int32_t* __restrict__ adj,
                                                 const uint32_t* __restrict__ pk, const T* __restrict__ cK,
                                                 const T* __restrict__ cM, T* __restrict__ valsK, T* __restrict__ valsM,
                                                 Fallback fb, int64_t* d_counters, int wmax, int emax) {
    constexpr int NLB = DIM + 1;
    extern __shared__ __align__(16) unsigned char smem[];
    T* f = reinterpret_cast<T*>(smem);                          // [DIM][wmax]
    T* kc = f + DIM * wmax;                                     // [emax][NLB]
    T* mo = kc + NLB * emax;                                    // [emax]
    uint32_t* pkl = reinterpret_cast<uint32_t*>(mo + emax);     // [emax]
    int32_t* rp = reinterpret_cast<int32_t*>(pkl + emax);       // [NR + 1]
    int32_t* ap = rp + (NR + 1);                                // [NR + 1]
    uint8_t* rloc = reinterpret_cast<uint8_t*>(ap + (NR + 1));  // [wmax]

    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * NR;
    const int nr = static_cast<int>((r0 + NR < nn) ? NR : nn - r0);
    if (threadIdx.x <= nr) {
        rp[threadIdx.x] = row_ptr[r0 + threadIdx.x];
        ap[threadIdx.x] = adj_ptr[r0 + threadIdx.x];
    }
    __syncthreads();
    const int32_t w0 = rp[0], e0 = ap[0];
    const int W = rp[nr] - w0, NE = ap[nr] - e0;

    // phase 0: edge vector per slot
    for (int w = threadIdx.x; w < W; w += NBT) {
        const int r = upper_pos(rp, nr, w0 + w);
        const int64_t i = r0 + r;
        const int32_t col = col_idx[w0 + w];
        rloc[w] = static_cast<uint8_t>(r | ((col == i) ? 128 : 0));
#pragma unroll
        for (int k = 0; k < DIM; ++k)
            f[k * wmax + w] = static_cast<T>(coords[static_cast<int64_t>(col) * DIM + k] - coords[i * DIM + k]);
    }
    __syncthreads();

    // phase 1: row a of every adjacent element
    int64_t routed = 0;
    for (int t = threadIdx.x; t < NE; t += NBT) {
        const int r = upper_pos(ap, nr, e0 + t);
        const int s0 = rp[r] - w0;
        const uint32_t p = pk[e0 + t];
        pkl[t] = p;
        T ck = T(1), cm = T(1);
        if constexpr (COEF) {
            const int64_t e = adj[e0 + t] >> 2;
            if (cK) ck = cK[e];
            if (cM) cm = cM[e];
        }
        T u[DIM][DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const int s = s0 + static_cast<int>((p >> (2 + 8 * k)) & 255);
#pragma unroll
            for (int q = 0; q < DIM; ++q) u[k][q] = f[q * wmax + s];
        }
        T krow[NLB], m;
        P1Geom<DIM, T> g;
        p1_geom_edges<DIM, T>(u, g);
        bool route = false;
        if constexpr (sizeof(T) == 4) route = should_route(g.det, g.absterms, fb);
        if (route) {
            // FP64 recomputation from the coordinates of the row's node and the three others
            const int64_t i = r0 + r;
            double ev[DIM][DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const int64_t col = col_idx[w0 + s0 + static_cast<int>((p >> (2 + 8 * k)) & 255)];
#pragma unroll
                for (int q = 0; q < DIM; ++q) ev[k][q] = coords[col * DIM + q] - coords[i * DIM + q];
            }
            P1Geom<DIM, double> gd;
            p1_geom<DIM, double>(ev, gd);
            double kd[NLB], md;
            origin_row<DIM, double>(gd, ck, cm, kd, md);
#pragma unroll
            for (int b = 0; b < NLB; ++b) krow[b] = static_cast<T>(kd[b]);
            m = static_cast<T>(md);
            if ((p & 3) == 0) ++routed;  // count each element once, at its first node's row
        } else {
            origin_row<DIM, T>(g, ck, cm, krow, m);
        }
#pragma unroll
        for (int b = 0; b < NLB; ++b) kc[t * NLB + b] = krow[b];
        mo[t] = m;
    }
    if (routed) count_add(d_counters, 0, routed);
    __syncthreads();

    // phase 2: one slot per thread, ascending element order, coalesced stores
    for (int w = threadIdx.x; w < W; w += NBT) {
        const int code = rloc[w];
        const int r = code & 127;
        const int s = w - (rp[r] - w0);
        const int t0 = ap[r] - e0, t1 = ap[r + 1] - e0;
        T sk = T(0), sm = T(0);
        if (code & 128) {
            for (int t = t0; t < t1; ++t) {
                sk += kc[t * NLB];
                sm += mo[t] + mo[t];
            }
        } else {
            for (int t = t0; t < t1; ++t) {
                const uint32_t p = pkl[t];
#pragma unroll
                for (int k = 0; k < DIM; ++k) {
                    if (static_cast<int>((p >> (2 + 8 * k)) & 255) == s) {
                        sk += kc[t * NLB + 1 + k];
                        sm += mo[t];
                    }
                }
            }
        }
        valsK[w0 + w] = sk;
        if (valsM) valsM[w0 + w] = sm;
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

template <int DIM, typename T, bool COEF, int NRB>
pf_status launch_numeric(const pf_csr* c, const double* coords, const void* cK, const void* cM, void* valsK,
                         void* valsM, Fallback f, int64_t* ctr, int wmax, int emax, hipStream_t s) {
    const size_t shm = numeric_lds_bytes<DIM, T>(NRB, wmax, emax);
    const unsigned g = static_cast<unsigned>(ceil_div(c->nn, NRB));
    hipLaunchKernelGGL((k_numeric<DIM, T, COEF, NRB>), dim3(g), dim3(NBT), shm, s, c->nn, coords, c->row_ptr,
                       c->col_idx, c->adj_ptr, c->adj, c->pk, static_cast<const T*>(cK), static_cast<const T*>(cM),
                       static_cast<T*>(valsK), static_cast<T*>(valsM), f, ctr, wmax, emax);
    return launch_check("pf_assemble");
}

template <int DIM, typename T>
pf_status numeric_dispatch(const pf_csr* c, const double* coords, const void* cK, const void* cM, void* valsK,
                           void* valsM, Fallback f, int64_t* ctr, hipStream_t s) {
    const bool coef = cK || cM;
    if (numeric_lds_bytes<DIM, T>(NR_BIG, c->wmax_big, c->emax_big) <= LDS_BYTES) {
        return coef ? launch_numeric<DIM, T, true, NR_BIG>(c, coords, cK, cM, valsK, valsM, f, ctr, c->wmax_big,
                                                           c->emax_big, s)
                    : launch_numeric<DIM, T, false, NR_BIG>(c, coords, cK, cM, valsK, valsM, f, ctr, c->wmax_big,
                                                            c->emax_big, s);
    }
    // 8 rows of at most MAXROW nonzeros and MAXADJ elements always fit
    return coef ? launch_numeric<DIM, T, true, NR_SMALL>(c, coords, cK, cM, valsK, valsM, f, ctr, c->wmax_small,
                                                         c->emax_small, s)
                : launch_numeric<DIM, T, false, NR_SMALL>(c, coords, cK, cM, valsK, valsM, f, ctr, c->wmax_small,
                                                          c->emax_small, s);
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
    (void)hipFree(c->pk);
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
    if ((st = grow(c->pk, c->cap_pk, m))) return st;
    const int64_t nb = std::max<int64_t>(ceil_div(nn + 1, SCAN_TILE), 1);
    if ((st = grow(c->bsum, c->cap_bsum, nb))) return st;
    if ((st = grow(c->info, c->cap_info, 8))) return st;
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, s, c->info, int64_t(8), int64_t(0));
    if (nn > 0) hipLaunchKernelGGL(k_fill_i32, dim3(flat_grid(nn)), dim3(SBS), 0, s, c->cnt, nn, 0);
    const unsigned gtile = static_cast<unsigned>(std::max<int64_t>(ceil_div(m, AG_TILE), 1));
    if (m > 0) hipLaunchKernelGGL(k_count, dim3(gtile), dim3(AG_BS), 0, s, elems, m, nn, c->cnt, c->info);
    if ((st = scan(c->cnt, nn, c->adj_ptr, c->bsum, c->info + 1, s))) return st;
    if (nn > 0) hipLaunchKernelGGL(k_fill_i32, dim3(flat_grid(nn)), dim3(SBS), 0, s, c->cnt, nn, 0);
    if (m > 0)
        hipLaunchKernelGGL(k_scatter, dim3(gtile), dim3(AG_BS), 0, s, elems, m, nlb, nn, c->adj_ptr, c->cnt, c->adj);
    const unsigned grows = static_cast<unsigned>(ceil_div(nn, RBS));
    if (nn > 0) {
        if (nlb == 4)
            hipLaunchKernelGGL(k_rows<4>, dim3(grows), dim3(RBS), 0, s, nn, elems, c->adj_ptr, c->adj, c->cnt, c->info);
        else
            hipLaunchKernelGGL(k_rows<3>, dim3(grows), dim3(RBS), 0, s, nn, elems, c->adj_ptr, c->adj, c->cnt, c->info);
    }
    if ((st = scan(c->cnt, nn, c->row_ptr, c->bsum, c->info + 2, s))) return st;
    for (int which = 0; which < 2 && nn > 0; ++which) {
        const int nr = which == 0 ? NR_BIG : NR_SMALL;
        const int64_t nblk = ceil_div(nn, nr);
        hipLaunchKernelGGL(k_block_stats, dim3(static_cast<unsigned>(ceil_div(nblk, 256))), dim3(256), 0, s, nn, nr,
                           c->row_ptr, c->adj_ptr, nblk, c->info, 3 + 2 * which);
    }
    if ((st = launch_check("pf_csr_symbolic"))) return st;
    int64_t info[8];
    PF_HIP_TRY(hipMemcpyAsync(info, c->info, sizeof(info), hipMemcpyDeviceToHost, s));
    PF_HIP_TRY(hipStreamSynchronize(s));
    if (info[0] & ERR_INDEX) return fail(PF_EINDEX, "pf_csr_symbolic: node index out of range in elems");
    if (info[0] & ERR_ADJ) return fail(PF_ELIMIT, "pf_csr_symbolic: a node belongs to more than 64 elements");
    if (info[0] & ERR_ROW) return fail(PF_ELIMIT, "pf_csr_symbolic: a row has more than 64 nonzeros");
    if (info[2] >= INT32_MAX) return fail(PF_ELIMIT, "pf_csr_symbolic: nnz must be < 2^31");
    const int64_t nnz = info[2];
    if ((st = grow(c->col_idx, c->cap_nnz, nnz))) return st;
    if (nn > 0) {
        if (nlb == 4)
            hipLaunchKernelGGL(k_cols<4>, dim3(grows), dim3(RBS), 0, s, nn, elems, c->adj_ptr, c->adj, c->row_ptr,
                               c->col_idx, c->pk);
        else
            hipLaunchKernelGGL(k_cols<3>, dim3(grows), dim3(RBS), 0, s, nn, elems, c->adj_ptr, c->adj, c->row_ptr,
                               c->col_idx, c->pk);
    }
    if ((st = launch_check("pf_csr_symbolic cols"))) return st;
    c->dim = dim;
    c->nlb = nlb;
    c->nn = nn;
    c->ne = ne;
    c->nnz = nnz;
    c->wmax_big = static_cast<int>(info[3]);
    c->emax_big = static_cast<int>(info[4]);
    c->wmax_small = static_cast<int>(info[5]);
    c->emax_small = static_cast<int>(info[6]);
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
    if (!coords || !valsK) return fail(PF_EINVAL, "pf_assemble: null coords or valsK");
    (void)elems;  // the structure carries the connectivity it was built from
    if (prec != PF_F32 && prec != PF_F64) return fail(PF_EDTYPE, "pf_assemble: prec must be PF_F32 or PF_F64");
    hipStream_t s = as_stream(stream);
    Fallback f = make_fallback(fb);
    if (prec == PF_F32)
        return c->dim == 3 ? numeric_dispatch<3, float>(c, coords, cK, cM, valsK, valsM, f, d_counters, s)
                           : numeric_dispatch<2, float>(c, coords, cK, cM, valsK, valsM, f, d_counters, s);
    return c->dim == 3 ? numeric_dispatch<3, double>(c, coords, cK, cM, valsK, valsM, f, d_counters, s)
                       : numeric_dispatch<2, double>(c, coords, cK, cM, valsK, valsM, f, d_counters, s);
}

}  // extern "C"
