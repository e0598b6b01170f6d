// assembly.hip -- COO -> CSR assembly of the P1 stiffness and mass matrices, i.e. the
// sparse(X3D(:), Y3D(:), K3D(:), nn, nn) call of the section 3.6 listings, without ever
// materialising the 16 (row, col, value) triples per element.
//
// Symbolic phase (integer-exact, kept in a pf_csr handle):
//   1. node -> element adjacency in a padded layout (MAXADJ entries per node): per-tile LDS
//      hash aggregation of the (element, local node) entries, one global atomic per
//      (tile, node) reserving positions in the node's row, LDS atomics inside the tile;
//   2. row patterns, one pass per block of rows: the distinct (row, node) pairs of its
//      elements in per-row LDS hash tables, each row's nodes ranked (ascending) into a
//      padded buffer, the row lengths, and for every adjacency entry the row positions
//      ("slots") of the element's other nodes;
//   3. scan of the row lengths into row_ptr, then the padded rows are moved into col_idx.
// Numeric phase (deterministic; see k_numeric): a block owns a contiguous range of rows,
// hence a contiguous window of the CSR arrays.  Node coordinates are staged in LDS as the
// FP64 difference vector of every window slot (column node minus row node, rounded once),
// each adjacency entry recomputes its element's row of K_e and M_e from three of those
// vectors, and the contributions are summed exactly (rounded onto a fixed grid first), so
// the result is bitwise reproducible whatever the order of the atomic adds.
#include "p1elem.hpp"
#include "internal.hpp"
#include "quadrature.hpp"
#include "exact.hpp"

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <new>
#include <vector>

struct pf_csr {
    int dim = 0, nlb = 0;
    int64_t nn = 0, ne = 0, nnz = 0;
    int wmax_big = 0;    // largest CSR window of a numeric block of NR_BIG rows
    int wmax_mid = 0;    // ... of NR_MID rows
    int wmax_small = 0;  // ... of NR_SMALL rows
    int wmax8 = 0;       // ... of 8 rows
    int wmax2 = 0;       // ... of 2 rows
    int max_adj = 0;     // largest number of elements around one node
    // resident: the CSR pattern, the node -> element adjacency in CSR form (node i's entries
    // at aptr[i] .. aptr[i+1]) with the packed slot words of every entry, the diagonal positions
    int32_t* aptr = nullptr;  // adjacency offsets (nn + 1)
    int32_t* adj = nullptr;   // entries (element << 2 | local index; P2: << 4), ne * nlb of them
    uint32_t* pk = nullptr;   // per adjacency entry: local index, slots of the other nodes
    uint64_t* pk2 = nullptr;  // P2 structures: row positions of the other nodes, 7 bits each
    int32_t* row_ptr = nullptr;
    int32_t* col_idx = nullptr;  // exactly nnz words
    // build scratch: one block (one pool allocation, one release when the build ends) holding
    int32_t* adj_len = nullptr;  // elements around each node (scatter cursors)
    int32_t* adj_pad = nullptr;  // node i's entries at i * MAXADJ ... (scatter output)
    int32_t* cnt = nullptr;      // row lengths
    int32_t* colblk = nullptr;   // sorted columns of every row-pattern block, RR * MAXROW per block
    uint64_t* look = nullptr;    // published counts / prefixes of the row-offset tiles
    int32_t* lrows_s = nullptr;  // the long rows found by the row-block pass
    unsigned char* scratch = nullptr;
    bool scratch_owned = false;  // a block of its own, not the device's scratch arena
    int32_t* lcol = nullptr;     // each long row's columns, LCAP words apiece (long-row phase)
    int64_t cap_lcol = 0;
    // long rows (more than MAXADJ elements or MAXROW nonzeros): their list (resident)
    int64_t nlong = 0;
    int32_t* lrows = nullptr;
    int64_t cap_lrows = 0;
    uint8_t* pk9 = nullptr;  // P2 long rows of 10-node elements: each entry's ninth position
    int64_t cap_pk9 = 0;
    bool p2 = false;            // built from P2 elements (pf_csr_symbolic_p2)
    int64_t* bsum = nullptr;  // scan workspace
    int64_t* info = nullptr;  // [0] error bits, [1] adjacency total, [2] nnz, [3..6] block stats
    // routed-element count of each FP32 numeric block (P1; one int per 4 rows at most), summed
    // into the caller's counter after the launch: calls on one structure whose numeric phases
    // overlap in time share it, so their routed counts may mix (their values do not)
    int32_t* bcnt = nullptr;
    void* work = nullptr;     // workspace of the energy reductions (pf_energies)
    // faces (pf_csr_faces): per-row counts and their scans, the lists, and the totals
    int32_t* dpos = nullptr;   // column position of each row's diagonal
    uint8_t* esign = nullptr;  // orientation of every element (1: det J < 0)
    int32_t *fcount = nullptr, *bcount = nullptr, *fptr = nullptr, *bptr = nullptr;
    int32_t *faces = nullptr, *fel = nullptr, *bfaces = nullptr, *bel = nullptr;
    int64_t* finfo = nullptr;  // [0] error bits, [1] faces, [2] boundary faces
    int64_t nf = 0, nfb = 0;
    bool faces_built = false;
    int64_t cap_fcount = 0, cap_bcount = 0, cap_fptr = 0, cap_bptr = 0, cap_faces = 0, cap_fel = 0,
            cap_bfaces = 0, cap_bel = 0, cap_finfo = 0, cap_esign = 0;
    // the resident arrays sized before the pattern (aptr, row_ptr, dpos, adj, pk or pk2, bsum,
    // info) share one block (one pool allocation); col_idx, sized by nnz, is its own
    unsigned char* res = nullptr;
    int64_t cap_res = 0, cap_nnz = 0, cap_work = 0, cap_scratch = 0;
    bool built = false;
    // per-stage timing of pf_csr_symbolic (events e0..e3: start, after the adjacency, after
    // the pattern, after the row offsets)
    bool timing = false, pending = false;
    int64_t* hinfo = nullptr;  // pinned host words for the status readbacks (allocated once)
    hipEvent_t ready = nullptr;  // recorded at the end of each enqueued build phase
    int stage = 0;               // 0 idle, 1 pattern phase enqueued, 3 long-row phase, 2 columns
    // pf_csr_symbolic returned with the column phase enqueued on q_stream and not yet seen
    // complete: work on another stream first waits for the ready event
    mutable bool cols_pending = false;
    int q_dim = 0, q_nlb = 0;    // ... the build's shape and stream
    int64_t q_nn = 0, q_ne = 0;
    hipStream_t q_stream = nullptr;
    const int32_t* q_elems = nullptr;
    bool q_long = false;  // the long-row phase has run for this build
    bool q_cols = false;  // phase 1 moved the columns into the col_idx kept from a former build
    hipEvent_t ev[PF_CSR_STAGES + 2] = {};  // stage k: ev[STAGE_EV[k][0]] .. ev[STAGE_EV[k][1]]
    double stage_ms[PF_CSR_STAGES] = {};
    int64_t stage_calls = 0;
};

namespace pf {

constexpr int SBS = 256;         // threads per block in the flat symbolic kernels
constexpr int SCAN_ITEMS = 8;    // items per thread in the scan
constexpr int SCAN_TILE = SBS * SCAN_ITEMS;
constexpr size_t LDS_BYTES = 65536;  // dynamic LDS budget of one numeric block

constexpr int64_t ERR_INDEX = 1, ERR_ROW = 4;
constexpr int INFO_WORDS = 16;  // status and statistics words of a symbolic build
constexpr int INFO_NLONG = 10;  // ... the number of long rows
// Long rows: a P1 row whose node lies in more than MAXADJ elements or that holds more than
// MAXROW nonzeros.  The row-block kernels skip them; kernels of one workgroup per long row
// build and assemble them.  A long row holds at most LCAP nonzeros (the packed slot words
// give a column position 8 bits).
constexpr int LCAP = 256;
constexpr int MAXADJ = 64;  // elements per node (adjacency rows are padded to this length)
constexpr int MAXROW = 64;  // nonzeros per row

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
// atomic per tile instead of one per entry.  The table uses linear probing with one
// compare-and-swap per probe; the first probes of all of a lane's entries are issued
// together.
#ifndef PF_SCATTER_BS
#define PF_SCATTER_BS 256
#endif
#ifndef PF_SCATTER_ITEMS
#define PF_SCATTER_ITEMS 4
#endif
constexpr int AG_BS = PF_SCATTER_BS;
constexpr int AG_ITEMS = PF_SCATTER_ITEMS;
constexpr int AG_TILE = AG_BS * AG_ITEMS;
constexpr int AG_HASH = 2 * AG_TILE;  // load factor <= 1/2, probing always ends
constexpr int AG_BITS = AG_HASH == 1024 ? 10 : AG_HASH == 2048 ? 11 : AG_HASH == 4096 ? 12 : AG_HASH == 8192 ? 13 : 0;
static_assert(AG_BITS > 0, "the scatter table holds 1024..8192 slots");

__device__ __forceinline__ int ag_hash(int32_t node) {
    return static_cast<int>((static_cast<uint32_t>(node) * 2654435761u) >> (32 - AG_BITS));
}

// Scatter (element << 2 | local index) into each node's padded row (MAXADJ entries).  One
// global atomic per (tile, node) on the node's length reserves the tile's positions; entries
// take positions inside them through LDS atomics.  The first inserter of a node lists its
// table slot, so the block issues the global atomics of all its distinct nodes at once (one
// round trip) instead of sweeping the table.  The order inside a row is not fixed: nothing
// downstream depends on it (the numeric phase sums exactly, so its result does not depend
// on the entry order).  Out-of-range node ids set an error bit and are not stored; entries
// beyond MAXADJ are not stored either (the node's row is a long row, whose entries the
// long-row phase places again), while the length counts them all.
template <int ASH>  // bits of the local index in an adjacency entry: 2 (P1), 4 (P2)
__global__ __launch_bounds__(AG_BS) void k_scatter(const int32_t* __restrict__ elems, int64_t m, int nlb, int64_t nn,
                                                   int32_t* __restrict__ adj_len, int32_t* __restrict__ adj,
                                                   int64_t* __restrict__ info) {
    __shared__ int32_t keys[AG_HASH];
    __shared__ int32_t vals[AG_HASH];
    __shared__ int16_t uniq[AG_TILE];  // table slots of the tile's distinct nodes (16 bits: LDS
                                       // under 20 KB, eight resident blocks per CU)
    static_assert(AG_HASH <= 32768, "table slots fit 16 bits");
    __shared__ int32_t nuniq;
    __shared__ int32_t guard[AG_BS];  // never -1: the first probes of empty entries
    const int64_t t0 = static_cast<int64_t>(blockIdx.x) * AG_TILE;
    int slot[AG_ITEMS];
    int32_t node[AG_ITEMS], cur[AG_ITEMS];
    bool bad = false;
#pragma unroll
    for (int q = 0; q < AG_ITEMS; ++q) {  // all loads in flight together, while the table is cleared
        const int64_t t = t0 + q * AG_BS + threadIdx.x;
        node[q] = elems[t < m ? t : m - 1];
    }
    for (int h = threadIdx.x; h < AG_HASH; h += AG_BS) {
        keys[h] = -1;
        vals[h] = 0;
    }
    guard[threadIdx.x] = -2;
    if (threadIdx.x == 0) nuniq = 0;
    __syncthreads();
    // first probes of all the lane's entries together; an entry outside the tile or with a
    // bad node id probes the lane's guard word (never -1, so nothing is stored)
#pragma unroll
    for (int q = 0; q < AG_ITEMS; ++q) {
        const int64_t t = t0 + q * AG_BS + threadIdx.x;
        const bool ok = t < m && node[q] >= 0 && node[q] < nn;
        bad = bad || (t < m && !ok);
        slot[q] = ok ? ag_hash(node[q]) : -1;
        cur[q] = atomicCAS(ok ? keys + slot[q] : guard + threadIdx.x, -1, node[q]);
    }
#pragma unroll
    for (int q = 0; q < AG_ITEMS; ++q) {
        if (slot[q] < 0) continue;
        int h = slot[q];
        int32_t c = cur[q];
        while (c != -1 && c != node[q]) {  // taken: linear probing (the table is at most half full)
            h = (h + 1) & (AG_HASH - 1);
            c = atomicCAS(keys + h, -1, node[q]);
        }
        slot[q] = h;
        if (c == -1) uniq[atomicAdd(&nuniq, 1)] = static_cast<int16_t>(h);
        atomicAdd(vals + h, 1);
    }
    if (bad) atomicOr(reinterpret_cast<unsigned long long*>(info), static_cast<unsigned long long>(ERR_INDEX));
    __syncthreads();
    const int nu = nuniq;
    int old[AG_ITEMS];
#pragma unroll
    for (int q = 0; q < AG_ITEMS; ++q) {  // independent atomics, all in flight together
        const int u = threadIdx.x + q * AG_BS;
        old[q] = 0;
        if (u < nu) {
            const int h = uniq[u];
            old[q] = atomicAdd(adj_len + keys[h], vals[h]);
        }
    }
#pragma unroll
    for (int q = 0; q < AG_ITEMS; ++q) {
        const int u = threadIdx.x + q * AG_BS;
        if (u < nu) vals[uniq[u]] = old[q];  // the tile's first position in the node's row
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < AG_ITEMS; ++q) {
        if (slot[q] >= 0) {
            const int64_t t = t0 + q * AG_BS + threadIdx.x;
            const int64_t e = nlb == 4 ? (t >> 2)
                                       : static_cast<int64_t>(static_cast<uint32_t>(t) / static_cast<uint32_t>(nlb));
            const int a = static_cast<int>(t - e * nlb);
            const int64_t node = keys[slot[q]];
            const int off = atomicAdd(vals + slot[q], 1);
            if (off < MAXADJ) adj[node * MAXADJ + off] = static_cast<int32_t>((e << ASH) | a);
        }
    }
}

// ---------------------------------------------------------------------------- row pattern
// Row patterns are built block-cooperatively: a block of RR rows inserts the nodes of all
// its adjacency entries into per-row open-addressing tables in LDS (linear probing, one
// compare-and-swap per probe, which returns the slot's node whether or not it stored the
// new one; the first probes of all of a lane's inserts are issued together); the first
// inserter of a node appends it to its row's list.  Lists are then ranked (sorted) in parallel and the
// ranks give both col_idx and, for every adjacency entry, the row positions ("slots") of the
// element's other nodes.  Entries are dealt to lanes row-interleaved (entry j of row r is
// item r + nr j), so the lanes of one instruction insert into different rows' tables.
#ifndef PF_PATTERN_RR
#define PF_PATTERN_RR 8
#endif
#ifndef PF_PATTERN_RT
#define PF_PATTERN_RT 128
#endif
constexpr int RR = PF_PATTERN_RR;  // rows per block in the row-pattern kernels
constexpr int RT = PF_PATTERN_RT;  // threads per block
constexpr int RSUB = MAXROW;     // slots of one row's table: every admissible row fits
static_assert(RR <= 64, "the row-count prefix runs in one wave");
static_assert(RT >= RR && RT >= 64, "one thread per row and a full first wave");

__device__ __forceinline__ int rsub_hash(int32_t v) {
    return static_cast<int>((static_cast<uint32_t>(v) * 2654435761u) >> 26);  // 6 bits
}
static_assert(RSUB == 64, "rsub_hash yields 6 bits");

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

// ---------------------------------------------------------------------------- P2 row pattern
// The same block-cooperative pattern for P2 meshes (6 or 10 nodes per element): rows hold up
// to MAXROW2 nonzeros (a vertex of the Kuhn cube's P2 mesh has 65), and every adjacency
// entry (element << 4 | local index a) gets pk2 = the row positions of the element's other
// nodes in local order, 7 bits each (9 x 7 = 63 bits).  A block takes RR2 = 16 rows and 1024
// table words: when every one of its rows can hold at most 64 nonzeros (1 + (NLB - 1) x its
// number of elements, which covers the mid-edge rows of a P2 mesh), all 16 rows go in one
// pass with 64-slot tables; otherwise in two passes of 8 rows with 128-slot tables.  Either
// way the sorted columns of rows 8k .. 8k+7 go to the region of RR * MAXROW2 words of
// colblk that the row offsets expect for that 8-row group.
constexpr int MAXROW2 = 128;
constexpr int RT2 = 128;
constexpr int RR2 = 2 * RR;          // rows of a P2 pattern block
constexpr int TAB2 = RR * MAXROW2;  // table (and list) words of a block: 16 x 64 or 8 x 128
static_assert(RT2 >= RR2 && RT2 >= 64 && RR2 <= 64, "one thread per row, one wave for the row prefix");
static_assert(RR2 * 64 == TAB2, "the two table layouts of a block take the same LDS");

template <int TS>
__device__ __forceinline__ int tsub_hash(int32_t v) {
    static_assert(TS == 64 || TS == 128, "6- or 7-bit table slots");
    return static_cast<int>((static_cast<uint32_t>(v) * 2654435761u) >> (TS == 64 ? 26 : 25));
}

struct P2Pattern {                  // LDS of a P2 pattern block
    alignas(16) int32_t tab[TAB2];  // node ids, -1 empty; then each row's nodes, compacted
    uint8_t seg_h[TAB2];            // table slot of each compacted node
    uint8_t slot_rank[TAB2];        // rank (column position) of each used table slot
    int32_t cnt[RR2];
    int32_t cpre[RR2 + 1];
    int32_t maxl;
};

// One pass over NRW rows (nrw of them in the matrix) starting at row rq, with TS-slot tables,
// one adjacency entry per thread at a time.  alen: the rows' numbers of elements (0 for a
// long row), abase: their first compact adjacency entries, rlong: their long-row flags (all
// LDS; a row whose table fills becomes long); dst: the colblk region of the pass's first 8
// rows (rows 8 .. 15 of a 16-row pass go to the next region); apre: this thread's entry of
// the first batch (item r + NRW j, j = thread / NRW), read at block start, used when `pre`.
// Every entry of a row kept here is copied to its compact place, with its pk2 word; a long
// row gets no columns, diagonal position -1, and joins the list of long rows.
template <int NLB, int NRW, int TS>
__device__ __forceinline__ void p2_pattern_pass(P2Pattern& S, const int32_t* alen, const int32_t* abase,
                                                int32_t* rlong, int64_t rq, int nrw, const int32_t* __restrict__ elems,
                                                const int32_t* __restrict__ adj, int32_t* __restrict__ rowlen,
                                                int32_t* __restrict__ dst, int32_t* __restrict__ adjc,
                                                uint64_t* __restrict__ pk2, int32_t* __restrict__ dpos,
                                                int32_t* __restrict__ lrows, int64_t* __restrict__ info, int32_t apre,
                                                bool pre) {
    constexpr int NO = NLB - 1;
    static_assert(NO * 7 <= 64, "the positions of the other nodes fit one 64-bit word");
    static_assert(NRW * TS == TAB2, "a pass fills the block's tables");
    static_assert((NRW & (NRW - 1)) == 0, "NRW is a power of two");
    const int64_t e0 = rq * MAXADJ;
    for (int h = threadIdx.x; h < TAB2; h += RT2) S.tab[h] = -1;
    if (threadIdx.x == 0) S.maxl = 0;
    __syncthreads();
    if (threadIdx.x < NRW) {
        const int r = threadIdx.x;
        const int L = r < nrw ? alen[r] : 0;
        if (r < nrw && L == 0 && !rlong[r]) dpos[rq + r] = 0;  // a node of no element has an empty row
        if (L > 0) {                              // the diagonal
            const int32_t self = static_cast<int32_t>(rq + r);
            S.tab[r * TS + tsub_hash<TS>(self)] = self;
            atomicMax(&S.maxl, L);
        }
    }
    __syncthreads();
    const int items = NRW * S.maxl;
    // items per thread: a one-pass row has at most 63 / NO elements, a two-pass row MAXADJ
    constexpr int ITMAX = (NRW * (NRW == RR2 ? 63 / NO : MAXADJ) + RT2 - 1) / RT2;
    // element node ids in 8-byte loads (NLB even: an element's ids start 8-byte aligned)
    static_assert(NLB % 2 == 0, "P2 elements have 6 or 10 nodes");
    const bool al8 = (reinterpret_cast<uintptr_t>(elems) & 7) == 0;
    uint64_t eslot[ITMAX];  // per item of this thread: table slot of other node k << 7k
#pragma unroll
    for (int it = 0; it < ITMAX; ++it) {
        const int idx = static_cast<int>(threadIdx.x) + it * RT2;
        eslot[it] = 0;
        if (idx >= items) break;
        const int r = idx % NRW, j = idx / NRW;
        const bool ok = j < alen[r] && r < nrw;
        const int32_t w = pre && it == 0 ? apre : adj[e0 + (ok ? r * MAXADJ + j : 0)];
        if (!ok) continue;
        adjc[abase[r] + j] = w;
        const int a = w & 15;
        const int64_t e = static_cast<uint32_t>(w) >> 4;
        int32_t nd[NLB];
        if (al8) {
            const int2* pe = reinterpret_cast<const int2*>(elems + e * NLB);
#pragma unroll
            for (int k = 0; k < NLB / 2; ++k) {
                const int2 v = pe[k];
                nd[2 * k] = v.x;
                nd[2 * k + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int k = 0; k < NLB; ++k) nd[k] = elems[e * NLB + k];
        }
        // the other nodes' first probes together, then every probe that met another node
        // retried together (one LDS round trip per probe depth, not per node)
        int32_t* rt = S.tab + r * TS;
        int32_t ov[NO];
        int hq[NO];
        uint32_t pend = 0;
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            ov[k] = k < a ? nd[k] : nd[k + 1];
            hq[k] = tsub_hash<TS>(ov[k]);
            const int32_t cur = atomicCAS(rt + hq[k], -1, ov[k]);
            pend |= static_cast<uint32_t>(cur != -1 && cur != ov[k]) << k;
        }
        for (int probe = 1; pend != 0u; ++probe) {  // linear probing
            if (probe == TS) {                      // a full table: a long row
                rlong[r] = 1;
                break;
            }
#pragma unroll
            for (int k = 0; k < NO; ++k) {
                if ((pend >> k) & 1u) {
                    hq[k] = (hq[k] + 1) & (TS - 1);
                    const int32_t cur = atomicCAS(rt + hq[k], -1, ov[k]);
                    if (cur == -1 || cur == ov[k]) pend &= ~(1u << k);
                }
            }
        }
        uint64_t word = 0;
#pragma unroll
        for (int k = 0; k < NO; ++k) word |= static_cast<uint64_t>(hq[k]) << (7 * k);
        eslot[it] = word;
    }
    __syncthreads();
    // each row's list: its used table slots, compacted in place (one wave per row, lane = slot
    // of each 64; a wave reads its 64 slots before it writes, and writes only below them)
    for (int r = threadIdx.x >> 6; r < NRW; r += RT2 / 64) {
        const int lane = threadIdx.x & 63;
        if (rlong[r]) {  // the same for the wave: no columns here
            if (lane == 0) S.cnt[r] = 0;
            continue;
        }
        int n = 0;
#pragma unroll
        for (int half = 0; half < TS / 64; ++half) {
            const int32_t v = S.tab[r * TS + 64 * half + lane];
            const unsigned long long m = __ballot(v != -1);
            const int below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                                        __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
            if (v != -1) {
                S.tab[r * TS + n + below] = v;
                S.seg_h[r * TS + n + below] = static_cast<uint8_t>(64 * half + lane);
            }
            n += __popcll(m);
        }
        if (lane == 0) S.cnt[r] = n;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int v = lane < nrw ? S.cnt[lane] : 0;
        int x = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane < nrw) S.cpre[lane] = x - v;
        if (lane == nrw - 1) S.cpre[nrw] = x;
    }
    if (static_cast<int>(threadIdx.x) < nrw) {
        rowlen[rq + threadIdx.x] = S.cnt[threadIdx.x];
        if (rlong[threadIdx.x]) {
            dpos[rq + threadIdx.x] = -1;
            lrows[atomicAdd(reinterpret_cast<unsigned long long*>(info + INFO_NLONG), 1ull)] =
                static_cast<int32_t>(rq + threadIdx.x);
        }
    }
    __syncthreads();
    // each node's rank in its row = its column position; the sorted columns go straight to
    // their region (a wave's stores cover a contiguous run of it): rows 0 .. 7 of the pass to
    // the first region, rows 8 .. 15 (a 16-row pass) to the next
    const int split = NRW > RR && nrw > RR ? S.cpre[RR] : S.cpre[nrw];
    for (int q = threadIdx.x; q < S.cpre[nrw]; q += RT2) {
        const int r = upper_pos(S.cpre, nrw, q);
        const int p = q - S.cpre[r];
        const int n = S.cnt[r];
        const int32_t* sr = S.tab + r * TS;
        const int32_t v = sr[p];
        int rank = 0;
        int j = 0;
        for (; j + 4 <= n; j += 4) {
            const int32_t a0 = sr[j], a1 = sr[j + 1], a2 = sr[j + 2], a3 = sr[j + 3];
            rank += (a0 < v) + (a1 < v) + (a2 < v) + (a3 < v);
        }
        for (; j < n; ++j) rank += sr[j] < v;
        S.slot_rank[r * TS + S.seg_h[r * TS + p]] = static_cast<uint8_t>(rank);
        if (v == rq + r) dpos[rq + r] = rank;
        const int pos = S.cpre[r] + rank;
        dst[pos < split ? pos : RR * MAXROW2 + (pos - split)] = v;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < ITMAX; ++it) {
        const int idx = static_cast<int>(threadIdx.x) + it * RT2;
        if (idx >= items) break;
        const int r = idx % NRW, j = idx / NRW;
        if (r >= nrw || j >= alen[r] || rlong[r]) continue;
        const uint64_t w = eslot[it];
        uint64_t word = 0;
#pragma unroll
        for (int k = 0; k < NO; ++k)
            word |= static_cast<uint64_t>(S.slot_rank[r * TS + static_cast<int>((w >> (7 * k)) & 127)]) << (7 * k);
        pk2[abase[r] + j] = word;
    }
    __syncthreads();  // the LDS is free for the next pass
}

template <int NLB>
__global__ __launch_bounds__(RT2) void k_pattern_p2(int64_t nn, const int32_t* __restrict__ elems,
                                                   const int32_t* __restrict__ adj_len, const int32_t* __restrict__ adj,
                                                   const int32_t* __restrict__ aptr, int32_t* __restrict__ rowlen,
                                                   int32_t* __restrict__ colblk, int32_t* __restrict__ adjc,
                                                   uint64_t* __restrict__ pk2, int32_t* __restrict__ dpos,
                                                   int32_t* __restrict__ lrows, int64_t* __restrict__ info) {
    constexpr int NO = NLB - 1;
    __shared__ P2Pattern S;
    __shared__ int32_t alen[RR2];
    __shared__ int32_t abase[RR2];
    __shared__ int32_t rlong[RR2];
    __shared__ int32_t longrows;
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * RR2;
    const int nr = static_cast<int>((r0 + RR2 < nn) ? RR2 : nn - r0);
    // the first batch of entries of the one-pass layout (item r + RR2 j) is read together with
    // the row lengths (padded rows: every entry below MAXADJ of a row of the matrix is in
    // bounds; entries past a row's length are dropped once the lengths are known)
    static_assert(RT2 / RR2 <= MAXADJ, "the first batch lies inside the padded rows");
    int32_t apre;
    {
        const int r = static_cast<int>(threadIdx.x) % RR2, j = static_cast<int>(threadIdx.x) / RR2;
        apre = adj[(r0 + (r < nr ? r : 0)) * MAXADJ + j];
    }
    const int32_t lv = adj_len[r0 + (static_cast<int>(threadIdx.x) < nr ? threadIdx.x : 0)];
    const int32_t av = aptr[r0 + (static_cast<int>(threadIdx.x) < nr ? threadIdx.x : 0)];
    if (threadIdx.x < 64) {  // row lengths, and whether a row may hold more than 64 nonzeros (wave 0)
        // a node of more than MAXADJ elements heads a long row: left to the long-row phase
        const bool lng = static_cast<int>(threadIdx.x) < nr && lv > MAXADJ;
        const int L = static_cast<int>(threadIdx.x) < nr && !lng ? lv : 0;
        if (threadIdx.x < RR2) {
            alen[threadIdx.x] = L;
            abase[threadIdx.x] = av;
            rlong[threadIdx.x] = lng;
        }
        const unsigned long long lg = __ballot(1 + NO * L > 64);
        if (threadIdx.x == 0) longrows = lg != 0ull;
    }
    __syncthreads();
    int32_t* dst = colblk + (static_cast<int64_t>(blockIdx.x) * 2) * (RR * MAXROW2);
    if (!longrows) {
        p2_pattern_pass<NLB, RR2, 64>(S, alen, abase, rlong, r0, nr, elems, adj, rowlen, dst, adjc, pk2, dpos, lrows,
                                      info, apre, true);
    } else {
        p2_pattern_pass<NLB, RR, MAXROW2>(S, alen, abase, rlong, r0, min(nr, RR), elems, adj, rowlen, dst, adjc, pk2,
                                          dpos, lrows, info, apre, false);
        if (nr > RR)
            p2_pattern_pass<NLB, RR, MAXROW2>(S, alen + RR, abase + RR, rlong + RR, r0 + RR, nr - RR, elems, adj,
                                              rowlen, dst + RR * MAXROW2, adjc, pk2, dpos, lrows, info, apre, false);
    }
}

// ---------------------------------------------------------------------------- row offsets
// row_ptr, nnz and the numeric launch statistics in one pass over tiles of SCAN_TILE rows (a
// single-pass scan with decoupled look-back); the columns follow once col_idx is allocated
// for exactly nnz words (k_row_columns).  Tile t publishes its nonzero count
// as soon as it has summed its row lengths (status AGG), then sums the published values of
// the tiles before it, nearest first, 64 at a time, until it meets one holding its
// inclusive prefix (status INC), and publishes its own.  A tile waits only for tiles of
// smaller index to publish their counts, which they do before waiting on anyone; every
// wait is bounded (LB_SPIN polls) and a wait that runs out sets ERR_SCAN.
constexpr uint64_t LB_AGG = uint64_t(1) << 62, LB_INC = uint64_t(2) << 62, LB_VAL = LB_AGG - 1;
constexpr int LB_SPIN = 1 << 13;
constexpr int64_t ERR_SCAN = 16;

__device__ __forceinline__ void lb_publish(uint64_t* look, int64_t t, uint64_t word) {
    __hip_atomic_store(look + t, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// exclusive prefix of tile t (> 0) over the published counts; run by one full wave
__device__ int64_t lb_exclusive(const uint64_t* look, int64_t t, bool& timeout) {
    const int lane = threadIdx.x & 63;
    int64_t excl = 0;
    for (int64_t end = t;; end -= 64) {  // tiles end-1-lane, lane 0 the nearest
        const int64_t j = end - 1 - lane;
        uint64_t d = LB_INC;  // before tile 0: an inclusive prefix of zero
        if (j >= 0) {
            d = __hip_atomic_load(look + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int spin = 0; (d >> 62) == 0; ++spin) {
                if (spin >= LB_SPIN) {
                    timeout = true;
                    d = LB_INC;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
                d = __hip_atomic_load(look + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        const unsigned long long inc = __ballot((d >> 62) == 2);
        const int first = inc ? __ffsll(static_cast<long long>(inc)) - 1 : 64;  // the nearest inclusive prefix
        int64_t v = lane <= first ? static_cast<int64_t>(d & LB_VAL) : 0;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        excl += v;
        if (inc) return excl;
    }
}

// Thread i of a tile holds rows 8i .. 8i+7, one 8-row group (a P1 row-pattern block, or half
// of a P2 one: a row-pattern block below).  Besides the offsets, the tile measures the largest
// CSR window of the numeric block classes (NR_BIG rows, NR_MID rows as sums over 4 and 2
// neighbouring lanes, NR_SMALL = 4 rows per half thread) and the largest number of elements
// around a node, and stores them as tstat[8t .. 8t+7] (no atomics on shared words: those
// serialise across the whole device); k_row_stats reduces them.
static_assert(SCAN_ITEMS == RR && SCAN_ITEMS == 8, "a scan thread owns one row-pattern block of 8 rows");
constexpr int TSTAT = 8;  // int32 statistics per tile (two 16-byte words)

__global__ __launch_bounds__(SBS) void k_row_offsets(int64_t nn, const int32_t* __restrict__ rowlen,
                                                     const int32_t* __restrict__ adj_len, int32_t* __restrict__ row_ptr,
                                                     uint64_t* __restrict__ look, int32_t* __restrict__ tstat,
                                                     int64_t* __restrict__ info) {
    __shared__ int red[TSTAT][SBS / 64];
    __shared__ int64_t excl_s;
    const int64_t t = blockIdx.x;
    const int64_t row0 = t * SCAN_TILE + static_cast<int64_t>(threadIdx.x) * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int sum = 0, amax = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        const bool in = row0 + i < nn;
        v[i] = in ? rowlen[row0 + i] : 0;
        const int al = in ? adj_len[row0 + i] : 0;
        amax = max(amax, al <= MAXADJ ? al : 0);  // long rows have a kernel of their own
        sum += v[i];
    }
    int64_t total;
    const int64_t pre = block_exclusive_scan(sum, total);  // synchronises the block
    if (threadIdx.x == 0) lb_publish(look, t, (t == 0 ? LB_INC : LB_AGG) | static_cast<uint64_t>(total));
    // launch statistics: 2-, 4-, 8-, 16- and 32-row windows (tiles and threads start on
    // multiples of 32 and 8 rows)
    int m[TSTAT];
    const int w4a = v[0] + v[1] + v[2] + v[3], w4b = v[4] + v[5] + v[6] + v[7];
    m[2] = max(w4a, w4b);
    m[1] = sum + __shfl_xor(sum, 1, 64);
    m[0] = m[1] + __shfl_xor(m[1], 2, 64);
    m[3] = amax;
    m[4] = sum;
    m[5] = max(max(v[0] + v[1], v[2] + v[3]), max(v[4] + v[5], v[6] + v[7]));
#pragma unroll
    for (int c = 6; c < TSTAT; ++c) m[c] = 0;
#pragma unroll
    for (int c = 0; c < TSTAT; ++c) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) m[c] = max(m[c], __shfl_xor(m[c], d, 64));
        if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = m[c];
    }
    if (threadIdx.x < 64) {  // the tile's offset, by wave 0
        bool timeout = false;
        int64_t excl = t == 0 ? 0 : lb_exclusive(look, t, timeout);
        const bool late = __any(timeout);  // wave-uniform
        excl = late ? 0 : excl;
        if (threadIdx.x == 0) {
            if (late) atomicOr(reinterpret_cast<unsigned long long*>(info), static_cast<unsigned long long>(ERR_SCAN));
            excl_s = excl;
            if (t != 0) lb_publish(look, t, LB_INC | static_cast<uint64_t>(excl + total));
            if (static_cast<int64_t>(t + 1) * SCAN_TILE >= nn) {  // the last tile
                row_ptr[nn] = static_cast<int32_t>(excl + total);
                info[2] = excl + total;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < TSTAT) {
        const int c = threadIdx.x;
        int x = red[c][0];
#pragma unroll
        for (int w = 1; w < SBS / 64; ++w) x = max(x, red[c][w]);
        tstat[t * TSTAT + c] = x;
    }
    int64_t o = excl_s + pre;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (row0 + i < nn) row_ptr[row0 + i] = static_cast<int32_t>(o);
        o += v[i];
    }
}

// The columns of every row into col_idx (sized exactly nnz), once the row offsets are known:
// tile t moves the row-pattern blocks of its SCAN_TILE rows (thread i: block t SBS + i, rows
// 8i .. 8i+7 of the tile, whose columns lie contiguous at the start of the block's region of
// colblk).  Each wave moves groups of 4 consecutive blocks (wave w takes groups w, w + 4,
// ...): the first 64 NRD words of the 4 blocks as 4 NRD loads in flight per lane
// (consecutive lanes on consecutive words of a block), then the rest of any longer block.
template <int RW, int NRD>
__global__ __launch_bounds__(SBS) void k_row_columns(int64_t nn, const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ colblk,
                                                     int32_t* __restrict__ col_idx, int64_t cap) {
    __shared__ int32_t boff[SBS];  // offset of each block's first column in col_idx
    __shared__ int32_t bcnt[SBS];  // its number of columns
    // enqueued ahead of the host's knowledge of nnz (col_idx kept from an earlier build):
    // nothing is written unless every column fits
    if (row_ptr[nn] > cap) return;
    const int64_t blk0 = static_cast<int64_t>(blockIdx.x) * SBS;  // the tile's first row-pattern block
    const int64_t nblk = (nn + RR - 1) / RR;
    const int nb = static_cast<int>(nblk - blk0 < SBS ? nblk - blk0 : SBS);
    {
        const int64_t b = blk0 + (static_cast<int>(threadIdx.x) < nb ? threadIdx.x : nb - 1);
        const int32_t lo = row_ptr[b * RR];
        const int32_t hi = row_ptr[(b + 1) * RR < nn ? (b + 1) * RR : nn];
        boff[threadIdx.x] = lo;
        bcnt[threadIdx.x] = hi - lo;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (int g = (threadIdx.x >> 6) * 4; g < nb; g += (SBS / 64) * 4) {
        int n[4], o[4];
        const int32_t* src[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int b = min(g + j, nb - 1);
            // a group with a long row holds more columns than its region: its columns are
            // rewritten by k_long_columns, here only the region is read
            n[j] = g + j < nb ? min(bcnt[b], RW) : 0;
            o[j] = boff[b];
            src[j] = colblk + (blk0 + b) * RW;
        }
        static_assert(RW % (64 * NRD) == 0, "rounds of 64 NRD words tile a row-pattern block's region");
        // rounds of 64 NRD words per block, all loads of a round (4 blocks) in flight before
        // its stores; the first round is read whole (inside the blocks' regions), later ones
        // only where a block has words left (wave-uniform count of rounds)
        const int nmax = max(max(n[0], n[1]), max(n[2], n[3]));
        for (int w0 = 0; w0 < nmax; w0 += 64 * NRD) {
            int32_t v[4][NRD];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < NRD; ++r) {
                    const int w = w0 + lane + 64 * r;
                    v[j][r] = (w0 == 0 || w < n[j]) ? src[j][w] : 0;
                }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int r = 0; r < NRD; ++r)
                    if (w0 + lane + 64 * r < n[j]) col_idx[o[j] + w0 + lane + 64 * r] = v[j][r];
        }
    }
}

// the tiles' statistics into info[3] (32-row windows), info[4] (16 rows), info[5] (4 rows),
// info[7] (elements around a node), info[8] (8 rows) and info[9] (2 rows); one block
__global__ __launch_bounds__(SBS) void k_row_stats(int64_t tiles, const int32_t* __restrict__ tstat,
                                                   int64_t* __restrict__ info) {
    __shared__ int red[TSTAT][SBS / 64];
    int m[TSTAT];
#pragma unroll
    for (int c = 0; c < TSTAT; ++c) m[c] = 0;
    for (int64_t t = threadIdx.x; t < tiles; t += SBS) {
        const int4 v = *reinterpret_cast<const int4*>(tstat + t * TSTAT);
        const int4 w = *reinterpret_cast<const int4*>(tstat + t * TSTAT + 4);
        m[0] = max(m[0], v.x);
        m[1] = max(m[1], v.y);
        m[2] = max(m[2], v.z);
        m[3] = max(m[3], v.w);
        m[4] = max(m[4], w.x);
        m[5] = max(m[5], w.y);
    }
#pragma unroll
    for (int c = 0; c < TSTAT; ++c) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) m[c] = max(m[c], __shfl_xor(m[c], d, 64));
        if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = m[c];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int c = threadIdx.x;
        int x = red[c][0];
#pragma unroll
        for (int w = 1; w < SBS / 64; ++w) x = max(x, red[c][w]);
        constexpr int slot[6] = {3, 4, 5, 7, 8, 9};
        info[slot[c]] = x;
    }
}

// ---------------------------------------------------------------------------- P1 rows
// The row pattern of a P1 mesh and its row offsets in one pass.  A block of PR = 32 rows and
// 256 threads: thread t owns row t % 32 (its adjacency entries t / 32 + 8 q and its distinct
// nodes t / 32 + 8 u), so no phase leaves lanes idle on per-row work.  Every entry enters the
// element's other nodes into its row's 64-slot LDS table (one compare-and-swap per probe, the
// first probes of a batch of entries issued together); the first inserter of a node appends it
// to the row's list; a row's own node is entered once, by the thread holding its first entry.
// Each list item's rank (ascending node id) is its column position.  The block writes the row
// lengths, the diagonal positions, every 8-row group's sorted columns at the start of the
// group's region of 8 x 64 words of colblk (the layout the column phase moves into col_idx once
// the lengths are scanned), and, at the entry's place aptr[row] + j of the compact adjacency,
// the entry itself and its packed slot word pk (bits 0-1 local index, bits 2+8k .. 9+8k column
// position of the k-th other node, in local order).
constexpr int PR = 32;            // rows per block
constexpr int PT = 256;           // threads per block
constexpr int PJ = PT / PR;       // threads per row
constexpr int PS = MAXROW + 1;    // LDS stride of a row's table (odd: rows fall in different banks)
constexpr int PL = MAXROW + 4;    // LDS stride of a row's list (16-byte rows for four-word reads)
constexpr int PB = 3;             // entries per thread per batch (all loads of a batch in flight)
constexpr int PQ = MAXADJ / PJ;   // entries per thread at most
static_assert(PT % PR == 0 && PQ * PJ == MAXADJ && MAXROW == 64 && PR % RR == 0, "row-block shape");

template <int NLB>
__global__ __launch_bounds__(PT) void k_rows_p1(int64_t nn, const int32_t* __restrict__ elems,
                                                const int32_t* __restrict__ adj_len, const int32_t* __restrict__ adj,
                                                const int32_t* __restrict__ aptr, int32_t* __restrict__ rowlen,
                                                int32_t* __restrict__ colblk, int32_t* __restrict__ adjc,
                                                uint32_t* __restrict__ pk, int32_t* __restrict__ dpos,
                                                int32_t* __restrict__ lrows, int64_t* __restrict__ info) {
    constexpr int NO = NLB - 1;        // other nodes of an element
    constexpr int NC = PB * NO;        // inserts of a batch
    static_assert(NC <= 32, "a batch's inserts fit one mask word");
    __shared__ int32_t tab[PR * PS];               // node ids, -1 empty
    __shared__ __align__(16) int32_t lst[PR * PL];  // each row's distinct nodes, insertion order
    __shared__ uint8_t lsth[PR * PL];              // table slot of each list item
    __shared__ uint8_t srank[PR * PS];             // column position of each used table slot
    __shared__ int32_t cnt[PR];
    __shared__ int32_t rlong[PR];                  // a probe of the row found its table full
    __shared__ int32_t cpre[PR + 1];
    __shared__ int32_t guard[PT];                  // never -1: the first probes of empty entries
    const int t = static_cast<int>(threadIdx.x);
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * PR;
    const int nr = static_cast<int>((r0 + PR < nn) ? PR : nn - r0);
    const int r = t % PR, jt = t / PR;
    const int64_t row = r0 + (r < nr ? r : nr - 1);  // in bounds for the loads of rows past the end
    const int32_t self = static_cast<int32_t>(r0 + r);
    // Round trip 1, before the tables are set up: the row's length, its adjacency offsets and
    // the block's, and the thread's first batch of padded entries (every word of a padded row
    // lies in the scratch; words past the length are dropped below).
    const int32_t Lfull = adj_len[row];
    const int64_t ao = aptr[row];                           // the row's first compact entry
    const int32_t ablk0 = aptr[r0], ablk1 = aptr[r0 + nr];  // the block's compact entries
    static_assert(PB * PJ <= MAXADJ, "the first batch lies inside the padded rows");
    int32_t apre[PB];
#pragma unroll
    for (int i = 0; i < PB; ++i) apre[i] = adj[row * MAXADJ + jt + i * PJ];
    // a node of more than MAXADJ elements heads a long row: left to the long-row phase
    const int L = r < nr && Lfull <= MAXADJ ? Lfull : 0;
    // round trip 2: the first batch's element node ids, in flight while the tables are cleared
    int ndpre[PB][4];
#pragma unroll
    for (int i = 0; i < PB; ++i) apre[i] = jt + i * PJ < L ? apre[i] : 0;
    auto gather = [&](const int32_t (&aqv)[PB], int (&ndv)[PB][4]) {
        if (NLB == 4 && (reinterpret_cast<uintptr_t>(elems) & 15) == 0) {
#pragma unroll
            for (int i = 0; i < PB; ++i) {
                const int4 v = *reinterpret_cast<const int4*>(elems + static_cast<int64_t>(aqv[i] >> 2) * 4);
                ndv[i][0] = v.x;
                ndv[i][1] = v.y;
                ndv[i][2] = v.z;
                ndv[i][3] = v.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < PB; ++i)
#pragma unroll
                for (int k = 0; k < NLB; ++k) ndv[i][k] = elems[static_cast<int64_t>(aqv[i] >> 2) * NLB + k];
        }
    };
    if (jt < L) gather(apre, ndpre);  // a thread with an entry (so the mesh has elements)
    for (int h = t; h < PR * PS; h += PT) tab[h] = -1;
    if (t < PR) {
        cnt[t] = 0;
        rlong[t] = 0;
    }
    guard[t] = -2;
    __syncthreads();
    int32_t* rt = tab + r * PS;
    int32_t* rl = lst + r * PL;
    uint8_t* rh = lsth + r * PL;
    bool bad = false;

    // rare path: linear probing from slot h after a first probe that found another node
    auto probe_on = [&](int32_t v, int h, int32_t& cur) -> int {
#pragma unroll 1
        for (int probe = 1; cur != -1 && cur != v; ++probe) {
            if (probe == MAXROW) return -1;
            h = (h + 1) & (MAXROW - 1);
            cur = atomicCAS(rt + h, -1, v);
        }
        return h;
    };
    if (jt == 0 && L > 0) {  // the diagonal (a row of entries always holds its own node)
        const int h0 = rsub_hash(self);
        int32_t cur = atomicCAS(rt + h0, -1, self);
        const int h = probe_on(self, h0, cur);
        bad = bad || h < 0;
        if (h >= 0 && cur == -1) {
            const int p = atomicAdd(cnt + r, 1);
            if (p < MAXROW) {
                rl[p] = self;
                rh[p] = static_cast<uint8_t>(h);
            }
        }
    }
    uint32_t iw[PQ];  // per entry: local index | table slot of the k-th other node << (2 + 6k)
    int32_t aw[PQ];   // the entries themselves
#pragma unroll
    for (int q0 = 0; q0 < PQ; q0 += PB) {
        if (jt + q0 * PJ >= L) break;
        int32_t aq[PB];
        int nd[PB][4];
        bool okq[PB];
#pragma unroll
        for (int i = 0; i < PB; ++i) {  // loads without branches: an empty entry reads entry 0 and is dropped
            const int q = q0 + i;
            const int j = jt + q * PJ;
            okq[i] = q < PQ && j < L;
            if (q0 == 0) aq[i] = apre[i];  // read at the start, already masked
            else aq[i] = adj[row * MAXADJ + (okq[i] ? j : 0)];
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            aq[i] = okq[i] ? aq[i] : 0;
            if (q0 + i < PQ) aw[q0 + i] = aq[i];
        }
        if (q0 == 0) {
#pragma unroll
            for (int i = 0; i < PB; ++i)
#pragma unroll
                for (int k = 0; k < 4; ++k) nd[i][k] = ndpre[i][k];
        } else {
            gather(aq, nd);
        }
        // the first probe of every insert of the batch, all in flight together; an empty entry
        // probes the thread's own guard word (never -1, so nothing is stored)
        int32_t ov[NC], cq[NC];
        int hq[NC];
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int a = aq[i] & 3;
#pragma unroll
            for (int k = 0; k < NO; ++k) {
                const int c = i * NO + k;
                ov[c] = k < a ? nd[i][k] : nd[i][k + 1];
                hq[c] = rsub_hash(ov[c]);
                cq[c] = atomicCAS(okq[i] ? rt + hq[c] : guard + t, -1, ov[c]);
            }
        }
        // most first probes find the node or an empty slot; the others probe on (rarely)
        bool coll = false;
#pragma unroll
        for (int c = 0; c < NC; ++c) coll = coll || (okq[c / NO] && cq[c] != -1 && cq[c] != ov[c]);
        if (__any(coll)) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (okq[c / NO] && cq[c] != -1 && cq[c] != ov[c]) {
                    hq[c] = probe_on(ov[c], hq[c], cq[c]);
                    bad = bad || hq[c] < 0;
                }
            }
        }
        // the nodes this thread entered first go to the row's list: one atomic per batch
        uint32_t fresh = 0;
#pragma unroll
        for (int c = 0; c < NC; ++c) fresh |= static_cast<uint32_t>(okq[c / NO] && cq[c] == -1 && hq[c] >= 0) << c;
        if (fresh) {
            const int base = atomicAdd(cnt + r, __popc(fresh));
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int p = base + __popc(fresh & ((1u << c) - 1u));
                if (((fresh >> c) & 1u) && p < MAXROW) {
                    rl[p] = ov[c];
                    rh[p] = static_cast<uint8_t>(hq[c]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            if (q0 + i >= PQ) break;
            uint32_t w = static_cast<uint32_t>(aq[i] & 3);
#pragma unroll
            for (int k = 0; k < NO; ++k) w |= static_cast<uint32_t>(hq[i * NO + k] & (MAXROW - 1)) << (2 + 6 * k);
            iw[q0 + i] = w;
        }
    }
    if (bad) rlong[r] = 1;
    __syncthreads();

    // a row whose distinct nodes overflow its table (more than MAXROW nonzeros), or whose node
    // has more than MAXADJ elements, is a long row: no columns here, its diagonal position
    // -1 (the mark the long-row phase reads), and it joins the list of long rows
    const bool lng = r < nr && (Lfull > MAXADJ || rlong[r] != 0);
    const int n = lng ? 0 : min(cnt[r], MAXROW);
    if (lng && jt == 0) {
        dpos[r0 + r] = -1;
        lrows[atomicAdd(reinterpret_cast<unsigned long long*>(info + INFO_NLONG), 1ull)] = static_cast<int32_t>(r0 + r);
    }
    for (int k = jt; k < n; k += PJ) {
        const int32_t v = rl[k];
        int rank = 0;
        for (int m = 0; m < n; m += 4) {
            const int4 w = *reinterpret_cast<const int4*>(rl + m);  // words past n are stale: masked
            rank += (w.x < v) + (m + 1 < n && w.y < v) + (m + 2 < n && w.z < v) + (m + 3 < n && w.w < v);
        }
        srank[r * PS + rh[k]] = static_cast<uint8_t>(rank);
        if (v == self) dpos[r0 + r] = rank;
    }
    if (jt == 0 && r < nr && Lfull == 0) dpos[r0 + r] = 0;  // a node of no element has an empty row
    // row lengths, and each 8-row group's prefix (wave 0)
    if (t < 64) {
        const int lane = t;
        const int v = lane < PR ? (lane < nr ? n : 0) : 0;
        int x = v;
#pragma unroll
        for (int d = 1; d < RR; d <<= 1) {  // inclusive prefix inside each group of RR lanes
            const int y = __shfl_up(x, d, 64);
            if ((lane & (RR - 1)) >= d) x += y;
        }
        if (lane < PR) cpre[lane] = x - v;
        if (lane < nr) rowlen[r0 + lane] = v;
    }
    __syncthreads();
    {
        int32_t* dst = colblk + (r0 + (r & ~(RR - 1))) * MAXROW + cpre[r];  // the row's group region
        for (int k = jt; k < n; k += PJ) dst[srank[r * PS + rh[k]]] = rl[k];
    }
    // packed slots of every adjacency entry from its kept table slots.  The block's entries
    // are one contiguous range of the compact adjacency: they are gathered in the (no longer
    // read) tables and stored with consecutive lanes on consecutive words, unless the range
    // is longer than the tables hold (then each entry is stored at its place directly)
    const int nent = ablk1 - ablk0;
    constexpr int STG = PR * PS / 2;  // entries the tables hold (entry words, then slot words)
    const bool staged = nent <= STG;  // the same for the whole block
    int32_t* stg = tab;
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
        const int j = jt + q * PJ;
        if (j >= L || lng) break;  // a long row's entries are placed by the long-row phase
        const uint32_t w = iw[q];
        uint32_t word = w & 3;
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            const int h = static_cast<int>((w >> (2 + 6 * k)) & (MAXROW - 1));
            word |= static_cast<uint32_t>(srank[r * PS + h]) << (2 + 8 * k);
        }
        if (staged) {
            const int loc = static_cast<int>(ao - ablk0) + j;
            stg[loc] = aw[q];
            stg[STG + loc] = static_cast<int32_t>(word);
        } else {
            adjc[ao + j] = aw[q];
            pk[ao + j] = word;
        }
    }
    if (staged) {
        __syncthreads();
        for (int k = t; k < nent; k += PT) {
            adjc[ablk0 + k] = stg[k];
            pk[ablk0 + k] = static_cast<uint32_t>(stg[STG + k]);
        }
    }
}

// ---------------------------------------------------------------------------- long rows, structure
// Long rows (LCAP above) are built after the row-block pass has listed them: their nodes'
// compact adjacency, then one workgroup per long row for the pattern.
constexpr int LT = 256;     // threads of a long-row workgroup
constexpr int LTAB = 1024;  // slots of a long row's hash table (at most LCAP nodes: load <= 1/4)

static_assert(CSR_MAXADJ == MAXADJ && CSR_MAXROW == MAXROW && CSR_LCAP == LCAP, "one long-row rule");
__device__ __forceinline__ bool is_long_row(int elements, int nonzeros) { return csr_long_row(elements, nonzeros); }

// every entry (element << ash | local index) of a long row's node (diagonal position -1) at
// aptr[node] + a cursor; the cursor is the node's row length, which the row-block pass left
// at 0 for long rows
// (four consecutive entries per thread and pass when elems is 16-byte aligned: one 16-byte
// load, then the four diagonal-position gathers in flight together)
__device__ __forceinline__ void long_adj_entry(int64_t t, int32_t node, int nlb, int ash,
                                               const int32_t* __restrict__ aptr, int32_t* __restrict__ cur,
                                               int32_t* __restrict__ adjc) {
    const int64_t e = t / nlb;
    const int a = static_cast<int>(t - e * nlb);
    const int pos = atomicAdd(cur + node, 1);
    adjc[aptr[node] + pos] = static_cast<int32_t>((e << ash) | a);
}

__global__ __launch_bounds__(SBS) void k_long_adj(const int32_t* __restrict__ elems, int64_t m, int nlb, int ash,
                                                  const int32_t* __restrict__ dpos, const int32_t* __restrict__ aptr,
                                                  int32_t* __restrict__ cur, int32_t* __restrict__ adjc) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * SBS;
    int64_t t0 = 0;
    if ((reinterpret_cast<uintptr_t>(elems) & 15) == 0) {
        const int64_t m4 = m >> 2;
        for (int64_t q = static_cast<int64_t>(blockIdx.x) * SBS + threadIdx.x; q < m4; q += stride) {
            const int4 v = reinterpret_cast<const int4*>(elems)[q];
            const int32_t nd[4] = {v.x, v.y, v.z, v.w};
            int32_t dp[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) dp[k] = dpos[nd[k]];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (dp[k] == -1) long_adj_entry(4 * q + k, nd[k], nlb, ash, aptr, cur, adjc);
        }
        t0 = m4 << 2;
    }
    for (int64_t t = t0 + static_cast<int64_t>(blockIdx.x) * SBS + threadIdx.x; t < m; t += stride) {
        const int32_t node = elems[t];
        if (dpos[node] == -1) long_adj_entry(t, node, nlb, ash, aptr, cur, adjc);
    }
}

__device__ __forceinline__ int long_hash(int32_t v) {
    return static_cast<int>((static_cast<uint32_t>(v) * 2654435761u) >> 22);  // 10 bits
}
static_assert(LTAB == 1024, "long_hash yields 10 bits");

// One workgroup per long row: the other nodes of all its entries (and the row's own) enter an
// LDS hash table; the distinct nodes are ranked (ascending: the column positions), written to
// the row's list in lcol (LCAP words per long row), and every entry's slot word is formed
// from the ranks of its element's other nodes: P1 (ASH = 2) pk as in the row-block pass, P2
// (ASH = 4) 8-bit positions in pk2 (k < 8) and pk9 (the ninth).  More than LCAP distinct
// nodes: ERR_ROW.
template <int NLB, int ASH>
__global__ __launch_bounds__(LT) void k_rows_long(const int32_t* __restrict__ lrows, const int32_t* __restrict__ elems,
                                                  const int32_t* __restrict__ aptr, const int32_t* __restrict__ adjc,
                                                  int32_t* __restrict__ rowlen, int32_t* __restrict__ lcol,
                                                  uint32_t* __restrict__ pk, uint64_t* __restrict__ pk2,
                                                  uint8_t* __restrict__ pk9, int32_t* __restrict__ dpos,
                                                  int64_t* __restrict__ info) {
    constexpr int NO = NLB - 1;
    static_assert((ASH == 2 && NO <= 3) || (ASH == 4 && NO <= 9), "P1 entries: 2-bit index; P2: 4-bit");
    __shared__ int32_t tab[LTAB];
    __shared__ uint8_t trank[LTAB];
    __shared__ int32_t lst[LCAP];
    __shared__ int16_t lsth[LCAP];
    __shared__ int32_t nlst;
    const int t = static_cast<int>(threadIdx.x);
    const int32_t row = lrows[blockIdx.x];
    const int64_t a0 = aptr[row];
    const int L = aptr[row + 1] - static_cast<int>(a0);
    for (int h = t; h < LTAB; h += LT) tab[h] = -1;
    if (t == 0) nlst = 0;
    __syncthreads();
    auto insert = [&](int32_t v) {
        int h = long_hash(v);
        for (int probe = 0; probe < LTAB; ++probe) {  // the table never fills: probing ends
            const int32_t c = atomicCAS(tab + h, -1, v);
            if (c == -1) {
                const int p = atomicAdd(&nlst, 1);
                if (p < LCAP) {
                    lst[p] = v;
                    lsth[p] = static_cast<int16_t>(h);
                }
                return;
            }
            if (c == v) return;
            h = (h + 1) & (LTAB - 1);
        }
    };
    if (t == 0) insert(row);
    for (int j = t; j < L; j += LT) {
        const int32_t w = adjc[a0 + j];
        const int64_t e = static_cast<uint32_t>(w) >> ASH;
        const int a = w & ((1 << ASH) - 1);
#pragma unroll
        for (int k = 0; k < NO; ++k) insert(elems[e * NLB + (k < a ? k : k + 1)]);
    }
    __syncthreads();
    const int n = nlst;  // the same for every thread
    if (n > LCAP) {
        if (t == 0) atomicOr(reinterpret_cast<unsigned long long*>(info), static_cast<unsigned long long>(ERR_ROW));
        return;
    }
    int32_t* out = lcol + static_cast<int64_t>(blockIdx.x) * LCAP;
    for (int k = t; k < n; k += LT) {
        const int32_t v = lst[k];
        int rank = 0;
        for (int u = 0; u < n; ++u) rank += lst[u] < v;
        trank[lsth[k]] = static_cast<uint8_t>(rank);
        out[rank] = v;
        if (v == row) dpos[row] = rank;
    }
    if (t == 0) rowlen[row] = n;
    __syncthreads();
    for (int j = t; j < L; j += LT) {
        const int32_t w = adjc[a0 + j];
        const int64_t e = static_cast<uint32_t>(w) >> ASH;
        const int a = w & ((1 << ASH) - 1);
        uint64_t word = ASH == 2 ? static_cast<uint64_t>(a) : 0ull;
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            const int32_t v = elems[e * NLB + (k < a ? k : k + 1)];
            int h = long_hash(v);
            while (tab[h] != v) h = (h + 1) & (LTAB - 1);  // present: entered above
            if constexpr (ASH == 2) word |= static_cast<uint64_t>(trank[h]) << (2 + 8 * k);
            else if (k < 8) word |= static_cast<uint64_t>(trank[h]) << (8 * k);
            else pk9[a0 + j] = trank[h];
        }
        if constexpr (ASH == 2) pk[a0 + j] = static_cast<uint32_t>(word);
        else pk2[a0 + j] = word;
    }
}

// The columns of the 8-row groups that hold a long row, rewritten once col_idx is sized: the
// long row's from its list, the group's other rows from the group's colblk region (RR x
// maxrow words: maxrow = MAXROW for P1, MAXROW2 for P2; in row order, lengths from row_ptr).
// Two long rows of one group write the same words for the group's other rows.
__global__ __launch_bounds__(LT) void k_long_columns(const int32_t* __restrict__ lrows, int64_t nn, int maxrow,
                                                     const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ aptr,
                                                     const int32_t* __restrict__ colblk,
                                                     const int32_t* __restrict__ lcol, int32_t* __restrict__ col_idx) {
    const int t = static_cast<int>(threadIdx.x);
    const int64_t row = lrows[blockIdx.x];
    {
        const int64_t w0 = row_ptr[row];
        const int len = row_ptr[row + 1] - static_cast<int>(w0);
        for (int k = t; k < len; k += LT) col_idx[w0 + k] = lcol[static_cast<int64_t>(blockIdx.x) * LCAP + k];
    }
    const int64_t g0 = row / RR * RR;
    const int32_t* src = colblk + g0 * maxrow;  // the group's region
    int off = 0;
    for (int64_t r = g0; r < g0 + RR && r < nn; ++r) {
        const int64_t w0 = row_ptr[r];
        const int len = row_ptr[r + 1] - static_cast<int>(w0);
        if (aptr[r + 1] - aptr[r] > MAXADJ || len > maxrow) continue;  // a long row (P1 or P2)
        for (int k = t; k < len; k += LT) col_idx[w0 + k] = src[off + k];
        off += len;
    }
}

// ---------------------------------------------------------------------------- faces
// All faces of the mesh (section 3.2: normals of all faces, or of the boundary faces only),
// grouped by their smallest node.  Node i owns the faces of its adjacent elements whose
// other nodes all come after i, i.e. lie after the diagonal in row i of the CSR structure;
// the packed slot words give those positions without a gather, so inside its row a face is
// keyed by the column positions of its other nodes, and ascending keys are ascending node
// ids.  Two passes over blocks of FR rows: pass 0 counts each row's faces and boundary
// faces (for the scans), pass 1 rebuilds the same tables and writes every face at its
// place -- nodes ordered outward of its first element (the smaller element id), the pair
// of elements, and the boundary faces in a list of their own.
constexpr int FR = 8;              // rows per block
constexpr int FT = 128;            // threads per block
constexpr int FSUB = 128;          // slots of one row's face table (faces a node owns, at most 128)
constexpr int64_t ERR_FACE = 8;    // a face in more than two elements
static_assert(FT >= FR && FT >= 64, "one thread per row");

__device__ __forceinline__ int fsub_hash(int32_t k) {
    return static_cast<int>((static_cast<uint32_t>(k) * 2654435761u) >> 25);  // 7 bits
}
static_assert(FSUB == 128, "fsub_hash yields 7 bits");

// find or insert k in a row's face table (one compare-and-swap per probe); -1 when full
// A face table word holds the face's key (bits 0-23) and the number of elements that
// reached it (bits 24-30: at most 64, the elements around a node), -1 when empty.
constexpr int32_t FKEY = (1 << 24) - 1;
constexpr int FCNT = 24;

__device__ __forceinline__ int fsub_insert(int32_t* tab, int32_t k, bool& fresh) {
    int h = fsub_hash(k);
#pragma unroll 1
    for (int probe = 0; probe < FSUB; ++probe) {
        const int32_t cur = atomicCAS(tab + h, -1, k);
        if (cur == -1 || (cur & FKEY) == k) {
            fresh = cur == -1;
            return h;
        }
        h = (h + 1) & (FSUB - 1);
    }
    fresh = false;
    return -1;
}

// local node order of the face opposite local node k, outward for a positively oriented
// element (det J > 0, first-node origin); reversed when det J < 0
__device__ __forceinline__ int face_local(int nlb, int k, int t) {
    if (nlb == 4) {
        constexpr int F3[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
        return F3[k][t];
    }
    constexpr int F2[3][2] = {{1, 2}, {2, 0}, {0, 1}};
    return F2[k][t];
}

// orientation of every element: esign[e] = 1 when det J < 0 (FP64, first-node origin)
template <int NLB>
__global__ __launch_bounds__(SBS) void k_elem_sign(int64_t ne, const double* __restrict__ coords,
                                                   const int32_t* __restrict__ elems, uint8_t* __restrict__ esign) {
    constexpr int D = NLB - 1;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * SBS + threadIdx.x;
    if (e >= ne) return;
    double ev[D][D];
    const int64_t n0 = elems[e * NLB];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int64_t nk = elems[e * NLB + k + 1];
#pragma unroll
        for (int c = 0; c < D; ++c) ev[k][c] = coords[nk * D + c] - coords[n0 * D + c];
    }
    double det;
    if constexpr (D == 3)
        det = ev[0][0] * (ev[1][1] * ev[2][2] - ev[1][2] * ev[2][1]) - ev[0][1] * (ev[1][0] * ev[2][2] - ev[1][2] * ev[2][0]) +
              ev[0][2] * (ev[1][0] * ev[2][1] - ev[1][1] * ev[2][0]);
    else
        det = ev[0][0] * ev[1][1] - ev[0][1] * ev[1][0];
    esign[e] = det < 0.0 ? 1 : 0;
}

// One face of row i written at its place f (and fb >= 0 in the boundary list): its first
// element is the smaller of the two that reached it (equal ids, a degenerate mesh, ordered by
// the opposite node and the slot word, so the choice never depends on arrival order); code:
// entry position in the row's adjacency << 2 | local node opposite the face, w and q: the
// entry's adjacency and slot words.  The nodes follow the face opposite that node, outward
// of the first element (reversed when its det J < 0): node i itself, or an other node of
// the element at its column position in row i.
template <int NLB>
__device__ __forceinline__ void emit_face(int64_t i, int c, int code0, int code1, int32_t w0, int32_t w1, uint32_t q0,
                                          uint32_t q1, int32_t rb, int64_t f, int64_t fb,
                                          const int32_t* __restrict__ col_idx, const uint8_t* __restrict__ esign,
                                          int32_t* __restrict__ faces, int32_t* __restrict__ fel,
                                          int32_t* __restrict__ bfaces, int32_t* __restrict__ bel) {
    constexpr int NV = NLB - 1;
    const uint32_t ea = static_cast<uint32_t>(w0) >> 2, eb = static_cast<uint32_t>(w1) >> 2;
    const uint32_t ka = (static_cast<uint32_t>(code0 & 3) << 26) | (q0 & 0x3ffffffu);
    const uint32_t kb = (static_cast<uint32_t>(code1 & 3) << 26) | (q1 & 0x3ffffffu);
    const bool second = c == 2 && (eb < ea || (eb == ea && kb < ka));
    const int64_t e1 = second ? eb : ea;
    const int32_t e2 = static_cast<int32_t>(second ? ea : eb);
    const int opp = (second ? code1 : code0) & 3;
    const uint32_t p1 = second ? q1 : q0;
    const int a1 = static_cast<int>(p1 & 3);  // local index of node i in e1
    const bool flip = esign[e1] != 0;
#pragma unroll
    for (int t = 0; t < NV; ++t) {
        const int L = face_local(NLB, opp, flip ? NV - 1 - t : t);  // local node of e1
        const int32_t v = L == a1 ? static_cast<int32_t>(i)
                                  : col_idx[rb + static_cast<int>((p1 >> (2 + 8 * (L < a1 ? L : L - 1))) & 255)];
        faces[f * NV + t] = v;
        if (fb >= 0) bfaces[fb * NV + t] = v;
    }
    fel[2 * f] = static_cast<int32_t>(e1);
    fel[2 * f + 1] = c == 2 ? e2 : -1;
    if (fb >= 0) bel[fb] = static_cast<int32_t>(e1);
}

template <int NLB, int PASS>
__global__ __launch_bounds__(FT) void k_faces(int64_t nn, const int32_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col_idx, const int32_t* __restrict__ aptr,
                                              const int32_t* __restrict__ adj, const uint32_t* __restrict__ pk,
                                              const int32_t* __restrict__ dpos, const uint8_t* __restrict__ esign,
                                              int32_t* __restrict__ fcount, int32_t* __restrict__ bcount,
                                              const int32_t* __restrict__ fptr, const int32_t* __restrict__ bptr,
                                              int32_t* __restrict__ faces, int32_t* __restrict__ fel,
                                              int32_t* __restrict__ bfaces, int32_t* __restrict__ bel,
                                              int64_t* __restrict__ info) {
    constexpr int NV = NLB - 1;  // nodes of a face = other nodes of an element
    __shared__ int32_t key[FR * FSUB];  // face key | element count << FCNT
    // the two elements of each face, in arrival order, as the position of their entry in the
    // row's adjacency << 2 | the local node opposite the face (pass 1 only; 2 KB per block
    // instead of two 64-bit words per slot, for twice the resident blocks): the writing phase
    // reads the two entries back and takes the smaller element as the face's first
    constexpr int WS = PASS == 1 ? FR * FSUB * 2 : 1;
    __shared__ uint8_t wj[WS];
    __shared__ int16_t list[FR * FSUB];  // used slots of each row
    __shared__ int32_t nlist[FR], dslot[FR], alen[FR], abase[FR], lpre[FR + 1];
    __shared__ int32_t maxl;
    __shared__ int32_t rowp[FR], rowf[FR], rowb[FR];
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * FR;
    const int nr = static_cast<int>((r0 + FR < nn) ? FR : nn - r0);
    // every load that does not depend on another is issued first: the rows' adjacency and
    // row offsets, diagonal positions and (pass 1) face offsets; then the first FPRE batches
    // of entries.  A long row counts as empty here: k_faces_long takes it.
    {
        const int r = static_cast<int>(threadIdx.x) < nr ? static_cast<int>(threadIdx.x) : 0;
        const int32_t a0 = aptr[r0 + r], a1 = aptr[r0 + r + 1], dv = dpos[r0 + r];
        const int32_t pv = row_ptr[r0 + r], pv1 = row_ptr[r0 + r + 1];
        int32_t fv = 0, bv = 0;
        if constexpr (PASS == 1) {
            fv = fptr[r0 + r];
            bv = bptr[r0 + r];
        }
        if (threadIdx.x < FR) {
            const int L = static_cast<int>(threadIdx.x) < nr && !is_long_row(a1 - a0, pv1 - pv) ? a1 - a0 : 0;
            alen[threadIdx.x] = L;
            abase[threadIdx.x] = a0;
            nlist[threadIdx.x] = 0;
            dslot[threadIdx.x] = L > 0 ? dv : 0;
            rowp[threadIdx.x] = pv;
            rowf[threadIdx.x] = fv;
            rowb[threadIdx.x] = bv;
        }
    }
    for (int h = threadIdx.x; h < FR * FSUB; h += FT) key[h] = -1;
    if (threadIdx.x == 0) maxl = 0;
    __syncthreads();
    if (threadIdx.x < FR) atomicMax(&maxl, alen[threadIdx.x]);
    // the first FPRE batches of entries, in flight together (an entry past its row's length
    // reads entry 0 and is dropped)
    constexpr int FPRE = 2;
    int32_t wpre[FPRE];
    uint32_t ppre[FPRE];
#pragma unroll
    for (int b = 0; b < FPRE; ++b) {
        const int idx = static_cast<int>(threadIdx.x) + b * FT;
        const int r = idx % FR, j = idx / FR;
        const int64_t t = j < alen[r] ? static_cast<int64_t>(abase[r]) + j : 0;
        wpre[b] = adj[t];
        ppre[b] = pk[t];
    }
    __syncthreads();
    bool full = false;
    // entries dealt r + FR j: the faces each one owns go into its row's table
    auto entry = [&](int r, int j, int32_t w, uint32_t p) {
        const int a = w & 3;
        int s[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] = static_cast<int>((p >> (2 + 8 * k)) & 255);
        int32_t* tab = key + r * FSUB;
#pragma unroll
        for (int k = 0; k < NV; ++k) {  // the face opposite the k-th other node
            int smin = 1 << 20, smax = -1;
#pragma unroll
            for (int k2 = 0; k2 < NV; ++k2) {
                if (k2 == k) continue;
                smin = min(smin, s[k2]);
                smax = max(smax, s[k2]);
            }
            if (smin <= dslot[r]) continue;  // a node before the row's own: another row owns it
            const int32_t kk = NV == 3 ? (smin << 6) | smax : smin;
            bool fresh;
            const int h = fsub_insert(tab, kk, fresh);
            if (h < 0) {
                full = true;
                continue;
            }
            if (fresh) list[r * FSUB + atomicAdd(&nlist[r], 1)] = static_cast<int16_t>(h);
            const int ord = atomicAdd(&key[r * FSUB + h], 1 << FCNT) >> FCNT;  // arrival order
            if constexpr (PASS == 1) {
                const int opp = k < a ? k : k + 1;  // local index of the opposite node
                if (ord < 2) wj[(r * FSUB + h) * 2 + ord] = static_cast<uint8_t>((j << 2) | opp);
            }
        }
    };
#pragma unroll
    for (int b = 0; b < FPRE; ++b) {
        const int idx = static_cast<int>(threadIdx.x) + b * FT;
        const int r = idx % FR, j = idx / FR;
        if (j < alen[r]) entry(r, j, wpre[b], ppre[b]);
    }
    for (int idx = threadIdx.x + FPRE * FT; idx < FR * maxl; idx += FT) {
        const int r = idx % FR, j = idx / FR;
        if (j >= alen[r]) continue;
        const int64_t t = static_cast<int64_t>(abase[r]) + j;
        entry(r, j, adj[t], pk[t]);
    }
    __syncthreads();
    if constexpr (PASS == 0) {
        bool bad = false;
        if (threadIdx.x < nr) {
            const int r = threadIdx.x;
            int nb = 0;
            const int nl = nlist[r];
            const int16_t* lr = list + r * FSUB;
            const int32_t* kr = key + r * FSUB;
            int u = 0;
            for (; u + 4 <= nl; u += 4) {  // four independent slot and key reads in flight
                int c[4];
#pragma unroll
                for (int z = 0; z < 4; ++z) c[z] = kr[lr[u + z]] >> FCNT;
#pragma unroll
                for (int z = 0; z < 4; ++z) {
                    nb += c[z] == 1;
                    bad = bad || c[z] > 2;
                }
            }
            for (; u < nl; ++u) {
                const int c = kr[lr[u]] >> FCNT;
                nb += c == 1;
                bad = bad || c > 2;
            }
            fcount[r0 + r] = nlist[r];
            bcount[r0 + r] = nb;
        }
        if (bad || full)
            atomicOr(reinterpret_cast<unsigned long long*>(info),
                     static_cast<unsigned long long>((bad ? ERR_FACE : 0) | (full ? ERR_ROW : 0)));
    } else {
        if (threadIdx.x == 0) {  // the block's faces, row after row
            int acc = 0;
            for (int r = 0; r < FR; ++r) {
                lpre[r] = acc;
                acc += nlist[r];
            }
            lpre[FR] = acc;
        }
        __syncthreads();
        for (int q = threadIdx.x; q < lpre[FR]; q += FT) {
            int r = 0;
            while (q >= lpre[r + 1]) ++r;
            const int h = list[r * FSUB + (q - lpre[r])];
            const int32_t kk = key[r * FSUB + h] & FKEY;
            const int c = key[r * FSUB + h] >> FCNT;
            // the face's entries, read back while the rank is counted (both, when it has two)
            const int c0 = wj[(r * FSUB + h) * 2], c1 = c == 2 ? wj[(r * FSUB + h) * 2 + 1] : c0;
            const int64_t t0 = static_cast<int64_t>(abase[r]) + (c0 >> 2), t1 = static_cast<int64_t>(abase[r]) + (c1 >> 2);
            const int32_t w0 = adj[t0], w1 = adj[t1];
            const uint32_t q0 = pk[t0], q1 = pk[t1];
            int rank = 0, brank = 0;
            const int nl = nlist[r];
            const int16_t* lr = list + r * FSUB;
            const int32_t* kr = key + r * FSUB;
            int v = 0;
            for (; v + 4 <= nl; v += 4) {  // four independent slot and key reads in flight
                int32_t w2[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) w2[u] = kr[lr[v + u]];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool before = (w2[u] & FKEY) < kk;
                    rank += before;
                    brank += before && (w2[u] >> FCNT) == 1;
                }
            }
            for (; v < nl; ++v) {
                const int32_t w2 = kr[lr[v]];
                const bool before = (w2 & FKEY) < kk;
                rank += before;
                brank += before && (w2 >> FCNT) == 1;
            }
            const int64_t f = rowf[r] + rank;
            const int64_t fb = c == 1 ? rowb[r] + brank : -1;
            emit_face<NLB>(r0 + r, c, c0, c1, w0, w1, q0, q1, rowp[r], f, fb, col_idx, esign, faces, fel, bfaces,
                           bel);
        }
    }
}

// The faces of the long rows (the rows the row-block passes leave empty), one workgroup per
// row with the same two passes: the entries' faces owned by the row go into one table of FLS
// slots keyed by the column positions of their other nodes (8 bits each here), each arrival
// keeps its entry position and opposite node (pass 1), and each face's rank among the row's
// keys is its place.  A row may own FLC faces (more sets ERR_ROW): the link of a node with at
// most 255 neighbours has fewer triangles.
constexpr int FLT = 256;   // threads of a long-row face workgroup
constexpr int FLS = 2048;  // slots of its table
constexpr int FLC = 1024;  // faces one long row may own
static_assert(FLC <= FLS / 2 && FLC <= 32767, "the table stays at most half full; list items fit 16 bits");

__device__ __forceinline__ int flong_hash(int32_t k) {
    return static_cast<int>((static_cast<uint32_t>(k) * 2654435761u) >> 21);  // 11 bits
}

template <int NLB, int PASS>
__global__ __launch_bounds__(FLT) void k_faces_long(const int32_t* __restrict__ lrows,
                                                    const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col_idx,
                                                    const int32_t* __restrict__ aptr, const int32_t* __restrict__ adj,
                                                    const uint32_t* __restrict__ pk, const int32_t* __restrict__ dpos,
                                                    const uint8_t* __restrict__ esign, int32_t* __restrict__ fcount,
                                                    int32_t* __restrict__ bcount, const int32_t* __restrict__ fptr,
                                                    const int32_t* __restrict__ bptr, int32_t* __restrict__ faces,
                                                    int32_t* __restrict__ fel, int32_t* __restrict__ bfaces,
                                                    int32_t* __restrict__ bel, int64_t* __restrict__ info) {
    constexpr int NV = NLB - 1;
    static_assert(FKEY >= (255 << 8 | 255), "two 8-bit positions fit a key");
    __shared__ int32_t key[FLS];  // face key | element count << FCNT
    __shared__ int16_t list[FLC];
    constexpr int WS = PASS == 1 ? 2 * FLS : 1;
    __shared__ int32_t wj[WS];  // per arrival: entry position << 2 | opposite local node
    __shared__ int32_t nlist, nbnd, flags;
    const int t = static_cast<int>(threadIdx.x);
    const int64_t i = lrows[blockIdx.x];
    const int64_t a0 = aptr[i];
    const int L = aptr[i + 1] - static_cast<int>(a0);
    const int ds = dpos[i];
    for (int h = t; h < FLS; h += FLT) key[h] = -1;
    if (t == 0) {
        nlist = 0;
        nbnd = 0;
        flags = 0;
    }
    __syncthreads();
    bool full = false;
    for (int j = t; j < L; j += FLT) {
        const int32_t w = adj[a0 + j];
        const uint32_t p = pk[a0 + j];
        const int a = w & 3;
        int sp[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) sp[k] = static_cast<int>((p >> (2 + 8 * k)) & 255);
#pragma unroll
        for (int k = 0; k < NV; ++k) {  // the face opposite the k-th other node
            int smin = 1 << 20, smax = -1;
#pragma unroll
            for (int k2 = 0; k2 < NV; ++k2) {
                if (k2 == k) continue;
                smin = min(smin, sp[k2]);
                smax = max(smax, sp[k2]);
            }
            if (smin <= ds) continue;  // a node before the row's own: another row owns it
            const int32_t kk = NV == 3 ? (smin << 8) | smax : smin;
            int h = flong_hash(kk);
            int cur = -1;
            int probe = 0;
            for (; probe < FLS; ++probe) {  // linear probing; the table never fills (FLC <= FLS / 2)
                cur = atomicCAS(key + h, -1, kk);
                if (cur == -1 || (cur & FKEY) == kk) break;
                h = (h + 1) & (FLS - 1);
            }
            if (probe == FLS) {
                full = true;
                continue;
            }
            if (cur == -1) {
                const int u = atomicAdd(&nlist, 1);
                if (u < FLC) list[u] = static_cast<int16_t>(h);
                else full = true;
            }
            const int ord = atomicAdd(key + h, 1 << FCNT) >> FCNT;  // arrival order
            if constexpr (PASS == 1) {
                if (ord < 2) wj[2 * h + ord] = (j << 2) | (k < a ? k : k + 1);
            }
        }
    }
    if (full) atomicOr(&flags, 1);
    __syncthreads();
    const int nl = min(nlist, FLC);
    if constexpr (PASS == 0) {
        int nb = 0;
        bool bad = false;
        for (int u = t; u < nl; u += FLT) {
            const int c = key[list[u]] >> FCNT;
            nb += c == 1;
            bad = bad || c > 2;
        }
        if (nb) atomicAdd(&nbnd, nb);
        if (bad) atomicOr(&flags, 2);
        __syncthreads();
        if (t == 0) {
            fcount[i] = nl;
            bcount[i] = nbnd;
            if (flags)
                atomicOr(reinterpret_cast<unsigned long long*>(info),
                         static_cast<unsigned long long>(((flags & 2) ? ERR_FACE : 0) | ((flags & 1) ? ERR_ROW : 0)));
        }
    } else {
        const int32_t rb = row_ptr[i];
        const int64_t f0 = fptr[i], b0 = bptr[i];
        for (int q = t; q < nl; q += FLT) {
            const int h = list[q];
            const int32_t kk = key[h] & FKEY;
            const int c = key[h] >> FCNT;
            const int c0 = wj[2 * h], c1 = c == 2 ? wj[2 * h + 1] : c0;
            const int32_t w0 = adj[a0 + (c0 >> 2)], w1 = adj[a0 + (c1 >> 2)];
            const uint32_t q0 = pk[a0 + (c0 >> 2)], q1 = pk[a0 + (c1 >> 2)];
            int rank = 0, brank = 0;
            for (int u = 0; u < nl; ++u) {
                const int32_t w2 = key[list[u]];
                const bool before = (w2 & FKEY) < kk;
                rank += before;
                brank += before && (w2 >> FCNT) == 1;
            }
            emit_face<NLB>(i, c, c0, c1, w0, w1, q0, q1, rb, f0 + rank, c == 1 ? b0 + brank : -1, col_idx, esign,
                           faces, fel, bfaces, bel);
        }
    }
}

// ---------------------------------------------------------------------------- numeric
#ifndef PF_NUMERIC_ROWS
#define PF_NUMERIC_ROWS 32
#endif
#ifndef PF_NUMERIC_ITEMS
#define PF_NUMERIC_ITEMS 3
#endif
constexpr int NR_BIG = PF_NUMERIC_ROWS;   // rows per block of the numeric kernel
constexpr int NR_MID = PF_NUMERIC_ROWS / 2;  // ... when a node has more elements than a big block covers
constexpr int NR_SMALL = 4;  // ... when neither fits
constexpr int NBT = 256;     // threads per block of the numeric kernel
constexpr int NITEMS = PF_NUMERIC_ITEMS;    // adjacency entries per thread (held in registers)
static_assert(MAXADJ <= NITEMS * NBT / NR_SMALL, "the small numeric blocks must cover any admissible row");
static_assert(NR_SMALL == 4 && NR_MID == 16 && NR_BIG == 32, "k_row_offsets measures windows of 4, 16 and 32 rows");
static_assert(MAXADJ == CSR_MAXADJ, "one padded adjacency layout");
// FP32 blocks: NT32 threads, with 8, 16 or 32 threads per row (rows per block NT32 / 8,
// NT32 / 16, NT32 / 32) so that NITEMS entries per thread cover 24, 48 or 96 elements per node
#ifndef PF_F32_THREADS
#define PF_F32_THREADS 128
#endif
constexpr int NT32 = PF_F32_THREADS;
static_assert(NT32 == 64 || NT32 == 128 || NT32 == 256, "FP32 numeric blocks of one, two or four waves");
static_assert(MAXADJ <= NITEMS * 32, "the FP32 class with 32 threads per row covers any admissible row");

template <typename T>
struct alignas(16) Vec4 {  // 16-byte LDS reads; the layout keeps Vec4 arrays 16-byte aligned
    T x, y, z, w;
};

// Row of K_e and M_e for the element's node that is the origin of the edge vectors (local
// vertex 0 of the geometry): k[b] = cK |T| grad phi_0 . grad phi_b, mo = cM |T| / ((d+1)(d+2)).
template <int DIM, typename C>
__device__ __forceinline__ void origin_row(const P1Geom<DIM, C>& g, C ck, C cm, C (&k)[DIM + 1], C& mo) {
    const C adet = fabs(g.det);
    C kf;
    if constexpr (sizeof(C) == 4) kf = ck * __builtin_amdgcn_rcpf(static_cast<C>(fact_dim<DIM>()) * adet);  // 1 ulp
    else kf = ck / (static_cast<C>(fact_dim<DIM>()) * adet);
#pragma unroll
    for (int b = 0; b <= DIM; ++b) {
        C s = g.c[0][0] * g.c[b][0];
#pragma unroll
        for (int q = 1; q < DIM; ++q) s = fmaT(g.c[0][q], g.c[b][q], s);
        k[b] = kf * s;
    }
    mo = cm * adet * static_cast<C>(1.0 / (fact_dim<DIM>() * (DIM + 1) * (DIM + 2)));
}

// Row of K_e and M_e from FP64 edge vectors, plain FP64 arithmetic (used for the elements the
// FP32 path routes: FP64 carries 29 more bits than the FP32 result needs, so no compensation
// is required, and the path stays light on registers).
template <int DIM>
__device__ __forceinline__ void origin_row_f64(const double (&u)[DIM][DIM], double ck, double cm,
                                               double (&k)[DIM + 1], double& mo, double& adet_out) {
    double c[DIM + 1][DIM];
    double det;
    if constexpr (DIM == 3) {
#pragma unroll
        for (int j = 1; j <= 3; ++j) {
            const double* x = u[j % 3];
            const double* y = u[(j + 1) % 3];
            c[j][0] = fmaT(x[1], y[2], -x[2] * y[1]);
            c[j][1] = fmaT(x[2], y[0], -x[0] * y[2]);
            c[j][2] = fmaT(x[0], y[1], -x[1] * y[0]);
        }
        det = fmaT(u[0][0], c[1][0], fmaT(u[0][1], c[1][1], u[0][2] * c[1][2]));
    } else {
        c[1][0] = u[1][1];
        c[1][1] = -u[1][0];
        c[2][0] = -u[0][1];
        c[2][1] = u[0][0];
        det = fmaT(u[0][0], u[1][1], -u[0][1] * u[1][0]);
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        double s = c[1][i];
#pragma unroll
        for (int j = 2; j <= DIM; ++j) s += c[j][i];
        c[0][i] = -s;
    }
    const double adet = fabs(det);
    adet_out = adet;
    const double kf = ck / (fact_dim<DIM>() * adet);
#pragma unroll
    for (int b = 0; b <= DIM; ++b) {
        double s = c[0][0] * c[b][0];
#pragma unroll
        for (int q = 1; q < DIM; ++q) s = fmaT(c[0][q], c[b][q], s);
        k[b] = kf * s;
    }
    mo = cm * adet * (1.0 / (fact_dim<DIM>() * (DIM + 1) * (DIM + 2)));
}

// FP32 routing test with thresholds already rounded to FP32: route unless 0 < |det| < inf,
// |det| >= tau_abs and absterms <= tau_cond |det| (a NaN fails every comparison, so NaN
// det or absterms route; an infinite absterms with finite det fails the last test)
__device__ __forceinline__ bool route32(float det, float absterms, double shape2, float tau_abs, float tau_cond,
                                        int enable) {
    const float ad = fabsf(det);
    const double d = ad;
    const bool keep = ad > 0.0f && ad < __builtin_huge_valf() && ad >= tau_abs && absterms <= tau_cond * ad &&
                      shape2 <= SHAPE_MAX * SHAPE_MAX * d * d;
    return enable && !keep;
}

// dynamic LDS of one numeric block of numeric_block
template <int DIM, typename T>
constexpr size_t numeric_lds_bytes(int nr, int wmax) {
    return static_cast<size_t>(wmax) * (2 * sizeof(typename Exact<T>::acc) + sizeof(Vec4<T>) + 8) +
           static_cast<size_t>(3 * (nr + 1) + 1) * 4;
}

// Numeric assembly, NR rows per block:
//   phase 0  every CSR slot of the block's window gets the edge vector from its row's node to
//            its column's node (FP64 difference, rounded once to T) in LDS;
//   phase 1  every adjacency entry (row node = element vertex a) computes, from three edge
//            vectors read from LDS, its element's row a of K_e and M_e (routed elements are
//            recomputed from the FP64 coordinates) and keeps it in registers; each slot's
//            largest contribution fixes that slot's grid, and the rounded contributions
//            are added into LDS accumulators with atomics (exact: order does not matter);
//   phase 2  every slot converts its sum and stores it once (coalesced).
// Entries and slots are dealt row-interleaved (item r + NR j), so the lanes of one
// instruction work on different rows and their LDS atomics hit different addresses.
// One block of NR rows starting at row r0 (the body of the numeric kernels).  QN > 0:
// cK and cM hold QN values per element at the integration points of the QuadRule<DIM, QN>
// (the stiffness takes their weighted mean, the mass row is integrated point by point).
template <int DIM, typename T, bool COEF, int NR, int QN = 0>
__device__ __forceinline__ void numeric_block(int64_t r0, int64_t nn, const double* __restrict__ coords,
                                              const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                                              const int32_t* __restrict__ aptr, const int32_t* __restrict__ adj,
                                              const uint32_t* __restrict__ pk, const T* __restrict__ cK,
                                              const T* __restrict__ cM, T* __restrict__ valsK, T* __restrict__ valsM,
                                              const Fallback& fb, int64_t* d_counters, int wmax) {
    constexpr int NLB = DIM + 1;
    using A = typename Exact<T>::acc;
    extern __shared__ __align__(16) unsigned char smem[];
    // 16-byte vectors first, then the accumulators, so every LDS access is naturally aligned
    Vec4<T>* f = reinterpret_cast<Vec4<T>*>(smem);               // [wmax] edge vector per slot
    A* accK = reinterpret_cast<A*>(f + wmax);                    // [wmax]
    A* accM = accK + wmax;                                       // [wmax]
    int32_t* shK = reinterpret_cast<int32_t*>(accM + wmax);      // [wmax] max bits, then shift
    int32_t* shM = shK + wmax;                                   // [wmax]
    int32_t* rp = shM + wmax;                                    // [NR + 1]
    int32_t* ap = rp + (NR + 1);                                 // [NR + 1] adjacency offsets of the rows
    int32_t* dslot = ap + (NR + 1);                              // [NR + 1]
    int32_t* maxlen = dslot + (NR + 1);                          // [1]
    static_assert(lds_carve_aligned<Vec4<T>, A, A, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t>(),
                  "numeric LDS carve-out: every array naturally aligned");

    // Items are dealt by NR (row r = item % NR, a power of two); rows past the end of the
    // matrix in the last block are empty (no elements, no slots).
    static_assert((NR & (NR - 1)) == 0, "NR is a power of two");
    const int nr = static_cast<int>((r0 + NR < nn) ? NR : nn - r0);
    {
        const int t = static_cast<int>(threadIdx.x);
        const int32_t rpv = row_ptr[r0 + (t <= nr ? t : nr)];  // both loads unconditional
        const int32_t apv = aptr[r0 + (t <= nr ? t : nr)];  // rows past the end: no elements
        if (t <= NR) rp[t] = rpv;
        if (t <= NR) ap[t] = apv;
    }
    if (threadIdx.x == 0) *maxlen = 0;
    __syncthreads();
    if (threadIdx.x < nr) atomicMax(maxlen, rp[threadIdx.x + 1] - rp[threadIdx.x]);
    const int32_t w0 = rp[0];
    const int W = rp[nr] - w0;
    // packed entries of this thread's items, loaded before phase 0 so their latency overlaps
    // it; the loads take no branch (an empty item reads entry 0 and drops it), so all of them
    // are in flight together
    uint32_t pw[NITEMS];
    int rr[NITEMS];
    int64_t tt[NITEMS];
#pragma unroll
    for (int q = 0; q < NITEMS; ++q) {
        // the host guarantees that NITEMS * NBT / NR covers the longest adjacency list
        const int idx = threadIdx.x + q * NBT;
        const int r = idx % NR, j = idx / NR;
        const int La = ap[r + 1] - ap[r];
        const bool ok = j < La && !is_long_row(La, rp[r + 1] - rp[r]);  // long rows: own workgroups
        rr[q] = ok ? r : -1;
        tt[q] = ok ? static_cast<int64_t>(ap[r]) + j : 0;
        pw[q] = pk[tt[q]];
    }
    __syncthreads();

    // phase 0: edge vector per slot (row-interleaved, no search), accumulators cleared
    for (int idx = threadIdx.x; idx < NR * *maxlen; idx += NBT) {
        const int r = idx % NR, k = idx / NR;
        if (k >= rp[r + 1] - rp[r]) continue;
        const int w = rp[r] - w0 + k;
        const int64_t i = r0 + r;
        const int64_t col = col_idx[w0 + w];
        if (col == i) dslot[r] = w;
        accK[w] = A(0);
        accM[w] = A(0);
        // a long row's slots are marked: neither graded nor stored here
        shK[w] = is_long_row(ap[r + 1] - ap[r], rp[r + 1] - rp[r]) ? INT32_MIN : 0;
        shM[w] = 0;
        Vec4<T> v;
        v.x = static_cast<T>(coords[col * DIM] - coords[i * DIM]);
        v.y = static_cast<T>(coords[col * DIM + 1] - coords[i * DIM + 1]);
        v.z = DIM == 3 ? static_cast<T>(coords[col * DIM + (DIM - 1)] - coords[i * DIM + (DIM - 1)]) : T(0);
        v.w = T(0);
        f[w] = v;
    }
    __syncthreads();

    // phase 1a: rows of the adjacent elements, in registers; per-slot maxima
    const float tau_abs = static_cast<float>(fb.tau_abs), tau_cond = static_cast<float>(fb.tau_cond);
    constexpr int MQ = QN > 0 ? DIM + 1 : 1;  // mass values per row: one per node with a rule, else one
    T kr[NITEMS][NLB], mr[NITEMS][MQ];
    int64_t routed = 0;
#pragma unroll
    for (int q = 0; q < NITEMS; ++q) {
        const int r = rr[q];
        if (r < 0) continue;
        const int64_t t = tt[q];
        const int s0 = rp[r] - w0;
        const uint32_t p = pw[q];
        T ck = T(1), cm = T(1);
        T cmq[QN > 0 ? QN : 1];
        if constexpr (COEF && QN == 0) {
            const int64_t e = adj[t] >> 2;
            if (cK) ck = cK[e];
            if (cM) cm = cM[e];
        }
        if constexpr (QN > 0) {
            const int64_t e = adj[t] >> 2;
            T sk = T(0);
#pragma unroll
            for (int iq = 0; iq < QN; ++iq) {
                sk += cK ? cK[e * QN + iq] : T(1);
                cmq[iq] = cM ? cM[e * QN + iq] : T(1);
            }
            ck = sk * static_cast<T>(1.0 / QN);  // equal weights: the weighted mean of the stiffness coefficient
        }
        T u[DIM][DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const Vec4<T> v = f[s0 + static_cast<int>((p >> (2 + 8 * k)) & 255)];
            u[k][0] = v.x;
            u[k][1] = v.y;
            if constexpr (DIM == 3) u[k][2] = v.z;
        }
        P1Geom<DIM, T> g;
        p1_geom_edges<DIM, T>(u, g);
        bool route = false;
        if constexpr (sizeof(T) == 4) route = route32(g.det, g.absterms, g.shape2, tau_abs, tau_cond, fb.enable);
        T adet_t = fabs(g.det);
        double adet_d = 0.0;
        if (route) {
            // FP64 recomputation from the coordinates of the row's node and the three others
            const int64_t i = r0 + r;
            double ev[DIM][DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const int64_t col = col_idx[w0 + s0 + static_cast<int>((p >> (2 + 8 * k)) & 255)];
#pragma unroll
                for (int c = 0; c < DIM; ++c) ev[k][c] = coords[col * DIM + c] - coords[i * DIM + c];
            }
            double kd[NLB], md;
            origin_row_f64<DIM>(ev, ck, cm, kd, md, adet_d);
#pragma unroll
            for (int b = 0; b < NLB; ++b) kr[q][b] = static_cast<T>(kd[b]);
            mr[q][0] = static_cast<T>(md);
            if ((p & 3) == 0) ++routed;  // count each element once, at its first node's row
        } else {
            origin_row<DIM, T>(g, ck, cm, kr[q], mr[q][0]);
        }
        if constexpr (QN > 0) {
            // mass row by the rule: |det| sum_q w cM_q lam_a(q) lam_b(q), b = the row's node,
            // then the other nodes in local order
            const int a = static_cast<int>(p & 3);
            T ms[NLB];
#pragma unroll
            for (int b = 0; b < NLB; ++b) ms[b] = T(0);
#pragma unroll
            for (int iq = 0; iq < QN; ++iq) {
                const T wl = static_cast<T>(quad_weight<DIM, QN>() * QuadRule<DIM, QN>::lam(iq, a)) * cmq[iq];
#pragma unroll
                for (int b = 0; b < NLB; ++b) {
                    const int lb = b == 0 ? a : (b - 1 < a ? b - 1 : b);
                    ms[b] = fmaT(wl, static_cast<T>(QuadRule<DIM, QN>::lam(iq, lb)), ms[b]);
                }
            }
#pragma unroll
            for (int b = 0; b < NLB; ++b)
                mr[q][b] = route ? static_cast<T>(adet_d * static_cast<double>(ms[b])) : adet_t * ms[b];
        }
        const int sd = dslot[r];
        atomicMax(reinterpret_cast<uint32_t*>(shK + sd), Exact<T>::mag(kr[q][0]));
        if constexpr (QN > 0) atomicMax(reinterpret_cast<uint32_t*>(shM + sd), Exact<T>::mag(mr[q][0]));
        else atomicMax(reinterpret_cast<uint32_t*>(shM + sd), Exact<T>::mag(mr[q][0] + mr[q][0]));
        const uint32_t mm = Exact<T>::mag(mr[q][0]);
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const int s = s0 + static_cast<int>((p >> (2 + 8 * k)) & 255);
            atomicMax(reinterpret_cast<uint32_t*>(shK + s), Exact<T>::mag(kr[q][1 + k]));
            atomicMax(reinterpret_cast<uint32_t*>(shM + s), QN > 0 ? Exact<T>::mag(mr[q][QN > 0 ? 1 + k : 0]) : mm);
        }
    }
    if (routed) count_add(d_counters, 0, routed);
    __syncthreads();
    // per-slot grid: maximum bits -> shift
    for (int w = threadIdx.x; w < W; w += NBT) {
        if (shK[w] == INT32_MIN) continue;
        shK[w] = Exact<T>::shift(static_cast<uint32_t>(shK[w]));
        shM[w] = Exact<T>::shift(static_cast<uint32_t>(shM[w]));
    }
    __syncthreads();

    // phase 1b: exact accumulation on each slot's grid
#pragma unroll
    for (int q = 0; q < NITEMS; ++q) {
        const int r = rr[q];
        if (r < 0) continue;
        const int s0 = rp[r] - w0;
        const int sd = dslot[r];
        atomicAdd(accK + sd, Exact<T>::quant(kr[q][0], shK[sd]));
        if constexpr (QN > 0) atomicAdd(accM + sd, Exact<T>::quant(mr[q][0], shM[sd]));
        else atomicAdd(accM + sd, Exact<T>::quant(mr[q][0] + mr[q][0], shM[sd]));
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const int s = s0 + static_cast<int>((pw[q] >> (2 + 8 * k)) & 255);
            atomicAdd(accK + s, Exact<T>::quant(kr[q][1 + k], shK[s]));
            atomicAdd(accM + s, Exact<T>::quant(mr[q][QN > 0 ? 1 + k : 0], shM[s]));
        }
    }
    __syncthreads();

    // phase 2: one slot per thread, coalesced stores
    for (int w = threadIdx.x; w < W; w += NBT) {
        if (shK[w] == INT32_MIN) continue;
        valsK[w0 + w] = Exact<T>::back(accK[w], shK[w]);
        if (valsM) valsM[w0 + w] = Exact<T>::back(accM[w], shM[w]);
    }
}

// LDS of one FP32 numeric block: per slot an edge vector, the two integer sums and the slot's
// row; per row the window bounds and the two row maxima
template <int DIM>
constexpr size_t numeric_lds_bytes_f32(int nr, int wmax) {
    return static_cast<size_t>(wmax) * (sizeof(Vec4<float>) + 2 * sizeof(uint64_t) + 1) +
           static_cast<size_t>(3 * (nr + 1) + 1) * 4;
}

// FP32 numeric assembly, NR rows per block of NT threads; thread t owns row t % NR: its
// adjacency entries j = t / NR + q NT / NR (q < NITEMS) and its slots k = t / NR + u NT / NR.
//   round trip 1  every load that depends on nothing: the window bounds, the row's adjacency
//                 offsets, diagonal position and node coordinates (the entries' packed words
//                 follow as soon as the offsets arrive);
//   round trips 2, 3  the columns of the thread's slots, then their coordinates (two slots of
//                 a row per pass, all loads in flight), giving every slot the edge vector from
//                 its row's node to its column's node (FP64 difference rounded once) in LDS;
//   phase 1a  every entry computes its element's row of K_e and M_e in registers (geometry
//             with the fast determinant, routed elements in FP64); every thread enters the
//             largest magnitude of its contributions into its row's maximum (one LDS atomic per
//             matrix);
//   phase 1b  every contribution is rounded onto its row's grid (RowGrid32) and added as a
//             64-bit integer: exact, so the order of the adds does not matter; a thread adds
//             its entries' diagonal contributions in registers first and enters them with one
//             atomic each;
//   phase 2   one slot per thread converts its sums and stores them (coalesced).
// A row that receives a non-finite contribution (a degenerate element, or a non-finite
// coefficient) is NaN in every slot.
template <int DIM, bool COEF, int NR, int NT, int QN = 0>
__device__ __forceinline__ void numeric_block_f32(int64_t r0, int64_t nn, const double* __restrict__ coords,
                                                  const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col_idx,
                                                  const int32_t* __restrict__ aptr, const int32_t* __restrict__ adj,
                                                  const uint32_t* __restrict__ pk, const int32_t* __restrict__ dpos,
                                                  const float* __restrict__ cK, const float* __restrict__ cM,
                                                  float* __restrict__ valsK, float* __restrict__ valsM,
                                                  const Fallback& fb, int64_t* d_counters, int32_t* bcnt, int wmax) {
    constexpr int NLB = DIM + 1;
    constexpr int JS = NT / NR;  // stride of a thread's entries and slots within its row
    using G = RowGrid32;
    extern __shared__ __align__(16) unsigned char smem[];
    Vec4<float>* f = reinterpret_cast<Vec4<float>*>(smem);         // [wmax] edge vector per slot
    uint64_t* accK = reinterpret_cast<uint64_t*>(f + wmax);         // [wmax]
    uint64_t* accM = accK + wmax;                                   // [wmax]
    int32_t* rp = reinterpret_cast<int32_t*>(accM + wmax);          // [NR + 1]
    uint32_t* rmK = reinterpret_cast<uint32_t*>(rp + (NR + 1));     // [NR + 1] row maxima (bits of |x|)
    uint32_t* rmM = rmK + (NR + 1);                                 // [NR + 1]
    int32_t* nrouted = reinterpret_cast<int32_t*>(rmM + (NR + 1));  // [1] the block's routed elements
    uint8_t* rowof = reinterpret_cast<uint8_t*>(nrouted + 1);       // [wmax] row of each slot
    static_assert(lds_carve_aligned<Vec4<float>, uint64_t, uint64_t, int32_t, uint32_t, uint32_t, int32_t, uint8_t>(),
                  "FP32 numeric LDS carve-out: every array naturally aligned");
    static_assert((NR & (NR - 1)) == 0 && NT % NR == 0 && NR <= 256, "a thread's items share one row");
    static_assert(NITEMS * JS >= 1, "items per row");

    const int nr = static_cast<int>((r0 + NR < nn) ? NR : nn - r0);
    const int t = static_cast<int>(threadIdx.x);
    const int r = t % NR, jt = t / NR;
    const int64_t row = r0 + (r < nr ? r : nr - 1);  // in bounds for the loads of rows past the end

    // round trip 1 (no load waits for another)
    const int32_t rpv = row_ptr[r0 + (t <= nr ? t : nr)];
    const int32_t a0v = aptr[row], a1v = aptr[row + 1];
    const int32_t dpv = dpos[row];
    double pi[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) pi[c] = coords[row * DIM + c];
    const int L = r < nr ? a1v - a0v : 0;  // elements around the row's node
    bool okq[NITEMS];
#pragma unroll
    for (int q = 0; q < NITEMS; ++q) okq[q] = jt + q * JS < L;  // the host keeps NITEMS * JS >= L
    // the entries' packed words (an empty item reads entry 0 and drops it)
    uint32_t pw[NITEMS];
    int64_t tt[NITEMS];
#pragma unroll
    for (int q = 0; q < NITEMS; ++q) {
        tt[q] = okq[q] ? static_cast<int64_t>(a0v) + jt + q * JS : 0;
        pw[q] = pk[tt[q]];
    }
    if (t <= NR) rp[t] = rpv;
    if (t < NR) {
        rmK[t] = 0u;
        rmM[t] = 0u;
    }
    if (t == 0) *nrouted = 0;
    __syncthreads();
    const int32_t w0 = rp[0];
    const int W = rp[nr] - w0;
    const int s0 = rp[r] - w0;
    const int len = rp[r + 1] - rp[r];  // 0 for rows past the end
    if (is_long_row(L, len)) {  // a long row: assembled by its own workgroup, not here
#pragma unroll
        for (int q = 0; q < NITEMS; ++q) okq[q] = false;
        if (jt == 0) rmK[r] = G::SKIP;
    }

    // coefficients of the thread's entries (their loads overlap the slot passes)
    float ckq[NITEMS], cmq0[NITEMS];
    float cmq[QN > 0 ? NITEMS : 1][QN > 0 ? QN : 1];
#pragma unroll
    for (int q = 0; q < NITEMS; ++q) {
        ckq[q] = 1.0f;
        cmq0[q] = 1.0f;
        if constexpr (COEF || QN > 0) {
            const int64_t e = okq[q] ? (adj[tt[q]] >> 2) : 0;
            if constexpr (QN == 0) {
                if (cK) ckq[q] = cK[e];
                if (cM) cmq0[q] = cM[e];
            } else {
                float sk = 0.0f;
#pragma unroll
                for (int iq = 0; iq < QN; ++iq) {
                    sk += cK ? cK[e * QN + iq] : 1.0f;
                    cmq[q][iq] = cM ? cM[e * QN + iq] : 1.0f;
                }
                ckq[q] = sk * static_cast<float>(1.0 / QN);  // equal weights: the mean of the stiffness coefficient
            }
        }
    }

    // round trips 2 and 3: edge vectors of the thread's slots, two per pass; sums cleared
    for (int k0 = jt; k0 < len; k0 += 2 * JS) {
        const int k1 = k0 + JS;
        const bool two = k1 < len;
        const int64_t c0 = col_idx[w0 + s0 + k0];
        const int64_t c1 = col_idx[w0 + s0 + (two ? k1 : k0)];
        double x0[DIM], x1[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            x0[c] = coords[c0 * DIM + c];
            x1[c] = coords[c1 * DIM + c];
        }
        Vec4<float> v;  // the edge vector, and the column's node id in the fourth lane
        v.x = static_cast<float>(x0[0] - pi[0]);
        v.y = static_cast<float>(x0[1] - pi[1]);
        v.z = DIM == 3 ? static_cast<float>(x0[DIM - 1] - pi[DIM - 1]) : 0.0f;
        v.w = __int_as_float(static_cast<int32_t>(c0));
        f[s0 + k0] = v;
        accK[s0 + k0] = 0;
        accM[s0 + k0] = 0;
        rowof[s0 + k0] = static_cast<uint8_t>(r);
        if (two) {
            v.x = static_cast<float>(x1[0] - pi[0]);
            v.y = static_cast<float>(x1[1] - pi[1]);
            v.z = DIM == 3 ? static_cast<float>(x1[DIM - 1] - pi[DIM - 1]) : 0.0f;
            v.w = __int_as_float(static_cast<int32_t>(c1));
            f[s0 + k1] = v;
            accK[s0 + k1] = 0;
            accM[s0 + k1] = 0;
            rowof[s0 + k1] = static_cast<uint8_t>(r);
        }
    }
    __syncthreads();

    // phase 1a: rows of the adjacent elements in registers; the thread's maxima
    const float tau_abs = static_cast<float>(fb.tau_abs), tau_cond = static_cast<float>(fb.tau_cond);
    constexpr int MQ = QN > 0 ? DIM + 1 : 1;  // mass values per row: one per node with a rule, else one
    float kr[NITEMS][NLB], mr[NITEMS][MQ];
    int64_t routed = 0;
    float mk = 0.0f, mm = 0.0f;
    bool finite = true;
#pragma unroll
    for (int q = 0; q < NITEMS; ++q) {
        if (!okq[q]) continue;
        const uint32_t p = pw[q];
        const float ck = ckq[q], cm = cmq0[q];
        float u[DIM][DIM];
        int32_t cn[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const Vec4<float> v = f[s0 + static_cast<int>((p >> (2 + 8 * k)) & 255)];
            u[k][0] = v.x;
            u[k][1] = v.y;
            if constexpr (DIM == 3) u[k][2] = v.z;
            cn[k] = __float_as_int(v.w);
        }
        P1Geom<DIM, float> g;
        p1_geom_edges_fast<DIM>(u, g);
        const bool route = route32(g.det, g.absterms, g.shape2, tau_abs, tau_cond, fb.enable);
        const float adet_t = fabsf(g.det);
        double adet_d = 0.0;
        if (route) {
            // FP64 recomputation from the coordinates of the row's node (read again: a rare path
            // that should not keep them in registers) and of the three others (their node ids
            // came with the edge vectors: one round trip)
            double ev[DIM][DIM];
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const int64_t col = cn[k];
#pragma unroll
                for (int c = 0; c < DIM; ++c) ev[k][c] = coords[col * DIM + c] - coords[row * DIM + c];
            }
            double kd[NLB], md;
            origin_row_f64<DIM>(ev, ck, cm, kd, md, adet_d);
#pragma unroll
            for (int b = 0; b < NLB; ++b) kr[q][b] = static_cast<float>(kd[b]);
            mr[q][0] = static_cast<float>(md);
            if ((p & 3) == 0) ++routed;  // count each element once, at its first node's row
        } else {
            origin_row<DIM, float>(g, ck, cm, kr[q], mr[q][0]);
        }
        if constexpr (QN > 0) {
            // mass row by the rule: |det| sum_q w cM_q lam_a(q) lam_b(q), b = the row's node,
            // then the other nodes in local order
            const int a = static_cast<int>(p & 3);
            float ms[NLB];
#pragma unroll
            for (int b = 0; b < NLB; ++b) ms[b] = 0.0f;
#pragma unroll
            for (int iq = 0; iq < QN; ++iq) {
                const float wl =
                    static_cast<float>(quad_weight<DIM, QN>() * QuadRule<DIM, QN>::lam(iq, a)) * cmq[QN > 0 ? q : 0][iq];
#pragma unroll
                for (int b = 0; b < NLB; ++b) {
                    const int lb = b == 0 ? a : (b - 1 < a ? b - 1 : b);
                    ms[b] = fmaf(wl, static_cast<float>(QuadRule<DIM, QN>::lam(iq, lb)), ms[b]);
                }
            }
#pragma unroll
            for (int b = 0; b < NLB; ++b) {
                mr[q][b] = route ? static_cast<float>(adet_d * static_cast<double>(ms[b])) : adet_t * ms[b];
                mm = fmaxf(mm, fabsf(mr[q][b]));
            }
        } else {
            mm = fmaxf(mm, fabsf(mr[q][0] + mr[q][0]));  // the diagonal takes 2 mo
        }
#pragma unroll
        for (int b = 0; b < NLB; ++b) mk = fmaxf(mk, fabsf(kr[q][b]));
        // K_e's row is kf times dot products of finite cofactors: all of it is finite exactly
        // when its diagonal entry kf |c_0|^2 is; the mass row carries |det| in its first entry
        finite = finite && __builtin_isfinite(kr[q][0]) && __builtin_isfinite(mr[q][0]);
    }
    if (routed) atomicAdd(nrouted, static_cast<int32_t>(routed));
    if (okq[0]) {  // items are dealt in order: a thread with any entry has its first
        atomicMax(rmK + r, finite ? G::mag(mk) : G::POISON);
        atomicMax(rmM + r, G::mag(mm));
    }
    __syncthreads();
    if (t == 0) {  // the block's routed count: into its slot of the launch's array, else the counter
        const int32_t nb = *nrouted;
        if (bcnt) bcnt[blockIdx.x] = nb;
        else if (nb) count_add(d_counters, 0, nb);
    }

    // phase 1b: every contribution onto its row's grid, exact integer sums
    const uint32_t mKr = rmK[r];
    if (okq[0] && mKr != G::POISON) {
        const int shK = G::shift(mKr), shM = G::shift(rmM[r]);
        uint64_t dK = 0, dM = 0;
#pragma unroll
        for (int q = 0; q < NITEMS; ++q) {
            if (!okq[q]) continue;
            dK += G::quant(kr[q][0], shK);
            uint64_t qm = 0;
            if constexpr (QN > 0) dM += G::quant(mr[q][0], shM);
            else {
                qm = G::quant(mr[q][0], shM);
                dM += qm + qm;
            }
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const int sl = s0 + static_cast<int>((pw[q] >> (2 + 8 * k)) & 255);
                atomicAdd(accK + sl, G::quant(kr[q][1 + k], shK));
                atomicAdd(accM + sl, QN > 0 ? G::quant(mr[q][QN > 0 ? 1 + k : 0], shM) : qm);
            }
        }
        const int sd = s0 + dpv;
        atomicAdd(accK + sd, dK);
        atomicAdd(accM + sd, dM);
    }
    __syncthreads();

    // phase 2: one slot per thread, coalesced stores
    for (int w = t; w < W; w += NT) {
        const int rr = rowof[w];
        const uint32_t mK = rmK[rr];
        if (mK == G::SKIP) continue;
        const bool poison = mK == G::POISON;
        valsK[w0 + w] = poison ? __builtin_nanf("") : G::back(accK[w], G::shift(mK));
        if (valsM) valsM[w0 + w] = poison ? __builtin_nanf("") : G::back(accM[w], G::shift(rmM[rr]));
    }
}

// waves per SIMD the numeric kernels are compiled for: the FP32 body with constant
// coefficients and 8 or more rows per block fits 64 VGPRs (8 waves) without spilling; the
// other variants keep the compiler's choice
template <int QN, bool COEF, int NR>
constexpr int numeric32_waves() {
    return QN == 0 && !COEF && NR >= 8 ? 8 : 1;
}

template <int DIM, typename T, bool COEF, int NR, int QN = 0>
__global__ __launch_bounds__(NBT) void k_numeric(int64_t nn, const double* __restrict__ coords,
                                                 const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                                                 const int32_t* __restrict__ aptr, const int32_t* __restrict__ adj,
                                                 const uint32_t* __restrict__ pk, const T* __restrict__ cK,
                                                 const T* __restrict__ cM, T* __restrict__ valsK, T* __restrict__ valsM,
                                                 Fallback fb, int64_t* d_counters, int wmax) {
    numeric_block<DIM, T, COEF, NR, QN>(static_cast<int64_t>(blockIdx.x) * NR, nn, coords, row_ptr, col_idx, aptr,
                                        adj, pk, cK, cM, valsK, valsM, fb, d_counters, wmax);
}

template <int DIM, bool COEF, int NR, int NT, int QN = 0>
__global__ __launch_bounds__(NT, (numeric32_waves<QN, COEF, NR>())) void k_numeric32(
    int64_t nn, const double* __restrict__ coords, const int32_t* __restrict__ row_ptr,
    const int32_t* __restrict__ col_idx, const int32_t* __restrict__ aptr, const int32_t* __restrict__ adj,
    const uint32_t* __restrict__ pk, const int32_t* __restrict__ dpos, const float* __restrict__ cK,
    const float* __restrict__ cM, float* __restrict__ valsK, float* __restrict__ valsM, Fallback fb,
    int64_t* d_counters, int32_t* bcnt, int wmax) {
    numeric_block_f32<DIM, COEF, NR, NT, QN>(static_cast<int64_t>(blockIdx.x) * NR, nn, coords, row_ptr, col_idx,
                                             aptr, adj, pk, dpos, cK, cM, valsK, valsM, fb, d_counters, bcnt, wmax);
}


// block b of a multi-mesh launch belongs to the job whose block range holds b
__device__ __forceinline__ const NumericJob& job_of_block(const NumericJob* __restrict__ jobs, int njobs, int64_t b) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].block0 <= b) lo = mid;
        else hi = mid - 1;
    }
    return jobs[lo];
}

// The numeric phase of several meshes in one launch: block b belongs to the job whose block
// range holds b (binary search over the jobs' first blocks); every job keeps its own
// structure, coordinates, outputs, routing thresholds and counters, and its rows are
// computed exactly as by k_numeric / k_numeric32, so a job's values do not depend on its batch.
template <int DIM, int NR>
__global__ __launch_bounds__(NBT) void k_numeric_jobs(const NumericJob* __restrict__ jobs, int njobs, int wmax) {
    const int64_t b = blockIdx.x;
    const NumericJob& j = job_of_block(jobs, njobs, b);
    numeric_block<DIM, double, false, NR>((b - j.block0) * NR, j.nn, j.coords, j.row_ptr, j.col_idx, j.aptr, j.adj,
                                          j.pk, nullptr, nullptr, static_cast<double*>(j.valsK),
                                          static_cast<double*>(j.valsM), j.fb, j.counters, wmax);
}

template <int DIM, int NR, int NT>
__global__ __launch_bounds__(NT, (numeric32_waves<0, false, NR>())) void k_numeric_jobs32(
    const NumericJob* __restrict__ jobs, int njobs, int wmax) {
    const int64_t b = blockIdx.x;
    const NumericJob& j = job_of_block(jobs, njobs, b);
    numeric_block_f32<DIM, false, NR, NT>((b - j.block0) * NR, j.nn, j.coords, j.row_ptr, j.col_idx, j.aptr,
                                          j.adj, j.pk, j.dpos, nullptr, nullptr, static_cast<float*>(j.valsK),
                                          static_cast<float*>(j.valsM), j.fb, j.counters, nullptr, wmax);
}

// ---------------------------------------------------------------------------- long rows, numeric
// One workgroup per long row (at most LCAP slots): every adjacency entry's row of K_e and M_e
// in FP64 from the coordinates of the row's node and of the element's other nodes (reached
// through the entry's slot word), entered in two passes -- the largest magnitude of each
// slot, then every contribution on the slot's LongGrid as a 64-bit integer (exact, so the
// result does not depend on the order of the adds).  FP32 outputs round the FP64 sum once.
// The routed counter counts, at each element's first node, the elements the FP32 geometry
// would route, as the row-block kernels do.
template <int DIM, typename T, bool COEF, int QN>
__device__ __forceinline__ void long_entry(int64_t row, int64_t w0, int sd, uint32_t p, int64_t e,
                                           const double* __restrict__ coords, const int32_t* __restrict__ col_idx,
                                           const T* __restrict__ cK, const T* __restrict__ cM, double (&kd)[DIM + 1],
                                           double (&md)[DIM + 1], int (&sl)[DIM + 1], double (&ev)[DIM][DIM]) {
    constexpr int NLB = DIM + 1;
    sl[0] = sd;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        sl[1 + k] = static_cast<int>((p >> (2 + 8 * k)) & 255);
        const int64_t col = col_idx[w0 + sl[1 + k]];
#pragma unroll
        for (int c = 0; c < DIM; ++c) ev[k][c] = coords[col * DIM + c] - coords[row * DIM + c];
    }
    double ck = 1.0, cm = 1.0;
    double cmq[QN > 0 ? QN : 1];
    if constexpr (COEF && QN == 0) {
        if (cK) ck = static_cast<double>(cK[e]);
        if (cM) cm = static_cast<double>(cM[e]);
    }
    if constexpr (QN > 0) {
        double sk = 0.0;
#pragma unroll
        for (int iq = 0; iq < QN; ++iq) {
            sk += cK ? static_cast<double>(cK[e * QN + iq]) : 1.0;
            cmq[iq] = cM ? static_cast<double>(cM[e * QN + iq]) : 1.0;
        }
        ck = sk * (1.0 / QN);
    }
    double mo, adet;
    origin_row_f64<DIM>(ev, ck, cm, kd, mo, adet);
    if constexpr (QN > 0) {
        const int a = static_cast<int>(p & 3);
#pragma unroll
        for (int b = 0; b < NLB; ++b) md[b] = 0.0;
#pragma unroll
        for (int iq = 0; iq < QN; ++iq) {
            const double wl = quad_weight<DIM, QN>() * QuadRule<DIM, QN>::lam(iq, a) * cmq[iq];
#pragma unroll
            for (int b = 0; b < NLB; ++b) {
                const int lb = b == 0 ? a : (b - 1 < a ? b - 1 : b);
                md[b] = fma(wl, QuadRule<DIM, QN>::lam(iq, lb), md[b]);
            }
        }
#pragma unroll
        for (int b = 0; b < NLB; ++b) md[b] *= adet;
    } else {
        md[0] = mo + mo;
#pragma unroll
        for (int b = 1; b < NLB; ++b) md[b] = mo;
    }
}

template <int DIM, typename T, bool COEF, int QN>
__global__ __launch_bounds__(LT) void k_numeric_long(const int32_t* __restrict__ lrows,
                                                     const double* __restrict__ coords,
                                                     const int32_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col_idx,
                                                     const int32_t* __restrict__ aptr, const int32_t* __restrict__ adj,
                                                     const uint32_t* __restrict__ pk, const int32_t* __restrict__ dpos,
                                                     const T* __restrict__ cK, const T* __restrict__ cM,
                                                     T* __restrict__ valsK, T* __restrict__ valsM, Fallback fb,
                                                     int64_t* d_counters) {
    constexpr int NLB = DIM + 1;
    using G = LongGrid;
    __shared__ uint32_t mxK[LCAP], mxM[LCAP];
    __shared__ int32_t shK[LCAP], shM[LCAP];
    __shared__ unsigned long long accK[LCAP], accM[LCAP];
    const int t = static_cast<int>(threadIdx.x);
    const int64_t row = lrows[blockIdx.x];
    const int64_t w0 = row_ptr[row];
    const int len = row_ptr[row + 1] - static_cast<int>(w0);  // at most LCAP
    const int64_t a0 = aptr[row];
    const int L = aptr[row + 1] - static_cast<int>(a0);
    const int sd = dpos[row];
    const int hb = G::headroom(L);
    for (int k = t; k < LCAP; k += LT) {
        mxK[k] = mxM[k] = 0u;
        accK[k] = accM[k] = 0ull;
    }
    __syncthreads();
    int64_t routed = 0;
    for (int j = t; j < L; j += LT) {  // pass 1: each slot's largest magnitude
        const uint32_t p = pk[a0 + j];
        const int64_t e = static_cast<uint32_t>(adj[a0 + j]) >> 2;
        double kd[NLB], md[NLB], ev[DIM][DIM];
        int sl[NLB];
        long_entry<DIM, T, COEF, QN>(row, w0, sd, p, e, coords, col_idx, cK, cM, kd, md, sl, ev);
#pragma unroll
        for (int b = 0; b < NLB; ++b) {
            atomicMax(mxK + sl[b], G::mag(kd[b]));
            atomicMax(mxM + sl[b], G::mag(md[b]));
        }
        if constexpr (sizeof(T) == 4) {
            if ((p & 3) == 0) {  // what the FP32 path would route, counted at the element's first node
                float u[DIM][DIM];
#pragma unroll
                for (int k = 0; k < DIM; ++k)
#pragma unroll
                    for (int c = 0; c < DIM; ++c) u[k][c] = static_cast<float>(ev[k][c]);
                P1Geom<DIM, float> g;
                p1_geom_edges_fast<DIM>(u, g);
                if (route32(g.det, g.absterms, g.shape2, static_cast<float>(fb.tau_abs), static_cast<float>(fb.tau_cond),
                            fb.enable))
                    ++routed;
            }
        }
    }
    if (routed) count_add(d_counters, 0, routed);
    __syncthreads();
    for (int k = t; k < len; k += LT) {
        shK[k] = mxK[k] == G::POISON ? 0 : G::shift(mxK[k], hb);
        shM[k] = mxM[k] == G::POISON ? 0 : G::shift(mxM[k], hb);
    }
    __syncthreads();
    for (int j = t; j < L; j += LT) {  // pass 2: exact sums
        const uint32_t p = pk[a0 + j];
        const int64_t e = static_cast<uint32_t>(adj[a0 + j]) >> 2;
        double kd[NLB], md[NLB], ev[DIM][DIM];
        int sl[NLB];
        long_entry<DIM, T, COEF, QN>(row, w0, sd, p, e, coords, col_idx, cK, cM, kd, md, sl, ev);
#pragma unroll
        for (int b = 0; b < NLB; ++b) {
            if (mxK[sl[b]] != G::POISON) atomicAdd(accK + sl[b], G::quant(kd[b], shK[sl[b]]));
            if (mxM[sl[b]] != G::POISON) atomicAdd(accM + sl[b], G::quant(md[b], shM[sl[b]]));
        }
    }
    __syncthreads();
    for (int k = t; k < len; k += LT) {
        valsK[w0 + k] = mxK[k] == G::POISON ? static_cast<T>(NAN) : static_cast<T>(G::back(accK[k], shK[k]));
        if (valsM) valsM[w0 + k] = mxM[k] == G::POISON ? static_cast<T>(NAN) : static_cast<T>(G::back(accM[k], shM[k]));
    }
}

// ---------------------------------------------------------------------------- host
namespace {

// Device memory of the structures comes from one stream-ordered memory pool per device that
// keeps released blocks for reuse (no release threshold): a build after another structure
// was released takes its pages back without mapping new ones, and a release enqueued on a
// stream (hipFreeAsync) waits for no device work.  pf_csr_destroy trims the pool.
constexpr int MAX_POOL_DEVICES = 64;
std::mutex g_pool_mu;
hipMemPool_t g_pool[MAX_POOL_DEVICES] = {};

pf_status pool_of_current(hipMemPool_t* out) {
    int dev = 0;
    PF_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_POOL_DEVICES) return fail(PF_EINVAL, "device index beyond the pool table");
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_pool[dev]) {
        hipMemPoolProps props = {};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t pool = nullptr;
        PF_HIP_TRY(hipMemPoolCreate(&pool, &props));
        uint64_t keep = UINT64_MAX;
        PF_HIP_TRY(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
        g_pool[dev] = pool;
    }
    *out = g_pool[dev];
    return PF_OK;
}

// an array of `need` elements on stream s; an existing smaller one is released first (after
// a device synchronisation: work on any stream may still read it)
template <typename P>
pf_status grow(P*& p, int64_t& cap, int64_t need, hipStream_t s) {
    if (need <= cap && p) return PF_OK;
    if (p) {
        PF_HIP_TRY(hipDeviceSynchronize());
        PF_HIP_TRY(hipFreeAsync(p, s));
        p = nullptr;
    }
    cap = 0;
    hipMemPool_t pool = nullptr;
    if (pf_status st = pool_of_current(&pool)) return st;
    const size_t bytes = sizeof(P) * static_cast<size_t>(need > 0 ? need : 1);
    hipError_t e = hipMallocFromPoolAsync(reinterpret_cast<void**>(&p), bytes, pool, s);
    if (e != hipSuccess) {
        p = nullptr;
        return fail(PF_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    }
    cap = need;
    return PF_OK;
}

// release an array in the order of stream s
template <typename P>
void drop(P*& p, int64_t& cap, hipStream_t s) {
    if (p) (void)hipFreeAsync(p, s);
    p = nullptr;
    cap = 0;
}

// pinned host words for the status readbacks, recycled across handles (pinning and unpinning
// host memory is slow, and its release may wait for the device)
std::mutex g_pin_mu;
std::vector<int64_t*> g_pin_free;

pf_status pinned_words(int64_t** out) {
    {
        std::lock_guard<std::mutex> lk(g_pin_mu);
        if (!g_pin_free.empty()) {
            *out = g_pin_free.back();
            g_pin_free.pop_back();
            return PF_OK;
        }
    }
    PF_HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(out), INFO_WORDS * sizeof(int64_t)));
    return PF_OK;
}

void recycle_pinned(int64_t* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_pin_mu);
    g_pin_free.push_back(p);
}

// The build scratch of one device: a block that one build at a time borrows and hands back
// by recording an event on its stream (no allocation or release call, each of which costs the
// host tens of microseconds); the next borrower's stream waits for that event on the device.
// A build that finds the block in use allocates scratch of its own from the pool.
struct ScratchArena {
    unsigned char* p = nullptr;
    int64_t cap = 0;
    bool busy = false;
    hipEvent_t done = nullptr;  // recorded when the last borrower's build stopped using it
    bool recorded = false;
};
ScratchArena g_arena[MAX_POOL_DEVICES];

// scratch of `bytes` for a build on stream s: the arena's block (*owned = false) or a block
// of the pool's (*owned = true)
pf_status scratch_borrow(int64_t bytes, hipStream_t s, unsigned char** out, bool* owned) {
    int dev = 0;
    PF_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_POOL_DEVICES) return fail(PF_EINVAL, "device index beyond the pool table");
    hipMemPool_t pool = nullptr;
    if (pf_status st = pool_of_current(&pool)) return st;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        ScratchArena& a = g_arena[dev];
        if (!a.busy) {
            a.busy = true;
            if (a.recorded) PF_HIP_TRY(hipStreamWaitEvent(s, a.done, 0));  // the last borrower is done
            if (a.cap < bytes) {
                if (a.p) PF_HIP_TRY(hipFreeAsync(a.p, s));
                a.p = nullptr;
                a.cap = 0;
                const hipError_t e = hipMallocFromPoolAsync(reinterpret_cast<void**>(&a.p), bytes, pool, s);
                if (e != hipSuccess) {
                    a.busy = false;
                    return fail(PF_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
                }
                a.cap = bytes;
            }
            *out = a.p;
            *owned = false;
            return PF_OK;
        }
    }
    const hipError_t e = hipMallocFromPoolAsync(reinterpret_cast<void**>(out), bytes, pool, s);
    if (e != hipSuccess) return fail(PF_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    *owned = true;
    return PF_OK;
}

// hand the scratch back: the arena's block once the work enqueued on s so far is done
void scratch_return(unsigned char* p, bool owned, hipStream_t s) {
    if (!p) return;
    if (owned) {
        (void)hipFreeAsync(p, s);
        return;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_POOL_DEVICES) return;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    ScratchArena& a = g_arena[dev];
    if (!a.done && hipEventCreateWithFlags(&a.done, hipEventDisableTiming) != hipSuccess) a.done = nullptr;
    a.recorded = a.done && hipEventRecord(a.done, s) == hipSuccess;
    if (!a.recorded) (void)hipStreamSynchronize(s);  // no event: wait here instead
    a.busy = false;
}

// release the arena's block of the current device (when no build holds it)
void scratch_trim() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_POOL_DEVICES) return;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    ScratchArena& a = g_arena[dev];
    if (a.busy || !a.p) return;
    if (a.recorded) (void)hipEventSynchronize(a.done);
    (void)hipFreeAsync(a.p, nullptr);
    (void)hipStreamSynchronize(nullptr);
    a.p = nullptr;
    a.cap = 0;
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

template <int DIM, typename T, bool COEF, int NRB, int QN = 0>
pf_status launch_numeric(const pf_csr* c, const double* coords, const void* cK, const void* cM, void* valsK,
                         void* valsM, Fallback f, int64_t* ctr, int wmax, hipStream_t s) {
    const size_t shm = numeric_lds_bytes<DIM, T>(NRB, wmax);
    const unsigned g = static_cast<unsigned>(ceil_div(c->nn, NRB));
    hipLaunchKernelGGL((k_numeric<DIM, T, COEF, NRB, QN>), dim3(g), dim3(NBT), shm, s, c->nn, coords, c->row_ptr,
                       c->col_idx, c->aptr, c->adj, c->pk, static_cast<const T*>(cK), static_cast<const T*>(cM),
                       static_cast<T*>(valsK), static_cast<T*>(valsM), f, ctr, wmax);
    return launch_check("pf_assemble");
}

// largest CSR window of nr consecutive rows starting at a multiple of nr
int window_of(const pf_csr* c, int nr) {
    switch (nr) {
        case 32: return c->wmax_big;
        case 16: return c->wmax_mid;
        case 8: return c->wmax8;
        case 4: return c->wmax_small;
        default: return c->wmax2;
    }
}

// rows per block (FP64): the largest of NR_BIG, NR_MID, NR_SMALL whose window fits the LDS
// budget and whose item budget covers the longest adjacency row
template <int DIM, typename T>
int numeric_rows(const pf_csr* c) {
    if (numeric_lds_bytes<DIM, T>(NR_BIG, c->wmax_big) <= LDS_BYTES && c->max_adj <= NITEMS * NBT / NR_BIG)
        return NR_BIG;
    if (numeric_lds_bytes<DIM, T>(NR_MID, c->wmax_mid) <= LDS_BYTES && c->max_adj <= NITEMS * NBT / NR_MID)
        return NR_MID;
    return NR_SMALL;  // 4 rows of at most MAXROW nonzeros and MAXADJ elements always fit
}

// rows per FP32 block: 8, 16 or 32 threads per row, the fewest that cover the longest
// adjacency row and whose window fits the LDS budget
template <int DIM>
int numeric_rows32(const pf_csr* c) {
    constexpr int R8 = NT32 / 8, R16 = NT32 / 16;
    if (c->max_adj <= NITEMS * 8 && numeric_lds_bytes_f32<DIM>(R8, window_of(c, R8)) <= LDS_BYTES) return R8;
    if (c->max_adj <= NITEMS * 16 && numeric_lds_bytes_f32<DIM>(R16, window_of(c, R16)) <= LDS_BYTES) return R16;
    return NT32 / 32;  // at most NT32 / 32 rows of MAXROW nonzeros: always fits
}

template <int DIM, bool COEF, int NR, int QN = 0>
pf_status launch_numeric32(const pf_csr* c, const double* coords, const void* cK, const void* cM, void* valsK,
                           void* valsM, Fallback f, int64_t* ctr, hipStream_t s) {
    const int wmax = window_of(c, NR);
    const size_t shm = numeric_lds_bytes_f32<DIM>(NR, wmax);
    const unsigned g = static_cast<unsigned>(ceil_div(c->nn, NR));
    // routed counts: every block stores its own in the structure's array of block counts, which
    // one more launch sums (blocks that all add to the one counter serialise on it where many
    // elements route)
    int32_t* bcnt = ctr && f.enable ? c->bcnt : nullptr;
    hipLaunchKernelGGL((k_numeric32<DIM, COEF, NR, NT32, QN>), dim3(g), dim3(NT32), shm, s, c->nn, coords, c->row_ptr,
                       c->col_idx, c->aptr, c->adj, c->pk, c->dpos, static_cast<const float*>(cK),
                       static_cast<const float*>(cM), static_cast<float*>(valsK), static_cast<float*>(valsM), f, ctr,
                       bcnt, wmax);
    if (bcnt) {
        const int64_t gs = ceil_div(static_cast<int64_t>(g), SUM_COUNTS_PER_BLOCK);
        hipLaunchKernelGGL((k_sum_counts<1>), dim3(static_cast<unsigned>(gs < 1 ? 1 : gs)), dim3(256), 0, s, bcnt,
                           static_cast<int64_t>(g), ctr, 0, 0, 0);
    }
    return launch_check("pf_assemble");
}

template <int DIM, bool COEF, int QN = 0>
pf_status numeric_dispatch32(const pf_csr* c, const double* coords, const void* cK, const void* cM, void* valsK,
                             void* valsM, Fallback f, int64_t* ctr, hipStream_t s) {
    const int nr = numeric_rows32<DIM>(c);
    if (nr == NT32 / 8)
        return launch_numeric32<DIM, COEF, NT32 / 8, QN>(c, coords, cK, cM, valsK, valsM, f, ctr, s);
    if (nr == NT32 / 16)
        return launch_numeric32<DIM, COEF, NT32 / 16, QN>(c, coords, cK, cM, valsK, valsM, f, ctr, s);
    return launch_numeric32<DIM, COEF, NT32 / 32, QN>(c, coords, cK, cM, valsK, valsM, f, ctr, s);
}

// the long rows of a structure (none for most meshes): one workgroup each
template <int DIM, typename T, bool COEF, int QN>
pf_status launch_long(const pf_csr* c, const double* coords, const void* cK, const void* cM, void* valsK, void* valsM,
                      Fallback f, int64_t* ctr, hipStream_t s) {
    if (c->nlong == 0) return PF_OK;
    hipLaunchKernelGGL((k_numeric_long<DIM, T, COEF, QN>), dim3(static_cast<unsigned>(c->nlong)), dim3(LT), 0, s,
                       c->lrows, coords, c->row_ptr, c->col_idx, c->aptr, c->adj, c->pk, c->dpos,
                       static_cast<const T*>(cK), static_cast<const T*>(cM), static_cast<T*>(valsK),
                       static_cast<T*>(valsM), f, ctr);
    return launch_check("pf_assemble (long rows)");
}

template <int DIM, typename T>
pf_status numeric_dispatch_rows(const pf_csr* c, const double* coords, const void* cK, const void* cM, void* valsK,
                                void* valsM, Fallback f, int64_t* ctr, hipStream_t s) {
    const bool coef = cK || cM;
    if constexpr (sizeof(T) == 4) {
        return coef ? numeric_dispatch32<DIM, true>(c, coords, cK, cM, valsK, valsM, f, ctr, s)
                    : numeric_dispatch32<DIM, false>(c, coords, cK, cM, valsK, valsM, f, ctr, s);
    }
    switch (numeric_rows<DIM, T>(c)) {
        case NR_BIG:
            return coef ? launch_numeric<DIM, T, true, NR_BIG>(c, coords, cK, cM, valsK, valsM, f, ctr, c->wmax_big, s)
                        : launch_numeric<DIM, T, false, NR_BIG>(c, coords, cK, cM, valsK, valsM, f, ctr, c->wmax_big, s);
        case NR_MID:
            return coef ? launch_numeric<DIM, T, true, NR_MID>(c, coords, cK, cM, valsK, valsM, f, ctr, c->wmax_mid, s)
                        : launch_numeric<DIM, T, false, NR_MID>(c, coords, cK, cM, valsK, valsM, f, ctr, c->wmax_mid, s);
        default:
            return coef ? launch_numeric<DIM, T, true, NR_SMALL>(c, coords, cK, cM, valsK, valsM, f, ctr,
                                                                  c->wmax_small, s)
                        : launch_numeric<DIM, T, false, NR_SMALL>(c, coords, cK, cM, valsK, valsM, f, ctr,
                                                                   c->wmax_small, s);
    }
}

template <int DIM, typename T>
pf_status numeric_dispatch(const pf_csr* c, const double* coords, const void* cK, const void* cM, void* valsK,
                           void* valsM, Fallback f, int64_t* ctr, hipStream_t s) {
    pf_status st = numeric_dispatch_rows<DIM, T>(c, coords, cK, cM, valsK, valsM, f, ctr, s);
    if (st != PF_OK) return st;
    return (cK || cM) ? launch_long<DIM, T, true, 0>(c, coords, cK, cM, valsK, valsM, f, ctr, s)
                      : launch_long<DIM, T, false, 0>(c, coords, cK, cM, valsK, valsM, f, ctr, s);
}

// coefficients at the QN integration points of every element
template <int DIM, typename T, int QN>
pf_status numeric_dispatch_quad_rows(const pf_csr* c, const double* coords, const void* cKq, const void* cMq,
                                     void* valsK, void* valsM, Fallback f, int64_t* ctr, hipStream_t s) {
    if constexpr (sizeof(T) == 4) return numeric_dispatch32<DIM, false, QN>(c, coords, cKq, cMq, valsK, valsM, f, ctr, s);
    switch (numeric_rows<DIM, T>(c)) {
        case NR_BIG:
            return launch_numeric<DIM, T, false, NR_BIG, QN>(c, coords, cKq, cMq, valsK, valsM, f, ctr, c->wmax_big, s);
        case NR_MID:
            return launch_numeric<DIM, T, false, NR_MID, QN>(c, coords, cKq, cMq, valsK, valsM, f, ctr, c->wmax_mid, s);
        default:
            return launch_numeric<DIM, T, false, NR_SMALL, QN>(c, coords, cKq, cMq, valsK, valsM, f, ctr,
                                                               c->wmax_small, s);
    }
}

template <int DIM, typename T, int QN>
pf_status numeric_dispatch_quad(const pf_csr* c, const double* coords, const void* cKq, const void* cMq, void* valsK,
                                void* valsM, Fallback f, int64_t* ctr, hipStream_t s) {
    pf_status st = numeric_dispatch_quad_rows<DIM, T, QN>(c, coords, cKq, cMq, valsK, valsM, f, ctr, s);
    if (st != PF_OK) return st;
    return launch_long<DIM, T, false, QN>(c, coords, cKq, cMq, valsK, valsM, f, ctr, s);
}

}  // namespace

pf_status device_pool_alloc(int64_t bytes, hipStream_t s, void** out) {
    hipMemPool_t pool = nullptr;
    if (pf_status st = pool_of_current(&pool)) return st;
    const hipError_t e = hipMallocFromPoolAsync(out, static_cast<size_t>(bytes), pool, s);
    if (e != hipSuccess) return fail(PF_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    return PF_OK;
}
void device_pool_free(void* p, hipStream_t s) {
    if (p) (void)hipFreeAsync(p, s);
}

// the long rows of a structure alone (the serving loop's fused launches skip them)
pf_status numeric_long(const pf_csr* c, pf_dtype prec, const double* coords, void* valsK, void* valsM,
                       const pf_fallback* fb, int64_t* ctr, hipStream_t s) {
    if (c->nlong == 0) return PF_OK;
    const Fallback f = make_fallback(fb);
    if (c->dim == 3)
        return prec == PF_F32 ? launch_long<3, float, false, 0>(c, coords, nullptr, nullptr, valsK, valsM, f, ctr, s)
                              : launch_long<3, double, false, 0>(c, coords, nullptr, nullptr, valsK, valsM, f, ctr, s);
    return prec == PF_F32 ? launch_long<2, float, false, 0>(c, coords, nullptr, nullptr, valsK, valsM, f, ctr, s)
                          : launch_long<2, double, false, 0>(c, coords, nullptr, nullptr, valsK, valsM, f, ctr, s);
}

// rows per block of a job's numeric phase (as pf_assemble chooses)
int numeric_class(const pf_csr* c, pf_dtype prec) {
    if (c->dim == 3) return prec == PF_F32 ? numeric_rows32<3>(c) : numeric_rows<3, double>(c);
    return prec == PF_F32 ? numeric_rows32<2>(c) : numeric_rows<2, double>(c);
}

int64_t numeric_blocks(const pf_csr* c, pf_dtype prec) { return ceil_div(c->nn, numeric_class(c, prec)); }

void numeric_describe(const pf_csr* c, const double* coords, void* valsK, void* valsM, const pf_fallback* fb,
                      int64_t* counters, int64_t block0, NumericJob* out) {
    out->nn = c->nn;
    out->coords = coords;
    out->row_ptr = c->row_ptr;
    out->col_idx = c->col_idx;
    out->aptr = c->aptr;
    out->adj = c->adj;
    out->pk = c->pk;
    out->dpos = c->dpos;
    out->valsK = valsK;
    out->valsM = valsM;
    out->counters = counters;
    out->fb = make_fallback(fb);
    out->block0 = block0;
}

int numeric_wmax(const pf_csr* c, int nr) { return window_of(c, nr); }

namespace {
template <int DIM, int NR>
pf_status launch_jobs64(const NumericJob* d_jobs, int njobs, int64_t nblocks, int wmax, hipStream_t s) {
    const size_t shm = numeric_lds_bytes<DIM, double>(NR, wmax);
    hipLaunchKernelGGL((k_numeric_jobs<DIM, NR>), dim3(static_cast<unsigned>(nblocks)), dim3(NBT), shm, s, d_jobs,
                       njobs, wmax);
    return launch_check("numeric batch");
}

template <int DIM, int NR>
pf_status launch_jobs32(const NumericJob* d_jobs, int njobs, int64_t nblocks, int wmax, hipStream_t s) {
    const size_t shm = numeric_lds_bytes_f32<DIM>(NR, wmax);
    hipLaunchKernelGGL((k_numeric_jobs32<DIM, NR, NT32>), dim3(static_cast<unsigned>(nblocks)), dim3(NT32), shm, s,
                       d_jobs, njobs, wmax);
    return launch_check("numeric batch");
}
}  // namespace

pf_status numeric_launch_many(int dim, pf_dtype prec, int nr, const NumericJob* d_jobs, int njobs, int64_t nblocks,
                              int wmax, hipStream_t s) {
    if (njobs <= 0 || nblocks <= 0) return PF_OK;
    if (nblocks >= (int64_t(1) << 31)) return fail(PF_ELIMIT, "numeric batch: too many row blocks");
    if (prec == PF_F32) {
        auto pick = [&](auto big, auto mid, auto small) {
            return nr == NT32 / 8 ? big(d_jobs, njobs, nblocks, wmax, s)
                                  : (nr == NT32 / 16 ? mid(d_jobs, njobs, nblocks, wmax, s)
                                                     : small(d_jobs, njobs, nblocks, wmax, s));
        };
        if (dim == 3)
            return pick(launch_jobs32<3, NT32 / 8>, launch_jobs32<3, NT32 / 16>, launch_jobs32<3, NT32 / 32>);
        return pick(launch_jobs32<2, NT32 / 8>, launch_jobs32<2, NT32 / 16>, launch_jobs32<2, NT32 / 32>);
    }
    auto pick = [&](auto big, auto mid, auto small) {
        return nr == NR_BIG ? big(d_jobs, njobs, nblocks, wmax, s)
                            : (nr == NR_MID ? mid(d_jobs, njobs, nblocks, wmax, s) : small(d_jobs, njobs, nblocks, wmax, s));
    };
    if (dim == 3) return pick(launch_jobs64<3, NR_BIG>, launch_jobs64<3, NR_MID>, launch_jobs64<3, NR_SMALL>);
    return pick(launch_jobs64<2, NR_BIG>, launch_jobs64<2, NR_MID>, launch_jobs64<2, NR_SMALL>);
}

size_t csr_bytes(const pf_csr* c) {
    return static_cast<size_t>(c->cap_scratch + c->cap_res) + static_cast<size_t>(c->cap_nnz + c->cap_lrows + c->cap_lcol) * 4 +
           static_cast<size_t>(c->cap_work) * 8 +
           static_cast<size_t>(c->cap_fcount + c->cap_bcount + c->cap_fptr + c->cap_bptr + c->cap_faces + c->cap_fel +
                               c->cap_bfaces + c->cap_bel) * 4 + static_cast<size_t>(c->cap_finfo) * 8 +
           static_cast<size_t>(c->cap_esign + c->cap_pk9);
}

int64_t csr_nnz(const pf_csr* c) { return c->built ? c->nnz : -1; }
int64_t csr_nn(const pf_csr* c) { return c->nn; }
int csr_dim(const pf_csr* c) { return c->dim; }
int64_t csr_ne(const pf_csr* c) { return c->ne; }
bool csr_built(const pf_csr* c) { return c->built && !c->p2; }
bool csr_view(const pf_csr* c, CsrView* v) {
    if (!c->built) return false;
    v->nn = c->nn;
    v->ne = c->ne;
    v->nnz = c->nnz;
    v->dim = c->dim;
    v->nlb = c->nlb;
    v->row_ptr = c->row_ptr;
    v->aptr = c->aptr;
    v->adj = c->adj;
    v->pk = c->p2 ? nullptr : c->pk;
    v->pk2 = c->p2 ? c->pk2 : nullptr;
    v->dpos = c->dpos;
    v->wmax4 = c->wmax_small;
    v->wmax16 = c->wmax_mid;
    v->wmax32 = c->wmax_big;
    v->max_adj = c->max_adj;
    v->nlong = c->nlong;
    v->lrows = c->lrows;
    v->pk9 = c->pk9;
    return true;
}
const int32_t* csr_adj(const pf_csr* c) { return c->adj; }
const int32_t* csr_aptr(const pf_csr* c) { return c->aptr; }

pf_status csr_order(const pf_csr* c, hipStream_t s) {
    if (!c->cols_pending) return PF_OK;
    const hipError_t e = hipEventQuery(c->ready);
    if (e == hipSuccess) {
        c->cols_pending = false;
        return PF_OK;
    }
    if (e != hipErrorNotReady) return fail(PF_EHIP, std::string("structure build: ") + hipGetErrorString(e));
    if (s != c->q_stream) PF_HIP_TRY(hipStreamWaitEvent(s, c->ready, 0));
    return PF_OK;
}

pf_status csr_workspace(pf_csr* c, int64_t words, double** out, hipStream_t s) {
    pf_status st;
    if ((st = grow(reinterpret_cast<double*&>(c->work), c->cap_work, words, s))) return st;
    *out = static_cast<double*>(c->work);
    return PF_OK;
}

void csr_pool_trim() {
    scratch_trim();
    hipMemPool_t pool = nullptr;
    if (pool_of_current(&pool) == PF_OK) (void)hipMemPoolTrimTo(pool, 0);
}

void csr_release(pf_csr* c, hipStream_t s) {
    if (!c) return;
    if ((c->stage != 0 || c->cols_pending) && c->ready) (void)hipEventSynchronize(c->ready);  // a build in flight
    for (hipEvent_t& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    scratch_return(c->scratch, c->scratch_owned, s);
    c->scratch = nullptr;
    c->cap_scratch = 0;
    drop(c->res, c->cap_res, s);
    drop(c->lrows, c->cap_lrows, s);
    drop(c->pk9, c->cap_pk9, s);
    drop(c->col_idx, c->cap_nnz, s);
    drop(c->work, c->cap_work, s);
    drop(c->fcount, c->cap_fcount, s);
    drop(c->bcount, c->cap_bcount, s);
    drop(c->fptr, c->cap_fptr, s);
    drop(c->bptr, c->cap_bptr, s);
    drop(c->faces, c->cap_faces, s);
    drop(c->fel, c->cap_fel, s);
    drop(c->bfaces, c->cap_bfaces, s);
    drop(c->bel, c->cap_bel, s);
    drop(c->esign, c->cap_esign, s);
    drop(c->finfo, c->cap_finfo, s);
    if (c->ready) (void)hipEventDestroy(c->ready);
    recycle_pinned(c->hinfo);
    delete c;
}

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
    // nothing may still read the arrays (as hipFree would, wait for the whole device)
    (void)hipDeviceSynchronize();
    csr_release(c, nullptr);
    (void)hipStreamSynchronize(nullptr);
    csr_pool_trim();
}

namespace {
// add the stage times of the last timed call to the sums
// the events that open and close each stage: the first three follow each other on the
// stream; the columns open when the host enqueues them, after the status readback
constexpr int STAGE_EV[PF_CSR_STAGES][2] = {{0, 1}, {1, 2}, {2, 3}, {4, 5}};

pf_status collect_stage_times(pf_csr* c) {
    if (!c->pending) return PF_OK;
    c->pending = false;
    PF_HIP_TRY(hipEventSynchronize(c->ev[PF_CSR_STAGES + 1]));
    for (int k = 0; k < PF_CSR_STAGES; ++k) {
        float ms = 0.0f;
        PF_HIP_TRY(hipEventElapsedTime(&ms, c->ev[STAGE_EV[k][0]], c->ev[STAGE_EV[k][1]]));
        c->stage_ms[k] += ms;
    }
    ++c->stage_calls;
    return PF_OK;
}

pf_status mark(pf_csr* c, int k, hipStream_t s) {
    if (c->timing) PF_HIP_TRY(hipEventRecord(c->ev[k], s));
    return PF_OK;
}
}  // namespace

pf_status pf_csr_set_timing(pf_csr* c, int on) {
    if (!c) return fail(PF_EINVAL, "pf_csr_set_timing: null handle");
    if (on)
        for (hipEvent_t& e : c->ev)
            if (!e) PF_HIP_TRY(hipEventCreate(&e));
    c->timing = on != 0;
    c->pending = false;
    for (double& v : c->stage_ms) v = 0.0;
    c->stage_calls = 0;
    return PF_OK;
}

pf_status pf_csr_stage_times(pf_csr* c, double* ms, int64_t* calls) {
    if (!c || !ms) return fail(PF_EINVAL, "pf_csr_stage_times: null argument");
    pf_status st;
    if ((st = collect_stage_times(c))) return st;
    for (int k = 0; k < PF_CSR_STAGES; ++k) ms[k] = c->stage_ms[k];
    if (calls) *calls = c->stage_calls;
    return PF_OK;
}

namespace {
pf_status enqueue_columns(pf_csr* c, hipStream_t s, const char* who);

// The structure of a P1 (nlb = dim + 1) or P2 (nlb = 6, 10) mesh, in two phases.  Phase 1
// (symbolic_enqueue): the adjacency scattered into padded rows, its offsets (a scan of the
// lengths), the row patterns (every 8-row group's sorted columns, the compact adjacency with
// the packed slot words of its entries, the diagonal positions), the row offsets, nnz and
// the launch statistics; it ends with the status words' copy to pinned host memory and the
// ready event.  Phase 2 (symbolic_columns, once the host holds nnz): col_idx allocated for
// exactly nnz words, the columns moved into it, the build's scratch released; it ends with
// the ready event again.  A rebuild in a handle whose col_idx already holds the new nnz moves
// the columns in phase 1 and needs no phase 2.  Every step is enqueued on one stream; nothing
// waits in between.
pf_status symbolic_enqueue(pf_csr* c, int dim, int nlb, int64_t nn, int64_t ne, const int32_t* elems, void* stream,
                           const char* who) {
    const bool p2 = nlb > dim + 1;
    const int maxrow = p2 ? MAXROW2 : MAXROW;
    if (nn >= INT32_MAX || ne * nlb >= INT32_MAX || ne >= (int64_t(1) << (p2 ? 27 : 29)))
        return fail(PF_ELIMIT, std::string(who) + ": mesh too large for 32-bit indices");
    if (ne > 0 && !elems) return fail(PF_EINVAL, std::string(who) + ": null elems");
    hipStream_t s = as_stream(stream);
    if (c->stage != 0) {  // an unfinished earlier build: its status is dropped
        PF_HIP_TRY(hipEventSynchronize(c->ready));
        c->stage = 0;
    }
    pf_status st;
    if ((st = csr_order(c, s))) return st;  // the previous build's columns, on another stream
    c->built = false;
    c->faces_built = false;
    const int64_t m = ne * nlb;
    if ((st = collect_stage_times(c))) return st;  // the previous call's events are reused below
    auto part = [](int64_t bytes) { return (std::max<int64_t>(bytes, 1) + 255) & ~int64_t(255); };
    {
        const int64_t nb = std::max<int64_t>(ceil_div(nn + 1, SCAN_TILE), 1);
        const int64_t b_rows = part(4 * (nn + 1)), b_adj = part(4 * m), b_pk = part((p2 ? 8 : 4) * m);
        const int64_t b_bsum = part(8 * nb), b_info = part(8 * INFO_WORDS);
        const int64_t b_bcnt = p2 ? 0 : part(4 * ceil_div(nn, 4));  // routed counts of the FP32 numeric blocks
        if ((st = grow(c->res, c->cap_res, 3 * b_rows + b_adj + b_pk + b_bsum + b_info + b_bcnt, s))) return st;
        unsigned char* q = c->res;
        c->aptr = reinterpret_cast<int32_t*>(q);
        c->row_ptr = reinterpret_cast<int32_t*>(q + b_rows);
        c->dpos = reinterpret_cast<int32_t*>(q + 2 * b_rows);
        q += 3 * b_rows;
        c->adj = reinterpret_cast<int32_t*>(q);
        c->pk = p2 ? nullptr : reinterpret_cast<uint32_t*>(q + b_adj);
        c->pk2 = p2 ? reinterpret_cast<uint64_t*>(q + b_adj) : nullptr;
        c->bsum = reinterpret_cast<int64_t*>(q + b_adj + b_pk);
        c->info = reinterpret_cast<int64_t*>(q + b_adj + b_pk + b_bsum);
        c->bcnt = p2 ? nullptr : reinterpret_cast<int32_t*>(q + b_adj + b_pk + b_bsum + b_info);
    }
    const int64_t tiles = ceil_div(nn, SCAN_TILE);
    {
        // every 8-row group's sorted columns wait at the start of its region of colblk (P1
        // pattern blocks of 32 rows write 4 groups; P2 blocks of 16 rows write groups 2b, 2b + 1);
        // look: tile descriptors, then TSTAT int32 statistics per tile
        const int64_t regions = p2 ? 2 * ceil_div(nn, RR2) : (PR / RR) * ceil_div(nn, PR);
        const int64_t b_len = part(4 * (nn + 1)), b_pad = part(4 * nn * MAXADJ), b_cnt = part(4 * (nn + 1));
        const int64_t b_blk = part(4 * std::max<int64_t>(regions * RR * maxrow, 1));
        const int64_t b_look = part(8 * ((1 + TSTAT / 2) * std::max<int64_t>(tiles, 1) + 1));
        const int64_t b_lst = part(4 * nn);  // the long rows' list
        if (c->scratch) {  // an earlier build's, still held (an error ended it early)
            scratch_return(c->scratch, c->scratch_owned, s);
            c->scratch = nullptr;
        }
        const int64_t bytes = b_len + b_pad + b_cnt + b_blk + b_look + b_lst;
        if ((st = scratch_borrow(bytes, s, &c->scratch, &c->scratch_owned))) return st;
        c->cap_scratch = bytes;
        unsigned char* q = c->scratch;
        c->adj_len = reinterpret_cast<int32_t*>(q);
        c->adj_pad = reinterpret_cast<int32_t*>(q + b_len);
        c->cnt = reinterpret_cast<int32_t*>(q + b_len + b_pad);
        c->colblk = reinterpret_cast<int32_t*>(q + b_len + b_pad + b_cnt);
        c->look = reinterpret_cast<uint64_t*>(q + b_len + b_pad + b_cnt + b_blk);
        c->lrows_s = reinterpret_cast<int32_t*>(q + b_len + b_pad + b_cnt + b_blk + b_look);
    }
    c->nlong = 0;
    c->q_long = false;
    if (!c->hinfo && (st = pinned_words(&c->hinfo))) return st;
    if ((st = mark(c, 0, s))) return st;
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, s, c->info, int64_t(INFO_WORDS), int64_t(0));
    if (nn > 0) hipLaunchKernelGGL(k_fill_i32, dim3(flat_grid(nn)), dim3(SBS), 0, s, c->adj_len, nn, 0);
    const unsigned gtile = static_cast<unsigned>(std::max<int64_t>(ceil_div(m, AG_TILE), 1));
    if (m > 0) {
        if (p2)
            hipLaunchKernelGGL(k_scatter<4>, dim3(gtile), dim3(AG_BS), 0, s, elems, m, nlb, nn, c->adj_len, c->adj_pad,
                               c->info);
        else
            hipLaunchKernelGGL(k_scatter<2>, dim3(gtile), dim3(AG_BS), 0, s, elems, m, nlb, nn, c->adj_len, c->adj_pad,
                               c->info);
    }
    // adjacency offsets (aptr[nn] = the adjacency total, into info[1])
    if ((st = scan(c->adj_len, nn, c->aptr, c->bsum, c->info + 1, s))) return st;
    if ((st = mark(c, 1, s))) return st;
    if (nn > 0) {
        const unsigned g1 = static_cast<unsigned>(ceil_div(nn, PR));   // P1: 32-row blocks
        const unsigned g2 = static_cast<unsigned>(ceil_div(nn, RR2));  // P2: 16-row blocks
        if (nlb == 10)
            hipLaunchKernelGGL((k_pattern_p2<10>), dim3(g2), dim3(RT2), 0, s, nn, elems, c->adj_len, c->adj_pad,
                               c->aptr, c->cnt, c->colblk, c->adj, c->pk2, c->dpos, c->lrows_s, c->info);
        else if (nlb == 6)
            hipLaunchKernelGGL((k_pattern_p2<6>), dim3(g2), dim3(RT2), 0, s, nn, elems, c->adj_len, c->adj_pad,
                               c->aptr, c->cnt, c->colblk, c->adj, c->pk2, c->dpos, c->lrows_s, c->info);
        else if (nlb == 4)
            hipLaunchKernelGGL((k_rows_p1<4>), dim3(g1), dim3(PT), 0, s, nn, elems, c->adj_len, c->adj_pad, c->aptr,
                               c->cnt, c->colblk, c->adj, c->pk, c->dpos, c->lrows_s, c->info);
        else
            hipLaunchKernelGGL((k_rows_p1<3>), dim3(g1), dim3(PT), 0, s, nn, elems, c->adj_len, c->adj_pad, c->aptr,
                               c->cnt, c->colblk, c->adj, c->pk, c->dpos, c->lrows_s, c->info);
    }
    if ((st = mark(c, 2, s))) return st;
    if (nn > 0) {
        hipLaunchKernelGGL(k_fill_i64, dim3(flat_grid(tiles)), dim3(SBS), 0, s, reinterpret_cast<int64_t*>(c->look),
                           tiles, int64_t(0));
        int32_t* tstat = reinterpret_cast<int32_t*>(c->look + ((tiles + 1) & ~int64_t(1)));  // 16-byte aligned
        hipLaunchKernelGGL(k_row_offsets, dim3(static_cast<unsigned>(tiles)), dim3(SBS), 0, s, nn, c->cnt, c->adj_len,
                           c->row_ptr, c->look, tstat, c->info);
        hipLaunchKernelGGL(k_row_stats, dim3(1), dim3(SBS), 0, s, tiles, tstat, c->info);
    } else {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, c->row_ptr, int64_t(1), 0);
    }
    if ((st = mark(c, 3, s))) return st;
    // a col_idx kept from an earlier build of the handle: the columns go in now (the kernel
    // writes nothing if nnz exceeds it), so that a rebuild of a mesh of no more nonzeros and no
    // long rows ends with this phase's readback
    c->q_cols = c->col_idx != nullptr && c->cap_nnz > 0 && nn > 0;
    c->q_nn = nn;  // (the helper reads the build's shape)
    c->q_dim = dim;
    c->q_nlb = nlb;
    if (c->q_cols && (st = enqueue_columns(c, s, who))) return st;  // no long rows listed yet: nlong is 0
    if ((st = launch_check(who))) return st;
    c->pending = c->timing;
    // pinned: a direct copy, no staging through pageable memory
    PF_HIP_TRY(hipMemcpyAsync(c->hinfo, c->info, INFO_WORDS * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (!c->ready) PF_HIP_TRY(hipEventCreateWithFlags(&c->ready, hipEventDisableTiming));
    PF_HIP_TRY(hipEventRecord(c->ready, s));
    c->stage = 1;
    c->q_dim = dim;
    c->q_nlb = nlb;
    c->q_nn = nn;
    c->q_ne = ne;
    c->q_stream = s;
    c->q_elems = elems;
    return PF_OK;
}

// the build's scratch, released in the order of its stream
void drop_scratch(pf_csr* c, hipStream_t s) {
    scratch_return(c->scratch, c->scratch_owned, s);
    c->scratch = nullptr;
    c->cap_scratch = 0;
    drop(c->lcol, c->cap_lcol, s);
    c->adj_len = c->adj_pad = c->cnt = c->colblk = c->lrows_s = nullptr;
    c->look = nullptr;
}

// Phase 1b, only for a mesh whose phase 1 listed long rows: their list made resident, their
// nodes' compact adjacency, one workgroup per long row for its pattern (columns into lcol,
// slot words, diagonal position, row length), then the row offsets and statistics again with
// the long rows' lengths; ends with the status readback and the ready event.
pf_status symbolic_long(pf_csr* c, const char* who) {
    hipStream_t s = c->q_stream;
    const int64_t nlong = c->hinfo[INFO_NLONG];
    const int64_t nn = c->q_nn, m = c->q_ne * c->q_nlb;
    const int nlb = c->q_nlb;
    const bool p2 = nlb > c->q_dim + 1;
    pf_status st;
    if ((st = grow(c->lrows, c->cap_lrows, nlong, s))) return st;
    if ((st = grow(c->lcol, c->cap_lcol, nlong * LCAP, s))) return st;
    if (nlb == 10 && (st = grow(c->pk9, c->cap_pk9, m, s))) return st;  // the ninth position of a P2 long row's entry
    c->nlong = nlong;
    c->q_long = true;
    PF_HIP_TRY(hipMemcpyAsync(c->lrows, c->lrows_s, nlong * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_long_adj, dim3(flat_grid(ceil_div(m, 4))), dim3(SBS), 0, s, c->q_elems, m, nlb, p2 ? 4 : 2,
                       c->dpos,
                       c->aptr, c->cnt, c->adj);
    const unsigned g = static_cast<unsigned>(nlong);
    switch (nlb) {
        case 4:
            hipLaunchKernelGGL((k_rows_long<4, 2>), dim3(g), dim3(LT), 0, s, c->lrows, c->q_elems, c->aptr, c->adj,
                               c->cnt, c->lcol, c->pk, nullptr, nullptr, c->dpos, c->info);
            break;
        case 3:
            hipLaunchKernelGGL((k_rows_long<3, 2>), dim3(g), dim3(LT), 0, s, c->lrows, c->q_elems, c->aptr, c->adj,
                               c->cnt, c->lcol, c->pk, nullptr, nullptr, c->dpos, c->info);
            break;
        case 10:
            hipLaunchKernelGGL((k_rows_long<10, 4>), dim3(g), dim3(LT), 0, s, c->lrows, c->q_elems, c->aptr, c->adj,
                               c->cnt, c->lcol, nullptr, c->pk2, c->pk9, c->dpos, c->info);
            break;
        default:
            hipLaunchKernelGGL((k_rows_long<6, 4>), dim3(g), dim3(LT), 0, s, c->lrows, c->q_elems, c->aptr, c->adj,
                               c->cnt, c->lcol, nullptr, c->pk2, nullptr, c->dpos, c->info);
            break;
    }
    const int64_t tiles = ceil_div(nn, SCAN_TILE);
    hipLaunchKernelGGL(k_fill_i64, dim3(flat_grid(tiles)), dim3(SBS), 0, s, reinterpret_cast<int64_t*>(c->look), tiles,
                       int64_t(0));
    int32_t* tstat = reinterpret_cast<int32_t*>(c->look + ((tiles + 1) & ~int64_t(1)));
    hipLaunchKernelGGL(k_row_offsets, dim3(static_cast<unsigned>(tiles)), dim3(SBS), 0, s, nn, c->cnt, c->adj_len,
                       c->row_ptr, c->look, tstat, c->info);
    hipLaunchKernelGGL(k_row_stats, dim3(1), dim3(SBS), 0, s, tiles, tstat, c->info);
    if ((st = launch_check(who))) return st;
    PF_HIP_TRY(hipMemcpyAsync(c->hinfo, c->info, INFO_WORDS * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PF_HIP_TRY(hipEventRecord(c->ready, s));
    c->stage = 3;
    return PF_OK;
}

// the columns of every row into col_idx (sized for at least nnz), the long rows' groups again
pf_status enqueue_columns(pf_csr* c, hipStream_t s, const char* who) {
    const int64_t nn = c->q_nn;
    const bool p2 = c->q_nlb > c->q_dim + 1;
    pf_status st;
    if ((st = mark(c, 4, s))) return st;
    if (nn > 0) {
        const unsigned tiles = static_cast<unsigned>(ceil_div(nn, SCAN_TILE));
        if (p2)
            hipLaunchKernelGGL((k_row_columns<RR * MAXROW2, 4>), dim3(tiles), dim3(SBS), 0, s, nn, c->row_ptr,
                               c->colblk, c->col_idx, c->cap_nnz);
        else
            hipLaunchKernelGGL((k_row_columns<RR * MAXROW, 2>), dim3(tiles), dim3(SBS), 0, s, nn, c->row_ptr,
                               c->colblk, c->col_idx, c->cap_nnz);
        if (c->nlong > 0)
            hipLaunchKernelGGL(k_long_columns, dim3(static_cast<unsigned>(c->nlong)), dim3(LT), 0, s, c->lrows, nn,
                               p2 ? MAXROW2 : MAXROW, c->row_ptr, c->aptr, c->colblk, c->lcol, c->col_idx);
    }
    if ((st = mark(c, 5, s))) return st;
    return launch_check(who);
}

// After phase 1 (or 1b): its status words have reached the host (the ready event has
// completed).  Check them; if phase 1 listed long rows, enqueue phase 1b; otherwise fix the
// structure's sizes and launch statistics and enqueue phase 2 (the columns).
pf_status symbolic_columns(pf_csr* c, const char* who) {
    c->stage = 0;
    hipStream_t s = c->q_stream;
    const int64_t* info = c->hinfo;
    const int dim = c->q_dim, nlb = c->q_nlb;
    const int64_t nn = c->q_nn, ne = c->q_ne;
    const bool p2 = nlb > dim + 1;
    pf_status st = PF_OK;
    if (info[0] & ERR_INDEX) st = fail(PF_EINDEX, std::string(who) + ": node index out of range in elems");
    else if (info[0] & ERR_ROW)
        st = fail(PF_ELIMIT, std::string(who) + ": a row has more than " + std::to_string(LCAP) + " nonzeros");
    else if (info[0] & ERR_SCAN) st = fail(PF_EINVAL, std::string(who) + ": the row offsets could not be formed");
    else if (info[2] >= INT32_MAX) st = fail(PF_ELIMIT, std::string(who) + ": nnz must be < 2^31");
    if (st == PF_OK && !c->q_long && info[INFO_NLONG] > 0) {
        if ((st = symbolic_long(c, who)) == PF_OK) return PF_OK;
    }
    const int64_t nnz = info[2];
    // phase 1 already moved the columns (they fitted, and no long rows): the build is complete
    const bool done = st == PF_OK && c->q_cols && !c->q_long && info[INFO_NLONG] == 0 && nnz <= c->cap_nnz;
    if (st == PF_OK && !done) st = grow(c->col_idx, c->cap_nnz, std::max<int64_t>(nnz, 1), s);
    if (st != PF_OK) {
        c->pending = false;  // the stage events of this call are incomplete
        drop_scratch(c, s);
        return st;
    }
    if (!done) {  // phase 2: the columns into col_idx, then the ready event
        if ((st = enqueue_columns(c, s, who))) return st;
        drop_scratch(c, s);
        PF_HIP_TRY(hipEventRecord(c->ready, s));
        c->stage = 2;
    } else {
        drop_scratch(c, s);
    }
    c->dim = dim;
    c->nlb = nlb;
    c->p2 = p2;
    c->nn = nn;
    c->ne = ne;
    c->nnz = nnz;
    c->wmax_big = static_cast<int>(info[3]);
    c->wmax_mid = static_cast<int>(info[4]);
    c->wmax_small = static_cast<int>(info[5]);
    c->max_adj = static_cast<int>(info[7]);
    c->wmax8 = static_cast<int>(info[8]);
    c->wmax2 = static_cast<int>(info[9]);
    return PF_OK;
}

pf_status symbolic(pf_csr* c, int dim, int nlb, int64_t nn, int64_t ne, const int32_t* elems, void* stream,
                   const char* who) {
    pf_status st = symbolic_enqueue(c, dim, nlb, nn, ne, elems, stream, who);
    if (st != PF_OK) return st;
    PF_HIP_TRY(hipEventSynchronize(c->ready));
    if ((st = symbolic_columns(c, who))) return st;
    if (c->stage == 3) {  // the long-row phase ran: its status, then the columns
        PF_HIP_TRY(hipEventSynchronize(c->ready));
        if ((st = symbolic_columns(c, who))) return st;
    }
    // the columns complete in the order of the stream: no wait here (csr_order orders the
    // work of other streams after them); stage 0: phase 1 already placed them
    c->cols_pending = c->stage == 2;
    c->stage = 0;
    c->built = true;
    return PF_OK;
}
}  // namespace

}  // extern "C"

namespace pf {
pf_status csr_symbolic_enqueue(pf_csr* c, int dim, int64_t nn, int64_t ne, const int32_t* elems, hipStream_t s) {
    if (dim != 2 && dim != 3) return fail(PF_EORDER, "pf_server build: dim must be 2 or 3");
    return symbolic_enqueue(c, dim, dim + 1, nn, ne, elems, s, "pf_server build");
}

int csr_symbolic_poll(pf_csr* c, pf_status* st) {
    if (c->stage == 0) {
        *st = c->built ? PF_OK : fail(PF_ESTATE, "pf_server build: nothing enqueued");
        return 1;
    }
    const hipError_t e = hipEventQuery(c->ready);
    if (e == hipErrorNotReady) return 0;
    if (e != hipSuccess) {
        c->stage = 0;
        *st = fail(PF_EHIP, std::string("pf_server build: ") + hipGetErrorString(e));
        return 1;
    }
    if (c->stage == 1 || c->stage == 3) {  // the pattern (or long-row) phase ended: what follows
        const pf_status s1 = symbolic_columns(c, "pf_server build");
        if (s1 != PF_OK) {
            c->stage = 0;
            *st = s1;
            return 1;
        }
        if (c->stage == 0) {  // complete already (columns placed in phase 1)
            c->built = true;
            *st = PF_OK;
            return 1;
        }
        return 0;
    }
    c->stage = 0;
    c->built = true;
    *st = PF_OK;
    return 1;
}

}  // namespace pf

extern "C" {

namespace {
}  // namespace

pf_status pf_csr_symbolic(pf_csr* c, int dim, int64_t nn, int64_t ne, const int32_t* elems, void* stream) {
    if (!c) return fail(PF_EINVAL, "pf_csr_symbolic: null handle");
    if (dim != 2 && dim != 3) return fail(PF_EORDER, "pf_csr_symbolic: dim must be 2 or 3");
    if (nn < 0 || ne < 0) return fail(PF_EINVAL, "pf_csr_symbolic: negative size");
    return symbolic(c, dim, dim + 1, nn, ne, elems, stream, "pf_csr_symbolic");
}

pf_status pf_csr_symbolic_p2(pf_csr* c, int dim, int64_t nn, int64_t ne, const int32_t* elems2, void* stream) {
    if (!c) return fail(PF_EINVAL, "pf_csr_symbolic_p2: null handle");
    if (dim != 2 && dim != 3) return fail(PF_EORDER, "pf_csr_symbolic_p2: dim must be 2 or 3");
    if (nn < 0 || ne < 0) return fail(PF_EINVAL, "pf_csr_symbolic_p2: negative size");
    return symbolic(c, dim, dim == 2 ? 6 : 10, nn, ne, elems2, stream, "pf_csr_symbolic_p2");
}

pf_status pf_assemble_quad(const pf_csr* c, pf_dtype prec, const double* coords, int order, const void* cKq,
                           const void* cMq, void* valsK, void* valsM, const pf_fallback* fb, int64_t* d_counters,
                           void* stream) {
    if (!c) return fail(PF_EINVAL, "pf_assemble_quad: null handle");
    if (!c->built) return fail(PF_ESTATE, "pf_assemble_quad: structure not built");
    if (c->p2) return fail(PF_ESTATE, "pf_assemble_quad: a P2 structure (pf_p2_assemble assembles it)");
    const int qn = quad_count(c->dim, order);
    if (!qn) return fail(PF_EINVAL, "pf_assemble_quad: order must be 1 or 2");
    if (c->nn == 0 || c->nnz == 0) return PF_OK;
    if (!coords || !valsK) return fail(PF_EINVAL, "pf_assemble_quad: null coords or valsK");
    if (prec != PF_F32 && prec != PF_F64) return fail(PF_EDTYPE, "pf_assemble_quad: prec must be PF_F32 or PF_F64");
    hipStream_t s = as_stream(stream);
    if (pf_status st = csr_order(c, s)) return st;
    Fallback f = make_fallback(fb);
    if (c->dim == 3) {
        if (prec == PF_F32)
            return qn == 1 ? numeric_dispatch_quad<3, float, 1>(c, coords, cKq, cMq, valsK, valsM, f, d_counters, s)
                           : numeric_dispatch_quad<3, float, 4>(c, coords, cKq, cMq, valsK, valsM, f, d_counters, s);
        return qn == 1 ? numeric_dispatch_quad<3, double, 1>(c, coords, cKq, cMq, valsK, valsM, f, d_counters, s)
                       : numeric_dispatch_quad<3, double, 4>(c, coords, cKq, cMq, valsK, valsM, f, d_counters, s);
    }
    if (prec == PF_F32)
        return qn == 1 ? numeric_dispatch_quad<2, float, 1>(c, coords, cKq, cMq, valsK, valsM, f, d_counters, s)
                       : numeric_dispatch_quad<2, float, 3>(c, coords, cKq, cMq, valsK, valsM, f, d_counters, s);
    return qn == 1 ? numeric_dispatch_quad<2, double, 1>(c, coords, cKq, cMq, valsK, valsM, f, d_counters, s)
                   : numeric_dispatch_quad<2, double, 3>(c, coords, cKq, cMq, valsK, valsM, f, d_counters, s);
}

pf_status pf_csr_faces(pf_csr* c, const double* coords, const int32_t* elems, void* stream) {
    if (!c) return fail(PF_EINVAL, "pf_csr_faces: null handle");
    if (!c->built) return fail(PF_ESTATE, "pf_csr_faces: structure not built");
    if (c->p2) return fail(PF_ESTATE, "pf_csr_faces: a P2 structure");
    if (c->ne > 0 && (!coords || !elems)) return fail(PF_EINVAL, "pf_csr_faces: null coords or elems");
    hipStream_t s = as_stream(stream);
    if (pf_status st = csr_order(c, s)) return st;
    c->faces_built = false;
    const int64_t nn = c->nn;
    pf_status st;
    if ((st = grow(c->fcount, c->cap_fcount, nn + 1, s))) return st;
    if ((st = grow(c->bcount, c->cap_bcount, nn + 1, s))) return st;
    if ((st = grow(c->fptr, c->cap_fptr, nn + 1, s))) return st;
    if ((st = grow(c->bptr, c->cap_bptr, nn + 1, s))) return st;
    if ((st = grow(c->finfo, c->cap_finfo, 4, s))) return st;
    if ((st = grow(c->esign, c->cap_esign, std::max<int64_t>(c->ne, 1), s))) return st;
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, s, c->finfo, int64_t(4), int64_t(0));
    if (c->ne > 0) {
        const unsigned ge = static_cast<unsigned>(ceil_div(c->ne, SBS));
        if (c->nlb == 4) hipLaunchKernelGGL((k_elem_sign<4>), dim3(ge), dim3(SBS), 0, s, c->ne, coords, elems, c->esign);
        else hipLaunchKernelGGL((k_elem_sign<3>), dim3(ge), dim3(SBS), 0, s, c->ne, coords, elems, c->esign);
    }
    const unsigned g = static_cast<unsigned>(std::max<int64_t>(ceil_div(nn, FR), 1));
    if (nn > 0) {
        if (c->nlb == 4)
            hipLaunchKernelGGL((k_faces<4, 0>), dim3(g), dim3(FT), 0, s, nn, c->row_ptr, c->col_idx, c->aptr,
                               c->adj, c->pk, c->dpos, c->esign, c->fcount, c->bcount, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr, c->finfo);
        else
            hipLaunchKernelGGL((k_faces<3, 0>), dim3(g), dim3(FT), 0, s, nn, c->row_ptr, c->col_idx, c->aptr,
                               c->adj, c->pk, c->dpos, c->esign, c->fcount, c->bcount, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr, c->finfo);
    }
    const unsigned gl = static_cast<unsigned>(c->nlong);  // the long rows, after the row blocks left them empty
    if (gl > 0) {
        if (c->nlb == 4)
            hipLaunchKernelGGL((k_faces_long<4, 0>), dim3(gl), dim3(FLT), 0, s, c->lrows, c->row_ptr, c->col_idx,
                               c->aptr, c->adj, c->pk, c->dpos, c->esign, c->fcount, c->bcount, nullptr, nullptr,
                               nullptr, nullptr, nullptr, nullptr, c->finfo);
        else
            hipLaunchKernelGGL((k_faces_long<3, 0>), dim3(gl), dim3(FLT), 0, s, c->lrows, c->row_ptr, c->col_idx,
                               c->aptr, c->adj, c->pk, c->dpos, c->esign, c->fcount, c->bcount, nullptr, nullptr,
                               nullptr, nullptr, nullptr, nullptr, c->finfo);
    }
    if ((st = scan(c->fcount, nn, c->fptr, c->bsum, c->finfo + 1, s))) return st;
    if ((st = scan(c->bcount, nn, c->bptr, c->bsum, c->finfo + 2, s))) return st;
    if (!c->hinfo && (st = pinned_words(&c->hinfo))) return st;
    int64_t* info = c->hinfo;
    PF_HIP_TRY(hipMemcpyAsync(info, c->finfo, 4 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PF_HIP_TRY(hipStreamSynchronize(s));
    if (info[0] & ERR_FACE)
        return fail(PF_EINVAL, "pf_csr_faces: a face belongs to more than two elements (not a conforming mesh)");
    if (info[0] & ERR_ROW)
        return fail(PF_ELIMIT, "pf_csr_faces: a node owns more than 128 faces (1024 for a node in more than 64 "
                               "elements or with more than 64 neighbours)");
    const int64_t nf = info[1], nfb = info[2];
    const int nv = c->dim;
    if ((st = grow(c->faces, c->cap_faces, nf * nv, s))) return st;
    if ((st = grow(c->fel, c->cap_fel, 2 * nf, s))) return st;
    if ((st = grow(c->bfaces, c->cap_bfaces, nfb * nv, s))) return st;
    if ((st = grow(c->bel, c->cap_bel, nfb, s))) return st;
    if (nn > 0 && nf > 0) {
        if (c->nlb == 4)
            hipLaunchKernelGGL((k_faces<4, 1>), dim3(g), dim3(FT), 0, s, nn, c->row_ptr, c->col_idx, c->aptr,
                               c->adj, c->pk, c->dpos, c->esign, nullptr, nullptr, c->fptr, c->bptr, c->faces,
                               c->fel, c->bfaces, c->bel, c->finfo);
        else
            hipLaunchKernelGGL((k_faces<3, 1>), dim3(g), dim3(FT), 0, s, nn, c->row_ptr, c->col_idx, c->aptr,
                               c->adj, c->pk, c->dpos, c->esign, nullptr, nullptr, c->fptr, c->bptr, c->faces,
                               c->fel, c->bfaces, c->bel, c->finfo);
        if (gl > 0) {
            if (c->nlb == 4)
                hipLaunchKernelGGL((k_faces_long<4, 1>), dim3(gl), dim3(FLT), 0, s, c->lrows, c->row_ptr, c->col_idx,
                                   c->aptr, c->adj, c->pk, c->dpos, c->esign, nullptr, nullptr, c->fptr, c->bptr,
                                   c->faces, c->fel, c->bfaces, c->bel, c->finfo);
            else
                hipLaunchKernelGGL((k_faces_long<3, 1>), dim3(gl), dim3(FLT), 0, s, c->lrows, c->row_ptr, c->col_idx,
                                   c->aptr, c->adj, c->pk, c->dpos, c->esign, nullptr, nullptr, c->fptr, c->bptr,
                                   c->faces, c->fel, c->bfaces, c->bel, c->finfo);
        }
    }
    if ((st = launch_check("pf_csr_faces"))) return st;
    c->nf = nf;
    c->nfb = nfb;
    c->faces_built = true;
    return PF_OK;
}

pf_status pf_csr_faces_info(const pf_csr* c, int64_t* nf, int64_t* nfb, const int32_t** faces, const int32_t** fel,
                            const int32_t** bfaces, const int32_t** bel) {
    if (!c) return fail(PF_EINVAL, "pf_csr_faces_info: null handle");
    if (!c->faces_built) return fail(PF_ESTATE, "pf_csr_faces_info: faces not built");
    if (nf) *nf = c->nf;
    if (nfb) *nfb = c->nfb;
    if (faces) *faces = c->faces;
    if (fel) *fel = c->fel;
    if (bfaces) *bfaces = c->bfaces;
    if (bel) *bel = c->bel;
    return PF_OK;
}

pf_status pf_csr_info(const pf_csr* c, int64_t* nn, int64_t* nnz, const int32_t** row_ptr, const int32_t** col_idx) {
    if (!c) return fail(PF_EINVAL, "pf_csr_info: null handle");
    if (!c->built) return fail(PF_ESTATE, "pf_csr_info: structure not built");
    if (c->cols_pending) {  // device pointers handed out: the arrays are complete
        PF_HIP_TRY(hipEventSynchronize(c->ready));
        c->cols_pending = false;
    }
    if (nn) *nn = c->nn;
    if (nnz) *nnz = c->nnz;
    if (row_ptr) *row_ptr = c->row_ptr;
    if (col_idx) *col_idx = c->col_idx;
    return PF_OK;
}

pf_status pf_csr_memory(const pf_csr* c, int64_t* resident, int64_t* scratch) {
    if (!c) return fail(PF_EINVAL, "pf_csr_memory: null handle");
    const int64_t all = static_cast<int64_t>(csr_bytes(c));
    const int64_t scr = c->cap_scratch + 4 * c->cap_lcol;
    if (resident) *resident = all - scr;
    if (scratch) *scratch = scr;
    return PF_OK;
}

pf_status pf_csr_numeric_info(const pf_csr* c, pf_dtype prec, int32_t* rows_per_block, int32_t* max_adj) {
    if (!c) return fail(PF_EINVAL, "pf_csr_numeric_info: null handle");
    if (!c->built || c->p2) return fail(PF_ESTATE, "pf_csr_numeric_info: no P1 structure built");
    if (prec != PF_F32 && prec != PF_F64) return fail(PF_EDTYPE, "pf_csr_numeric_info: prec must be PF_F32 or PF_F64");
    if (rows_per_block) *rows_per_block = numeric_class(c, prec);
    if (max_adj) *max_adj = c->max_adj;
    return PF_OK;
}

pf_status pf_assemble(const pf_csr* c, pf_dtype prec, const double* coords, const int32_t* elems, const void* cK,
                      const void* cM, void* valsK, void* valsM, const pf_fallback* fb, int64_t* d_counters,
                      void* stream) {
    if (!c) return fail(PF_EINVAL, "pf_assemble: null handle");
    if (!c->built) return fail(PF_ESTATE, "pf_assemble: structure not built");
    if (c->p2) return fail(PF_ESTATE, "pf_assemble: a P2 structure (pf_p2_assemble assembles it)");
    if (c->nn == 0 || c->nnz == 0) return PF_OK;
    if (!coords || !valsK) return fail(PF_EINVAL, "pf_assemble: null coords or valsK");
    (void)elems;  // the structure carries the connectivity it was built from
    if (prec != PF_F32 && prec != PF_F64) return fail(PF_EDTYPE, "pf_assemble: prec must be PF_F32 or PF_F64");
    hipStream_t s = as_stream(stream);
    if (pf_status st = csr_order(c, s)) return st;
    Fallback f = make_fallback(fb);
    if (prec == PF_F32)
        return c->dim == 3 ? numeric_dispatch<3, float>(c, coords, cK, cM, valsK, valsM, f, d_counters, s)
                           : numeric_dispatch<2, float>(c, coords, cK, cM, valsK, valsM, f, d_counters, s);
    return c->dim == 3 ? numeric_dispatch<3, double>(c, coords, cK, cM, valsK, valsM, f, d_counters, s)
                       : numeric_dispatch<2, double>(c, coords, cK, cM, valsK, valsM, f, d_counters, s);
}

}  // extern "C"
