// internal.hpp -- declarations shared between the library's own translation units (not
// part of the C ABI): the multi-mesh numeric assembly used by the serving loop, and the
// structure handle's adjacency and workspace for the load vector and energy kernels.
#pragma once

#include "common.hpp"

namespace pf {

// Device descriptor of one mesh in a multi-mesh numeric launch (k_numeric_jobs).
struct NumericJob {
    int64_t nn;
    const double* coords;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const int32_t* aptr;
    const int32_t* adj;
    const uint32_t* pk;
    const int32_t* dpos;
    void* valsK;
    void* valsM;
    int64_t* counters;
    Fallback fb;
    int64_t block0;  // first block of this job in the launch
};

// rows per block (16 or 4) that pf_assemble would use for this structure and precision
int numeric_class(const pf_csr* c, pf_dtype prec);
int64_t numeric_blocks(const pf_csr* c, pf_dtype prec);
int numeric_wmax(const pf_csr* c, int nr);
void numeric_describe(const pf_csr* c, const double* coords, void* valsK, void* valsM, const pf_fallback* fb,
                      int64_t* counters, int64_t block0, NumericJob* out);
// one launch over njobs descriptors (device array) of the same dim, precision and rows per
// block; wmax = the largest window of those jobs, nblocks = the total block count
pf_status numeric_launch_many(int dim, pf_dtype prec, int nr, const NumericJob* d_jobs, int njobs, int64_t nblocks,
                              int wmax, hipStream_t s);
// the numeric phase of the structure's long rows alone, constant coefficients (the fused
// multi-mesh launches skip long rows)
pf_status numeric_long(const pf_csr* c, pf_dtype prec, const double* coords, void* valsK, void* valsM,
                       const pf_fallback* fb, int64_t* counters, hipStream_t s);
size_t csr_bytes(const pf_csr* c);
int64_t csr_nnz(const pf_csr* c);
int64_t csr_nn(const pf_csr* c);
int csr_dim(const pf_csr* c);
int64_t csr_ne(const pf_csr* c);
bool csr_built(const pf_csr* c);  // a built P1 structure
// a built structure, P1 or P2: node i's adjacency entries at aptr[i] .. aptr[i+1] of adj,
// (element << 2 | local index) with pk (P1: row positions of the element's other nodes in
// local order, 8 bits each from bit 2), or (element << 4 | local index) with pk2 (P2: 7 bits
// each from bit 0), at most CSR_MAXADJ per node; dpos = the diagonal's
// position in each row; wmax4 / wmax16 / wmax32 = the largest CSR window of 4 / 16 / 32
// consecutive rows starting at a multiple of their count; max_adj = the longest adjacency list
struct CsrView {
    int64_t nn, ne, nnz;
    int dim, nlb;
    const int32_t* row_ptr;
    const int32_t* aptr;
    const int32_t* adj;
    const uint32_t* pk;
    const uint64_t* pk2;
    const int32_t* dpos;
    int wmax4, wmax16, wmax32;
    int max_adj;
    int64_t nlong;         // long rows ...
    const int32_t* lrows;  // ... and their list
    const uint8_t* pk9;    // P2 long rows of 10-node elements: the ninth 8-bit position
};
bool csr_view(const pf_csr* c, CsrView* v);  // false unless built
// node -> element adjacency of the structure: entries (element << 2 | local index) of node i
// at adj[aptr[i]] .. adj[aptr[i+1] - 1], at most CSR_MAXADJ of them
constexpr int CSR_MAXADJ = 64;
// A P1 row is long when its node lies in more than CSR_MAXADJ elements or the row holds
// more than CSR_MAXROW nonzeros (a P2 row: more than CSR_MAXROW2): the row-block kernels skip
// it, and kernels of one workgroup per long row (listed in lrows, nlong of them) assemble it;
// a long row holds at most CSR_LCAP nonzeros.  The slot words of a P2 long row's entries
// hold 8-bit positions (pk2 bits 8k .. 8k+7 for the k-th other node, k < 8; the ninth of a
// 10-node element in pk9).
constexpr int CSR_MAXROW = 64;
constexpr int CSR_MAXROW2 = 128;
constexpr int CSR_LCAP = 256;
__host__ __device__ inline bool csr_long_row(int elements, int nonzeros) {
    return elements > CSR_MAXADJ || nonzeros > CSR_MAXROW;
}
__host__ __device__ inline bool csr_long_row_p2(int elements, int nonzeros) {
    return elements > CSR_MAXADJ || nonzeros > CSR_MAXROW2;
}
const int32_t* csr_adj(const pf_csr* c);
const int32_t* csr_aptr(const pf_csr* c);
// asynchronous structure build (the serving loop): csr_symbolic_enqueue issues the first
// phase of pf_csr_symbolic on stream s without waiting; csr_symbolic_poll, called until it
// returns 1, enqueues the second phase once the first one's status words have reached the
// host and returns 1 when the build has ended (*st: its outcome, the structure usable on any
// stream if PF_OK), 0 while it runs
pf_status csr_symbolic_enqueue(pf_csr* c, int dim, int64_t nn, int64_t ne, const int32_t* elems, hipStream_t s);
int csr_symbolic_poll(pf_csr* c, pf_status* st);
// a device workspace of at least `words` doubles owned by the handle (grown on stream s when
// needed)
pf_status csr_workspace(pf_csr* c, int64_t words, double** out, hipStream_t s);

// a stream-ordered block of the library's device pool, and its release on a stream
pf_status device_pool_alloc(int64_t bytes, hipStream_t s, void** out);
void device_pool_free(void* p, hipStream_t s);

// Per-workgroup count slots for one launch of nb workgroups and W tallies (block_counts), a
// stream-ordered pool block taken only when the caller asked for counters; finish() sums
// them into the counters (k_sum_counts) and releases the block on the same stream.
template <int W>
struct BlockCountSlots {
    void* p = nullptr;
    int64_t nb = 0;
    pf_status init(const int64_t* d_counters, int64_t nblocks, hipStream_t s) {
        nb = nblocks;
        if (!d_counters || nblocks <= 0) return PF_OK;
        return device_pool_alloc(static_cast<int64_t>(W) * 4 * nblocks, s, &p);
    }
    int32_t* slots() const { return static_cast<int32_t*>(p); }
    void finish(int64_t* d_counters, hipStream_t s, int w0, int w1 = 0, int w2 = 0) {
        if (!p) return;
        const int64_t g = (nb + SUM_COUNTS_PER_BLOCK - 1) / SUM_COUNTS_PER_BLOCK;
        hipLaunchKernelGGL((k_sum_counts<W>), dim3(static_cast<unsigned>(g)), dim3(256), 0, s, slots(), nb,
                           d_counters, w0, w1, w2);
        device_pool_free(p, s);
        p = nullptr;
    }
};
// pf_csr_destroy without its device-wide wait: the handle's arrays are released in the order
// of stream s (every earlier use of the structure must be ordered before that point of s, or
// have completed); a build still in flight is waited for first
void csr_release(pf_csr* c, hipStream_t s);
// return the unused blocks of the current device's structure pool to the device
void csr_pool_trim();
// order the work about to be enqueued on stream s after the end of the structure's build
// (pf_csr_symbolic returns with its last phase still in flight on its own stream)
pf_status csr_order(const pf_csr* c, hipStream_t s);

}  // namespace pf
