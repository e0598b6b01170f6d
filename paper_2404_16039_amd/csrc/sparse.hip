// sparse.hip -- assembly of element pages into the CSR structure: the sparse(X3D(:),
// Y3D(:), K3D(:)) step that ends the P1 and P2 listings of section 3.6, for pages computed
// by any kernel (pf_elem_stiffness_mass, pf_p2_elements) or by the caller.
//
// In the listings Y3D(a, b, e) = elems(e, a) and X3D is its page transpose, so the page
// entry (a, b) of element e goes to row elems(e, b), column elems(e, a).  Row-owned and
// exact, like the fused P1 numeric phase: a block owns PR consecutive rows (a contiguous
// window of the CSR arrays); every adjacency entry of a row (element e with the row's node
// at local index a) reads column a of its element's page (contiguous), entry (b, a) for all
// b, and adds it to the slot of node b; the slot positions come from the structure (the
// diagonal position, and pk / pk2 for the other nodes).  Each slot's largest contribution
// fixes its grid, the contributions are rounded to it once and summed exactly in integers,
// so the result does not depend on the order of the additions.
#include "exact.hpp"
#include "internal.hpp"

#include <string>
#include <type_traits>

namespace pf {

constexpr int PBT = 256;   // threads per block
constexpr int PITEMS = 2;  // adjacency entries per thread (held in registers)
constexpr int PCAP = PITEMS * PBT;  // entries per block at most
static_assert(PCAP >= 4 * CSR_MAXADJ, "the smallest blocks (4 rows) cover any admissible rows");

__device__ __forceinline__ int last_le(const int32_t* v, int n, int x) {
    // last index r in [0, n) with v[r] <= x (v ascending, v[0] <= x)
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (v[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// column a of a page (NB consecutive values from base) into v, zeros without pages.  With
// NB even a column starts 8 bytes (FP32) or 16 bytes (FP64) into an aligned page array, and
// 16 bytes in FP32 when NB = 4, so VEC (the host found the arrays 16-byte aligned) allows
// vector loads; a compile-time choice, so no scalar copy of the loads exists beside them.
template <int NB, typename T, bool VEC>
__device__ __forceinline__ void load_column(const T* __restrict__ pg, int64_t base, T (&v)[NB]) {
    constexpr bool vec = VEC;
    if (pg == nullptr) {
#pragma unroll
        for (int b = 0; b < NB; ++b) v[b] = T(0);
        return;
    }
    if constexpr (sizeof(T) == 4 && NB == 4) {
        if constexpr (vec) {
            const float4 x = *reinterpret_cast<const float4*>(pg + base);
            v[0] = x.x;
            v[1] = x.y;
            v[2] = x.z;
            v[3] = x.w;
            return;
        }
    } else if constexpr (NB % 2 == 0) {
        using V2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
        if constexpr (vec) {
            const V2* x = reinterpret_cast<const V2*>(pg + base);
#pragma unroll
            for (int k = 0; k < NB / 2; ++k) {
                const V2 y = x[k];
                v[2 * k] = y.x;
                v[2 * k + 1] = y.y;
            }
            return;
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) v[b] = pg[base + b];
}

// NB nodes per element; P2: entries are (element << 4 | a) with pk2, else (element << 2 | a)
// with pk.  pages: ne x NB x NB, column-major (entry (a, b) at a + b NB).  PR rows per block,
// chosen by the host so that PR times the longest adjacency list fits PCAP; the block's
// entries are dealt flat (row after row), entry k to thread k mod PBT.
template <int NB, bool P2, typename T, int PR, bool VEC>
__global__ __launch_bounds__(PBT) void k_assemble_pages(int64_t nn, const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ aptr,
                                                        const int32_t* __restrict__ adj, const uint32_t* __restrict__ pk,
                                                        const uint64_t* __restrict__ pk2, const int32_t* __restrict__ dpos,
                                                        const T* __restrict__ pagesK, const T* __restrict__ pagesM,
                                                        T* __restrict__ valsK, T* __restrict__ valsM) {
    using A = typename Exact<T>::acc;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t rp[PR + 1], abase[PR + 1], apre[PR + 1], dslot[PR];
    __shared__ int32_t anylong;
    auto is_long = [](int elements, int nonzeros) {
        return P2 ? csr_long_row_p2(elements, nonzeros) : csr_long_row(elements, nonzeros);
    };
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * PR;
    const int nr = static_cast<int>((r0 + PR < nn) ? PR : nn - r0);
    if (threadIdx.x <= PR) {  // rows past the end: no slots, no entries
        const int r = threadIdx.x <= nr ? threadIdx.x : nr;
        rp[threadIdx.x] = row_ptr[r0 + r];
        abase[threadIdx.x] = aptr[r0 + r];
    }
    if (threadIdx.x < PR) dslot[threadIdx.x] = static_cast<int>(threadIdx.x) < nr ? dpos[r0 + threadIdx.x] : 0;
    __syncthreads();
    static_assert(PR <= 64, "the row prefix runs in one wave");
    if (threadIdx.x < 64) {  // prefix of the rows' entries in wave 0; P1 long rows count none
        const int r = threadIdx.x;
        const int La = r < nr ? abase[r + 1] - abase[r] : 0;
        const bool lng = r < nr && is_long(La, rp[r + 1] - rp[r]);
        const int Lk = lng ? 0 : La;
        int x = Lk;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(x, d, 64);
            if (r >= d) x += y;
        }
        if (r < PR) apre[r] = x - Lk;
        if (r == PR - 1) apre[PR] = x;
        const unsigned long long lm = __ballot(lng);
        if (r == 0) anylong = lm != 0ull;
    }
    __syncthreads();
    const int32_t w0 = rp[0];
    const int W = rp[nr] - w0;
    A* accK = reinterpret_cast<A*>(smem);
    A* accM = accK + W;
    int32_t* shK = reinterpret_cast<int32_t*>(accM + W);
    int32_t* shM = shK + W;
    static_assert(lds_carve_aligned<A, A, int32_t, int32_t>(), "page assembly LDS carve-out: every array naturally aligned");
    for (int w = threadIdx.x; w < W; w += PBT) {
        accK[w] = A(0);
        accM[w] = A(0);
        shK[w] = 0;
        shM[w] = 0;
    }
    // this thread's entries k = thread + q PBT of the block's flat list; loads without branches
    int rq[PITEMS];
    int64_t eq[PITEMS];
    int aq[PITEMS];
    uint64_t pq[PITEMS];
#pragma unroll
    for (int q = 0; q < PITEMS; ++q) {
        const int idx = threadIdx.x + q * PBT;
        const bool ok = idx < apre[PR];
        const int r = ok ? last_le(apre, PR, idx) : 0;
        const int64_t t = ok ? static_cast<int64_t>(abase[r]) + (idx - apre[r]) : 0;
        const int32_t w = adj[t];
        pq[q] = P2 ? pk2[t] : static_cast<uint64_t>(pk[t]);
        rq[q] = ok ? r : -1;
        eq[q] = ok ? static_cast<int64_t>(static_cast<uint32_t>(w) >> (P2 ? 4 : 2)) : 0;
        aq[q] = ok ? (w & (P2 ? 15 : 3)) : 0;
    }
    __syncthreads();  // accumulators cleared
    if (anylong) {  // a long row's slots are marked: neither graded nor stored here
        for (int r = 0; r < nr; ++r)
            if (is_long(abase[r + 1] - abase[r], rp[r + 1] - rp[r]))
                for (int k = rp[r] - w0 + threadIdx.x; k < rp[r + 1] - w0; k += PBT) shK[k] = INT32_MIN;
        __syncthreads();
    }
    // window position of local node b of the entry's element in its row
    auto slot = [&](int q, int b) -> int {
        const int r = rq[q], a = aq[q];
        if (b == a) return rp[r] - w0 + dslot[r];
        const int k = b < a ? b : b - 1;
        const int pos = P2 ? static_cast<int>((pq[q] >> (7 * k)) & 127) : static_cast<int>((pq[q] >> (2 + 8 * k)) & 255);
        return rp[r] - w0 + pos;
    };
    T kv[PITEMS][NB], mv[PITEMS][NB];
#pragma unroll
    for (int q = 0; q < PITEMS; ++q) {
        const int64_t base = eq[q] * (NB * NB) + aq[q] * NB;  // column a
        load_column<NB, T, VEC>(pagesK, base, kv[q]);
        load_column<NB, T, VEC>(pagesM, base, mv[q]);
    }
    // per-slot grid: the largest contribution
#pragma unroll
    for (int q = 0; q < PITEMS; ++q) {
        if (rq[q] < 0) continue;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int s = slot(q, b);
            atomicMax(reinterpret_cast<uint32_t*>(shK + s), Exact<T>::mag(kv[q][b]));
            atomicMax(reinterpret_cast<uint32_t*>(shM + s), Exact<T>::mag(mv[q][b]));
        }
    }
    __syncthreads();
    for (int w = threadIdx.x; w < W; w += PBT) {
        if (shK[w] == INT32_MIN) continue;
        shK[w] = Exact<T>::shift(static_cast<uint32_t>(shK[w]));
        shM[w] = Exact<T>::shift(static_cast<uint32_t>(shM[w]));
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PITEMS; ++q) {
        if (rq[q] < 0) continue;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int s = slot(q, b);
            atomicAdd(accK + s, Exact<T>::quant(kv[q][b], shK[s]));
            atomicAdd(accM + s, Exact<T>::quant(mv[q][b], shM[s]));
        }
    }
    __syncthreads();
    for (int w = threadIdx.x; w < W; w += PBT) {
        if (shK[w] == INT32_MIN) continue;
        if (valsK) valsK[w0 + w] = Exact<T>::back(accK[w], shK[w]);
        if (valsM) valsM[w0 + w] = Exact<T>::back(accM[w], shM[w]);
    }
}

// The long rows (one workgroup each, at most CSR_LCAP slots): every entry's column of its
// element's pages, graded and summed on each slot's LongGrid as in the long-row numeric
// kernel (page values are exact in FP64).  Slot positions: P1 from pk, P2 from the 8-bit
// positions of a long row's entries (pk2, and pk9 for the ninth other node).
template <int NB, bool P2, typename T>
__global__ __launch_bounds__(PBT) void k_assemble_pages_long(const int32_t* __restrict__ lrows,
                                                             const int32_t* __restrict__ row_ptr,
                                                             const int32_t* __restrict__ aptr,
                                                             const int32_t* __restrict__ adj,
                                                             const uint32_t* __restrict__ pk,
                                                             const uint64_t* __restrict__ pk2,
                                                             const uint8_t* __restrict__ pk9,
                                                             const int32_t* __restrict__ dpos,
                                                             const T* __restrict__ pagesK, const T* __restrict__ pagesM,
                                                             T* __restrict__ valsK, T* __restrict__ valsM) {
    static_assert(P2 ? NB <= 10 : NB <= 4, "P2 long rows: 8-bit positions of up to nine other nodes");
    using G = LongGrid;
    __shared__ uint32_t mxK[CSR_LCAP], mxM[CSR_LCAP];
    __shared__ int32_t shK[CSR_LCAP], shM[CSR_LCAP];
    __shared__ unsigned long long accK[CSR_LCAP], accM[CSR_LCAP];
    const int t = static_cast<int>(threadIdx.x);
    const int64_t row = lrows[blockIdx.x];
    const int64_t w0 = row_ptr[row];
    const int len = row_ptr[row + 1] - static_cast<int>(w0);
    const int64_t a0 = aptr[row];
    const int L = aptr[row + 1] - static_cast<int>(a0);
    const int sd = dpos[row];
    const int hb = G::headroom(L);
    for (int k = t; k < CSR_LCAP; k += PBT) {
        mxK[k] = mxM[k] = 0u;
        accK[k] = accM[k] = 0ull;
    }
    __syncthreads();
    auto entry = [&](int j, double (&kv)[NB], double (&mv)[NB], int (&sl)[NB]) {
        const int32_t w = adj[a0 + j];
        const uint64_t p = P2 ? pk2[a0 + j] : static_cast<uint64_t>(pk[a0 + j]);
        const int p9 = P2 && NB == 10 ? pk9[a0 + j] : 0;
        const int64_t e = static_cast<uint32_t>(w) >> (P2 ? 4 : 2);
        const int a = w & (P2 ? 15 : 3);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int k = b < a ? b : b - 1;  // index among the other nodes
            const int pos = P2 ? (k == 8 ? p9 : static_cast<int>((p >> (8 * k)) & 255))
                               : static_cast<int>((p >> (2 + 8 * k)) & 255);
            sl[b] = b == a ? sd : pos;
            const int64_t idx = e * (NB * NB) + a * NB + b;  // column a, entry b
            kv[b] = pagesK ? static_cast<double>(pagesK[idx]) : 0.0;
            mv[b] = pagesM ? static_cast<double>(pagesM[idx]) : 0.0;
        }
    };
    for (int j = t; j < L; j += PBT) {
        double kv[NB], mv[NB];
        int sl[NB];
        entry(j, kv, mv, sl);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            atomicMax(mxK + sl[b], G::mag(kv[b]));
            atomicMax(mxM + sl[b], G::mag(mv[b]));
        }
    }
    __syncthreads();
    for (int k = t; k < len; k += PBT) {
        shK[k] = mxK[k] == G::POISON ? 0 : G::shift(mxK[k], hb);
        shM[k] = mxM[k] == G::POISON ? 0 : G::shift(mxM[k], hb);
    }
    __syncthreads();
    for (int j = t; j < L; j += PBT) {
        double kv[NB], mv[NB];
        int sl[NB];
        entry(j, kv, mv, sl);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (mxK[sl[b]] != G::POISON) atomicAdd(accK + sl[b], G::quant(kv[b], shK[sl[b]]));
            if (mxM[sl[b]] != G::POISON) atomicAdd(accM + sl[b], G::quant(mv[b], shM[sl[b]]));
        }
    }
    __syncthreads();
    for (int k = t; k < len; k += PBT) {
        if (valsK) valsK[w0 + k] = mxK[k] == G::POISON ? static_cast<T>(NAN) : static_cast<T>(G::back(accK[k], shK[k]));
        if (valsM) valsM[w0 + k] = mxM[k] == G::POISON ? static_cast<T>(NAN) : static_cast<T>(G::back(accM[k], shM[k]));
    }
}

constexpr size_t PLDS = 65536;  // LDS budget of the window

template <typename T>
size_t window_bytes(int w) {
    return static_cast<size_t>(w) * (2 * sizeof(typename Exact<T>::acc) + 8);
}

// rows per block: the largest of 32, 16, 8, 4 whose entries fit PCAP and whose window fits
template <typename T>
int pages_rows(const CsrView& v) {
    if (32 * v.max_adj <= PCAP && window_bytes<T>(v.wmax32) <= PLDS) return 32;
    if (16 * v.max_adj <= PCAP && window_bytes<T>(v.wmax16) <= PLDS) return 16;
    if (8 * v.max_adj <= PCAP && window_bytes<T>(v.wmax16) <= PLDS) return 8;
    return window_bytes<T>(v.wmax4) <= PLDS ? 4 : 0;
}

template <int NB, bool P2, typename T, int PR>
void launch_pages_rows(const CsrView& v, const void* pK, const void* pM, void* vK, void* vM, hipStream_t s) {
    const int w = PR == 32 ? v.wmax32 : PR == 4 ? v.wmax4 : v.wmax16;  // 8 rows lie inside an aligned 16
    const unsigned g = static_cast<unsigned>(ceil_div(v.nn, PR));
    // vector column loads: an even page order and 16-byte aligned page arrays
    const bool vec = NB % 2 == 0 && (reinterpret_cast<uintptr_t>(pK) & 15) == 0 && (reinterpret_cast<uintptr_t>(pM) & 15) == 0;
    if (vec)
        hipLaunchKernelGGL((k_assemble_pages<NB, P2, T, PR, NB % 2 == 0>), dim3(g), dim3(PBT), window_bytes<T>(w), s, v.nn,
                           v.row_ptr, v.aptr, v.adj, v.pk, v.pk2, v.dpos, static_cast<const T*>(pK),
                           static_cast<const T*>(pM), static_cast<T*>(vK), static_cast<T*>(vM));
    else
        hipLaunchKernelGGL((k_assemble_pages<NB, P2, T, PR, false>), dim3(g), dim3(PBT), window_bytes<T>(w), s, v.nn,
                           v.row_ptr, v.aptr, v.adj, v.pk, v.pk2, v.dpos, static_cast<const T*>(pK),
                           static_cast<const T*>(pM), static_cast<T*>(vK), static_cast<T*>(vM));
}

template <int NB, bool P2, typename T>
void launch_pages(const CsrView& v, int pr, const void* pK, const void* pM, void* vK, void* vM, hipStream_t s) {
    if (pr == 32) launch_pages_rows<NB, P2, T, 32>(v, pK, pM, vK, vM, s);
    else if (pr == 16) launch_pages_rows<NB, P2, T, 16>(v, pK, pM, vK, vM, s);
    else if (pr == 8) launch_pages_rows<NB, P2, T, 8>(v, pK, pM, vK, vM, s);
    else launch_pages_rows<NB, P2, T, 4>(v, pK, pM, vK, vM, s);
}

template <int NB, bool P2, typename T>
void launch_pages_long(const CsrView& v, unsigned g, const void* pK, const void* pM, void* vK, void* vM,
                       hipStream_t s) {
    hipLaunchKernelGGL((k_assemble_pages_long<NB, P2, T>), dim3(g), dim3(PBT), 0, s, v.lrows, v.row_ptr, v.aptr, v.adj,
                       v.pk, v.pk2, v.pk9, v.dpos, static_cast<const T*>(pK), static_cast<const T*>(pM),
                       static_cast<T*>(vK), static_cast<T*>(vM));
}

}  // namespace pf

using namespace pf;

pf_status pf_csr_assemble_pages(const pf_csr* csr, pf_dtype prec, const void* pagesK, const void* pagesM, void* valsK,
                                void* valsM, void* stream) {
    if (!csr) return fail(PF_EINVAL, "pf_csr_assemble_pages: null handle");
    CsrView v{};
    if (!csr_view(csr, &v)) return fail(PF_ESTATE, "pf_csr_assemble_pages: structure not built");
    if (prec != PF_F32 && prec != PF_F64) return fail(PF_EDTYPE, "pf_csr_assemble_pages: prec must be PF_F32 or PF_F64");
    if ((valsK && !pagesK) || (valsM && !pagesM) || (!valsK && !valsM))
        return fail(PF_EINVAL, "pf_csr_assemble_pages: each output needs its pages, and one output is needed");
    if (v.nn == 0 || v.nnz == 0) return PF_OK;
    const bool f32 = prec == PF_F32;
    const int pr = f32 ? pages_rows<float>(v) : pages_rows<double>(v);
    if (pr == 0) return fail(PF_ELIMIT, "pf_csr_assemble_pages: a CSR window of 4 rows exceeds the LDS budget");
    hipStream_t s = as_stream(stream);
    if (pf_status st = csr_order(csr, s)) return st;
    // an output without its request still gets the other's pages read as zero
    const void* pK = valsK ? pagesK : nullptr;
    const void* pM = valsM ? pagesM : nullptr;
    switch (v.nlb) {
        case 3:
            f32 ? launch_pages<3, false, float>(v, pr, pK, pM, valsK, valsM, s) : launch_pages<3, false, double>(v, pr, pK, pM, valsK, valsM, s);
            break;
        case 4:
            f32 ? launch_pages<4, false, float>(v, pr, pK, pM, valsK, valsM, s) : launch_pages<4, false, double>(v, pr, pK, pM, valsK, valsM, s);
            break;
        case 6:
            f32 ? launch_pages<6, true, float>(v, pr, pK, pM, valsK, valsM, s) : launch_pages<6, true, double>(v, pr, pK, pM, valsK, valsM, s);
            break;
        case 10:
            f32 ? launch_pages<10, true, float>(v, pr, pK, pM, valsK, valsM, s) : launch_pages<10, true, double>(v, pr, pK, pM, valsK, valsM, s);
            break;
        default:
            return fail(PF_EINVAL, "pf_csr_assemble_pages: unsupported element");
    }
    if (v.nlong > 0) {  // the long rows, one workgroup each
        const unsigned g = static_cast<unsigned>(v.nlong);
        switch (v.nlb) {
            case 3:
                f32 ? launch_pages_long<3, false, float>(v, g, pK, pM, valsK, valsM, s)
                    : launch_pages_long<3, false, double>(v, g, pK, pM, valsK, valsM, s);
                break;
            case 4:
                f32 ? launch_pages_long<4, false, float>(v, g, pK, pM, valsK, valsM, s)
                    : launch_pages_long<4, false, double>(v, g, pK, pM, valsK, valsM, s);
                break;
            case 6:
                f32 ? launch_pages_long<6, true, float>(v, g, pK, pM, valsK, valsM, s)
                    : launch_pages_long<6, true, double>(v, g, pK, pM, valsK, valsM, s);
                break;
            default:
                f32 ? launch_pages_long<10, true, float>(v, g, pK, pM, valsK, valsM, s)
                    : launch_pages_long<10, true, double>(v, g, pK, pM, valsK, valsM, s);
                break;
        }
    }
    return launch_check("pf_csr_assemble_pages");
}
