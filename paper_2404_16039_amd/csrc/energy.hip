// energy.hip -- load vector and local energy parts of P1 elements (section 3.6: the
// right-hand side listing with its accumarray step, and the element-wise contributions to
// the gradient, reactive and linear parts of the energy functional).
//
// Load vector: one element per lane computes its local vector b2D (|det J| times the rule
// applied to f phi_j); half a wave per node then sums the entries of the elements around it,
// read through the structure handle's node -> element adjacency, exactly on a grid fixed by
// the node's largest entry, so b does not depend on the order of the adjacency lists.
//
// Energies: one element per lane; with c_j = det * grad phi_j (the cofactor columns of the
// Jacobian),
//   1/2 u^T K_e u = 1/2 cK_mean |sum_j u_j c_j|^2 / (d! |det|),  sum_j u_j c_j = sum_{j>=1} (u_j - u_0) c_j,
//   1/2 u^T M_e u = 1/2 |det| sum_q w_q cM_q u(x_q)^2,          u(x_q) = sum_j lam_qj u_j,
// which are the page bilinear forms with the element matrices of the quadrature assembly
// (stiffness with the weighted mean of the coefficient, mass integrated point by point), in
// a form that takes differences of u before any product.  The three sums over elements are
// FP64 block sums in a fixed order, then one block adds the block sums in order.
#include "p1elem.hpp"
#include "quadrature.hpp"
#include "exact.hpp"
#include "internal.hpp"

#include <mutex>
#include <string>

namespace pf {

constexpr int RBS = 256;  // threads per block
constexpr int ETOT_BLOCKS = 2048;  // blocks of the energy kernel at most (one partial each)

template <int DIM>
__device__ __forceinline__ bool gather_edges(const double* __restrict__ coords, int64_t nn,
                                             const int32_t* __restrict__ elems, int64_t e, int (&nd)[DIM + 1],
                                             double (&ev)[DIM][DIM]) {
    load_nodes<DIM>(elems, e, nd);
    return p1_edges<DIM>(coords, nn, nd, ev);
}

// |det J| of one element in precision C, with the FP32 routing to FP64 of pf_fallback
template <int DIM, typename T>
__device__ __forceinline__ double abs_det(const double (&ev)[DIM][DIM], const Fallback& fb, bool& routed) {
    routed = false;
    if constexpr (sizeof(T) == 4) {
        P1Geom<DIM, float> g;
        p1_geom<DIM, float>(ev, g);
        routed = route_elem<DIM>(g, fb);
        if (!routed) return fabsf(g.det);
    }
    P1Geom<DIM, double> gd;
    p1_geom<DIM, double>(ev, gd);
    return fabs(gd.det);
}

// ------------------------------------------------------------------------- load vector
// b2D[e*nlb + j] = |det| sum_q w_q f_q lam_qj; the rule sum in T, |det| in T (FP64 when routed)
template <int DIM, typename T, int QN>
__global__ __launch_bounds__(RBS) void k_rhs_elem(int64_t nn, const double* __restrict__ coords, int64_t ne,
                                                  const int32_t* __restrict__ elems, const T* __restrict__ fq,
                                                  T* __restrict__ b2D, Fallback fb, int64_t* d_counters,
                                                  int32_t* __restrict__ bcnt) {
    constexpr int NLB = DIM + 1;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * RBS + threadIdx.x;
    bool routed = false, bad = false;
    if (e < ne) {
        int nd[NLB];
        double ev[DIM][DIM];
        bad = !gather_edges<DIM>(coords, nn, elems, e, nd, ev);
        T s[NLB];
#pragma unroll
        for (int j = 0; j < NLB; ++j) s[j] = T(0);
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const T wf = static_cast<T>(quad_weight<DIM, QN>()) * fq[e * QN + q];
#pragma unroll
            for (int j = 0; j < NLB; ++j) s[j] = fmaT(wf, static_cast<T>(QuadRule<DIM, QN>::lam(q, j)), s[j]);
        }
        if (bad) {
#pragma unroll
            for (int j = 0; j < NLB; ++j) b2D[e * NLB + j] = static_cast<T>(NAN);
        } else {
            const double ad = abs_det<DIM, T>(ev, fb, routed);
#pragma unroll
            for (int j = 0; j < NLB; ++j)
                b2D[e * NLB + j] = routed ? static_cast<T>(ad * static_cast<double>(s[j])) : static_cast<T>(ad) * s[j];
        }
    }
    block_counts<2, RBS>(d_counters, bcnt, {0, 2}, {routed ? 1 : 0, bad ? 1 : 0});
}

// b[i] = sum of the entries of the elements around node i, exact on the grid of the node's
// largest entry (a node of more than 64 elements: on a LongGrid, every entry in turn).  Half a wave per node: lane l reads adjacency entries l and l + 32 of the
// node (contiguous words from aptr[i]) and gathers their local-vector values; the row maximum and then
// the integer sum of the rounded values are reduced across the 32 lanes with shuffles
// (integer adds: exact, so the result does not depend on the entry order).  Each half wave
// takes RHS_ROWS nodes at once, issuing all of their loads before the first reduction.
constexpr int RHS_ROWS = 8;
template <typename T>
__global__ __launch_bounds__(RBS) void k_rhs_nodes(int64_t nn, int nlb, const int32_t* __restrict__ aptr,
                                                   const int32_t* __restrict__ adj, const T* __restrict__ b2D,
                                                   T* __restrict__ b) {
    using A = typename Exact<T>::acc;
    static_assert(CSR_MAXADJ == 64, "two entries per lane of a half wave");
    const int64_t h = (static_cast<int64_t>(blockIdx.x) * RBS + threadIdx.x) >> 5;  // half wave
    const int l = threadIdx.x & 31;
    int64_t i[RHS_ROWS];
    int L[RHS_ROWS];
    int32_t w0[RHS_ROWS];
    T v0[RHS_ROWS], v1[RHS_ROWS];
    // the rows' adjacency offsets, then their first 32 entries (a lane past its row's
    // length reads entry 0 and drops it)
    int32_t a0[RHS_ROWS], a1[RHS_ROWS];
#pragma unroll
    for (int k = 0; k < RHS_ROWS; ++k) {  // every lane takes part in the shuffles
        i[k] = h * RHS_ROWS + k;
        const int64_t ic = i[k] < nn ? i[k] : nn - 1;
        a0[k] = aptr[ic];
        a1[k] = aptr[ic + 1];
    }
#pragma unroll
    for (int k = 0; k < RHS_ROWS; ++k) {
        L[k] = i[k] < nn ? min(a1[k] - a0[k], CSR_MAXADJ) : 0;
        w0[k] = adj[l < L[k] ? static_cast<int64_t>(a0[k]) + l : 0];
    }
#pragma unroll
    for (int k = 0; k < RHS_ROWS; ++k) w0[k] = l < L[k] ? w0[k] : 0;
#pragma unroll
    for (int k = 0; k < RHS_ROWS; ++k) {
        v0[k] = l < L[k] ? b2D[static_cast<int64_t>(w0[k] >> 2) * nlb + (w0[k] & 3)] : T(0);
        v1[k] = T(0);
        if (l + 32 < L[k]) {  // only nodes with more than 32 elements read the second half
            const int32_t w1 = adj[static_cast<int64_t>(a0[k]) + l + 32];
            v1[k] = b2D[static_cast<int64_t>(w1 >> 2) * nlb + (w1 & 3)];
        }
    }
#pragma unroll
    for (int k = 0; k < RHS_ROWS; ++k) {
        const int Lf = i[k] < nn ? a1[k] - a0[k] : 0;  // the same for the half wave
        if (Lf > CSR_MAXADJ) {
            // a node of more than 64 elements: every entry in turn, summed on a LongGrid
            using G = LongGrid;
            const int hb = G::headroom(Lf);
            uint32_t mx = 0u;
            for (int j = l; j < Lf; j += 32) {
                const int32_t w = adj[static_cast<int64_t>(a0[k]) + j];
                mx = max(mx, G::mag(static_cast<double>(b2D[static_cast<int64_t>(w >> 2) * nlb + (w & 3)])));
            }
#pragma unroll
            for (int d = 16; d >= 1; d >>= 1)
                mx = max(mx, static_cast<uint32_t>(__shfl_xor(static_cast<int>(mx), d, 32)));
            const int sh = mx == G::POISON ? 0 : G::shift(mx, hb);
            unsigned long long acc = 0ull;
            for (int j = l; j < Lf; j += 32) {
                const int32_t w = adj[static_cast<int64_t>(a0[k]) + j];
                acc += G::quant(static_cast<double>(b2D[static_cast<int64_t>(w >> 2) * nlb + (w & 3)]), sh);
            }
#pragma unroll
            for (int d = 16; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 32);
            if (l == 0) b[i[k]] = mx == G::POISON ? static_cast<T>(NAN) : static_cast<T>(G::back(acc, sh));
            continue;
        }
        uint32_t mx = max(Exact<T>::mag(v0[k]), Exact<T>::mag(v1[k]));
#pragma unroll
        for (int d = 16; d >= 1; d >>= 1)
            mx = max(mx, static_cast<uint32_t>(__shfl_xor(static_cast<int>(mx), d, 32)));
        const int sh = Exact<T>::shift(mx);
        A acc = Exact<T>::quant(v0[k], sh) + Exact<T>::quant(v1[k], sh);
#pragma unroll
        for (int d = 16; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 32);
        if (i[k] < nn && l == 0) b[i[k]] = Exact<T>::back(acc, sh);
    }
}

// ----------------------------------------------------------------------------- energies
// The three parts of one element from its cofactor columns (precision C) and nodal values.
template <int DIM, int QN, typename C>
__device__ __forceinline__ void energy_parts(const P1Geom<DIM, C>& g, const C (&uj)[DIM + 1], C ckm,
                                             const C (&cmq)[QN], C (&J)[2]) {
    C gu[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        C s = (uj[1] - uj[0]) * g.c[1][i];
#pragma unroll
        for (int j = 2; j <= DIM; ++j) s = fmaT(uj[j] - uj[0], g.c[j][i], s);
        gu[i] = s;
    }
    C g2 = gu[0] * gu[0];
#pragma unroll
    for (int i = 1; i < DIM; ++i) g2 = fmaT(gu[i], gu[i], g2);
    const C adet = fabs(g.det);
    J[0] = C(0.5) * ckm * g2 / (static_cast<C>(fact_dim<DIM>()) * adet);
    C m = C(0);
#pragma unroll
    for (int q = 0; q < QN; ++q) {
        C uq = static_cast<C>(QuadRule<DIM, QN>::lam(q, 0)) * uj[0];
#pragma unroll
        for (int j = 1; j <= DIM; ++j) uq = fmaT(static_cast<C>(QuadRule<DIM, QN>::lam(q, j)), uj[j], uq);
        m = fmaT(cmq[q] * uq, uq, m);
    }
    J[1] = C(0.5) * adet * static_cast<C>(quad_weight<DIM, QN>()) * m;
}

// one element per lane (grid-strided over a fixed grid); J[c * ne + e] in T (nullable);
// per-block FP64 sums of the three parts into part[3 * blockIdx.x + c]
template <int DIM, typename T, int QN>
__global__ __launch_bounds__(RBS) void k_energies(int64_t nn, const double* __restrict__ coords, int64_t ne,
                                                  const int32_t* __restrict__ elems, const T* __restrict__ cKq,
                                                  const T* __restrict__ cMq, const T* __restrict__ u,
                                                  const T* __restrict__ b2D, T* __restrict__ J,
                                                  double* __restrict__ part, Fallback fb, int64_t* d_counters) {
    constexpr int NLB = DIM + 1;
    __shared__ double red[3][RBS / 64];
    double sum[3] = {0.0, 0.0, 0.0};
    int64_t nrouted = 0, nbad = 0;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * RBS + threadIdx.x; e < ne;
         e += static_cast<int64_t>(gridDim.x) * RBS) {
        int nd[NLB];
        double ev[DIM][DIM];
        const bool ok = gather_edges<DIM>(coords, nn, elems, e, nd, ev);
        double Je[3];
        if (!ok) {
            ++nbad;
            Je[0] = Je[1] = Je[2] = NAN;
        } else {
            T uj[NLB], ck = T(0), cmq[QN];
#pragma unroll
            for (int j = 0; j < NLB; ++j) uj[j] = u[nd[j]];
#pragma unroll
            for (int q = 0; q < QN; ++q) {
                ck += cKq ? cKq[e * QN + q] : T(1);
                cmq[q] = cMq ? cMq[e * QN + q] : T(1);
            }
            ck *= static_cast<T>(1.0 / QN);  // equal weights: the weighted mean
            T j3 = T(0);
            if (b2D)
#pragma unroll
                for (int j = 0; j < NLB; ++j) j3 = fmaT(-b2D[e * NLB + j], uj[j], j3);
            Je[2] = static_cast<double>(j3);
            bool routed = false;
            if constexpr (sizeof(T) == 4) {
                P1Geom<DIM, float> g;
                p1_geom<DIM, float>(ev, g);
                routed = route_elem<DIM>(g, fb);
                if (!routed) {
                    float Jf[2];
                    energy_parts<DIM, QN, float>(g, uj, ck, cmq, Jf);
                    Je[0] = Jf[0];
                    Je[1] = Jf[1];
                }
            }
            if (sizeof(T) == 8 || routed) {
                P1Geom<DIM, double> gd;
                p1_geom<DIM, double>(ev, gd);
                double ud[NLB], cmd[QN], Jd[2];
#pragma unroll
                for (int j = 0; j < NLB; ++j) ud[j] = uj[j];
#pragma unroll
                for (int q = 0; q < QN; ++q) cmd[q] = cmq[q];
                energy_parts<DIM, QN, double>(gd, ud, static_cast<double>(ck), cmd, Jd);
                Je[0] = Jd[0];
                Je[1] = Jd[1];
            }
            nrouted += routed;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T v = static_cast<T>(Je[c]);
            if (J) J[c * ne + e] = v;
            sum[c] += static_cast<double>(v);  // the totals add the stored values
        }
    }
    // one atomic per workgroup and tally (at most ETOT_BLOCKS workgroups)
    block_counts<2, RBS>(d_counters, nullptr, {0, 2}, {static_cast<int>(nrouted), static_cast<int>(nbad)});
    // fixed-order block reduction: wave tree (xor shuffles), then the waves in order
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) sum[c] += __shfl_xor(sum[c], d, 64);
        if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = sum[c];
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int w = 0; w < RBS / 64; ++w) s += red[threadIdx.x][w];
        part[3 * blockIdx.x + threadIdx.x] = s;
    }
}

// totals[c] = sum over the block sums in block order (one wave per part, fixed tree)
__global__ __launch_bounds__(192) void k_energy_totals(const double* __restrict__ part, int nblocks,
                                                       double* __restrict__ totals) {
    const int c = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double s = 0.0;
    for (int b = lane; b < nblocks; b += 64) s += part[3 * b + c];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if (lane == 0) totals[c] = s;
}

namespace {

pf_status check_csr_mesh(const pf_csr* csr, const double* coords, const int32_t* elems, const char* who) {
    if (!csr) return fail(PF_EINVAL, std::string(who) + ": null handle");
    if (!csr_built(csr)) return fail(PF_ESTATE, std::string(who) + ": structure not built");
    if (csr_ne(csr) > 0 && (!coords || !elems)) return fail(PF_EINVAL, std::string(who) + ": null coords or elems");
    return PF_OK;
}

template <int DIM, typename T>
pf_status launch_rhs_elem(int qn, int64_t nn, const double* coords, int64_t ne, const int32_t* elems, const void* fq,
                          void* b2D, Fallback f, int64_t* ctr, hipStream_t s) {
    const unsigned g = static_cast<unsigned>(ceil_div(ne, RBS));
    constexpr int Q2 = DIM == 2 ? 3 : 4;
    BlockCountSlots<2> cs;
    if (pf_status st = cs.init(ctr, g, s)) return st;
    if (qn == 1)
        hipLaunchKernelGGL((k_rhs_elem<DIM, T, 1>), dim3(g), dim3(RBS), 0, s, nn, coords, ne, elems,
                           static_cast<const T*>(fq), static_cast<T*>(b2D), f, ctr, cs.slots());
    else
        hipLaunchKernelGGL((k_rhs_elem<DIM, T, Q2>), dim3(g), dim3(RBS), 0, s, nn, coords, ne, elems,
                           static_cast<const T*>(fq), static_cast<T*>(b2D), f, ctr, cs.slots());
    cs.finish(ctr, s, 0, 2);
    return PF_OK;
}

template <int DIM, typename T>
void launch_energies(int qn, int grid, int64_t nn, const double* coords, int64_t ne, const int32_t* elems,
                     const void* cKq, const void* cMq, const void* u, const void* b2D, void* J, double* part,
                     Fallback f, int64_t* ctr, hipStream_t s) {
    constexpr int Q2 = DIM == 2 ? 3 : 4;
    if (qn == 1)
        hipLaunchKernelGGL((k_energies<DIM, T, 1>), dim3(grid), dim3(RBS), 0, s, nn, coords, ne, elems,
                           static_cast<const T*>(cKq), static_cast<const T*>(cMq), static_cast<const T*>(u),
                           static_cast<const T*>(b2D), static_cast<T*>(J), part, f, ctr);
    else
        hipLaunchKernelGGL((k_energies<DIM, T, Q2>), dim3(grid), dim3(RBS), 0, s, nn, coords, ne, elems,
                           static_cast<const T*>(cKq), static_cast<const T*>(cMq), static_cast<const T*>(u),
                           static_cast<const T*>(b2D), static_cast<T*>(J), part, f, ctr);
}

}  // namespace
}  // namespace pf

using namespace pf;

pf_status pf_rhs(const pf_csr* csr, pf_dtype prec, const double* coords, const int32_t* elems, int order,
                 const void* fq, void* b2D, void* b, const pf_fallback* fb, int64_t* d_counters, void* stream) {
    pf_status st = check_csr_mesh(csr, coords, elems, "pf_rhs");
    if (st) return st;
    const int dim = csr_dim(csr);
    const int qn = quad_count(dim, order);
    if (!qn) return fail(PF_EINVAL, "pf_rhs: order must be 1 or 2");
    if (prec != PF_F32 && prec != PF_F64) return fail(PF_EDTYPE, "pf_rhs: prec must be PF_F32 or PF_F64");
    const int64_t nn = csr_nn(csr), ne = csr_ne(csr);
    if (ne > 0 && (!fq || !b2D)) return fail(PF_EINVAL, "pf_rhs: null fq or b2D");
    hipStream_t s = as_stream(stream);
    if ((st = csr_order(csr, s))) return st;
    const Fallback f = make_fallback(fb);
    if (ne > 0) {
        if (dim == 3)
            st = prec == PF_F32 ? launch_rhs_elem<3, float>(qn, nn, coords, ne, elems, fq, b2D, f, d_counters, s)
                                : launch_rhs_elem<3, double>(qn, nn, coords, ne, elems, fq, b2D, f, d_counters, s);
        else
            st = prec == PF_F32 ? launch_rhs_elem<2, float>(qn, nn, coords, ne, elems, fq, b2D, f, d_counters, s)
                                : launch_rhs_elem<2, double>(qn, nn, coords, ne, elems, fq, b2D, f, d_counters, s);
        if (st) return st;
        if ((st = launch_check("pf_rhs elements"))) return st;
    }
    if (b && nn > 0) {
        const unsigned g = static_cast<unsigned>(ceil_div(ceil_div(nn, RHS_ROWS) * 32, RBS));  // half waves
        if (prec == PF_F32)
            hipLaunchKernelGGL(k_rhs_nodes<float>, dim3(g), dim3(RBS), 0, s, nn, dim + 1, csr_aptr(csr),
                               csr_adj(csr), static_cast<const float*>(b2D), static_cast<float*>(b));
        else
            hipLaunchKernelGGL(k_rhs_nodes<double>, dim3(g), dim3(RBS), 0, s, nn, dim + 1, csr_aptr(csr),
                               csr_adj(csr), static_cast<const double*>(b2D), static_cast<double*>(b));
        if ((st = launch_check("pf_rhs nodes"))) return st;
    }
    return PF_OK;
}

namespace pf {
namespace {

// Shared body of pf_energies and pf_energies_noalloc: `part` holds 3 FP64 block sums per
// block of the energy kernel (every block writes its three, so nothing needs clearing).
pf_status energies_into(const pf_csr* csr, pf_dtype prec, const double* coords, const int32_t* elems, int order,
                        const void* cKq, const void* cMq, const void* u, const void* b2D, void* J, double* totals,
                        const pf_fallback* fb, int64_t* d_counters, hipStream_t s, double* part, int grid) {
    const int dim = csr_dim(csr);
    const int qn = quad_count(dim, order);
    const int64_t nn = csr_nn(csr), ne = csr_ne(csr);
    const Fallback f = make_fallback(fb);
    pf_status st;
    if (dim == 3) {
        if (prec == PF_F32)
            launch_energies<3, float>(qn, grid, nn, coords, ne, elems, cKq, cMq, u, b2D, J, part, f, d_counters, s);
        else
            launch_energies<3, double>(qn, grid, nn, coords, ne, elems, cKq, cMq, u, b2D, J, part, f, d_counters, s);
    } else {
        if (prec == PF_F32)
            launch_energies<2, float>(qn, grid, nn, coords, ne, elems, cKq, cMq, u, b2D, J, part, f, d_counters, s);
        else
            launch_energies<2, double>(qn, grid, nn, coords, ne, elems, cKq, cMq, u, b2D, J, part, f, d_counters, s);
    }
    if ((st = launch_check("pf_energies"))) return st;
    if (totals) {
        hipLaunchKernelGGL(k_energy_totals, dim3(1), dim3(192), 0, s, part, grid, totals);
        if ((st = launch_check("pf_energies totals"))) return st;
    }
    return PF_OK;
}

// argument checks of both entry points; on success *grid = the energy kernel's block count
pf_status energies_check(const pf_csr* csr, pf_dtype prec, const double* coords, const int32_t* elems, int order,
                         const void* u, const char* who, int* grid) {
    pf_status st = check_csr_mesh(csr, coords, elems, who);
    if (st) return st;
    if (!quad_count(csr_dim(csr), order)) return fail(PF_EINVAL, std::string(who) + ": order must be 1 or 2");
    if (prec != PF_F32 && prec != PF_F64)
        return fail(PF_EDTYPE, std::string(who) + ": prec must be PF_F32 or PF_F64");
    const int64_t ne = csr_ne(csr);
    if (ne > 0 && !u) return fail(PF_EINVAL, std::string(who) + ": null u");
    *grid = static_cast<int>(std::max<int64_t>(std::min<int64_t>(ceil_div(ne, RBS), ETOT_BLOCKS), 1));
    return PF_OK;
}

// Block sums of pf_energies_noalloc: one copy of this array per device, held until the process
// ends.  Host code never passes the array's name to a kernel (on the host it is a stand-in,
// not a device address): it uses the address hipGetSymbolAddress returns for the current
// device, kept in scratch_dev.
constexpr int SCRATCH_WORDS = 3 * ETOT_BLOCKS;
__device__ __align__(256) double scratch[SCRATCH_WORDS];
constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_dev[SCRATCH_DEVICES] = {};

pf_status scratch_of_current_device(double** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(PF_EHIP, "pf_energies_noalloc: hipGetDevice failed");
    if (dev < 0 || dev >= SCRATCH_DEVICES)
        return fail(PF_EINVAL, "pf_energies_noalloc: device ordinal beyond the supported 64");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PF_EHIP, std::string("pf_energies_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = scratch_dev[dev];
    return PF_OK;
}

}  // namespace
}  // namespace pf

pf_status pf_energies(pf_csr* csr, pf_dtype prec, const double* coords, const int32_t* elems, int order,
                      const void* cKq, const void* cMq, const void* u, const void* b2D, void* J, double* totals,
                      const pf_fallback* fb, int64_t* d_counters, void* stream) {
    int grid = 0;
    pf_status st = energies_check(csr, prec, coords, elems, order, u, "pf_energies", &grid);
    if (st) return st;
    double* part = nullptr;
    if ((st = csr_workspace(csr, 3 * static_cast<int64_t>(grid), &part, as_stream(stream)))) return st;
    return energies_into(csr, prec, coords, elems, order, cKq, cMq, u, b2D, J, totals, fb, d_counters,
                         as_stream(stream), part, grid);
}

pf_status pf_energies_noalloc(const pf_csr* csr, pf_dtype prec, const double* coords, const int32_t* elems,
                              int order, const void* cKq, const void* cMq, const void* u, const void* b2D, void* J,
                              double* totals, const pf_fallback* fb, int64_t* d_counters, void* stream) {
    int grid = 0;
    pf_status st = energies_check(csr, prec, coords, elems, order, u, "pf_energies_noalloc", &grid);
    if (st) return st;
    if (3 * grid > SCRATCH_WORDS)
        return fail(PF_EINVAL, "pf_energies_noalloc: the energy kernel needs more block sums than the static "
                               "scratch holds");
    double* part = nullptr;
    if ((st = scratch_of_current_device(&part))) return st;
    return energies_into(csr, prec, coords, elems, order, cKq, cMq, u, b2D, J, totals, fb, d_counters,
                         as_stream(stream), part, grid);
}
