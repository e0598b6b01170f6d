// p2.hip -- P2 element matrices of straight-sided triangles and tetrahedra (section 3.6,
// stiffness_matrixP2 / mass_matrixP2): one element per lane, K3D and M3D pages written
// once.
//
// Local nodes: the dim + 1 vertices, then the mid-edge nodes of the local edges (0,1),
// (0,2), (1,2) in 2-D or (0,1), (0,2), (0,3), (1,2), (1,3), (2,3) in 3-D.  In barycentric
// coordinates the basis is lam_i (2 lam_i - 1) at vertex i and 4 lam_i lam_j at edge (i,j),
// so grad phi_a = sum_k D_ak grad lam_k with D affine in lam (vertex i: D_ii = 4 lam_i - 1;
// edge (i,j): D_ai = 4 lam_j, D_aj = 4 lam_i).  Hence
//   K_ab = |T| sum_kl G_kl sum_q w_q c_q D_ak(x_q) D_bl(x_q),   G_kl = grad lam_k . grad lam_l,
// needs only the coefficient-weighted moments S0 = sum w c, S1_i = sum w c lam_i and
// S2_ij = sum w c lam_i lam_j of the stiffness rule (any rule), and M_ab = |T| sum_q w_q c_q
// phi_a phi_b is summed point by point.  G comes from the P1 cofactors (grad lam_k = c_k /
// det) in the working precision, with the FP64 recomputation of routed elements.
#include "p1elem.hpp"
#include "internal.hpp"

#include <string>

namespace pf {

constexpr int P2BS = 64;  // elements per block (one wave)

struct P2Rules {
    int nqK, nqM;
    double lamK[PF_P2_RULE_MAX * 4], wK[PF_P2_RULE_MAX];
    double lamM[PF_P2_RULE_MAX * 4], wM[PF_P2_RULE_MAX];
};

template <int DIM>
struct P2Local {
    static constexpr int N = DIM + 1;               // vertices
    static constexpr int NB = DIM == 2 ? 6 : 10;    // basis functions
    // vertices of edge node a (a >= N)
    __device__ static constexpr int ei(int a) {
        return DIM == 2 ? (a == 3 ? 0 : a == 4 ? 0 : 1) : (a <= 6 ? 0 : a <= 8 ? 1 : 2);
    }
    __device__ static constexpr int ej(int a) {
        return DIM == 2 ? (a == 3 ? 1 : 2) : (a == 4 ? 1 : a == 5 ? 2 : a == 6 ? 3 : a == 7 ? 2 : 3);
    }
};

// the stiffness entry (a, b) from the moments: sum_kl G_kl <D_ak D_bl>
template <int DIM, typename C>
__device__ __forceinline__ C p2_kentry(int a, int b, const C (&G)[DIM + 1][DIM + 1], C S0, const C (&S1)[DIM + 1],
                                       const C (&S2)[DIM + 1][DIM + 1]) {
    using L = P2Local<DIM>;
    constexpr int N = L::N;
    // D_ak as (constant, coefficient of lam_m, index m) pairs over the nonzero k of row a
    int ka[2], kb[2], ma[2], mb[2];
    C ca[2], cm_a[2], cb[2], cm_b[2];
    int na, nb;
    if (a < N) {
        na = 1; ka[0] = a; ca[0] = C(-1); cm_a[0] = C(4); ma[0] = a;
    } else {
        na = 2; ka[0] = L::ei(a); ma[0] = L::ej(a); ka[1] = L::ej(a); ma[1] = L::ei(a);
        ca[0] = ca[1] = C(0); cm_a[0] = cm_a[1] = C(4);
    }
    if (b < N) {
        nb = 1; kb[0] = b; cb[0] = C(-1); cm_b[0] = C(4); mb[0] = b;
    } else {
        nb = 2; kb[0] = L::ei(b); mb[0] = L::ej(b); kb[1] = L::ej(b); mb[1] = L::ei(b);
        cb[0] = cb[1] = C(0); cm_b[0] = cm_b[1] = C(4);
    }
    C s = C(0);
    for (int u = 0; u < na; ++u)
        for (int v = 0; v < nb; ++v) {
            // <(ca + cma lam_ma)(cb + cmb lam_mb)> = ca cb S0 + ca cmb S1_mb + cb cma S1_ma + cma cmb S2
            const C mom = ca[u] * cb[v] * S0 + ca[u] * cm_b[v] * S1[mb[v]] + cb[v] * cm_a[u] * S1[ma[u]] +
                          cm_a[u] * cm_b[v] * S2[ma[u]][mb[v]];
            s = fmaT(G[ka[u]][kb[v]], mom, s);
        }
    return s;
}

// position of entry (a, b), a >= b, of a symmetric page stored as its lower triangle
__device__ __forceinline__ constexpr int tri(int a, int b) {
    return a * (a + 1) / 2 + b;
}

// K and M of one element into the staging pages kp, mp (nullable: not requested), each a
// lower triangle (entry (a, b), a >= b, at tri(a, b): both matrices are symmetric); ck, cm:
// the element's coefficients at the points of each rule (nullable: 1)
template <int DIM, typename C, typename T>
__device__ __forceinline__ void p2_write(const P1Geom<DIM, C>& g, const P2Rules& R, const T* ck, const T* cm, T* kp,
                                         T* mp) {
    using L = P2Local<DIM>;
    constexpr int N = L::N, NB = L::NB;
    const C adet = fabs(g.det);
    const C vol = adet / static_cast<C>(fact_dim<DIM>());
    if (kp) {
        // G_kl = c_k . c_l / det^2
        const C id2 = C(1) / (g.det * g.det);
        C G[N][N];
#pragma unroll
        for (int k = 0; k < N; ++k)
#pragma unroll
            for (int l = k; l < N; ++l) {
                C s = g.c[k][0] * g.c[l][0];
#pragma unroll
                for (int i = 1; i < DIM; ++i) s = fmaT(g.c[k][i], g.c[l][i], s);
                G[k][l] = G[l][k] = s * id2;
            }
        C S0 = C(0), S1[N], S2[N][N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            S1[k] = C(0);
#pragma unroll
            for (int l = 0; l < N; ++l) S2[k][l] = C(0);
        }
        for (int q = 0; q < R.nqK; ++q) {
            const C wc = static_cast<C>(R.wK[q]) * (ck ? static_cast<C>(ck[q]) : C(1));
            S0 += wc;
            C lam[N];
#pragma unroll
            for (int k = 0; k < N; ++k) {
                lam[k] = static_cast<C>(R.lamK[q * N + k]);
                S1[k] = fmaT(wc, lam[k], S1[k]);
            }
#pragma unroll
            for (int k = 0; k < N; ++k)
#pragma unroll
                for (int l = k; l < N; ++l) S2[k][l] = fmaT(wc * lam[k], lam[l], S2[k][l]);
        }
#pragma unroll
        for (int k = 0; k < N; ++k)
#pragma unroll
            for (int l = 0; l < k; ++l) S2[k][l] = S2[l][k];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int a = b; a < NB; ++a) {
                kp[tri(a, b)] = static_cast<T>(vol * p2_kentry<DIM, C>(a, b, G, S0, S1, S2));
            }
    }
    if (mp) {
        C m[NB][NB];
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) m[a][b] = C(0);
        for (int q = 0; q < R.nqM; ++q) {
            const C wc = static_cast<C>(R.wM[q]) * (cm ? static_cast<C>(cm[q]) : C(1));
            C lam[N], phi[NB];
#pragma unroll
            for (int k = 0; k < N; ++k) lam[k] = static_cast<C>(R.lamM[q * N + k]);
#pragma unroll
            for (int k = 0; k < N; ++k) phi[k] = lam[k] * fmaT(C(2), lam[k], C(-1));
#pragma unroll
            for (int a = N; a < NB; ++a) phi[a] = C(4) * lam[L::ei(a)] * lam[L::ej(a)];
#pragma unroll
            for (int a = 0; a < NB; ++a) {
                const C wa = wc * phi[a];
#pragma unroll
                for (int b = 0; b <= a; ++b) m[a][b] = fmaT(wa, phi[b], m[a][b]);
            }
        }
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                mp[tri(a, b)] = static_cast<T>(vol * m[a][b]);
            }
    }
}

// One element per lane.  The lanes build their pages in LDS as lower triangles (stride
// NB(NB+1)/2 words, odd, so the lanes' writes fall in different banks; half the LDS of full
// pages, hence more resident waves), then the block copies its elements' contiguous run of
// full pages out with consecutive lanes on consecutive words (coalesced), each word read
// from its triangle position: first the K pages, then the M pages through the same
// staging area.
template <int DIM, typename T>
__global__ __launch_bounds__(P2BS) void k_p2_elem(int64_t nn, const double* __restrict__ coords, int64_t ne,
                                                  const int32_t* __restrict__ elems2, P2Rules R,
                                                  const T* __restrict__ cKq, const T* __restrict__ cMq,
                                                  T* __restrict__ K3D, T* __restrict__ M3D, Fallback fb,
                                                  int64_t* d_counters, int32_t* __restrict__ bcnt) {
    constexpr int NB = P2Local<DIM>::NB;
    constexpr int PS = NB * (NB + 1) / 2;  // staging stride of one page (its lower triangle)
    static_assert(PS % 2 == 1, "an odd stride spreads the lanes over the banks");
    __shared__ T stage[P2BS * PS];
    __shared__ uint8_t trimap[NB * NB];  // column-major page word -> its triangle position
    for (int w = threadIdx.x; w < NB * NB; w += P2BS) {
        const int a = w % NB, b = w / NB;
        trimap[w] = static_cast<uint8_t>(a >= b ? tri(a, b) : tri(b, a));
    }
    const int64_t e0 = static_cast<int64_t>(blockIdx.x) * P2BS;
    const int64_t e = e0 + threadIdx.x;
    const int nel = static_cast<int>(ne - e0 < P2BS ? ne - e0 : P2BS);
    bool routed = false, bad = false;
    double ev[DIM][DIM];
    if (e < ne) {
        int nd[DIM + 1];
#pragma unroll
        for (int j = 0; j <= DIM; ++j) nd[j] = elems2[e * NB + j];
        bad = !p1_edges<DIM>(coords, nn, nd, ev);
#pragma unroll
        for (int j = DIM + 1; j < NB; ++j) {
            const int32_t v = elems2[e * NB + j];
            bad = bad || v < 0 || v >= nn;
        }
    }
    T* page = stage + threadIdx.x * PS;
    for (int which = 0; which < 2; ++which) {  // 0: K, 1: M
        T* out = which == 0 ? K3D : M3D;
        if (!out) continue;
        const T* cq = which == 0 ? cKq : cMq;
        const int nq = which == 0 ? R.nqK : R.nqM;
        const T* cl = cq ? cq + e * nq : nullptr;
        if (e < ne) {
            if (bad) {
                for (int k = 0; k < PS; ++k) page[k] = static_cast<T>(NAN);
            } else {
                T* kp = which == 0 ? page : nullptr;
                T* mp = which == 1 ? page : nullptr;
                bool r = false;
                if constexpr (sizeof(T) == 4) {
                    P1Geom<DIM, float> g;
                    p1_geom<DIM, float>(ev, g);
                    r = route_elem<DIM>(g, fb);
                    if (!r) p2_write<DIM, float, T>(g, R, cl, cl, kp, mp);
                }
                if (sizeof(T) == 8 || r) {
                    P1Geom<DIM, double> gd;
                    p1_geom<DIM, double>(ev, gd);
                    p2_write<DIM, double, T>(gd, R, cl, cl, kp, mp);
                }
                routed = routed || r;
            }
        }
        __syncthreads();
        T* dst = out + e0 * (NB * NB);
        static_assert((NB * NB) % 4 == 0, "a page is a whole number of 4-word groups");
        bool vec = false;
        if constexpr (sizeof(T) == 4) {
            vec = (reinterpret_cast<uintptr_t>(dst) & 15) == 0;
            if (vec) {  // 16-byte stores: four consecutive words per lane
                for (int k = 4 * threadIdx.x; k < nel * NB * NB; k += 4 * P2BS) {
                    const int el = k / (NB * NB), w = k - el * (NB * NB);
                    const T* sp = stage + el * PS;
                    float4 v;
                    v.x = sp[trimap[w]];
                    v.y = sp[trimap[w + 1]];
                    v.z = sp[trimap[w + 2]];
                    v.w = sp[trimap[w + 3]];
                    *reinterpret_cast<float4*>(dst + k) = v;
                }
            }
        }
        if (!vec) {
            for (int k = threadIdx.x; k < nel * NB * NB; k += P2BS) {
                const int el = k / (NB * NB);
                dst[k] = stage[el * PS + trimap[k - el * (NB * NB)]];
            }
        }
        __syncthreads();
    }
    block_counts<2, P2BS>(d_counters, bcnt, {0, 2}, {routed ? 1 : 0, (bad && e < ne) ? 1 : 0});
}

}  // namespace pf

using namespace pf;

pf_status pf_p2_elements(int dim, pf_dtype prec, int64_t nn, const double* coords, int64_t ne, const int32_t* elems2,
                         int nqK, const double* lamK, const double* wK, const void* cKq, int nqM, const double* lamM,
                         const double* wM, const void* cMq, void* K3D, void* M3D, const pf_fallback* fb,
                         int64_t* d_counters, void* stream) {
    if (dim != 2 && dim != 3) return fail(PF_EORDER, "pf_p2_elements: dim must be 2 or 3");
    if (prec != PF_F32 && prec != PF_F64) return fail(PF_EDTYPE, "pf_p2_elements: prec must be PF_F32 or PF_F64");
    if (nn < 0 || ne < 0) return fail(PF_EINVAL, "pf_p2_elements: negative size");
    if (nn > INT32_MAX) return fail(PF_ELIMIT, "pf_p2_elements: nn must be < 2^31");
    if ((K3D && (nqK < 1 || nqK > PF_P2_RULE_MAX || !lamK || !wK)) ||
        (M3D && (nqM < 1 || nqM > PF_P2_RULE_MAX || !lamM || !wM)))
        return fail(PF_EINVAL, "pf_p2_elements: each requested matrix needs a rule of 1..PF_P2_RULE_MAX points");
    if (ne == 0) return PF_OK;
    if (!coords || !elems2) return fail(PF_EINVAL, "pf_p2_elements: null coords or elems");
    P2Rules R{};
    const int n = dim + 1;
    R.nqK = K3D ? nqK : 0;
    R.nqM = M3D ? nqM : 0;
    for (int q = 0; q < R.nqK; ++q) {
        R.wK[q] = wK[q];
        for (int k = 0; k < n; ++k) R.lamK[q * n + k] = lamK[q * n + k];
    }
    for (int q = 0; q < R.nqM; ++q) {
        R.wM[q] = wM[q];
        for (int k = 0; k < n; ++k) R.lamM[q * n + k] = lamM[q * n + k];
    }
    hipStream_t s = as_stream(stream);
    const Fallback f = make_fallback(fb);
    const unsigned g = static_cast<unsigned>(ceil_div(ne, P2BS));
    BlockCountSlots<2> cs;
    if (pf_status st = cs.init(d_counters, g, s)) return st;
    int32_t* bc = cs.slots();
    if (dim == 3) {
        if (prec == PF_F32)
            hipLaunchKernelGGL((k_p2_elem<3, float>), dim3(g), dim3(P2BS), 0, s, nn, coords, ne, elems2, R,
                               static_cast<const float*>(cKq), static_cast<const float*>(cMq),
                               static_cast<float*>(K3D), static_cast<float*>(M3D), f, d_counters, bc);
        else
            hipLaunchKernelGGL((k_p2_elem<3, double>), dim3(g), dim3(P2BS), 0, s, nn, coords, ne, elems2, R,
                               static_cast<const double*>(cKq), static_cast<const double*>(cMq),
                               static_cast<double*>(K3D), static_cast<double*>(M3D), f, d_counters, bc);
    } else {
        if (prec == PF_F32)
            hipLaunchKernelGGL((k_p2_elem<2, float>), dim3(g), dim3(P2BS), 0, s, nn, coords, ne, elems2, R,
                               static_cast<const float*>(cKq), static_cast<const float*>(cMq),
                               static_cast<float*>(K3D), static_cast<float*>(M3D), f, d_counters, bc);
        else
            hipLaunchKernelGGL((k_p2_elem<2, double>), dim3(g), dim3(P2BS), 0, s, nn, coords, ne, elems2, R,
                               static_cast<const double*>(cKq), static_cast<const double*>(cMq),
                               static_cast<double*>(K3D), static_cast<double*>(M3D), f, d_counters, bc);
    }
    cs.finish(d_counters, s, 0, 2);
    return launch_check("pf_p2_elements");
}
