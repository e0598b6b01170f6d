// elements.hip -- per-element P1 geometry, stiffness and mass matrices (section 3.6), and
// boundary facet normals and measures (section 3.2).  One element (or facet) per lane.
#include "p1elem.hpp"
#include "quadrature.hpp"
#include "internal.hpp"

namespace pf {

constexpr int EBS = 256;

struct ElemOut {
    void* det;
    void* vol;
    void* grads;
    void* normals;
    void* facet;
    void* K3D;
    void* M3D;
};

// Every output of one element in precision C, rounded to T, in registers: the gradients of
// the barycentric functions (their negatives are the normals3D columns), the facet measures,
// the K page (column-major, symmetric) and the two values of the M page.
template <int DIM, typename T>
struct ElemVals {
    static constexpr int NLB = DIM + 1;
    T det, vol;
    T grad[DIM * NLB];
    T facet[NLB];
    T K[NLB * NLB];
    T mo, md;
};

template <int DIM, typename C, typename T>
__device__ __forceinline__ void elem_values(const P1Geom<DIM, C>& g, C ck, C cm, const ElemOut& o,
                                            ElemVals<DIM, T>& v) {
    constexpr int NLB = DIM + 1;
    const C det = g.det;
    const C adet = fabs(det);
    const C vol = adet / static_cast<C>(fact_dim<DIM>());
    v.det = static_cast<T>(det);
    v.vol = static_cast<T>(vol);
    if (o.grads || o.normals) {
        const C inv_det = C(1) / det;
#pragma unroll
        for (int j = 0; j < NLB; ++j)
#pragma unroll
            for (int i = 0; i < DIM; ++i) v.grad[i + j * DIM] = static_cast<T>(g.c[j][i] * inv_det);
    }
    if (o.facet) {
        // facet opposite node j: dim |T| |grad phi_j| = |c_j| / (dim-1)!
#pragma unroll
        for (int j = 0; j < NLB; ++j) {
            C s = g.c[j][0] * g.c[j][0];
#pragma unroll
            for (int i = 1; i < DIM; ++i) s = fmaT(g.c[j][i], g.c[j][i], s);
            v.facet[j] = static_cast<T>(DIM == 3 ? C(0.5) * sqrt(s) : sqrt(s));
        }
    }
    if (o.K3D) {
        const C kf = ck / (static_cast<C>(fact_dim<DIM>()) * adet);
#pragma unroll
        for (int b = 0; b < NLB; ++b)
#pragma unroll
            for (int a = b; a < NLB; ++a) {
                C s = g.c[a][0] * g.c[b][0];
#pragma unroll
                for (int i = 1; i < DIM; ++i) s = fmaT(g.c[a][i], g.c[b][i], s);
                const T x = static_cast<T>(kf * s);
                v.K[a + b * NLB] = x;
                v.K[b + a * NLB] = x;
            }
    }
    if (o.M3D) {
        const C mo = cm * vol / static_cast<C>((DIM + 1) * (DIM + 2));
        v.mo = static_cast<T>(mo);
        v.md = static_cast<T>(mo + mo);
    }
}

// One output array of W values per element, through LDS: every lane puts its element's
// values at stride W + 1 (odd: the lanes of a wave hit different banks), then the block
// stores its elements' contiguous run with consecutive lanes on consecutive words.  Elements
// with a bad node index (okb 0) keep the caller's values.  Called by every thread.
template <int W, typename T>
__device__ __forceinline__ void stage_store(T* __restrict__ out, int64_t e0, int nloc, const T (&v)[W],
                                            T* __restrict__ buf, const uint8_t* __restrict__ okb) {
    const int t = static_cast<int>(threadIdx.x);
#pragma unroll
    for (int i = 0; i < W; ++i) buf[t * (W + 1) + i] = v[i];
    __syncthreads();
    for (int k = t; k < nloc * W; k += EBS) {
        const int el = k / W;
        if (okb[el]) out[e0 * W + k] = buf[el * (W + 1) + (k - el * W)];
    }
    __syncthreads();
}

template <int DIM, typename T>
__global__ __launch_bounds__(EBS) void k_elem(int64_t nn, const double* __restrict__ coords, int64_t ne,
                                              const int32_t* __restrict__ elems, const T* __restrict__ cK,
                                              const T* __restrict__ cM, ElemOut o, Fallback fb,
                                              uint8_t* __restrict__ flags, int64_t* d_counters,
                                              int32_t* __restrict__ bcnt) {
    constexpr int NLB = DIM + 1;
    constexpr int WMAX = NLB * NLB;
    __shared__ __align__(16) T buf[EBS * (WMAX + 1)];
    __shared__ uint8_t okb[EBS];
    const int64_t e0 = static_cast<int64_t>(blockIdx.x) * EBS;
    const int64_t e = e0 + threadIdx.x;
    const int nloc = static_cast<int>(ne - e0 < EBS ? ne - e0 : EBS);
    bool routed = false, sing = false, bad = false;
    ElemVals<DIM, T> v{};
    if (e < ne) {
        int nd[DIM + 1];
        load_nodes<DIM>(elems, e, nd);
        double ev[DIM][DIM];
        bad = !p1_edges<DIM>(coords, nn, nd, ev);
        if (!bad) {
            const T ck = cK ? cK[e] : T(1);
            const T cm = cM ? cM[e] : T(1);
            if constexpr (sizeof(T) == 4) {
                P1Geom<DIM, float> g;
                p1_geom<DIM, float>(ev, g);
                routed = route_elem<DIM>(g, fb);
                if (routed) {
                    P1Geom<DIM, double> gd;
                    p1_geom<DIM, double>(ev, gd);
                    sing = (gd.det == 0.0);
                    elem_values<DIM, double, T>(gd, ck, cm, o, v);
                } else {
                    sing = (g.det == 0.0f);
                    elem_values<DIM, float, T>(g, ck, cm, o, v);
                }
            } else {
                P1Geom<DIM, double> gd;
                p1_geom<DIM, double>(ev, gd);
                sing = (gd.det == 0.0);
                elem_values<DIM, double, T>(gd, ck, cm, o, v);
            }
            // one value per element: consecutive lanes, consecutive words already
            if (o.det) static_cast<T*>(o.det)[e] = v.det;
            if (o.vol) static_cast<T*>(o.vol)[e] = v.vol;
        }
        if (flags)
            flags[e] = (sing ? FLAG_SINGULAR : 0) | (routed ? FLAG_ROUTED : 0) | (bad ? FLAG_BADINDEX : 0);
    }
    okb[threadIdx.x] = (e < ne && !bad) ? 1 : 0;
    block_counts<3, EBS>(d_counters, bcnt, {0, 1, 2}, {routed ? 1 : 0, sing ? 1 : 0, bad ? 1 : 0});
    // the multi-value outputs, one array at a time through LDS (the requests are the same for
    // the whole block)
    if (o.grads) stage_store<DIM * NLB, T>(static_cast<T*>(o.grads), e0, nloc, v.grad, buf, okb);
    if (o.normals) {
        T nv[DIM * NLB];
#pragma unroll
        for (int i = 0; i < DIM * NLB; ++i) nv[i] = -v.grad[i];
        stage_store<DIM * NLB, T>(static_cast<T*>(o.normals), e0, nloc, nv, buf, okb);
    }
    if (o.facet) stage_store<NLB, T>(static_cast<T*>(o.facet), e0, nloc, v.facet, buf, okb);
    if (o.K3D) stage_store<NLB * NLB, T>(static_cast<T*>(o.K3D), e0, nloc, v.K, buf, okb);
    if (o.M3D) {
        T mv[NLB * NLB];
#pragma unroll
        for (int b = 0; b < NLB; ++b)
#pragma unroll
            for (int a = 0; a < NLB; ++a) mv[a + b * NLB] = a == b ? v.md : v.mo;
        stage_store<NLB * NLB, T>(static_cast<T*>(o.M3D), e0, nloc, mv, buf, okb);
    }
}

// boundary facets: 3-D triangles (a,b,c): n = (b-a) x (c-a), measure |n|/2;
// 2-D edges (a,b): n = (b_y - a_y, a_x - b_x), measure |n|
template <int DIM, typename T>
__global__ __launch_bounds__(EBS) void k_boundary(int64_t nn, const double* __restrict__ coords, int64_t nf,
                                                  const int32_t* __restrict__ faces, T* __restrict__ unit,
                                                  T* __restrict__ measure) {
    const int64_t f = static_cast<int64_t>(blockIdx.x) * EBS + threadIdx.x;
    if (f >= nf) return;
    int nd[DIM];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        nd[j] = faces[f * DIM + j];
        ok = ok && nd[j] >= 0 && nd[j] < nn;
    }
    T n[DIM];
    if (!ok) {
#pragma unroll
        for (int i = 0; i < DIM; ++i) n[i] = static_cast<T>(NAN);
    } else if constexpr (DIM == 3) {
        double pa[3], u[3], v[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) pa[i] = coords[static_cast<int64_t>(nd[0]) * 3 + i];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            u[i] = coords[static_cast<int64_t>(nd[1]) * 3 + i] - pa[i];
            v[i] = coords[static_cast<int64_t>(nd[2]) * 3 + i] - pa[i];
        }
        T x[3], y[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            x[i] = static_cast<T>(u[i]);
            y[i] = static_cast<T>(v[i]);
        }
        n[0] = det2(x[1], x[2], y[1], y[2]);
        n[1] = det2(x[2], x[0], y[2], y[0]);
        n[2] = det2(x[0], x[1], y[0], y[1]);
    } else {
        const int64_t a = nd[0], b = nd[1];
        n[0] = static_cast<T>(coords[b * 2 + 1] - coords[a * 2 + 1]);
        n[1] = static_cast<T>(coords[a * 2] - coords[b * 2]);
    }
    T s = n[0] * n[0];
#pragma unroll
    for (int i = 1; i < DIM; ++i) s = fmaT(n[i], n[i], s);
    const T len = sqrt(s);
    if (measure) measure[f] = DIM == 3 ? T(0.5) * len : len;
    if (unit) {
        const T il = T(1) / len;
#pragma unroll
        for (int i = 0; i < DIM; ++i) unit[f * DIM + i] = n[i] * il;
    }
}

// Physical integration points x_q = sum_j lam(q, j) p_j of every element (FP64, products
// and sums in node order without contraction), stored element-major: xq[(e*QN + q)*DIM + i].
template <int DIM, int QN>
__global__ __launch_bounds__(EBS) void k_quad_points(int64_t nn, const double* __restrict__ coords, int64_t ne,
                                                     const int32_t* __restrict__ elems, double* __restrict__ xq) {
    constexpr int NLB = DIM + 1;
    const int64_t e = static_cast<int64_t>(blockIdx.x) * EBS + threadIdx.x;
    if (e >= ne) return;
    double p[NLB][DIM];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < NLB; ++j) {
        const int64_t node = elems[e * NLB + j];
        ok = ok && node >= 0 && node < nn;
#pragma unroll
        for (int i = 0; i < DIM; ++i) p[j][i] = ok ? coords[node * DIM + i] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < QN; ++q)
#pragma unroll
        for (int i = 0; i < DIM; ++i) {
            double x = 0.0;
#pragma unroll
            for (int j = 0; j < NLB; ++j) x += QuadRule<DIM, QN>::lam(q, j) * p[j][i];
            xq[(e * QN + q) * DIM + i] = ok ? x : NAN;
        }
}

namespace {

pf_status check_mesh(int dim, int64_t nn, const double* coords, int64_t ne, const int32_t* elems, const char* who) {
    if (dim != 2 && dim != 3) return fail(PF_EORDER, std::string(who) + ": dim must be 2 or 3");
    if (nn < 0 || ne < 0) return fail(PF_EINVAL, std::string(who) + ": negative size");
    if (nn > INT32_MAX) return fail(PF_ELIMIT, std::string(who) + ": nn must be < 2^31");
    if (ne > 0 && (!coords || !elems)) return fail(PF_EINVAL, std::string(who) + ": null coords or elems");
    return PF_OK;
}

template <int DIM, typename T>
pf_status launch_elem(int64_t nn, const double* coords, int64_t ne, const int32_t* elems, const void* cK,
                      const void* cM, const ElemOut& o, Fallback fb, uint8_t* flags, int64_t* ctr, hipStream_t s) {
    const int64_t g = ceil_div(ne, EBS);
    BlockCountSlots<3> cs;
    if (pf_status st = cs.init(ctr, g, s)) return st;
    hipLaunchKernelGGL((k_elem<DIM, T>), dim3(static_cast<unsigned>(g)), dim3(EBS), 0, s, nn, coords, ne, elems,
                       static_cast<const T*>(cK), static_cast<const T*>(cM), o, fb, flags, ctr, cs.slots());
    cs.finish(ctr, s, 0, 1, 2);
    return launch_check("element kernel");
}

pf_status elem_dispatch(int dim, pf_dtype prec, int64_t nn, const double* coords, int64_t ne, const int32_t* elems,
                        const void* cK, const void* cM, const ElemOut& o, const pf_fallback* fb, uint8_t* flags,
                        int64_t* ctr, void* stream, const char* who) {
    pf_status st = check_mesh(dim, nn, coords, ne, elems, who);
    if (st) return st;
    if (ne == 0) return PF_OK;
    Fallback f = make_fallback(fb);
    hipStream_t s = as_stream(stream);
    if (prec == PF_F32) {
        return dim == 2 ? launch_elem<2, float>(nn, coords, ne, elems, cK, cM, o, f, flags, ctr, s)
                        : launch_elem<3, float>(nn, coords, ne, elems, cK, cM, o, f, flags, ctr, s);
    }
    if (prec == PF_F64) {
        return dim == 2 ? launch_elem<2, double>(nn, coords, ne, elems, cK, cM, o, f, flags, ctr, s)
                        : launch_elem<3, double>(nn, coords, ne, elems, cK, cM, o, f, flags, ctr, s);
    }
    return fail(PF_EDTYPE, std::string(who) + ": prec must be PF_F32 or PF_F64");
}

}  // namespace
}  // namespace pf

using namespace pf;

extern "C" {

pf_status pf_elem_geometry(int dim, pf_dtype prec, int64_t nn, const double* coords, int64_t ne, const int32_t* elems,
                           void* det, void* vol, void* grads, void* normals, void* facet, const pf_fallback* fb,
                           uint8_t* flags, int64_t* d_counters, void* stream) {
    ElemOut o{det, vol, grads, normals, facet, nullptr, nullptr};
    return elem_dispatch(dim, prec, nn, coords, ne, elems, nullptr, nullptr, o, fb, flags, d_counters, stream,
                         "pf_elem_geometry");
}

pf_status pf_elem_stiffness_mass(int dim, pf_dtype prec, int64_t nn, const double* coords, int64_t ne,
                                 const int32_t* elems, const void* cK, const void* cM, void* K3D, void* M3D,
                                 const pf_fallback* fb, uint8_t* flags, int64_t* d_counters, void* stream) {
    ElemOut o{nullptr, nullptr, nullptr, nullptr, nullptr, K3D, M3D};
    return elem_dispatch(dim, prec, nn, coords, ne, elems, cK, cM, o, fb, flags, d_counters, stream,
                         "pf_elem_stiffness_mass");
}

pf_status pf_quad_points(int dim, int order, int64_t nn, const double* coords, int64_t ne, const int32_t* elems,
                         double* xq, void* stream) {
    pf_status st = check_mesh(dim, nn, coords, ne, elems, "pf_quad_points");
    if (st) return st;
    const int qn = quad_count(dim, order);
    if (!qn) return fail(PF_EINVAL, "pf_quad_points: order must be 1 or 2");
    if (ne == 0) return PF_OK;
    if (!xq) return fail(PF_EINVAL, "pf_quad_points: null xq");
    hipStream_t s = as_stream(stream);
    const unsigned g = static_cast<unsigned>(ceil_div(ne, EBS));
    if (dim == 2) {
        if (qn == 1) hipLaunchKernelGGL((k_quad_points<2, 1>), dim3(g), dim3(EBS), 0, s, nn, coords, ne, elems, xq);
        else hipLaunchKernelGGL((k_quad_points<2, 3>), dim3(g), dim3(EBS), 0, s, nn, coords, ne, elems, xq);
    } else {
        if (qn == 1) hipLaunchKernelGGL((k_quad_points<3, 1>), dim3(g), dim3(EBS), 0, s, nn, coords, ne, elems, xq);
        else hipLaunchKernelGGL((k_quad_points<3, 4>), dim3(g), dim3(EBS), 0, s, nn, coords, ne, elems, xq);
    }
    return launch_check("pf_quad_points");
}

pf_status pf_boundary_normals(int dim, pf_dtype prec, int64_t nn, const double* coords, int64_t nf,
                              const int32_t* faces, void* unit, void* measure, void* stream) {
    if (dim != 2 && dim != 3) return fail(PF_EORDER, "pf_boundary_normals: dim must be 2 or 3");
    if (nf < 0 || nn < 0) return fail(PF_EINVAL, "pf_boundary_normals: negative size");
    if (nf == 0) return PF_OK;
    if (!coords || !faces) return fail(PF_EINVAL, "pf_boundary_normals: null coords or faces");
    hipStream_t s = as_stream(stream);
    unsigned g = static_cast<unsigned>(ceil_div(nf, EBS));
    if (prec == PF_F32) {
        if (dim == 3)
            hipLaunchKernelGGL((k_boundary<3, float>), dim3(g), dim3(EBS), 0, s, nn, coords, nf, faces, (float*)unit,
                               (float*)measure);
        else
            hipLaunchKernelGGL((k_boundary<2, float>), dim3(g), dim3(EBS), 0, s, nn, coords, nf, faces, (float*)unit,
                               (float*)measure);
    } else if (prec == PF_F64) {
        if (dim == 3)
            hipLaunchKernelGGL((k_boundary<3, double>), dim3(g), dim3(EBS), 0, s, nn, coords, nf, faces,
                               (double*)unit, (double*)measure);
        else
            hipLaunchKernelGGL((k_boundary<2, double>), dim3(g), dim3(EBS), 0, s, nn, coords, nf, faces,
                               (double*)unit, (double*)measure);
    } else {
        return fail(PF_EDTYPE, "pf_boundary_normals: bad prec");
    }
    return launch_check("pf_boundary_normals");
}

}  // extern "C"
