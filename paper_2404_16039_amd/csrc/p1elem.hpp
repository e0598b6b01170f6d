// p1elem.hpp -- per-element P1 geometry in registers (section 3.6 derivative routine with
// one integration point; section 3.2 volumes and normals).
//
// With edges e_k = p_{k+1} - p_1 (the columns of J), the inverse transpose of J has the
// cofactor vectors as columns: c_1 = e_2 x e_3, c_2 = e_3 x e_1, c_3 = e_1 x e_2 (3-D), or
// the rotated edges (2-D), divided by det J = e_1 . c_1.  The barycentric gradients
// (the routine's dphi = tjac^{-1} dshape with the P1 reference derivatives) are therefore
// grad phi_j = c_j / det for j >= 1 and grad phi_0 = -(c_1 + ... + c_d) / det, and the P1
// stiffness entry |T| grad phi_a . grad phi_b equals (c_a . c_b) / (d! |det|).
// Precision: the determinant is compensated -- c_1 by Kahan's FMA scheme (each component
// within 2 ulp), then det = e_1 . c_1 as a Dot2 sum (FMA-split products, compensated sum) --
// so its arithmetic error is at most (1 + 2 kappa) u |det| with kappa the det-condition
// sum_j |e_1j c_1j| / |det| that the routing predicate tests.  The other cofactors take one
// FMA per component: their error stays within a few u |e_k||e_l|, the size of what the
// rounding of the edge vectors themselves (from FP64 coordinates) already puts there.
#pragma once

#include "smallmat.hpp"

namespace pf {

template <int DIM, typename C>
struct P1Geom {
    C c[DIM + 1][DIM];  // c[j] = det * grad phi_j
    C det;              // signed det J (first node origin)
    C absterms;         // sum_j |e_1j c_1j|, numerator of the det-condition
    double shape2;      // FP32 geometry: prod_k |e_k|^2 (FP64), numerator of the squared vertex shape
};

// Vertex shape of an element seen from its origin node: sigma = prod_k |e_k| / |det J|, the
// product of the lengths of the edges from that node over the volume factor.  sigma >= 1/sin
// of every angle between two of those edges and bounds the cancellation in the origin node's
// gradient -(c_1 + ... + c_d), so it bounds what the FP32 rounding of the edge vectors costs
// the gradients and the stiffness entries relative to their scale |grad phi_a| |grad phi_b|:
// about 7 sigma u_32.  The FP32 element paths send an element with sigma > SHAPE_MAX to FP64
// (whenever routing is enabled), which keeps that cost below 1e-5 of the scale; sigma >= the
// det-condition / sqrt(d), so this also covers det-conditions above ~28.  Regular elements
// have sigma of a few units (the jittered Kuhn tetrahedra at most 6.5).
constexpr double SHAPE_MAX = 16.0;

template <int DIM, typename C>
__device__ __forceinline__ double edge_lengths2(const C (&u)[DIM][DIM]) {
    double p = 1.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        C l = u[k][0] * u[k][0];
#pragma unroll
        for (int i = 1; i < DIM; ++i) l = fmaT(u[k][i], u[k][i], l);
        p *= static_cast<double>(l);
    }
    return p;
}

// the vertex shape test of an FP32 geometry (sigma > SHAPE_MAX, FP64 comparison: no range of
// coordinates overflows it)
template <int DIM>
__device__ __forceinline__ bool shape_exceeds(const P1Geom<DIM, float>& g) {
    const double d = static_cast<double>(g.det);
    return g.shape2 > SHAPE_MAX * SHAPE_MAX * d * d;
}

// Geometry from edge vectors already in precision C (u[k] = p_{k+1} - p_origin).
template <int DIM, typename C>
__device__ __forceinline__ void p1_geom_edges(const C (&u)[DIM][DIM], P1Geom<DIM, C>& g) {
    if constexpr (DIM == 3) {
        // c_1 = e_2 x e_3 (Kahan), det = e_1 . c_1 compensated
        g.c[1][0] = det2(u[1][1], u[1][2], u[2][1], u[2][2]);
        g.c[1][1] = det2(u[1][2], u[1][0], u[2][2], u[2][0]);
        g.c[1][2] = det2(u[1][0], u[1][1], u[2][0], u[2][1]);
        g.det = dot_comp<C, 3>(u[0], g.c[1], g.absterms);
#pragma unroll
        for (int j = 2; j <= 3; ++j) {
            const C* x = u[j % 3];  // c_2 = e_3 x e_1, c_3 = e_1 x e_2, one FMA per component
            const C* y = u[(j + 1) % 3];
            g.c[j][0] = fmaT(x[1], y[2], -(x[2] * y[1]));
            g.c[j][1] = fmaT(x[2], y[0], -(x[0] * y[2]));
            g.c[j][2] = fmaT(x[0], y[1], -(x[1] * y[0]));
        }
    } else {
        g.c[1][0] = u[1][1];
        g.c[1][1] = -u[1][0];
        g.c[2][0] = -u[0][1];
        g.c[2][1] = u[0][0];
        g.det = det2(u[0][0], u[0][1], u[1][0], u[1][1]);
        g.absterms = fabs(u[0][0] * u[1][1]) + fabs(u[0][1] * u[1][0]);
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
        C s = g.c[1][i];
#pragma unroll
        for (int j = 2; j <= DIM; ++j) s += g.c[j][i];
        g.c[0][i] = -s;
    }
    g.shape2 = sizeof(C) == 4 ? edge_lengths2<DIM, C>(u) : 0.0;
}

// FP32 geometry for the bulk of well-shaped elements: c_1 and det are first evaluated with one
// rounding per product (FMA), which is within (3 kappa + 2 kappa_L) u of |det| (kappa the
// det-condition, kappa_L the sum of the six |Leibniz products| over |det|); only where kappa > 4
// (or det is not finite) are c_1 and det recomputed compensated as in p1_geom_edges, so the
// determinant of every element is within a few tens of u of the exact one, and within
// (1 + 2 kappa) u wherever kappa is large.  2-D elements take p1_geom_edges.
template <int DIM>
__device__ __forceinline__ void p1_geom_edges_fast(const float (&u)[DIM][DIM], P1Geom<DIM, float>& g) {
    if constexpr (DIM == 3) {
        g.c[1][0] = fmaf(u[1][1], u[2][2], -(u[1][2] * u[2][1]));
        g.c[1][1] = fmaf(u[1][2], u[2][0], -(u[1][0] * u[2][2]));
        g.c[1][2] = fmaf(u[1][0], u[2][1], -(u[1][1] * u[2][0]));
        g.det = fmaf(u[0][0], g.c[1][0], fmaf(u[0][1], g.c[1][1], u[0][2] * g.c[1][2]));
        g.absterms = fmaf(fabsf(u[0][0]), fabsf(g.c[1][0]),
                          fmaf(fabsf(u[0][1]), fabsf(g.c[1][1]), fabsf(u[0][2]) * fabsf(g.c[1][2])));
        if (!(g.absterms <= 4.0f * fabsf(g.det))) {
            g.c[1][0] = det2(u[1][1], u[1][2], u[2][1], u[2][2]);
            g.c[1][1] = det2(u[1][2], u[1][0], u[2][2], u[2][0]);
            g.c[1][2] = det2(u[1][0], u[1][1], u[2][0], u[2][1]);
            g.det = dot_comp<float, 3>(u[0], g.c[1], g.absterms);
        }
#pragma unroll
        for (int j = 2; j <= 3; ++j) {
            const float* x = u[j % 3];
            const float* y = u[(j + 1) % 3];
            g.c[j][0] = fmaf(x[1], y[2], -(x[2] * y[1]));
            g.c[j][1] = fmaf(x[2], y[0], -(x[0] * y[2]));
            g.c[j][2] = fmaf(x[0], y[1], -(x[1] * y[0]));
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) g.c[0][i] = -(g.c[1][i] + g.c[2][i] + g.c[3][i]);
        g.shape2 = edge_lengths2<DIM, float>(u);
    } else {
        p1_geom_edges<DIM, float>(u, g);
    }
}

// routing of an FP32 element geometry: pf_fallback's predicate on |det| and the det-condition,
// or (routing enabled) a vertex shape above SHAPE_MAX
template <int DIM>
__device__ __forceinline__ bool route_elem(const P1Geom<DIM, float>& g, const Fallback& fb) {
    return should_route(g.det, g.absterms, fb) || (fb.enable && shape_exceeds<DIM>(g));
}

// Geometry from FP64 edge vectors, rounded once to precision C.
template <int DIM, typename C>
__device__ __forceinline__ void p1_geom(const double (&e)[DIM][DIM], P1Geom<DIM, C>& g) {
    C u[DIM][DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int i = 0; i < DIM; ++i) u[k][i] = static_cast<C>(e[k][i]);
    p1_geom_edges<DIM, C>(u, g);
}

template <int DIM>
__device__ __forceinline__ constexpr double fact_dim() {
    return DIM == 2 ? 2.0 : 6.0;
}

// gather the element's node coordinates and form the FP64 edge vectors; returns false on
// an out-of-range node id
template <int DIM>
__device__ __forceinline__ bool p1_edges(const double* __restrict__ coords, int64_t nn, const int (&nd)[DIM + 1],
                                         double (&e)[DIM][DIM]) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j <= DIM; ++j) ok = ok && (nd[j] >= 0) && (nd[j] < nn);
    if (!ok) return false;
    double p0[DIM];
#pragma unroll
    for (int i = 0; i < DIM; ++i) p0[i] = coords[static_cast<int64_t>(nd[0]) * DIM + i];
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int i = 0; i < DIM; ++i) e[k][i] = coords[static_cast<int64_t>(nd[k + 1]) * DIM + i] - p0[i];
    return true;
}

template <int DIM>
__device__ __forceinline__ void load_nodes(const int32_t* __restrict__ elems, int64_t e, int (&nd)[DIM + 1]) {
    if constexpr (DIM == 3) {
        if ((reinterpret_cast<uintptr_t>(elems) & 15) == 0) {
            const int4 v = *reinterpret_cast<const int4*>(elems + e * 4);
            nd[0] = v.x;
            nd[1] = v.y;
            nd[2] = v.z;
            nd[3] = v.w;
        } else {
            const int32_t* p = elems + e * 4;
            nd[0] = p[0];
            nd[1] = p[1];
            nd[2] = p[2];
            nd[3] = p[3];
        }
    } else {
        const int32_t* p = elems + e * 3;
        nd[0] = p[0];
        nd[1] = p[1];
        nd[2] = p[2];
    }
}

}  // namespace pf
