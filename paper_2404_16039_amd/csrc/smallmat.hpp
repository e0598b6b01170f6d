// smallmat.hpp -- register-resident determinants, cofactors and inverses of 1x1..4x4
// column-major pages (element (r, c) at a[r + c*N]).
//
// Determinant and inverse follow section 2.3 of the paper (page-wise determinant; inverse
// on the pages with non-zero determinant) through the adjugate, inv = adj / det.  Accuracy
// in the working precision (FP32 or FP64) does not depend on cancellation:
//   - 2x2 minors are evaluated as double-word values (error-free products and sums), or
//     with Kahan's FMA scheme (within 2 ulp) where a single rounding is enough;
//   - the determinant is the expansion along the first row with double-word cofactors and
//     a compensated sum, so it is within about one ulp of the exact value;
//   - 3x3 cofactors of a 4x4 page are compensated 3-term sums of double-word 2x2 minors.
// Every inverse entry is therefore within a few ulps of the exact entry (componentwise),
// as long as u * (det-condition) stays small; the routing threshold guards that.
#pragma once

#include "common.hpp"

namespace pf {

#define A_(r, c) a[(r) + (c) * N]

template <typename T>
__device__ __forceinline__ T dw_val(const DW<T>& v) {
    return v.hi + v.lo;
}

// 3-term compensated combination x0 y0 + x1 y1 + x2 y2 of double-word y's, as double-word
template <typename T>
__device__ __forceinline__ DW<T> comb3(T x0, DW<T> y0, T x1, DW<T> y1, T x2, DW<T> y2) {
    T x[3] = {x0, x1, x2}, s;
    DW<T> y[3] = {y0, y1, y2};
    return dot_dw<T, 3>(x, y, s);
}

// First-row cofactors C_0j (rounded), determinant (expansion along the first row,
// double-word cofactors, compensated) and the expansion's absolute term sum
// sum_j |a_0j C_0j| (numerator of the det-condition).
template <typename T, int N>
__device__ __forceinline__ void det_first_row(const T* a, T* c0, T& det, T& absterms) {
    if constexpr (N == 1) {
        c0[0] = T(1);
        det = a[0];
        absterms = fabs(a[0]);
    } else if constexpr (N == 2) {
        c0[0] = A_(1, 1);
        c0[1] = -A_(1, 0);
        det = dw_val(dw_det2(A_(0, 0), A_(0, 1), A_(1, 0), A_(1, 1)));
        absterms = fabs(A_(0, 0) * A_(1, 1)) + fabs(A_(0, 1) * A_(1, 0));
    } else if constexpr (N == 3) {
        DW<T> c[3];
        c[0] = dw_det2(A_(1, 1), A_(1, 2), A_(2, 1), A_(2, 2));
        c[1] = dw_det2(A_(1, 2), A_(1, 0), A_(2, 2), A_(2, 0));
        c[2] = dw_det2(A_(1, 0), A_(1, 1), A_(2, 0), A_(2, 1));
        T r0[3] = {A_(0, 0), A_(0, 1), A_(0, 2)};
        det = dw_val(dot_dw<T, 3>(r0, c, absterms));
#pragma unroll
        for (int j = 0; j < 3; ++j) c0[j] = dw_val(c[j]);
    } else {
        // complementary 2x2 minors of rows 2 and 3
        const DW<T> q0 = dw_det2(A_(2, 0), A_(2, 1), A_(3, 0), A_(3, 1));
        const DW<T> q1 = dw_det2(A_(2, 0), A_(2, 2), A_(3, 0), A_(3, 2));
        const DW<T> q2 = dw_det2(A_(2, 0), A_(2, 3), A_(3, 0), A_(3, 3));
        const DW<T> q3 = dw_det2(A_(2, 1), A_(2, 2), A_(3, 1), A_(3, 2));
        const DW<T> q4 = dw_det2(A_(2, 1), A_(2, 3), A_(3, 1), A_(3, 3));
        const DW<T> q5 = dw_det2(A_(2, 2), A_(2, 3), A_(3, 2), A_(3, 3));
        DW<T> c[4];
        c[0] = comb3(A_(1, 1), q5, -A_(1, 2), q4, A_(1, 3), q3);
        c[1] = comb3(-A_(1, 0), q5, A_(1, 2), q2, -A_(1, 3), q1);
        c[2] = comb3(A_(1, 0), q4, -A_(1, 1), q2, A_(1, 3), q0);
        c[3] = comb3(-A_(1, 0), q3, A_(1, 1), q1, -A_(1, 2), q0);
        T r0[4] = {A_(0, 0), A_(0, 1), A_(0, 2), A_(0, 3)};
        det = dw_val(dot_dw<T, 4>(r0, c, absterms));
#pragma unroll
        for (int j = 0; j < 4; ++j) c0[j] = dw_val(c[j]);
    }
}

// Full adjugate: adj[r + c*N] = C_cr (cofactor of a_cr), so that inv = adj / det.
template <typename T, int N>
__device__ __forceinline__ void adjugate(const T* a, T* adj) {
    if constexpr (N == 1) {
        adj[0] = T(1);
    } else if constexpr (N == 2) {
        adj[0] = A_(1, 1);
        adj[1] = -A_(1, 0);
        adj[2] = -A_(0, 1);
        adj[3] = A_(0, 0);
    } else if constexpr (N == 3) {
        // signed cofactor C_ij from cyclic indices, each within 2 ulp (Kahan)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
                adj[j + i * 3] = det2(A_(i1, j1), A_(i1, j2), A_(i2, j1), A_(i2, j2));
            }
    } else {
        const DW<T> s0 = dw_det2(A_(0, 0), A_(0, 1), A_(1, 0), A_(1, 1));
        const DW<T> s1 = dw_det2(A_(0, 0), A_(0, 2), A_(1, 0), A_(1, 2));
        const DW<T> s2 = dw_det2(A_(0, 0), A_(0, 3), A_(1, 0), A_(1, 3));
        const DW<T> s3 = dw_det2(A_(0, 1), A_(0, 2), A_(1, 1), A_(1, 2));
        const DW<T> s4 = dw_det2(A_(0, 1), A_(0, 3), A_(1, 1), A_(1, 3));
        const DW<T> s5 = dw_det2(A_(0, 2), A_(0, 3), A_(1, 2), A_(1, 3));
        const DW<T> q0 = dw_det2(A_(2, 0), A_(2, 1), A_(3, 0), A_(3, 1));
        const DW<T> q1 = dw_det2(A_(2, 0), A_(2, 2), A_(3, 0), A_(3, 2));
        const DW<T> q2 = dw_det2(A_(2, 0), A_(2, 3), A_(3, 0), A_(3, 3));
        const DW<T> q3 = dw_det2(A_(2, 1), A_(2, 2), A_(3, 1), A_(3, 2));
        const DW<T> q4 = dw_det2(A_(2, 1), A_(2, 3), A_(3, 1), A_(3, 3));
        const DW<T> q5 = dw_det2(A_(2, 2), A_(2, 3), A_(3, 2), A_(3, 3));
        // adj(r, c) = C_cr
        adj[0 + 0 * 4] = dw_val(comb3(A_(1, 1), q5, -A_(1, 2), q4, A_(1, 3), q3));
        adj[0 + 1 * 4] = dw_val(comb3(-A_(0, 1), q5, A_(0, 2), q4, -A_(0, 3), q3));
        adj[0 + 2 * 4] = dw_val(comb3(A_(3, 1), s5, -A_(3, 2), s4, A_(3, 3), s3));
        adj[0 + 3 * 4] = dw_val(comb3(-A_(2, 1), s5, A_(2, 2), s4, -A_(2, 3), s3));
        adj[1 + 0 * 4] = dw_val(comb3(-A_(1, 0), q5, A_(1, 2), q2, -A_(1, 3), q1));
        adj[1 + 1 * 4] = dw_val(comb3(A_(0, 0), q5, -A_(0, 2), q2, A_(0, 3), q1));
        adj[1 + 2 * 4] = dw_val(comb3(-A_(3, 0), s5, A_(3, 2), s2, -A_(3, 3), s1));
        adj[1 + 3 * 4] = dw_val(comb3(A_(2, 0), s5, -A_(2, 2), s2, A_(2, 3), s1));
        adj[2 + 0 * 4] = dw_val(comb3(A_(1, 0), q4, -A_(1, 1), q2, A_(1, 3), q0));
        adj[2 + 1 * 4] = dw_val(comb3(-A_(0, 0), q4, A_(0, 1), q2, -A_(0, 3), q0));
        adj[2 + 2 * 4] = dw_val(comb3(A_(3, 0), s4, -A_(3, 1), s2, A_(3, 3), s0));
        adj[2 + 3 * 4] = dw_val(comb3(-A_(2, 0), s4, A_(2, 1), s2, -A_(2, 3), s0));
        adj[3 + 0 * 4] = dw_val(comb3(-A_(1, 0), q3, A_(1, 1), q1, -A_(1, 2), q0));
        adj[3 + 1 * 4] = dw_val(comb3(A_(0, 0), q3, -A_(0, 1), q1, A_(0, 2), q0));
        adj[3 + 2 * 4] = dw_val(comb3(-A_(3, 0), s3, A_(3, 1), s1, -A_(3, 2), s0));
        adj[3 + 3 * 4] = dw_val(comb3(A_(2, 0), s3, -A_(2, 1), s1, A_(2, 2), s0));
    }
}

#undef A_

// Routing decision of the FP32 path (see pf_fallback): route when |det| < tau_abs, the
// det-condition exceeds tau_cond, or det is zero or not finite (the det-condition of a zero
// determinant is infinite, also when every term of the expansion is zero).
template <typename T>
__device__ __forceinline__ bool should_route(T det, T absterms, const Fallback& fb) {
    if (!fb.enable) return false;
    T ad = fabs(det);
    if (!finiteT(det) || !finiteT(absterms)) return true;
    if (ad == T(0) || static_cast<double>(ad) < fb.tau_abs) return true;
    // absterms / |det| > tau_cond  <=>  absterms > tau_cond * |det| (no division)
    return static_cast<double>(absterms) > fb.tau_cond * static_cast<double>(ad);
}

}  // namespace pf
