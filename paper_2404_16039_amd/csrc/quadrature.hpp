// quadrature.hpp -- integration rules on the reference simplex for coefficients given at
// integration points (the loop over integration points of the section 3.6 stiffness and
// mass listings).  Barycentric coordinate lam(q, j) of local node j at point q; every rule
// here has equal weights w = (1/dim!) / QN, summing to the reference measure.
//   order 1 (QN = 1):         the centroid;
//   order 2, 2-D (QN = 3):    the edge midpoints, point q on the edge (q, q+1 mod 3);
//   order 2, 3-D (QN = 4):    the symmetric 4-point rule, lam = A at node q, B elsewhere,
//                             A = (5 + 3 sqrt 5)/20, B = (5 - sqrt 5)/20.
// Both order-2 rules are exact for polynomials of degree 2.
#pragma once

#include "common.hpp"

namespace pf {

template <int DIM, int QN>
struct QuadRule;

template <int DIM>
struct QuadRule<DIM, 1> {
    __device__ static double lam(int, int) { return 1.0 / (DIM + 1); }
};

template <>
struct QuadRule<2, 3> {
    __device__ static double lam(int q, int j) { return (j == q || j == (q + 1) % 3) ? 0.5 : 0.0; }
};

template <>
struct QuadRule<3, 4> {
    __device__ static double lam(int q, int j) {
        return j == q ? (5.0 + 3.0 * __builtin_sqrt(5.0)) / 20.0 : (5.0 - __builtin_sqrt(5.0)) / 20.0;
    }
};

template <int DIM, int QN>
__device__ __forceinline__ double quad_weight() {
    return (DIM == 2 ? 0.5 : 1.0 / 6.0) / QN;
}

// integration points of a rule of `order` (1 or 2) in dimension dim, 0 if unsupported
inline int quad_count(int dim, int order) {
    if ((dim != 2 && dim != 3) || (order != 1 && order != 2)) return 0;
    return order == 1 ? 1 : dim + 1;
}

}  // namespace pf
