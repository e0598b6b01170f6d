/*
 * pf_oracle.c -- plain FP64 CPU oracle for the page-wise linear algebra and P1 finite
 * element assembly of "On a vectorized basic linear algebra package for prototyping
 * codes in MATLAB" (Moskovka, Rahman, Valdman, Vatne; arXiv 2404.16039).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link or call
 * this file; only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * use it.  It shares no source, header, table or helper with the HIP path.
 *
 * Everything is computed from the plain mathematical definitions, one page / one element
 * at a time, in double precision, with no blocking, fusion or reordering:
 *   - determinant: Leibniz sum over all permutations (section 2.3, page-wise determinant)
 *   - inverse: Gauss-Jordan elimination with partial pivoting (section 2.3, page-wise
 *     inverse on the set of pages with non-zero determinant)
 *   - transpose / products: index definitions (section 2.2, page-wise transpose and
 *     page-wise matrix multiplication; section 2.4 library functions)
 *   - P1 elements: Jacobian from the reference shape-function derivatives, its inverse,
 *     global gradients, stiffness and mass by quadrature (section 3.6, the derivative
 *     routine and the P1 stiffness / P2 mass listings specialised to P1, c = 1)
 *   - assembly: (row, col, value) triples in element-major order, stable sort by
 *     (row, col), sum of each run (section 3.6, the sparse() call of the listings)
 *   - boundary faces: cross product normals and areas (section 3.2)
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math, no FMA contraction).
 * All matrices are column-major pages (MATLAB order); page k of an r x c array starts
 * at k*r*c unless a page stride is given.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXN 4

/* ------------------------------------------------------------------------------------ */
/* permutations of {0..n-1} in lexicographic order, with signs                          */
/* ------------------------------------------------------------------------------------ */
static int next_perm(int* p, int n) {
    int i = n - 2;
    while (i >= 0 && p[i] > p[i + 1]) i--;
    if (i < 0) return 0;
    int j = n - 1;
    while (p[j] < p[i]) j--;
    int t = p[i]; p[i] = p[j]; p[j] = t;
    for (int a = i + 1, b = n - 1; a < b; a++, b--) { t = p[a]; p[a] = p[b]; p[b] = t; }
    return 1;
}

static int perm_sign(const int* p, int n) {
    int s = 1;
    for (int a = 0; a < n; a++)
        for (int b = a + 1; b < n; b++)
            if (p[a] > p[b]) s = -s;
    return s;
}

/* element (r, c) of a column-major rows x cols page */
#define AT(a, rows, r, c) ((a)[(r) + (int64_t)(c) * (rows)])

/* Leibniz determinant and its absolute scale perm(|A|) = sum over sigma of prod |a| */
static double leibniz(const double* a, int n, double* perm_abs) {
    int p[OR_MAXN];
    for (int i = 0; i < n; i++) p[i] = i;
    double sum = 0.0, sabs = 0.0;
    do {
        double prod = 1.0, pabs = 1.0;
        for (int i = 0; i < n; i++) {
            prod *= AT(a, n, i, p[i]);
            pabs *= fabs(AT(a, n, i, p[i]));
        }
        sum += perm_sign(p, n) * prod;
        sabs += pabs;
    } while (next_perm(p, n));
    if (perm_abs) *perm_abs = sabs;
    return sum;
}

/* Gauss-Jordan with partial pivoting on [A | I].  Returns 1 if a zero pivot occurs. */
static int gauss_jordan(const double* a, int n, double* inv) {
    /* extended precision (64-bit significand on x86-64), one rounding to FP64 at the end:
     * FP64 elimination loses up to ~10 bits on pages where partial pivoting still leaves a
     * cancelling back substitution, more than the inverse's error scale allows */
    long double m[OR_MAXN][2 * OR_MAXN];
    for (int r = 0; r < n; r++) {
        for (int c = 0; c < n; c++) m[r][c] = AT(a, n, r, c);
        for (int c = 0; c < n; c++) m[r][n + c] = (r == c) ? 1.0 : 0.0;
    }
    for (int col = 0; col < n; col++) {
        int piv = col;
        for (int r = col + 1; r < n; r++)
            if (fabsl(m[r][col]) > fabsl(m[piv][col])) piv = r;
        if (m[piv][col] == 0.0L) {
            for (int i = 0; i < n * n; i++) inv[i] = NAN;
            return 1;
        }
        if (piv != col)
            for (int c = 0; c < 2 * n; c++) { long double t = m[col][c]; m[col][c] = m[piv][c]; m[piv][c] = t; }
        long double d = m[col][col];
        for (int c = 0; c < 2 * n; c++) m[col][c] /= d;
        for (int r = 0; r < n; r++) {
            if (r == col) continue;
            long double f = m[r][col];
            if (f != 0.0L)
                for (int c = 0; c < 2 * n; c++) m[r][c] -= f * m[col][c];
        }
    }
    for (int r = 0; r < n; r++)
        for (int c = 0; c < n; c++) AT(inv, n, r, c) = (double)m[r][n + c];
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* page operations (sections 2.2-2.4)                                                  */
/* ------------------------------------------------------------------------------------ */

/* det[k] = det of page k (n x n), perm_abs[k] = perm(|A_k|) (nullable) */
int or_page_det(int n, int64_t count, const double* a, double* det, double* perm_abs) {
    if (n < 1 || n > OR_MAXN) return -1;
    for (int64_t k = 0; k < count; k++) {
        double s;
        det[k] = leibniz(a + k * n * n, n, &s);
        if (perm_abs) perm_abs[k] = s;
    }
    return 0;
}

/* inv[k] = A_k^{-1}; singular[k] = 1 when elimination meets a zero pivot (inv = NaN).
 * scale (nullable) = |A^{-1}| |A| |A^{-1}| per page, the componentwise error scale.   */
int or_page_inv(int n, int64_t count, const double* a, double* inv, uint8_t* singular, double* scale) {
    if (n < 1 || n > OR_MAXN) return -1;
    for (int64_t k = 0; k < count; k++) {
        const double* ak = a + k * n * n;
        double* xk = inv + k * n * n;
        int s = gauss_jordan(ak, n, xk);
        if (singular) singular[k] = (uint8_t)s;
        if (scale) {
            double* sk = scale + k * n * n;
            double t[OR_MAXN * OR_MAXN];
            for (int r = 0; r < n; r++)
                for (int c = 0; c < n; c++) {
                    double acc = 0.0;
                    for (int p = 0; p < n; p++) acc += fabs(AT(xk, n, r, p)) * fabs(AT(ak, n, p, c));
                    AT(t, n, r, c) = acc;
                }
            for (int r = 0; r < n; r++)
                for (int c = 0; c < n; c++) {
                    double acc = 0.0;
                    for (int p = 0; p < n; p++) acc += AT(t, n, r, p) * fabs(AT(xk, n, p, c));
                    AT(sk, n, r, c) = acc;
                }
        }
    }
    return 0;
}

/* t[k] = A_k^T for rows x cols pages */
int or_page_transpose(int rows, int cols, int64_t count, const double* a, double* t) {
    for (int64_t k = 0; k < count; k++) {
        const double* ak = a + k * rows * cols;
        double* tk = t + k * rows * cols;
        for (int r = 0; r < rows; r++)
            for (int c = 0; c < cols; c++) AT(tk, cols, c, r) = AT(ak, rows, r, c);
    }
    return 0;
}

/* C_k = op(A_k) op(B_k); op(A) is m x kk, op(B) is kk x n, C is m x n.
 * transA: A is stored kk x m; else m x kk.  transB: B stored n x kk; else kk x n.
 * sA / sB: page strides of A and B in elements (0 broadcasts a single page, the copy map
 * of section 2.2).  absC (nullable) = (|op(A)| |op(B)|)_ij, the error scale.          */
int or_page_mtimes(int m, int kk, int n, int64_t count,
                   const double* A, int transA, int64_t sA,
                   const double* B, int transB, int64_t sB,
                   double* C, double* absC) {
    if (m < 1 || kk < 1 || n < 1) return -1;
    for (int64_t k = 0; k < count; k++) {
        const double* ak = A + k * sA;
        const double* bk = B + k * sB;
        double* ck = C + k * (int64_t)m * n;
        for (int i = 0; i < m; i++)
            for (int j = 0; j < n; j++) {
                double acc = 0.0, aacc = 0.0;
                for (int p = 0; p < kk; p++) {
                    double av = transA ? AT(ak, kk, p, i) : AT(ak, m, i, p);
                    double bv = transB ? AT(bk, n, j, p) : AT(bk, kk, p, j);
                    acc += av * bv;
                    aacc += fabs(av) * fabs(bv);
                }
                AT(ck, m, i, j) = acc;
                if (absC) AT(absC + k * (int64_t)m * n, m, i, j) = aacc;
            }
    }
    return 0;
}

/* C_k = s_k * A_k (page-wise scalar multiplication, section 2.2) */
int or_page_scale(int rows, int cols, int64_t count, const double* s, const double* a, double* c) {
    int64_t ps = (int64_t)rows * cols;
    for (int64_t k = 0; k < count; k++)
        for (int64_t q = 0; q < ps; q++) c[k * ps + q] = s[k] * a[k * ps + q];
    return 0;
}

/* q_k = u_k^T A_k v_k (page-wise bilinear form, section 2.2) */
int or_page_bilinear(int n, int64_t count, const double* u, const double* a, const double* v, double* q) {
    for (int64_t k = 0; k < count; k++) {
        const double* ak = a + k * n * n;
        double acc = 0.0;
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) acc += u[k * n + i] * AT(ak, n, i, j) * v[k * n + j];
        q[k] = acc;
    }
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* P1 elements (section 3.6): one quadrature point for the gradients (constant on a P1  */
/* element), a degree-2 exact rule for the mass matrix, coefficients c_K = c_M = 1.     */
/* ------------------------------------------------------------------------------------ */

/* reference derivatives of the P1 shape functions phi_1 = 1 - sum xi, phi_{i+1} = xi_i,
 * stored dim x nlb column-major: dshape(i, j) = d phi_j / d xi_i                       */
static void p1_dshape(int dim, double* ds) {
    int nlb = dim + 1;
    for (int i = 0; i < dim; i++)
        for (int j = 0; j < nlb; j++) AT(ds, dim, i, j) = (j == 0) ? -1.0 : ((j == i + 1) ? 1.0 : 0.0);
}

/* degree-2 exact quadrature on the reference simplex in barycentric coordinates:
 * triangle: the 3 edge midpoints, weight 1/6 each; tetrahedron: the 4 points
 * (a,b,b,b) and permutations with a = (5+3 sqrt5)/20, b = (5-sqrt5)/20, weight 1/24.   */
static int p1_mass_rule(int dim, double lam[4][4], double* w) {
    if (dim == 2) {
        double mid[3][3] = {{0.5, 0.5, 0.0}, {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}};
        for (int q = 0; q < 3; q++) { for (int j = 0; j < 3; j++) lam[q][j] = mid[q][j]; w[q] = 1.0 / 6.0; }
        return 3;
    }
    double a = (5.0 + 3.0 * sqrt(5.0)) / 20.0, b = (5.0 - sqrt(5.0)) / 20.0;
    for (int q = 0; q < 4; q++) {
        for (int j = 0; j < 4; j++) lam[q][j] = (j == q) ? a : b;
        w[q] = 1.0 / 24.0;
    }
    return 4;
}

/* Per element e (nlb = dim+1 nodes):
 *   det[e]   signed det of the Jacobian tjac = dshape * coords3D^T (first node origin)
 *   vol[e]   |det| / dim!
 *   grads    dim x nlb per element: dphi = tjac^{-1} dshape (column j = grad phi_j)
 *   Ke, Me   nlb x nlb per element: Ke = w |det| dphi^T dphi, Me = sum_q w_q |det| phi phi^T
 *   Kabs     nlb x nlb per element: w |det| |dphi(:,a)| |dphi(:,b)|, the error scale of Ke
 *            (Cauchy-Schwarz bound of the integrand grad phi_a . grad phi_b)
 *   facet    nlb per element: measure of the facet opposite node j = dim |T| |grad phi_j|
 * Any output pointer may be NULL.  Returns the number of elements whose Jacobian is singular. */
int64_t or_p1_elements(int dim, int64_t nn, const double* coords, int64_t ne, const int32_t* elems,
                       double* det, double* vol, double* grads, double* Ke, double* Me,
                       double* Kabs, double* facet) {
    if (dim != 2 && dim != 3) return -1;
    int nlb = dim + 1;
    double ds[3 * 4];
    p1_dshape(dim, ds);
    double fact = (dim == 2) ? 2.0 : 6.0;
    double w1 = 1.0 / fact; /* one-point rule: weight = reference measure */
    double lam[4][4], wq[4];
    int nq = p1_mass_rule(dim, lam, wq);
    int64_t nsing = 0;
    for (int64_t e = 0; e < ne; e++) {
        double c3[3 * 4]; /* coords3D: dim x nlb */
        for (int j = 0; j < nlb; j++) {
            int64_t node = elems[e * nlb + j];
            if (node < 0 || node >= nn) return -2;
            for (int i = 0; i < dim; i++) AT(c3, dim, i, j) = coords[node * dim + i];
        }
        double tjac[9]; /* tjac = dshape * coords3D^T : dim x dim */
        for (int r = 0; r < dim; r++)
            for (int c = 0; c < dim; c++) {
                double acc = 0.0;
                for (int j = 0; j < nlb; j++) acc += AT(ds, dim, r, j) * AT(c3, dim, c, j);
                AT(tjac, dim, r, c) = acc;
            }
        double dt = leibniz(tjac, dim, NULL);
        double tinv[9];
        int sing = gauss_jordan(tjac, dim, tinv);
        nsing += sing;
        double dphi[12]; /* tjac^{-1} * dshape : dim x nlb */
        for (int r = 0; r < dim; r++)
            for (int j = 0; j < nlb; j++) {
                double acc = 0.0;
                for (int p = 0; p < dim; p++) acc += AT(tinv, dim, r, p) * AT(ds, dim, p, j);
                AT(dphi, dim, r, j) = acc;
            }
        double adet = fabs(dt);
        double T = adet / fact;
        if (det) det[e] = dt;
        if (vol) vol[e] = T;
        if (grads)
            for (int q = 0; q < dim * nlb; q++) grads[e * dim * nlb + q] = dphi[q];
        double gnorm[4];
        for (int j = 0; j < nlb; j++) {
            double g2 = 0.0;
            for (int i = 0; i < dim; i++) g2 += AT(dphi, dim, i, j) * AT(dphi, dim, i, j);
            gnorm[j] = sqrt(g2);
        }
        for (int a = 0; a < nlb; a++)
            for (int b = 0; b < nlb; b++) {
                double acc = 0.0;
                for (int i = 0; i < dim; i++) acc += AT(dphi, dim, i, a) * AT(dphi, dim, i, b);
                if (Ke) Ke[e * nlb * nlb + a + b * nlb] = w1 * adet * acc;
                /* error scale of the integrand: |grad phi_a . grad phi_b| <= |grad phi_a| |grad phi_b| */
                if (Kabs) Kabs[e * nlb * nlb + a + b * nlb] = w1 * adet * gnorm[a] * gnorm[b];
                if (Me) {
                    double m = 0.0;
                    for (int q = 0; q < nq; q++) m += wq[q] * adet * lam[q][a] * lam[q][b];
                    Me[e * nlb * nlb + a + b * nlb] = m;
                }
            }
        if (facet)
            for (int j = 0; j < nlb; j++) {
                double g2 = 0.0;
                for (int i = 0; i < dim; i++) g2 += AT(dphi, dim, i, j) * AT(dphi, dim, i, j);
                facet[e * nlb + j] = dim * T * sqrt(g2);
            }
    }
    return nsing;
}

/* Integration rules on the reference simplex (the integration points and weights of the
 * section 3.6 listings; weights sum to the reference measure 1/dim!), in barycentric
 * coordinates lam[q][j] of local node j:
 *   order 1: the centroid, weight 1/dim!;
 *   order 2: the degree-2 exact rules of p1_mass_rule.                                  */
static int quad_rule(int dim, int order, double lam[4][4], double* w) {
    if (order == 2) return p1_mass_rule(dim, lam, w);
    int nlb = dim + 1;
    for (int j = 0; j < nlb; j++) lam[0][j] = 1.0 / nlb;
    w[0] = (dim == 2) ? 0.5 : 1.0 / 6.0;
    return 1;
}

int or_quad_count(int dim, int order) {
    double lam[4][4], w[4];
    if ((dim != 2 && dim != 3) || (order != 1 && order != 2)) return -1;
    return quad_rule(dim, order, lam, w);
}

/* Physical integration points x_q = sum_j lam[q][j] p_j of every element: ne x nq x dim */
int or_quad_points(int dim, int order, int64_t nn, const double* coords, int64_t ne, const int32_t* elems,
                   double* xq) {
    double lam[4][4], w[4];
    if ((dim != 2 && dim != 3) || (order != 1 && order != 2)) return -1;
    int nq = quad_rule(dim, order, lam, w), nlb = dim + 1;
    for (int64_t e = 0; e < ne; e++)
        for (int q = 0; q < nq; q++)
            for (int i = 0; i < dim; i++) {
                double x = 0.0;
                for (int j = 0; j < nlb; j++) {
                    int64_t node = elems[e * nlb + j];
                    if (node < 0 || node >= nn) return -2;
                    x += lam[q][j] * coords[node * dim + i];
                }
                xq[(e * nq + q) * dim + i] = x;
            }
    return 0;
}

/* Element matrices with coefficients given at the integration points, as the loop over
 * integration points of the stiffness / mass listings of section 3.6 computes them:
 *   Ke = sum_q w_q cK_q |det| dphi^T dphi,  Me = sum_q w_q cM_q |det| phi(x_q) phi(x_q)^T,
 * with error scales Kabs = sum_q w_q |cK_q| |det| |dphi_a| |dphi_b| and
 * Mabs = sum_q w_q |cM_q| |det| phi_a phi_b.  cKq, cMq: ne x nq values (NULL = 1).
 * The Jacobian, its inverse and the gradients follow or_p1_elements step by step. */
int64_t or_p1_elements_q(int dim, int order, int64_t nn, const double* coords, int64_t ne, const int32_t* elems,
                         const double* cKq, const double* cMq, double* Ke, double* Me, double* Kabs, double* Mabs) {
    if ((dim != 2 && dim != 3) || (order != 1 && order != 2)) return -1;
    int nlb = dim + 1;
    double ds[3 * 4];
    p1_dshape(dim, ds);
    double lam[4][4], wq[4];
    int nq = quad_rule(dim, order, lam, wq);
    int64_t nsing = 0;
    for (int64_t e = 0; e < ne; e++) {
        double c3[3 * 4];
        for (int j = 0; j < nlb; j++) {
            int64_t node = elems[e * nlb + j];
            if (node < 0 || node >= nn) return -2;
            for (int i = 0; i < dim; i++) AT(c3, dim, i, j) = coords[node * dim + i];
        }
        double tjac[9];
        for (int r = 0; r < dim; r++)
            for (int c = 0; c < dim; c++) {
                double acc = 0.0;
                for (int j = 0; j < nlb; j++) acc += AT(ds, dim, r, j) * AT(c3, dim, c, j);
                AT(tjac, dim, r, c) = acc;
            }
        double adet = fabs(leibniz(tjac, dim, NULL));
        double tinv[9];
        nsing += gauss_jordan(tjac, dim, tinv);
        double dphi[12];
        for (int r = 0; r < dim; r++)
            for (int j = 0; j < nlb; j++) {
                double acc = 0.0;
                for (int p = 0; p < dim; p++) acc += AT(tinv, dim, r, p) * AT(ds, dim, p, j);
                AT(dphi, dim, r, j) = acc;
            }
        double gnorm[4];
        for (int j = 0; j < nlb; j++) {
            double g2 = 0.0;
            for (int i = 0; i < dim; i++) g2 += AT(dphi, dim, i, j) * AT(dphi, dim, i, j);
            gnorm[j] = sqrt(g2);
        }
        for (int a = 0; a < nlb; a++)
            for (int b = 0; b < nlb; b++) {
                double gg = 0.0;
                for (int i = 0; i < dim; i++) gg += AT(dphi, dim, i, a) * AT(dphi, dim, i, b);
                double k = 0.0, ka = 0.0, m = 0.0, ma = 0.0;
                for (int q = 0; q < nq; q++) {
                    double ck = cKq ? cKq[e * nq + q] : 1.0, cm = cMq ? cMq[e * nq + q] : 1.0;
                    k += wq[q] * ck * adet * gg;
                    ka += wq[q] * fabs(ck) * adet * gnorm[a] * gnorm[b];
                    m += wq[q] * cm * adet * lam[q][a] * lam[q][b];
                    ma += wq[q] * fabs(cm) * adet * lam[q][a] * lam[q][b];
                }
                if (Ke) Ke[e * nlb * nlb + a + b * nlb] = k;
                if (Kabs) Kabs[e * nlb * nlb + a + b * nlb] = ka;
                if (Me) Me[e * nlb * nlb + a + b * nlb] = m;
                if (Mabs) Mabs[e * nlb * nlb + a + b * nlb] = ma;
            }
    }
    return nsing;
}

/* coords3D and vectors3D of the coordinate-structure listing (section 3.1):
 * coords3D dim x nlb x ne, vectors3D dim x (nlb-1) x ne with column j = node j - last node */
int or_create_coords3d(int dim, int nlb, int64_t nn, const double* coords, int64_t ne,
                       const int32_t* elems, double* coords3d, double* vectors3d) {
    for (int64_t e = 0; e < ne; e++) {
        for (int j = 0; j < nlb; j++) {
            int64_t node = elems[e * nlb + j];
            if (node < 0 || node >= nn) return -2;
            for (int i = 0; i < dim; i++)
                if (coords3d) coords3d[e * dim * nlb + i + j * dim] = coords[node * dim + i];
        }
        if (vectors3d) {
            int64_t last = elems[e * nlb + nlb - 1];
            for (int j = 0; j < nlb - 1; j++) {
                int64_t node = elems[e * nlb + j];
                for (int i = 0; i < dim; i++)
                    vectors3d[e * dim * (nlb - 1) + i + j * dim] = coords[node * dim + i] - coords[last * dim + i];
            }
        }
    }
    return 0;
}

/* FP64 routing predicate on the Jacobian (first node origin): route when |det| < tau_abs
 * or when the det-condition sum_j |a_1j C_1j| / |det| exceeds tau_cond (C = cofactors of
 * the first row, each from its own Leibniz determinant).                              */
int or_route_predicate(int dim, const double* tjac_pages, int64_t count, double tau_abs, double tau_cond,
                       uint8_t* routed, double* cond) {
    for (int64_t k = 0; k < count; k++) {
        const double* a = tjac_pages + k * dim * dim;
        double d = leibniz(a, dim, NULL);
        double s = 0.0;
        for (int j = 0; j < dim; j++) {
            double minor[9];
            int q = 0;
            for (int c = 0; c < dim; c++) {
                if (c == j) continue;
                for (int r = 1; r < dim; r++) minor[(r - 1) + q * (dim - 1)] = AT(a, dim, r, c);
                q++;
            }
            double cof = leibniz(minor, dim - 1, NULL);
            s += fabs(AT(a, dim, 0, j) * cof);
        }
        double kappa = (d == 0.0) ? INFINITY : s / fabs(d);
        if (cond) cond[k] = kappa;
        routed[k] = (uint8_t)((fabs(d) < tau_abs) || (kappa > tau_cond));
    }
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* assembly: sparse(rows, cols, vals) with duplicates summed                            */
/* ------------------------------------------------------------------------------------ */
typedef struct { int32_t row, col; int64_t seq; } or_triple;

static int cmp_triple(const void* x, const void* y) {
    const or_triple* a = (const or_triple*)x;
    const or_triple* b = (const or_triple*)y;
    if (a->row != b->row) return a->row < b->row ? -1 : 1;
    if (a->col != b->col) return a->col < b->col ? -1 : 1;
    if (a->seq != b->seq) return a->seq < b->seq ? -1 : 1; /* stable */
    return 0;
}

/* Assemble K and M from element matrices (nlb x nlb column-major per element) into CSR.
 * The listing's index arrays give, for local (a, b) of element e, the global entry
 * (row, col) = (elems[e][b], elems[e][a]) with value K_e(a, b).  Triples are emitted in
 * element-major, then a, then b order, stably sorted by (row, col), and each run is
 * summed in that order.  Every pair is kept (entries summing to zero included).
 * Outputs: row_ptr[nn+1]; col_idx, valK, valM, scaleK, scaleM[cap] (any value array
 * nullable; scale = sum of |contributions|, using Kabs when given).  Returns nnz, or -1
 * if cap is too small, -2 on a bad index.                                             */
int64_t or_assemble(int nlb, int64_t nn, int64_t ne, const int32_t* elems,
                    const double* Ke, const double* Me, const double* Kabs,
                    int64_t* row_ptr, int32_t* col_idx, double* valK, double* valM,
                    double* scaleK, double* scaleM, int64_t cap) {
    int64_t nt = ne * nlb * nlb;
    or_triple* t = (or_triple*)malloc(sizeof(or_triple) * (size_t)(nt > 0 ? nt : 1));
    if (!t) return -3;
    int64_t q = 0;
    for (int64_t e = 0; e < ne; e++)
        for (int a = 0; a < nlb; a++)
            for (int b = 0; b < nlb; b++) {
                int32_t r = elems[e * nlb + b], c = elems[e * nlb + a];
                if (r < 0 || r >= nn || c < 0 || c >= nn) { free(t); return -2; }
                t[q].row = r;
                t[q].col = c;
                t[q].seq = e * nlb * nlb + a + (int64_t)b * nlb; /* position of K_e(a,b) */
                q++;
            }
    qsort(t, (size_t)nt, sizeof(or_triple), cmp_triple);
    for (int64_t i = 0; i <= nn; i++) row_ptr[i] = 0;
    int64_t nnz = 0;
    for (int64_t s = 0; s < nt;) {
        int64_t u = s;
        double sk = 0.0, sm = 0.0, ak = 0.0, am = 0.0;
        while (u < nt && t[u].row == t[s].row && t[u].col == t[s].col) {
            int64_t p = t[u].seq;
            if (Ke) { sk += Ke[p]; ak += fabs(Kabs ? Kabs[p] : Ke[p]); }
            if (Me) { sm += Me[p]; am += fabs(Me[p]); }
            u++;
        }
        if (nnz >= cap) { free(t); return -1; }
        col_idx[nnz] = t[s].col;
        if (valK) valK[nnz] = sk;
        if (valM) valM[nnz] = sm;
        if (scaleK) scaleK[nnz] = ak;
        if (scaleM) scaleM[nnz] = am;
        row_ptr[t[s].row + 1]++;
        nnz++;
        s = u;
    }
    for (int64_t i = 0; i < nn; i++) row_ptr[i + 1] += row_ptr[i];
    free(t);
    return nnz;
}

/* Sampled rows of the assembled K and M, computed one by one: scan every element, and for
 * each sampled row node i in it, add the element's contributions to row i (in element
 * order, the order the full assembly sums them in).  rows[nr] are distinct node ids.
 * For sampled row r: its sorted columns go to cols[r*cap ..], values to valK/valM (and
 * scales) at the same positions, its length to len[r].  Returns 0, -1 if a row exceeds
 * cap, -2 on a bad index.                                                             */
int or_assemble_rows(int dim, int64_t nn, const double* coords, int64_t ne, const int32_t* elems,
                     int nr, const int32_t* rows, int cap, int32_t* cols, double* valK, double* valM,
                     double* scaleK, double* scaleM, int32_t* len) {
    int nlb = dim + 1;
    int32_t* which = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nn > 0 ? nn : 1));
    if (!which) return -3;
    for (int64_t i = 0; i < nn; i++) which[i] = -1;
    for (int r = 0; r < nr; r++) { which[rows[r]] = r; len[r] = 0; }
    double Ke[16], Me[16], Ka[16];
    for (int64_t e = 0; e < ne; e++) {
        int hit = 0;
        for (int a = 0; a < nlb; a++) {
            int32_t node = elems[e * nlb + a];
            if (node < 0 || node >= nn) { free(which); return -2; }
            if (which[node] >= 0) hit = 1;
        }
        if (!hit) continue;
        if (or_p1_elements(dim, nn, coords, 1, elems + e * nlb, NULL, NULL, NULL, Ke, Me, Ka, NULL) < 0) {
            free(which);
            return -2;
        }
        /* triple (row = elems[b], col = elems[a]) += K_e(a, b); visit in a-major, b order */
        for (int a = 0; a < nlb; a++)
            for (int b = 0; b < nlb; b++) {
                int32_t row = elems[e * nlb + b];
                int r = which[row];
                if (r < 0) continue;
                int32_t col = elems[e * nlb + a];
                int32_t* cr = cols + (int64_t)r * cap;
                int L = len[r], pos = 0;
                while (pos < L && cr[pos] < col) pos++;
                int64_t base = (int64_t)r * cap;
                if (pos == L || cr[pos] != col) {
                    if (L >= cap) { free(which); return -1; }
                    for (int m = L; m > pos; m--) {
                        cr[m] = cr[m - 1];
                        valK[base + m] = valK[base + m - 1];
                        valM[base + m] = valM[base + m - 1];
                        scaleK[base + m] = scaleK[base + m - 1];
                        scaleM[base + m] = scaleM[base + m - 1];
                    }
                    cr[pos] = col;
                    valK[base + pos] = 0.0;
                    valM[base + pos] = 0.0;
                    scaleK[base + pos] = 0.0;
                    scaleM[base + pos] = 0.0;
                    len[r] = L + 1;
                }
                int p = a + b * nlb;
                valK[base + pos] += Ke[p];
                valM[base + pos] += Me[p];
                scaleK[base + pos] += fabs(Ka[p]);
                scaleM[base + pos] += fabs(Me[p]);
            }
    }
    free(which);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* boundary facets (section 3.2): 3-D triangles (a,b,c): n = (b-a) x (c-a), area |n|/2;  */
/* 2-D edges (a,b): n = (b_y - a_y, a_x - b_x), length |n|.  unit = n / |n|.            */
/* ------------------------------------------------------------------------------------ */
int or_boundary(int dim, int64_t nn, const double* coords, int64_t nf, const int32_t* faces,
                double* unit, double* measure, double* raw) {
    for (int64_t f = 0; f < nf; f++) {
        double n[3] = {0, 0, 0};
        double meas;
        if (dim == 3) {
            int64_t ia = faces[f * 3], ib = faces[f * 3 + 1], ic = faces[f * 3 + 2];
            if (ia < 0 || ia >= nn || ib < 0 || ib >= nn || ic < 0 || ic >= nn) return -2;
            double u[3], v[3];
            for (int i = 0; i < 3; i++) {
                u[i] = coords[ib * 3 + i] - coords[ia * 3 + i];
                v[i] = coords[ic * 3 + i] - coords[ia * 3 + i];
            }
            n[0] = u[1] * v[2] - u[2] * v[1];
            n[1] = u[2] * v[0] - u[0] * v[2];
            n[2] = u[0] * v[1] - u[1] * v[0];
            meas = 0.5 * sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        } else if (dim == 2) {
            int64_t ia = faces[f * 2], ib = faces[f * 2 + 1];
            if (ia < 0 || ia >= nn || ib < 0 || ib >= nn) return -2;
            n[0] = coords[ib * 2 + 1] - coords[ia * 2 + 1];
            n[1] = coords[ia * 2] - coords[ib * 2];
            meas = sqrt(n[0] * n[0] + n[1] * n[1]);
        } else {
            return -1;
        }
        double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int i = 0; i < dim; i++) {
            if (unit) unit[f * dim + i] = n[i] / len;
            if (raw) raw[f * dim + i] = n[i];
        }
        if (measure) measure[f] = meas;
    }
    return 0;
}

/* Load vector of the right-hand side listing (section 3.6): on every element the local
 * vector b2D[e*nlb + j] = sum_q w_q |det J_e| f_eq phi_j(x_q) over the integration points
 * of the rule of `order` (phi_j(x_q) = lam[q][j]), then the accumarray step b[i] = sum of
 * b2D[e*nlb + j] over all (e, j) with elems[e*nlb + j] == i, taken in element order.
 * babs[i] = the same sum of absolute values (the error scale of b[i]).  f: ne x nq values
 * (element-major).  b2D, b, babs may be NULL.  Returns 0, or -1 / -2 on a bad rule or node. */
int or_rhs_p1(int dim, int order, int64_t nn, const double* coords, int64_t ne, const int32_t* elems,
              const double* fq, double* b2D, double* b, double* babs) {
    if ((dim != 2 && dim != 3) || (order != 1 && order != 2)) return -1;
    int nlb = dim + 1;
    double ds[3 * 4];
    p1_dshape(dim, ds);
    double lam[4][4], wq[4];
    int nq = quad_rule(dim, order, lam, wq);
    if (b)
        for (int64_t i = 0; i < nn; i++) b[i] = 0.0;
    if (babs)
        for (int64_t i = 0; i < nn; i++) babs[i] = 0.0;
    for (int64_t e = 0; e < ne; e++) {
        double c3[3 * 4];
        for (int j = 0; j < nlb; j++) {
            int64_t node = elems[e * nlb + j];
            if (node < 0 || node >= nn) return -2;
            for (int i = 0; i < dim; i++) AT(c3, dim, i, j) = coords[node * dim + i];
        }
        double tjac[9];
        for (int r = 0; r < dim; r++)
            for (int c = 0; c < dim; c++) {
                double acc = 0.0;
                for (int j = 0; j < nlb; j++) acc += AT(ds, dim, r, j) * AT(c3, dim, c, j);
                AT(tjac, dim, r, c) = acc;
            }
        double adet = fabs(leibniz(tjac, dim, NULL));
        for (int j = 0; j < nlb; j++) {
            double v = 0.0;
            for (int q = 0; q < nq; q++) v += wq[q] * adet * fq[e * nq + q] * lam[q][j];
            if (b2D) b2D[e * nlb + j] = v;
            int64_t node = elems[e * nlb + j];
            if (b) b[node] += v;
            if (babs) babs[node] += fabs(v);
        }
    }
    return 0;
}

/* All faces of a simplicial mesh (section 3.2, normals of all faces or of boundary faces
 * only): every element contributes its nlb faces (the face opposite local node k), each
 * keyed by its node ids in ascending order; the keys are sorted (ties by element id) and
 * equal keys merged.  Outputs, faces in ascending key order:
 *   faces[f*nv ...]  the face's nodes ordered so that its normal points out of its first
 *                    element e1 (the smaller element id): for a positively oriented
 *                    element (det J > 0, first-node origin) the face opposite node k is
 *                    taken in the order that makes (b-a)x(c-a) (3-D) or (b_y-a_y, a_x-b_x)
 *                    (2-D) outward, reversed when det J < 0;
 *   fel[f*2 ...]     (e1, e2), e2 = -1 on the boundary.
 * Returns the number of faces, or -1 / -2 / -3 (bad dim, bad node, a face in more than two
 * elements); cap is the capacity of the outputs (at least nlb * ne faces). */
typedef struct {
    int32_t key[3];
    int64_t e;
    int k;
} or_face_t;

static int face_cmp(const void* pa, const void* pb) {
    const or_face_t* a = (const or_face_t*)pa;
    const or_face_t* b = (const or_face_t*)pb;
    for (int i = 0; i < 3; i++)
        if (a->key[i] != b->key[i]) return a->key[i] < b->key[i] ? -1 : 1;
    return (a->e > b->e) - (a->e < b->e);
}

/* local node order of the face opposite node k, outward for a positively oriented element */
static const int FACE3[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};
static const int FACE2[3][2] = {{1, 2}, {2, 0}, {0, 1}};

int64_t or_faces(int dim, int64_t nn, const double* coords, int64_t ne, const int32_t* elems, int32_t* faces,
                 int32_t* fel, int64_t cap) {
    if (dim != 2 && dim != 3) return -1;
    int nlb = dim + 1, nv = dim;
    int64_t m = ne * nlb;
    or_face_t* all = (or_face_t*)malloc(sizeof(or_face_t) * (size_t)(m > 0 ? m : 1));
    if (!all) return -4;
    for (int64_t e = 0; e < ne; e++)
        for (int k = 0; k < nlb; k++) {
            or_face_t* f = &all[e * nlb + k];
            int t = 0;
            for (int j = 0; j < nlb; j++) {
                if (j == k) continue;
                int32_t v = elems[e * nlb + j];
                if (v < 0 || v >= nn) { free(all); return -2; }
                f->key[t++] = v;
            }
            for (int a = 0; a < nv; a++)       /* insertion sort of the key */
                for (int b = a + 1; b < nv; b++)
                    if (f->key[b] < f->key[a]) { int32_t x = f->key[a]; f->key[a] = f->key[b]; f->key[b] = x; }
            if (nv == 2) f->key[2] = -1;
            f->e = e;
            f->k = k;
        }
    qsort(all, (size_t)m, sizeof(or_face_t), face_cmp);
    int64_t nf = 0;
    for (int64_t i = 0; i < m;) {
        int64_t j = i + 1;
        while (j < m && all[j].key[0] == all[i].key[0] && all[j].key[1] == all[i].key[1] &&
               all[j].key[2] == all[i].key[2])
            j++;
        if (j - i > 2) { free(all); return -3; }
        if (nf >= cap) { free(all); return -5; }
        const or_face_t* f = &all[i];
        /* sign of det J of e1 (first-node origin), Leibniz */
        double J[9];
        int64_t e = f->e;
        for (int r = 0; r < dim; r++)
            for (int c = 0; c < dim; c++)
                J[r + c * dim] = coords[(int64_t)elems[e * nlb + c + 1] * dim + r] - coords[(int64_t)elems[e * nlb] * dim + r];
        double det = leibniz(J, dim, NULL);
        for (int t = 0; t < nv; t++) {
            int loc = (dim == 3) ? FACE3[f->k][det < 0 ? nv - 1 - t : t] : FACE2[f->k][det < 0 ? nv - 1 - t : t];
            faces[nf * nv + t] = elems[e * nlb + loc];
        }
        fel[nf * 2] = (int32_t)e;
        fel[nf * 2 + 1] = (j - i == 2) ? (int32_t)all[i + 1].e : -1;
        nf++;
        i = j;
    }
    free(all);
    return nf;
}

/* Points of an integration rule on every cell (sections 3.3 and 3.5, X_ip = amsm(coords3D, ip)):
 * X[(c*nq + q)*dim + i] = sum_j lam[q*nv + j] * coords[cells[c*nv + j]*dim + i]. */
int or_simplex_points(int dim, int nv, int64_t nn, const double* coords, int64_t nc, const int32_t* cells, int nq,
                      const double* lam, double* X) {
    for (int64_t c = 0; c < nc; c++)
        for (int q = 0; q < nq; q++)
            for (int i = 0; i < dim; i++) {
                double x = 0.0;
                for (int j = 0; j < nv; j++) {
                    int64_t v = cells[c * nv + j];
                    if (v < 0 || v >= nn) return -2;
                    x += lam[q * nv + j] * coords[v * dim + i];
                }
                X[(c * nq + q) * dim + i] = x;
            }
    return 0;
}

/* The GI function (section 3.4): value = sum_c sizes[c] * f_c with f_c = sum_q w_q fip[c, q]
 * for a scalar (d = 1), or f_c = sum_i n_ci sum_q w_q fip[c, q, i] for a vector field with
 * normals n (nc x d).  fip: nc x nq x d, component fastest.  Plain sum in cell order. */
double or_gi(int64_t nc, int nq, int d, const double* fip, const double* w, const double* sizes,
             const double* normals) {
    double value = 0.0;
    for (int64_t c = 0; c < nc; c++) {
        double fc = 0.0;
        for (int i = 0; i < d; i++) {
            double s = 0.0;
            for (int q = 0; q < nq; q++) s += w[q] * fip[(c * nq + q) * d + i];
            fc += normals ? normals[c * d + i] * s : s;
        }
        value += sizes[c] * fc;
    }
    return value;
}

/* P2 element matrices (section 3.6, stiffness_matrixP2 / mass_matrixP2) of straight-sided
 * triangles (dim 2) and tetrahedra (dim 3).  Local nodes: the nlb1 = dim + 1 vertices, then
 * the midpoints of the local edges (0,1), (0,2), (1,2) (2-D) or (0,1), (0,2), (0,3), (1,2),
 * (1,3), (2,3) (3-D).  Basis in barycentric coordinates: vertex i: lam_i (2 lam_i - 1),
 * edge (i,j): 4 lam_i lam_j; gradients from grad lam = the P1 gradients of or_p1_elements.
 * With |T| the element measure and rules (lamK, wK), (lamM, wM) whose weights sum to 1:
 *   K3D[e, a, b] = |T| sum_q wK_q cK[e, q] grad phi_a(x_q) . grad phi_b(x_q),
 *   M3D[e, a, b] = |T| sum_q wM_q cM[e, q] phi_a(x_q) phi_b(x_q)
 * (column-major nlb2 x nlb2 pages; cK, cM NULL = 1), and the error scales with |cK|,
 * |grad phi_a| |grad phi_b| and |cM| |phi_a phi_b|.  Returns the number of singular
 * Jacobians, or -1 / -2. */
static void p2_basis(int dim, const double* lam, double* phi) {
    int nlb1 = dim + 1, t = nlb1;
    for (int i = 0; i < nlb1; i++) phi[i] = lam[i] * (2.0 * lam[i] - 1.0);
    for (int i = 0; i < nlb1; i++)
        for (int j = i + 1; j < nlb1; j++) phi[t++] = 4.0 * lam[i] * lam[j];
}

static void p2_grads(int dim, const double* lam, const double* glam /* dim x nlb1, col-major */, double* gphi) {
    int nlb1 = dim + 1, t = nlb1;
    for (int i = 0; i < nlb1; i++)
        for (int r = 0; r < dim; r++) gphi[r + i * dim] = (4.0 * lam[i] - 1.0) * glam[r + i * dim];
    for (int i = 0; i < nlb1; i++)
        for (int j = i + 1; j < nlb1; j++, t++)
            for (int r = 0; r < dim; r++) gphi[r + t * dim] = 4.0 * (lam[i] * glam[r + j * dim] + lam[j] * glam[r + i * dim]);
}

int64_t or_p2_elements(int dim, int64_t nn, const double* coords, int64_t ne, const int32_t* elems, int nqK,
                       const double* lamK, const double* wK, const double* cK, int nqM, const double* lamM,
                       const double* wM, const double* cM, double* K3D, double* M3D, double* Kabs, double* Mabs) {
    if (dim != 2 && dim != 3) return -1;
    int nlb1 = dim + 1, nlb2 = (dim == 2) ? 6 : 10;
    double ds[3 * 4];
    p1_dshape(dim, ds);
    int64_t nsing = 0;
    for (int64_t e = 0; e < ne; e++) {
        double c3[3 * 4];
        for (int j = 0; j < nlb1; j++) {
            int64_t node = elems[e * nlb2 + j];
            if (node < 0 || node >= nn) return -2;
            for (int i = 0; i < dim; i++) AT(c3, dim, i, j) = coords[node * dim + i];
        }
        for (int j = nlb1; j < nlb2; j++)
            if (elems[e * nlb2 + j] < 0 || elems[e * nlb2 + j] >= nn) return -2;
        double tjac[9];
        for (int r = 0; r < dim; r++)
            for (int c = 0; c < dim; c++) {
                double acc = 0.0;
                for (int j = 0; j < nlb1; j++) acc += AT(ds, dim, r, j) * AT(c3, dim, c, j);
                AT(tjac, dim, r, c) = acc;
            }
        double vol = fabs(leibniz(tjac, dim, NULL)) / ((dim == 2) ? 2.0 : 6.0);
        double tinv[9];
        nsing += gauss_jordan(tjac, dim, tinv);
        double glam[3 * 4];
        for (int r = 0; r < dim; r++)
            for (int j = 0; j < nlb1; j++) {
                double acc = 0.0;
                for (int p = 0; p < dim; p++) acc += AT(tinv, dim, r, p) * AT(ds, dim, p, j);
                AT(glam, dim, r, j) = acc;
            }
        double* Ke = K3D ? K3D + e * nlb2 * nlb2 : NULL;
        double* Me = M3D ? M3D + e * nlb2 * nlb2 : NULL;
        double* Ka = Kabs ? Kabs + e * nlb2 * nlb2 : NULL;
        double* Ma = Mabs ? Mabs + e * nlb2 * nlb2 : NULL;
        for (int k = 0; k < nlb2 * nlb2; k++) {
            if (Ke) Ke[k] = 0.0;
            if (Me) Me[k] = 0.0;
            if (Ka) Ka[k] = 0.0;
            if (Ma) Ma[k] = 0.0;
        }
        for (int q = 0; q < nqK; q++) {
            double gphi[3 * 10], gn[10];
            p2_grads(dim, lamK + q * nlb1, glam, gphi);
            for (int a = 0; a < nlb2; a++) {
                double g2 = 0.0;
                for (int r = 0; r < dim; r++) g2 += gphi[r + a * dim] * gphi[r + a * dim];
                gn[a] = sqrt(g2);
            }
            double c = cK ? cK[e * nqK + q] : 1.0;
            for (int a = 0; a < nlb2; a++)
                for (int b = 0; b < nlb2; b++) {
                    double gg = 0.0;
                    for (int r = 0; r < dim; r++) gg += gphi[r + a * dim] * gphi[r + b * dim];
                    if (Ke) Ke[a + b * nlb2] += vol * wK[q] * c * gg;
                    if (Ka) Ka[a + b * nlb2] += vol * wK[q] * fabs(c) * gn[a] * gn[b];
                }
        }
        for (int q = 0; q < nqM; q++) {
            double phi[10];
            p2_basis(dim, lamM + q * nlb1, phi);
            double c = cM ? cM[e * nqM + q] : 1.0;
            for (int a = 0; a < nlb2; a++)
                for (int b = 0; b < nlb2; b++) {
                    if (Me) Me[a + b * nlb2] += vol * wM[q] * c * phi[a] * phi[b];
                    if (Ma) Ma[a + b * nlb2] += vol * wM[q] * fabs(c * phi[a] * phi[b]);
                }
        }
    }
    return nsing;
}
