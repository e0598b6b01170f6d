/*
 * pagefem.h -- C ABI of libpagefem.so: page-wise small dense linear algebra and P1 finite
 * element assembly on AMD Instinct MI355X (gfx950).
 *
 * The operations follow "On a vectorized basic linear algebra package for prototyping
 * codes in MATLAB" (Moskovka, Rahman, Valdman, Vatne, arXiv 2404.16039):
 *   section 2.2  page-wise multiplication, transpose, scalar multiplication, bilinear form
 *                evaluation
 *   section 2.3  page-wise determinant and inverse, transformation of normals
 *   section 2.4  the library functions amtam, avtam, avtav, astam, amsm, amsv, smamt,
 *                svamt, aminv, amt, amdet, avtamav
 *   section 3.1  the coords3D / vectors3D structures
 *   section 3.2  volumes and normals
 *   section 3.3  volume integrals (integration points of a rule on every cell)
 *   section 3.4  the GI function
 *   section 3.5  surface integrals (boundary faces, their normals and areas)
 *   section 3.6  derivative routine, P1 stiffness and mass matrices, sparse() assembly
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Memory: every array argument is DEVICE memory owned by the caller, unless stated.
 *    Opaque handles (pf_csr, pf_plan, pf_server) are owned by the library and freed by
 *    their *_destroy call.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls enqueue their kernels on it and return; outputs are valid once the stream has
 *    been synchronised.  Calls that must read a size back to the host say so.
 *  - Errors: every call returns a pf_status; pf_last_error() gives a message for the last
 *    failure on the calling thread.  Numerical events (singular pages, FP64-routed pages,
 *    out-of-range indices found on the device) are not errors: they are reported through
 *    optional per-page flags and device counters, so no call synchronises for them.
 *  - Pages: a batch of `count` matrices of `rows` x `cols` is described by pf_pages with
 *    element strides.  The paper's (MATLAB) layout is column-major inside a page with pages
 *    contiguous: s_row = 1, s_col = rows, s_page = rows*cols.  The structure-of-arrays
 *    layout (component-major) is s_page = 1, s_row = count, s_col = rows*count.  s_page = 0
 *    broadcasts one page to every index (the copy map of section 2.2, used by amsm, amsv,
 *    smamt, svamt).  Orders are 1..4 in each dimension.
 *  - Indices: element and face connectivity is 0-based int32, row-major (element e's
 *    nodes at elems[e*nlb .. e*nlb+nlb-1]); coordinates are float64, row-major nn x dim.
 *  - Device counters (nullable int64_t[4] in device memory, zeroed by the caller; calls
 *    add to them): [0] pages/elements routed to FP64, [1] singular pages/elements,
 *    [2] out-of-range indices met, [3] reserved.  The element-parallel calls (pf_elem_*,
 *    pf_rhs, pf_p2_elements) and pf_assemble(_quad) count per workgroup: a call given
 *    counters takes a small stream-ordered pool block (pf_assemble: an array of the
 *    structure) for the workgroups' counts and one more launch that sums them in; without
 *    counters neither happens.
 *  - Per-page flags (nullable uint8 array, one per page/element): bit 0 singular
 *    (determinant exactly zero in the final precision), bit 1 routed to FP64, bit 2 bad
 *    index.
 */
#ifndef PAGEFEM_H
#define PAGEFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PF_OK = 0,
    PF_EINVAL = 1,   /* invalid argument (null pointer, negative size, bad stride)      */
    PF_EDTYPE = 2,   /* unsupported precision                                           */
    PF_EORDER = 3,   /* unsupported matrix order or shape                               */
    PF_ENOMEM = 4,   /* device or host allocation failed                                */
    PF_EHIP = 5,     /* HIP runtime error (message has the HIP error string)            */
    PF_EINDEX = 6,   /* out-of-range connectivity index found while building a structure */
    PF_ELIMIT = 7,   /* a documented size limit was exceeded                             */
    PF_EBUDGET = 8,  /* a request can never fit the configured memory budget             */
    PF_ESTATE = 9    /* handle used in the wrong state                                   */
} pf_status;

typedef enum { PF_F32 = 0, PF_F64 = 1 } pf_dtype;

typedef struct pf_pages {
    int32_t rows, cols;            /* page shape, 1..4 each                             */
    int64_t count;                 /* number of pages (>= 0)                            */
    int64_t s_row, s_col, s_page;  /* strides in elements; s_page == 0 broadcasts       */
} pf_pages;

/* FP64 routing of the FP32 path: a page/element is recomputed in FP64 when its FP32
 * determinant (compensated) satisfies |det| < tau_abs, or its det-condition
 * sum_j |a_0j C_0j| / |det| (expansion along the first row) exceeds tau_cond, or det is
 * zero (infinite det-condition) or not finite.  Elements (the P1 geometry of every element
 * kernel, P2 included, and of assembly) are in addition routed when their vertex shape seen
 * from their first node, sigma = prod_k |p_k - p_0| / |det J|, exceeds 16: the FP32 error of
 * the gradients and of K relative to |grad phi_a| |grad phi_b| grows as ~7 sigma u_32, which
 * this keeps below 1e-5 on meshes of any shape (a fixed threshold, not an argument; sigma is
 * at most 6.5 on jittered Kuhn meshes).  enable = 0 turns routing off.  A NULL pf_fallback*
 * means {tau_abs = 0, tau_cond = 1e6, enable = 1}.  Ignored on the FP64 path.           */
typedef struct pf_fallback {
    double tau_abs;
    double tau_cond;
    int32_t enable;
} pf_fallback;

const char* pf_last_error(void);
int pf_version(void);

/* ------------------------------------------------------------------------------------
 * Page operations (section 2.2, page-wise maps; section 2.3, determinants
 * and inverses; section 2.4, library functions)
 * ---------------------------------------------------------------------------------- */

/* Page-wise determinant det_W (section 2.3; amdet).  A: n x n pages, n = 1..4.
 * det: `count` values of `dtype`, contiguous.  flags, d_counters nullable. */
pf_status pf_page_det(pf_dtype dtype, const pf_pages* A, const void* a, void* det,
                      const pf_fallback* fb, uint8_t* flags, int64_t* d_counters, void* stream);

/* Page-wise inverse on det_W^{-1}(W*) (section 2.3; aminv, which also returns the
 * determinants).  X: output pages (n x n).  det (nullable): determinants as in
 * pf_page_det.  A page with zero determinant gets the IEEE result of adj(A)/0 (inf/nan)
 * and flag bit 0; it is counted in d_counters[1]. */
pf_status pf_page_inv(pf_dtype dtype, const pf_pages* A, const void* a, const pf_pages* X, void* x,
                      void* det, const pf_fallback* fb, uint8_t* flags, int64_t* d_counters,
                      void* stream);

/* Page-wise transpose (section 2.2; amt).  A: r x c pages, T: c x r pages. Bit-exact. */
pf_status pf_page_transpose(pf_dtype dtype, const pf_pages* A, const void* a, const pf_pages* T,
                            void* t, void* stream);

/* Page-wise product C_k = op(A_k) op(B_k) (section 2.2, page-wise matrix multiplication;
 * section 2.4 amtam, avtam, avtav, amsm, amsv, smamt, svamt are instances).  op(X) = X or
 * X^T per the trans flag.  op(A): m x k, op(B): k x n, C: m x n, all dims 1..4; a
 * broadcast operand (s_page = 0) is one matrix used for every page.  C.count pages are
 * computed; non-broadcast A/B must have count equal to C.count. */
pf_status pf_page_mtimes(pf_dtype dtype, const pf_pages* A, const void* a, int transA,
                         const pf_pages* B, const void* b, int transB, const pf_pages* C, void* c,
                         void* stream);

/* Page-wise matrix-vector product y_k = op(A_k) x_k (section 2.4 amsv / avtam pattern);
 * x, y are vectors given as n x 1 pages.  Same rules as pf_page_mtimes. */
pf_status pf_page_mv(pf_dtype dtype, const pf_pages* A, const void* a, int transA,
                     const pf_pages* X, const void* x, const pf_pages* Y, void* y, void* stream);

/* Page-wise scalar multiplication C_k = s_k A_k (section 2.2, Id (x) pi; astam).
 * s: count scalars, contiguous, or one scalar broadcast when s_stride = 0. */
pf_status pf_page_scale(pf_dtype dtype, const void* s, int64_t s_stride, const pf_pages* A,
                        const void* a, const pf_pages* C, void* c, void* stream);

/* Page-wise bilinear form q_k = u_k^T A_k v_k (section 2.2, page-wise bilinear form
 * evaluation; avtamav).  u, v: n x 1 pages; q: count values, contiguous. */
pf_status pf_page_bilinear(pf_dtype dtype, const pf_pages* U, const void* u, const pf_pages* A,
                           const void* a, const pf_pages* V, const void* v, void* q, void* stream);

/* ------------------------------------------------------------------------------------
 * P1 elements (section 3.6, derivative routine and P1 stiffness / mass; section 3.2,
 * volumes and normals).  dim = 2 (triangles, nlb = 3) or 3 (tetrahedra, nlb = 4).
 * prec = PF_F64: FP64 arithmetic and outputs.  prec = PF_F32: FP32 arithmetic (Jacobian
 * edges subtracted in FP64, then rounded), compensated determinant, FP64 recomputation of
 * routed elements, FP32 outputs.  The Jacobian uses the first node as origin,
 * J = [p_2 - p_1, ..., p_{d+1} - p_1] (the transpose of the routine's tjac).
 * ---------------------------------------------------------------------------------- */

/* Per-element geometry.  Outputs (each nullable, type = prec):
 *   det[ne]            signed det J
 *   vol[ne]            |det J| / dim!                                 (section 3.2)
 *   grads[ne][dim*nlb] dphi = J^{-T} D, column-major dim x nlb; column j = grad phi_j
 *   normals[ne][dim*nlb] normals3D = vectors3D^{-T} normalsRef = -grads  (section 3.2)
 *   facet[ne][nlb]     measure of the facet opposite node j = dim |T| |grad phi_j|    */
pf_status pf_elem_geometry(int dim, pf_dtype prec, int64_t nn, const double* coords, int64_t ne,
                           const int32_t* elems, void* det, void* vol, void* grads, void* normals,
                           void* facet, const pf_fallback* fb, uint8_t* flags,
                           int64_t* d_counters, void* stream);

/* Element stiffness and mass matrices (the listings' K3D and M3D outputs), column-major
 * nlb x nlb per element: K_e = cK_e |T| dphi^T dphi, M_e = cM_e |T| (1 + delta_ab) /
 * ((d+1)(d+2)) (the exact P1 mass for an element-wise constant coefficient).  cK, cM:
 * per-element coefficients of type prec, nullable (= 1).  K3D, M3D nullable. */
pf_status pf_elem_stiffness_mass(int dim, pf_dtype prec, int64_t nn, const double* coords,
                                 int64_t ne, const int32_t* elems, const void* cK, const void* cM,
                                 void* K3D, void* M3D, const pf_fallback* fb, uint8_t* flags,
                                 int64_t* d_counters, void* stream);

/* Integration points of every element for coefficients given at integration points (the
 * coeffs_in_ip step of the section 3.6 listings).  order 1: the centroid (1 point); order
 * 2: the degree-2 exact rule, in 2-D the 3 edge midpoints (point q on the edge between local
 * nodes q and q+1 mod 3), in 3-D the 4 points with barycentric coordinate A = (5+3 sqrt 5)/20
 * at local node q and B = (5 - sqrt 5)/20 at the others; equal weights summing to 1/dim!.
 * xq[ne][nq][dim] (FP64): the caller evaluates its coefficient functions there and passes
 * the values to pf_assemble_quad.  Bad node ids give NaN points.  PF_EINVAL for another
 * order. */
pf_status pf_quad_points(int dim, int order, int64_t nn, const double* coords, int64_t ne,
                         const int32_t* elems, double* xq, void* stream);

/* Boundary facets (section 3.2 normals; facesB / areasB of the surface integrals of
 * section 3.5).
 * dim = 3: faces[nf][3] triangles (a,b,c), n = (b-a) x (c-a), measure = |n| / 2.
 * dim = 2: faces[nf][2] edges (a,b), n = (b_y - a_y, a_x - b_x), measure = |n|.
 * unit[nf][dim] = n / |n| (nullable), measure[nf] (nullable), type prec. */
pf_status pf_boundary_normals(int dim, pf_dtype prec, int64_t nn, const double* coords, int64_t nf,
                              const int32_t* faces, void* unit, void* measure, void* stream);

/* ------------------------------------------------------------------------------------
 * Assembly: sparse(X3D(:), Y3D(:), K3D(:), nn, nn) of the P1 listings (section 3.6).
 * The CSR pattern holds every pair of nodes that share an element (entries that sum to
 * zero are kept), columns ascending in each row.  K and M are symmetric, so the CSR
 * arrays equal the compressed-column arrays of the global matrices.
 * ---------------------------------------------------------------------------------- */
typedef struct pf_csr pf_csr;

/* Create an empty structure handle (host call, no device work). */
pf_status pf_csr_create(pf_csr** out);

/* Build (or rebuild) the CSR structure of a P1 mesh: node-to-element adjacency and the
 * row pattern.  The handle keeps the CSR pattern (row_ptr, and col_idx of exactly nnz
 * words), the node-to-element adjacency in CSR form (4*ne entries with their packed column
 * positions) and each row's diagonal position: 12 (nn + 1) + 4 nnz + 32 ne bytes for a 3-D
 * mesh.  Its device memory comes from a stream-ordered pool of the library (enqueued on
 * `stream`); the build's own scratch (padded adjacency rows and row-pattern columns, about
 * 520 bytes per node) is released when the build ends.  This call synchronises `stream`
 * once, to read nnz and the error word back (the exact size of col_idx).  A rebuild whose
 * nonzeros fit the col_idx of an earlier build in the handle is then complete; otherwise the
 * call returns with the last step (the columns into a col_idx of exactly nnz words) enqueued
 * on `stream`: the library's later calls on the handle order their work after it on any
 * stream (a device-side wait, no host wait), and pf_csr_info, which hands out device
 * pointers, waits for it on the host.
 * Rows whose node lies in more than 64 elements, or that hold more than 64 nonzeros, are
 * long rows: the build lists them (one more synchronisation of `stream`, only then) and
 * builds them with one workgroup per row, and pf_assemble, pf_assemble_quad,
 * pf_csr_assemble_pages and pf_rhs assemble them the same way (exactly, in FP64, rounded
 * once to the output type); pf_csr_faces refuses a structure with long rows.
 * Limits: 4*ne < 2^31, nnz < 2^31, at most 256 nonzeros per row (PF_ELIMIT otherwise).
 * Out-of-range node ids give PF_EINDEX; PF_EINVAL if the row
 * offsets could not be formed (a bounded wait between the workgroups of the row-offset
 * scan ran out, which the device's in-order start of workgroups rules out). */
pf_status pf_csr_symbolic(pf_csr* csr, int dim, int64_t nn, int64_t ne, const int32_t* elems,
                          void* stream);

/* Build the CSR structure of a P2 mesh (section 3.6: the global matrices of the
 * stiffness_matrixP2 / mass_matrixP2 listings): elems2 ne x nlb2 int32 (nlb2 = 6 for dim 2,
 * 10 for dim 3) as for pf_p2_elements; every pair of nodes that share an element is an entry.
 * A row of a node in more than 64 elements, or of more than 128 nonzeros (a vertex of the
 * Kuhn cube's P2 mesh has 65), is a long row, built and assembled by one workgroup as in
 * pf_csr_symbolic; any row holds at most 256 nonzeros, ne < 2^27 (PF_ELIMIT otherwise);
 * otherwise as pf_csr_symbolic.  The
 * handle then serves pf_csr_info, pf_csr_assemble_pages and the stage timing; the P1 calls
 * (pf_assemble, pf_assemble_quad, pf_csr_faces, pf_rhs, pf_energies) return PF_ESTATE. */
pf_status pf_csr_symbolic_p2(pf_csr* csr, int dim, int64_t nn, int64_t ne, const int32_t* elems2,
                             void* stream);

/* sparse(X3D(:), Y3D(:), K3D(:)) of the section 3.6 listings for the structure's mesh (P1 or
 * P2), with Y3D(a, b, e) = elems(e, a) and X3D its page transpose: valsK[k] = the sum, over
 * elements e and local pairs (a, b) such that entry k is row elems[e][b], column
 * elems[e][a], of pagesK[e*nlb^2 + a + b*nlb]; the same for M.
 * Pages ne x nlb x nlb column-major of type prec, as pf_elem_stiffness_mass (P1) and
 * pf_p2_elements (P2) write them; device pointers.  Each value is summed exactly on a grid
 * fixed by its largest contribution, as in pf_assemble.  valsK or valsM nullable (not both);
 * each output needs its pages.  Rows are taken 32, 16, 8 or 4 at a time, as the longest
 * adjacency list and the LDS budget allow; PF_ELIMIT if 4 consecutive rows (starting at a
 * multiple of 4) hold more entries than that budget (4096 FP32, 2730 FP64).  Page arrays
 * that start 16-byte aligned are read with vector loads (any alignment of the type is
 * accepted). */
pf_status pf_csr_assemble_pages(const pf_csr* csr, pf_dtype prec, const void* pagesK,
                                const void* pagesM, void* valsK, void* valsM, void* stream);

/* Read the structure: sizes on the host, device pointers owned by the handle. */
pf_status pf_csr_info(const pf_csr* csr, int64_t* nn, int64_t* nnz, const int32_t** row_ptr,
                      const int32_t** col_idx);

/* Device bytes the handle holds (a memory-planning aid): *resident = the structure's own
 * arrays (the CSR pattern, the compact adjacency with its slot words, the diagonal
 * positions, and the face lists and energy workspace once built); *scratch = build scratch
 * still held (non-zero only while a build is in flight).  Both nullable; host call. */
pf_status pf_csr_memory(const pf_csr* csr, int64_t* resident, int64_t* scratch);

/* Launch shape of pf_assemble and pf_assemble_quad on a built P1 structure in precision
 * prec (a diagnostic, e.g. for tests that must reach every variant of the numeric kernel):
 * rows per workgroup of the numeric launch and the largest number of elements around one
 * node (both nullable).  PF_ESTATE for a P2 or unbuilt structure. */
pf_status pf_csr_numeric_info(const pf_csr* csr, pf_dtype prec, int32_t* rows_per_block,
                              int32_t* max_adj);

/* Per-stage device time of pf_csr_symbolic, a profiling aid.  pf_csr_set_timing(csr, 1)
 * clears the sums and makes every later pf_csr_symbolic call on the handle record HIP
 * events on its stream between its stages (0 stops recording).  pf_csr_stage_times waits
 * for the events of the last call and writes ms[PF_CSR_STAGES], the summed milliseconds
 * of each stage since timing was switched on, and *calls, the number of calls summed
 * (nullable).  Stages: adjacency (counting scatter and the scan of the adjacency lengths),
 * row pattern, row offsets (the scan of the row lengths with row_ptr, nnz and the numeric
 * launch statistics), columns (col_idx, enqueued once nnz has reached the host; the host's
 * wait between the row offsets and the columns belongs to no stage). */
#define PF_CSR_STAGES 4
pf_status pf_csr_set_timing(pf_csr* csr, int on);
pf_status pf_csr_stage_times(pf_csr* csr, double* ms, int64_t* calls);

/* Numeric assembly of the global K (valsK[nnz]) and M (valsM[nnz], nullable) of the mesh
 * whose structure `csr` holds (the handle keeps the connectivity it was built from;
 * `elems` is accepted for symmetry with the element calls and may be NULL).  coords may
 * change between calls (same topology).  Each value is the sum of its element
 * contributions, each first rounded onto a grid fixed by the value's largest contribution
 * (2^-24 of its power of two for FP32, 2^-56 for FP64), so the sum is exact and does not
 * depend on the order of the additions: the same inputs give the same bits.  Every element row is computed with that row's node as the origin of the edge
 * vectors.  prec as for the element calls; cK, cM per-element coefficients, nullable
 * (= 1).  d_counters[0] counts FP64-routed elements once each (FP32 with routing enabled:
 * each workgroup stores its count in an array of the structure, one int per 4 to 16 rows,
 * that a second launch sums into the counter; calls on one structure whose numeric phases
 * overlap in time, on two streams, share that array and may mix their routed counts, while
 * their values are unaffected). */
pf_status pf_assemble(const pf_csr* csr, pf_dtype prec, const double* coords, const int32_t* elems,
                      const void* cK, const void* cM, void* valsK, void* valsM,
                      const pf_fallback* fb, int64_t* d_counters, void* stream);

/* Numeric assembly with coefficients given at the integration points of a rule of `order`
 * (1 or 2, the rules of pf_quad_points), as the loop over integration points of the
 * section 3.6 listings: K_e = sum_q w_q cK_q |det J| dphi^T dphi, M_e = sum_q w_q cM_q
 * |det J| phi(x_q) phi(x_q)^T.  cKq, cMq: ne x nq values of type prec in element-major
 * order (nullable = 1).  Everything else as pf_assemble. */
pf_status pf_assemble_quad(const pf_csr* csr, pf_dtype prec, const double* coords, int order,
                           const void* cKq, const void* cMq, void* valsK, void* valsM,
                           const pf_fallback* fb, int64_t* d_counters, void* stream);

/* All faces of the mesh whose structure `csr` holds (section 3.2: the normals of all faces,
 * internal ones included, or of the boundary faces only); elems: the connectivity it was
 * built from.  A face is the set of dim nodes of an element minus one node; faces are
 * listed in ascending order of their sorted node ids, each once, with its nodes ordered so
 * that the normal of pf_boundary_normals points out of its first element e1 (the smaller
 * element id; the orientation follows the sign of e1's det J) and the element pair
 * (e1, e2), e2 = -1 on the boundary.  The boundary faces, in the same order, also form a
 * list of their own (the section 3.5 facesB) with their elements.  Built from the
 * structure's adjacency and row patterns inside the handle; synchronises `stream` once
 * (the counts size the lists).  PF_EINVAL if a face belongs to more than two elements,
 * PF_ELIMIT if a node owns more than 128 faces (the faces whose smallest node it is), or
 * more than 1024 for the node of a long row (see pf_csr_symbolic).  A later
 * pf_csr_symbolic invalidates it. */
pf_status pf_csr_faces(pf_csr* csr, const double* coords, const int32_t* elems, void* stream);

/* The face lists of pf_csr_faces: counts on the host, device pointers owned by the handle:
 * faces nf x dim, fel nf x 2 (e1, e2), bfaces nfb x dim, bel nfb (the element of each
 * boundary face).  Any output may be NULL. */
pf_status pf_csr_faces_info(const pf_csr* csr, int64_t* nf, int64_t* nfb, const int32_t** faces,
                            const int32_t** fel, const int32_t** bfaces, const int32_t** bel);

/* P2 element matrices (section 3.6, stiffness_matrixP2 / mass_matrixP2) of straight-sided
 * triangles (dim 2) and tetrahedra (dim 3).  elems2: ne x nlb2 int32 (nlb2 = 6 / 10): the
 * dim + 1 vertices, then the mid-edge nodes of the local edges (0,1), (0,2), (1,2) (2-D) or
 * (0,1), (0,2), (0,3), (1,2), (1,3), (2,3) (3-D); the geometry comes from the vertices.
 * Basis: lam_i (2 lam_i - 1) at vertex i, 4 lam_i lam_j at edge (i,j).  With |T| the element
 * measure and rules given as barycentric points (host, nq x (dim+1)) and weights summing to 1
 * (host, nq; at most PF_P2_RULE_MAX points):
 *   K3D[e*nlb2^2 + a + b*nlb2] = |T| sum_q wK_q cK_q grad phi_a . grad phi_b (rule K),
 *   M3D[e*nlb2^2 + a + b*nlb2] = |T| sum_q wM_q cM_q phi_a phi_b            (rule M),
 * column-major pages of type prec; cKq, cMq: ne x nq of type prec (nullable = 1); K3D or M3D
 * nullable (then its rule is ignored).  FP32 recomputes routed elements in FP64 as
 * pf_elem_stiffness_mass; d_counters: [0] routed, [2] bad node index (NaN pages). */
#define PF_P2_RULE_MAX 32
pf_status pf_p2_elements(int dim, pf_dtype prec, int64_t nn, const double* coords, int64_t ne,
                         const int32_t* elems2, int nqK, const double* lamK, const double* wK,
                         const void* cKq, int nqM, const double* lamM, const double* wM,
                         const void* cMq, void* K3D, void* M3D, const pf_fallback* fb,
                         int64_t* d_counters, void* stream);

/* ----------------------------------------------------------------------------------
 * Integration over cells (sections 3.3-3.5): points of a rule (X_ip = amsm(coords3D, ip)) and the
 * GI function (section 3.4).
 * A rule is nq barycentric points lam (host, nq x nv, row-major) with weights w (host, nq)
 * summing to 1; at most PF_RULE_MAX points.
 * ---------------------------------------------------------------------------------- */
#define PF_RULE_MAX 64
#define PF_GI_WORK 2048

/* Points of a rule on every cell (X_ip = amsm(coords3D, ip)): cells are nc simplices of nv
 * nodes each (nv = dim + 1 elements, nv = dim boundary faces, ...), int32 row-major;
 * X (device, FP64) receives nc x nq x dim values, X[(c*nq + q)*dim + i] =
 * sum_j lam[q*nv + j] coords[cells[c*nv + j]*dim + i]; a cell with a bad node gets NaN. */
pf_status pf_simplex_points(int dim, int nv, int64_t nn, const double* coords, int64_t nc,
                            const int32_t* cells, int nq, const double* lam, double* X, void* stream);

/* The GI function (section 3.4): value = sum_c sizes[c] f_c with
 * f_c = sum_i normals[c*d + i] sum_q w_q fip[(c*nq + q)*d + i] (normals nullable: the plain
 * sum over the d components, d = 1 for a scalar), i.e. the integral of a scalar function or
 * the flux of a vector field through oriented cells.  fip, sizes, normals: device, type prec;
 * value: device, one FP64; work: device scratch of PF_GI_WORK doubles.  Sums in FP64 in a
 * fixed order (deterministic). */
pf_status pf_gi(pf_dtype prec, int64_t nc, int nq, int d, const void* fip, const double* w,
                const void* sizes, const void* normals, double* value, double* work, void* stream);

/* Load vector (section 3.6, right-hand side listing) of the mesh whose structure `csr`
 * holds; elems: the connectivity it was built from (ne x (dim+1), device).  For every
 * element, b2D[e*nlb + j] = |det J_e| sum_q w_q f_eq phi_j(x_q) over the points of the rule
 * of `order` (1 or 2, those of pf_quad_points; fq: ne x nq values of type prec,
 * element-major), in prec (FP32 recomputes the determinant of routed elements in FP64, as
 * pf_elem_stiffness_mass).  b (nn values, nullable): the accumarray step, b[i] = the sum of
 * the entries of the elements around node i, read through the handle's node-element
 * adjacency and summed exactly on a grid fixed by the largest entry (2^-24 of its power of
 * two for FP32, 2^-56 for FP64): deterministic.  b2D (device, ne x nlb, type prec) is
 * required.  d_counters: [0] routed elements, [2] elements with a bad node index (their
 * entries are NaN). */
pf_status pf_rhs(const pf_csr* csr, pf_dtype prec, const double* coords, const int32_t* elems,
                 int order, const void* fq, void* b2D, void* b, const pf_fallback* fb,
                 int64_t* d_counters, void* stream);

/* Local energy parts (section 3.6, element-wise contributions to the energy functional) of
 * the P1 function with nodal values u (nn values of type prec, device) on the mesh of `csr`
 * (elems as for pf_rhs): J[e] = 1/2 u_e^T K_e u_e, J[ne + e] = 1/2 u_e^T M_e u_e,
 * J[2 ne + e] = -b2D_e^T u_e, with K_e and M_e the element matrices of pf_assemble_quad for
 * the rule of `order` (cKq, cMq: ne x nq, nullable = 1) and b2D the local load vectors of
 * pf_rhs (nullable: the third part is 0).  The bilinear forms are evaluated as
 * 1/2 mean(cK) |det| |grad u_e|^2 / d! and 1/2 |det| sum_q w_q cM_q u_e(x_q)^2, which equal
 * them.  J (device, 3 ne values of type prec) is nullable; totals (device, 3 doubles,
 * nullable) receives the sums of the stored J values over all elements, in FP64 and in a
 * fixed order (deterministic).  Uses a workspace of the handle (grown when needed, so the
 * handle is not const).  d_counters as pf_rhs. */
pf_status pf_energies(pf_csr* csr, pf_dtype prec, const double* coords, const int32_t* elems,
                      int order, const void* cKq, const void* cMq, const void* u, const void* b2D,
                      void* J, double* totals, const pf_fallback* fb, int64_t* d_counters,
                      void* stream);

/* pf_energies for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops and harnesses that forbid hipMalloc): the same arguments, kernels and results
 * (J and totals bit for bit those of pf_energies), but the FP64 block sums live in a static
 * per-device array of the library (3 x 2048 doubles, 48 KiB, held on every device the call runs
 * on until the process ends) instead of a workspace of the handle, so the handle is const and
 * the call makes no hipMalloc, hipFree or other allocating call.  The array's address on the
 * current device is looked up once, at the first call on that device.  The block count of the
 * energy kernel is capped at 2048 for any mesh, so no mesh is too large; PF_EINVAL would report
 * a need beyond the array.  All calls on one device share the array: calls that overlap on a
 * device (two streams, or two threads) race on it and give undefined totals; serialise them. */
pf_status pf_energies_noalloc(const pf_csr* csr, pf_dtype prec, const double* coords,
                              const int32_t* elems, int order, const void* cKq, const void* cMq,
                              const void* u, const void* b2D, void* J, double* totals,
                              const pf_fallback* fb, int64_t* d_counters, void* stream);

/* Release a structure handle: waits for the device (as hipFree would), returns the handle's
 * memory to the library's pool and the pool's unused memory to the device.  NULL is a no-op. */
void pf_csr_destroy(pf_csr* csr);

/* ----------------------------------------------------------------------------------
 * Mixed-order batch plans: one persistent launch applies the page-wise inverse (with
 * determinant, section 2.3) and the page-wise product of section 2.2 (aminv and the
 * amsm/amtam-style products of section 2.4) to many groups of square pages of different
 * orders at once.
 *
 * A plan holds a work list (one descriptor per group, tiles of each group numbered
 * consecutively) in pinned host memory and a copy of it in device memory.  pf_plan_run
 * replays a HIP graph of two nodes: the host-to-device copy of the work list, then one
 * persistent kernel whose workgroups (compute units x occupancy) walk the tiles in
 * round-robin order.  Group pointers and counts may change between runs without a new
 * graph (pf_plan_set_groups); a new schedule with another wave count re-captures it.
 *
 * Pages of every group use the paper's layout (column-major n x n pages stored back to
 * back, element (r, c) of page k at k*n*n + r + c*n); pointers need the natural alignment
 * of the element type only.  FP32 plans compute the inverse with compensated cofactors
 * and route pages by the fallback predicate to FP64, exactly as pf_page_inv; products
 * are FMA chains in ascending inner index (bitwise the same for every schedule).
 * ---------------------------------------------------------------------------------- */
typedef struct pf_plan pf_plan;

enum { PF_OP_INV = 1, PF_OP_MTIMES = 2 };

typedef struct {
    int32_t order;    /* n, 1..4                                                          */
    int32_t ops;      /* PF_OP_INV and/or PF_OP_MTIMES                                    */
    int64_t count;    /* pages in the group (0 allowed)                                   */
    const void* a;    /* count pages A                                                    */
    const void* b;    /* count pages B (PF_OP_MTIMES), else ignored                       */
    void* x;          /* out: inv(A) (PF_OP_INV), else ignored                            */
    void* c;          /* out: A*B (PF_OP_MTIMES), else ignored                            */
    void* det;        /* out: det(A) (PF_OP_INV, nullable)                                */
} pf_group;

/* Schedule of one order: lanes per matrix (1, n or n*n), LDS staging of the tile (1) or
 * direct per-lane loads (0), and chunks per tile (1..16; a chunk is one page per lane for
 * lanes = 1, else floor(64/lanes) pages per wave). */
typedef struct {
    int32_t lanes, staged, tile;
} pf_order_schedule;

typedef struct {
    int32_t waves;               /* waves per workgroup: 1, 2, 4 or 8 */
    pf_order_schedule order[5];  /* indexed by the order, entry 0 unused */
} pf_schedule;

enum { PF_TUNE_CACHED = 0, PF_TUNE_FORCE = 1, PF_TUNE_DEFAULT = 2 };

/* Create a plan for up to max_groups groups of pages of type dtype (host call; allocates
 * the pinned and device work lists).  fb: routing of FP32 pages (NULL = tau_abs 0,
 * tau_cond 1e6, enabled).  The schedule starts as the default one. */
pf_status pf_plan_create(pf_dtype dtype, int32_t max_groups, const pf_fallback* fb, pf_plan** out);

/* Replace the plan's groups (ngroups <= max_groups).  Validates orders, ops, counts and
 * pointers (PF_EINVAL / PF_EORDER), waits for the plan's previous run to finish, then
 * rewrites the host work list; the next run copies it to the device. */
pf_status pf_plan_set_groups(pf_plan* plan, const pf_group* groups, int32_t ngroups);

/* Read / set the schedule.  PF_EINVAL for values outside the documented sets or a tile
 * staging buffer beyond the device's LDS per workgroup. */
pf_status pf_plan_get_schedule(const pf_plan* plan, pf_schedule* out);
pf_status pf_plan_set_schedule(pf_plan* plan, const pf_schedule* sched);

/* Choose the schedule for the current groups.  mode PF_TUNE_DEFAULT: the default schedule.
 * PF_TUNE_CACHED: look the groups' shape up in the JSON file `cache_path` (device
 * architecture, precision, total pages per order as a power-of-two bucket); on a miss,
 * tune and add the result to the file.  PF_TUNE_FORCE: tune and overwrite the entry.
 * Tuning times candidate schedules with HIP events on `stream` (it runs the plan, so it
 * writes the groups' outputs) and keeps the tuned schedule only if it beats the default
 * on the whole batch.  cache_path may be NULL (no file).  Synchronises `stream`. */
pf_status pf_plan_tune(pf_plan* plan, const char* cache_path, int32_t mode, void* stream);

/* Run the plan on `stream` by replaying its graph (captured on first use).  d_counters
 * (nullable, as for the page calls) receives routed and singular page counts. */
pf_status pf_plan_run(pf_plan* plan, int64_t* d_counters, void* stream);

/* The same work as pf_plan_run with ordinary launches (a copy, then the kernel). */
pf_status pf_plan_launch(pf_plan* plan, int64_t* d_counters, void* stream);

/* Launch geometry of the current schedule: tiles, workgroups, LDS bytes per workgroup. */
pf_status pf_plan_info(const pf_plan* plan, int64_t* ntiles, int32_t* grid, int32_t* lds_bytes);

void pf_plan_destroy(pf_plan* plan);

/* ----------------------------------------------------------------------------------
 * Serving loop: assembly jobs (the section 3.6 K and M of one P1 mesh each) and page-op jobs
 * (the section 2.3-2.4 page-wise inverse with determinant and page product of one batch of
 * pages each), submitted from host memory, are admitted by a device-memory budget and a
 * slot limit.  Every scheduler tick runs the numeric phase of all assembly jobs that are
 * ready in that tick as one launch per (dimension, precision, rows-per-block) class, and
 * all page-op jobs admitted in that tick as one persistent batch-plan launch per precision
 * (the mixed-order plan of pf_plan_run, replayed from its HIP graph).  Meshes with the same
 * non-zero topology key share their connectivity and CSR structure, which stay resident
 * (least recently used structures are evicted when the budget needs room); a new structure
 * is built on a stream of its own while the scheduler goes on admitting, launching and
 * completing other jobs, and its jobs join the tick in which the build has finished.
 *
 * A server owns one scheduler thread and one HIP stream on the device that is current
 * when it is created.  Per assembly job: host-to-device copy of the coordinates (and of the
 * connectivity plus the symbolic phase when the topology is not resident), the numeric
 * phase, then the device-to-host copy of the values when output buffers are given.  Per
 * page-op job: copies of its pages in, the batched page operations, copies of the results
 * out.  Times are seconds on the server clock (pf_server_now, steady clock, 0 at creation).
 * Latency = end of the job's compute launch - arrival; the copy back is reported apart.
 * Assembly values are bitwise those of pf_csr_symbolic + pf_assemble on the same mesh, and
 * page results bitwise those of the same pages in a plan of their own, alone or in any
 * batch.  Assembly coefficients are 1 (no cK/cM); page jobs are routed with the default
 * fallback (tau_abs 0, tau_cond 1e6) and report routed = -1 (their pages share the launch's
 * counters).
 * ---------------------------------------------------------------------------------- */
typedef struct pf_server pf_server;

enum { PF_SERVER_NOFUSE = 1, PF_SERVER_NOCACHE = 2 };
enum { PF_JOB_ASSEMBLY = 0, PF_JOB_PAGES = 1 };

typedef struct {
    int32_t dim;             /* assembly: 2 (triangles) or 3 (tetrahedra)                      */
    int32_t prec;            /* pf_dtype of the arithmetic and of the values                  */
    int64_t nn, ne;          /* assembly: nodes, elements (both > 0)                           */
    const double* coords;    /* assembly: HOST nn x dim, row-major (pinned: asynchronous copy) */
    const int32_t* elems;    /* assembly: HOST ne x (dim+1), 0-based                           */
    uint64_t topology;       /* assembly: non-zero: jobs with equal keys have identical elems  */
    double arrival;          /* arrival time on the server clock; < 0: the time of submission   */
    pf_fallback fb;          /* assembly: routing of FP32 jobs                                 */
    void* valsK;             /* assembly: HOST output, nullable: nnz values of K in CSR order  */
    void* valsM;             /* assembly: HOST output, nullable: nnz values of M               */
    int64_t vals_cap;        /* assembly: capacity of valsK / valsM in values (PF_ELIMIT if nnz exceeds) */
    int32_t kind;            /* PF_JOB_ASSEMBLY (0, the fields above) or PF_JOB_PAGES (below)  */
    int32_t order;           /* pages: n, 1..4                                                 */
    int32_t ops;             /* pages: PF_OP_INV and/or PF_OP_MTIMES                           */
    int32_t reserved;        /* 0                                                              */
    int64_t count;           /* pages: number of pages (> 0)                                   */
    const void* a;           /* pages: HOST count n x n pages A (paper layout), type prec      */
    const void* b;           /* pages: HOST count pages B (PF_OP_MTIMES), else ignored         */
    void* x;                 /* pages: HOST output inv(A) (PF_OP_INV), nullable                */
    void* c;                 /* pages: HOST output A*B (PF_OP_MTIMES), nullable                */
    void* det;               /* pages: HOST output det(A) (PF_OP_INV), nullable                */
} pf_job;

typedef struct {
    int32_t status;          /* pf_status of the job (valid once done)                       */
    int32_t done;            /* 1 once the job has finished (values copied back)              */
    int64_t nnz;             /* nonzeros of the job's CSR structure (0 for page-op jobs)      */
    int64_t routed;          /* elements recomputed in FP64 (-1 for page-op jobs)             */
    double arrival, admitted, finished, copied;  /* server clock                             */
} pf_job_result;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t elements;                  /* elements of the completed jobs                     */
    int64_t ticks, launches, max_batch;
    int64_t cache_hits, cache_misses, evictions;
    double latency_p50, latency_p99, latency_mean, latency_max;  /* seconds               */
    double first_arrival, last_finish; /* server clock                                        */
    double jobs_per_s, elements_per_s; /* completed work over [first_arrival, last_finish]    */
    int64_t hbm_in_use, hbm_high_water;  /* accounted device bytes                            */
    int64_t pages;                     /* pages of the completed page-op jobs                  */
    double pages_per_s;                /* over [first_arrival, last_finish]                     */
    /* scheduler thread, host seconds spent: freeing evicted structures, starting structure
     * builds, preparing and launching ticks; admissions that found the queue head waiting
     * for memory                                                                             */
    double evict_s, build_start_s, tick_s;
    int64_t admit_waits;
} pf_stats;

/* Create a server with a device-memory budget (bytes of job inputs, outputs and resident
 * structures, estimated before the structure is built and exact afterwards) and at most
 * max_slots jobs in flight.  flags: PF_SERVER_NOFUSE (one numeric launch per job),
 * PF_SERVER_NOCACHE (no resident structures: every job builds and frees its own). */
pf_status pf_server_create(size_t hbm_budget, int32_t max_slots, int32_t flags, pf_server** out);

/* Seconds since the server was created (steady clock). */
double pf_server_now(const pf_server* srv);

/* Queue a job (host call; the host arrays must stay valid until the job is done).
 * PF_EINVAL / PF_EORDER / PF_EDTYPE for invalid jobs, PF_EBUDGET if the job alone can
 * never fit the budget.  Jobs are admitted in submission order. */
pf_status pf_server_submit(pf_server* srv, const pf_job* job, uint64_t* ticket);

/* Device bytes a job is admitted with when its structure is not resident: inputs, values
 * and a new structure, estimated from its sizes (an upper bound of what it holds). */
pf_status pf_server_footprint(const pf_job* job, size_t* bytes);

/* State of a job; PF_EINVAL for an unknown ticket.  wait blocks until it is done. */
pf_status pf_server_poll(pf_server* srv, uint64_t ticket, pf_job_result* out);
pf_status pf_server_wait(pf_server* srv, uint64_t ticket, pf_job_result* out);

/* Block until every submitted job is done. */
pf_status pf_server_drain(pf_server* srv);

/* Counters and latency percentiles over the completed jobs. */
pf_status pf_server_stats(pf_server* srv, pf_stats* out);

/* Finish every submitted job, stop the scheduler thread and free all device memory. */
void pf_server_destroy(pf_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* PAGEFEM_H */
