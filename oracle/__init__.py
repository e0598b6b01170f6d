"""Plain FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It wraps ``pf_oracle.c`` (plain loops, double precision, built with
``-O2 -ffp-contract=off``) through ctypes and shares nothing with the HIP library.
Every function follows a definition of the paper (arXiv 2404.16039); the C source names
the section each one comes from.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# PF_ORACLE_LIB: an oracle library built elsewhere (the tests that plant mistakes in a copy
# of pf_oracle.c and check that the pins catch them load their build through it)
_ALT = os.environ.get("PF_ORACLE_LIB")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle into oracle/liboracle.so (plain gcc, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if _ALT:
            lib = C.CDLL(_ALT)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            lib = C.CDLL(_LIB)
        P = C.c_void_p
        I64 = C.c_int64
        INT = C.c_int
        D = C.c_double
        lib.or_page_det.argtypes = [INT, I64, P, P, P]
        lib.or_page_inv.argtypes = [INT, I64, P, P, P, P]
        lib.or_page_transpose.argtypes = [INT, INT, I64, P, P]
        lib.or_page_mtimes.argtypes = [INT, INT, INT, I64, P, INT, I64, P, INT, I64, P, P]
        lib.or_page_scale.argtypes = [INT, INT, I64, P, P, P]
        lib.or_page_bilinear.argtypes = [INT, I64, P, P, P, P]
        lib.or_p1_elements.argtypes = [INT, I64, P, I64, P, P, P, P, P, P, P, P]
        lib.or_p1_elements.restype = I64
        lib.or_create_coords3d.argtypes = [INT, INT, I64, P, I64, P, P, P]
        lib.or_quad_count.argtypes = [INT, INT]
        lib.or_quad_points.argtypes = [INT, INT, I64, P, I64, P, P]
        lib.or_p1_elements_q.argtypes = [INT, INT, I64, P, I64, P, P, P, P, P, P, P]
        lib.or_p1_elements_q.restype = I64
        lib.or_rhs_p1.argtypes = [INT, INT, I64, P, I64, P, P, P, P, P]
        lib.or_faces.argtypes = [INT, I64, P, I64, P, P, P, I64]
        lib.or_faces.restype = I64
        lib.or_simplex_points.argtypes = [INT, INT, I64, P, I64, P, INT, P, P]
        lib.or_gi.argtypes = [I64, INT, INT, P, P, P, P]
        lib.or_gi.restype = D
        lib.or_p2_elements.argtypes = [INT, I64, P, I64, P, INT, P, P, P, INT, P, P, P, P, P, P, P]
        lib.or_p2_elements.restype = I64
        lib.or_route_predicate.argtypes = [INT, P, I64, D, D, P, P]
        lib.or_assemble.argtypes = [INT, I64, I64, P, P, P, P, P, P, P, P, P, P, I64]
        lib.or_assemble.restype = I64
        lib.or_assemble_rows.argtypes = [INT, I64, P, I64, P, INT, P, INT, P, P, P, P, P, P]
        lib.or_boundary.argtypes = [INT, I64, P, I64, P, P, P, P]
        for f in ("or_page_det", "or_page_inv", "or_page_transpose", "or_page_mtimes", "or_page_scale",
                  "or_page_bilinear", "or_create_coords3d", "or_route_predicate", "or_assemble_rows",
                  "or_boundary", "or_quad_count", "or_quad_points"):
            getattr(lib, f).restype = INT
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")
    return rc


# ----------------------------------------------------------------------------- page ops
def page_det(a, n):
    """Leibniz determinant of each n x n column-major page. Returns (det, perm(|A|))."""
    a = _f64(a).reshape(-1, n * n)
    det = np.empty(a.shape[0])
    pa = np.empty(a.shape[0])
    _check(_load().or_page_det(n, a.shape[0], _p(a), _p(det), _p(pa)), "page_det")
    return det, pa


def page_inv(a, n):
    """Gauss-Jordan inverse of each page. Returns (inv, singular flags, |A^-1||A||A^-1|)."""
    a = _f64(a).reshape(-1, n * n)
    inv = np.empty_like(a)
    sing = np.empty(a.shape[0], dtype=np.uint8)
    sc = np.empty_like(a)
    _check(_load().or_page_inv(n, a.shape[0], _p(a), _p(inv), _p(sing), _p(sc)), "page_inv")
    return inv, sing, sc


def page_transpose(a, rows, cols):
    a = _f64(a).reshape(-1, rows * cols)
    t = np.empty_like(a)
    _check(_load().or_page_transpose(rows, cols, a.shape[0], _p(a), _p(t)), "page_transpose")
    return t


def page_mtimes(A, B, m, k, n, transA=False, transB=False, count=None):
    """C_k = op(A_k) op(B_k) (m x k times k x n). A or B with a single page is broadcast.
    Returns (C, (|op A||op B|))."""
    A = _f64(A).reshape(-1, m * k)
    B = _f64(B).reshape(-1, k * n)
    if count is None:
        count = max(A.shape[0], B.shape[0])
    sA = 0 if A.shape[0] == 1 and count != 1 else m * k
    sB = 0 if B.shape[0] == 1 and count != 1 else k * n
    Cm = np.empty((count, m * n))
    absC = np.empty_like(Cm)
    _check(_load().or_page_mtimes(m, k, n, count, _p(A), int(transA), sA, _p(B), int(transB), sB,
                                  _p(Cm), _p(absC)), "page_mtimes")
    return Cm, absC


def page_scale(s, a, rows, cols):
    a = _f64(a).reshape(-1, rows * cols)
    s = _f64(s).reshape(-1)
    c = np.empty_like(a)
    _check(_load().or_page_scale(rows, cols, a.shape[0], _p(s), _p(a), _p(c)), "page_scale")
    return c


def page_bilinear(u, a, v, n):
    a = _f64(a).reshape(-1, n * n)
    u = _f64(u).reshape(-1, n)
    v = _f64(v).reshape(-1, n)
    q = np.empty(a.shape[0])
    _check(_load().or_page_bilinear(n, a.shape[0], _p(u), _p(a), _p(v), _p(q)), "page_bilinear")
    return q


# ----------------------------------------------------------------------------- elements
def p1_elements(coords, elems):
    """Per-element det, vol, grads (dim x nlb col-major), Ke, Me, Kabs, facet measures."""
    coords = _f64(coords)
    elems = _i32(elems)
    nn, dim = coords.shape
    ne, nlb = elems.shape
    assert nlb == dim + 1
    det = np.empty(ne)
    vol = np.empty(ne)
    grads = np.empty((ne, dim * nlb))
    Ke = np.empty((ne, nlb * nlb))
    Me = np.empty((ne, nlb * nlb))
    Ka = np.empty((ne, nlb * nlb))
    fac = np.empty((ne, nlb))
    rc = _load().or_p1_elements(dim, nn, _p(coords), ne, _p(elems), _p(det), _p(vol), _p(grads), _p(Ke),
                                _p(Me), _p(Ka), _p(fac))
    _check(rc, "p1_elements")
    return {"det": det, "vol": vol, "grads": grads, "Ke": Ke, "Me": Me, "Kabs": Ka, "facet": fac,
            "nsingular": int(rc)}


def quad_count(dim, order):
    """Number of integration points of the order-1 / order-2 rule."""
    n = _load().or_quad_count(int(dim), int(order))
    _check(0 if n > 0 else n, "quad_count")
    return n


def quad_points(coords, elems, order):
    """Physical integration points of every element: (ne, nq, dim)."""
    coords = _f64(coords)
    elems = _i32(elems)
    nn, dim = coords.shape
    ne = elems.shape[0]
    nq = quad_count(dim, order)
    xq = np.empty((ne, nq, dim))
    _check(_load().or_quad_points(dim, int(order), nn, _p(coords), ne, _p(elems), _p(xq)), "quad_points")
    return xq


def p1_elements_q(coords, elems, order, cKq=None, cMq=None):
    """Ke, Me (and error scales Kabs, Mabs) with coefficients at the integration points
    (cKq, cMq: (ne, nq) or None for 1)."""
    coords = _f64(coords)
    elems = _i32(elems)
    nn, dim = coords.shape
    ne, nlb = elems.shape
    nq = quad_count(dim, order)
    ck = None if cKq is None else _f64(np.asarray(cKq).reshape(ne, nq))
    cm = None if cMq is None else _f64(np.asarray(cMq).reshape(ne, nq))
    Ke, Me, Ka, Ma = (np.empty((ne, nlb * nlb)) for _ in range(4))
    rc = _load().or_p1_elements_q(dim, int(order), nn, _p(coords), ne, _p(elems), _p(ck), _p(cm), _p(Ke), _p(Me),
                                  _p(Ka), _p(Ma))
    _check(rc, "p1_elements_q")
    return {"Ke": Ke, "Me": Me, "Kabs": Ka, "Mabs": Ma, "nsingular": int(rc)}


def rhs_p1(coords, elems, order, fq):
    """Load vector of the right-hand side listing: local vectors b2D (ne, nlb), the
    accumarray sum b (nn), and its error scale babs (nn).  fq: (ne, nq) values of f at the
    integration points of the rule of `order`."""
    coords = _f64(coords)
    elems = _i32(elems)
    nn, dim = coords.shape
    ne, nlb = elems.shape
    nq = quad_count(dim, order)
    f = _f64(np.asarray(fq).reshape(ne, nq))
    b2D = np.empty((ne, nlb))
    b = np.empty(nn)
    babs = np.empty(nn)
    _check(_load().or_rhs_p1(dim, int(order), nn, _p(coords), ne, _p(elems), _p(f), _p(b2D), _p(b), _p(babs)),
           "rhs_p1")
    return {"b2D": b2D, "b": b, "babs": babs}


def local_energies(coords, elems, order, u, cKq=None, cMq=None, b2D=None):
    """Local energy contributions of the section 3.6 energy functional, as the page
    bilinear form (section 2.2) of the element matrices with the nodal values u_k of each
    element: J1k = 1/2 u_k^T K_k u_k, J2k = 1/2 u_k^T M_k u_k, J3k = -b_k^T u_k (K_k, M_k with
    coefficients at the integration points of the rule of `order`; b_k the local load
    vector b2D, or None for J3k = 0).  Returns J1k, J2k, J3k and their error scales."""
    coords = _f64(coords)
    elems = _i32(elems)
    ne, nlb = elems.shape
    u = _f64(u)
    el = p1_elements_q(coords, elems, order, cKq, cMq)
    ue = u[elems]                        # (ne, nlb): u restricted to each element
    ua = np.abs(ue)
    J1 = 0.5 * page_bilinear(ue, el["Ke"], ue, nlb)
    J2 = 0.5 * page_bilinear(ue, el["Me"], ue, nlb)
    J1abs = 0.5 * page_bilinear(ua, el["Kabs"], ua, nlb)
    J2abs = 0.5 * page_bilinear(ua, el["Mabs"], ua, nlb)
    if b2D is None:
        J3 = np.zeros(ne)
        J3abs = np.zeros(ne)
    else:
        b2 = _f64(np.asarray(b2D).reshape(ne, nlb))
        J3 = -(b2 * ue).sum(axis=1)
        J3abs = (np.abs(b2) * ua).sum(axis=1)
    return {"J1k": J1, "J2k": J2, "J3k": J3, "J1abs": J1abs, "J2abs": J2abs, "J3abs": J3abs}


def faces(coords, elems):
    """All faces by sorting the nlb faces of every element (keys = ascending node ids, ties
    by element): (faces (nf, dim) oriented outward of their first element, fel (nf, 2) with
    e2 = -1 on the boundary), in ascending key order."""
    coords = _f64(coords)
    elems = _i32(elems)
    nn, dim = coords.shape
    ne, nlb = elems.shape
    cap = max(ne * nlb, 1)
    f = np.empty((cap, dim), dtype=np.int32)
    fe = np.empty((cap, 2), dtype=np.int32)
    nf = _load().or_faces(dim, nn, _p(coords), ne, _p(elems), _p(f), _p(fe), cap)
    _check(0 if nf >= 0 else int(nf), "faces")
    return f[:nf].copy(), fe[:nf].copy()


def simplex_points(coords, cells, lam):
    """Points of a rule with barycentric coordinates lam (nq, nv) on every cell: (nc, nq, dim)."""
    coords = _f64(coords)
    cells = _i32(cells)
    lam = _f64(lam)
    nn, dim = coords.shape
    nc, nv = cells.shape
    nq = lam.shape[0]
    X = np.empty((nc, nq, dim))
    _check(_load().or_simplex_points(dim, nv, nn, _p(coords), nc, _p(cells), nq, _p(lam), _p(X)), "simplex_points")
    return X


def gi(fip, w, sizes, normals=None):
    """The GI function: fip (nc, nq) or (nc, nq, d), w (nq) summing to 1, sizes (nc)."""
    fip = _f64(fip)
    nc, nq = fip.shape[0], fip.shape[1]
    d = fip.shape[2] if fip.ndim == 3 else 1
    nrm = None if normals is None else _f64(np.asarray(normals).reshape(nc, d))
    return float(_load().or_gi(nc, nq, d, _p(fip), _p(_f64(w)), _p(_f64(sizes)), _p(nrm)))


def p2_elements(coords, elems2, ruleK, ruleM, cK=None, cM=None):
    """P2 element matrices K3D, M3D (ne, nlb2*nlb2, column-major pages) and their error
    scales, for rules (lam, w) with weights summing to 1 and coefficients (ne, nq) or None."""
    coords = _f64(coords)
    elems2 = _i32(elems2)
    nn, dim = coords.shape
    ne, nlb2 = elems2.shape
    lamK, wK = (_f64(x) for x in ruleK)
    lamM, wM = (_f64(x) for x in ruleM)
    ck = None if cK is None else _f64(np.asarray(cK).reshape(ne, lamK.shape[0]))
    cm = None if cM is None else _f64(np.asarray(cM).reshape(ne, lamM.shape[0]))
    K, M, Ka, Ma = (np.empty((ne, nlb2 * nlb2)) for _ in range(4))
    rc = _load().or_p2_elements(dim, nn, _p(coords), ne, _p(elems2), lamK.shape[0], _p(lamK), _p(wK), _p(ck),
                                lamM.shape[0], _p(lamM), _p(wM), _p(cm), _p(K), _p(M), _p(Ka), _p(Ma))
    _check(rc, "p2_elements")
    return {"K3D": K, "M3D": M, "Kabs": Ka, "Mabs": Ma, "nsingular": int(rc)}


def stroud_rule(d, m):
    """Conical product (collapsed-coordinate) rule on the reference d-simplex (d = 2, 3;
    Stroud, Approximate Calculation of Multiple Integrals, 1971): m Gauss-Jacobi points per
    direction, exact for degree 2m - 1.  Returns (lam (m^d, d+1) barycentric, w summing to 1)."""
    from scipy.special import roots_jacobi
    ax = []
    for k in range(d):  # direction k carries the Jacobian factor (1 - u_k)^(d - 1 - k)
        a = d - 1 - k
        x, wx = roots_jacobi(m, a, 0)
        ax.append(((1 + x) / 2, wx / 2 ** (a + 1)))
    pts, wts = [], []
    for idx in np.ndindex(*([m] * d)):
        u = [ax[k][0][idx[k]] for k in range(d)]
        w = np.prod([ax[k][1][idx[k]] for k in range(d)])
        xi, rest = [], 1.0
        for k in range(d):
            xi.append(u[k] * rest)
            rest *= 1 - u[k]
        pts.append([1 - sum(xi)] + xi)
        wts.append(w)
    w = np.array(wts)
    return np.array(pts), w / w.sum()


def create_coords3d(coords, elems):
    """coords3D (ne, dim*nlb) and vectors3D (ne, dim*(nlb-1)), column-major pages."""
    coords = _f64(coords)
    elems = _i32(elems)
    nn, dim = coords.shape
    ne, nlb = elems.shape
    c3 = np.empty((ne, dim * nlb))
    v3 = np.empty((ne, dim * (nlb - 1)))
    _check(_load().or_create_coords3d(dim, nlb, nn, _p(coords), ne, _p(elems), _p(c3), _p(v3)), "coords3d")
    return c3, v3


def route_predicate(tjac_pages, dim, tau_abs, tau_cond):
    t = _f64(tjac_pages).reshape(-1, dim * dim)
    routed = np.empty(t.shape[0], dtype=np.uint8)
    cond = np.empty(t.shape[0])
    _check(_load().or_route_predicate(dim, _p(t), t.shape[0], float(tau_abs), float(tau_cond), _p(routed),
                                      _p(cond)), "route_predicate")
    return routed.astype(bool), cond


def jacobians(coords, elems):
    """tjac pages (first-node origin, column-major dim x dim): column c holds d x_c / d xi."""
    c3, _ = create_coords3d(coords, elems)
    dim = _f64(coords).shape[1]
    nlb = dim + 1
    ds = np.zeros((dim, nlb))
    ds[:, 0] = -1.0
    ds[np.arange(dim), np.arange(1, nlb)] = 1.0
    # tjac = dshape * coords3D^T  (smamt of the derivative routine)
    Cm, _ = page_mtimes(ds.T.reshape(1, -1), c3, dim, nlb, dim, transA=False, transB=True)
    return Cm


# ----------------------------------------------------------------------------- assembly
def assemble(elems, nn, Ke, Me=None, Kabs=None):
    """sparse() of the listings: CSR (row_ptr, col_idx, valK, valM, scaleK, scaleM)."""
    elems = _i32(elems)
    ne, nlb = elems.shape
    Ke = _f64(Ke)
    Me = None if Me is None else _f64(Me)
    Kabs = None if Kabs is None else _f64(Kabs)
    cap = ne * nlb * nlb
    row_ptr = np.empty(nn + 1, dtype=np.int64)
    col = np.empty(max(cap, 1), dtype=np.int32)
    vk = np.empty(max(cap, 1))
    vm = np.empty(max(cap, 1))
    sk = np.empty(max(cap, 1))
    sm = np.empty(max(cap, 1))
    nnz = _load().or_assemble(nlb, nn, ne, _p(elems), _p(Ke), _p(Me), _p(Kabs), _p(row_ptr), _p(col),
                              _p(vk), _p(vm), _p(sk), _p(sm), cap)
    _check(nnz, "assemble")
    return {"row_ptr": row_ptr, "col_idx": col[:nnz].copy(), "valK": vk[:nnz].copy(),
            "valM": vm[:nnz].copy() if Me is not None else None, "scaleK": sk[:nnz].copy(),
            "scaleM": sm[:nnz].copy() if Me is not None else None, "nnz": int(nnz)}


def assemble_rows(coords, elems, rows, cap=64):
    """Sampled CSR rows computed one by one. Returns list of (cols, valK, valM, scaleK, scaleM)."""
    coords = _f64(coords)
    elems = _i32(elems)
    rows = _i32(rows)
    nn, dim = coords.shape
    ne = elems.shape[0]
    nr = rows.shape[0]
    cols = np.zeros((nr, cap), dtype=np.int32)
    vk = np.zeros((nr, cap))
    vm = np.zeros((nr, cap))
    sk = np.zeros((nr, cap))
    sm = np.zeros((nr, cap))
    ln = np.zeros(nr, dtype=np.int32)
    _check(_load().or_assemble_rows(dim, nn, _p(coords), ne, _p(elems), nr, _p(rows), cap, _p(cols), _p(vk),
                                    _p(vm), _p(sk), _p(sm), _p(ln)), "assemble_rows")
    return [(cols[r, :ln[r]].copy(), vk[r, :ln[r]].copy(), vm[r, :ln[r]].copy(), sk[r, :ln[r]].copy(),
             sm[r, :ln[r]].copy()) for r in range(nr)]


def boundary(coords, faces):
    """Boundary facets: (unit normals, measures, raw normals)."""
    coords = _f64(coords)
    faces = _i32(faces)
    nn, dim = coords.shape
    nf = faces.shape[0]
    unit = np.empty((nf, dim))
    meas = np.empty(nf)
    raw = np.empty((nf, dim))
    _check(_load().or_boundary(dim, nn, _p(coords), nf, _p(faces), _p(unit), _p(meas), _p(raw)), "boundary")
    return unit, meas, raw
