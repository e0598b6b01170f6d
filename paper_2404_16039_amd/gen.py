"""Seeded synthetic inputs: structured jittered simplex meshes and random page batches.

This module only builds inputs (connectivity, coordinates, random matrices, job traces).
It holds none of the method's arithmetic: no determinant, inverse, gradient, element
matrix or assembly is computed here, so both the HIP path and the CPU oracle can take
their inputs from it without sharing any of the computation.

Mesh conventions (0-based int32 connectivity, float64 coordinates, row-major):

* 2-D: unit square cut into n x n squares, each into two counter-clockwise triangles.
  Node id = i + (n+1) j.  Square s = i + n j gives triangles 2s = (v00, v10, v11) and
  2s+1 = (v00, v11, v01).
* 3-D: unit cube cut into n^3 cubes, each into the six Kuhn (Freudenthal) tetrahedra.
  Node id = i + (n+1) j + (n+1)^2 k.  Cube c = i + n j + n^2 k gives tetrahedra 6c+p for
  the permutations p of (0,1,2) in lexicographic order, with vertices v0, v0+e_s1,
  v0+e_s1+e_s2, v0+(1,1,1); the 2nd and 3rd vertex are swapped for odd permutations so
  every tetrahedron is positively oriented before jitter.  The mesh is conforming and its
  counts (6n^3 tetrahedra, (n+1)^3 nodes, 12 n^2 boundary triangles) equal those of the
  paper's uniformly refined meshes (section 3, volume and normal tables, level 6 = 128^3).
* Jitter: every node moves by uniform(-a h, a h) per coordinate, then boundary nodes are
  reset, so the domain is exactly the unit square/cube.

Seeds: stream k of base seed 16039 is numpy's PCG64 seeded with SeedSequence(16039,
spawn_key=(k,)), i.e. SeedSequence(16039).spawn(k+1)[k].
"""
from __future__ import annotations

import itertools
import math

import numpy as np

SEED_BASE = 16039

# named streams (spawn keys) so that every workload draws from its own independent stream
STREAM_SQUARE = 1
STREAM_CUBE = 2
STREAM_PAGES_A = 3
STREAM_PAGES_B = 4
STREAM_PAGES_X = 5
STREAM_SLIVER = 6
STREAM_MIXED = 7
STREAM_SERVE = 8
STREAM_PERM = 9
STREAM_FAN = 10
STREAM_SERVE_PAGES = 11
STREAM_DELAUNAY = 12


def rng(stream: int, sub: int | None = None) -> np.random.Generator:
    """Independent generator for a named stream (and optional sub-stream, e.g. a job id)."""
    key = (int(stream),) if sub is None else (int(stream), int(sub))
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED_BASE, spawn_key=key)))


# --------------------------------------------------------------------------------------
# 2-D square mesh
# --------------------------------------------------------------------------------------
def square_mesh(n: int, jitter: float = 0.2, seed_sub: int | None = None, stream: int = STREAM_SQUARE):
    """Unit square, n x n squares, two triangles each.

    Returns (coords[nn,2] f64, elems[ne,3] i32, bedges[4n,2] i32).  Boundary edges are
    listed counter-clockwise around the domain (outward normal on the right of a->b).
    """
    n = int(n)
    if n < 1:
        raise ValueError("n must be >= 1")
    h = 1.0 / n
    m = n + 1
    I, J = np.meshgrid(np.arange(m), np.arange(m), indexing="xy")  # J rows, I columns
    coords = np.stack([I.ravel() * h, J.ravel() * h], axis=1).astype(np.float64)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    v00 = i + m * j
    v10 = v00 + 1
    v01 = v00 + m
    v11 = v01 + 1
    elems = np.empty((2 * n * n, 3), dtype=np.int32)
    elems[0::2] = np.stack([v00, v10, v11], axis=1)
    elems[1::2] = np.stack([v00, v11, v01], axis=1)
    if jitter:
        g = rng(stream, seed_sub)
        d = g.uniform(-jitter * h, jitter * h, size=coords.shape)
        inner = _interior_mask_grid(m, 2)
        coords[inner] += d[inner]
    # boundary edges, counter-clockwise: bottom (left->right), right (up), top (right->left), left (down)
    b = []
    for ii in range(n):
        b.append((ii, ii + 1))
    for jj in range(n):
        b.append((n + m * jj, n + m * (jj + 1)))
    for ii in range(n, 0, -1):
        b.append((ii + m * n, ii - 1 + m * n))
    for jj in range(n, 0, -1):
        b.append((m * jj, m * (jj - 1)))
    bedges = np.asarray(b, dtype=np.int32)
    return coords, elems, bedges


# --------------------------------------------------------------------------------------
# 3-D Kuhn cube mesh
# --------------------------------------------------------------------------------------
_PERMS = list(itertools.permutations((0, 1, 2)))  # lexicographic


def lshape_mesh(n: int):
    """L-shaped domain of the section 3.6 boundary value problem: the unit square without
    the quarter-open square (0.25, 1) x (0.25, 1), i.e. the union of (0, 0.25)^2,
    (0, 0.25) x (0.25, 1) and (0.25, 1) x (0, 0.25).  A (4n x 4n) grid of squares of side
    h = 1 / (4n) keeps the 7 n^2 squares inside the domain, each cut into two triangles as
    in square_mesh; nodes are renumbered consecutively (x fastest).  No jitter.

    Returns (coords[nn,2] f64, elems[ne,3] i32)."""
    n = int(n)
    if n < 1:
        raise ValueError("n must be >= 1")
    m = 4 * n
    h = 1.0 / m
    i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    keep = (i < n) | (j < n)  # squares left of x = 0.25 or below y = 0.25
    i = i[keep]
    j = j[keep]
    g = m + 1
    v00 = i + g * j
    v10 = v00 + 1
    v01 = v00 + g
    v11 = v01 + 1
    elems = np.empty((2 * i.size, 3), dtype=np.int64)
    elems[0::2] = np.stack([v00, v10, v11], axis=1)
    elems[1::2] = np.stack([v00, v11, v01], axis=1)
    used = np.unique(elems)
    new_id = np.full(g * g, -1, dtype=np.int64)
    new_id[used] = np.arange(used.size)
    coords = np.stack([(used % g) * h, (used // g) * h], axis=1).astype(np.float64)
    return coords, new_id[elems].astype(np.int32)


P2_EDGES = {2: ((0, 1), (0, 2), (1, 2)), 3: ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))}


def p2_mesh(coords: np.ndarray, elems: np.ndarray):
    """P2 mesh of a P1 mesh: one new node at the midpoint of every edge (numbered after the
    vertices, edges in ascending (min, max) order), and per element its vertices followed by
    the mid-edge nodes of its local edges in the order of P2_EDGES.

    Returns (coords2[nn + nedges, dim] f64, elems2[ne, nlb2] i32, nedges)."""
    nn, dim = coords.shape
    ne = elems.shape[0]
    loc = P2_EDGES[dim]
    a = np.stack([elems[:, i] for i, _ in loc], axis=1).astype(np.int64)
    b = np.stack([elems[:, j] for _, j in loc], axis=1).astype(np.int64)
    lo, hi = np.minimum(a, b).ravel(), np.maximum(a, b).ravel()
    key = lo * nn + hi
    uniq, inv = np.unique(key, return_inverse=True)
    ulo, uhi = uniq // nn, uniq % nn
    mid = 0.5 * (coords[ulo] + coords[uhi])
    coords2 = np.concatenate([coords, mid], axis=0)
    elems2 = np.concatenate([elems.astype(np.int64), nn + inv.reshape(ne, len(loc))], axis=1).astype(np.int32)
    return coords2, elems2, uniq.size


def _perm_sign(p):
    s = 1
    p = list(p)
    for a in range(len(p)):
        for b in range(a + 1, len(p)):
            if p[a] > p[b]:
                s = -s
    return s


def _interior_mask_grid(m: int, dim: int) -> np.ndarray:
    idx = np.arange(m)
    inner1 = (idx > 0) & (idx < m - 1)
    if dim == 2:
        J, I = np.meshgrid(inner1, inner1, indexing="ij")
        return (I & J).ravel()
    K, J, I = np.meshgrid(inner1, inner1, inner1, indexing="ij")
    return (I & J & K).ravel()


def cube_mesh(n: int, jitter: float = 0.15, seed_sub: int | None = None, stream: int = STREAM_CUBE,
              with_faces: bool = True):
    """Unit cube, n^3 cubes, six Kuhn tetrahedra each.

    Returns (coords[nn,3] f64, elems[ne,4] i32, faces[12 n^2,3] i32 or None).  Boundary
    triangles are oriented so that (b-a) x (c-a) points out of the cube.
    """
    n = int(n)
    if n < 1:
        raise ValueError("n must be >= 1")
    h = 1.0 / n
    m = n + 1
    K, J, I = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    coords = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1).astype(np.float64) * h
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    v0 = (ii + m * jj + m * m * kk).ravel().astype(np.int64)
    step = np.array([1, m, m * m], dtype=np.int64)
    ne = 6 * n ** 3
    elems = np.empty((ne, 4), dtype=np.int32)
    for p, perm in enumerate(_PERMS):
        a = v0
        b = v0 + step[perm[0]]
        c = b + step[perm[1]]
        d = v0 + step.sum()
        if _perm_sign(perm) < 0:
            b, c = c, b
        elems[p::6, 0] = a
        elems[p::6, 1] = b
        elems[p::6, 2] = c
        elems[p::6, 3] = d
    if jitter:
        g = rng(stream, seed_sub)
        dlt = g.uniform(-jitter * h, jitter * h, size=coords.shape)
        inner = _interior_mask_grid(m, 3)
        coords[inner] += dlt[inner]
    faces = _cube_boundary_faces(n) if with_faces else None
    return coords, elems, faces


def _cube_boundary_faces(n: int) -> np.ndarray:
    """Boundary triangles of the Kuhn mesh, outward oriented.

    Every boundary square of the Kuhn mesh is split along the diagonal from its lowest
    corner (0,0) to (1,1) in its two in-plane axes; the tetrahedra of the mesh carry
    exactly these triangles on the domain boundary.
    """
    m = n + 1
    step = np.array([1, m, m * m], dtype=np.int64)
    out = []
    for axis in range(3):
        u, v = [ax for ax in range(3) if ax != axis]
        a_idx, b_idx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        a_idx = a_idx.ravel()
        b_idx = b_idx.ravel()
        for side in (0, n):
            base = a_idx * step[u] + b_idx * step[v] + side * step[axis]
            p00 = base
            p10 = base + step[u]
            p01 = base + step[v]
            p11 = base + step[u] + step[v]
            # (u, v, axis) right-handed <=> cyclic order; normal of (p00,p10,p11) is +axis
            # when (u, v, axis) is a cyclic permutation of (0, 1, 2)
            cyc = (u, v, axis) in ((0, 1, 2), (1, 2, 0), (2, 0, 1))
            outward_pos = side == n
            keep = cyc == outward_pos
            t1 = np.stack([p00, p10, p11], axis=1) if keep else np.stack([p00, p11, p10], axis=1)
            t2 = np.stack([p00, p11, p01], axis=1) if keep else np.stack([p00, p01, p11], axis=1)
            tri = np.empty((2 * len(base), 3), dtype=np.int64)
            tri[0::2] = t1
            tri[1::2] = t2
            out.append(tri)
    return np.concatenate(out).astype(np.int32)


def append_slivers(coords: np.ndarray, elems: np.ndarray, count: int, h: float,
                   lo: float = 1e-6, hi: float = 1e-3, stream: int = STREAM_SLIVER):
    """Append `count` isolated sliver tetrahedra on new nodes.

    Each sliver has edge lengths ~h and |det J| = t h^3 with t log-uniform in [lo, hi]; it is
    randomly rotated and placed inside the unit cube.  Returns (coords, elems, t) with the
    slivers' element ids ne .. ne+count-1 and their nominal det factors t.
    """
    g = rng(stream)
    t = np.exp(g.uniform(math.log(lo), math.log(hi), size=count))
    base = g.uniform(0.1, 0.9, size=(count, 3))
    q, r = np.linalg.qr(g.standard_normal((count, 3, 3)))
    # make q a proper rotation (det +1)
    s = np.sign(np.einsum("kii->ki", r))
    q = q * s[:, None, :]
    dq = np.linalg.det(q)
    q[dq < 0, :, 0] *= -1.0
    local = np.zeros((count, 4, 3))
    local[:, 1, 0] = h
    local[:, 2, 1] = h
    local[:, 3, 0] = 0.5 * h
    local[:, 3, 1] = 0.5 * h
    local[:, 3, 2] = t * h
    pts = base[:, None, :] + np.einsum("kij,kpj->kpi", q, local)
    nn0 = coords.shape[0]
    new_coords = np.concatenate([coords, pts.reshape(-1, 3)], axis=0)
    new_elems = np.concatenate(
        [elems, (nn0 + np.arange(4 * count, dtype=np.int64)).reshape(count, 4).astype(np.int32)], axis=0)
    return new_coords, new_elems, t


def fan_mesh(dim: int, k: int, seed_sub: int = 0, stream: int = STREAM_FAN):
    """A closed fan of k simplices around one hub, i.e. a node in k elements (high valence).

    2-D: hub at the origin, k rim nodes on a jittered circle, triangles (hub, r_i, r_i+1).
    3-D: an axis edge (a, b) at z = -1 and z = +1 with k rim nodes on a jittered circle in the
    plane z = 0, tetrahedra (a, b, r_i, r_i+1): both axis nodes lie in k elements and their
    rows hold k + 2 nonzeros.  Rim angles are jittered by up to a quarter of the spacing and
    radii by up to 20%, from the seeded stream.  Returns (coords, elems).
    """
    g = rng(stream, seed_sub)
    ang = 2.0 * math.pi * (np.arange(k) + g.uniform(-0.25, 0.25, k)) / k
    rad = 1.0 + g.uniform(-0.2, 0.2, k)
    rim = np.stack([rad * np.cos(ang), rad * np.sin(ang)], axis=1)
    nxt = (np.arange(k) + 1) % k
    if dim == 2:
        coords = np.concatenate([[[0.0, 0.0]], rim])
        elems = np.stack([np.zeros(k, np.int64), 1 + np.arange(k), 1 + nxt], axis=1)
    else:
        axis = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, 1.0]]) + g.uniform(-0.1, 0.1, (2, 3)) * [1, 1, 0]
        coords = np.concatenate([axis, np.concatenate([rim, np.zeros((k, 1))], axis=1)])
        elems = np.stack([np.zeros(k, np.int64), np.ones(k, np.int64), 2 + np.arange(k), 2 + nxt], axis=1)
    return coords.astype(np.float64), elems.astype(np.int32)


def join_meshes(*meshes):
    """Disjoint union of (coords, elems) meshes: node ids of each later mesh shifted."""
    cs, es, off = [], [], 0
    for c, e in meshes:
        cs.append(np.asarray(c, np.float64))
        es.append(np.asarray(e, np.int64) + off)
        off += c.shape[0]
    return np.concatenate(cs), np.concatenate(es).astype(np.int32)


def permute_nodes(coords: np.ndarray, elems: np.ndarray, faces=None, stream: int = STREAM_PERM):
    """Random relabelling of the nodes (numbering with no structure).

    Returns (coords', elems', faces', perm) with coords'[perm[i]] = coords[i].
    """
    g = rng(stream)
    nn = coords.shape[0]
    perm = g.permutation(nn).astype(np.int64)
    c2 = np.empty_like(coords)
    c2[perm] = coords
    e2 = perm[elems].astype(np.int32)
    f2 = None if faces is None else perm[faces].astype(np.int32)
    return c2, e2, f2, perm


def _morton_code(q: np.ndarray) -> np.ndarray:
    """Z-order key of integer grid coordinates q (npts, dim), 21 bits per axis."""
    def spread(v, dim):
        v = v.astype(np.uint64) & np.uint64((1 << 21) - 1)
        out = np.zeros_like(v)
        for b in range(21):
            out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(dim * b)
        return out
    dim = q.shape[1]
    code = np.zeros(q.shape[0], dtype=np.uint64)
    for a in range(dim):
        code |= spread(q[:, a], dim) << np.uint64(a)
    return code


def delaunay_mesh(npts: int, dim: int = 3, stream: int = STREAM_DELAUNAY, sub: int | None = None):
    """Unstructured mesh: the Delaunay triangulation (scipy's Qhull) of npts uniform random
    points in the unit square/cube.  Nodes are numbered along a Z-order curve of the points
    and elements sorted by their smallest node, the locality a mesh generator's reordering
    gives; elements keep Qhull's vertex order, so both orientations occur.  About 6.7 tets
    (3-D) or 2 triangles (2-D) per point.  Returns (coords, elems)."""
    from scipy.spatial import Delaunay

    pts = rng(stream, sub).random((npts, dim))
    code = _morton_code(np.minimum((pts * (1 << 21)).astype(np.int64), (1 << 21) - 1))
    order = np.argsort(code, kind="stable")
    coords = np.ascontiguousarray(pts[order])
    elems = Delaunay(coords).simplices.astype(np.int32)
    elems = elems[np.argsort(elems.min(axis=1), kind="stable")]
    return coords, np.ascontiguousarray(elems)


# --------------------------------------------------------------------------------------
# page batches
# --------------------------------------------------------------------------------------
def page_batch(count: int, n: int, stream: int = STREAM_PAGES_A, shift: float = 3.0,
               layout: str = "pages", sub: int | None = None) -> np.ndarray:
    """`count` random n x n float64 matrices with N(0,1) entries plus shift * I.

    layout "pages": array[count, n, n] holding each page column-major (MATLAB order,
    element (r, c) of page k at flat offset k n^2 + r + c n); returned as shape
    (count, n*n) flat pages.
    layout "soa": array[n*n, count], component (r + c n) of every page contiguous.
    """
    g = rng(stream, sub)
    a = g.standard_normal((count, n, n))
    a += shift * np.eye(n)[None, :, :]
    # a[k, r, c]; column-major flat index r + c n -> transpose to [k, c, r]
    flat = np.ascontiguousarray(np.transpose(a, (0, 2, 1)).reshape(count, n * n))
    if layout == "pages":
        return flat
    if layout == "soa":
        return np.ascontiguousarray(flat.T)
    raise ValueError(layout)


def vector_batch(count: int, n: int, stream: int = STREAM_PAGES_X, sub: int | None = None) -> np.ndarray:
    """`count` random n-vectors with N(0,1) entries, shape (count, n)."""
    return rng(stream, sub).standard_normal((count, n))


def mixed_groups(ngroups: int = 64, lo: float = 1e3, hi: float = 1e6, stream: int = STREAM_MIXED):
    """Uneven mixed-order batch: (order, size) per group, order uniform in {2,3,4},
    size = round(10^U(log10 lo, log10 hi))."""
    g = rng(stream)
    orders = g.integers(2, 5, size=ngroups)
    sizes = np.rint(10.0 ** g.uniform(math.log10(lo), math.log10(hi), size=ngroups)).astype(np.int64)
    return [(int(o), int(s)) for o, s in zip(orders, sizes)]


def serving_trace(njobs: int, rate: float = 200.0, lo: float = 1e3, hi: float = 2e6,
                  stream: int = STREAM_SERVE):
    """Poisson arrivals: list of dicts {t, dim, n, target} with inter-arrival Exp(1/rate),
    dim uniform in {2,3}, target element count log-uniform in [lo, hi], and the mesh
    parameter n chosen so that the structured mesh has about `target` elements."""
    g = rng(stream)
    gaps = g.exponential(1.0 / rate, size=njobs)
    t = np.cumsum(gaps) - gaps[0]
    dims = g.integers(2, 4, size=njobs)
    tgt = 10.0 ** g.uniform(math.log10(lo), math.log10(hi), size=njobs)
    jobs = []
    for k in range(njobs):
        d = int(dims[k])
        if d == 2:
            n = max(1, int(round(math.sqrt(tgt[k] / 2.0))))
        else:
            n = max(1, int(round((tgt[k] / 6.0) ** (1.0 / 3.0))))
        jobs.append({"id": k, "t": float(t[k]), "dim": d, "n": n, "target": float(tgt[k])})
    return jobs


def jittered_coords(base: np.ndarray, n: int, dim: int, seed_sub: int, stream: int = STREAM_SERVE,
                    jitter: float | None = None) -> np.ndarray:
    """The coordinates square_mesh / cube_mesh(n, seed_sub=seed_sub, stream=stream) return,
    from the same mesh's unjittered coordinates `base` (jitter 0.2 h in 2-D, 0.15 h in 3-D
    unless given): the same draws, so serving traces can keep one connectivity per size."""
    if jitter is None:
        jitter = 0.2 if dim == 2 else 0.15
    h = 1.0 / n
    g = rng(stream, seed_sub)
    d = g.uniform(-jitter * h, jitter * h, size=base.shape)
    inner = _interior_mask_grid(n + 1, dim)
    c = base.copy()
    c[inner] += d[inner]
    return c


def serving_page_jobs(njobs: int, frac: float = 0.25, lo: float = 1e3, hi: float = 1e6,
                      stream: int = STREAM_SERVE_PAGES):
    """Which jobs of a serving trace are page-op jobs, and their shape: a list with None for
    an assembly job, else {order, count, prec} (order uniform in {2,3,4}, count log-uniform in
    [lo, hi], FP32 or FP64 with p = 1/2) for a page-op job (probability `frac`)."""
    g = rng(stream)
    is_page = g.random(njobs) < frac
    order = g.integers(2, 5, size=njobs)
    count = np.round(10.0 ** g.uniform(math.log10(lo), math.log10(hi), size=njobs)).astype(np.int64)
    prec = g.integers(0, 2, size=njobs)
    return [{"order": int(order[k]), "count": int(count[k]), "prec": int(prec[k])} if is_page[k] else None
            for k in range(njobs)]


def kuhn_counts(n: int) -> dict:
    """Closed-form counts of the Kuhn n^3 mesh: tetrahedra, nodes, edges, CSR nonzeros
    (nodes + 2 edges), boundary triangles and all triangles."""
    tets = 6 * n ** 3
    nodes = (n + 1) ** 3
    edges = 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3
    fb = 12 * n * n
    return {"tets": tets, "nodes": nodes, "edges": edges, "nnz": nodes + 2 * edges,
            "bfaces": fb, "faces": (4 * tets + fb) // 2}


def square_counts(n: int) -> dict:
    """Closed-form counts of the two-triangle n x n mesh."""
    tris = 2 * n * n
    nodes = (n + 1) ** 2
    edges = 2 * n * (n + 1) + n * n
    return {"tris": tris, "nodes": nodes, "edges": edges, "nnz": nodes + 2 * edges, "bedges": 4 * n}
