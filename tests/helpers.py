"""Shared helpers of the GPU parity tests (input marshalling and tolerance checks)."""
import functools
import sys

import numpy as np
import torch

from paper_2404_16039_amd import gen

# tolerances of the two paths: relative to the natural error scale of each result
TOL = {torch.float64: 1e-12, torch.float32: 1e-5}
F64, F32 = 1, 0


def prec_of(dtype):
    return F64 if dtype == torch.float64 else F32


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu").numpy()


def counters():
    return torch.zeros(4, dtype=torch.int64, device="cuda")


def say(*a):
    """Name the case before each GPU step (so a failing run says what it was doing)."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def within(got, ref, scale, tol, what):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    err = np.abs(got - ref)
    bound = tol * scale
    bad = ~(err <= bound)
    if bad.any():
        i = np.flatnonzero(bad.ravel())[:5]
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} outside tol {tol}: got {got.ravel()[i]} "
                             f"ref {ref.ravel()[i]} scale {scale.ravel()[i]} max rel "
                             f"{np.max(err / np.maximum(scale, 1e-300)):.3e}")
    return float(np.max(err / np.maximum(scale, 1e-300))) if err.size else 0.0


@functools.lru_cache(maxsize=4)
def cube(n, jitter=0.15):
    return gen.cube_mesh(n, jitter=jitter)


@functools.lru_cache(maxsize=4)
def square(n, jitter=0.2):
    return gen.square_mesh(n, jitter=jitter)


def flip_half(elems, seed=7):
    """The mesh with half its elements (seeded choice) given local nodes 1 and 2 swapped:
    det J < 0 for those (the generators orient every element positively)."""
    flip = np.random.default_rng(seed).random(len(elems)) < 0.5
    e = np.array(elems, copy=True)
    e[flip, 1], e[flip, 2] = elems[flip, 2], elems[flip, 1]
    return e


def kuhn_pattern(n):
    """CSR pattern of the Kuhn cube mesh of n^3 cubes, from its closed form (no elements):
    node v and v + d are joined by an edge iff d or -d is a nonzero 0/1 vector and both
    nodes lie in the grid (two vertices of a Kuhn tetrahedron differ by such a vector, and
    any such pair lies on a monotone path through one cube).  Node id = i + s j + s^2 k with
    s = n + 1, so the columns of a row are the row plus the valid offsets in ascending order."""
    s = n + 1
    vecs = [(dx, dy, dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]  # includes 0 = diagonal
    offs = []
    for d in vecs:
        offs.append(d)
        if any(d):
            offs.append(tuple(-c for c in d))
    offs.sort(key=lambda d: d[0] + s * d[1] + s * s * d[2])
    i, j, k = np.meshgrid(np.arange(s), np.arange(s), np.arange(s), indexing="ij")
    i, j, k = (a.transpose(2, 1, 0).ravel() for a in (i, j, k))  # node order: i fastest
    node = i + s * j + s * s * k
    cols = np.full((node.size, len(offs)), -1, np.int64)
    for q, (dx, dy, dz) in enumerate(offs):
        ok = (i + dx >= 0) & (i + dx <= n) & (j + dy >= 0) & (j + dy <= n) & (k + dz >= 0) & (k + dz <= n)
        cols[ok, q] = node[ok] + dx + s * dy + s * s * dz
    valid = cols >= 0
    row_ptr = np.concatenate([[0], np.cumsum(valid.sum(axis=1))]).astype(np.int64)
    return row_ptr, cols[valid].astype(np.int32)


def pair_pattern(elems, nn, chunk=1 << 22):
    """CSR pattern of sparse() on any mesh: every ordered pair of nodes that share an element
    (diagonal included), by sorting the pairs (np.unique), in element chunks to bound memory."""
    elems = np.asarray(elems, np.int64)
    keys = []
    for e0 in range(0, elems.shape[0], chunk):
        e = elems[e0:e0 + chunk]
        k = (e[:, :, None] * nn + e[:, None, :]).ravel()
        keys.append(np.unique(k))
    k = np.unique(np.concatenate(keys)) if len(keys) > 1 else (keys[0] if keys else np.zeros(0, np.int64))
    rows = k // nn
    row_ptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=nn))]).astype(np.int64)
    return row_ptr, (k % nn).astype(np.int32)
