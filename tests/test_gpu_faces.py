"""Parity of the face lists (section 3.2, normals of all faces or of boundary faces) against
the oracle's sorted face keys, the 128^3 counts of the section 3.2 normals table, and the
GI function (section 3.4) with integration points: the divergence theorem by a volume and
a surface integral, against the oracle's GI."""
import os

import numpy as np
import pytest
import torch

import oracle
from helpers import TOL, cube, dev, flip_half, host, say, square
from paper_2404_16039_amd import gen

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def lib():
    from paper_2404_16039_amd import lib as L
    return L


def _gpu_faces(L, coords, elems):
    dim = coords.shape[1]
    te = dev(elems)
    csr = L.Csr().symbolic(dim, coords.shape[0], te)
    csr.faces(dev(coords), te)
    f, fe, bf, be = (host(t) for t in csr.face_lists())
    csr.close()
    return f, fe, bf, be


@pytest.mark.parametrize("mesh", ["cube1", "cube2", "cube5", "square6", "cube4_perm", "square5_perm", "cube4_flip",
                                  "square5_flip"])
def test_faces_match_oracle(lib, mesh):
    """_perm: a random node numbering; _flip: half the elements with two local nodes swapped
    (det J < 0), so the faces' node order follows the element's orientation."""
    say("faces", mesh)
    base, perm = mesh.split("_")[0], mesh.endswith("_perm")
    coords, elems, _ = cube(int(base[4:])) if base.startswith("cube") else square(int(base[6:]))
    if perm:
        coords, elems, _, _ = gen.permute_nodes(coords, elems)
    if mesh.endswith("_flip"):
        elems = flip_half(elems)
    f, fe, bf, be = _gpu_faces(lib, coords, elems)
    F, FE = oracle.faces(coords, elems)
    assert np.array_equal(f, F) and np.array_equal(fe, FE)
    b = FE[:, 1] < 0
    assert np.array_equal(bf, F[b]) and np.array_equal(be, FE[b, 0])


def test_faces_full_size_counts_and_orientation(lib):
    """128^3 Kuhn cube: the counts of the section 3.2 normals table at level 6 (25,264,128
    faces, 196,608 boundary faces), boundary faces = the generator's, outward (sum of
    area n = 0, flux of x = 3)."""
    say("faces 128^3")
    gold = {}
    with open(os.path.join(GOLD, "sphere_levels.txt")) as fh:
        for line in fh:
            p = line.split()
            if p and not p[0].startswith("#"):
                gold[int(p[0])] = (int(p[3]), int(p[4]))
    coords, elems, bfaces = gen.cube_mesh(128, jitter=0.15)
    tc, te = dev(coords), dev(elems)
    csr = lib.Csr().symbolic(3, coords.shape[0], te)
    csr.faces(tc, te)
    f, fe, bf, be = csr.face_lists()
    assert (f.shape[0], bf.shape[0]) == gold[6]
    fe_h = host(fe)
    assert int((fe_h[:, 1] < 0).sum()) == gold[6][1]
    assert np.all(fe_h[:, 0] < np.where(fe_h[:, 1] < 0, np.iinfo(np.int32).max, fe_h[:, 1]))
    got = np.sort(host(bf), axis=1)
    want = np.sort(bfaces, axis=1)
    order = np.lexsort(want.T[::-1])
    assert np.array_equal(got, want[order])
    unit = torch.empty(bf.shape[0] * 3, dtype=torch.float64, device="cuda")
    area = torch.empty(bf.shape[0], dtype=torch.float64, device="cuda")
    lib.boundary_normals(lib.F64, tc, bf.contiguous(), unit=unit, measure=area)
    u, a = host(unit).reshape(-1, 3), host(area)
    assert np.allclose((u * a[:, None]).sum(axis=0), 0.0, atol=1e-10)
    cent = coords[host(bf)].mean(axis=1)
    assert abs((cent * u * a[:, None]).sum() - 3.0) < 1e-10
    csr.close()


def _stroud(d, m):
    lam, w = oracle.stroud_rule(d, m)
    return lam, w


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_gi_divergence_theorem(lib, dtype):
    """Volume integral of div F and flux of F through the boundary faces with rules exact
    for their degrees (GPU points, volumes, boundary normals and GI) both give 8/15, and
    each GI equals the oracle's GI of the same values."""
    say("GI", dtype)
    coords, elems, _ = cube(6)
    tc, te = dev(coords), dev(elems)
    lam3, w3 = _stroud(3, 3)
    lam2, w2 = _stroud(2, 3)
    X = lib.simplex_points(tc, te, lam3)
    Xo = oracle.simplex_points(coords, elems, lam3)
    assert np.allclose(host(X), Xo, rtol=0, atol=1e-15)
    ne = elems.shape[0]
    vol = torch.empty(ne, dtype=dtype, device="cuda")
    lib.elem_geometry(lib.F64 if dtype == torch.float64 else lib.F32, tc, te, vol=vol)
    div = ((X[..., 0] ** 2 + X[..., 1] ** 2) * (X[..., 1] ** 2 + X[..., 2] ** 2)).to(dtype).contiguous()
    p = lib.F64 if dtype == torch.float64 else lib.F32
    v = host(lib.gi(p, div, w3, vol))[0]
    ref = oracle.gi(host(div), w3, host(vol))
    scale = oracle.gi(np.abs(host(div)), w3, np.abs(host(vol)))
    assert abs(v - ref) <= 1e-12 * scale
    tol = 1e-12 if dtype == torch.float64 else TOL[dtype]
    assert abs(v - 8 / 15) <= tol * scale, v
    csr = lib.Csr().symbolic(3, coords.shape[0], te)
    csr.faces(tc, te)
    _, _, bf, _ = csr.face_lists()
    bf = bf.contiguous()
    Y = lib.simplex_points(tc, bf, lam2)
    unit = torch.empty(bf.shape[0] * 3, dtype=dtype, device="cuda")
    area = torch.empty(bf.shape[0], dtype=dtype, device="cuda")
    lib.boundary_normals(p, tc, bf, unit=unit, measure=area)
    Fv = torch.stack([Y[..., 0] ** 3 * (Y[..., 1] ** 2 + Y[..., 2] ** 2) / 3, Y[..., 1] ** 5 / 5,
                      Y[..., 1] ** 2 * Y[..., 2] ** 3 / 3], dim=2).to(dtype).contiguous()
    s = host(lib.gi(p, Fv, w2, area, normals=unit))[0]
    ref = oracle.gi(host(Fv), w2, host(area), host(unit).reshape(-1, 3))
    scale = oracle.gi(np.abs(host(Fv)), w2, np.abs(host(area)), np.abs(host(unit)).reshape(-1, 3))
    assert abs(s - ref) <= 1e-12 * scale
    assert abs(s - 8 / 15) <= tol * scale, s
    csr.close()


def test_gi_deterministic_and_edge_cases(lib):
    say("GI edge cases")
    rng = np.random.default_rng(16039)
    fip = dev(rng.random((100000, 4)))
    sizes = dev(rng.random(100000))
    w = np.full(4, 0.25)
    a = host(lib.gi(lib.F64, fip, w, sizes))[0]
    b = host(lib.gi(lib.F64, fip, w, sizes))[0]
    assert a == b
    assert abs(a - (host(fip).mean(axis=1) * host(sizes)).sum()) < 1e-9
    z = lib.gi(lib.F64, fip[:0], w, sizes[:0])
    assert host(z)[0] == 0.0
    with pytest.raises(lib.PagefemError):
        lib.gi(lib.F64, torch.zeros(4, 65, dtype=torch.float64, device="cuda"), np.ones(65) / 65,
               torch.ones(4, dtype=torch.float64, device="cuda"))
    csr = lib.Csr()
    with pytest.raises(lib.PagefemError):
        csr.faces(None, None)
    coords, elems, _ = cube(2)
    csr.symbolic(3, coords.shape[0], dev(elems))
    with pytest.raises(lib.PagefemError):
        csr.face_lists()
    csr.close()


@pytest.mark.parametrize("case", ["tet27", "tet1", "tet64", "tri9", "edge3"])
def test_simplex_points_parity(lib, case):
    """Points of caller-given rules on every cell (section 3.5: the coordinates combined with
    the rule's barycentric points) against the oracle: tetrahedra with 27, 1 and 64 points,
    triangles, and boundary edges, over several blocks of cells with a ragged last one."""
    say("simplex points", case)
    if case.startswith("tet"):
        coords, cells, _ = cube(6)
        nq = int(case[3:])
        lam = np.full((1, 4), 0.25) if nq == 1 else _stroud(3, 3 if nq == 27 else 4)[0]
    elif case == "tri9":
        coords, cells, _ = square(40)
        lam = _stroud(2, 3)[0]
    else:
        coords, _, cells = square(40)  # the boundary edges
        g, _ = np.polynomial.legendre.leggauss(3)
        t = (g + 1) / 2
        lam = np.stack([1 - t, t], axis=1)
    X = host(lib.simplex_points(dev(coords), dev(cells), lam))
    Xo = oracle.simplex_points(coords, cells, lam)
    assert X.shape == Xo.shape == (cells.shape[0], lam.shape[0], coords.shape[1])
    assert np.allclose(X, Xo, rtol=0, atol=4e-16 * np.abs(coords).max() * 4), np.abs(X - Xo).max()


def test_simplex_points_bad_node(lib):
    """A cell with a node index out of range gets NaN points; every other cell is unaffected."""
    say("simplex points bad node")
    coords, cells, _ = cube(6)
    lam = _stroud(3, 3)[0]
    bad = cells.copy()
    bad[700, 2] = coords.shape[0] + 3
    X = host(lib.simplex_points(dev(coords), dev(bad), lam))
    Xo = oracle.simplex_points(coords, cells, lam)
    assert np.all(np.isnan(X[700]))
    keep = np.ones(cells.shape[0], dtype=bool)
    keep[700] = False
    assert np.allclose(X[keep], Xo[keep], rtol=0, atol=4e-15)
