"""Parity of the load vector (section 3.6 right-hand side listing with its accumarray step)
and of the local energy parts against the oracle, closed forms at full size, and the
boundary value problem of section 3.6 on the L-shaped domain against the printed energies."""
import math
import os

import numpy as np
import pytest
import torch

import oracle
from helpers import TOL, counters, cube, dev, flip_half, host, prec_of, say, square, within
from paper_2404_16039_amd import gen

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def lib():
    from paper_2404_16039_amd import lib as L
    return L


def _fields(xq, dim):
    """smooth coefficient and source fields at the points: f changes sign, c > 0"""
    s = xq.sum(axis=-1)
    f = np.sin(3.0 * s) + 0.5 * xq[..., 0]
    cK = np.exp(s)
    cM = 1.0 + xq[..., -1] ** 2
    return f, cK, cM


def _gpu_rhs_energies(L, coords, elems, dtype, order, fq, cKq, cMq, u, csr=None):
    dim = coords.shape[1]
    ne, nlb = elems.shape
    tc, te = dev(coords), dev(elems)
    csr = csr or L.Csr()
    csr.symbolic(dim, coords.shape[0], te)
    p = prec_of(dtype)
    b2D = torch.empty(ne * nlb, dtype=dtype, device="cuda")
    b = torch.empty(coords.shape[0], dtype=dtype, device="cuda")
    ctr = counters()
    csr.rhs(p, tc, te, order, dev(fq, dtype), b2D, b, counters=ctr)
    J = torch.empty(3 * ne, dtype=dtype, device="cuda")
    tot = torch.zeros(3, dtype=torch.float64, device="cuda")
    csr.energies(p, tc, te, order, dev(u, dtype), cKq=dev(cKq, dtype), cMq=dev(cMq, dtype), b2D=b2D, J=J,
                 totals=tot, counters=ctr)
    return {"b2D": host(b2D).reshape(ne, nlb), "b": host(b), "J": host(J).reshape(3, ne), "tot": host(tot),
            "ctr": host(ctr), "csr": csr, "tb": b}


def _rounded(x, dtype):
    return np.asarray(x, dtype=np.float64).astype(np.float32 if dtype == torch.float32 else np.float64).astype(
        np.float64)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dim,order", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_rhs_and_energies_parity(lib, dtype, dim, order):
    say("rhs/energies", dim, order, dtype)
    coords, elems, _ = square(13) if dim == 2 else cube(7)
    xq = oracle.quad_points(coords, elems, order)
    f, cK, cM = (_rounded(v, dtype) for v in _fields(xq, dim))
    u = _rounded(np.cos(2.0 * coords[:, 0]) + coords[:, 1] ** 2 - 0.3 * coords[:, -1], dtype)
    got = _gpu_rhs_energies(lib, coords, elems, dtype, order, f, cK, cM, u)
    tol = TOL[dtype]
    r = oracle.rhs_p1(coords, elems, order, f)
    rabs = oracle.rhs_p1(coords, elems, order, np.abs(f))
    within(got["b2D"], r["b2D"], rabs["b2D"], tol, "b2D")
    within(got["b"], r["b"], r["babs"], tol, "b")
    J = oracle.local_energies(coords, elems, order, u, cKq=cK, cMq=cM, b2D=_rounded(got["b2D"], dtype))
    for c, k in enumerate(("J1", "J2", "J3")):
        within(got["J"][c], J[k + "k"], J[k + "abs"], tol, k)
        # totals: FP64 sums of the stored values
        want = got["J"][c].astype(np.float64).sum()
        assert abs(got["tot"][c] - want) <= 1e-12 * np.abs(got["J"][c]).sum() + 1e-300, (k, got["tot"][c], want)
    assert got["ctr"][2] == 0


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_rhs_and_energies_negatively_oriented(lib, dtype):
    """Half the tetrahedra with det J < 0: local vectors, node sums and the energy parts
    against the oracle."""
    say("rhs/energies flipped", dtype)
    coords, elems, _ = cube(5)
    elems = flip_half(elems)
    xq = oracle.quad_points(coords, elems, 2)
    f, cK, cM = (_rounded(v, dtype) for v in _fields(xq, 3))
    u = _rounded(np.cos(2.0 * coords[:, 0]) + coords[:, 1] ** 2 - 0.3 * coords[:, -1], dtype)
    got = _gpu_rhs_energies(lib, coords, elems, dtype, 2, f, cK, cM, u)
    tol = TOL[dtype]
    r = oracle.rhs_p1(coords, elems, 2, f)
    rabs = oracle.rhs_p1(coords, elems, 2, np.abs(f))
    within(got["b2D"], r["b2D"], rabs["b2D"], tol, "b2D")
    within(got["b"], r["b"], r["babs"], tol, "b")
    J = oracle.local_energies(coords, elems, 2, u, cKq=cK, cMq=cM, b2D=_rounded(got["b2D"], dtype))
    for c, k in enumerate(("J1", "J2", "J3")):
        within(got["J"][c], J[k + "k"], J[k + "abs"], tol, k)


def test_rhs_deterministic_across_adjacency_orders(lib):
    """b is summed exactly, so rebuilding the structure (which may order the adjacency lists
    differently) and a node renumbering give the same bits."""
    say("rhs determinism")
    coords, elems, _ = cube(9)
    xq = oracle.quad_points(coords, elems, 2)
    f = _rounded(_fields(xq, 3)[0], torch.float32)
    u = np.zeros(coords.shape[0])
    a = _gpu_rhs_energies(lib, coords, elems, torch.float32, 2, f, f, f, u)
    b = _gpu_rhs_energies(lib, coords, elems, torch.float32, 2, f, f, f, u, csr=a["csr"])
    assert np.array_equal(a["b"], b["b"]) and np.array_equal(a["b2D"], b["b2D"])
    pc, pe, _, perm = gen.permute_nodes(coords, elems)  # pc[perm[i]] = coords[i]
    p = _gpu_rhs_energies(lib, pc, pe, torch.float32, 2, f, f, f, np.zeros(pc.shape[0]))
    assert np.array_equal(p["b"][perm], a["b"])


def test_edge_cases(lib):
    say("rhs edge cases")
    # single element, isolated node, nodes of no element get b = 0
    coords = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [5, 5, 5]], dtype=np.float64)
    elems = np.array([[0, 1, 2, 3]], dtype=np.int32)
    fq = np.ones((1, 4))
    got = _gpu_rhs_energies(lib, coords, elems, torch.float64, 2, fq, fq, fq, np.arange(5.0))
    assert np.allclose(got["b"], [1 / 24, 1 / 24, 1 / 24, 1 / 24, 0.0], rtol=1e-15, atol=0)
    assert got["b"][4] == 0.0
    # J1 = 1/2 |grad u|^2 |T| with u = x + 2y + 3z on nodes 0..3
    assert abs(got["J"][0][0] - 0.5 * 14 / 6) < 1e-14
    # errors: unbuilt handle, bad order
    csr = lib.Csr()
    b2D = torch.empty(4, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.PagefemError):
        csr.rhs(lib.F64, dev(coords), dev(elems), 2, dev(fq), b2D)
    csr.symbolic(3, 5, dev(elems))
    with pytest.raises(lib.PagefemError):
        csr.rhs(lib.F64, dev(coords), dev(elems), 3, dev(fq), b2D)
    with pytest.raises(lib.PagefemError):
        csr.energies(lib.F64, dev(coords), dev(elems), 2, None)


def test_full_size_fp32_closed_forms(lib):
    """128^3 Kuhn cube, FP32, u linear, unit coefficients, f = 1: the totals equal the closed
    forms 1/2 |g|^2, 1/2 int u^2 and -int u over the unit cube, b sums to 1, and sampled
    nodes of b match the oracle's element sums."""
    say("energies 128^3")
    n = 128
    coords, elems, _ = gen.cube_mesh(n, jitter=0.15, with_faces=False)
    ne, nq = elems.shape[0], 4
    g = np.array([0.8, -1.1, 0.5])
    c = 0.25
    u = coords @ g + c
    ones = np.ones((ne, nq), dtype=np.float32)
    L = lib
    tc, te = dev(coords), dev(elems)
    csr = L.Csr().symbolic(3, coords.shape[0], te)
    b2D = torch.empty(ne * 4, dtype=torch.float32, device="cuda")
    b = torch.empty(coords.shape[0], dtype=torch.float32, device="cuda")
    tf = dev(ones, torch.float32)
    csr.rhs(L.F32, tc, te, 2, tf, b2D, b)
    tot = torch.zeros(3, dtype=torch.float64, device="cuda")
    csr.energies(L.F32, tc, te, 2, dev(u, torch.float32), cKq=tf, cMq=tf, b2D=b2D, totals=tot)
    tot = host(tot)
    want1 = 0.5 * g @ g
    s = g.sum()
    want2 = 0.5 * (c * c + c * s + (g @ g) / 3 + (s * s - g @ g) / 4)
    want3 = -(c + s / 2)
    assert abs(tot[0] - want1) < 1e-5 * want1, (tot[0], want1)
    assert abs(tot[1] - want2) < 1e-5 * want2, (tot[1], want2)
    assert abs(tot[2] - want3) < 1e-5 * abs(want3), (tot[2], want3)
    hb = host(b).astype(np.float64)
    assert abs(hb.sum() - 1.0) < 1e-5
    ref = oracle.rhs_p1(coords, elems, 2, ones)
    rows = np.random.default_rng(7).choice(coords.shape[0], 4096, replace=False)
    within(hb[rows], ref["b"][rows], ref["babs"][rows], TOL[torch.float32], "b sampled")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_bvp_energies_lshape(lib, dtype):
    """The section 3.6 boundary value problem on the L-shaped domain: the GPU's energy parts
    of the interpolant of u equal the oracle's, and converge to the printed values."""
    say("BVP", dtype)
    pi = math.pi
    pr = {}
    with open(os.path.join(GOLD, "energies_bvp.txt")) as fh:
        for line in fh:
            p = line.split()
            if p and p[0] == "printed":
                pr[p[1]] = float(p[2])
    errs = []
    for n in (8, 16, 32):
        coords, elems = gen.lshape_mesh(n)
        xq = oracle.quad_points(coords, elems, 2)
        x1, x2 = xq[..., 0], xq[..., 1]
        f = (8 * pi * x1 * np.sin(4 * pi * x1) * np.cos(4 * pi * x2) + np.cos(4 * pi * x1) *
             (-4 * pi * np.sin(4 * pi * x2) + (1 - x1 + 32 * pi ** 2 * (1 + x1 ** 2 - x2) + x2 ** 2) *
              np.cos(4 * pi * x2)))
        cK = 1 + x1 ** 2 - x2
        cM = 1 - x1 + x2 ** 2
        u = np.cos(4 * pi * coords[:, 0]) * np.cos(4 * pi * coords[:, 1])
        f, cK, cM, u = (_rounded(v, dtype) for v in (f, cK, cM, u))
        got = _gpu_rhs_energies(lib, coords, elems, dtype, 2, f, cK, cM, u)
        ref = oracle.local_energies(coords, elems, 2, u, cKq=cK, cMq=cM,
                                    b2D=oracle.rhs_p1(coords, elems, 2, f)["b2D"])
        for c, k in enumerate(("J1", "J2", "J3")):
            scale = ref[k + "abs"].sum()
            assert abs(got["tot"][c] - ref[k + "k"].sum()) <= TOL[dtype] * scale, (k, got["tot"][c])
        errs.append([abs(got["tot"][c] - pr[k]) for c, k in enumerate(("J1", "J2", "J3"))])
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 3.3) and np.all(ratios < 4.8), (errs, ratios)
