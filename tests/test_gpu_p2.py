"""Parity of the P2 element matrices (section 3.6, stiffness_matrixP2 / mass_matrixP2)
against the oracle, the exact energies of quadratic functions, and the fourth-order
benchmark of section 3.6 computed from the GPU's element matrices."""
import os

import numpy as np
import pytest
import torch

import oracle
from helpers import TOL, counters, cube, dev, flip_half, host, pair_pattern, prec_of, say, square, within
from paper_2404_16039_amd import gen

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def lib():
    from paper_2404_16039_amd import lib as L
    return L


def _gpu_p2(L, coords2, elems2, dtype, ruleK, ruleM, cK=None, cM=None):
    ne, nb = elems2.shape
    K = torch.empty(ne * nb * nb, dtype=dtype, device="cuda")
    M = torch.empty(ne * nb * nb, dtype=dtype, device="cuda")
    ctr = counters()
    L.p2_elements(prec_of(dtype), dev(coords2), dev(elems2), ruleK, ruleM,
                  cKq=None if cK is None else dev(cK, dtype), cMq=None if cM is None else dev(cM, dtype),
                  K3D=K, M3D=M, counters=ctr)
    return host(K).reshape(ne, nb * nb), host(M).reshape(ne, nb * nb), host(ctr)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("flip", [False, True])
def test_p2_parity(lib, dtype, dim, flip):
    """flip: half the elements with det J < 0 (vertices 1 and 2 swapped before the mid-edge
    nodes are added)."""
    say("p2 parity", dim, dtype, flip)
    coords, elems, _ = square(9) if dim == 2 else cube(5)
    if flip:
        elems = flip_half(elems)
    c2, e2, _ = gen.p2_mesh(coords, elems)
    rK, rM = oracle.stroud_rule(dim, 2), oracle.stroud_rule(dim, 3)
    xK = oracle.simplex_points(coords, elems, rK[0])
    xM = oracle.simplex_points(coords, elems, rM[0])
    rnd = lambda a: a.astype(np.float32).astype(np.float64) if dtype == torch.float32 else a
    cK, cM = rnd(np.exp(xK.sum(axis=-1))), rnd(1.0 + xM[..., 0] ** 2)
    K, M, ctr = _gpu_p2(lib, c2, e2, dtype, rK, rM, cK, cM)
    ref = oracle.p2_elements(c2, e2, rK, rM, cK, cM)
    within(K, ref["K3D"], ref["Kabs"], TOL[dtype], "P2 K3D")
    within(M, ref["M3D"], ref["Mabs"], TOL[dtype], "P2 M3D")
    assert ctr[0] == 0 and ctr[2] == 0


@pytest.mark.parametrize("dim", [2, 3])
def test_p2_quadratics_exact(lib, dim):
    """Sum over elements of v_e^T K_e v_e and v_e^T M_e v_e for a quadratic v equals the
    exact integrals over the unit square / cube (FP64)."""
    say("p2 quadratics", dim)
    coords, elems, _ = gen.square_mesh(6, jitter=0.2) if dim == 2 else gen.cube_mesh(4, jitter=0.15)
    c2, e2, _ = gen.p2_mesh(coords, elems)
    K, M, _ = _gpu_p2(lib, c2, e2, torch.float64, oracle.stroud_rule(dim, 2), oracle.stroud_rule(dim, 3))
    nb = e2.shape[1]
    v = c2[:, 0] ** 2 + 2 * c2[:, 1] * c2[:, -1] - c2[:, -1] + 0.5
    ve = v[e2]
    vK = np.einsum("ea,eab,eb->", ve, K.reshape(-1, nb, nb), ve)
    vM = np.einsum("ea,eab,eb->", ve, M.reshape(-1, nb, nb), ve)
    gl, gw = np.polynomial.legendre.leggauss(4)
    gl, gw = (gl + 1) / 2, gw / 2
    grid = np.stack(np.meshgrid(*([gl] * dim), indexing="ij"), axis=-1).reshape(-1, dim)
    wts = np.prod(np.stack(np.meshgrid(*([gw] * dim), indexing="ij"), axis=-1).reshape(-1, dim), axis=1)
    x = grid
    vv = x[:, 0] ** 2 + 2 * x[:, 1] * x[:, -1] - x[:, -1] + 0.5
    if dim == 2:
        g2 = (2 * x[:, 0]) ** 2 + (4 * x[:, 1] - 1) ** 2
    else:
        g2 = (2 * x[:, 0]) ** 2 + (2 * x[:, 2]) ** 2 + (2 * x[:, 1] - 1) ** 2
    assert abs(vK - (wts * g2).sum()) < 1e-11
    assert abs(vM - (wts * vv ** 2).sum()) < 1e-12


def test_p2_benchmark_fourth_order(lib):
    """The section 3.6 3-D P2 benchmark from the GPU's FP64 element matrices: the errors
    against the printed I_K, I_M fall at fourth order."""
    say("p2 benchmark")
    ik = im = None
    with open(os.path.join(GOLD, "energies.txt")) as fh:
        for line in fh:
            p = line.split()
            if p[:3] == ["closed", "3d", "IK"]:
                ik = float(p[3])
            if p[:3] == ["closed", "3d", "IM"]:
                im = float(p[3])
    errs = []
    for n in (4, 8, 16):
        c, e, _ = gen.cube_mesh(n, jitter=0.0, with_faces=False)
        c2, e2, _ = gen.p2_mesh(c, e)
        r = oracle.stroud_rule(3, 3)
        cq = np.exp(oracle.simplex_points(c, e, r[0]).sum(axis=-1))
        K, M, _ = _gpu_p2(lib, c2, e2, torch.float64, r, r, cq, cq)
        v = np.cos(np.pi * c2[:, 0]) * np.cos(np.pi * c2[:, 1]) * np.cos(np.pi * c2[:, 2])
        ve = v[e2]
        errs.append((abs(np.einsum("ea,eab,eb->", ve, K.reshape(-1, 10, 10), ve) - ik),
                     abs(np.einsum("ea,eab,eb->", ve, M.reshape(-1, 10, 10), ve) - im)))
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 13) and np.all(ratios < 19), (errs, ratios)


def test_p2_edge_cases(lib):
    say("p2 edge cases")
    coords, elems, _ = cube(1)
    c2, e2, _ = gen.p2_mesh(coords, elems)
    e2 = e2.copy()
    e2[0, 7] = c2.shape[0] + 5  # a bad mid-edge node
    r = oracle.stroud_rule(3, 2)
    K, M, ctr = _gpu_p2(lib, c2, e2, torch.float64, r, r)
    assert np.all(np.isnan(K[0])) and np.all(np.isnan(M[0])) and ctr[2] == 1
    assert np.all(np.isfinite(K[1:]))
    big = oracle.stroud_rule(3, 4)  # 64 points: more than the P2 limit
    with pytest.raises(lib.PagefemError):
        _gpu_p2(lib, c2, gen.p2_mesh(coords, elems)[1], torch.float64, big, r)
    Kt = torch.empty(e2.shape[0] * 100, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.PagefemError):  # K requested without a rule
        lib.p2_elements(lib.F64, dev(c2), dev(e2), None, r, K3D=Kt)


def _gpu_p2_global(L, coords2, elems2, dtype, ruleK, ruleM, cK=None, cM=None, csr=None):
    """P2 pages on the GPU, the P2 structure, and sparse() of the pages into it."""
    dim = coords2.shape[1]
    ne, nb = elems2.shape
    K = torch.empty(ne * nb * nb, dtype=dtype, device="cuda")
    M = torch.empty(ne * nb * nb, dtype=dtype, device="cuda")
    L.p2_elements(prec_of(dtype), dev(coords2), dev(elems2), ruleK, ruleM,
                  cKq=None if cK is None else dev(cK, dtype), cMq=None if cM is None else dev(cM, dtype), K3D=K, M3D=M)
    csr = csr or L.Csr()
    csr.symbolic_p2(dim, coords2.shape[0], dev(elems2))
    nn, nnz, _, _ = csr.info()
    vK = torch.empty(nnz, dtype=dtype, device="cuda")
    vM = torch.empty(nnz, dtype=dtype, device="cuda")
    csr.assemble_pages(prec_of(dtype), K, M, vK, vM)
    rp, ci = (host(t) for t in csr.structure())
    return {"K": host(K), "M": host(M), "rp": rp, "ci": ci, "vK": host(vK), "vM": host(vM), "csr": csr}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("mesh", ["cube3", "square7", "cube3_perm", "cube8", "square24"])
def test_p2_global_assembly(lib, dtype, mesh):
    """The global P2 K and M (section 3.6: sparse() of the P2 pages): the structure equals the
    oracle's sparse() pattern bit for bit, the values equal the oracle's sums of the same
    pages, and of the oracle's own pages, within the tolerance.  cube8 (4,913 P2 nodes) and
    square24 (2,401) span several tiles of the row-offset scan."""
    say("p2 global", mesh, dtype)
    base = mesh.split("_")[0]
    coords, elems, _ = cube(int(base[4:])) if base.startswith("cube") else square(int(base[6:]))
    if mesh.endswith("_perm"):
        coords, elems, _, _ = gen.permute_nodes(coords, elems)
    dim = coords.shape[1]
    c2, e2, _ = gen.p2_mesh(coords, elems)
    rK, rM = oracle.stroud_rule(dim, 2), oracle.stroud_rule(dim, 3)
    rnd = lambda a: a.astype(np.float32).astype(np.float64) if dtype == torch.float32 else a
    cK = rnd(np.exp(oracle.simplex_points(coords, elems, rK[0]).sum(axis=-1)))
    cM = rnd(1.0 + oracle.simplex_points(coords, elems, rM[0])[..., 0] ** 2)
    got = _gpu_p2_global(lib, c2, e2, dtype, rK, rM, cK, cM)
    nn = c2.shape[0]
    ref = oracle.assemble(e2, nn, got["K"].astype(np.float64), got["M"].astype(np.float64))
    assert np.array_equal(got["rp"], ref["row_ptr"]) and np.array_equal(got["ci"], ref["col_idx"])
    tol = TOL[dtype]
    within(got["vK"], ref["valK"], ref["scaleK"], tol, "P2 K from GPU pages")
    within(got["vM"], ref["valM"], ref["scaleM"], tol, "P2 M from GPU pages")
    pages = oracle.p2_elements(c2, e2, rK, rM, cK, cM)
    own = oracle.assemble(e2, nn, pages["K3D"], pages["M3D"], Kabs=pages["Kabs"])
    own_m = oracle.assemble(e2, nn, pages["Mabs"])
    within(got["vK"], own["valK"], own["scaleK"], tol, "P2 K vs oracle pages")
    within(got["vM"], own["valM"], own_m["valK"], tol, "P2 M vs oracle pages")
    got["csr"].close()


def test_p2_global_permutation_bitwise(lib):
    """Exact sums: renumbering the P2 nodes gives the same global values, bit for bit."""
    say("p2 permutation")
    coords, elems, _ = cube(4)
    c2, e2, _ = gen.p2_mesh(coords, elems)
    r = oracle.stroud_rule(3, 2)
    a = _gpu_p2_global(lib, c2, e2, torch.float32, r, r)
    pc, pe, _, perm = gen.permute_nodes(c2, e2)  # pc[perm[i]] = c2[i]
    b = _gpu_p2_global(lib, pc, pe, torch.float32, r, r)
    # entry (i, j) of a is entry (perm[i], perm[j]) of b
    def dense_entries(d, p):
        rows = np.repeat(np.arange(len(d["rp"]) - 1), np.diff(d["rp"]))
        return {(int(p[i]), int(p[j])): (k, m) for i, j, k, m in zip(rows, d["ci"], d["vK"], d["vM"])}
    ident = np.arange(c2.shape[0])
    da, db = dense_entries(a, perm), dense_entries(b, ident)
    assert da.keys() == db.keys()
    assert all(da[k][0] == db[k][0] and da[k][1] == db[k][1] for k in da)
    a["csr"].close()
    b["csr"].close()


def test_p2_global_full_size_properties(lib):
    """The 64^3 P2 mesh of the section 3.6 benchmark (2,146,689 nodes), FP32 with c = exp(x1+x2+x3)
    at 27 points: the structure equals every node pair of the elements (all rows), interior
    vertex rows hold 65 entries, K rows sum to 0, the entries of M sum to 1,
    v^T K v and v^T M v of a quadratic v equal its exact energies with c = 1, and sampled rows
    equal the FP64 sums of their pages."""
    say("p2 global 64^3")
    n = 64
    coords, elems, _ = gen.cube_mesh(n, jitter=0.15, with_faces=False)
    c2, e2, _ = gen.p2_mesh(coords, elems)
    r = oracle.stroud_rule(3, 3)
    got = _gpu_p2_global(lib, c2, e2, torch.float32, r, r)
    rp, ci, vK, vM = got["rp"], got["ci"], got["vK"].astype(np.float64), got["vM"].astype(np.float64)
    assert c2.shape[0] == 2146689 and np.diff(rp).max() == 65
    # the whole structure, bit for bit, against the sorted node pairs of the elements
    prp, pci = pair_pattern(e2, c2.shape[0], chunk=1 << 19)
    assert np.array_equal(rp.astype(np.int64), prp) and np.array_equal(ci, pci)
    del prp, pci
    rows = np.repeat(np.arange(c2.shape[0]), np.diff(rp))
    rs = np.bincount(rows, weights=vK, minlength=c2.shape[0])
    ra = np.bincount(rows, weights=np.abs(vK), minlength=c2.shape[0])
    assert np.all(np.abs(rs) <= 1e-5 * ra)
    assert abs(vM.sum() - 1.0) < 1e-5
    v = c2[:, 0] ** 2 + 2 * c2[:, 1] * c2[:, 2] - c2[:, 2] + 0.5
    vKv = (v[rows] * vK * v[ci]).sum()
    vMv = (v[rows] * vM * v[ci]).sum()
    gl, gw = np.polynomial.legendre.leggauss(4)
    gl, gw = (gl + 1) / 2, gw / 2
    x = np.stack(np.meshgrid(gl, gl, gl, indexing="ij"), axis=-1).reshape(-1, 3)
    w = np.prod(np.stack(np.meshgrid(gw, gw, gw, indexing="ij"), axis=-1).reshape(-1, 3), axis=1)
    ik = (w * ((2 * x[:, 0]) ** 2 + (2 * x[:, 2]) ** 2 + (2 * x[:, 1] - 1) ** 2)).sum()
    im = (w * (x[:, 0] ** 2 + 2 * x[:, 1] * x[:, 2] - x[:, 2] + 0.5) ** 2).sum()
    assert abs(vKv - ik) < 2e-4 * ik and abs(vMv - im) < 2e-5 * im, (vKv, ik, vMv, im)
    K, M = got["K"].reshape(-1, 10, 10), got["M"].reshape(-1, 10, 10)
    rng = np.random.default_rng(5)
    for i in rng.choice(c2.shape[0], 24, replace=False):
        es, as_ = np.nonzero(e2 == i)
        for vals, P in ((vK, K), (vM, M)):
            want, scale = {}, {}
            for e, a in zip(es, as_):
                for b in range(10):
                    j = int(e2[e, b])
                    x_ = float(P[e, a, b])  # page entry (b, a) (at b + 10 a) goes to row e2[e, a] = i
                    want[j] = want.get(j, 0.0) + x_
                    scale[j] = scale.get(j, 0.0) + abs(x_)
            cols = ci[rp[i]:rp[i + 1]]
            assert sorted(want) == list(cols)
            for k, j in enumerate(cols):
                assert abs(vals[rp[i] + k] - want[j]) <= TOL[torch.float32] * scale[j]
    got["csr"].close()


def test_p2_structure_errors(lib):
    say("p2 structure errors")
    coords, elems, _ = cube(2)
    c2, e2, _ = gen.p2_mesh(coords, elems)
    csr = lib.Csr().symbolic_p2(3, c2.shape[0], dev(e2))
    nn, nnz, _, _ = csr.info()
    v = torch.empty(nnz, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.PagefemError):  # a P1 call on a P2 structure
        csr.assemble(lib.F64, dev(c2), dev(e2), v, v)
    with pytest.raises(lib.PagefemError):  # an output without pages
        csr.assemble_pages(lib.F64, None, None, v, None)
    bad = e2.copy()
    bad[3, 7] = c2.shape[0] + 1
    with pytest.raises(lib.PagefemError):
        lib.Csr().symbolic_p2(3, c2.shape[0], dev(bad))
    csr.close()


def test_p1_pages_assembly_matches_fused(lib):
    """sparse() of the P1 pages of pf_elem_stiffness_mass into a P1 structure equals the fused
    numeric assembly within the tolerance (both sum exactly; the pages take the first node as
    the origin, the fused rows their own node)."""
    say("p1 pages")
    coords, elems, _ = cube(5)
    tc, te = dev(coords), dev(elems)
    csr = lib.Csr().symbolic(3, coords.shape[0], te)
    nn, nnz, _, _ = csr.info()
    ne = elems.shape[0]
    K = torch.empty(ne * 16, dtype=torch.float64, device="cuda")
    M = torch.empty(ne * 16, dtype=torch.float64, device="cuda")
    lib.elem_stiffness_mass(lib.F64, tc, te, K3D=K, M3D=M)
    a = [torch.empty(nnz, dtype=torch.float64, device="cuda") for _ in range(4)]
    csr.assemble_pages(lib.F64, K, M, a[0], a[1])
    csr.assemble(lib.F64, tc, te, a[2], a[3])
    ref = oracle.assemble(elems, coords.shape[0], host(K), host(M))
    within(host(a[0]), ref["valK"], ref["scaleK"], TOL[torch.float64], "P1 pages K")
    within(host(a[1]), ref["valM"], ref["scaleM"], TOL[torch.float64], "P1 pages M")
    # against the fused rows: contributions that vanish in exact arithmetic round differently
    # with the two origins, so K takes the Cauchy-Schwarz scale of each contribution
    el = oracle.p1_elements(coords, elems)
    cs = oracle.assemble(elems, coords.shape[0], el["Ke"], el["Me"], Kabs=el["Kabs"])
    within(host(a[0]), cs["valK"], cs["scaleK"], TOL[torch.float64], "P1 pages K (CS scale)")
    within(host(a[2]), cs["valK"], cs["scaleK"], TOL[torch.float64], "P1 fused K (CS scale)")
    within(host(a[3]), host(a[1]), cs["scaleM"], TOL[torch.float64], "P1 fused M")
    csr.close()


def _unaligned(t):
    """A copy of t in device memory that starts one element past a 16-byte boundary."""
    buf = torch.empty(t.numel() + 1, dtype=t.dtype, device="cuda")
    buf[1:].copy_(t)
    v = buf[1:]
    assert v.data_ptr() % 16 != 0
    return v


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_pages_assembly_unaligned_pages(lib, dtype):
    """sparse() reads page columns with vector loads only from 16-byte aligned page arrays;
    arrays that start elsewhere take element loads and give the same values bit for bit (P2
    pages of 10 nodes, P1 pages of 4 nodes, and one output alone)."""
    say("pages unaligned", dtype)
    coords, elems, _ = cube(3)
    c2, e2, _ = gen.p2_mesh(coords, elems)
    r = oracle.stroud_rule(3, 2)
    a = _gpu_p2_global(lib, c2, e2, dtype, r, r)
    K = torch.from_numpy(a["K"]).cuda()
    M = torch.from_numpy(a["M"]).cuda()
    nnz = a["vK"].shape[0]
    vK = torch.empty(nnz, dtype=dtype, device="cuda")
    vM = torch.empty(nnz, dtype=dtype, device="cuda")
    a["csr"].assemble_pages(prec_of(dtype), _unaligned(K), _unaligned(M), vK, vM)
    assert np.array_equal(host(vK), a["vK"]) and np.array_equal(host(vM), a["vM"])
    vK.fill_(0)
    a["csr"].assemble_pages(prec_of(dtype), _unaligned(K), None, vK, None)
    assert np.array_equal(host(vK), a["vK"])
    a["csr"].close()
    # P1 pages (4 x 4: one 16-byte vector per FP32 column when aligned)
    tc, te = dev(coords), dev(elems)
    csr = lib.Csr().symbolic(3, coords.shape[0], te)
    _, nnz1, _, _ = csr.info()
    ne = elems.shape[0]
    K1 = torch.empty(ne * 16, dtype=dtype, device="cuda")
    M1 = torch.empty(ne * 16, dtype=dtype, device="cuda")
    lib.elem_stiffness_mass(prec_of(dtype), tc, te, K3D=K1, M3D=M1)
    out = [torch.empty(nnz1, dtype=dtype, device="cuda") for _ in range(4)]
    csr.assemble_pages(prec_of(dtype), K1, M1, out[0], out[1])
    csr.assemble_pages(prec_of(dtype), _unaligned(K1), _unaligned(M1), out[2], out[3])
    assert np.array_equal(host(out[0]), host(out[2])) and np.array_equal(host(out[1]), host(out[3]))
    csr.close()


def test_p2_routed_slivers(lib):
    """FP32 pages of elements whose Jacobian fails the routing test (isolated slivers with det
    down to 1e-6 h^3) are recomputed in FP64: every page matches the FP64 oracle within 1e-5
    of each entry's scale, and the routed count is exactly the number of slivers."""
    say("p2 routed slivers")
    n, ns = 4, 96
    h = 1.0 / n
    coords, elems, _ = cube(n)
    cs, es, _ = gen.append_slivers(coords, elems, ns, h)
    c2, e2, _ = gen.p2_mesh(cs, es)
    r = oracle.stroud_rule(3, 2)
    ne, nb = e2.shape
    K = torch.empty(ne * nb * nb, dtype=torch.float32, device="cuda")
    M = torch.empty(ne * nb * nb, dtype=torch.float32, device="cuda")
    ctr = counters()
    lib.p2_elements(lib.F32, dev(c2), dev(e2), r, r, K3D=K, M3D=M, fb=lib.fallback(1e-3 * h ** 3, 1e6, True),
                    counters=ctr)
    ctr = host(ctr)
    assert ctr[0] == ns and ctr[2] == 0, ctr
    ref = oracle.p2_elements(c2, e2, r, r)
    within(host(K).reshape(ne, nb * nb), ref["K3D"], ref["Kabs"], TOL[torch.float32], "P2 K3D with slivers")
    within(host(M).reshape(ne, nb * nb), ref["M3D"], ref["Mabs"], TOL[torch.float32], "P2 M3D with slivers")
    # K alone takes the same path
    K2 = torch.empty_like(K)
    lib.p2_elements(lib.F32, dev(c2), dev(e2), r, None, K3D=K2, fb=lib.fallback(1e-3 * h ** 3, 1e6, True))
    assert np.array_equal(host(K2), host(K))
