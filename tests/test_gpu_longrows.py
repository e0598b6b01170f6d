"""Long rows: P1 meshes with a node in more than 64 elements or a row of more than 64
nonzeros (the spill class of the row-owned assembly).  The structure is compared bit for
bit with the oracle's sparse() pattern, the values of K and M (constant, per-element and
quadrature coefficients, FP32 and FP64), the load vector and sparse() of element pages
within the tolerance of each entry's scale; meshes mix long rows with ordinary ones, also
after a random renumbering (long rows then fall anywhere in the 8-row groups)."""
import numpy as np
import pytest
import torch

import oracle
from helpers import TOL, counters, cube, dev, host, prec_of, say, within
from paper_2404_16039_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2404_16039_amd import lib as L
    return L


def fan2d(k, seed=0):
    """A centre node in k triangles (its row: k + 1 nonzeros); radii jittered."""
    g = np.random.default_rng(seed)
    ang = np.linspace(0, 2 * np.pi, k, endpoint=False) + g.uniform(-0.2, 0.2, k) * (2 * np.pi / k)
    rad = g.uniform(0.8, 1.2, k)
    coords = np.concatenate([[[0.0, 0.0]], np.stack([rad * np.cos(ang), rad * np.sin(ang)], 1)])
    elems = np.array([[0, 1 + i, 1 + (i + 1) % k] for i in range(k)], np.int32)
    return coords, elems


def star3d(k, seed=0):
    """A centre node in 2k tetrahedra around a ring of k nodes with an apex above and below
    (centre row: k + 3 nonzeros; each apex lies in k tetrahedra)."""
    g = np.random.default_rng(seed)
    ang = np.linspace(0, 2 * np.pi, k, endpoint=False) + g.uniform(-0.2, 0.2, k) * (2 * np.pi / k)
    rad = g.uniform(0.8, 1.2, k)
    ring = np.stack([rad * np.cos(ang), rad * np.sin(ang), g.uniform(-0.1, 0.1, k)], 1)
    coords = np.concatenate([[[0.0, 0.0, 0.0]], ring, [[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]]])
    top, bot = k + 1, k + 2
    el = []
    for i in range(k):
        a, b = 1 + i, 1 + (i + 1) % k
        el.append([0, a, b, top])
        el.append([0, b, a, bot])
    return coords, np.array(el, np.int32)


def with_block(coords, elems, n=3, shift=(3.0, 0.0, 0.0)):
    """The mesh after a Kuhn block of n^3 cubes (or an n x n square), node ids offset."""
    dim = coords.shape[1]
    bc, be, _ = cube(n) if dim == 3 else gen.square_mesh(n, jitter=0.2)
    c = np.concatenate([bc, coords + np.array(shift[:dim])])
    e = np.concatenate([be, elems + bc.shape[0]]).astype(np.int32)
    return c, e


def renumber(coords, elems, seed):
    perm = np.random.default_rng(seed).permutation(coords.shape[0])  # old id -> new id
    c = np.empty_like(coords)
    c[perm] = coords
    return c, perm[elems].astype(np.int32)


def meshes():
    c2, e2 = with_block(*fan2d(70, 1), n=6)
    c3, e3 = with_block(*star3d(80, 2), n=3)
    c4, e4 = with_block(*star3d(40, 3), n=3)  # centre in 80 tets, row of 43 nonzeros
    return {"fan70": (c2, e2), "star80": (c3, e3), "star40": (c4, e4),
            "fan70_perm": renumber(c2, e2, 5), "star80_perm": renumber(c3, e3, 6), "fan100": fan2d(100, 4)}


MESHES = meshes()


def _gpu(L, coords, elems, dtype, cK=None, cM=None):
    dim = coords.shape[1]
    tc, te = dev(coords), dev(elems)
    csr = L.Csr().symbolic(dim, coords.shape[0], te)
    _, nnz, _, _ = csr.info()
    vk = torch.empty(nnz, dtype=dtype, device="cuda")
    vm = torch.empty(nnz, dtype=dtype, device="cuda")
    ctr = counters()
    csr.assemble(prec_of(dtype), tc, te, vk, vm, cK=None if cK is None else dev(cK, dtype),
                 cM=None if cM is None else dev(cM, dtype), counters=ctr)
    rp, ci = csr.structure()
    return csr, {"row_ptr": host(rp).astype(np.int64), "col_idx": host(ci), "valK": host(vk), "valM": host(vm),
                 "nnz": nnz, "ctr": host(ctr)}


def _oracle(coords, elems, cK=None, cM=None):
    el = oracle.p1_elements(coords, elems)
    Ke, Me, Ka = el["Ke"], el["Me"], el["Kabs"]
    if cK is not None:
        Ke, Ka = Ke * cK[:, None], Ka * np.abs(cK[:, None])
    if cM is not None:
        Me = Me * cM[:, None]
    return oracle.assemble(elems, coords.shape[0], Ke, Me, Ka)


def _long_rows(ref):
    rp = ref["row_ptr"]
    return int(np.sum(np.diff(rp) > 64))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name", list(MESHES))
def test_long_rows_parity(lib, name, dtype):
    say("long rows", name, dtype)
    coords, elems = MESHES[name]
    g = np.random.default_rng(11)
    for coef in (False, True):
        cK = cM = None
        if coef:
            cK = g.uniform(0.5, 2.0, len(elems))
            cM = g.uniform(0.5, 2.0, len(elems))
            if dtype == torch.float32:
                cK = cK.astype(np.float32).astype(np.float64)
                cM = cM.astype(np.float32).astype(np.float64)
        csr, got = _gpu(lib, coords, elems, dtype, cK, cM)
        ref = _oracle(coords, elems, cK, cM)
        assert got["nnz"] == ref["nnz"]
        assert np.array_equal(got["row_ptr"], ref["row_ptr"]) and np.array_equal(got["col_idx"], ref["col_idx"])
        within(got["valK"], ref["valK"], ref["scaleK"], TOL[dtype], f"{name} K")
        within(got["valM"], ref["valM"], ref["scaleM"], TOL[dtype], f"{name} M")
        assert got["ctr"][2] == 0
        csr.close()


@pytest.mark.parametrize("name", list(MESHES))
def test_long_rows_faces(lib, name):
    """Every face of meshes with long rows (the long rows' own faces from the long-row face
    kernel, the others from the row blocks), with its element pair and orientation, and the
    boundary list, equal to the oracle's; twice on one handle (the second call reuses the
    lists)."""
    say("long-row faces", name)
    coords, elems = MESHES[name]
    te = dev(elems)
    csr = lib.Csr().symbolic(coords.shape[1], coords.shape[0], te)
    F, FE = oracle.faces(coords, elems)
    b = FE[:, 1] < 0
    for _ in range(2):
        csr.faces(dev(coords), te)
        f, fe, bf, be = (host(t) for t in csr.face_lists())
        assert np.array_equal(f, F) and np.array_equal(fe, FE)
        assert np.array_equal(bf, F[b]) and np.array_equal(be, FE[b, 0])
    csr.close()


def test_long_rows_are_listed(lib):
    """The meshes above really hold long rows of both kinds (elements > 64, nonzeros > 64)."""
    for name, (coords, elems) in MESHES.items():
        nn = coords.shape[0]
        per_node = np.bincount(elems.ravel(), minlength=nn)
        ref = _oracle(coords, elems)
        nz = np.diff(ref["row_ptr"])
        assert np.any(per_node > 64) or np.any(nz > 64), name
    c, e = MESHES["star40"]
    assert np.bincount(e.ravel()).max() == 80 and np.diff(_oracle(c, e)["row_ptr"]).max() <= 64


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_long_rows_quadrature(lib, dtype):
    """Coefficients at the 4 points of the degree-2 rule (the section 3.6 benchmark's form)."""
    say("long rows quad", dtype)
    coords, elems = MESHES["star80_perm"]
    tc, te = dev(coords), dev(elems)
    xq = lib.quad_points(tc, te, 2)
    cq = torch.exp(xq.sum(dim=2)).to(dtype).contiguous()
    csr = lib.Csr().symbolic(3, coords.shape[0], te)
    _, nnz, _, _ = csr.info()
    vk = torch.empty(nnz, dtype=dtype, device="cuda")
    vm = torch.empty(nnz, dtype=dtype, device="cuda")
    csr.assemble_quad(prec_of(dtype), tc, 2, vk, vm, cKq=cq, cMq=cq)
    c64 = host(cq).astype(np.float64)
    q = oracle.p1_elements_q(coords, elems, 2, c64, c64)
    ref = oracle.assemble(elems, coords.shape[0], q["Ke"], q["Me"], q["Kabs"])
    within(host(vk), ref["valK"], ref["scaleK"], TOL[dtype], "quad K")
    within(host(vm), ref["valM"], ref["scaleM"], TOL[dtype], "quad M")
    csr.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_long_rows_pages_and_rhs(lib, dtype):
    """sparse() of element pages and the load vector's node sums on meshes with long rows."""
    say("long rows pages rhs", dtype)
    for name in ("fan70_perm", "star80", "fan100"):
        coords, elems = MESHES[name]
        dim = coords.shape[1]
        nlb = dim + 1
        tc, te = dev(coords), dev(elems)
        csr = lib.Csr().symbolic(dim, coords.shape[0], te)
        _, nnz, _, _ = csr.info()
        ne = elems.shape[0]
        K = torch.empty(ne * nlb * nlb, dtype=dtype, device="cuda")
        M = torch.empty(ne * nlb * nlb, dtype=dtype, device="cuda")
        lib.elem_stiffness_mass(prec_of(dtype), tc, te, K3D=K, M3D=M)
        vk = torch.empty(nnz, dtype=dtype, device="cuda")
        vm = torch.empty(nnz, dtype=dtype, device="cuda")
        csr.assemble_pages(prec_of(dtype), K, M, vk, vm)
        ref = oracle.assemble(elems, coords.shape[0], host(K).astype(np.float64), host(M).astype(np.float64))
        within(host(vk), ref["valK"], ref["scaleK"], TOL[dtype], f"{name} pages K")
        within(host(vm), ref["valM"], ref["scaleM"], TOL[dtype], f"{name} pages M")
        # load vector, order 2, f = 1 + x1 at the points
        xq = oracle.quad_points(coords, elems, 2)
        f = (1.0 + xq[..., 0]).astype(np.float32 if dtype == torch.float32 else np.float64).astype(np.float64)
        b2D = torch.empty(ne * nlb, dtype=dtype, device="cuda")
        b = torch.empty(coords.shape[0], dtype=dtype, device="cuda")
        csr.rhs(prec_of(dtype), tc, te, 2, dev(f, dtype), b2D, b)
        r = oracle.rhs_p1(coords, elems, 2, f)
        within(host(b), r["b"], r["babs"], TOL[dtype], f"{name} b")
        csr.close()


def test_long_rows_deterministic(lib):
    """Long rows sum exactly: a rebuild in the same handle and a renumbering give the same bits."""
    say("long rows determinism")
    coords, elems = MESHES["star80"]
    csr, a = _gpu(lib, coords, elems, torch.float32)
    csr.close()
    csr, b = _gpu(lib, coords, elems, torch.float32)
    assert np.array_equal(a["valK"], b["valK"]) and np.array_equal(a["valM"], b["valM"])
    csr.close()
    pc, pe = renumber(coords, elems, 9)
    csr, p = _gpu(lib, pc, pe, torch.float32)
    csr.close()
    perm = np.random.default_rng(9).permutation(coords.shape[0])

    def entries(got, relabel):
        rows = np.repeat(np.arange(len(got["row_ptr"]) - 1), np.diff(got["row_ptr"]))
        r, c = relabel[rows], relabel[got["col_idx"]]
        o = np.lexsort((c, r))
        return got["valK"][o], got["valM"][o]

    ka, ma = entries(a, perm)
    kp, mp = entries(p, np.arange(pc.shape[0]))
    assert np.array_equal(ka, kp) and np.array_equal(ma, mp)


def p2_meshes():
    """P2 meshes (one node per edge midpoint) with long rows: a centre vertex in 80 tets (a
    row of 205 nonzeros), one in 60 tets whose row of 155 nonzeros overflows the 128-slot
    tables, a 2-D centre in 70 triangles (211 nonzeros); each after a Kuhn block, and
    renumbered."""
    base = {"p2star40": with_block(*star3d(40, 3), n=2), "p2star30": with_block(*star3d(30, 7), n=2),
            "p2fan70": with_block(*fan2d(70, 1), n=4)}
    out = {}
    for name, (c, e) in base.items():
        c2, e2, _ = gen.p2_mesh(c, e)
        out[name] = (c2, e2)
        out[name + "_perm"] = renumber(c2, e2, 13)
    return out


P2_MESHES = p2_meshes()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name", list(P2_MESHES))
def test_p2_long_rows(lib, name, dtype):
    """sparse() of P2 element pages on meshes with long rows: the structure equals the
    oracle's sparse() pattern bit for bit (long rows listed), the values the oracle's exact
    sums of the same pages within the tolerance; the same pages again give the same bits."""
    say("p2 long rows", name, dtype)
    c2, e2 = P2_MESHES[name]
    dim, nn = c2.shape[1], c2.shape[0]
    rK, rM = oracle.stroud_rule(dim, 2), oracle.stroud_rule(dim, 3)
    pages = oracle.p2_elements(c2, e2, rK, rM)
    K = pages["K3D"].astype(np.float32).astype(np.float64) if dtype == torch.float32 else pages["K3D"]
    M = pages["M3D"].astype(np.float32).astype(np.float64) if dtype == torch.float32 else pages["M3D"]
    ref = oracle.assemble(e2, nn, K, M)
    lens, counts = np.diff(ref["row_ptr"]), np.bincount(e2.ravel(), minlength=nn)
    assert np.any((counts > 64) | (lens > 128))  # the mesh has P2 long rows
    csr = lib.Csr().symbolic_p2(dim, nn, dev(e2))
    _, nnz, _, _ = csr.info()
    rp, ci = (host(t) for t in csr.structure())
    assert np.array_equal(rp, ref["row_ptr"]) and np.array_equal(ci, ref["col_idx"])
    tK, tM = dev(K.ravel(), dtype), dev(M.ravel(), dtype)
    outs = []
    for _ in range(2):
        vK = torch.empty(nnz, dtype=dtype, device="cuda")
        vM = torch.empty(nnz, dtype=dtype, device="cuda")
        csr.assemble_pages(prec_of(dtype), tK, tM, vK, vM)
        outs.append((host(vK), host(vM)))
    within(outs[0][0], ref["valK"], ref["scaleK"], TOL[dtype], f"{name} P2 K")
    within(outs[0][1], ref["valM"], ref["scaleM"], TOL[dtype], f"{name} P2 M")
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    csr.close()


def test_rebuilds_with_and_without_long_rows(lib):
    """One handle rebuilt in turn for P2 meshes with long rows, without, and P1 meshes with
    and without (the speculative column phase, the long-row list, the ninth-position bytes
    and the face lists carried over from the previous build): every structure, sparse() of
    the oracle's pages and the face lists equal the oracle's."""
    say("long-row rebuilds")
    c3, e3, _ = cube(3)
    p2cube = gen.p2_mesh(c3, e3)[:2]
    seq = [("p2", P2_MESHES["p2star40"]), ("p2", p2cube), ("p1", MESHES["star80"]), ("p2", P2_MESHES["p2fan70"]),
           ("p1", (c3, e3)), ("p2", P2_MESHES["p2star30_perm"]), ("p1", MESHES["fan70_perm"])]
    csr = lib.Csr()
    for kind, (c, e) in seq:
        dim, nn = c.shape[1], c.shape[0]
        if kind == "p2":
            rK, rM = oracle.stroud_rule(dim, 2), oracle.stroud_rule(dim, 3)
            pages = oracle.p2_elements(c, e, rK, rM)
            K, M = pages["K3D"], pages["M3D"]
            csr.symbolic_p2(dim, nn, dev(e))
        else:
            el = oracle.p1_elements(c, e)
            K, M = el["Ke"], el["Me"]
            csr.symbolic(dim, nn, dev(e))
        ref = oracle.assemble(e, nn, K, M)
        _, nnz, _, _ = csr.info()
        rp, ci = (host(t) for t in csr.structure())
        assert np.array_equal(rp, ref["row_ptr"]) and np.array_equal(ci, ref["col_idx"]), kind
        vK = torch.empty(nnz, dtype=torch.float64, device="cuda")
        vM = torch.empty(nnz, dtype=torch.float64, device="cuda")
        csr.assemble_pages(lib.F64, dev(K.ravel()), dev(M.ravel()), vK, vM)
        within(host(vK), ref["valK"], ref["scaleK"], TOL[torch.float64], f"rebuild {kind} K")
        within(host(vM), ref["valM"], ref["scaleM"], TOL[torch.float64], f"rebuild {kind} M")
        if kind == "p1":
            csr.faces(dev(c), dev(e))
            F, FE = oracle.faces(c, e)
            f, fe, _, _ = (host(t) for t in csr.face_lists())
            assert np.array_equal(f, F) and np.array_equal(fe, FE)
    csr.close()


def test_row_beyond_256_nonzeros_is_refused(lib):
    """A long row holds at most 256 nonzeros (8-bit column positions of the slot words)."""
    say("long row limit")
    coords, elems = fan2d(300, 7)
    with pytest.raises(lib.PagefemError) as ei:
        lib.Csr().symbolic(2, coords.shape[0], dev(elems))
    assert ei.value.code == 7
    c2, e2, _ = gen.p2_mesh(*fan2d(100, 7))  # a P2 centre row of 301 nonzeros
    with pytest.raises(lib.PagefemError) as ei:
        lib.Csr().symbolic_p2(2, c2.shape[0], dev(e2))
    assert ei.value.code == 7
    coords, elems = fan2d(255, 8)  # a row of 256 nonzeros is still accepted
    csr, got = _gpu(lib, coords, elems, torch.float64)
    ref = _oracle(coords, elems)
    assert np.array_equal(got["col_idx"], ref["col_idx"])
    within(got["valK"], ref["valK"], ref["scaleK"], TOL[torch.float64], "fan255 K")
    csr.close()


def test_long_rows_through_the_server(lib):
    """A job whose mesh has long rows, fused with ordinary jobs, gets the values of the same
    mesh assembled alone, bit for bit."""
    say("long rows server")
    srv = lib.Server(1 << 30, 16)
    jobs = []
    for k, name in enumerate(("star80", "star40")):
        coords, elems = MESHES[name]
        nn = coords.shape[0]
        csr, alone = _gpu(lib, coords, elems, torch.float32)
        csr.close()
        vk = torch.empty(alone["nnz"], dtype=torch.float32).pin_memory()
        vm = torch.empty(alone["nnz"], dtype=torch.float32).pin_memory()
        t = srv.submit(3, lib.F32, torch.from_numpy(coords).pin_memory(), torch.from_numpy(elems).pin_memory(),
                       topology=3000 + k, valsK=vk, valsM=vm)
        jobs.append((t, vk, vm, alone))
    c, e, _ = cube(4)
    srv.submit(3, lib.F32, torch.from_numpy(c).pin_memory(), torch.from_numpy(e).pin_memory(), topology=3100)
    for t, vk, vm, alone in jobs:
        r = srv.wait(t)
        assert r["status"] == 0
        assert np.array_equal(vk.numpy(), alone["valK"]) and np.array_equal(vm.numpy(), alone["valM"])
    srv.close()
