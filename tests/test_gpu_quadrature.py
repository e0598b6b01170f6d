"""Assembly with coefficients given at integration points (the loop over integration points
of the section 3.6 stiffness and mass listings): integration points bitwise equal to the
oracle's, assembled values against the oracle, and the section 3.6 energy benchmark
(c = exp(sum x)) converging at second order up to the 128^3 mesh, where the errors match the
printed table."""
import os

import numpy as np
import pytest
import torch

import oracle
from helpers import TOL, counters, dev, flip_half, host, prec_of, say, within
from paper_2404_16039_amd import gen

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def lib():
    from paper_2404_16039_amd import lib as L
    return L


def _closed():
    out, table = {}, {}
    for line in open(os.path.join(GOLD, "energies.txt")):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "closed":
            out[(f[1], f[2])] = float(f[3])
        elif f[0] == "p1_3d":
            table[int(f[2])] = (float(f[3]), float(f[4]))
    return out, table


def _gpu_quad(L, coords, elems, dtype, order, fb=None):
    dim = coords.shape[1]
    tc, te = dev(coords), dev(elems)
    xq = L.quad_points(tc, te, order)
    cq = torch.exp(xq.sum(dim=2)).to(dtype).contiguous()
    csr = L.Csr().symbolic(dim, coords.shape[0], te)
    _, nnz, _, _ = csr.info()
    vk = torch.empty(nnz, dtype=dtype, device="cuda")
    vm = torch.empty(nnz, dtype=dtype, device="cuda")
    ctr = counters()
    csr.assemble_quad(prec_of(dtype), tc, order, vk, vm, cKq=cq, cMq=cq, fb=fb, counters=ctr)
    rp, ci = csr.structure()
    out = {"xq": host(xq), "cq": host(cq).astype(np.float64), "row_ptr": host(rp).astype(np.int64),
           "col_idx": host(ci), "valK": host(vk), "valM": host(vm), "ctr": host(ctr)}
    csr.close()
    return out


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("dim,n", [(2, 12), (3, 5)])
@pytest.mark.parametrize("flip", [False, True])
def test_quadrature_assembly_matches_oracle(lib, dtype, order, dim, n, flip):
    """flip: half the elements with det J < 0."""
    say("quadrature assembly", dtype, order, dim, n, flip)
    coords, elems, _ = (gen.square_mesh(n) if dim == 2 else gen.cube_mesh(n))
    if flip:
        elems = flip_half(elems)
    got = _gpu_quad(lib, coords, elems, dtype, order)
    xq = oracle.quad_points(coords, elems, order)
    assert np.array_equal(got["xq"], xq), "integration points differ from the oracle's"
    q = oracle.p1_elements_q(coords, elems, order, got["cq"], got["cq"])
    ref = oracle.assemble(elems, coords.shape[0], q["Ke"], q["Me"], q["Kabs"])
    assert np.array_equal(got["row_ptr"], ref["row_ptr"]) and np.array_equal(got["col_idx"], ref["col_idx"])
    within(got["valK"], ref["valK"], ref["scaleK"], TOL[dtype], "K")
    within(got["valM"], ref["valM"], ref["scaleM"], TOL[dtype], "M")


def _energies(coords, got):
    pi = np.pi
    if coords.shape[1] == 2:
        v = np.sin(pi * coords[:, 0]) * np.sin(pi * coords[:, 1])
    else:
        v = np.cos(pi * coords[:, 0]) * np.cos(pi * coords[:, 1]) * np.cos(pi * coords[:, 2])
    rows = np.repeat(np.arange(coords.shape[0]), np.diff(got["row_ptr"]))
    vl, vr = v[rows], v[got["col_idx"]]
    return (float(np.sum(vl * got["valK"].astype(np.float64) * vr)),
            float(np.sum(vl * got["valM"].astype(np.float64) * vr)))


def test_energy_benchmark_3d_up_to_128(lib):
    """e_K, e_M on the Kuhn meshes with the node counts of the printed levels 3..7 (up to
    2,146,689 nodes): second order, and within 25% of the printed errors."""
    closed, table = _closed()
    errs = []
    for n in (8, 16, 32, 64, 128):
        say("energy 3d", n)
        coords, elems, _ = gen.cube_mesh(n, jitter=0.0, with_faces=False)
        got = _gpu_quad(lib, coords, elems, torch.float64, 2)
        k, m = _energies(coords, got)
        eK, eM = abs(k - closed[("3d", "IK")]), abs(m - closed[("3d", "IM")])
        pK, pM = table[coords.shape[0]]
        print(f"n={n}: e_K {eK:.3e} (printed {pK:.2e})  e_M {eM:.3e} (printed {pM:.2e})")
        assert 0.8 < eK / pK < 1.25 and 0.8 < eM / pM < 1.25
        errs.append((eK, eM))
    for (k0, m0), (k1, m1) in zip(errs, errs[1:]):
        assert 3.6 < k0 / k1 < 4.4 and 3.6 < m0 / m1 < 4.4


def test_energy_benchmark_2d_rate(lib):
    closed, _ = _closed()
    errs = []
    for n in (32, 64, 128, 256):
        coords, elems, _ = gen.square_mesh(n, jitter=0.0)
        got = _gpu_quad(lib, coords, elems, torch.float64, 2)
        k, m = _energies(coords, got)
        errs.append((abs(k - closed[("2d", "IK")]), abs(m - closed[("2d", "IM")])))
    for (k0, m0), (k1, m1) in zip(errs, errs[1:]):
        assert 3.8 < k0 / k1 < 4.2 and 3.8 < m0 / m1 < 4.2


def test_fp32_quadrature_with_slivers(lib):
    """FP32 with routed slivers: the routed elements' rows are recomputed in FP64 and match."""
    n = 6
    h = 1.0 / n
    coords, elems, _ = gen.cube_mesh(n)
    c2, e2, _ = gen.append_slivers(coords, elems, 64, h)
    fb = lib.fallback(1e-3 * h ** 3, 1e6, True)
    got = _gpu_quad(lib, c2, e2, torch.float32, 2, fb=fb)
    assert got["ctr"][0] == 64
    q = oracle.p1_elements_q(c2, e2, 2, got["cq"], got["cq"])
    ref = oracle.assemble(e2, c2.shape[0], q["Ke"], q["Me"], q["Kabs"])
    within(got["valK"], ref["valK"], ref["scaleK"], TOL[torch.float32], "K")
    within(got["valM"], ref["valM"], ref["scaleM"], TOL[torch.float32], "M")
