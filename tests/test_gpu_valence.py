"""sparse() (section 3.6) of meshes with high-valence nodes: a node in 30 to 63 elements and
rows of up to 64 nonzeros, every entry against the oracle, in FP32 and FP64, with constant,
per-element and integration-point coefficients.  These meshes take the numeric kernel's
workgroup shapes for long adjacency lists (the launch shape is read back and checked), and
fill the row-pattern tables up to their capacity."""
import numpy as np
import pytest
import torch

import oracle
from helpers import TOL, counters, dev, host, prec_of, say, within
from paper_2404_16039_amd import gen

pytestmark = pytest.mark.gpu

# (name, builder): fans joined to a small structured block (a second component with
# ordinary valence, so both kinds of rows share the launch)
MESHES = {
    "fan2_30+square": lambda: gen.join_meshes(gen.fan_mesh(2, 30, 1), gen.square_mesh(4)[:2]),
    "fan2_63": lambda: gen.fan_mesh(2, 63, 2),
    "fan3_30+cube": lambda: gen.join_meshes(gen.fan_mesh(3, 30, 3), gen.cube_mesh(3)[:2]),
    "fan3_44": lambda: gen.fan_mesh(3, 44, 4),
    "fan3_60+cube": lambda: gen.join_meshes(gen.cube_mesh(2)[:2], gen.fan_mesh(3, 60, 5)),
    "fan3_62": lambda: gen.fan_mesh(3, 62, 6),
}


def expected_rows_per_block(max_adj, dtype):
    """workgroup shape of the numeric kernel for the longest adjacency list: FP64 blocks of
    256 threads take 32 rows (24 elements per node), 16 rows (48) or 4 rows (any admissible
    list); FP32 blocks of 128 threads take 16, 8 or 4 rows (8, 16 or 32 threads per row,
    three entries each: 24, 48 or 96 elements per node)"""
    if dtype == torch.float64:
        return 32 if max_adj <= 24 else (16 if max_adj <= 48 else 4)
    return 16 if max_adj <= 24 else (8 if max_adj <= 48 else 4)


@pytest.fixture(scope="module")
def lib():
    from paper_2404_16039_amd import lib as L
    return L


def _coef(ne, nq, dtype, seed):
    g = np.random.default_rng(seed)
    c = g.uniform(0.5, 2.0, (ne, nq)) if nq else g.uniform(0.5, 2.0, ne)
    if dtype == torch.float32:
        c = c.astype(np.float32).astype(np.float64)
    return c


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("coef", ["none", "element", "quad2"])
@pytest.mark.parametrize("name", list(MESHES))
def test_high_valence_assembly(lib, name, coef, dtype):
    coords, elems = MESHES[name]()
    dim = coords.shape[1]
    nn, ne = coords.shape[0], elems.shape[0]
    say("high valence", name, coef, dtype)
    tc, te = dev(coords), dev(elems)
    csr = lib.Csr().symbolic(dim, nn, te)
    _, nnz, _, _ = csr.info()
    counts = np.bincount(elems.ravel(), minlength=nn)
    rows, madj = csr.numeric_info(prec_of(dtype))
    assert madj == counts.max()
    assert rows == expected_rows_per_block(madj, dtype), (rows, madj)
    vk = torch.empty(nnz, dtype=dtype, device="cuda")
    vm = torch.empty(nnz, dtype=dtype, device="cuda")
    ctr = counters()
    if coef == "quad2":
        nq = dim + 1
        cKq, cMq = _coef(ne, nq, dtype, 7), _coef(ne, nq, dtype, 8)
        csr.assemble_quad(prec_of(dtype), tc, 2, vk, vm, cKq=dev(cKq, dtype), cMq=dev(cMq, dtype), counters=ctr)
        q = oracle.p1_elements_q(coords, elems, 2, cKq, cMq)
        ref = oracle.assemble(elems, nn, q["Ke"], q["Me"], q["Kabs"])
    else:
        el = oracle.p1_elements(coords, elems)
        Ke, Me, Ka = el["Ke"], el["Me"], el["Kabs"]
        if coef == "element":
            cK, cM = _coef(ne, 0, dtype, 7), _coef(ne, 0, dtype, 8)
            csr.assemble(prec_of(dtype), tc, te, vk, vm, cK=dev(cK, dtype), cM=dev(cM, dtype), counters=ctr)
            Ke, Ka, Me = Ke * cK[:, None], Ka * cK[:, None], Me * cM[:, None]
        else:
            csr.assemble(prec_of(dtype), tc, te, vk, vm, counters=ctr)
        ref = oracle.assemble(elems, nn, Ke, Me, Ka)
    rp, ci = csr.structure()
    assert nnz == ref["nnz"]
    assert np.array_equal(host(rp).astype(np.int64), ref["row_ptr"])
    assert np.array_equal(host(ci), ref["col_idx"])
    assert np.diff(ref["row_ptr"]).max() == counts.max() + (dim - 1)  # the hub rows: hub, axis partner, rim
    within(host(vk), ref["valK"], ref["scaleK"], TOL[dtype], "K values")
    within(host(vm), ref["valM"], ref["scaleM"], TOL[dtype], "M values")
    assert host(ctr)[2] == 0
    csr.close()


def test_launch_shapes_cover_every_variant(lib):
    """the meshes above reach every numeric workgroup shape (together with the Kuhn cube)"""
    seen = set()
    for name, build in list(MESHES.items()) + [("cube3", lambda: gen.cube_mesh(3)[:2])]:
        coords, elems = build()
        say("launch shape", name)
        csr = lib.Csr().symbolic(coords.shape[1], coords.shape[0], dev(elems))
        for p in (0, 1):
            seen.add((p, csr.numeric_info(p)[0]))
        csr.close()
    assert seen == {(1, 32), (1, 16), (1, 4), (0, 16), (0, 8), (0, 4)}, seen
