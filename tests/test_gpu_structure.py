"""The structure handle's device memory and stream semantics: the resident arrays of a built
structure match their closed-form sizes (the CSR pattern, the compact node-to-element
adjacency with one slot word per entry, the diagonal positions), no build scratch outlives
the build, and a structure whose last build phase is still in flight on one stream is used
correctly by calls on another stream."""
import numpy as np
import pytest
import torch

from helpers import cube, dev, host, say, square

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2404_16039_amd import lib as L
    return L


def _part(b):
    """bytes of one 256-byte aligned part of a pooled block"""
    return (max(b, 1) + 255) // 256 * 256


@pytest.mark.parametrize("dim,n,p2", [(3, 24, False), (2, 64, False), (3, 6, True), (2, 9, True)])
def test_resident_memory_closed_form(lib, dim, n, p2):
    say("structure memory", dim, n, p2)
    from paper_2404_16039_amd import gen
    coords, elems, _ = cube(n) if dim == 3 else square(n)
    nn = coords.shape[0]
    if p2:
        coords, elems, _ = gen.p2_mesh(coords, elems)
        nn = coords.shape[0]
    te = dev(elems)
    csr = lib.Csr()
    (csr.symbolic_p2 if p2 else csr.symbolic)(dim, nn, te)
    _, nnz, _, _ = csr.info()
    m = elems.shape[0] * elems.shape[1]
    res, scr = csr.memory()
    nb = max(-(-(nn + 1) // 2048), 1)
    want = 3 * _part(4 * (nn + 1)) + _part(4 * m) + _part((8 if p2 else 4) * m) + _part(8 * nb) + _part(8 * 16)
    want += 0 if p2 else _part(4 * -(-nn // 4))  # routed counts of the FP32 numeric blocks
    want += 4 * nnz  # col_idx, exactly nnz words
    assert scr == 0 and res == want, (res, want)
    # the pattern and the adjacency: at most 12 (nn + 1) + 4 nnz + (8 or 12) m bytes plus alignment
    csr_bytes = 4 * (nn + 1) + 4 * nnz
    assert res <= csr_bytes + 9 * (nn + 1) + (12 if p2 else 8) * m + 8 * 256 + 8 * nb + 128
    csr.close()


def test_full_size_memory_ratio(lib):
    """128^3 Kuhn cube: the resident structure is within 4.12x the CSR pattern's bytes (was
    about 16x with padded adjacency rows and columns; 4.107x with the numeric blocks' routed
    counts, one int per 4 rows)."""
    say("structure memory 128^3")
    from paper_2404_16039_amd import gen
    coords, elems, _ = gen.cube_mesh(128, jitter=0.15, with_faces=False)
    csr = lib.Csr().symbolic(3, coords.shape[0], dev(elems))
    nn, nnz, _, _ = csr.info()
    res, scr = csr.memory()
    assert scr == 0
    ratio = res / (4 * (nn + 1) + 4 * nnz)
    assert ratio < 4.12, ratio
    csr.close()


def test_structure_used_on_another_stream(lib):
    """pf_csr_symbolic on stream s1 returns with its column phase in flight; an assembly on
    stream s2 enqueued at once (no host synchronisation) must see the finished structure.
    Three rebuilds in a row, alternating the streams, each checked bitwise against a
    reference assembled after a full synchronisation."""
    say("structure across streams")
    coords, elems, _ = cube(40)
    nn = coords.shape[0]
    tc, te = dev(coords), dev(elems)
    ref = lib.Csr().symbolic(3, nn, te)
    _, nnz, _, _ = ref.info()
    rk = torch.empty(nnz, dtype=torch.float32, device="cuda")
    rm = torch.empty(nnz, dtype=torch.float32, device="cuda")
    ref.assemble(lib.F32, tc, te, rk, rm)
    rk, rm = host(rk), host(rm)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    csr = lib.Csr()
    vk = torch.empty(nnz, dtype=torch.float32, device="cuda")
    vm = torch.empty(nnz, dtype=torch.float32, device="cuda")
    for rep in range(3):
        a, b = (s1, s2) if rep % 2 == 0 else (s2, s1)
        vk.fill_(float("nan"))
        vm.fill_(float("nan"))
        torch.cuda.synchronize()
        csr.symbolic(3, nn, te, stream=a)
        csr.assemble(lib.F32, tc, te, vk, vm, stream=b)
        b.synchronize()
        assert np.array_equal(host(vk), rk) and np.array_equal(host(vm), rm), rep
    # the pattern handed out by info() is complete (info waits for the build's end)
    csr.symbolic(3, nn, te, stream=s1)
    for x, y in zip(csr.structure(), ref.structure()):
        assert torch.equal(x, y)
    csr.close()
    ref.close()
