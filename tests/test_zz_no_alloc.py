"""pf_energies_noalloc (block sums in the library's static per-device array) against
pf_energies (block sums in a workspace of the handle): the same kernels, so the local energy
parts J and their FP64 totals must agree bit for bit.  Two calls in a row on one device, the
second on a smaller mesh, so a stale block sum left by the first call in the shared array
would change the second call's totals."""
import numpy as np
import pytest
import torch

from helpers import cube, dev, host, prec_of, say, square

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2404_16039_amd import lib as L
    return L


def _inputs(coords, elems, dtype, seed):
    rng = np.random.default_rng(seed)
    ne, nq = elems.shape[0], (4 if coords.shape[1] == 3 else 3)
    u = rng.standard_normal(coords.shape[0])
    cK = 1.0 + rng.random((ne, nq))
    cM = 0.5 + rng.random((ne, nq))
    return dev(u, dtype), dev(cK, dtype), dev(cM, dtype)


def _both(L, coords, elems, dtype, seed):
    """J and totals from both entry points on the same inputs (the b2D part left out)."""
    dim = coords.shape[1]
    tc, te = dev(coords), dev(elems)
    csr = L.Csr().symbolic(dim, coords.shape[0], te)
    u, cK, cM = _inputs(coords, elems, dtype, seed)
    p = prec_of(dtype)
    ne = elems.shape[0]
    out = []
    for call in (csr.energies, csr.energies_noalloc):
        J = torch.full((3 * ne,), float("nan"), dtype=dtype, device="cuda")
        tot = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        call(p, tc, te, 2, u, cKq=cK, cMq=cM, J=J, totals=tot)
        out.append((host(J), host(tot)))
    csr.close()
    return out


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_matches_workspace_entry_point(lib, dtype):
    # first call: 48^3 cubes (663,552 tets: the energy kernel's full 2048 blocks fill the
    # static array); second call: 6^3 cubes (1,296 tets, 6 blocks)
    for n in (48, 6):
        say("energies_noalloc cube", n, dtype)
        coords, elems, _ = cube(n)
        (J0, t0), (J1, t1) = _both(lib, coords, elems, dtype, seed=100 + n)
        assert np.all(np.isfinite(J0)) and np.all(np.isfinite(t0))
        assert np.array_equal(J0, J1), f"J differs at n={n}"
        assert np.array_equal(t0, t1), f"totals differ at n={n}: {t0} vs {t1}"
    # and a 2-D mesh after them (3 blocks)
    say("energies_noalloc square 40", dtype)
    coords, elems, _ = square(40)
    (J0, t0), (J1, t1) = _both(lib, coords, elems, dtype, seed=7)
    assert np.array_equal(J0, J1) and np.array_equal(t0, t1)


def test_noalloc_rejects_unbuilt_handle(lib):
    csr = lib.Csr()
    with pytest.raises(lib.PagefemError):
        csr.energies_noalloc(lib.F32, None, None, 2, None)
    csr.close()
