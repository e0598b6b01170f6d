"""The serving loop (row a14): jobs admitted by a device-memory budget, fused numeric
launches per scheduler tick, resident structures per topology.  A job's values are bitwise
those of the same mesh assembled alone, and match the oracle."""
import numpy as np
import pytest
import torch

import oracle
from helpers import TOL, host, say, within
from paper_2404_16039_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2404_16039_amd import lib as L
    return L


def _mesh(dim, n, sub):
    if dim == 2:
        c, e, _ = gen.square_mesh(n, seed_sub=sub, stream=gen.STREAM_SERVE)
    else:
        c, e, _ = gen.cube_mesh(n, seed_sub=sub, stream=gen.STREAM_SERVE, with_faces=False)
    return c, e


def _alone(L, dim, prec, coords, elems, fb=None):
    """The same mesh through pf_csr_symbolic + pf_assemble on its own."""
    dt = torch.float32 if prec == L.F32 else torch.float64
    csr = L.Csr().symbolic(dim, coords.shape[0], torch.from_numpy(elems).cuda())
    _, nnz, _, _ = csr.info()
    vk = torch.empty(nnz, dtype=dt, device="cuda")
    vm = torch.empty(nnz, dtype=dt, device="cuda")
    csr.assemble(prec, torch.from_numpy(coords).cuda(), None, vk, vm, fb=fb)
    rp, ci = csr.structure()
    out = host(vk), host(vm), host(rp), host(ci)
    csr.close()
    return out


def _outputs(nnz_cap, prec):
    dt = torch.float32 if prec == 0 else torch.float64
    return (torch.full((nnz_cap,), float("nan"), dtype=dt).pin_memory(),
            torch.full((nnz_cap,), float("nan"), dtype=dt).pin_memory())


SPEC = [(2, 1, 12), (3, 0, 5), (3, 0, 4), (2, 1, 20), (3, 1, 3), (2, 0, 7), (3, 0, 9), (2, 1, 1)]


@pytest.mark.parametrize("flags", [0, 1 | 2])
def test_jobs_match_alone_bitwise(lib, flags):
    """Fused (flags 0) and one-launch-per-job without resident structures (flags 3)."""
    say("server identity", flags)
    srv = lib.Server(1 << 30, 16, flags)
    start = srv.now() + 0.05  # every job arrives at the same instant: one tick, fused launches
    tickets = []
    for k, (dim, prec, n) in enumerate(SPEC):
        c, e = _mesh(dim, n, k)
        cap = (gen.square_counts(n) if dim == 2 else gen.kuhn_counts(n))["nnz"]
        vk, vm = _outputs(cap, prec)
        t = srv.submit(dim, prec, torch.from_numpy(c).pin_memory(), torch.from_numpy(e).pin_memory(),
                       topology=1000 + k, arrival=start, valsK=vk, valsM=vm)
        tickets.append((t, dim, prec, c, e, vk, vm, cap))
    srv.drain()
    for t, dim, prec, c, e, vk, vm, cap in tickets:
        r = srv.poll(t)
        assert r["done"] == 1 and r["status"] == 0 and r["nnz"] == cap
        ak, am, _, _ = _alone(lib, dim, prec, c, e)
        assert np.array_equal(vk.numpy(), ak) and np.array_equal(vm.numpy(), am), f"job {t} differs from alone"
        assert r["arrival"] <= r["admitted"] <= r["finished"] <= r["copied"]
    s = srv.stats()
    assert s["completed"] == len(SPEC) and s["failed"] == 0
    if flags == 0:
        assert s["max_batch"] == len(SPEC) and s["launches"] <= 4  # one launch per (dim, prec, rows) class
    else:
        assert s["launches"] == len(SPEC)
    assert s["hbm_in_use"] >= 0 and s["hbm_high_water"] <= 1 << 30
    srv.close()


def test_values_match_oracle(lib):
    say("server oracle")
    srv = lib.Server(1 << 28, 4)
    for dim, prec, n in [(2, lib.F64, 9), (3, lib.F32, 4)]:
        c, e = _mesh(dim, n, 7)
        cap = (gen.square_counts(n) if dim == 2 else gen.kuhn_counts(n))["nnz"]
        vk, vm = _outputs(cap, prec)
        t = srv.submit(dim, prec, torch.from_numpy(c).pin_memory(), torch.from_numpy(e).pin_memory(),
                       valsK=vk, valsM=vm)
        r = srv.wait(t)
        assert r["status"] == 0
        el = oracle.p1_elements(c, e)
        ref = oracle.assemble(e, c.shape[0], el["Ke"], el["Me"], el["Kabs"])
        tol = TOL[torch.float64 if prec == lib.F64 else torch.float32]
        within(vk.numpy(), ref["valK"], ref["scaleK"], tol, "server K")
        within(vm.numpy(), ref["valM"], ref["scaleM"], tol, "server M")
    srv.close()


def test_budget_queueing_and_rejection(lib):
    """A budget that holds about two jobs: all ten finish, in turn, under the budget; a job
    that can never fit is refused at submission."""
    say("server budget")
    c, e = _mesh(3, 8, 1)
    budget = int(2.5 * lib.server_footprint(3, lib.F32, c.shape[0], e.shape[0]))
    srv = lib.Server(budget, 64)
    with pytest.raises(lib.PagefemError) as ei:
        big_c, big_e = _mesh(3, 20, 2)
        srv.submit(3, lib.F32, big_c, big_e)
    assert ei.value.code == 8
    tc, te = torch.from_numpy(c).pin_memory(), torch.from_numpy(e).pin_memory()
    ts = [srv.submit(3, lib.F32, tc, te) for _ in range(10)]
    srv.drain()
    for t in ts:
        r = srv.poll(t)
        assert r["done"] == 1 and r["status"] == 0
    s = srv.stats()
    assert s["completed"] == 10 and s["hbm_high_water"] <= budget and s["hbm_in_use"] == 0
    assert s["max_batch"] < 10  # the budget split the jobs over several ticks
    srv.close()


def test_resident_structures(lib):
    """Jobs of one topology share its structure (one miss, then hits) and still get their
    own values; a small budget evicts idle structures."""
    say("server cache")
    srv = lib.Server(1 << 28, 8)
    outs = []
    for k in range(4):
        c, e = _mesh(3, 6, 50 + k)  # same connectivity, different jitter
        cap = gen.kuhn_counts(6)["nnz"]
        vk, vm = _outputs(cap, 0)
        t = srv.submit(3, lib.F32, torch.from_numpy(c).pin_memory(), torch.from_numpy(e).pin_memory(),
                       topology=77, valsK=vk, valsM=vm)
        srv.wait(t)
        outs.append((c, e, vk, vm))
    s = srv.stats()
    assert s["cache_misses"] == 1 and s["cache_hits"] == 3
    for c, e, vk, vm in outs:
        ak, am, _, _ = _alone(lib, 3, lib.F32, c, e)
        assert np.array_equal(vk.numpy(), ak) and np.array_equal(vm.numpy(), am)
    assert not np.array_equal(outs[0][2].numpy(), outs[1][2].numpy())
    srv.close()
    # eviction: two topologies that do not fit together
    c1, e1 = _mesh(3, 10, 1)
    c2, e2 = _mesh(3, 11, 2)
    # room for one new job, not for a resident structure next to it
    budget = lib.server_footprint(3, lib.F32, c2.shape[0], e2.shape[0]) + 65536
    srv = lib.Server(budget, 8)
    for k in range(3):
        srv.wait(srv.submit(3, lib.F32, c1, e1, topology=1))
        srv.wait(srv.submit(3, lib.F32, c2, e2, topology=2))
    s = srv.stats()
    assert s["completed"] == 6 and s["evictions"] >= 1 and s["hbm_high_water"] <= budget
    srv.close()


def test_job_errors_do_not_stop_the_server(lib):
    say("server errors")
    srv = lib.Server(1 << 28, 4)
    c, e = _mesh(2, 6, 3)
    with pytest.raises(lib.PagefemError) as ei:
        srv.submit(4, lib.F32, c, e)
    assert ei.value.code == 3
    small = torch.empty(10, dtype=torch.float64).pin_memory()
    t = srv.submit(2, lib.F64, c, e, valsK=small)  # vals_cap below nnz
    r = srv.wait(t)
    assert r["done"] == 1 and r["status"] == 7
    bad = e.copy()
    bad[3, 1] = 10 ** 6  # out-of-range node id
    r = srv.wait(srv.submit(2, lib.F64, c, bad))
    assert r["status"] == 6
    r = srv.wait(srv.submit(2, lib.F64, c, e))
    assert r["status"] == 0
    with pytest.raises(lib.PagefemError):
        srv.poll(12345)
    s = srv.stats()
    assert s["failed"] == 2 and s["completed"] == 1
    srv.close()


def test_poisson_trace(lib):
    """A short Poisson trace (200 jobs/s, small meshes) submitted at its arrival times."""
    import time
    trace = gen.serving_trace(60, rate=200.0, hi=3e4)
    say("server trace", len(trace))
    srv = lib.Server(1 << 30, 64)
    meshes = {}
    for j in trace:
        c, e = _mesh(j["dim"], j["n"], j["id"])
        meshes[j["id"]] = (torch.from_numpy(c).pin_memory(), torch.from_numpy(e).pin_memory())
    t0 = srv.now() + 0.01
    ts = []
    for j in trace:
        while srv.now() < t0 + j["t"]:
            time.sleep(0.0002)
        c, e = meshes[j["id"]]
        prec = lib.F64 if j["dim"] == 2 else lib.F32
        ts.append(srv.submit(j["dim"], prec, c, e, topology=(j["dim"] << 32) | j["n"], arrival=t0 + j["t"]))
    srv.drain()
    s = srv.stats()
    assert s["completed"] == len(trace) and s["failed"] == 0
    assert 0 < s["latency_p50"] <= s["latency_p99"] <= s["latency_max"]
    assert s["jobs_per_s"] > 0 and s["elements"] == sum(m[1].shape[0] for m in meshes.values())
    srv.close()


# page-op jobs: (prec, order, ops, count)
PAGE_SPEC = [(0, 3, 3, 5000), (1, 2, 1, 777), (0, 4, 2, 1234), (1, 3, 3, 3000), (0, 1, 3, 99), (1, 4, 3, 2500)]


def _page_job_arrays(prec, n, ops, count, sub):
    dt = np.float32 if prec == 0 else np.float64
    a = gen.page_batch(count, n, sub=sub).astype(dt)
    b = gen.page_batch(count, n, stream=gen.STREAM_PAGES_B, sub=sub).astype(dt)
    x = np.full((count, n * n), np.nan, dtype=dt) if ops & 1 else None
    c = np.full((count, n * n), np.nan, dtype=dt) if ops & 2 else None
    d = np.full(count, np.nan, dtype=dt) if ops & 1 else None
    return a, (b if ops & 2 else None), x, c, d


def _submit_pages(srv, spec, sub, arrival=-1.0):
    prec, n, ops, count = spec
    a, b, x, c, d = _page_job_arrays(prec, n, ops, count, sub)
    t = srv.submit_pages(prec, n, ops, a, b=b, x=x, c=c, det=d, arrival=arrival)
    return t, (a, b, x, c, d)


@pytest.mark.parametrize("flags", [0, 1])
def test_page_jobs_alone_and_in_a_mix(lib, flags):
    """Page-op jobs (inverse with determinant, product; orders 1..4, FP32 and FP64) submitted
    together with assembly jobs, all arriving in one tick: each page job's results are bitwise
    those of the same job through a server of its own, and match the oracle."""
    say("server page jobs", flags)
    srv = lib.Server(1 << 30, 32, flags)
    nasm = (len(PAGE_SPEC) + 1) // 2
    meshes = {}
    for k in range(0, len(PAGE_SPEC), 2):  # the assembly jobs' structures, built beforehand
        dim, prec, n = SPEC[k]
        c, e = _mesh(dim, n, k)
        meshes[k] = (torch.from_numpy(c).pin_memory(), torch.from_numpy(e).pin_memory())
        srv.wait(srv.submit(dim, prec, *meshes[k], topology=2000 + k))
    warm = srv.stats()["launches"]
    start = srv.now() + 0.05
    mixed = []
    for k, sp in enumerate(PAGE_SPEC):
        mixed.append((sp, k) + _submit_pages(srv, sp, 300 + k, arrival=start))
        if k % 2 == 0:  # assembly jobs in the same tick
            dim, prec, n = SPEC[k]
            srv.submit(dim, prec, *meshes[k], topology=2000 + k, arrival=start)
    srv.drain()
    s = srv.stats()
    assert s["failed"] == 0 and s["completed"] == len(PAGE_SPEC) + 2 * nasm
    assert s["pages"] == sum(sp[3] for sp in PAGE_SPEC)
    if flags == 0:  # one batch-plan launch per precision, plus the numeric classes
        assert s["max_batch"] == len(PAGE_SPEC) + nasm and s["launches"] - warm <= 2 + 4
    srv.close()
    for sp, k, t, (a, b, x, c, d) in mixed:
        prec, n, ops, count = sp
        alone = lib.Server(1 << 28, 2, flags)
        t2, (a2, b2, x2, c2, d2) = _submit_pages(alone, sp, 300 + k)
        r = alone.wait(t2)
        assert r["status"] == 0 and r["routed"] == -1 and r["nnz"] == 0
        alone.close()
        for got, ref in ((x, x2), (c, c2), (d, d2)):
            if got is not None:
                assert np.array_equal(got, ref), f"page job {k} differs from alone"
        tol = TOL[torch.float32 if prec == 0 else torch.float64]
        a64 = a.astype(np.float64)
        if ops & 1:
            inv, sing, sc = oracle.page_inv(a64, n)
            assert not sing.any()
            within(x, inv, sc, tol, f"page job {k} inverse")
            det, perm = oracle.page_det(a64, n)
            within(d, det, perm, tol, f"page job {k} det")
        if ops & 2:
            cm, ab = oracle.page_mtimes(a64, b.astype(np.float64), n, n, n)
            within(c, cm, ab, tol, f"page job {k} product")


def test_shared_new_structure_built_once(lib):
    """Jobs of one new topology arriving in one tick share one structure build (one miss,
    the others hits) and get their own values; a build that fails (bad node id) fails every
    job that shares it, and the server goes on."""
    say("server shared build")
    srv = lib.Server(1 << 29, 16)
    start = srv.now() + 0.05
    jobs = []
    for k in range(3):
        c, e = _mesh(3, 7, 400 + k)  # one connectivity, three jitters
        cap = gen.kuhn_counts(7)["nnz"]
        vk, vm = _outputs(cap, 0)
        t = srv.submit(3, lib.F32, torch.from_numpy(c).pin_memory(), torch.from_numpy(e).pin_memory(),
                       topology=555, arrival=start, valsK=vk, valsM=vm)
        jobs.append((t, c, e, vk, vm))
    c2, e2 = _mesh(2, 5, 9)
    bad = e2.copy()
    bad[2, 0] = -5
    fails = [srv.submit(2, lib.F64, c2, bad, topology=666, arrival=start) for _ in range(2)]
    srv.drain()
    s = srv.stats()
    assert s["cache_misses"] == 2 and s["cache_hits"] == 3, s
    assert s["completed"] == 3 and s["failed"] == 2
    for t, c, e, vk, vm in jobs:
        assert srv.poll(t)["status"] == 0
        ak, am, _, _ = _alone(lib, 3, lib.F32, c, e)
        assert np.array_equal(vk.numpy(), ak) and np.array_equal(vm.numpy(), am)
    for t in fails:
        assert srv.poll(t)["status"] == 6
    r = srv.wait(srv.submit(2, lib.F64, c2, e2, topology=666))  # the key builds again, correctly
    assert r["status"] == 0
    srv.close()
