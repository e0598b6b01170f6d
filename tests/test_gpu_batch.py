"""Parity of the mixed-order batch plans (page-wise inverse with determinant of section
2.3 and page-wise product of section 2.2, many groups of orders 1..4 in one persistent launch) against the
oracle, under every schedule, through the graph replay path, and at the 64-group
uneven-batch size (about 9.3 million pages) on sampled pages."""
import json

import numpy as np
import pytest
import torch

import oracle
from helpers import TOL, counters, host, say, within
from paper_2404_16039_amd import gen

pytestmark = pytest.mark.gpu

# (order, count, ops, misaligned by one element)
SPEC = [(1, 37, 3, 0), (2, 1000, 3, 1), (3, 777, 3, 0), (4, 513, 3, 1), (2, 0, 3, 0), (3, 1, 1, 0),
        (4, 300, 2, 0), (3, 327, 3, 1), (2, 65, 1, 1), (4, 1, 3, 0)]


@pytest.fixture(scope="module")
def lib():
    from paper_2404_16039_amd import lib as L
    return L


def _buf(host_pages, dtype, shift):
    """Device copy of flat pages, `shift` elements into a fresh buffer (misaligned views)."""
    flat = torch.from_numpy(np.ascontiguousarray(host_pages).reshape(-1)).to(dtype)
    t = torch.zeros(flat.numel() + shift, dtype=dtype, device="cuda")
    t[shift:] = flat.cuda()
    return t[shift:]


def _make(L, dtype, spec=SPEC, seed=0, a_override=None):
    groups = []
    for gi, (n, count, ops, mis) in enumerate(spec):
        a = gen.page_batch(count, n, sub=1000 * seed + gi)
        b = gen.page_batch(count, n, stream=gen.STREAM_PAGES_B, sub=1000 * seed + gi)
        if a_override is not None and gi in a_override:
            a = a_override[gi]
        if dtype == torch.float32:
            a = a.astype(np.float32).astype(np.float64)
            b = b.astype(np.float32).astype(np.float64)
        nn = n * n
        g = {"order": n, "ops": ops, "count": count, "ha": a, "hb": b, "a": _buf(a, dtype, mis)}
        if ops & L.OP_MTIMES:
            g["b"] = _buf(b, dtype, mis)
            g["c"] = _buf(np.full((count, nn), np.nan), dtype, 1 - mis)
        if ops & L.OP_INV:
            g["x"] = _buf(np.full((count, nn), np.nan), dtype, mis)
            g["det"] = torch.full((count,), float("nan"), dtype=dtype, device="cuda")
        groups.append(g)
    return groups


def _check(groups, dtype, what):
    tol = TOL[dtype]
    for gi, g in enumerate(groups):
        n, count = g["order"], g["count"]
        if count == 0:
            continue
        if "x" in g:
            inv, sing, sc = oracle.page_inv(g["ha"], n)
            within(host(g["x"]).reshape(count, n * n), inv, sc, tol, f"{what} group {gi} inv")
            d, perm = oracle.page_det(g["ha"], n)
            within(host(g["det"]), d, perm, tol, f"{what} group {gi} det")
        if "c" in g:
            c, absc = oracle.page_mtimes(g["ha"], g["hb"], n, n, n)
            within(host(g["c"]).reshape(count, n * n), c, absc, tol, f"{what} group {gi} product")


def _schedules(L, waves_set=(1, 4, 8)):
    for waves in waves_set:
        for li in range(3):
            for staged in (0, 1):
                for tile in (1, 3):
                    per = {n: ([1, n, n * n][li], staged, tile) for n in range(1, 5)}
                    yield waves, li, staged, tile, per


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_every_schedule_matches_oracle(lib, dtype):
    """All lane mappings x staging x tile sizes x wave counts on ragged, misaligned groups;
    the products are bitwise the same under every schedule."""
    prec = lib.F32 if dtype == torch.float32 else lib.F64
    groups = _make(lib, dtype)
    plan = lib.Plan(prec, 16).set_groups(groups)
    ref_c = None
    ran = 0
    for waves, li, staged, tile, per in _schedules(lib):
        try:
            plan.set_schedule(waves, per)
        except lib.PagefemError as e:
            assert e.code == 1 and "LDS" in str(e)  # a staging buffer beyond one workgroup's LDS
            continue
        say("plan schedule", dtype, waves, li, staged, tile)
        for g in groups:
            if "x" in g:
                g["x"].fill_(float("nan"))
            if "c" in g:
                g["c"].fill_(float("nan"))
        ctr = counters()
        plan.launch(counters=ctr)
        _check(groups, dtype, f"waves {waves} lanes#{li} staged {staged} tile {tile}")
        cs = [g["c"].clone() for g in groups if "c" in g]
        if ref_c is None:
            ref_c = cs
        else:
            assert all(torch.equal(p, q) for p, q in zip(cs, ref_c)), "products differ between schedules"
        assert int(host(ctr)[1]) == 0
        ran += 1
    assert ran >= 30
    plan.close()


def _hard_pages(count, n, rng):
    """FP32 pages whose det-condition is far above 1e6 (row 1 = row 0 except one entry one
    ulp away) and exactly singular integer pages (a repeated column, first row non-zero),
    mixed with ordinary ones."""
    a = gen.page_batch(count, n, sub=77 + n).astype(np.float32)
    near = np.arange(2, count, 9)
    sing = np.arange(5, count, 9)
    for idx in near:
        m = (rng.standard_normal((n, n)) + 3 * np.eye(n)).astype(np.float32)
        m[1] = m[0]
        m[1, 0] = np.nextafter(m[0, 0], np.float32(np.inf))
        a[idx] = m.T.reshape(-1)
    for idx in sing:
        m = rng.integers(-4, 5, size=(n, n)).astype(np.float32)
        m[0, 0] = 1 + abs(m[0, 0])
        m[:, n - 1] = m[:, 0]
        a[idx] = m.T.reshape(-1)
    return a.astype(np.float64), near, sing


def test_fp32_routing_and_singular_pages(lib):
    rng = np.random.default_rng(5)
    spec = [(2, 300, 3, 0), (3, 400, 3, 1), (4, 350, 3, 0)]
    hard = {}
    nsing = 0
    near_idx, sing_idx = {}, {}
    for gi, (n, count, _, _) in enumerate(spec):
        hard[gi], near_idx[gi], sing_idx[gi] = _hard_pages(count, n, rng)
        nsing += len(sing_idx[gi])
    groups = _make(lib, torch.float32, spec=spec, a_override=hard)
    plan = lib.Plan(lib.F32, 4, lib.fallback(0.0, 1e6, True)).set_groups(groups)
    for waves, li, staged, tile, per in _schedules(lib, waves_set=(4,)):
        plan.set_schedule(waves, per)
        say("plan routing", li, staged, tile)
        ctr = counters()
        plan.launch(counters=ctr)
        c = host(ctr)
        assert int(c[1]) == nsing
        routed_expected = 0
        for gi, g in enumerate(groups):
            n, count = g["order"], g["count"]
            r_or, cond = oracle.route_predicate(g["ha"], n, 0.0, 1e6)
            assert r_or[near_idx[gi]].mean() > 0.8  # the construction does reach the FP64 path
            routed_expected += int(r_or.sum())
            inv, _, sc = oracle.page_inv(g["ha"], n)
            sing = np.zeros(count, bool)
            sing[sing_idx[gi]] = True  # exactly singular by construction
            x = host(g["x"]).reshape(count, -1)
            within(x[~sing], inv[~sing], sc[~sing], TOL[torch.float32], f"group {gi} inv")
            assert not np.isfinite(x[sing]).all(axis=1).any()
            d, perm = oracle.page_det(g["ha"], n)
            within(host(g["det"]), d, perm, TOL[torch.float32], f"group {gi} det")
        assert int(c[0]) == routed_expected
    plan.close()


def test_graph_replay_matches_eager(lib):
    """Replays of the captured graph, with eager work and new inputs in between, give the
    eager launch's bits every time; new group pointers need no new capture."""
    groups = _make(lib, torch.float32, seed=3)
    plan = lib.Plan(lib.F32, 16).set_groups(groups)
    outs = lambda: [g[k].clone() for g in groups for k in ("x", "c", "det") if k in g]  # noqa: E731
    for rep in range(4):
        say("graph replay", rep)
        for g in groups:
            if g["count"]:
                g["a"].mul_(1.0 + 0.125 * rep)  # eager work on the inputs between replays
        plan.launch()
        eager = outs()
        for g in groups:
            for k in ("x", "c"):
                if k in g:
                    g[k].zero_()
        plan.run()
        torch.cuda.synchronize()
        got = outs()
        assert all(torch.equal(p, q) for p, q in zip(got, eager)), f"replay {rep} differs from eager"
    # new tensors for the same shapes: the graph copies the new work list on replay
    g2 = _make(lib, torch.float32, seed=4)
    plan.set_groups(g2)
    plan.run()
    torch.cuda.synchronize()
    _check(g2, torch.float32, "replay after set_groups")
    plan.close()


def test_group_validation(lib):
    say("plan validation")
    plan = lib.Plan(lib.F32, 2)
    a = torch.zeros(64, device="cuda")
    with pytest.raises(lib.PagefemError) as e:
        plan.set_groups([{"order": 5, "ops": 1, "count": 1, "a": a, "x": a}])
    assert e.value.code == 3
    with pytest.raises(lib.PagefemError) as e:
        plan.set_groups([{"order": 2, "ops": 3, "count": 2, "a": a, "x": a}])  # no b, c
    assert e.value.code == 1
    with pytest.raises(lib.PagefemError) as e:
        plan.set_groups([{"order": 2, "ops": 9, "count": 2, "a": a, "x": a}])
    assert e.value.code == 1
    with pytest.raises(lib.PagefemError) as e:
        plan.set_groups([{"order": 2, "ops": 1, "count": 1, "a": a, "x": a}] * 3)  # above max_groups
    assert e.value.code == 1
    with pytest.raises(lib.PagefemError) as e:
        plan.set_schedule(3, {})
    assert e.value.code == 1
    with pytest.raises(lib.PagefemError) as e:
        plan.set_schedule(4, {3: (2, 1, 1)})  # lanes must be 1, n or n*n
    assert e.value.code == 1
    plan.set_groups([])
    plan.run()  # an empty plan is a no-op
    torch.cuda.synchronize()
    plan.close()


def test_tuner_and_cache(lib, tmp_path):
    groups = _make(lib, torch.float32, seed=6)
    plan = lib.Plan(lib.F32, 16).set_groups(groups)
    cache = tmp_path / "tune.json"
    say("tuner force")
    s1 = plan.tune(str(cache), lib.TUNE_FORCE).as_dict()
    data = json.loads(cache.read_text())
    assert any("|f32|waves|" in k for k in data) and any("|n4|" in k for k in data)
    before = cache.read_text()
    say("tuner cached")
    s2 = plan.tune(str(cache), lib.TUNE_CACHED).as_dict()
    assert s1 == s2 and cache.read_text() == before
    plan.run()
    torch.cuda.synchronize()
    _check(groups, torch.float32, "tuned")
    assert plan.tune(None, lib.TUNE_DEFAULT).as_dict()["waves"] == 4
    plan.close()


def test_uneven_batch_full_size(lib):
    """64 groups, orders uniform in {2,3,4}, sizes 10^U(3,6) (about 9.3 million pages):
    tuned plan replayed from its graph against the oracle on sampled pages and against the
    one-launch-per-group page operations on every page."""
    spec = gen.mixed_groups(64)
    total = sum(c for _, c in spec)
    say("uneven batch", total)
    rng = np.random.default_rng(9)
    groups, host_in = [], []
    for gi, (n, count) in enumerate(spec):
        a = gen.page_batch(count, n, sub=gi).astype(np.float32)
        b = gen.page_batch(count, n, stream=gen.STREAM_PAGES_B, sub=gi).astype(np.float32)
        ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        groups.append({"order": n, "ops": 3, "a": ta, "b": tb, "x": torch.empty_like(ta),
                       "c": torch.empty_like(ta), "det": torch.empty(count, device="cuda")})
        pick = np.unique(np.concatenate([rng.choice(count, min(count, 200), replace=False), [0, count - 1]]))
        host_in.append((pick, a[pick].astype(np.float64), b[pick].astype(np.float64)))
    fb = lib.fallback(0.0, 1e6, True)
    plan = lib.Plan(lib.F32, 64, fb).set_groups(groups)
    plan.tune(None, lib.TUNE_FORCE)
    ctr = counters()
    plan.run(counters=ctr)
    torch.cuda.synchronize()
    for gi, (g, (pick, a, b)) in enumerate(zip(groups, host_in)):
        n = g["order"]
        x = host(g["x"])[pick].astype(np.float64)
        inv, sing, sc = oracle.page_inv(a, n)
        within(x, inv, sc, TOL[torch.float32], f"group {gi} inv")
        d, perm = oracle.page_det(a, n)
        within(host(g["det"])[pick], d, perm, TOL[torch.float32], f"group {gi} det")
        c, absc = oracle.page_mtimes(a, b, n, n, n)
        within(host(g["c"])[pick], c, absc, TOL[torch.float32], f"group {gi} product")
    # the plain form: one pf_page_inv and one pf_page_mtimes launch per group; products
    # are bitwise equal, inverses agree within twice the tolerance of |X||A||X|
    routed = 0
    for gi, g in enumerate(groups):
        n, count = g["order"], g["a"].shape[0]
        P = lib.pages(count, n, n)
        x2, c2, d2 = torch.empty_like(g["x"]), torch.empty_like(g["c"]), torch.empty_like(g["det"])
        ctr2 = counters()
        lib.page_inv(P, g["a"], P, x2, det=d2, fb=fb, counters=ctr2)
        lib.page_mtimes(P, g["a"], 0, P, g["b"], 0, P, c2)
        routed += int(host(ctr2)[0])
        assert torch.equal(c2, g["c"]), f"group {gi}: products differ from pf_page_mtimes"
        xa = host(x2).astype(np.float64).reshape(count, n, n)
        xb = host(g["x"]).astype(np.float64).reshape(count, n, n)
        am = host(g["a"]).astype(np.float64).reshape(count, n, n)
        # pages are column-major: entry (r, c) at [c, r]; |X||A||X| in that storage order
        sc = np.abs(xa) @ np.abs(am) @ np.abs(xa)
        assert np.all(np.abs(xa - xb) <= 2 * TOL[torch.float32] * sc), f"group {gi}: inverse vs pf_page_inv"
    assert int(host(ctr)[0]) == routed
    plan.close()
