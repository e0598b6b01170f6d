#!/usr/bin/env python3
"""Benchmark: P1 tetrahedral stiffness + mass assembly on one MI355X.

Workload (one step = the whole hot path over one mesh, inputs resident in HBM):
  unit cube cut into 128^3 cubes, 6 Kuhn tetrahedra each (12,582,912 tets, 2,146,689
  nodes), interior nodes jittered uniformly by +-0.15 h (seeded), FP64 coordinates, FP32
  arithmetic and values with FP64 recomputation of elements whose det is below 1e-3 h^3:
    1. CSR structure of the mesh (node->element adjacency, row pattern; symbolic phase)
    2. numeric assembly of K and M (per-element geometry, stiffness and mass in registers,
       deterministic row-wise sums into the CSR values)
    3. boundary triangle normals and areas (196,608 faces)
Prints one JSON line: the metric and its value, the step time, per-phase and per-kernel
times, the roofline of the dominant kernel and the CPU oracle's rate on the same work.

Other workloads (one JSON line each, same contract):
  --workload pages   page operations on 1e7 random 3x3 pages (N(0,1) + 3 I), FP64 and FP32,
                     paper layout and structure-of-arrays: det, inv + det, transpose,
                     mat-vec, mat-mat
  --workload batch   64 groups of pages of orders 2..4, sizes 10^U(3,6) (about 9.3 million
                     pages), FP32 inverse + product per group in one persistent launch
                     replayed from a HIP graph, against one launch per group and operation
  --workload energy  load vector (local vectors + node sums) and local energy parts on the
                     128^3 cube mesh, FP32, fields at the 4 points of the degree-2 rule
  --workload faces   all faces of the 128^3 cube mesh with the normals of all of them, and
                     GI volume / surface integrals of the divergence theorem
  --workload p2      global P2 stiffness and mass matrices on the 64^3 cube mesh (2,146,689
                     P2 nodes), coefficients at 27 points: the 10 x 10 element pages, the P2
                     CSR structure and sparse() of the pages
  --workload serve   a Poisson stream of assembly jobs (200 jobs/s, 2-D FP64 / 3-D FP32,
                     1e3..2e6 elements) through the serving loop: p50/p99 latency and
                     throughput, fused + resident structures vs one launch per job without
                     them, and a 10x overload run
  --workload unstructured  the assembly step on a 3-D Delaunay mesh of --points random
                     points (default 1e6: about 6.7 million tets, nodes in up to ~110 tets),
                     FP32 with FP64 fallback
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "assembly_cube128_traffic.json")
KERNEL_SOURCES = ["assembly.hip", "p1elem.hpp", "smallmat.hpp", "common.hpp", "exact.hpp", "quadrature.hpp"]
BATCH_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "batch_plan_64groups_traffic.json")
ENERGY_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "energy_cube128_traffic.json")
ENERGY_SOURCES = ["energy.hip", "p1elem.hpp", "smallmat.hpp", "common.hpp", "exact.hpp", "quadrature.hpp"]
FACES_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "faces_cube128_traffic.json")
FACES_SOURCES = ["assembly.hip", "integrals.hip", "common.hpp"]
P2_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "p2_cube64_traffic.json")
P2_SOURCES = ["p2.hip", "sparse.hip", "assembly.hip", "p1elem.hpp", "smallmat.hpp", "common.hpp", "exact.hpp",
              "internal.hpp"]
BATCH_SOURCES = ["batch.hip", "smallmat.hpp", "common.hpp"]
PAGES_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "page_ops_1e7_traffic.json")
PAGES_SOURCES = ["page_ops.hip", "smallmat.hpp", "common.hpp"]
ELEM_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "elements_cube128_traffic.json")
ELEM_SOURCES = ["elements.hip", "p1elem.hpp", "smallmat.hpp", "common.hpp", "quadrature.hpp"]


def kernel_hash(files=KERNEL_SOURCES) -> str:
    """Hash of the kernel sources with comments and blank space removed (a counter file
    stays valid across comment-only edits)."""
    import re
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2404_16039_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update("".join(src.split()).encode())
    return h.hexdigest()[:16]


def traffic_of(path, files, kernel=None, **match):
    """HBM bytes per launch from a committed counter file, if it matches these sources
    (files holding several kernels list them under "kernels")."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        tr = json.load(f)
    if tr.get("kernel_hash") != kernel_hash(files) or any(tr.get(k) != v for k, v in match.items()):
        return None
    if kernel is not None:
        return tr.get("kernels", {}).get(kernel)
    return tr.get("hbm_bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128, help="cubes per side of the mesh (default 128)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=128, help="cubes per side of the CPU oracle sample")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    ap.add_argument("--workload", choices=["assembly", "square", "elements", "pages", "batch", "serve", "energy",
                                           "faces", "p2", "unstructured"],
                    default="assembly")
    ap.add_argument("--coef", choices=["one", "quad"], default="one",
                    help="assembly coefficients: c = 1, or c = exp(x1+x2+x3) at the 4 points of the degree-2 rule "
                         "(the paper's section 3.6 benchmark)")
    ap.add_argument("--jobs", type=int, default=10000, help="jobs of the serving trace")
    ap.add_argument("--page-frac", type=float, default=0.25, help="share of page-op jobs in the serving trace")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0, help="device-memory budget of the server")
    ap.add_argument("--rate", type=float, default=200.0, help="arrival rate of the serving trace (jobs/s)")
    ap.add_argument("--tuner-cache", default=None, help="JSON schedule cache of the batch workload")
    ap.add_argument("--prec", choices=["f32", "f64"], default="f32",
                    help="assembly precision: FP32 bulk with FP64 fallback, or FP64 throughout")
    ap.add_argument("--points", type=int, default=1000000,
                    help="points of the Delaunay mesh of the unstructured workload")
    ap.add_argument("--rotate", type=int, default=4,
                    help="copies of the assembly inputs used in turn (defeats the last-level cache)")
    return ap.parse_args()


def _events(n):
    import torch
    return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]


def _timed(fn, steps, warmup, stream):
    """Per-call times (ms) of fn() from HIP events on `stream`, after `warmup` calls."""
    import numpy as np
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = _events(steps)
    for e0, e1 in ev:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return np.array([e0.elapsed_time(e1) for e0, e1 in ev])


def _calib_copy(mib):
    import torch
    if mib:
        src = torch.empty((mib << 20) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()


def run_pages(args):
    """1e7 random 3x3 pages: every page operation, FP64 and FP32, both layouts."""
    import numpy as np
    import torch

    from paper_2404_16039_amd import gen
    from paper_2404_16039_amd import lib as L

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    count, n = 10_000_000, 3
    _calib_copy(args.copy_calib_mib)
    a64 = gen.page_batch(count, n)
    b64 = gen.page_batch(count, n, stream=gen.STREAM_PAGES_B)
    x64 = gen.vector_batch(count, n)
    rows = []
    fb = L.fallback(0.0, 1e6, True)
    ctr = torch.zeros(4, dtype=torch.int64, device="cuda")
    for dtype, prec, es in ((torch.float64, L.F64, 8), (torch.float32, L.F32, 4)):
        for layout in ("pages", "soa"):
            if layout == "pages":
                ta = torch.from_numpy(a64).to(dtype).cuda()
                tb = torch.from_numpy(b64).to(dtype).cuda()
                D = L.pages(count, n, n)
                V = L.pages(count, n, 1)
                tx = torch.from_numpy(x64).to(dtype).cuda()
            else:
                ta = torch.from_numpy(np.ascontiguousarray(a64.T)).to(dtype).cuda()
                tb = torch.from_numpy(np.ascontiguousarray(b64.T)).to(dtype).cuda()
                D = L.pages_soa(count, n, n)
                V = L.pages_soa(count, n, 1)
                tx = torch.from_numpy(np.ascontiguousarray(x64.T)).to(dtype).cuda()
            out = torch.empty_like(ta)
            det = torch.empty(count, dtype=dtype, device="cuda")
            y = torch.empty_like(tx)
            ops = {
                "det": (lambda: L.page_det(D, ta, det, fb=fb, counters=ctr), 9 * es + es),
                "inv+det": (lambda: L.page_inv(D, ta, D, out, det=det, fb=fb, counters=ctr), 18 * es + es),
                "transpose": (lambda: L.page_transpose(D, ta, D, out), 18 * es),
                "mv": (lambda: L.page_mv(D, ta, 0, V, tx, V, y), 15 * es),
                "mtimes": (lambda: L.page_mtimes(D, ta, 0, D, tb, 0, D, out), 27 * es),
            }
            for name, (fn, bpp) in ops.items():
                t = _timed(fn, args.steps, args.warmup, stream)
                med = float(np.median(t))
                gbs = bpp * count / (med * 1e-3) / 1e9
                rows.append({"op": name, "dtype": "f64" if es == 8 else "f32", "layout": layout,
                             "ms_median": round(med, 4), "ms_p10": round(float(np.percentile(t, 10)), 4),
                             "ms_p90": round(float(np.percentile(t, 90)), 4), "bytes_per_page": bpp,
                             "gbps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
            del ta, tb, tx, out, det, y
            torch.cuda.empty_cache()
    head = next(r for r in rows if r["op"] == "inv+det" and r["dtype"] == "f32" and r["layout"] == "pages")
    out = {
        "metric": "3x3 page inverses (with det) per second, FP32, paper layout",
        "value": count / (head["ms_median"] * 1e-3), "unit": "pages/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_median"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "1e7 random 3x3 pages, N(0,1) + 3 I; FP64 and FP32; paper layout and SoA",
                   "pages": count},
        "roofline": {"kernel": "k_page_inv<float,3,true> (pf_page_inv)", "bound": "hbm",
                     "achieved": head["gbps"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": head["frac"],
                     "traffic": traffic_of(PAGES_TRAFFIC_FILE, PAGES_SOURCES, kernel="k_page_inv<float,3,true>",
                                           pages=count),
                     "algorithmic_bytes_per_launch": head["bytes_per_page"] * count},
        "ops": rows,
    }
    if not args.no_cpu_baseline:
        import oracle
        a32 = a64.astype(np.float32).astype(np.float64)
        t1 = time.perf_counter()
        done = 0
        while time.perf_counter() - t1 < 10.0:  # whole passes over the 1e7 pages, >= 10 s in total
            oracle.page_inv(a32, n)
            oracle.page_det(a32, n)
            done += count
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": done / dt, "unit": "pages/s", "cores": 1, "kind": "oracle",
                               "sample": "FP64 oracle Gauss-Jordan inverse + Leibniz det of all 1e7 FP32 pages, "
                                         "%d pass(es), single thread, %.1f s" % (done // count, dt)}
    print(json.dumps(out))


def run_batch(args):
    """64-group uneven mixed batch: inverse + product per group, one persistent launch."""
    import tempfile

    import numpy as np
    import torch

    from paper_2404_16039_amd import gen
    from paper_2404_16039_amd import lib as L

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    spec = gen.mixed_groups(64)
    total = sum(c for _, c in spec)
    groups, host_a = [], []
    for gi, (n, count) in enumerate(spec):
        a = gen.page_batch(count, n, sub=gi).astype(np.float32)
        b = gen.page_batch(count, n, stream=gen.STREAM_PAGES_B, sub=gi).astype(np.float32)
        ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        groups.append({"order": n, "ops": L.OP_INV | L.OP_MTIMES, "a": ta, "b": tb, "x": torch.empty_like(ta),
                       "c": torch.empty_like(ta), "det": torch.empty(count, device="cuda")})
        host_a.append((n, a, b))
    # algorithmic bytes: A and B read, inv(A), A*B and det(A) written once, FP32
    alg = sum(4 * (4 * n * n + 1) * c for n, c in spec)
    fb = L.fallback(0.0, 1e6, True)
    ctr = torch.zeros(4, dtype=torch.int64, device="cuda")
    plan = L.Plan(L.F32, 64, fb).set_groups(groups)
    _calib_copy(args.copy_calib_mib)

    plan.tune(None, L.TUNE_DEFAULT)
    t_def = _timed(lambda: plan.run(counters=ctr), args.steps, args.warmup, stream)
    cache = args.tuner_cache or os.path.join(tempfile.gettempdir(), "pagefem_tuner_cache.json")
    t0 = time.perf_counter()
    sched = plan.tune(cache, L.TUNE_CACHED, stream=stream).as_dict()
    tune_s = time.perf_counter() - t0
    t_tuned = _timed(lambda: plan.run(counters=ctr), args.steps, args.warmup, stream)
    ntiles, grid, lds = plan.info()

    def plain():
        for g in groups:
            n, count = g["order"], g["a"].shape[0]
            P = L.pages(count, n, n)
            L.page_inv(P, g["a"], P, g["x"], det=g["det"], fb=fb, counters=ctr)
            L.page_mtimes(P, g["a"], 0, P, g["b"], 0, P, g["c"])
    t_plain = _timed(plain, args.steps, args.warmup, stream)
    med = float(np.median(t_tuned))
    gbs = alg / (med * 1e-3) / 1e9
    out = {
        "metric": "matrices/s (mixed-order inverse + product, one persistent graph-replayed launch)",
        "value": total / (med * 1e-3), "unit": "matrices/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": med, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64 groups, orders uniform in {2,3,4}, sizes round(10^U(3,6)), A, B = N(0,1) + 3 I, "
                               "FP32 inv(A) with det and A*B per group", "matrices": total,
                   "per_order": {str(n): sum(c for m, c in spec if m == n) for n in (2, 3, 4)}},
        "ms_tuned": {"median": med, "p10": float(np.percentile(t_tuned, 10)), "p90": float(np.percentile(t_tuned, 90))},
        "ms_default_schedule": float(np.median(t_def)),
        "ms_one_launch_per_group_and_op": float(np.median(t_plain)),
        "schedule": sched, "tune_seconds": round(tune_s, 3), "tiles": ntiles, "grid": grid, "lds_bytes": lds,
        "roofline": {"kernel": "k_plan<float,%d> (pf_plan_run)" % sched["waves"], "bound": "hbm", "achieved": gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                     "traffic": traffic_of(BATCH_TRAFFIC_FILE, BATCH_SOURCES, matrices=total),
                     "algorithmic_bytes_per_launch": alg},
    }
    if not args.no_cpu_baseline:
        import oracle
        t1 = time.perf_counter()
        done = 0
        while time.perf_counter() - t1 < 10.0:  # whole passes over every group, >= 10 s in total
            for n, a, b in host_a:
                a64, b64 = a.astype(np.float64).reshape(-1, n * n), b.astype(np.float64).reshape(-1, n * n)
                oracle.page_inv(a64, n)
                oracle.page_det(a64, n)
                oracle.page_mtimes(a64, b64, n, n, n)
                done += a.shape[0]
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": done / dt, "unit": "matrices/s", "cores": 1, "kind": "oracle",
                               "sample": "FP64 oracle inverse + det + product of every matrix of the batch, "
                                         "%d pass(es), single thread, %.1f s" % (done // total, dt)}
    plan.close()
    print(json.dumps(out))


def run_energy(args):
    """Load vector and local energy parts on the 3-D cube mesh (FP32, degree-2 rule)."""
    import numpy as np
    import torch

    from paper_2404_16039_amd import gen
    from paper_2404_16039_amd import lib as L

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n = args.n
    coords, elems, _ = gen.cube_mesh(n, jitter=0.15, with_faces=False)
    nn, ne = coords.shape[0], elems.shape[0]
    tc, te = torch.from_numpy(coords).cuda(), torch.from_numpy(elems).cuda()
    # fields at the 4 integration points of every element, resident before the clock
    xq = L.quad_points(tc, te, 2)
    s = xq.sum(dim=2)
    fq = (torch.sin(3.0 * s) + 0.5 * xq[..., 0]).to(torch.float32).contiguous()
    cKq = torch.exp(s).to(torch.float32).contiguous()
    cMq = (1.0 + xq[..., 2] ** 2).to(torch.float32).contiguous()
    u = (torch.cos(2.0 * tc[:, 0]) + tc[:, 1] ** 2 - 0.3 * tc[:, 2]).to(torch.float32).contiguous()
    del xq, s
    csr = L.Csr().symbolic(3, nn, te)
    b2D = torch.empty(ne * 4, dtype=torch.float32, device="cuda")
    b = torch.empty(nn, dtype=torch.float32, device="cuda")
    J = torch.empty(3 * ne, dtype=torch.float32, device="cuda")
    tot = torch.zeros(3, dtype=torch.float64, device="cuda")
    fb = L.fallback(1e-3 / n ** 3, 1e6, True)
    _calib_copy(args.copy_calib_mib)

    def step():
        csr.rhs(L.F32, tc, te, 2, fq, b2D, b, fb=fb, stream=stream)
        csr.energies(L.F32, tc, te, 2, u, cKq=cKq, cMq=cMq, b2D=b2D, J=J, totals=tot, fb=fb, stream=stream)

    # per-kernel durations: the element part of the load vector alone, the whole load
    # vector (the node sums are the difference), the energies (element kernel + totals)
    t_elem = _timed(lambda: csr.rhs(L.F32, tc, te, 2, fq, b2D, None, fb=fb, stream=stream), args.steps,
                    args.warmup, stream)
    t_rhs = _timed(lambda: csr.rhs(L.F32, tc, te, 2, fq, b2D, b, fb=fb, stream=stream), args.steps, args.warmup,
                   stream)
    t_en = _timed(lambda: csr.energies(L.F32, tc, te, 2, u, cKq=cKq, cMq=cMq, b2D=b2D, J=J, totals=tot, fb=fb,
                                       stream=stream), args.steps, args.warmup, stream)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    ms = {"k_rhs_elem<3,float,4>": float(np.mean(t_elem)),
          "k_rhs_nodes<float>": max(float(np.mean(t_rhs) - np.mean(t_elem)), 1e-6),
          "k_energies<3,float,4> + totals": float(np.mean(t_en))}
    # algorithmic bytes per launch: element node ids 16 B/tet, FP64 coordinates 24 B/node,
    # FP32 values at 4 points 16 B/tet each (f; c_K; c_M), local vectors 16 B/tet, node sums
    # 4 B/node, the adjacency words 16 B/tet and lengths 4 B/node, nodal u 4 B/node, J 12 B/tet
    alg = {"k_rhs_elem<3,float,4>": 48 * ne + 24 * nn,
           "k_rhs_nodes<float>": 32 * ne + 8 * nn,
           "k_energies<3,float,4> + totals": 76 * ne + 28 * nn}
    dom = max(ms, key=ms.get)

    def roof(k):
        gbs = alg[k] / (ms[k] * 1e-3) / 1e9
        return {"kernel": k, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS,
                "traffic": traffic_of(ENERGY_TRAFFIC_FILE, ENERGY_SOURCES, kernel=k.split(" ")[0], n=n),
                "algorithmic_bytes_per_launch": alg[k], "launch_us": round(ms[k] * 1e3, 1)}

    th = tot.cpu().numpy()
    out = {
        "metric": "P1 tet elements/s (load vector with node sums + local energy parts)",
        "value": ne / (wall / args.steps), "unit": "tets/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3-D P1 tets: unit cube, %d^3 cubes x 6 Kuhn tets, jitter 0.15 h; f, c_K, c_M at the "
                               "4 points of the degree-2 rule, FP32; b2D + b (pf_rhs) and J1k, J2k, J3k + totals "
                               "(pf_energies)" % n, "tets": ne, "nodes": nn},
        "kernels_us": {k: round(v * 1e3, 1) for k, v in ms.items()},
        "totals": [float(x) for x in th],
        "roofline": roof(dom),
        "rooflines": {k: roof(k) for k in ms},
    }
    if not args.no_cpu_baseline:
        import oracle
        cn = args.cpu_n
        c2, e2, _ = gen.cube_mesh(cn, jitter=0.15, with_faces=False)
        xq2 = oracle.quad_points(c2, e2, 2)
        s2 = xq2.sum(axis=2)
        f2, ck2, cm2 = np.sin(3.0 * s2) + 0.5 * xq2[..., 0], np.exp(s2), 1.0 + xq2[..., 2] ** 2
        u2 = np.cos(2.0 * c2[:, 0]) + c2[:, 1] ** 2 - 0.3 * c2[:, 2]
        t1 = time.perf_counter()
        passes = 0
        while passes == 0 or time.perf_counter() - t1 < 10.0:  # whole passes, >= 10 s in total
            r = oracle.rhs_p1(c2, e2, 2, f2)
            oracle.local_energies(c2, e2, 2, u2, cKq=ck2, cMq=cm2, b2D=r["b2D"])
            passes += 1
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": passes * e2.shape[0] / dt, "unit": "tets/s", "cores": 1, "kind": "oracle",
                               "sample": "FP64 oracle load vector (local vectors + accumarray) and local energies "
                                         "(element matrices + page bilinear forms), single thread, %d^3 Kuhn mesh, "
                                         "%d tets, %d pass(es), %.1f s" % (cn, e2.shape[0], passes, dt)}
    csr.close()
    print(json.dumps(out))


def _collapsed_rule(d, m):
    """Collapsed-coordinate (conical product) rule on the d-simplex, m Gauss-Jacobi points per
    direction (exact for degree 2m - 1): barycentric points and weights summing to 1."""
    import numpy as np
    from scipy.special import roots_jacobi
    ax = []
    for k in range(d):
        a = d - 1 - k
        x, wx = roots_jacobi(m, a, 0)
        ax.append(((1 + x) / 2, wx / 2 ** (a + 1)))
    pts, wts = [], []
    for idx in np.ndindex(*([m] * d)):
        xi, rest, w = [], 1.0, 1.0
        for k in range(d):
            u = ax[k][0][idx[k]]
            xi.append(u * rest)
            rest *= 1 - u
            w *= ax[k][1][idx[k]]
        pts.append([1 - sum(xi)] + xi)
        wts.append(w)
    w = np.array(wts)
    return np.array(pts), w / w.sum()


def run_faces(args):
    """All faces with their normals (section 3.2 normals benchmark) and GI volume / surface
    integrals (section 3.5) on the 3-D cube mesh."""
    import numpy as np
    import torch

    from paper_2404_16039_amd import gen
    from paper_2404_16039_amd import lib as L

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n = args.n
    coords, elems, _ = gen.cube_mesh(n, jitter=0.15, with_faces=False)
    nn, ne = coords.shape[0], elems.shape[0]
    tc, te = torch.from_numpy(coords).cuda(), torch.from_numpy(elems).cuda()
    csr = L.Csr().symbolic(3, nn, te)
    csr.faces(tc, te)
    f, fe, bf, be = csr.face_lists()
    nf, nfb = f.shape[0], bf.shape[0]
    unit = torch.empty(nf * 3, dtype=torch.float32, device="cuda")
    area = torch.empty(nf, dtype=torch.float32, device="cuda")
    _calib_copy(args.copy_calib_mib)

    def normals():  # faces of the mesh and the normals of all of them
        csr.faces(tc, te, stream=stream)
        fl = csr.face_lists(stream=stream)[0]
        L.boundary_normals(L.F32, tc, fl, unit=unit, measure=area, stream=stream)

    t_faces = _timed(lambda: csr.faces(tc, te, stream=stream), args.steps, args.warmup, stream)
    t_norm = _timed(normals, args.steps, args.warmup, stream)
    # GI: the moment of inertia of rho = x1^2 + x2^2 about the x1 axis, int rho (x2^2 + x3^2),
    # by a volume integral (degree-5 rule on the tets) and as the flux of
    # F = (x1^3 (x2^2 + x3^2)/3, x2^5/5, x2^2 x3^3/3) through the boundary (degree-5 rule on
    # the faces); both 8/15 on the unit cube
    lam3, w3 = _collapsed_rule(3, 3)
    lam2, w2 = _collapsed_rule(2, 3)
    vol = torch.empty(ne, dtype=torch.float64, device="cuda")
    L.elem_geometry(L.F64, tc, te, vol=vol)
    bfc = bf.contiguous()
    bunit = torch.empty(nfb * 3, dtype=torch.float64, device="cuda")
    barea = torch.empty(nfb, dtype=torch.float64, device="cuda")
    L.boundary_normals(L.F64, tc, bfc, unit=bunit, measure=barea)
    value = torch.empty(1, dtype=torch.float64, device="cuda")
    work = torch.empty(L.GI_WORK, dtype=torch.float64, device="cuda")
    X = L.simplex_points(tc, te, lam3)
    div = ((X[..., 0] ** 2 + X[..., 1] ** 2) * (X[..., 1] ** 2 + X[..., 2] ** 2)).contiguous()
    t_pts = _timed(lambda: L.simplex_points(tc, te, lam3, stream=stream), 5, 1, stream)
    t_gi = _timed(lambda: L.gi(L.F64, div, w3, vol, value=value, work=work, stream=stream), args.steps, args.warmup,
                  stream)
    i_vol = float(value.item())
    Y = L.simplex_points(tc, bfc, lam2)
    Fv = torch.stack([Y[..., 0] ** 3 * (Y[..., 1] ** 2 + Y[..., 2] ** 2) / 3, Y[..., 1] ** 5 / 5,
                      Y[..., 1] ** 2 * Y[..., 2] ** 3 / 3], dim=2).contiguous()
    L.gi(L.F64, Fv, w2, barea, normals=bunit, value=value, work=work)
    i_surf = float(value.item())
    del X, div
    nq3 = lam3.shape[0]
    ms = {"faces (k_faces x 2 + scans)": float(np.mean(t_faces)),
          "faces + all normals": float(np.mean(t_norm)),
          "k_simplex_points<3,4> (27 points)": float(np.mean(t_pts)),
          "k_gi<double> (27 points)": float(np.mean(t_gi))}
    # algorithmic bytes: faces -- the adjacency words and slot words read once per pass
    # (2 x 32 B/tet), the faces written (5 x 4 B per face) and the boundary list (4 x 4 B);
    # points -- element node ids 16 B/tet, coordinates 24 B/node, points 24 B each;
    # GI -- the values 8 B per point and the volume 8 B per tet
    alg = {"faces (k_faces x 2 + scans)": 64 * ne + 20 * nf + 16 * nfb,
           "k_simplex_points<3,4> (27 points)": 16 * ne + 24 * nn + 24 * nq3 * ne,
           "k_gi<double> (27 points)": 8 * nq3 * ne + 8 * ne}
    dom = max(alg, key=lambda k: ms[k])

    def roof(k):
        gbs = alg[k] / (ms[k] * 1e-3) / 1e9
        tk = {"k_simplex_points<3,4> (27 points)": ["k_simplex_points<3,4>"], "k_gi<double> (27 points)": ["k_gi<double>"],
              "faces (k_faces x 2 + scans)": ["k_faces<4,0>", "k_faces<4,1>"]}[k]
        tr = [traffic_of(FACES_TRAFFIC_FILE, FACES_SOURCES, kernel=x, n=n) for x in tk]
        return {"kernel": k, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": None if None in tr else sum(tr),
                "algorithmic_bytes_per_launch": alg[k], "launch_us": round(ms[k] * 1e3, 1)}

    step_ms = ms["faces + all normals"]
    out = {
        "metric": "P1 tet elements/s (all faces with their outward normals and areas)",
        "value": ne / (step_ms * 1e-3), "unit": "tets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": step_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3-D P1 tets: unit cube, %d^3 cubes x 6 Kuhn tets, jitter 0.15 h; all faces (sorted, "
                               "oriented outward of their first element, element pairs, boundary list) and the FP32 "
                               "normals and areas of all of them; GI volume and surface integrals" % n,
                   "tets": ne, "nodes": nn, "faces": nf, "boundary_faces": nfb},
        "kernels_us": {k: round(v * 1e3, 1) for k, v in ms.items()},
        "gi": {"volume_integral": i_vol, "surface_integral": i_surf, "closed_form": 8 / 15},
        "roofline": roof(dom),
        "rooflines": {k: roof(k) for k in alg},
        "paper_context": {"what": "all-face normals of a 12,582,912-tet sphere mesh (25,264,128 faces) in MATLAB, "
                                  "mesh generation included, hardware not stated", "s": 10.9},
    }
    if not args.no_cpu_baseline:
        import oracle
        cn = args.cpu_n
        c2, e2, _ = gen.cube_mesh(cn, jitter=0.15, with_faces=False)
        t1 = time.perf_counter()
        passes = 0
        while passes == 0 or time.perf_counter() - t1 < 10.0:  # whole passes, >= 10 s in total
            F2, FE2 = oracle.faces(c2, e2)
            oracle.boundary(c2, F2)
            del F2, FE2
            passes += 1
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": passes * e2.shape[0] / dt, "unit": "tets/s", "cores": 1, "kind": "oracle",
                               "sample": "FP64 oracle: all faces by sorting the element faces, then the normals and "
                                         "areas of all faces, single thread, %d^3 Kuhn mesh, %d tets, %d pass(es), "
                                         "%.1f s" % (cn, e2.shape[0], passes, dt)}
    csr.close()
    print(json.dumps(out))


def run_p2(args):
    """P2 stiffness and mass matrices of the 3-D benchmark (section 3.6): element pages, the
    P2 structure and sparse() of the pages, i.e. the global K and M as the P2 listings return."""
    import numpy as np
    import torch

    from paper_2404_16039_amd import gen
    from paper_2404_16039_amd import lib as L

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n = args.n if args.n != 128 else 64  # the paper's largest 3-D P2 case: 64^3 cubes, 2,146,689 nodes
    coords, elems, _ = gen.cube_mesh(n, jitter=0.15, with_faces=False)
    c2, e2, _ = gen.p2_mesh(coords, elems)
    ne, nn2 = e2.shape[0], c2.shape[0]
    tc, te = torch.from_numpy(c2).cuda(), torch.from_numpy(e2).cuda()
    rule = _collapsed_rule(3, 3)  # 27 points, degree 5
    nq = rule[0].shape[0]
    X = L.simplex_points(torch.from_numpy(coords).cuda(), torch.from_numpy(elems).cuda(), rule[0])
    cq = torch.exp(X.sum(dim=2)).to(torch.float32).contiguous()
    del X
    K = torch.empty(ne * 100, dtype=torch.float32, device="cuda")
    M = torch.empty(ne * 100, dtype=torch.float32, device="cuda")
    fb = L.fallback(1e-3 / n ** 3, 1e6, True)
    _calib_copy(args.copy_calib_mib)
    csr = L.Csr().symbolic_p2(3, nn2, te)
    nnz = csr.info()[1]
    vK = torch.empty(nnz, dtype=torch.float32, device="cuda")
    vM = torch.empty(nnz, dtype=torch.float32, device="cuda")
    t_k = _timed(lambda: L.p2_elements(L.F32, tc, te, rule, None, cKq=cq, K3D=K, fb=fb, stream=stream), args.steps,
                 args.warmup, stream)
    t_m = _timed(lambda: L.p2_elements(L.F32, tc, te, None, rule, cMq=cq, M3D=M, fb=fb, stream=stream), args.steps,
                 args.warmup, stream)
    t_km = _timed(lambda: L.p2_elements(L.F32, tc, te, rule, rule, cKq=cq, cMq=cq, K3D=K, M3D=M, fb=fb,
                                        stream=stream), args.steps, args.warmup, stream)
    t_sp = _timed(lambda: csr.assemble_pages(L.F32, K, M, vK, vM, stream=stream), args.steps, args.warmup, stream)

    def step():  # the whole P2 assembly: pages, structure, sparse()
        L.p2_elements(L.F32, tc, te, rule, rule, cKq=cq, cMq=cq, K3D=K, M3D=M, fb=fb, stream=stream)
        csr.symbolic_p2(3, nn2, te, stream=stream)
        csr.assemble_pages(L.F32, K, M, vK, vM, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    csr.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms, stage_calls = csr.stage_times()
    csr.set_timing(False)
    ms_step = wall * 1e3 / args.steps
    # algorithmic bytes per launch:
    #  pages (K and M): the 10 node ids 40 B/tet, FP64 vertex coordinates 24 B per vertex node, the
    #    coefficient at 27 points for K and for M (2 x 108 B/tet), two FP32 10 x 10 pages 800 B/tet
    #  scatter: node ids 40 B/tet read, adjacency entries 40 B/tet written, 4 B/node counts
    #  pattern: adjacency 40 B/tet, node ids once 40 B/tet, compact entries 40 B/tet and position
    #    words 80 B/tet written, 4 B/nonzero (columns), 8 B/node (row lengths, diagonal positions)
    #  row offsets: 12 B/node; columns: 8 B/nonzero + 4 B/node;  sparse(): adjacency + position
    #    words 120 B/tet, the pages once 800 B/tet, 12 B/node, FP32 K and M 8 B/nonzero
    nv = coords.shape[0]
    kernels = {
        "k_p2_elem<3,float> K+M": (float(np.mean(t_km)), 40 * ne + 24 * nv + 2 * 4 * nq * ne + 800 * ne),
        "k_scatter<4> (P2)": (stage_ms["adjacency"] / stage_calls, 80 * ne + 4 * nn2),
        "k_pattern_p2<10>": (stage_ms["pattern"] / stage_calls, 200 * ne + 4 * nnz + 8 * nn2),
        "k_row_offsets": (stage_ms["row offsets"] / stage_calls, 12 * nn2),
        "k_row_columns<1024,4>": (stage_ms["columns"] / stage_calls, 8 * nnz + 4 * nn2),
        "k_assemble_pages<10,P2,float>": (float(np.mean(t_sp)), 920 * ne + 12 * nn2 + 8 * nnz),
    }
    dominant = max(kernels, key=lambda k: kernels[k][0])

    def roofline(name):
        kms, alg = kernels[name]
        gbs = alg / (kms * 1e-3) / 1e9
        return {"kernel": name, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS,
                "traffic": traffic_of(P2_TRAFFIC_FILE, P2_SOURCES, kernel=name.split(" ")[0], n=n),
                "algorithmic_bytes_per_launch": alg, "launch_us": round(kms * 1e3, 1)}

    out = {
        "metric": "P2 tet elements/s (global stiffness + mass matrices: element pages, structure, sparse())",
        "value": ne / (ms_step * 1e-3), "unit": "tets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3-D P2 tets: unit cube, %d^3 cubes x 6 Kuhn tets, jitter 0.15 h, mid-edge nodes; "
                               "global K and M (FP32, CSR) with c_K = c_M = exp(x1+x2+x3) at the 27 points of a "
                               "degree-5 rule" % n, "tets": ne, "nodes_p2": nn2, "nnz": nnz},
        "kernels_us": dict({k: round(v[0] * 1e3, 1) for k, v in kernels.items()},
                           **{"k_p2_elem<3,float> K": round(float(np.mean(t_k)) * 1e3, 1),
                              "k_p2_elem<3,float> M": round(float(np.mean(t_m)) * 1e3, 1)}),
        "roofline": roofline(dominant),
        "rooflines": {k: roofline(k) for k in kernels},
        "paper_context": {"what": "P2 K and M in MATLAB at 2,146,689 nodes (3-D level 6), hardware not stated",
                          "K_s": 87.6, "M_s": 16.4},
    }
    if not args.no_cpu_baseline:
        import oracle
        cn = 48  # about 10 s of oracle work
        cc, ce, _ = gen.cube_mesh(cn, jitter=0.15, with_faces=False)
        cc2, ce2, _ = gen.p2_mesh(cc, ce)
        cqq = np.exp(oracle.simplex_points(cc, ce, rule[0]).sum(axis=-1))
        t1 = time.perf_counter()
        pg = oracle.p2_elements(cc2, ce2, rule, rule, cqq, cqq)
        oracle.assemble(ce2, cc2.shape[0], pg["K3D"], pg["M3D"])
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": ce.shape[0] / dt, "unit": "tets/s", "cores": 1, "kind": "oracle",
                               "sample": "FP64 oracle P2 K3D + M3D (27-point rules, error scales included) and "
                                         "sparse() of both by sorting, single thread, %d^3 Kuhn mesh, %d tets, "
                                         "%.1f s" % (cn, ce.shape[0], dt)}
    csr.close()
    print(json.dumps(out))


def run_serve(args):
    """Poisson stream of assembly and page-op jobs through the serving loop."""
    import numpy as np
    import torch

    from paper_2404_16039_amd import gen
    from paper_2404_16039_amd import lib as L

    torch.cuda.set_device(0)
    trace = gen.serving_trace(args.jobs, rate=args.rate)
    kinds = gen.serving_page_jobs(args.jobs, frac=args.page_frac)
    base_of, meshes = {}, []
    t_gen = time.perf_counter()
    for j, pg in zip(trace, kinds):  # inputs in host memory before the clock starts (pinned)
        if pg is not None:
            meshes.append(None)
            continue
        key = (j["dim"] << 32) | j["n"]
        if key not in base_of:  # one connectivity (and unjittered coordinates) per mesh size
            if j["dim"] == 2:
                c0, e0, _ = gen.square_mesh(j["n"], jitter=0.0)
            else:
                c0, e0, _ = gen.cube_mesh(j["n"], jitter=0.0, with_faces=False)
            base_of[key] = (c0, e0)
        c0, e0 = base_of[key]
        c = gen.jittered_coords(c0, j["n"], j["dim"], j["id"], stream=gen.STREAM_SERVE)
        meshes.append((torch.from_numpy(c).pin_memory(), e0, key))
    # page-op jobs read prefixes of one pool of pages per (order, precision); their results
    # are computed on the device, and the first 64 page jobs also copy them back
    pool = {}
    for pg in kinds:
        if pg is not None:
            k = (pg["order"], pg["prec"])
            pool[k] = max(pool.get(k, 0), pg["count"])
    for (n, prec), cnt in list(pool.items()):
        dt = np.float32 if prec == 0 else np.float64
        a = gen.page_batch(cnt, n, sub=100 + n).astype(dt)
        b = gen.page_batch(cnt, n, stream=gen.STREAM_PAGES_B, sub=100 + n).astype(dt)
        pool[(n, prec)] = (torch.from_numpy(a).pin_memory(), torch.from_numpy(b).pin_memory())
    t_gen = time.perf_counter() - t_gen
    print(f"serve: inputs ready in {t_gen:.1f} s", file=sys.stderr, flush=True)
    asm = [k for k, m in enumerate(meshes) if m is not None]
    pgs = [k for k, m in enumerate(meshes) if m is None]
    total_el = sum(meshes[k][1].shape[0] for k in asm)
    total_pages = sum(kinds[k]["count"] for k in pgs)
    n_out = 64  # these jobs of each kind also copy their results back (pinned outputs)
    outs = {}
    for k in asm[:n_out]:
        j = trace[k]
        cnt = gen.square_counts(j["n"]) if j["dim"] == 2 else gen.kuhn_counts(j["n"])
        dt = torch.float64 if j["dim"] == 2 else torch.float32
        outs[k] = (torch.empty(cnt["nnz"], dtype=dt).pin_memory(), torch.empty(cnt["nnz"], dtype=dt).pin_memory())
    for k in pgs[:n_out]:
        pg = kinds[k]
        dt = torch.float32 if pg["prec"] == 0 else torch.float64
        nn2 = pg["count"] * pg["order"] ** 2
        outs[k] = (torch.empty(nn2, dtype=dt).pin_memory(), torch.empty(nn2, dtype=dt).pin_memory(),
                   torch.empty(pg["count"], dtype=dt).pin_memory())
    budget = int(args.serve_budget_gib * (1 << 30))

    def pct(v, q):
        return float(np.percentile(np.asarray(v), q)) * 1e3 if len(v) else None

    def replay(flags, speed):
        srv = L.Server(budget, 256, flags)
        t0 = srv.now() + 0.05
        tickets = []
        for k, j in enumerate(trace):
            at = t0 + j["t"] / speed
            while srv.now() < at:
                pass
            if k % 1000 == 0:
                print(f"serve: flags {flags} speed {speed}: {k} jobs submitted", file=sys.stderr, flush=True)
            pg = kinds[k]
            if pg is None:
                c, e, key = meshes[k]
                prec = L.F64 if j["dim"] == 2 else L.F32
                vk, vm = outs.get(k, (None, None))
                tickets.append(srv.submit(j["dim"], prec, c, e, topology=key, arrival=at, valsK=vk, valsM=vm))
            else:
                a, b = pool[(pg["order"], pg["prec"])]
                cnt = pg["count"]
                x, cc, d = outs.get(k, (None, None, None))
                tickets.append(srv.submit_pages(pg["prec"], pg["order"], L.OP_INV | L.OP_MTIMES, a[:cnt], b=b[:cnt],
                                                x=x, c=cc, det=d, arrival=at))
        srv.drain()
        st = srv.stats()
        res = [srv.poll(t) for t in tickets]
        srv.close()
        print(f"serve: flags {flags} speed {speed}: done, p50 {st['latency_p50'] * 1e3:.2f} ms", file=sys.stderr,
              flush=True)
        bad = [r for r in res if r["status"] != 0]
        if bad:
            raise RuntimeError(f"{len(bad)} serving jobs failed, first status {bad[0]['status']}")
        lat_a = [res[k]["finished"] - res[k]["arrival"] for k in asm]
        lat_p = [res[k]["finished"] - res[k]["arrival"] for k in pgs]
        copy = [res[k]["copied"] - res[k]["finished"] for k in outs]
        return {"jobs": st["completed"], "elements": st["elements"], "pages": st["pages"],
                "latency_ms": {"p50": st["latency_p50"] * 1e3, "p99": st["latency_p99"] * 1e3,
                               "mean": st["latency_mean"] * 1e3, "max": st["latency_max"] * 1e3},
                "latency_ms_assembly": {"p50": pct(lat_a, 50), "p99": pct(lat_a, 99)},
                "latency_ms_pages": {"p50": pct(lat_p, 50), "p99": pct(lat_p, 99)},
                "jobs_per_s": st["jobs_per_s"], "elements_per_s": st["elements_per_s"],
                "pages_per_s": st["pages_per_s"],
                "copy_back_ms_median": float(np.median(copy)) * 1e3 if copy else None,
                "ticks": st["ticks"], "launches": st["launches"], "max_batch": st["max_batch"],
                "structure_hits": st["cache_hits"], "structure_misses": st["cache_misses"],
                "evictions": st["evictions"], "admit_waits": st["admit_waits"],
                "scheduler_s": {"evict": round(st["evict_s"], 3), "build_start": round(st["build_start_s"], 3),
                                "tick": round(st["tick_s"], 3)},
                "hbm_high_water_bytes": st["hbm_high_water"], "span_s": st["last_finish"] - st["first_arrival"]}

    served = replay(0, 1.0)
    plain = replay(L.SERVER_NOFUSE | L.SERVER_NOCACHE, 1.0)
    overload = replay(0, 10.0)
    out = {
        "metric": "P1 elements assembled/s under a Poisson stream of assembly and page-op jobs (+ p50/p99 job "
                  "latency)",
        "value": served["elements_per_s"], "unit": "elements/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": served["span_s"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (2-D jobs) / f32 (3-D jobs); page jobs f32 or f64", "data": "synthetic",
        "config": {"workload": "%d jobs, Poisson arrivals %.0f jobs/s; %.0f%% page-op jobs (inverse with det + "
                               "product, order 2..4, 10^U(3,6) pages, FP32 or FP64), the others assembly jobs of "
                               "dim 2 (FP64) or 3 (FP32 + FP64 fallback) with p = 1/2, 10^U(3, log10 2e6) "
                               "elements, jittered structured meshes, 64 GiB budget, 256 slots"
                               % (len(trace), args.rate, 100 * args.page_frac),
                   "assembly_jobs": len(asm), "page_jobs": len(pgs), "elements": total_el, "pages": total_pages,
                   "input_generation_s": round(t_gen, 1)},
        "served": served, "one_launch_per_job_no_resident_structures": plain, "overload_10x": overload,
        "roofline": None,
        "roofline_note": "latency-bound job stream; the kernels' rooflines are those of the assembly and pages "
                         "workloads",
    }
    if not args.no_cpu_baseline:
        import oracle
        hi = host_info()
        t1 = time.perf_counter()
        done = 0
        for k in asm:
            c, e, _ = meshes[k]
            cn = c.numpy()
            el = oracle.p1_elements(cn, e)
            oracle.assemble(e, cn.shape[0], el["Ke"], el["Me"], el["Kabs"])
            done += e.shape[0]
            if time.perf_counter() - t1 > 10.0:
                break
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": done / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
                               "sample": "FP64 oracle element matrices + sparse assembly of the trace's first "
                                         "assembly jobs (%d elements), single thread, %.1f s" % (done, dt),
                               "host": hi}
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: pagefem runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the assembly would shard by rows: each GPU owns a node range and the elements around it)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "pages":
        return run_pages(args)
    if args.workload == "square":
        return run_square(args)
    if args.workload == "elements":
        return run_elements(args)
    if args.workload == "batch":
        return run_batch(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "energy":
        return run_energy(args)
    if args.workload == "faces":
        return run_faces(args)
    if args.workload == "p2":
        return run_p2(args)
    if args.workload == "unstructured":
        return run_unstructured(args)

    return run_assembly(args)


def run_square(args):
    """Latency of the whole 2-D P1 FP64 pipeline on the unit square cut into 32 x 32 squares
    (2,048 triangles, 1,089 nodes): per-triangle Jacobian determinant, inverse (the gradients
    of the barycentric coordinates hold J^-T), element stiffness and mass matrices, the CSR
    structure and the assembly of K and M."""
    import numpy as np
    import torch

    from paper_2404_16039_amd import gen
    from paper_2404_16039_amd import lib as L

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n = 32
    coords, elems, _ = gen.square_mesh(n)
    nn, ne = coords.shape[0], elems.shape[0]
    tc, te = torch.from_numpy(coords).cuda(), torch.from_numpy(elems).cuda()
    f64 = torch.float64
    det = torch.empty(ne, dtype=f64, device="cuda")
    vol = torch.empty(ne, dtype=f64, device="cuda")
    grads = torch.empty(ne * 6, dtype=f64, device="cuda")
    K3D = torch.empty(ne * 9, dtype=f64, device="cuda")
    M3D = torch.empty(ne * 9, dtype=f64, device="cuda")
    csr = L.Csr()
    csr.symbolic(2, nn, te)
    _, nnz, _, _ = csr.info()
    vk = torch.empty(nnz, dtype=f64, device="cuda")
    vm = torch.empty(nnz, dtype=f64, device="cuda")
    ctr = torch.zeros(4, dtype=torch.int64, device="cuda")

    def step():
        L.elem_geometry(L.F64, tc, te, det=det, vol=vol, grads=grads, counters=ctr, stream=stream)
        L.elem_stiffness_mass(L.F64, tc, te, K3D=K3D, M3D=M3D, counters=ctr, stream=stream)
        csr.symbolic(2, nn, te, stream=stream)
        csr.assemble(L.F64, tc, te, vk, vm, counters=ctr, stream=stream)

    steps = max(args.steps, 200)
    t = _timed(step, steps, max(args.warmup, 20), stream)
    med = float(np.median(t))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / steps
    out = {
        "metric": "triangles/s of the whole 2-D P1 FP64 pipeline (latency-bound)",
        "value": ne / (med * 1e-3), "unit": "triangles/s", "n_gpus": 1, "steps": steps,
        "warmup": max(args.warmup, 20), "ms_per_step": med, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2-D P1 plain FP64: unit square, 32 x 32 squares x 2 triangles, jitter 0.2 h; "
                               "Jacobian det and inverse, 3 x 3 element K and M, CSR structure and assembly",
                   "triangles": ne, "nodes": nn, "nnz": int(nnz)},
        "latency_us": {"median": round(med * 1e3, 2), "p10": round(float(np.percentile(t, 10)) * 1e3, 2),
                       "p90": round(float(np.percentile(t, 90)) * 1e3, 2),
                       "host_wall_per_step": round(wall_ms * 1e3, 2)},
        "note": "194 KB of data per step: launch- and latency-bound, so no roofline fraction is reported",
    }
    if not args.no_cpu_baseline:
        import oracle
        hi = host_info()
        t1 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t1 < 5.0:
            el = oracle.p1_elements(coords, elems)
            ref = oracle.assemble(elems, nn, el["Ke"], el["Me"], el["Kabs"])
            reps += 1
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": reps * ne / dt, "unit": "triangles/s", "cores": 1, "kind": "oracle",
                               "sample": "FP64 oracle (element matrices incl. Jacobian inverse + stable-sort sparse "
                                         "assembly), the same 2,048 triangles repeated %d times in %.1f s" % (reps, dt),
                               "host": hi}
        rp, ci = csr.structure()
        out["errors_vs_oracle"] = {
            "structure_identical": bool(np.array_equal(rp.cpu().numpy(), ref["row_ptr"]) and
                                        np.array_equal(ci.cpu().numpy(), ref["col_idx"])),
            "K": value_errors(vk.cpu().numpy(), {"val": ref["valK"], "scale": ref["scaleK"]}, 1e-12),
            "M": value_errors(vm.cpu().numpy(), {"val": ref["valM"], "scale": ref["scaleM"]}, 1e-12),
            "det_max_rel": float(np.max(np.abs(det.cpu().numpy() - el["det"]) / np.abs(el["det"])))}
    print(json.dumps(out))
    csr.close()


def run_elements(args):
    """Per-element work on the 3-D cube (section 3.2 volumes and normals, section 3.6 element
    matrices), FP32 with FP64 fallback: one launch for det, volume and the outward normals of
    the four faces (normals3D), one for the 4 x 4 element stiffness and mass pages."""
    import numpy as np
    import torch

    from paper_2404_16039_amd import gen
    from paper_2404_16039_amd import lib as L

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n = args.n
    h = 1.0 / n
    coords, elems, _ = gen.cube_mesh(n, jitter=0.15, with_faces=False)
    nn, ne = coords.shape[0], elems.shape[0]
    R = max(1, args.rotate)
    tcs = [torch.from_numpy(coords).cuda() for _ in range(R)]
    tes = [torch.from_numpy(elems).cuda() for _ in range(R)]
    fb = L.fallback(1e-3 * h ** 3, 1e6, True)
    _calib_copy(args.copy_calib_mib)
    f32 = torch.float32
    det = torch.empty(ne, dtype=f32, device="cuda")
    vol = torch.empty(ne, dtype=f32, device="cuda")
    nrm = torch.empty(ne * 12, dtype=f32, device="cuda")
    K3D = torch.empty(ne * 16, dtype=f32, device="cuda")
    M3D = torch.empty(ne * 16, dtype=f32, device="cuda")
    ctr = torch.zeros(4, dtype=torch.int64, device="cuda")
    geo = [lambda k=k: L.elem_geometry(L.F32, tcs[k], tes[k], det=det, vol=vol, normals=nrm, fb=fb, counters=ctr,
                                       stream=stream) for k in range(R)]
    mats = [lambda k=k: L.elem_stiffness_mass(L.F32, tcs[k], tes[k], K3D=K3D, M3D=M3D, fb=fb, counters=ctr,
                                              stream=stream) for k in range(R)]
    for w in range(args.warmup):
        geo[w % R]()
        mats[w % R]()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        geo[k % R]()
        evs[k][1].record(stream)
        mats[k % R]()
        evs[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tg = np.array([e[0].elapsed_time(e[1]) for e in evs])
    tm = np.array([e[1].elapsed_time(e[2]) for e in evs])
    # algorithmic bytes: elems 16 B/tet and FP64 coordinates 24 B/node read once; written:
    # det + volume 8 B/tet and normals3D 48 B/tet, or the two 4 x 4 FP32 pages 128 B/tet
    alg_g = 16 * ne + 24 * nn + 56 * ne
    alg_m = 16 * ne + 24 * nn + 128 * ne
    ms_step = wall * 1e3 / args.steps

    def roof(name, key, alg, ms):
        gbs = alg / (ms * 1e-3) / 1e9
        return {"kernel": name, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": traffic_of(ELEM_TRAFFIC_FILE, ELEM_SOURCES, kernel=key, n=n),
                "algorithmic_bytes_per_launch": alg, "launch_us": round(ms * 1e3, 1)}
    rg = roof("k_elem<3,float> (det, volume, normals3D)", "k_elem<3,float>/geometry", alg_g, float(np.median(tg)))
    rm = roof("k_elem<3,float> (K3D, M3D)", "k_elem<3,float>/pages", alg_m, float(np.median(tm)))
    out = {
        "metric": "P1 tets/s: volumes + normals3D, then element K and M pages",
        "value": ne / (ms_step * 1e-3), "unit": "tets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3-D P1 tets, FP32 with FP64 fallback: unit cube, %d^3 cubes x 6 Kuhn tets, jitter "
                               "0.15 h; det, volume and normals3D per tet, then the 4 x 4 K and M pages" % n,
                   "tets": ne, "nodes": nn, "input_sets_rotated": R},
        "roofline": rm if rm["launch_us"] >= rg["launch_us"] else rg,
        "rooflines": [rg, rm],
        "paper_context": {"what": "MATLAB timings at 12,582,912 tets (hardware not stated): volumes 4.42 s "
                                  "(with mesh generation), normals of all faces 10.9 s"},
    }
    if not args.no_cpu_baseline:
        import oracle
        hi = host_info()
        m = ne
        t1 = time.perf_counter()
        passes = 0
        while time.perf_counter() - t1 < 10.0:  # whole passes over the mesh, >= 10 s in total
            el = oracle.p1_elements(coords, elems)
            passes += 1
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": passes * ne / dt, "unit": "tets/s", "cores": 1, "kind": "oracle",
                               "sample": "FP64 oracle element loop (det, volume, gradients, K_e, M_e, facet "
                                         "measures) over all %d tets, %d pass(es), single thread, %.1f s"
                                         % (ne, passes, dt), "host": hi}
        d = det.cpu().numpy()[:m].astype(np.float64)
        out["errors_vs_oracle"] = {
            "det_max_rel": float(np.max(np.abs(d - el["det"]) / np.abs(el["det"]))),
            "K3D_max_err_over_scale": float(np.max(np.abs(K3D.cpu().numpy().reshape(ne, 16)[:m] - el["Ke"]) /
                                                   el["Kabs"])),
            "normals_max_rel": float(np.max(np.abs(-nrm.cpu().numpy().reshape(ne, 12)[:m] - el["grads"]) /
                                            np.abs(el["grads"]).max(axis=1, keepdims=True)))}
    print(json.dumps(out))


def host_info():
    """Host cores this process may use and the CPU model (for the oracle legs)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cap = int(os.environ.get("OMP_NUM_THREADS", avail) or avail)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": avail, "threads": max(1, min(avail, cap)), "cpu_model": model}


def _flush(buf):
    """Read a 1 GiB device buffer (evicts the 256 MB last-level cache and the L2s with clean
    lines: nothing is left to write back while the timed kernel runs); not timed."""
    buf.sum()


def oracle_p1_rate(coords, elems, threads, quad=None):
    """The oracle's element matrices and sparse() over `elems`: one thread on the whole mesh,
    or `threads` threads on contiguous element chunks (each chunk assembled on its own, then
    the chunk matrices summed).  Returns (tets/s, seconds, result of the single-thread run)."""
    import threading

    import numpy as np

    import oracle
    nn, ne = coords.shape[0], elems.shape[0]

    def one(c0, c1, out, k):
        e = elems[c0:c1]
        if quad is not None:
            el = oracle.p1_elements_q(coords, e, 2, quad[c0:c1], quad[c0:c1])
        else:
            el = oracle.p1_elements(coords, e)
        out[k] = oracle.assemble(e, nn, el["Ke"], el["Me"], el["Kabs"])

    if threads == 1:
        res = [None]
        t0 = time.perf_counter()
        one(0, ne, res, 0)
        dt = time.perf_counter() - t0
        return ne / dt, dt, res[0]
    import scipy.sparse as sp
    cuts = np.linspace(0, ne, threads + 1).astype(np.int64)
    res = [None] * threads
    t0 = time.perf_counter()
    th = [threading.Thread(target=one, args=(int(cuts[k]), int(cuts[k + 1]), res, k)) for k in range(threads)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    # chunk matrices summed (in the timed region): their entries concatenated, duplicates added
    rows = np.concatenate([np.repeat(np.arange(nn, dtype=np.int64), np.diff(r["row_ptr"])) for r in res])
    cols = np.concatenate([r["col_idx"] for r in res])
    for key in ("valK", "valM"):
        sp.coo_matrix((np.concatenate([r[key] for r in res]), (rows, cols)), shape=(nn, nn)).tocsr()
    dt = time.perf_counter() - t0
    return ne / dt, dt, None


def value_errors(got, ref, tol):
    """Largest error of every value against the oracle's, relative to the oracle's error scale
    (the sum of the magnitudes of the contributions), and how many exceed the tolerance."""
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    e = np.abs(got - ref["val"]) / np.maximum(ref["scale"], 1e-300)
    big = np.abs(ref["val"]) >= 1e-3 * ref["scale"]
    rel = np.abs(got - ref["val"])[big] / np.abs(ref["val"][big]) if big.any() else np.zeros(1)
    return {"max_err_over_scale": float(e.max()) if e.size else 0.0, "over_tol": int((e > tol).sum()),
            "tol": tol, "max_rel_err_where_not_cancelling": float(rel.max()),
            "frobenius_rel": float(np.linalg.norm(got - ref["val"]) / max(np.linalg.norm(ref["val"]), 1e-300))}


def run_assembly(args):
    """The headline step: CSR structure + numeric K and M + boundary normals on the 3-D cube."""
    import numpy as np
    import torch

    from paper_2404_16039_amd import gen
    from paper_2404_16039_amd import lib as L

    torch.cuda.set_device(0)
    n = args.n
    h = 1.0 / n
    f64 = args.prec == "f64"
    dt_val = torch.float64 if f64 else torch.float32
    prec = L.F64 if f64 else L.F32
    es = 8 if f64 else 4
    coords, elems, faces = gen.cube_mesh(n, jitter=0.15)
    nn, ne, nf = coords.shape[0], elems.shape[0], faces.shape[0]
    # R copies of the inputs, used in turn: R x (elems + coords) well above the 256 MB
    # last-level cache, so no step finds its inputs left in the cache by the step before
    R = max(1, args.rotate)
    tcs = [torch.from_numpy(coords).cuda() for _ in range(R)]
    tes = [torch.from_numpy(elems).cuda() for _ in range(R)]
    tf = torch.from_numpy(faces).cuda()
    fb = L.fallback(1e-3 * h ** 3, 1e6, True)
    stream = torch.cuda.current_stream()
    _calib_copy(args.copy_calib_mib)

    quad = args.coef == "quad"
    cqs = []
    if quad:  # coefficient values at the integration points: inputs resident in HBM before the clock
        for k in range(R):
            xq = L.quad_points(tcs[k], tes[k], 2)
            cqs.append(torch.exp(xq.sum(dim=2)).to(dt_val).contiguous())
            del xq
    csr = L.Csr()
    csr.symbolic(3, nn, tes[0])
    _, nnz, _, _ = csr.info()
    valsK = torch.empty(nnz, dtype=dt_val, device="cuda")
    valsM = torch.empty(nnz, dtype=dt_val, device="cuda")
    unit = torch.empty(nf * 3, dtype=dt_val, device="cuda")
    area = torch.empty(nf, dtype=dt_val, device="cuda")
    ctr = torch.zeros(4, dtype=torch.int64, device="cuda")

    def numeric(k):
        if quad:
            csr.assemble_quad(prec, tcs[k], 2, valsK, valsM, cKq=cqs[k], cMq=cqs[k], fb=fb, counters=ctr,
                              stream=stream)
        else:
            csr.assemble(prec, tcs[k], tes[k], valsK, valsM, fb=fb, counters=ctr, stream=stream)

    def step(k, ev=None):
        if ev:
            ev[0].record(stream)
        csr.symbolic(3, nn, tes[k], stream=stream)
        if ev:
            ev[1].record(stream)
        numeric(k)
        if ev:
            ev[2].record(stream)
        L.boundary_normals(prec, tcs[k], tf, unit=unit, measure=area, stream=stream)
        if ev:
            ev[3].record(stream)

    for w in range(args.warmup):
        step(w % R)
    torch.cuda.synchronize()
    ctr.zero_()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    csr.set_timing(True)  # HIP events between the symbolic kernels, on the same stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k % R, evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms, stage_calls = csr.stage_times()
    csr.set_timing(False)
    sym = np.array([e[0].elapsed_time(e[1]) for e in evs])
    num = np.array([e[1].elapsed_time(e[2]) for e in evs])
    bnd = np.array([e[2].elapsed_time(e[3]) for e in evs])
    routed = int(ctr[0].item()) // max(args.steps, 1)
    bad = int(ctr[2].item())
    step_out = (valsK.cpu().numpy(), valsM.cpu().numpy(), csr.structure())

    # the numeric phase alone on the resident structure (the roofline's kernel): a 1 GiB
    # buffer is read between repetitions, outside the events (cold caches, no dirty lines)
    flush = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
    reps = max(args.steps, 5)
    tn = []
    for r in range(reps):
        _flush(flush)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        numeric(r % R)
        e1.record(stream)
        torch.cuda.synchronize()
        tn.append(e0.elapsed_time(e1))
    tn = np.array(tn)
    del flush

    ms_step = wall * 1e3 / args.steps
    value = ne / (wall / args.steps)
    # algorithmic bytes of the numeric assembly kernel: elems (16 B/tet), FP64 coordinates
    # (24 B/node), K and M values (2 x es B/nonzero); with quadrature also the coefficients at
    # 4 points for K and for M (8 es B/tet)
    alg_num = 16 * ne + 24 * nn + 2 * es * nnz + (8 * es * ne if quad else 0)
    # symbolic phase: the method's bytes are the connectivity read and the structure written
    alg_sym = 16 * ne + 4 * (nn + 1) + 4 * nnz
    # whole step: numeric + the structure written once + boundary faces (12 B of indices and
    # 4 es B of outputs per face)
    alg_step = alg_num + 4 * (nn + 1) + 4 * nnz + nf * (12 + 4 * es)
    num_ms = float(np.median(tn))
    sym_ms = float(sym.mean())
    phases = {"symbolic_ms": round(sym_ms, 4), "numeric_ms": round(float(num.mean()), 4),
              "boundary_ms": round(float(bnd.mean()), 4), "numeric_flushed_ms_median": round(num_ms, 4),
              "numeric_flushed_ms_p10": round(float(np.percentile(tn, 10)), 4),
              "numeric_flushed_ms_p90": round(float(np.percentile(tn, 90)), 4)}
    kname = ("k_numeric<3,double>" if f64 else "k_numeric32<3>") + (" (QN=4)" if quad else "")
    stage_names = {"adjacency": "k_scatter + adjacency scan", "pattern": "k_rows_p1<4>",
                   "row offsets": "k_row_offsets + k_row_stats", "columns": "k_row_columns"}
    kernels_us = {stage_names.get(k, k): round(v / stage_calls * 1e3, 1) for k, v in stage_ms.items()}
    kernels_us[kname] = round(num_ms * 1e3, 1)
    gbs = alg_num / (num_ms * 1e-3) / 1e9
    tr = None if (quad or f64) else traffic_of(TRAFFIC_FILE, KERNEL_SOURCES, kernel=kname, n=n)
    roof = {"kernel": kname, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "traffic": tr, "algorithmic_bytes_per_launch": alg_num,
            "launch_us": round(num_ms * 1e3, 1),
            "bytes": "16 B/tet (elems) + 24 B/node (FP64 coords) + %d B/nonzero (K, M)%s"
                     % (2 * es, " + 8 coefficients/tet" if quad else "")}
    sgbs = alg_sym / (sym_ms * 1e-3) / 1e9
    roof_sym = {"phase": "symbolic (k_scatter, adjacency scan, k_rows_p1, k_row_offsets, k_row_columns)", "bound": "hbm", "achieved": sgbs,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": sgbs / HBM_PEAK_GBS,
                "algorithmic_bytes": alg_sym, "ms": round(sym_ms, 4),
                "bytes": "16 B/tet (elems read) + 4 B/row (row_ptr) + 4 B/nonzero (col_idx) written"}
    # the paper's level-7 cube (2,146,689 nodes, 12,582,912 tets), K + M with c = exp(x1+x2+x3)
    # at quadrature points: 66.6 s + 20.4 s in MATLAB (hardware not stated)
    paper_tets_per_s = 12582912 / (66.6 + 20.4)
    vs = value / paper_tets_per_s if (quad and n == 128) else None

    out = {
        "metric": "P1 tet elements assembled/sec (stiffness + mass, CSR) + achieved HBM GB/s",
        "value": value,
        "unit": "tets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": vs,
        "dtype": "f64" if f64 else "f32",
        "data": "synthetic",
        "config": {"workload": "3-D P1 tets, %s: unit cube, %d^3 cubes x 6 Kuhn tets, jitter 0.15 h; K + M CSR "
                               "assembly (symbolic + numeric) and boundary normals/areas%s"
                               % ("FP64" if f64 else "FP32 bulk with FP64 fallback", n,
                                  "; c_K = c_M = exp(x1+x2+x3) at the 4 points of the degree-2 rule" if quad else ""),
                   "tets": ne, "nodes": nn, "nnz": int(nnz), "boundary_faces": nf,
                   "fallback": None if f64 else "det < 1e-3 h^3, det-condition > 1e6 or vertex shape > 16 -> FP64",
                   "coords": "f64",
                   "input_sets_rotated": R},
        "hbm_gbps_step": alg_step / (ms_step * 1e-3) / 1e9,
        "phases_ms": phases,
        "numeric_tets_per_s": ne / (num_ms * 1e-3),
        "routed_per_step": routed,
        "bad_index": bad,
        "kernels_us": kernels_us,
        "roofline": roof,
        "roofline_symbolic": roof_sym,
        "paper_context": {"what": "MATLAB page-function library, 3-D P1 K and M at 2,146,689 nodes (level 7), "
                                  "hardware not stated, c = exp(x1+x2+x3) with quadrature",
                          "K_s": 66.6, "M_s": 20.4},
    }

    if not args.no_cpu_baseline:
        hi = host_info()
        cn = args.cpu_n
        c2, e2, _ = (coords, elems, None) if cn == n else gen.cube_mesh(cn, jitter=0.15, with_faces=False)
        q2 = None
        if quad:  # coefficients at the integration points are inputs, as on the GPU side
            import oracle
            q2 = np.exp(oracle.quad_points(c2, e2, 2).sum(axis=2))
        rate1, dt1, ref = oracle_p1_rate(c2, e2, 1, q2)
        rateT, dtT, _ = oracle_p1_rate(c2, e2, hi["threads"], q2) if hi["threads"] > 1 else (rate1, dt1, None)
        out["cpu_baseline"] = {
            "value": rateT, "unit": "tets/s", "cores": hi["threads"], "kind": "oracle",
            "sample": "FP64 oracle (element matrices%s + stable-sort sparse assembly of K and M) on the %d^3 Kuhn "
                      "mesh, %d tets: %d threads on contiguous element chunks, chunk matrices summed, %.2f s; "
                      "one thread on the whole mesh %.1f s"
                      % (" with coefficients at the integration points" if quad else "", cn, e2.shape[0],
                         hi["threads"], dtT, dt1),
            "single_core": {"value": rate1, "cores": 1, "seconds": round(dt1, 2)},
            "host": hi}
        if cn == n:  # the step's results against the oracle's (every nonzero)
            vk, vm, (rp, ci) = step_out
            tol = 1e-12 if f64 else 1e-5
            out["errors_vs_oracle"] = {
                "structure_identical": bool(np.array_equal(rp.cpu().numpy(), ref["row_ptr"]) and
                                            np.array_equal(ci.cpu().numpy(), ref["col_idx"])),
                "K": value_errors(vk, {"val": ref["valK"], "scale": ref["scaleK"]}, tol),
                "M": value_errors(vm, {"val": ref["valM"], "scale": ref["scaleM"]}, tol)}
    print(json.dumps(out))
    csr.close()


def run_unstructured(args):
    """The assembly step (structure + numeric K and M, FP32 with FP64 fallback) on a 3-D
    Delaunay mesh of random points: nodes of valence up to ~110 (long rows), both element
    orientations, and the vertex-shape routing of its ill-shaped tets."""
    import numpy as np
    import torch

    from paper_2404_16039_amd import gen
    from paper_2404_16039_amd import lib as L

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    coords, elems = gen.delaunay_mesh(args.points, 3)
    t_mesh = time.perf_counter() - t0
    print(f"delaunay mesh: {elems.shape[0]} tets in {t_mesh:.1f} s", file=sys.stderr, flush=True)
    nn, ne = coords.shape[0], elems.shape[0]
    deg = np.bincount(elems.ravel(), minlength=nn)
    tc, te = torch.from_numpy(coords).cuda(), torch.from_numpy(elems).cuda()
    fb = L.fallback(0.0, 1e6, True)
    stream = torch.cuda.current_stream()
    csr = L.Csr()
    csr.symbolic(3, nn, te)
    _, nnz, _, _ = csr.info()
    valsK = torch.empty(nnz, dtype=torch.float32, device="cuda")
    valsM = torch.empty(nnz, dtype=torch.float32, device="cuda")
    ctr = torch.zeros(4, dtype=torch.int64, device="cuda")

    def numeric():
        csr.assemble(L.F32, tc, te, valsK, valsM, fb=fb, counters=ctr, stream=stream)

    def step():
        csr.symbolic(3, nn, te, stream=stream)
        numeric()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctr.zero_()
    csr.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms, stage_calls = csr.stage_times()
    csr.set_timing(False)
    routed = int(ctr[0].item()) // max(args.steps, 1)
    bad = int(ctr[2].item())
    flush = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
    tn = []
    for _ in range(max(args.steps, 5)):
        _flush(flush)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        numeric()
        e1.record(stream)
        torch.cuda.synchronize()
        tn.append(e0.elapsed_time(e1))
    del flush
    num_ms = float(np.median(tn))
    ms_step = wall * 1e3 / args.steps
    alg_num = 16 * ne + 24 * nn + 8 * nnz
    gbs = alg_num / (num_ms * 1e-3) / 1e9
    kernels_us = {k: round(v / stage_calls * 1e3, 1) for k, v in stage_ms.items()}
    kernels_us["numeric (k_numeric32<3> + long rows)"] = round(num_ms * 1e3, 1)
    out = {
        "metric": "P1 tet elements assembled/sec (stiffness + mass, CSR) + achieved HBM GB/s",
        "value": ne / (wall / args.steps), "unit": "tets/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3-D P1 tets, FP32 bulk with FP64 fallback: Delaunay mesh of %d uniform random points "
                               "in the unit cube (Z-order node numbering); K + M CSR assembly (symbolic + numeric)"
                               % args.points,
                   "tets": ne, "nodes": nn, "nnz": int(nnz), "max_valence": int(deg.max()),
                   "long_rows": int(((deg > 64)).sum()),
                   "fallback": "det-condition > 1e6 or vertex shape > 16 -> FP64", "coords": "f64"},
        "routed_per_step": routed, "bad_index": bad, "kernels_us": kernels_us,
        "numeric_tets_per_s": ne / (num_ms * 1e-3),
        "roofline": {"kernel": "k_numeric32<3> + k_numeric_long", "bound": "hbm", "achieved": gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": alg_num, "launch_us": round(num_ms * 1e3, 1),
                     "bytes": "16 B/tet (elems) + 24 B/node (FP64 coords) + 8 B/nonzero (K, M)"},
    }
    if not args.no_cpu_baseline:
        hi = host_info()
        rate1, dt1, ref = oracle_p1_rate(coords, elems, 1)
        out["cpu_baseline"] = {"value": rate1, "unit": "tets/s", "cores": 1, "kind": "oracle",
                               "sample": "FP64 oracle (element matrices + stable-sort sparse assembly of K and M) "
                                         "on the whole mesh, one thread, %.1f s" % dt1, "host": hi}
        rp, ci = csr.structure()
        out["errors_vs_oracle"] = {
            "structure_identical": bool(np.array_equal(rp.cpu().numpy(), ref["row_ptr"]) and
                                        np.array_equal(ci.cpu().numpy(), ref["col_idx"])),
            "K": value_errors(valsK.cpu().numpy(), {"val": ref["valK"], "scale": ref["scaleK"]}, 1e-5),
            "M": value_errors(valsM.cpu().numpy(), {"val": ref["valM"], "scale": ref["scaleM"]}, 1e-5)}
    print(json.dumps(out))
    csr.close()


if __name__ == "__main__":
    main()
