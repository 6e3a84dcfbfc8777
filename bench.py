#!/usr/bin/env python3
"""Benchmark of the DD projection hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-cpu] [--skip-fp64]
                    [--skip-ann | --ann-only]

Workload (one step = one projection P_D of the whole query batch through the
C ABI): N = 2^27 synthetic material data points, m = 65536 query states, BF16
MFMA scan on tile-centred data with certified candidates reranked in FP64
(indices equal to the FP64 nearest neighbour).  The plain FP64 MFMA scan of the
same batch is timed beside it.  Inputs are resident in HBM before timing; the
dataset (whitening, spatial order, packs) is built once, outside the timed
region.  Beside the headline: DD solve latency (8^3 hex, N = 1e6) and the ANN
walk at N = 10^9 (exact and budgeted, 16^3 DD solve).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BF16_PEAK_TFLOPS = 2500.0     # MI355X dense bf16 MFMA
FP32_PEAK_TFLOPS = 157.3      # MI355X fp32 MFMA
FP64_PEAK_TFLOPS = 78.6       # MI355X fp64 MFMA
FLOPS_PER_PAIR = 24.0         # K = 12 dot product per (query, data point)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(mode, tile, N, m):
    """HBM bytes per launch of the main scan kernel from the committed rocprofv3
    counter summary, or None when that summary is for another kernel, workload
    or an older version of the kernel source."""
    if mode != "bf16":
        return None
    return profile_traffic("scan16_pass_bf16_N2e27_m65536.md", f"N={N} m={m} tile={tile}")


def profile_traffic(name, workload):
    """traffic_bytes_per_launch of a committed profile summary when its workload
    matches and the profiled kernel source is unchanged, else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        line = line.strip()
        if ":" in line and line.split(":")[0] in ("kernel", "workload", "traffic_bytes_per_launch",
                                                  "source", "source_sha256_16"):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    try:
        src = open(os.path.join(ROOT, fields["source"]), "rb").read()
    except (KeyError, OSError):
        return None
    if hashlib.sha256(src).hexdigest()[:16] != fields.get("source_sha256_16"):
        return None
    if fields.get("workload") != workload:
        return None
    return float(fields["traffic_bytes_per_launch"])


def host_cpu():
    """CPU model, sockets, physical cores and logical CPUs of this host (for the
    CPU baseline), from /proc/cpuinfo and the scheduler's affinity mask."""
    model, phys = "unknown", set()
    try:
        cur = {}
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                if "physical id" in cur and "core id" in cur:
                    phys.add((cur["physical id"], cur["core id"]))
                cur = {}
                continue
            k, v = (x.strip() for x in line.split(":", 1))
            cur[k] = v
            if k == "model name":
                model = v
        if "physical id" in cur and "core id" in cur:
            phys.add((cur["physical id"], cur["core id"]))
    except OSError:
        pass
    return {"model": model, "sockets": len({p for p, _ in phys}) or None,
            "physical_cores": len(phys) or None, "logical_cpus": os.cpu_count(),
            "cpus_available": len(os.sched_getaffinity(0))}


def dd_solve_latency(L, C, R):
    """p50/p99 wall latency of complete DD solves: 8^3 hexahedra (4096 material
    points), clamped at x = 0, 100 MPa traction on x = 1, N = 1e6 data points,
    random initial associations with seeds 0..R-1, until the association stops
    changing."""
    import numpy as np
    import torch

    import ddsynth
    N, n = 1_000_000, 8
    e, s = ddsynth.data_points(N, 1001)
    ds = L.dd_dataset_create(torch.from_numpy(e).cuda(), torch.from_numpy(s).cuda(), C,
                             packs=0x1 | 0x4 | 0x10)
    mask, force = ddsynth.box_bc(n, 100.0)
    out = {"workload": "DD solve, 8^3 hex (4096 material points), N=1e6, clamp + 100 MPa; "
                       "P_C by the cached K^-1, P_D exact in every mode",
           "solves": R}
    for mode in ("bf16", "fp64", "ann"):
        L.dd_solve(ds, (n, n, n), mask, force, ddsynth.indices(8 * n ** 3, N, 999), mode=mode)
        lat, iters, conv = [], [], 0
        for seed in range(R):
            init = ddsynth.indices(8 * n ** 3, N, seed)
            torch.cuda.synchronize()
            t = time.time()
            r = L.dd_solve(ds, (n, n, n), mask, force, init, mode=mode)
            lat.append((time.time() - t) * 1e3)
            iters.append(r["iterations"])
            conv += int(r["converged"])
        lat = np.array(lat)
        out[mode] = {"p50_ms": round(float(np.percentile(lat, 50)), 2),
                     "p99_ms": round(float(np.percentile(lat, 99)), 2),
                     "mean_iterations": round(float(np.mean(iters)), 2), "converged": conv}
        log(f"dd_solve {mode}: p50 {out[mode]['p50_ms']} ms, p99 {out[mode]['p99_ms']} ms, "
            f"iterations {np.mean(iters):.1f}, converged {conv}/{R}")
    ds.close()
    return out


ANN_BYTES_PER_POINT = 24.0    # FP16 scaled offsets (12) read per visited point
ANN_BYTES_PER_LEAF = 64.0     # leaf centre, radius (FP32) read per visited leaf
ANN_BYTES_PER_LEAF_BOX = 24.0  # quantised leaf box (lo[12], hi[12] as bytes) per test
ANN_BYTES_PER_BOX = 96.0      # FP32 box (lo[12], hi[12]) read per test of a higher box
KMT_BYTES_PER_RECORD = 80.0   # k-means tree child record (centre, radius, code, byte box) per test
KMT_BYTES_PER_NODE = 96.0     # FP32 box of an expanded k-means tree node (decodes its children)
HBM_PEAK_GBS = 8000.0         # MI355X HBM3E


def ann_leg(L, C, steps, budgets=(4, 64), solve=True, index="ann", fds=()):
    """Tree walks at scale: N = 10^9 points generated on the device (streamed
    into the dataset), m = 32768 queries around generated points; index "ann"
    (box tree) or "kmeans" (k-means tree).  Exact walks cold and warm-started
    from the exact answer (the steady state of the DD loop), a few budgets (and
    for the k-means tree radius factors f_d < 1) with the generating point as
    warm start, and the 16^3 DD solve."""
    import numpy as np
    import torch

    import ddsynth
    N, m = 1_000_000_000, 32768
    kmt = index == "kmeans"
    gen = ddsynth.DevicePoints(1003)
    torch.cuda.synchronize()
    t = time.time()
    ds = L.dd_dataset_create_streamed(N, C, gen.fill_fn, gen.user,
                                      packs=0x1 | (0x20 if kmt else 0x10))
    torch.cuda.synchronize()
    create_s = time.time() - t
    qe, qs, base = ddsynth.queries_generated(N, 1003, m, 2003)
    states = torch.from_numpy(ddsynth.states(qe, qs)).cuda()
    name = "k-means tree" if kmt else "box tree"
    out = {"workload": f"{name} walk, N=1e9 (generated on device, streamed), m=32768 queries",
           "N": N, "m": m, "dataset_create_s": round(create_s, 3),
           "dataset_gb": round(ds.info()[1] / 1e9, 2), "index": L.dd_dataset_index_info(ds)}

    def run(warm, budget, fd=None):
        walk, tot, vis, box, lvs, lbox, nds, ovf = [], [], 0, 0, 0, 0, 0, 0
        L.dd_project(ds, states, warm_start_idx=warm, mode=index, ann_budget=budget, ann_fd=fd)
        for _ in range(steps):
            i, d, st = L.dd_project(ds, states, warm_start_idx=warm, mode=index,
                                    ann_budget=budget, ann_fd=fd, stats=True)
            walk.append(st["scan_ms"])
            tot.append(st["total_ms"])
            vis += st["visited"]
            box += st["boxes"]
            lvs += st["leaves"]
            lbox += st["leaf_boxes"]
            nds += st["nodes"]
            ovf += st["overflowed"]
        w, tt = sum(walk) / steps, sum(tot) / steps
        if kmt:
            byts = (ANN_BYTES_PER_POINT * vis + ANN_BYTES_PER_LEAF * lvs
                    + KMT_BYTES_PER_RECORD * box + KMT_BYTES_PER_NODE * nds) / steps
        else:
            byts = (ANN_BYTES_PER_POINT * vis + ANN_BYTES_PER_LEAF * lvs
                    + ANN_BYTES_PER_LEAF_BOX * lbox + ANN_BYTES_PER_BOX * (box - lbox)) / steps
        return i, d, {"walk_ms": round(w, 3), "total_ms": round(tt, 3),
                      "proj_per_s": round(m / (tt / 1e3), 1),
                      "points_per_query": round(vis / steps / m, 1),
                      "boxes_per_query": round(box / steps / m, 1),
                      "leaves_per_query": round(lvs / steps / m, 1),
                      "leaf_boxes_per_query": round(lbox / steps / m, 1),
                      "nodes_per_query": round(nds / steps / m, 1),
                      "fallback_queries": ovf // steps,
                      "algorithmic_bytes_per_launch": round(byts), "achieved_gbs": round(byts / w / 1e6, 1)}

    ie, de, cold = run(None, 0)
    _, _, warm = run(ie.clone(), 0)
    out["exact_cold"], out["exact_warm"] = cold, warm
    out["roofline"] = {"bound": "hbm", "achieved": warm["achieved_gbs"], "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(warm["achieved_gbs"] / HBM_PEAK_GBS, 4),
                       "traffic": profile_traffic(f"{index}_walk_N1e9_m32768.md",
                                                  f"N={N} m={m} exact warm"),
                       "kernel": f"ann_walk_kernel<false, {'true' if kmt else 'false'}> "
                                 "(exact, warm-started)",
                       "bytes_per_point": ANN_BYTES_PER_POINT, "bytes_per_leaf": ANN_BYTES_PER_LEAF}
    if kmt:
        out["roofline"]["bytes_per_record"] = KMT_BYTES_PER_RECORD
        out["roofline"]["bytes_per_node"] = KMT_BYTES_PER_NODE
    else:
        out["roofline"]["bytes_per_leaf_box"] = ANN_BYTES_PER_LEAF_BOX
        out["roofline"]["bytes_per_box"] = ANN_BYTES_PER_BOX
    log(f"{index} 1e9: create {create_s:.2f}s, exact cold {cold['walk_ms']} ms, "
        f"warm {warm['walk_ms']} ms ({warm['achieved_gbs']} GB/s)")
    wb = torch.from_numpy(base).cuda()
    out["budgeted"] = {}
    for b in budgets:
        ib, db, r = run(wb, b)
        r["recall"] = round(float((ib == ie).double().mean()), 4)
        r["mean_rel_dist_excess"] = float(((db - de) / de).mean())
        out["budgeted"][str(b)] = r
        log(f"{index} 1e9 budget {b}: recall {r['recall']}, walk {r['walk_ms']} ms")
    if fds:
        out["radius_factor"] = {}
        for fd in fds:
            ib, db, r = run(wb, 0, fd)
            r["recall"] = round(float((ib == ie).double().mean()), 4)
            r["mean_rel_dist_excess"] = float(((db - de) / de).mean())
            out["radius_factor"][str(fd)] = r
            log(f"{index} 1e9 f_d {fd}: recall {r['recall']}, walk {r['walk_ms']} ms")
    if not solve:
        ds.close()
        return out
    n = 16
    mask, force = ddsynth.box_bc(n, 100.0)
    init = ddsynth.indices(8 * n ** 3, N, 7)
    L.dd_solve(ds, (n, n, n), mask, force, init, mode=index)
    t = time.time()
    r = L.dd_solve(ds, (n, n, n), mask, force, init, mode=index)
    solve_ms = (time.time() - t) * 1e3
    out["dd_solve_16cube"] = {"workload": "16^3 hex (32768 material points), clamp + 100 MPa, "
                                          f"exact {name} walks",
                              "ms": round(solve_ms, 1), "iterations": r["iterations"],
                              "converged": bool(r["converged"])}
    log(f"{index} 1e9 dd_solve 16^3: {solve_ms:.0f} ms, {r['iterations']} iterations")
    t = time.time()
    rs = L.dd_solve(ds, (n, n, n), mask, force, init, mode=index, skip=True)
    skip_ms = (time.time() - t) * 1e3
    out["dd_solve_16cube_skip"] = {
        "ms": round(skip_ms, 1), "iterations": rs["iterations"],
        "projections_skipped": rs["skipped"], "projections": rs["iterations"] * 8 * n ** 3,
        "same_u_as_without": bool(np.array_equal(rs["u"], r["u"]))}
    log(f"{index} 1e9 dd_solve 16^3 with skipping: {skip_ms:.0f} ms, skipped {rs['skipped']} of "
        f"{rs['iterations'] * 8 * n ** 3} projections")
    sched = []
    runs = [dict(ann_budget=4), dict(ann_budget=4, ann_ramp=10),
            dict(ann_budget=4, ann_ramp=10, local_accuracy=True), dict(ann_budget=16, ann_ramp=10),
            dict(ann_budget=16, ann_ramp=10, local_accuracy=True)]
    if kmt:
        runs += [dict(ann_fd=0.4, ann_ramp=10), dict(ann_fd=0.4, ann_ramp=10, local_accuracy=True),
                 dict(ann_fd=0.0, ann_ramp=10), dict(ann_fd=0.0, ann_ramp=10, local_accuracy=True)]
    for kw in runs:
        t = time.time()
        rb = L.dd_solve(ds, (n, n, n), mask, force, init, mode=index, **kw)
        ms_b = (time.time() - t) * 1e3
        err = float(np.linalg.norm(rb["u"] - r["u"]) / np.linalg.norm(r["u"]))
        row = {"budget": kw.get("ann_budget", 0), "ramp": kw.get("ann_ramp", 0),
               "f_d_final": kw.get("ann_fd", 1.0), "local_accuracy": kw.get("local_accuracy", False),
               "ms": round(ms_b, 1), "search_ms": round(rb["project_ms"], 1),
               "iterations": rb["iterations"], "stop_reason": rb["stop_reason"],
               "final_global_distance": float(rb["d_full"][-1]), "u_rel_err_vs_exact": err}
        sched.append(row)
        log(f"{index} 1e9 dd_solve 16^3 {kw}: {ms_b:.0f} ms (search {rb['project_ms']:.0f} ms), "
            f"{rb['iterations']} iterations, final distance {rb['d_full'][-1]:.5g}, "
            f"u rel err {err:.3e}")
    out["dd_solve_16cube_exact_distance"] = float(r["d_full"][-1])
    out["dd_solve_16cube_budgeted"] = sched
    ds.close()
    return out


def serve_leg(L, C, n_solves, fracs=(0.5, 0.9), n_cap=8, modes=("bf16", "ann")):
    """Serving: N = 2^26 resident data points (BF16 + FP64 packs); DD solves on
    4^3, 8^3, 16^3 and 24^3 hexahedra in equal mix, clamp + normal traction drawn
    in [50, 200] MPa, random initial associations.  Capacity = solves/s of a burst
    of n_cap solves submitted at once; then Poisson arrivals at each fraction of
    that capacity, n_solves per run, each run on a fresh server."""
    import numpy as np
    import torch

    import ddsynth
    N = 1 << 26
    e, s = ddsynth.data_points(N, 1004)
    ds = L.dd_dataset_create(torch.from_numpy(e).cuda(), torch.from_numpy(s).cuda(), C,
                             packs=0x1 | 0x4 | 0x10)
    del e, s
    torch.cuda.empty_cache()
    sizes = (4, 8, 16, 24)
    rng = np.random.default_rng(4)
    bcs = {n: ddsynth.box_bc(n, 1.0) for n in sizes}

    def request(k):
        n = sizes[k % 4]
        t = float(rng.uniform(50.0, 200.0))
        mask, unit = bcs[n]
        return ((n, n, n), mask, unit * t, ddsynth.indices(8 * n ** 3, N, 40000 + k))

    out = {"workload": "serving, N=2^26 resident (BF16 + FP64 packs and the tree), DD solves on "
                       "4^3/8^3/16^3/24^3 hex (equal mix), traction U[50,200] MPa, projections "
                       "batched across solves (exact in every mode)",
           "N": N}
    for mode in modes:
        res = {}
        # warm-up: one solve of each size (forms the cached inverses)
        srv = L.DDServer(ds, mode=mode)
        for t in [srv.submit(*request(k)) for k in range(4)]:
            srv.wait(t)
        srv.close()
        # capacity: a burst submitted at once
        srv = L.DDServer(ds, mode=mode)
        t0 = time.time()
        for t in [srv.submit(*request(100 + k)) for k in range(n_cap)]:
            srv.wait(t)
        cap = n_cap / (time.time() - t0)
        st = srv.stats()
        srv.close()
        res["capacity_solves_per_s"] = round(cap, 3)
        res["capacity_queries_per_s"] = round(st["queries_per_s"], 1)
        log(f"serving ({mode}) capacity: {cap:.3f} solves/s ({st['queries_per_s']:.0f} queries/s)")
        res["runs"] = []
        for frac in fracs:
            lam = frac * cap
            arrivals = np.cumsum(rng.exponential(1.0 / lam, n_solves))
            srv = L.DDServer(ds, mode=mode)
            tickets, lat, iters, conv = [], [], [], 0
            t0 = time.time()
            for k, ta in enumerate(arrivals):
                dt = ta - (time.time() - t0)
                if dt > 0:
                    time.sleep(dt)
                tickets.append(srv.submit(*request(1000 * (1 + int(frac * 10)) + k)))
            for t in tickets:
                r = srv.wait(t)
                lat.append(r["elapsed_ms"])
                iters.append(r["iterations"])
                conv += int(r["converged"])
            wall = time.time() - t0
            st = srv.stats()
            srv.close()
            lat = np.array(lat)
            run = {"rate_fraction": frac, "lambda_solves_per_s": round(lam, 3), "solves": n_solves,
                   "solve_p50_ms": round(float(np.percentile(lat, 50)), 1),
                   "solve_p99_ms": round(float(np.percentile(lat, 99)), 1),
                   "projection_p50_ms": round(st["proj_p50_ms"], 2),
                   "projection_p99_ms": round(st["proj_p99_ms"], 2),
                   "queue_p50_ms": round(st["queue_p50_ms"], 2),
                   "queue_p99_ms": round(st["queue_p99_ms"], 2),
                   "queries_per_s": round(st["queries"] / wall, 1),
                   "batches": st["batches"],
                   "mean_batch": round(st["queries"] / max(st["batches"], 1), 1),
                   "peak_active": st["peak_active"], "peak_hbm_bytes": st["peak_bytes"],
                   "mean_iterations": round(float(np.mean(iters)), 2), "converged": conv}
            res["runs"].append(run)
            log(f"serving ({mode}) at {frac} x capacity ({lam:.3f}/s): solve p50 "
                f"{run['solve_p50_ms']} ms, p99 {run['solve_p99_ms']} ms, projection p50 "
                f"{run['projection_p50_ms']} ms, p99 {run['projection_p99_ms']} ms, "
                f"{run['queries_per_s']:.0f} queries/s")
        out[mode] = res
    ds.close()
    return out


def paper_leg(L, C=None, Ns=(1_000, 10_000, 100_000, 1_000_000, 100_000_000, 1_000_000_000),
              seeds=5, mode="ann", kmeans_Ns=(100_000_000, 1_000_000_000),
              kmeans_fds=(1.0, 0.0, 0.4, 0.6, 0.8), kmeans_ramp=20):
    """The paper's own example (Section 3): cube of edge 10 mm, 20^3 hexahedra
    (64000 material points), bottom fixed, top rotated by 2 degrees; data from
    the nonlinear law with strains in +-0.025; metric from the PCA of the data;
    exact projections.  Per data-set size: iterations, final global distance,
    solve time and the GPU time of the projections over `seeds` random initial
    associations.  For the sizes in kmeans_Ns also the k-means tree of
    Sections 4.2 and 4.5: f_d ramped linearly from 0 to f_d^f over the first
    kmeans_ramp iterations, for each f_d^f in kmeans_fds (1.0: the exact walk
    over the k-means tree, no ramp)."""
    import numpy as np
    import torch

    import ddsynth
    n, size = 20, 10.0
    mask, val, force = ddsynth.torsion_bc(n, size, 2.0)
    out = {"workload": "paper example: 20^3 hex cube (edge 10 mm, 64000 material points), bottom "
                       "fixed, top rotated 2 deg; nonlinear law E=1000 MPa, alpha=500, strains "
                       "+-0.025; PCA metric; exact " + mode + " projections",
           "runs": [], "kmeans_runs": []}

    def dataset(N, seed, packs):
        if N <= 1_000_000:
            e, s = ddsynth.data_points_nonlinear(N, seed)
            de, dsg = torch.from_numpy(e).cuda(), torch.from_numpy(s).cuda()
            C = L.dd_metric_pca(de, dsg)
            ds = L.dd_dataset_create(de, dsg, C, packs=packs)
            del de, dsg
            return ds
        # generated on the device and streamed into the dataset; the metric
        # from the PCA of the first 2^24 points (a uniform sample of the set)
        gen = ddsynth.DevicePoints(seed, law="nonlinear")
        se, ss = gen.generate(0, 1 << 24)
        C = L.dd_metric_pca(se, ss)
        del se, ss
        torch.cuda.empty_cache()
        return L.dd_dataset_create_streamed(N, C, gen.fill_fn, gen.user, packs=packs)

    def solves(ds, N, **kw):
        its, dist, ms, pms = [], [], [], []
        for seed in range(seeds):
            init = ddsynth.indices(8 * n ** 3, N, 5000 + seed)
            t = time.time()
            r = L.dd_solve(ds, (n, n, n, size, size, size), mask, force, init,
                           dirichlet_values=val, **kw)
            ms.append((time.time() - t) * 1e3)
            its.append(r["iterations"])
            dist.append(float(r["d_full"][-1]))
            pms.append(r["project_ms"])
        return {"mean_iterations": round(float(np.mean(its)), 2),
                "mean_final_global_distance": float(np.mean(dist)),
                "mean_solve_ms": round(float(np.mean(ms)), 1),
                "p50_solve_ms": round(float(np.percentile(ms, 50)), 1),
                "mean_search_ms": round(float(np.mean(pms)), 1)}

    for N in Ns:
        seed = 3000 + N % 997
        t = time.time()
        ds = dataset(N, seed, 0x1 | 0x10 | (0x4 if N <= 1_000_000 else 0))
        torch.cuda.synchronize()
        run = {"N": N, "dataset_build_s": round(time.time() - t, 2)}
        run.update(solves(ds, N, mode=mode))
        out["runs"].append(run)
        log(f"paper example N={N}: {run['mean_iterations']} iterations, final distance "
            f"{run['mean_final_global_distance']:.4g}, {run['mean_solve_ms']} ms "
            f"(search {run['mean_search_ms']} ms)")
        ds.close()
        torch.cuda.empty_cache()
        if N not in kmeans_Ns or not kmeans_fds:
            continue
        t = time.time()
        ds = dataset(N, seed, 0x1 | 0x20)
        torch.cuda.synchronize()
        build_s = round(time.time() - t, 2)
        for fd in kmeans_fds:
            ramp = kmeans_ramp if fd < 1.0 else 0
            for local in ((False, True) if 0.0 <= fd <= 0.4 else (False,)):
                run = {"N": N, "f_d_final": fd, "ramp_iterations": ramp, "local_accuracy": local,
                       "dataset_build_s": build_s}
                run.update(solves(ds, N, mode="kmeans", ann_fd=fd, ann_ramp=ramp,
                                  local_accuracy=local))
                out["kmeans_runs"].append(run)
                log(f"paper example N={N}, k-means tree f_d^f {fd}{' local' if local else ''}: "
                    f"{run['mean_iterations']} iterations, final distance "
                    f"{run['mean_final_global_distance']:.4g}, {run['mean_solve_ms']} ms "
                    f"(search {run['mean_search_ms']} ms)")
        ds.close()
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--log2n", type=int, default=27)
    ap.add_argument("--m", type=int, default=65536)
    ap.add_argument("--mode", default="bf16", choices=["bf16", "fp16", "fp64"])
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--fp32-steps", type=int, default=2)
    ap.add_argument("--skip-fp32", action="store_true")
    ap.add_argument("--cpu-queries", type=int, default=256)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--tile", type=int, default=2048)
    ap.add_argument("--passes", type=int, default=0)
    ap.add_argument("--dd-solves", type=int, default=100,
                    help="DD solves (8^3 hex, N=1e6) timed for the p50/p99 latency leg; 0 = skip")
    ap.add_argument("--skip-ann", action="store_true", help="skip the N=1e9 ANN leg")
    ap.add_argument("--serve-solves", type=int, default=200,
                    help="solves per Poisson run of the serving leg (N=2^26); 0 = skip")
    ap.add_argument("--serve-modes", default="ann",
                    help="projection modes of the serving leg, comma separated (bf16 serves "
                         "about 0.7 solves/s of this mix: 200 solves take minutes per rate)")
    ap.add_argument("--paper-seeds", type=int, default=3,
                    help="random starts per data-set size in the paper-example leg; 0 = skip")
    ap.add_argument("--paper-only", action="store_true",
                    help="run only the paper-example leg and print its JSON object")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg and print its JSON object")
    ap.add_argument("--ann-only", action="store_true",
                    help="run only the N=1e9 ANN leg and print its JSON object")
    ap.add_argument("--kmeans-only", action="store_true",
                    help="run only the N=1e9 k-means tree leg and print its JSON object")
    ap.add_argument("--skip-kmeans", action="store_true",
                    help="leave out the N=1e9 k-means tree leg")
    ap.add_argument("--ann-no-solve", action="store_true",
                    help="with --ann-only: leave out the 16^3 DD solve (for counter runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the projection shards by data or by query; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import ddsynth
    from paper_2012_00357_amd import _lib as L

    torch.cuda.set_device(0)
    N, m = 1 << args.log2n, args.m
    C = ddsynth.isotropic_stiffness()
    if args.paper_only:
        print(json.dumps({"paper_example": paper_leg(L, seeds=max(args.paper_seeds, 1))}),
              flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": serve_leg(L, C, args.serve_solves,
                                               modes=tuple(args.serve_modes.split(",")))}),
              flush=True)
        return
    if args.ann_only:
        res = {"ann": ann_leg(L, C, args.steps, solve=not args.ann_no_solve)}
        if not args.skip_kmeans:
            res["kmeans"] = ann_leg(L, C, args.steps, solve=not args.ann_no_solve, index="kmeans",
                                    fds=(0.5, 0.8))
        print(json.dumps(res), flush=True)
        return
    if args.kmeans_only:
        print(json.dumps({"kmeans": ann_leg(L, C, args.steps, solve=not args.ann_no_solve,
                                            index="kmeans", fds=(0.5, 0.8))}), flush=True)
        return
    t = time.time()
    e, s = ddsynth.data_points(N, 1002)
    qe, qs, _ = ddsynth.queries(e, s, m, 2002)
    log(f"generated N={N} m={m} in {time.time() - t:.1f}s")
    t = time.time()
    de, dsg = torch.from_numpy(e).cuda(), torch.from_numpy(s).cuda()
    states = torch.from_numpy(ddsynth.states(qe, qs)).cuda()
    packs = 0x1 | (0x8 if args.mode == "fp16" else 0x4)
    torch.cuda.synchronize()
    t = time.time()
    ds = L.dd_dataset_create(de, dsg, C, packs=packs, tile=args.tile)
    torch.cuda.synchronize()
    build_s = time.time() - t
    del de, dsg
    torch.cuda.empty_cache()
    log(f"dataset built in {build_s:.2f}s, {ds.info()[1] / 1e9:.2f} GB on device")

    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written by one copy kernel")
        del a, b
    idx = torch.empty(m, dtype=torch.int64, device="cuda")
    dist = torch.empty(m, dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        L.dd_project(ds, states, mode=args.mode, idx_out=idx, dist_out=dist, passes=args.passes)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    scan_ms, cand, ovf, slow = [], 0, 0, 0
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        _, _, st = L.dd_project(ds, states, mode=args.mode, idx_out=idx, dist_out=dist, stats=True,
                                passes=args.passes)
        scan_ms.append(st["scan_ms"])
        slow += st["slow_tiles"]
        cand += st["candidates"]
        ovf += st["overflowed"]
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    value = m / (ms / 1e3)
    scan_avg = sum(scan_ms) / len(scan_ms)
    idx_mixed = idx.cpu().numpy().copy()
    dist_mixed = dist.cpu().numpy().copy()
    log(f"{args.mode}: {ms:.2f} ms/step, scan {scan_avg:.2f} ms, {value:.4g} proj/s, "
        f"cand/query {cand / (m * args.steps):.2f}, fallback/step {ovf / args.steps:.1f}, "
        f"slow tiles/step {slow / args.steps:.0f}")

    # the same dataset from host arrays (DD_DATASET_HOST_INPUT): creation including the
    # chunked host-to-device copies of the raw points, outside the timed region
    torch.cuda.synchronize()
    t = time.time()
    dsh = L.dd_dataset_create(e, s, C, packs=packs, tile=args.tile)
    torch.cuda.synchronize()
    host_build_s = time.time() - t
    ih, _ = L.dd_project(dsh, states, mode=args.mode)
    host_same = bool(np.array_equal(ih.cpu().numpy(), idx_mixed))
    dsh.close()
    del ih
    torch.cuda.empty_cache()
    log(f"dataset from host arrays built in {host_build_s:.2f}s "
        f"({N * 96 / host_build_s / 1e9:.1f} GB/s of raw points), indices equal: {host_same}")

    peak = FP64_PEAK_TFLOPS if args.mode == "fp64" else BF16_PEAK_TFLOPS
    traffic = measured_traffic(args.mode, args.tile, N, m)
    achieved = FLOPS_PER_PAIR * N * m / (scan_avg / 1e3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "kernel": f"scan16_pass_kernel<{args.mode}, {args.tile}, mark>",
                "flops_per_pair": FLOPS_PER_PAIR,
                "issued_frac": round(achieved * 32.0 / FLOPS_PER_PAIR / peak, 4)}

    walk = None
    if not args.skip_ann:
        # the exact tree walk on the same dataset and queries (its own pack and tree)
        torch.cuda.synchronize()
        t = time.time()
        dsa = L.dd_dataset_create(torch.from_numpy(e).cuda(), torch.from_numpy(s).cuda(), C,
                                  packs=0x1 | 0x10)
        torch.cuda.synchronize()
        walk_build = time.time() - t
        L.dd_project(dsa, states, mode="ann")
        torch.cuda.synchronize()
        w_ms, tot = [], []
        for _ in range(args.steps):
            iw, dw, st = L.dd_project(dsa, states, mode="ann", stats=True)
            w_ms.append(st["scan_ms"])
            tot.append(st["total_ms"])
        same = bool(np.array_equal(iw.cpu().numpy(), idx_mixed))
        walk = {"proj_per_s": round(m / (sum(tot) / len(tot) / 1e3), 1),
                "walk_ms": round(sum(w_ms) / len(w_ms), 3), "total_ms": round(sum(tot) / len(tot), 3),
                "points_per_query": round(st["visited"] / m, 1),
                "dataset_build_s": round(walk_build, 3), "indices_equal_mixed": same}
        log(f"exact tree walk at N=2^{args.log2n}: {walk['total_ms']} ms/step "
            f"({walk['proj_per_s']:.4g} proj/s), indices equal to {args.mode}: {same}")
        dsa.close()
        torch.cuda.empty_cache()

    fp64 = None
    if not args.skip_fp64 and args.mode != "fp64":
        if not (packs & 0x1):
            pass
        for _ in range(args.fp64_steps):
            torch.cuda.synchronize()
            t = time.time()
            i64, d64, st = L.dd_project(ds, states, mode="fp64", stats=True)
            torch.cuda.synchronize()
            wall = time.time() - t
        same = bool(np.array_equal(i64.cpu().numpy(), idx_mixed))
        fp64 = {"proj_per_s": round(m / wall, 2), "ms_per_step": round(wall * 1e3, 2),
                "scan_ms": round(st["scan_ms"], 2),
                "frac_fp64_mfma": round(FLOPS_PER_PAIR * N * m / (st["scan_ms"] / 1e3) / 1e12
                                        / FP64_PEAK_TFLOPS, 4),
                "indices_equal_mixed": same,
                "max_dist_rel_diff": float(np.max(np.abs(d64.cpu().numpy() - dist_mixed)
                                                  / dist_mixed))}
        log(f"fp64: {wall * 1e3:.1f} ms/step, indices equal to {args.mode}: {same}")

    fp32 = None
    if not args.skip_fp32 and args.mode != "fp64":
        # the FP32 MFMA scan of the same batch (its own pack; FP64 rerank and fallback)
        ds.close()
        torch.cuda.empty_cache()
        t = time.time()
        ds = L.dd_dataset_create(torch.from_numpy(e).cuda(), torch.from_numpy(s).cuda(), C,
                                 packs=0x1 | 0x2, tile=args.tile)
        torch.cuda.synchronize()
        log(f"FP32 dataset built in {time.time() - t:.2f}s")
        L.dd_project(ds, states, mode="fp32")
        walls, scans = [], []
        for _ in range(args.fp32_steps):
            torch.cuda.synchronize()
            t = time.time()
            i32, d32, st = L.dd_project(ds, states, mode="fp32", stats=True)
            torch.cuda.synchronize()
            walls.append(time.time() - t)
            scans.append(st["scan_ms"])
        wall, scan = sum(walls) / len(walls), sum(scans) / len(scans)
        same = bool(np.array_equal(i32.cpu().numpy(), idx_mixed))
        ach = FLOPS_PER_PAIR * N * m / (scan / 1e3) / 1e12
        fp32 = {"proj_per_s": round(m / wall, 2), "ms_per_step": round(wall * 1e3, 2),
                "scan_ms": round(scan, 2), "achieved_tflops": round(ach, 2),
                "frac_fp32_mfma": round(ach / FP32_PEAK_TFLOPS, 4),
                "kernel": "scan32_kernel (v_mfma_f32_32x32x2_f32, K=12, norms as accumulator input)",
                "candidates_per_query": round(st["candidates"] / m, 3),
                "fallback_queries": st["overflowed"], "indices_equal_mixed": same,
                "dist_equal_mixed": bool(np.array_equal(d32.cpu().numpy(), dist_mixed))}
        log(f"fp32: {wall * 1e3:.1f} ms/step, scan {scan:.1f} ms ({ach:.1f} TFLOP/s, "
            f"{ach / FP32_PEAK_TFLOPS:.3f} of peak), indices equal to {args.mode}: {same}")

    dd = None
    if args.dd_solves > 0:
        dd = dd_solve_latency(L, C, args.dd_solves)

    ds.close()
    torch.cuda.empty_cache()
    ann = None
    if not args.skip_ann:
        ann = ann_leg(L, C, args.steps)
    kmeans = None
    if not args.skip_ann and not args.skip_kmeans:
        kmeans = ann_leg(L, C, args.steps, index="kmeans", fds=(0.5, 0.8))
    serving = None
    if args.serve_solves > 0:
        serving = serve_leg(L, C, args.serve_solves, modes=tuple(args.serve_modes.split(",")))
    paper = None
    if args.paper_seeds > 0:
        paper = paper_leg(L, seeds=args.paper_seeds)

    cpu = None
    if not args.skip_cpu:
        # the oracle's whitened brute force (equal to its raw-metric form on the
        # N = 65536 workload, a CPU test) over a sample of the queries against
        # all N points; the whitening of the data set is set-up, not timed
        import oracle
        k = args.cpu_queries
        W = oracle.whiten(e, s, C)
        QW = oracle.whiten(qe[:k], qs[:k], C)
        t = time.time()
        oi, od, o2 = oracle.pd_white(W, QW)
        cpu_s = time.time() - t
        del W
        clear = o2 > od * (1 + 1e-12)
        agree = bool(np.array_equal(oi[clear], idx_mixed[:k][clear]))
        host = host_cpu()
        cpu = {"value": round(k / cpu_s, 4), "unit": "projections/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"{k} of the {m} queries against all N={N} points, the oracle's "
                         f"whitened FP64 brute force (1/2 |q - x|^2 in index order, OpenMP over "
                         f"queries), {cpu_s:.1f}s",
               "per_core": round(k / cpu_s / oracle.threads(), 4),
               "host": host, "indices_equal_gpu": agree}
        log(f"cpu oracle: {k} queries in {cpu_s:.1f}s ({oracle.threads()} threads, {host}), "
            f"agree={agree}")

    out = {
        "metric": "NN projections/s at N=2^27 (FP64 scan vs BF16+rerank); p50/p99 DD solve latency",
        "value": round(value, 2), "unit": "projections/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.mode, "data": "synthetic",
        "config": {"workload": f"mixed-precision NN projection, N=2^{args.log2n} data points, "
                               f"m={m} queries, {args.mode.upper()} MFMA scan + FP64 rerank",
                   "N": N, "m": m, "mode": args.mode, "dataset_build_s": round(build_s, 3),
                   "dataset_build_from_host_s": round(host_build_s, 3),
                   "host_input_gbs": round(N * 96 / host_build_s / 1e9, 2),
                   "candidates_per_query": round(cand / (m * args.steps), 3),
                   "fallback_queries_per_step": ovf / args.steps,
                   "slow_tiles_per_step": slow / args.steps, "tile": args.tile},
        "roofline": roofline,
        "fp64_scan": fp64,
        "fp32_scan": fp32,
        "exact_tree_walk": walk,
        "dd_solve": dd,
        "ann": ann,
        "kmeans_tree": kmeans,
        "serving": serving,
        "paper_example": paper,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
