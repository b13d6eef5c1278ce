#!/usr/bin/env python3
"""Benchmark of the P2M++ query stage on one MI355X.

Workload: displaced icosphere split 7 times (327,680 triangles), 10M query
points (5M uniform in the mesh box x1.2, 5M near-surface with sigma = 0.5% of
the box diagonal), float32.  Preprocessing (p2m_build) is excluded; inputs
are resident in HBM when timing starts.

One step = one forward pass over all 10M points: the query sort
(p2m_sort_points) followed by the search kernel (p2m_query_ordered), the two
halves of p2m_query.  HIP events on the stream the kernels run on time both
halves of every step.  Forward+backward and fused forward+backward are timed
the same way after the forward steps and reported as extra fields, followed
by the other workloads (the 960-triangle UV sphere, the cylinder + cone
symmetry stress case, the 4M-point gradient set, the batched multi-mesh form
and the augmentation ablation), none of them inside the timed steps.

Roofline of the search kernel: HBM-compulsory bytes of one launch (each
point read once, its outputs written once, and every distinct item of the
search structure the launch reads, counted once at its size by the
instrumented forward) over the kernel's event-timed average.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("kernels.hip", "device.h"):
        with open(os.path.join(ROOT, "paper_2605_00429_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_hash, n_points):
    """HBM traffic of the search kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "search_c2_10M_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash or t.get("n_points") != n_points:
        return None
    return t.get("hbm_bytes_per_launch")


def load_limiter(kernel_hash, n_points):
    """What limits the search kernel, from the committed rocprofv3 pipeline
    counters, if they were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "search_c2_10M_pipeline.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash or t.get("n_points") != n_points:
        return None
    return t.get("limiter")


def bytes_per_query(ctr, n):
    """Bytes one forward query touches, each touch at its plain size (point
    12, outputs 20, seed cell 4; per walk step the site's position and
    adjacency range 8 and 16 per neighbour read; the located site's list
    range 8; 16 per list entry scanned (bounding sphere); per exact test the
    triangle id 4 and its record 48), from the instrumented counts of this
    run.  Sorted queries share most of these touches through the caches, so
    this is the method's work per query, not HBM traffic."""
    return (12 + 20 + 4 + 8 * ctr["walk_steps"] / n + 16 * ctr["adj_read"] / n + 8
            + 16 * ctr["list_read"] / n + 52 * ctr["exact_tests"] / n)


def layout_bytes_per_query(ctr, n):
    """Bytes the kernel's own layout reads per query (each touch counted
    once): point 12, order 4, seed 4, per visited site 32, adjacency entries
    16, located site 32, 16 per scanned list entry (its sphere), 48 more per
    exact test (first vertex and both edges), the winner's record 48 + id 4,
    outputs 20."""
    return (12 + 4 + 4 + 32 * ctr["walk_steps"] / n + 16 * ctr["adj_read"] / n + 32
            + 16 * ctr["list_read"] / n + 48 * ctr["exact_tests"] / n + 52 + 20)


# Per-query input and output bytes of the search kernel: the point 12, its
# place in the visiting order 4, distance 4, triangle id 4, closest point 12.
QUERY_IO_BYTES = 12 + 4 + 20


def compulsory_bytes(items, n):
    """HBM-compulsory bytes of one search launch over n points: each point
    and its outputs once, plus every distinct structure item the launch read
    (p2m_query_touched), once at its size."""
    return QUERY_IO_BYTES * n + sum(b for _, b in items.values())


# Per-query bytes a gradient pass adds to the forward's input and output:
# dL/dD 4 in, dL/dq 12 out.
GRAD_IO_BYTES = 4 + 12


def timed(fn, steps, warmup, stream):
    """Average ms of fn() over `steps` calls after `warmup`, HIP events on
    `stream`."""
    import torch
    for _ in range(max(1, warmup)):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_batched(args, plain_c2_mqps, stream):
    """The batched multi-mesh form: 64 meshes of uneven sizes and kinds with
    uneven query counts, forward and fused forward+backward as one
    graph-captured persistent launch each, against the same work as one plain
    call per mesh on the same stream."""
    import numpy as np
    import torch

    import gen
    import paper_2605_00429_amd as p2m

    plan = gen.c4_plan()[: args.batched_meshes]
    log(f"batched workload: generating {len(plan)} meshes and their points")
    cfg = gen.config_c4(plan)
    t0 = time.time()
    meshes = []
    for k, c in enumerate(cfg):
        t1 = time.time()
        meshes.append(p2m.Mesh(c["V"], c["F"]))
        log(f"  mesh {k + 1}/{len(cfg)}: {c['name']}, {len(c['F'])} triangles, {len(c['Q'])} points, "
            f"built in {time.time() - t1:.1f}s")
    build_s = time.time() - t0
    stages = {k: 0.0 for k in ("voronoi", "optimize", "lists", "layout")}
    cells = [0, 0]
    for mm in meshes:
        sm = mm.stats()
        for k in stages:
            stages[k] += sm[f"t_{k}_s"]
        cells[0] += sm["n_cells_device"]
        cells[1] += sm["n_cells_host"]
    counts = [len(c["Q"]) for c in cfg]
    n = int(sum(counts))
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    n_tris = int(sum(len(c["F"]) for c in cfg))
    n_verts = [len(c["V"]) for c in cfg]
    n_tri_each = [len(c["F"]) for c in cfg]
    kinds = [c["name"].split()[-1] for c in cfg]
    log(f"batched workload: {len(cfg)} meshes, {n_tris} triangles, {n} points; build {build_s:.1f}s")
    dev = torch.device("cuda", 0)
    q = torch.from_numpy(np.concatenate([c["Q"] for c in cfg], 0)).to(dev)
    # a few meshes' points to check against the oracle afterwards
    picks = sorted({0, len(cfg) // 2, len(cfg) - 1})
    sample_src = [(cfg[i]["V"], cfg[i]["F"], cfg[i]["D"], i) for i in picks]
    del cfg
    g = torch.from_numpy(np.random.default_rng(2605_00429 + 4).normal(size=n).astype(np.float32)).to(dev)
    dist = torch.empty(n, device=dev)
    tri = torch.empty(n, dtype=torch.int32, device=dev)
    cl = torch.empty((n, 3), device=dev)
    gq = torch.empty((n, 3), device=dev)
    voff = np.concatenate([[0], np.cumsum(n_verts)]).astype(np.int64)
    gv_flat = torch.zeros((int(voff[-1]), 3), device=dev)
    gvs = [gv_flat[voff[i]:voff[i + 1]] for i in range(len(meshes))]
    qs = [q[off[i]:off[i + 1]] for i in range(len(meshes))]

    # compulsory bytes: per-mesh instrumented forwards (untimed), each
    # mesh's distinct structure items plus every point's input and output
    comp = 0.0
    ctrs = []
    for i, m in enumerate(meshes):
        ctrs.append(None)
        if counts[i]:
            _, _, _, ctrs[i], items = p2m.query_touched(m, qs[i])
            comp += compulsory_bytes(items, counts[i])
    torch.cuda.synchronize()

    b_fwd = p2m.Batch(meshes, counts, autotune=True)
    b_fwd.bind(q, dist, tri, cl, stream=stream)
    b_fus = p2m.Batch(meshes, counts, autotune=True)
    b_fus.bind(q, dist, tri, cl, grad_dist=g, grad_points=gq, grad_vertices=gvs, stream=stream)

    outs = [(dist[off[i]:off[i + 1]], tri[off[i]:off[i + 1]], cl[off[i]:off[i + 1]]) for i in range(len(meshes))]

    def plain_fwd():
        for i, m in enumerate(meshes):
            p2m.lib().p2m_query(m.handle, p2m._ptr(qs[i]), counts[i], p2m._ptr(outs[i][0]), p2m._ptr(outs[i][1]),
                                p2m._ptr(outs[i][2]), p2m._stream(stream))

    def plain_fused():
        gv_flat.zero_()
        for i, m in enumerate(meshes):
            p2m.lib().p2m_query_fused(m.handle, p2m._ptr(qs[i]), counts[i], p2m._ptr(g[off[i]:off[i + 1]]),
                                      p2m._ptr(outs[i][0]), p2m._ptr(outs[i][1]), p2m._ptr(outs[i][2]),
                                      p2m._ptr(gq[off[i]:off[i + 1]]), p2m._ptr(gvs[i]), p2m._stream(stream))

    def batched_fused():
        gv_flat.zero_()
        b_fus.launch(stream=stream)

    steps, warm = max(3, args.steps // 2), max(1, args.warmup)
    # where the time goes: each mesh's plain forward timed alone, summed by
    # mesh kind with the instrumented per-query counts
    by_kind = {}
    for i, m in enumerate(meshes):
        if not counts[i]:
            continue
        ms_i = timed(lambda: p2m.lib().p2m_query(m.handle, p2m._ptr(qs[i]), counts[i], p2m._ptr(outs[i][0]),
                                                 p2m._ptr(outs[i][1]), p2m._ptr(outs[i][2]), p2m._stream(stream)),
                     3, 1, stream)
        k = by_kind.setdefault(kinds[i], {"meshes": 0, "points": 0, "triangles": 0, "plain_ms": 0.0,
                                          "list_len": 0, "list_read": 0, "exact_tests": 0})
        k["meshes"] += 1
        k["points"] += counts[i]
        k["triangles"] += n_tri_each[i]
        k["plain_ms"] += ms_i
        for c in ("list_len", "list_read", "exact_tests"):
            k[c] += ctrs[i][c]
    for k in by_kind.values():
        k["plain_ms"] = round(k["plain_ms"], 3)
        k["mqps"] = round(k["points"] / (k["plain_ms"] * 1e-3) / 1e6, 1)
        for c in ("list_len", "list_read", "exact_tests"):
            k[c] = round(k[c] / max(k["points"], 1), 1)
        k["queried"] = k.pop("list_len")
    ms_b = timed(lambda: b_fwd.launch(stream=stream), steps, warm, stream)
    ms_p = timed(plain_fwd, steps, warm, stream)
    ms_bf = timed(batched_fused, steps, warm, stream)
    ms_pf = timed(plain_fused, steps, warm, stream)
    mq = lambda ms: round(n / (ms * 1e-3) / 1e6, 2)
    gbs = lambda per, ms: round(per / (ms * 1e-3) / 1e9, 1)
    res = {
        "workload": (f"the 64-mesh plan" if len(meshes) == 64 else f"the first {len(meshes)} of a 64-mesh plan") +
                    " (uv sphere, capped cylinder, capped cone, torus, displaced icosphere): "
                    f"{n_tris} triangles, log-uniform 1e3-5e5 per mesh; {n} points, log-uniform 1e4-2e6 per "
                    "mesh, half uniform in box x1.2, half near-surface sigma 0.5% diag",
        "n_points": n, "n_triangles": n_tris, "build_s": round(build_s, 1),
        "build_stages_s": {**{k: round(v, 1) for k, v in stages.items()}, "cells_device": cells[0],
                           "cells_host": cells[1]},
        "fwd_ms": round(ms_b, 4), "fwd_mqps": mq(ms_b),
        "plain_fwd_ms": round(ms_p, 4), "plain_fwd_mqps": mq(ms_p),
        "fwd_vs_plain": round(ms_p / ms_b, 4),
        "fwd_vs_c2_plain_forward": round(mq(ms_b) / plain_c2_mqps, 4),
        "fwd_bwd_ms": round(ms_bf, 4), "fwd_bwd_mqps": mq(ms_bf),
        "plain_fwd_bwd_ms": round(ms_pf, 4), "plain_fwd_bwd_mqps": mq(ms_pf),
        "fwd_bwd_vs_plain": round(ms_pf / ms_bf, 4),
        "compulsory_bytes_per_query": round(comp / n, 1),
        "fwd_compulsory_GBps": gbs(comp, ms_b),
        "fwd_compulsory_frac": round(gbs(comp, ms_b) / HBM_PEAK_GBS, 4),
        "fwd_bwd_compulsory_GBps": gbs(comp + GRAD_IO_BYTES * n + 24 * int(voff[-1]), ms_bf),
        "launch_config": b_fwd.config(),
        "by_kind": by_kind,
    }
    log(f"batched forward {ms_b:.3f} ms ({res['fwd_mqps']:.1f} Mq/s) vs {len(meshes)} plain calls "
        f"{ms_p:.3f} ms; fused batched {ms_bf:.3f} ms vs plain {ms_pf:.3f} ms")
    b_fwd.launch(stream=stream)
    torch.cuda.synchronize()
    samples = []
    for V, F, D, i in sample_src:
        k = min(500, counts[i])
        sl = slice(int(off[i]), int(off[i]) + k)
        samples.append((V, F, D, q[sl].cpu().numpy(), dist[sl].cpu().numpy()))
    b_fwd.close()
    b_fus.close()
    return res, samples


def bench_ablation(args, stream):
    """Auxiliary sites on and off (the shape of the paper's Tab. 4): list
    Max / Avg / Queried, preprocessing seconds and query rate, on a
    tessellated sphere with the paper's Sphere face count, a capped cylinder
    and cone (rotational symmetry) and the organic displaced icosphere, for
    1M points uniform in the mesh box scaled 10x (the paper's query region)
    and for the 50/50 uniform (box x1.2) / near-surface mix."""
    import numpy as np
    import torch

    import gen
    import paper_2605_00429_amd as p2m

    meshes = [("icosphere-5", gen.icosphere(5)),
              ("capped cylinder 256x64", gen.capped_cylinder(1.0, 2.0, 256, 64)),
              ("capped cone 256x64", gen.capped_cone(1.0, 2.0, 256, 64)),
              ("displaced icosphere-6", gen.displaced_icosphere(6, np.random.default_rng(2605_00429 + 5)))]
    out = []
    for name, (V, F) in meshes:
        rng = np.random.default_rng(2605_00429 + 6)
        lo, hi = gen.scaled_box(V, 10.0)
        sets = {"box x10": gen.uniform_box(rng, 1_000_000, lo, hi)}
        lo, hi = gen.scaled_box(V, 1.2)
        D = float(np.linalg.norm(V.max(0) - V.min(0)))
        sets["mix"] = np.concatenate([gen.uniform_box(rng, 500_000, lo, hi),
                                      gen.near_surface(rng, 500_000, V, F, 0.005 * D)]).astype(np.float32)
        for aug in (0, 1):
            t0 = time.time()
            m = p2m.Mesh(V, F, augment=aug)
            pre = time.time() - t0
            st = m.stats()
            row = {"mesh": name, "faces": len(F), "augment": aug, "aux_sites": st["n_aux_sites"],
                   "pre_s": round(pre, 2), "list_max": st["list_max"], "list_avg": round(st["list_avg"], 1)}
            for key, Q in sets.items():
                q = torch.from_numpy(np.ascontiguousarray(Q, dtype=np.float32)).cuda()
                n = len(q)
                _, _, _, ctr = p2m.query_counters(m, q)
                d = torch.empty(n, device=q.device)
                t = torch.empty(n, dtype=torch.int32, device=q.device)
                c = torch.empty((n, 3), device=q.device)
                ms = timed(lambda: p2m.lib().p2m_query(m.handle, p2m._ptr(q), n, p2m._ptr(d), p2m._ptr(t),
                                                        p2m._ptr(c), p2m._stream(stream)), 5, 2, stream)
                row[f"queried[{key}]"] = round(ctr["list_len"] / n, 1)
                row[f"mqps[{key}]"] = round(n / (ms * 1e-3) / 1e6, 1)
                if not args.no_exact:
                    torch.cuda.synchronize()
                    e, _, _, _, _ = forward_errors(V, F, Q, d.cpu().numpy(), D)
                    row[f"fp64_error_over_diag[{key}]"] = e
            log(f"ablation {row}")
            out.append(row)
            del m
    return out


def err_stats(x):
    """max and p99.9 of an error array (NaN-free), as floats."""
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    if len(x) == 0:
        return {"max": None, "p99.9": None}
    return {"max": float(x.max()), "p99.9": float(np.quantile(x, 0.999))}


def forward_errors(V, F, Q, d_gpu, D, n_threads=0):
    """|d_gpu - d64| / D against the oracle's exact result for every point
    (tier-B branch-and-bound, bit-identical to the brute force); returns the
    max / p99.9 and the oracle's (d64, tri64, seconds, threads)."""
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    d64, t64, _, used = oracle.distance_exact(V, F, Q, n_threads=n_threads, want_closest=False)
    sec = time.perf_counter() - t0
    ok = np.isfinite(d64)
    e = err_stats(np.abs(np.asarray(d_gpu, np.float64)[ok] - d64[ok]) / D)
    e["points"] = int(ok.sum())
    return e, d64, t64, sec, used


def grad_row_errors(G, G64):
    """Per-row relative error of a gradient against the FP64 one: the row's
    error over the row's norm, floored at 1e-3 of the rms row."""
    import numpy as np
    G, G64 = np.asarray(G, np.float64), np.asarray(G64, np.float64)
    rms = float(np.sqrt(np.mean(np.sum(G64 ** 2, axis=1)))) if len(G64) else 0.0
    row = np.linalg.norm(G - G64, axis=1) / np.maximum(np.linalg.norm(G64, axis=1), max(1e-3 * rms, 1e-30))
    out = err_stats(row)
    out["normwise"] = float(np.linalg.norm(G - G64) / max(np.linalg.norm(G64), 1e-30))
    return out


def time_query(p2m, mesh, q, stream, steps, warmup):
    """ms of one p2m_query (sort + search) over q, outputs preallocated."""
    import torch
    n = len(q)
    d = torch.empty(n, device=q.device)
    t = torch.empty(n, dtype=torch.int32, device=q.device)
    c = torch.empty((n, 3), device=q.device)
    ms = timed(lambda: p2m.lib().p2m_query(mesh.handle, p2m._ptr(q), n, p2m._ptr(d), p2m._ptr(t), p2m._ptr(c),
                                           p2m._stream(stream)), steps, warmup, stream)
    torch.cuda.synchronize()
    return ms, (d, t, c)


def bench_small_configs(args, stream):
    """The 960-triangle UV sphere (10k points) and the cylinder + cone
    symmetry stress case (263,168 triangles, 1M uniform + 1M near-surface
    points): forward rate, list statistics and FP64 error over every point."""
    import numpy as np
    import torch

    import gen
    import paper_2605_00429_amd as p2m

    out = {}
    for key, mk in (("C0", gen.config_c0), ("C1", gen.config_c1)):
        c = mk()
        V, F, Q, D = c["V"], c["F"], c["Q"], c["D"]
        t0 = time.time()
        m = p2m.Mesh(V, F)
        build_s = time.time() - t0
        st = m.stats()
        q = torch.from_numpy(Q).cuda()
        n = len(Q)
        _, _, _, ctr = p2m.query_counters(m, q)
        ms, (d, _, _) = time_query(p2m, m, q, stream, args.steps, args.warmup)
        err, _, _, sec, used = forward_errors(V, F, Q, d.cpu().numpy(), D)
        out[key] = {"workload": c["name"], "n_points": n, "n_triangles": len(F), "build_s": round(build_s, 2),
                    "aux_sites": st["n_aux_sites"], "list_avg": round(st["list_avg"], 1),
                    "list_max": st["list_max"], "queried": round(ctr["list_len"] / n, 1),
                    "list_read": round(ctr["list_read"] / n, 1), "exact_tests": round(ctr["exact_tests"] / n, 2),
                    "walk_steps": round(ctr["walk_steps"] / n, 3), "ms": round(ms, 4),
                    "mqps": round(n / (ms * 1e-3) / 1e6, 2), "fp64_error_over_diag": err,
                    "oracle_tier_b_s": round(sec, 2)}
        log(f"{key}: {out[key]}")
        del m, q
    return out


def bench_c3(args, mesh, V, F, D, stream):
    """The gradient set: the 327,680-triangle mesh with 4M near-surface
    points and dL/dd ~ N(0, 1): forward, backward alone (the forward's
    order and triangles given), forward + backward and fused, and the FP64
    error of the distances and of both gradients over every point."""
    import numpy as np
    import torch

    import gen
    import oracle
    import paper_2605_00429_amd as p2m

    c = gen.config_c3()
    Q, G = c["Q"], c["G"]
    n = len(Q)
    dev = torch.device("cuda", 0)
    q = torch.from_numpy(Q).to(dev)
    g = torch.from_numpy(G).to(dev)
    order = torch.empty(n, dtype=torch.int32, device=dev)
    d = torch.empty(n, device=dev)
    t = torch.empty(n, dtype=torch.int32, device=dev)
    cl = torch.empty((n, 3), device=dev)
    gq = torch.empty((n, 3), device=dev)
    gv = torch.zeros((len(V), 3), device=dev)
    L = p2m.lib()
    S = p2m._stream(stream)

    def fwd():
        L.p2m_sort_points(mesh.handle, p2m._ptr(q), n, p2m._ptr(order), None, S)
        L.p2m_query_ordered(mesh.handle, p2m._ptr(q), p2m._ptr(order), n, p2m._ptr(d), p2m._ptr(t), p2m._ptr(cl), S)

    def bwd():
        gv.zero_()
        L.p2m_query_backward_ordered(mesh.handle, p2m._ptr(q), p2m._ptr(order), n, p2m._ptr(t), p2m._ptr(g),
                                     p2m._ptr(gq), p2m._ptr(gv), S)

    def fwd_bwd():
        fwd()
        bwd()

    def fused():
        gv.zero_()
        L.p2m_query_fused(mesh.handle, p2m._ptr(q), n, p2m._ptr(g), p2m._ptr(d), p2m._ptr(t), p2m._ptr(cl),
                          p2m._ptr(gq), p2m._ptr(gv), S)

    res = {"workload": c["name"] + f": {n} near-surface points, sigma 0.5% diag, dL/dd ~ N(0, 1)", "n_points": n}
    fwd()
    torch.cuda.synchronize()
    for name, fn in (("fwd", fwd), ("bwd", bwd), ("fwd_bwd", fwd_bwd), ("fused", fused)):
        ms = timed(fn, args.steps, args.warmup, stream)
        res[f"{name}_ms"] = round(ms, 4)
        res[f"{name}_mqps"] = round(n / (ms * 1e-3) / 1e6, 2)
    for name in ("fwd_bwd", "fused"):
        res[f"{name}_vs_fwd"] = round(res[f"{name}_mqps"] / res["fwd_mqps"], 4)
    # FP64 error of the fused outputs (the last run) and gradients
    fused()
    torch.cuda.synchronize()
    dn, tn = d.cpu().numpy(), t.cpu().numpy()
    err, _, _, sec, _ = forward_errors(V, F, Q, dn, D)
    res["fp64_error_over_diag"] = err
    dq64, dV64 = oracle.gradient(V, F, Q, tn, G)
    res["fused_grad_points_error"] = grad_row_errors(gq.cpu().numpy(), dq64)
    res["fused_grad_vertices_error"] = grad_row_errors(gv.cpu().numpy(), dV64)
    fwd_bwd()
    torch.cuda.synchronize()
    res["bwd_grad_points_error"] = grad_row_errors(gq.cpu().numpy(), dq64)
    res["bwd_grad_vertices_error"] = grad_row_errors(gv.cpu().numpy(), dV64)
    log(f"C3: {res}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--points", type=int, default=10_000_000, help="total points (half uniform, half near-surface)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grad", action="store_true", help="skip the forward+backward timings")
    ap.add_argument("--cpu-sample", type=int, default=16000)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched multi-mesh measurement")
    ap.add_argument("--no-point-set", action="store_true",
                    help="skip the point-set distance measurement (profiling runs: it launches the search "
                         "kernel with fewer outputs)")
    ap.add_argument("--batched-meshes", type=int, default=64,
                    help="meshes of the batched workload: the first k of its 64-mesh plan (all 64: about "
                         "2 minutes of preprocessing)")
    ap.add_argument("--octree", action="store_true",
                    help="add the octree decomposition (leaf boxes instead of Voronoi cells) on the same workload")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the augmentation ablation (with and without auxiliary sites) on symmetric meshes")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (UV sphere, cylinder + cone, the 4M-point gradient set)")
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the FP64 error over every point (the exact tree oracle on the host)")
    ap.add_argument("--xcd-groups", type=int, default=None,
                    help="launch configuration of the main workload: give each of this many XCDs a "
                         "contiguous range of the sorted points (default: the library's)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device copy, the reference kernel for scaling "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the query path shards "
              "by replicating the mesh structure and splitting the points, which this build does not run.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2605_00429_amd as p2m

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written by one copy kernel")
        del src, dst

    log("generating workload")
    n_half = args.points // 2
    c = gen.config_c2(n_half, args.points - n_half)
    V, F, Q, D = c["V"], c["F"], c["Q"], c["D"]
    n = len(Q)
    log(f"mesh {len(V)} vertices / {len(F)} triangles, {n} points; building search structure")
    t0 = time.time()
    mesh = p2m.Mesh(V, F)
    build_s = time.time() - t0
    if args.xcd_groups is not None:
        mesh.set_query_config(xcd_groups=args.xcd_groups)
    st = mesh.stats()
    log(f"build {build_s:.1f}s: {st['n_sites']} sites ({st['n_aux_sites']} auxiliary), "
        f"lists avg {st['list_avg']:.1f} max {st['list_max']}, adjacency avg {st['adj_avg']:.1f}")

    q = torch.from_numpy(Q).to(dev)
    stream = torch.cuda.current_stream()

    # per-query counts and the distinct structure items one launch reads,
    # from the instrumented forward (same results, untimed)
    _, _, _, ctr, items = p2m.query_touched(mesh, q)
    torch.cuda.synchronize()
    bpq = bytes_per_query(ctr, n)
    lbpq = layout_bytes_per_query(ctr, n)
    comp = compulsory_bytes(items, n)
    log(f"per query: walk steps {ctr['walk_steps'] / n:.2f}, adjacency read {ctr['adj_read'] / n:.1f}, "
        f"list read {ctr['list_read'] / n:.1f} of {ctr['list_len'] / n:.1f}, exact tests "
        f"{ctr['exact_tests'] / n:.2f}, fallback {ctr['fallback']}; touched {bpq:.0f} B/query; "
        f"compulsory {comp / n:.1f} B/query (structure read: {sum(b for _, b in items.values()) / 1e6:.1f} MB)")

    order = torch.empty(n, dtype=torch.int32, device=dev)
    out = (torch.empty(n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
           torch.empty((n, 3), dtype=torch.float32, device=dev))

    def step():
        p2m.lib().p2m_sort_points(mesh.handle, p2m._ptr(q), n, p2m._ptr(order), None, p2m._stream(stream))
        ev_mid.record(stream)
        p2m.query_ordered(mesh, q, order, out=out, stream=stream)

    ev_mid = torch.cuda.Event(enable_timing=True)
    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    mids = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        ev_mid = mids[k]
        step()
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    step_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    sort_ms = [s.elapsed_time(m) for s, m in zip(starts, mids)]
    search_ms = [m.elapsed_time(e) for m, e in zip(mids, ends)]
    ms_per_step = sum(step_ms) / args.steps
    search_avg = sum(search_ms) / args.steps
    mqps = n / (ms_per_step * 1e-3) / 1e6
    log(f"forward: {ms_per_step:.3f} ms/step (sort {sum(sort_ms) / args.steps:.3f}, search "
        f"{search_avg:.3f}) = {mqps:.1f} Mq/s; wall {wall:.3f}s")

    result = {
        "metric": "Mqueries/s fwd and fwd+bwd, 327k-tri mesh, 10M pts; achieved HBM GB/s",
        "value": round(mqps, 2),
        "unit": "Mqueries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "displaced icosphere-7 (327,680 triangles, 163,842 vertices); "
                        f"{n} points: {n_half} uniform in box x1.2 + {n - n_half} near-surface sigma 0.5% diag",
            "n_points": n, "n_triangles": len(F),
        },
    }

    kh = kernel_source_hash()
    # which search the library ran (p2m_query_config.group; 2 = automatic)
    grp = mesh.query_config()["group"]
    grouped = grp == 1 or (grp == 2 and n >= 2000000)
    search_path = ("search phase of p2m_query_ordered: locate_kernel, sort by site, grouped_kernel "
                   "(list chunks shared through LDS)" if grouped else
                   "search phase of p2m_query_ordered: fwd_kernel (walk, regroup, per-lane list scans)")
    achieved = comp / (search_avg * 1e-3) / 1e9
    traffic = load_traffic(kh, n)
    result["roofline"] = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
        "kernel": search_path, "kernel_ms": round(search_avg, 4),
        "compulsory_bytes_per_launch": int(comp), "compulsory_bytes_per_query": round(comp / n, 1),
        "structure_items_read": {k: v[0] for k, v in items.items()},
        "touched_bytes_per_query": round(bpq, 1),
        "touched_GBps": round(bpq * n / (search_avg * 1e-3) / 1e9, 1),
        "layout_bytes_per_query": round(lbpq, 1), "kernel_hash": kh,
    }
    if traffic:
        result["roofline"]["traffic_GBps"] = round(traffic / (search_avg * 1e-3) / 1e9, 1)
        result["roofline"]["traffic_counts"] = "FETCH_SIZE + WRITE_SIZE: L2-to-fabric requests (MALL or HBM)"
    lim = load_limiter(kh, n)
    if lim:
        result["roofline"]["limiter"] = lim
    result["forward_step_compulsory_GBps"] = round(comp / (ms_per_step * 1e-3) / 1e9, 1)
    result["sort_ms"] = round(sum(sort_ms) / args.steps, 4)
    result["per_query"] = {k: round(v / n, 3) for k, v in ctr.items()}
    result["structure"] = {k: st[k] for k in ("n_sites", "n_aux_sites", "list_avg", "list_max", "adj_avg",
                                              "list_nnz", "device_bytes")}
    result["build_s"] = round(build_s, 2)
    # the stages of a second build of the same mesh (the first one also pays
    # the device's one-time set-up): Tab. 3's Voronoi build / optimize / list
    # build columns, and where the Voronoi cells were built
    t0 = time.time()
    st2 = p2m.Mesh(V, F).stats()
    result["build_stages_s"] = {"total": round(time.time() - t0, 3),
                                **{k: round(st2[f"t_{k}_s"], 3) for k in ("voronoi", "optimize", "lists", "layout")},
                                "cells_device": st2["n_cells_device"], "cells_host": st2["n_cells_host"]}

    # mesh-to-mesh building block: the same points reduced on the device to
    # max / argmax / sums (one-sided Hausdorff distance and Chamfer term)
    red = torch.empty(5, dtype=torch.float64, device=dev)
    ms_red = None if args.no_point_set else timed(lambda: p2m.lib().p2m_point_set_distance(mesh.handle, p2m._ptr(q), n, p2m._ptr(red),
                                                            p2m._stream(stream)), args.steps, args.warmup, stream)
    if ms_red is not None:
        result["point_set_distance"] = {"ms": round(ms_red, 4), "mqps": round(n / (ms_red * 1e-3) / 1e6, 2),
                                        "vs_forward": round(ms_per_step / ms_red, 4)}
        log(f"point-set distance (query + reduction): {ms_red:.3f} ms")

    if not args.no_grad:
        g = torch.from_numpy(np.random.default_rng(2605_00429 + 3).normal(size=n).astype(np.float32)).to(dev)
        gv = torch.zeros((len(V), 3), dtype=torch.float32, device=dev)
        gq = torch.empty((n, 3), dtype=torch.float32, device=dev)

        # forward then backward, the points sorted once for both passes
        def fwd_bwd():
            gv.zero_()
            p2m.lib().p2m_sort_points(mesh.handle, p2m._ptr(q), n, p2m._ptr(order), None, p2m._stream(stream))
            p2m.query_ordered(mesh, q, order, out=out, stream=stream)
            p2m.lib().p2m_query_backward_ordered(mesh.handle, p2m._ptr(q), p2m._ptr(order), n, p2m._ptr(out[1]),
                                                 p2m._ptr(g), p2m._ptr(gq), p2m._ptr(gv), p2m._stream(stream))

        def fused():
            gv.zero_()
            p2m.lib().p2m_query_fused(mesh.handle, p2m._ptr(q), n, p2m._ptr(g), p2m._ptr(out[0]),
                                      p2m._ptr(out[1]), p2m._ptr(out[2]), p2m._ptr(gq), p2m._ptr(gv),
                                      p2m._stream(stream))

        for name, fn in (("fwd_bwd", fwd_bwd), ("fused", fused)):
            for _ in range(max(1, args.warmup)):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.steps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            result[f"{name}_mqps"] = round(n / (ms * 1e-3) / 1e6, 2)
            result[f"{name}_ms"] = round(ms, 4)
            # compulsory bytes of the whole job: the forward's, plus g and
            # dL/dq per point and dL/dV read and written once per vertex
            comp_g = comp + GRAD_IO_BYTES * n + 24 * len(V)
            result[f"{name}_compulsory_GBps"] = round(comp_g / (ms * 1e-3) / 1e9, 1)
            result[f"{name}_compulsory_frac"] = round(result[f"{name}_compulsory_GBps"] / HBM_PEAK_GBS, 4)
            result[f"{name}_vs_forward"] = round(result[f"{name}_mqps"] / mqps, 4)
            log(f"{name}: {ms:.3f} ms/step = {result[f'{name}_mqps']:.1f} Mq/s")

    if not args.no_batched:
        result["batched"], batched_samples = bench_batched(args, mqps, stream)

    if args.octree:
        t0 = time.time()
        mo = p2m.Mesh(V, F, decomposition=1, octree_max_list=512, octree_max_depth=8)
        ob = time.time() - t0
        so = mo.stats()
        _, _, _, ctr_o = p2m.query_counters(mo, q)
        ms_o = timed(lambda: p2m.lib().p2m_query(mo.handle, p2m._ptr(q), n, p2m._ptr(out[0]), p2m._ptr(out[1]),
                                                  p2m._ptr(out[2]), p2m._stream(stream)), args.steps, args.warmup, stream)
        result["octree"] = {"max_list": 512, "max_depth": 8, "leaves": so["n_sites"], "list_avg": round(so["list_avg"], 1),
                            "list_nnz": so["list_nnz"], "device_bytes": so["device_bytes"], "build_s": round(ob, 1),
                            "queried": round(ctr_o["list_len"] / n, 1), "list_read": round(ctr_o["list_read"] / n, 1),
                            "exact_tests": round(ctr_o["exact_tests"] / n, 2), "descent_steps": round(ctr_o["walk_steps"] / n, 2),
                            "ms": round(ms_o, 4), "mqps": round(n / (ms_o * 1e-3) / 1e6, 2),
                            "vs_voronoi": round(ms_per_step / ms_o, 4)}
        log(f"octree: {result['octree']}")
        del mo

    if not args.no_configs:
        result["configs"] = bench_small_configs(args, stream)
        result["configs"]["C3"] = bench_c3(args, mesh, V, F, D, stream)

    if not args.no_ablation:
        result["ablation"] = bench_ablation(args, stream)

    fp64 = {}
    if not args.no_exact:
        # every one of the 10M distances against the oracle's exact result
        # (re-run the forward: the fused timings above overwrote the outputs)
        step()
        torch.cuda.synchronize()
        e, d64, t64, sec, used = forward_errors(V, F, Q, out[0].cpu().numpy(), D)
        fp64["forward_over_diag"] = e
        result["oracle_tier_b"] = {"mqps": round(n / sec / 1e6, 4), "seconds": round(sec, 2), "cores": int(used),
                                   "kind": "exact FP64 branch-and-bound over a box tree (the oracle's own)"}
        log(f"forward FP64 error over {n} points: {e}; exact oracle {sec:.1f}s on {used} threads")
        if not args.no_grad:
            import oracle
            fused()
            torch.cuda.synchronize()
            tg = out[1].cpu().numpy()
            dq64, dV64 = oracle.gradient(V, F, Q, tg, g.cpu().numpy())
            fp64["fused_grad_points"] = grad_row_errors(gq.cpu().numpy(), dq64)
            fp64["fused_grad_vertices"] = grad_row_errors(gv.cpu().numpy(), dV64)
            log(f"fused gradient FP64 error: {fp64['fused_grad_points']}, {fp64['fused_grad_vertices']}")

    if not args.no_cpu_baseline:
        import oracle
        k = max(2, args.cpu_sample)
        idx = np.concatenate([np.arange(k // 2), n_half + np.arange(k - k // 2)])
        Qs = np.ascontiguousarray(Q[idx])
        log(f"oracle on {len(Qs)} sampled points (brute force over {len(F)} triangles)")
        t0 = time.perf_counter()
        d64, t64, _, used = oracle.distance(V, F, Qs, want_closest=False)
        cpu_s = time.perf_counter() - t0
        d_gpu = out[0][torch.from_numpy(idx).to(dev)].cpu().numpy()
        err = np.abs(d_gpu.astype(np.float64) - d64) / D
        result["cpu_baseline"] = {
            "value": round(len(Qs) / cpu_s / 1e6, 6), "unit": "Mqueries/s", "cores": int(used),
            "kind": "oracle",
            "sample": f"{len(Qs)} points ({k // 2} uniform + {k - k // 2} near-surface, the first of each "
                      f"half of the workload), FP64 brute force over all {len(F)} triangles, {cpu_s:.1f}s",
        }
        log(f"oracle {cpu_s:.1f}s on {used} threads; GPU max |d - d64| / D on the sample = {err.max():.2e}")
        if not args.no_batched:
            bmax = 0.0
            for Vb, Fb, Db, Qb, db in batched_samples:
                d64b, _, _, _ = oracle.distance(Vb, Fb, Qb, want_closest=False)
                bmax = max(bmax, float(np.max(np.abs(db.astype(np.float64) - d64b)) / Db))
            fp64["batched_max_abs_err_over_diag"] = bmax
            fp64["batched_points_compared"] = int(sum(len(x[3]) for x in batched_samples))
    result["fp64_error"] = fp64
    log(f"FP64 error: {fp64}")

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
