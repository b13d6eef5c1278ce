"""Batched multi-mesh queries: one persistent, graph-captured launch must give
exactly the per-mesh plain-launch results (the per-point code is shared)."""
import os

import numpy as np
import pytest

import gen
import oracle

from gpu_util import check_forward, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_00429_amd as p2m
    return p2m


@pytest.fixture(scope="module")
def c4_small(dev):
    """The C4 recipe with the first 10 meshes, triangle counts capped at 8,000
    and 5% of the points (host preprocessing of the full set takes minutes)."""
    plan = [(k, min(t, 8000), q) for k, t, q in gen.c4_plan()[:10]]
    cfg = gen.config_c4(plan, query_scale=0.05)
    meshes = [dev.Mesh(c["V"], c["F"]) for c in cfg]
    return cfg, meshes


def concat_points(cfg):
    Q = np.concatenate([c["Q"] for c in cfg], 0)
    off = np.concatenate([[0], np.cumsum([len(c["Q"]) for c in cfg])])
    return Q, off


def test_batched_forward_equals_plain(dev, c4_small, tmp_path):
    cfg, meshes = c4_small
    Q, off = concat_points(cfg)
    n = len(Q)
    q = torch.from_numpy(Q).cuda()
    dist = torch.empty(n, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    cl = torch.empty((n, 3), device="cuda")
    cache = str(tmp_path / "tune.txt")
    b = dev.Batch(meshes, [len(c["Q"]) for c in cfg], autotune=True, cache_path=cache)
    b.bind(q, dist, tri, cl)
    ref = []
    for i, m in enumerate(meshes):
        ref.append(dev.query(m, q[off[i]:off[i + 1]].contiguous()))
    for rep in range(3):
        dist.fill_(-1.0)
        tri.fill_(-7)
        b.launch()
        torch.cuda.synchronize()
        # eager work between graph replays
        _ = (q * 2).sum().item()
        for i in range(len(meshes)):
            s = slice(off[i], off[i + 1])
            assert torch.equal(dist[s], ref[i][0]), (rep, i)
            assert torch.equal(tri[s], ref[i][1]), (rep, i)
            assert torch.equal(cl[s], ref[i][2]), (rep, i)
    # a second batch over the same sizes takes the cached configuration
    cfg1 = b.config()
    b2 = dev.Batch(meshes, [len(c["Q"]) for c in cfg], autotune=True, cache_path=cache)
    b2.bind(q, dist, tri, cl)
    assert b2.config() == cfg1
    assert os.path.exists(cache)
    # and both match the oracle on a sample
    for i in (0, len(meshes) - 1):
        s = slice(off[i], off[i + 1])
        idx = np.arange(off[i], min(off[i + 1], off[i] + 1500))
        check_forward(cfg[i]["V"], cfg[i]["F"], Q[idx], to_np(dist)[idx], to_np(tri)[idx], to_np(cl)[idx],
                      cfg[i]["D"], label=cfg[i]["name"])


def test_batched_fused_equals_plain(dev, c4_small):
    cfg, meshes = c4_small
    Q, off = concat_points(cfg)
    n = len(Q)
    rng = np.random.default_rng(31)
    q = torch.from_numpy(Q).cuda()
    g = torch.from_numpy(rng.normal(size=n).astype(np.float32)).cuda()
    dist = torch.empty(n, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    cl = torch.empty((n, 3), device="cuda")
    gq = torch.empty((n, 3), device="cuda")
    gvs = [torch.zeros((len(m.V), 3), device="cuda") for m in meshes]
    b = dev.Batch(meshes, [len(c["Q"]) for c in cfg], autotune=False)
    b.bind(q, dist, tri, cl, grad_dist=g, grad_points=gq, grad_vertices=gvs)
    for rep in range(2):
        for t in gvs:
            t.zero_()
        b.launch()
        torch.cuda.synchronize()
        for i, m in enumerate(meshes):
            s = slice(off[i], off[i + 1])
            gv_ref = torch.zeros_like(gvs[i])
            d, t, c, gq_ref = dev.query_fused(m, q[s].contiguous(), g[s].contiguous(), grad_vertices=gv_ref)
            torch.cuda.synchronize()
            assert torch.equal(dist[s], d) and torch.equal(tri[s], t) and torch.equal(gq[s], gq_ref)
            err = torch.linalg.norm(gvs[i] - gv_ref) / max(torch.linalg.norm(gv_ref).item(), 1e-30)
            assert err <= 1e-5, (rep, i, err)


@pytest.mark.parametrize("tile,grid,block,stage", [(256, 0, 256, 0), (512, 0, 512, 1), (2048, 512, 256, 0),
                                                   (1024, 1024, 512, 1)])
def test_batched_launch_modes_equal_plain(dev, c4_small, tile, grid, block, stage):
    """Both launch modes (one workgroup per item, or a persistent grid taking
    items from the queue), at two workgroup sizes, with and without LDS
    staging: forward and fused outputs equal one plain call per mesh bit for
    bit (dL/dV up to the order of float32 additions)."""
    cfg, meshes = c4_small
    Q, off = concat_points(cfg)
    n = len(Q)
    q = torch.from_numpy(Q).cuda()
    g = torch.from_numpy(np.random.default_rng(33).normal(size=n).astype(np.float32)).cuda()
    dist = torch.empty(n, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    cl = torch.empty((n, 3), device="cuda")
    gq = torch.empty((n, 3), device="cuda")
    gvs = [torch.zeros((len(m.V), 3), device="cuda") for m in meshes]
    b = dev.Batch(meshes, [len(c["Q"]) for c in cfg], autotune=False)
    b.set_config(tile, grid, block, stage)
    b.bind(q, dist, tri, cl)
    assert b.config() == {"tile": tile, "grid": grid, "block": block, "stage": stage}
    bf = dev.Batch(meshes, [len(c["Q"]) for c in cfg], autotune=False)
    bf.set_config(tile, grid, block, stage)
    bf.bind(q, torch.empty_like(dist), torch.empty_like(tri), torch.empty_like(cl), grad_dist=g, grad_points=gq,
            grad_vertices=gvs)
    for rep in range(2):
        for t in gvs:
            t.zero_()
        b.launch()
        bf.launch()
        torch.cuda.synchronize()
        for i, m in enumerate(meshes):
            s = slice(off[i], off[i + 1])
            d, t, c = dev.query(m, q[s].contiguous())
            gv_ref = torch.zeros_like(gvs[i])
            _, _, _, gq_ref = dev.query_fused(m, q[s].contiguous(), g[s].contiguous(), grad_vertices=gv_ref)
            torch.cuda.synchronize()
            assert torch.equal(dist[s], d) and torch.equal(tri[s], t) and torch.equal(cl[s], c), (rep, i)
            assert torch.equal(gq[s], gq_ref), (rep, i)
            err = torch.linalg.norm(gvs[i] - gv_ref) / max(torch.linalg.norm(gv_ref).item(), 1e-30)
            assert err <= 1e-5, (rep, i, err)


def test_batched_fused_against_oracle_gradient(dev, c4_small):
    """The batched fused form's dL/dq and every mesh's dL/dV against the
    FP64 envelope-theorem gradient of the oracle (at the GPU's triangles;
    their distances are checked against the oracle first), on the first
    5,000 points of each mesh."""
    cfg, meshes = c4_small
    sub = [dict(c, Q=c["Q"][:5000]) for c in cfg]
    Q, off = concat_points(sub)
    n = len(Q)
    rng = np.random.default_rng(32)
    gnp = rng.normal(size=n).astype(np.float32)
    q = torch.from_numpy(Q).cuda()
    g = torch.from_numpy(gnp).cuda()
    dist = torch.empty(n, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    cl = torch.empty((n, 3), device="cuda")
    gq = torch.empty((n, 3), device="cuda")
    gvs = [torch.zeros((len(m.V), 3), device="cuda") for m in meshes]
    b = dev.Batch(meshes, [len(c["Q"]) for c in sub], autotune=False)
    b.bind(q, dist, tri, cl, grad_dist=g, grad_points=gq, grad_vertices=gvs)
    b.launch()
    torch.cuda.synchronize()
    dn, tn, cn, gqn = to_np(dist), to_np(tri), to_np(cl), to_np(gq)
    for i, c in enumerate(sub):
        s = slice(off[i], off[i + 1])
        V, F = c["V"], c["F"]
        check_forward(V, F, Q[s], dn[s], tn[s], cn[s], c["D"], label=c["name"])
        dq64, dV64 = oracle.gradient(V, F, Q[s], tn[s], gnp[s])
        eq = np.linalg.norm(gqn[s] - dq64) / max(np.linalg.norm(dq64), 1e-30)
        ev = np.linalg.norm(to_np(gvs[i]) - dV64) / max(np.linalg.norm(dV64), 1e-30)
        assert eq <= 1e-3 and ev <= 1e-3, (c["name"], eq, ev)


def test_batched_plan_prefix_full_meshes(dev):
    """The first 11 meshes of the 64-mesh plan at their full triangle counts
    (up to 81,608) with 10% of their points: the batched forward equals one
    plain call per mesh bit for bit, and 200 points of every mesh match the
    oracle."""
    cfg = gen.config_c4(gen.c4_plan()[:11], query_scale=0.1)
    meshes = [dev.Mesh(c["V"], c["F"]) for c in cfg]
    Q, off = concat_points(cfg)
    n = len(Q)
    q = torch.from_numpy(Q).cuda()
    dist = torch.empty(n, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    cl = torch.empty((n, 3), device="cuda")
    b = dev.Batch(meshes, [len(c["Q"]) for c in cfg], autotune=True)
    b.bind(q, dist, tri, cl)
    b.launch()
    torch.cuda.synchronize()
    for i, m in enumerate(meshes):
        s = slice(off[i], off[i + 1])
        d, t, c = dev.query(m, q[s].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(dist[s], d) and torch.equal(tri[s], t) and torch.equal(cl[s], c), i
        k = min(200, off[i + 1] - off[i])
        idx = np.arange(off[i], off[i] + k)
        check_forward(cfg[i]["V"], cfg[i]["F"], Q[idx], to_np(dist)[idx], to_np(tri)[idx], to_np(cl)[idx],
                      cfg[i]["D"], label=cfg[i]["name"])


def test_batched_full_plan(dev):
    """The whole 64-mesh plan at its stated size (7.35M triangles, 16.9M
    points; built with the device preprocessing): the batched forward, in
    the configuration the autotuner picks, equals one plain call per mesh
    bit for bit, and 200 points of every mesh match the oracle."""
    import time
    t0 = time.time()
    cfg = gen.config_c4(gen.c4_plan())
    meshes = []
    for k, c in enumerate(cfg):
        meshes.append(dev.Mesh(c["V"], c["F"]))
        print(f"mesh {k + 1}/64 ({c['name']}, {len(c['F'])} triangles) built at {time.time() - t0:.1f}s", flush=True)
    print(f"64 meshes built in {time.time() - t0:.1f}s")
    Q, off = concat_points(cfg)
    n = len(Q)
    q = torch.from_numpy(Q).cuda()
    dist = torch.empty(n, device="cuda")
    tri = torch.empty(n, dtype=torch.int32, device="cuda")
    cl = torch.empty((n, 3), device="cuda")
    b = dev.Batch(meshes, [len(c["Q"]) for c in cfg], autotune=True)
    b.bind(q, dist, tri, cl)
    b.launch()
    torch.cuda.synchronize()
    print(f"launch configuration {b.config()}")
    dn, tn, cn = to_np(dist), to_np(tri), to_np(cl)
    for i, m in enumerate(meshes):
        s = slice(off[i], off[i + 1])
        d, t, c = dev.query(m, q[s].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(dist[s], d) and torch.equal(tri[s], t) and torch.equal(cl[s], c), i
        idx = np.arange(off[i], off[i] + min(200, off[i + 1] - off[i]))
        check_forward(cfg[i]["V"], cfg[i]["F"], Q[idx], dn[idx], tn[idx], cn[idx], cfg[i]["D"], label=cfg[i]["name"])

