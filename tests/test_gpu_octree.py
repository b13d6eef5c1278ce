"""The octree decomposition on the GPU: the same search kernel with the
octree descent in place of the Delaunay walk, against the FP64 oracle."""
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


def run(p2m, m, Q):
    d, t, cl = p2m.query(m, torch.from_numpy(np.ascontiguousarray(Q, np.float32)).cuda())
    torch.cuda.synchronize()
    return to_np(d), to_np(t), to_np(cl)


def test_octree_c0_full(dev):
    c = gen.config_c0()
    m = dev.Mesh(c["V"], c["F"], decomposition=1, octree_max_list=32)
    d, t, cl = run(dev, m, c["Q"])
    check_forward(c["V"], c["F"], c["Q"], d, t, cl, c["D"], label="C0 octree")


@pytest.mark.parametrize("max_list,max_depth", [(32, 12), (128, 6), (64, 3)])
def test_octree_organic_mixed_and_outside(dev, max_list, max_depth):
    V, F = gen.displaced_icosphere(5, np.random.default_rng(71))
    D = float(np.linalg.norm(V.max(0) - V.min(0)))
    rng = np.random.default_rng(72)
    Q = np.concatenate([gen.uniform_box(rng, 20000, *gen.scaled_box(V, 1.2)),
                        gen.near_surface(rng, 20000, V, F, 0.005 * D),
                        gen.uniform_box(rng, 3000, *gen.scaled_box(V, 4.0)),   # partly outside the root box
                        V[rng.integers(0, len(V), 200)]]).astype(np.float32)
    m = dev.Mesh(V, F, decomposition=1, octree_max_list=max_list, octree_max_depth=max_depth)
    d, t, cl = run(dev, m, Q)
    check_forward(V, F, Q, d, t, cl, D, label="octree")
    _, _, _, ctr = dev.query_counters(m, torch.from_numpy(Q).cuda())
    assert ctr["fallback"] > 0          # the points outside the root box


def test_octree_fused_and_batched_equal_plain(dev):
    V, F = gen.displaced_icosphere(4, np.random.default_rng(73))
    rng = np.random.default_rng(74)
    Q = gen.near_surface(rng, 30000, V, F, 0.02).astype(np.float32)
    mo = dev.Mesh(V, F, decomposition=1, octree_max_list=48)
    mv = dev.Mesh(V, F)
    q = torch.from_numpy(Q).cuda()
    g = torch.from_numpy(rng.normal(size=len(Q)).astype(np.float32)).cuda()
    d, t, cl = dev.query(mo, q)
    gv = torch.zeros((len(V), 3), device="cuda")
    d2, t2, cl2, gq = dev.query_fused(mo, q, g, grad_vertices=gv)
    torch.cuda.synchronize()
    assert torch.equal(d, d2) and torch.equal(t, t2) and torch.equal(cl, cl2)
    # the two decompositions agree on the distance (both exact)
    dv, _, _ = dev.query(mv, q)
    assert torch.max(torch.abs(dv - d)).item() <= 1e-5 * 2.6
    # one batch mixing an octree mesh and a Voronoi mesh equals plain calls
    n = len(Q)
    qq = torch.cat([q, q])
    dist = torch.empty(2 * n, device="cuda")
    tri = torch.empty(2 * n, dtype=torch.int32, device="cuda")
    clo = torch.empty((2 * n, 3), device="cuda")
    b = dev.Batch([mo, mv], [n, n], autotune=False)
    b.bind(qq, dist, tri, clo)
    b.launch()
    torch.cuda.synchronize()
    assert torch.equal(dist[:n], d) and torch.equal(tri[:n], t)
    assert torch.equal(dist[n:], dv)
