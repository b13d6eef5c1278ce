"""GPU forward parity: the HIP query path (through the C ABI) against the FP64
brute-force oracle, on the workload meshes and on edge cases."""
import os

import numpy as np
import pytest

import gen
import oracle

from gpu_util import check_forward, exact_reference, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_00429_amd as p2m
    return p2m


def run(p2m, mesh, Q):
    q = torch.from_numpy(np.ascontiguousarray(Q, np.float32)).cuda()
    d, t, c = p2m.query(mesh, q)
    torch.cuda.synchronize()
    return to_np(d), to_np(t), to_np(c)


@pytest.fixture(scope="module")
def c0(dev):
    c = gen.config_c0()
    return c, dev.Mesh(c["V"], c["F"])


def test_c0_full(dev, c0):
    c, m = c0
    d, t, cl = run(dev, m, c["Q"])
    print("C0 max|dd|/D, p99.9:", check_forward(c["V"], c["F"], c["Q"], d, t, cl, c["D"], label="C0"))


def test_c0_launch_configs_bitwise(dev, c0):
    c, m = c0
    m.set_query_config(group=0)
    ref = run(dev, m, c["Q"])
    for group in (0, 1):
        for bs in (64, 512, 1024):
            for reorder in (0, 1):
                for xcd in (1, 3, 8):
                    for stage in (0, 1):
                        m.set_query_config(block_size=bs, reorder=reorder, xcd_groups=xcd, stage=stage, group=group)
                        out = run(dev, m, c["Q"])
                        for a, b in zip(ref, out):
                            assert np.array_equal(a, b, equal_nan=True), (group, bs, reorder, xcd, stage)
    m.set_query_config(block_size=256, reorder=1, xcd_groups=1, stage=0, group=2)


@pytest.mark.parametrize("n", [1, 4095, 4097, 300_001])
def test_sort_points_is_a_permutation(dev, c0, n):
    c, m = c0
    rng = np.random.default_rng(50 + n)
    Q = rng.uniform(-1.5, 1.5, (n, 3)).astype(np.float32)
    Q[: n // 10] *= 30.0                      # some points outside the domain box
    qt = torch.from_numpy(Q).cuda()
    order_t, sq = dev.sort_points(m, qt, want_sorted=True)
    order = to_np(order_t)
    assert np.array_equal(np.sort(order), np.arange(n))
    assert np.array_equal(to_np(sq), Q[order])
    # the two halves give exactly p2m_query's results
    ref = dev.query(m, qt)
    for a, b in zip(ref, dev.query_sorted(m, sq, order_t)):
        assert torch.equal(a, b)
    for a, b in zip(ref, dev.query_ordered(m, qt, order_t)):
        assert torch.equal(a, b)
    # spatially coherent: consecutive points are much closer than random pairs
    if n > 1000:
        inside = np.all(np.abs(Q[order]) <= 1.5, axis=1)
        qs = Q[order][inside].astype(np.float64)
        step = np.linalg.norm(np.diff(qs, axis=0), axis=1)
        assert np.median(step) < 0.1 * np.median(np.linalg.norm(qs - qs[::-1], axis=1))


@pytest.mark.parametrize("group", [0, 1])
@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 4097, 100_003])
def test_ragged_sizes(dev, c0, n, group):
    c, m = c0
    rng = np.random.default_rng(100 + n)
    Q = rng.uniform(-1.5, 1.5, (n, 3)).astype(np.float32)
    m.set_query_config(group=group)
    d, t, cl = run(dev, m, Q)
    m.set_query_config(group=2)
    assert d.shape == (n,)
    if n:
        idx = rng.choice(n, min(n, 3000), replace=False)
        check_forward(c["V"], c["F"], Q[idx], d[idx], t[idx], cl[idx], c["D"], label=f"n={n}")


@pytest.mark.parametrize("group", [0, 1])
def test_special_points(dev, c0, group):
    c, m = c0
    m.set_query_config(group=group)
    V, F = c["V"], c["F"]
    Q = np.concatenate([
        V[:40],                                             # exactly at vertices
        (V[F[:40, 0]] + V[F[:40, 1]]) * 0.5,                # on edges
        V[F[:40]].mean(axis=1),                             # on faces
        np.zeros((1, 3)),                                   # the co-spherical centre
        np.array([[30.0, 0, 0], [0, -40, 2], [1e3, 1e3, -1e3]]),  # outside the domain box: fallback
    ]).astype(np.float32)
    d, t, cl = run(dev, m, Q)
    check_forward(V, F, Q, d, t, cl, c["D"], label="special")
    assert np.all(d[:40] <= 1e-5 * c["D"])
    Qn = np.array([[np.nan, 0, 0], [0, np.inf, 0], [-np.inf, 1, 1]], np.float32)
    d, t, cl = run(dev, m, Qn)
    m.set_query_config(group=2)
    assert np.all(np.isnan(d)) and np.all(t == -1) and np.all(np.isnan(cl))


def test_counters_match_plain_forward(dev, c0):
    c, m = c0
    q = torch.from_numpy(c["Q"]).cuda()
    d0, t0, c0_ = dev.query(m, q)
    d1, t1, c1, ctr = dev.query_counters(m, q)
    assert torch.equal(d0, d1) and torch.equal(t0, t1) and torch.equal(c0_, c1)
    assert ctr["walk_steps"] >= len(c["Q"]) and ctr["exact_tests"] >= len(c["Q"])
    assert ctr["list_read"] <= ctr["list_len"] and ctr["fallback"] == 0 and ctr["walk_capped"] == 0


def test_small_and_degenerate_meshes(dev):
    rng = np.random.default_rng(7)
    cases = {
        "one_triangle": (np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32), np.array([[0, 1, 2]], np.int32)),
        "tetrahedron": gen.tetrahedron(1.0),
        "cube": gen.cube(0.5),
    }
    V, F = gen.uv_sphere(12, 6)
    V2 = np.concatenate([V, [[5, 5, 5]], V[:3]], 0).astype(np.float32)
    F2 = np.concatenate([F, [[0, len(V) + 1, len(V) + 2]], [[1, 1, 2]]], 0).astype(np.int32)
    cases["degenerate_soup"] = (V2, F2)
    for name, (V, F) in cases.items():
        m = dev.Mesh(V, F)
        D = float(np.linalg.norm(V[np.unique(F)].max(0) - V[np.unique(F)].min(0)))
        Q = rng.uniform(-2, 2, (5000, 3)).astype(np.float32)
        d, t, cl = run(dev, m, Q)
        check_forward(V, F, Q, d, t, cl, D, label=name)


@pytest.fixture(scope="module")
def c1(dev):
    # C1's recipe at 128 x 32 segments (16,640 triangles), every output
    # checked against the oracle
    c = gen.config_c1(20_000, 20_000, n_seg=128, n_ring=32)
    return c, dev.Mesh(c["V"], c["F"])


def test_c1_subset(dev, c1):
    c, m = c1
    d, t, cl = run(dev, m, c["Q"])
    print("C1 max|dd|/D, p99.9:", check_forward(c["V"], c["F"], c["Q"], d, t, cl, c["D"], label="C1"))
    # the grouped search forced on (C1 has few points per site): the same bits
    m.set_query_config(group=1)
    d1, t1, cl1 = run(dev, m, c["Q"])
    m.set_query_config(group=2)
    assert np.array_equal(d, d1) and np.array_equal(t, t1) and np.array_equal(cl, cl1)


def check_full_size(dev, c, m):
    """The whole workload through p2m_query (the benchmark's launch
    configuration), run twice (deterministic), and every output checked
    against the oracle's exact result under the acceptance rules."""
    q = torch.from_numpy(c["Q"]).cuda()
    d, t, cl = dev.query(m, q)
    d2, t2, cl2 = dev.query(m, q)
    torch.cuda.synchronize()
    assert torch.equal(d, d2) and torch.equal(t, t2) and torch.equal(cl, cl2)   # deterministic
    d, t, cl = to_np(d), to_np(t), to_np(cl)
    d64, _, _ = exact_reference(c["V"], c["F"], c["Q"], want_closest=False)
    return check_forward(c["V"], c["F"], c["Q"], d, t, cl, c["D"], d64=d64, label=c["name"])


def test_c1_full_size(dev):
    """C1 at its full size: 512 x 128 cylinder + cone (263,168 triangles),
    1M uniform + 1M near-surface points, every output against the oracle."""
    c = gen.config_c1()
    m = dev.Mesh(c["V"], c["F"])
    print("C1 full max|dd|/D, p99.9:", check_full_size(dev, c, m))


@pytest.fixture(scope="module")
def c2(dev):
    c = gen.config_c2()     # full size: 10M points
    return c, dev.Mesh(c["V"], c["F"])


def test_c2_full_size(dev, c2):
    """Full C2 workload (10M points) in the benchmark's launch configuration,
    every output against the oracle."""
    c, m = c2
    print("C2 full max|dd|/D, p99.9:", check_full_size(dev, c, m))


def test_c2_staging_is_exact(dev, c2):
    """Staging the list spheres in LDS changes where the scan reads them,
    not what it computes: 2M points of C2 give bit-identical outputs with
    and without it, plain and fused, at 256 and 1,024 threads per block."""
    c, m = c2
    q = torch.from_numpy(c["Q"][::5].copy()).cuda()
    g = torch.from_numpy(np.random.default_rng(81).normal(size=len(q)).astype(np.float32)).cuda()
    outs = {}
    for bs in (256, 1024):
        for stage in (0, 1):
            m.set_query_config(block_size=bs, stage=stage)
            outs[(bs, stage)] = dev.query(m, q) + dev.query_fused(m, q, g)
    m.set_query_config(block_size=256, stage=0)
    torch.cuda.synchronize()
    ref = outs[(256, 0)]
    for key, o in outs.items():
        for a, b in zip(ref, o):
            assert torch.equal(a, b), key


def test_c2_grouped_equals_one_pass(dev, c2):
    """The grouped search (locate, sort by site, list chunks shared through
    LDS) against the one-pass kernel on 2M points of C2, plain and fused
    with dL/dV, both through the library's own sort and in a given order:
    the same bits (dL/dV up to the order of float32 additions)."""
    c, m = c2
    q = torch.from_numpy(c["Q"][::5].copy()).cuda()
    n = len(q)
    g = torch.from_numpy(np.random.default_rng(82).normal(size=n).astype(np.float32)).cuda()
    nv = len(c["V"])
    outs = {}
    for group in (0, 1):
        m.set_query_config(group=group)
        gv = torch.zeros((nv, 3), device="cuda")
        outs[group] = dev.query(m, q) + dev.query_fused(m, q, g, grad_vertices=gv) + (gv,)
    m.set_query_config(group=2)
    torch.cuda.synchronize()
    for a, b in zip(outs[0][:-1], outs[1][:-1]):
        assert torch.equal(a, b)
    gv0, gv1 = outs[0][-1], outs[1][-1]
    assert (torch.linalg.norm(gv0 - gv1) / torch.linalg.norm(gv0)).item() <= 1e-5


def test_c2_no_walk_reaches_the_step_cap(dev, c2):
    """The instrumented forward on 1M points of C2: no walk stops at the step
    cap, nothing falls back, and the outputs equal the plain forward's."""
    c, m = c2
    q = torch.from_numpy(c["Q"][::10].copy()).cuda()
    d0, t0, c0_ = dev.query(m, q)
    d1, t1, c1_, ctr = dev.query_counters(m, q)
    assert torch.equal(d0, d1) and torch.equal(t0, t1) and torch.equal(c0_, c1_)
    assert ctr["walk_capped"] == 0 and ctr["fallback"] == 0


def test_c2_touched_items(dev, c2):
    """p2m_query_touched: same outputs as the plain forward; the distinct
    items it reports are within the arrays' sizes and at least what the
    counters imply (every located site, one seed cell per point cell)."""
    c, m = c2
    q = torch.from_numpy(c["Q"][:500_000].copy()).cuda()
    d0, t0, c0_ = dev.query(m, q)
    d1, t1, c1_, ctr, items = dev.query_touched(m, q)
    assert torch.equal(d0, d1) and torch.equal(t0, t1) and torch.equal(c0_, c1_)
    st = m.stats()
    assert 0 < items["site_rec"][0] <= st["n_sites"]
    assert 0 < items["adjacency"][0] <= st["adj_nnz"]
    assert 0 < items["list_sphere"][0] <= st["list_nnz"]
    assert 0 < items["list_record"][0] <= items["list_sphere"][0]
    assert items["list_sphere"][0] <= ctr["list_read"] + 3 * ctr["walk_steps"]     # at most what was read
    assert items["fallback_triangle"][0] == 0 and items["fallback_bvh_node"][0] == 0


@pytest.mark.parametrize("name", ["C0", "icosphere-5"])
def test_without_augmentation(dev, name):
    """augment = 0 (vertex sites only, the ablation of the paper's Tab. 4):
    on the UV sphere and the icosphere every vertex cell reaches the centre,
    so lists hold about every triangle and the wavefront completes long
    lists on nearly every query.  Every output against the oracle."""
    if name == "C0":
        c = gen.config_c0()
        V, F, Q, D = c["V"], c["F"], c["Q"], c["D"]
    else:
        V, F = gen.icosphere(5)
        D = float(np.linalg.norm(V.max(0) - V.min(0)))
        rng = np.random.default_rng(61)
        lo, hi = gen.scaled_box(V, 1.2)
        Q = np.concatenate([gen.uniform_box(rng, 20_000, lo, hi), gen.near_surface(rng, 20_000, V, F, 0.005 * D),
                            gen.uniform_box(rng, 5_000, *gen.scaled_box(V, 10.0))]).astype(np.float32)
    m = dev.Mesh(V, F, augment=0)
    st = m.stats()
    assert st["n_aux_sites"] == 0 and st["list_max"] > 0.5 * len(F)
    d, t, cl = run(dev, m, Q)
    d64, _, _ = exact_reference(V, F, Q, want_closest=False)
    print(name, "augment=0 max|dd|/D, p99.9:", check_forward(V, F, Q, d, t, cl, D, d64=d64, label=name))
    _, _, _, ctr = dev.query_counters(m, torch.from_numpy(Q).cuda())
    assert ctr["walk_capped"] == 0


def test_two_streams_one_handle(dev, c0):
    """The handle is read-only after build: queries of different point sets
    enqueued on two streams at once (each stream with its own scratch) give
    the results of the same queries run one after the other."""
    c, m = c0
    rng = np.random.default_rng(71)
    sets = [rng.uniform(-1.5, 1.5, (n, 3)).astype(np.float32) for n in (200_003, 150_001)]
    qs = [torch.from_numpy(Q).cuda() for Q in sets]
    ref = [dev.query(m, q) for q in qs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(3):
        outs = [None, None]
        for k in (0, 1):
            streams[k].wait_stream(torch.cuda.current_stream())
        for k in (0, 1):
            with torch.cuda.stream(streams[k]):
                outs[k] = dev.query(m, qs[k], stream=streams[k])
        # larger sets on the second round: the scratch regrows per stream
        torch.cuda.synchronize()
        for k in (0, 1):
            for a, b in zip(ref[k], outs[k]):
                assert torch.equal(a, b), (rep, k)
    Q = rng.uniform(-1.5, 1.5, (400_000, 3)).astype(np.float32)
    q = torch.from_numpy(Q).cuda()
    r0 = dev.query(m, q)
    torch.cuda.synchronize()
    with torch.cuda.stream(streams[1]):
        r1 = dev.query(m, q, stream=streams[1])
    torch.cuda.synchronize()
    for a, b in zip(r0, r1):
        assert torch.equal(a, b)


def test_rejects_bad_counts_before_any_launch(dev):
    """Point counts beyond 2^31 - 1 or negative are refused with
    P2M_ERR_INVALID_ARG before any device memory is touched (the pointers
    below are never read)."""
    import ctypes
    from paper_2605_00429_amd import _lib
    V, F = gen.icosphere(2)
    m = dev.Mesh(V, F)
    buf = torch.empty(16, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    lib = dev.lib()
    for n in (1 << 31, -1):
        assert lib.p2m_query(m.handle, p, n, p, None, None, None) == _lib.P2M_ERR_INVALID_ARG
        assert lib.p2m_point_set_distance(m.handle, p, n, p, None) == _lib.P2M_ERR_INVALID_ARG
        assert lib.p2m_sort_points(m.handle, p, n, p, None, None) == _lib.P2M_ERR_INVALID_ARG
        assert lib.p2m_query_backward(m.handle, p, n, p, p, None, None, None) == _lib.P2M_ERR_INVALID_ARG
        assert lib.p2m_mesh_distance(m.handle, m.handle, p, n, None, 0, p, None) == _lib.P2M_ERR_INVALID_ARG
    assert lib.p2m_query(m.handle, p, 5, None, None, None, None) == _lib.P2M_ERR_INVALID_ARG   # null distance
    assert lib.p2m_mesh_distance(m.handle, m.handle, None, 5, None, 0, p, None) == _lib.P2M_ERR_INVALID_ARG
