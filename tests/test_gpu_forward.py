"""GPU forward parity: the HIP query path (through the C ABI) against the FP64
brute-force oracle, on the workload meshes and on edge cases."""
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
    ref = run(dev, m, c["Q"])
    for bs in (64, 512, 1024):
        for reorder in (0, 1):
            for xcd in (1, 3, 8):
                m.set_query_config(block_size=bs, reorder=reorder, xcd_groups=xcd)
                out = run(dev, m, c["Q"])
                for a, b in zip(ref, out):
                    assert np.array_equal(a, b, equal_nan=True), (bs, reorder, xcd)
    m.set_query_config(block_size=256, reorder=1, xcd_groups=8)


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


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 4097, 100_003])
def test_ragged_sizes(dev, c0, n):
    c, m = c0
    rng = np.random.default_rng(100 + n)
    Q = rng.uniform(-1.5, 1.5, (n, 3)).astype(np.float32)
    d, t, cl = run(dev, m, Q)
    assert d.shape == (n,)
    if n:
        idx = rng.choice(n, min(n, 3000), replace=False)
        check_forward(c["V"], c["F"], Q[idx], d[idx], t[idx], cl[idx], c["D"], label=f"n={n}")


def test_special_points(dev, c0):
    c, m = c0
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
    assert np.all(np.isnan(d)) and np.all(t == -1) and np.all(np.isnan(cl))


def test_counters_match_plain_forward(dev, c0):
    c, m = c0
    q = torch.from_numpy(c["Q"]).cuda()
    d0, t0, c0_ = dev.query(m, q)
    d1, t1, c1, ctr = dev.query_counters(m, q)
    assert torch.equal(d0, d1) and torch.equal(t0, t1) and torch.equal(c0_, c1)
    assert ctr["walk_steps"] >= len(c["Q"]) and ctr["exact_tests"] >= len(c["Q"])
    assert ctr["list_read"] <= ctr["list_len"] and ctr["fallback"] == 0


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


def check_full_size(dev, c, m, n_sample, seed):
    """The whole workload through p2m_query (the benchmark's launch
    configuration); the oracle checks a seeded sample of outputs one by one,
    invariants check all of them."""
    q = torch.from_numpy(c["Q"]).cuda()
    d, t, cl = dev.query(m, q)
    d2, t2, cl2 = dev.query(m, q)
    torch.cuda.synchronize()
    assert torch.equal(d, d2) and torch.equal(t, t2) and torch.equal(cl, cl2)   # deterministic
    d, t, cl = to_np(d), to_np(t), to_np(cl)
    n = len(c["Q"])
    rng = np.random.default_rng(seed)
    h = n_sample // 2
    idx = np.concatenate([rng.choice(n // 2, h, replace=False), n // 2 + rng.choice(n - n // 2, h, replace=False)])
    res = check_forward(c["V"], c["F"], c["Q"][idx], d[idx], t[idx], cl[idx], c["D"], label=c["name"])
    tol = 1e-5 * c["D"]
    assert t.min() >= 0 and t.max() < len(c["F"])
    on = oracle.distance_to_triangles64(c["V"], c["F"], cl.astype(np.float64), t)
    assert on.max() <= tol                                  # closest point on its triangle
    dq = np.linalg.norm(c["Q"].astype(np.float64) - cl, axis=1)
    assert np.abs(dq - d).max() <= tol                      # |q - p| = d
    return res


def test_c1_full_size_sampled(dev):
    """C1 at its full size: 512 x 128 cylinder + cone (263,168 triangles),
    1M uniform + 1M near-surface points."""
    c = gen.config_c1()
    m = dev.Mesh(c["V"], c["F"])
    print("C1 full sample max|dd|/D, p99.9:", check_full_size(dev, c, m, 3000, 2025))


@pytest.fixture(scope="module")
def c2(dev):
    c = gen.config_c2()     # full size: 10M points
    return c, dev.Mesh(c["V"], c["F"])


def test_c2_full_size_sampled(dev, c2):
    """Full C2 workload (10M points) in the benchmark's launch configuration."""
    c, m = c2
    print("C2 sample max|dd|/D, p99.9:", check_full_size(dev, c, m, 3000, 2024))


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
        assert lib.p2m_query_backward(m.handle, p, n, p, None, None, p, None, None, None) == _lib.P2M_ERR_INVALID_ARG
    assert lib.p2m_query(m.handle, p, 5, None, None, None, None) == _lib.P2M_ERR_INVALID_ARG   # null distance
