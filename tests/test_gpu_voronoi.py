"""Voronoi corner checks on the GPU (gpu_voronoi = 1) give the host's cells:
the same sites (vertex and auxiliary, whose placement depends on the
first pass's cells), the same Delaunay neighbours and the same interception
lists, site by site, on meshes with every kind of degeneracy the builder
meets (co-spherical and co-circular sites, line clusters, budgeted checks
that give up), and at the 327,680-triangle size, where the time of the
Voronoi stage on each side is printed."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_00429_amd as p2m
    return p2m


def assert_same_structure(m0, m1, label, sites=None):
    s0, s1 = m0.stats(), m1.stats()
    for k in ("n_sites", "n_aux_sites", "n_dense_cells", "adj_nnz", "adj_max", "list_nnz", "list_max"):
        assert s0[k] == s1[k], (label, k, s0[k], s1[k])
    (x0, a0), (x1, a1) = m0.host_sites(), m1.host_sites()
    assert np.array_equal(x0, x1) and np.array_equal(a0, a1), label
    for s in (range(s0["n_sites"]) if sites is None else sites):
        assert np.array_equal(m0.host_neighbors(s), m1.host_neighbors(s)), (label, "neighbours", s)
        assert np.array_equal(m0.host_list(s), m1.host_list(s)), (label, "list", s)
    assert list(s0["seed_dims"]) == list(s1["seed_dims"]), label
    # the seed grids (walk starts, also computed on the device) agree: the
    # same walks take the same steps and give the same answers
    import paper_2605_00429_amd as p2m
    V = x0[~a0]
    lo, hi = V.min(0), V.max(0)
    rng = np.random.default_rng(54)
    Q = (lo + (hi - lo) * rng.uniform(-0.1, 1.1, size=(20000, 3))).astype(np.float32)
    q = torch.from_numpy(Q).cuda()
    r0, r1 = p2m.query_counters(m0, q), p2m.query_counters(m1, q)
    torch.cuda.synchronize()
    for a, b in zip(r0[:3], r1[:3]):
        assert torch.equal(a, b), label
    assert r0[3] == r1[3], (label, r0[3], r1[3])
    return s0, s1


CASES = {
    "uv sphere 32x16": lambda: gen.uv_sphere(32, 16),
    "icosphere-5": lambda: gen.icosphere(5),
    "cylinder+cone 128x32": lambda: gen.cylinder_cone(128, 32),
    "displaced icosphere-5": lambda: gen.displaced_icosphere(5, np.random.default_rng(51)),
    "torus": lambda: gen.torus(1.0, 0.3, 64, 20),
}


@pytest.mark.parametrize("name", list(CASES))
def test_device_checks_give_the_host_cells(dev, name):
    V, F = CASES[name]()
    m0 = dev.Mesh(V, F, gpu_voronoi=0)
    m1 = dev.Mesh(V, F, gpu_voronoi=1)
    assert_same_structure(m0, m1, name)


def test_device_checks_without_augmentation_and_degenerate(dev):
    V, F = gen.icosphere(4)
    m0, m1 = dev.Mesh(V, F, gpu_voronoi=0, augment=0), dev.Mesh(V, F, gpu_voronoi=1, augment=0)
    assert_same_structure(m0, m1, "icosphere-4 augment=0")
    # a far-away vertex and a triangle with a repeated vertex
    V, F = gen.uv_sphere(12, 6)
    V2 = np.concatenate([V, [[5, 5, 5]], V[:3]], 0).astype(np.float32)
    F2 = np.concatenate([F, [[0, len(V) + 1, len(V) + 2]], [[1, 1, 2]]], 0).astype(np.int32)
    m0, m1 = dev.Mesh(V2, F2, gpu_voronoi=0), dev.Mesh(V2, F2, gpu_voronoi=1)
    assert_same_structure(m0, m1, "degenerate")


def test_device_checks_full_size(dev):
    """The displaced icosphere-7 (327,680 triangles): identical statistics
    and site positions, 3,000 sampled sites' neighbours and lists."""
    from gen.configs import c2_mesh
    V, F, _ = c2_mesh()
    m0, m1 = dev.Mesh(V, F, gpu_voronoi=0), dev.Mesh(V, F, gpu_voronoi=1)
    rng = np.random.default_rng(53)
    n = m0.stats()["n_sites"]
    s0, s1 = assert_same_structure(m0, m1, "C2", sites=rng.choice(n, 3000, replace=False))
    print(f"Voronoi stage: host checks {s0['t_voronoi_s']:.2f}s, device checks {s1['t_voronoi_s']:.2f}s; "
          f"whole build {s0['t_total_s']:.2f}s / {s1['t_total_s']:.2f}s")
