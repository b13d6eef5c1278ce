"""The Voronoi stage on the GPU gives the host's cells.  Three modes build
the same structure: gpu_voronoi = 0 (all on the host), 2 (corner checks on
the device, clipping on the host) and 1 (whole cells on the device, one
wavefront per cell, cells that outgrow the device capacity on the host).
Compared: the sites (vertex and auxiliary, whose placement depends on the
first pass's cells), the Delaunay neighbours and the interception lists,
site by site, on meshes with every kind of degeneracy the builder meets
(co-spherical and co-circular sites, line clusters, budgeted checks that
give up, axis cells too large for the device), and at the 327,680-triangle
size, where the time of the Voronoi stage in each mode is printed."""
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
def test_device_cells_give_the_host_cells(dev, name):
    V, F = CASES[name]()
    m0 = dev.Mesh(V, F, gpu_voronoi=0)
    for mode in (1, 2):
        m = dev.Mesh(V, F, gpu_voronoi=mode)
        assert_same_structure(m0, m, f"{name} mode {mode}")
        st = m.stats()
        if mode == 1:
            assert st["n_cells_device"] > 0, name
        else:
            assert st["n_cells_device"] == 0, name
    print(name, {k: m0.stats()[k] for k in ("n_sites", "n_aux_sites")},
          "device mode 1 cells:", dev.Mesh(V, F, gpu_voronoi=1).stats()["n_cells_device"])


def test_device_cells_without_augmentation_and_degenerate(dev):
    V, F = gen.icosphere(4)
    m0 = dev.Mesh(V, F, gpu_voronoi=0, augment=0)
    for mode in (1, 2):
        assert_same_structure(m0, dev.Mesh(V, F, gpu_voronoi=mode, augment=0), f"icosphere-4 augment=0 mode {mode}")
    # a far-away vertex and a triangle with a repeated vertex
    V, F = gen.uv_sphere(12, 6)
    V2 = np.concatenate([V, [[5, 5, 5]], V[:3]], 0).astype(np.float32)
    F2 = np.concatenate([F, [[0, len(V) + 1, len(V) + 2]], [[1, 1, 2]]], 0).astype(np.int32)
    m0 = dev.Mesh(V2, F2, gpu_voronoi=0)
    for mode in (1, 2):
        assert_same_structure(m0, dev.Mesh(V2, F2, gpu_voronoi=mode), f"degenerate mode {mode}")


def test_device_cells_hand_large_cells_back(dev):
    """A capped cylinder: the cells of the vertices on its axis are cut by
    every vertex of the wall and outgrow the device's per-cell capacity;
    they are built on the host and the structure is still the host's."""
    V, F = gen.cylinder_cone(256, 16)
    m0, m1 = dev.Mesh(V, F, gpu_voronoi=0), dev.Mesh(V, F, gpu_voronoi=1)
    assert_same_structure(m0, m1, "cylinder 256x16")
    st = m1.stats()
    assert st["n_cells_host"] > 0 and st["n_cells_device"] > 0, st


def test_device_cells_in_small_passes(dev):
    """gpu_cell_pass splits the device cells into passes (here of 1,000 and
    of 777 cells, so that the last pass is ragged): the structure is still
    the host's, with and without cells handed back to the host."""
    for name, (V, F) in (("icosphere-5", gen.icosphere(5)), ("cylinder 256x16", gen.cylinder_cone(256, 16))):
        m0 = dev.Mesh(V, F, gpu_voronoi=0)
        for per in (1000, 777):
            m = dev.Mesh(V, F, gpu_voronoi=1, gpu_cell_pass=per)
            assert_same_structure(m0, m, f"{name} passes of {per}")
            assert m.stats()["n_cells_device"] > 0


def test_device_cells_full_size(dev):
    """The displaced icosphere-7 (327,680 triangles): identical statistics
    and site positions, 3,000 sampled sites' neighbours and lists, in each
    device mode; nearly every cell is built on the device."""
    from gen.configs import c2_mesh
    V, F, _ = c2_mesh()
    m0 = dev.Mesh(V, F, gpu_voronoi=0)
    rng = np.random.default_rng(53)
    n = m0.stats()["n_sites"]
    pick = rng.choice(n, 3000, replace=False)
    s0 = m0.stats()
    times = {0: (s0["t_voronoi_s"], s0["t_total_s"])}
    for mode in (2, 1):
        m = dev.Mesh(V, F, gpu_voronoi=mode)
        _, s = assert_same_structure(m0, m, f"C2 mode {mode}", sites=pick)
        times[mode] = (s["t_voronoi_s"], s["t_total_s"])
        if mode == 1:
            assert s["n_cells_device"] >= 0.99 * (s["n_cells_device"] + s["n_cells_host"]), s
        del m
    print("Voronoi stage / whole build (s): host " + "%.2f / %.2f" % times[0]
          + ", device checks " + "%.2f / %.2f" % times[2] + ", device cells " + "%.2f / %.2f" % times[1])
