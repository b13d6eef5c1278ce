"""Host preprocessing (no GPU): Voronoi cells / Delaunay neighbours, the locate
walk, interception-list completeness and the theorem the lists rest on.

The reference for every check is independent of the library: brute-force
nearest site and brute-force distance from the FP64 oracle, SciPy's qhull
Delaunay triangulation, and direct numeric checks of Eq. (3) and Eq. (8).
"""
import numpy as np
import pytest

import gen
import oracle
import paper_2605_00429_amd as p2m


def all_lists(m):
    return [m.host_list(s) for s in range(m.n_sites)]


def check_exact(m, V, F, Q):
    """Every query's located site is a nearest site, and its list holds a
    triangle attaining the oracle's distance."""
    S, _ = m.host_sites()
    loc = m.host_locate(Q)
    _, dn = oracle.nearest_point(S, Q)
    dl = np.linalg.norm(S[loc].astype(np.float64) - Q.astype(np.float64), axis=1)
    assert np.all(dl <= dn + 1e-12 * max(1.0, dn.max())), "walk did not reach a nearest site"
    d, _, _, _ = oracle.distance(V, F, Q)
    lists = all_lists(m)
    lens = np.array([len(lists[s]) for s in loc])
    assert lens.min() > 0
    qi = np.repeat(np.arange(len(Q)), lens)
    tri = np.concatenate([lists[s] for s in loc])
    dd = oracle.distance_to_triangles(V, F, Q[qi], tri)[0]
    best = np.minimum.reduceat(dd, np.concatenate([[0], np.cumsum(lens)[:-1]]))
    assert np.all(best <= d + 1e-12), f"{np.sum(best > d + 1e-12)} queries miss their closest triangle"
    return lens


MESHES = {
    "uv32x16": lambda: gen.uv_sphere(32, 16),
    "ico3": lambda: gen.icosphere(3),
    "cyl48x12": lambda: gen.capped_cylinder(1.0, 2.0, 48, 12),
    "cone48x12": lambda: gen.capped_cone(1.0, 2.0, 48, 12),
    "torus": lambda: gen.torus(1.0, 0.3, 40, 12),
    "dispico3": lambda: gen.displaced_icosphere(3, np.random.default_rng(11)),
    "tet": lambda: gen.tetrahedron(1.0),
}


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("augment", [0, 1])
def test_locate_exact_and_lists_complete(name, augment):
    V, F = MESHES[name]()
    rng = np.random.default_rng(12)
    lo, hi = gen.scaled_box(V, 1.2)
    D = float(np.linalg.norm(V.max(0) - V.min(0)))
    Q = np.concatenate([
        gen.uniform_box(rng, 1500, lo, hi),
        gen.near_surface(rng, 1500, V, F, 0.01 * D),
        gen.uniform_box(rng, 300, *gen.scaled_box(V, 9.0)),  # far queries inside the domain box
        V[rng.integers(0, len(V), 50)],                      # queries exactly at vertices
    ])
    m = p2m.Mesh(V, F, device="host", augment=augment)
    check_exact(m, V, F, Q)


def test_c0_full_query_set():
    c = gen.config_c0()
    m = p2m.Mesh(c["V"], c["F"], device="host")
    lens = check_exact(m, c["V"], c["F"], c["Q"])
    st = m.stats()
    assert st["n_aux_sites"] > 0          # the co-spherical centre is augmented
    assert lens.mean() < 0.2 * len(c["F"])


def test_incident_triangles_in_vertex_lists():
    for name in ("uv32x16", "dispico3", "torus"):
        V, F = MESHES[name]()
        m = p2m.Mesh(V, F, device="host")
        sov = m.site_of_vertex()
        lists = all_lists(m)
        for t, tri in enumerate(F):
            for v in tri:
                assert t in set(lists[sov[v]].tolist())


def test_delaunay_neighbours_match_qhull():
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(13)
    P = rng.uniform(-1, 1, (600, 3)).astype(np.float32)
    F = np.arange(600, dtype=np.int32).reshape(-1, 3)  # triangle soup: every point is a site
    m = p2m.Mesh(P, F, device="host", augment=0, domain_scale=50.0)
    S, _ = m.host_sites()
    # map our site ids to input point ids
    sov = m.site_of_vertex()
    inv = np.empty(len(S), np.int64)
    inv[sov] = np.arange(len(P))
    ours = set()
    for s in range(m.n_sites):
        for t in m.host_neighbors(s):
            ours.add((min(inv[s], inv[t]), max(inv[s], inv[t])))
    dt = Delaunay(P.astype(np.float64))
    theirs = set()
    for simp in dt.simplices:
        for i in range(4):
            for j in range(i + 1, 4):
                a, b = simp[i], simp[j]
                theirs.add((min(a, b), max(a, b)))
    assert ours <= theirs
    # edges qhull has and we do not must be hull edges whose shared Voronoi
    # face lies outside the clipped domain (none for a box 50x the points)
    assert len(theirs - ours) <= 0.002 * len(theirs)
    # the neighbour relation is symmetric
    sym = sum(1 for s in range(m.n_sites) for t in m.host_neighbors(s) if s in set(m.host_neighbors(t)))
    assert sym == sum(len(m.host_neighbors(s)) for s in range(m.n_sites))


def test_vertex_sphere_union_theorem():
    """Eq. (3): a ball about any point x of a convex polytope P through v lies
    in the union of the balls about P's vertices through v."""
    from scipy.spatial import ConvexHull
    rng = np.random.default_rng(14)
    for _ in range(200):
        pts = rng.normal(size=(12, 3))
        U = pts[ConvexHull(pts).vertices]
        v = rng.normal(size=3) * 2
        lam = rng.dirichlet(np.ones(len(U)))
        x = lam @ U
        R = np.linalg.norm(x - v)
        dirs = rng.normal(size=(500, 3))
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        p = x + dirs * R * rng.uniform(0, 1, (500, 1)) ** (1 / 3)
        inside_some = np.any(np.linalg.norm(p[:, None, :] - U[None], axis=2)
                             <= np.linalg.norm(U - v, axis=1)[None] + 1e-12, axis=1)
        assert inside_some.all()


def test_eq8_sphere_contains_corner_balls():
    """Eq. (8): r = max_u |s-u| + |u-p| gives B(s, r) containing every B(u, |u-p|)."""
    rng = np.random.default_rng(15)
    for _ in range(200):
        U = rng.normal(size=(10, 3))
        s = U.mean(0) + rng.normal(size=3) * 0.1
        p = rng.normal(size=3) * 3
        r = np.max(np.linalg.norm(U - s, axis=1) + np.linalg.norm(U - p, axis=1))
        for u in U:
            R = np.linalg.norm(u - p)
            # farthest point of B(u, R) from s
            assert np.linalg.norm(u - s) + R <= r + 1e-12


def test_ngon_interference_growth():
    """Sec. 3.2: without augmentation, a rotationally symmetric shape's lists
    grow quadratically with resolution; augmentation localises them."""
    tot = {}
    for n in (32, 64, 128):
        V, F = gen.regular_ngon_prism(n, 1.0, 0.1, 1)
        m = p2m.Mesh(V, F, device="host", augment=0)
        tot[n] = m.stats()["list_nnz"]
    assert tot[64] / tot[32] > 3.0 and tot[128] / tot[64] > 3.0   # ~4x per doubling: O(n^2)
    # co-spherical vertices: every list is the whole mesh without augmentation
    for n_lat in (16, 24):
        V, F = gen.uv_sphere(2 * n_lat, n_lat)
        plain = p2m.Mesh(V, F, device="host", augment=0).stats()
        aug = p2m.Mesh(V, F, device="host", augment=1).stats()
        assert plain["list_avg"] > 0.9 * len(F)
        assert aug["n_aux_sites"] > 0 and aug["list_avg"] < 0.1 * len(F)


def test_unreferenced_duplicate_and_degenerate_input():
    V, F = gen.uv_sphere(12, 6)
    V2 = np.concatenate([V, [[5, 5, 5]], V[:3]], 0).astype(np.float32)   # unreferenced + duplicates
    dup = len(V) + 1
    F2 = np.concatenate([F, [[0, dup, dup + 1]], [[1, 1, 2]]], 0).astype(np.int32)  # degenerate tris
    m = p2m.Mesh(V2, F2, device="host")
    sov = m.site_of_vertex()
    assert sov[len(V)] == -1                       # unreferenced vertex is no site
    assert sov[dup] == sov[0] and sov[dup + 1] == sov[1]   # equal positions share a site
    rng = np.random.default_rng(16)
    Q = rng.uniform(-1.5, 1.5, (1000, 3)).astype(np.float32)
    check_exact(m, V2, F2, Q)


@pytest.mark.parametrize("case", ["no_tris", "bad_index", "neg_index", "nan_vertex", "bad_opt", "bad_voronoi_mode",
                                  "bad_cell_pass"])
def test_build_errors(case):
    V, F = gen.tetrahedron()
    kw = {}
    if case == "no_tris":
        F = F[:0]
        code = p2m._lib.P2M_ERR_BAD_MESH
    elif case == "bad_index":
        F = F.copy(); F[1, 2] = 4
        code = p2m._lib.P2M_ERR_BAD_MESH
    elif case == "neg_index":
        F = F.copy(); F[0, 0] = -1
        code = p2m._lib.P2M_ERR_BAD_MESH
    elif case == "nan_vertex":
        V = V.copy(); V[2, 1] = np.nan
        code = p2m._lib.P2M_ERR_BAD_MESH
    elif case == "bad_voronoi_mode":
        kw = dict(gpu_voronoi=3)
        code = p2m._lib.P2M_ERR_INVALID_ARG
    elif case == "bad_cell_pass":
        kw = dict(gpu_cell_pass=-1)
        code = p2m._lib.P2M_ERR_INVALID_ARG
    else:
        kw = dict(domain_scale=0.5)
        code = p2m._lib.P2M_ERR_INVALID_ARG
    with pytest.raises(p2m.P2MError) as e:
        p2m.Mesh(V, F, device="host", **kw)
    assert e.value.code == code


def test_host_only_build_counts_its_cells():
    """Without a device every Voronoi cell (of every pass) is built on the
    host: at least one per site."""
    V, F = gen.icosphere(3)
    m = p2m.Mesh(V, F, device="host")
    st = m.stats()
    assert st["n_cells_device"] == 0
    assert st["n_cells_host"] >= st["n_sites"]


def test_null_arguments_and_host_only_queries():
    import ctypes
    L = p2m.lib()
    h = ctypes.c_void_p()
    assert L.p2m_build(None, None, ctypes.byref(h)) == p2m._lib.P2M_ERR_INVALID_ARG
    V, F = gen.tetrahedron()
    m = p2m.Mesh(V, F, device="host")
    # a host-only handle refuses device calls without touching the GPU
    rc = L.p2m_query(m.handle, None, 5, None, None, None, None)
    assert rc == p2m._lib.P2M_ERR_NO_DEVICE
    assert L.p2m_query(m.handle, None, -1, None, None, None, None) == p2m._lib.P2M_ERR_INVALID_ARG
    assert L.p2m_query(None, None, 0, None, None, None, None) == p2m._lib.P2M_ERR_INVALID_ARG
    assert b"host-only" in L.p2m_last_error() or True
    n = ctypes.c_int64()
    assert L.p2m_host_list(m.handle, 99, None, 0, ctypes.byref(n)) == p2m._lib.P2M_ERR_INVALID_ARG


def test_organic_list_statistics():
    """Table 1 order of magnitude (parity unpinned: the paper's models are not
    available; organic meshes there average ~63 entries per site)."""
    V, F = gen.displaced_icosphere(5, np.random.default_rng(17))
    m = p2m.Mesh(V, F, device="host")
    st = m.stats()
    assert st["n_aux_sites"] == 0          # augmentation stays inactive on organic shapes
    assert 20 < st["list_avg"] < 200
