"""The octree decomposition (decomposition = 1): leaf boxes as the convex
cells, each with the corner-ball list of Eq. (3) about the mesh point
closest to its centre.  Host-side checks against the FP64 oracle: every
point inside the root box is located into the leaf box that contains it,
and that leaf's list holds a triangle attaining the oracle's distance."""
import numpy as np
import pytest

import gen
import oracle
import paper_2605_00429_amd as p2m

MESHES = {
    "uv32x16": lambda: gen.uv_sphere(32, 16),
    "ico3": lambda: gen.icosphere(3),
    "cyl48x12": lambda: gen.capped_cylinder(1.0, 2.0, 48, 12),
    "torus": lambda: gen.torus(1.0, 0.3, 40, 12),
    "dispico3": lambda: gen.displaced_icosphere(3, np.random.default_rng(11)),
    "cube": lambda: gen.cube(1.0),
}


@pytest.mark.parametrize("name", sorted(MESHES))
def test_octree_lists_complete(name):
    V, F = MESHES[name]()
    rng = np.random.default_rng(61)
    lo, hi = gen.scaled_box(V, 1.2)
    D = float(np.linalg.norm(V.max(0) - V.min(0)))
    Q = np.concatenate([
        gen.uniform_box(rng, 2000, lo, hi),
        gen.near_surface(rng, 2000, V, F, 0.01 * D),
        V[rng.integers(0, len(V), 50)],
    ]).astype(np.float32)
    m = p2m.Mesh(V, F, device="host", decomposition=1, octree_max_list=32)
    st = m.stats()
    assert st["n_vertex_sites"] == 0 and st["n_sites"] == st["n_aux_sites"] and st["adj_nnz"] == 0
    loc = m.host_locate(Q)
    assert loc.min() >= 0
    lists = [m.host_list(s) for s in range(m.n_sites)]
    lens = np.array([len(lists[s]) for s in loc])
    assert lens.min() > 0
    d, _, _, _ = oracle.distance(V, F, Q)
    qi = np.repeat(np.arange(len(Q)), lens)
    tri = np.concatenate([lists[s] for s in loc])
    dd = oracle.distance_to_triangles(V, F, Q[qi], tri)[0]
    best = np.minimum.reduceat(dd, np.concatenate([[0], np.cumsum(lens)[:-1]]))
    assert np.all(best <= d + 1e-12), f"{np.sum(best > d + 1e-12)} queries miss their closest triangle"


def test_octree_options_and_outside_points():
    V, F = gen.icosphere(2)
    with pytest.raises(p2m.P2MError):
        p2m.Mesh(V, F, device="host", decomposition=2)
    with pytest.raises(p2m.P2MError):
        p2m.Mesh(V, F, device="host", decomposition=1, octree_max_depth=17)
    m = p2m.Mesh(V, F, device="host", decomposition=1)
    far = np.array([[100.0, 0, 0], [np.nan, 0, 0]], np.float32)
    assert list(m.host_locate(far)) == [-1, -1]
