"""Mesh-to-mesh distance on the GPU (p2m_point_set_distance and the
Hausdorff / Chamfer helpers) against the FP64 oracle."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_00429_amd as p2m
    return p2m


def check_against_oracle(p2m, V, F, P, D):
    m = p2m.Mesh(V, F)
    r = p2m.point_set_distance(m, torch.from_numpy(P).cuda())
    o = oracle.point_set_distance(V, F, P)
    tol = 1e-5 * D
    assert r["count"] == o["count"]
    assert abs(r["max"] - o["max"]) <= tol
    # the point the GPU names attains the maximum (ties within tol may differ)
    d_at, _, _, _ = oracle.distance(V, F, P[r["argmax"]:r["argmax"] + 1], want_closest=False)
    assert abs(d_at[0] - o["max"]) <= tol
    assert abs(r["sum"] - o["sum"]) <= tol * o["count"]
    assert abs(r["sum_sq"] - o["sum_sq"]) <= 2 * tol * (o["max"] + tol) * o["count"]
    return r, o


def test_translated_cube_closed_form(dev):
    V, F = gen.cube(1.0)
    A = (V + np.array([0.5, 0.0, 0.0], np.float32)).astype(np.float32)
    r, _ = check_against_oracle(dev, V, F, A, 2 * np.sqrt(3))
    assert abs(r["max"] - 0.5) <= 1e-6 and abs(r["sum"] - 2.0) <= 1e-5 and r["count"] == 8


def test_surface_samples_and_vertices_against_oracle(dev):
    rng = np.random.default_rng(41)
    V, F = gen.displaced_icosphere(5, rng)
    D = float(np.linalg.norm(V.max(0) - V.min(0)))
    # samples of a second surface (a torus through the first), its vertices,
    # and points off both
    Vt, Ft = gen.torus(0.9, 0.3, 96, 32)
    P = np.concatenate([gen.near_surface(rng, 3000, Vt, Ft, 0.0), Vt[::7],
                        gen.uniform_box(rng, 1000, *gen.scaled_box(V, 3.0))]).astype(np.float32)
    check_against_oracle(dev, V, F, P, D)


def test_ragged_sizes_nan_and_empty(dev):
    V, F = gen.icosphere(3)
    m = dev.Mesh(V, F)
    rng = np.random.default_rng(42)
    for n in (1, 63, 255, 256, 257, 4097, 70001):
        P = rng.uniform(-2, 2, (n, 3)).astype(np.float32)
        check_against_oracle(dev, V, F, P, 2 * np.sqrt(3))
    P = np.array([[2.0, 0, 0], [np.nan, 0, 0], [0, 3.0, 0]], np.float32)
    r = dev.point_set_distance(m, torch.from_numpy(P).cuda())
    assert r["count"] == 2 and r["argmax"] == 2
    r = dev.point_set_distance(m, torch.zeros((0, 3), device="cuda"))
    assert r == {"max": -1.0, "argmax": -1, "sum": 0.0, "sum_sq": 0.0, "count": 0}


def test_hausdorff_and_chamfer_helpers(dev):
    """Two different tessellations of shapes offset from each other: the
    helpers equal the oracle's one-sided measures composed on the host."""
    Va, Fa = gen.icosphere(3)
    Vb, Fb = gen.uv_sphere(40, 20, radius=1.1, center=(0.05, 0.0, 0.0))
    ma, mb = dev.Mesh(Va, Fa), dev.Mesh(Vb, Fb)
    pa, pb = Va[np.unique(Fa)], Vb[np.unique(Fb)]
    oab = oracle.point_set_distance(Vb, Fb, pa)
    oba = oracle.point_set_distance(Va, Fa, pb)
    tol = 1e-5 * 2.2 * np.sqrt(3)
    assert abs(dev.hausdorff(ma, mb, symmetric=False) - oab["max"]) <= tol
    assert abs(dev.hausdorff(ma, mb) - max(oab["max"], oba["max"])) <= tol
    ch = oab["sum"] / oab["count"] + oba["sum"] / oba["count"]
    assert abs(dev.chamfer(ma, mb) - ch) <= 2 * tol


def test_mesh_distance_call_against_oracle(dev):
    """p2m_mesh_distance: both one-sided Hausdorff distances, the symmetric
    one, the Chamfer distances (means of d and d^2) and the count, on the
    default vertex sets and on caller point sets of different sizes, against
    the oracle's one-sided reductions composed here; a mesh against itself
    is 0."""
    Va, Fa = gen.displaced_icosphere(4, np.random.default_rng(43))
    Vb, Fb = gen.torus(0.9, 0.35, 80, 30)
    ma, mb = dev.Mesh(Va, Fa), dev.Mesh(Vb, Fb)
    tol = 1e-5 * 3.0
    rng = np.random.default_rng(44)
    sa = gen.near_surface(rng, 7001, Va, Fa, 0.0)
    sb = np.concatenate([gen.near_surface(rng, 3000, Vb, Fb, 0.0), [[np.nan, 0, 0]]]).astype(np.float32)
    for pa, pb in ((None, None), (sa, sb), (sa, None)):
        ua = Va[np.unique(Fa)] if pa is None else pa
        ub = Vb[np.unique(Fb)] if pb is None else pb
        oab = oracle.point_set_distance(Vb, Fb, ua)
        oba = oracle.point_set_distance(Va, Fa, ub)
        r = dev.mesh_distance(ma, mb, None if pa is None else torch.from_numpy(pa).cuda(),
                              None if pb is None else torch.from_numpy(pb).cuda())
        assert r["count"] == oab["count"] + oba["count"]
        assert abs(r["hausdorff_ab"] - oab["max"]) <= tol and abs(r["hausdorff_ba"] - oba["max"]) <= tol
        assert r["hausdorff"] == max(r["hausdorff_ab"], r["hausdorff_ba"])
        ch = oab["sum"] / oab["count"] + oba["sum"] / oba["count"]
        ch2 = oab["sum_sq"] / oab["count"] + oba["sum_sq"] / oba["count"]
        assert abs(r["chamfer"] - ch) <= 2 * tol
        assert abs(r["chamfer_sq"] - ch2) <= 4 * tol * (oab["max"] + oba["max"] + tol)
    r = dev.mesh_distance(ma, ma)
    assert r["hausdorff"] <= 1e-6 and r["chamfer"] <= 1e-6


def test_full_size_consistent_with_query(dev):
    """10M points on the 327,680-triangle mesh: the reduction equals the same
    reduction of p2m_query's distances."""
    c = gen.config_c2()
    m = dev.Mesh(c["V"], c["F"])
    q = torch.from_numpy(c["Q"]).cuda()
    r = dev.point_set_distance(m, q)
    d, _, _ = dev.query(m, q, want_tri=False, want_closest=False)
    d64 = d.double()
    assert r["count"] == len(q)
    assert r["max"] == d64.max().item()
    assert d[r["argmax"]].item() == d.max().item() and r["argmax"] == int(torch.nonzero(d == d.max())[0, 0])
    assert abs(r["sum"] - d64.sum().item()) <= 1e-9 * d64.sum().item()
    assert abs(r["sum_sq"] - (d64 * d64).sum().item()) <= 1e-9 * (d64 * d64).sum().item()
