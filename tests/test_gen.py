"""The seeded workload generators: sizes, closedness, orientation, determinism."""
import numpy as np
import pytest

import gen


def signed_volume(V, F):
    V = V.astype(np.float64)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    return np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0


def is_closed_oriented(F):
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]).astype(np.int64)
    key = e[:, 0] * (F.max() + 1) + e[:, 1]
    rkey = e[:, 1] * (F.max() + 1) + e[:, 0]
    return len(np.unique(key)) == len(key) and np.all(np.isin(rkey, key))


@pytest.mark.parametrize("mk,nv,nt", [
    (lambda: gen.uv_sphere(32, 16), 482, 960),
    (lambda: gen.cylinder_cone(512, 128), 131_588, 263_168),
    (lambda: gen.icosphere(7), 163_842, 327_680),
    (lambda: gen.torus(1.0, 0.3, 40, 12), 480, 960),
    (lambda: gen.cube(), 8, 12),
    (lambda: gen.tetrahedron(), 4, 4),
])
def test_mesh_sizes_closed_outward(mk, nv, nt):
    V, F = mk()
    assert V.shape == (nv, 3) and F.shape == (nt, 3)
    assert V.dtype == np.float32 and F.dtype == np.int32
    assert is_closed_oriented(F)
    assert signed_volume(V, F) > 0


def test_c2_displacement_range_and_determinism():
    V1, F1, _ = gen.configs.c2_mesh()
    V2, F2, _ = gen.configs.c2_mesh()
    assert np.array_equal(V1, V2) and np.array_equal(F1, F2)
    r = np.linalg.norm(V1.astype(np.float64), axis=1)
    assert r.min() >= 0.592 - 1e-6 and r.max() <= 1.408 + 1e-6


def test_config_prefix_and_query_regions():
    c = gen.config_c2(1000, 1000)
    assert c["Q"].shape == (2000, 3) and c["Q"].dtype == np.float32
    lo, hi = gen.scaled_box(c["V"], 1.2)
    assert np.all(c["Q"][:1000] >= lo - 1e-6) and np.all(c["Q"][:1000] <= hi + 1e-6)
    c0 = gen.config_c0()
    assert c0["Q"].shape == (10_000, 3) and np.abs(c0["Q"]).max() <= 1.5


def test_c4_plan_ranges():
    plan = gen.c4_plan()
    assert len(plan) == 64
    for kind, t, q in plan:
        assert 1e3 <= t <= 5e5 and 1e4 <= q <= 2e6
        assert kind in gen.configs.C4_KINDS
