"""The tier-B oracle (exact branch-and-bound over the oracle's own box tree)
pinned to the brute force: identical distance, lowest-index triangle and
closest point, bit for bit, on seeded points of every workload mesh.  The
brute force itself is pinned in test_oracle_pins.py."""
import numpy as np
import pytest

import gen
import oracle


def assert_same_as_bruteforce(V, F, Q, label):
    d0, t0, p0, _ = oracle.distance(V, F, Q)
    d1, t1, p1, _ = oracle.distance_exact(V, F, Q)
    bad = np.nonzero((d0 != d1) & ~(np.isnan(d0) & np.isnan(d1)))[0]
    assert len(bad) == 0, f"{label}: {len(bad)} distances differ, e.g. {bad[:5]}"
    assert np.array_equal(t0, t1), f"{label}: triangle ids differ at {np.nonzero(t0 != t1)[0][:5]}"
    assert np.array_equal(p0, p1, equal_nan=True), f"{label}: closest points differ"


def mixed(V, F, n, seed, sigma_rel=0.005, box=1.2):
    rng = np.random.default_rng(seed)
    lo, hi = gen.scaled_box(V, box)
    D = float(np.linalg.norm(V.max(0) - V.min(0)))
    return np.concatenate([gen.uniform_box(rng, n // 2, lo, hi),
                           gen.near_surface(rng, n - n // 2, V, F, sigma_rel * D)]).astype(np.float32)


def test_c0_full_and_extra():
    c = gen.config_c0()
    Q = np.concatenate([c["Q"], mixed(c["V"], c["F"], 10_000, 1)])
    assert_same_as_bruteforce(c["V"], c["F"], Q, "C0")


@pytest.mark.parametrize("name,mk", [
    ("icosphere-5", lambda: gen.icosphere(5)),
    ("cylinder+cone 128x32", lambda: gen.cylinder_cone(128, 32)),
    ("torus", lambda: gen.torus(1.0, 0.3, 120, 36)),
    ("displaced icosphere-5", lambda: gen.displaced_icosphere(5, np.random.default_rng(3))),
    ("capped cone", lambda: gen.capped_cone(1.0, 2.0, 96, 24)),
])
def test_smaller_meshes_of_the_workload_kinds(name, mk):
    V, F = mk()
    Q = mixed(V, F, 20_000, 2)
    # the paper's query region (box x10) too
    lo, hi = gen.scaled_box(V, 10.0)
    Q = np.concatenate([Q, gen.uniform_box(np.random.default_rng(3), 2000, lo, hi).astype(np.float32)])
    assert_same_as_bruteforce(V, F, Q, name)


def test_ties_duplicates_and_special_points():
    """Every triangle duplicated (exact ties everywhere: the lower index must
    win, as in the brute force), zero-area triangles, points on vertices,
    edges and faces, non-finite points."""
    V, F = gen.uv_sphere(24, 12)
    F2 = np.concatenate([F, F[::-1], [[0, 0, 1]], [[2, 3, 2]]], 0).astype(np.int32)
    rng = np.random.default_rng(4)
    Q = np.concatenate([
        V, (V[F[:, 0]] + V[F[:, 1]]) * 0.5, V[F].mean(axis=1),
        rng.uniform(-1.5, 1.5, (3000, 3)), np.zeros((1, 3)),
        [[np.nan, 0, 0], [0, np.inf, 0]]]).astype(np.float32)
    assert_same_as_bruteforce(V, F2, Q, "duplicated uv sphere")
    d, t, _, _ = oracle.distance_exact(V, F2, Q)
    assert np.nanmax(t) < len(F)          # duplicates (higher ids) never win a tie


def test_empty_mesh_and_empty_queries():
    V, F = gen.cube(1.0)
    d, t, p, _ = oracle.distance_exact(V, F[:0], np.zeros((3, 3), np.float32))
    assert np.all(np.isnan(d)) and np.all(t == -1)
    d, t, p, _ = oracle.distance_exact(V, F, np.zeros((0, 3), np.float32))
    assert len(d) == 0


@pytest.mark.slow
@pytest.mark.parametrize("cfg", ["C1", "C2"])
def test_full_size_config_meshes_20k(cfg):
    """The full-size C1 (263,168 triangles) and C2 (327,680) meshes with 20k
    seeded points each (10k uniform in the box x1.2, 10k near-surface)."""
    if cfg == "C1":
        c = gen.config_c1(10_000, 10_000)
    else:
        c = gen.config_c2(10_000, 10_000)
    assert_same_as_bruteforce(c["V"], c["F"], c["Q"], cfg)
