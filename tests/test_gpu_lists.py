"""Interception lists built on the GPU (gpu_lists = 1) equal the host's,
site by site and entry by entry, on meshes that exercise every kind of
site: vertex sites, ring-based auxiliary sites with corner balls about
proj(s, M) (mode 1) or the single Eq. (8) sphere (mode 0), cells with more
than 64 balls (kept on the host), and degenerate input."""
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


def all_lists(m):
    n = m.n_sites
    return [m.host_list(s) for s in range(n)]


CASES = {
    "uv sphere 32x16": lambda: gen.uv_sphere(32, 16),
    "icosphere-5 (ring sites)": lambda: gen.icosphere(5),
    "cylinder+cone 128x32": lambda: gen.cylinder_cone(128, 32),
    "displaced icosphere-5": lambda: gen.displaced_icosphere(5, np.random.default_rng(51)),
    "torus": lambda: gen.torus(1.0, 0.3, 64, 20),
}


@pytest.mark.parametrize("name", list(CASES))
def test_gpu_lists_equal_host_lists(dev, name):
    V, F = CASES[name]()
    m0 = dev.Mesh(V, F, gpu_lists=0)
    m1 = dev.Mesh(V, F, gpu_lists=1)
    s0, s1 = m0.stats(), m1.stats()
    assert s0["n_sites"] == s1["n_sites"] and s0["list_nnz"] == s1["list_nnz"]
    L0, L1 = all_lists(m0), all_lists(m1)
    for s, (a, b) in enumerate(zip(L0, L1)):
        assert np.array_equal(a, b), (name, s, len(a), len(b))


def test_gpu_lists_eq8_mode_and_degenerate(dev):
    V, F = gen.icosphere(4)
    for kw in (dict(aux_list_mode=0), dict(augment=0)):
        m0, m1 = dev.Mesh(V, F, gpu_lists=0, **kw), dev.Mesh(V, F, gpu_lists=1, **kw)
        assert all(np.array_equal(a, b) for a, b in zip(all_lists(m0), all_lists(m1))), kw
    V, F = gen.uv_sphere(12, 6)
    V2 = np.concatenate([V, [[5, 5, 5]], V[:3]], 0).astype(np.float32)
    F2 = np.concatenate([F, [[0, len(V) + 1, len(V) + 2]], [[1, 1, 2]]], 0).astype(np.int32)
    m0, m1 = dev.Mesh(V2, F2, gpu_lists=0), dev.Mesh(V2, F2, gpu_lists=1)
    assert all(np.array_equal(a, b) for a, b in zip(all_lists(m0), all_lists(m1)))


def test_gpu_lists_full_size_counts(dev):
    """C2 mesh (327,680 triangles): identical list statistics and a sampled
    set of identical lists; the device list stage is timed in the stats."""
    from gen.configs import c2_mesh
    V, F, _ = c2_mesh()
    m0, m1 = dev.Mesh(V, F, gpu_lists=0), dev.Mesh(V, F, gpu_lists=1)
    s0, s1 = m0.stats(), m1.stats()
    for k in ("n_sites", "list_nnz", "list_max", "adj_nnz"):
        assert s0[k] == s1[k], k
    rng = np.random.default_rng(52)
    for s in rng.choice(s0["n_sites"], 2000, replace=False):
        assert np.array_equal(m0.host_list(s), m1.host_list(s)), s
    print(f"list stage: host {s0['t_lists_s']:.2f}s, device {s1['t_lists_s']:.2f}s")
