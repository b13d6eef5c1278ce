"""The five synthetic workloads, each from its own seed ``SEED_BASE + c``.

* C0: closed UV sphere (r=1, 32 longitudes x 16 latitude bands, 960
  triangles), 10,000 points uniform in [-1.5, 1.5]^3.
* C1: closed cylinder (r=1, h=2, 512 x 128) plus closed cone (r=1, h=2,
  512 x 128) offset by 3 along x; 1M points uniform in the box x1.2 and 1M
  near-surface points (sigma = 1% of the box diagonal).
* C2: icosphere split 7 times (327,680 triangles) displaced radially by a
  sum of 8 random sines; 5M points uniform in the box x1.2 and 5M
  near-surface points (sigma = 0.5% of the diagonal).
* C3: the C2 mesh, 4M near-surface points (sigma = 0.5%), upstream gradient
  dL/dD ~ N(0, 1).
* C4: 64 meshes with log-uniform triangle counts in [1e3, 5e5], generators
  drawn from {UV sphere, capped cylinder, capped cone, torus R=1 r=0.3,
  displaced icosphere}, log-uniform query counts in [1e4, 2e6], half uniform
  in the box x1.2 and half near-surface (sigma = 0.5%).

Each config function takes the point counts as arguments so that tests can
draw a prefix-sized version of the same recipe.
"""
import math

import numpy as np

from . import meshes as M
from .queries import scaled_box, uniform_box, near_surface

SEED_BASE = 260500429


def _diag(V):
    V = np.asarray(V, dtype=np.float64)
    return float(np.linalg.norm(V.max(0) - V.min(0)))


def _mixed_queries(rng, V, F, n_uniform, n_near, sigma_rel):
    lo, hi = scaled_box(V, 1.2)
    qu = uniform_box(rng, n_uniform, lo, hi)
    qn = near_surface(rng, n_near, V, F, sigma_rel * _diag(V))
    return np.ascontiguousarray(np.concatenate([qu, qn], axis=0))


def config_c0(n_queries=10_000):
    rng = np.random.default_rng(SEED_BASE + 0)
    V, F = M.uv_sphere(32, 16)
    Q = uniform_box(rng, n_queries, (-1.5, -1.5, -1.5), (1.5, 1.5, 1.5))
    return dict(name="C0 uv-sphere 32x16", V=V, F=F, Q=Q, D=_diag(V))


def config_c1(n_uniform=1_000_000, n_near=1_000_000, n_seg=512, n_ring=128):
    rng = np.random.default_rng(SEED_BASE + 1)
    V, F = M.cylinder_cone(n_seg, n_ring)
    Q = _mixed_queries(rng, V, F, n_uniform, n_near, 0.01)
    return dict(name="C1 cylinder+cone 512x128", V=V, F=F, Q=Q, D=_diag(V))


def c2_mesh():
    rng = np.random.default_rng(SEED_BASE + 2)
    V, F = M.displaced_icosphere(7, rng)
    return V, F, rng


def config_c2(n_uniform=5_000_000, n_near=5_000_000):
    V, F, rng = c2_mesh()
    Q = _mixed_queries(rng, V, F, n_uniform, n_near, 0.005)
    return dict(name="C2 displaced icosphere-7", V=V, F=F, Q=Q, D=_diag(V))


def config_c3(n_queries=4_000_000):
    V, F, _ = c2_mesh()
    rng = np.random.default_rng(SEED_BASE + 3)
    Q = near_surface(rng, n_queries, V, F, 0.005 * _diag(V))
    G = rng.normal(0.0, 1.0, n_queries).astype(np.float32)
    return dict(name="C3 gradient on displaced icosphere-7", V=V, F=F, Q=Q, G=G, D=_diag(V))


C4_KINDS = ("uv_sphere", "cylinder", "cone", "torus", "icosphere")


def c4_plan(n_meshes=64, t_range=(1e3, 5e5), q_range=(1e4, 2e6)):
    """Per-mesh (kind, target triangle count, query count) for C4.

    Draw order per mesh from the C4 seed: log-uniform triangle count, kind
    index, log-uniform query count.
    """
    rng = np.random.default_rng(SEED_BASE + 4)
    plan = []
    for _ in range(n_meshes):
        t = math.exp(rng.uniform(math.log(t_range[0]), math.log(t_range[1])))
        kind = C4_KINDS[int(rng.integers(len(C4_KINDS)))]
        q = math.exp(rng.uniform(math.log(q_range[0]), math.log(q_range[1])))
        plan.append((kind, int(round(t)), int(round(q))))
    return plan


def c4_mesh(kind, t, mesh_index):
    """A mesh of the given kind with about ``t`` triangles."""
    if kind == "uv_sphere":
        n_lat = max(3, int(round((1.0 + math.sqrt(1.0 + t)) / 2.0)))
        return M.uv_sphere(2 * n_lat, n_lat)
    if kind == "cylinder":
        n_ring = max(1, int(round((-8.0 + math.sqrt(64.0 + 32.0 * t)) / 16.0)))
        return M.capped_cylinder(1.0, 2.0, 4 * n_ring, n_ring)
    if kind == "cone":
        n_ring = max(2, int(round(math.sqrt(t / 8.0))))
        return M.capped_cone(1.0, 2.0, 4 * n_ring, n_ring)
    if kind == "torus":
        n_minor = max(3, int(round(math.sqrt(t * 3.0 / 20.0))))
        n_major = max(3, int(round(n_minor * 10.0 / 3.0)))
        return M.torus(1.0, 0.3, n_major, n_minor)
    if kind == "icosphere":
        levels = np.arange(3, 8)
        counts = 20.0 * 4.0 ** levels
        level = int(levels[np.argmin(np.abs(np.log(counts) - math.log(t)))])
        rng = np.random.default_rng([SEED_BASE + 4, mesh_index])
        return M.displaced_icosphere(level, rng)
    raise ValueError(kind)


def config_c4(plan=None, query_scale=1.0):
    """Meshes and query sets of C4.  ``query_scale`` shrinks every query count
    (at least 2 points per mesh) for smaller test runs of the same recipe."""
    if plan is None:
        plan = c4_plan()
    out = []
    for i, (kind, t, q) in enumerate(plan):
        V, F = c4_mesh(kind, t, i)
        n = max(2, int(round(q * query_scale)))
        rng = np.random.default_rng([SEED_BASE + 4, 1000 + i])
        Q = _mixed_queries(rng, V, F, n // 2, n - n // 2, 0.005)
        out.append(dict(name=f"C4[{i}] {kind}", kind=kind, V=V, F=F, Q=Q, D=_diag(V)))
    return out
