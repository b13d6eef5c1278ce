"""Closed triangle meshes used as synthetic workloads.

Every generator returns ``(V, F)`` with ``V`` an ``(nV, 3)`` float32 array and
``F`` an ``(nT, 3)`` int32 array of 0-based vertex indices, triangles wound so
that their normals point out of the enclosed volume.  Positions are computed in
float64 and rounded once to float32.
"""
import numpy as np


def _out(V, F):
    return np.ascontiguousarray(V, dtype=np.float32), np.ascontiguousarray(F, dtype=np.int32)


def _band(ring_a, ring_b, n):
    """Triangles joining two closed vertex rings of ``n`` vertices each.

    ``ring_a`` lies above ``ring_b`` (larger z); both run counter-clockwise
    seen from +z, which makes the quads face outward.
    """
    j = np.arange(n)
    jn = (j + 1) % n
    a0, a1 = ring_a[j], ring_a[jn]
    b0, b1 = ring_b[j], ring_b[jn]
    t1 = np.stack([a0, b0, b1], axis=1)
    t2 = np.stack([a0, b1, a1], axis=1)
    return np.concatenate([t1, t2], axis=0)


def _fan_top(center, ring, n):
    j = np.arange(n)
    return np.stack([np.full(n, center), ring[j], ring[(j + 1) % n]], axis=1)


def _fan_bottom(center, ring, n):
    j = np.arange(n)
    return np.stack([np.full(n, center), ring[(j + 1) % n], ring[j]], axis=1)


def uv_sphere(n_lon=32, n_lat=16, radius=1.0, center=(0.0, 0.0, 0.0)):
    """Closed UV sphere: two poles, ``n_lat - 1`` rings of ``n_lon`` vertices.

    Triangle count is ``2 * n_lon * (n_lat - 1)`` (960 for 32 x 16).
    """
    th = np.arange(1, n_lat) * np.pi / n_lat
    ph = np.arange(n_lon) * 2.0 * np.pi / n_lon
    st, ct = np.sin(th)[:, None], np.cos(th)[:, None]
    ring_xyz = np.stack([st * np.cos(ph)[None, :], st * np.sin(ph)[None, :],
                         np.broadcast_to(ct, (n_lat - 1, n_lon))], axis=2).reshape(-1, 3)
    V = np.concatenate([[[0.0, 0.0, 1.0]], ring_xyz, [[0.0, 0.0, -1.0]]], axis=0)
    V = V * radius + np.asarray(center, dtype=np.float64)
    rings = [1 + i * n_lon + np.arange(n_lon) for i in range(n_lat - 1)]
    south = 1 + (n_lat - 1) * n_lon
    F = [_fan_top(0, rings[0], n_lon)]
    for i in range(n_lat - 2):
        F.append(_band(rings[i], rings[i + 1], n_lon))
    F.append(_fan_bottom(south, rings[-1], n_lon))
    return _out(V, np.concatenate(F, axis=0))


def capped_cylinder(radius=1.0, height=2.0, n_seg=512, n_ring=128, center=(0.0, 0.0, 0.0)):
    """Closed cylinder along z: ``n_ring + 1`` vertex rings, caps fanned to a centre vertex."""
    z = np.linspace(height / 2, -height / 2, n_ring + 1)
    ph = np.arange(n_seg) * 2.0 * np.pi / n_seg
    ring_xyz = np.stack([np.broadcast_to(radius * np.cos(ph), (n_ring + 1, n_seg)),
                         np.broadcast_to(radius * np.sin(ph), (n_ring + 1, n_seg)),
                         np.broadcast_to(z[:, None], (n_ring + 1, n_seg))], axis=2).reshape(-1, 3)
    top_c = len(ring_xyz)
    bot_c = top_c + 1
    V = np.concatenate([ring_xyz, [[0.0, 0.0, height / 2], [0.0, 0.0, -height / 2]]], axis=0)
    V = V + np.asarray(center, dtype=np.float64)
    rings = [i * n_seg + np.arange(n_seg) for i in range(n_ring + 1)]
    F = [_fan_top(top_c, rings[0], n_seg)]
    for i in range(n_ring):
        F.append(_band(rings[i], rings[i + 1], n_seg))
    F.append(_fan_bottom(bot_c, rings[-1], n_seg))
    return _out(V, np.concatenate(F, axis=0))


def capped_cone(radius=1.0, height=2.0, n_seg=512, n_ring=128, center=(0.0, 0.0, 0.0)):
    """Closed cone along z: base ring at z=-h/2, apex at z=+h/2.

    ``n_ring`` vertex rings (radius falling linearly from ``radius``), the top
    band fanned to the apex and the base fanned to a centre vertex.
    """
    k = np.arange(n_ring)
    z = -height / 2 + height * k / n_ring
    rr = radius * (1.0 - k / n_ring)
    ph = np.arange(n_seg) * 2.0 * np.pi / n_seg
    # ring 0 is the base; order rings top-down for _band (upper ring first)
    ring_xyz = np.stack([rr[:, None] * np.cos(ph)[None, :], rr[:, None] * np.sin(ph)[None, :],
                         np.broadcast_to(z[:, None], (n_ring, n_seg))], axis=2).reshape(-1, 3)
    apex = len(ring_xyz)
    base_c = apex + 1
    V = np.concatenate([ring_xyz, [[0.0, 0.0, height / 2], [0.0, 0.0, -height / 2]]], axis=0)
    V = V + np.asarray(center, dtype=np.float64)
    rings = [i * n_seg + np.arange(n_seg) for i in range(n_ring)]
    F = [_fan_top(apex, rings[-1], n_seg)]
    for i in range(n_ring - 1, 0, -1):
        F.append(_band(rings[i], rings[i - 1], n_seg))
    F.append(_fan_bottom(base_c, rings[0], n_seg))
    return _out(V, np.concatenate(F, axis=0))


def cylinder_cone(n_seg=512, n_ring=128):
    """Union of a closed cylinder (r=1, h=2, at the origin) and a closed cone
    (r=1, h=2, base centre (3,0,-1), apex (3,0,1)), as two disjoint shells."""
    V1, F1 = capped_cylinder(1.0, 2.0, n_seg, n_ring)
    V2, F2 = capped_cone(1.0, 2.0, n_seg, n_ring, center=(3.0, 0.0, 0.0))
    return _out(np.concatenate([V1, V2], 0), np.concatenate([F1, F2 + len(V1)], 0))


_ICO_V = None


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    V = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    F = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return V / np.linalg.norm(V, axis=1, keepdims=True), F


def icosphere_f64(level):
    """Icosahedron split ``level`` times at edge midpoints, re-projected to the
    unit sphere after every split.  Returns float64 vertices and int64 faces:
    ``10 * 4**level + 2`` vertices and ``20 * 4**level`` triangles."""
    V, F = _icosahedron()
    for _ in range(level):
        e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
        e.sort(axis=1)
        uniq, inv = np.unique(e, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = (V[uniq[:, 0]] + V[uniq[:, 1]]) * 0.5
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = len(V)
        V = np.concatenate([V, mid], axis=0)
        nf = len(F)
        m01 = base + inv[:nf]
        m12 = base + inv[nf:2 * nf]
        m20 = base + inv[2 * nf:]
        a, b, c = F[:, 0], F[:, 1], F[:, 2]
        F = np.concatenate([np.stack([a, m01, m20], 1), np.stack([b, m12, m01], 1),
                            np.stack([c, m20, m12], 1), np.stack([m01, m12, m20], 1)], axis=0)
    return V, F


def icosphere(level, radius=1.0):
    V, F = icosphere_f64(level)
    return _out(V * radius, F)


def displaced_icosphere(level, rng, amplitude=0.15, n_waves=8, freq_std=4.0):
    """Icosphere with vertices moved radially by
    ``r(x) = 1 + amplitude * sum_k a_k sin(f_k . x + phi_k)``.

    Draw order from ``rng``: ``a`` (n_waves uniforms on [0.2, 1), divided by k),
    then ``f`` (n_waves x 3 normals, std ``freq_std``), then ``phi``
    (n_waves uniforms on [0, 2 pi)).
    """
    V, F = icosphere_f64(level)
    k = np.arange(1, n_waves + 1, dtype=np.float64)
    a = rng.uniform(0.2, 1.0, n_waves) / k
    f = rng.normal(0.0, freq_std, (n_waves, 3))
    phi = rng.uniform(0.0, 2.0 * np.pi, n_waves)
    r = 1.0 + amplitude * np.sin(V @ f.T + phi[None, :]) @ a
    return _out(V * r[:, None], F)


def torus(R=1.0, r=0.3, n_major=64, n_minor=20):
    """Closed torus around the z axis, ``2 * n_major * n_minor`` triangles."""
    u = np.arange(n_major) * 2.0 * np.pi / n_major
    v = np.arange(n_minor) * 2.0 * np.pi / n_minor
    cu, su = np.cos(u)[:, None], np.sin(u)[:, None]
    cv, sv = np.cos(v)[None, :], np.sin(v)[None, :]
    X = (R + r * cv) * cu
    Y = (R + r * cv) * su
    Z = np.broadcast_to(r * sv, X.shape)
    V = np.stack([X, Y, Z], axis=2).reshape(-1, 3)
    i = np.arange(n_major)[:, None]
    j = np.arange(n_minor)[None, :]
    a = i * n_minor + j
    b = ((i + 1) % n_major) * n_minor + j
    c = ((i + 1) % n_major) * n_minor + (j + 1) % n_minor
    d = i * n_minor + (j + 1) % n_minor
    F = np.concatenate([np.stack([a, b, c], 2).reshape(-1, 3),
                        np.stack([a, c, d], 2).reshape(-1, 3)], axis=0)
    return _out(V, F)


def cube(h=1.0):
    """Axis-aligned cube [-h, h]^3 as 12 outward triangles."""
    V = np.array([[x, y, z] for x in (-h, h) for y in (-h, h) for z in (-h, h)], dtype=np.float64)

    def idx(x, y, z):
        return (x > 0) * 4 + (y > 0) * 2 + (z > 0)
    quads = [
        [idx(1, -1, -1), idx(1, 1, -1), idx(1, 1, 1), idx(1, -1, 1)],      # +x
        [idx(-1, -1, -1), idx(-1, -1, 1), idx(-1, 1, 1), idx(-1, 1, -1)],  # -x
        [idx(-1, 1, -1), idx(-1, 1, 1), idx(1, 1, 1), idx(1, 1, -1)],      # +y
        [idx(-1, -1, -1), idx(1, -1, -1), idx(1, -1, 1), idx(-1, -1, 1)],  # -y
        [idx(-1, -1, 1), idx(1, -1, 1), idx(1, 1, 1), idx(-1, 1, 1)],      # +z
        [idx(-1, -1, -1), idx(-1, 1, -1), idx(1, 1, -1), idx(1, -1, -1)],  # -z
    ]
    F = []
    for q in quads:
        F.append([q[0], q[1], q[2]])
        F.append([q[0], q[2], q[3]])
    return _out(V, np.array(F))


def tetrahedron(a=1.0):
    """Regular tetrahedron of edge ``a`` centred at the origin."""
    s = a / (2.0 * 2.0 ** 0.5)
    V = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64) * s
    F = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]])
    return _out(V, F)


def regular_ngon_prism(n, radius=1.0, height=0.2, n_ring=1):
    """Thin closed prism over a regular n-gon (the 3D analogue of the
    n-gon example used to motivate site augmentation)."""
    return capped_cylinder(radius, height, n, n_ring)
