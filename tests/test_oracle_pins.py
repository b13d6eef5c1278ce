"""Pins of the FP64 oracle against facts fixed by geometry, not by the oracle.

Each test compares the oracle with a closed form, an invariant, an
independent formulation or brute-force sampling, chosen so that a dropped
term, a wrong sign, a swapped index or a transposed operand in the oracle
fails at least one of them.
"""
import math

import numpy as np
import pytest

import gen
import oracle


# ---------------------------------------------------------------- helpers

def ericson_region_walk(q, a, b, c):
    """Closest point on triangle by Voronoi-region classification
    (Ericson, Real-Time Collision Detection, Sec. 5.1.5), written
    independently of the oracle's KKT enumeration."""
    ab, ac, ap = b - a, c - a, q - a
    d1, d2 = ab @ ap, ac @ ap
    if d1 <= 0 and d2 <= 0:
        return a
    bp = q - b
    d3, d4 = ab @ bp, ac @ bp
    if d3 >= 0 and d4 <= d3:
        return b
    vc = d1 * d4 - d3 * d2
    if vc <= 0 and d1 >= 0 and d3 <= 0:
        return a + ab * (d1 / (d1 - d3))
    cp = q - c
    d5, d6 = ab @ cp, ac @ cp
    if d6 >= 0 and d5 <= d6:
        return c
    vb = d5 * d2 - d1 * d6
    if vb <= 0 and d2 >= 0 and d6 <= 0:
        return a + ac * (d2 / (d2 - d6))
    va = d3 * d6 - d5 * d4
    if va <= 0 and (d4 - d3) >= 0 and (d5 - d6) >= 0:
        return b + (c - b) * ((d4 - d3) / ((d4 - d3) + (d5 - d6)))
    den = 1.0 / (va + vb + vc)
    return a + ab * (vb * den) + ac * (vc * den)


def random_rotation(rng):
    A = rng.normal(size=(3, 3))
    Qm, R = np.linalg.qr(A)
    Qm = Qm * np.sign(np.diag(R))
    if np.linalg.det(Qm) < 0:
        Qm[:, 0] = -Qm[:, 0]
    return Qm


def bary_of_point(p, a, b, c):
    """Barycentrics of p in the plane of (a, b, c) by least squares."""
    A = np.stack([b - a, c - a], axis=1)
    st, *_ = np.linalg.lstsq(A, p - a, rcond=None)
    return np.array([1.0 - st[0] - st[1], st[0], st[1]]), np.linalg.norm(A @ st + a - p)


# ---------------------------------------------------------- closed forms

def test_cube_outside_and_inside_closed_form():
    h = 0.75
    V, F = gen.cube(h)
    rng = np.random.default_rng(1)
    Q = rng.uniform(-3 * h, 3 * h, (3000, 3)).astype(np.float32)
    d, tri, p, _ = oracle.distance(V, F, Q)
    q = Q.astype(np.float64)
    outside = np.any(np.abs(q) > h, axis=1)
    exp_out = np.linalg.norm(np.maximum(np.abs(q) - h, 0.0), axis=1)
    exp_in = h - np.max(np.abs(q), axis=1)
    exp = np.where(outside, exp_out, exp_in)
    assert np.max(np.abs(d - exp)) < 1e-12
    # outside: the closest point is the clamp of q onto the box
    assert np.max(np.abs(p[outside] - np.clip(q[outside], -h, h))) < 1e-12
    # inside: projection onto the face of the largest |coordinate|
    k = np.argmax(np.abs(q), axis=1)
    p_in = q.copy()
    p_in[np.arange(len(q)), k] = np.sign(q[np.arange(len(q)), k]) * h
    ins = ~outside
    assert np.max(np.abs(p[ins] - p_in[ins])) < 1e-12
    assert ins.sum() > 50 and outside.sum() > 1000


def test_regular_tetrahedron_inradius_and_vertex_ray():
    a = 1.3
    V, F = gen.tetrahedron(a)
    Vd = V.astype(np.float64)
    d, tri, p, _ = oracle.distance(V, F, np.zeros((1, 3), np.float32))
    assert abs(d[0] - a * math.sqrt(6) / 12) < 1e-7  # float32 vertices
    R = np.linalg.norm(Vd, axis=1)
    assert np.allclose(R, a * math.sqrt(6) / 4, atol=1e-6)
    for i in range(4):
        u = Vd[i] / R[i]
        for t in (R[i] * 1.01, R[i] * 1.5, R[i] * 4.0):
            q = (u * t).astype(np.float32)[None]
            d, tri, p, _ = oracle.distance(V, F, q)
            assert abs(d[0] - (np.linalg.norm(q[0].astype(np.float64)) - R[i])) < 2e-7
            assert np.linalg.norm(p[0] - Vd[i]) < 1e-6


@pytest.mark.parametrize("mesh", ["cube", "tet", "uv", "ico", "cyl", "cone"])
def test_convex_mesh_interior_is_min_plane_distance(mesh):
    V, F = {"cube": lambda: gen.cube(1.0), "tet": lambda: gen.tetrahedron(2.0),
            "uv": lambda: gen.uv_sphere(12, 7), "ico": lambda: gen.icosphere(2),
            "cyl": lambda: gen.capped_cylinder(1.0, 2.0, 24, 3),
            "cone": lambda: gen.capped_cone(1.0, 2.0, 24, 3)}[mesh]()
    Vd = V.astype(np.float64)
    a, b, c = Vd[F[:, 0]], Vd[F[:, 1]], Vd[F[:, 2]]
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    off = np.einsum("ij,ij->i", n, a)
    rng = np.random.default_rng(2)
    Q = rng.uniform(Vd.min(0), Vd.max(0), (4000, 3))
    inside = np.all(Q @ n.T <= off[None, :] - 1e-9, axis=1)
    Q = Q[inside].astype(np.float32)
    assert len(Q) > 200
    d, tri, p, _ = oracle.distance(V, F, Q)
    plane = np.min(off[None, :] - Q.astype(np.float64) @ n.T, axis=1)
    # cube and tetrahedron vertices are exact in float32; the other meshes'
    # split quads are planar only up to float32 rounding of their vertices
    tol = 1e-12 if mesh in ("cube", "tet") else 5e-7
    assert np.max(np.abs(d - plane)) < tol


@pytest.mark.parametrize("mk", [lambda: gen.uv_sphere(32, 16), lambda: gen.icosphere(3)])
def test_inscribed_convex_mesh_vertex_ray(mk):
    V, F = mk()
    Vd = V.astype(np.float64)
    rng = np.random.default_rng(3)
    idx = rng.choice(len(V), 60, replace=False)
    t = rng.uniform(1.01, 3.0, 60)
    Q = (Vd[idx] * t[:, None]).astype(np.float32)
    d, tri, p, _ = oracle.distance(V, F, Q)
    q = Q.astype(np.float64)
    # q is (up to float32 rounding of q) on the ray through the vertex: d = |q| - |v|
    exp = np.linalg.norm(q, axis=1) - np.linalg.norm(Vd[idx], axis=1)
    assert np.max(np.abs(d - exp)) < 1e-6
    assert np.max(np.linalg.norm(p - Vd[idx], axis=1)) < 1e-5
    # tie rule: the returned triangle is the lowest-index triangle incident to the vertex
    for i, v in enumerate(idx):
        inc = np.nonzero(np.any(F == v, axis=1))[0]
        dd = oracle.distance_to_triangles(V, F, np.repeat(Q[i:i + 1], len(inc), 0), inc)[0]
        best = inc[np.argmin(dd)] if np.ptp(dd) > 1e-12 else inc.min()
        assert tri[i] in inc
        assert dd[list(inc).index(tri[i])] <= dd.min() + 1e-12
        if np.ptp(dd) <= 1e-12:
            assert tri[i] == best


def test_flat_uv_sphere_centre_closed_form():
    n_lon, n_lat = 32, 16
    V, F = gen.uv_sphere(n_lon, n_lat)
    d, tri, p, _ = oracle.distance(V, F, np.zeros((1, 3), np.float32))
    half = math.pi / n_lon
    th = np.arange(n_lat + 1) * math.pi / n_lat
    best = np.inf
    for i in range(n_lat):
        t1, t2 = th[i], th[i + 1]
        x1, z1 = math.sin(t1) * math.cos(half), math.cos(t1)
        x2, z2 = math.sin(t2) * math.cos(half), math.cos(t2)
        best = min(best, abs(x1 * z2 - z1 * x2) / math.hypot(x1 - x2, z1 - z2))
    assert abs(d[0] - best) < 1e-7  # float32 vertex rounding


# ------------------------------------------- independent formulation

def test_matches_region_walk_formulation():
    rng = np.random.default_rng(4)
    worst = 0.0
    for trial in range(3000):
        tri = rng.normal(size=(3, 3))
        if trial % 7 == 0:   # near-degenerate slivers
            tri[2] = tri[0] + (tri[1] - tri[0]) * rng.uniform(-0.5, 1.5) + rng.normal(size=3) * 1e-7
        q = rng.normal(size=3) * 2.0
        d, p, lam = oracle.point_triangle(q, *tri)
        pr = ericson_region_walk(q, *tri)
        worst = max(worst, abs(d - np.linalg.norm(q - pr)))
        assert np.linalg.norm(p - (lam[0] * tri[0] + lam[1] * tri[1] + lam[2] * tri[2])) < 1e-9
        assert lam.min() >= -1e-12 and abs(lam.sum() - 1.0) < 1e-12
    assert worst < 1e-12 * 10


def test_dense_barycentric_sampling_upper_bound():
    rng = np.random.default_rng(5)
    g = np.linspace(0.0, 1.0, 161)
    S, T = np.meshgrid(g, g)
    keep = S + T <= 1.0
    S, T = S[keep], T[keep]
    for _ in range(40):
        tri = rng.normal(size=(3, 3))
        q = rng.normal(size=3) * 1.5
        d, p, lam = oracle.point_triangle(q, *tri)
        pts = tri[0][None] + S[:, None] * (tri[1] - tri[0])[None] + T[:, None] * (tri[2] - tri[0])[None]
        ds = np.linalg.norm(pts - q[None], axis=1).min()
        h = np.max(np.linalg.norm(tri - np.roll(tri, 1, 0), axis=1)) / 160
        assert d <= ds + 1e-12
        assert ds - d <= h * 1.5


def test_degenerate_triangles():
    a = np.array([0.0, 0.0, 0.0])
    b = np.array([2.0, 0.0, 0.0])
    c = np.array([1.0, 0.0, 0.0])  # collinear: the triangle is the segment [a, b]
    q = np.array([1.5, 3.0, 4.0])
    d, p, lam = oracle.point_triangle(q, a, b, c)
    assert abs(d - 5.0) < 1e-14 and np.allclose(p, [1.5, 0, 0])
    q = np.array([-3.0, 4.0, 0.0])
    d, p, lam = oracle.point_triangle(q, a, b, c)
    assert abs(d - 5.0) < 1e-14 and np.allclose(p, a)
    d, p, lam = oracle.point_triangle(q, a, a, a)  # a point
    assert abs(d - 5.0) < 1e-14


# ------------------------------------------------------------ invariants

def test_invariants_on_mesh_queries():
    c = gen.config_c0(2000)
    V, F, Q = c["V"], c["F"], c["Q"]
    d, tri, p, _ = oracle.distance(V, F, Q)
    Vd, q = V.astype(np.float64), Q.astype(np.float64)
    # the closest point is on its triangle and at distance d
    for i in range(0, len(Q), 7):
        a, b, cc = Vd[F[tri[i]]]
        lam, res = bary_of_point(p[i], a, b, cc)
        assert res < 1e-12 and lam.min() > -1e-12
    assert np.max(np.abs(np.linalg.norm(q - p, axis=1) - d)) < 1e-12
    # no vertex is closer than the surface
    used = np.unique(F)
    vd = np.min(np.linalg.norm(q[:, None, :] - Vd[None, used, :], axis=2), axis=1)
    assert np.all(d <= vd + 1e-12)
    # distance is 1-Lipschitz
    j = np.random.default_rng(6).permutation(len(Q))
    assert np.all(np.abs(d - d[j]) <= np.linalg.norm(q - q[j], axis=1) + 1e-12)


def test_rigid_motion_invariance():
    rng = np.random.default_rng(7)
    V, F = gen.torus(1.0, 0.3, 24, 10)
    Q = rng.uniform(-1.5, 1.5, (500, 3)).astype(np.float32)
    d0, _, _, _ = oracle.distance(V, F, Q)
    R = random_rotation(rng)
    t = rng.normal(size=3)
    V2 = (V.astype(np.float64) @ R.T + t).astype(np.float32)
    Q2 = (Q.astype(np.float64) @ R.T + t).astype(np.float32)
    d1, _, _, _ = oracle.distance(V2, F, Q2)
    assert np.max(np.abs(d0 - d1)) < 2e-6  # float32 rounding of the moved inputs


def test_lowest_index_tie_rule_and_nan():
    V, F = gen.cube(1.0)
    Fd = np.concatenate([F, F], 0)  # every triangle duplicated: ties everywhere
    Q = np.random.default_rng(8).uniform(-2, 2, (300, 3)).astype(np.float32)
    d, tri, _, _ = oracle.distance(V, Fd, Q)
    assert tri.max() < len(F)
    Qn = np.array([[np.nan, 0, 0], [0, np.inf, 0]], np.float32)
    d, tri, _, _ = oracle.distance(V, F, Qn)
    assert np.all(np.isnan(d)) and np.all(tri == -1)


def test_nearest_point_brute_force_vs_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(9)
    P = rng.normal(size=(500, 3)).astype(np.float32)
    Q = rng.normal(size=(2000, 3)).astype(np.float32) * 2
    idx, dist = oracle.nearest_point(P, Q)
    dk, ik = cKDTree(P.astype(np.float64)).query(Q.astype(np.float64))
    assert np.max(np.abs(dist - dk)) < 1e-12
    assert np.mean(idx == ik) > 0.999


# --------------------------------------------------------------- gradient

def test_gradient_single_triangle_closed_form():
    V = np.array([[0, 0, 0], [2, 0, 0], [0, 2, 0]], np.float32)
    F = np.array([[0, 1, 2]], np.int32)
    Q = np.array([[0.5, 0.25, 1.5], [0.5, 0.5, -2.0]], np.float32)
    g = np.array([1.0, 2.0], np.float32)
    d, tri, p, _ = oracle.distance(V, F, Q)
    assert np.allclose(d, [1.5, 2.0])
    dq, dV = oracle.gradient(V, F, Q, tri, g)
    assert np.allclose(dq, [[0, 0, 1.0], [0, 0, -2.0]], atol=1e-14)
    lam0 = np.array([1 - 0.25 - 0.125, 0.25, 0.125])
    lam1 = np.array([0.5, 0.25, 0.25])
    exp = -1.0 * lam0[:, None] * np.array([0, 0, 1.0]) - 2.0 * lam1[:, None] * np.array([0, 0, -1.0])
    assert np.allclose(dV, exp, atol=1e-14)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(10)
    V, F = gen.uv_sphere(10, 6)
    Q = rng.uniform(-1.6, 1.6, (40, 3)).astype(np.float32)
    g = rng.normal(size=40).astype(np.float32)
    d, tri, p, _ = oracle.distance(V, F, Q)
    dq, dV = oracle.gradient(V, F, Q, tri, g)
    Vd = V.astype(np.float64)

    def dist64(Vx, Qx):
        a, b, c = Vx[F[:, 0]], Vx[F[:, 1]], Vx[F[:, 2]]
        out = np.empty(len(Qx))
        for i, q in enumerate(Qx):
            out[i] = min(oracle.point_triangle(q, a[f], b[f], c[f])[0] for f in range(len(F)))
        return out

    h = 1e-6
    q64 = Q.astype(np.float64)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (dist64(Vd, q64 + e) - dist64(Vd, q64 - e)) / (2 * h)
        assert np.max(np.abs(g * fd - dq[:, k])) < 1e-5
    # vertex gradient on a few vertices touched by the argmin triangles
    for v in np.unique(F[tri])[:6]:
        for k in range(3):
            Vp, Vm = Vd.copy(), Vd.copy()
            Vp[v, k] += h
            Vm[v, k] -= h
            fd = np.sum(g * (dist64(Vp, q64) - dist64(Vm, q64))) / (2 * h)
            assert abs(fd - dV[v, k]) < 1e-5 * max(1.0, abs(fd))


# ---------------------------------------------------------------------------
# Point-set reduction (mesh-to-mesh distance built on the point query)

def test_point_set_distance_translated_cube_closed_form():
    """Vertices of a cube translated by delta along x, against the cube: the
    four at x = h + delta lie delta from the face x = h, the four at
    x = -h + delta lie on the edges y, z = +-h of the cube (distance 0)."""
    V, F = gen.cube(1.0)
    for delta in (0.25, 0.5, 1.5):
        A = (V + np.array([delta, 0.0, 0.0], np.float32)).astype(np.float32)
        r = oracle.point_set_distance(V, F, A)
        far = np.nonzero(np.isclose(A[:, 0], 1.0 + delta))[0]
        assert r["count"] == 8
        assert abs(r["max"] - delta) <= 1e-12
        assert r["argmax"] == far.min()
        assert abs(r["sum"] - 4 * delta) <= 1e-12
        assert abs(r["sum_sq"] - 4 * delta * delta) <= 1e-12


def test_point_set_distance_self_is_zero_and_nan_left_out():
    V, F = gen.icosphere(2)
    r = oracle.point_set_distance(V, F, V[np.unique(F)])
    assert r["max"] <= 1e-7 and r["sum"] <= 1e-5
    P = np.array([[2.0, 0, 0], [np.nan, 0, 0], [0, 3.0, 0]], np.float32)
    r = oracle.point_set_distance(V, F, P)
    assert r["count"] == 2 and r["argmax"] == 2
    empty = oracle.point_set_distance(V, F, np.zeros((0, 3), np.float32))
    assert empty == {"max": -1.0, "argmax": -1, "sum": 0.0, "sum_sq": 0.0, "count": 0}


def test_point_set_distance_concentric_spheres_bounds():
    """Vertices of a radius-2 icosphere against a unit one (convex, inscribed
    in the unit sphere, inradius rho): every distance lies in [1, 2 - rho]."""
    V, F = gen.icosphere(3)
    A = (2.0 * gen.icosphere(2)[0]).astype(np.float32)
    a, b, c = (V[F[:, k]].astype(np.float64) for k in range(3))
    n = np.cross(b - a, c - a)
    rho = np.min(np.abs(np.sum(n * a, axis=1)) / np.linalg.norm(n, axis=1))
    d, _, _, _ = oracle.distance(V, F, A, want_closest=False)
    assert d.min() >= 1.0 - 1e-6 and d.max() <= 2.0 - rho + 1e-6
    r = oracle.point_set_distance(V, F, A)
    assert abs(r["max"] - d.max()) == 0 and r["count"] == len(A)


# -------------------------------------------- per-triangle helper closed forms

# One right triangle a = (0,0,0), b = (1,0,0), c = (0,1,0) in the plane z = 0,
# placed in each coordinate plane and translated by exactly representable
# offsets, so that every closed form below is exact in FP64.  Each point is
# (local x, local y, height h) with its region, the expected closest point
# (local) and distance.  A helper that returned 0, or too small or too large
# a value, or the closest point of another region, fails.
_REGION_CASES = [
    # face: straight above an interior point
    ((0.25, 0.5, 0.75), "face", (0.25, 0.5, 0.0)),
    ((0.125, 0.125, -2.0), "face", (0.125, 0.125, 0.0)),
    # edge ab (y = 0), edge ca (x = 0), edge bc (x + y = 1)
    ((0.5, -0.75, 0.5), "ab", (0.5, 0.0, 0.0)),
    ((-0.5, 0.25, -1.0), "ca", (0.0, 0.25, 0.0)),
    ((0.75, 0.75, 0.25), "bc", (0.5, 0.5, 0.0)),
    # vertices a, b, c
    ((-0.5, -0.25, 1.0), "a", (0.0, 0.0, 0.0)),
    ((1.5, -0.5, -0.25), "b", (1.0, 0.0, 0.0)),
    ((-0.25, 1.75, 0.5), "c", (0.0, 1.0, 0.0)),
]


def _placed_triangle(plane, offset, scale):
    """Vertices and the local->world map of the unit right triangle placed
    in coordinate plane ``plane`` (0: z = const, 1: x = const, 2: y = const)."""
    axes = [(0, 1, 2), (1, 2, 0), (2, 0, 1)][plane]

    def world(u):
        w = np.zeros(3)
        for k in range(3):
            w[axes[k]] = scale * u[k]
        return w + np.asarray(offset)

    return world


@pytest.mark.parametrize("plane", [0, 1, 2])
@pytest.mark.parametrize("offset,scale", [((0.0, 0.0, 0.0), 1.0), ((2.5, -1.25, 0.375), 4.0),
                                          ((-100.0, 50.0, 12.0), 0.0625)])
def test_distance_to_triangles_closed_forms(plane, offset, scale):
    world = _placed_triangle(plane, offset, scale)
    V = np.array([world((0, 0, 0)), world((1, 0, 0)), world((0, 1, 0))], np.float32)
    F = np.array([[0, 1, 2]], np.int32)
    assert np.array_equal(V.astype(np.float64),
                          np.array([world((0, 0, 0)), world((1, 0, 0)), world((0, 1, 0))]))
    Q = np.array([world(u) for u, _, _ in _REGION_CASES])
    P = np.array([world(p) for _, _, p in _REGION_CASES])
    exp = np.linalg.norm(Q - P, axis=1)
    assert np.all(exp > 0.1 * scale)
    assert np.array_equal(Q.astype(np.float32).astype(np.float64), Q)   # exact in float32
    tri = np.zeros(len(Q), np.int32)
    d, p, lam = oracle.distance_to_triangles(V, F, Q.astype(np.float32), tri)
    assert np.max(np.abs(d - exp)) <= 1e-14 * max(1.0, np.abs(Q).max())
    assert np.max(np.abs(p - P)) <= 1e-13 * max(1.0, np.abs(Q).max())
    assert np.allclose(lam.sum(1), 1.0, atol=1e-14) and lam.min() >= 0.0
    assert np.max(np.abs(lam @ V.astype(np.float64) - P)) <= 1e-12 * max(1.0, np.abs(Q).max())
    d64 = oracle.distance_to_triangles64(V, F, Q, tri)
    assert np.max(np.abs(d64 - exp)) <= 1e-14 * max(1.0, np.abs(Q).max())
    # the float64 variant takes points that are not float32 values
    Q2 = Q + np.array([1e-9, -3e-10, 7e-10]) * scale
    P2 = np.array([world(p) for _, _, p in _REGION_CASES])
    d2 = oracle.distance_to_triangles64(V, F, Q2, tri)
    assert np.max(np.abs(d2 - np.linalg.norm(Q2 - P2, axis=1))) <= 4e-9 * scale


def test_distance_to_triangles_picks_the_given_triangle():
    """Two triangles at different known distances: each query is measured
    against the triangle named for it, not the nearer one."""
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 2], [1, 0, 2], [0, 1, 2]], np.float32)
    F = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    Q = np.array([[0.25, 0.25, 0.5], [0.25, 0.25, 0.5], [0.25, 0.25, 3.0]], np.float32)
    tri = np.array([0, 1, 0], np.int32)
    d, p, _ = oracle.distance_to_triangles(V, F, Q, tri)
    assert np.array_equal(d, [0.5, 1.5, 3.0])
    assert np.array_equal(p, [[0.25, 0.25, 0.0], [0.25, 0.25, 2.0], [0.25, 0.25, 0.0]])
    d64 = oracle.distance_to_triangles64(V, F, Q.astype(np.float64), tri)
    assert np.array_equal(d64, [0.5, 1.5, 3.0])


def test_distance_to_triangles_matches_region_walk_on_random_meshes():
    rng = np.random.default_rng(11)
    V = rng.normal(size=(60, 3)).astype(np.float32)
    # distinct corners (the region walk divides by zero on a repeated one)
    F = np.array([rng.choice(60, 3, replace=False) for _ in range(200)], np.int32)
    Q = (rng.normal(size=(2000, 3)) * 2).astype(np.float32)
    tri = rng.integers(0, 200, 2000).astype(np.int32)
    d, p, _ = oracle.distance_to_triangles(V, F, Q, tri)
    Vd = V.astype(np.float64)
    ref = np.array([np.linalg.norm(Q[i].astype(np.float64) - ericson_region_walk(Q[i].astype(np.float64),
                                                                                *Vd[F[tri[i]]]))
                    for i in range(len(Q))])
    assert np.max(np.abs(d - ref)) <= 1e-12
    P = Q.astype(np.float64) + rng.normal(size=(2000, 3)) * 1e-3
    d64 = oracle.distance_to_triangles64(V, F, P, tri)
    ref64 = np.array([np.linalg.norm(P[i] - ericson_region_walk(P[i], *Vd[F[tri[i]]])) for i in range(len(P))])
    assert np.max(np.abs(d64 - ref64)) <= 1e-12
