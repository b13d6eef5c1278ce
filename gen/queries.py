"""Seeded query point sets.

All points are drawn in float64 and rounded once to float32.
"""
import numpy as np


def scaled_box(V, scale):
    """Axis-aligned bounding box of ``V`` scaled by ``scale`` about its centre."""
    V = np.asarray(V, dtype=np.float64)
    lo, hi = V.min(0), V.max(0)
    c, h = (lo + hi) * 0.5, (hi - lo) * 0.5 * scale
    return c - h, c + h


def uniform_box(rng, n, lo, hi):
    """``n`` points uniform in the box ``[lo, hi]`` (one (n,3) uniform draw)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return rng.uniform(lo, hi, (n, 3)).astype(np.float32)


def near_surface(rng, n, V, F, sigma):
    """``n`` points near the surface: a triangle picked with probability
    proportional to its area, a uniform point on it, plus isotropic Gaussian
    noise of standard deviation ``sigma``.

    Draw order: ``n`` uniforms for the triangle pick (inverse CDF over the
    cumulative areas), then an (n,2) uniform draw (r1, r2), then an (n,3)
    normal draw for the offset.  The point on the triangle is
    ``(1-sqrt r1) a + sqrt r1 (1-r2) b + sqrt r1 r2 c`` (Osada et al. 2002).
    """
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    cdf = np.cumsum(area)
    u = rng.uniform(0.0, cdf[-1], n)
    t = np.minimum(np.searchsorted(cdf, u, side="right"), len(F) - 1)
    r = rng.uniform(0.0, 1.0, (n, 2))
    s1 = np.sqrt(r[:, :1])
    p = (1.0 - s1) * a[t] + s1 * (1.0 - r[:, 1:]) * b[t] + s1 * r[:, 1:] * c[t]
    p += rng.normal(0.0, sigma, (n, 3))
    return p.astype(np.float32)
