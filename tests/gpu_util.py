"""Shared helpers for the GPU parity tests: acceptance rules against the FP64
oracle.

For mesh box diagonal D and tol = 1e-5 D (the stated correctness bound):
  * |d_gpu - d64| <= tol;
  * the GPU triangle is accepted iff its FP64 distance is within tol of d64
    (several triangles are correct at shared edges, vertices and medial ties);
  * the GPU closest point lies on the GPU triangle within tol and
    | |q - closest| - d_gpu | <= tol.
"""
import numpy as np

import oracle


def to_np(t):
    return t.detach().cpu().numpy()


def exact_reference(V, F, Q, want_closest=True):
    """The oracle's exact FP64 result for every point of ``Q``: the tier-B
    branch-and-bound, bit-identical to the brute force (which its own tests
    pin), fast enough for the full-size point sets.  ``(d, tri, closest)``."""
    d, t, p, _ = oracle.distance_exact(V, F, Q, want_closest=want_closest)
    return d, t, p


def check_forward(V, F, Q, dist, tri, closest, D, d64=None, label=""):
    """Assert the acceptance rules; returns (max |dd|/D, p99.9 |dd|/D)."""
    tol = 1e-5 * D
    dist, tri, closest = np.asarray(dist), np.asarray(tri), np.asarray(closest)
    if d64 is None:
        d64, _, _, _ = oracle.distance(V, F, Q, want_closest=False)
    assert len(dist) == len(Q) == len(d64)
    err = np.abs(dist.astype(np.float64) - d64)
    bad = np.nonzero(~(err <= tol))[0]
    assert len(bad) == 0, f"{label}: {len(bad)} distances off, worst {err[bad].max() if len(bad) else 0}, first {bad[:5]}"
    assert tri.min() >= 0 and tri.max() < len(F)
    dt, _, _ = oracle.distance_to_triangles(V, F, Q, tri)
    bad = np.nonzero(dt > d64 + tol)[0]
    assert len(bad) == 0, f"{label}: {len(bad)} triangle ids not within tol of the minimum, e.g. {bad[:5]}"
    on = oracle.distance_to_triangles64(V, F, closest.astype(np.float64), tri)
    assert on.max() <= tol, f"{label}: closest point off its triangle by {on.max()}"
    dq = np.linalg.norm(Q.astype(np.float64) - closest.astype(np.float64), axis=1)
    assert np.abs(dq - dist).max() <= tol, f"{label}: |q - closest| differs from distance"
    return err.max() / D, float(np.quantile(err, 0.999)) / D
