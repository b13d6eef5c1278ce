"""FP64 brute-force CPU oracle for point-to-mesh distance (ctypes binding).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this package; the library's product path never
imports it.  It shares no code with the HIP library.

The C source (``p2m_oracle.c``) states what is computed: the minimum
point-triangle distance over all triangles (the definition the paper's query
reaches exactly, Sec. 1, Eq. (1) and Sec. 3.4), the lowest-index argmin, the
closest point, and the envelope-theorem gradient.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "p2m_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc (OpenMP, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                           "-std=c99", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_bruteforce.argtypes = [P, i64, P, i64, P, i64, P, P, P, ctypes.c_int]
        lib.oracle_bruteforce.restype = ctypes.c_int
        lib.oracle_point_triangle_batch.argtypes = [P, P, P, P, i64, P, P, P]
        lib.oracle_point_triangle_batch64.argtypes = [P, P, P, P, i64, P]
        lib.oracle_gradient.argtypes = [P, i64, P, P, P, P, i64, P, P]
        lib.oracle_nearest_point.argtypes = [P, i64, P, i64, P, P]
        lib.oracle_threads.argtypes = [ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_point_triangle_sq.argtypes = [P, P, P, P, P, P]
        lib.oracle_point_triangle_sq.restype = ctypes.c_double
        lib.oracle_tree_build.argtypes = [P, i64, P, i64]
        lib.oracle_tree_build.restype = P
        lib.oracle_tree_free.argtypes = [P]
        lib.oracle_tree_query.argtypes = [P, P, i64, P, P, P, ctypes.c_int]
        lib.oracle_tree_query.restype = ctypes.c_int
        _lib = lib
    return _lib


def _f32(a, cols=3):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a.reshape(-1, cols) if cols else a.reshape(-1)


def _i32(a, cols=3):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a.reshape(-1, cols) if cols else a.reshape(-1)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def threads(n_threads=0):
    """Threads the oracle's parallel loops use (``0`` = OpenMP default)."""
    return _load().oracle_threads(int(n_threads))


def distance(V, F, Q, n_threads=0, want_closest=True):
    """Brute-force FP64 distance.  Returns ``(d, tri, closest, threads_used)``.

    ``d`` and ``closest`` are float64; ``tri`` is int32 (lowest index on ties).
    """
    V, F, Q = _f32(V), _i32(F), _f32(Q)
    n = len(Q)
    d = np.empty(n, np.float64)
    tri = np.empty(n, np.int32)
    p = np.empty((n, 3), np.float64) if want_closest else None
    used = _load().oracle_bruteforce(_p(V), len(V), _p(F), len(F), _p(Q), n, _p(d), _p(tri),
                                     _p(p), int(n_threads))
    return d, tri, p, used


class ExactTree:
    """Tier-B oracle: the same exact FP64 result as ``distance`` (distance,
    lowest-index triangle, closest point, bit for bit), found by
    branch-and-bound over the oracle's own box tree of the triangles, for
    query sets too large for the brute force."""

    def __init__(self, V, F):
        self.V, self.F = _f32(V), _i32(F)
        self._h = _load().oracle_tree_build(_p(self.V), len(self.V), _p(self.F), len(self.F))
        if not self._h:
            raise MemoryError("oracle tree build failed")

    def distance(self, Q, n_threads=0, want_closest=True):
        """``(d, tri, closest, threads_used)`` as ``distance``."""
        Q = _f32(Q)
        n = len(Q)
        d = np.empty(n, np.float64)
        tri = np.empty(n, np.int32)
        p = np.empty((n, 3), np.float64) if want_closest else None
        used = _load().oracle_tree_query(self._h, _p(Q), n, _p(d), _p(tri), _p(p), int(n_threads))
        return d, tri, p, used

    def close(self):
        if getattr(self, "_h", None):
            _load().oracle_tree_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def distance_exact(V, F, Q, n_threads=0, want_closest=True):
    """Tier-B oracle in one call: builds the tree, answers ``Q``."""
    t = ExactTree(V, F)
    try:
        return t.distance(Q, n_threads=n_threads, want_closest=want_closest)
    finally:
        t.close()


def point_triangle(q, a, b, c):
    """Squared-distance-free helper: ``(d, p, lam)`` for one point and triangle."""
    q = np.ascontiguousarray(q, np.float64)
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    c = np.ascontiguousarray(c, np.float64)
    p = np.empty(3, np.float64)
    lam = np.empty(3, np.float64)
    d2 = _load().oracle_point_triangle_sq(_p(q), _p(a), _p(b), _p(c), _p(p), _p(lam))
    return float(np.sqrt(d2)), p, lam


def distance_to_triangles(V, F, Q, tri):
    """FP64 distance from each ``Q[i]`` (float32) to triangle ``tri[i]``.
    Returns ``(d, closest, barycentrics)``."""
    V, F, Q, tri = _f32(V), _i32(F), _f32(Q), _i32(tri, None)
    n = len(Q)
    d = np.empty(n, np.float64)
    p = np.empty((n, 3), np.float64)
    lam = np.empty((n, 3), np.float64)
    _load().oracle_point_triangle_batch(_p(V), _p(F), _p(Q), _p(tri), n, _p(d), _p(p), _p(lam))
    return d, p, lam


def distance_to_triangles64(V, F, P, tri):
    """FP64 distance from float64 points ``P[i]`` to triangle ``tri[i]``."""
    V, F, tri = _f32(V), _i32(F), _i32(tri, None)
    P = np.ascontiguousarray(P, np.float64).reshape(-1, 3)
    d = np.empty(len(P), np.float64)
    _load().oracle_point_triangle_batch64(_p(V), _p(F), _p(P), _p(tri), len(P), _p(d))
    return d


def gradient(V, F, Q, tri, g):
    """Envelope-theorem gradient of ``sum_i g_i d(q_i)``: ``(dL/dQ, dL/dV)`` in FP64,
    dL/dV accumulated sequentially in query order."""
    V, F, Q, tri = _f32(V), _i32(F), _f32(Q), _i32(tri, None)
    g = _f32(g, None)
    dq = np.empty((len(Q), 3), np.float64)
    dV = np.empty((len(V), 3), np.float64)
    _load().oracle_gradient(_p(V), len(V), _p(F), _p(Q), _p(tri), _p(g), len(Q), _p(dq), _p(dV))
    return dq, dV


def point_set_distance(V, F, P, n_threads=0):
    """Distances of the points ``P`` to the mesh, reduced as the mesh-to-mesh
    measures need them (Sec. 5 names mesh-to-mesh distance as an application
    of the point query): the largest distance and the first point attaining
    it, the FP64 sums of d and d^2 and the number of finite points (points
    with a non-finite coordinate are left out).  ``max`` / ``argmax`` are -1
    when no point counts."""
    P = np.asarray(P, dtype=np.float32).reshape(-1, 3)
    if len(P) == 0:
        return {"max": -1.0, "argmax": -1, "sum": 0.0, "sum_sq": 0.0, "count": 0}
    d, _, _, _ = distance(V, F, P, n_threads=n_threads, want_closest=False)
    ok = np.isfinite(P).all(axis=1)
    if not ok.any():
        return {"max": -1.0, "argmax": -1, "sum": 0.0, "sum_sq": 0.0, "count": 0}
    dd = np.where(ok, d, -np.inf)
    k = int(np.argmax(dd))          # first index among equal maxima
    return {"max": float(dd[k]), "argmax": k, "sum": float(d[ok].sum()), "sum_sq": float((d[ok] ** 2).sum()),
            "count": int(ok.sum())}


def nearest_point(P, Q):
    """Brute-force nearest of the points ``P`` for each query: ``(idx, dist)``."""
    P, Q = _f32(P), _f32(Q)
    idx = np.empty(len(Q), np.int32)
    d = np.empty(len(Q), np.float64)
    _load().oracle_nearest_point(_p(P), len(P), _p(Q), len(Q), _p(idx), _p(d))
    return idx, d
