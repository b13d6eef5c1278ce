"""MI355X-native P2M++ point-to-mesh distance queries.

``Mesh(V, F)`` runs the host preprocessing (site augmentation, Voronoi cells,
interception lists) and uploads the search structure; ``distance(mesh, pts)``
answers queries on the GPU with hand-written HIP kernels and is
differentiable with respect to the points and the mesh vertices.

Every call goes through the C ABI of ``libp2m.so`` (``include/p2m.h``); this
module only marshals arguments.  PyTorch supplies device memory and streams.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import P2MError, check, lib

__all__ = ["Mesh", "Batch", "distance", "query", "query_backward", "query_fused", "point_set_distance",
           "mesh_distance", "hausdorff", "chamfer", "query_counters", "query_touched", "sort_points",
           "query_sorted", "query_ordered", "P2MError", "build_opts"]


def build_opts(**kw):
    """A ``p2m_build_opts`` with the library defaults, overridden by ``kw``."""
    o = _lib.default_opts()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown build option {k!r}")
        setattr(o, k, v)
    return o


def _np_mesh(V, F):
    try:
        import torch
        if isinstance(V, torch.Tensor):
            V = V.detach().cpu().numpy()
        if isinstance(F, torch.Tensor):
            F = F.detach().cpu().numpy()
    except ImportError:
        pass
    V = np.ascontiguousarray(V, dtype=np.float32).reshape(-1, 3)
    F = np.ascontiguousarray(F, dtype=np.int32).reshape(-1, 3)
    return V, F


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Mesh:
    """A triangle mesh preprocessed for P2M++ queries.

    ``device``: a CUDA/HIP device (index or ``torch.device``) to upload to,
    ``"host"`` for a host-only build (inspection, no queries), or ``None``
    for torch's current device.  Extra keyword arguments set
    ``p2m_build_opts`` fields.
    """

    def __init__(self, V, F, device=None, **opts):
        V_np, F_np = _np_mesh(V, F)
        self.V = V_np
        self.F = F_np
        self.vertices = V if not isinstance(V, np.ndarray) else None  # torch tensor for autograd
        o = build_opts(**opts)
        if device == "host":
            o.device = -1
            self.device = None
        else:
            import torch
            if device is None:
                dev = torch.cuda.current_device()
            else:
                dev = torch.device(device).index if not isinstance(device, int) else device
                if dev is None:
                    dev = torch.cuda.current_device()
            o.device = int(dev)
            self.device = torch.device("cuda", int(dev))
        desc = _lib.p2m_mesh_desc(V_np.ctypes.data_as(ctypes.c_void_p), len(V_np),
                                  F_np.ctypes.data_as(ctypes.c_void_p), len(F_np))
        h = ctypes.c_void_p()
        check(lib().p2m_build(ctypes.byref(desc), ctypes.byref(o), ctypes.byref(h)))
        self.handle = h
        self.opts = o

    def close(self):
        if getattr(self, "handle", None):
            lib().p2m_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ inspection
    def stats(self):
        s = _lib.p2m_stats()
        check(lib().p2m_get_stats(self.handle, ctypes.byref(s)))
        return s.as_dict()

    @property
    def n_sites(self):
        return self.stats()["n_sites"]

    def query_config(self):
        c = _lib.p2m_query_config()
        check(lib().p2m_get_query_config(self.handle, ctypes.byref(c)))
        return {"block_size": c.block_size, "reorder": c.reorder, "xcd_groups": c.xcd_groups,
                "sort_bits": c.sort_bits, "stage": c.stage, "group": c.group}

    def set_query_config(self, block_size=None, reorder=None, xcd_groups=None, sort_bits=None, stage=None,
                         group=None):
        """Launch configuration of this handle's queries (see p2m_query_config)."""
        cur = self.query_config()
        c = _lib.p2m_query_config(block_size if block_size is not None else cur["block_size"],
                                  int(reorder) if reorder is not None else cur["reorder"],
                                  xcd_groups if xcd_groups is not None else cur["xcd_groups"],
                                  sort_bits if sort_bits is not None else cur["sort_bits"],
                                  int(stage) if stage is not None else cur["stage"],
                                  int(group) if group is not None else cur["group"])
        check(lib().p2m_set_query_config(self.handle, ctypes.byref(c)))

    def host_sites(self):
        n = self.n_sites
        xyz = np.empty((n, 3), np.float32)
        aux = np.empty(n, np.uint8)
        check(lib().p2m_host_sites(self.handle, xyz.ctypes.data_as(ctypes.c_void_p),
                                   aux.ctypes.data_as(ctypes.c_void_p)))
        return xyz, aux.astype(bool)

    def site_of_vertex(self):
        out = np.empty(len(self.V), np.int32)
        check(lib().p2m_host_site_of_vertex(self.handle, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def host_list(self, site):
        n = ctypes.c_int64()
        check(lib().p2m_host_list(self.handle, int(site), None, 0, ctypes.byref(n)))
        out = np.empty(n.value, np.int32)
        check(lib().p2m_host_list(self.handle, int(site), out.ctypes.data_as(ctypes.c_void_p),
                                  n.value, ctypes.byref(n)))
        return out

    def host_neighbors(self, site):
        n = ctypes.c_int64()
        check(lib().p2m_host_neighbors(self.handle, int(site), None, 0, ctypes.byref(n)))
        out = np.empty(n.value, np.int32)
        check(lib().p2m_host_neighbors(self.handle, int(site), out.ctypes.data_as(ctypes.c_void_p),
                                       n.value, ctypes.byref(n)))
        return out

    def host_locate(self, P):
        P = np.ascontiguousarray(P, np.float32).reshape(-1, 3)
        out = np.empty(len(P), np.int32)
        check(lib().p2m_host_locate(self.handle, P.ctypes.data_as(ctypes.c_void_p), len(P),
                                    out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def list_lengths(self):
        n = self.n_sites
        out = np.empty(n, np.int64)
        L = ctypes.c_int64()
        for s in range(n):
            check(lib().p2m_host_list(self.handle, s, None, 0, ctypes.byref(L)))
            out[s] = L.value
        return out


def _check_points(mesh, points):
    import torch
    if mesh.device is None:
        raise P2MError(_lib.P2M_ERR_NO_DEVICE, "mesh was built host-only")
    if not isinstance(points, torch.Tensor) or points.device != mesh.device:
        raise ValueError(f"points must be a tensor on {mesh.device}")
    if points.dtype != torch.float32 or points.dim() != 2 or points.shape[1] != 3:
        raise ValueError("points must be an (n, 3) float32 tensor")
    return points.contiguous()


def query(mesh, points, want_tri=True, want_closest=True, stream=None):
    """Forward query: ``(dist, tri, closest)`` (tri / closest may be None)."""
    import torch
    p = _check_points(mesh, points)
    n = p.shape[0]
    dist = torch.empty(n, dtype=torch.float32, device=p.device)
    tri = torch.empty(n, dtype=torch.int32, device=p.device) if want_tri else None
    closest = torch.empty((n, 3), dtype=torch.float32, device=p.device) if want_closest else None
    check(lib().p2m_query(mesh.handle, _ptr(p), n, _ptr(dist), _ptr(tri), _ptr(closest), _stream(stream)))
    return dist, tri, closest


def point_set_distance(mesh, points, stream=None):
    """Distances of a point set to ``mesh``, reduced on the device
    (``p2m_point_set_distance``): a dict with ``max``, ``argmax`` (lowest
    index on ties), ``sum``, ``sum_sq`` and ``count`` (non-finite points are
    left out; ``max`` and ``argmax`` are -1 when none is counted)."""
    import torch
    p = _check_points(mesh, points)
    out = torch.empty(5, dtype=torch.float64, device=p.device)
    check(lib().p2m_point_set_distance(mesh.handle, _ptr(p), p.shape[0], _ptr(out), _stream(stream)))
    v = out.cpu().tolist()
    return {"max": v[0], "argmax": int(v[1]), "sum": v[2], "sum_sq": v[3], "count": int(v[4])}


def mesh_distance(mesh_a, mesh_b, points_a=None, points_b=None, stream=None):
    """Distances between two meshes measured on point sets of each
    (``p2m_mesh_distance``): ``points_a`` on A against mesh B and
    ``points_b`` on B against mesh A, by default each mesh's referenced
    vertices.  Returns a dict with the one-sided Hausdorff distances
    ``hausdorff_ab`` and ``hausdorff_ba``, the symmetric ``hausdorff``, the
    Chamfer distances ``chamfer`` (means of d) and ``chamfer_sq`` (means of
    d^2), and ``count``, the number of points counted."""
    import torch
    dev = mesh_a.device
    if mesh_b.device != dev:
        raise ValueError("both meshes must be on one device")
    pa = _check_points(mesh_a, points_a) if points_a is not None else None
    pb = _check_points(mesh_b, points_b) if points_b is not None else None
    out = torch.empty(6, dtype=torch.float64, device=dev)
    check(lib().p2m_mesh_distance(mesh_a.handle, mesh_b.handle, _ptr(pa), pa.shape[0] if pa is not None else 0,
                                  _ptr(pb), pb.shape[0] if pb is not None else 0, _ptr(out), _stream(stream)))
    v = out.cpu().tolist()
    return {"hausdorff_ab": v[0], "hausdorff_ba": v[1], "hausdorff": v[2], "chamfer": v[3], "chamfer_sq": v[4],
            "count": int(v[5])}


def hausdorff(mesh_a, mesh_b, points_a=None, points_b=None, symmetric=True, stream=None):
    """Hausdorff distance between two meshes measured on point sets of each
    (``points_a`` on A, ``points_b`` on B; by default their referenced
    vertices).  One-sided (A to B) unless ``symmetric``."""
    r = mesh_distance(mesh_a, mesh_b, points_a, points_b, stream)
    return r["hausdorff"] if symmetric else r["hausdorff_ab"]


def chamfer(mesh_a, mesh_b, points_a=None, points_b=None, squared=False, stream=None):
    """Chamfer distance: the mean distance from points of A to mesh B plus
    the mean distance from points of B to mesh A (mean squared distances
    with ``squared``)."""
    r = mesh_distance(mesh_a, mesh_b, points_a, points_b, stream)
    return r["chamfer_sq"] if squared else r["chamfer"]


def sort_points(mesh, points, want_sorted=False, stream=None):
    """The order (int32 permutation) in which ``query`` visits the points, and
    with ``want_sorted`` also the points in that order: ``(order, sorted)``."""
    import torch
    p = _check_points(mesh, points)
    order = torch.empty(p.shape[0], dtype=torch.int32, device=p.device)
    sp = torch.empty_like(p) if want_sorted else None
    check(lib().p2m_sort_points(mesh.handle, _ptr(p), p.shape[0], _ptr(order), _ptr(sp), _stream(stream)))
    return (order, sp) if want_sorted else order


def query_sorted(mesh, sorted_points, order, out=None, stream=None):
    """The search half of ``query`` on points already in visiting order;
    outputs land at ``order`` positions.  ``out`` may supply preallocated
    ``(dist, tri, closest)`` tensors."""
    import torch
    p = _check_points(mesh, sorted_points)
    n = p.shape[0]
    if out is None:
        out = (torch.empty(n, dtype=torch.float32, device=p.device),
               torch.empty(n, dtype=torch.int32, device=p.device),
               torch.empty((n, 3), dtype=torch.float32, device=p.device))
    dist, tri, closest = out
    check(lib().p2m_query_sorted(mesh.handle, _ptr(p), _ptr(order), n, _ptr(dist), _ptr(tri), _ptr(closest),
                                 _stream(stream)))
    return dist, tri, closest


def query_ordered(mesh, points, order, out=None, stream=None):
    """The search half of ``query`` with a given visiting order (or None).
    ``out`` may supply preallocated ``(dist, tri, closest)`` tensors."""
    import torch
    p = _check_points(mesh, points)
    n = p.shape[0]
    if out is None:
        out = (torch.empty(n, dtype=torch.float32, device=p.device),
               torch.empty(n, dtype=torch.int32, device=p.device),
               torch.empty((n, 3), dtype=torch.float32, device=p.device))
    dist, tri, closest = out
    check(lib().p2m_query_ordered(mesh.handle, _ptr(p), _ptr(order), n, _ptr(dist), _ptr(tri),
                                  _ptr(closest), _stream(stream)))
    return dist, tri, closest


def query_counters(mesh, points, stream=None):
    """Instrumented forward: ``(dist, tri, closest, counters)`` with counters a
    dict of totals over the points."""
    import torch
    p = _check_points(mesh, points)
    n = p.shape[0]
    dist = torch.empty(n, dtype=torch.float32, device=p.device)
    tri = torch.empty(n, dtype=torch.int32, device=p.device)
    closest = torch.empty((n, 3), dtype=torch.float32, device=p.device)
    ctr = torch.zeros(8, dtype=torch.int64, device=p.device)
    check(lib().p2m_query_counters(mesh.handle, _ptr(p), n, _ptr(dist), _ptr(tri), _ptr(closest),
                                   _ptr(ctr), _stream(stream)))
    c = ctr.cpu().tolist()
    return dist, tri, closest, dict(zip(COUNTER_NAMES, c))


COUNTER_NAMES = ["walk_steps", "adj_read", "list_read", "exact_tests", "fallback", "list_len", "walk_capped"]
# the structure arrays p2m_query_touched reports on, and the bytes of one item
TOUCH_ITEMS = [("site_rec", 32), ("adjacency", 16), ("list_sphere", 16), ("list_record", 48), ("seed", 4),
               ("fallback_triangle", 48), ("fallback_bvh_node", 32)]


def query_touched(mesh, points, stream=None):
    """Instrumented forward that also counts the distinct structure items the
    launch reads (``p2m_query_touched``): ``(dist, tri, closest, counters,
    items)`` with ``items`` a dict name -> (distinct items, bytes)."""
    import torch
    p = _check_points(mesh, points)
    n = p.shape[0]
    dist = torch.empty(n, dtype=torch.float32, device=p.device)
    tri = torch.empty(n, dtype=torch.int32, device=p.device)
    closest = torch.empty((n, 3), dtype=torch.float32, device=p.device)
    ctr = torch.zeros(8, dtype=torch.int64, device=p.device)
    items = (ctypes.c_int64 * 7)()
    check(lib().p2m_query_touched(mesh.handle, _ptr(p), n, _ptr(dist), _ptr(tri), _ptr(closest), _ptr(ctr),
                                  items, _stream(stream)))
    c = ctr.cpu().tolist()
    touched = {name: (int(items[k]), int(items[k]) * size) for k, (name, size) in enumerate(TOUCH_ITEMS)}
    return dist, tri, closest, dict(zip(COUNTER_NAMES, c)), touched


def query_backward(mesh, points, tri, grad_dist, grad_points=True, grad_vertices=None, order=None, stream=None):
    """Gradients of ``sum(grad_dist * dist)``: ``(dL/dpoints, dL/dV)``.
    ``grad_vertices`` may be a zeroed (nV, 3) tensor to accumulate into.
    ``order``: the visiting order ``sort_points`` gave for the forward pass
    (``p2m_query_backward_ordered``); without it the points are sorted again
    when dL/dV is wanted."""
    import torch
    p = _check_points(mesh, points)
    n = p.shape[0]
    g = grad_dist.contiguous().to(torch.float32)
    gq = torch.empty((n, 3), dtype=torch.float32, device=p.device) if grad_points else None
    if order is not None:
        check(lib().p2m_query_backward_ordered(mesh.handle, _ptr(p), _ptr(order), n, _ptr(tri.contiguous()),
                                               _ptr(g), _ptr(gq), _ptr(grad_vertices), _stream(stream)))
    else:
        check(lib().p2m_query_backward(mesh.handle, _ptr(p), n, _ptr(tri.contiguous()), _ptr(g), _ptr(gq),
                                       _ptr(grad_vertices), _stream(stream)))
    return gq, grad_vertices


def query_fused(mesh, points, grad_dist, grad_vertices=None, stream=None):
    """Forward and gradient in one pass: ``(dist, tri, closest, dL/dpoints)``;
    dL/dV is accumulated into ``grad_vertices`` when given."""
    import torch
    p = _check_points(mesh, points)
    n = p.shape[0]
    g = grad_dist.contiguous().to(torch.float32)
    dist = torch.empty(n, dtype=torch.float32, device=p.device)
    tri = torch.empty(n, dtype=torch.int32, device=p.device)
    closest = torch.empty((n, 3), dtype=torch.float32, device=p.device)
    gq = torch.empty((n, 3), dtype=torch.float32, device=p.device)
    check(lib().p2m_query_fused(mesh.handle, _ptr(p), n, _ptr(g), _ptr(dist), _ptr(tri), _ptr(closest),
                                _ptr(gq), _ptr(grad_vertices), _stream(stream)))
    return dist, tri, closest, gq


def _make_fn():
    import torch

    class _P2MDistance(torch.autograd.Function):
        @staticmethod
        def forward(ctx, points, vertices, mesh):
            p = points.detach()
            # sort once: the backward visits the points in the same order
            order = sort_points(mesh, p) if mesh.query_config()["reorder"] else None
            dist, tri, closest = query_ordered(mesh, p, order)
            ctx.mesh = mesh
            ctx.order = order
            ctx.save_for_backward(p, tri)
            ctx.has_vertices = vertices is not None
            ctx.mark_non_differentiable(tri, closest)
            return dist, tri, closest

        @staticmethod
        def backward(ctx, g_dist, g_tri, g_closest):
            points, tri = ctx.saved_tensors
            mesh = ctx.mesh
            need_p = ctx.needs_input_grad[0]
            need_v = ctx.has_vertices and ctx.needs_input_grad[1]
            if g_dist is None or not (need_p or need_v):
                return None, None, None
            gv = torch.zeros((len(mesh.V), 3), dtype=torch.float32, device=points.device) if need_v else None
            gq, gv = query_backward(mesh, points, tri, g_dist, grad_points=need_p, grad_vertices=gv, order=ctx.order)
            return gq, gv, None

    return _P2MDistance


_FN = None


def distance(mesh, points):
    """Differentiable distance: ``(dist, tri, closest)``.  Gradients flow to
    ``points`` and, if the mesh was built from a tensor that requires grad,
    to those vertices (the distance at the built positions)."""
    global _FN
    if _FN is None:
        _FN = _make_fn()
    v = mesh.vertices
    import torch
    if not (isinstance(v, torch.Tensor) and v.requires_grad):
        v = None
    return _FN.apply(points, v, mesh)


class Batch:
    """Many meshes and query sets in one persistent, graph-captured launch."""

    def __init__(self, meshes, counts, autotune=True, cache_path=None):
        self.meshes = list(meshes)
        self.counts = [int(c) for c in counts]
        arr = (ctypes.c_void_p * len(self.meshes))(*[m.handle.value for m in self.meshes])
        cnt = (ctypes.c_int64 * len(self.counts))(*self.counts)
        h = ctypes.c_void_p()
        check(lib().p2m_batch_create(arr, len(self.meshes), cnt, int(bool(autotune)),
                                     cache_path.encode() if cache_path else None, ctypes.byref(h)))
        self.handle = h
        self._keep = None

    def bind(self, points, dist, tri=None, closest=None, grad_dist=None, grad_points=None,
             grad_vertices=None, stream=None):
        gv = None
        if grad_vertices is not None:
            gv = (ctypes.c_void_p * len(self.meshes))(*[t.data_ptr() if t is not None else 0
                                                        for t in grad_vertices])
        self._keep = (points, dist, tri, closest, grad_dist, grad_points, grad_vertices)
        check(lib().p2m_batch_bind(self.handle, _ptr(points), _ptr(dist), _ptr(tri), _ptr(closest),
                                   _ptr(grad_dist), _ptr(grad_points), gv, _stream(stream)))

    def launch(self, stream=None):
        check(lib().p2m_batch_launch(self.handle, _stream(stream)))

    def config(self):
        t, g, b, st = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().p2m_batch_config(self.handle, ctypes.byref(t), ctypes.byref(g), ctypes.byref(b),
                                     ctypes.byref(st)))
        return {"tile": t.value, "grid": g.value, "block": b.value, "stage": st.value}

    def set_config(self, tile, grid, block, stage=0):
        """Pin the launch configuration (see ``p2m_batch_set_config``); call
        before ``bind``."""
        check(lib().p2m_batch_set_config(self.handle, int(tile), int(grid), int(block), int(stage)))

    def close(self):
        if getattr(self, "handle", None):
            lib().p2m_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
