"""ctypes binding of ``libp2m.so``: the C ABI of ``include/p2m.h`` with the
same names, argument marshalling only.

Loading fails loudly if the library has not been built: there is no
fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libp2m.so")

P2M_OK = 0
P2M_ERR_INVALID_ARG = 1
P2M_ERR_BAD_MESH = 2
P2M_ERR_OOM = 3
P2M_ERR_HIP = 4
P2M_ERR_INTERNAL = 5
P2M_ERR_NO_DEVICE = 6


class P2MError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"p2m error {code}: {msg}")
        self.code = code


class p2m_mesh_desc(ctypes.Structure):
    _fields_ = [("vertices", ctypes.c_void_p), ("n_vertices", ctypes.c_int64),
                ("triangles", ctypes.c_void_p), ("n_triangles", ctypes.c_int64)]


class p2m_build_opts(ctypes.Structure):
    _fields_ = [("domain_scale", ctypes.c_float), ("augment", ctypes.c_int32),
                ("tau_scale", ctypes.c_float), ("dense_min_sites", ctypes.c_int32),
                ("dense_rel", ctypes.c_float), ("ring_sites", ctypes.c_int32), ("ring_layers", ctypes.c_int32),
                ("aux_list_mode", ctypes.c_int32), ("list_inflation_rel", ctypes.c_float),
                ("seed_cell_scale", ctypes.c_float), ("seed_max_cells", ctypes.c_int64),
                ("n_threads", ctypes.c_int32), ("decomposition", ctypes.c_int32),
                ("octree_max_list", ctypes.c_int32), ("octree_max_depth", ctypes.c_int32),
                ("gpu_lists", ctypes.c_int32), ("gpu_voronoi", ctypes.c_int32),
                ("device", ctypes.c_int32), ("gpu_cell_pass", ctypes.c_int32)]


class p2m_stats(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("n_triangles", ctypes.c_int64),
                ("n_sites", ctypes.c_int64), ("n_vertex_sites", ctypes.c_int64),
                ("n_aux_sites", ctypes.c_int64), ("n_dense_cells", ctypes.c_int64),
                ("adj_nnz", ctypes.c_int64), ("adj_max", ctypes.c_int64),
                ("list_nnz", ctypes.c_int64), ("list_max", ctypes.c_int64),
                ("adj_avg", ctypes.c_double), ("list_avg", ctypes.c_double),
                ("seed_dims", ctypes.c_int32 * 3),
                ("t_voronoi_s", ctypes.c_double), ("t_optimize_s", ctypes.c_double),
                ("t_lists_s", ctypes.c_double), ("t_layout_s", ctypes.c_double),
                ("t_total_s", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("diag", ctypes.c_double), ("n_cells_device", ctypes.c_int64),
                ("n_cells_host", ctypes.c_int64)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if name == "seed_dims" else v
        return d


class p2m_query_config(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_int32), ("reorder", ctypes.c_int32), ("xcd_groups", ctypes.c_int32),
                ("sort_bits", ctypes.c_int32), ("stage", ctypes.c_int32), ("group", ctypes.c_int32)]


_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64

# name -> (restype, argtypes)
SIGNATURES = {
    "p2m_default_opts": (None, [ctypes.POINTER(p2m_build_opts)]),
    "p2m_build": (_I32, [ctypes.POINTER(p2m_mesh_desc), ctypes.POINTER(p2m_build_opts),
                         ctypes.POINTER(_VP)]),
    "p2m_destroy": (_I32, [_VP]),
    "p2m_query": (_I32, [_VP, _VP, _I64, _VP, _VP, _VP, _VP]),
    "p2m_query_noalloc": (_I32, [_VP, _VP, _I64, _VP, _VP, _VP, _VP]),
    "p2m_point_set_distance": (_I32, [_VP, _VP, _I64, _VP, _VP]),
    "p2m_mesh_distance": (_I32, [_VP, _VP, _VP, _I64, _VP, _I64, _VP, _VP]),
    "p2m_query_touched": (_I32, [_VP, _VP, _I64, _VP, _VP, _VP, _VP, _VP, _VP]),
    "p2m_query_backward": (_I32, [_VP, _VP, _I64, _VP, _VP, _VP, _VP, _VP]),
    "p2m_query_backward_ordered": (_I32, [_VP, _VP, _VP, _I64, _VP, _VP, _VP, _VP, _VP]),
    "p2m_query_fused": (_I32, [_VP, _VP, _I64, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "p2m_get_stats": (_I32, [_VP, ctypes.POINTER(p2m_stats)]),
    "p2m_get_query_config": (_I32, [_VP, ctypes.POINTER(p2m_query_config)]),
    "p2m_set_query_config": (_I32, [_VP, ctypes.POINTER(p2m_query_config)]),
    "p2m_query_counters": (_I32, [_VP, _VP, _I64, _VP, _VP, _VP, _VP, _VP]),
    "p2m_sort_points": (_I32, [_VP, _VP, _I64, _VP, _VP, _VP]),
    "p2m_query_sorted": (_I32, [_VP, _VP, _VP, _I64, _VP, _VP, _VP, _VP]),
    "p2m_query_ordered": (_I32, [_VP, _VP, _VP, _I64, _VP, _VP, _VP, _VP]),
    "p2m_host_sites": (_I32, [_VP, _VP, _VP]),
    "p2m_host_site_of_vertex": (_I32, [_VP, _VP]),
    "p2m_host_list": (_I32, [_VP, _I64, _VP, _I64, ctypes.POINTER(_I64)]),
    "p2m_host_neighbors": (_I32, [_VP, _I64, _VP, _I64, ctypes.POINTER(_I64)]),
    "p2m_host_locate": (_I32, [_VP, _VP, _I64, _VP]),
    "p2m_batch_create": (_I32, [_VP, _I32, _VP, _I32, ctypes.c_char_p, ctypes.POINTER(_VP)]),
    "p2m_batch_bind": (_I32, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "p2m_batch_launch": (_I32, [_VP, _VP]),
    "p2m_batch_config": (_I32, [_VP, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "p2m_batch_set_config": (_I32, [_VP, _I32, _I32, _I32, _I32]),
    "p2m_batch_destroy": (_I32, [_VP]),
    "p2m_status_string": (ctypes.c_char_p, [_I32]),
    "p2m_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """The loaded library (raises if it was never built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first "
                              "(python -m paper_2605_00429_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != P2M_OK:
        msg = lib().p2m_last_error().decode(errors="replace")
        raise P2MError(rc, msg)
    return rc


def default_opts():
    o = p2m_build_opts()
    lib().p2m_default_opts(ctypes.byref(o))
    return o
