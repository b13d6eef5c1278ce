"""The C-ABI library loads and exports every function include/p2m.h declares
(no GPU calls)."""
import ctypes
import os
import re

import paper_2605_00429_amd as p2m
from paper_2605_00429_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "p2m.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(p2m_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("p2m_build", "p2m_query", "p2m_query_backward", "p2m_query_fused",
                     "p2m_batch_create", "p2m_batch_bind", "p2m_batch_launch", "p2m_destroy",
                     "p2m_get_stats", "p2m_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_status_strings_and_defaults():
    L = p2m.lib()
    assert L.p2m_status_string(0) == b"ok"
    assert L.p2m_status_string(2) == b"bad mesh"
    o = _lib.default_opts()
    assert o.domain_scale == 10.0 and o.augment == 1 and o.device == -2
