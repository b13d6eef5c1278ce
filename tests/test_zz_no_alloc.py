"""The no-allocation query (p2m_query_noalloc) against p2m_query through the
C ABI: the same kernels on the same inputs, so the outputs must be equal bit
for bit, on two calls in a row (the second with fewer points, so the shared
scratch holds the first call's leftovers), and a point count beyond its
scratch is refused before any launch."""
import ctypes

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


def run_both(p2m, mesh, q):
    n = q.shape[0]
    outs = []
    for fn in ("p2m_query", "p2m_query_noalloc"):
        d = torch.full((n,), -1.0, device="cuda")
        t = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        c = torch.full((n, 3), -1.0, device="cuda")
        rc = getattr(p2m.lib(), fn)(mesh.handle, p2m._ptr(q), n, p2m._ptr(d), p2m._ptr(t), p2m._ptr(c),
                                    p2m._stream())
        assert rc == 0, (fn, p2m.lib().p2m_last_error())
        outs.append((d, t, c))
    torch.cuda.synchronize()
    return outs


def test_noalloc_equals_query_two_calls(dev):
    c = gen.config_c2(900_000, 900_000)
    m = dev.Mesh(c["V"], c["F"])
    q1 = torch.from_numpy(c["Q"]).cuda()
    q2 = torch.from_numpy(c["Q"][::7].copy()).cuda()
    for q in (q1, q2):
        ref, got = run_both(dev, m, q)
        for a, b in zip(ref, got):
            assert torch.equal(a, b)
        assert int((got[1] < 0).sum()) == 0


def test_noalloc_refuses_counts_beyond_its_scratch(dev):
    from paper_2605_00429_amd import _lib
    V, F = gen.icosphere(3)
    m = dev.Mesh(V, F)
    buf = torch.empty(16, device="cuda")
    p = ctypes.c_void_p(buf.data_ptr())
    # pointers are never read: the count is refused first
    assert dev.lib().p2m_query_noalloc(m.handle, p, 3_000_000, p, None, None, None) == _lib.P2M_ERR_INVALID_ARG
    assert b"scratch" in dev.lib().p2m_last_error()
    assert dev.lib().p2m_query_noalloc(m.handle, p, 0, p, None, None, None) == _lib.P2M_OK
