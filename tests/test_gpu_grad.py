"""GPU gradients: the hand-written backward and fused kernels against the FP64
oracle gradient (envelope theorem), central finite differences of the FP64
oracle distance, and invariants at the full C3 size."""
import numpy as np
import pytest

import gen
import oracle

from gpu_util import check_forward, exact_reference, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_00429_amd as p2m
    return p2m


@pytest.fixture(scope="module")
def c3(dev):
    c = gen.config_c3()      # C2 mesh, 4M near-surface points, g ~ N(0, 1)
    return c, dev.Mesh(c["V"], c["F"])


def gpu_grads(p2m, m, Q, g):
    q = torch.from_numpy(np.ascontiguousarray(Q)).cuda()
    gt = torch.from_numpy(np.ascontiguousarray(g)).cuda()
    d, t, cl = p2m.query(m, q)
    gv = torch.zeros((len(m.V), 3), dtype=torch.float32, device="cuda")
    gq, gv = p2m.query_backward(m, q, t, gt, grad_vertices=gv)
    torch.cuda.synchronize()
    return to_np(d), to_np(t), to_np(cl), to_np(gq), to_np(gv)


def rel_err(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def test_c3_sample_against_oracle_gradient(dev, c3):
    c, m = c3
    V, F, D = c["V"], c["F"], c["D"]
    Q, g = c["Q"][:4000], c["G"][:4000].copy()
    d, t, cl, gq, gv = gpu_grads(dev, m, Q, g)
    d64, t64, p64, _ = oracle.distance(V, F, Q)
    # medial ties: a different triangle with a different closest point; the
    # gradient is discontinuous there, so those points are masked in both runs
    tie = (t != t64) & (np.linalg.norm(cl - p64, axis=1) > 1e-5 * D)
    assert tie.mean() < 0.01
    g[tie] = 0.0
    d, t, cl, gq, gv = gpu_grads(dev, m, Q, g)
    dq64, dV64 = oracle.gradient(V, F, Q, t64, g)
    assert rel_err(gq, dq64) <= 1e-3
    assert rel_err(gv, dV64) <= 1e-3
    # Per row, against the FP64 gradient taken at the GPU's own triangle: at
    # near-ties (distances equal within float32) the GPU may pick a
    # neighbouring triangle, which moves O(lambda) of a row to another vertex.
    # The forward tests already accept that triangle as a minimiser.
    dt, _, _ = oracle.distance_to_triangles(V, F, Q, t)
    assert np.all(dt <= d64 + 1e-5 * D)
    dq64, dV64 = oracle.gradient(V, F, Q, t, g)
    # relative to the row or, for rows that nearly cancel, to 1e-2 of the
    # rms row: a few float32 atomic additions round at ~1e-7 absolute
    rms = np.sqrt(np.mean(np.sum(dV64 ** 2, axis=1)))
    row = np.linalg.norm(gv - dV64, axis=1)
    lim = 1e-3 * np.maximum(np.linalg.norm(dV64, axis=1), 1e-2 * rms)
    worst = np.argsort(row - lim)[-3:]
    assert np.all(row <= lim), [(int(k), row[k], lim[k], dV64[k], gv[k]) for k in worst]
    rowq = np.linalg.norm(gq - dq64, axis=1)
    assert np.all(rowq <= 1e-3 * np.maximum(np.linalg.norm(dq64, axis=1), 1e-3))


def test_c3_full_size_against_oracle_gradient(dev, c3):
    """All 4M points of C3: the forward against the oracle's exact result,
    and the whole dL/dq (4M x 3) and dL/dV (163,842 x 3) against the FP64
    envelope-theorem gradient taken at the oracle's own argmins.  Medial ties
    (a different triangle with a different closest point, where the gradient
    jumps) are masked with g = 0 in both runs."""
    c, m = c3
    V, F, D, Q = c["V"], c["F"], c["D"], c["Q"]
    d64, t64, p64 = exact_reference(V, F, Q)
    q = torch.from_numpy(Q).cuda()
    d, t, cl = dev.query(m, q)
    torch.cuda.synchronize()
    d, t, cl = to_np(d), to_np(t), to_np(cl)
    print("C3 forward max|dd|/D, p99.9:", check_forward(V, F, Q, d, t, cl, D, d64=d64, label="C3"))
    tie = (t != t64) & (np.linalg.norm(cl - p64, axis=1) > 1e-5 * D)
    assert tie.mean() < 1e-3, tie.mean()
    g = c["G"].copy()
    g[tie] = 0.0
    gt = torch.from_numpy(g).cuda()
    gv = torch.zeros((len(V), 3), dtype=torch.float32, device="cuda")
    gq, gv = dev.query_backward(m, q, torch.from_numpy(t).cuda(), gt, grad_vertices=gv)
    gv2 = torch.zeros_like(gv)
    _, _, _, gq2 = dev.query_fused(m, q, gt, grad_vertices=gv2)
    torch.cuda.synchronize()
    dq64, dV64 = oracle.gradient(V, F, Q, t64, g)
    for name, a, b in (("backward dL/dq", to_np(gq), dq64), ("backward dL/dV", to_np(gv), dV64),
                       ("fused dL/dq", to_np(gq2), dq64), ("fused dL/dV", to_np(gv2), dV64)):
        e = rel_err(a, b)
        print(f"C3 {name}: norm-wise relative error {e:.3e}")
        assert e <= 1e-3, (name, e)
    # row by row against the FP64 gradient at the GPU's own triangles (at
    # shared edges and vertices those are equally correct)
    dq64g, dV64g = oracle.gradient(V, F, Q, t, g)
    rms = np.sqrt(np.mean(np.sum(dV64g ** 2, axis=1)))
    for a in (to_np(gv), to_np(gv2)):
        row = np.linalg.norm(a - dV64g, axis=1)
        assert np.all(row <= 1e-3 * np.maximum(np.linalg.norm(dV64g, axis=1), 1e-3 * rms))
    for a in (to_np(gq), to_np(gq2)):
        rowq = np.linalg.norm(a - dq64g, axis=1)
        assert np.all(rowq <= 1e-3 * np.maximum(np.linalg.norm(dq64g, axis=1), 1e-3))


def test_c3_full_size_invariants_and_fused(dev, c3):
    c, m = c3
    q = torch.from_numpy(c["Q"]).cuda()
    g = torch.from_numpy(c["G"]).cuda()
    d, t, cl = dev.query(m, q)
    gv = torch.zeros((len(m.V), 3), dtype=torch.float32, device="cuda")
    gq, gv = dev.query_backward(m, q, t, g, grad_vertices=gv)
    gv2 = torch.zeros_like(gv)
    d2, t2, cl2, gq2 = dev.query_fused(m, q, g, grad_vertices=gv2)
    torch.cuda.synchronize()
    assert torch.equal(d, d2) and torch.equal(t, t2) and torch.equal(cl, cl2)
    assert torch.equal(gq, gq2)
    assert rel_err(to_np(gv2), to_np(gv)) <= 1e-5          # atomics order only
    # without dL/dV (no LDS table, no barrier): the same outputs and dL/dq
    d3, t3, cl3, gq3 = dev.query_fused(m, q, g)
    torch.cuda.synchronize()
    assert torch.equal(d, d3) and torch.equal(t, t3) and torch.equal(cl, cl3)
    assert torch.equal(gq, gq3)
    dn, gqn, gn = to_np(d), to_np(gq), np.abs(c["G"])
    pos = dn > 1e-6
    assert np.allclose(np.linalg.norm(gqn[pos], axis=1), gn[pos], rtol=1e-5, atol=1e-6)   # |dd/dq| = 1
    # translating mesh and points together leaves d unchanged
    s = gqn.astype(np.float64).sum(0) + to_np(gv).astype(np.float64).sum(0)
    assert np.linalg.norm(s) <= 1e-4 * np.abs(gqn).sum()


def region_key(V, F, Q, tri):
    """Triangle and closest-point region (which barycentrics vanish)."""
    _, _, lam = oracle.distance_to_triangles(V, F, Q, tri)
    return tri.astype(np.int64) * 8 + ((lam > 1e-12) * np.array([1, 2, 4])).sum(1)


def fd_points(V, F, Q, h):
    """Central differences of the FP64 oracle distance at Q, per axis, and a
    mask of points where q and all q +- h e_k keep the same closest triangle
    and region: there d is one smooth formula (plane, line or point distance)
    and the central difference is accurate to O(h^2 / d^2).  Across a region
    boundary d is only C1 and the difference errs by O(h / d)."""
    d, t, _, _ = oracle.distance(V, F, Q, want_closest=False)
    key = region_key(V, F, Q, t)
    fd = np.zeros((len(Q), 3))
    ok = d >= 20 * h
    for k in range(3):
        e = np.zeros(3, np.float32)
        e[k] = h
        Qp, Qm = (Q + e).astype(np.float32), (Q - e).astype(np.float32)
        dp, tp, _, _ = oracle.distance(V, F, Qp, want_closest=False)
        dm, tm, _, _ = oracle.distance(V, F, Qm, want_closest=False)
        # the float32 step actually taken
        hs = Qp[:, k].astype(np.float64) - Qm[:, k].astype(np.float64)
        fd[:, k] = (dp - dm) / hs
        ok &= (region_key(V, F, Qp, tp) == key) & (region_key(V, F, Qm, tm) == key)
    return fd, ok


def test_fd_point_gradient(dev, c3):
    c, m = c3
    V, F = c["V"], c["F"]
    h = 1e-3
    # candidates at least 25 h from the surface (selection only: the finite
    # differences below come from the FP64 oracle)
    pool = c["Q"][-40000:]
    dpool, _, _ = dev.query(m, torch.from_numpy(pool).cuda())
    far = np.nonzero(to_np(dpool) >= 25 * h)[0][:6000]
    Q = pool[far]
    fd, ok = fd_points(V, F, Q, h)
    assert ok.sum() >= 1000
    sel = np.nonzero(ok)[0][:1000]
    _, _, _, gq, _ = gpu_grads(dev, m, Q[sel], np.ones(len(sel), np.float32))
    err = np.linalg.norm(gq - fd[sel], axis=1)
    assert np.all(err <= 1e-3), err.max()


def test_fd_vertex_gradient(dev):
    V, F = gen.displaced_icosphere(5, np.random.default_rng(21))
    m = dev.Mesh(V, F)
    D = float(np.linalg.norm(V.max(0) - V.min(0)))
    rng = np.random.default_rng(22)
    Q = gen.near_surface(rng, 3000, V, F, 0.02 * D)
    # moving a vertex rotates its triangles' planes, so d is curved in the
    # vertex position on the scale of an edge (0.04 here): a step of 2e-4
    # keeps the O(h^2) truncation error of the central difference below 1e-4
    h = 2e-4
    d64, t64, p64, _ = oracle.distance(V, F, Q)
    keep = d64 >= 100 * h
    Q = Q[keep][:1000]
    g = rng.normal(size=len(Q)).astype(np.float32)
    _, t, _, _, gv = gpu_grads(dev, m, Q, g)
    verts = np.unique(F[t])[:: max(1, len(np.unique(F[t])) // 12)][:12]
    base, tb, _, _ = oracle.distance(V, F, Q, want_closest=False)
    key = region_key(V, F, Q, tb)
    for v in verts:
        for k in range(3):
            Vp, Vm = V.copy(), V.copy()
            Vp[v, k] += h
            Vm[v, k] -= h
            dp, tp, _, _ = oracle.distance(Vp, F, Q, want_closest=False)
            dm, tm, _, _ = oracle.distance(Vm, F, Q, want_closest=False)
            # points whose closest triangle and region stay put (smooth d)
            smooth = (region_key(Vp, F, Q, tp) == key) & (region_key(Vm, F, Q, tm) == key)
            hs = (Vp[v, k].astype(np.float64) - V[v, k]) + (V[v, k] - Vm[v, k].astype(np.float64))
            fd = np.sum((g * (dp - dm))[smooth]) / hs
            # the GPU gradient restricted to the same smooth points
            gsel = np.where(smooth, g, 0.0).astype(np.float32)
            _, _, _, _, gvs = gpu_grads(dev, m, Q, gsel)
            assert abs(gvs[v, k] - fd) <= 1e-3 * max(1.0, abs(fd)), (v, k, gvs[v, k], fd)


def test_autograd_matches_kernels(dev):
    V, F = gen.displaced_icosphere(4, np.random.default_rng(23))
    Vt = torch.from_numpy(V).cuda().requires_grad_(True)
    m = dev.Mesh(Vt, torch.from_numpy(F))
    rng = np.random.default_rng(24)
    Q = gen.near_surface(rng, 5000, V, F, 0.05)
    q = torch.from_numpy(Q).cuda().requires_grad_(True)
    g = torch.from_numpy(rng.normal(size=len(Q)).astype(np.float32)).cuda()
    d, t, cl = dev.distance(m, q)
    assert not t.requires_grad and not cl.requires_grad
    (d * g).sum().backward()
    gv = torch.zeros_like(Vt)
    gq, gv = dev.query_backward(m, q.detach(), t, g, grad_vertices=gv)
    torch.cuda.synchronize()
    assert torch.equal(q.grad, gq)
    assert rel_err(to_np(Vt.grad), to_np(gv)) <= 1e-5


def test_backward_ordered_equals_backward(dev, c3):
    """p2m_query_backward_ordered with the forward's visiting order (the
    points sorted once) gives the same dL/dq and, up to the order of float32
    additions, the same dL/dV as p2m_query_backward; so does the input order
    (order None)."""
    c, m = c3
    q = torch.from_numpy(c["Q"][:500000]).cuda()
    g = torch.from_numpy(c["G"][:500000]).cuda()
    order = dev.sort_points(m, q)
    d, t, cl = dev.query_ordered(m, q, order)
    d0, t0, cl0 = dev.query(m, q)
    assert torch.equal(d, d0) and torch.equal(t, t0)
    gv0 = torch.zeros((len(m.V), 3), device="cuda")
    gq0, gv0 = dev.query_backward(m, q, t, g, grad_vertices=gv0)
    for o in (order, None):
        gv1 = torch.zeros_like(gv0)
        gq1, gv1 = dev.query_backward(m, q, t, g, grad_vertices=gv1, order=o)
        torch.cuda.synchronize()
        assert torch.equal(gq1, gq0)
        assert rel_err(to_np(gv1), to_np(gv0)) <= 1e-5


def test_backward_table_flushes(dev, c3):
    """At 4M points a backward workgroup runs over several tiles with one LDS
    table of vertex gradients.  In input order (random in space) the table
    fills within a tile or two and is flushed and cleared between tiles;
    sorted, it is flushed at the end.  Both give the same dL/dV up to the
    order of float32 additions, and dL/dq bit for bit."""
    c, m = c3
    q = torch.from_numpy(c["Q"]).cuda()
    g = torch.from_numpy(c["G"]).cuda()
    order = dev.sort_points(m, q)
    d, t, cl = dev.query_ordered(m, q, order)
    ident = torch.arange(len(q), dtype=torch.int32, device="cuda")
    gv0 = torch.zeros((len(m.V), 3), device="cuda")
    gq0, gv0 = dev.query_backward(m, q, t, g, grad_vertices=gv0, order=order)
    gv1 = torch.zeros_like(gv0)
    gq1, gv1 = dev.query_backward(m, q, t, g, grad_vertices=gv1, order=ident)
    torch.cuda.synchronize()
    assert torch.equal(gq1, gq0)
    assert rel_err(to_np(gv1), to_np(gv0)) <= 1e-5
    # translating mesh and points together leaves d unchanged
    for gv in (gv0, gv1):
        s = to_np(gq0).astype(np.float64).sum(0) + to_np(gv).astype(np.float64).sum(0)
        assert np.linalg.norm(s) <= 1e-4 * np.abs(to_np(gq0)).sum()


def test_fused_block_sizes(dev, c3):
    """The fused kernel's LDS holds the regroup area and, with dL/dV, the
    vertex-gradient table (shrunk to fit 64 KB at 1,024 threads): every
    workgroup size gives the same outputs and dL/dq bit for bit, and dL/dV up
    to the order of float32 additions."""
    c, m = c3
    q = torch.from_numpy(c["Q"][:200000]).cuda()
    g = torch.from_numpy(c["G"][:200000]).cuda()
    outs = {}
    for bs in (256, 64, 1024):
        m.set_query_config(block_size=bs)
        gv = torch.zeros((len(m.V), 3), device="cuda")
        d, t, cl, gq = dev.query_fused(m, q, g, grad_vertices=gv)
        torch.cuda.synchronize()
        outs[bs] = (d, t, cl, gq, gv)
    m.set_query_config(block_size=256)
    ref = outs[256]
    for bs in (64, 1024):
        for a, b in zip(ref[:4], outs[bs][:4]):
            assert torch.equal(a, b), bs
        assert rel_err(to_np(outs[bs][4]), to_np(ref[4])) <= 1e-5, bs
