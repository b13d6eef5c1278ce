// C ABI of the library (declared in include/p2m.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <list>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "device.h"
#include "host/build.h"
#include "p2m.h"

namespace {

thread_local std::string g_last_error;

int32_t fail(int32_t code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

int32_t hip_fail(hipError_t e, const char* what)
{
    return fail(P2M_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Makes `dev` current for the scope and restores the caller's device.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

// Scratch memory of the calls made on one stream: the query sort's
// workspace, and the distances and reduction partials of the point-set
// reduction.  Each stream that queries a handle gets its own, so that calls
// on different streams never share memory; a buffer is regrown only after
// its own stream has finished with it.
struct StreamScratch {
    hipStream_t stream = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    void* gws = nullptr;  // the grouped search's locate keys and site sort
    size_t gws_bytes = 0;
    void* rws = nullptr;
    size_t rws_bytes = 0;
    double* pair = nullptr;  // mesh distances: the two one-sided reductions (10 doubles)
};

struct p2m_handle_ {
    p2m::HostStructure H;
    int device = -1;
    p2m::DevMesh dm{};
    std::vector<void*> allocs;
    int64_t device_bytes = 0;
    p2m_query_config cfg{256, 1, 1, 0, 0, 2};
    // the caller's referenced vertices (index order), for mesh distances
    const float* ref_v = nullptr;
    int64_t n_ref = 0;
    std::recursive_mutex mu;  // guards `scratch` and the enqueues that use it
    std::list<StreamScratch> scratch;  // a list: references stay valid as streams are added

    ~p2m_handle_()
    {
        if (device >= 0) {
            DeviceGuard g(device);
            for (void* p : allocs) (void)hipFree(p);
            for (StreamScratch& sc : scratch) {
                if (sc.ws) (void)hipFree(sc.ws);
                if (sc.gws) (void)hipFree(sc.gws);
                if (sc.rws) (void)hipFree(sc.rws);
                if (sc.pair) (void)hipFree(sc.pair);
            }
        }
    }

    template <typename T>
    const T* upload(const void* src, size_t bytes)
    {
        void* p = nullptr;
        const size_t nb = bytes ? bytes : 16;
        hipError_t e = hipMalloc(&p, nb);
        if (e != hipSuccess) throw p2m::Error(P2M_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
        allocs.push_back(p);
        device_bytes += (int64_t)nb;
        if (bytes) {
            e = hipMemcpy(p, src, bytes, hipMemcpyHostToDevice);
            if (e != hipSuccess) throw p2m::Error(P2M_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
        }
        return (const T*)p;
    }

    void upload_all(const p2m_mesh_desc& mesh)
    {
        using namespace p2m;
        const HostStructure& h = H;
        static_assert(sizeof(SiteRec) == 32 && sizeof(ListRec) == 64, "device record layout");
        dm.site_rec = upload<float4>(h.site_rec.data(), h.site_rec.size() * sizeof(SiteRec));
        dm.adj = upload<float4>(h.adj.data(), h.adj.size() * 4);
        // list entries split into a dense sphere array (what the scan reads
        // for every entry) and the records at the same index
        {
            const size_t ne = h.list_rec.size();
            std::vector<float> sph(4 * ne), rec(12 * ne);
            for (size_t k = 0; k < ne; ++k) {
                const ListRec& L = h.list_rec[k];
                std::memcpy(&sph[4 * k], &L.cx, 16);
                std::memcpy(&rec[12 * k], &L.ax, 48);
            }
            dm.list_sph = upload<float4>(sph.data(), sph.size() * 4);
            dm.list_rec = upload<float4>(rec.data(), rec.size() * 4);
        }
        dm.tri_rec = upload<float4>(h.tri_rec.data(), h.tri_rec.size() * 4);
        dm.tri_user = upload<int32_t>(h.tri_user.data(), h.tri_user.size() * 4);
        dm.tri_vid = upload<int4>(h.tri_vid.data(), h.tri_vid.size() * 4);
        {
            std::vector<float> v4(4 * (size_t)mesh.n_vertices, 0.f);
            for (int64_t v = 0; v < mesh.n_vertices; ++v) std::memcpy(&v4[4 * v], mesh.vertices + 3 * v, 12);
            dm.verts = upload<float4>(v4.data(), v4.size() * 4);
        }
        std::vector<int32_t> slot(h.n_triangles);
        for (int64_t i = 0; i < h.n_triangles; ++i) slot[h.tri_user[i]] = (int32_t)i;
        dm.tri_slot = upload<int32_t>(slot.data(), slot.size() * 4);
        dm.seed = upload<int32_t>(h.seed.data(), h.seed.size() * 4);
        dm.bvh = upload<float4>(h.bvh.data(), h.bvh.size() * 4);
        dm.oct = h.oct.empty() ? nullptr : upload<int32_t>(h.oct.data(), h.oct.size() * 4);
        for (int k = 0; k < 4; ++k) dm.oroot[k] = h.oroot[k];
        for (int k = 0; k < 3; ++k) {
            dm.gdim[k] = h.gdim[k];
            dm.gorg[k] = h.gorg[k];
            dm.dlo[k] = h.dlo[k];
            dm.dhi[k] = h.dhi[k];
        }
        dm.ginv = 1.0f / h.gcell;
        dm.n_sites = h.n_sites;
        dm.n_tris = (int32_t)h.n_triangles;
        dm.n_vertices = (int32_t)h.n_vertices;
        // referenced vertices in index order (the default point set of a
        // mesh-to-mesh distance)
        std::vector<char> used((size_t)mesh.n_vertices, 0);
        for (int64_t k = 0; k < 3 * mesh.n_triangles; ++k) used[mesh.triangles[k]] = 1;
        std::vector<float> rv;
        for (int64_t v = 0; v < mesh.n_vertices; ++v)
            if (used[v]) rv.insert(rv.end(), mesh.vertices + 3 * v, mesh.vertices + 3 * v + 3);
        n_ref = (int64_t)rv.size() / 3;
        ref_v = upload<float>(rv.data(), rv.size() * 4);
    }

    // This stream's scratch (created on first use); the caller holds mu.
    StreamScratch& scratch_for(hipStream_t st)
    {
        for (StreamScratch& sc : scratch)
            if (sc.stream == st) return sc;
        scratch.push_back(StreamScratch{});
        scratch.back().stream = st;
        return scratch.back();
    }

    // Grows one scratch buffer of `st` to at least `bytes`; waits for earlier
    // work on `st` first (the only stream that used it).  The caller holds mu.
    int32_t grow(void*& buf, size_t& have, size_t bytes, hipStream_t st)
    {
        if (have >= bytes) return P2M_OK;
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        if (buf) (void)hipFree(buf);
        buf = nullptr;
        have = 0;
        const size_t nb = bytes + bytes / 4;
        e = hipMalloc(&buf, nb);
        if (e != hipSuccess) return fail(P2M_ERR_OOM, std::string("workspace hipMalloc: ") + hipGetErrorString(e));
        have = nb;
        return P2M_OK;
    }

    // The sort workspace of `st`, at least `bytes` (caller holds mu).
    int32_t ensure_ws(size_t bytes, hipStream_t st, void** out)
    {
        StreamScratch& sc = scratch_for(st);
        const int32_t rc = grow(sc.ws, sc.ws_bytes, bytes, st);
        *out = sc.ws;
        return rc;
    }

    // The point-set reduction buffer of `st`, at least `bytes` (caller holds mu).
    // The grouped search's workspace of `st`, at least `bytes` (caller holds mu).
    int32_t ensure_gws(size_t bytes, hipStream_t st, void** out)
    {
        StreamScratch& sc = scratch_for(st);
        const int32_t rc = grow(sc.gws, sc.gws_bytes, bytes, st);
        *out = sc.gws;
        return rc;
    }

    // Whether a non-instrumented search of n points runs as the grouped
    // passes (locate, sort by site, shared list scans): config group = 1,
    // or automatic (2) for a forward or fused call of at least 2M points.
    // The grouped passes cost a few hundred microseconds more in fixed
    // work and win on large sets: forwards measured 2.53 against 3.03 ms
    // on 10M points of the 327k-triangle mesh, 1.01 against 1.07 on its 4M
    // near-surface points, 3.26 against 3.60 on C1's 2M, but 0.87 against
    // 0.73 on 1M points of the same mesh and 0.54 against 0.38 on 10k;
    // fused calls 2.87 against 3.61 ms on the 10M points, 1.18 against
    // 1.30 on the 4M, 3.32 against 3.75 on C1, 0.92 against 0.85 on 1M.
    bool grouped(int64_t n) const
    {
        if (cfg.group == 0) return false;
        if (cfg.group == 1) return true;
        return n >= 2000000;
    }

    // The search of `a` (sorted or not): the grouped passes or the one-pass
    // kernel.  The caller holds mu.
    int32_t search(const p2m::FwdArgs& a, bool fused, hipStream_t st)
    {
        if (grouped(a.n)) {
            void* gw = nullptr;
            const int32_t rc = ensure_gws(p2m::grouped_workspace_bytes(a.n, dm.n_sites), st, &gw);
            if (rc != P2M_OK) return rc;
            const hipError_t e = p2m::launch_grouped(dm, a, gw, fused, st);
            if (e != hipSuccess) return hip_fail(e, "grouped search launch");
            return P2M_OK;
        }
        const hipError_t e = p2m::launch_forward(dm, a, cfg.block_size, fused, false, st);
        if (e != hipSuccess) return hip_fail(e, "forward launch");
        return P2M_OK;
    }

    int32_t ensure_rws(size_t bytes, hipStream_t st, void** out)
    {
        StreamScratch& sc = scratch_for(st);
        const int32_t rc = grow(sc.rws, sc.rws_bytes, bytes, st);
        *out = sc.rws;
        return rc;
    }
};

namespace p2m {
const DevMesh& handle_devmesh(const p2m_handle_* h) { return h->dm; }
int handle_device(const p2m_handle_* h) { return h->device; }
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace p2m

extern "C" {

void p2m_default_opts(p2m_build_opts* o)
{
    if (!o) return;
    o->domain_scale = 10.0f;
    o->augment = 1;
    o->tau_scale = 2.0f;
    o->dense_min_sites = 256;
    o->dense_rel = 8.0f;
    o->ring_sites = 12;
    o->ring_layers = 8;
    o->aux_list_mode = 1;
    o->gpu_lists = 1;
    o->gpu_voronoi = 1;
    o->gpu_cell_pass = 0;
    o->decomposition = 0;
    o->octree_max_list = 64;
    o->octree_max_depth = 12;
    o->list_inflation_rel = 1e-7f;
    o->seed_cell_scale = 2.0f;
    o->seed_max_cells = 16 << 20;
    o->n_threads = 0;
    o->device = -2;
}

int32_t p2m_build(const p2m_mesh_desc* mesh, const p2m_build_opts* opts, p2m_handle* out)
{
    if (!mesh || !out) return fail(P2M_ERR_INVALID_ARG, "null mesh or output pointer");
    *out = nullptr;
    p2m_build_opts o;
    p2m_default_opts(&o);
    if (opts) o = *opts;
    p2m_handle h = nullptr;
    try {
        h = new p2m_handle_();
        int dev = o.device;
        if (dev == -2) {
            hipError_t e = hipGetDevice(&dev);
            if (e != hipSuccess) {
                delete h;
                return hip_fail(e, "hipGetDevice");
            }
        }
        if (dev >= 0) {
            DeviceGuard g(dev);
            if (!g.ok) {
                delete h;
                return fail(P2M_ERR_HIP, "cannot select HIP device " + std::to_string(dev));
            }
            const p2m::GpuListFn on_device = p2m::gpu_build_lists;
            const p2m::CheckFn checks_on_device = p2m::gpu_corner_checks;
            const p2m::CellFn cells_on_device = p2m::gpu_cells;
            p2m::build_host(*mesh, o, h->H, o.gpu_lists ? &on_device : nullptr,
                            o.gpu_voronoi ? &checks_on_device : nullptr,
                            o.gpu_voronoi == 1 ? &cells_on_device : nullptr);
            h->device = dev;
            h->upload_all(*mesh);
        } else {
            p2m::build_host(*mesh, o, h->H);
        }
        h->H.stats.device_bytes = h->device_bytes;
        // The host keeps only the triangle id of each list entry (for the
        // inspection calls); the full 64 B records live on the device.
        h->H.list_tri.resize(h->H.list_rec.size());
        for (size_t k = 0; k < h->H.list_rec.size(); ++k) h->H.list_tri[k] = h->H.list_rec[k].tri;
        std::vector<p2m::ListRec>().swap(h->H.list_rec);
    } catch (const p2m::Error& e) {
        delete h;
        return fail(e.code, e.what());
    } catch (const std::bad_alloc&) {
        delete h;
        return fail(P2M_ERR_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        delete h;
        return fail(P2M_ERR_INTERNAL, e.what());
    }
    *out = h;
    return P2M_OK;
}

int32_t p2m_destroy(p2m_handle h)
{
    delete h;
    return P2M_OK;
}

int32_t p2m_get_stats(p2m_handle h, p2m_stats* out)
{
    if (!h || !out) return fail(P2M_ERR_INVALID_ARG, "null handle or output");
    *out = h->H.stats;
    return P2M_OK;
}

int32_t p2m_get_query_config(p2m_handle h, p2m_query_config* out)
{
    if (!h || !out) return fail(P2M_ERR_INVALID_ARG, "null handle or output");
    *out = h->cfg;
    return P2M_OK;
}

int32_t p2m_set_query_config(p2m_handle h, const p2m_query_config* c)
{
    if (!h || !c) return fail(P2M_ERR_INVALID_ARG, "null handle or config");
    if (c->block_size < 64 || c->block_size > 1024 || c->block_size % 64 != 0)
        return fail(P2M_ERR_INVALID_ARG, "block_size must be a multiple of 64 in [64, 1024]");
    if (c->xcd_groups < 1 || c->xcd_groups > 64)
        return fail(P2M_ERR_INVALID_ARG, "xcd_groups must be in [1, 64]");
    if (c->sort_bits < 0 || c->sort_bits > 8)
        return fail(P2M_ERR_INVALID_ARG, "sort_bits must be in [0, 8]");
    if (c->stage != 0 && c->stage != 1) return fail(P2M_ERR_INVALID_ARG, "stage must be 0 or 1");
    if (c->group < 0 || c->group > 2) return fail(P2M_ERR_INVALID_ARG, "group must be 0, 1 or 2");
    h->cfg = *c;
    return P2M_OK;
}

static int32_t query_common(p2m_handle h, const float* q, int64_t n, float* dist, int32_t* tri, float* closest,
                            const float* g, float* gq, float* gv, unsigned long long* ctr, bool fused,
                            void* stream, const p2m::Touch* touch = nullptr)
{
    if (!h) return fail(P2M_ERR_INVALID_ARG, "null handle");
    if (n < 0) return fail(P2M_ERR_INVALID_ARG, "negative point count");
    if (h->device < 0) return fail(P2M_ERR_NO_DEVICE, "handle was built host-only");
    if (n == 0) return P2M_OK;
    if (!q || !dist) return fail(P2M_ERR_INVALID_ARG, "null points or distance output");
    if (fused && !g) return fail(P2M_ERR_INVALID_ARG, "null upstream gradient");
    if (n > 0x7fffffffLL) return fail(P2M_ERR_INVALID_ARG, "more than 2^31-1 points per call");
    DeviceGuard dg(h->device);
    hipStream_t st = (hipStream_t)stream;
    p2m::FwdArgs a{};
    a.q = q;
    a.n = n;
    a.dist = dist;
    a.tri = tri;
    a.closest = closest;
    a.grad_dist = g;
    a.grad_q = gq;
    a.grad_v = gv;
    a.ctr = ctr;
    if (touch) a.touch = *touch;
    a.xcds = h->cfg.xcd_groups;
    a.stage = h->cfg.stage;
    std::lock_guard<std::recursive_mutex> lk(h->mu);
    if (h->cfg.reorder) {
        // The search gathers each point through the order: measured faster
        // than having the sort also write the points in visiting order.
        void* ws = nullptr;
        int32_t rc = h->ensure_ws(p2m::reorder_workspace_bytes(n, h->cfg.sort_bits), st, &ws);
        if (rc != P2M_OK) return rc;
        hipError_t e = p2m::launch_reorder(h->dm, q, n, h->cfg.sort_bits, ws, &a.perm, st);
        if (e != hipSuccess) return hip_fail(e, "reorder launch");
    }
    if (!ctr) return h->search(a, fused, st);
    hipError_t e = p2m::launch_forward(h->dm, a, h->cfg.block_size, fused, true, st);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return P2M_OK;
}

int32_t p2m_query(p2m_handle h, const float* d_points, int64_t n, float* d_out_dist, int32_t* d_out_tri,
                  float* d_out_closest, void* stream)
{
    return query_common(h, d_points, n, d_out_dist, d_out_tri, d_out_closest, nullptr, nullptr, nullptr,
                        nullptr, false, stream);
}

// ------------------------------------------------------- no-allocation query
// Scratch of p2m_query_noalloc: the query sort's workspace, in a device
// array of the library rather than in memory allocated per call.  Each GPU
// the library runs on holds its own copy until the process ends.  Host code
// never uses the array's name as an address: its device address is looked
// up once per device (hipGetSymbolAddress, with that device current) and
// kept in g_scratch_ptr.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device ordinal; null until looked up

// The scratch array's address on `dev`, which must be the current device.
int32_t scratch_address(int dev, void** out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(P2M_ERR_HIP, "hipGetSymbolAddress(scratch) returned no address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return P2M_OK;
}
}  // namespace

int32_t p2m_query_noalloc(p2m_handle h, const float* d_points, int64_t n, float* d_out_dist, int32_t* d_out_tri,
                          float* d_out_closest, void* stream)
{
    if (!h) return fail(P2M_ERR_INVALID_ARG, "null handle");
    if (n < 0) return fail(P2M_ERR_INVALID_ARG, "negative point count");
    if (h->device < 0) return fail(P2M_ERR_NO_DEVICE, "handle was built host-only");
    if (n == 0) return P2M_OK;
    if (!d_points || !d_out_dist) return fail(P2M_ERR_INVALID_ARG, "null points or distance output");
    const size_t need = h->cfg.reorder ? p2m::reorder_workspace_bytes(n, h->cfg.sort_bits) : 0;
    if (n > 0x7fffffffLL || need > kNoAllocScratchBytes)
        return fail(P2M_ERR_INVALID_ARG, "p2m_query_noalloc: " + std::to_string(n) + " points need " +
                                             std::to_string(need) + " bytes of sort workspace; its scratch holds " +
                                             std::to_string(kNoAllocScratchBytes) + " (use p2m_query)");
    DeviceGuard dg(h->device);
    if (!dg.ok) return fail(P2M_ERR_HIP, "cannot select the handle's HIP device");
    hipStream_t st = (hipStream_t)stream;
    p2m::FwdArgs a{};
    a.q = d_points;
    a.n = n;
    a.dist = d_out_dist;
    a.tri = d_out_tri;
    a.closest = d_out_closest;
    a.xcds = h->cfg.xcd_groups;
    a.stage = h->cfg.stage;
    if (h->cfg.reorder) {
        void* ws = nullptr;
        const int32_t rc = scratch_address(h->device, &ws);
        if (rc != P2M_OK) return rc;
        const hipError_t e = p2m::launch_reorder(h->dm, d_points, n, h->cfg.sort_bits, ws, &a.perm, st);
        if (e != hipSuccess) return hip_fail(e, "reorder launch");
    }
    const hipError_t e = p2m::launch_forward(h->dm, a, h->cfg.block_size, false, false, st);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return P2M_OK;
}

int32_t p2m_point_set_distance(p2m_handle h, const float* d_points, int64_t n, double* d_out, void* stream)
{
    if (!h) return fail(P2M_ERR_INVALID_ARG, "null handle");
    if (n < 0) return fail(P2M_ERR_INVALID_ARG, "negative point count");
    if (h->device < 0) return fail(P2M_ERR_NO_DEVICE, "handle was built host-only");
    if (!d_out || (n > 0 && !d_points)) return fail(P2M_ERR_INVALID_ARG, "null points or output");
    if (n > 0x7fffffffLL) return fail(P2M_ERR_INVALID_ARG, "more than 2^31-1 points per call");
    DeviceGuard dg(h->device);
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::recursive_mutex> lk(h->mu);
    const size_t dist_bytes = ((size_t)n * sizeof(float) + 255) & ~(size_t)255;
    const size_t need = dist_bytes + 5 * sizeof(double) * (size_t)p2m::reduce_blocks(n);
    void* rws = nullptr;
    int32_t rc = h->ensure_rws(need, st, &rws);
    if (rc != P2M_OK) return rc;
    float* dist = (float*)rws;
    double* part = (double*)((char*)rws + dist_bytes);
    if (n > 0) {
        rc = query_common(h, d_points, n, dist, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, false, stream);
        if (rc != P2M_OK) return rc;
    }
    const hipError_t e = p2m::launch_reduce_dist(dist, n, part, d_out, st);
    if (e != hipSuccess) return hip_fail(e, "reduction launch");
    return P2M_OK;
}

int32_t p2m_mesh_distance(p2m_handle a, p2m_handle b, const float* d_points_a, int64_t n_a,
                          const float* d_points_b, int64_t n_b, double* d_out, void* stream)
{
    if (!a || !b) return fail(P2M_ERR_INVALID_ARG, "null handle");
    if (a->device < 0 || b->device < 0) return fail(P2M_ERR_NO_DEVICE, "handle was built host-only");
    if (a->device != b->device) return fail(P2M_ERR_INVALID_ARG, "handles on different devices");
    if (!d_out) return fail(P2M_ERR_INVALID_ARG, "null output");
    if ((d_points_a && n_a < 0) || (d_points_b && n_b < 0)) return fail(P2M_ERR_INVALID_ARG, "negative point count");
    if ((!d_points_a && n_a != 0) || (!d_points_b && n_b != 0))
        return fail(P2M_ERR_INVALID_ARG, "a point count without points (pass 0 with NULL for the vertices)");
    const float* pa = d_points_a ? d_points_a : a->ref_v;
    const int64_t na = d_points_a ? n_a : a->n_ref;
    const float* pb = d_points_b ? d_points_b : b->ref_v;
    const int64_t nb = d_points_b ? n_b : b->n_ref;
    DeviceGuard dg(a->device);
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::recursive_mutex> lk(a->mu);
    // the two one-sided reductions (5 doubles each), in a's scratch of this
    // stream
    StreamScratch& sc = a->scratch_for(st);
    if (!sc.pair) {
        const hipError_t e = hipMalloc(&sc.pair, 10 * sizeof(double));
        if (e != hipSuccess) {
            sc.pair = nullptr;
            return fail(P2M_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
    }
    double* pair = sc.pair;
    int32_t rc = p2m_point_set_distance(b, pa, na, pair, stream);      // A's points against mesh B
    if (rc != P2M_OK) return rc;
    rc = p2m_point_set_distance(a, pb, nb, pair + 5, stream);  // B's points against mesh A
    if (rc != P2M_OK) return rc;
    const hipError_t e = p2m::launch_mesh_distance_combine(pair, pair + 5, d_out, st);
    if (e != hipSuccess) return hip_fail(e, "combine launch");
    return P2M_OK;
}

int32_t p2m_sort_points(p2m_handle h, const float* d_points, int64_t n, int32_t* d_order,
                        float* d_sorted_points, void* stream)
{
    if (!h) return fail(P2M_ERR_INVALID_ARG, "null handle");
    if (n < 0) return fail(P2M_ERR_INVALID_ARG, "negative point count");
    if (h->device < 0) return fail(P2M_ERR_NO_DEVICE, "handle was built host-only");
    if (n == 0) return P2M_OK;
    if (!d_points || !d_order) return fail(P2M_ERR_INVALID_ARG, "null points or order");
    if (n > 0x7fffffffLL) return fail(P2M_ERR_INVALID_ARG, "more than 2^31-1 points per call");
    DeviceGuard dg(h->device);
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::recursive_mutex> lk(h->mu);
    void* ws = nullptr;
    int32_t rc = h->ensure_ws(p2m::reorder_workspace_bytes(n, h->cfg.sort_bits), st, &ws);
    if (rc != P2M_OK) return rc;
    const int32_t* perm = nullptr;
    hipError_t e = p2m::launch_reorder(h->dm, d_points, n, h->cfg.sort_bits, ws, &perm, st, d_sorted_points);
    if (e == hipSuccess) e = hipMemcpyAsync(d_order, perm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "sort launch");
    return P2M_OK;
}

int32_t p2m_query_ordered(p2m_handle h, const float* d_points, const int32_t* d_order, int64_t n,
                          float* d_out_dist, int32_t* d_out_tri, float* d_out_closest, void* stream)
{
    if (!h) return fail(P2M_ERR_INVALID_ARG, "null handle");
    if (n < 0) return fail(P2M_ERR_INVALID_ARG, "negative point count");
    if (h->device < 0) return fail(P2M_ERR_NO_DEVICE, "handle was built host-only");
    if (n == 0) return P2M_OK;
    if (!d_points || !d_out_dist) return fail(P2M_ERR_INVALID_ARG, "null points or distance output");
    if (n > 0x7fffffffLL) return fail(P2M_ERR_INVALID_ARG, "more than 2^31-1 points per call");
    DeviceGuard dg(h->device);
    p2m::FwdArgs a{};
    a.q = d_points;
    a.perm = d_order;
    a.n = n;
    a.dist = d_out_dist;
    a.tri = d_out_tri;
    a.closest = d_out_closest;
    a.xcds = h->cfg.xcd_groups;
    a.stage = h->cfg.stage;
    std::lock_guard<std::recursive_mutex> lk(h->mu);
    return h->search(a, false, (hipStream_t)stream);
}

int32_t p2m_query_sorted(p2m_handle h, const float* d_sorted_points, const int32_t* d_order, int64_t n,
                         float* d_out_dist, int32_t* d_out_tri, float* d_out_closest, void* stream)
{
    if (!h) return fail(P2M_ERR_INVALID_ARG, "null handle");
    if (n < 0) return fail(P2M_ERR_INVALID_ARG, "negative point count");
    if (h->device < 0) return fail(P2M_ERR_NO_DEVICE, "handle was built host-only");
    if (n == 0) return P2M_OK;
    if (!d_sorted_points || !d_out_dist) return fail(P2M_ERR_INVALID_ARG, "null points or distance output");
    if (n > 0x7fffffffLL) return fail(P2M_ERR_INVALID_ARG, "more than 2^31-1 points per call");
    DeviceGuard dg(h->device);
    p2m::FwdArgs a{};
    a.q = d_sorted_points;
    a.q_sorted = 1;
    a.perm = d_order;
    a.n = n;
    a.dist = d_out_dist;
    a.tri = d_out_tri;
    a.closest = d_out_closest;
    a.xcds = h->cfg.xcd_groups;
    a.stage = h->cfg.stage;
    std::lock_guard<std::recursive_mutex> lk(h->mu);
    return h->search(a, false, (hipStream_t)stream);
}

int32_t p2m_query_counters(p2m_handle h, const float* d_points, int64_t n, float* d_out_dist,
                           int32_t* d_out_tri, float* d_out_closest, unsigned long long* d_counters,
                           void* stream)
{
    if (!d_counters) return fail(P2M_ERR_INVALID_ARG, "null counters");
    return query_common(h, d_points, n, d_out_dist, d_out_tri, d_out_closest, nullptr, nullptr, nullptr,
                        d_counters, false, stream);
}

int32_t p2m_query_touched(p2m_handle h, const float* d_points, int64_t n, float* d_out_dist,
                          int32_t* d_out_tri, float* d_out_closest, unsigned long long* d_counters,
                          int64_t* h_items, void* stream)
{
    if (!d_counters || !h_items) return fail(P2M_ERR_INVALID_ARG, "null counters or item counts");
    if (!h) return fail(P2M_ERR_INVALID_ARG, "null handle");
    if (h->device < 0) return fail(P2M_ERR_NO_DEVICE, "handle was built host-only");
    DeviceGuard dg(h->device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t sizes[7] = {(int64_t)h->H.site_rec.size(), (int64_t)h->H.adj.size() / 4,
                              (int64_t)h->H.list_tri.size(), (int64_t)h->H.list_tri.size(),
                              (int64_t)h->H.seed.size(), (int64_t)h->H.n_triangles,
                              (int64_t)h->H.bvh.size() / 8};
    int64_t total = 0;
    for (int64_t k : sizes) total += (k + 3) / 4 * 4;
    void* flags = nullptr;
    hipError_t e = hipMalloc(&flags, (size_t)std::max<int64_t>(total, 4));
    if (e != hipSuccess) return fail(P2M_ERR_OOM, std::string("flag hipMalloc: ") + hipGetErrorString(e));
    e = p2m::launch_fill_u32((uint32_t*)flags, 0u, total / 4, st);
    p2m::Touch t{};
    uint8_t* ptr[7];
    {
        uint8_t* p = (uint8_t*)flags;
        for (int k = 0; k < 7; ++k) {
            ptr[k] = p;
            p += (sizes[k] + 3) / 4 * 4;
        }
    }
    t.site = ptr[0];
    t.adj = ptr[1];
    t.sph = ptr[2];
    t.rec = ptr[3];
    t.seed = ptr[4];
    t.tri = ptr[5];
    t.bvh = ptr[6];
    int32_t rc = P2M_OK;
    if (e != hipSuccess) rc = hip_fail(e, "flag clear");
    if (rc == P2M_OK)
        rc = query_common(h, d_points, n, d_out_dist, d_out_tri, d_out_closest, nullptr, nullptr, nullptr,
                          d_counters, false, stream, &t);
    std::vector<uint8_t> host((size_t)std::max<int64_t>(total, 4));
    if (rc == P2M_OK) {
        e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = hipMemcpy(host.data(), flags, (size_t)total, hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = hip_fail(e, "flag copy");
    }
    (void)hipFree(flags);
    if (rc != P2M_OK) return rc;
    size_t off = 0;
    for (int k = 0; k < 7; ++k) {
        int64_t c = 0;
        for (int64_t i = 0; i < sizes[k]; ++i) c += host[off + (size_t)i] != 0;
        h_items[k] = c;
        off += (size_t)((sizes[k] + 3) / 4 * 4);
    }
    return P2M_OK;
}

int32_t p2m_query_fused(p2m_handle h, const float* d_points, int64_t n, const float* d_grad_dist,
                        float* d_out_dist, int32_t* d_out_tri, float* d_out_closest, float* d_grad_points,
                        float* d_grad_vertices, void* stream)
{
    return query_common(h, d_points, n, d_out_dist, d_out_tri, d_out_closest, d_grad_dist, d_grad_points,
                        d_grad_vertices, nullptr, true, stream);
}

int32_t p2m_query_backward(p2m_handle h, const float* d_points, int64_t n, const int32_t* d_tri,
                           const float* d_grad_dist, float* d_grad_points, float* d_grad_vertices, void* stream)
{
    if (!h) return fail(P2M_ERR_INVALID_ARG, "null handle");
    if (n < 0) return fail(P2M_ERR_INVALID_ARG, "negative point count");
    if (h->device < 0) return fail(P2M_ERR_NO_DEVICE, "handle was built host-only");
    if (n == 0) return P2M_OK;
    if (!d_points || !d_tri || !d_grad_dist) return fail(P2M_ERR_INVALID_ARG, "null points, triangles or gradient");
    if (n > 0x7fffffffLL) return fail(P2M_ERR_INVALID_ARG, "more than 2^31-1 points per call");
    DeviceGuard dg(h->device);
    hipStream_t st = (hipStream_t)stream;
    // Visiting the points in spatial order lets a workgroup combine the
    // vertex gradients of neighbouring points before the global atomics.
    const int32_t* order = nullptr;
    std::lock_guard<std::recursive_mutex> lk(h->mu);
    if (h->cfg.reorder && d_grad_vertices) {
        void* ws = nullptr;
        int32_t rc = h->ensure_ws(p2m::reorder_workspace_bytes(n, h->cfg.sort_bits), st, &ws);
        if (rc != P2M_OK) return rc;
        hipError_t e = p2m::launch_reorder(h->dm, d_points, n, h->cfg.sort_bits, ws, &order, st);
        if (e != hipSuccess) return hip_fail(e, "reorder launch");
    }
    hipError_t e = p2m::launch_backward(h->dm, d_points, n, order, d_tri, d_grad_dist, d_grad_points,
                                        d_grad_vertices, h->cfg.block_size, st);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return P2M_OK;
}

int32_t p2m_query_backward_ordered(p2m_handle h, const float* d_points, const int32_t* d_order, int64_t n,
                                   const int32_t* d_tri, const float* d_grad_dist, float* d_grad_points,
                                   float* d_grad_vertices, void* stream)
{
    if (!h) return fail(P2M_ERR_INVALID_ARG, "null handle");
    if (n < 0) return fail(P2M_ERR_INVALID_ARG, "negative point count");
    if (h->device < 0) return fail(P2M_ERR_NO_DEVICE, "handle was built host-only");
    if (n == 0) return P2M_OK;
    if (!d_points || !d_tri || !d_grad_dist) return fail(P2M_ERR_INVALID_ARG, "null points, triangles or gradient");
    if (n > 0x7fffffffLL) return fail(P2M_ERR_INVALID_ARG, "more than 2^31-1 points per call");
    DeviceGuard dg(h->device);
    hipError_t e = p2m::launch_backward(h->dm, d_points, n, d_order, d_tri, d_grad_dist, d_grad_points,
                                        d_grad_vertices, h->cfg.block_size, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return P2M_OK;
}

// ------------------------------------------------------------ inspection

int32_t p2m_host_sites(p2m_handle h, float* out_xyz, uint8_t* out_is_aux)
{
    if (!h) return fail(P2M_ERR_INVALID_ARG, "null handle");
    for (int32_t s = 0; s < h->H.n_sites; ++s) {
        if (out_xyz) std::memcpy(out_xyz + 3 * (int64_t)s, &h->H.site_rec[s].x, 12);
        if (out_is_aux) out_is_aux[s] = h->H.site_is_aux[s];
    }
    return P2M_OK;
}

int32_t p2m_host_site_of_vertex(p2m_handle h, int32_t* out)
{
    if (!h || !out) return fail(P2M_ERR_INVALID_ARG, "null handle or output");
    std::memcpy(out, h->H.site_of_vertex.data(), sizeof(int32_t) * h->H.site_of_vertex.size());
    return P2M_OK;
}

int32_t p2m_host_list(p2m_handle h, int64_t site, int32_t* out_tris, int64_t cap, int64_t* len)
{
    if (!h || !len || cap < 0) return fail(P2M_ERR_INVALID_ARG, "null handle or length");
    if (site < 0 || site >= h->H.n_sites) return fail(P2M_ERR_INVALID_ARG, "site out of range");
    const int32_t b = h->H.site_rec[site].list_begin, e = h->H.site_rec[site].list_end;
    *len = e - b;
    for (int64_t k = 0; k < std::min<int64_t>(cap, e - b) && out_tris; ++k)
        out_tris[k] = h->H.list_tri[b + k];
    return P2M_OK;
}

int32_t p2m_host_neighbors(p2m_handle h, int64_t site, int32_t* out, int64_t cap, int64_t* len)
{
    if (!h || !len || cap < 0) return fail(P2M_ERR_INVALID_ARG, "null handle or length");
    if (site < 0 || site >= h->H.n_sites) return fail(P2M_ERR_INVALID_ARG, "site out of range");
    const int32_t b = h->H.site_rec[site].adj_begin, e = h->H.site_rec[site].adj_end;
    *len = e - b;
    for (int64_t k = 0; k < std::min<int64_t>(cap, e - b) && out; ++k) {
        int32_t id;
        std::memcpy(&id, &h->H.adj[4 * (b + k) + 3], 4);
        out[k] = id;
    }
    return P2M_OK;
}

int32_t p2m_host_locate(p2m_handle h, const float* pts, int64_t n, int32_t* out_site)
{
    if (!h || (n > 0 && (!pts || !out_site))) return fail(P2M_ERR_INVALID_ARG, "null argument");
    const p2m::HostStructure& H = h->H;
    const float ginv = 1.0f / H.gcell;
    for (int64_t i = 0; i < n; ++i) {
        const float qx = pts[3 * i], qy = pts[3 * i + 1], qz = pts[3 * i + 2];
        if (!std::isfinite(qx) || !std::isfinite(qy) || !std::isfinite(qz)) {
            out_site[i] = -1;
            continue;
        }
        if (!H.oct.empty()) {
            // octree: the leaf box (float32 descent, as on the device); -1 outside the root
            const float q[3] = {qx, qy, qz};
            float c[3] = {H.oroot[0], H.oroot[1], H.oroot[2]};
            float hh = H.oroot[3];
            bool inside = true;
            for (int k = 0; k < 3; ++k) inside &= q[k] >= c[k] - hh && q[k] <= c[k] + hh;
            int32_t v = inside ? H.oct[0] : -1;
            while (inside && v >= 0) {
                int mk = 0;
                hh *= 0.5f;
                for (int k = 0; k < 3; ++k) {
                    const bool up = q[k] >= c[k];
                    mk |= (int)up << k;
                    c[k] = up ? c[k] + hh : c[k] - hh;
                }
                v = H.oct[v + mk];
            }
            out_site[i] = inside ? -v - 1 : -1;
            continue;
        }
        auto cell = [&](float v, int k) {
            const int c = (int)std::floor((v - H.gorg[k]) * ginv);
            return std::min(std::max(c, 0), H.gdim[k] - 1);
        };
        int s = H.seed[((int64_t)cell(qz, 2) * H.gdim[1] + cell(qy, 1)) * H.gdim[0] + cell(qx, 0)];
        for (int it = 0; it < 4096; ++it) {
            const p2m::SiteRec& sr = H.site_rec[s];
            const float sp[3] = {sr.x, sr.y, sr.z};
            const double wx = (double)qx - sp[0], wy = (double)qy - sp[1], wz = (double)qz - sp[2];
            double best = 0.0;
            int nxt = -1;
            for (int32_t k = sr.adj_begin; k < sr.adj_end; ++k) {
                const float* a = &H.adj[4 * (int64_t)k];
                const double dx = (double)a[0] - sp[0], dy = (double)a[1] - sp[1], dz = (double)a[2] - sp[2];
                const double val = wx * dx + wy * dy + wz * dz - 0.5 * (dx * dx + dy * dy + dz * dz);
                if (val > best) {
                    best = val;
                    std::memcpy(&nxt, &a[3], 4);
                }
            }
            if (nxt < 0) break;
            s = nxt;
        }
        out_site[i] = s;
    }
    return P2M_OK;
}

const char* p2m_status_string(int32_t s)
{
    switch (s) {
    case P2M_OK: return "ok";
    case P2M_ERR_INVALID_ARG: return "invalid argument";
    case P2M_ERR_BAD_MESH: return "bad mesh";
    case P2M_ERR_OOM: return "out of memory";
    case P2M_ERR_HIP: return "HIP error";
    case P2M_ERR_INTERNAL: return "internal error";
    case P2M_ERR_NO_DEVICE: return "no device data";
    default: return "unknown status";
    }
}

const char* p2m_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
