// Batched multi-mesh queries (not in the paper): one persistent launch over
// many meshes, captured in a HIP graph together with the per-mesh query
// sort.  Work items of `tile` sorted queries are handed out from a global
// counter, so uneven mesh and query-set sizes balance across the chip.  The
// tile and grid sizes are chosen by timing candidates on the bound data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "device.h"
#include "host/build.h"
#include "p2m.h"

// Defined in capi.hip.
struct p2m_handle_;
namespace p2m {
const DevMesh& handle_devmesh(const p2m_handle_* h);
int handle_device(const p2m_handle_* h);
void set_last_error(const std::string& msg);
}  // namespace p2m

namespace {

int32_t fail(int32_t code, const std::string& msg)
{
    p2m::set_last_error(msg);
    return code;
}

int32_t hip_fail(hipError_t e, const char* what)
{
    return fail(P2M_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int d)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(d);
    }
    ~DevGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct p2m_batch_ {
    std::vector<p2m_handle> meshes;
    std::vector<int64_t> counts, q_off;
    int device = 0;
    int autotune = 1;
    std::string cache_path;
    int tile = 256, grid = 0, block = 256, stage = 0;  // one workgroup per item until tuned
    bool tuned = false;
    // device buffers
    p2m::DevMesh* d_meshes = nullptr;
    int64_t* d_qoff = nullptr;
    int32_t** d_perm = nullptr;
    float** d_gradv = nullptr;
    int32_t* d_item_mesh = nullptr;
    int64_t* d_item_first = nullptr;
    unsigned* d_counter = nullptr;
    void* ws = nullptr;
    int32_t n_items = 0;
    int32_t items_tile = 0;
    std::vector<size_t> ws_off;
    // bound arguments
    p2m::BatchArgs args{};
    bool fused = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~p2m_batch_()
    {
        DevGuard g(device);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (void* p : {(void*)d_meshes, (void*)d_qoff, (void*)d_perm, (void*)d_gradv, (void*)d_item_mesh,
                        (void*)d_item_first, (void*)d_counter, ws})
            if (p) (void)hipFree(p);
    }

    // Work items for tile size t: per mesh, ceil(count / t) items.
    int32_t build_items(int t)
    {
        std::vector<int32_t> im;
        std::vector<int64_t> first;
        // largest meshes first so long items start early
        std::vector<int> order(meshes.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return counts[a] > counts[b]; });
        for (int i : order)
            for (int64_t f = 0; f < counts[i]; f += t) {
                im.push_back(i);
                first.push_back(f);
            }
        if (d_item_mesh) (void)hipFree(d_item_mesh);
        if (d_item_first) (void)hipFree(d_item_first);
        d_item_mesh = nullptr;
        d_item_first = nullptr;
        n_items = (int32_t)im.size();
        items_tile = t;
        const size_t n = std::max<size_t>(im.size(), 1);
        hipError_t e = hipMalloc(&d_item_mesh, n * sizeof(int32_t));
        if (e != hipSuccess) return hip_fail(e, "hipMalloc items");
        e = hipMalloc(&d_item_first, n * sizeof(int64_t));
        if (e != hipSuccess) return hip_fail(e, "hipMalloc items");
        if (!im.empty()) {
            e = hipMemcpy(d_item_mesh, im.data(), im.size() * sizeof(int32_t), hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(d_item_first, first.data(), first.size() * sizeof(int64_t), hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy items");
        }
        return P2M_OK;
    }

    // The whole batched sequence on `st` (also what the graph records).
    hipError_t enqueue(hipStream_t st)
    {
        hipError_t e = p2m::launch_fill_u32(d_counter, 0u, 1, st);
        if (e != hipSuccess) return e;
        std::vector<const int32_t*> perms(meshes.size(), nullptr);
        for (size_t i = 0; i < meshes.size(); ++i) {
            if (counts[i] == 0) continue;
            e = p2m::launch_reorder(p2m::handle_devmesh(meshes[i]), args.q + 3 * q_off[i], counts[i], 0,
                                    (char*)ws + ws_off[i], &perms[i], st);
            if (e != hipSuccess) return e;
        }
        p2m::BatchArgs a = args;
        a.item_mesh = d_item_mesh;
        a.item_first = d_item_first;
        a.n_items = n_items;
        a.tile = items_tile;
        a.counter = d_counter;
        return p2m::launch_batch(d_meshes, a, grid, block, fused, stage, st);
    }
};

namespace {

// The autotuner's cache key: the device, the fused flag and every mesh's
// triangle and query counts (a batch of other sizes gets its own entry).
std::string cache_key(const p2m_batch_* b)
{
    uint64_t h = 1469598103934665603ull;  // FNV-1a over the per-mesh sizes
    auto mix = [&](uint64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (v >> (8 * k)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    int64_t tris = 0, total = 0;
    for (size_t i = 0; i < b->meshes.size(); ++i) {
        p2m_stats s;
        p2m_get_stats(b->meshes[i], &s);
        tris += s.n_triangles;
        total += b->counts[i];
        mix((uint64_t)s.n_triangles);
        mix((uint64_t)s.n_sites);
        mix((uint64_t)b->counts[i]);
    }
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) arch = prop.gcnArchName;
    std::ostringstream os;
    os << arch << "_m" << b->meshes.size() << "_t" << tris << "_q" << total << "_f" << (b->fused ? 1 : 0) << "_h"
       << std::hex << h;
    return os.str();
}

bool cache_lookup(const std::string& path, const std::string& key, int& tile, int& grid, int& block, int& stage)
{
    std::ifstream f(path);
    std::string k;
    int t, g, bl, sg;
    while (f >> k >> t >> g >> bl >> sg)
        if (k == key) {
            tile = t;
            grid = g;
            block = bl;
            stage = sg;
            return true;
        }
    return false;
}

void cache_store(const std::string& path, const std::string& key, int tile, int grid, int block, int stage)
{
    std::ofstream f(path, std::ios::app);
    if (f) f << key << " " << tile << " " << grid << " " << block << " " << stage << "\n";
}

}  // namespace

extern "C" {

int32_t p2m_batch_create(const p2m_handle* meshes, int32_t n_meshes, const int64_t* h_query_counts,
                         int32_t autotune, const char* cache_path, p2m_batch* out)
{
    if (!out || n_meshes <= 0 || !meshes || !h_query_counts)
        return fail(P2M_ERR_INVALID_ARG, "null argument or no meshes");
    *out = nullptr;
    const int dev = p2m::handle_device(meshes[0]);
    for (int i = 0; i < n_meshes; ++i) {
        if (!meshes[i]) return fail(P2M_ERR_INVALID_ARG, "null mesh handle");
        if (p2m::handle_device(meshes[i]) < 0) return fail(P2M_ERR_NO_DEVICE, "mesh handle built host-only");
        if (p2m::handle_device(meshes[i]) != dev) return fail(P2M_ERR_INVALID_ARG, "meshes on different devices");
        if (h_query_counts[i] < 0) return fail(P2M_ERR_INVALID_ARG, "negative query count");
    }
    p2m_batch_* b = new (std::nothrow) p2m_batch_();
    if (!b) return fail(P2M_ERR_OOM, "host allocation failed");
    b->device = dev;
    b->autotune = autotune;
    if (cache_path) b->cache_path = cache_path;
    b->meshes.assign(meshes, meshes + n_meshes);
    b->counts.assign(h_query_counts, h_query_counts + n_meshes);
    b->q_off.assign(n_meshes + 1, 0);
    for (int i = 0; i < n_meshes; ++i) b->q_off[i + 1] = b->q_off[i] + b->counts[i];
    DevGuard g(dev);
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "hipGetDeviceProperties");
    }
    b->grid = 0;
    std::vector<p2m::DevMesh> dm(n_meshes);
    for (int i = 0; i < n_meshes; ++i) dm[i] = p2m::handle_devmesh(meshes[i]);
    size_t ws_total = 0;
    b->ws_off.resize(n_meshes);
    for (int i = 0; i < n_meshes; ++i) {
        b->ws_off[i] = ws_total;
        ws_total += (p2m::reorder_workspace_bytes(b->counts[i], 0) + 255) / 256 * 256;
    }
    e = hipMalloc(&b->d_meshes, sizeof(p2m::DevMesh) * n_meshes);
    if (e == hipSuccess) e = hipMalloc(&b->d_qoff, sizeof(int64_t) * (n_meshes + 1));
    if (e == hipSuccess) e = hipMalloc(&b->d_perm, sizeof(int32_t*) * n_meshes);
    if (e == hipSuccess) e = hipMalloc(&b->d_gradv, sizeof(float*) * n_meshes);
    if (e == hipSuccess) e = hipMalloc(&b->d_counter, 256);
    if (e == hipSuccess) e = hipMalloc(&b->ws, std::max<size_t>(ws_total, 256));
    if (e != hipSuccess) {
        delete b;
        return fail(P2M_ERR_OOM, std::string("batch hipMalloc: ") + hipGetErrorString(e));
    }
    // Each mesh's sorted order lands at the same place in its workspace on every call.
    std::vector<int32_t*> perm(n_meshes, nullptr);
    for (int i = 0; i < n_meshes; ++i)
        if (b->counts[i] > 0)
            perm[i] = (int32_t*)p2m::reorder_perm_location((char*)b->ws + b->ws_off[i], b->counts[i], 0);
    e = hipMemcpy(b->d_meshes, dm.data(), sizeof(p2m::DevMesh) * n_meshes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_qoff, b->q_off.data(), sizeof(int64_t) * (n_meshes + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_perm, perm.data(), sizeof(int32_t*) * n_meshes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch hipMemcpy");
    }
    int32_t rc = b->build_items(b->tile);
    if (rc != P2M_OK) {
        delete b;
        return rc;
    }
    *out = b;
    return P2M_OK;
}

int32_t p2m_batch_bind(p2m_batch b, const float* d_points, float* d_out_dist, int32_t* d_out_tri,
                       float* d_out_closest, const float* d_grad_dist, float* d_grad_points,
                       float* const* d_grad_vertices, void* stream)
{
    if (!b) return fail(P2M_ERR_INVALID_ARG, "null batch");
    const int64_t total = b->q_off.back();
    if (total > 0 && (!d_points || !d_out_dist)) return fail(P2M_ERR_INVALID_ARG, "null points or distances");
    DevGuard g(b->device);
    hipStream_t st = (hipStream_t)stream;
    b->fused = d_grad_dist != nullptr;
    std::vector<float*> gv(b->meshes.size(), nullptr);
    if (b->fused && d_grad_vertices)
        for (size_t i = 0; i < gv.size(); ++i) gv[i] = d_grad_vertices[i];
    hipError_t e = hipMemcpy(b->d_gradv, gv.data(), sizeof(float*) * gv.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy grad pointers");
    b->args = p2m::BatchArgs{};
    b->args.q = d_points;
    b->args.dist = d_out_dist;
    b->args.tri = d_out_tri;
    b->args.closest = d_out_closest;
    b->args.grad_dist = d_grad_dist;
    b->args.grad_q = b->fused ? d_grad_points : nullptr;
    b->args.grad_v = b->d_gradv;
    b->args.perm = b->d_perm;
    b->args.q_off = b->d_qoff;

    if (!b->tuned) {
        const std::string key = cache_key(b);
        int t = b->tile, gr = b->grid, bl = b->block, sg = b->stage;
        if (!b->cache_path.empty() && cache_lookup(b->cache_path, key, t, gr, bl, sg)) {
            b->tile = t;
            b->grid = gr;
            b->block = bl;
            b->stage = sg;
        } else if (b->autotune && total > 0) {
            // Time the plain sequence for each candidate (work-item size,
            // persistent workgroups per CU, workgroup size, LDS staging); the
            // fused form accumulates into the caller's gradient buffers, so
            // tune on the forward form and reuse the choice.
            const bool fused = b->fused;
            b->fused = false;
            hipDeviceProp_t prop;
            (void)hipGetDeviceProperties(&prop, b->device);
            const int cus = prop.multiProcessorCount;
            hipEvent_t e0, e1;
            (void)hipEventCreate(&e0);
            (void)hipEventCreate(&e1);
            float best = 1e30f;
            int bt = b->tile, bg = b->grid, bb = b->block, bs = b->stage;
            // mult 0: one workgroup per item of one block of queries (no
            // queue); else a persistent grid of mult workgroups per CU taking
            // items of tile_blocks blocks from the queue
            for (int block : {256, 512})
                for (int tile_blocks : {1, 2, 8, 32})
                    for (int mult : {0, 2, 4, 8})
                        for (int stage : {0, 1}) {
                            if ((mult == 0) != (tile_blocks == 1)) continue;
                            const int tile = tile_blocks * block;
                            int32_t rc = b->build_items(tile);
                            if (rc != P2M_OK) return rc;
                            b->grid = cus * mult;
                            b->block = block;
                            b->stage = stage;
                            float ms = 0.f;
                            for (int rep = 0; rep < 2; ++rep) {
                                (void)hipEventRecord(e0, st);
                                e = b->enqueue(st);
                                if (e != hipSuccess) return hip_fail(e, "autotune launch");
                                (void)hipEventRecord(e1, st);
                                e = hipEventSynchronize(e1);
                                if (e != hipSuccess) return hip_fail(e, "autotune sync");
                                (void)hipEventElapsedTime(&ms, e0, e1);
                            }
                            if (ms < best) {
                                best = ms;
                                bt = tile;
                                bg = b->grid;
                                bb = block;
                                bs = stage;
                            }
                        }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            b->fused = fused;
            b->tile = bt;
            b->grid = bg;
            b->block = bb;
            b->stage = bs;
            if (!b->cache_path.empty()) cache_store(b->cache_path, key, bt, bg, bb, bs);
        }
        b->tuned = true;
    }
    int32_t rc = b->build_items(b->tile);
    if (rc != P2M_OK) return rc;

    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    // Record into a private stream (the caller's may be the null stream,
    // which cannot be captured); the graph is launched on the caller's stream.
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    hipError_t le = b->enqueue(cap);
    e = hipStreamEndCapture(cap, &b->graph);
    (void)hipStreamDestroy(cap);
    if (le != hipSuccess) return hip_fail(le, "captured launch");
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return P2M_OK;
}

int32_t p2m_batch_launch(p2m_batch b, void* stream)
{
    if (!b || !b->exec) return fail(P2M_ERR_INVALID_ARG, "batch not bound");
    DevGuard g(b->device);
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return P2M_OK;
}

int32_t p2m_batch_set_config(p2m_batch b, int32_t tile, int32_t grid, int32_t block, int32_t stage)
{
    if (!b) return fail(P2M_ERR_INVALID_ARG, "null batch");
    if (block < 64 || block > 1024 || block % 64 != 0)
        return fail(P2M_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
    if (grid < 0 || tile < 1 || (grid == 0 && tile != block))
        return fail(P2M_ERR_INVALID_ARG, "tile >= 1, grid >= 0, and tile == block when grid is 0");
    if (stage != 0 && stage != 1) return fail(P2M_ERR_INVALID_ARG, "stage must be 0 or 1");
    b->tile = tile;
    b->grid = grid;
    b->block = block;
    b->stage = stage;
    b->tuned = true;
    return P2M_OK;
}

int32_t p2m_batch_config(p2m_batch b, int32_t* tile, int32_t* grid, int32_t* block, int32_t* stage)
{
    if (!b) return fail(P2M_ERR_INVALID_ARG, "null batch");
    if (tile) *tile = b->tile;
    if (grid) *grid = b->grid;
    if (block) *block = b->block;
    if (stage) *stage = b->stage;
    return P2M_OK;
}

int32_t p2m_batch_destroy(p2m_batch b)
{
    delete b;
    return P2M_OK;
}

}  // extern "C"
