// Corner checks of the Voronoi stage (Sec. 3.2 builds the cells the walk
// and the interception lists use) on the GPU.
//
// A cell is the domain box clipped by the bisector half-spaces of nearby
// sites; it is final once no site lies closer than its own site to any of
// its corners.  The host clips; each round it hands over every corner that
// still needs that check, over all cells in progress, and this file answers
// them: for corner x with limit r^2 (1 - slack), the nearest site below the
// limit that is not already among the cell's planes, or none, or "gave up"
// when a budget of examined sites runs out.
//
// One lane per check.  Each lane runs the host's depth-first search of the
// site kd-tree step for step: the same nearer-child-first order, the same
// pruning against the best distance so far and the same count of examined
// sites, in FP64 with the host's operation order and no contraction into
// fused multiply-adds.  The answers, including the budget decisions that
// depend on the search order, are therefore the host's, and so are the
// cells.  The search stacks (one node id per level) live in LDS; a node's
// distance is recomputed when it is taken off the stack.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "host/build.h"
#include "host/kdtree.h"

namespace p2m {
namespace {

constexpr int kBlock = 256;
// Stack slots per lane: a depth-first search of a tree of depth d holds at
// most d + 1 entries; median splits into leaves of <= 8 sites keep d below
// 32 for any int32 site count.
constexpr int kMaxStack = 32;

struct KdView {
    const double* box;     // 6 per node: lo xyz, hi xyz
    const int4* link;      // per node: begin, end, left (-1 for a leaf), right
    const int32_t* order;  // leaf ranges index this
    const double* pts;     // 3 per site
};

// Squared distance from q to the node's box; the host's
// max(lo - q, 0, q - hi) per axis, summed in the same order.
__host__ __device__ __forceinline__ double box_d2(const double* b, double qx, double qy, double qz)
{
    const double dx = fmax(fmax(b[0] - qx, 0.0), qx - b[3]);
    const double dy = fmax(fmax(b[1] - qy, 0.0), qy - b[4]);
    const double dz = fmax(fmax(b[2] - qz, 0.0), qz - b[5]);
    return dx * dx + dy * dy + dz * dz;
}

__host__ __device__ __forceinline__ bool excluded(const int32_t* ex, int64_t lo, int64_t hi, int32_t p)
{
    const int64_t end = hi;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (ex[mid] < p) lo = mid + 1;
        else hi = mid;
    }
    return lo < end && ex[lo] == p;
}

// One check: the search of KdTree::below, with its stack at st[k * stride]
// for k < slots.  Returns the site, -1, -2 (budget spent) or -3 (stack too
// small, which the host's depth bound rules out).
__host__ __device__ inline int32_t check_one(const KdView& kd, double qx, double qy, double qz, double best,
                                             const int32_t* excl, int64_t e0, int64_t e1, int64_t budget,
                                             int32_t* st, int stride, int slots)
{
    int32_t bi = -1;
    int top = 0;
    st[0] = 0;
    top = 1;
    while (top > 0) {
        const int32_t node = st[--top * stride];
        const double d2n = box_d2(kd.box + 6 * (int64_t)node, qx, qy, qz);
        if (d2n >= best) continue;
        const int4 lk = kd.link[node];
        if (lk.z < 0) {
            if (budget >= 0) {
                budget -= lk.y - lk.x;
                if (budget < 0) return -2;
            }
            for (int32_t k = lk.x; k < lk.y; ++k) {
                const int32_t p = kd.order[k];
                const double* pp = kd.pts + 3 * (int64_t)p;
                const double ax = pp[0] - qx, ay = pp[1] - qy, az = pp[2] - qz;
                const double d2 = ax * ax + ay * ay + az * az;
                if (d2 < best || (d2 == best && bi >= 0 && p < bi)) {
                    if (excluded(excl, e0, e1, p)) continue;
                    best = d2;
                    bi = p;
                }
            }
            continue;
        }
        const double dl = box_d2(kd.box + 6 * (int64_t)lk.z, qx, qy, qz);
        const double dr = box_d2(kd.box + 6 * (int64_t)lk.w, qx, qy, qz);
        // the host pushes the farther child first and takes the nearer next;
        // a pushed node is tested against the best distance when taken
        if (top + 2 > slots) return -3;
        if (dl <= dr) {
            st[top++ * stride] = lk.w;
            st[top++ * stride] = lk.z;
        } else {
            st[top++ * stride] = lk.z;
            st[top++ * stride] = lk.w;
        }
    }
    return bi;
}

__global__ __launch_bounds__(kBlock) void corner_check_kernel(KdView kd, const double* __restrict__ q,
                                                              const double* __restrict__ limit2,
                                                              const int32_t* __restrict__ list,
                                                              const int64_t* __restrict__ excl_off,
                                                              const int32_t* __restrict__ excl, int64_t n,
                                                              int64_t budget, int stack_slots, int32_t* out)
{
    extern __shared__ int32_t stack_lds[];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t l = list[i];
    // slot k of this lane's stack at stack_lds[k * blockDim.x + tid]
    out[i] = check_one(kd, q[3 * i], q[3 * i + 1], q[3 * i + 2], limit2[i], excl, excl_off[l], excl_off[l + 1],
                       budget, stack_lds + threadIdx.x, (int)blockDim.x, stack_slots);
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    template <typename T>
    T* get() const { return (T*)p; }
};

void check(hipError_t e, const char* what)
{
    if (e != hipSuccess) throw Error(P2M_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
void upload(DevBuf& b, const T* src, size_t n)
{
    check(hipMalloc(&b.p, n ? n * sizeof(T) : 16), "hipMalloc (corner checks)");
    if (n) check(hipMemcpy(b.p, src, n * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy (corner checks)");
}

// The device copy of the last tree checked against, per host thread: the
// rounds of one build check against the same tree many times.  It is
// replaced when a thread checks against another tree (or device), and kept
// otherwise until the thread ends (a few MB; the buffers are not freed at
// exit, when the HIP runtime may already be gone).
struct TreeCache {
    int device = -1;
    uint64_t stamp = 0;
    void* box = nullptr;
    void* link = nullptr;
    void* order = nullptr;
    void* pts = nullptr;
};
thread_local TreeCache t_tree;

void release(TreeCache& c)
{
    for (void* p : {c.box, c.link, c.order, c.pts})
        if (p) (void)hipFree(p);
    c = TreeCache{};
}

template <typename T>
void upload_raw(void*& dst, const std::vector<T>& v)
{
    check(hipMalloc(&dst, v.empty() ? 16 : v.size() * sizeof(T)), "hipMalloc (corner checks)");
    if (!v.empty()) check(hipMemcpy(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy (corner checks)");
}

const TreeCache& device_tree(const KdTree& kd)
{
    int dev = -1;
    check(hipGetDevice(&dev), "hipGetDevice");
    if (t_tree.stamp == kd.stamp() && t_tree.device == dev) return t_tree;
    if (t_tree.device >= 0) {
        // free the old copy on the device that holds it
        const int old = t_tree.device;
        if (old != dev) check(hipSetDevice(old), "hipSetDevice");
        release(t_tree);
        if (old != dev) check(hipSetDevice(dev), "hipSetDevice");
    }
    std::vector<double> box, pts;
    std::vector<int32_t> link, order;
    kd.export_flat(box, link, order, pts);
    TreeCache c;
    c.device = dev;
    try {
        upload_raw(c.box, box);
        upload_raw(c.link, link);
        upload_raw(c.order, order);
        upload_raw(c.pts, pts);
    } catch (...) {
        release(c);
        throw;
    }
    c.stamp = kd.stamp();
    t_tree = c;
    return t_tree;
}

}  // namespace

void gpu_corner_checks(const CornerChecks& job, std::vector<int32_t>& out)
{
    const int64_t n = (int64_t)job.q.size();
    out.assign(n, -1);
    if (n == 0 || job.kd->n_nodes() == 0) return;
    const int slots = job.kd->depth() + 1;
    if (slots > kMaxStack) throw Error(P2M_ERR_INTERNAL, "site tree too deep for the device corner checks");
    const TreeCache& tc = device_tree(*job.kd);
    std::vector<double> qv(3 * n);
    for (int64_t i = 0; i < n; ++i) {
        qv[3 * i] = job.q[i].x;
        qv[3 * i + 1] = job.q[i].y;
        qv[3 * i + 2] = job.q[i].z;
    }
    DevBuf d_q, d_lim, d_list, d_eoff, d_excl, d_out;
    upload(d_q, qv.data(), qv.size());
    upload(d_lim, job.limit2.data(), job.limit2.size());
    upload(d_list, job.list.data(), job.list.size());
    upload(d_eoff, job.excl_off.data(), job.excl_off.size());
    upload(d_excl, job.excl.data(), job.excl.size());
    check(hipMalloc(&d_out.p, n * sizeof(int32_t)), "hipMalloc (corner checks)");
    const KdView kv{(const double*)tc.box, (const int4*)tc.link, (const int32_t*)tc.order, (const double*)tc.pts};
    const int64_t grid = (n + kBlock - 1) / kBlock;
    const size_t lds = (size_t)slots * kBlock * sizeof(int32_t);
    corner_check_kernel<<<(unsigned)grid, kBlock, lds>>>(kv, d_q.get<double>(), d_lim.get<double>(),
                                                         d_list.get<int32_t>(), d_eoff.get<int64_t>(),
                                                         d_excl.get<int32_t>(), n, job.budget, slots,
                                                         d_out.get<int32_t>());
    check(hipGetLastError(), "corner check launch");
    check(hipMemcpy(out.data(), d_out.p, n * sizeof(int32_t), hipMemcpyDeviceToHost), "hipMemcpy (corner checks)");
    for (int64_t i = 0; i < n; ++i)
        if (out[i] == -3) throw Error(P2M_ERR_INTERNAL, "device corner check stack overflow");
}

}  // namespace p2m
