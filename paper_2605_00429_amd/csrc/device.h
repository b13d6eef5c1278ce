// Device-side layout of one built mesh and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace p2m {

// Read-only search structure of one mesh in device memory (see build.h for
// the meaning of each array).  Passed to kernels by value.
struct DevMesh {
    const float4* site_rec;  // 2 per site: (x, y, z, 0), int4 (adj begin, end, list begin, end)
    const float4* adj;       // neighbour xyz + id bits
    const float4* list_sph;  // 1 per list entry: bounding sphere (c, r); the scan recomputes a lower
                             // bound of ell from it
    const float4* list_rec;  // 3 per list entry, same index: (a, ell), (e1, e1.e2), (e2, caller triangle id bits)
    const float4* tri_rec;   // 3 per slot: (a, |e1|^2), (e1, e1.e2), (e2, |e2|^2)
    const int32_t* tri_user; // slot -> caller triangle id
    const int4* tri_vid;     // caller triangle id -> caller vertex ids
    const float4* verts;     // caller vertices (x, y, z, 0): the winner's exact FP64 closest point
    const int32_t* tri_slot; // caller triangle id -> slot
    const int32_t* seed;     // seed grid (x fastest)
    const float4* bvh;       // 2 per node
    const int32_t* oct;      // octree decomposition: nodes (first child, or -(site + 1)); null for Voronoi cells
    float oroot[4];          // octree root centre xyz, half size
    int32_t gdim[3];
    float gorg[3];
    float ginv;              // 1 / seed cell size
    float dlo[3], dhi[3];    // domain box
    int32_t n_sites, n_tris, n_vertices;
};

// A load from device memory issued as a global-memory access.  Left to
// itself the compiler issued the search kernel's loads as flat (generic)
// ones, which take 64-bit address arithmetic per lane and also wait on the
// LDS counter.  T is a 4-, 8- or 16-byte type (int, float, int2, float4,
// int4).
template <class T>
__device__ __forceinline__ T gload(const T* p)
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8 || sizeof(T) == 16, "gload: 4, 8 or 16 bytes");
    if constexpr (sizeof(T) == 16) {
        typedef int v4 __attribute__((ext_vector_type(4)));
        return __builtin_bit_cast(T, *(const __attribute__((address_space(1))) v4*)p);
    } else if constexpr (sizeof(T) == 8) {
        typedef int v2 __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(T, *(const __attribute__((address_space(1))) v2*)p);
    } else {
        return __builtin_bit_cast(T, *(const __attribute__((address_space(1))) int*)p);
    }
}

// Counter slots of the instrumented forward.
// CTR_WALK_CAP counts walks stopped at the step cap (answered by the exact
// BVH fallback, so also counted in CTR_FALLBACK).
enum { CTR_WALK_STEPS = 0, CTR_ADJ_READ, CTR_LIST_READ, CTR_EXACT, CTR_FALLBACK, CTR_LIST_LEN, CTR_WALK_CAP, CTR_N };

// Instrumented forward only: one flag per item of each structure array,
// set to 1 when a load touches the item, so that the distinct bytes one
// launch reads can be counted (each array zeroed by the caller; null =
// not recorded).  Items: site records (32 B), adjacency entries (16 B), list
// spheres (16 B), list records (48 B), seed cells (4 B), triangle records
// of the fallback (48 B), fallback BVH nodes (32 B).
struct Touch {
    uint8_t* site;
    uint8_t* adj;
    uint8_t* sph;
    uint8_t* rec;
    uint8_t* seed;
    uint8_t* tri;
    uint8_t* bvh;
};

struct FwdArgs {
    const float* q;          // n x 3: caller order, or visiting order when q_sorted
    const int32_t* perm;     // optional processing order (output positions)
    int32_t q_sorted;        // q[j] is the j-th point visited (already permuted)
    int64_t n;
    float* dist;
    int32_t* tri;            // nullable
    float* closest;          // nullable
    const float* grad_dist;  // fused only
    float* grad_q;           // fused only, nullable
    float* grad_v;           // fused only, nullable
    unsigned long long* ctr; // counters only
    Touch touch;             // counters only: distinct items read (see Touch)
    int32_t xcds;            // blocks are spread over this many XCD groups (see launch_forward)
    int32_t acc_slots;       // fused: LDS hash slots for vertex gradients (set by launch_forward)
    int32_t stage;           // 1: stage the located sites' list spheres in LDS before the scan
};

// Arguments of the persistent batched kernel.  Queries of mesh i occupy
// [q_off[i], q_off[i+1]) of the concatenated arrays; work item t covers
// sorted positions [item_first[t], item_first[t] + tile) of mesh item_mesh[t].
struct BatchArgs {
    const float* q;
    float* dist;
    int32_t* tri;
    float* closest;
    const float* grad_dist;
    float* grad_q;
    float* const* grad_v;        // per mesh (device array of device pointers)
    const int32_t* const* perm;  // per mesh, or null entries
    const int64_t* q_off;        // n_meshes + 1
    const int32_t* item_mesh;
    const int64_t* item_first;
    int32_t n_items;
    int32_t tile;
    unsigned* counter;
    int32_t stage;      // LDS staging capacity per wavefront (0: off; set by launch_batch)
    int32_t acc_slots;  // fused: LDS hash slots for vertex gradients (set by launch_batch)
};

// stage: 1 to stage list spheres in LDS (capacity chosen here), 0 not.
hipError_t launch_batch(const DevMesh* meshes, const BatchArgs& a, int grid, int block, bool fused, int stage,
                        hipStream_t st);
hipError_t launch_forward(const DevMesh& m, const FwdArgs& a, int block, bool fused, bool counters,
                          hipStream_t st);
// order (nullable): visit point order[j] at thread j.  The closest point
// of each point's triangle is recomputed exactly (FP64), as the forward
// computed it for its winner.
hipError_t launch_backward(const DevMesh& m, const float* q, int64_t n, const int32_t* order,
                           const int32_t* tri, const float* g, float* grad_q, float* grad_v, int block,
                           hipStream_t st);
// The search as three passes for point sets with many points per cell:
// locate in the visiting order (a.perm / a.q_sorted as launch_forward),
// sort by located site, scan each site's list once per run of lanes sharing
// it (through LDS).  Same outputs as launch_forward (not instrumented).
// ws must hold grouped_workspace_bytes(a.n, m.n_sites) bytes.
size_t grouped_workspace_bytes(int64_t n, int64_t n_sites);
hipError_t launch_grouped(const DevMesh& m, const FwdArgs& a, void* ws, bool fused, hipStream_t st);
// Radix sort of queries by the Morton code of their cell in a 2^k grid
// over the seed-grid box (k from n when bits = 0).  ws must hold
// reorder_workspace_bytes(n) bytes; writes the order to *perm_out.
// bits = 0 picks the resolution from n.
size_t reorder_workspace_bytes(int64_t n, int bits);
// sorted_q (nullable, n x 3): also receives the points in the sorted order.
hipError_t launch_reorder(const DevMesh& m, const float* q, int64_t n, int bits, void* ws,
                          const int32_t** perm_out, hipStream_t st, float* sorted_q = nullptr);
// Where launch_reorder leaves the order inside ws (fixed for given n, bits).
const int32_t* reorder_perm_location(void* ws, int64_t n, int bits);
// Max (with index), sum, sum of squares and count of the non-NaN entries of
// d[0..n): 5 doubles to out; part holds 5 doubles per block of the first
// stage (reduce_blocks(n) blocks).
int reduce_blocks(int64_t n);
hipError_t launch_reduce_dist(const float* d, int64_t n, double* part, double* out, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
// Combines two point-set reductions (5 doubles each, as launch_reduce_dist
// leaves them: A's points against B, B's points against A) into the six
// mesh-distance values of p2m_mesh_distance.
hipError_t launch_mesh_distance_combine(const double* ab, const double* ba, double* out, hipStream_t st);

}  // namespace p2m
