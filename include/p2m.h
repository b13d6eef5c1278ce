/*
 * p2m.h - C ABI of the MI355X (gfx950) P2M++ point-to-mesh distance library.
 *
 * The method (P2M++, Sec. 3): partition space by the Voronoi diagram of a
 * site set (the mesh vertices plus auxiliary sites placed where Voronoi
 * vertices cluster, Sec. 3.2), precompute for every site an interception
 * list of the triangles that can be closer to some point of its cell than
 * the site's reference point (Sec. 3.3, Eq. (2), the Vertex Sphere Union
 * theorem Eq. (3) and the conservative sphere Eq. (8)), and answer a query
 * by locating the nearest site and taking the minimum exact point-triangle
 * distance over its list with bounding-sphere pruning (Sec. 3.4).
 *
 * Conventions for every call below:
 *   - Return value: P2M_OK (0) or one of the P2M_ERR_* codes;
 *     p2m_last_error() gives a thread-local message for the last failure.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the device current when the handle was built.
 *   - Arrays of points are row-major float32 x, y, z triples.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Query calls only enqueue work; they do not synchronise.  Errors of
 *     asynchronous kernels surface at the caller's next synchronisation.
 *   - n == 0 is a valid no-op.
 */
#ifndef P2M_H
#define P2M_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    P2M_OK = 0,
    P2M_ERR_INVALID_ARG = 1, /* null required pointer, negative size, bad option */
    P2M_ERR_BAD_MESH = 2,    /* no triangles, index out of range, non-finite vertex */
    P2M_ERR_OOM = 3,         /* host or device allocation failed, or a size limit hit */
    P2M_ERR_HIP = 4,         /* HIP runtime or launch error (see p2m_last_error) */
    P2M_ERR_INTERNAL = 5,    /* invariant violated inside the library */
    P2M_ERR_NO_DEVICE = 6    /* handle built host-only (device = -1): no query calls */
};

typedef struct p2m_handle_* p2m_handle;
typedef struct p2m_batch_* p2m_batch;

/* A triangle mesh, in host memory.  vertices: n_vertices x 3 float32;
 * triangles: n_triangles x 3 int32 0-based vertex indices.  p2m_build copies
 * both; the caller may free them on return. */
typedef struct {
    const float* vertices;
    int64_t n_vertices;
    const int32_t* triangles;
    int64_t n_triangles;
} p2m_mesh_desc;

/* Preprocessing options.  p2m_default_opts() fills the defaults below.
 * The augmentation constants are the ones the paper leaves to experiment
 * (Sec. 3.2, "Choice of Parameters"); none of them affects exactness. */
typedef struct {
    float domain_scale;        /* cells are clipped to the mesh box scaled by this about its
                                  centre (default 10, the query region of Sec. 4); queries
                                  outside it take an exact BVH fallback */
    int32_t augment;           /* 1: ring-based auxiliary sites (Sec. 3.2), 0: vertex sites only */
    float tau_scale;           /* density grid cell tau = tau_scale * mean edge length (2) */
    int32_t dense_min_sites;   /* a grid cell is dense when at least max(this, dense_rel *
                                  median) distinct sites have a Voronoi vertex in it; the
                                  median is over grid cells holding mesh vertices (256) */
    float dense_rel;           /* (8) */
    int32_t ring_sites;        /* ring_layers = 0: sites on the one enclosing sphere of a dense
                                  cluster (12, the icosahedron's directions); > 0: the fewest
                                  sites of one ring (12) */
    int32_t ring_layers;       /* > 0 (default 8): about a dense cluster at distance d from the
                                  mesh, up to this many layers of auxiliary sites at radii d/2,
                                  d/4, ... (down to tau), each about tau apart: rings normal to
                                  the cluster's axis when its Voronoi vertices lie along a line
                                  (cylinder, cone and torus cores), else spherical shells;
                                  0: the one enclosing sphere of ring_sites sites */
    int32_t aux_list_mode;     /* 0: one conservative sphere per auxiliary site, Eq. (8);
                                  1: corner balls about the site's projection on the mesh
                                  (Eq. (3) with that reference point; a subset of mode 0) (1) */
    float list_inflation_rel;  /* corner-ball radius inflation / mesh box diagonal (1e-7) */
    float seed_cell_scale;     /* seed grid cell = this * mean edge length (2) */
    int64_t seed_max_cells;    /* cap on seed grid cells (16M) */
    int32_t n_threads;         /* host preprocessing threads, 0 = all */
    int32_t decomposition;     /* convex cells of the domain: 0 = Voronoi cells of the sites
                                  (the paper's, default); 1 = an adaptive octree over the mesh
                                  box x1.25 whose leaf boxes get corner-ball lists about the
                                  mesh point closest to their centre (the paper's remark that
                                  any convex decomposition with point location serves) */
    int32_t octree_max_list;   /* octree: split a box while its list is longer (64) */
    int32_t octree_max_depth;  /* octree: at most this many levels below the root (12, <= 16) */
    int32_t gpu_lists;         /* 1: the list stage's sphere-union tests run on the device
                                  (same lists; sites with more than 256 balls stay on the
                                  host); 0: all on the host (default 1; needs device >= 0) */
    int32_t gpu_voronoi;       /* 1 (default): the Voronoi stage's cells are built on the
                                  device, one wavefront per cell (kNN, clipping, corner
                                  checks in rounds over all cells in progress); cells that
                                  outgrow the device's per-cell capacity (128 faces, 1,024
                                  polygon vertices) are built on the host; 2: only the
                                  corner checks (is a site closer than the cell's own to
                                  this corner?) run on the device, the host clips; 0: all
                                  on the host.  The cells are the same, bit for bit, in all
                                  three (needs device >= 0 for 1 and 2) */
    int32_t device;            /* HIP device to upload to; -2 (default) = the current
                                  device; -1 = host only (inspection, no query calls) */
    int32_t gpu_cell_pass;     /* with gpu_voronoi = 1: cells built per device pass, each
                                  taking about 118 KB of device memory during the build;
                                  0 (default) = as many as a quarter of the free device
                                  memory holds, at most 32 GiB of them.  The cells are the
                                  same for any value (>= 0) */
} p2m_build_opts;

/* Statistics of a built handle (list lengths as in Table 1 of the paper). */
typedef struct {
    int64_t n_vertices, n_triangles;
    int64_t n_sites, n_vertex_sites, n_aux_sites, n_dense_cells;
    int64_t adj_nnz, adj_max;
    int64_t list_nnz, list_max;
    double adj_avg, list_avg;
    int32_t seed_dims[3];
    double t_voronoi_s, t_optimize_s, t_lists_s, t_layout_s, t_total_s;
    int64_t device_bytes;
    double diag;
    int64_t n_cells_device;    /* Voronoi cells (over every pass) built on the device */
    int64_t n_cells_host;      /* ... and on the host (all of them with gpu_voronoi != 1) */
} p2m_stats;

/* Per-handle launch configuration of the query kernels. */
typedef struct {
    int32_t block_size; /* threads per block: 64..1024, multiple of 64 (default 256) */
    int32_t reorder;    /* 1: sort queries spatially before the search (default 1) */
    int32_t xcd_groups; /* > 1: give each of this many XCDs (workgroups are dispatched
                           round-robin over them) a contiguous range of the sorted points;
                           1 (default, measured faster on MI355X) = plain block order */
    int32_t sort_bits;  /* sort grid of 2^sort_bits cells per axis (1..8); 0 = automatic,
                           the finest grid with at most two cells per point */
    int32_t stage;      /* 1: each wavefront copies the bounding spheres of its located sites'
                           lists into LDS with coalesced loads before the list scan (up to 256
                           per wavefront); 0 (default, measured faster on MI355X): the scan
                           gathers them from device memory.  Results are identical. */
    int32_t group;      /* the search of a non-instrumented query: 0 = one pass (walk, regroup by
                           site within each workgroup, per-lane list scans); 1 = three passes
                           (locate every point, sort the points by located site, then each run of
                           lanes sharing a site scans its list once, loaded 32 entries at a time
                           through LDS); 2 (default) = the three passes for a forward or
                           fused call of at least 2,000,000 points.  Results are identical. */
} p2m_query_config;

void p2m_default_opts(p2m_build_opts* opts);

/* Preprocess a mesh (Sec. 3.2-3.3) and upload the search structure.
 * Synchronous; runs on host threads.  opts may be NULL (defaults).
 * Unreferenced vertices are not sites; vertices at equal positions share one
 * site.  On success *out owns all host and device memory of the structure. */
int32_t p2m_build(const p2m_mesh_desc* mesh, const p2m_build_opts* opts, p2m_handle* out);

/* Free a handle.  The caller must first synchronise streams that used it. */
int32_t p2m_destroy(p2m_handle h);

/* Distance query (Sec. 3.4): for each point, locate the nearest site, then
 * the minimum exact point-triangle distance over its interception list.
 *   d_points:      device, n x 3 float32
 *   d_out_dist:    device, n float32 (required); NaN for a non-finite point
 *   d_out_tri:     device, n int32 (nullable); caller's triangle id, -1 for NaN
 *   d_out_closest: device, n x 3 float32 (nullable); closest point on the mesh
 * The handle is read-only after p2m_build: calls on different streams may
 * run concurrently, each stream getting its own scratch memory (the query
 * sort's workspace, about 16 B per point, allocated on a stream's first call
 * and grown as needed; held until p2m_destroy).  Calls on one stream run in
 * stream order; calls from several host threads are serialised while they
 * enqueue. */
int32_t p2m_query(p2m_handle h, const float* d_points, int64_t n, float* d_out_dist,
                  int32_t* d_out_tri, float* d_out_closest, void* stream);

/* p2m_query for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same results as p2m_query, with the query sort's workspace taken from
 * a 32 MiB device array of the library (one per GPU, held until the process
 * ends) instead of the stream's scratch.  It calls no hipMalloc, hipFree or
 * allocating library routine.  Point counts whose sort workspace exceeds
 * the array (about 2,000,000 points at the default settings; roughly 16.25
 * bytes per point) are refused with P2M_ERR_INVALID_ARG before any launch.
 * The array needs no clearing between calls (every byte a call reads it
 * first writes).  All calls on one GPU share it: calls that overlap on one
 * GPU (on different streams, or from different host threads) race and must
 * not be issued. */
int32_t p2m_query_noalloc(p2m_handle h, const float* d_points, int64_t n, float* d_out_dist,
                          int32_t* d_out_tri, float* d_out_closest, void* stream);

/* Distance from a point set to the mesh, reduced on the device: the
 * building block of mesh-to-mesh distance (named as an application in
 * Sec. 5).  With the points sampled on (or the vertices of) a second surface
 * A, d_out[0] is the one-sided Hausdorff distance from A to this mesh and
 * d_out[2] / d_out[4] the mean distance (one Chamfer term).
 *   d_points: device, n x 3 float32
 *   d_out:    device, 5 float64: max distance, index of the point attaining it
 *             (lowest index on ties), sum of distances, sum of squared
 *             distances, number of points counted; non-finite points (NaN
 *             distance) are left out.  n = 0 (or no finite point) gives
 *             max = -1, index = -1, sums and count 0.
 * Runs p2m_query's sort and search into a buffer of the stream's scratch
 * (n floats, allocated on first use and grown as needed; see p2m_query) and
 * two reduction kernels, all on `stream`. */
int32_t p2m_point_set_distance(p2m_handle h, const float* d_points, int64_t n, double* d_out, void* stream);

/* Distances between two meshes A (handle a) and B (handle b) measured on
 * point sets, built on the point query (Sec. 5 names mesh-to-mesh distance
 * as an application; the measures are defined here): points on A against
 * mesh B and points on B against mesh A, each reduced as in
 * p2m_point_set_distance.
 *   d_points_a: device, n_a x 3 float32 points on A; NULL with n_a = 0 for
 *               A's referenced vertices (every vertex some triangle uses, in
 *               index order: the exact vertex-to-mesh distances)
 *   d_points_b: likewise for B
 *   d_out:      device, 6 float64: [0] one-sided Hausdorff distance A to B
 *               (largest distance of A's points to B), [1] B to A, [2] the
 *               symmetric Hausdorff distance max([0], [1]), [3] the Chamfer
 *               distance mean_A d + mean_B d, [4] the squared Chamfer
 *               distance mean_A d^2 + mean_B d^2, [5] the number of points
 *               counted.  Points with a non-finite coordinate are left out;
 *               a side without points gives -1 in [0] or [1] and adds 0 to
 *               [3] and [4].
 * Both handles must be on one device.  Enqueues two point-set distances and
 * one small kernel on `stream`; the two reductions are kept in a's scratch
 * of that stream (80 bytes). */
int32_t p2m_mesh_distance(p2m_handle a, p2m_handle b, const float* d_points_a, int64_t n_a,
                          const float* d_points_b, int64_t n_b, double* d_out, void* stream);

/* The two halves of p2m_query, for callers that sort once and query several
 * times (or time the search kernel alone).
 * p2m_sort_points: writes to d_order (device, n int32) the order in which
 *   p2m_query visits the points: by the Morton code of each point's cell in a
 *   2^k-per-axis grid over the mesh box x1.25, points outside the domain box
 *   last; and, if d_sorted_points (device, n x 3, nullable) is given, the
 *   points themselves in that order.  Uses the handle's workspace (same
 *   concurrency rule as p2m_query).
 * p2m_query_ordered: the search of p2m_query, reading the caller's
 *   d_points and visiting point d_order[j] at thread j (d_order a permutation
 *   of 0..n-1, or NULL for 0..n-1); outputs are indexed like d_points.
 *   p2m_query is p2m_sort_points followed by p2m_query_ordered.
 * p2m_query_sorted: the same search on points already in visiting order
 *   (d_sorted_points[j] = d_points[d_order[j]], e.g. kept from an earlier
 *   sort); the outputs for point j go to position d_order[j] (or j if
 *   d_order is NULL). */
int32_t p2m_sort_points(p2m_handle h, const float* d_points, int64_t n, int32_t* d_order,
                        float* d_sorted_points, void* stream);
int32_t p2m_query_sorted(p2m_handle h, const float* d_sorted_points, const int32_t* d_order, int64_t n,
                         float* d_out_dist, int32_t* d_out_tri, float* d_out_closest, void* stream);
int32_t p2m_query_ordered(p2m_handle h, const float* d_points, const int32_t* d_order, int64_t n,
                          float* d_out_dist, int32_t* d_out_tri, float* d_out_closest,
                          void* stream);

/* Gradient of L = sum_i g_i d_i (not in the paper; envelope theorem):
 *   dL/dq_i = g_i (q_i - p_i) / d_i;
 *   dL/dv_k += -g_i lambda_k (q_i - p_i) / d_i for the 3 vertices of tri_i,
 * with lambda the barycentrics of the closest point p_i; 0 when d_i = 0.
 * p_i, d_i and lambda are recomputed exactly (FP64 from the float32 inputs)
 * for the triangle d_tri[i], as the forward computed them for its winner:
 * the forward's rounded closest point and distance would give the direction
 * (q - p) / d only to about 1e-7 / d (norm-wise 2.5e-3 on 4M near-surface
 * points, measured), so they are not inputs.
 *   d_tri:           device, n int32: the forward's triangle ids
 *   d_grad_dist:     device, n float32
 *   d_grad_points:   device, n x 3 float32 (nullable), overwritten
 *   d_grad_vertices: device, n_vertices x 3 float32 (nullable), accumulated
 *                    with float32 atomics (caller zeroes it) */
int32_t p2m_query_backward(p2m_handle h, const float* d_points, int64_t n, const int32_t* d_tri,
                           const float* d_grad_dist, float* d_grad_points, float* d_grad_vertices,
                           void* stream);

/* p2m_query_backward visiting the points in the caller's order (nullable:
 * input order), e.g. the d_order p2m_sort_points wrote for the forward pass,
 * so that the points are sorted once for both passes.  d_order must be a
 * permutation of [0, n) (not checked); other arguments as in
 * p2m_query_backward. */
int32_t p2m_query_backward_ordered(p2m_handle h, const float* d_points, const int32_t* d_order, int64_t n,
                                   const int32_t* d_tri, const float* d_grad_dist, float* d_grad_points,
                                   float* d_grad_vertices, void* stream);

/* Forward and backward in one pass when dL/dd is known up front.  Outputs as
 * in p2m_query and p2m_query_backward (d_out_tri and d_out_closest nullable). */
int32_t p2m_query_fused(p2m_handle h, const float* d_points, int64_t n,
                        const float* d_grad_dist, float* d_out_dist, int32_t* d_out_tri,
                        float* d_out_closest, float* d_grad_points, float* d_grad_vertices,
                        void* stream);

int32_t p2m_get_stats(p2m_handle h, p2m_stats* out);
int32_t p2m_get_query_config(p2m_handle h, p2m_query_config* out);
int32_t p2m_set_query_config(p2m_handle h, const p2m_query_config* cfg);

/* Instrumented forward (same results as p2m_query) that also accumulates,
 * into d_counters (device, 7 uint64, caller-zeroed): walk steps, adjacency
 * entries read, list entries read, exact point-triangle tests, queries
 * answered by the exact BVH fallback (points outside the domain box, and
 * walks stopped at the step cap), sum of the located site's list length,
 * walks stopped at the step cap (4,096 steps; not reached on a valid
 * Delaunay graph). */
int32_t p2m_query_counters(p2m_handle h, const float* d_points, int64_t n, float* d_out_dist,
                           int32_t* d_out_tri, float* d_out_closest,
                           unsigned long long* d_counters, void* stream);

/* p2m_query_counters that also records which items of the search structure
 * the launch reads, and writes to h_items (host, 7 int64) the number of
 * distinct items read per array: site records (32 B each), adjacency
 * entries (16 B), list spheres (16 B), list records (48 B), seed-grid cells
 * (4 B), triangle records of the fallback (48 B), fallback BVH nodes (32 B).
 * Their sum times the sizes is the structure's share of the launch's
 * compulsory bytes.  Synchronous: waits for `stream`; allocates and frees
 * one flag byte per item. */
int32_t p2m_query_touched(p2m_handle h, const float* d_points, int64_t n, float* d_out_dist,
                          int32_t* d_out_tri, float* d_out_closest, unsigned long long* d_counters,
                          int64_t* h_items, void* stream);

/* Host-side inspection of the built structure (no GPU needed).
 * p2m_host_sites: n_sites x 3 float32 positions and is-auxiliary flags
 *   (either pointer nullable); sites in device order.
 * p2m_host_site_of_vertex: n_vertices int32 site id per caller vertex (-1 if
 *   unreferenced).
 * p2m_host_list: caller triangle ids of site `site`'s list (in scan order);
 *   writes min(len, cap) ids and the full length to *len.
 * p2m_host_neighbors: Delaunay neighbours of `site` used by the locate walk.
 * p2m_host_locate: nearest site of each host point as the device walk finds
 *   it (a host replay of the walk, for testing). */
int32_t p2m_host_sites(p2m_handle h, float* out_xyz, uint8_t* out_is_aux);
int32_t p2m_host_site_of_vertex(p2m_handle h, int32_t* out);
int32_t p2m_host_list(p2m_handle h, int64_t site, int32_t* out_tris, int64_t cap, int64_t* len);
int32_t p2m_host_neighbors(p2m_handle h, int64_t site, int32_t* out, int64_t cap, int64_t* len);
int32_t p2m_host_locate(p2m_handle h, const float* points, int64_t n, int32_t* out_site);

/* Batched form (not in the paper): many meshes and query sets of uneven
 * sizes in one persistent launch, captured in a HIP graph.
 *   p2m_batch_create: meshes[n_meshes] (handles outlive the batch),
 *     h_query_counts[n_meshes] (host); autotune = 1 times candidate launch
 *     configurations on the first bind (see p2m_batch_config); cache_path
 *     (nullable) keeps the choice.  Each workgroup takes work items (a tile
 *     of one mesh's sorted queries) from a global counter and runs them
 *     through the same search as p2m_query, regroup by site included.
 *   p2m_batch_bind: device buffers for the concatenated queries of all
 *     meshes (mesh i's points follow mesh i-1's), outputs laid out the same
 *     way; d_grad_dist nullable (forward only), else d_grad_vertices[i] is
 *     mesh i's n_vertices x 3 accumulator (device, caller-zeroed, entries
 *     nullable) and d_grad_points (nullable) is n_total x 3.  Captures the
 *     graph on `stream`.
 *   p2m_batch_launch: replays the graph on `stream`. */
int32_t p2m_batch_create(const p2m_handle* meshes, int32_t n_meshes, const int64_t* h_query_counts,
                         int32_t autotune, const char* cache_path, p2m_batch* out);
int32_t p2m_batch_bind(p2m_batch b, const float* d_points, float* d_out_dist, int32_t* d_out_tri,
                       float* d_out_closest, const float* d_grad_dist, float* d_grad_points,
                       float* const* d_grad_vertices, void* stream);
int32_t p2m_batch_launch(p2m_batch b, void* stream);
/* The launch configuration in use (each output nullable): tile = queries
 * per work item, grid = persistent workgroups taking items from the queue,
 * or 0 for one workgroup per item (tile = block), block = threads per
 * workgroup, stage = LDS staging of list spheres (0/1).  With autotune, the
 * first bind times candidates (block 256 or 512; one workgroup per item, or
 * items of 2, 8 or 32 blocks for 2, 4 or 8 persistent workgroups per CU;
 * staging off or on) and keeps the fastest, cached under a key of the
 * device and every mesh's sizes. */
int32_t p2m_batch_config(p2m_batch b, int32_t* tile, int32_t* grid, int32_t* block, int32_t* stage);
/* Sets the launch configuration (same meaning as p2m_batch_config's outputs;
 * grid = 0 requires tile == block) instead of tuning; takes effect at the
 * next p2m_batch_bind. */
int32_t p2m_batch_set_config(p2m_batch b, int32_t tile, int32_t grid, int32_t block, int32_t stage);
int32_t p2m_batch_destroy(p2m_batch b);

const char* p2m_status_string(int32_t status);
const char* p2m_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* P2M_H */
