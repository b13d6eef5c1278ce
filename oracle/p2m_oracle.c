/*
 * FP64 brute-force oracle for point-to-mesh distance.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP library.
 *
 * What it computes is the plain definition the paper's method reaches
 * exactly (Sec. 1 and Eq. (1), the distance from a point to a mesh is the
 * minimum of the point-triangle distances over all triangles; Sec. 3.4, the
 * query returns that minimum):
 *
 *     d(q)       = min_f d(q, f)
 *     tri(q)     = smallest index f attaining the minimum in FP64
 *     closest(q) = the closest point of tri(q) to q
 *
 * Point-triangle distance is found by enumerating the KKT cases of
 *     min_{s,t >= 0, s+t <= 1} |a + s e1 + t e2 - q|^2 :
 * the unconstrained minimiser over the plane when it lies inside the
 * triangle, otherwise the best of the three clamped edge projections.  A
 * triangle whose Gram determinant vanishes is treated through its edges
 * only (a degenerate triangle is the union of its edges).
 *
 * The gradient (not in the paper) follows the envelope theorem:
 *     d(q, f) = min_{lambda in simplex} |q - sum_k lambda_k v_k|,
 *     dd/dq   = (q - p) / d,   dd/dv_k = -lambda_k (q - p) / d,
 * with lambda the barycentrics of the closest point p; zero when d = 0.
 *
 * Built with -ffp-contract=off so no result depends on FMA contraction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Closest point of segment [a, b] to q.  Returns the squared distance and
 * writes the parameter t of p = a + t (b - a). */
static double seg_closest(const double q[3], const double a[3], const double b[3],
                          double p[3], double *t_out)
{
    double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double aq[3] = {q[0] - a[0], q[1] - a[1], q[2] - a[2]};
    double L = dot3(ab, ab);
    double t = 0.0;
    if (L > 0.0) {
        t = dot3(aq, ab) / L;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
    }
    double r[3];
    for (int k = 0; k < 3; ++k) {
        p[k] = a[k] + t * ab[k];
        r[k] = q[k] - p[k];
    }
    *t_out = t;
    return dot3(r, r);
}

/* Squared distance from q to triangle (a, b, c); writes the closest point
 * and its barycentrics (weights of a, b, c). */
double oracle_point_triangle_sq(const double q[3], const double a[3], const double b[3],
                                const double c[3], double p[3], double lam[3])
{
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double w[3] = {q[0] - a[0], q[1] - a[1], q[2] - a[2]};
    double g11 = dot3(e1, e1), g12 = dot3(e1, e2), g22 = dot3(e2, e2);
    double det = g11 * g22 - g12 * g12;
    if (det > 1e-30 * g11 * g22 && det > 0.0) {
        double r1 = dot3(e1, w), r2 = dot3(e2, w);
        double s = (g22 * r1 - g12 * r2) / det;
        double t = (g11 * r2 - g12 * r1) / det;
        if (s >= 0.0 && t >= 0.0 && s + t <= 1.0) {
            double r[3];
            for (int k = 0; k < 3; ++k) {
                p[k] = a[k] + s * e1[k] + t * e2[k];
                r[k] = q[k] - p[k];
            }
            lam[0] = 1.0 - s - t;
            lam[1] = s;
            lam[2] = t;
            return dot3(r, r);
        }
    }
    /* Boundary: best of the three edges, first one on ties. */
    double pe[3], te, best;
    best = seg_closest(q, a, b, p, &te);
    lam[0] = 1.0 - te; lam[1] = te; lam[2] = 0.0;
    double d = seg_closest(q, b, c, pe, &te);
    if (d < best) {
        best = d;
        memcpy(p, pe, sizeof pe);
        lam[0] = 0.0; lam[1] = 1.0 - te; lam[2] = te;
    }
    d = seg_closest(q, c, a, pe, &te);
    if (d < best) {
        best = d;
        memcpy(p, pe, sizeof pe);
        lam[0] = te; lam[1] = 0.0; lam[2] = 1.0 - te;
    }
    return best;
}

static inline void load_vertex(const float *V, int32_t i, double out[3])
{
    out[0] = (double)V[3 * (int64_t)i + 0];
    out[1] = (double)V[3 * (int64_t)i + 1];
    out[2] = (double)V[3 * (int64_t)i + 2];
}

static int set_threads(int n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
    return omp_get_max_threads();
#else
    (void)n_threads;
    return 1;
#endif
}

/* Number of threads the parallel loops below use. */
int oracle_threads(int n_threads) { return set_threads(n_threads); }

/*
 * Brute force over all triangles for each query.
 *   V: nV x 3 float32, F: nT x 3 int32 (0-based), Q: nQ x 3 float32.
 *   out_d: nQ doubles, out_tri: nQ int32 (-1 if nT == 0 or q not finite),
 *   out_p: nQ x 3 doubles (may be NULL).
 * Returns the number of threads used.
 */
int oracle_bruteforce(const float *V, int64_t nV, const int32_t *F, int64_t nT,
                      const float *Q, int64_t nQ, double *out_d, int32_t *out_tri,
                      double *out_p, int n_threads)
{
    (void)nV;
    int used = set_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nQ; ++i) {
        double q[3] = {(double)Q[3 * i + 0], (double)Q[3 * i + 1], (double)Q[3 * i + 2]};
        double best = INFINITY, bp[3] = {NAN, NAN, NAN};
        int32_t bt = -1;
        if (isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2])) {
            for (int64_t f = 0; f < nT; ++f) {
                double a[3], b[3], c[3], p[3], lam[3];
                load_vertex(V, F[3 * f + 0], a);
                load_vertex(V, F[3 * f + 1], b);
                load_vertex(V, F[3 * f + 2], c);
                double d2 = oracle_point_triangle_sq(q, a, b, c, p, lam);
                if (d2 < best) {
                    best = d2;
                    bt = (int32_t)f;
                    bp[0] = p[0]; bp[1] = p[1]; bp[2] = p[2];
                }
            }
        }
        out_d[i] = bt >= 0 ? sqrt(best) : NAN;
        out_tri[i] = bt;
        if (out_p) {
            out_p[3 * i + 0] = bp[0];
            out_p[3 * i + 1] = bp[1];
            out_p[3 * i + 2] = bp[2];
        }
    }
    return used;
}

/*
 * Distance from each query to one given triangle (tri[i]), in FP64.  Used to
 * judge a candidate triangle id and closest point against the oracle.
 *   out_d: nQ doubles; out_p, out_lam: nQ x 3 doubles (either may be NULL).
 */
void oracle_point_triangle_batch(const float *V, const int32_t *F, const float *Q,
                                 const int32_t *tri, int64_t nQ, double *out_d,
                                 double *out_p, double *out_lam)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nQ; ++i) {
        double q[3] = {(double)Q[3 * i], (double)Q[3 * i + 1], (double)Q[3 * i + 2]};
        int64_t f = tri[i];
        double a[3], b[3], c[3], p[3], lam[3];
        load_vertex(V, F[3 * f + 0], a);
        load_vertex(V, F[3 * f + 1], b);
        load_vertex(V, F[3 * f + 2], c);
        double d2 = oracle_point_triangle_sq(q, a, b, c, p, lam);
        out_d[i] = sqrt(d2);
        if (out_p) for (int k = 0; k < 3; ++k) out_p[3 * i + k] = p[k];
        if (out_lam) for (int k = 0; k < 3; ++k) out_lam[3 * i + k] = lam[k];
    }
}

/*
 * Distance from arbitrary (double) points to one triangle each; the points
 * need not be float32 (used for closest points reported in FP32 and for
 * finite-difference probes).
 */
void oracle_point_triangle_batch64(const float *V, const int32_t *F, const double *P,
                                   const int32_t *tri, int64_t n, double *out_d)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t f = tri[i];
        double a[3], b[3], c[3], p[3], lam[3];
        load_vertex(V, F[3 * f + 0], a);
        load_vertex(V, F[3 * f + 1], b);
        load_vertex(V, F[3 * f + 2], c);
        out_d[i] = sqrt(oracle_point_triangle_sq(&P[3 * i], a, b, c, p, lam));
    }
}

/*
 * Gradient of L = sum_i g_i d(q_i) given the oracle's argmin triangles.
 *   tri: nQ int32 (the triangle whose closest point defines d(q_i)),
 *   g: nQ float32 upstream gradient,
 *   out_dq: nQ x 3 doubles (overwritten; may be NULL),
 *   out_dV: nV x 3 doubles (overwritten with the sequential FP64 sum; may be NULL).
 * Queries with tri < 0 or d == 0 contribute zero.
 */
void oracle_gradient(const float *V, int64_t nV, const int32_t *F, const float *Q,
                     const int32_t *tri, const float *g, int64_t nQ, double *out_dq,
                     double *out_dV)
{
    if (out_dV) memset(out_dV, 0, sizeof(double) * 3 * (size_t)nV);
    for (int64_t i = 0; i < nQ; ++i) {
        double dq[3] = {0.0, 0.0, 0.0};
        int64_t f = tri[i];
        if (f >= 0) {
            double q[3] = {(double)Q[3 * i], (double)Q[3 * i + 1], (double)Q[3 * i + 2]};
            double a[3], b[3], c[3], p[3], lam[3];
            load_vertex(V, F[3 * f + 0], a);
            load_vertex(V, F[3 * f + 1], b);
            load_vertex(V, F[3 * f + 2], c);
            double d = sqrt(oracle_point_triangle_sq(q, a, b, c, p, lam));
            if (d > 0.0) {
                double gi = (double)g[i];
                double n[3] = {(q[0] - p[0]) / d, (q[1] - p[1]) / d, (q[2] - p[2]) / d};
                for (int k = 0; k < 3; ++k) dq[k] = gi * n[k];
                if (out_dV) {
                    for (int j = 0; j < 3; ++j) {
                        int64_t vj = F[3 * f + j];
                        for (int k = 0; k < 3; ++k) out_dV[3 * vj + k] -= gi * lam[j] * n[k];
                    }
                }
            }
        }
        if (out_dq) for (int k = 0; k < 3; ++k) out_dq[3 * i + k] = dq[k];
    }
}

/*
 * Brute-force nearest point: for each query, the index of the closest of the
 * nP points P (smallest index on exact FP64 ties) and the distance.
 */
void oracle_nearest_point(const float *P, int64_t nP, const float *Q, int64_t nQ,
                          int32_t *out_idx, double *out_d)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nQ; ++i) {
        double q[3] = {(double)Q[3 * i], (double)Q[3 * i + 1], (double)Q[3 * i + 2]};
        double best = INFINITY;
        int32_t bi = -1;
        for (int64_t j = 0; j < nP; ++j) {
            double r[3] = {q[0] - (double)P[3 * j], q[1] - (double)P[3 * j + 1],
                           q[2] - (double)P[3 * j + 2]};
            double d2 = dot3(r, r);
            if (d2 < best) {
                best = d2;
                bi = (int32_t)j;
            }
        }
        out_idx[i] = bi;
        if (out_d) out_d[i] = sqrt(best);
    }
}

/* ------------------------------------------------------------------------
 * Tier B: the same definition evaluated by an exact branch-and-bound over an
 * axis-aligned bounding-box tree of the triangles, for query sets too large
 * for the brute force.  Nothing in it departs from the definition above: a
 * subtree is skipped only when its box lies farther from q than the best
 * distance so far plus a slack (1e-12 of the mesh scale) that covers the
 * rounding of both the box distance and the triangle distances, and every
 * triangle that is evaluated goes through oracle_point_triangle_sq with the
 * rule "smaller squared distance, or equal with a smaller index, wins".
 * The result is therefore the brute force's, bit for bit: the same
 * distance, the same lowest-index triangle and the same closest point.
 * The tree is the oracle's own (median split of triangle centroids along
 * the widest axis, at most 4 triangles per leaf).
 * ---------------------------------------------------------------------- */

typedef struct {
    double lo[3], hi[3];
    int64_t a, b; /* leaf: b < 0, triangles perm[a .. a - b - 1]; inner: children a, b */
} onode;

typedef struct {
    const float *V;
    const int32_t *F;
    int64_t nT;
    onode *nodes;
    int64_t n_nodes;
    int32_t *perm;
    double *cen;  /* 3 per triangle, centroid (split key) */
    double *tv;   /* 9 per leaf slot: the triangle's vertices, in leaf order */
    double *tb;   /* 6 per leaf slot: the triangle's box (lo, hi) */
    double slack;
} otree;

static int g_sort_axis; /* used only during the (serial) build */
static const double *g_sort_cen;

static int cmp_cen(const void *x, const void *y)
{
    double a = g_sort_cen[3 * (int64_t)*(const int32_t *)x + g_sort_axis];
    double b = g_sort_cen[3 * (int64_t)*(const int32_t *)y + g_sort_axis];
    if (a < b) return -1;
    if (a > b) return 1;
    return (*(const int32_t *)x > *(const int32_t *)y) - (*(const int32_t *)x < *(const int32_t *)y);
}

static void tri_box(const otree *t, int32_t f, double lo[3], double hi[3])
{
    for (int k = 0; k < 3; ++k) {
        lo[k] = INFINITY;
        hi[k] = -INFINITY;
    }
    for (int j = 0; j < 3; ++j) {
        double v[3];
        load_vertex(t->V, t->F[3 * (int64_t)f + j], v);
        for (int k = 0; k < 3; ++k) {
            if (v[k] < lo[k]) lo[k] = v[k];
            if (v[k] > hi[k]) hi[k] = v[k];
        }
    }
}

static int64_t build_node(otree *t, int64_t first, int64_t count)
{
    int64_t me = t->n_nodes++;
    onode *n = &t->nodes[me];
    for (int k = 0; k < 3; ++k) {
        n->lo[k] = INFINITY;
        n->hi[k] = -INFINITY;
    }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = first; i < first + count; ++i) {
        double lo[3], hi[3];
        int32_t f = t->perm[i];
        tri_box(t, f, lo, hi);
        for (int k = 0; k < 3; ++k) {
            if (lo[k] < n->lo[k]) n->lo[k] = lo[k];
            if (hi[k] > n->hi[k]) n->hi[k] = hi[k];
            double c = t->cen[3 * (int64_t)f + k];
            if (c < clo[k]) clo[k] = c;
            if (c > chi[k]) chi[k] = c;
        }
    }
    if (count <= 4) {
        n->a = first;
        n->b = -count;
        return me;
    }
    int axis = 0;
    for (int k = 1; k < 3; ++k)
        if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
    g_sort_axis = axis;
    g_sort_cen = t->cen;
    qsort(t->perm + first, (size_t)count, sizeof(int32_t), cmp_cen);
    int64_t half = count / 2;
    int64_t left = build_node(t, first, half);
    int64_t right = build_node(t, first + half, count - half);
    t->nodes[me].a = left;
    t->nodes[me].b = right;
    return me;
}

/* Build the tree of mesh (V, F).  V and F must stay alive while the tree is
 * used.  Returns NULL on allocation failure. */
void *oracle_tree_build(const float *V, int64_t nV, const int32_t *F, int64_t nT)
{
    otree *t = (otree *)calloc(1, sizeof(otree));
    if (!t) return NULL;
    t->V = V;
    t->F = F;
    t->nT = nT;
    t->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nT > 0 ? nT : 1));
    t->cen = (double *)malloc(sizeof(double) * 3 * (size_t)(nT > 0 ? nT : 1));
    t->nodes = (onode *)malloc(sizeof(onode) * (size_t)(2 * nT + 1));
    t->tv = (double *)malloc(sizeof(double) * 9 * (size_t)(nT > 0 ? nT : 1));
    t->tb = (double *)malloc(sizeof(double) * 6 * (size_t)(nT > 0 ? nT : 1));
    if (!t->perm || !t->cen || !t->nodes || !t->tv || !t->tb) {
        free(t->perm);
        free(t->cen);
        free(t->nodes);
        free(t->tv);
        free(t->tb);
        free(t);
        return NULL;
    }
    double scale = 0.0;
    for (int64_t i = 0; i < nV; ++i)
        for (int k = 0; k < 3; ++k) {
            double a = fabs((double)V[3 * i + k]);
            if (a > scale) scale = a;
        }
    t->slack = 1e-12 * (scale > 0.0 ? scale : 1.0);
    for (int64_t f = 0; f < nT; ++f) {
        t->perm[f] = (int32_t)f;
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int j = 0; j < 3; ++j) s += (double)V[3 * (int64_t)F[3 * f + j] + k];
            t->cen[3 * f + k] = s / 3.0;
        }
    }
    if (nT > 0) build_node(t, 0, nT);
    for (int64_t k = 0; k < nT; ++k) {
        int32_t f = t->perm[k];
        for (int j = 0; j < 3; ++j) load_vertex(V, F[3 * (int64_t)f + j], &t->tv[9 * k + 3 * j]);
        tri_box(t, f, &t->tb[6 * k], &t->tb[6 * k + 3]);
    }
    return t;
}

void oracle_tree_free(void *h)
{
    otree *t = (otree *)h;
    if (!t) return;
    free(t->perm);
    free(t->cen);
    free(t->nodes);
    free(t->tv);
    free(t->tb);
    free(t);
}

static double box_dist2(const double q[3], const double lo[3], const double hi[3])
{
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        double d = 0.0;
        if (q[k] < lo[k]) d = lo[k] - q[k];
        else if (q[k] > hi[k]) d = q[k] - hi[k];
        s += d * d;
    }
    return s;
}

/* True when a box at squared distance lb can still hold a triangle at most
 * as far as the best squared distance so far. */
static int may_hold(double lb, double best, double slack)
{
    return best == INFINITY || sqrt(lb) <= sqrt(best) + slack;
}

/*
 * Exact distance of each query by branch-and-bound over the tree; outputs
 * as oracle_bruteforce (identical values).  Returns the threads used.
 */
int oracle_tree_query(const void *h, const float *Q, int64_t nQ, double *out_d, int32_t *out_tri,
                      double *out_p, int n_threads)
{
    const otree *t = (const otree *)h;
    int used = set_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < nQ; ++i) {
        double q[3] = {(double)Q[3 * i + 0], (double)Q[3 * i + 1], (double)Q[3 * i + 2]};
        double best = INFINITY;
        int32_t bt = -1;
        if (t->nT > 0 && isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2])) {
            int64_t stack[128];
            int sp = 0;
            stack[sp++] = 0;
            while (sp > 0) {
                const onode *n = &t->nodes[stack[--sp]];
                if (!may_hold(box_dist2(q, n->lo, n->hi), best, t->slack)) continue;
                if (n->b < 0) {
                    for (int64_t k = n->a; k < n->a - n->b; ++k) {
                        /* the triangle's own box bounds it like a node's */
                        if (!may_hold(box_dist2(q, &t->tb[6 * k], &t->tb[6 * k + 3]), best, t->slack)) continue;
                        int32_t f = t->perm[k];
                        const double *v = &t->tv[9 * k];
                        double p[3], lam[3];
                        double d2 = oracle_point_triangle_sq(q, v, v + 3, v + 6, p, lam);
                        if (d2 < best || (d2 == best && f < bt)) {
                            best = d2;
                            bt = f;
                        }
                    }
                } else {
                    /* nearer child on top of the stack */
                    const onode *na = &t->nodes[n->a], *nb = &t->nodes[n->b];
                    double la = box_dist2(q, na->lo, na->hi), lb = box_dist2(q, nb->lo, nb->hi);
                    int64_t near = la <= lb ? n->a : n->b, far = la <= lb ? n->b : n->a;
                    if (sp + 2 > 128) abort(); /* depth is about log2(nT): never reached */
                    stack[sp++] = far;
                    stack[sp++] = near;
                }
            }
        }
        double bp[3] = {NAN, NAN, NAN};
        if (bt >= 0) {
            double a[3], b[3], c[3], lam[3];
            load_vertex(t->V, t->F[3 * (int64_t)bt + 0], a);
            load_vertex(t->V, t->F[3 * (int64_t)bt + 1], b);
            load_vertex(t->V, t->F[3 * (int64_t)bt + 2], c);
            oracle_point_triangle_sq(q, a, b, c, bp, lam);
        }
        out_d[i] = bt >= 0 ? sqrt(best) : NAN;
        out_tri[i] = bt;
        if (out_p) {
            out_p[3 * i + 0] = bp[0];
            out_p[3 * i + 1] = bp[1];
            out_p[3 * i + 2] = bp[2];
        }
    }
    return used;
}
