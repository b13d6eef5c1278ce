/* A plain C99 client of the library: builds a host-only handle for a cube
 * and checks, without a GPU, that the header works from C and that the
 * calls behave as it states.  Prints "ok" and exits 0 on success. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "p2m.h"

#define CHECK(c, msg) do { if (!(c)) { fprintf(stderr, "FAIL: %s (%s)\n", msg, p2m_last_error()); return 1; } } while (0)

int main(void)
{
    const float V[8][3] = {{-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {-1, 1, 1},
                           {1, -1, -1},  {1, -1, 1},  {1, 1, -1},  {1, 1, 1}};
    const int32_t F[12][3] = {{0, 1, 3}, {0, 3, 2}, {4, 6, 7}, {4, 7, 5}, {0, 4, 5}, {0, 5, 1},
                              {2, 3, 7}, {2, 7, 6}, {0, 2, 6}, {0, 6, 4}, {1, 5, 7}, {1, 7, 3}};
    p2m_mesh_desc mesh = {&V[0][0], 8, &F[0][0], 12};
    p2m_build_opts opts;
    p2m_default_opts(&opts);
    CHECK(opts.domain_scale == 10.0f && opts.augment == 1 && opts.device == -2, "defaults");
    opts.device = -1; /* host only: no GPU needed */
    p2m_handle h = NULL;
    CHECK(p2m_build(&mesh, &opts, &h) == P2M_OK && h != NULL, "build");

    p2m_stats st;
    CHECK(p2m_get_stats(h, &st) == P2M_OK, "stats");
    CHECK(st.n_triangles == 12 && st.n_vertices == 8 && st.n_vertex_sites == 8, "stats values");
    CHECK(st.list_nnz >= 8 * 3, "every vertex lists its incident triangles");

    /* points near each corner are located at that corner's site */
    int32_t sov[8];
    CHECK(p2m_host_site_of_vertex(h, sov) == P2M_OK, "site_of_vertex");
    for (int v = 0; v < 8; ++v) {
        const float p[3] = {1.5f * V[v][0], 1.5f * V[v][1], 1.5f * V[v][2]};
        int32_t s = -7;
        CHECK(p2m_host_locate(h, p, 1, &s) == P2M_OK && s == sov[v], "locate");
        int64_t len = 0;
        CHECK(p2m_host_list(h, s, NULL, 0, &len) == P2M_OK && len >= 3, "list length");
    }

    /* query calls refuse a host-only handle; bad arguments are refused */
    float d = 0.f;
    const float q[3] = {0.f, 0.f, 2.f};
    CHECK(p2m_query(h, q, 1, &d, NULL, NULL, NULL) == P2M_ERR_NO_DEVICE, "host-only query refused");
    CHECK(strlen(p2m_status_string(P2M_ERR_NO_DEVICE)) > 0, "status string");
    CHECK(p2m_build(NULL, &opts, &h) == P2M_ERR_INVALID_ARG, "null mesh refused");
    const int32_t bad[3] = {0, 1, 8};
    p2m_mesh_desc badmesh = {&V[0][0], 8, bad, 1};
    p2m_handle h2 = NULL;
    CHECK(p2m_build(&badmesh, &opts, &h2) == P2M_ERR_BAD_MESH && h2 == NULL, "out-of-range index refused");
    CHECK(strlen(p2m_last_error()) > 0, "last error message");

    CHECK(p2m_destroy(h) == P2M_OK, "destroy");
    printf("ok\n");
    return 0;
}
