/*
 * Test driver (host only): runs every oracle entry point on small seeded cases so
 * that a build with AddressSanitizer and UndefinedBehaviorSanitizer checks the
 * oracle's memory accesses and arithmetic.  Exit status 0 and "ok" on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sphbuf_oracle.h"

static unsigned long long rng = 88172645463325252ull;
static double urand(void) { /* xorshift64, uniform in [0, 1) */
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) / 9007199254740992.0;
}

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                   \
        }                                                               \
    } while (0)

static int channel(int dim) {
    const double dp = 0.05;
    const int64_t nx = 40, ny = 8, nz = dim == 3 ? 8 : 1;
    const int64_t n0 = nx * ny * nz, cap = n0 + 400;
    orc_state s;
    memset(&s, 0, sizeof(s));
    s.dim = dim;
    s.n_carried = 4;
    s.capacity = cap;
    for (int c = 0; c < 3; c++) s.pos[c] = (float *)calloc((size_t)cap, sizeof(float));
    for (int f = 0; f < s.n_carried; f++) s.carried[f] = (float *)calloc((size_t)cap, sizeof(float));
    s.label = (int32_t *)calloc((size_t)cap, sizeof(int32_t));
    s.id = (int64_t *)calloc((size_t)cap, sizeof(int64_t));
    int64_t i = 0;
    for (int64_t kz = 0; kz < nz; kz++)
        for (int64_t ky = 0; ky < ny; ky++)
            for (int64_t kx = 0; kx < nx; kx++, i++) {
                s.pos[0][i] = (float)((kx + 0.5 + 0.3 * (urand() - 0.5)) * dp);
                s.pos[1][i] = (float)((ky + 0.5 + 0.3 * (urand() - 0.5)) * dp);
                if (dim == 3) s.pos[2][i] = (float)((kz + 0.5 + 0.3 * (urand() - 0.5)) * dp);
                s.carried[3][i] = 1000.0f;
                s.id[i] = i;
            }
    s.n = n0;
    s.next_id = n0;
    const double wy = ny * dp, wz = nz * dp, L = nx * dp;
    orc_buffer b[2];
    memset(b, 0, sizeof(b));
    b[0].kind = ORC_INLET;
    b[1].kind = ORC_OUTLET;
    const double d_in[3] = {1.0, 0.0, 0.0};
    CHECK(orc_rotation_from_direction(d_in, b[0].rot) == ORC_OK);
    CHECK(orc_rotation_from_direction(d_in, b[1].rot) == ORC_OK);
    for (int k = 0; k < 2; k++) {
        b[k].half[0] = 2.0 * dp;
        b[k].half[1] = 0.5 * wy + dp;
        b[k].half[2] = dim == 3 ? 0.5 * wz + dp : 0.0;
        b[k].margin = 2.6 * dp;
        b[k].origin[1] = 0.5 * wy;
        b[k].origin[2] = dim == 3 ? 0.5 * wz : 0.0;
    }
    b[0].origin[0] = 2.0 * dp;
    b[1].origin[0] = L - 2.0 * dp;
    int64_t nl[ORC_MAX_BUFFERS];
    CHECK(orc_identify(b, 2, -1, &s, nl) == ORC_OK);
    orc_bc bcs[2];
    memset(bcs, 0, sizeof(bcs));
    bcs[0].kind = ORC_BC_VELOCITY;
    bcs[0].profile = dim == 3 ? ORC_PROFILE_PARABOLIC_R : ORC_PROFILE_PARABOLIC_Y;
    bcs[0].u = 1.0;
    bcs[0].radius = 0.5 * wy;
    bcs[1].kind = ORC_BC_PRESSURE;
    bcs[1].p_b = 10.0;
    bcs[1].rho0 = 1000.0;
    bcs[1].c0 = 10.0;
    orc_fields fields = {{0, 1, dim == 3 ? 2 : -1}, 3};
    int64_t *gen = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    int64_t *del = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    int64_t total_g = 0, total_d = 0;
    for (int step = 0; step < 60; step++) {
        for (int64_t p = 0; p < s.n; p++) s.pos[0][p] += (float)(0.25 * dp * (1.0 + 0.05 * (urand() - 0.5)));
        int64_t ng = 0, nd = 0;
        const int st = orc_update_bc(b, bcs, &fields, 2, &s, gen, &ng, del, &nd, nl);
        CHECK(st == ORC_OK);
        total_g += ng;
        total_d += nd;
        CHECK(orc_apply_bc(b, bcs, &fields, 2, &s) == ORC_OK);
    }
    CHECK(total_g > 0 && total_d > 0);
    CHECK(s.n == n0 + total_g - total_d);
    /* a small turn of the inlet about its own origin */
    double m[9];
    orc_rotation_2d(0.01, m);
    const double center[3] = {b[0].origin[0], b[0].origin[1], b[0].origin[2]};
    const int rs = orc_rotate_buffer(b, 2, 1, center, m, &fields, &s);
    CHECK(rs == ORC_OK || rs == ORC_ERR_CFL);
    /* local coordinates, literal recycle, Rodrigues */
    double *xl = (double *)malloc(sizeof(double) * (size_t)s.n);
    double *yl = (double *)malloc(sizeof(double) * (size_t)s.n);
    double *zl = (double *)malloc(sizeof(double) * (size_t)s.n);
    orc_local_coords(dim, &b[1], s.n, s.pos[0], s.pos[1], s.pos[2], xl, yl, zl);
    double r[3] = {0.3, 0.2, 0.1}, out[3];
    orc_recycle_literal(dim, &b[0], r, out);
    const double axis[3] = {0.0, 0.6, 0.8};
    double R[9];
    orc_rodrigues(axis, 0.3, R);
    /* cell lists, dense and brick-sparse, and the neighbour search */
    const float lo[3] = {-0.1f, -0.1f, -0.1f};
    const float inv = (float)(1.0 / (2.6 * dp));
    const int32_t dims[3] = {20, 6, dim == 3 ? 6 : 1};
    const int64_t C = (int64_t)dims[0] * dims[1] * dims[2];
    int32_t *cs = (int32_t *)malloc(sizeof(int32_t) * (size_t)(C + 2));
    int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(s.n > 0 ? s.n : 1));
    CHECK(orc_cell_list(dim, lo, inv, dims, s.n, s.pos[0], s.pos[1], s.pos[2], cs, ci) == ORC_OK);
    CHECK(cs[C] == (int32_t)s.n);
    const int blog2 = 2;
    const int64_t bd0 = (dims[0] + 3) >> 2, bd1 = (dims[1] + 3) >> 2, bd2 = dim == 3 ? (dims[2] + 3) >> 2 : 1;
    unsigned char *act = (unsigned char *)calloc((size_t)(bd0 * bd1 * bd2), 1);
    const int64_t na = orc_sparse_active(dim, lo, inv, dims, blog2, 1, s.n, s.pos[0], s.pos[1], s.pos[2], act);
    CHECK(na > 0);
    const int64_t cells = na * (dim == 3 ? 64 : 16) + 1;
    int32_t *css = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cells + 1));
    CHECK(orc_cell_list_sparse(dim, lo, inv, dims, blog2, act, s.n, s.pos[0], s.pos[1], s.pos[2], css, ci) ==
          ORC_OK);
    int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(s.n > 0 ? s.n : 1));
    orc_neighbor_count(dim, s.n, s.pos[0], s.pos[1], s.pos[2], 2.6 * dp, NULL, s.n, cnt);
    int64_t q[3] = {0, s.n / 2, s.n - 1};
    int32_t cq[3];
    orc_neighbor_count(dim, s.n, s.pos[0], s.pos[1], s.pos[2], 2.6 * dp, q, 3, cq);
    CHECK(cq[0] == cnt[0] && cq[1] == cnt[s.n / 2] && cq[2] == cnt[s.n - 1]);
    free(cnt);
    free(css);
    free(act);
    free(ci);
    free(cs);
    free(xl);
    free(yl);
    free(zl);
    free(gen);
    free(del);
    for (int c = 0; c < 3; c++) free(s.pos[c]);
    for (int f = 0; f < s.n_carried; f++) free(s.carried[f]);
    free(s.label);
    free(s.id);
    printf("dim %d: %lld generated, %lld deleted, N = %lld\n", dim, (long long)total_g, (long long)total_d,
           (long long)s.n);
    return 0;
}

int main(void) {
    if (channel(2) || channel(3)) return 1;
    printf("ok\n");
    return 0;
}
