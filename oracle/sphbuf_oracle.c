/*
 * sphbuf_oracle.c -- TEST INFRASTRUCTURE, not part of the product.
 *
 * A plain, deliberately slow FP64 CPU oracle for one update of the
 * arbitrary-positioned SPH in-/outlet buffer (arXiv 2406.16786, Section 3,
 * Algorithms 1-3).  Every particle is checked against every buffer (brute
 * force): the paper's local cell-linked lists are an efficiency device that must
 * not change the result, so the oracle does without them.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math (no FMA contraction,
 * so every FP64 expression below is evaluated exactly as written, left to right).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library; it shares no code with the GPU library.
 */
#include "sphbuf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- frames --- */

/* Eq. (2D_transformation): X' =  cos(t) (X - X_O') + sin(t) (Y - Y_O'),
 *                          Y' = -sin(t) (X - X_O') + cos(t) (Y - Y_O'),
 * theta positive anticlockwise.  Embedded in 3x3 with Z' = Z - Z_O'. */
void orc_rotation_2d(double theta, double q[9]) {
    double c = cos(theta), s = sin(theta);
    q[0] = c;    q[1] = s;   q[2] = 0.0;
    q[3] = -s;   q[4] = c;   q[5] = 0.0;
    q[6] = 0.0;  q[7] = 0.0; q[8] = 1.0;
}

/* Eq. (antisymmetric_matrix) and Eq. (rotation_matrix):
 * S = [[0, -nz, ny], [nz, 0, -nx], [-ny, nx, 0]],  R = I + S sin(t) + S^2 (1 - cos(t)). */
void orc_rodrigues(const double n[3], double theta, double r[9]) {
    double S[9] = {0.0, -n[2], n[1], n[2], 0.0, -n[0], -n[1], n[0], 0.0};
    double S2[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double acc = 0.0;
            for (int m = 0; m < 3; m++) acc += S[3 * i + m] * S[3 * m + j];
            S2[3 * i + j] = acc;
        }
    double st = sin(theta), omc = 1.0 - cos(theta);
    for (int i = 0; i < 9; i++) r[i] = ((i % 4 == 0) ? 1.0 : 0.0) + S[i] * st + S2[i] * omc;
}

/* Frame whose X' axis is the unit vector along d (Section 3.1, 3-D case).
 * Eq. (rotation_axis): n = (OX x O'X') / |OX x O'X'| with OX = e_x and O'X' = d.
 * theta is the angle between e_x and d (positive).  Rodrigues' R of Eq.
 * (rotation_matrix) is the active rotation taking e_x onto d, so the local
 * coordinate of a point along d is (R e_x).(r - O') = [R^T (r - O')]_x: the
 * global->local matrix of Eq. (3D_transformation) is read as Q = R^T.  With
 * n = e_z this Q is exactly the 2-D matrix of Eq. (2D_transformation).
 * Degenerate axis (d parallel to e_x, where the cross product vanishes):
 * d = +e_x gives Q = I; d = -e_x gives a half turn about e_z. */
int orc_rotation_from_direction(const double d[3], double q[9]) {
    double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(len > 0.0) || !isfinite(len)) return ORC_ERR_ARG;
    double u[3] = {d[0] / len, d[1] / len, d[2] / len};
    /* e_x x u = (0, -u_z, u_y) */
    double cx[3] = {0.0, -u[2], u[1]};
    double s = sqrt(cx[1] * cx[1] + cx[2] * cx[2]);
    if (s == 0.0) {
        for (int i = 0; i < 9; i++) q[i] = 0.0;
        if (u[0] > 0.0) {
            q[0] = 1.0; q[4] = 1.0; q[8] = 1.0;
        } else {
            q[0] = -1.0; q[4] = -1.0; q[8] = 1.0;
        }
        return ORC_OK;
    }
    double n[3] = {cx[0] / s, cx[1] / s, cx[2] / s};
    double theta = atan2(s, u[0]);
    double r[9];
    orc_rodrigues(n, theta, r);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) q[3 * i + j] = r[3 * j + i];
    return ORC_OK;
}

/* r' = Q (r - O'), Eq. (2D_transformation) / Eq. (3D_transformation).
 * FP64, each component summed left to right: ((q0 d0 + q1 d1) + q2 d2). */
static void local_of(int dim, const orc_buffer *b, double x, double y, double z, double lc[3]) {
    double d0 = x - b->origin[0];
    double d1 = y - b->origin[1];
    if (dim == 2) {
        lc[0] = b->rot[0] * d0 + b->rot[1] * d1;
        lc[1] = b->rot[3] * d0 + b->rot[4] * d1;
        lc[2] = 0.0;
    } else {
        double d2 = z - b->origin[2];
        lc[0] = (b->rot[0] * d0 + b->rot[1] * d1) + b->rot[2] * d2;
        lc[1] = (b->rot[3] * d0 + b->rot[4] * d1) + b->rot[5] * d2;
        lc[2] = (b->rot[6] * d0 + b->rot[7] * d1) + b->rot[8] * d2;
    }
}

void orc_local_coords(int dim, const orc_buffer *b, int64_t n, const float *x, const float *y,
                      const float *z, double *xl, double *yl, double *zl) {
    for (int64_t i = 0; i < n; i++) {
        double lc[3];
        local_of(dim, b, (double)x[i], (double)y[i], dim == 3 ? (double)z[i] : 0.0, lc);
        xl[i] = lc[0];
        yl[i] = lc[1];
        if (zl) zl[i] = lc[2];
    }
}

void orc_recycle_literal(int dim, const orc_buffer *b, const double r[3], double out[3]) {
    double lc[3];
    local_of(dim, b, r[0], r[1], dim == 3 ? r[2] : 0.0, lc);
    lc[0] = lc[0] - 2.0 * b->half[0]; /* r' - [a, 0, 0] */
    int m = dim;
    for (int j = 0; j < m; j++) {     /* Q^T (...) + O' */
        double acc = 0.0;
        for (int i = 0; i < m; i++) acc += b->rot[3 * i + j] * lc[i];
        out[j] = acc + b->origin[j];
    }
    if (dim == 2) out[2] = 0.0;
}

/* ------------------------------------------------------------ predicates --- */

/* Buffer box (Section 3.1): |X'| < a/2 and |Y'| < b/2 (and |Z'| < c/2 in 3-D). */
static int in_box(int dim, const orc_buffer *b, const double lc[3]) {
    if (!(fabs(lc[0]) < b->half[0])) return 0;
    if (!(fabs(lc[1]) < b->half[1])) return 0;
    if (dim == 3 && !(fabs(lc[2]) < b->half[2])) return 0;
    return 1;
}

/* Check region: the box dilated by the margin on every side, standing for the
 * local cell-linked lists, which reach slightly past the buffer (Section 3.1). */
static int in_check(int dim, const orc_buffer *b, const double lc[3]) {
    if (!(fabs(lc[0]) < b->half[0] + b->margin)) return 0;
    if (!(fabs(lc[1]) < b->half[1] + b->margin)) return 0;
    if (dim == 3 && !(fabs(lc[2]) < b->half[2] + b->margin)) return 0;
    return 1;
}

static void position_of(const orc_state *s, int64_t i, double r[3]) {
    r[0] = (double)s->pos[0][i];
    r[1] = (double)s->pos[1][i];
    r[2] = s->dim == 3 ? (double)s->pos[2][i] : 0.0;
}

static int valid_args(const orc_buffer *bufs, int nb, const orc_state *s) {
    if (!s || (s->dim != 2 && s->dim != 3)) return 0;
    if (nb < 0 || nb > ORC_MAX_BUFFERS || (nb > 0 && !bufs)) return 0;
    if (s->n < 0 || s->n > s->capacity) return 0;
    if (s->n_carried < 0 || s->n_carried > ORC_MAX_CARRIED) return 0;
    for (int k = 0; k < nb; k++)
        if (bufs[k].kind < ORC_INLET || bufs[k].kind > ORC_BIDIR) return 0;
    return 1;
}

static void count_labels(int nb, const orc_state *s, int64_t *n_labelled) {
    if (!n_labelled) return;
    for (int k = 0; k < nb; k++) n_labelled[k] = 0;
    for (int64_t i = 0; i < s->n; i++) {
        int32_t l = s->label[i];
        if (l >= 1 && l <= nb) n_labelled[l - 1]++;
    }
}

/* ------------------------------------------------------- identification --- */

/* Algorithm 1, first procedure (run a single time, at set-up): every particle inside the
 * box of buffer k is added to buffer k's set, i.e. receives label k. */
int orc_identify(const orc_buffer *bufs, int nb, int which, orc_state *s, int64_t *n_labelled) {
    if (!valid_args(bufs, nb, s)) return ORC_ERR_ARG;
    if (which != -1 && (which < 1 || which > nb)) return ORC_ERR_ARG;
    for (int64_t i = 0; i < s->n; i++)
        for (int c = 0; c < s->dim; c++)
            if (!isfinite(s->pos[c][i])) return ORC_ERR_NONFINITE;
    for (int64_t i = 0; i < s->n; i++) {
        double r[3], lc[3];
        position_of(s, i, r);
        for (int k = 0; k < nb; k++) {
            if (which != -1 && which != k + 1) continue;
            local_of(s->dim, &bufs[k], r[0], r[1], r[2], lc);
            if (in_box(s->dim, &bufs[k], lc)) s->label[i] = k + 1;
        }
    }
    count_labels(nb, s, n_labelled);
    return ORC_OK;
}

/* ---------------------------------------------------------------- update --- */

enum { EV_NONE = 0, EV_GEN = 1, EV_DEL = 2 };

static int cmp_i64(const void *a, const void *b) {
    const int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static void copy_particle(orc_state *s, int64_t dst, int64_t src) {
    for (int c = 0; c < s->dim; c++) s->pos[c][dst] = s->pos[c][src];
    for (int f = 0; f < s->n_carried; f++) s->carried[f][dst] = s->carried[f][src];
    s->label[dst] = s->label[src];
    s->id[dst] = s->id[src];
}

/*
 * One update, every decision taken on the input state:
 *  1. Inflow (Algorithm 1, second procedure; Algorithm 3 first branch): a particle
 *     of buffer k (label k) with X' > a/2 is duplicated, and the original is moved
 *     back one buffer length, r' <- r' - [a, 0, 0], mapped back by the inverse
 *     transform (Eqs. 2D/3D_Inverse_transformation).  That map is exactly
 *     r <- r - a d with d = Q^T e_x; it is evaluated in FP64 and rounded to FP32.
 *  2. Outflow (Algorithm 2): any particle in the check region of an outlet with
 *     X' > a/2 is deleted; at a bidirectional buffer (Algorithm 3 second branch) a
 *     particle of the buffer with X' < -a/2 is deleted.
 *  3. Relabel (Algorithms 2 and 3, second procedure): for outlets and
 *     bidirectional buffers, every surviving particle in the check region, at its
 *     post-recycle position, gets label k if it is inside the box, otherwise loses
 *     label k (other labels are left alone).
 *  Candidates of every buffer are restricted to its check region; a particle of
 *  buffer k found outside it (moved more than the margin in one step) is an
 *  error.  Layout: deleted slots below the new count are refilled in ascending
 *  order from the surviving tail, then the duplicates are appended in ascending
 *  source order with label 0 and ids next_id, next_id + 1, ...
 */
int orc_update(const orc_buffer *bufs, int nb, orc_state *s, int64_t *gen_src, int64_t *n_gen,
               int64_t *del_idx, int64_t *n_del, int64_t *n_labelled) {
    return orc_update_bc(bufs, NULL, NULL, nb, s, gen_src, n_gen, del_idx, n_del, n_labelled);
}

/* Field roles must name existing carried arrays (or be -1). */
static int valid_fields(const orc_fields *f, const orc_state *s) {
    if (!f) return 1;
    for (int c = 0; c < 3; c++)
        if (f->vel[c] < -1 || f->vel[c] >= s->n_carried) return 0;
    return f->rho >= -1 && f->rho < s->n_carried;
}

/* Density of a particle recycled at a pressure boundary, Eq. (postulate-density)
 * with the EoS p = c0^2 (rho - rho0) (Eq. state_equation). */
static float recycled_density(const orc_bc *bc) {
    return (float)(bc->rho0 + bc->p_b / (bc->c0 * bc->c0));
}

/* Event of a particle in the check region of buffer b (local coordinates lc,
 * mine: it carries the buffer's label): Algorithm 1 (inlet generation),
 * Algorithm 2 (outlet deletion), Algorithm 3 (bidirectional: both). */
static unsigned char event_of(const orc_buffer *b, int mine, const double lc[3]) {
    if (b->kind == ORC_INLET) return (mine && lc[0] > b->half[0]) ? EV_GEN : EV_NONE;
    if (b->kind == ORC_OUTLET) return lc[0] > b->half[0] ? EV_DEL : EV_NONE;
    if (mine && lc[0] > b->half[0]) return EV_GEN;
    if (mine && lc[0] < -b->half[0]) return EV_DEL;
    return EV_NONE;
}

/* Particle i against every buffer on the input state: its event and owning
 * buffer (written only when it is in order), ORC_ERR_CFL if it carries label k
 * but lies outside C_k, ORC_ERR_ARG if two check regions hold it. */
static int classify_particle(const orc_buffer *bufs, int nb, const orc_state *s, int64_t i, unsigned char *ev,
                             unsigned char *owner) {
    double r[3], lc[3];
    position_of(s, i, r);
    unsigned char e = EV_NONE, own = 0;
    for (int k = 0; k < nb; k++) {
        const orc_buffer *b = &bufs[k];
        local_of(s->dim, b, r[0], r[1], r[2], lc);
        if (!in_check(s->dim, b, lc)) {
            if (s->label[i] == k + 1) return ORC_ERR_CFL;
            continue;
        }
        if (own != 0) return ORC_ERR_ARG; /* overlapping regions */
        own = (unsigned char)(k + 1);
        e = event_of(b, s->label[i] == k + 1, lc);
    }
    ev[i] = e;
    owner[i] = own;
    return ORC_OK;
}

/* Relabel of outlets / bidirectional buffers (Algorithms 2 and 3, second
 * procedure) for one surviving particle, on its post-recycle position. */
static void relabel_particle(const orc_buffer *bufs, int nb, orc_state *s, int64_t i) {
    double r[3], lc[3];
    position_of(s, i, r);
    for (int k = 0; k < nb; k++) {
        const orc_buffer *b = &bufs[k];
        if (b->kind == ORC_INLET) continue;
        local_of(s->dim, b, r[0], r[1], r[2], lc);
        if (!in_check(s->dim, b, lc)) continue;
        if (in_box(s->dim, b, lc)) s->label[i] = k + 1;
        else if (s->label[i] == k + 1) s->label[i] = 0;
    }
}

/* Everything after the classification: index sets (ascending), capacity check,
 * duplicates (pre-recycle state), recycle, relabel of the survivors (cand: the
 * particles to relabel, NULL for all), hole refill and append. */
static int apply_events(const orc_buffer *bufs, const orc_bc *bcs, const orc_fields *fields, int nb, orc_state *s,
                        unsigned char *ev, const unsigned char *owner, const int64_t *cand, int64_t n_cand,
                        int64_t *gen_src, int64_t *n_gen, int64_t *del_idx, int64_t *n_del, int64_t *n_labelled) {
    const int dim = s->dim;
    const int64_t N = s->n;
    int64_t G = 0, D = 0;
    if (cand) {
        /* index sets from the candidates, then sorted */
        for (int64_t j = 0; j < n_cand; j++) {
            const int64_t i = cand[j];
            if (ev[i] == EV_GEN) gen_src[G++] = i;
            if (ev[i] == EV_DEL) del_idx[D++] = i;
        }
        qsort(gen_src, (size_t)G, sizeof(int64_t), cmp_i64);
        qsort(del_idx, (size_t)D, sizeof(int64_t), cmp_i64);
    } else {
        /* index sets, ascending because i runs upwards */
        for (int64_t i = 0; i < N; i++) {
            if (ev[i] == EV_GEN) gen_src[G++] = i;
            if (ev[i] == EV_DEL) del_idx[D++] = i;
        }
    }
    const int64_t Np = N - D;
    if (Np + G > s->capacity) return ORC_ERR_CAPACITY;

    /* ---- duplicates: a copy of the crossing particle's state, before recycling ---- */
    const int nf = s->n_carried;
    float *dup_pos = (float *)malloc(sizeof(float) * (size_t)(G * 3 + 1));
    float *dup_car = (float *)malloc(sizeof(float) * (size_t)(G * (nf > 0 ? nf : 1) + 1));
    for (int64_t j = 0; j < G; j++) {
        int64_t i = gen_src[j];
        for (int c = 0; c < dim; c++) dup_pos[3 * j + c] = s->pos[c][i];
        for (int f = 0; f < nf; f++) dup_car[(size_t)nf * j + f] = s->carried[f][i];
    }

    /* ---- recycle: r <- fl32(r - a d), d = first row of Q ---- */
    for (int64_t j = 0; j < G; j++) {
        int64_t i = gen_src[j];
        const orc_buffer *b = &bufs[owner[i] - 1];
        const double a = 2.0 * b->half[0];
        for (int c = 0; c < dim; c++) {
            double shift = a * b->rot[c];
            s->pos[c][i] = (float)((double)s->pos[c][i] - shift);
        }
        const orc_bc *bc = bcs ? &bcs[owner[i] - 1] : NULL;
        if (bc && bc->kind == ORC_BC_PRESSURE && fields && fields->rho >= 0)
            s->carried[fields->rho][i] = recycled_density(bc);
    }

    /* ---- relabel outlets / bidirectional buffers on post-recycle positions ---- */
    int64_t nl_cand[ORC_MAX_BUFFERS] = {0};
    if (cand) {
        /* every particle of a buffer is one of its candidates: the labelled counts
         * after the update are those of the surviving candidates */
        for (int64_t j = 0; j < n_cand; j++) {
            const int64_t i = cand[j];
            if (ev[i] == EV_DEL) continue;
            relabel_particle(bufs, nb, s, i);
            if (s->label[i] == owner[i]) nl_cand[owner[i] - 1]++;
        }
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < N; i++)
            if (ev[i] != EV_DEL) relabel_particle(bufs, nb, s, i);
    }

    /* ---- layout: refill holes below Np from the surviving tail, ascending ---- */
    {
        int64_t t = Np;
        for (int64_t j = 0; j < D; j++) {
            int64_t hole = del_idx[j];
            if (hole >= Np) break;
            while (t < N && ev[t] == EV_DEL) t++;
            copy_particle(s, hole, t);
            t++;
        }
    }

    /* ---- append duplicates: label 0, fresh ids ---- */
    for (int64_t j = 0; j < G; j++) {
        int64_t dst = Np + j;
        for (int c = 0; c < dim; c++) s->pos[c][dst] = dup_pos[3 * j + c];
        for (int f = 0; f < nf; f++) s->carried[f][dst] = dup_car[(size_t)nf * j + f];
        s->label[dst] = 0;
        s->id[dst] = s->next_id + j;
    }
    s->next_id += G;
    s->n = Np + G;

    free(dup_pos);
    free(dup_car);

    *n_gen = G;
    *n_del = D;
    if (!cand) count_labels(nb, s, n_labelled);
    else if (n_labelled)
        for (int k = 0; k < nb; k++) n_labelled[k] = nl_cand[k];
    return ORC_OK;
}

int orc_update_bc(const orc_buffer *bufs, const orc_bc *bcs, const orc_fields *fields, int nb, orc_state *s,
                  int64_t *gen_src, int64_t *n_gen, int64_t *del_idx, int64_t *n_del, int64_t *n_labelled) {
    if (!valid_args(bufs, nb, s) || !valid_fields(fields, s)) return ORC_ERR_ARG;
    const int dim = s->dim;
    const int64_t N = s->n;

    for (int64_t i = 0; i < N; i++)
        for (int c = 0; c < dim; c++)
            if (!isfinite(s->pos[c][i])) return ORC_ERR_NONFINITE;

    unsigned char *ev = (unsigned char *)calloc((size_t)(N > 0 ? N : 1), 1);
    unsigned char *owner = (unsigned char *)calloc((size_t)(N > 0 ? N : 1), 1);
    if (!ev || !owner) {
        free(ev);
        free(owner);
        return ORC_ERR_ARG;
    }

    /* ---- classification on the input state: every particle against every
     *      buffer; the error reported is that of the lowest index ---- */
    int64_t first_bad = N;
#pragma omp parallel for schedule(static) reduction(min : first_bad)
    for (int64_t i = 0; i < N; i++)
        if (classify_particle(bufs, nb, s, i, ev, owner) != ORC_OK && i < first_bad) first_bad = i;
    int status = first_bad < N ? classify_particle(bufs, nb, s, first_bad, ev, owner) : ORC_OK;
    if (status == ORC_OK)
        status = apply_events(bufs, bcs, fields, nb, s, ev, owner, NULL, 0, gen_src, n_gen, del_idx, n_del,
                              n_labelled);
    free(ev);
    free(owner);
    return status;
}

/* The paper's own method on the CPU (Section 3.1): candidates come only from
 * the cells of a cell list (cell_start, cell_idx: cell keys as in orc_cell_list
 * on a dense grid lo, inv_cs, dims) that meet the axis-aligned box around each
 * buffer's check region, widened by one cell on every side (more than the FP32
 * binning error).  A buffer particle outside its check region is caught by
 * counting: n_labelled_in[k] particles carry label k.  Same decisions, index
 * sets and layout as orc_update_bc. */
int orc_update_local(const orc_buffer *bufs, int nb, orc_state *s, const float lo[3], float inv_cs,
                     const int32_t dims[3], const int32_t *cell_start, const int32_t *cell_idx,
                     const int64_t *n_labelled_in, int64_t *gen_src, int64_t *n_gen, int64_t *del_idx,
                     int64_t *n_del, int64_t *n_labelled) {
    if (!valid_args(bufs, nb, s) || !n_labelled_in) return ORC_ERR_ARG;
    const int dim = s->dim;
    const int64_t N = s->n;
    const double cs = 1.0 / (double)inv_cs;
    unsigned char *ev = (unsigned char *)calloc((size_t)(N > 0 ? N : 1), 1);
    unsigned char *owner = (unsigned char *)calloc((size_t)(N > 0 ? N : 1), 1);
    int64_t n_cand = 0, cap = 1024;
    int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    int status = (ev && owner && cand) ? ORC_OK : ORC_ERR_ARG;
    for (int k = 0; k < nb && status == ORC_OK; k++) {
        const orc_buffer *b = &bufs[k];
        int64_t c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0}, found = 0;
        for (int j = 0; j < dim; j++) {
            double ext = 0.0;
            for (int i = 0; i < dim; i++) ext += fabs(b->rot[3 * i + j]) * (b->half[i] + b->margin);
            double a = floor((b->origin[j] - ext - (double)lo[j]) / cs) - 1.0;
            double z = floor((b->origin[j] + ext - (double)lo[j]) / cs) + 1.0;
            a = a < 0.0 ? 0.0 : (a > dims[j] - 1 ? dims[j] - 1 : a);
            z = z < 0.0 ? 0.0 : (z > dims[j] - 1 ? dims[j] - 1 : z);
            c0[j] = (int64_t)a;
            c1[j] = (int64_t)z;
        }
        for (int64_t iz = c0[2]; iz <= c1[2] && status == ORC_OK; iz++)
            for (int64_t iy = c0[1]; iy <= c1[1] && status == ORC_OK; iy++)
                for (int64_t ix = c0[0]; ix <= c1[0] && status == ORC_OK; ix++) {
                    const int64_t key = ix + (int64_t)dims[0] * (iy + (int64_t)dims[1] * iz);
                    for (int32_t t = cell_start[key]; t < cell_start[key + 1]; t++) {
                        const int64_t i = cell_idx[t];
                        double r[3], lc[3];
                        position_of(s, i, r);
                        if (!(isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]))) {
                            status = ORC_ERR_NONFINITE;
                            break;
                        }
                        local_of(dim, b, r[0], r[1], r[2], lc);
                        if (!in_check(dim, b, lc)) continue;
                        if (owner[i] != 0) {
                            status = ORC_ERR_ARG;
                            break;
                        }
                        owner[i] = (unsigned char)(k + 1);
                        found += s->label[i] == k + 1;
                        ev[i] = event_of(b, s->label[i] == k + 1, lc);
                        if (n_cand == cap) {
                            cap *= 2;
                            cand = (int64_t *)realloc(cand, sizeof(int64_t) * (size_t)cap);
                        }
                        cand[n_cand++] = i;
                    }
                }
        if (status == ORC_OK && found != n_labelled_in[k]) status = ORC_ERR_CFL;
    }
    if (status == ORC_OK)
        status = apply_events(bufs, NULL, NULL, nb, s, ev, owner, cand, n_cand, gen_src, n_gen, del_idx, n_del,
                              n_labelled);
    free(cand);
    free(ev);
    free(owner);
    return status;
}

/* Threads of the parallel loops (OpenMP; 1 when built without it); returns the
 * number the next call will use. */
int orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------- boundary conditions --- */

/* Profile factor f(Y', Z') of the velocity boundary condition (Section 4.2). */
static double profile_factor(const orc_bc *bc, const double lc[3]) {
    if (bc->profile == ORC_PROFILE_PARABOLIC_Y) {
        double q = lc[1] / bc->radius;
        return 1.0 - q * q;
    }
    if (bc->profile == ORC_PROFILE_PARABOLIC_R) {
        double r2 = lc[1] * lc[1] + lc[2] * lc[2];
        return 1.0 - r2 / (bc->radius * bc->radius);
    }
    return 1.0;
}

int orc_apply_bc(const orc_buffer *bufs, const orc_bc *bcs, const orc_fields *fields, int nb, orc_state *s) {
    if (!valid_args(bufs, nb, s) || !bcs || !fields || !valid_fields(fields, s)) return ORC_ERR_ARG;
    const int dim = s->dim;
    for (int c = 0; c < dim; c++)
        if (fields->vel[c] < 0) return ORC_ERR_ARG;
    int st = ORC_OK;
    for (int64_t i = 0; i < s->n; i++) {
        int32_t l = s->label[i];
        if (l < 1 || l > nb) continue;
        const orc_buffer *b = &bufs[l - 1];
        const orc_bc *bc = &bcs[l - 1];
        if (bc->kind == ORC_BC_NONE) continue;
        double r[3], lc[3];
        position_of(s, i, r);
        local_of(dim, b, r[0], r[1], r[2], lc);
        if (!in_check(dim, b, lc)) {
            st = ORC_ERR_CFL;
            continue;
        }
        if (bc->kind == ORC_BC_VELOCITY) {
            /* v' = (u f, 0, 0); v = Q^T v' */
            double w = bc->u * profile_factor(bc, lc);
            for (int c = 0; c < dim; c++) s->carried[fields->vel[c]][i] = (float)(b->rot[c] * w);
        } else {
            /* v <- (v . u_hat) u_hat, u_hat = Q^T e_x = first row of Q */
            double v[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < dim; c++) v[c] = (double)s->carried[fields->vel[c]][i];
            double dot = b->rot[0] * v[0] + b->rot[1] * v[1];
            if (dim == 3) dot = dot + b->rot[2] * v[2];
            for (int c = 0; c < dim; c++) s->carried[fields->vel[c]][i] = (float)(dot * b->rot[c]);
        }
    }
    return st;
}

/* y = m x for a row-major 3x3 m, each row summed left to right (two terms in 2-D). */
static void mat_vec(int dim, const double m[9], const double x[3], double y[3]) {
    for (int r = 0; r < 3; r++) {
        double acc = m[3 * r] * x[0] + m[3 * r + 1] * x[1];
        if (dim == 3) acc = acc + m[3 * r + 2] * x[2];
        y[r] = acc;
    }
}

int orc_rotate_buffer(orc_buffer *bufs, int nb, int which, const double center[3], const double m[9],
                      const orc_fields *fields, orc_state *s) {
    if (!valid_args(bufs, nb, s) || which < 1 || which > nb || !center || !m || !valid_fields(fields, s))
        return ORC_ERR_ARG;
    const int dim = s->dim;
    orc_buffer *b = &bufs[which - 1];
    int st = ORC_OK;
    for (int64_t i = 0; i < s->n; i++) {
        if (s->label[i] != which) continue;
        double r[3], lc[3];
        position_of(s, i, r);
        local_of(dim, b, r[0], r[1], r[2], lc);
        if (!in_check(dim, b, lc)) {
            st = ORC_ERR_CFL;
            continue;
        }
        double d[3] = {r[0] - center[0], r[1] - center[1], dim == 3 ? r[2] - center[2] : 0.0}, e[3];
        mat_vec(dim, m, d, e);
        for (int c = 0; c < dim; c++) s->pos[c][i] = (float)(center[c] + e[c]);
        if (fields && fields->vel[0] >= 0) {
            double v[3] = {0.0, 0.0, 0.0}, w[3];
            for (int c = 0; c < dim; c++) v[c] = fields->vel[c] >= 0 ? (double)s->carried[fields->vel[c]][i] : 0.0;
            mat_vec(dim, m, v, w);
            for (int c = 0; c < dim; c++)
                if (fields->vel[c] >= 0) s->carried[fields->vel[c]][i] = (float)w[c];
        }
    }
    /* the frame follows the body: O' <- C + m (O' - C), rows of Q <- m (rows of Q) */
    double d[3] = {b->origin[0] - center[0], b->origin[1] - center[1], dim == 3 ? b->origin[2] - center[2] : 0.0};
    double e[3];
    mat_vec(dim, m, d, e);
    for (int c = 0; c < dim; c++) b->origin[c] = center[c] + e[c];
    double q[9];
    for (int r = 0; r < 3; r++) {
        double row[3] = {b->rot[3 * r], b->rot[3 * r + 1], b->rot[3 * r + 2]}, nr[3];
        mat_vec(dim, m, row, nr);
        for (int c = 0; c < 3; c++) q[3 * r + c] = c < dim ? nr[c] : b->rot[3 * r + c];
    }
    memcpy(b->rot, q, sizeof q);
    return st;
}

/* ------------------------------------------------------------- cell list --- */

static int64_t axis_cell(float v, float lo, float inv_cs, int32_t n) {
    float f = floorf((v - lo) * inv_cs);
    if (!(f >= 0.0f)) f = 0.0f; /* also maps NaN to cell 0 */
    if (f > (float)(n - 1)) f = (float)(n - 1);
    return (int64_t)f;
}

int orc_cell_list(int dim, const float lo[3], float inv_cs, const int32_t dims[3], int64_t n, const float *x,
                  const float *y, const float *z, int32_t *cell_start, int32_t *cell_idx) {
    if (dim != 2 && dim != 3) return ORC_ERR_ARG;
    const int64_t nz = dim == 3 ? dims[2] : 1;
    const int64_t C = (int64_t)dims[0] * dims[1] * nz;
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!key) return ORC_ERR_ARG;
    for (int64_t c = 0; c <= C; c++) cell_start[c] = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t k = axis_cell(x[i], lo[0], inv_cs, dims[0]) + (int64_t)dims[0] * axis_cell(y[i], lo[1], inv_cs, dims[1]);
        if (dim == 3) k += (int64_t)dims[0] * dims[1] * axis_cell(z[i], lo[2], inv_cs, dims[2]);
        key[i] = k;
        cell_start[k + 1]++;
    }
    for (int64_t c = 0; c < C; c++) cell_start[c + 1] += cell_start[c];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(C > 0 ? C : 1));
    for (int64_t c = 0; c < C; c++) fill[c] = cell_start[c];
    for (int64_t i = 0; i < n; i++) cell_idx[fill[key[i]]++] = (int32_t)i;
    free(fill);
    free(key);
    return ORC_OK;
}

/* ------------------------------------------------------ brick-sparse grid --- */

static void cell_of(int dim, const float lo[3], float inv_cs, const int32_t dims[3], float x, float y, float z,
                    int64_t c[3]) {
    c[0] = axis_cell(x, lo[0], inv_cs, dims[0]);
    c[1] = axis_cell(y, lo[1], inv_cs, dims[1]);
    c[2] = dim == 3 ? axis_cell(z, lo[2], inv_cs, dims[2]) : 0;
}

int64_t orc_sparse_active(int dim, const float lo[3], float inv_cs, const int32_t dims[3], int blog2, int margin,
                          int64_t n, const float *x, const float *y, const float *z, unsigned char *active) {
    if ((dim != 2 && dim != 3) || blog2 < 1 || margin < 0) return -1;
    int64_t bd[3] = {1, 1, 1};
    for (int a = 0; a < dim; a++) bd[a] = (dims[a] + (1 << blog2) - 1) >> blog2;
    const int64_t nb = bd[0] * bd[1] * bd[2];
    unsigned char *occ = (unsigned char *)calloc((size_t)nb, 1);
    for (int64_t b = 0; b < nb; b++) active[b] = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t c[3];
        cell_of(dim, lo, inv_cs, dims, x[i], y[i], dim == 3 ? z[i] : 0.0f, c);
        occ[(c[0] >> blog2) + bd[0] * ((c[1] >> blog2) + bd[1] * (c[2] >> blog2))] = 1;
    }
    const int mz = dim == 3 ? margin : 0;
    for (int64_t bz = 0; bz < bd[2]; bz++)
        for (int64_t by = 0; by < bd[1]; by++)
            for (int64_t bx = 0; bx < bd[0]; bx++) {
                if (!occ[bx + bd[0] * (by + bd[1] * bz)]) continue;
                for (int64_t dz = -mz; dz <= mz; dz++)
                    for (int64_t dy = -margin; dy <= margin; dy++)
                        for (int64_t dx = -margin; dx <= margin; dx++) {
                            int64_t X = bx + dx, Y = by + dy, Z = bz + dz;
                            if (X < 0 || Y < 0 || Z < 0 || X >= bd[0] || Y >= bd[1] || Z >= bd[2]) continue;
                            active[X + bd[0] * (Y + bd[1] * Z)] = 1;
                        }
            }
    free(occ);
    int64_t na = 0;
    for (int64_t b = 0; b < nb; b++) na += active[b];
    return na;
}

int orc_cell_list_sparse(int dim, const float lo[3], float inv_cs, const int32_t dims[3], int blog2,
                         const unsigned char *active, int64_t n, const float *x, const float *y, const float *z,
                         int32_t *cell_start, int32_t *cell_idx) {
    if ((dim != 2 && dim != 3) || blog2 < 1) return ORC_ERR_ARG;
    int64_t bd[3] = {1, 1, 1};
    for (int a = 0; a < dim; a++) bd[a] = (dims[a] + (1 << blog2) - 1) >> blog2;
    const int64_t nb = bd[0] * bd[1] * bd[2];
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
    int64_t na = 0;
    for (int64_t b = 0; b < nb; b++) slot[b] = active[b] ? na++ : -1;
    const int64_t per = (int64_t)1 << (dim * blog2), mask = (1 << blog2) - 1;
    const int64_t C = na * per + 1; /* the last key is the overflow cell */
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t c = 0; c <= C; c++) cell_start[c] = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t c[3];
        cell_of(dim, lo, inv_cs, dims, x[i], y[i], dim == 3 ? z[i] : 0.0f, c);
        int64_t s = slot[(c[0] >> blog2) + bd[0] * ((c[1] >> blog2) + bd[1] * (c[2] >> blog2))];
        int64_t local = (c[0] & mask) + ((c[1] & mask) << blog2) + ((c[2] & mask) << (2 * blog2));
        key[i] = s < 0 ? na * per : s * per + local;
        cell_start[key[i] + 1]++;
    }
    for (int64_t c = 0; c < C; c++) cell_start[c + 1] += cell_start[c];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)C);
    for (int64_t c = 0; c < C; c++) fill[c] = cell_start[c];
    for (int64_t i = 0; i < n; i++) cell_idx[fill[key[i]]++] = (int32_t)i;
    free(fill);
    free(key);
    free(slot);
    return ORC_OK;
}

/* ------------------------------------------------------ neighbour search -- */

void orc_neighbor_count(int dim, int64_t n, const float *x, const float *y, const float *z, double radius,
                        const int64_t *query, int64_t nq, int32_t *counts) {
    const double r2 = radius * radius;
    for (int64_t k = 0; k < nq; k++) {
        const int64_t q = query ? query[k] : k;
        int32_t c = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == q) continue;
            const double dx = (double)x[q] - (double)x[j];
            const double dy = (double)y[q] - (double)y[j];
            double d2 = dx * dx + dy * dy;
            if (dim == 3) {
                const double dz = (double)z[q] - (double)z[j];
                d2 = d2 + dz * dz;
            }
            if (d2 < r2) c++;
        }
        counts[k] = c;
    }
}
