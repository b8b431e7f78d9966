/*
 * sphbuf_oracle.h -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Plain, slow, FP64 CPU oracle for one buffer update of the arbitrary-positioned
 * SPH in-/outlet buffer of Zhang, Fan, Ren, Qian & Hu, "Generalized and
 * high-efficiency arbitrary-positioned buffer for smoothed particle
 * hydrodynamics" (arXiv 2406.16786), Section 3 and Algorithms 1-3.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  It shares no code, header, table or helper with the
 * GPU library, and the GPU library never calls it.
 *
 * Conventions (all readings of the paper are listed in the design notes):
 *   - rot is a row-major 3x3 matrix Q mapping global to local coordinates,
 *     r' = Q (r - O'); its rows are the local axes X', Y', Z' in global
 *     coordinates (Eq. 2D_transformation; Eq. 3D_transformation with Q = R^T,
 *     see orc_rotation_from_direction).
 *   - half = (a/2, b/2, c/2): buffer half-extents along X', Y', Z'.
 *   - margin = delta: the check region C = box dilated by delta on every side
 *     stands for the cell-linked lists local to the buffer of Section 3.1,
 *     which reach slightly past it.
 *   - label 0 = ordinary fluid particle, label k (1..n_buffers) = buffer k.
 */
#ifndef SPHBUF_ORACLE_H
#define SPHBUF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_ERR_ARG = 1, ORC_ERR_CAPACITY = 4, ORC_ERR_CFL = 5, ORC_ERR_NONFINITE = 6 };
enum { ORC_INLET = 1, ORC_OUTLET = 2, ORC_BIDIR = 3 };
#define ORC_MAX_BUFFERS 15
#define ORC_MAX_CARRIED 16

typedef struct {
    int32_t kind;      /* ORC_INLET / ORC_OUTLET / ORC_BIDIR                    */
    int32_t pad_;
    double origin[3];  /* O' in global coordinates                              */
    double rot[9];     /* Q, row-major, global -> local                          */
    double half[3];    /* a/2, b/2, c/2 (c ignored in 2-D)                       */
    double margin;     /* delta > 0                                              */
} orc_buffer;

typedef struct {
    int32_t dim;                      /* 2 or 3                                   */
    int32_t n_carried;                /* number of extra float fields             */
    int64_t n;                        /* live particles, updated in place         */
    int64_t capacity;                 /* length of every array                    */
    int64_t next_id;                  /* id handed to the next duplicate          */
    float *pos[3];                    /* x, y, z (z unused in 2-D)                */
    float *carried[ORC_MAX_CARRIED];  /* velocity, mass, density, pressure, ...   */
    int32_t *label;
    int64_t *id;
} orc_state;

/* Eq. (2D_transformation) embedded in 3x3: [[c, s, 0], [-s, c, 0], [0, 0, 1]]. */
void orc_rotation_2d(double theta, double q[9]);
/* Eq. (rotation_matrix): R = I + S sin(theta) + S^2 (1 - cos(theta)), S from
 * Eq. (antisymmetric_matrix).  Returns the matrix exactly as printed. */
void orc_rodrigues(const double n[3], double theta, double r[9]);
/* Global->local frame whose X' axis is the unit vector d (Eqs. rotation_axis to
 * 3D_transformation, read with Q = R^T).  Returns ORC_ERR_ARG if |d| == 0. */
int orc_rotation_from_direction(const double d[3], double q[9]);

/* FP64 local coordinates of FP32 positions, one buffer, n points. */
void orc_local_coords(int dim, const orc_buffer *b, int64_t n, const float *x, const float *y,
                      const float *z, double *xl, double *yl, double *zl);

/* Paper's literal inverse transform, r = Q^T (Q (r - O') - [a,0,0]) + O', in FP64
 * (Eqs. 2D_Inverse_transformation and 3D_Inverse_transformation). */
void orc_recycle_literal(int dim, const orc_buffer *b, const double r[3], double out[3]);

/* Buffer-particle identification (Algorithm 1, first procedure): every particle
 * inside buffer k's box gets label k.  which = buffer index 1..nb, or -1 = all.
 * n_labelled[k-1] receives the count of label k afterwards. */
int orc_identify(const orc_buffer *bufs, int nb, int which, orc_state *s, int64_t *n_labelled);

/* One buffer update (Algorithms 1-3).  gen_src / del_idx (capacity >= n) receive
 * the generated-source and deleted index sets, ascending.  On error nothing is
 * mutated and the return value says why. */
int orc_update(const orc_buffer *bufs, int nb, orc_state *s, int64_t *gen_src, int64_t *n_gen,
               int64_t *del_idx, int64_t *n_del, int64_t *n_labelled);

/* Cell-linked list of the first n particles on a dense grid of dims cells with
 * FP32 origin lo and FP32 inverse cell size inv_cs: cell index per axis is
 * floor(fl32(fl32(x - lo) * inv_cs)) clamped to [0, dims-1] (the binning
 * precision is the GPU library's own choice, so the oracle takes the same FP32
 * decision), linear key ix + dims0 * (iy + dims1 * iz).  cell_start has
 * dims0*dims1*dims2 + 1 entries (exclusive prefix counts), cell_idx n entries
 * in ascending particle order within each cell (stable counting sort). */
int orc_cell_list(int dim, const float lo[3], float inv_cs, const int32_t dims[3], int64_t n, const float *x,
                  const float *y, const float *z, int32_t *cell_start, int32_t *cell_idx);

/* Brick-sparse grid.  Bricks of 2^blog2 cells per axis cover the dense grid of
 * dims cells (cell coordinates as in orc_cell_list).  A brick is active if a
 * brick holding one of the n particles lies within Chebyshev distance margin of
 * it.  active must hold bdims0*bdims1*bdims2 bytes, bdims = ceil(dims / 2^blog2).
 * Returns the number of active bricks (or -1 on bad arguments). */
int64_t orc_sparse_active(int dim, const float lo[3], float inv_cs, const int32_t dims[3], int blog2, int margin,
                          int64_t n, const float *x, const float *y, const float *z, unsigned char *active);
/* Cell list on the brick-sparse grid: an active brick's slot is its rank among
 * active bricks in ascending brick index; its cells have keys
 * slot * 2^(dim blog2) + lx + 2^blog2 (ly + 2^blog2 lz); every cell of an
 * inactive brick has the single overflow key n_active * 2^(dim blog2).
 * cell_start has n_active * 2^(dim blog2) + 2 entries. */
int orc_cell_list_sparse(int dim, const float lo[3], float inv_cs, const int32_t dims[3], int blog2,
                         const unsigned char *active, int64_t n, const float *x, const float *y, const float *z,
                         int32_t *cell_start, int32_t *cell_idx);

/* ------------- in-/outlet boundary conditions (Section 4) and moving buffers --- */

enum { ORC_BC_NONE = 0, ORC_BC_VELOCITY = 1, ORC_BC_PRESSURE = 2 };
enum { ORC_PROFILE_PLUG = 0, ORC_PROFILE_PARABOLIC_Y = 1, ORC_PROFILE_PARABOLIC_R = 2 };

typedef struct {
    int32_t kind;      /* ORC_BC_NONE / ORC_BC_VELOCITY / ORC_BC_PRESSURE             */
    int32_t profile;   /* velocity BC: ORC_PROFILE_*                                  */
    double u;          /* velocity BC: speed scale of the profile along X'             */
    double radius;     /* velocity BC: R of the parabolic profiles                     */
    double p_b;        /* pressure BC: boundary pressure                               */
    double rho0;       /* pressure BC: reference density of the EoS                   */
    double c0;         /* pressure BC: artificial sound speed of the EoS               */
} orc_bc;

typedef struct {
    int32_t vel[3];    /* carried-field index of v_x, v_y, v_z (-1: absent)             */
    int32_t rho;       /* carried-field index of the density (-1: absent)               */
} orc_fields;

/* orc_update with the pressure boundary condition on the recycle path: a
 * particle recycled by a pressure-BC buffer takes the density
 * fl32(rho0 + p_b / (c0 c0)) (Eq. postulate-density); its duplicate keeps the
 * state before the recycle.  bcs and fields may be NULL (no boundary conditions). */
int orc_update_bc(const orc_buffer *bufs, const orc_bc *bcs, const orc_fields *fields, int nb, orc_state *s,
                  int64_t *gen_src, int64_t *n_gen, int64_t *del_idx, int64_t *n_del, int64_t *n_labelled);

/* Boundary conditions on the particles of each buffer (label k) inside its check
 * region:
 *   velocity BC (Section 4.2): the prescribed profile in the local frame,
 *     v' = (u f(Y', Z'), 0, 0), mapped to global by Q^T (Eqs. 2D/3D_velocity_profile
 *     and 2D/3D_velocity_transformation): v_c = fl32(Q[0][c] * (u * f)), with
 *     f = 1 (plug), f = 1 - (Y'/R)^2 (parabolic in Y', as printed), or
 *     f = 1 - (Y'^2 + Z'^2) / (R R) (parabolic in the radius of a pipe);
 *   pressure BC (Section 4.1): the velocity projected on the boundary normal
 *     u_hat = Q^T e_x (Eqs. velocity_correction, 2D/3D_normal_transformation):
 *     v_c = fl32((v . u_hat) u_hat_c), the dot product summed left to right.
 * Particles of a buffer found outside its check region are left alone and the
 * call returns ORC_ERR_CFL (the others are still set). */
int orc_apply_bc(const orc_buffer *bufs, const orc_bc *bcs, const orc_fields *fields, int nb, orc_state *s);

/* Rotate buffer `which` (1..nb) rigidly about `center` by the orthonormal matrix
 * m (row-major, global coordinates), as the rotating sprinkler of Section 5.3
 * turns its buffer each step: every particle of the buffer inside its check
 * region moves to r = C + m (r - C) and its velocity to m v (FP64, rounded to
 * FP32); then the buffer's frame follows, O' <- C + m (O' - C) and Q <- Q m^T,
 * so that the particle keeps its local coordinates.  Labelled particles outside
 * the check region are left alone and the call returns ORC_ERR_CFL. */
int orc_rotate_buffer(orc_buffer *bufs, int nb, int which, const double center[3], const double m[9],
                      const orc_fields *fields, orc_state *s);

/* Neighbour search by its definition, brute force over all particles (the solver's
 * search for neighbours within the kernel support 2h, Section 3): for each query
 * particle q = query[k], counts[k] = number of j != q, 0 <= j < n, with
 * ((dx*dx + dy*dy) + dz*dz) < radius*radius, dx = (double)x_q - (double)x_j,
 * every operation rounded in FP64 (no contraction), dz = 0 in 2-D.  query = NULL
 * queries every particle (nq = n).  O(n) per query. */
/* The paper's method on the CPU: one update with candidates gathered only from
 * the cells of a cell list (orc_cell_list on the dense grid lo, inv_cs, dims)
 * near each buffer's check region; n_labelled_in[k] is the number of particles
 * carrying label k.  Same results as orc_update.  CPU-baseline mode. */
int orc_update_local(const orc_buffer *bufs, int nb, orc_state *s, const float lo[3], float inv_cs,
                     const int32_t dims[3], const int32_t *cell_start, const int32_t *cell_idx,
                     const int64_t *n_labelled_in, int64_t *gen_src, int64_t *n_gen, int64_t *del_idx,
                     int64_t *n_del, int64_t *n_labelled);

/* Threads of the oracle's parallel loops (OpenMP over particles; the arithmetic
 * of each particle is unchanged); returns the count the next call uses. */
int orc_set_threads(int n);

void orc_neighbor_count(int dim, int64_t n, const float *x, const float *y, const float *z, double radius,
                        const int64_t *query, int64_t nq, int32_t *counts);

#ifdef __cplusplus
}
#endif
#endif
