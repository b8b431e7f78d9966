// Host FP64 geometry of the buffer library: local frames (Section 3.1,
// Eqs. 2D_transformation, rotation_axis, antisymmetric_matrix, rotation_matrix,
// 3D_transformation), frame validation, the cell cover of a buffer's check
// region (separating-axis test of the oriented check box against cell boxes) and
// the FP32 guard band.  Pure host code: callable without a GPU.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "sphbuf.h"
#include "sphbuf_internal.h"

namespace {

inline bool finite3(const double v[3]) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Rodrigues in the expanded form R = cos(t) I + sin(t) [n]x + (1 - cos(t)) n n^T,
// which equals I + S sin(t) + S^2 (1 - cos(t)) because S^2 = n n^T - I for unit n.
void rodrigues_cs(const double n[3], double c, double s, double r[9]) {
    const double omc = 1.0 - c;
    r[0] = c + omc * n[0] * n[0];
    r[1] = omc * n[0] * n[1] - s * n[2];
    r[2] = omc * n[0] * n[2] + s * n[1];
    r[3] = omc * n[1] * n[0] + s * n[2];
    r[4] = c + omc * n[1] * n[1];
    r[5] = omc * n[1] * n[2] - s * n[0];
    r[6] = omc * n[2] * n[0] - s * n[1];
    r[7] = omc * n[2] * n[1] + s * n[0];
    r[8] = c + omc * n[2] * n[2];
}

}  // namespace

extern "C" sph_status sph_rotation_2d(double theta, double rot[9]) {
    if (!rot || !std::isfinite(theta)) return SPH_ERR_ARG;
    const double c = std::cos(theta), s = std::sin(theta);
    const double q[9] = {c, s, 0.0, -s, c, 0.0, 0.0, 0.0, 1.0};
    std::copy(q, q + 9, rot);
    return SPH_OK;
}

extern "C" sph_status sph_rotation_axis_angle(const double n[3], double theta, double rot[9]) {
    if (!n || !rot || !finite3(n) || !std::isfinite(theta)) return SPH_ERR_ARG;
    const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (!(len > 0.0)) return SPH_ERR_ARG;
    const double u[3] = {n[0] / len, n[1] / len, n[2] / len};
    rodrigues_cs(u, std::cos(theta), std::sin(theta), rot);
    return SPH_OK;
}

// The local X' axis must point along dir.  Rodrigues' matrix for the axis
// e_x x dir and the angle between them rotates e_x onto dir, so it maps local
// to global; the global->local frame is its transpose (with the axis e_z this
// reproduces the 2-D matrix of Eq. 2D_transformation).
extern "C" sph_status sph_rotation_from_direction(const double dir[3], double rot[9]) {
    if (!dir || !rot || !finite3(dir)) return SPH_ERR_ARG;
    const double len = std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    if (!(len > 0.0) || !std::isfinite(len)) return SPH_ERR_ARG;
    const double d[3] = {dir[0] / len, dir[1] / len, dir[2] / len};
    const double ax[3] = {0.0, -d[2], d[1]};  // e_x x d
    const double s = std::sqrt(ax[1] * ax[1] + ax[2] * ax[2]);
    if (s == 0.0) {
        const double sgn = d[0] > 0.0 ? 1.0 : -1.0;  // -e_x: half turn about e_z
        const double q[9] = {sgn, 0.0, 0.0, 0.0, sgn, 0.0, 0.0, 0.0, 1.0};
        std::copy(q, q + 9, rot);
        return SPH_OK;
    }
    const double n[3] = {0.0, ax[1] / s, ax[2] / s};
    double r[9];
    rodrigues_cs(n, d[0], s, r);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) rot[3 * i + j] = r[3 * j + i];
    return SPH_OK;
}

extern "C" sph_status sph_check_rotation(int32_t dim, const double rot[9]) {
    if (!rot || (dim != 2 && dim != 3)) return SPH_ERR_ARG;
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(rot[i])) return SPH_ERR_ROTATION;
    const int m = dim;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            double acc = 0.0;
            for (int k = 0; k < m; ++k) acc += rot[3 * i + k] * rot[3 * j + k];
            if (std::fabs(acc - (i == j ? 1.0 : 0.0)) > 1e-9) return SPH_ERR_ROTATION;
        }
    double det;
    if (dim == 2) {
        det = rot[0] * rot[4] - rot[1] * rot[3];
    } else {
        det = rot[0] * (rot[4] * rot[8] - rot[5] * rot[7]) - rot[1] * (rot[3] * rot[8] - rot[5] * rot[6]) +
              rot[2] * (rot[3] * rot[7] - rot[4] * rot[6]);
    }
    if (std::fabs(det - 1.0) > 1e-9) return SPH_ERR_ROTATION;
    return SPH_OK;
}

namespace sphbuf {

const double kMaxBinningError = 0.25;

// Oriented box: centre, axes (rows of rot), half-extents.
struct Obb {
    int dim;
    double c[3];
    double ax[3][3];
    double h[3];
};

Obb check_box(int dim, const double origin[3], const double rot[9], const double half[3], double margin) {
    Obb b{};
    b.dim = dim;
    for (int i = 0; i < 3; ++i) {
        b.c[i] = (dim == 2 && i == 2) ? 0.0 : origin[i];
        for (int j = 0; j < 3; ++j) b.ax[i][j] = rot[3 * i + j];
        b.h[i] = (dim == 2 && i == 2) ? 0.0 : half[i] + margin;
    }
    if (dim == 2) {
        b.ax[0][2] = b.ax[1][2] = 0.0;
        b.ax[2][0] = b.ax[2][1] = 0.0;
        b.ax[2][2] = 1.0;
    }
    return b;
}

void obb_aabb(const Obb &b, double lo[3], double hi[3]) {
    for (int j = 0; j < 3; ++j) {
        double r = 0.0;
        for (int i = 0; i < 3; ++i) r += b.h[i] * std::fabs(b.ax[i][j]);
        lo[j] = b.c[j] - r;
        hi[j] = b.c[j] + r;
    }
}

// Separating-axis test between an oriented box and an axis-aligned box given by
// its corners; true when they may intersect (conservative near touching).
bool obb_aabb_overlap(const Obb &b, const double lo[3], const double hi[3]) {
    double ac[3], ah[3], t[3];
    for (int j = 0; j < 3; ++j) {
        ac[j] = 0.5 * (lo[j] + hi[j]);
        ah[j] = 0.5 * (hi[j] - lo[j]);
        t[j] = ac[j] - b.c[j];
    }
    const int m = b.dim;
    auto separated = [&](const double L[3]) {
        double proj_t = 0.0, ra = 0.0, rb = 0.0;
        for (int j = 0; j < m; ++j) {
            proj_t += L[j] * t[j];
            ra += ah[j] * std::fabs(L[j]);
        }
        for (int i = 0; i < m; ++i) {
            double d = 0.0;
            for (int j = 0; j < m; ++j) d += L[j] * b.ax[i][j];
            rb += b.h[i] * std::fabs(d);
        }
        const double slack = 1e-12 * (std::fabs(proj_t) + ra + rb);
        return std::fabs(proj_t) > ra + rb + slack;
    };
    for (int j = 0; j < m; ++j) {  // world axes
        double L[3] = {0, 0, 0};
        L[j] = 1.0;
        if (separated(L)) return false;
    }
    for (int i = 0; i < m; ++i)  // box axes
        if (separated(b.ax[i])) return false;
    if (m == 3) {
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) {
                double E[3] = {0, 0, 0};
                E[j] = 1.0;
                const double *a = b.ax[i];
                double L[3] = {E[1] * a[2] - E[2] * a[1], E[2] * a[0] - E[0] * a[2], E[0] * a[1] - E[1] * a[0]};
                const double n2 = L[0] * L[0] + L[1] * L[1] + L[2] * L[2];
                if (n2 < 1e-20) continue;  // parallel axes: covered by the face axes
                if (separated(L)) return false;
            }
    }
    return true;
}

bool obb_obb_overlap(const Obb &a, const Obb &b) {
    const int m = a.dim;
    double t[3];
    for (int j = 0; j < 3; ++j) t[j] = b.c[j] - a.c[j];
    auto radius = [&](const Obb &o, const double L[3]) {
        double r = 0.0;
        for (int i = 0; i < m; ++i) {
            double d = 0.0;
            for (int j = 0; j < m; ++j) d += L[j] * o.ax[i][j];
            r += o.h[i] * std::fabs(d);
        }
        return r;
    };
    auto separated = [&](const double L[3]) {
        double p = 0.0;
        for (int j = 0; j < m; ++j) p += L[j] * t[j];
        const double r = radius(a, L) + radius(b, L);
        return std::fabs(p) > r + 1e-12 * (std::fabs(p) + r);
    };
    for (int i = 0; i < m; ++i)
        if (separated(a.ax[i]) || separated(b.ax[i])) return false;
    if (m == 3)
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) {
                const double *u = a.ax[i], *v = b.ax[k];
                double L[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
                if (L[0] * L[0] + L[1] * L[1] + L[2] * L[2] < 1e-20) continue;
                if (separated(L)) return false;
            }
    return true;
}

// Bound, in cells, on how far the FP32 cell coordinate of a particle can lie from
// the exact one.  The kernels bin a position x (an FP32 value) by
// t = fl32(fl32(x - lo32) * ic) with lo32 = fl32(lo) and ic = fl32(1/cs), so
//   t = [(x - lo) + (lo - lo32)] / cs * (1 + d1)(1 + d2)(1 + d3),  |di| <= u,
// and |t - (x - lo)/cs| <= |lo - lo32|/cs + 3.0001 u |x - lo32|/cs.  Positions
// beyond the grid are clamped into the edge cells, whose cover extends to
// infinity, so |x - lo32|/cs <= dims + 1 + |lo - lo32|/cs is all that matters.
double binning_error_cells(int dim, const double glo[3], double cs, const int32_t dims[3]) {
    const double u = std::ldexp(1.0, -24);
    double off = 0.0, span = 0.0;
    for (int j = 0; j < dim; ++j) {
        off = std::max(off, std::fabs(glo[j] - (double)(float)glo[j]) / cs);
        span = std::max(span, (double)dims[j] + 1.0);
    }
    return off + 3.0001 * u * (span + off);
}

sph_status cover_box(int dim, const double glo[3], double cs, const int32_t dims[3], const double origin[3],
                     const double rot[9], const double half[3], double margin, CoverBox &out) {
    const Obb b = check_box(dim, origin, rot, half, margin);
    for (int i = 0; i < 3; ++i) {
        out.c[i] = b.c[i];
        out.h[i] = b.h[i];
        for (int j = 0; j < 3; ++j) out.ax[i][j] = b.ax[i][j];
        out.lo_i[i] = out.hi_i[i] = 0;
    }
    obb_aabb(b, out.blo, out.bhi);
    // Cell boxes are dilated by more than the FP32 binning error, so a particle of
    // the check region binned into a cell puts that cell in the cover; grids whose
    // error reaches a quarter cell are refused.
    const double err = binning_error_cells(dim, glo, cs, dims);
    if (!(err < kMaxBinningError)) return SPH_ERR_ARG;
    out.eps = std::max(1e-2, 1.5 * err) * cs;
    for (int j = 0; j < dim; ++j) {
        double a = std::floor((out.blo[j] - out.eps - glo[j]) / cs) - 1.0;
        double z = std::floor((out.bhi[j] + out.eps - glo[j]) / cs) + 1.0;
        a = std::max(0.0, std::min(a, (double)dims[j] - 1.0));
        z = std::max(0.0, std::min(z, (double)dims[j] - 1.0));
        out.lo_i[j] = (int)a;
        out.hi_i[j] = (int)z;
        if ((double)out.hi_i[j] - (double)out.lo_i[j] > (double)(1 << 20)) return SPH_ERR_ARG;
    }
    return SPH_OK;
}

sph_status grid_cover(int dim, const double glo[3], double cs, const int32_t dims[3], const double origin[3],
                      const double rot[9], const double half[3], double margin, std::vector<int32_t> &first,
                      std::vector<int32_t> &len) {
    first.clear();
    len.clear();
    const Obb b = check_box(dim, origin, rot, half, margin);
    CoverBox cb;
    const sph_status st = cover_box(dim, glo, cs, dims, origin, rot, half, margin, cb);
    if (st != SPH_OK) return st;
    const double *blo = cb.blo, *bhi = cb.bhi;
    const double eps = cb.eps;
    const int32_t *lo_i = cb.lo_i, *hi_i = cb.hi_i;
    const int nz = dim == 3 ? hi_i[2] - lo_i[2] + 1 : 1;
    for (int kz = 0; kz < nz; ++kz) {
        const int iz = lo_i[2] + kz;
        for (int iy = lo_i[1]; iy <= hi_i[1]; ++iy) {
            int run_start = -1;
            for (int ix = lo_i[0]; ix <= hi_i[0] + 1; ++ix) {
                bool in = false;
                if (ix <= hi_i[0]) {
                    const int idx[3] = {ix, iy, iz};
                    double clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
                    for (int j = 0; j < dim; ++j) {
                        clo[j] = glo[j] + idx[j] * cs - eps;
                        chi[j] = glo[j] + (idx[j] + 1) * cs + eps;
                        // edge cells also hold every particle beyond the grid on that side
                        if (idx[j] == 0) clo[j] = std::min(clo[j], blo[j] - cs);
                        if (idx[j] == dims[j] - 1) chi[j] = std::max(chi[j], bhi[j] + cs);
                    }
                    in = obb_aabb_overlap(b, clo, chi);
                }
                if (in && run_start < 0) run_start = ix;
                if (!in && run_start >= 0) {
                    const int64_t lin = (int64_t)run_start + (int64_t)dims[0] * ((int64_t)iy + (int64_t)dims[1] * iz);
                    first.push_back((int32_t)lin);
                    len.push_back(ix - run_start);
                    run_start = -1;
                }
            }
        }
    }
    return SPH_OK;
}

double guard_band(int dim, const double origin[3], const double half[3], double margin, double cs, double dp) {
    (void)cs;
    const double u = std::ldexp(1.0, -24);
    double r2 = 0.0, hmax = 0.0, osum = 0.0;
    for (int j = 0; j < dim; ++j) {
        const double e = half[j] + margin;
        r2 += e * e;
        hmax = std::max(hmax, e);
        osum += std::fabs(origin[j]);
    }
    // Candidates reaching the threshold tests lie inside the sphere of radius R
    // around O' (a cheaper test rejects the rest), so with a hi/lo split origin
    // |X'_fp32 - X'| <= 6u |r - O'| + u^2 |O'|_1 (recursive 3-term dot product,
    // Higham Thm 3.1); the FP32 thresholds and the comparison add u (h + delta) each.
    const double R = std::sqrt(r2) * (1.0 + 2e-4);
    const double E = 6.1 * u * R + 4.0 * u * u * osum + 2.0 * u * hmax;
    return std::max(1e-4 * dp, 2.0 * E);
}

bool check_regions_overlap(int dim, const double o1[3], const double r1[9], const double h1[3], double m1,
                           const double o2[3], const double r2[9], const double h2[3], double m2) {
    return obb_obb_overlap(check_box(dim, o1, r1, h1, m1), check_box(dim, o2, r2, h2, m2));
}

double sphere_radius(int dim, const double half[3], double margin) {
    double r2 = 0.0;
    for (int j = 0; j < dim; ++j) r2 += (half[j] + margin) * (half[j] + margin);
    return std::sqrt(r2) * (1.0 + 1e-4);
}

}  // namespace sphbuf

extern "C" sph_status sph_grid_cover(int32_t dim, const double lo[3], double cell_size, const int32_t dims[3],
                                     const double origin[3], const double rot[9], const double half[3],
                                     double margin, int32_t *run_first, int32_t *run_len, int64_t cap,
                                     int64_t *n_runs) {
    if ((dim != 2 && dim != 3) || !lo || !dims || !origin || !rot || !half || !n_runs || !(cell_size > 0.0))
        return SPH_ERR_ARG;
    std::vector<int32_t> f, l;
    sph_status st = sphbuf::grid_cover(dim, lo, cell_size, dims, origin, rot, half, margin, f, l);
    if (st != SPH_OK) return st;
    *n_runs = (int64_t)f.size();
    if ((int64_t)f.size() > cap) return SPH_ERR_ARG;
    if (!f.empty() && (!run_first || !run_len)) return SPH_ERR_ARG;
    std::copy(f.begin(), f.end(), run_first);
    std::copy(l.begin(), l.end(), run_len);
    return SPH_OK;
}

extern "C" double sph_guard_band(int32_t dim, const double origin[3], const double half[3], double margin,
                                 double cell_size, double dp) {
    if ((dim != 2 && dim != 3) || !origin || !half) return -1.0;
    return sphbuf::guard_band(dim, origin, half, margin, cell_size, dp);
}

extern "C" const char *sph_status_str(sph_status s) {
    switch (s) {
        case SPH_OK: return "ok";
        case SPH_ERR_ARG: return "invalid argument";
        case SPH_ERR_ROTATION: return "rotation is not orthonormal with determinant +1";
        case SPH_ERR_OVERLAP: return "check region overlaps another buffer's";
        case SPH_ERR_CAPACITY: return "particle capacity exceeded";
        case SPH_ERR_CFL: return "a buffer particle left its buffer's check region";
        case SPH_ERR_NONFINITE: return "non-finite particle position";
        case SPH_ERR_TOO_MANY_BUFFERS: return "too many buffers";
        case SPH_ERR_EVENTS: return "more events than max_events in one update";
        case SPH_ERR_HIP: return "HIP runtime error";
        case SPH_ERR_STATE: return "call out of order";
    }
    return "unknown status";
}
