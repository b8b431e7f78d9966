// Internal declarations shared by the host geometry and the HIP translation unit.
#pragma once
#include <cstdint>
#include <vector>

#include "sphbuf.h"

namespace sphbuf {

struct Obb;

// Where a check region's cover is searched: the oriented check box (centre,
// axes as rows, half-extents), its axis-aligned box, the dilation of the cell
// boxes and the inclusive cell ranges per axis.
struct CoverBox {
    double c[3];
    double ax[3][3];
    double h[3];
    double blo[3], bhi[3];
    double eps;
    int32_t lo_i[3], hi_i[3];
};
sph_status cover_box(int dim, const double glo[3], double cs, const int32_t dims[3], const double origin[3],
                     const double rot[9], const double half[3], double margin, CoverBox &out);
sph_status grid_cover(int dim, const double glo[3], double cs, const int32_t dims[3], const double origin[3],
                      const double rot[9], const double half[3], double margin, std::vector<int32_t> &first,
                      std::vector<int32_t> &len);
// FP32 cell binning: bound on the error of a cell coordinate (in cells), and the
// largest bound a grid may have (the cover dilates cell boxes by 1.5 times it).
double binning_error_cells(int dim, const double glo[3], double cs, const int32_t dims[3]);
extern const double kMaxBinningError;
double guard_band(int dim, const double origin[3], const double half[3], double margin, double cs, double dp);
double sphere_radius(int dim, const double half[3], double margin);
bool check_regions_overlap(int dim, const double o1[3], const double r1[9], const double h1[3], double m1,
                           const double o2[3], const double r2[9], const double h2[3], double m2);

// Per-buffer record read by the kernels.  FP32 members drive the bulk test; the
// FP64 members reproduce the exact FP64 decision inside the guard band.
struct BufDev {
    float qf[9];      // rotation, FP32
    float ohi[3];     // origin, FP32 high part
    float olo[3];     // origin, FP32 low part (origin - ohi)
    float thrf[6];    // FP32 thresholds: a/2, b/2, c/2, a/2 + d, b/2 + d, c/2 + d
    float guard;      // FP32 guard band
    float rsq;        // squared radius of a sphere around O' holding the check region
    int32_t kind;     // SPH_INLET / SPH_OUTLET / SPH_BIDIR
    int32_t pad_[3];
    double q[9];      // rotation, FP64
    double o[3];      // origin, FP64
    double thr[6];    // FP64 thresholds, same order as thrf
    double shift[3];  // recycle shift a d = (2 * a/2) * q[0..2], FP64
    int32_t bc_kind;  // SPH_BC_NONE / SPH_BC_VELOCITY / SPH_BC_PRESSURE
    int32_t profile;  // velocity BC: SPH_PROFILE_*
    float rho_rec;    // pressure BC: density of a recycled particle, fl32(rho0 + p_b / c0^2)
    int32_t pad2_;
    double bc_u;      // velocity BC: speed scale of the profile along X'
    double bc_radius; // velocity BC: radius R of the parabolic profiles
    float bmin[3];    // axis-aligned box holding the check region, rounded outward in FP32
    float bmax[3];    // (+-inf on the axes a 2-D domain does not have)
};

}  // namespace sphbuf
