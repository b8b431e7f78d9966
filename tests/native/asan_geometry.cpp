// Test driver (host only): the library's host FP64 geometry (frames, frame
// validation, cell cover of check regions, guard band) on seeded random frames,
// built with AddressSanitizer and UndefinedBehaviorSanitizer.  Exit status 0 and
// "ok" on success.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "sphbuf.h"

#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                          \
        }                                                                      \
    } while (0)

int main() {
    std::mt19937_64 gen(7);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    double rot[9];
    CHECK(sph_rotation_2d(0.4, rot) == SPH_OK);
    CHECK(sph_check_rotation(2, rot) == SPH_OK);
    const double zero[3] = {0.0, 0.0, 0.0};
    CHECK(sph_rotation_from_direction(zero, rot) == SPH_ERR_ARG);
    const double bad[9] = {1, 0, 0, 0, 2, 0, 0, 0, 1};
    CHECK(sph_check_rotation(3, bad) == SPH_ERR_ROTATION);
    for (int s = SPH_OK; s <= SPH_ERR_STATE; ++s) CHECK(sph_status_str((sph_status)s) != nullptr);
    const double lo[3] = {-1.0, -1.0, -1.0};
    const double cs = 0.05;
    const int32_t dims[3] = {40, 40, 40};
    std::vector<int32_t> first(1 << 16), len(1 << 16);
    long long total = 0;
    for (int t = 0; t < 200; ++t) {
        const int dim = 2 + (t & 1);
        const double dir[3] = {U(gen), U(gen), dim == 3 ? U(gen) : 0.0};
        if (sph_rotation_from_direction(dir, rot) != SPH_OK) continue;
        if (dim == 2) CHECK(sph_rotation_2d(std::atan2(dir[1], dir[0]), rot) == SPH_OK);
        CHECK(sph_check_rotation(dim, rot) == SPH_OK);
        const double n[3] = {U(gen), U(gen), U(gen)};
        double r2[9];
        const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (nn > 1e-3) {
            const double un[3] = {n[0] / nn, n[1] / nn, n[2] / nn};
            CHECK(sph_rotation_axis_angle(un, U(gen) * 3.0, r2) == SPH_OK);
        }
        const double origin[3] = {0.6 * U(gen), 0.6 * U(gen), dim == 3 ? 0.6 * U(gen) : 0.0};
        const double half[3] = {0.1 * std::fabs(U(gen)) + 0.01, 0.2 * std::fabs(U(gen)) + 0.01,
                                dim == 3 ? 0.2 * std::fabs(U(gen)) + 0.01 : 0.0};
        int64_t nr = 0;
        // too small a run buffer first (reports the need), then a large enough one
        const sph_status small = sph_grid_cover(dim, lo, cs, dims, origin, rot, half, cs, first.data(), len.data(),
                                                1, &nr);
        CHECK(small == SPH_OK || (small == SPH_ERR_ARG && nr > 1));
        CHECK(sph_grid_cover(dim, lo, cs, dims, origin, rot, half, cs, first.data(), len.data(),
                             (int64_t)first.size(), &nr) == SPH_OK);
        CHECK(nr > 0);
        for (int64_t r = 0; r < nr; ++r) {
            CHECK(first[r] >= 0 && len[r] > 0);
            total += len[r];
        }
        const double g = sph_guard_band(dim, origin, half, cs, cs, cs / 2.6);
        CHECK(g >= 1e-4 * cs / 2.6 && std::isfinite(g));
    }
    CHECK(total > 0);
    std::printf("%lld cover cells over 200 random frames\nok\n", total);
    return 0;
}
