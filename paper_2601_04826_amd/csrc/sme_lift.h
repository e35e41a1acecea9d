// sme_lift.h -- arguments of the 3D lifting kernel (interpolate_3d postprocessing).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sme {

constexpr int kLiftMaxLevels = 64;  // sigma levels per call

struct LiftArgs {
    const double *q;          // state, SoA with `stride`, internal cell order
    const double *b;          // bathymetry, internal order
    int64_t stride;
    int64_t ncells;
    // 1D / structured
    int nx, ny;
    double inv_dx, inv_dy;
    int bc[4];
    // triangles (internal order)
    const int32_t *nbr;       // [3][stride], -1 = wall
    const double *cx, *cy;    // centroids
    const int64_t *to_caller; // internal -> caller cell (null: identity)
    // sigma levels and output
    int nz;
    double zeta[kLiftMaxLevels];
    double rho_g;             // rho * g
    double *out;              // [5][nz][ncells]: z, u, v, w, p in caller order
};

hipError_t launch_lift(int level, int kind, const LiftArgs &a, hipStream_t s);

}  // namespace sme
