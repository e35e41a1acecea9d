// sme_host.h -- host helpers shared by the single-grid and batched front ends.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "sme_kernels.h"

namespace sme {
namespace host {

// Gauss-Legendre points on [0, 1] (weights sum to 1) by Newton's method on P_n.
inline void gauss_legendre01(int n, double *s, double *w)
{
    for (int i = 0; i < n; ++i) {
        long double x = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
        long double dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = x;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) {
                p1 = x;
                p0 = 1;
            }
            dp = n * (x * p1 - p0) / (x * x - 1);
            long double dx = p1 / dp;
            x -= dx;
            if (fabsl(dx) < 1e-30L) break;
        }
        long double p0 = 1, p1 = x;
        for (int k = 2; k <= n; ++k) {
            long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) {
            p1 = x;
            p0 = 1;
        }
        dp = n * (x * p1 - p0) / (x * x - 1);
        long double wi = 2.0L / ((1 - x * x) * dp * dp);
        s[i] = (double)(0.5L * (1.0L - x));
        w[i] = (double)(0.5L * wi);
    }
}

// compute units of the current device (256 on an MI355X)
inline int device_cus()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        return prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    return 256;
}

// Height of the row band each wave of the structured kernel marches up.
// Every band costs its rows plus about 1.5 rows of halo work, and waves run in
// generations of (compute units x 4 SIMDs x waves per SIMD); a short last
// generation costs a full band time.  Pick the height that minimises
// generations x (rows + 1.5) for this grid, level and device.
inline int pick_rows(int level, int64_t nx, int64_t ny, int cus)
{
    const int per_simd = step_2d_waves_per_simd(level);
    const int64_t slots = (int64_t)cus * 4 * per_simd;
    const int64_t nsx = (nx + 61) / 62;
    int best = 8;
    double best_cost = 1e300;
    for (int rows = 2; rows <= 64; ++rows) {
        const int64_t waves = nsx * ((ny + rows - 1) / rows);
        const int64_t gens = (waves + slots - 1) / slots;
        const double cost = (double)gens * (rows + 1.5);
        if (cost < best_cost - 1e-9) {
            best_cost = cost;
            best = rows;
        }
    }
    return best;
}

}  // namespace host
}  // namespace sme
