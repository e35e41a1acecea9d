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
// Every band costs its rows plus about 1.5 rows of halo work; N waves (strips
// x bands) run on S resident wave slots (compute units x 4 SIMDs x waves per
// SIMD).
// - In step: the waves of a generation start and end together, and a short
//   last generation costs a whole band time: cost ceil(N / S) x (rows + 1.5).
//   This holds at one wave per SIMD, and where the best such choice needs at
//   most two generations.
// - Otherwise (more generations at two or more waves per SIMD) the waves
//   drift apart, and the step costs about N / S band times plus one band at
//   the end: (N / S + 1) x (rows + 1.5).
// (Measured with warm clocks, same box, against the first rule everywhere:
// 2-5 % faster at 4096^2 levels 1, 2 and 4 and at 6144^2 level 2, 9 % at
// 8192^2 level 0; 3072^2 level 2 and every smaller grid measured keep the
// first rule's choice.)
inline int rows_by_cost(bool drift, int64_t slots, int64_t nsx, int64_t ny, int64_t *gens_out)
{
    int best = 8;
    double best_cost = 1e300;
    int64_t best_gens = 1;
    for (int rows = 2; rows <= 64; ++rows) {
        const int64_t waves = nsx * ((ny + rows - 1) / rows);
        const int64_t g = (waves + slots - 1) / slots;
        const double gens = drift ? (double)waves / (double)slots + 1.0 : (double)g;
        const double cost = gens * (rows + 1.5);
        if (cost < best_cost - 1e-9) {
            best_cost = cost;
            best = rows;
            best_gens = g;
        }
    }
    if (gens_out) *gens_out = best_gens;
    return best;
}

inline int pick_rows_for(int per_simd, int64_t nx, int64_t ny, int cus)
{
    const int64_t slots = (int64_t)cus * 4 * per_simd;
    const int64_t nsx = (nx + 61) / 62;
    int64_t gens = 1;
    const int in_step = rows_by_cost(false, slots, nsx, ny, &gens);
    if (per_simd < 2 || gens <= 2) return in_step;
    return rows_by_cost(true, slots, nsx, ny, nullptr);
}

inline int pick_rows(int level, int64_t nx, int64_t ny, int cus)
{
    return pick_rows_for(step_2d_waves_per_simd(level), nx, ny, cus);
}

}  // namespace host
}  // namespace sme
