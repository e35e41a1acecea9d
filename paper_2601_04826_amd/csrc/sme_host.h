// sme_host.h -- host helpers shared by the single-grid and batched front ends.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

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

}  // namespace host
}  // namespace sme
