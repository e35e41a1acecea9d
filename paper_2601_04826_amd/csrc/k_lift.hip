// k_lift.hip -- 3D lifting of an SME state (the interpolate_3d postprocessing).
//
// For every cell and sigma level zeta_l in [0, 1] the kernel writes the
// elevation z = b + zeta h, the velocity profile u = sum_k alpha_k phi_k(zeta)
// (v likewise with beta_k), the vertical velocity from incompressibility and
// the kinematic bed condition,
//     w = -sum_k (d_x qx_k + d_y qy_k) Phi_k(zeta) + u (d_x b + zeta d_x h) + v (d_y b + zeta d_y h),
// and the hydrostatic pressure p = rho g h (1 - zeta) (Sec. 2.2.1
// postprocessing; the level-0 case is the printed SWE lifting of Sec. 3.1).
// Horizontal derivatives are least-squares gradients over the face neighbours
// inside the domain (compute_derivatives, Sec. 2.1.2): on uniform grids the
// normal matrix is diagonal (central differences inside, one-sided at a wall
// or open end); on triangles a 2x2 solve from the centroid displacements, the
// minimum-norm gradient d (d . grad) / |d|^2 for a cell with one neighbour.
// phi_k(zeta) = P_k(x), x = 1 - 2 zeta, by Bonnet's recurrence, and
// Phi_k(zeta) = int_0^zeta phi_k = -(P_{k+1}(x) - P_{k-1}(x)) / (2 (2k + 1)) for
// k >= 1 (Phi_0 = zeta), from (2k+1) P_k = (P_{k+1} - P_{k-1})'.
// One lane per cell; the write of 5 nz values per cell dominates the traffic,
// stored as out[(var * nz + l) * ncells + cell] in the caller's cell order.
#include <hip/hip_runtime.h>

#include "sme_lift.h"
#include "sme_step_common.h"

namespace sme {

using namespace detail;

namespace {

// gradient along one axis of a uniform grid from the neighbours that exist
// (displacements -d and +d): central, one-sided or zero
__device__ __forceinline__ double axis_grad(bool lo, bool hi, double fl, double fc, double fr, double inv_d)
{
    if (lo && hi) return 0.5 * (fr - fl) * inv_d;
    if (hi) return (fr - fc) * inv_d;
    if (lo) return (fc - fl) * inv_d;
    return 0.0;
}

// neighbour index along one axis (periodic wrap), -1 if none
__device__ __forceinline__ int axis_nbr(int c, int n, int bc_lo, int bc_hi, int dir)
{
    const int m = c + dir;
    if (m < 0) return bc_lo == BC_PERIODIC ? n - 1 : -1;
    if (m >= n) return bc_hi == BC_PERIODIC ? 0 : -1;
    return m;
}

template <int N, int KIND>
__global__ __launch_bounds__(kBlock) void k_lift(LiftArgs a)
{
    constexpr int n = N + 1;
    constexpr int nv = 2 + 2 * n;  // h, b, qx_0..qx_N, qy_0..qy_N
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.ncells) return;
    auto val = [&](int v, int64_t c) -> double {
        if (v == 1) return a.b[c];
        if (v == 0) return a.q[c];
        return a.q[(int64_t)(v - 1) * a.stride + c];  // v = 2 + k -> field 1 + k
    };
    double f[nv], gx[nv], gy[nv];
#pragma unroll
    for (int v = 0; v < nv; ++v) {
        f[v] = (KIND == 1 && v >= 2 + n) ? 0.0 : val(v, i);
        gx[v] = 0.0;
        gy[v] = 0.0;
    }
    if constexpr (KIND == 1 || KIND == 2) {
        const int ix = (int)(i % a.nx), iy = (int)(i / a.nx);
        const int wl = axis_nbr(ix, a.nx, a.bc[0], a.bc[1], -1), wr = axis_nbr(ix, a.nx, a.bc[0], a.bc[1], 1);
        const double idx = a.inv_dx;
#pragma unroll
        for (int v = 0; v < nv; ++v) {
            if (KIND == 1 && v >= 2 + n) continue;
            const double fl = wl >= 0 ? val(v, (int64_t)iy * a.nx + wl) : 0.0;
            const double fr = wr >= 0 ? val(v, (int64_t)iy * a.nx + wr) : 0.0;
            gx[v] = axis_grad(wl >= 0, wr >= 0, fl, f[v], fr, idx);
        }
        if constexpr (KIND == 2) {
            const int sl = axis_nbr(iy, a.ny, a.bc[2], a.bc[3], -1), sr = axis_nbr(iy, a.ny, a.bc[2], a.bc[3], 1);
#pragma unroll
            for (int v = 0; v < nv; ++v) {
                const double fl = sl >= 0 ? val(v, (int64_t)sl * a.nx + ix) : 0.0;
                const double fr = sr >= 0 ? val(v, (int64_t)sr * a.nx + ix) : 0.0;
                gy[v] = axis_grad(sl >= 0, sr >= 0, fl, f[v], fr, a.inv_dy);
            }
        }
    } else {
        // triangles: least squares over the (up to three) interior neighbours
        const double cx = a.cx[i], cy = a.cy[i];
        double sxx = 0.0, sxy = 0.0, syy = 0.0;
        double rx[nv], ry[nv];
#pragma unroll
        for (int v = 0; v < nv; ++v) {
            rx[v] = 0.0;
            ry[v] = 0.0;
        }
        int cnt = 0;
        double d1x = 0.0, d1y = 0.0;
        for (int s = 0; s < 3; ++s) {
            const int j = a.nbr[s * a.stride + i];
            if (j < 0) continue;
            const double dx = a.cx[j] - cx, dy = a.cy[j] - cy;
            sxx = fma(dx, dx, sxx);
            sxy = fma(dx, dy, sxy);
            syy = fma(dy, dy, syy);
            d1x = dx;
            d1y = dy;
            ++cnt;
#pragma unroll
            for (int v = 0; v < nv; ++v) {
                const double df = val(v, j) - f[v];
                rx[v] = fma(dx, df, rx[v]);
                ry[v] = fma(dy, df, ry[v]);
            }
        }
        if (cnt >= 2) {
            const double idet = 1.0 / (sxx * syy - sxy * sxy);
#pragma unroll
            for (int v = 0; v < nv; ++v) {
                gx[v] = (syy * rx[v] - sxy * ry[v]) * idet;
                gy[v] = (sxx * ry[v] - sxy * rx[v]) * idet;
            }
        } else if (cnt == 1) {
            // minimum-norm solution of d . g = df: g = d df / |d|^2, and here
            // (rx, ry) = d df
            const double id2 = 1.0 / (d1x * d1x + d1y * d1y);
#pragma unroll
            for (int v = 0; v < nv; ++v) {
                gx[v] = rx[v] * id2;
                gy[v] = ry[v] * id2;
            }
        }
    }
    const double h = f[0], b = f[1];
    const double ih = 1.0 / h;
    const int64_t dst = a.to_caller ? a.to_caller[i] : i;
    const int64_t vs = (int64_t)a.nz * a.ncells;  // stride between output variables
    for (int l = 0; l < a.nz; ++l) {
        const double zeta = a.zeta[l];
        const double x = 1.0 - 2.0 * zeta;
        // P_0..P_{N+1}(x)
        double P[n + 1];
        P[0] = 1.0;
        if constexpr (n >= 1) P[1] = x;
#pragma unroll
        for (int k = 1; k < n; ++k) P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
        double u = 0.0, v = 0.0, div = 0.0;
#pragma unroll
        for (int k = 0; k < n; ++k) {
            const double Phi = k == 0 ? zeta : -(P[k + 1] - P[k - 1 < 0 ? 0 : k - 1]) / (2.0 * (2 * k + 1));
            u = fma(f[2 + k] * ih, P[k], u);
            v = fma(f[2 + n + k] * ih, P[k], v);
            div = fma(gx[2 + k] + gy[2 + n + k], Phi, div);
        }
        const double w = -div + u * fma(zeta, gx[0], gx[1]) + v * fma(zeta, gy[0], gy[1]);
        const int64_t o = (int64_t)l * a.ncells + dst;
        a.out[o] = fma(zeta, h, b);
        a.out[vs + o] = u;
        a.out[2 * vs + o] = v;
        a.out[3 * vs + o] = w;
        a.out[4 * vs + o] = a.rho_g * h * (1.0 - zeta);
    }
}

}  // namespace

hipError_t launch_lift(int level, int kind, const LiftArgs &a, hipStream_t s)
{
    if (a.ncells == 0) return hipSuccess;
    const unsigned grid = blocks_for(a.ncells);
#define LL1(N) hipLaunchKernelGGL((k_lift<N, 1>), dim3(grid), dim3(kBlock), 0, s, a)
#define LL2(N) hipLaunchKernelGGL((k_lift<N, 2>), dim3(grid), dim3(kBlock), 0, s, a)
#define LL3(N) hipLaunchKernelGGL((k_lift<N, 3>), dim3(grid), dim3(kBlock), 0, s, a)
    if (kind == 1) {
        SME_LEVEL_SWITCH(level, LL1)
    } else if (kind == 2) {
        SME_LEVEL_SWITCH(level, LL2)
    } else {
        SME_LEVEL_SWITCH(level, LL3)
    }
#undef LL1
#undef LL2
#undef LL3
    return hipGetLastError();
}

}  // namespace sme
