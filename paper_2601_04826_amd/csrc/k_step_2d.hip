// k_step_2d.hip -- SME step on structured 2D grids (one launch per step).
#include <hip/hip_runtime.h>

#include "sme_step_common.h"

namespace sme {

using namespace detail;

namespace {

// ----------------------------------------------------------------------------
// Structured 2D: fields (h, qx_0..qx_N, qy_0..qy_N), cell index j * nx + i.
template <int N>
__device__ __forceinline__ void load_2d(const StepArgs &a, int64_t cell, bool mx, bool my, double &h,
                                        double &b, double *qx, double *qy)
{
    constexpr int n = N + 1;
    h = a.q[cell];
    b = a.b[cell];
#pragma unroll
    for (int k = 0; k < n; ++k) {
        double vx = a.q[(1 + k) * a.stride + cell];
        double vy = a.q[(1 + n + k) * a.stride + cell];
        qx[k] = mx ? -vx : vx;
        qy[k] = my ? -vy : vy;
    }
}

// finish one cell: predictor, friction, store, CFL ratio of the new state
template <int N>
__device__ __forceinline__ double finish_2d(const StepArgs &a, double dt, int64_t cell, bool out, double h0,
                                            const double *qx0, const double *qy0, const double *acc)
{
    constexpr int n = N + 1;
    double h = fma(-dt, acc[0], h0);
    double qx[n], qy[n];
#pragma unroll
    for (int k = 0; k < n; ++k) {
        qx[k] = fma(-dt, acc[1 + k], qx0[k]);
        qy[k] = fma(-dt, acc[1 + n + k], qy0[k]);
    }
    const double ih = rcp(h);
    friction<N>(qx, ih, dt, a.c_slip, a.nu);
    friction<N>(qy, ih, dt, a.c_slip, a.nu);
    double r = 0.0;
    if (out) {
        a.qn[cell] = h;
        bool bad = !(h > 0.0) || !isfinite(h);
#pragma unroll
        for (int k = 0; k < n; ++k) {
            a.qn[(1 + k) * a.stride + cell] = qx[k];
            a.qn[(1 + n + k) * a.stride + cell] = qy[k];
            bad |= !isfinite(qx[k]) || !isfinite(qy[k]);
        }
        flag_bad(a, bad);
        double lm;
        r = cfl_ratio_2d<N>(a.g, h, ih, qx, qy, a.idx, a.idy, &lm);
        if (!(r >= 0.0)) r = 0.0;
    }
    return r;
}

template <int N>
__global__ __launch_bounds__(kBlock) void k_step_2d(StepArgs a)
{
    constexpr int n = N + 1;
    constexpr int nf = 2 * n + 1;
    const double dt = step_dt(a);
    if (blockIdx.x == 0 && threadIdx.x == 0) slot_update(a, dt);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int nsx = (a.nx + kOut - 1) / kOut;
    const int nsy = (a.ny + a.rows - 1) / a.rows;
    if (wave >= nsx * nsy) return;
    const int sx = wave % nsx;
    const int sy = wave / nsx;
    const int c = sx * kOut - 1 + lane;
    const int j0 = sy * a.rows;
    const int j1 = min(j0 + a.rows, a.ny);
    bool mx;
    const int col = ghost_index(c, a.nx, a.bc[0], a.bc[1], mx);
    const bool outc = lane >= 1 && lane <= kOut && c < a.nx;

    // previous row, y-frame: qa = qy, qt = qx
    Side<N, true> P;
    double accP[nf];
    {
        bool my;
        const int row = ghost_index(j0 - 1, a.ny, a.bc[2], a.bc[3], my);
        double qx[n], qy[n];
        load_2d<N>(a, (int64_t)row * a.nx + col, mx, my, P.h, P.b, qx, qy);
#pragma unroll
        for (int k = 0; k < n; ++k) {
            P.qa[k] = qy[k];
            P.qt[k] = qx[k];
        }
        side_flux<N, true>(P, a.g);
    }
    double rmax = 0.0;
    for (int j = j0; j < j1; ++j) {
        Side<N, true> C;  // y-frame of the current row
        double qx[n], qy[n];
        load_2d<N>(a, (int64_t)j * a.nx + col, mx, false, C.h, C.b, qx, qy);
#pragma unroll
        for (int k = 0; k < n; ++k) {
            C.qa[k] = qy[k];
            C.qt[k] = qx[k];
        }
        side_flux<N, true>(C, a.g);
        double Fh[nf], D[nf], accC[nf];
        face_flux<N, true>(P, C, a.g, a.quad, Fh, D);
        // frame [h, y.., x..] -> physical [h, x.., y..]
        if (j > j0) {
            accP[0] = fma(a.idy, fma(0.5, D[0], Fh[0]), accP[0]);
#pragma unroll
            for (int k = 0; k < n; ++k) {
                accP[1 + n + k] = fma(a.idy, fma(0.5, D[1 + k], Fh[1 + k]), accP[1 + n + k]);
                accP[1 + k] = fma(a.idy, fma(0.5, D[1 + n + k], Fh[1 + n + k]), accP[1 + k]);
            }
            rmax = fmax(rmax, finish_2d<N>(a, dt, (int64_t)(j - 1) * a.nx + c, outc, P.h, P.qt, P.qa, accP));
        }
        accC[0] = a.idy * fma(0.5, D[0], -Fh[0]);
#pragma unroll
        for (int k = 0; k < n; ++k) {
            accC[1 + n + k] = a.idy * fma(0.5, D[1 + k], -Fh[1 + k]);
            accC[1 + k] = a.idy * fma(0.5, D[1 + n + k], -Fh[1 + n + k]);
        }
        // x-faces of this row: x-frame qa = qx, qt = qy
        {
            Side<N, true> X;
            X.h = C.h;
            X.b = C.b;
#pragma unroll
            for (int k = 0; k < n; ++k) {
                X.qa[k] = qx[k];
                X.qt[k] = qy[k];
            }
            side_flux<N, true>(X, a.g);
            Side<N, true> R;
            R.h = shfl_dn(X.h);
            R.b = shfl_dn(X.b);
            R.Fh = shfl_dn(X.Fh);
            R.lam = shfl_dn(X.lam);
#pragma unroll
            for (int k = 0; k < n; ++k) {
                R.qa[k] = shfl_dn(X.qa[k]);
                R.qt[k] = shfl_dn(X.qt[k]);
                R.Fa[k] = shfl_dn(X.Fa[k]);
                R.Ft[k] = shfl_dn(X.Ft[k]);
            }
            double Gh[nf], E[nf];
            face_flux<N, true>(X, R, a.g, a.quad, Gh, E);
#pragma unroll
            for (int f = 0; f < nf; ++f) {
                double own = fma(0.5, E[f], Gh[f]);
                double oth = fma(0.5, E[f], -Gh[f]);
                accC[f] = fma(a.idx, own + shfl_up1(oth), accC[f]);
            }
        }
        P = C;
#pragma unroll
        for (int f = 0; f < nf; ++f) accP[f] = accC[f];
    }
    // closing y-face of the strip
    {
        bool my;
        const int row = ghost_index(j1, a.ny, a.bc[2], a.bc[3], my);
        Side<N, true> C;
        double qx[n], qy[n];
        load_2d<N>(a, (int64_t)row * a.nx + col, mx, my, C.h, C.b, qx, qy);
#pragma unroll
        for (int k = 0; k < n; ++k) {
            C.qa[k] = qy[k];
            C.qt[k] = qx[k];
        }
        side_flux<N, true>(C, a.g);
        double Fh[nf], D[nf];
        face_flux<N, true>(P, C, a.g, a.quad, Fh, D);
        accP[0] = fma(a.idy, fma(0.5, D[0], Fh[0]), accP[0]);
#pragma unroll
        for (int k = 0; k < n; ++k) {
            accP[1 + n + k] = fma(a.idy, fma(0.5, D[1 + k], Fh[1 + k]), accP[1 + n + k]);
            accP[1 + k] = fma(a.idy, fma(0.5, D[1 + n + k], Fh[1 + n + k]), accP[1 + k]);
        }
        rmax = fmax(rmax, finish_2d<N>(a, dt, (int64_t)(j1 - 1) * a.nx + c, outc, P.h, P.qt, P.qa, accP));
    }
    publish_max(&a.slots[a.sb].rbits, rmax);
}

}  // namespace

hipError_t launch_step_2d(int level, const StepArgs &a, hipStream_t s)
{
    const int64_t nsx = (a.nx + kOut - 1) / kOut;
    const int64_t nsy = (a.ny + a.rows - 1) / a.rows;
    const unsigned grid = blocks_for(nsx * nsy * kWave);
#define L2(N) hipLaunchKernelGGL(k_step_2d<N>, dim3(grid), dim3(kBlock), 0, s, a)
    SME_LEVEL_SWITCH(level, L2)
#undef L2
    return hipGetLastError();
}

}  // namespace sme
