// k_step_tri.hip -- SME step on triangle meshes (one launch per step).
#include <hip/hip_runtime.h>

#include "sme_step_common.h"

namespace sme {

using namespace detail;

namespace {

// ----------------------------------------------------------------------------
// Triangles: one lane per cell (internal order), faces s = 0, 1, 2.
template <int N>
__device__ __forceinline__ void frame_side(Side<N, true> &S, double h, double b, const double *qx, const double *qy,
                                           double nx, double ny, double g)
{
    S.h = h;
    S.b = b;
#pragma unroll
    for (int k = 0; k <= N; ++k) {
        S.qa[k] = fma(qx[k], nx, qy[k] * ny);
        S.qt[k] = fma(qy[k], nx, -qx[k] * ny);
    }
    side_flux<N, true>(S, g);
}

template <int N>
__global__ __launch_bounds__(kBlock) void k_step_tri(StepArgs a)
{
    constexpr int n = N + 1;
    constexpr int nf = 2 * n + 1;
    const double dt = step_dt(a);
    if (blockIdx.x == 0 && threadIdx.x == 0) slot_update(a, dt);
    if (dt == 0.0) {
        noop_step(a, nf);
        return;
    }
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double r = 0.0;
    if (i < a.ncells) {
        double h0, b0, qx0[n], qy0[n];
        h0 = a.q[i];
        b0 = a.b[i];
#pragma unroll
        for (int k = 0; k < n; ++k) {
            qx0[k] = a.q[(1 + k) * a.stride + i];
            qy0[k] = a.q[(1 + n + k) * a.stride + i];
        }
        double acc[nf];
#pragma unroll
        for (int f = 0; f < nf; ++f) acc[f] = 0.0;
        double fw[3], fnx[3], fny[3];
        for (int s = 0; s < 3; ++s) {
            const int j = a.nbr[s * a.stride + i];
            const double nx = a.fnx[s * a.stride + i];
            const double ny = a.fny[s * a.stride + i];
            const double w = a.fw[s * a.stride + i];
            fw[s] = w;
            fnx[s] = nx;
            fny[s] = ny;
            double h1, b1, qx1[n], qy1[n];
            if (j >= 0) {
                h1 = a.q[j];
                b1 = a.b[j];
#pragma unroll
                for (int k = 0; k < n; ++k) {
                    qx1[k] = a.q[(1 + k) * a.stride + j];
                    qy1[k] = a.q[(1 + n + k) * a.stride + j];
                }
            } else {  // reflective wall: mirror the normal momenta
                h1 = h0;
                b1 = b0;
#pragma unroll
                for (int k = 0; k < n; ++k) {
                    double qn = fma(qx0[k], nx, qy0[k] * ny);
                    qx1[k] = fma(-2.0 * qn, nx, qx0[k]);
                    qy1[k] = fma(-2.0 * qn, ny, qy0[k]);
                }
            }
            // canonical orientation: from the lower to the higher cell index
            const bool own_left = (j < 0) || (i < j);
            const double sx = own_left ? nx : -nx;
            const double sy = own_left ? ny : -ny;
            Side<N, true> L, R;
            if (own_left) {
                frame_side<N>(L, h0, b0, qx0, qy0, sx, sy, a.g);
                frame_side<N>(R, h1, b1, qx1, qy1, sx, sy, a.g);
            } else {
                frame_side<N>(L, h1, b1, qx1, qy1, sx, sy, a.g);
                frame_side<N>(R, h0, b0, qx0, qy0, sx, sy, a.g);
            }
            double Fh[nf], D[nf];
            face_flux<N, true>(L, R, a.g, a.quad, Fh, D);
            double cf[nf];
#pragma unroll
            for (int f = 0; f < nf; ++f) cf[f] = own_left ? fma(0.5, D[f], Fh[f]) : fma(0.5, D[f], -Fh[f]);
            acc[0] = fma(w, cf[0], acc[0]);
#pragma unroll
            for (int k = 0; k < n; ++k) {
                // frame (a, t) -> (x, y) with the frame normal (sx, sy)
                double cx = fma(cf[1 + k], sx, -cf[1 + n + k] * sy);
                double cy = fma(cf[1 + k], sy, cf[1 + n + k] * sx);
                acc[1 + k] = fma(w, cx, acc[1 + k]);
                acc[1 + n + k] = fma(w, cy, acc[1 + n + k]);
            }
        }
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
        a.qn[i] = h;
        bool bad = !(h > 0.0) || !isfinite(h);
#pragma unroll
        for (int k = 0; k < n; ++k) {
            a.qn[(1 + k) * a.stride + i] = qx[k];
            a.qn[(1 + n + k) * a.stride + i] = qy[k];
            bad |= !isfinite(qx[k]) || !isfinite(qy[k]);
        }
        flag_bad(a, bad);
        double lm;
        r = cfl_ratio_tri<N>(a.g, h, ih, qx, qy, fnx, fny, fw, &lm);
        if (!(r >= 0.0)) r = 0.0;
    }
    publish_max(&a.slots[a.sb].rbits, r);
}

}  // namespace

hipError_t launch_step_tri(int level, const StepArgs &a, hipStream_t s)
{
    const unsigned grid = blocks_for(a.ncells);
#define L3(N) hipLaunchKernelGGL(k_step_tri<N>, dim3(grid), dim3(kBlock), 0, s, a)
    SME_LEVEL_SWITCH(level, L3)
#undef L3
    return hipGetLastError();
}

}  // namespace sme
