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

// Raw state of one face's neighbour and the face's scaled normal n |e|.
template <int N>
struct Gather {
    double h, b, qx[N + 1], qy[N + 1];
    double sx, sy;
};

// Loads for the face at geometry index gi whose neighbour is j (a wall if j < 0:
// only the geometry is loaded, the mirror state is formed at use).
template <int N>
__device__ __forceinline__ void gather(const StepArgs &a, int j, int64_t gi, Gather<N> &G)
{
    constexpr int n = N + 1;
    G.sx = a.fsx[gi];
    G.sy = a.fsy[gi];
    if (j >= 0) {
        G.h = a.q[j];
        G.b = a.b[j];
#pragma unroll
        for (int k = 0; k < n; ++k) {
            G.qx[k] = a.q[(1 + k) * a.stride + j];
            G.qy[k] = a.q[(1 + n + k) * a.stride + j];
        }
    }
}

// IMP: the friction step is backward Euler (compile-time copy of the flag)
template <int N, bool IMP>
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
    // XCD-aware order: block b runs on die b % kXcd; each die gets one
    // contiguous range of the (bandwidth-reduced) cell order, so the neighbour
    // gathers of a die hit its own L2 instead of being fetched by every die
    const int64_t per_xcd = ((int64_t)gridDim.x + kXcd - 1) / kXcd;
    const int64_t slot = (int64_t)(blockIdx.x % kXcd) * per_xcd + blockIdx.x / kXcd;
    const int64_t i = slot * kBlock + threadIdx.x;
    double r = 0.0;
    if (i < a.ncells) {
        double h0, b0, qx0[n], qy0[n];
        h0 = a.q[i];
        b0 = a.b[i];
        const double iv = a.ivol[i];
#pragma unroll
        for (int k = 0; k < n; ++k) {
            qx0[k] = a.q[(1 + k) * a.stride + i];
            qy0[k] = a.q[(1 + n + k) * a.stride + i];
        }
        double acc[nf];
#pragma unroll
        for (int f = 0; f < nf; ++f) acc[f] = 0.0;
        // One face at a time (rolled: the live set is one face's two sides),
        // with the gather of the next face's neighbour issued before the
        // current face is evaluated, so its latency overlaps the arithmetic.
        int jn[3];
#pragma unroll
        for (int s = 0; s < 3; ++s) jn[s] = a.nbr[s * a.stride + i];
        Gather<N> nxt;
        gather<N>(a, jn[0], i, nxt);
#pragma unroll 1
        for (int s = 0; s < 3; ++s) {
            const Gather<N> cur = nxt;
            if (s < 2) gather<N>(a, s == 0 ? jn[1] : jn[2], i + (s + 1) * a.stride, nxt);
            const int j = s == 0 ? jn[0] : (s == 1 ? jn[1] : jn[2]);
            double nx, ny, w;
            face_geom(cur.sx, cur.sy, iv, nx, ny, w);
            double h1, b1, qx1[n], qy1[n];
            if (j >= 0) {
                h1 = cur.h;
                b1 = cur.b;
#pragma unroll
                for (int k = 0; k < n; ++k) {
                    qx1[k] = cur.qx[k];
                    qy1[k] = cur.qy[k];
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
            // canonical orientation: from the lower to the higher cell index,
            // so both cells of a face evaluate it on bitwise equal inputs
            const bool own_left = (j < 0) || (i < j);
            const double sx = own_left ? nx : -nx;
            const double sy = own_left ? ny : -ny;
            double qxl[n], qyl[n], qxr[n], qyr[n];
#pragma unroll
            for (int k = 0; k < n; ++k) {
                qxl[k] = own_left ? qx0[k] : qx1[k];
                qyl[k] = own_left ? qy0[k] : qy1[k];
                qxr[k] = own_left ? qx1[k] : qx0[k];
                qyr[k] = own_left ? qy1[k] : qy0[k];
            }
            Side<N, true> L, R;
            frame_side<N>(L, own_left ? h0 : h1, own_left ? b0 : b1, qxl, qyl, sx, sy, a.g);
            frame_side<N>(R, own_left ? h1 : h0, own_left ? b1 : b0, qxr, qyr, sx, sy, a.g);
            double Fh[nf], D[nf];
            face_flux<N, true>(L, R, a.g, a.quad, Fh, D);
            // this cell's share, rotated from the frame (a, t) with normal (sx, sy) back to (x, y)
            const double sgn = own_left ? 1.0 : -1.0;
            acc[0] = fma(w, fma(0.5, D[0], sgn * Fh[0]), acc[0]);
#pragma unroll
            for (int k = 0; k < n; ++k) {
                const double ca = fma(0.5, D[1 + k], sgn * Fh[1 + k]);
                const double ct = fma(0.5, D[1 + n + k], sgn * Fh[1 + n + k]);
                acc[1 + k] = fma(w, fma(ca, sx, -ct * sy), acc[1 + k]);
                acc[1 + n + k] = fma(w, fma(ca, sy, ct * sx), acc[1 + n + k]);
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
        friction_step<N, true, IMP>(qx, qy, ih, dt, a.c_slip, a.nu);
        a.qn[i] = h;
        bool bad = !(h > 0.0) || !isfinite(h);
#pragma unroll
        for (int k = 0; k < n; ++k) {
            a.qn[(1 + k) * a.stride + i] = qx[k];
            a.qn[(1 + n + k) * a.stride + i] = qy[k];
            bad |= !isfinite(qx[k]) || !isfinite(qy[k]);
        }
        flag_bad(a, bad);
        double fw[3], fnx[3], fny[3];  // reloaded (cached) rather than held across the face loop
        tri_geom(a, i, fnx, fny, fw);
        double lm;
        r = cfl_ratio_tri<N>(a.g, h, ih, qx, qy, fnx, fny, fw, &lm);
        if (!(r >= 0.0)) r = 0.0;
    }
    publish_ratio(a.slots[a.sb], r);
}

}  // namespace

hipError_t launch_step_tri(int level, const StepArgs &a, hipStream_t s)
{
    // whole dies' worth of blocks, so the die-major slot order covers every cell
    const unsigned grid = (blocks_for(a.ncells) + kXcd - 1) / kXcd * kXcd;
#define L3(N) hipLaunchKernelGGL((k_step_tri<N, false>), dim3(grid), dim3(kBlock), 0, s, a)
#define L3X(N) hipLaunchKernelGGL((k_step_tri<N, true>), dim3(grid), dim3(kBlock), 0, s, a)
    if (a.implicit) {
        SME_LEVEL_SWITCH(level, L3X)
    } else {
        SME_LEVEL_SWITCH(level, L3)
    }
#undef L3
#undef L3X
    return hipGetLastError();
}

}  // namespace sme
