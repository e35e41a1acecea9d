// k_step_1d.hip -- SME step on uniform 1D grids (one launch per step).
//
// A 64-lane wave owns 64 consecutive cells (62 outputs and one halo cell on
// each side); each lane computes the face to its right, the right cell's share
// moves one lane up through a cross-lane shift.  With a learned closure
// attached (level 1 only) every cell also adds dt times the network's
// correction rates of (q_0, q_1), which the rates pass computed from Q^n.
#include <hip/hip_runtime.h>

#include "sme_step_common.h"

namespace sme {

using namespace detail;

namespace {

template <int N, bool CLOS>
__global__ __launch_bounds__(kBlock) void k_step_1d(StepArgs a)
{
    constexpr int n = N + 1;
    const double dt = step_dt(a);
    if (blockIdx.x == 0 && threadIdx.x == 0) slot_update(a, dt);
    if (dt == 0.0) {
        noop_step(a, N + 2);
        return;
    }
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int x0 = wave * kOut;
    double r = 0.0;
    if (x0 < a.nx) {  // waves beyond the grid only join the reduction
        const int c = x0 - 1 + lane;
        bool mir;
        const int src = ghost_index(c, a.nx, a.bc[0], a.bc[1], mir);
        const bool out = lane >= 1 && lane <= kOut && c < a.nx;

        Side<N, false> S;
        S.h = a.q[src];
        S.b = a.b[src];
#pragma unroll
        for (int k = 0; k < n; ++k) {
            double v = a.q[(1 + k) * a.stride + src];
            S.qa[k] = mir ? -v : v;
        }
        side_flux<N, false>(S, a.g);

        Side<N, false> R;
        R.h = shfl_dn(S.h);
        R.b = shfl_dn(S.b);
        R.lam = shfl_dn(S.lam);
#pragma unroll
        for (int k = 0; k < n; ++k) {
            R.qa[k] = shfl_dn(S.qa[k]);
            R.Fa[k] = shfl_dn(S.Fa[k]);
        }
        double Fh[1 + n], D[1 + n];
        face_flux<N, false>(S, R, a.g, a.quad, Fh, D);
        double acc[1 + n];
#pragma unroll
        for (int f = 0; f < 1 + n; ++f) {
            double own = fma(0.5, D[f], Fh[f]);
            double oth = fma(0.5, D[f], -Fh[f]);
            acc[f] = own + shfl_up1(oth);
        }
        // predictor and friction
        const double sc = dt * a.idx;
        double h = fma(-sc, acc[0], S.h);
        double q[n];
#pragma unroll
        for (int k = 0; k < n; ++k) q[k] = fma(-sc, acc[1 + k], S.qa[k]);
        const double ih = rcp(h);
        friction<N>(q, ih, dt, a.c_slip, a.nu);
        if constexpr (CLOS) {
            static_assert(N == 1, "the closure acts on level 1");
            if (out) {  // rates of (q_0, q_1) from the rates pass over Q^n
                const float2 cr = reinterpret_cast<const float2 *>(a.rates)[c];
                q[0] = fma(dt, (double)cr.x, q[0]);
                q[1] = fma(dt, (double)cr.y, q[1]);
            }
        }
        if (out) {
            a.qn[c] = h;
            bool bad = !(h > 0.0) || !isfinite(h);
#pragma unroll
            for (int k = 0; k < n; ++k) {
                a.qn[(1 + k) * a.stride + c] = q[k];
                bad |= !isfinite(q[k]);
            }
            flag_bad(a, bad);
            double lm;
            r = cfl_ratio_1d<N>(a.g, h, ih, q, a.idx, &lm);
            if (!(r >= 0.0)) r = 0.0;
        }
    }
    publish_ratio(a.slots[a.sb], r);
}

}  // namespace

hipError_t launch_step_1d(int level, const StepArgs &a, hipStream_t s)
{
    const int64_t waves = (a.nx + kOut - 1) / kOut;
    const unsigned grid = blocks_for(waves * kWave);
    if (a.closure) {
        if (level != 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_step_1d<1, true>), dim3(grid), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
#define L1(N) hipLaunchKernelGGL((k_step_1d<N, false>), dim3(grid), dim3(kBlock), 0, s, a)
    SME_LEVEL_SWITCH(level, L1)
#undef L1
    return hipGetLastError();
}

}  // namespace sme
