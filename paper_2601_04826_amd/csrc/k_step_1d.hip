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

// Faces, predictor and friction of this lane's cell from the lane's side S
// (its state, with side_flux applied): the right face through a cross-lane
// shift, the left face's share from the lane below.  Returns h of Q^{n+1}
// and writes its momenta to q and 1/h to ih.  Shared by the step kernel and
// the multi-step kernel, so both give bitwise equal states.
template <int N, bool IMP>
__device__ __forceinline__ double update_1d(const StepArgs &a, double dt, const Side<N, false> &S, double *q,
                                            double &ih)
{
    constexpr int n = N + 1;
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
    const double sc = dt * a.idx;
    const double h = fma(-sc, acc[0], S.h);
#pragma unroll
    for (int k = 0; k < n; ++k) q[k] = fma(-sc, acc[1 + k], S.qa[k]);
    ih = rcp(h);
    friction_step<N, false, IMP>(q, nullptr, ih, dt, a.c_slip, a.nu);
    return h;
}

// IMP: the friction step is backward Euler (a compile-time copy of the flag,
// so the explicit kernels keep their own register allocation)
template <int N, bool CLOS, bool IMP>
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
        // faces, predictor and friction
        double q[n], ih;
        const double h = update_1d<N, IMP>(a, dt, S, q, ih);
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

// Many steps of a small 1D grid in one launch: a single workgroup keeps the
// state (two buffers) and the bathymetry in LDS and runs up to nsteps steps,
// each one exactly as k_step_1d computes it (same cell arithmetic, the same
// step from the exact maximum of the CFL ratios, the same clock sum), with a
// workgroup barrier where the per-step path has a kernel boundary.  A grid of
// a thousand cells is otherwise bound by the launch of each step.  Steps past
// the end time change nothing, so the loop stops at the first one.  At the end
// the state goes to dst (the buffer the per-step path would hold after
// nsteps steps) and the time slots are left as nsteps steps would leave them.
constexpr int kRunBlock = 1024;

template <int N, bool IMP>
__global__ __launch_bounds__(kRunBlock) void k_run_1d_lds(StepArgs a, int nsteps, double *dst)
{
    constexpr int n = N + 1;
    constexpr int nf = N + 2;
    constexpr int nw = kRunBlock / kWave;
    extern __shared__ __attribute__((aligned(16))) double lds[];  // [2][nf][nx] state, [nx] bathymetry
    __shared__ double part[nw];
    const int nx = a.nx;
    double *const bl = lds + 2 * nf * nx;
    for (int i = threadIdx.x; i < nx; i += kRunBlock) {
#pragma unroll
        for (int f = 0; f < nf; ++f) lds[f * nx + i] = a.q[f * a.stride + i];
        bl[i] = a.b[i];
    }
    const Slot &s0 = a.slots[a.sa];
    double t = s0.t, r = slot_ratio(s0), dt_last = s0.dt;
    long long step = s0.step;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
    const int chunks = (nx + kOut - 1) / kOut;
    int cur = 0;
    bool stopped = false;
    __syncthreads();
    for (int k = 0; k < nsteps; ++k) {
        double dt = a.dt_fixed > 0.0 ? a.dt_fixed : (r > 0.0 ? a.cfl / r : 0.0);
        if (a.t_end > 0.0) dt = fmin(dt, fmax(a.t_end - t, 0.0));
        if (dt == 0.0) {
            stopped = true;
            break;
        }
        const double *src = lds + cur * nf * nx;
        double *out = lds + (1 - cur) * nf * nx;
        double rl = 0.0;
        for (int w = wave; w < chunks; w += nw) {
            const int c = w * kOut - 1 + lane;
            bool mir;
            const int sc = ghost_index(c, nx, a.bc[0], a.bc[1], mir);
            const bool o = lane >= 1 && lane <= kOut && c < nx;
            Side<N, false> S;
            S.h = src[sc];
            S.b = bl[sc];
#pragma unroll
            for (int j = 0; j < n; ++j) {
                const double v = src[(1 + j) * nx + sc];
                S.qa[j] = mir ? -v : v;
            }
            side_flux<N, false>(S, a.g);
            double q[n], ih;
            const double h = update_1d<N, IMP>(a, dt, S, q, ih);
            if (o) {
                out[c] = h;
                bool bad = !(h > 0.0) || !isfinite(h);
#pragma unroll
                for (int j = 0; j < n; ++j) {
                    out[(1 + j) * nx + c] = q[j];
                    bad |= !isfinite(q[j]);
                }
                flag_bad_at(a, bad, step + 1);
                double lm;
                double rr = cfl_ratio_1d<N>(a.g, h, ih, q, a.idx, &lm);
                if (!(rr >= 0.0)) rr = 0.0;
                rl = fmax(rl, rr);
            }
        }
        rl = wave_max(rl);
        if (lane == 0) part[wave] = rl;
        __syncthreads();  // the new state and every wave's ratio are in LDS
        double m = part[0];
#pragma unroll
        for (int w = 1; w < nw; ++w) m = fmax(m, part[w]);
        __syncthreads();  // part is rewritten by the next step
        t = t + dt;
        dt_last = dt;
        ++step;
        r = m;
        cur = 1 - cur;
    }
    const double *fin = lds + cur * nf * nx;
    for (int i = threadIdx.x; i < nx; i += kRunBlock) {
#pragma unroll
        for (int f = 0; f < nf; ++f) dst[f * a.stride + i] = fin[f * nx + i];
    }
    if (threadIdx.x == 0) {
        // the slot of the state after nsteps steps, and the cleared one after it
        Slot &sf = a.slots[(a.sa + nsteps) % 3];
        Slot &sn = a.slots[(a.sa + nsteps + 1) % 3];
        sf.r[0].bits = (unsigned long long)__double_as_longlong(r);
#pragma unroll
        for (int w = 1; w < kRatioWords; ++w) sf.r[w].bits = 0ull;
        sf.lbits = 0ull;
        sf.t = t;
        sf.dt = stopped ? 0.0 : dt_last;  // a step past the end time records dt = 0
        sf.step = step;
#pragma unroll
        for (int w = 0; w < kRatioWords; ++w) sn.r[w].bits = 0ull;
        sn.lbits = 0ull;
    }
}

}  // namespace

// bytes of dynamic LDS the multi-step kernel needs for this grid
size_t run_1d_lds_bytes(int level, int nx) { return (size_t)(2 * (level + 2) + 1) * (size_t)nx * sizeof(double); }

hipError_t launch_run_1d_lds(int level, const StepArgs &a, int nsteps, double *dst, hipStream_t s)
{
    const size_t bytes = run_1d_lds_bytes(level, a.nx);
    hipError_t e = hipSuccess;
#define R1I(N, I)                                                                                                \
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_run_1d_lds<N, I>),                                  \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);                              \
    if (e == hipSuccess) hipLaunchKernelGGL((k_run_1d_lds<N, I>), dim3(1), dim3(kRunBlock), bytes, s, a, nsteps, dst)
#define R1(N) R1I(N, false)
#define R1X(N) R1I(N, true)
    if (a.implicit) {
        SME_LEVEL_SWITCH(level, R1X)
    } else {
        SME_LEVEL_SWITCH(level, R1)
    }
#undef R1
#undef R1X
#undef R1I
    return e == hipSuccess ? hipGetLastError() : e;
}

hipError_t launch_step_1d(int level, const StepArgs &a, hipStream_t s)
{
    const int64_t waves = (a.nx + kOut - 1) / kOut;
    const unsigned grid = blocks_for(waves * kWave);
    if (a.closure) {
        if (level != 1) return hipErrorInvalidValue;
        if (a.implicit)
            hipLaunchKernelGGL((k_step_1d<1, true, true>), dim3(grid), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((k_step_1d<1, true, false>), dim3(grid), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
#define L1(N) hipLaunchKernelGGL((k_step_1d<N, false, false>), dim3(grid), dim3(kBlock), 0, s, a)
#define L1X(N) hipLaunchKernelGGL((k_step_1d<N, false, true>), dim3(grid), dim3(kBlock), 0, s, a)
    if (a.implicit) {
        SME_LEVEL_SWITCH(level, L1X)
    } else {
        SME_LEVEL_SWITCH(level, L1)
    }
#undef L1
#undef L1X
    return hipGetLastError();
}

}  // namespace sme
