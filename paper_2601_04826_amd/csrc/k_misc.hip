// k_misc.hip -- eigenvalue-bound reduction, slot reset and permutation kernels.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sme_step_common.h"

namespace sme {

using namespace detail;

namespace {

// ----------------------------------------------------------------------------
// Eigenvalue bound over the current state: max CFL ratio and max lam into slot sa.
// A grid-stride loop over a few blocks per compute unit: one atomic per block
// and quantity, so the atomics on the two slot words stay few.
template <int N, int KIND>
__global__ __launch_bounds__(kBlock) void k_eig(StepArgs a)
{
    constexpr int n = N + 1;
    double rm = 0.0, lm = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.ncells; i += (int64_t)gridDim.x * kBlock) {
        double r = 0.0, lmax = 0.0;
        const double h = a.q[i];
        const double ih = rcp(h);
        double qx[n], qy[n];
#pragma unroll
        for (int k = 0; k < n; ++k) {
            qx[k] = a.q[(1 + k) * a.stride + i];
            qy[k] = KIND == 1 ? 0.0 : a.q[(1 + n + k) * a.stride + i];
        }
        if (KIND == 1) {
            r = cfl_ratio_1d<N>(a.g, h, ih, qx, a.idx, &lmax);
        } else if (KIND == 2) {
            r = cfl_ratio_2d<N>(a.g, h, ih, qx, qy, a.idx, a.idy, &lmax);
        } else {
            double fnx[3], fny[3], fw[3];
            tri_geom(a, i, fnx, fny, fw);
            r = cfl_ratio_tri<N>(a.g, h, ih, qx, qy, fnx, fny, fw, &lmax);
        }
        // a loaded state must be physical too (step index = current step count)
        bool bad = !(h > 0.0) || !isfinite(h);
#pragma unroll
        for (int k = 0; k < n; ++k) bad |= !isfinite(qx[k]) || !isfinite(qy[k]);
        flag_bad_at(a, bad, a.slots[a.sa].step);
        if (r >= 0.0) rm = fmax(rm, r);
        if (lmax >= 0.0) lm = fmax(lm, lmax);
    }
    publish_ratio(a.slots[a.sa], rm);
    publish_max(&a.slots[a.sa].lbits, lm);
}

__global__ void k_slots_reset(Slot *slots, ErrWord *err, int sa)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int s = 0; s < 3; ++s) {
            for (int w = 0; w < kRatioWords; ++w) slots[s].r[w].bits = 0ull;
            slots[s].lbits = 0ull;
            slots[s].t = 0.0;
            slots[s].dt = 0.0;
            slots[s].step = 0;
        }
        if (err) {
            err->flag = 0u;
            err->first_step = ~0ull;
        }
    }
}

// dst[f * dstride + map[i]] = src[f * sstride + i]   (map == nullptr: identity)
__global__ __launch_bounds__(kBlock) void k_permute(const double *src, int64_t sstride, double *dst, int64_t dstride,
                                                   const int64_t *map, int64_t ncells, int nf)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= ncells) return;
    const int64_t d = map ? map[i] : i;
    for (int f = 0; f < nf; ++f) dst[f * dstride + d] = src[f * sstride + i];
}

}  // namespace

hipError_t launch_eig(int dim, int kind, int level, const StepArgs &a, hipStream_t s)
{
    (void)dim;
    const unsigned grid = std::min(blocks_for(a.ncells), 1024u);
#define LE1(N) hipLaunchKernelGGL((k_eig<N, 1>), dim3(grid), dim3(kBlock), 0, s, a)
#define LE2(N) hipLaunchKernelGGL((k_eig<N, 2>), dim3(grid), dim3(kBlock), 0, s, a)
#define LE3(N) hipLaunchKernelGGL((k_eig<N, 3>), dim3(grid), dim3(kBlock), 0, s, a)
    if (kind == 1) {
        SME_LEVEL_SWITCH(level, LE1)
    } else if (kind == 2) {
        SME_LEVEL_SWITCH(level, LE2)
    } else {
        SME_LEVEL_SWITCH(level, LE3)
    }
#undef LE1
#undef LE2
#undef LE3
    return hipGetLastError();
}

hipError_t launch_slots_reset(Slot *slots, ErrWord *err, int sa, hipStream_t s)
{
    hipLaunchKernelGGL(k_slots_reset, dim3(1), dim3(64), 0, s, slots, err, sa);
    return hipGetLastError();
}

hipError_t launch_permute(const double *src, int64_t sstride, double *dst, int64_t dstride, const int64_t *map,
                          int64_t ncells, int nf, hipStream_t s)
{
    if (ncells == 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute, dim3(blocks_for(ncells)), dim3(kBlock), 0, s, src, sstride, dst, dstride, map,
                       ncells, nf);
    return hipGetLastError();
}

}  // namespace sme
