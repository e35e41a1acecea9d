// k_batch.hip -- many structured SME grids of mixed size and level advanced by
// one persistent launch per step.
//
// The work list holds one item per (grid, strip, band), sorted by level
// (costliest first).  Each resident wave takes the next item from a device
// counter when it is done with the previous one, so the waves finish together
// even when the items are few and tall (a fixed deal of a few tall items per
// wave leaves some waves one item behind the rest).  Each grid keeps its own
// three time slots, so every grid takes its own CFL step; the item holding the
// grid's first band also advances that grid's clock.  The band code is the one
// of the single-grid kernel, so a grid advanced here is bitwise identical to
// the same grid advanced alone.
#include <hip/hip_runtime.h>

#include "sme_band2d.h"

namespace sme {

using namespace detail;

namespace {

// IMP: the friction step is backward Euler (compile-time copy of the flag)
template <bool IMP>
__global__ __launch_bounds__(kBlock) void k_batch_step(BatchArgs B)
{
    const int lane = threadIdx.x & (kWave - 1);
    // one staging area per wave, sized for the highest level of the ensemble
    constexpr int sd = stage_doubles<kBatchMaxLevel>();
    __shared__ __attribute__((aligned(16))) double stage_all[(kBlock / kWave) * sd];
    double *const stage = stage_all + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * sd;
    // This step counts on work[sa] and clears work[sc] for the step after
    // next (the next step counts on work[sb], which the previous step cleared).
    unsigned *const ctr = B.work + B.sa * kWorkStride;
    if (blockIdx.x == 0 && threadIdx.x == 0) (void)atomicExch(B.work + B.sc * kWorkStride, 0u);
    unsigned got = 0;
    if (lane == 0) got = atomicAdd(ctr, 1u);
    unsigned it = (unsigned)__builtin_amdgcn_readfirstlane(got);
    while (it < (unsigned)B.nitems) {
        // the index of the wave's next item is fetched while this one runs
        got = 0;
        if (lane == 0) got = atomicAdd(ctr, 1u);
        const BatchItem item = B.items[it];
        const BatchInst I = B.inst[item.inst];
        StepArgs a;
        a.q = B.q + I.offset;
        a.qn = B.qn + I.offset;
        a.b = B.b + I.boff;
        a.stride = I.stride;
        a.ncells = (int64_t)I.nx * I.ny;
        a.nx = I.nx;
        a.ny = I.ny;
        a.idx = I.idx;
        a.idy = I.idy;
        a.bc[0] = I.bc[0];
        a.bc[1] = I.bc[1];
        a.bc[2] = I.bc[2];
        a.bc[3] = I.bc[3];
        a.rows = I.rows;
        a.nbr = nullptr;
        a.fsx = a.fsy = a.ivol = nullptr;
        a.g = B.g;
        a.c_slip = B.c_slip;
        a.implicit = B.implicit;
        a.nu = B.nu;
        a.cfl = B.cfl;
        a.quad = B.quad;
        a.dt_fixed = 0.0;
        a.t_end = 0.0;
        a.slots = B.slots + 3 * item.inst;
        a.sa = B.sa;
        a.sb = B.sb;
        a.sc = B.sc;
        a.err = B.err;
        a.closure = nullptr;
        a.oor = nullptr;
        a.rates = nullptr;
        const double dt = step_dt(a);
        if (item.sx == 0 && item.sy == 0 && lane == 0) slot_update(a, dt);
        double r = 0.0;
        switch (I.level) {
        case 0: r = band2d<0, false, IMP>(a, dt, item.sx, item.sy, stage); break;
        case 1: r = band2d<1, false, IMP>(a, dt, item.sx, item.sy, stage); break;
        case 2: r = band2d<2, false, IMP>(a, dt, item.sx, item.sy, stage); break;
        case 3: r = band2d<3, false, IMP>(a, dt, item.sx, item.sy, stage); break;
        case 4: r = band2d<4, false, IMP>(a, dt, item.sx, item.sy, stage); break;
        default: break;
        }
        r = wave_max(r);
        if (lane == 0 && r > 0.0)
            atomicMax(&a.slots[a.sb].r[blockIdx.x % kRatioWords].bits, (unsigned long long)__double_as_longlong(r));
        it = (unsigned)__builtin_amdgcn_readfirstlane(got);
    }
}

}  // namespace

hipError_t launch_batch_step(const BatchArgs &a, int grid, hipStream_t s)
{
    if (a.implicit)
        hipLaunchKernelGGL(k_batch_step<true>, dim3(grid), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_batch_step<false>, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// resident waves per SIMD of the ensemble kernel (runtime occupancy query:
// VGPRs, AGPRs and LDS together; a block is one wave per SIMD); 1 on failure
int batch_waves_per_simd()
{
    int blocks = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch_step<false>, kBlock, 0);
    return e == hipSuccess && blocks > 0 ? blocks * (kBlock / kWave) / 4 : 1;
}

}  // namespace sme
