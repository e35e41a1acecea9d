// k_step_2d.hip -- SME step on structured 2D grids (one launch per step).
#include <hip/hip_runtime.h>

#include "sme_band2d.h"

namespace sme {

using namespace detail;

namespace {

// resident waves per SIMD the register allocation aims for, per level
template <int N>
constexpr int waves_target()
{
    return N == 2 ? 3 : (N == 4 ? 2 : 1);
}

template <int N, bool CLOS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(waves_target<N>()))) void k_step_2d(StepArgs a)
{
    const double dt = step_dt(a);
    if (blockIdx.x == 0 && threadIdx.x == 0) slot_update(a, dt);
    if (dt == 0.0) {
        noop_step(a, 2 * N + 3);
        return;
    }
    const int nsx = (a.nx + kOut - 1) / kOut;
    const int nsy = (a.ny + a.rows - 1) / a.rows;
    // XCD-aware order: blocks are dealt round-robin to the kXcd dies, so block b
    // runs on die b % kXcd.  Give each die one contiguous range of (strip,
    // band) pairs so the halo rows two bands share stay in that die's L2.
    const int nblk = (int)gridDim.x;
    const int per_xcd = (nblk + kXcd - 1) / kXcd;
    const int slot = (int)(blockIdx.x % kXcd) * per_xcd + (int)(blockIdx.x / kXcd);
    // wave-uniform (scalar) band coordinates: the staged loads need uniform row addresses
    const int wave = __builtin_amdgcn_readfirstlane(slot * (kBlock / kWave) + (int)(threadIdx.x >> 6));
    constexpr int sd = stage_doubles<N>();
    __shared__ __attribute__((aligned(16))) double stage[(kBlock / kWave) * (sd > 0 ? sd : 1)];
    double rmax = 0.0;
    if (wave < nsx * nsy)  // waves beyond the grid only join the reduction
        rmax = band2d<N, CLOS>(a, dt, wave % nsx, wave / nsx, stage + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * sd);
    publish_ratio(a.slots[a.sb], rmax);
}

}  // namespace

hipError_t launch_step_2d(int level, const StepArgs &a, hipStream_t s)
{
    const int64_t nsx = (a.nx + kOut - 1) / kOut;
    const int64_t nsy = (a.ny + a.rows - 1) / a.rows;
    // whole dies' worth of blocks, so the die-major slot order covers every wave
    const int64_t blocks = (nsx * nsy * kWave + kBlock - 1) / kBlock;
    const unsigned grid = (unsigned)((blocks + kXcd - 1) / kXcd * kXcd);
    if (a.closure) {
        if (level != 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_step_2d<1, true>), dim3(grid), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
#define L2(N) hipLaunchKernelGGL((k_step_2d<N, false>), dim3(grid), dim3(kBlock), 0, s, a)
    SME_LEVEL_SWITCH(level, L2)
#undef L2
    return hipGetLastError();
}

int step_2d_vgprs(int level)
{
    hipFuncAttributes fa{};
    hipError_t e = hipErrorInvalidValue;
#define A2(N) e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&k_step_2d<N, false>))
    switch (level) {
    case 0: A2(0); break;
    case 1: A2(1); break;
    case 2: A2(2); break;
    case 3: A2(3); break;
    case 4: A2(4); break;
    case 5: A2(5); break;
    case 6: A2(6); break;
    case 7: A2(7); break;
    case 8: A2(8); break;
    default: break;
    }
#undef A2
    return e == hipSuccess ? fa.numRegs : -1;
}

}  // namespace sme
