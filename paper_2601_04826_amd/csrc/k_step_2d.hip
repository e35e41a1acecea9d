// k_step_2d.hip -- SME step on structured 2D grids (one launch per step).
#include <hip/hip_runtime.h>

#include "sme_band2d.h"

namespace sme {

using namespace detail;

namespace {

// resident waves per SIMD the register allocation aims for, per level.  At
// level 2 two waves (172 registers, nothing spilled) run the 4096^2 step 3%
// faster than three (168 registers and a spill) and the 1024^2 step as fast:
// the row loop is bound by its FP64 arithmetic and by HBM, not by latency.
template <int N>
constexpr int waves_target()
{
    return N == 4 || N == 2 ? 2 : 1;
}

// IMP: the friction step is backward Euler (a compile-time copy of the flag,
// so the explicit kernels keep their own register allocation)
template <int N, bool CLOS, bool IMP>
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
    __shared__ __attribute__((aligned(16))) double stage[(kBlock / kWave) * sd];
    double rmax = 0.0;
    if (wave < nsx * nsy)  // waves beyond the grid only join the reduction
        rmax = band2d<N, CLOS, IMP>(a, dt, wave % nsx, wave / nsx, stage + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * sd);
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
        if (a.implicit)
            hipLaunchKernelGGL((k_step_2d<1, true, true>), dim3(grid), dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((k_step_2d<1, true, false>), dim3(grid), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
#define L2(N) hipLaunchKernelGGL((k_step_2d<N, false, false>), dim3(grid), dim3(kBlock), 0, s, a)
#define L2X(N) hipLaunchKernelGGL((k_step_2d<N, false, true>), dim3(grid), dim3(kBlock), 0, s, a)
    if (a.implicit) {
        SME_LEVEL_SWITCH(level, L2X)
    } else {
        SME_LEVEL_SWITCH(level, L2)
    }
#undef L2
#undef L2X
    return hipGetLastError();
}

// resident waves per SIMD of the structured step kernel at this level, from
// the runtime's occupancy calculation (VGPRs, AGPRs and LDS together); a block
// is one wave per SIMD.  1 if the query fails.
int step_2d_waves_per_simd(int level)
{
    int blocks = 0;
    hipError_t e = hipErrorInvalidValue;
#define O2(N) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_step_2d<N, false, false>, kBlock, 0)
    switch (level) {
    case 0: O2(0); break;
    case 1: O2(1); break;
    case 2: O2(2); break;
    case 3: O2(3); break;
    case 4: O2(4); break;
    case 5: O2(5); break;
    case 6: O2(6); break;
    case 7: O2(7); break;
    case 8: O2(8); break;
    default: break;
    }
#undef O2
    return e == hipSuccess && blocks > 0 ? blocks * (kBlock / kWave) / 4 : 1;
}

}  // namespace sme
