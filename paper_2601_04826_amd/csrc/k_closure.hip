// k_closure.hip -- closure rates of every cell from the current level-1 state.
//
// Runs before each level-1 step that has a learned closure attached.  One
// lane per cell and direction: it forms the nine features (the cell's depth
// and normal momenta q_0, q_1 and their differences to the two neighbours
// along that direction, boundary ghosts as in the step), evaluates the network
// and stores the two correction rates as FP32 float2 at [dir * stride + cell].
// A direction whose features leave the training box gets zero rates and is
// counted.  The network's parameters are staged in LDS.
#include <hip/hip_runtime.h>

#include "sme_step_common.h"

namespace sme {

using namespace detail;

namespace {

// (h, q_0, q_1) normal to the axis of the neighbour at offset (di, dj) of cell
// (i, j); blk = field index of q_0 of the momenta normal to that axis
__device__ __forceinline__ void nb_normal(const StepArgs &a, int i, int j, int di, int dj, int blk, double &h,
                                          double &q0, double &q1)
{
    bool mx = false, my = false;
    const int ii = di ? ghost_index(i + di, a.nx, a.bc[0], a.bc[1], mx) : i;
    const int jj = dj ? ghost_index(j + dj, a.ny, a.bc[2], a.bc[3], my) : j;
    const int64_t cell = (int64_t)jj * a.nx + ii;
    const double s = (mx || my) ? -1.0 : 1.0;  // a wall mirrors the normal momenta
    h = a.q[cell];
    q0 = s * a.q[(blk + 0) * a.stride + cell];
    q1 = s * a.q[(blk + 1) * a.stride + cell];
}

// grid = nblk blocks per direction; blocks [0, nblk) do x, [nblk, 2 nblk) do y
__global__ __launch_bounds__(kBlock) void k_closure_rates_valu(StepArgs a, unsigned nblk)
{
    __shared__ float P[kMlpParams];
    mlp_stage(a.closure->params, P);
    const int dir = blockIdx.x >= nblk ? 1 : 0;
    const int64_t cell = (int64_t)(blockIdx.x - dir * nblk) * kBlock + threadIdx.x;
    float2 *rates = reinterpret_cast<float2 *>(const_cast<float *>(a.rates)) + dir * a.stride;
    const bool live = step_dt(a) > 0.0;  // a step past the end time changes nothing
    unsigned out = 0;
    if (cell < a.ncells) {
        float2 r = make_float2(0.0f, 0.0f);
        if (live) {
            const int i = (int)(cell % a.nx), j = (int)(cell / a.nx);
            const int blk = dir ? 3 : 1;  // level 1: fields h, qx_0, qx_1, qy_0, qy_1
            const double h = a.q[cell];
            const double q0 = a.q[blk * a.stride + cell], q1 = a.q[(blk + 1) * a.stride + cell];
            double hp, q0p, q1p, hm, q0m, q1m;
            nb_normal(a, i, j, dir ? 0 : 1, dir, blk, hp, q0p, q1p);
            nb_normal(a, i, j, dir ? 0 : -1, -dir, blk, hm, q0m, q1m);
            out = closure_rate(P, a.closure, h, q0, q1, hp, q0p, q1p, hm, q0m, q1m, r.x, r.y) ? 0u : 1u;
        }
        rates[cell] = r;
    }
    publish_count(a.oor, out);
}

}  // namespace

hipError_t launch_closure_rates(const StepArgs &a, int dims, int mode, hipStream_t s)
{
    if (mode != 0 || dims < 1 || dims > 2) return hipErrorInvalidValue;
    const unsigned nblk = blocks_for(a.ncells);
    const unsigned dirs = (unsigned)dims;
    hipLaunchKernelGGL(k_closure_rates_valu, dim3(nblk * dirs), dim3(kBlock), 0, s, a, nblk);
    return hipGetLastError();
}

}  // namespace sme
