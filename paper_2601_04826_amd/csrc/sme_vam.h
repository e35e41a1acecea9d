// sme_vam.h -- launch interface of the non-hydrostatic VAM step (k_vam.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sme_kernels.h"

namespace sme {

// One channel of nx cells, fields (h, h u0, h u1, h w0, h w1) at
// q[f * stride + cell].  The corrector's unknowns (p0, p1) of cells 2k and
// 2k + 1 form block k of a block-tridiagonal system with 4 x 4 blocks; the
// blocks are held entry-major: entry e of block k at M[e * nb + k] (coalesced
// for consecutive blocks).
struct VamSystem {
    double *A, *B, *C;  // [16][nb] couplings to blocks k - 1, k, k + 1
    double *d;          // [4][nb] right-hand side
};

struct VamArgs {
    const double *q;    // Q^n
    double *qs;         // Q* and then Q^{n+1} (in place)
    const double *b;    // bathymetry [nx]
    double *p;          // pressure (p0, p1) at p[c * stride + cell]
    int64_t stride;
    int nx, nb;         // cells, blocks = ceil(nx / 2)
    double dx, g, cfl;
    Quad quad;
    double t_end;       // > 0: clamp simulated time
    double dt_fixed;    // > 0: fixed step
    Slot *slots;
    int sa, sb, sc;
    ErrWord *err;
};

hipError_t launch_vam_eig(const VamArgs &a, hipStream_t s);       // CFL ratio of a.q into slot sa
hipError_t launch_vam_predict(const VamArgs &a, hipStream_t s);   // dt, Q* into a.qs
// constraint rows of the corrector, right-hand side -R at the pressure pcur (null: 0)
hipError_t launch_vam_assemble(const VamArgs &a, const VamSystem &m, const double *pcur, hipStream_t s);
// block cyclic reduction: the n / 2 odd equations of a level of n equations
// (src) into the next level (dst)
hipError_t launch_vam_reduce(int n, const VamSystem &src, const VamSystem &dst, hipStream_t s);
// back substitution of a level of n equations into x ([4][n]) from the
// unknowns xup of the level above (null at the top)
hipError_t launch_vam_back(int n, const VamSystem &m, const double *xup, double *x, hipStream_t s);
// P = x (or P += x if accumulate)
hipError_t launch_vam_scatter(const VamArgs &a, const double *x, int accumulate, hipStream_t s);
hipError_t launch_vam_correct(const VamArgs &a, hipStream_t s);   // Q** in place, CFL ratio into slot sb

}  // namespace sme
