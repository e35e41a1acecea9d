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
    double *fac;        // [52][ceil(nb / 2)] factors of the even equations (E, F, g, B^-1)
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

// The last levels of a reduction, from the first level of at most kTailMax
// equations up to the one-equation top, reduced and back-substituted by one
// wave of kTailThreads threads in LDS.  m[i], x[i] and n[i] (i < count) are
// the system, unknowns and size of the tail's level i; i = 0 is its largest.
constexpr int kTailMax = 64;
constexpr int kTailLevels = 16;
constexpr int kTailThreads = 64;
static_assert((1 << (kTailLevels - 1)) > kTailMax, "a tail of n <= kTailMax equations has at most log2(n) + 1 levels");
struct VamTail {
    VamSystem m[kTailLevels];
    double *x[kTailLevels];
    int n[kTailLevels];
    int count;
};

hipError_t launch_vam_eig(const VamArgs &a, hipStream_t s);       // CFL ratio of a.q into slot sa
hipError_t launch_vam_predict(const VamArgs &a, hipStream_t s);   // dt, Q* into a.qs
// constraint rows of the corrector, right-hand side -R at P = 0
hipError_t launch_vam_assemble(const VamArgs &a, const VamSystem &m, hipStream_t s);
// right-hand side -R(Q**(P)) at the pressure a.p (the matrix is unchanged)
hipError_t launch_vam_residual(const VamArgs &a, const VamSystem &m, hipStream_t s);
// block cyclic reduction: the even equations of a level of n equations (src)
// factored, its n / 2 odd equations into the next level (dst); rhs_only: the
// right-hand side alone, on the factors stored by a full reduction
hipError_t launch_vam_reduce(int n, const VamSystem &src, const VamSystem &dst, bool rhs_only, hipStream_t s);
// back substitution of a level of n > 1 equations into x ([4][n]) from the
// unknowns xup of the level above
hipError_t launch_vam_back(int n, const VamSystem &m, const double *xup, double *x, hipStream_t s);
// the tail of a reduction, described by lv_dev (device memory)
hipError_t launch_vam_tail(const VamTail *lv_dev, bool rhs_only, hipStream_t s);
// P = x (or P += x if accumulate)
hipError_t launch_vam_scatter(const VamArgs &a, const double *x, int accumulate, hipStream_t s);
hipError_t launch_vam_correct(const VamArgs &a, hipStream_t s);   // Q** in place, CFL ratio into slot sb

}  // namespace sme
