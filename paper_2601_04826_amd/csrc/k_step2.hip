// k_step2.hip -- second-order SME step on 1D and structured 2D grids.
//
// Reconstruction (compute_derivatives, Sec. 2.1.2, with a limiter): per cell
// and axis the variables v = (eta = h + b, q_1 .. q_{nf-1}, b) get the slope
// sigma = minmod(v_i - v_minus, v_plus - v_i) per cell width (across a
// boundary the neighbour is the cell's ghost: a copy, or for a wall the copy
// with its normal momenta mirrored); the face values are v_i -/+ sigma / 2 and
// h = eta - b, so the lake at rest stays exact.  A cell whose face depth would
// not be positive keeps zero slopes.  k_recon writes the slopes to a scratch
// array slopes[(axis * nv + f) * stride + cell].
//
// Semi-discrete operator (path-conservative finite volumes of second order,
// Sec. 2.1.2): every face carries the Rusanov flux and the path fluctuation
// between the two reconstructed face values (the neighbour's own face value,
// or the ghost of this cell's one at a boundary), evaluated in the canonical
// orientation (minus side left, normal +axis) so the two cells of a face see
// bitwise equal values; the left cell takes Fhat + D/2, the right -Fhat + D/2.
// Each cell adds, per axis, the fluctuation inside it along the straight path
// from its minus-face to its plus-face value (normal +axis).
//
// Time: two-stage SSP Runge-Kutta (Heun) for the hyperbolic part,
//   stage 1  Q1 = Q^n + dt L(Q^n)                       (written to the other buffer)
//   stage 2  Q2 = Q^n / 2 + (Q1 + dt L(Q1)) / 2         (in place over Q^n)
// then the friction step of the splitting (Eq. (3d)) on Q2, and the CFL ratio
// of the new state is reduced for the next step (Sec. 3.1).  One lane per
// cell; blocks are dealt die-major so neighbouring rows share an L2.
#include <hip/hip_runtime.h>

#include "sme_step_common.h"

namespace sme {

using namespace detail;

namespace {

template <int N, int DIM>
struct Shape2 {
    static constexpr int n = N + 1;
    static constexpr int nf = DIM == 1 ? N + 2 : 2 * N + 3;  // state fields
    static constexpr int nv = nf + 1;                          // reconstruction variables
};

__device__ __forceinline__ double minmod(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}

// die-major cell index of this lane (each XCD walks one contiguous range)
__device__ __forceinline__ int64_t cell_index()
{
    const int nblk = (int)gridDim.x;
    const int per_xcd = (nblk + kXcd - 1) / kXcd;
    const int64_t blk = (int64_t)(blockIdx.x % kXcd) * per_xcd + (blockIdx.x / kXcd);
    return blk * kBlock + threadIdx.x;
}

// reconstruction variables of cell c (mirror: the normal momenta of axis ax
// change sign, the ghost of a wall)
template <int N, int DIM>
__device__ __forceinline__ void load_v(const StepArgs &a, int64_t c, bool mirror, int ax, double *v)
{
    using S = Shape2<N, DIM>;
    const double h = a.q[c], b = a.b[c];
    v[0] = h + b;
#pragma unroll
    for (int f = 1; f < S::nf; ++f) v[f] = a.q[(int64_t)f * a.stride + c];
    v[S::nf] = b;
    if (mirror) {
        const int first = 1 + ax * S::n;  // qx block (axis 0) or qy block (axis 1)
#pragma unroll
        for (int k = 0; k < S::n; ++k) v[first + k] = -v[first + k];
    }
}

// neighbour of (ix, iy) along axis ax (side -1 or +1): cell index and mirror flag
template <int DIM>
__device__ __forceinline__ int64_t nbr_of(const StepArgs &a, int ix, int iy, int ax, int side, bool &mirror)
{
    if (ax == 0) {
        const int c = ghost_index(ix + side, a.nx, a.bc[0], a.bc[1], mirror);
        return (int64_t)iy * a.nx + c;
    }
    const int r = ghost_index(iy + side, a.ny, a.bc[2], a.bc[3], mirror);
    return (int64_t)r * a.nx + ix;
}

template <int N, int DIM>
__global__ __launch_bounds__(kBlock) void k_recon(StepArgs a, double *slopes)
{
    using S = Shape2<N, DIM>;
    const int64_t i = cell_index();
    if (i >= a.ncells) return;
    const int ix = (int)(i % a.nx), iy = (int)(i / a.nx);
    double vi[S::nv];
    load_v<N, DIM>(a, i, false, 0, vi);
    double sg[DIM][S::nv];
    bool ok = true;
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax) {
        double vm[S::nv], vp[S::nv];
        bool mm, mp;
        const int64_t cm = nbr_of<DIM>(a, ix, iy, ax, -1, mm);
        const int64_t cp = nbr_of<DIM>(a, ix, iy, ax, 1, mp);
        load_v<N, DIM>(a, cm, mm, ax, vm);
        load_v<N, DIM>(a, cp, mp, ax, vp);
#pragma unroll
        for (int f = 0; f < S::nv; ++f) sg[ax][f] = minmod(vi[f] - vm[f], vp[f] - vi[f]);
        // positive face depths on both sides, else first order
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const double hs = side ? 0.5 : -0.5;
            const double eta = vi[0] + hs * sg[ax][0], b = vi[S::nf] + hs * sg[ax][S::nf];
            ok = ok && (eta - b > 0.0);
        }
    }
#pragma unroll
    for (int ax = 0; ax < DIM; ++ax)
#pragma unroll
        for (int f = 0; f < S::nv; ++f) slopes[(int64_t)(ax * S::nv + f) * a.stride + i] = ok ? sg[ax][f] : 0.0;
}

// reconstructed face value of cell c on side hs (-0.5 minus, +0.5 plus) of
// axis ax, as a frame side of that axis (normal +axis): h, b, qa, qt
template <int N, int DIM>
__device__ __forceinline__ void face_side(const StepArgs &a, const double *slopes, int64_t c, int ax, double hs,
                                          Side<N, DIM == 2> &S)
{
    using Sh = Shape2<N, DIM>;
    constexpr int n = Sh::n;
    const double *sl = slopes + (int64_t)ax * Sh::nv * a.stride;
    const double b = a.b[c] + hs * sl[(int64_t)Sh::nf * a.stride + c];
    const double eta = (a.q[c] + a.b[c]) + hs * sl[c];
    S.h = eta - b;
    S.b = b;
    double qx[n], qy[DIM == 2 ? n : 1];
#pragma unroll
    for (int k = 0; k < n; ++k) qx[k] = a.q[(int64_t)(1 + k) * a.stride + c] + hs * sl[(int64_t)(1 + k) * a.stride + c];
    if constexpr (DIM == 2) {
#pragma unroll
        for (int k = 0; k < n; ++k)
            qy[k] = a.q[(int64_t)(1 + n + k) * a.stride + c] + hs * sl[(int64_t)(1 + n + k) * a.stride + c];
    }
#pragma unroll
    for (int k = 0; k < n; ++k) {
        if constexpr (DIM == 2) {
            S.qa[k] = ax == 0 ? qx[k] : qy[k];
            S.qt[k] = ax == 0 ? qy[k] : -qx[k];
        } else {
            S.qa[k] = qx[k];
        }
    }
}

// add a frame-field contribution (weight wgt) to the x/y accumulators
template <int N, int DIM>
__device__ __forceinline__ void add_frame(double *acc, const double *F, int ax, double wgt)
{
    constexpr int n = N + 1;
    acc[0] = fma(wgt, F[0], acc[0]);
#pragma unroll
    for (int k = 0; k < n; ++k) {
        if constexpr (DIM == 2) {
            if (ax == 0) {
                acc[1 + k] = fma(wgt, F[1 + k], acc[1 + k]);
                acc[1 + n + k] = fma(wgt, F[1 + n + k], acc[1 + n + k]);
            } else {
                acc[1 + n + k] = fma(wgt, F[1 + k], acc[1 + n + k]);
                acc[1 + k] = fma(-wgt, F[1 + n + k], acc[1 + k]);
            }
        } else {
            acc[1 + k] = fma(wgt, F[1 + k], acc[1 + k]);
        }
    }
}

// STAGE 1: qn = q + dt L(q).  STAGE 2: qn = qn / 2 + (q + dt L(q)) / 2 in
// place over qn, then friction, store, CFL ratio of the new state.
template <int N, int DIM, int STAGE, bool IMP>
__global__ __launch_bounds__(kBlock) void k_flux2(StepArgs a, const double *slopes)
{
    using Sh = Shape2<N, DIM>;
    constexpr int n = N + 1;
    constexpr int nf = Sh::nf;
    constexpr bool TAN = DIM == 2;
    const double dt = step_dt(a);
    if (STAGE == 2 && blockIdx.x == 0 && threadIdx.x == 0) slot_update(a, dt);
    const int64_t i = cell_index();
    const bool live = i < a.ncells;
    double rmax = 0.0;
    if (live && dt == 0.0) {
        // past the end time: the state stays (stage 1 copies it for stage 2,
        // stage 2 leaves it in place) and the CFL ratio carries over
        if (STAGE == 1)
            for (int f = 0; f < nf; ++f) a.qn[(int64_t)f * a.stride + i] = a.q[(int64_t)f * a.stride + i];
    } else if (live) {
        const int ix = (int)(i % a.nx), iy = (int)(i / a.nx);
        double acc[nf];
#pragma unroll
        for (int f = 0; f < nf; ++f) acc[f] = 0.0;
        for (int ax = 0; ax < DIM; ++ax) {
            const double inv_d = ax == 0 ? a.idx : a.idy;  // |e| / |V| of this axis' faces
            for (int side = 0; side < 2; ++side) {
                // the face on this side: L = minus-side value, R = plus-side value
                bool mirror;
                const int64_t j = nbr_of<DIM>(a, ix, iy, ax, side ? 1 : -1, mirror);
                const bool ghost = (ax == 0) ? (side ? ix + 1 >= a.nx && a.bc[1] != BC_PERIODIC
                                                     : ix == 0 && a.bc[0] != BC_PERIODIC)
                                             : (side ? iy + 1 >= a.ny && a.bc[3] != BC_PERIODIC
                                                     : iy == 0 && a.bc[2] != BC_PERIODIC);
                Side<N, TAN> own, oth;
                face_side<N, DIM>(a, slopes, i, ax, side ? 0.5 : -0.5, own);
                if (ghost) {
                    oth = own;
                    if (mirror) {
#pragma unroll
                        for (int k = 0; k < n; ++k) oth.qa[k] = -oth.qa[k];
                    }
                } else {
                    face_side<N, DIM>(a, slopes, j, ax, side ? -0.5 : 0.5, oth);
                }
                Side<N, TAN> &L = side ? own : oth;
                Side<N, TAN> &R = side ? oth : own;
                side_flux<N, TAN>(L, a.g);
                side_flux<N, TAN>(R, a.g);
                double Fh[nf], D[nf];
                face_flux<N, TAN>(L, R, a.g, a.quad, Fh, D);
                // this cell is the left one on its plus face, the right one on its minus face
                double C[nf];
#pragma unroll
                for (int f = 0; f < nf; ++f) C[f] = side ? fma(0.5, D[f], Fh[f]) : fma(0.5, D[f], -Fh[f]);
                add_frame<N, DIM>(acc, C, ax, inv_d);
            }
            // in-cell fluctuation from the minus-face to the plus-face value
            Side<N, TAN> m, p;
            face_side<N, DIM>(a, slopes, i, ax, -0.5, m);
            face_side<N, DIM>(a, slopes, i, ax, 0.5, p);
            double dqa[n], dqt[TAN ? n : 1], D[nf];
#pragma unroll
            for (int k = 0; k < n; ++k) {
                dqa[k] = p.qa[k] - m.qa[k];
                if constexpr (TAN) dqt[k] = p.qt[k] - m.qt[k];
            }
            nc_fluct<N, TAN>(m, p, a.g, a.quad, dqa, dqt, D);
            add_frame<N, DIM>(acc, D, ax, inv_d);
        }
        double qnew[nf];
#pragma unroll
        for (int f = 0; f < nf; ++f) {
            const double q1 = fma(-dt, acc[f], a.q[(int64_t)f * a.stride + i]);
            qnew[f] = STAGE == 1 ? q1 : 0.5 * a.qn[(int64_t)f * a.stride + i] + 0.5 * q1;
        }
        if constexpr (STAGE == 2) {
            const double ih = rcp(qnew[0]);
            friction_step<N, DIM == 2, IMP>(qnew + 1, DIM == 2 ? qnew + 1 + n : nullptr, ih, dt, a.c_slip, a.nu);
            bool bad = !(qnew[0] > 0.0) || !isfinite(qnew[0]);
#pragma unroll
            for (int f = 1; f < nf; ++f) bad |= !isfinite(qnew[f]);
            flag_bad(a, bad);
            double lm;
            if constexpr (DIM == 2)
                rmax = cfl_ratio_2d<N>(a.g, qnew[0], ih, qnew + 1, qnew + 1 + n, a.idx, a.idy, &lm);
            else
                rmax = cfl_ratio_1d<N>(a.g, qnew[0], ih, qnew + 1, a.idx, &lm);
            if (!(rmax >= 0.0)) rmax = 0.0;
        }
#pragma unroll
        for (int f = 0; f < nf; ++f) a.qn[(int64_t)f * a.stride + i] = qnew[f];
    }
    if constexpr (STAGE == 2) {
        if (dt == 0.0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
                for (int w = 0; w < kRatioWords; ++w) a.slots[a.sb].r[w].bits = a.slots[a.sa].r[w].bits;
                a.slots[a.sb].lbits = a.slots[a.sa].lbits;
            }
        } else {
            publish_ratio(a.slots[a.sb], rmax);
        }
    }
}

}  // namespace

unsigned step2_grid(int64_t ncells) { return (blocks_for(ncells) + kXcd - 1) / kXcd * kXcd; }

hipError_t launch_recon2(int level, int dim, const StepArgs &a, double *slopes, hipStream_t s)
{
    const unsigned grid = step2_grid(a.ncells);
#define RC1(N) hipLaunchKernelGGL((k_recon<N, 1>), dim3(grid), dim3(kBlock), 0, s, a, slopes)
#define RC2(N) hipLaunchKernelGGL((k_recon<N, 2>), dim3(grid), dim3(kBlock), 0, s, a, slopes)
    if (dim == 1) {
        SME_LEVEL_SWITCH(level, RC1)
    } else {
        SME_LEVEL_SWITCH(level, RC2)
    }
#undef RC1
#undef RC2
    return hipGetLastError();
}

hipError_t launch_flux2(int level, int dim, int stage, const StepArgs &a, const double *slopes, hipStream_t s)
{
    const unsigned grid = step2_grid(a.ncells);
#define FX(N, D, S, I) hipLaunchKernelGGL((k_flux2<N, D, S, I>), dim3(grid), dim3(kBlock), 0, s, a, slopes)
#define F11(N) FX(N, 1, 1, false)
#define F12(N) FX(N, 1, 2, false)
#define F12I(N) FX(N, 1, 2, true)
#define F21(N) FX(N, 2, 1, false)
#define F22(N) FX(N, 2, 2, false)
#define F22I(N) FX(N, 2, 2, true)
    if (dim == 1) {
        if (stage == 1) {
            SME_LEVEL_SWITCH(level, F11)
        } else if (a.implicit) {
            SME_LEVEL_SWITCH(level, F12I)
        } else {
            SME_LEVEL_SWITCH(level, F12)
        }
    } else {
        if (stage == 1) {
            SME_LEVEL_SWITCH(level, F21)
        } else if (a.implicit) {
            SME_LEVEL_SWITCH(level, F22I)
        } else {
            SME_LEVEL_SWITCH(level, F22)
        }
    }
#undef FX
#undef F11
#undef F12
#undef F12I
#undef F21
#undef F22
#undef F22I
    return hipGetLastError();
}

}  // namespace sme
