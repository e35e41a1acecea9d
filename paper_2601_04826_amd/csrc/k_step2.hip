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
// of the new state is reduced for the next step (Sec. 3.1).
//
// Two implementations: on structured grids up to level 6 each stage is one
// banded launch that computes the slopes itself and evaluates every face once
// (k_stage2_band, below); on 1D grids and at levels 7-8, k_recon writes the
// slopes and k_flux2 takes one lane per cell (blocks dealt die-major so
// neighbouring rows share an L2), each face evaluated by both of its cells.
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


// ---- structured grids: reconstruction fused into the stage, one wave per band
//
// A 64-lane wave owns 64 consecutive columns (62 outputs and one halo column
// on each side) of a band of a.rows rows and marches up the band, as the
// first-order step does.  Per row it computes the limited slopes itself
// (along x from the neighbouring lanes, the two edge lanes reading their
// outer neighbour; along y from the rows below and above, held in registers),
// the four reconstructed face values of each cell with their fluxes, the
// x-face to the right of each lane (the right cell's share moves one lane up),
// the y-face between the previous and the current row (the previous row's
// upper face value held in registers) and both in-cell fluctuations.  Each
// face is evaluated once; no slopes array is written or read.  The slopes,
// face values and faces are computed by the same code from the same inputs
// whichever wave computes them, so results do not depend on the cut into
// strips and bands.

// index of column or row c of a grid of n with up to two halo cells per side:
// periodic ends wrap; beyond a wall or open end the nearest cell (mirror:
// the ghost of a wall, whose normal momenta change sign)
__device__ __forceinline__ int halo_index(int c, int n, int bc_lo, int bc_hi, bool &mirror)
{
    mirror = false;
    if (c < 0) {
        if (bc_lo == BC_PERIODIC) return ((c % n) + n) % n;
        mirror = bc_lo == BC_WALL;
        return 0;
    }
    if (c >= n) {
        if (bc_hi == BC_PERIODIC) return c % n;
        mirror = bc_hi == BC_WALL;
        return n - 1;
    }
    return c;
}

// the reconstruction variables (eta = h + b, qx, qy, b) of the cell at
// (column col, row row), x momenta mirrored if mx, y momenta if my
template <int N>
__device__ __forceinline__ void load_rv(const StepArgs &a, int col, int row, bool mx, bool my, double *v)
{
    constexpr int n = N + 1, nf = 2 * n + 1;
    const int64_t c = (int64_t)row * a.nx + col;
    const double h = a.q[c], b = a.b[c];
    v[0] = h + b;
#pragma unroll
    for (int k = 0; k < n; ++k) {
        const double qx = a.q[(int64_t)(1 + k) * a.stride + c];
        const double qy = a.q[(int64_t)(1 + n + k) * a.stride + c];
        v[1 + k] = mx ? -qx : qx;
        v[1 + n + k] = my ? -qy : qy;
    }
    v[nf] = b;
}

// one row of the wave: this lane's column, mapped, and its mirror flags
struct Lane2 {
    int col;      // column of this lane (halo columns mapped)
    bool mx;      // this lane's column is a wall ghost
    int colo;     // outer neighbour column of an edge lane (lane 0: c - 1, lane 63: c + 1)
    bool mxo;
};

// reconstruction variables of row j at this lane, and the outer neighbour's
// for the two edge lanes
template <int N>
__device__ __forceinline__ void load_row_rv(const StepArgs &a, const Lane2 &L, int j, double *v, double *vo,
                                            bool edge)
{
    bool my;
    const int row = halo_index(j, a.ny, a.bc[2], a.bc[3], my);
    load_rv<N>(a, L.col, row, L.mx, my, v);
    if (edge) load_rv<N>(a, L.colo, row, L.mxo, my, vo);
}

// Face value of a cell on side hs of axis AX (normal +axis frame) from its
// variables v and slopes s, with the flux of that side.
template <int N, int AX>
__device__ __forceinline__ void rv_side(const double *v, const double *s, double hs, double g, Side<N, true> &S)
{
    constexpr int n = N + 1, nf = 2 * n + 1;
    const double b = v[nf] + hs * s[nf];
    const double eta = v[0] + hs * s[0];
    S.h = eta - b;
    S.b = b;
#pragma unroll
    for (int k = 0; k < n; ++k) {
        const double qx = v[1 + k] + hs * s[1 + k];
        const double qy = v[1 + n + k] + hs * s[1 + n + k];
        S.qa[k] = AX == 0 ? qx : qy;
        S.qt[k] = AX == 0 ? qy : -qx;
    }
    side_flux<N, true>(S, g);
}

// the value outside a wall or open end: this side's value, the normal
// momenta (and so the tangential flux block) negated at a wall
template <int N>
__device__ __forceinline__ void outside_of(const Side<N, true> &s, bool wall, Side<N, true> &o)
{
    o = s;
    if (wall) {
#pragma unroll
        for (int k = 0; k <= N; ++k) {
            o.qa[k] = -s.qa[k];
            o.Ft[k] = -s.Ft[k];
        }
    }
}

template <int N>
__device__ __forceinline__ void shfl_dn_side(const Side<N, true> &s, Side<N, true> &r)
{
    r.h = shfl_dn(s.h);
    r.b = shfl_dn(s.b);
    r.lam = shfl_dn(s.lam);
#pragma unroll
    for (int k = 0; k <= N; ++k) {
        r.qa[k] = shfl_dn(s.qa[k]);
        r.qt[k] = shfl_dn(s.qt[k]);
        r.Fa[k] = shfl_dn(s.Fa[k]);
        r.Ft[k] = shfl_dn(s.Ft[k]);
    }
}

// in-cell fluctuation of axis AX from the minus to the plus face value, added
// to the physical-order accumulator with weight w
template <int N, int AX>
__device__ __forceinline__ void in_cell(const StepArgs &a, const Side<N, true> &m, const Side<N, true> &p, double w,
                                        double *acc)
{
    constexpr int n = N + 1, nf = 2 * n + 1;
    double dqa[n], dqt[n], D[nf];
#pragma unroll
    for (int k = 0; k < n; ++k) {
        dqa[k] = p.qa[k] - m.qa[k];
        dqt[k] = p.qt[k] - m.qt[k];
    }
    nc_fluct<N, true>(m, p, a.g, a.quad, dqa, dqt, D);
    add_frame<N, 2>(acc, D, AX, w);
}

// the stage update of a finished cell (row j, this lane), and for stage 2
// friction, the non-physical-state flag and the CFL ratio of the result
template <int N, int STAGE, bool IMP>
__device__ __forceinline__ double finish2(const StepArgs &a, double dt, int j, int c, bool out, const double *acc,
                                          long long step1)
{
    constexpr int n = N + 1, nf = 2 * n + 1;
    if (!out) return 0.0;
    const int64_t i = (int64_t)j * a.nx + c;
    double qnew[nf];
#pragma unroll
    for (int f = 0; f < nf; ++f) {
        const double q1 = fma(-dt, acc[f], a.q[(int64_t)f * a.stride + i]);
        qnew[f] = STAGE == 1 ? q1 : 0.5 * a.qn[(int64_t)f * a.stride + i] + 0.5 * q1;
    }
    double r = 0.0;
    if constexpr (STAGE == 2) {
        const double ih = rcp(qnew[0]);
        friction_step<N, true, IMP>(qnew + 1, qnew + 1 + n, ih, dt, a.c_slip, a.nu);
        bool bad = !(qnew[0] > 0.0) || !isfinite(qnew[0]);
#pragma unroll
        for (int f = 1; f < nf; ++f) bad |= !isfinite(qnew[f]);
        flag_bad_at(a, bad, step1);
        double lm;
        r = cfl_ratio_2d<N>(a.g, qnew[0], ih, qnew + 1, qnew + 1 + n, a.idx, a.idy, &lm);
        if (!(r >= 0.0)) r = 0.0;
    }
#pragma unroll
    for (int f = 0; f < nf; ++f) a.qn[(int64_t)f * a.stride + i] = qnew[f];
    return r;
}

// limited slope of variable f along x of this lane's cell, from its
// neighbours' values (lanes -/+ 1, or the edge lanes' outer neighbours vo)
__device__ __forceinline__ double slope_x(const double *v, const double *vo, int lane, int f)
{
    const double vl = shfl_up1(v[f]), vr = shfl_dn(v[f]);
    const double l = lane == 0 ? vo[f] : vl;
    const double r = lane == kWave - 1 ? vo[f] : vr;
    return minmod(v[f] - l, r - v[f]);
}

// Whole band (strip sxi, band syi) of one stage; returns the largest CFL
// ratio of the cells written (stage 2).  All 64 lanes of the wave must call
// it.  Per row the work is ordered so that one slope vector and at most three
// face values are live at a time.
template <int N, int STAGE, bool IMP>
__device__ __forceinline__ double band2_o2(const StepArgs &a, double dt, int sxi, int syi, long long step1)
{
    constexpr int n = N + 1, nf = 2 * n + 1, nv = nf + 1;
    const int lane = threadIdx.x & (kWave - 1);
    const int c = sxi * kOut - 1 + lane;
    const int j0 = syi * a.rows;
    const int j1 = min(j0 + a.rows, a.ny);
    Lane2 L;
    L.col = halo_index(c, a.nx, a.bc[0], a.bc[1], L.mx);
    L.colo = halo_index(lane == 0 ? c - 1 : c + 1, a.nx, a.bc[0], a.bc[1], L.mxo);
    const bool edge = lane == 0 || lane == kWave - 1;
    const bool outc = lane >= 1 && lane <= kOut && c < a.nx;
    // x boundary faces: this lane's face to the right is the west boundary
    // (c == -1) or the east boundary (c == nx - 1); the inner cell's own face
    // value stands outside
    const bool bnd_lo = c == -1 && a.bc[0] != BC_PERIODIC;
    const bool bnd_hi = c == a.nx - 1 && a.bc[1] != BC_PERIODIC;
    const bool wall_lo = a.bc[0] == BC_WALL, wall_hi = a.bc[1] == BC_WALL;
    double vd[nv], v[nv], vu[nv], vo[nv];
    double rmax = 0.0;
    // rows j0 - 2 .. j0 - 1 in registers: the slopes of the halo row j0 - 1 need the row below it
    load_row_rv<N>(a, L, j0 - 2, vd, vo, false);
    load_row_rv<N>(a, L, j0 - 1, v, vo, edge);
    Side<N, true> Pp;  // upper face value of the previous row
    double accP[nf];   // the previous row's accumulator
    for (int j = j0 - 1; j <= j1; ++j) {
        // v: row j (vo: its edge-lane outer neighbours); vd: row j - 1
        load_row_rv<N>(a, L, j + 1, vu, vo, false);
        // first order where a face depth would not be positive (eta and b slopes of both axes)
        bool ok = true;
        {
            const double se = slope_x(v, vo, lane, 0), sb = slope_x(v, vo, lane, nf);
            const double te = minmod(v[0] - vd[0], vu[0] - v[0]), tb = minmod(v[nf] - vd[nf], vu[nf] - v[nf]);
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const double hs = side ? 0.5 : -0.5;
                ok = ok && ((v[0] + hs * se) - (v[nf] + hs * sb) > 0.0);
            }
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const double hs = side ? 0.5 : -0.5;
                ok = ok && ((v[0] + hs * te) - (v[nf] + hs * tb) > 0.0);
            }
        }
        double sl[nv];
#pragma unroll
        for (int f = 0; f < nv; ++f) sl[f] = ok ? minmod(v[f] - vd[f], vu[f] - v[f]) : 0.0;
        Side<N, true> ym;
        rv_side<N, 1>(v, sl, -0.5, a.g, ym);
        double accC[nf];
        if (j >= j0) {
            // y-face between rows j - 1 (Pp) and j (ym); at a south or north
            // wall or open end the inner value stands outside
            if (j == 0 && a.bc[2] != BC_PERIODIC) outside_of<N>(ym, a.bc[2] == BC_WALL, Pp);
            if (j == a.ny && a.bc[3] != BC_PERIODIC) outside_of<N>(Pp, a.bc[3] == BC_WALL, ym);
            double Fh[nf], D[nf];
            face_flux<N, true>(Pp, ym, a.g, a.quad, Fh, D);
            if (j > j0) {
                double C[nf];
#pragma unroll
                for (int f = 0; f < nf; ++f) C[f] = fma(0.5, D[f], Fh[f]);
                add_frame<N, 2>(accP, C, 1, a.idy);
                rmax = fmax(rmax, finish2<N, STAGE, IMP>(a, dt, j - 1, c, outc, accP, step1));
            }
            if (j == j1) break;
#pragma unroll
            for (int f = 0; f < nf; ++f) accC[f] = 0.0;
            double C[nf];
#pragma unroll
            for (int f = 0; f < nf; ++f) C[f] = fma(0.5, D[f], -Fh[f]);
            add_frame<N, 2>(accC, C, 1, a.idy);
        }
        rv_side<N, 1>(v, sl, 0.5, a.g, Pp);
        if (j >= j0) {
            in_cell<N, 1>(a, ym, Pp, a.idy, accC);
#pragma unroll
            for (int f = 0; f < nv; ++f) sl[f] = ok ? slope_x(v, vo, lane, f) : 0.0;
            Side<N, true> xm, xp;
            rv_side<N, 0>(v, sl, -0.5, a.g, xm);
            rv_side<N, 0>(v, sl, 0.5, a.g, xp);
            in_cell<N, 0>(a, xm, xp, a.idx, accC);
            // x-face to the right: this lane's plus value, the next lane's minus value
            Side<N, true> R;
            shfl_dn_side<N>(xm, R);
            if (bnd_lo) outside_of<N>(R, wall_lo, xp);
            if (bnd_hi) outside_of<N>(xp, wall_hi, R);
            double Gh[nf], E[nf];
            face_flux<N, true>(xp, R, a.g, a.quad, Gh, E);
#pragma unroll
            for (int f = 0; f < nf; ++f) {
                const double own = fma(0.5, E[f], Gh[f]);
                const double oth = fma(0.5, E[f], -Gh[f]);
                accP[f] = fma(a.idx, own + shfl_up1(oth), accC[f]);
            }
        }
#pragma unroll
        for (int f = 0; f < nv; ++f) {
            vd[f] = v[f];
            v[f] = vu[f];
        }
        // the edge lanes' outer neighbours of the next row
        if (edge) {
            bool my;
            const int row = halo_index(j + 1, a.ny, a.bc[2], a.bc[3], my);
            load_rv<N>(a, L.colo, row, L.mxo, my, vo);
        }
    }
    return rmax;
}

// resident waves per SIMD the band stages aim for: two while the row's live
// set fits 256 registers, one above (the accumulation registers then hold
// what does not fit)
template <int N>
constexpr int waves_o2()
{
    return N <= 1 ? 2 : 1;
}

// STAGE 1: Q1 = Q^n + dt L(Q^n) into a.qn.  STAGE 2: Q = Q^n / 2 + (Q1 + dt L(Q1)) / 2
// in place over a.qn (= Q^n), then friction, the CFL ratio of the result.
template <int N, int STAGE, bool IMP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(waves_o2<N>()))) void k_stage2_band(StepArgs a)
{
    constexpr int nf = 2 * N + 3;
    const double dt = step_dt(a);
    if (STAGE == 2 && blockIdx.x == 0 && threadIdx.x == 0) slot_update(a, dt);
    if (dt == 0.0) {
        // past the end time: the state stays and the CFL ratio carries over
        const int64_t nth = (int64_t)gridDim.x * blockDim.x;
        const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (STAGE == 1)
            for (int f = 0; f < nf; ++f)
                for (int64_t i = t0; i < a.ncells; i += nth) a.qn[f * a.stride + i] = a.q[f * a.stride + i];
        if (STAGE == 2 && t0 == 0) {
#pragma unroll
            for (int w = 0; w < kRatioWords; ++w) a.slots[a.sb].r[w].bits = a.slots[a.sa].r[w].bits;
            a.slots[a.sb].lbits = a.slots[a.sa].lbits;
        }
        return;
    }
    const int nsx = (a.nx + kOut - 1) / kOut;
    const int nsy = (a.ny + a.rows - 1) / a.rows;
    const int nblk = (int)gridDim.x;
    const int per_xcd = (nblk + kXcd - 1) / kXcd;
    const int slot = (int)(blockIdx.x % kXcd) * per_xcd + (int)(blockIdx.x / kXcd);
    const int wave = __builtin_amdgcn_readfirstlane(slot * (kBlock / kWave) + (int)(threadIdx.x >> 6));
    const long long st = a.slots[a.sa].step + 1;
    double rmax = 0.0;
    if (wave < nsx * nsy) rmax = band2_o2<N, STAGE, IMP>(a, dt, wave % nsx, wave / nsx, st);
    if constexpr (STAGE == 2) publish_ratio(a.slots[a.sb], rmax);
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

hipError_t launch_stage2_band(int level, int stage, const StepArgs &a, hipStream_t s)
{
    const int64_t nsx = (a.nx + kOut - 1) / kOut;
    const int64_t nsy = (a.ny + a.rows - 1) / a.rows;
    const int64_t blocks = (nsx * nsy * kWave + kBlock - 1) / kBlock;
    const unsigned grid = (unsigned)((blocks + kXcd - 1) / kXcd * kXcd);
#define B(N, S, I) hipLaunchKernelGGL((k_stage2_band<N, S, I>), dim3(grid), dim3(kBlock), 0, s, a)
#define B1(N) B(N, 1, false)
#define B2(N) B(N, 2, false)
#define B2I(N) B(N, 2, true)
#define BAND_SWITCH(CALL)        \
    switch (level) {             \
    case 0: CALL(0); break;      \
    case 1: CALL(1); break;      \
    case 2: CALL(2); break;      \
    case 3: CALL(3); break;      \
    case 4: CALL(4); break;      \
    case 5: CALL(5); break;      \
    case 6: CALL(6); break;      \
    default: return hipErrorInvalidValue; \
    }
    static_assert(kStage2BandMaxLevel == 6, "the switch below lists the band levels");
    if (stage == 1) {
        BAND_SWITCH(B1)
    } else if (a.implicit) {
        BAND_SWITCH(B2I)
    } else {
        BAND_SWITCH(B2)
    }
#undef BAND_SWITCH
#undef B
#undef B1
#undef B2
#undef B2I
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
