// sme_band2d.h -- one band of the structured-grid SME step (device side).
//
// Fields (h, qx_0..qx_N, qy_0..qy_N), cell index j * nx + i.  A 64-lane wave
// owns 64 consecutive columns (62 outputs and one halo column on each side) of
// a band of `rows` rows and marches up the band:
//   * each cell's flux is evaluated once for both directions; the x-frame and
//     y-frame tangential blocks are the same quadratic form (A is symmetric);
//   * each lane computes the x-face to its right; the right cell's share moves
//     one lane up through a cross-lane shift;
//   * the y-face between the previous and the current row is computed once,
//     with the previous row held in registers (two register sets that swap
//     roles every row, so nothing is copied);
//   * rows reach registers through LDS: the loads of row j + 1 go straight
//     from memory into one of two per-wave LDS row buffers (buffer loads with
//     the LDS destination, one 4-byte word per lane) while row j is computed,
//     so the next row is in flight during the arithmetic without holding
//     registers.
// With a learned closure (CLOS, level 1) each finished cell also adds dt times
// the network's correction rates, computed from Q^n by the rates pass.
// Every face value is computed from the same inputs by the same code whichever
// wave computes it, so the result does not depend on how a grid is cut into
// strips and bands.
#pragma once

#include <hip/hip_runtime.h>

#include "sme_step_common.h"

namespace sme {
namespace detail {


template <int N>
struct Cell2 {
    static constexpr int n = N + 1;
    double h, b;
    double qx[n], qy[n];  // state as loaded (ghosts mirrored)
    double Fxx[n];        // x-frame normal block (x momenta), gravity included
    double Fyy[n];        // y-frame normal block (y momenta), gravity included
    double Ft[n];         // tangential block, identical in both frames
    double lx, ly;        // wave-speed bounds along x and y
};

template <int N>
struct Raw2 {
    double h, b;
    double qx[N + 1], qy[N + 1];
};

// ---- row staging through LDS

// doubles of one wave's staging area: two row buffers of (h, b, qx_0..qx_N,
// qy_0..qy_N), 64 columns each
template <int N>
constexpr int stage_doubles()
{
    return 2 * (2 * (N + 1) + 2) * kWave;
}

typedef __attribute__((address_space(3))) void lds_void_t;

// Per-lane byte offsets, within a row, of the two 4-byte words a lane stages:
// word w = 64 h + lane of a field row is half (lane & 1) of the double in
// column c0 + 32 h + lane / 2 (c0 = first column of the wave, ghosts mapped).
__device__ __forceinline__ void stage_offsets(const StepArgs &a, int c0, unsigned *voff)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        bool m;
        const int col = ghost_index(c0 + 32 * h + (lane >> 1), a.nx, a.bc[0], a.bc[1], m);
        voff[h] = (unsigned)col * 8u + 4u * (unsigned)(lane & 1);
    }
}

// Issue the loads of row j (ghost rows mapped) into a row buffer: field f of
// the row lands at buf[f * 64 + column - c0].  Returns at once; wait_staged()
// makes the data visible.
template <int N>
__device__ __forceinline__ void stage_row(const StepArgs &a, int j, const unsigned *voff, double *buf)
{
    constexpr int n = N + 1;
    bool my;
    const int row = ghost_index(j, a.ny, a.bc[2], a.bc[3], my);
    const int64_t r0 = (int64_t)row * a.nx;
    const int bytes = a.nx * 8;
    auto one = [&](const double *base, int f) {
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc((void *)(base + r0), (short)0, bytes, 0x00020000);
#pragma unroll
        for (int h = 0; h < 2; ++h)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t *)(buf + f * kWave + 32 * h), 4, voff[h], 0, 0,
                                                     0);
    };
    one(a.q, 0);
    one(a.b, 1);
#pragma unroll
    for (int k = 0; k < n; ++k) {
        one(a.q + (1 + k) * a.stride, 2 + k);
        one(a.q + (1 + n + k) * a.stride, 2 + n + k);
    }
}

// Every staged row (and every store) of this wave has landed.  Written as an
// asm statement with a memory clobber: the compiler does not track the LDS
// destination of these loads, and the intrinsic form of the wait is not a
// memory barrier, so the reads of a staged row could otherwise be scheduled
// before it.
__device__ __forceinline__ void wait_staged() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// row j from a row buffer into registers, with this lane's mirrors
template <int N>
__device__ __forceinline__ void read_row(const StepArgs &a, int j, bool mx, const double *buf, Raw2<N> &r)
{
    constexpr int n = N + 1;
    bool my;
    (void)ghost_index(j, a.ny, a.bc[2], a.bc[3], my);
    const int lane = threadIdx.x & (kWave - 1);
    r.h = buf[lane];
    r.b = buf[kWave + lane];
#pragma unroll
    for (int k = 0; k < n; ++k) {
        const double vx = buf[(2 + k) * kWave + lane];
        const double vy = buf[(2 + n + k) * kWave + lane];
        r.qx[k] = mx ? -vx : vx;
        r.qy[k] = my ? -vy : vy;
    }
}

template <int N>
__device__ __forceinline__ void cell_flux(Cell2<N> &c, const Raw2<N> &r, double g)
{
    constexpr int n = N + 1;
    c.h = r.h;
    c.b = r.b;
#pragma unroll
    for (int k = 0; k < n; ++k) {
        c.qx[k] = r.qx[k];
        c.qy[k] = r.qy[k];
    }
    const double ih = rcp(c.h);
    double al[n], be[n];
#pragma unroll
    for (int k = 0; k < n; ++k) {
        al[k] = c.qx[k] * ih;
        be[k] = c.qy[k] * ih;
    }
    quad_form<N>(c.qx, al, c.Fxx);
    quad_form<N>(c.qy, be, c.Fyy);
    quad_form<N>(c.qx, be, c.Ft);
    const double gh = g * c.h;
    const double p = 0.5 * gh * c.h;
    c.Fxx[0] += p;
    c.Fyy[0] += p;
    c.lx = lam_bound<N>(gh, al);
    c.ly = lam_bound<N>(gh, be);
}

template <int N>
__device__ __forceinline__ void x_side(const Cell2<N> &c, Side<N, true> &s)
{
    s.h = c.h;
    s.b = c.b;
#pragma unroll
    for (int k = 0; k <= N; ++k) {
        s.qa[k] = c.qx[k];
        s.qt[k] = c.qy[k];
        s.Fa[k] = c.Fxx[k];
        s.Ft[k] = c.Ft[k];
    }
    s.lam = c.lx;
}

template <int N>
__device__ __forceinline__ void y_side(const Cell2<N> &c, Side<N, true> &s)
{
    s.h = c.h;
    s.b = c.b;
#pragma unroll
    for (int k = 0; k <= N; ++k) {
        s.qa[k] = c.qy[k];
        s.qt[k] = c.qx[k];
        s.Fa[k] = c.Fyy[k];
        s.Ft[k] = c.Ft[k];
    }
    s.lam = c.ly;
}

// y-face between P (below) and C (above), normal +y.  Adds P's share to accP
// (if add_p) and, if SET_C, sets accC to C's share; both in physical field
// order, scaled by 1/dy.  (A compile-time flag rather than a null accC: a
// pointer test keeps the accumulator array in scratch memory at higher levels.)
template <int N, bool SET_C>
__device__ __forceinline__ void y_face(const StepArgs &a, const Cell2<N> &P, const Cell2<N> &C, double *accP,
                                       double *accC, bool add_p)
{
    constexpr int n = N + 1;
    Side<N, true> L, R;
    y_side<N>(P, L);
    y_side<N>(C, R);
    double Fh[2 * n + 1], D[2 * n + 1];
    face_flux<N, true>(L, R, a.g, a.quad, Fh, D);
    // frame [h, y.., x..] -> physical [h, x.., y..]
    if (add_p) {
        accP[0] = fma(a.idy, fma(0.5, D[0], Fh[0]), accP[0]);
#pragma unroll
        for (int k = 0; k < n; ++k) {
            accP[1 + n + k] = fma(a.idy, fma(0.5, D[1 + k], Fh[1 + k]), accP[1 + n + k]);
            accP[1 + k] = fma(a.idy, fma(0.5, D[1 + n + k], Fh[1 + n + k]), accP[1 + k]);
        }
    }
    if constexpr (SET_C) {
        accC[0] = a.idy * fma(0.5, D[0], -Fh[0]);
#pragma unroll
        for (int k = 0; k < n; ++k) {
            accC[1 + n + k] = a.idy * fma(0.5, D[1 + k], -Fh[1 + k]);
            accC[1 + k] = a.idy * fma(0.5, D[1 + n + k], -Fh[1 + n + k]);
        }
    }
}

// x-faces of the row of C: face to the right of each lane, neighbour via shuffle.
template <int N>
__device__ __forceinline__ void x_faces(const StepArgs &a, const Cell2<N> &C, double *accC)
{
    constexpr int n = N + 1;
    constexpr int nf = 2 * n + 1;
    Side<N, true> X, R;
    x_side<N>(C, X);
    R.h = shfl_dn(X.h);
    R.b = shfl_dn(X.b);
    R.lam = shfl_dn(X.lam);
#pragma unroll
    for (int k = 0; k < n; ++k) {
        R.qa[k] = shfl_dn(X.qa[k]);
        R.qt[k] = shfl_dn(X.qt[k]);
        R.Fa[k] = shfl_dn(X.Fa[k]);
        R.Ft[k] = shfl_dn(X.Ft[k]);
    }
    double Gh[nf], E[nf];
    face_flux<N, true>(X, R, a.g, a.quad, Gh, E);
#pragma unroll
    for (int f = 0; f < nf; ++f) {
        const double own = fma(0.5, E[f], Gh[f]);
        const double oth = fma(0.5, E[f], -Gh[f]);
        accC[f] = fma(a.idx, own + shfl_up1(oth), accC[f]);
    }
}

// predictor, friction, store, CFL ratio of the new state.  The cell is
// column col of the row starting at element rowoff (a wave-uniform value, so
// the stores address memory as a uniform base plus a 32-bit lane offset and
// no 64-bit per-lane address is held); step1 is the index of this step for
// the non-physical-state word (read once per band: a load of the slot here
// would make every row wait for its stores before reusing the register).
template <int N, bool CLOS, bool IMP>
__device__ __forceinline__ double finish_cell(const StepArgs &a, double dt, int64_t rowoff, int col, bool out,
                                              const Cell2<N> &c, const double *acc, long long step1)
{
    constexpr int n = N + 1;
    const double h = fma(-dt, acc[0], c.h);
    double qx[n], qy[n];
#pragma unroll
    for (int k = 0; k < n; ++k) {
        qx[k] = fma(-dt, acc[1 + k], c.qx[k]);
        qy[k] = fma(-dt, acc[1 + n + k], c.qy[k]);
    }
    const double ih = rcp(h);
    friction_step<N, true, IMP>(qx, qy, ih, dt, a.c_slip, a.nu);
    const unsigned uc = (unsigned)col;
    if constexpr (CLOS) {
        // learned closure: rates of (q_0, q_1) normal to x and to y from the rates pass
        if (out) {
            const float2 *rr = reinterpret_cast<const float2 *>(a.rates) + rowoff;
            const float2 rx = rr[uc];
            const float2 ry = (rr + a.stride)[uc];
            qx[0] = fma(dt, (double)rx.x, qx[0]);
            qx[1] = fma(dt, (double)rx.y, qx[1]);
            qy[0] = fma(dt, (double)ry.x, qy[0]);
            qy[1] = fma(dt, (double)ry.y, qy[1]);
        }
    }
    double r = 0.0;
    if (out) {
        double *const base = a.qn + rowoff;
        base[uc] = h;
        double sum = h;
#pragma unroll
        for (int k = 0; k < n; ++k) {
            (base + (int64_t)(1 + k) * a.stride)[uc] = qx[k];
            (base + (int64_t)(1 + n + k) * a.stride)[uc] = qy[k];
            sum += qx[k] + qy[k];
        }
        flag_bad_at(a, !(h > 0.0) || !isfinite(sum), step1);
        double lm;
        r = cfl_ratio_2d<N>(a.g, h, ih, qx, qy, a.idx, a.idy, &lm);
        if (!(r >= 0.0)) r = 0.0;
    }
    return r;
}

// one row: C <- row j (state in `raw`), y-face with P, finish P (row j-1) if
// requested, x-faces of C.
template <int N, bool CLOS, bool IMP>
__device__ __forceinline__ void row(const StepArgs &a, double dt, Cell2<N> &P, double *accP, Cell2<N> &C,
                                    double *accC, const Raw2<N> &raw, int j, int c, bool outc, bool finish_p,
                                    double &rmax, long long step1)
{
    cell_flux<N>(C, raw, a.g);
    y_face<N, true>(a, P, C, accP, accC, finish_p);
    if (finish_p)
        rmax = fmax(rmax, finish_cell<N, CLOS, IMP>(a, dt, (int64_t)(j - 1) * a.nx, c, outc, P, accP, step1));
    x_faces<N>(a, C, accC);
}

// closing y-face of the band: P is the last row (j1 - 1), raw the row above
template <int N, bool CLOS, bool IMP>
__device__ __forceinline__ void close_band(const StepArgs &a, double dt, Cell2<N> &P, double *accP,
                                           Cell2<N> &G, const Raw2<N> &raw, int j1, int c, bool outc,
                                           double &rmax, long long step1)
{
    cell_flux<N>(G, raw, a.g);
    y_face<N, false>(a, P, G, accP, nullptr, true);
    rmax = fmax(rmax, finish_cell<N, CLOS, IMP>(a, dt, (int64_t)(j1 - 1) * a.nx, c, outc, P, accP, step1));
}

// Whole band (strip sx, band sy) of one grid: returns the largest CFL ratio
// of the cells it wrote.  All 64 lanes of the wave must call it.  stage is
// this wave's staging area (stage_doubles<N>() doubles of LDS).
template <int N, bool CLOS = false, bool IMP = false>
__device__ __forceinline__ double band2d(const StepArgs &a, double dt, int sx, int sy, double *stage)
{
    constexpr int n = N + 1;
    constexpr int nf = 2 * n + 1;
    constexpr int rowd = (2 * n + 2) * kWave;  // doubles of one row buffer
    const int lane = threadIdx.x & (kWave - 1);
    const int c = sx * kOut - 1 + lane;
    const int j0 = sy * a.rows;
    const int j1 = min(j0 + a.rows, a.ny);
    bool mx;  // this lane's column is a wall ghost: its x momenta are mirrored
    (void)ghost_index(c, a.nx, a.bc[0], a.bc[1], mx);
    const bool outc = lane >= 1 && lane <= kOut && c < a.nx;
    double rmax = 0.0;
    // index of this step for the non-physical-state word, wave-uniform
    const long long st = a.slots[a.sa].step + 1;
    const long long step1 = (long long)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(st >> 32)) << 32) |
                                        (unsigned)__builtin_amdgcn_readfirstlane((int)st));
    Cell2<N> A, B;
    double accA[nf], accB[nf];
#pragma unroll
    for (int f = 0; f < nf; ++f) accA[f] = 0.0;
    double *const buf0 = stage, *const buf1 = stage + rowd;
    unsigned voff[2];
    stage_offsets(a, sx * kOut - 1, voff);
    Raw2<N> cur;
    stage_row<N>(a, j0 - 1, voff, buf0);
    stage_row<N>(a, j0, voff, buf1);
    wait_staged();
    read_row<N>(a, j0 - 1, mx, buf0, cur);
    cell_flux<N>(A, cur, a.g);  // halo row below the band
    int j = j0;                 // row j is staged in buf1
    while (true) {
        // buf0's previous row was read into registers before its arithmetic
        read_row<N>(a, j, mx, buf1, cur);
        stage_row<N>(a, j + 1, voff, buf0);  // next row, or the closing halo row
        row<N, CLOS, IMP>(a, dt, A, accA, B, accB, cur, j, c, outc, j > j0, rmax, step1);
        wait_staged();
        if (++j == j1) {
            read_row<N>(a, j1, mx, buf0, cur);
            close_band<N, CLOS, IMP>(a, dt, B, accB, A, cur, j1, c, outc, rmax, step1);
            break;
        }
        read_row<N>(a, j, mx, buf0, cur);
        stage_row<N>(a, j + 1, voff, buf1);
        row<N, CLOS, IMP>(a, dt, B, accB, A, accA, cur, j, c, outc, true, rmax, step1);
        wait_staged();
        if (++j == j1) {
            read_row<N>(a, j1, mx, buf1, cur);
            close_band<N, CLOS, IMP>(a, dt, A, accA, B, cur, j1, c, outc, rmax, step1);
            break;
        }
    }
    return rmax;
}

}  // namespace detail
}  // namespace sme
