// k_vam.hip -- non-hydrostatic VAM predictor-corrector step in 1D (Sec. 3.3,
// the splitting of Sec. 2.1.2).
//
// Fields (h, h u0, h u1, h w0, h w1); the vertical velocity's quadratic
// coefficient w2 = -(w0 + w1) + (u0 + u1) b_x follows from the kinematic bed
// condition.  A step is
//   predictor  Q* = Q^n - dt/dx (F^_{i+1/2} - F^_{i-1/2} + D_{i+1/2}/2 + D_{i-1/2}/2)
//              path-conservative Rusanov with the printed flux F and
//              non-conservative matrix (bed as an NC column g h b_x beside g h h_x),
//              straight path, G-point Gauss, speed bound |u0| + sqrt(g h + u1^2);
//   corrector  Q** = Q* + dt S^P(Q*, P), with the non-hydrostatic pressure
//              P = (p0, p1) chosen so that the two incompressibility
//              constraints R0, R1 hold at Q** (central differences, copies of
//              the end cells beyond the channel).  R(Q**(P)) is affine in P, so
//              the corrector is one linear solve:
//   assemble   each cell's two constraint rows as affine forms in the unknowns
//              of its five-cell neighbourhood (pairs of cells form the 4 x 4
//              blocks of a block-tridiagonal system);
//   reduce     parallel cyclic reduction, ceil(log2(blocks)) launches, each
//              block eliminating its neighbours at distance 1, 2, 4, ...;
//   solve      the decoupled 4 x 4 blocks (Gauss-Jordan, partial pivoting);
//   newton     assemble again with the right-hand side -R(Q**(P)) at the
//              pressure found, reduce, solve, and add the increment: one Newton
//              step on the affine constraints (the reduction loses digits on
//              long channels -- a relative residual of 1e-6 at 2^20 cells --
//              and one such step brings it to the rounding level of a direct
//              solve);
//   correct    Q** in place, and the CFL ratio of the new state.
#include <hip/hip_runtime.h>

#include "sme_step_common.h"
#include "sme_vam.h"

namespace sme {

using namespace detail;

namespace {

__device__ __forceinline__ int clampi(int m, int n) { return m < 0 ? 0 : (m > n - 1 ? n - 1 : m); }

__device__ __forceinline__ void quad_node(const Quad &q, int g, double &s, double &w)
{
    if (q.n == 3) {
        s = g == 0 ? q.s0 : (g == 1 ? q.s1 : q.s2);
        w = g == 0 ? q.w0 : (g == 1 ? q.w1 : q.w2);
    } else {
        s = q.s[g];
        w = q.w[g];
    }
}

// state of cell j: (h, h u0, h u1, h w0, h w1)
__device__ __forceinline__ void load_cell(const double *q, int64_t stride, int j, double *v)
{
#pragma unroll
    for (int f = 0; f < 5; ++f) v[f] = q[f * stride + j];
}

__device__ __forceinline__ double bx_at(const VamArgs &a, int j)
{
    return (a.b[clampi(j + 1, a.nx)] - a.b[clampi(j - 1, a.nx)]) * (0.5 / a.dx);
}

// w2 of a cell from its state and bed slope
__device__ __forceinline__ double w2_of(const double *v, double bx)
{
    const double ih = rcp(v[0]);
    return -(v[3] * ih + v[4] * ih) + (v[1] * ih + v[2] * ih) * bx;
}

__device__ __forceinline__ double lam_vam(double g, const double *v)
{
    const double ih = rcp(v[0]);
    const double u1 = v[2] * ih;
    return fabs(v[1] * ih) + sqrt_pos(fma(u1, u1, g * v[0]));
}

__device__ __forceinline__ void flux_vam(const double *v, double w2, double *F)
{
    const double h = v[0], ih = rcp(h);
    const double u0 = v[1] * ih, u1 = v[2] * ih;
    F[0] = v[1];
    F[1] = v[1] * u0 + v[2] * u1 / 3.0;
    F[2] = 2.0 * v[1] * u1;
    F[3] = v[1] * v[3] * ih + v[2] * v[4] * ih / 3.0;
    F[4] = u0 * v[4] + u1 * (v[3] + 0.4 * h * w2);
}

// Rusanov flux Fh and path-integrated NC fluctuation D between L and R
__device__ __forceinline__ void face_vam(const VamArgs &a, const double *L, double bL, double w2L, const double *R,
                                         double bR, double w2R, double *Fh, double *D)
{
    double FL[5], FR[5];
    flux_vam(L, w2L, FL);
    flux_vam(R, w2R, FR);
    const double s = fmax(lam_vam(a.g, L), lam_vam(a.g, R));
    Fh[0] = 0.5 * (FL[0] + FR[0]) - 0.5 * s * ((R[0] + bR) - (L[0] + bL));
#pragma unroll
    for (int f = 1; f < 5; ++f) Fh[f] = 0.5 * (FL[f] + FR[f]) - 0.5 * s * (R[f] - L[f]);
    double dq[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) dq[f] = R[f] - L[f];
    double iu0 = 0.0, iw = 0.0;
    for (int g = 0; g < a.quad.n; ++g) {
        double sg, wg;
        quad_node(a.quad, g, sg, wg);
        const double ih = 1.0 / (L[0] + sg * dq[0]);
        iu0 += wg * ((L[1] + sg * dq[1]) * ih);
        iw += wg * (0.2 * (w2L + sg * (w2R - w2L)) - (L[3] + sg * dq[3]) * ih);
    }
    D[0] = 0.0;
    D[1] = a.g * (0.5 * (L[0] + R[0])) * (dq[0] + (bR - bL));
    D[2] = -iu0 * dq[2];
    D[3] = 0.0;
    D[4] = iw * dq[2];
}

__device__ __forceinline__ double vam_dt(const VamArgs &a)
{
    const Slot &sl = a.slots[a.sa];
    double dt;
    if (a.dt_fixed > 0.0) {
        dt = a.dt_fixed;
    } else {
        const double r = slot_ratio(sl);
        dt = r > 0.0 ? a.cfl / r : 0.0;
    }
    if (a.t_end > 0.0) dt = fmin(dt, fmax(a.t_end - sl.t, 0.0));
    return dt;
}

__device__ __forceinline__ void flag_bad_vam(const VamArgs &a, bool bad, long long step)
{
    if (bad) {
        atomicOr(&a.err->flag, 1u);
        atomicMin(&a.err->first_step, (unsigned long long)step);
    }
}

__global__ __launch_bounds__(kBlock) void k_vam_eig(VamArgs a)
{
    double rm = 0.0;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < a.nx; i += gridDim.x * kBlock) {
        double v[5];
        load_cell(a.q, a.stride, i, v);
        const double r = lam_vam(a.g, v) / a.dx;
        bool bad = !(v[0] > 0.0);
#pragma unroll
        for (int f = 0; f < 5; ++f) bad |= !isfinite(v[f]);
        flag_bad_vam(a, bad, a.slots[a.sa].step);
        if (r >= 0.0) rm = fmax(rm, r);
    }
    publish_ratio(a.slots[a.sa], rm);
}

__global__ __launch_bounds__(kBlock) void k_vam_predict(VamArgs a)
{
    const double dt = vam_dt(a);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const Slot &sl = a.slots[a.sa];
        Slot &nx = a.slots[a.sb];
        nx.t = sl.t + dt;
        nx.dt = dt;
        nx.step = sl.step + (dt > 0.0 ? 1 : 0);
#pragma unroll
        for (int w = 0; w < kRatioWords; ++w) a.slots[a.sc].r[w].bits = 0ull;
        a.slots[a.sc].lbits = 0ull;
    }
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.nx) return;
    double C[5], Lc[5], Rc[5];
    load_cell(a.q, a.stride, i, C);
    if (dt == 0.0) {
#pragma unroll
        for (int f = 0; f < 5; ++f) a.qs[f * a.stride + i] = C[f];
        return;
    }
    const int im = clampi(i - 1, a.nx), ip = clampi(i + 1, a.nx);
    load_cell(a.q, a.stride, im, Lc);
    load_cell(a.q, a.stride, ip, Rc);
    const double bC = a.b[i], bL = a.b[im], bR = a.b[ip];
    const double w2C = w2_of(C, bx_at(a, i)), w2L = w2_of(Lc, bx_at(a, im)), w2R = w2_of(Rc, bx_at(a, ip));
    double FhL[5], DL[5], FhR[5], DR[5];
    face_vam(a, Lc, bL, w2L, C, bC, w2C, FhL, DL);
    face_vam(a, C, bC, w2C, Rc, bR, w2R, FhR, DR);
    const double k = dt / a.dx;
#pragma unroll
    for (int f = 0; f < 5; ++f) a.qs[f * a.stride + i] = C[f] - k * (((FhR[f] - FhL[f]) + 0.5 * DR[f]) + 0.5 * DL[f]);
}

// ---- corrector assembly: affine forms in the unknowns p0, p1 of the cells at
// offsets -2..2 from the row's cell (c[o + 2] for p0, c[7 + o] for p1)
struct Aff {
    double c[10];
    double k;
};

__device__ __forceinline__ void aff_zero(Aff &x)
{
#pragma unroll
    for (int e = 0; e < 10; ++e) x.c[e] = 0.0;
    x.k = 0.0;
}

__device__ __forceinline__ void aff_scale(Aff &x, double s)
{
#pragma unroll
    for (int e = 0; e < 10; ++e) x.c[e] *= s;
    x.k *= s;
}

// coefficient slot for unknown component comp of the cell at offset o
__device__ __forceinline__ void aff_add(Aff &x, int comp, int o, double v)
{
#pragma unroll
    for (int e = 0; e < 5; ++e)
        if (e - 2 == o) x.c[comp * 5 + e] += v;
}

struct Nbhd {
    double h[5], b[5];  // cells i-2..i+2 (clamped)
    int cell[5];        // the clamped cell indices
};

// h u0 at cell j (offset oj from the row's cell i, |oj| <= 1) after the correction
__device__ __forceinline__ void hu0_aff(const VamArgs &a, const Nbhd &n, int i, int oj, double q0, double dt, Aff &x)
{
    const double inv2dx = 0.5 / a.dx;
    const int j = n.cell[oj + 2];
    const int jp = clampi(j + 1, a.nx), jm = clampi(j - 1, a.nx);
    const double hp = a.qs[jp], hm = a.qs[jm];
    const double bx = (a.b[jp] - a.b[jm]) * inv2dx;
    aff_zero(x);
    x.k = q0;
    aff_add(x, 0, jp - i, -dt * hp * inv2dx);
    aff_add(x, 0, jm - i, dt * hm * inv2dx);
    aff_add(x, 1, j - i, -2.0 * dt * bx);
}

__device__ __forceinline__ void hu1_aff(const VamArgs &a, const Nbhd &n, int i, int oj, double q1, double dt, Aff &x)
{
    const double inv2dx = 0.5 / a.dx;
    const int j = n.cell[oj + 2];
    const int jp = clampi(j + 1, a.nx), jm = clampi(j - 1, a.nx);
    const double hp = a.qs[jp], hm = a.qs[jm];
    const double hx = (hp - hm) * inv2dx;
    const double bx = (a.b[jp] - a.b[jm]) * inv2dx;
    aff_zero(x);
    x.k = q1;
    aff_add(x, 1, jp - i, -dt * hp * inv2dx);
    aff_add(x, 1, jm - i, dt * hm * inv2dx);
    aff_add(x, 0, j - i, dt * (3.0 * hx + 6.0 * bx));
    aff_add(x, 1, j - i, -dt * (hx + 6.0 * bx));
}

// rows of the constraints at cell i; right-hand side -R(Q**(P)) at the
// pressure pcur (null: P = 0)
__global__ __launch_bounds__(kBlock) void k_vam_assemble(VamArgs a, VamSystem m, const double *pcur)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int ncell = 2 * a.nb;  // nx, or nx + 1 with one padding cell
    if (i >= ncell) return;
    const double dt = a.slots[a.sb].dt;
    const int k = i >> 1, r0 = 2 * (i & 1);
    double rowA[2][4], rowB[2][4], rowC[2][4], dd[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
#pragma unroll
        for (int c = 0; c < 4; ++c) rowA[e][c] = rowB[e][c] = rowC[e][c] = 0.0;
        dd[e] = 0.0;
    }
    if (i >= a.nx || dt == 0.0) {
        // padding cell, or a step of length zero: p = 0
        rowB[0][r0] = 1.0;
        rowB[1][r0 + 1] = 1.0;
    } else {
        const double inv2dx = 0.5 / a.dx;
        Nbhd n;
#pragma unroll
        for (int o = -2; o <= 2; ++o) {
            n.cell[o + 2] = clampi(i + o, a.nx);
            n.h[o + 2] = a.qs[n.cell[o + 2]];
            n.b[o + 2] = a.b[n.cell[o + 2]];
        }
        const double h = n.h[2], ih = 1.0 / h;
        const double hx = (n.h[3] - n.h[1]) * inv2dx, bx = (n.b[3] - n.b[1]) * inv2dx;
        const int jm = n.cell[1], jp = n.cell[3];
        Aff u0p, u0m, a1p, a1m, a1, a0;
        hu0_aff(a, n, i, 1, a.qs[a.stride + jp], dt, u0p);
        aff_scale(u0p, 1.0 / n.h[3]);
        hu0_aff(a, n, i, -1, a.qs[a.stride + jm], dt, u0m);
        aff_scale(u0m, 1.0 / n.h[1]);
        hu1_aff(a, n, i, 1, a.qs[2 * a.stride + jp], dt, a1p);
        hu1_aff(a, n, i, -1, a.qs[2 * a.stride + jm], dt, a1m);
        hu1_aff(a, n, i, 0, a.qs[2 * a.stride + i], dt, a1);
        hu0_aff(a, n, i, 0, a.qs[a.stride + i], dt, a0);
        const double r0v = a.qs[3 * a.stride + i], r1v = a.qs[4 * a.stride + i];
        // R0 = h (u0)_x + (h u1)_x / 3 + u1 h_x / 3 + 2 (w0 - u0 b_x)
        // R1 = h (u0)_x + u1 h_x + 2 (u1 b_x - w1)
        Aff R0, R1;
#pragma unroll
        for (int e = 0; e < 10; ++e) {
            const double du0 = h * ((u0p.c[e] - u0m.c[e]) * inv2dx);
            const double u1 = a1.c[e] * ih, u0 = a0.c[e] * ih;
            R0.c[e] = du0 + (a1p.c[e] - a1m.c[e]) * inv2dx / 3.0 + u1 * hx / 3.0 + 2.0 * (-(u0 * bx));
            R1.c[e] = du0 + u1 * hx + 2.0 * (u1 * bx);
        }
        {
            const double du0 = h * ((u0p.k - u0m.k) * inv2dx);
            const double u1 = a1.k * ih, u0 = a0.k * ih;
            R0.k = du0 + (a1p.k - a1m.k) * inv2dx / 3.0 + u1 * hx / 3.0 + 2.0 * (r0v * ih - u0 * bx);
            R1.k = du0 + u1 * hx + 2.0 * (u1 * bx - r1v * ih);
        }
        // the pressure terms of w0 = (h w0 + 2 dt p1) / h and w1 = (h w1 - 6 dt (p0 - p1)) / h
        R0.c[7] += 2.0 * (2.0 * dt * ih);
        R1.c[2] += -2.0 * (-6.0 * dt * ih);
        R1.c[7] += -2.0 * (6.0 * dt * ih);
        // scatter into the rows of block k
#pragma unroll
        for (int comp = 0; comp < 2; ++comp) {
#pragma unroll
            for (int o = -2; o <= 2; ++o) {
                const int mc = i + o;
                if (mc < 0 || mc >= a.nx) continue;
                const int which = (mc >> 1) - k;  // -1, 0, 1
                const int pos = 2 * (mc & 1) + comp;
                const double v0 = R0.c[comp * 5 + o + 2], v1 = R1.c[comp * 5 + o + 2];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (c != pos) continue;
                    if (which < 0) {
                        rowA[0][c] += v0;
                        rowA[1][c] += v1;
                    } else if (which == 0) {
                        rowB[0][c] += v0;
                        rowB[1][c] += v1;
                    } else {
                        rowC[0][c] += v0;
                        rowC[1][c] += v1;
                    }
                }
            }
        }
        double v0 = R0.k, v1 = R1.k;
        if (pcur) {
#pragma unroll
            for (int comp = 0; comp < 2; ++comp)
#pragma unroll
                for (int o = -2; o <= 2; ++o) {
                    const int mc = i + o;
                    if (mc < 0 || mc >= a.nx) continue;
                    const double pv = pcur[comp * a.stride + mc];
                    v0 = fma(R0.c[comp * 5 + o + 2], pv, v0);
                    v1 = fma(R1.c[comp * 5 + o + 2], pv, v1);
                }
        }
        dd[0] = -v0;
        dd[1] = -v1;
    }
    const int nb = a.nb;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int r = r0 + e;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            m.A[(r * 4 + c) * nb + k] = rowA[e][c];
            m.B[(r * 4 + c) * nb + k] = rowB[e][c];
            m.C[(r * 4 + c) * nb + k] = rowC[e][c];
        }
        m.d[r * nb + k] = dd[e];
    }
}

// ---- 4 x 4 block algebra (row-major, registers only: every index is static)
__device__ __forceinline__ void load4(const double *M, int nb, int k, double *X)
{
#pragma unroll
    for (int e = 0; e < 16; ++e) X[e] = M[e * nb + k];
}

__device__ __forceinline__ void store4(double *M, int nb, int k, const double *X)
{
#pragma unroll
    for (int e = 0; e < 16; ++e) M[e * nb + k] = X[e];
}

// X = inverse of M by Gauss-Jordan elimination with partial pivoting
__device__ __forceinline__ void inv4(const double *M, double *X)
{
    double a[4][8];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 8; ++c) a[r][c] = c < 4 ? M[r * 4 + c] : (c - 4 == r ? 1.0 : 0.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        // bring the largest |a[r][c]|, r >= c, to row c by compare-and-swap
#pragma unroll
        for (int r = c + 1; r < 4; ++r) {
            const bool sw = fabs(a[r][c]) > fabs(a[c][c]);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const double t = a[c][e];
                a[c][e] = sw ? a[r][e] : t;
                a[r][e] = sw ? t : a[r][e];
            }
        }
        const double ip = 1.0 / a[c][c];
#pragma unroll
        for (int e = 0; e < 8; ++e) a[c][e] *= ip;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r == c) continue;
            const double f = a[r][c];
#pragma unroll
            for (int e = 0; e < 8; ++e) a[r][e] = fma(-f, a[c][e], a[r][e]);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) X[r * 4 + c] = a[r][c + 4];
}

// Z = X Y
__device__ __forceinline__ void mul4(const double *X, const double *Y, double *Z)
{
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double s = X[r * 4] * Y[c];
#pragma unroll
            for (int e = 1; e < 4; ++e) s = fma(X[r * 4 + e], Y[e * 4 + c], s);
            Z[r * 4 + c] = s;
        }
}

// Z += X Y
__device__ __forceinline__ void muladd4(const double *X, const double *Y, double *Z)
{
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double s = Z[r * 4 + c];
#pragma unroll
            for (int e = 0; e < 4; ++e) s = fma(X[r * 4 + e], Y[e * 4 + c], s);
            Z[r * 4 + c] = s;
        }
}

// Block cyclic reduction with the equations of every level stored apart and
// contiguously.  Level l holds n_l equations, equation j coupled to j - 1 and
// j + 1 of the same level.  Level l + 1 holds the odd equations of level l,
// j = 2t + 1, each updated by eliminating its couplings with the equations
// j - 1 and j + 1 (which then couple it to j -/+ 2, the equations t -/+ 1 of
// level l + 1):
//   a = -A_j B_{j-1}^-1,  g = -C_j B_{j+1}^-1,
//   A' = a A_{j-1},  C' = g C_{j+1},  B' = B_j + a C_{j-1} + g A_{j+1},
//   d' = d_j + a d_{j-1} + g d_{j+1};
// an equation without a right neighbour has no coupling to it.  The one
// equation of the top level is decoupled; back substitution then visits the
// levels downwards: the odd unknowns of level l are those of level l + 1, the
// even ones follow from x_j = B_j^-1 (d_j - A_j x_{j-1} - C_j x_{j+1}).
// Every access is to consecutive equations (the compaction keeps the loads
// coalesced at every level), and work and traffic halve from level to level.
__global__ __launch_bounds__(kBlock) void k_vam_cr_reduce(int n, VamSystem src, VamSystem dst)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int nd = n / 2;
    if (t >= nd) return;
    const int j = 2 * t + 1;
    double Bj[16], dj[4], T[16], G[16], Z[16];
    load4(src.B, n, j, Bj);
#pragma unroll
    for (int r = 0; r < 4; ++r) dj[r] = src.d[r * n + j];
    {
        load4(src.B, n, j - 1, T);
        inv4(T, Z);                    // B_{j-1}^-1
        load4(src.A, n, j, T);
        mul4(T, Z, G);                 // A_j B_{j-1}^-1
#pragma unroll
        for (int e = 0; e < 16; ++e) G[e] = -G[e];
        load4(src.A, n, j - 1, T);
        mul4(G, T, Z);
        store4(dst.A, nd, t, Z);
        load4(src.C, n, j - 1, T);
        muladd4(G, T, Bj);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double acc = dj[r];
#pragma unroll
            for (int e = 0; e < 4; ++e) acc = fma(G[r * 4 + e], src.d[e * n + j - 1], acc);
            dj[r] = acc;
        }
    }
    if (j + 1 < n) {
        load4(src.B, n, j + 1, T);
        inv4(T, Z);                    // B_{j+1}^-1
        load4(src.C, n, j, T);
        mul4(T, Z, G);                 // C_j B_{j+1}^-1
#pragma unroll
        for (int e = 0; e < 16; ++e) G[e] = -G[e];
        load4(src.C, n, j + 1, T);
        mul4(G, T, Z);
        store4(dst.C, nd, t, Z);
        load4(src.A, n, j + 1, T);
        muladd4(G, T, Bj);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double acc = dj[r];
#pragma unroll
            for (int e = 0; e < 4; ++e) acc = fma(G[r * 4 + e], src.d[e * n + j + 1], acc);
            dj[r] = acc;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) Z[e] = 0.0;
        store4(dst.C, nd, t, Z);
    }
    store4(dst.B, nd, t, Bj);
#pragma unroll
    for (int r = 0; r < 4; ++r) dst.d[r * nd + t] = dj[r];
}

// back substitution of level l (n equations) into x ([4][n]); xup holds the
// unknowns of level l + 1 (null at the top level, which has one equation)
__global__ __launch_bounds__(kBlock) void k_vam_cr_back(int n, VamSystem m, const double *xup, double *x)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int nu = n / 2;
    if (j & 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r * n + j] = xup[r * nu + (j >> 1)];
        return;
    }
    double rhs[4], T[16], Z[16];
#pragma unroll
    for (int r = 0; r < 4; ++r) rhs[r] = m.d[r * n + j];
    if (j >= 1) {
        load4(m.A, n, j, T);
        const int u = (j - 1) >> 1;  // x_{j-1} is unknown u of level l + 1
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) rhs[r] = fma(-T[r * 4 + e], xup[e * nu + u], rhs[r]);
    }
    if (j + 1 < n) {
        load4(m.C, n, j, T);
        const int u = j >> 1;        // x_{j+1}
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) rhs[r] = fma(-T[r * 4 + e], xup[e * nu + u], rhs[r]);
    }
    load4(m.B, n, j, T);
    inv4(T, Z);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double v = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) v = fma(Z[r * 4 + e], rhs[e], v);
        x[r * n + j] = v;
    }
}

// the solved blocks -> (p0, p1) of cells 2k, 2k + 1 (added to the pressure if
// accumulate)
__global__ __launch_bounds__(kBlock) void k_vam_scatter(VamArgs a, const double *x, int accumulate)
{
    const int cell = blockIdx.x * kBlock + threadIdx.x;
    if (cell >= a.nx) return;
    const int k = cell >> 1, c = cell & 1;
    const double x0 = x[(2 * c) * a.nb + k], x1 = x[(2 * c + 1) * a.nb + k];
    a.p[cell] = accumulate ? a.p[cell] + x0 : x0;
    a.p[a.stride + cell] = accumulate ? a.p[a.stride + cell] + x1 : x1;
}

__global__ __launch_bounds__(kBlock) void k_vam_correct(VamArgs a)
{
    const double dt = a.slots[a.sb].dt;
    const long long step = a.slots[a.sb].step;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double r = 0.0;
    if (i < a.nx) {
        const int im = clampi(i - 1, a.nx), ip = clampi(i + 1, a.nx);
        double v[5];
        load_cell(a.qs, a.stride, i, v);
        if (dt != 0.0) {
            const double inv2dx = 0.5 / a.dx;
            const double hm = a.qs[im], hp = a.qs[ip];
            const double hx = (hp - hm) * inv2dx, bx = (a.b[ip] - a.b[im]) * inv2dx;
            const double p0 = a.p[i], p1 = a.p[a.stride + i];
            const double dhp0 = (hp * a.p[ip] - hm * a.p[im]) * inv2dx;
            const double dhp1 = (hp * a.p[a.stride + ip] - hm * a.p[a.stride + im]) * inv2dx;
            v[1] = v[1] - dt * (dhp0 + 2.0 * p1 * bx);
            v[2] = v[2] - dt * (dhp1 - (3.0 * p0 - p1) * hx - 6.0 * (p0 - p1) * bx);
            v[3] = v[3] + dt * (2.0 * p1);
            v[4] = v[4] - dt * (6.0 * (p0 - p1));
#pragma unroll
            for (int f = 1; f < 5; ++f) a.qs[f * a.stride + i] = v[f];
        }
        bool bad = !(v[0] > 0.0);
#pragma unroll
        for (int f = 0; f < 5; ++f) bad |= !isfinite(v[f]);
        flag_bad_vam(a, bad, step);
        r = lam_vam(a.g, v) / a.dx;
        if (!(r >= 0.0)) r = 0.0;
    }
    publish_ratio(a.slots[a.sb], r);
}

}  // namespace

hipError_t launch_vam_eig(const VamArgs &a, hipStream_t s)
{
    const unsigned grid = blocks_for(a.nx) < 1024u ? blocks_for(a.nx) : 1024u;
    hipLaunchKernelGGL(k_vam_eig, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vam_predict(const VamArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_vam_predict, dim3(blocks_for(a.nx)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vam_assemble(const VamArgs &a, const VamSystem &m, const double *pcur, hipStream_t s)
{
    hipLaunchKernelGGL(k_vam_assemble, dim3(blocks_for(2 * (int64_t)a.nb)), dim3(kBlock), 0, s, a, m, pcur);
    return hipGetLastError();
}

hipError_t launch_vam_reduce(int n, const VamSystem &src, const VamSystem &dst, hipStream_t s)
{
    if (n / 2 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_vam_cr_reduce, dim3(blocks_for(n / 2)), dim3(kBlock), 0, s, n, src, dst);
    return hipGetLastError();
}

hipError_t launch_vam_back(int n, const VamSystem &m, const double *xup, double *x, hipStream_t s)
{
    hipLaunchKernelGGL(k_vam_cr_back, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, m, xup, x);
    return hipGetLastError();
}

hipError_t launch_vam_scatter(const VamArgs &a, const double *x, int accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(k_vam_scatter, dim3(blocks_for(a.nx)), dim3(kBlock), 0, s, a, x, accumulate);
    return hipGetLastError();
}

hipError_t launch_vam_correct(const VamArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_vam_correct, dim3(blocks_for(a.nx)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace sme
