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
//   reduce     block cyclic reduction: each level factors its even
//              equations once and folds them into its odd ones, which form
//              the next level (one launch per level down to a few thousand
//              equations, the rest and their back substitution in one
//              workgroup);
//   back       back substitution from the one-equation top level down;
//   newton     the right-hand side -R(Q**(P)) at the pressure found,
//              evaluated on the corrected state itself, carried through the
//              stored factors (the matrix does not depend on P), back
//              substitution, and the increment added: one step of iterative
//              refinement, which takes the constraint residual from the
//              reduction's rounding to that of the residual evaluation;
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

// rows of the constraints at cell i, right-hand side -R(Q**(0))
__global__ __launch_bounds__(kBlock) void k_vam_assemble(VamArgs a, VamSystem m)
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
        dd[0] = -R0.k;
        dd[1] = -R1.k;
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
// X = M^-1 by the adjugate: the 2 x 2 minors of the top two rows (s) and of
// the bottom two rows (c) give the determinant (Laplace expansion along the
// top two rows) and every cofactor as a three-term sum.  About 100 FP64
// operations with a dependency depth of about 17, against about 370 and 75
// for Gauss-Jordan elimination with pivoting; the blocks of the corrector's
// system are well conditioned (diagonal blocks of a discrete second-order
// operator and their Schur complements), and the second Newton solve on the
// residual corrects what the inverse's rounding leaves.
__device__ __forceinline__ void inv4(const double *a, double *X)
{
    auto m2 = [](double p, double q, double r, double t) { return fma(p, q, -(r * t)); };  // p q - r t
    const double s0 = m2(a[0], a[5], a[4], a[1]);
    const double s1 = m2(a[0], a[6], a[4], a[2]);
    const double s2 = m2(a[0], a[7], a[4], a[3]);
    const double s3 = m2(a[1], a[6], a[5], a[2]);
    const double s4 = m2(a[1], a[7], a[5], a[3]);
    const double s5 = m2(a[2], a[7], a[6], a[3]);
    const double c5 = m2(a[10], a[15], a[14], a[11]);
    const double c4 = m2(a[9], a[15], a[13], a[11]);
    const double c3 = m2(a[9], a[14], a[13], a[10]);
    const double c2 = m2(a[8], a[15], a[12], a[11]);
    const double c1 = m2(a[8], a[14], a[12], a[10]);
    const double c0 = m2(a[8], a[13], a[12], a[9]);
    const double det = fma(s0, c5, fma(-s1, c4, s2 * c3)) + fma(s3, c2, fma(-s4, c1, s5 * c0));
    const double r = rcp(det);
    auto e3 = [r](double x0, double y0, double x1, double y1, double x2, double y2) {
        return r * fma(x0, y0, fma(x1, y1, x2 * y2));
    };
    X[0] = e3(a[5], c5, -a[6], c4, a[7], c3);
    X[1] = e3(-a[1], c5, a[2], c4, -a[3], c3);
    X[2] = e3(a[13], s5, -a[14], s4, a[15], s3);
    X[3] = e3(-a[9], s5, a[10], s4, -a[11], s3);
    X[4] = e3(-a[4], c5, a[6], c2, -a[7], c1);
    X[5] = e3(a[0], c5, -a[2], c2, a[3], c1);
    X[6] = e3(-a[12], s5, a[14], s2, -a[15], s1);
    X[7] = e3(a[8], s5, -a[10], s2, a[11], s1);
    X[8] = e3(a[4], c4, -a[5], c2, a[7], c0);
    X[9] = e3(-a[0], c4, a[1], c2, -a[3], c0);
    X[10] = e3(a[12], s4, -a[13], s2, a[15], s0);
    X[11] = e3(-a[8], s4, a[9], s2, -a[11], s0);
    X[12] = e3(-a[4], c3, a[5], c1, -a[6], c0);
    X[13] = e3(a[0], c3, -a[1], c1, a[2], c0);
    X[14] = e3(-a[12], s3, a[13], s1, -a[14], s0);
    X[15] = e3(a[8], s3, -a[9], s1, a[10], s0);
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

// Block cyclic reduction with the equations of every level stored apart and
// contiguously.  Level l holds n_l equations A_j x_{j-1} + B_j x_j + C_j x_{j+1}
// = d_j (no A for the first, no C for the last).  Every even equation i = 2u
// is factored once:
//   E_i = B_i^-1 A_i,  F_i = B_i^-1 C_i,  g_i = B_i^-1 d_i,
// so that x_i = g_i - E_i x_{i-1} - F_i x_{i+1}.  Level l + 1 holds the odd
// equations j = 2t + 1 with both even neighbours substituted, which couples
// them to j -/+ 2 (equations t -/+ 1 of level l + 1):
//   A' = -A_j E_{j-1},  C' = -C_j F_{j+1},  B' = B_j - A_j F_{j-1} - C_j E_{j+1},
//   d' = d_j - A_j g_{j-1} - C_j g_{j+1}.
// The top level's one equation is decoupled (x = g); back substitution then
// visits the levels downwards: the odd unknowns of level l are those of level
// l + 1, the even ones follow from their factors.  The factors, with B_i^-1,
// are kept per level: a second solve with the same matrix and a new
// right-hand side (the Newton step on the residual) only carries the
// right-hand side down, g_i = B_i^-1 d_i and d' as above.
// Every access is to consecutive equations (the compaction keeps the loads
// coalesced at every level), and work and traffic halve from level to level.

// a level's equations: entry e of equation j at A[e * s + j] (B, C: 16
// entries, d: 4), in device memory or in LDS
struct Eqs {
    double *A, *B, *C, *d;
    int s;
};
// factors of a level's even equations: entry e of even equation u at
// f[e * s + u]; entries 0..15 E, 16..31 F, 32..35 g, 36..51 B^-1
struct Facs {
    double *f;
    int s;
};
constexpr int kFacE = 0, kFacF = 16, kFacG = 32, kFacBi = 36, kFac = 52;

__device__ __forceinline__ int evens(int n) { return (n + 1) / 2; }
__device__ __forceinline__ Eqs eqs_of(const VamSystem &m, int n) { return Eqs{m.A, m.B, m.C, m.d, n}; }
__device__ __forceinline__ Facs facs_of(const VamSystem &m, int n) { return Facs{m.fac, evens(n)}; }

__device__ __forceinline__ void ld4(const Eqs &m, const double *M, int j, double *X)
{
#pragma unroll
    for (int e = 0; e < 16; ++e) X[e] = M[e * m.s + j];
}

// Z -= X Y
__device__ __forceinline__ void mulsub4(const double *X, const double *Y, double *Z)
{
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double s = Z[r * 4 + c];
#pragma unroll
            for (int e = 0; e < 4; ++e) s = fma(-X[r * 4 + e], Y[e * 4 + c], s);
            Z[r * 4 + c] = s;
        }
}

// factors of the even equation 2u of a level of n; the first equation has no
// A (E = 0) and, for odd n, the last no C (F = 0)
__device__ __forceinline__ void factor_even(int n, const Eqs &m, int u, double *E, double *F, double *g, double *Bi)
{
    const int i = 2 * u;
    double T[16];
    ld4(m, m.B, i, T);
    inv4(T, Bi);
    if (i >= 1) {
        ld4(m, m.A, i, T);
        mul4(Bi, T, E);
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) E[e] = 0.0;
    }
    if (i + 1 < n) {
        ld4(m, m.C, i, T);
        mul4(Bi, T, F);
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) F[e] = 0.0;
    }
    double d[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) d[r] = m.d[r * m.s + i];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double v = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) v = fma(Bi[r * 4 + e], d[e], v);
        g[r] = v;
    }
}

__device__ __forceinline__ void store_factors(const Facs &f, int u, const double *E, const double *F, const double *g,
                                              const double *Bi)
{
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        f.f[(kFacE + e) * f.s + u] = E[e];
        f.f[(kFacF + e) * f.s + u] = F[e];
        f.f[(kFacBi + e) * f.s + u] = Bi[e];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) f.f[(kFacG + r) * f.s + u] = g[r];
}

// The odd equation j = 2t + 1 of a level of n (src; its A_j, B_j, d_j
// already loaded) into equation t of the next level (dst); the factors of
// j - 1 at fm[e * sm] and of j + 1 at fp[e * sp] (read only if j + 1 < n).
__device__ __forceinline__ void reduce_odd(int n, const Eqs &src, const Eqs &dst, int t, const double *Aj,
                                           double *Bj, double *dj, const double *fm, int sm, const double *fp, int sp)
{
    const int j = 2 * t + 1;
    double M[16], X[16], Y[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) X[e] = fm[(kFacE + e) * sm];
    mul4(Aj, X, Y);
#pragma unroll
    for (int e = 0; e < 16; ++e) dst.A[e * dst.s + t] = -Y[e];
#pragma unroll
    for (int e = 0; e < 16; ++e) X[e] = fm[(kFacF + e) * sm];
    mulsub4(Aj, X, Bj);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) dj[r] = fma(-Aj[r * 4 + e], fm[(kFacG + e) * sm], dj[r]);
    if (j + 1 < n) {
        ld4(src, src.C, j, M);
#pragma unroll
        for (int e = 0; e < 16; ++e) X[e] = fp[(kFacE + e) * sp];
        mulsub4(M, X, Bj);
#pragma unroll
        for (int e = 0; e < 16; ++e) X[e] = fp[(kFacF + e) * sp];
        mul4(M, X, Y);
#pragma unroll
        for (int e = 0; e < 16; ++e) Y[e] = -Y[e];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) dj[r] = fma(-M[r * 4 + e], fp[(kFacG + e) * sp], dj[r]);
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) Y[e] = 0.0;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        dst.C[e * dst.s + t] = Y[e];
        dst.B[e * dst.s + t] = Bj[e];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) dst.d[r * dst.s + t] = dj[r];
}

__device__ __forceinline__ void load_odd(const Eqs &m, int j, double *Aj, double *Bj, double *dj)
{
    ld4(m, m.A, j, Aj);
    ld4(m, m.B, j, Bj);
#pragma unroll
    for (int r = 0; r < 4; ++r) dj[r] = m.d[r * m.s + j];
}

// g of the even equation 2u from its stored B^-1 and the level's new d
__device__ __forceinline__ void g_even(const Eqs &m, const Facs &f, int u, double *g)
{
    double d[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) d[r] = m.d[r * m.s + 2 * u];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double v = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) v = fma(f.f[(kFacBi + r * 4 + e) * f.s + u], d[e], v);
        g[r] = v;
    }
}

// d of equation t of the next level for a new right-hand side; gm, gp the g
// of the even neighbours 2t and 2t + 2, entry e at gm[e * sg] (gp read only
// if 2t + 2 < n)
__device__ __forceinline__ void rhs_odd(int n, const Eqs &src, const Eqs &dst, int t, const double *gm, int sg,
                                        const double *gp)
{
    const int j = 2 * t + 1;
    double dj[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) dj[r] = src.d[r * src.s + j];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) dj[r] = fma(-src.A[(r * 4 + e) * src.s + j], gm[e * sg], dj[r]);
    if (j + 1 < n) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) dj[r] = fma(-src.C[(r * 4 + e) * src.s + j], gp[e * sg], dj[r]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) dst.d[r * dst.s + t] = dj[r];
}

// unknowns x_j of a level of n (entry r at x[r * sx + j]) from its factors
// and the unknowns of the level above (xup[r * su + (j >> 1)])
__device__ __forceinline__ void back_one(int n, const Facs &f, const double *xup, int su, double *x, int sx, int j)
{
    if (j & 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r * sx + j] = xup[r * su + (j >> 1)];
        return;
    }
    const int u = j >> 1;
    double v[4], xs[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = f.f[(kFacG + r) * f.s + u];
    if (j >= 1) {
#pragma unroll
        for (int e = 0; e < 4; ++e) xs[e] = xup[e * su + ((j - 1) >> 1)];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) v[r] = fma(-f.f[(kFacE + r * 4 + e) * f.s + u], xs[e], v[r]);
    }
    if (j + 1 < n) {
#pragma unroll
        for (int e = 0; e < 4; ++e) xs[e] = xup[e * su + (j >> 1)];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) v[r] = fma(-f.f[(kFacF + r * 4 + e) * f.s + u], xs[e], v[r]);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) x[r * sx + j] = v[r];
}

// A workgroup barrier that orders LDS only: the device-memory stores issued
// before it are not waited for (a plain barrier would wait for all of them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One level of the reduction.  A workgroup factors kRedThreads consecutive
// even equations (into LDS, and into the level's factors) and then reduces
// the kRedThreads - 1 odd equations between them; the last even equation of
// a workgroup is the first of the next one, which alone stores it (if there
// is a next one).  The odd equation's loads are issued before the even one's
// arithmetic, so a level costs one round trip to memory.
constexpr int kRedThreads = 256;

__global__ __launch_bounds__(kRedThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_vam_cr_reduce(int n, VamSystem src, VamSystem dst)
{
    __shared__ double f[(kFacG + 4) * kRedThreads];  // E, F, g of the workgroup's even equations
    const Eqs se = eqs_of(src, n), de = eqs_of(dst, n / 2);
    const int ne = evens(n), nd = n / 2;
    const int k = threadIdx.x;
    const int u = blockIdx.x * (kRedThreads - 1) + k;
    const bool odd = k < kRedThreads - 1 && u < nd;
    double Aj[16], Bj[16], dj[4];
    if (odd) load_odd(se, 2 * u + 1, Aj, Bj, dj);
    if (u < ne) {
        double E[16], F[16], g[4], Bi[16];
        factor_even(n, se, u, E, F, g, Bi);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            f[(kFacE + e) * kRedThreads + k] = E[e];
            f[(kFacF + e) * kRedThreads + k] = F[e];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) f[(kFacG + r) * kRedThreads + k] = g[r];
        // the last one is stored by the next workgroup, if there is one
        if (k < kRedThreads - 1 || (int)(blockIdx.x + 1) * (kRedThreads - 1) >= nd)
            store_factors(facs_of(src, n), u, E, F, g, Bi);
    }
    lds_barrier();
    if (odd) reduce_odd(n, se, de, u, Aj, Bj, dj, f + k, kRedThreads, f + k + 1, kRedThreads);
}

// The same level for a new right-hand side of the factored matrix.  Thread
// t: g of the even equations 2t (stored) and 2t + 2 (stored only if it is
// the last), then d of the next level's equation t.
__global__ __launch_bounds__(kBlock) void k_vam_cr_rhs(int n, VamSystem src, VamSystem dst)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= n / 2) return;
    const Eqs se = eqs_of(src, n), de = eqs_of(dst, n / 2);
    const Facs fs = facs_of(src, n);
    double gm[4], gp[4];
    g_even(se, fs, t, gm);
#pragma unroll
    for (int r = 0; r < 4; ++r) fs.f[(kFacG + r) * fs.s + t] = gm[r];
    if (2 * t + 2 < n) {
        g_even(se, fs, t + 1, gp);
        if (t + 2 == fs.s) {
#pragma unroll
            for (int r = 0; r < 4; ++r) fs.f[(kFacG + r) * fs.s + t + 1] = gp[r];
        }
    }
    rhs_odd(n, se, de, t, gm, 1, gp);
}

// back substitution of level l (n > 1 equations) into x ([4][n]) from the
// unknowns xup of level l + 1
__global__ __launch_bounds__(kBlock) void k_vam_cr_back(int n, VamSystem m, const double *xup, double *x)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j < n) back_one(n, facs_of(m, n), xup, n / 2, x, n, j);
}

// The last levels of the reduction (at most kTailMax equations), the top
// equation and the back substitution of those levels in one wave, with every
// level in LDS: below a few hundred equations a level is too small to fill
// the chip, and its cost is a launch and the latency of memory round trips
// (about 2 us each); here the tail's first level is read once, everything
// after it stays in LDS, and the unknowns of the first level are written
// once.  The full solve also writes what a right-hand-side solve needs (the
// tail levels' A and C and the factors) to device memory; the
// right-hand-side solve (RHS) reads them back in one round trip.
// Device memory as such: a pointer read from memory (here from the tail's
// description) is generic to the compiler, and a generic access may alias
// LDS, so it would be kept in order with every LDS access and never batched.
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ const gdouble *gptr(const double *p) { return (const gdouble *)p; }
__device__ __forceinline__ gdouble *gptr(double *p) { return (gdouble *)p; }

constexpr int kTailEq = 2 * kTailMax;   // equations of all tail levels, padded
constexpr int kTailEv = kTailMax;       // even equations of all tail levels
static_assert(kTailThreads == kWave, "the tail runs in one wave");

template <bool RHS>
__global__ __launch_bounds__(kTailThreads) void k_vam_cr_tail(const VamTail *tail)
{
    __shared__ double sA[16 * kTailEq], sB[16 * kTailEq], sC[16 * kTailEq], sd[4 * kTailEq], sx[4 * kTailEq];
    __shared__ double sf[kFac * kTailEv];
    __shared__ int eq[kTailLevels], ev[kTailLevels];  // level i's first equation and first even equation
    const VamTail &lv = *tail;
    const int top = lv.count - 1, tid = threadIdx.x;
    if (tid == 0) {
        eq[0] = ev[0] = 0;
        for (int i = 1; i <= top; ++i) {
            eq[i] = eq[i - 1] + lv.n[i - 1];
            ev[i] = ev[i - 1] + evens(lv.n[i - 1]);
        }
    }
    lds_barrier();
    auto leqs = [&](int i) { return Eqs{sA + eq[i], sB + eq[i], sC + eq[i], sd + eq[i], kTailEq}; };
    auto lfacs = [&](int i) { return Facs{sf + ev[i], kTailEv}; };
    const int n0 = lv.n[0];
    if constexpr (!RHS) {
        const Eqs g0 = eqs_of(lv.m[0], n0);
        for (int j = tid; j < n0; j += kTailThreads) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                sA[e * kTailEq + j] = gptr(g0.A)[e * n0 + j];
                sB[e * kTailEq + j] = gptr(g0.B)[e * n0 + j];
                sC[e * kTailEq + j] = gptr(g0.C)[e * n0 + j];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) sd[r * kTailEq + j] = gptr(g0.d)[r * n0 + j];
        }
    } else {
        for (int i = 0; i <= top; ++i) {
            const int n = lv.n[i];
            const Eqs g = eqs_of(lv.m[i], n);
            const Facs gf = facs_of(lv.m[i], n);
            for (int j = tid; j < n; j += kTailThreads) {
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    sA[e * kTailEq + eq[i] + j] = gptr(g.A)[e * n + j];
                    sC[e * kTailEq + eq[i] + j] = gptr(g.C)[e * n + j];
                }
                if (i == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) sd[r * kTailEq + j] = gptr(g.d)[r * n + j];
                }
            }
            for (int u = tid; u < gf.s; u += kTailThreads) {
#pragma unroll
                for (int e = 0; e < kFac; ++e) sf[e * kTailEv + ev[i] + u] = gptr(gf.f)[e * gf.s + u];
            }
        }
    }
    lds_barrier();
    for (int i = 0; i < top; ++i) {
        const int n = lv.n[i], ne = evens(n), nd = n / 2;
        const Eqs se = leqs(i), de = leqs(i + 1);
        const Facs sfi = lfacs(i);
        if constexpr (RHS) {
            for (int u = tid; u < ne; u += kTailThreads) {
                double g[4];
                g_even(se, sfi, u, g);
#pragma unroll
                for (int r = 0; r < 4; ++r) sfi.f[(kFacG + r) * sfi.s + u] = g[r];
            }
            lds_barrier();
            for (int t = tid; t < nd; t += kTailThreads)
                rhs_odd(n, se, de, t, sfi.f + kFacG * sfi.s + t, sfi.s, sfi.f + kFacG * sfi.s + t + 1);
        } else {
            for (int u = tid; u < ne; u += kTailThreads) {
                double E[16], F[16], g[4], Bi[16];
                factor_even(n, se, u, E, F, g, Bi);
                store_factors(sfi, u, E, F, g, Bi);
            }
            lds_barrier();
            for (int t = tid; t < nd; t += kTailThreads) {
                double Aj[16], Bj[16], dj[4];
                load_odd(se, 2 * t + 1, Aj, Bj, dj);
                reduce_odd(n, se, de, t, Aj, Bj, dj, sfi.f + t, sfi.s, sfi.f + t + 1, sfi.s);
            }
        }
        lds_barrier();
    }
    if (tid == 0) {
        const Eqs se = leqs(top);
        const Facs sft = lfacs(top);
        double g[4];
        if constexpr (RHS) {
            g_even(se, sft, 0, g);
        } else {
            double E[16], F[16], Bi[16];
            factor_even(1, se, 0, E, F, g, Bi);
            store_factors(sft, 0, E, F, g, Bi);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            sft.f[(kFacG + r) * sft.s] = g[r];
            sx[r * kTailEq + eq[top]] = g[r];
        }
    }
    lds_barrier();
    for (int i = top - 1; i >= 0; --i) {
        const int n = lv.n[i];
        for (int j = tid; j < n; j += kTailThreads)
            back_one(n, lfacs(i), sx + eq[i + 1], kTailEq, sx + eq[i], kTailEq, j);
        lds_barrier();
    }
    for (int j = tid; j < n0; j += kTailThreads) {
#pragma unroll
        for (int r = 0; r < 4; ++r) gptr(lv.x[0])[r * n0 + j] = sx[r * kTailEq + j];
    }
    if constexpr (!RHS) {
        // what a right-hand-side solve reads: A and C of every tail level
        // after the first, the factors of every tail level
        for (int i = 0; i <= top; ++i) {
            const int n = lv.n[i];
            const Eqs g = eqs_of(lv.m[i], n);
            const Facs gf = facs_of(lv.m[i], n);
            if (i > 0) {
                for (int j = tid; j < n; j += kTailThreads) {
#pragma unroll
                    for (int e = 0; e < 16; ++e) {
                        gptr(g.A)[e * n + j] = sA[e * kTailEq + eq[i] + j];
                        gptr(g.C)[e * n + j] = sC[e * kTailEq + eq[i] + j];
                    }
                }
            }
            for (int u = tid; u < gf.s; u += kTailThreads) {
#pragma unroll
                for (int e = 0; e < kFac; ++e) gptr(gf.f)[e * gf.s + u] = sf[e * kTailEv + ev[i] + u];
            }
        }
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

// Q** = Q* + dt S^P(Q*, P) at cell i (v holds Q* on entry); P at p[c * stride + cell]
__device__ __forceinline__ void corrected(const VamArgs &a, const double *p, int i, double dt, double *v)
{
    const int im = clampi(i - 1, a.nx), ip = clampi(i + 1, a.nx);
    const double inv2dx = 0.5 / a.dx;
    const double hm = a.qs[im], hp = a.qs[ip];
    const double hx = (hp - hm) * inv2dx, bx = (a.b[ip] - a.b[im]) * inv2dx;
    const double p0 = p[i], p1 = p[a.stride + i];
    const double dhp0 = (hp * p[ip] - hm * p[im]) * inv2dx;
    const double dhp1 = (hp * p[a.stride + ip] - hm * p[a.stride + im]) * inv2dx;
    v[1] = v[1] - dt * (dhp0 + 2.0 * p1 * bx);
    v[2] = v[2] - dt * (dhp1 - (3.0 * p0 - p1) * hx - 6.0 * (p0 - p1) * bx);
    v[3] = v[3] + dt * (2.0 * p1);
    v[4] = v[4] - dt * (6.0 * (p0 - p1));
}

// right-hand side -R(Q**(P)) of cell i's two constraint rows at the pressure
// P = a.p, from the corrected state itself (Q** at i - 1, i, i + 1): the
// Newton step's residual, for the matrix factored by the first solve
__global__ __launch_bounds__(kBlock) void k_vam_residual(VamArgs a, VamSystem m)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int ncell = 2 * a.nb;
    if (i >= ncell) return;
    const double dt = a.slots[a.sb].dt;
    double R0 = 0.0, R1 = 0.0;
    if (i < a.nx && dt != 0.0) {
        const int im = clampi(i - 1, a.nx), ip = clampi(i + 1, a.nx);
        const double inv2dx = 0.5 / a.dx;
        double vm[5], v[5], vp[5];
        load_cell(a.qs, a.stride, im, vm);
        load_cell(a.qs, a.stride, i, v);
        load_cell(a.qs, a.stride, ip, vp);
        corrected(a, a.p, im, dt, vm);
        corrected(a, a.p, i, dt, v);
        corrected(a, a.p, ip, dt, vp);
        const double h = v[0], ih = 1.0 / h;
        const double hx = (vp[0] - vm[0]) * inv2dx, bx = (a.b[ip] - a.b[im]) * inv2dx;
        const double u0x = (vp[1] / vp[0] - vm[1] / vm[0]) * inv2dx;
        const double u0 = v[1] * ih, u1 = v[2] * ih, w0 = v[3] * ih, w1 = v[4] * ih;
        R0 = h * u0x + (vp[2] - vm[2]) * inv2dx / 3.0 + u1 * hx / 3.0 + 2.0 * (w0 - u0 * bx);
        R1 = h * u0x + u1 * hx + 2.0 * (u1 * bx - w1);
    }
    const int k = i >> 1, r0 = 2 * (i & 1);
    m.d[r0 * a.nb + k] = -R0;
    m.d[(r0 + 1) * a.nb + k] = -R1;
}

__global__ __launch_bounds__(kBlock) void k_vam_correct(VamArgs a)
{
    const double dt = a.slots[a.sb].dt;
    const long long step = a.slots[a.sb].step;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double r = 0.0;
    if (i < a.nx) {
        double v[5];
        load_cell(a.qs, a.stride, i, v);
        if (dt != 0.0) {
            corrected(a, a.p, i, dt, v);
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

hipError_t launch_vam_assemble(const VamArgs &a, const VamSystem &m, hipStream_t s)
{
    hipLaunchKernelGGL(k_vam_assemble, dim3(blocks_for(2 * (int64_t)a.nb)), dim3(kBlock), 0, s, a, m);
    return hipGetLastError();
}

hipError_t launch_vam_residual(const VamArgs &a, const VamSystem &m, hipStream_t s)
{
    hipLaunchKernelGGL(k_vam_residual, dim3(blocks_for(2 * (int64_t)a.nb)), dim3(kBlock), 0, s, a, m);
    return hipGetLastError();
}

hipError_t launch_vam_reduce(int n, const VamSystem &src, const VamSystem &dst, bool rhs_only, hipStream_t s)
{
    const int nd = n / 2;
    if (nd == 0) return hipSuccess;
    if (rhs_only)
        hipLaunchKernelGGL(k_vam_cr_rhs, dim3(blocks_for(nd)), dim3(kBlock), 0, s, n, src, dst);
    else
        hipLaunchKernelGGL(k_vam_cr_reduce, dim3((nd + kRedThreads - 2) / (kRedThreads - 1)), dim3(kRedThreads), 0, s,
                           n, src, dst);
    return hipGetLastError();
}

hipError_t launch_vam_back(int n, const VamSystem &m, const double *xup, double *x, hipStream_t s)
{
    hipLaunchKernelGGL(k_vam_cr_back, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, m, xup, x);
    return hipGetLastError();
}

hipError_t launch_vam_tail(const VamTail *lv_dev, bool rhs_only, hipStream_t s)
{
    if (rhs_only)
        hipLaunchKernelGGL(k_vam_cr_tail<true>, dim3(1), dim3(kTailThreads), 0, s, lv_dev);
    else
        hipLaunchKernelGGL(k_vam_cr_tail<false>, dim3(1), dim3(kTailThreads), 0, s, lv_dev);
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
