// sme_device.h -- per-cell and per-face arithmetic of the SME step (device side).
//
// Everything is written in the frame of a face normal n: for a state with
// depth h and moment momenta (qx_k, qy_k) the normal and tangential moment
// momenta are qa_k = qx_k n_x + qy_k n_y and qt_k = -qx_k n_y + qy_k n_x
// (1D: qa_k = q_k, no tangential block).  In that frame, with a_k = qa_k / h,
// t_k = qt_k / h, the SME flux of Sec. 3.4 (the 2D flux blocks; Eq. (1) in 1D)
// projected on n reads
//     F_h     = qa_0
//     F_a,k   = (1/M_k) sum_ij qa_i a_j A_ijk + delta_k0 g h^2 / 2
//     F_t,k   = (1/M_k) sum_ij qa_i t_j A_ijk
// (A is symmetric, so this equals n_x F_x + n_y F_y rotated into the frame).
// The non-conservative product of Eq. (1) / Sec. 3.4 contributes, for k >= 1,
//     (1/M_k) sum_i abar_i sum_{j>=1} B_ijk d(qa_j)     (normal row)
//     (1/M_k) sum_i tbar_i sum_{j>=1} B_ijk d(qa_j)     (tangential row)
// and the bed slope adds g h d(b) to the k = 0 normal row.
//
// Face scheme (Sec. 2.1.2: path-conservative finite volumes): Rusanov flux on
// W = (h + b, qa, qt) with speed s = max(lam_L, lam_R), and the fluctuation of
// the non-conservative product integrated along the straight path
// Q(s) = Q_L + s (Q_R - Q_L) with Gauss-Legendre points.  Along that path the
// product is linear in the velocities, so the integral only needs the path
// averages abar_i = int_0^1 qa_i(s)/h(s) ds = c0 qa_i^L + c1 d(qa_i) with
// c0 = sum_g w_g / h(s_g), c1 = sum_g w_g s_g / h(s_g).
// The left cell receives Fhat + D/2, the right cell -Fhat + D/2.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "sme_basis.h"

namespace sme {

constexpr int kMaxQuad = 8;

// 1/x for the positive depths of the scheme: hardware estimate refined by two
// Newton steps (error below one ulp after the second step).
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Wave-speed bound lam = |a_0| + sqrt(g h + (sum_{j>=1} |a_j|)^2)
template <int N>
__device__ __forceinline__ double lam_bound(double gh, const double *a)
{
    double s = 0.0;
#pragma unroll
    for (int j = 1; j <= N; ++j) s += fabs(a[j]);
    return fabs(a[0]) + sqrt(fma(s, s, gh));
}

// One side of a face in the face frame.
template <int N, bool TAN>
struct Side {
    static constexpr int n = N + 1;
    double h, b;
    double qa[n];
    double qt[TAN ? n : 1];
    double Fh;
    double Fa[n];
    double Ft[TAN ? n : 1];
    double lam;
};

// Fill the flux and speed of a side whose h, b, qa, qt are set.
template <int N, bool TAN>
__device__ __forceinline__ void side_flux(Side<N, TAN> &s, double g)
{
    constexpr int n = N + 1;
    const auto &T = Basis<N>::T;
    double ih = rcp(s.h);
    double a[n], t[TAN ? n : 1];
#pragma unroll
    for (int k = 0; k < n; ++k) a[k] = s.qa[k] * ih;
    if constexpr (TAN) {
#pragma unroll
        for (int k = 0; k < n; ++k) t[k] = s.qt[k] * ih;
    }
    s.Fh = s.qa[0];
#pragma unroll
    for (int k = 0; k < n; ++k) {
        double fa = 0.0, ft = 0.0;
#pragma unroll
        for (int i = 0; i < n; ++i) {
            double sa = 0.0, st = 0.0;
#pragma unroll
            for (int j = 0; j < n; ++j) {
                if (T.A[i][j][k] != 0.0) {
                    sa = fma(T.A[i][j][k], a[j], sa);
                    if constexpr (TAN) st = fma(T.A[i][j][k], t[j], st);
                }
            }
            fa = fma(s.qa[i], sa, fa);
            if constexpr (TAN) ft = fma(s.qa[i], st, ft);
        }
        s.Fa[k] = fa * T.invM[k];
        if constexpr (TAN) s.Ft[k] = ft * T.invM[k];
    }
    s.Fa[0] = fma(0.5 * g * s.h, s.h, s.Fa[0]);
    s.lam = lam_bound<N>(g * s.h, a);
}

struct Quad {
    int n;
    double s[kMaxQuad];
    double w[kMaxQuad];
};

// Face fluxes: Fhat (Rusanov) and D (path-integrated NC fluctuation), frame fields.
// Output layout: [h, a_0..a_N, t_0..t_N].
template <int N, bool TAN>
__device__ __forceinline__ void face_flux(const Side<N, TAN> &L, const Side<N, TAN> &R, double g,
                                          const Quad &q, double *Fhat, double *D)
{
    constexpr int n = N + 1;
    const auto &T = Basis<N>::T;
    const double s = fmax(L.lam, R.lam);
    const double hs = 0.5 * s;
    // Rusanov on W = (h + b, qa, qt)
    Fhat[0] = 0.5 * (L.Fh + R.Fh) - hs * ((R.h + R.b) - (L.h + L.b));
#pragma unroll
    for (int k = 0; k < n; ++k) Fhat[1 + k] = 0.5 * (L.Fa[k] + R.Fa[k]) - hs * (R.qa[k] - L.qa[k]);
    if constexpr (TAN) {
#pragma unroll
        for (int k = 0; k < n; ++k)
            Fhat[1 + n + k] = 0.5 * (L.Ft[k] + R.Ft[k]) - hs * (R.qt[k] - L.qt[k]);
    }
    // path averages of the velocities
    const double dh = R.h - L.h;
    double c0 = 0.0, c1 = 0.0;
    for (int gq = 0; gq < q.n; ++gq) {
        double r = rcp(fma(q.s[gq], dh, L.h));
        double wr = q.w[gq] * r;
        c0 += wr;
        c1 = fma(wr, q.s[gq], c1);
    }
    double dqa[n];
#pragma unroll
    for (int k = 0; k < n; ++k) dqa[k] = R.qa[k] - L.qa[k];
    // W_ik = sum_{j>=1} B_ijk d(qa_j)
    D[0] = 0.0;
    D[1] = g * 0.5 * (L.h + R.h) * (R.b - L.b);
#pragma unroll
    for (int k = 1; k < n; ++k) {
        double va = 0.0, vt = 0.0;
#pragma unroll
        for (int i = 0; i < n; ++i) {
            double w = 0.0;
#pragma unroll
            for (int j = 1; j < n; ++j)
                if (T.B[i][j][k] != 0.0) w = fma(T.B[i][j][k], dqa[j], w);
            double abar = fma(c0, L.qa[i], c1 * dqa[i]);
            va = fma(abar, w, va);
            if constexpr (TAN) {
                double tbar = fma(c0, L.qt[i], c1 * (R.qt[i] - L.qt[i]));
                vt = fma(tbar, w, vt);
            }
        }
        D[1 + k] = va * T.invM[k];
        if constexpr (TAN) D[1 + n + k] = vt * T.invM[k];
    }
    if constexpr (TAN) D[1 + n] = 0.0;
}

// Friction source (Sec. 3.4: slip at the bed, Newtonian bulk), explicit Euler
// on the predicted state: q_k += dt * S_k,
//   S_k = -(1/M_k) [ C u_b phi_k(0) + (nu / h) sum_j K_jk alpha_j ],  u_b = sum_j alpha_j,
// (phi_j(0) = 1 for the shifted Legendre basis).  q points at one moment block.
template <int N>
__device__ __forceinline__ void friction(double *q, double ih, double dt, double c_slip, double nu)
{
    constexpr int n = N + 1;
    const auto &T = Basis<N>::T;
    double al[n];
    double ub = 0.0;
#pragma unroll
    for (int k = 0; k < n; ++k) {
        al[k] = q[k] * ih;
        ub += al[k];
    }
    const double cub = c_slip * ub;
    const double nuh = nu * ih;
#pragma unroll
    for (int k = 0; k < n; ++k) {
        double bulk = 0.0;
#pragma unroll
        for (int j = 0; j < n; ++j)
            if (T.K[j][k] != 0.0) bulk = fma(T.K[j][k], al[j], bulk);
        double S = -(cub + nuh * bulk) * T.invM[k];
        q[k] = fma(dt, S, q[k]);
    }
}

}  // namespace sme
