// sme_device.h -- per-cell and per-face arithmetic of the SME step (device side).
//
// Everything is written in the frame of a face normal n: for a state with
// depth h and moment momenta (qx_k, qy_k) the normal and tangential moment
// momenta are qa_k = qx_k n_x + qy_k n_y and qt_k = -qx_k n_y + qy_k n_x
// (1D: qa_k = q_k, no tangential block).  In that frame, with a_k = qa_k / h,
// t_k = qt_k / h, the SME flux of Sec. 3.4 (the 2D flux blocks; Eq. (1) in 1D)
// projected on n reads
//     F_h     = qa_0
//     F_a,k   = (1/M_k) h sum_ij a_i a_j A_ijk + delta_k0 g h^2 / 2
//     F_t,k   = (1/M_k) h sum_ij a_i t_j A_ijk
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
//
// All tensor contractions are unrolled at compile time over the constexpr
// basis tensors (sfor below), so only their structurally nonzero entries
// generate instructions.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "sme_basis.h"

namespace sme {

constexpr int kMaxQuad = 8;

// compile-time loop: f(integral_constant<int, I>) for I = B .. E-1
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F &&f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        sfor<B + 1, E>(f);
    }
}

// first j in [j0, n) with A[i][j][k] != 0 (or -1)
template <int N>
constexpr int first_nz_A(int i, int k, int j0 = 0)
{
    for (int j = j0; j <= N; ++j)
        if (Basis<N>::T.AM[i][j][k] != 0.0) return j;
    return -1;
}
template <int N>
constexpr int first_nz_B(int i, int k)
{
    for (int j = 1; j <= N; ++j)
        if (Basis<N>::T.BM[i][j][k] != 0.0) return j;
    return -1;
}
template <int N>
constexpr int first_nz_K(int k)
{
    for (int j = 0; j <= N; ++j)
        if (Basis<N>::T.KM[j][k] != 0.0) return j;
    return -1;
}

// sum_j A[i][j][k] v[j] / M_k over the nonzero entries (0 if none)
template <int N, int I, int K>
__device__ __forceinline__ double contract_A(const double *v)
{
    constexpr int j0 = first_nz_A<N>(I, K);
    if constexpr (j0 < 0) {
        return 0.0;
    } else {
        double s = Basis<N>::T.AM[I][j0][K] * v[j0];
        sfor<j0 + 1, N + 1>([&](auto J) {
            constexpr int j = decltype(J)::value;
            constexpr double c = Basis<N>::T.AM[I][j][K];
            if constexpr (c != 0.0) s = fma(c, v[j], s);
        });
        return s;
    }
}

// sum_{j>=1} B[i][j][k] v[j] / M_k
template <int N, int I, int K>
__device__ __forceinline__ double contract_B(const double *v)
{
    constexpr int j0 = first_nz_B<N>(I, K);
    if constexpr (j0 < 0) {
        return 0.0;
    } else {
        double s = Basis<N>::T.BM[I][j0][K] * v[j0];
        sfor<j0 + 1, N + 1>([&](auto J) {
            constexpr int j = decltype(J)::value;
            constexpr double c = Basis<N>::T.BM[I][j][K];
            if constexpr (c != 0.0) s = fma(c, v[j], s);
        });
        return s;
    }
}

// qf_k = (1/M_k) sum_ij u_i v_j A_ijk (the quadratic forms of the flux), k = 0..N
template <int N>
__device__ __forceinline__ void quad_form(const double *u, const double *v, double *out)
{
    sfor<0, N + 1>([&](auto K) {
        constexpr int k = decltype(K)::value;
        double acc = 0.0;
        bool first = true;
        sfor<0, N + 1>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (first_nz_A<N>(i, k) >= 0) {
                double c = contract_A<N, i, k>(v);
                acc = first ? u[i] * c : fma(u[i], c, acc);
                first = false;
            }
        });
        out[k] = acc;
    });
}

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

// sqrt(x) for x > 0 by Goldschmidt's iteration from the hardware reciprocal
// square-root estimate (about 26 correct bits): one coupled iteration doubles
// the bits, a final residual correction rounds to within an ulp.  Negative
// or NaN input gives NaN (the estimate does).
__device__ __forceinline__ double sqrt_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    return fma(d, h, g);
}

// Wave-speed bound lam = |a_0| + sqrt(g h + (sum_{j>=1} |a_j|)^2)
template <int N>
__device__ __forceinline__ double lam_bound(double gh, const double *a)
{
    double s = 0.0;
#pragma unroll
    for (int j = 1; j <= N; ++j) s += fabs(a[j]);
    return fabs(a[0]) + sqrt_pos(fma(s, s, gh));
}

// One side of a face in the face frame (F_h = qa_0 is not stored).
template <int N, bool TAN>
struct Side {
    static constexpr int n = N + 1;
    double h, b;
    double qa[n];
    double qt[TAN ? n : 1];
    double Fa[n];
    double Ft[TAN ? n : 1];
    double lam;
};

// Fill the flux and speed of a side whose h, b, qa, qt are set.
template <int N, bool TAN>
__device__ __forceinline__ void side_flux(Side<N, TAN> &s, double g)
{
    constexpr int n = N + 1;
    const double ih = rcp(s.h);
    double a[n], t[TAN ? n : 1];
#pragma unroll
    for (int k = 0; k < n; ++k) a[k] = s.qa[k] * ih;
    quad_form<N>(s.qa, a, s.Fa);
    if constexpr (TAN) {
#pragma unroll
        for (int k = 0; k < n; ++k) t[k] = s.qt[k] * ih;
        quad_form<N>(s.qa, t, s.Ft);
    }
    s.Fa[0] = fma(0.5 * g * s.h, s.h, s.Fa[0]);
    s.lam = lam_bound<N>(g * s.h, a);
}

// Gauss-Legendre points on [0, 1]: the 3-point rule in scalars (no indexing),
// any other rule through a device pointer read with uniform loads.
struct Quad {
    int n;
    double s0, s1, s2, w0, w1, w2;
    const double *s;
    const double *w;
};

// c0 = sum_g w_g / h(s_g), c1 = sum_g w_g s_g / h(s_g),  h(s) = hL + s dh
__device__ __forceinline__ void path_weights(const Quad &q, double hL, double dh, double &c0, double &c1)
{
    if (q.n == 3) {
        const double r0 = q.w0 * rcp(fma(q.s0, dh, hL));
        const double r1 = q.w1 * rcp(fma(q.s1, dh, hL));
        const double r2 = q.w2 * rcp(fma(q.s2, dh, hL));
        c0 = r0 + r1 + r2;
        c1 = fma(r0, q.s0, fma(r1, q.s1, r2 * q.s2));
    } else {
        c0 = 0.0;
        c1 = 0.0;
        for (int g = 0; g < q.n; ++g) {
            const double sg = q.s[g];
            const double r = q.w[g] * rcp(fma(sg, dh, hL));
            c0 += r;
            c1 = fma(r, sg, c1);
        }
    }
}

// Path-integrated NC fluctuation D between the frame states L and R (only
// their h, b, qa, qt are read), given dqa = R.qa - L.qa and dqt = R.qt - L.qt.
template <int N, bool TAN>
__device__ __forceinline__ void nc_fluct(const Side<N, TAN> &L, const Side<N, TAN> &R, double g, const Quad &q,
                                         const double *dqa, const double *dqt, double *D)
{
    constexpr int n = N + 1;
    // path averages of the velocities
    double c0, c1;
    path_weights(q, L.h, R.h - L.h, c0, c1);
    D[0] = 0.0;
    D[1] = g * (0.5 * (L.h + R.h)) * (R.b - L.b);
    if constexpr (TAN) D[1 + n] = 0.0;
    sfor<1, n>([&](auto K) {
        constexpr int k = decltype(K)::value;
        double va = 0.0, vt = 0.0;
        bool first = true;
        sfor<0, n>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (first_nz_B<N>(i, k) >= 0) {
                const double w = contract_B<N, i, k>(dqa);
                const double abar = fma(c0, L.qa[i], c1 * dqa[i]);
                va = first ? abar * w : fma(abar, w, va);
                if constexpr (TAN) {
                    const double tbar = fma(c0, L.qt[i], c1 * dqt[i]);
                    vt = first ? tbar * w : fma(tbar, w, vt);
                }
                first = false;
            }
        });
        D[1 + k] = va;
        if constexpr (TAN) D[1 + n + k] = vt;
    });
}

// Face fluxes: Fhat (Rusanov) and D (path-integrated NC fluctuation), frame
// fields [h, a_0..a_N, t_0..t_N].
template <int N, bool TAN>
__device__ __forceinline__ void face_flux(const Side<N, TAN> &L, const Side<N, TAN> &R, double g,
                                          const Quad &q, double *Fhat, double *D)
{
    constexpr int n = N + 1;
    const double hs = 0.5 * fmax(L.lam, R.lam);
    // Rusanov on W = (h + b, qa, qt)
    Fhat[0] = fma(0.5, L.qa[0] + R.qa[0], -hs * ((R.h + R.b) - (L.h + L.b)));
    double dqa[n];
#pragma unroll
    for (int k = 0; k < n; ++k) {
        dqa[k] = R.qa[k] - L.qa[k];
        Fhat[1 + k] = fma(0.5, L.Fa[k] + R.Fa[k], -hs * dqa[k]);
    }
    double dqt[TAN ? n : 1];
    if constexpr (TAN) {
#pragma unroll
        for (int k = 0; k < n; ++k) {
            dqt[k] = R.qt[k] - L.qt[k];
            Fhat[1 + n + k] = fma(0.5, L.Ft[k] + R.Ft[k], -hs * dqt[k]);
        }
    }
    nc_fluct<N, TAN>(L, R, g, q, dqa, dqt, D);
}

// Friction source (Sec. 3.4: slip at the bed, Newtonian bulk), explicit Euler
// on the predicted state: q_k += dt * S_k,
//   S_k = -(1/M_k) [ C u_b phi_k(0) + (nu / h) sum_j K_jk alpha_j ],  u_b = sum_j alpha_j,
// (phi_j(0) = 1 for the shifted Legendre basis).  q points at one moment block.
template <int N>
__device__ __forceinline__ void friction(double *q, double ih, double dt, double c_slip, double nu)
{
    constexpr int n = N + 1;
    double al[n];
    double ub = 0.0;
#pragma unroll
    for (int k = 0; k < n; ++k) {
        al[k] = q[k] * ih;
        ub += al[k];
    }
    const double cub = c_slip * ub;
    const double nuh = nu * ih;
    sfor<0, n>([&](auto K) {
        constexpr int k = decltype(K)::value;
        double bulk = 0.0;
        constexpr int j0 = first_nz_K<N>(k);
        if constexpr (j0 >= 0) {
            bulk = Basis<N>::T.KM[j0][k] * al[j0];
            sfor<j0 + 1, n>([&](auto J) {
                constexpr int j = decltype(J)::value;
                constexpr double c = Basis<N>::T.KM[j][k];
                if constexpr (c != 0.0) bulk = fma(c, al[j], bulk);
            });
        }
        // S_k = -(C u_b / M_k + (nu/h) sum_j K_jk alpha_j / M_k)
        const double S = -fma(nuh, bulk, cub * Basis<N>::T.invM[k]);
        q[k] = fma(dt, S, q[k]);
    });
}

// Friction ODE (same source S) by one backward-Euler step: q solves
//   q = q* + dt S(q)   <=>   (M + c 1 1^T + e K) q = M q*,   c = C dt / h, e = nu dt / h^2
// per moment block (h is not changed by S).  With the friction modes
// (M + e K)^{-1} = P diag(g) P^T, g_m = 1 / (1 + e mu_m), and the rank-one
// slip term by Sherman-Morrison:
//   z = g o (R q*),  beta = c (w . z) / (1 + c sum_m w_m^2 g_m),  q = P (z - beta g o w).
// The matrix is symmetric positive definite for any dt, so the step is stable
// at any nu dt / h^2 (no stiffness limit).  TWO: qy holds a second block.
template <int N, bool TWO>
__device__ __forceinline__ void friction_implicit(double *qx, double *qy, double ih, double dt, double c_slip,
                                                  double nu)
{
    constexpr int n = N + 1;
    using F = Modes<N>;  // F::F holds mu, P, R, w
    const double c = dt * c_slip * ih;
    const double e = dt * nu * (ih * ih);
    double g[n];
    double s2 = 0.0;
    sfor<0, n>([&](auto Mi) {
        constexpr int m = decltype(Mi)::value;
        if constexpr (F::F.mu[m] == 0.0)
            g[m] = 1.0;
        else
            g[m] = rcp(fma(e, F::F.mu[m], 1.0));
        s2 = fma(F::F.w[m] * F::F.w[m], g[m], s2);
    });
    const double ic = rcp(fma(c, s2, 1.0));
    auto solve = [&](double *q) {
        double z[n];
        double s1 = 0.0;
        sfor<0, n>([&](auto Mi) {
            constexpr int m = decltype(Mi)::value;
            double y = 0.0;
            sfor<0, n>([&](auto J) {
                constexpr int j = decltype(J)::value;
                if constexpr (F::F.R[m][j] != 0.0) y = fma(F::F.R[m][j], q[j], y);
            });
            z[m] = g[m] * y;
            s1 = fma(F::F.w[m], z[m], s1);
        });
        const double beta = c * s1 * ic;
        sfor<0, n>([&](auto Mi) {
            constexpr int m = decltype(Mi)::value;
            z[m] = fma(-beta * F::F.w[m], g[m], z[m]);
        });
        sfor<0, n>([&](auto J) {
            constexpr int j = decltype(J)::value;
            double v = 0.0;
            sfor<0, n>([&](auto Mi) {
                constexpr int m = decltype(Mi)::value;
                if constexpr (F::F.P[j][m] != 0.0) v = fma(F::F.P[j][m], z[m], v);
            });
            q[j] = v;
        });
    };
    solve(qx);
    if constexpr (TWO) solve(qy);
}

// The friction step of the splitting on one cell: explicit (forward Euler)
// or implicit (backward Euler, IMP); a kernel instantiation takes one of them.
template <int N, bool TWO, bool IMP>
__device__ __forceinline__ void friction_step(double *qx, double *qy, double ih, double dt, double c_slip, double nu)
{
    if constexpr (IMP) {
        friction_implicit<N, TWO>(qx, qy, ih, dt, c_slip, nu);
    } else {
        friction<N>(qx, ih, dt, c_slip, nu);
        if constexpr (TWO) friction<N>(qy, ih, dt, c_slip, nu);
    }
}

}  // namespace sme
