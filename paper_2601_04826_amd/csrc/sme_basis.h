// sme_basis.h -- compile-time basis tensors of the shallow moment equations.
//
// The vertical velocity is expanded in the shifted Legendre family
// phi_k(zeta) = P_k(1 - 2 zeta), zeta in [0, 1] with zeta = 0 at the bed
// (Sec. 2.1.1, "Basismatrices"; Eq. (1)).  The model needs the depth integrals
//   M_k   = <phi_k, phi_k>,      A_ijk = <phi_i phi_j, phi_k>,
//   B_ijk = <phi_i Phi_j, phi_k'> with Phi_j(zeta) = int_0^zeta phi_j,
//   K_jk  = <phi_j', phi_k'>     (Newtonian bulk friction, Sec. 3.4).
// They are evaluated here at compile time, exactly: every phi_k has integer
// coefficients in zeta, products stay integer (__int128), and the integral over
// [0, 1] of sum_m c_m zeta^m is the fraction sum_m c_m / (m + 1), reduced once
// and rounded once to double.  Being constexpr, the kernels see the tensors as
// literals, so structurally zero entries cost nothing after unrolling.
#pragma once

#include <stdint.h>

namespace sme {

constexpr int kMaxLevel = 8;
constexpr int kMaxDeg = 3 * kMaxLevel + 2;  // degree bound of any triple product below

struct IPoly {               // integer polynomial in zeta, scaled by `scale`
    __int128 c[kMaxDeg + 1];
    int deg;
};

constexpr __int128 iabs128(__int128 a) { return a < 0 ? -a : a; }
constexpr __int128 gcd128(__int128 a, __int128 b)
{
    a = iabs128(a);
    b = iabs128(b);
    while (b != 0) {
        __int128 t = a % b;
        a = b;
        b = t;
    }
    return a;
}

constexpr IPoly pzero()
{
    IPoly p{};
    for (int i = 0; i <= kMaxDeg; ++i) p.c[i] = 0;
    p.deg = 0;
    return p;
}

constexpr IPoly pmul(const IPoly &a, const IPoly &b)
{
    IPoly r = pzero();
    for (int i = 0; i <= a.deg; ++i)
        for (int j = 0; j <= b.deg; ++j) r.c[i + j] += a.c[i] * b.c[j];
    r.deg = a.deg + b.deg;
    return r;
}

constexpr IPoly pder(const IPoly &a)
{
    IPoly r = pzero();
    for (int i = 1; i <= a.deg; ++i) r.c[i - 1] = a.c[i] * i;
    r.deg = a.deg > 0 ? a.deg - 1 : 0;
    return r;
}

// shifted Legendre phi_k(zeta) = P_k(1 - 2 zeta) has integer coefficients:
// phi_k(zeta) = sum_m (-1)^m C(k, m) C(k + m, m) zeta^m.
constexpr __int128 binom(int n, int k)
{
    __int128 r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

constexpr IPoly phi(int k)
{
    IPoly r = pzero();
    for (int m = 0; m <= k; ++m) r.c[m] = ((m % 2) ? -1 : 1) * binom(k, m) * binom(k + m, m);
    r.deg = k;
    return r;
}

// lcm(1..9) = 2520 makes 2520 * Phi_j an integer polynomial for every j <= 8
constexpr __int128 kPhiScale = 2520;

// kPhiScale * Phi_j(zeta), Phi_j(0) = 0
constexpr IPoly phi_int_scaled(int j)
{
    IPoly p = phi(j);
    IPoly r = pzero();
    for (int m = 0; m <= p.deg; ++m) r.c[m + 1] = p.c[m] * (kPhiScale / (m + 1));
    r.deg = p.deg + 1;
    return r;
}

struct Rat {
    __int128 num, den;
};

// exact int_0^1 p / scale as a reduced fraction
constexpr Rat integrate(const IPoly &p, __int128 scale)
{
    __int128 den = 1;  // lcm(1..deg+1)
    for (int m = 1; m <= p.deg + 1; ++m) den = den / gcd128(den, m) * m;
    __int128 num = 0;
    for (int m = 0; m <= p.deg; ++m) num += p.c[m] * (den / (m + 1));
    den *= scale;
    __int128 g = gcd128(num, den);
    if (g != 0) {
        num /= g;
        den /= g;
    }
    return Rat{num, den};
}

// mul * r rounded once to double
constexpr double to_double(Rat r, __int128 mul = 1)
{
    __int128 num = r.num * mul, den = r.den;
    __int128 g = gcd128(num, den);
    if (g != 0) {
        num /= g;
        den /= g;
    }
    return (double)num / (double)den;
}

template <int N>
struct Tensors {
    static constexpr int n = N + 1;
    double M[n];
    double invM[n];
    double A[n][n][n];
    double B[n][n][n];
    double K[n][n];
    // the same tensors divided by M_k (their last index), each rounded once:
    // AM_ijk = A_ijk / M_k, BM_ijk = B_ijk / M_k, KM_jk = K_jk / M_k
    double AM[n][n][n];
    double BM[n][n][n];
    double KM[n][n];
};

template <int N>
constexpr Tensors<N> make_tensors()
{
    constexpr int n = N + 1;
    Tensors<N> t{};
    IPoly ph[n] = {}, dph[n] = {}, Ph[n] = {};
    for (int k = 0; k < n; ++k) {
        ph[k] = phi(k);
        dph[k] = pder(ph[k]);
        Ph[k] = phi_int_scaled(k);
    }
    for (int k = 0; k < n; ++k) {
        t.M[k] = to_double(integrate(pmul(ph[k], ph[k]), 1));
        t.invM[k] = (double)(2 * k + 1);  // exact: M_k = 1 / (2k + 1)
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            IPoly pij = pmul(ph[i], ph[j]);
            IPoly qij = pmul(ph[i], Ph[j]);
            for (int k = 0; k < n; ++k) {
                const Rat a = integrate(pmul(pij, ph[k]), 1);
                const Rat b = integrate(pmul(qij, dph[k]), kPhiScale);
                t.A[i][j][k] = to_double(a);
                t.B[i][j][k] = to_double(b);
                t.AM[i][j][k] = to_double(a, 2 * k + 1);  // 1 / M_k = 2k + 1 exactly
                t.BM[i][j][k] = to_double(b, 2 * k + 1);
            }
        }
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) {
            const Rat kk = integrate(pmul(dph[j], dph[k]), 1);
            t.K[j][k] = to_double(kk);
            t.KM[j][k] = to_double(kk, 2 * k + 1);
        }
    return t;
}

template <int N>
struct Basis {
    static constexpr Tensors<N> T = make_tensors<N>();
};

// ---------------------------------------------------------------------------
// Modes of the bulk friction for its implicit step.  With M = diag(M_k) the
// generalized eigenproblem K v = mu M v has M-orthonormal eigenvectors: the
// symmetric G = M^{-1/2} K M^{-1/2} = V diag(mu) V^T (V orthogonal), and
// P = M^{-1/2} V satisfies P^T M P = I, P^T K P = diag(mu).  Then
//   (M + e K)^{-1} = P diag(1 / (1 + e mu)) P^T,
// so a solve with M + e K needs only the constant matrices P and R = P^T M
// (= V^T M^{1/2}) and one reciprocal per mode.  K couples only moments of
// equal parity and K_0k = 0, so V is block-sparse by parity and the mean
// mode (mu = 0) is e_0.  G is diagonalised at compile time by cyclic Jacobi
// rotations in double precision; w = P^T 1 serves the rank-one slip term.
constexpr double csqrt(double a)
{
    if (!(a > 0.0)) return 0.0;
    double x = a > 1.0 ? a : 1.0;  // Newton from above decreases monotonically
    for (int i = 0; i < 400; ++i) {
        const double nx = 0.5 * (x + a / x);
        if (!(nx < x)) break;
        x = nx;
    }
    return x;
}

constexpr double cabs(double a) { return a < 0.0 ? -a : a; }

template <int N>
struct FrictionModes {
    static constexpr int n = N + 1;
    double mu[n];     // eigenvalues of K v = mu M v
    double P[n][n];   // P[j][m]: component j of mode m (M-orthonormal)
    double R[n][n];   // R[m][j] = (P^T M)[m][j]: modal coordinate m of a momentum vector
    double w[n];      // w[m] = sum_j P[j][m]
};

template <int N>
constexpr FrictionModes<N> make_modes()
{
    constexpr int n = N + 1;
    const auto &T = Basis<N>::T;
    double G[n][n] = {}, V[n][n] = {}, sq[n] = {};
    for (int k = 0; k < n; ++k) sq[k] = csqrt((double)(2 * k + 1));  // M_k^{-1/2}
    for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) {
            G[j][k] = T.K[j][k] * sq[j] * sq[k];
            V[j][k] = j == k ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) (p == q ? diag : off) += G[p][q] * G[p][q];
        if (off <= 1e-34 * diag) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                if (G[p][q] == 0.0) continue;
                const double th = (G[q][q] - G[p][p]) / (2.0 * G[p][q]);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (cabs(th) + csqrt(th * th + 1.0));
                const double c = 1.0 / csqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // G <- G J (columns p, q)
                    const double gp = G[k][p], gq = G[k][q];
                    G[k][p] = c * gp - s * gq;
                    G[k][q] = s * gp + c * gq;
                }
                for (int k = 0; k < n; ++k) {  // G <- J^T G (rows p, q)
                    const double gp = G[p][k], gq = G[q][k];
                    G[p][k] = c * gp - s * gq;
                    G[q][k] = s * gp + c * gq;
                }
                G[p][q] = G[q][p] = 0.0;
                for (int k = 0; k < n; ++k) {  // V <- V J
                    const double vp = V[k][p], vq = V[k][q];
                    V[k][p] = c * vp - s * vq;
                    V[k][q] = s * vp + c * vq;
                }
            }
    }
    FrictionModes<N> f{};
    for (int m = 0; m < n; ++m) {
        f.mu[m] = G[m][m];
        f.w[m] = 0.0;
        for (int j = 0; j < n; ++j) {
            f.P[j][m] = sq[j] * V[j][m];
            f.R[m][j] = V[j][m] / sq[j];
            f.w[m] += f.P[j][m];
        }
    }
    return f;
}

template <int N>
struct Modes {
    static constexpr FrictionModes<N> F = make_modes<N>();
};

}  // namespace sme
