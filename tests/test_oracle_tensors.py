"""Pins of the oracle's exact basis tensors against closed forms.

Definitions (Eq. (1), Sec. 2.1.1 ``Basismatrices``, Sec. 3.4): phi_k(zeta) =
P_k(1 - 2 zeta); M_k = <phi_k, phi_k>; A_ijk = <phi_i phi_j, phi_k>;
B_ijk = <phi_i Phi_j, phi_k'> with Phi_j = int_0^zeta phi_j; K_jk = <phi_j', phi_k'>.
The closed forms below follow from Legendre orthogonality and integration by
parts, not from the oracle's code.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import tensors as T

LEVELS = list(range(0, 9))


@pytest.mark.parametrize("N", LEVELS)
def test_mass_matrix_closed_form(N):
    e = T.exact(N)
    assert e["M"] == [Fraction(1, 2 * k + 1) for k in range(N + 1)]


@pytest.mark.parametrize("N", LEVELS)
def test_bed_value_and_mean(N):
    # phi_k(0) = P_k(1) = 1 and <1, phi_k> = delta_k0 (zero mean for k >= 1)
    e = T.exact(N)
    assert e["phi0"] == [1] * (N + 1)
    for k in range(N + 1):
        # <1, phi_k> = A_00k (phi_0 = 1)
        assert e["A"][0][0][k] == (1 if k == 0 else 0)


@pytest.mark.parametrize("N", LEVELS)
def test_A_symmetry_and_first_slice(N):
    e = T.exact(N)
    n = N + 1
    for i in range(n):
        for j in range(n):
            for k in range(n):
                a = e["A"][i][j][k]
                assert a == e["A"][j][i][k] == e["A"][k][j][i]
                if i == 0:
                    assert a == (Fraction(1, 2 * k + 1) if j == k else 0)
                # Legendre triple products vanish unless i+j+k even and triangle inequality
                if (i + j + k) % 2 == 1 or i > j + k or j > i + k or k > i + j:
                    assert a == 0


@pytest.mark.parametrize("N", LEVELS)
def test_B_first_slice_by_parts(N):
    # B_0jk = int Phi_j phi_k' = [Phi_j phi_k]_0^1 - <phi_j, phi_k> = -delta_jk M_k (j >= 1)
    e = T.exact(N)
    for j in range(1, N + 1):
        for k in range(N + 1):
            assert e["B"][0][j][k] == (-Fraction(1, 2 * k + 1) if j == k else 0)
    # k = 0 slice vanishes because phi_0' = 0
    for i in range(N + 1):
        for j in range(N + 1):
            assert e["B"][i][j][0] == 0


@pytest.mark.parametrize("N", LEVELS)
def test_B_integration_by_parts_identity(N):
    # For j >= 1, Phi_j(0) = Phi_j(1) = 0, so integrating (phi_i phi_k)' Phi_j by parts
    # gives  <phi_i' Phi_j, phi_k> + <phi_i Phi_j, phi_k'> = -<phi_i phi_k, phi_j>,
    # i.e.  B_kji + B_ijk = -A_ijk.
    e = T.exact(N)
    for i in range(N + 1):
        for j in range(1, N + 1):
            for k in range(N + 1):
                assert e["B"][k][j][i] + e["B"][i][j][k] == -e["A"][i][j][k]


@pytest.mark.parametrize("N", LEVELS)
def test_K_closed_form(N):
    # int_0^1 phi_j' phi_k' = 2 int_{-1}^1 P_j' P_k' = 2 m (m+1), m = min(j,k), j+k even
    e = T.exact(N)
    for j in range(N + 1):
        for k in range(N + 1):
            m = min(j, k)
            want = 2 * m * (m + 1) if (j + k) % 2 == 0 else 0
            assert e["K"][j][k] == want


def test_level2_values():
    # hand-integrated values at N = 2 (phi_1 = 1 - 2z, phi_2 = 1 - 6z + 6z^2)
    e = T.exact(2)
    B = e["B"]
    assert B[1][1][2] == Fraction(-1, 5)
    assert B[1][2][1] == Fraction(-1, 15)
    assert B[2][1][1] == Fraction(1, 15)
    assert B[2][2][2] == Fraction(-1, 35)
    assert e["A"][1][1][2] == Fraction(2, 15)
    assert e["A"][2][2][2] == Fraction(2, 35)


@pytest.mark.parametrize("N", [3, 8])
def test_float_tensors_match_quadrature(N):
    # independent route: numpy's Legendre series (legder/legint) on a Gauss grid
    L = np.polynomial.legendre
    x, w = L.leggauss(20)
    z = 0.5 * (1 - x)             # zeta with x = 1 - 2 zeta
    wz = 0.5 * w
    n = N + 1
    phi = np.array([L.legval(x, np.eye(n)[k]) for k in range(n)])
    dphi = np.array([-2.0 * L.legval(x, L.legder(np.eye(n)[k])) for k in range(n)])
    # Phi_j(zeta) = int_0^zeta P_j(1 - 2s) ds = -1/2 (Q_j(1-2 zeta) - Q_j(1)), Q_j' = P_j
    Q = [L.legint(np.eye(n)[k]) for k in range(n)]
    Phi = np.array([-0.5 * (L.legval(x, Q[k]) - L.legval(1.0, Q[k])) for k in range(n)])
    t = T.tensors(N)
    A = np.einsum("ig,jg,kg,g->ijk", phi, phi, phi, wz)
    B = np.einsum("ig,jg,kg,g->ijk", phi, Phi, dphi, wz)
    K = np.einsum("jg,kg,g->jk", dphi, dphi, wz)
    np.testing.assert_allclose(t["A"], A, atol=1e-13)
    np.testing.assert_allclose(t["B"], B, atol=1e-13)
    np.testing.assert_allclose(t["K"], K, atol=1e-11)
