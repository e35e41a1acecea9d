"""Exact basis tensors of the shallow moment equations (oracle side).

Test infrastructure only (see ``oracle/__init__``).

The paper (Sec. 2.1.1, the ``Basismatrices`` description, and Eq. (1)) builds
the SME from depth integrals of products of the vertical basis functions
phi_k(zeta), zeta in [0, 1] with zeta = 0 at the bed.  The basis is the
shifted Legendre family; the reading used here is phi_k(zeta) = P_k(1 - 2 zeta)
so that phi_k(0) = 1 (any other sign convention maps alpha_j -> (-1)^j alpha_j
and leaves every physical quantity unchanged).

All integrals are over zeta in [0, 1] and are computed exactly with
``fractions.Fraction`` polynomial arithmetic, then rounded once to float:

    M_k    = <phi_k, phi_k>                       (mass matrix, diagonal)
    A_ijk  = <phi_i phi_j, phi_k>                 (conservative flux, Eq. (1))
    B_ijk  = <phi_i Phi_j, phi_k'>,  Phi_j(z) = int_0^z phi_j   (NC term, Eq. (1))
    K_jk   = <phi_j', phi_k'>                     (Newtonian bulk friction, Sec. 3.4)
    phi_k(0)                                      (bed value, slip closure, Sec. 3.4)
"""
from fractions import Fraction
from functools import lru_cache

import numpy as np

MAX_LEVEL = 8


# --- polynomial helpers: coefficient lists, index = power of zeta -----------
def _padd(p, q):
    n = max(len(p), len(q))
    return [(p[i] if i < len(p) else 0) + (q[i] if i < len(q) else 0) for i in range(n)]


def _pscale(p, c):
    return [c * a for a in p]


def _pmul(p, q):
    out = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        if a == 0:
            continue
        for j, b in enumerate(q):
            out[i + j] += a * b
    return out


def _pder(p):
    return [i * p[i] for i in range(1, len(p))] or [Fraction(0)]


def _pint0(p):
    """Antiderivative that vanishes at zeta = 0."""
    return [Fraction(0)] + [p[i] / (i + 1) for i in range(len(p))]


def _pint01(p):
    """Exact integral over [0, 1]."""
    return sum((p[i] / (i + 1) for i in range(len(p))), Fraction(0))


def _peval(p, x):
    return sum((c * x ** i for i, c in enumerate(p)), Fraction(0))


@lru_cache(maxsize=None)
def basis(level):
    """phi_0..phi_level as exact coefficient lists in zeta.

    Legendre P_k(x) by Bonnet's recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1},
    then x = 1 - 2 zeta.
    """
    x = [Fraction(1), Fraction(-2)]           # 1 - 2 zeta
    polys = [[Fraction(1)]]
    if level >= 1:
        polys.append(list(x))
    for k in range(1, level):
        t = _pscale(_pmul(x, polys[k]), Fraction(2 * k + 1, k + 1))
        u = _pscale(polys[k - 1], Fraction(-k, k + 1))
        polys.append(_padd(t, u))
    return tuple(tuple(p) for p in polys)


@lru_cache(maxsize=None)
def exact(level):
    """Exact tensors for levels 0..level as dict of nested Fraction lists."""
    phi = [list(p) for p in basis(level)]
    dphi = [_pder(p) for p in phi]
    Phi = [_pint0(p) for p in phi]
    n = level + 1
    M = [_pint01(_pmul(phi[k], phi[k])) for k in range(n)]
    A = [[[_pint01(_pmul(_pmul(phi[i], phi[j]), phi[k])) for k in range(n)]
          for j in range(n)] for i in range(n)]
    B = [[[_pint01(_pmul(_pmul(phi[i], Phi[j]), dphi[k])) for k in range(n)]
          for j in range(n)] for i in range(n)]
    K = [[_pint01(_pmul(dphi[j], dphi[k])) for k in range(n)] for j in range(n)]
    phi0 = [_peval(phi[k], Fraction(0)) for k in range(n)]
    return {"M": M, "A": A, "B": B, "K": K, "phi0": phi0}


def tensors(level):
    """Float64 tensors for ``level``: M (n,), A (n,n,n), B (n,n,n), K (n,n), phi0 (n,)."""
    if not 0 <= level <= MAX_LEVEL:
        raise ValueError(f"level must be in 0..{MAX_LEVEL}")
    e = exact(level)
    return {
        "M": np.array([float(v) for v in e["M"]]),
        "A": np.array([[[float(v) for v in r] for r in m] for m in e["A"]]),
        "B": np.array([[[float(v) for v in r] for r in m] for m in e["B"]]),
        "K": np.array([[float(v) for v in r] for r in e["K"]]),
        "phi0": np.array([float(v) for v in e["phi0"]]),
    }


def phi_eval(level, zeta):
    """Evaluate phi_0..phi_level at the points ``zeta`` (float array) -> (n, len(zeta))."""
    zeta = np.asarray(zeta, dtype=np.float64)
    out = []
    for p in basis(level):
        c = [float(v) for v in p]
        out.append(np.polynomial.polynomial.polyval(zeta, c))
    return np.array(out)
