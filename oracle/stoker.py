"""Exact solution of the wet-bed dam break (Stoker) for the level-0 pin.

Test infrastructure only (see ``oracle/__init__``).

Level 0 of the SME hierarchy is the shallow water system (Sec. 3.1 of the
paper, which validates against the wet dam break without friction).  For a
left state (h_L, 0) and a right state (h_R, 0) with h_L > h_R > 0 the exact
solution is a left rarefaction, a constant middle state (h_m, u_m) and a right
shock.  h_m solves

    2 (sqrt(g h_L) - sqrt(g h_m)) = (h_m - h_R) sqrt(g (h_m + h_R) / (2 h_m h_R)),

i.e. the velocity behind the rarefaction equals the velocity behind the shock
(Riemann invariant across the rarefaction, Rankine-Hugoniot across the shock).
"""
import math

import numpy as np


def middle_state(hl, hr, g):
    """(h_m, u_m, shock speed) by bisection on the relation above."""
    def f(hm):
        ur = 2.0 * (math.sqrt(g * hl) - math.sqrt(g * hm))
        us = (hm - hr) * math.sqrt(g * (hm + hr) / (2.0 * hm * hr))
        return ur - us

    lo, hi = hr, hl
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    hm = 0.5 * (lo + hi)
    um = 2.0 * (math.sqrt(g * hl) - math.sqrt(g * hm))
    s = hm * um / (hm - hr)
    return hm, um, s


def solution(x, t, x0, hl, hr, g):
    """Exact (h, u) at positions x and time t > 0, dam at x0."""
    x = np.asarray(x, dtype=np.float64)
    hm, um, s = middle_state(hl, hr, g)
    cl = math.sqrt(g * hl)
    cm = math.sqrt(g * hm)
    xi = (x - x0) / t
    h = np.empty_like(xi)
    u = np.empty_like(xi)
    left = xi <= -cl
    fan = (xi > -cl) & (xi <= um - cm)
    mid = (xi > um - cm) & (xi <= s)
    right = xi > s
    h[left], u[left] = hl, 0.0
    h[fan] = (2.0 * cl - xi[fan]) ** 2 / (9.0 * g)
    u[fan] = 2.0 * (cl + xi[fan]) / 3.0
    h[mid], u[mid] = hm, um
    h[right], u[right] = hr, 0.0
    return h, u
