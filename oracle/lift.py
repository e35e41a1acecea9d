"""3D lifting of an SME state (the paper's ``interpolate_3d`` postprocessing).

Test infrastructure only (see ``oracle/__init__``).

The depth-averaged state is mapped back to the flow variables of the 3D
incompressible setting (Sec. 2.2.1 postprocessing; the SWE lifting printed in
Sec. 3.1 is the level-0 case):

  z(zeta)  = b + zeta h                           elevation of sigma level zeta in [0, 1]
  u(zeta)  = sum_k alpha_k phi_k(zeta),  v(zeta) = sum_k beta_k phi_k(zeta)
  p(zeta)  = rho g h (1 - zeta)                   hydrostatic pressure
  w(zeta)  from incompressibility d_x u + d_y v + d_z w = 0 with the kinematic
           bed condition w(b) = u(b) d_x b + v(b) d_y b.  With
           int_b^z u dz' = h sum_k alpha_k Phi_k(zeta), Phi_k(zeta) = int_0^zeta phi_k,
           and Leibniz' rule at fixed z this gives
           w = -sum_k (d_x qx_k + d_y qy_k) Phi_k(zeta)
               + u(zeta) (d_x b + zeta d_x h) + v(zeta) (d_y b + zeta d_y h).
           At level 0 on a flat bed w(1) = -h (d_x u + d_y v), the printed SWE case.

The horizontal derivatives come from least-squares gradients over the face
neighbours (the ``compute_derivatives`` building block, Sec. 2.1.2): for each
cell the gradient g minimising sum_j (f_j - f_i - g . d_j)^2 over its interior
neighbours j (d_j the displacement from cell i to cell j), the minimum-norm
solution where that problem is
rank deficient (numpy.linalg.lstsq).  On a uniform grid the displacement
across a face is its outward normal times the spacing (across a periodic
boundary too), and the gradient is the central difference inside and the
one-sided difference at a wall or open end.
"""
import numpy as np

from . import tensors as _tensors


def _phi_and_Phi(level, zeta):
    """phi_k(zeta) and Phi_k(zeta) = int_0^zeta phi_k from the exact polynomials."""
    polys = _tensors.basis(level)
    phi, Phi = [], []
    for p in polys:
        c = [float(v) for v in p]
        ci = [0.0] + [float(v) / (i + 1) for i, v in enumerate(p)]  # antiderivative, 0 at zeta = 0
        phi.append(np.polynomial.polynomial.polyval(zeta, c))
        Phi.append(np.polynomial.polynomial.polyval(zeta, ci))
    return np.array(phi), np.array(Phi)


def lsq_gradients(m, F, spacing=None, cells=None):
    """Least-squares gradients of the rows of F ([nfield, ncells]) on mesh m.

    spacing: (dx, dy) of a uniform 1D or structured grid; the displacement
    across a face is then its outward normal times the spacing (which also
    holds across a periodic boundary).  None: centre-to-centre displacements
    (triangles).  cells: only these cells (default all).
    Returns G [nfield, len(cells), dim]."""
    nf, nc = F.shape
    dim = m.dim
    cells = np.arange(nc) if cells is None else np.asarray(cells)
    G = np.zeros((nf, len(cells), dim))
    cen = np.asarray(m.centers, dtype=np.float64).reshape(nc, -1)
    for c, i in enumerate(cells):
        rows, rhs = [], []
        for s in range(m.maxf):
            j = m.nbr[i, s]
            if j < 0:
                continue                      # wall, open end or unused slot: no interior neighbour
            if spacing is not None:
                d = np.array([m.nx[i, s] * spacing[0], m.ny[i, s] * spacing[1]])
            else:
                d = cen[j] - cen[i]
            rows.append(d[:dim])
            rhs.append(F[:, j] - F[:, i])
        if not rows:
            continue
        A = np.array(rows)
        R = np.array(rhs)                     # [nnbr, nfield]
        g, *_ = np.linalg.lstsq(A, R, rcond=None)
        G[:, c, :] = g.T
    return G


def interpolate_3d(level, m, Q, b, zeta, rho=1.0, g=9.81, spacing=None, cells=None):
    """Lifted fields at the sigma levels zeta: dict of z, u, v, w, p, each
    [len(zeta), ncells] (v = 0 in 1D); cells: only these cells (columns in
    that order)."""
    zeta = np.asarray(zeta, dtype=np.float64)
    n = level + 1
    Q = np.asarray(Q, dtype=np.float64)
    h = Q[0]
    qx = Q[1:1 + n]
    qy = Q[1 + n:1 + 2 * n] if m.dim == 2 else np.zeros_like(qx)
    b = np.zeros(h.shape) if b is None else np.asarray(b, dtype=np.float64)
    fields = np.vstack([h[None], b[None], qx, qy])
    G = lsq_gradients(m, fields, spacing, cells)
    if cells is not None:
        h, b, qx, qy = h[cells], b[cells], qx[:, cells], qy[:, cells]
    gx = G[..., 0]
    gy = G[..., 1] if m.dim == 2 else np.zeros_like(gx)
    dh_x, db_x, dqx_x = gx[0], gx[1], gx[2:2 + n]
    dh_y, db_y, dqy_y = gy[0], gy[1], gy[2 + n:2 + 2 * n]
    phi, Phi = _phi_and_Phi(level, zeta)          # [n, nz]
    al, be = qx / h, qy / h
    u = phi.T @ al                                 # [nz, ncells]
    v = phi.T @ be
    div = dqx_x + dqy_y                            # [n, ncells]
    w = (-(Phi.T @ div) + u * (db_x + zeta[:, None] * dh_x) + v * (db_y + zeta[:, None] * dh_y))
    p = rho * g * h[None, :] * (1.0 - zeta[:, None])
    z = b[None, :] + zeta[:, None] * h[None, :]
    return dict(z=z, u=u, v=v, w=w, p=p)


def spacing_of(problem):
    """(dx, dy) of a 1D or structured workload, None for triangles."""
    if problem["kind"] == "tri":
        return None
    dx = (problem["x1"] - problem["x0"]) / problem["nx"]
    dy = (problem.get("y1", 1.0) - problem.get("y0", 0.0)) / problem.get("ny", 1)
    return (dx, dy)
