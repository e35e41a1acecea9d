"""Non-hydrostatic VAM predictor-corrector step in 1D (Sec. 3.3 of the paper).

Test infrastructure only (see ``oracle/__init__``).

Model (the 1D vertically averaged momentum equations with linear u, quadratic
w and quadratic non-hydrostatic pressure p, Legendre basis phi_k(zeta) =
P_k(1 - 2 zeta), so phi_k(0) = 1 at the bed):

  Q = (h, h u0, h u1, h w0, h w1),  P = (p0, p1),
  w2 = -(w0 + w1) + (u0 + u1) b_x                   (kinematic bed condition)
  F  = (h u0, h u0^2 + h u1^2 / 3, 2 h u0 u1, h u0 w0 + h u1 w1 / 3,
        h u0 w1 + u1 (h w0 + 2 h w2 / 5))
  NC Q_x = (0, g h (h + b)_x, -u0 (h u1)_x, 0, (w2 / 5 - w0) (h u1)_x)

The printed NC matrix has g h only in the h column; the bed enters here as
g h b_x beside it (the same bed column as in the SME scheme), which makes the
lake at rest exact.

Scheme (the splitting of Sec. 2.1.2):

  predictor   Q* = Q^n - dt/dx [F^_{i+1/2} - F^_{i-1/2} + D_{i+1/2}/2 + D_{i-1/2}/2]
              (path-conservative Rusanov on the straight path, G-point Gauss,
               speed bound |u0| + sqrt(g h + u1^2), viscosity on h + b);
  corrector   Q** = Q* + dt S^P(Q*, P) with R(Q**) = 0 solved for P;
  no friction (the paper's VAM case has none).

S^P is the non-hydrostatic pressure source obtained by depth-averaging
-grad p against phi_0 and phi_1 (its signs follow that derivation; the
printed vector and the printed substitution code disagree in two entries):

  S^P = -(0, (h p0)_x + 2 p1 b_x, (h p1)_x - (3 p0 - p1) h_x - 6 (p0 - p1) b_x,
          -2 p1, 6 (p0 - p1))

and R the two incompressibility constraints:

  R0 = h (u0)_x + (h u1)_x / 3 + u1 h_x / 3 + 2 (w0 - u0 b_x)
  R1 = h (u0)_x + u1 h_x + 2 (u1 b_x - w1)

Spatial derivatives are central differences; at the two ends of the channel
every quantity is extended by a copy of the boundary cell (extrapolation
ends).  R(Q**(P)) is affine in P (h is not changed by S^P), so the corrector's
Newton iteration converges in one step: the oracle probes the affine map for
its sparse matrix (stencil of five cells, so five colour classes per
component) and solves it with a sparse direct solver.
"""
import numpy as np
import scipy.sparse
import scipy.sparse.linalg


def gauss01(G):
    x, w = np.polynomial.legendre.leggauss(G)
    return 0.5 * (x + 1.0), 0.5 * w


class Vam1D:
    """One 1D channel: nx cells on [x0, x1], extrapolation ends."""

    def __init__(self, nx, x0, x1, b=None, g=9.81, cfl=0.45, quad_points=3, periodic=False):
        self.nx = int(nx)
        self.dx = (x1 - x0) / nx
        self.b = np.zeros(nx) if b is None else np.asarray(b, dtype=np.float64).copy()
        self.g = g
        self.cfl = cfl
        self.s, self.w = gauss01(quad_points)
        self.periodic = periodic  # periodic ends: only for the dispersion pin

    # -- helpers ------------------------------------------------------------
    def pad(self, f):
        """f with one ghost value at each end (copy, or wrap if periodic)."""
        return np.pad(f, 1, mode="wrap" if self.periodic else "edge")

    def ddx(self, f):
        fp = self.pad(f)
        return (fp[2:] - fp[:-2]) / (2.0 * self.dx)

    def w2(self, Q):
        h = Q[0]
        u0, u1, w0, w1 = Q[1] / h, Q[2] / h, Q[3] / h, Q[4] / h
        return -(w0 + w1) + (u0 + u1) * self.ddx(self.b)

    def flux(self, Q, w2):
        h, q0, q1, r0, r1 = Q
        u0, u1 = q0 / h, q1 / h
        return np.array([q0, q0 * u0 + q1 * u1 / 3.0, 2.0 * q0 * u1, q0 * r0 / h + q1 * r1 / (3.0 * h),
                         u0 * r1 + u1 * (r0 + 0.4 * h * w2)])

    def lam(self, Q):
        h = Q[0]
        return np.abs(Q[1] / h) + np.sqrt(self.g * h + (Q[2] / h) ** 2)

    def cfl_dt(self, Q):
        lm = self.lam(Q)
        return self.cfl * self.dx / lm.max(), lm.max()

    # -- predictor ------------------------------------------------------------
    def face_terms(self, QL, QR, bL, bR, w2L, w2R):
        """Rusanov flux and NC fluctuation of faces between states QL, QR."""
        FL, FR = self.flux(QL, w2L), self.flux(QR, w2R)
        s = np.maximum(self.lam(QL), self.lam(QR))
        WL = QL.copy()
        WL[0] = QL[0] + bL
        WR = QR.copy()
        WR[0] = QR[0] + bR
        Fh = 0.5 * (FL + FR) - 0.5 * s * (WR - WL)
        dQ = QR - QL
        D = np.zeros_like(dQ)
        D[1] = self.g * 0.5 * (QL[0] + QR[0]) * (dQ[0] + (bR - bL))
        iu0 = np.zeros_like(QL[0])
        iw = np.zeros_like(QL[0])
        for sg, wg in zip(self.s, self.w):
            Qs = QL + sg * dQ
            h = Qs[0]
            iu0 += wg * Qs[1] / h
            iw += wg * (0.2 * (w2L + sg * (w2R - w2L)) - Qs[3] / h)
        D[2] = -iu0 * dQ[2]
        D[4] = iw * dQ[2]
        return Fh, D

    def predict(self, Q, dt):
        w2 = self.w2(Q)
        Qp = np.pad(Q, ((0, 0), (1, 1)), mode="wrap" if self.periodic else "edge")
        bp, w2p = self.pad(self.b), self.pad(w2)
        Fh, D = self.face_terms(Qp[:, :-1], Qp[:, 1:], bp[:-1], bp[1:], w2p[:-1], w2p[1:])
        # face f sits between padded cells f and f + 1, i.e. left of cell f
        return Q - dt / self.dx * (Fh[:, 1:] - Fh[:, :-1] + 0.5 * D[:, 1:] + 0.5 * D[:, :-1])

    # -- corrector ------------------------------------------------------------
    def correct_state(self, Qs, P, dt):
        """Q** = Q* + dt S^P(Q*, P)."""
        h = Qs[0]
        p0, p1 = P
        hx, bx = self.ddx(h), self.ddx(self.b)
        Q2 = Qs.copy()
        Q2[1] = Qs[1] - dt * (self.ddx(h * p0) + 2.0 * p1 * bx)
        Q2[2] = Qs[2] - dt * (self.ddx(h * p1) - (3.0 * p0 - p1) * hx - 6.0 * (p0 - p1) * bx)
        Q2[3] = Qs[3] + dt * 2.0 * p1
        Q2[4] = Qs[4] - dt * 6.0 * (p0 - p1)
        return Q2

    def residual(self, Q2):
        """(R0, R1) of a state."""
        h = Q2[0]
        u0, u1, w0, w1 = Q2[1] / h, Q2[2] / h, Q2[3] / h, Q2[4] / h
        hx, bx = self.ddx(h), self.ddx(self.b)
        u0x = self.ddx(u0)
        R0 = h * u0x + self.ddx(Q2[2]) / 3.0 + u1 * hx / 3.0 + 2.0 * (w0 - u0 * bx)
        R1 = h * u0x + u1 * hx + 2.0 * (u1 * bx - w1)
        return np.array([R0, R1])

    def pressure_system(self, Qs, dt):
        """Sparse matrix J and vector r with R(Q**(P)) = J P + r, P = [p0; p1]."""
        n = self.nx
        zero = np.zeros((2, n))
        r = self.residual(self.correct_state(Qs, zero, dt)).ravel()
        rows, cols, vals = [], [], []
        if n >= 5:
            assert not self.periodic or n % 5 == 0, "periodic colouring needs nx divisible by 5"
            ncol = 5
        else:
            ncol = n
        for comp in range(2):
            for c in range(ncol):
                P = np.zeros((2, n))
                P[comp, c::ncol] = 1.0
                dR = self.residual(self.correct_state(Qs, P, dt)).ravel() - r
                row = np.nonzero(dR)[0]
                cell = row % n
                # the one probed cell of colour c within two cells of `cell`
                if ncol == 5:
                    m = cell + ((c - cell + 2) % 5) - 2
                    m = m % n if self.periodic else m
                    assert np.all((m >= 0) & (m < n) & (np.abs(m - cell) % n <= 2) | (np.abs(m - cell) >= n - 2))
                else:
                    m = np.full_like(cell, c)
                rows.append(row)
                cols.append(comp * n + m)
                vals.append(dR[row])
        J = scipy.sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                    shape=(2 * n, 2 * n))
        return J, r

    def correct(self, Qs, dt):
        J, r = self.pressure_system(Qs, dt)
        P = scipy.sparse.linalg.spsolve(J.tocsc(), -r).reshape(2, self.nx)
        return self.correct_state(Qs, P, dt), P

    # -- whole step -----------------------------------------------------------
    def step(self, Q, dt=None):
        if dt is None:
            dt, _ = self.cfl_dt(Q)
        Qs = self.predict(Q, dt)
        Q2, P = self.correct(Qs, dt)
        return Q2, P, dt

    def run(self, Q, nsteps):
        t = 0.0
        P = None
        for _ in range(nsteps):
            Q, P, dt = self.step(Q)
            t += dt
        return Q, P, t
