/*
 * CPU FP64 oracle of the shallow-moment-equation (SME) time step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py.  It shares no code with the HIP library.
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 *
 * The method, stated per cell i with faces f (outward unit normal n, length
 * |e_f|, neighbour j or a ghost), follows the paper:
 *   - PDE template  dQ/dt + div F(Q) + B(Q) : grad Q = S(Q)      (Eq. (2))
 *   - 2D SME flux F_x, F_y, NC matrices and friction source        (Sec. 3.4)
 *   - 1D SME system                                               (Eq. (1))
 *   - explicit hydrostatic predictor, then the friction ODE      (Eqs. (3a), (3d))
 *   - path-conservative finite volumes for non-conservative systems (Sec. 2.1.2)
 *   - adaptive CFL time step (Sec. 3.1, CFL = 0.45)
 * with these readings where the paper is silent or inconsistent:
 *   * NC term in row k: sum_{i>=0} sum_{j>=1} alpha_i B_ijk d(h alpha_j) / M_k,
 *     with B_ijk = <phi_i Phi_j, phi_k'>; it vanishes for k = 0 (phi_0' = 0).
 *   * the bed enters as an NC column: row of the k = 0 momentum, g h n dot grad b.
 *   * friction: S_k = -(1/M_k) [ C u_b phi_k(0) + (nu/h) sum_j K_jk alpha_j ],
 *     u_b = sum_j alpha_j phi_j(0), K_jk = <phi_j', phi_k'>, for every k = 0..N.
 *   * Rusanov flux on W = (h + b, q): Fhat = (F(Q_i).n + F(Q_j).n)/2 - s/2 (W_j - W_i),
 *     s = max(lam(Q_i, n), lam(Q_j, n)); the fluctuation of the NC term along the
 *     straight path Q_i -> Q_j (Gauss-Legendre in s) is split half/half.
 *   * lam(Q, n) = |a_0| + sqrt(g h + (sum_{j>=1} |a_j|)^2), a_j = normal moment velocity.
 *   * dt = CFL * min_i 2 |V_i| / sum_f |e_f| lam(Q_i, n_f).
 *   * the friction ODE of the splitting (Eq. (3d)) is integrated by one
 *     forward-Euler step on the predicted state, or (implicit = 1) by one
 *     backward-Euler step: S is linear in the momenta for the fixed depth of
 *     the source step, so Q^{n+1} solves (I - dt L) q = q* per moment block,
 *     L the (N+1)x(N+1) matrix of S; Gaussian elimination with partial pivoting.
 *
 * State layout: SoA, Q[f * ncells + i].  1D fields (h, q_0..q_N);
 * 2D fields (h, qx_0..qx_N, qy_0..qy_N) with qx_k = h alpha_k, qy_k = h beta_k.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXN 9            /* levels 0..8 */
#define OR_MAXF (2 * OR_MAXN + 1)
#define OR_MAXQ 16

/* neighbour codes for boundary faces */
#define OR_WALL (-1)         /* reflective wall: ghost mirrors the normal velocity */
#define OR_EXTRAP (-2)       /* extrapolation: ghost = copy of the cell */

typedef struct {
    int level;                /* N */
    int dim;                  /* 1 or 2 */
    int64_t ncells;
    int maxf;                 /* face slots per cell */
    const int64_t *nbr;       /* [ncells*maxf]; >=0 neighbour, OR_WALL, OR_EXTRAP; < -2 unused slot */
    const double *fnx, *fny;  /* [ncells*maxf] outward unit normal */
    const double *flen;       /* [ncells*maxf] face length (1 in 1D) */
    const double *vol;        /* [ncells] cell volume (dx in 1D) */
    const double *b;          /* [ncells] bathymetry */
    double g, c_slip, nu, cfl;
    int nquad;                /* Gauss points for the path integral */
    const double *qs, *qw;    /* nodes on [0,1], weights summing to 1 */
    const double *M;          /* [n] */
    const double *A;          /* [n*n*n], A[(i*n+j)*n+k] */
    const double *B;          /* [n*n*n] */
    const double *K;          /* [n*n] */
    const double *phi0;       /* [n] */
    int implicit;             /* 0: explicit friction step, 1: implicit (backward Euler) */
} omesh;

static int nfields(const omesh *o) { return o->dim == 1 ? o->level + 2 : 2 * o->level + 3; }

/* ------------------------------------------------------------------------ */
/* physical flux F(Q).n, written as n_x F_x + n_y F_y with F_x, F_y as in the
 * 2D SME system (Sec. 3.4); the 1D system of Eq. (1) is the x part.        */
void oracle_flux(const omesh *o, const double *q, double nx, double ny, double *out)
{
    int n = o->level + 1, nf = nfields(o);
    double h = q[0];
    double al[OR_MAXN], be[OR_MAXN];
    for (int k = 0; k < n; k++) {
        al[k] = q[1 + k] / h;
        be[k] = (o->dim == 2) ? q[1 + n + k] / h : 0.0;
    }
    for (int f = 0; f < nf; f++) out[f] = 0.0;
    /* mass */
    out[0] = nx * h * al[0] + ny * h * be[0];
    for (int k = 0; k < n; k++) {
        double fxx = 0.0, fxy = 0.0, fyx = 0.0, fyy = 0.0;
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) {
                double a = o->A[(i * n + j) * n + k];
                fxx += h * al[i] * al[j] * a;   /* F_x, x-momentum */
                fxy += h * al[i] * be[j] * a;   /* F_x, y-momentum */
                fyx += h * be[i] * al[j] * a;   /* F_y, x-momentum */
                fyy += h * be[i] * be[j] * a;   /* F_y, y-momentum */
            }
        fxx /= o->M[k]; fxy /= o->M[k]; fyx /= o->M[k]; fyy /= o->M[k];
        if (k == 0) {
            fxx += 0.5 * o->g * h * h;
            fyy += 0.5 * o->g * h * h;
        }
        out[1 + k] = nx * fxx + ny * fyx;
        if (o->dim == 2) out[1 + n + k] = nx * fxy + ny * fyy;
    }
}

/* Non-conservative matrix B(Q).n in the convention dQ/dt + ... + B(Q).grad(Q, b) = ...
 * Output: nf rows x (nf + 1) columns, last column = bathymetry.            */
void oracle_ncmat(const omesh *o, const double *q, double nx, double ny, double *mat)
{
    int n = o->level + 1, nf = nfields(o), nc = nf + 1;
    double h = q[0];
    double al[OR_MAXN], be[OR_MAXN];
    for (int k = 0; k < n; k++) {
        al[k] = q[1 + k] / h;
        be[k] = (o->dim == 2) ? q[1 + n + k] / h : 0.0;
    }
    for (int r = 0; r < nf * nc; r++) mat[r] = 0.0;
    for (int k = 0; k < n; k++) {
        for (int j = 1; j < n; j++) {          /* derivative index: j >= 1 only */
            double sa = 0.0, sb = 0.0;
            for (int i = 0; i < n; i++) {
                sa += al[i] * o->B[(i * n + j) * n + k];
                sb += be[i] * o->B[(i * n + j) * n + k];
            }
            sa /= o->M[k];
            sb /= o->M[k];
            /* row x_k: columns x_j (x-derivative) and y_j (y-derivative) */
            mat[(1 + k) * nc + (1 + j)] += nx * sa;
            if (o->dim == 2) {
                mat[(1 + k) * nc + (1 + n + j)] += ny * sa;
                mat[(1 + n + k) * nc + (1 + j)] += nx * sb;
                mat[(1 + n + k) * nc + (1 + n + j)] += ny * sb;
            }
        }
    }
    /* bed slope: -<1, phi_k> g h grad b moved to the left-hand side; <1, phi_k> / M_k
     * is 1 for k = 0 and 0 otherwise (phi_k, k >= 1, has zero mean).          */
    mat[1 * nc + nf] = o->g * h * nx;
    if (o->dim == 2) mat[(1 + n) * nc + nf] = o->g * h * ny;
}

/* lam(Q, n) = |a_0| + sqrt(g h + (sum_{j>=1}|a_j|)^2) */
double oracle_lambda(const omesh *o, const double *q, double nx, double ny)
{
    int n = o->level + 1;
    double h = q[0];
    double a[OR_MAXN];
    for (int k = 0; k < n; k++) {
        double qn = nx * q[1 + k];
        if (o->dim == 2) qn += ny * q[1 + n + k];
        a[k] = qn / h;
    }
    double s = 0.0;
    for (int j = 1; j < n; j++) s += fabs(a[j]);
    return fabs(a[0]) + sqrt(o->g * h + s * s);
}

/* friction source S(Q) (Sec. 3.4 closure: slip at the bed, Newtonian bulk) */
void oracle_source(const omesh *o, const double *q, double *out)
{
    int n = o->level + 1, nf = nfields(o);
    double h = q[0];
    for (int f = 0; f < nf; f++) out[f] = 0.0;
    int nblk = (o->dim == 2) ? 2 : 1;
    for (int d = 0; d < nblk; d++) {
        const double *qq = q + 1 + d * n;
        double al[OR_MAXN];
        for (int k = 0; k < n; k++) al[k] = qq[k] / h;
        double ub = 0.0;
        for (int j = 0; j < n; j++) ub += al[j] * o->phi0[j];
        for (int k = 0; k < n; k++) {
            double bulk = 0.0;
            for (int j = 0; j < n; j++) bulk += o->K[j * n + k] * al[j];
            out[1 + d * n + k] = -(o->c_slip * ub * o->phi0[k] + o->nu / h * bulk) / o->M[k];
        }
    }
}

/* Matrix L of the friction source of one moment block at depth h:
 * S_k(q) = sum_j L_kj q_j with q_j = h alpha_j, i.e.
 * L_kj = -(1/M_k) [ C phi_j(0) phi_k(0) / h + nu K_jk / h^2 ]  (Sec. 3.4 closure). */
static void source_matrix(const omesh *o, double h, double *L)
{
    int n = o->level + 1;
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            L[k * n + j] = -(o->c_slip * o->phi0[j] * o->phi0[k] / h + o->nu * o->K[j * n + k] / (h * h)) / o->M[k];
}

/* Solve A x = r (n x n, row-major, destroyed) by Gaussian elimination with
 * partial pivoting; x overwrites r. */
static void gauss_solve(int n, double *A, double *r)
{
    for (int c = 0; c < n; c++) {
        int piv = c;
        for (int i = c + 1; i < n; i++)
            if (fabs(A[i * n + c]) > fabs(A[piv * n + c])) piv = i;
        if (piv != c) {
            for (int j = 0; j < n; j++) {
                double t = A[c * n + j];
                A[c * n + j] = A[piv * n + j];
                A[piv * n + j] = t;
            }
            double t = r[c];
            r[c] = r[piv];
            r[piv] = t;
        }
        for (int i = c + 1; i < n; i++) {
            double f = A[i * n + c] / A[c * n + c];
            for (int j = c; j < n; j++) A[i * n + j] -= f * A[c * n + j];
            r[i] -= f * r[c];
        }
    }
    for (int c = n - 1; c >= 0; c--) {
        double v = r[c];
        for (int j = c + 1; j < n; j++) v -= A[c * n + j] * r[j];
        r[c] = v / A[c * n + c];
    }
}

/* The friction ODE dq/dt = S(q) over one step dt from the predicted state
 * qstar (h is not changed by S): forward Euler q* + dt S(q*), or backward
 * Euler q = q* + dt S(q) solved per moment block. */
void oracle_friction_step(const omesh *o, const double *qstar, double dt, double *out)
{
    int n = o->level + 1, nf = nfields(o);
    if (!o->implicit) {
        double src[OR_MAXF];
        oracle_source(o, qstar, src);
        for (int f = 0; f < nf; f++) out[f] = qstar[f] + dt * src[f];
        return;
    }
    double h = qstar[0];
    out[0] = h;
    int nblk = (o->dim == 2) ? 2 : 1;
    for (int d = 0; d < nblk; d++) {
        double L[OR_MAXN * OR_MAXN], A[OR_MAXN * OR_MAXN], r[OR_MAXN];
        source_matrix(o, h, L);
        for (int k = 0; k < n; k++) {
            for (int j = 0; j < n; j++) A[k * n + j] = (k == j ? 1.0 : 0.0) - dt * L[k * n + j];
            r[k] = qstar[1 + d * n + k];
        }
        gauss_solve(n, A, r);
        for (int k = 0; k < n; k++) out[1 + d * n + k] = r[k];
    }
}

/* state and bathymetry of cell i into a local vector */
static void load_cell(const omesh *o, const double *Q, int64_t i, double *q, double *b)
{
    int nf = nfields(o);
    for (int f = 0; f < nf; f++) q[f] = Q[(int64_t)f * o->ncells + i];
    *b = o->b[i];
}

/* ghost state for a boundary face */
static void ghost(const omesh *o, const double *qi, double bi, int64_t code, double nx, double ny,
                  double *qg, double *bg)
{
    int n = o->level + 1, nf = nfields(o);
    for (int f = 0; f < nf; f++) qg[f] = qi[f];
    *bg = bi;
    if (code == OR_WALL) {
        for (int k = 0; k < n; k++) {
            if (o->dim == 1) {
                qg[1 + k] = -qi[1 + k];
            } else {
                double qx = qi[1 + k], qy = qi[1 + n + k];
                double qn = qx * nx + qy * ny;
                qg[1 + k] = qx - 2.0 * qn * nx;
                qg[1 + n + k] = qy - 2.0 * qn * ny;
            }
        }
    }
}

/* Path-conservative NC fluctuation along the straight path from (qi, bi) to
 * (qj, bj): nc = int_0^1 B(Phi(s)).n ds (Q_j - Q_i, b_j - b_i), Gauss-Legendre in s. */
static void nc_path(const omesh *o, const double *qi, double bi, const double *qj, double bj, double nx, double ny,
                    double *nc_)
{
    int nf = nfields(o), nc = nf + 1;
    double dq[OR_MAXF + 1];
    for (int f = 0; f < nf; f++) dq[f] = qj[f] - qi[f];
    dq[nf] = bj - bi;
    for (int f = 0; f < nf; f++) nc_[f] = 0.0;
    double mat[OR_MAXF * (OR_MAXF + 1)];
    for (int g = 0; g < o->nquad; g++) {
        double qs[OR_MAXF];
        for (int f = 0; f < nf; f++) qs[f] = qi[f] + o->qs[g] * dq[f];
        oracle_ncmat(o, qs, nx, ny, mat);
        for (int r = 0; r < nf; r++) {
            double v = 0.0;
            for (int c = 0; c < nc; c++) v += mat[r * nc + c] * dq[c];
            nc_[r] += o->qw[g] * v;
        }
    }
}

/* Per-face contribution for cell i: |e| (Fhat + NC/2), accumulated into acc. */
static void face_term(const omesh *o, const double *qi, double bi, const double *qj, double bj,
                      double nx, double ny, double len, double *acc)
{
    int nf = nfields(o);
    double fi[OR_MAXF], fj[OR_MAXF];
    oracle_flux(o, qi, nx, ny, fi);
    oracle_flux(o, qj, nx, ny, fj);
    double li = oracle_lambda(o, qi, nx, ny);
    double lj = oracle_lambda(o, qj, nx, ny);
    double s = li > lj ? li : lj;
    double wi[OR_MAXF], wj[OR_MAXF];
    for (int f = 0; f < nf; f++) { wi[f] = qi[f]; wj[f] = qj[f]; }
    wi[0] += bi;            /* Rusanov viscosity acts on the free surface h + b */
    wj[0] += bj;
    double nc_[OR_MAXF];
    nc_path(o, qi, bi, qj, bj, nx, ny, nc_);
    for (int f = 0; f < nf; f++) {
        double fhat = 0.5 * (fi[f] + fj[f]) - 0.5 * s * (wj[f] - wi[f]);
        acc[f] += len * (fhat + 0.5 * nc_[f]);
    }
}

/* One time step for the cells idx[0..nidx) (or all cells if idx == NULL):
 * out[f * nidx + c] = Q^{n+1} of cell idx[c].  Hydrostatic predictor, then the
 * explicit friction step on the predicted state.                          */
void oracle_step_cells(const omesh *o, const double *Q, double dt, const int64_t *idx, int64_t nidx,
                       double *out)
{
    int nf = nfields(o);
    int64_t cnt = idx ? nidx : o->ncells;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < cnt; c++) {
        int64_t i = idx ? idx[c] : c;
        double qi[OR_MAXF], bi, qj[OR_MAXF], bj, acc[OR_MAXF];
        load_cell(o, Q, i, qi, &bi);
        for (int f = 0; f < nf; f++) acc[f] = 0.0;
        for (int s = 0; s < o->maxf; s++) {
            int64_t code = o->nbr[i * o->maxf + s];
            if (code < OR_EXTRAP) continue;
            double nx = o->fnx[i * o->maxf + s], ny = o->fny[i * o->maxf + s];
            double len = o->flen[i * o->maxf + s];
            if (code >= 0)
                load_cell(o, Q, code, qj, &bj);
            else
                ghost(o, qi, bi, code, nx, ny, qj, &bj);
            face_term(o, qi, bi, qj, bj, nx, ny, len, acc);
        }
        double qstar[OR_MAXF], qn[OR_MAXF];
        for (int f = 0; f < nf; f++) qstar[f] = qi[f] - dt / o->vol[i] * acc[f];
        oracle_friction_step(o, qstar, dt, qn);
        for (int f = 0; f < nf; f++) out[(int64_t)f * cnt + c] = qn[f];
    }
}

/* Only the hyperbolic predictor Q* (no friction), for the cells idx (or all). */
void oracle_predict_cells(const omesh *o, const double *Q, double dt, const int64_t *idx, int64_t nidx,
                          double *out)
{
    int nf = nfields(o);
    int64_t cnt = idx ? nidx : o->ncells;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < cnt; c++) {
        int64_t i = idx ? idx[c] : c;
        double qi[OR_MAXF], bi, qj[OR_MAXF], bj, acc[OR_MAXF];
        load_cell(o, Q, i, qi, &bi);
        for (int f = 0; f < nf; f++) acc[f] = 0.0;
        for (int s = 0; s < o->maxf; s++) {
            int64_t code = o->nbr[i * o->maxf + s];
            if (code < OR_EXTRAP) continue;
            double nx = o->fnx[i * o->maxf + s], ny = o->fny[i * o->maxf + s];
            double len = o->flen[i * o->maxf + s];
            if (code >= 0)
                load_cell(o, Q, code, qj, &bj);
            else
                ghost(o, qi, bi, code, nx, ny, qj, &bj);
            face_term(o, qi, bi, qj, bj, nx, ny, len, acc);
        }
        for (int f = 0; f < nf; f++) out[(int64_t)f * cnt + c] = qi[f] - dt / o->vol[i] * acc[f];
    }
}

/* CFL time step from the state Q; also returns max lam over all cells/faces. */
double oracle_cfl_dt(const omesh *o, const double *Q, double *lam_max)
{
    double rmax = 0.0, lmax = 0.0;
    int nf = nfields(o);
#pragma omp parallel for reduction(max : rmax, lmax)
    for (int64_t i = 0; i < o->ncells; i++) {
        double q[OR_MAXF];
        for (int f = 0; f < nf; f++) q[f] = Q[(int64_t)f * o->ncells + i];
        double sum = 0.0;
        for (int s = 0; s < o->maxf; s++) {
            if (o->nbr[i * o->maxf + s] < OR_EXTRAP) continue;
            double l = oracle_lambda(o, q, o->fnx[i * o->maxf + s], o->fny[i * o->maxf + s]);
            if (l > lmax) lmax = l;
            sum += o->flen[i * o->maxf + s] * l;
        }
        double r = sum / (2.0 * o->vol[i]);
        if (r > rmax) rmax = r;
    }
    if (lam_max) *lam_max = lmax;
    return o->cfl / rmax;
}

/* n_steps steps; dt_fixed > 0 uses that dt, else the CFL dt of each Q^n.
 * Q is updated in place (work holds one state); returns simulated time.    */
double oracle_run(const omesh *o, double *Q, double *work, int64_t n_steps, double dt_fixed)
{
    double t = 0.0;
    int nf = nfields(o);
    for (int64_t s = 0; s < n_steps; s++) {
        double dt = dt_fixed > 0.0 ? dt_fixed : oracle_cfl_dt(o, Q, NULL);
        oracle_step_cells(o, Q, dt, NULL, 0, work);
        memcpy(Q, work, sizeof(double) * (size_t)nf * (size_t)o->ncells);
        t += dt;
    }
    return t;
}

/* ------------------------------------------------------------------------ */
/* Second-order scheme on 1D and structured grids (face slot s lies on axis
 * s / 2, on its minus side for even s and its plus side for odd s).
 *
 * Reconstruction (compute_derivatives, Sec. 2.1.2, with a limiter): per cell
 * and axis the variables v = (eta = h + b, q_1 .. q_{nf-1}, b) get the slope
 * sigma = minmod(v_i - v_minus, v_plus - v_i) (per cell width; the neighbour
 * across a boundary face is the ghost of the cell), and the face values are
 * v_i -/+ sigma / 2, with h = eta - b.  Reconstructing the free surface keeps
 * the lake at rest exact.  If a face depth would not be positive the cell
 * keeps zero slopes (first order).
 * Semi-discrete operator: for every face the Rusanov flux and half the path
 * fluctuation between the two reconstructed face values (the cell's own and
 * the neighbour's, or its ghost), plus per axis the fluctuation inside the
 * cell along the straight path from its minus-face to its plus-face value
 * (the in-cell term of path-conservative schemes of second order).
 * Time: two-stage SSP Runge-Kutta (Heun) for the hyperbolic part, then the
 * friction step of the splitting (Eq. (3d)) on the result.                */

static double minmod(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}

/* state (q, b) of cell i -> reconstruction variables v[0..nf] */
static void to_recon(int nf, const double *q, double b, double *v)
{
    v[0] = q[0] + b;
    for (int f = 1; f < nf; f++) v[f] = q[f];
    v[nf] = b;
}

/* reconstruction variables -> (q, b) */
static void from_recon(int nf, const double *v, double *q, double *b)
{
    q[0] = v[0] - v[nf];
    for (int f = 1; f < nf; f++) q[f] = v[f];
    *b = v[nf];
}

/* limited slopes sig[cell][axis][nf + 1] */
static void recon_slopes(const omesh *o, const double *Q, double *sig)
{
    int nf = nfields(o), na = o->maxf / 2, nv = nf + 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < o->ncells; i++) {
        double qi[OR_MAXF], bi, vi[OR_MAXF + 1];
        load_cell(o, Q, i, qi, &bi);
        to_recon(nf, qi, bi, vi);
        double *si = sig + i * na * nv;
        for (int a = 0; a < na; a++) {
            double vn[2][OR_MAXF + 1];
            for (int side = 0; side < 2; side++) {
                int s = 2 * a + side;
                int64_t code = o->nbr[i * o->maxf + s];
                double qn[OR_MAXF], bn;
                if (code >= 0)
                    load_cell(o, Q, code, qn, &bn);
                else
                    ghost(o, qi, bi, code, o->fnx[i * o->maxf + s], o->fny[i * o->maxf + s], qn, &bn);
                to_recon(nf, qn, bn, vn[side]);
            }
            for (int f = 0; f < nv; f++) si[a * nv + f] = minmod(vi[f] - vn[0][f], vn[1][f] - vi[f]);
        }
        /* positive face depths, else first order */
        int ok = 1;
        for (int a = 0; a < na; a++)
            for (int side = 0; side < 2; side++) {
                double sg = side ? 0.5 : -0.5;
                double eta = vi[0] + sg * si[a * nv + 0], b = vi[nf] + sg * si[a * nv + nf];
                if (!(eta - b > 0.0)) ok = 0;
            }
        if (!ok)
            for (int f = 0; f < na * nv; f++) si[f] = 0.0;
    }
}

/* reconstructed (q, b) of cell i at its face slot s */
static void face_value(const omesh *o, const double *Q, const double *sig, int64_t i, int s, double *q, double *b)
{
    int nf = nfields(o), na = o->maxf / 2, nv = nf + 1;
    double qi[OR_MAXF], bi, v[OR_MAXF + 1];
    load_cell(o, Q, i, qi, &bi);
    to_recon(nf, qi, bi, v);
    const double *si = sig + (i * na + s / 2) * nv;
    double sg = (s % 2) ? 0.5 : -0.5;
    for (int f = 0; f < nv; f++) v[f] += sg * si[f];
    from_recon(nf, v, q, b);
}

/* R = dQ/dt of the hyperbolic part at second order (all cells) */
void oracle_rhs2(const omesh *o, const double *Q, double *R)
{
    int nf = nfields(o), na = o->maxf / 2;
    double *sig = (double *)malloc(sizeof(double) * (size_t)o->ncells * na * (nf + 1));
    recon_slopes(o, Q, sig);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < o->ncells; i++) {
        double acc[OR_MAXF];
        for (int f = 0; f < nf; f++) acc[f] = 0.0;
        for (int s = 0; s < o->maxf; s++) {
            int64_t code = o->nbr[i * o->maxf + s];
            double nx = o->fnx[i * o->maxf + s], ny = o->fny[i * o->maxf + s];
            double len = o->flen[i * o->maxf + s];
            double qL[OR_MAXF], bL, qR[OR_MAXF], bR;
            face_value(o, Q, sig, i, s, qL, &bL);
            if (code >= 0)
                face_value(o, Q, sig, code, s ^ 1, qR, &bR);   /* the neighbour's value on the same face */
            else
                ghost(o, qL, bL, code, nx, ny, qR, &bR);
            face_term(o, qL, bL, qR, bR, nx, ny, len, acc);
        }
        for (int a = 0; a < na; a++) {
            /* inside the cell, from the minus face to the plus face, normal +axis */
            double qm[OR_MAXF], bm, qp[OR_MAXF], bp, ncc[OR_MAXF];
            face_value(o, Q, sig, i, 2 * a, qm, &bm);
            face_value(o, Q, sig, i, 2 * a + 1, qp, &bp);
            double nx = o->fnx[i * o->maxf + 2 * a + 1], ny = o->fny[i * o->maxf + 2 * a + 1];
            double len = o->flen[i * o->maxf + 2 * a + 1];
            nc_path(o, qm, bm, qp, bp, nx, ny, ncc);
            for (int f = 0; f < nf; f++) acc[f] += len * ncc[f];
        }
        for (int f = 0; f < nf; f++) R[(int64_t)f * o->ncells + i] = -acc[f] / o->vol[i];
    }
    free(sig);
}

/* One second-order step of the whole mesh: out = Q^{n+1}. */
void oracle_step2(const omesh *o, const double *Q, double dt, double *out)
{
    int nf = nfields(o);
    size_t n = (size_t)nf * (size_t)o->ncells;
    double *R = (double *)malloc(sizeof(double) * n), *Q1 = (double *)malloc(sizeof(double) * n);
    oracle_rhs2(o, Q, R);
    for (size_t k = 0; k < n; k++) Q1[k] = Q[k] + dt * R[k];
    oracle_rhs2(o, Q1, R);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < o->ncells; i++) {
        double q2[OR_MAXF], qn[OR_MAXF];
        for (int f = 0; f < nf; f++) {
            size_t k = (size_t)f * o->ncells + i;
            q2[f] = 0.5 * Q[k] + 0.5 * (Q1[k] + dt * R[k]);
        }
        oracle_friction_step(o, q2, dt, qn);
        for (int f = 0; f < nf; f++) out[(size_t)f * o->ncells + i] = qn[f];
    }
    free(R);
    free(Q1);
}

/* n_steps second-order steps (dt_fixed > 0, else the CFL step of each Q^n);
 * Q in place, work holds one state; returns the simulated time. */
double oracle_run2(const omesh *o, double *Q, double *work, int64_t n_steps, double dt_fixed)
{
    double t = 0.0;
    int nf = nfields(o);
    for (int64_t s = 0; s < n_steps; s++) {
        double dt = dt_fixed > 0.0 ? dt_fixed : oracle_cfl_dt(o, Q, NULL);
        oracle_step2(o, Q, dt, work);
        memcpy(Q, work, sizeof(double) * (size_t)nf * (size_t)o->ncells);
        t += dt;
    }
    return t;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
