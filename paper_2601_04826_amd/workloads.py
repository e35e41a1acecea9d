"""Seeded synthetic workloads (inputs only; no SME arithmetic lives here).

Both the HIP library's tests/benchmarks and the CPU oracle take their inputs
from these generators, so every field below is *input*: meshes (vertices and
triangles), bathymetry and initial states in the caller's cell order, plus the
run settings.  Nothing here computes fluxes, sources or wave speeds.

Workloads (all FP64, numpy PCG64 seeds stated per generator):

dam_break_1d      1000 cells on [0, 10] m, level 1, h = 2 m for x < 5 else 1 m,
                  velocity moments 0, extrapolation ends, 1000 steps.
struct_2d         1024^2 periodic cells on [0, 10]^2 m, level 2; bathymetry = sum
                  of 16 Gaussians (amplitude U(0, 0.2) m, width U(0.2, 1) m,
                  periodic minimum-image distance, seed 0); depth 1 m plus a
                  0.5 m Gaussian hump (width 0.5 m) at a centre U[2, 8]^2 (seed 1);
                  200 steps.
tri_2d            Delaunay triangulation of 2,000,000 points U[0, 1]^2 (seed 2),
                  about 4.0 M triangles, level 3, reflective walls; bathymetry =
                  16 Gaussians (a ~ U(0, 0.2), sigma ~ U(0.02, 0.1), seed 3);
                  circular dam: depth 2 m inside r < 0.25 around (0.5, 0.5), 1 m
                  outside; 100 steps.
smooth_1d/2d      random smooth periodic fields (sums of low Fourier modes) at any
                  level: the training runs (1D, 4096 cells, seeds 1000..1255,
                  held out 1256..1287) and the 2D evaluation (2048^2, seed 2000)
                  of the learned closure.
batch             512 instances on [0, 1]^2, side U{64..512}, level U{1..4}, walls,
                  flat bed, dam centre U[0.25, 0.75]^2, radius U(0.05, 0.2), inner
                  depth U(1, 3) m, outer 1 m (seed 4); 500 steps.

Friction defaults (every workload except the frictionless Stoker check):
g = 9.81 m/s^2, slip coefficient C = nu / slip_length = 0.1 / 0.1 = 1.0 m/s,
nu = 0.1 m^2/s, CFL 0.45, 3 Gauss points on the path integral.
"""
import numpy as np

DEFAULT_PARAMS = dict(g=9.81, c_slip=1.0, nu=0.1, cfl=0.45, quad_points=3, implicit_friction=0, order=1)


def nfields(level, dim):
    return level + 2 if dim == 1 else 2 * level + 3


def _problem(kind, level, ncells, q, b, steps, params=None, **mesh):
    p = dict(DEFAULT_PARAMS)
    if params:
        p.update(params)
    d = dict(kind=kind, level=level, ncells=ncells, q=q, b=b, steps=steps, params=p)
    d.update(mesh)
    return d


# ---------------------------------------------------------------------------
def dam_break_1d(n=1000, level=1, hl=2.0, hr=1.0, steps=1000, bc=("extrap", "extrap"),
                 params=None, x0=0.0, x1=10.0):
    dx = (x1 - x0) / n
    xc = x0 + (np.arange(n) + 0.5) * dx
    q = np.zeros((nfields(level, 1), n))
    q[0] = np.where(xc < 0.5 * (x0 + x1), hl, hr)
    return _problem("1d", level, n, q, np.zeros(n), steps, params,
                    nx=n, ny=1, x0=x0, x1=x1, y0=0.0, y1=1.0, bc=tuple(bc) + ("periodic", "periodic"))


def smooth_1d(n=4096, level=8, seed=1000, steps=2000, L=10.0, params=None):
    """Random smooth periodic 1D state: depth, mean velocity and moments
    (training runs of the learned closure)."""
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) * (L / n)
    h = np.ones(n)
    u = np.zeros(n)
    for m in range(1, 5):
        h += rng.uniform(-0.3, 0.3) / m * np.sin(2 * np.pi * m * x / L + rng.uniform(0, 2 * np.pi))
        u += rng.uniform(-0.5, 0.5) / m * np.sin(2 * np.pi * m * x / L + rng.uniform(0, 2 * np.pi))
    q = np.zeros((nfields(level, 1), n))
    q[0] = h
    q[1] = h * u
    for j in range(1, level + 1):
        amp = rng.uniform(-0.3, 0.3) / j ** 2
        mode = rng.integers(1, 4)
        q[1 + j] = h * amp * (1.0 + np.sin(2 * np.pi * mode * x / L + rng.uniform(0, 2 * np.pi)))
    return _problem("1d", level, n, q, np.zeros(n), steps, params,
                    nx=n, ny=1, x0=0.0, x1=L, y0=0.0, y1=1.0, bc=("periodic",) * 4)


def smooth_2d(n=2048, level=8, seed=2000, steps=1000, L=10.0, params=None):
    """Random smooth periodic 2D state from the family of ``smooth_1d``: depth
    and both mean velocities are sums of four Fourier modes (wave number m along
    x or y, random phases), each moment j >= 1 a scaled random mode (evaluation
    of the learned closure)."""
    rng = np.random.default_rng(seed)
    d = L / n
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x = ((ii + 0.5) * d).ravel()
    y = ((jj + 0.5) * d).ravel()

    def mode(m, amp):
        # wave number m along x or along y (so each direction sees the 1D family)
        kx, ky = (m, 0) if rng.integers(0, 2) == 0 else (0, m)
        return amp * np.sin(2 * np.pi * (kx * x + ky * y) / L + rng.uniform(0, 2 * np.pi))

    h = np.ones(n * n)
    u = np.zeros(n * n)
    v = np.zeros(n * n)
    for m in range(1, 5):
        h += mode(m, rng.uniform(-0.3, 0.3) / m)
        u += mode(m, rng.uniform(-0.5, 0.5) / m)
        v += mode(m, rng.uniform(-0.5, 0.5) / m)
    k = level + 1
    q = np.zeros((nfields(level, 2), n * n))
    q[0] = h
    q[1] = h * u
    q[1 + k] = h * v
    for j in range(1, level + 1):
        q[1 + j] = h * rng.uniform(-0.3, 0.3) / j ** 2 * (1.0 + mode(rng.integers(1, 4), 1.0))
        q[1 + k + j] = h * rng.uniform(-0.3, 0.3) / j ** 2 * (1.0 + mode(rng.integers(1, 4), 1.0))
    return _problem("2d", level, n * n, q, np.zeros(n * n), steps, params,
                    nx=n, ny=n, x0=0.0, x1=L, y0=0.0, y1=L, bc=("periodic",) * 4)


def _periodic_gaussians(xc, yc, L, n, amp, sig, rng):
    b = np.zeros_like(xc)
    for _ in range(n):
        a = rng.uniform(*amp)
        s = rng.uniform(*sig)
        cx, cy = rng.uniform(0, L, size=2)
        dx = np.abs(xc - cx)
        dy = np.abs(yc - cy)
        dx = np.minimum(dx, L - dx)
        dy = np.minimum(dy, L - dy)
        b += a * np.exp(-(dx * dx + dy * dy) / (2 * s * s))
    return b


def struct_2d(n=1024, level=2, L=10.0, steps=200, seed_b=0, seed_h=1, params=None, bc=("periodic",) * 4):
    d = L / n
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    xc = ((ii + 0.5) * d).ravel()
    yc = ((jj + 0.5) * d).ravel()
    b = _periodic_gaussians(xc, yc, L, 16, (0.0, 0.2), (0.2, 1.0), np.random.default_rng(seed_b))
    rng = np.random.default_rng(seed_h)
    cx, cy = rng.uniform(2, 8, size=2) * (L / 10.0)
    dx = np.abs(xc - cx)
    dy = np.abs(yc - cy)
    dx = np.minimum(dx, L - dx)
    dy = np.minimum(dy, L - dy)
    q = np.zeros((nfields(level, 2), n * n))
    q[0] = 1.0 + 0.5 * np.exp(-(dx * dx + dy * dy) / (2 * 0.5 ** 2))
    return _problem("2d", level, n * n, q, b, steps, params,
                    nx=n, ny=n, x0=0.0, x1=L, y0=0.0, y1=L, bc=tuple(bc))


def random_state_2d(level, ncells, seed, h_range=(0.8, 1.5), vel=0.5, mom=0.3):
    """Unstructured random state (for parity at the level of single steps)."""
    rng = np.random.default_rng(seed)
    q = np.zeros((nfields(level, 2), ncells))
    h = rng.uniform(*h_range, size=ncells)
    q[0] = h
    n = level + 1
    for k in range(n):
        s = vel if k == 0 else mom / k
        q[1 + k] = h * rng.uniform(-s, s, size=ncells)
        q[1 + n + k] = h * rng.uniform(-s, s, size=ncells)
    return q


def delaunay_unit_square(npts, seed):
    """Delaunay triangulation of npts uniform points in [0,1]^2 plus the four
    corners; triangles returned counter-clockwise, int32."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    pts = np.concatenate([np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]]),
                          rng.uniform(0.0, 1.0, size=(npts, 2))])
    tri = Delaunay(pts).simplices.astype(np.int64)
    p = pts[tri]
    cross = ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
             - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    flip = cross < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    keep = cross != 0
    return pts, np.ascontiguousarray(tri[keep].astype(np.int32))


def tri_2d(npts=2_000_000, level=3, steps=100, seed_mesh=2, seed_b=3, params=None):
    vert, tri = delaunay_unit_square(npts, seed_mesh)
    c = vert[tri].mean(axis=1)
    rng = np.random.default_rng(seed_b)
    b = np.zeros(len(tri))
    for _ in range(16):
        a = rng.uniform(0.0, 0.2)
        s = rng.uniform(0.02, 0.1)
        cx, cy = rng.uniform(0, 1, size=2)
        b += a * np.exp(-((c[:, 0] - cx) ** 2 + (c[:, 1] - cy) ** 2) / (2 * s * s))
    q = np.zeros((nfields(level, 2), len(tri)))
    r = np.hypot(c[:, 0] - 0.5, c[:, 1] - 0.5)
    q[0] = np.where(r < 0.25, 2.0, 1.0)
    return _problem("tri", level, len(tri), q, b, steps, params, vert=vert, tri=tri,
                    bc=("wall",) * 4)


def batch(n_inst=512, seed=4, steps=500, side=(64, 512), levels=(1, 4), params=None):
    """List of independent struct-2D wall-bounded dam-break problems."""
    out = []
    for i in range(n_inst):
        rng = np.random.default_rng(seed + i)
        n = int(rng.integers(side[0], side[1] + 1))
        level = int(rng.integers(levels[0], levels[1] + 1))
        cx, cy = rng.uniform(0.25, 0.75, size=2)
        rad = rng.uniform(0.05, 0.2)
        hin = rng.uniform(1.0, 3.0)
        d = 1.0 / n
        jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        xc = ((ii + 0.5) * d).ravel()
        yc = ((jj + 0.5) * d).ravel()
        q = np.zeros((nfields(level, 2), n * n))
        q[0] = np.where(np.hypot(xc - cx, yc - cy) < rad, hin, 1.0)
        out.append(_problem("2d", level, n * n, q, np.zeros(n * n), steps, params,
                            nx=n, ny=n, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc=("wall",) * 4))
    return out

def vam_1d(n=2000, L=20.0, steps=200, seed=7, params=None, moments=True):
    """1D channel for the non-hydrostatic VAM step: a smoothed 0.3 m dam
    (undular bore) upstream of a 0.2 m Gaussian hump, still water level 1 m
    downstream, extrapolation ends; fields (h, h u0, h u1, h w0, h w1).  With
    `moments`, small seeded smooth profiles of u1, w0 and w1 are added so that
    every field of the step is active."""
    rng = np.random.default_rng(seed)
    dx = L / n
    x = (np.arange(n) + 0.5) * dx
    b = 0.2 * np.exp(-((x - 0.6 * L) / (0.05 * L)) ** 2)
    eta = 1.0 + 0.15 * (1.0 - np.tanh((x - 0.3 * L) / (0.01 * L)))
    h = eta - b
    q = np.zeros((5, n))
    q[0] = h
    q[1] = h * 0.2 * (1.0 - np.tanh((x - 0.3 * L) / (0.01 * L)))
    if moments:
        for f, amp in ((2, 0.05), (3, 0.02), (4, 0.02)):
            k = rng.integers(1, 4)
            q[f] = h * amp * rng.uniform(0.5, 1.0) * np.sin(2 * np.pi * k * x / L + rng.uniform(0, 2 * np.pi))
    p = dict(g=9.81, cfl=0.45, quad_points=3)
    if params:
        p.update(params)
    return dict(kind="vam", ncells=n, nx=n, x0=0.0, x1=L, q=q, b=b, steps=steps, params=p)
