"""Generic finite-volume meshes for the oracle (cell -> face slots).

Test infrastructure only (see ``oracle/__init__``).

Every mesh is reduced to the same plain description the oracle step loops over
(collocated finite volumes on 1D/2D grids, Sec. 2.1.2 of the paper):

    nbr[i, s]   neighbour cell across face slot s of cell i, or
                WALL (-1, reflective), EXTRAP (-2, copy), UNUSED (-3)
    nx, ny      outward unit normal of that face
    flen        face length (1 in 1D)
    vol[i]      cell volume (dx in 1D, area in 2D)

Boundary kinds follow the paper's generic conditions (Sec. 2.1.1): periodic
(a neighbour index wrapped around), extrapolation, plus a reflective wall.
"""
import numpy as np

WALL, EXTRAP, UNUSED = -1, -2, -3
PERIODIC = "periodic"
BC_CODES = {"wall": WALL, "extrap": EXTRAP}


class Mesh:
    def __init__(self, dim, nbr, nx, ny, flen, vol, centers):
        self.dim = dim
        self.nbr = np.ascontiguousarray(nbr, dtype=np.int64)
        self.nx = np.ascontiguousarray(nx, dtype=np.float64)
        self.ny = np.ascontiguousarray(ny, dtype=np.float64)
        self.flen = np.ascontiguousarray(flen, dtype=np.float64)
        self.vol = np.ascontiguousarray(vol, dtype=np.float64)
        self.centers = centers
        self.ncells, self.maxf = self.nbr.shape


def _bc_neighbor(kind, wrap_index):
    return wrap_index if kind == PERIODIC else BC_CODES[kind]


def mesh_1d(n, x0, x1, bc=("extrap", "extrap")):
    """Uniform 1D grid of n cells on [x0, x1]; face slot 0 = left, 1 = right."""
    dx = (x1 - x0) / n
    i = np.arange(n)
    nbr = np.stack([i - 1, i + 1], axis=1)
    nbr[0, 0] = _bc_neighbor(bc[0], n - 1)
    nbr[n - 1, 1] = _bc_neighbor(bc[1], 0)
    nx = np.tile([-1.0, 1.0], (n, 1))
    ny = np.zeros((n, 2))
    flen = np.ones((n, 2))
    vol = np.full(n, dx)
    centers = x0 + (i + 0.5) * dx
    return Mesh(1, nbr, nx, ny, flen, vol, centers)


def mesh_2d_struct(nxc, nyc, x0, x1, y0, y1, bc=("periodic",) * 4):
    """nxc x nyc cells, cell index j*nxc + i; slots W, E, S, N; bc = (W, E, S, N)."""
    dx = (x1 - x0) / nxc
    dy = (y1 - y0) / nyc
    jj, ii = np.meshgrid(np.arange(nyc), np.arange(nxc), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    cid = lambda a, b: b * nxc + a

    def edge(kind, wrap):
        return wrap if kind == PERIODIC else BC_CODES[kind]

    w = np.where(ii > 0, cid(ii - 1, jj), edge(bc[0], cid(nxc - 1, jj)))
    e = np.where(ii < nxc - 1, cid(ii + 1, jj), edge(bc[1], cid(0, jj)))
    s = np.where(jj > 0, cid(ii, jj - 1), edge(bc[2], cid(ii, nyc - 1)))
    nn = np.where(jj < nyc - 1, cid(ii, jj + 1), edge(bc[3], cid(ii, 0)))
    nbr = np.stack([w, e, s, nn], axis=1)
    ncell = nxc * nyc
    nx = np.tile([-1.0, 1.0, 0.0, 0.0], (ncell, 1))
    ny = np.tile([0.0, 0.0, -1.0, 1.0], (ncell, 1))
    flen = np.tile([dy, dy, dx, dx], (ncell, 1))
    vol = np.full(ncell, dx * dy)
    centers = np.stack([x0 + (ii + 0.5) * dx, y0 + (jj + 0.5) * dy], axis=1)
    return Mesh(2, nbr, nx, ny, flen, vol, centers)


def mesh_tri(vert, tri):
    """Triangle mesh (CCW triangles).  Face slot s is the edge from vertex s to
    vertex s+1; its outward normal is the edge vector turned clockwise.  An
    edge used by one triangle only is a reflective wall."""
    vert = np.asarray(vert, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    nt = tri.shape[0]
    p = vert[tri]                                  # (nt, 3, 2)
    area = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                  - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    if np.any(area <= 0):
        raise ValueError("triangles must be counter-clockwise and non-degenerate")
    a = p
    bnext = np.roll(p, -1, axis=1)
    ex = bnext[..., 0] - a[..., 0]
    ey = bnext[..., 1] - a[..., 1]
    flen = np.hypot(ex, ey)
    nx = ey / flen
    ny = -ex / flen
    # neighbours: match each edge with its reverse
    v0 = tri
    v1 = np.roll(tri, -1, axis=1)
    lo = np.minimum(v0, v1).ravel()
    hi = np.maximum(v0, v1).ravel()
    order = np.lexsort((hi, lo))
    lo_s, hi_s = lo[order], hi[order]
    nbr = np.full(3 * nt, WALL, dtype=np.int64)
    same = (lo_s[1:] == lo_s[:-1]) & (hi_s[1:] == hi_s[:-1])
    k = np.nonzero(same)[0]
    if np.any(same[1:] & same[:-1]):
        raise ValueError("non-manifold edge")
    e1, e2 = order[k], order[k + 1]
    nbr[e1] = e2 // 3
    nbr[e2] = e1 // 3
    centers = p.mean(axis=1)
    return Mesh(2, nbr.reshape(nt, 3), nx, ny, flen, area, centers)
