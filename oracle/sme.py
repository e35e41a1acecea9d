"""Python driver of the C oracle (``sme_oracle.c``).

Test infrastructure only (see ``oracle/__init__``).  Each call builds the
plain ``omesh`` description (mesh face slots, exact tensors rounded to FP64,
Gauss-Legendre nodes for the path integral) and calls the C routines.
"""
import ctypes
import os
import subprocess

import numpy as np

from . import tensors as _tensors

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sme_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=True):
    """Compile the oracle with gcc (strict FP64: no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        d, i64, p = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
        _lib.oracle_flux.argtypes = [p, p, d, d, p]
        _lib.oracle_ncmat.argtypes = [p, p, d, d, p]
        _lib.oracle_lambda.argtypes = [p, p, d, d]
        _lib.oracle_lambda.restype = d
        _lib.oracle_source.argtypes = [p, p, p]
        _lib.oracle_friction_step.argtypes = [p, p, d, p]
        _lib.oracle_rhs2.argtypes = [p, p, p]
        _lib.oracle_step2.argtypes = [p, p, d, p]
        _lib.oracle_run2.argtypes = [p, p, p, i64, d]
        _lib.oracle_run2.restype = d
        _lib.oracle_step_cells.argtypes = [p, p, d, p, i64, p]
        _lib.oracle_predict_cells.argtypes = [p, p, d, p, i64, p]
        _lib.oracle_cfl_dt.argtypes = [p, p, p]
        _lib.oracle_cfl_dt.restype = d
        _lib.oracle_run.argtypes = [p, p, p, i64, d]
        _lib.oracle_run.restype = d
        _lib.oracle_max_threads.restype = ctypes.c_int
    return _lib


class _OMesh(ctypes.Structure):
    _fields_ = [
        ("level", ctypes.c_int), ("dim", ctypes.c_int), ("ncells", ctypes.c_int64),
        ("maxf", ctypes.c_int),
        ("nbr", ctypes.c_void_p), ("fnx", ctypes.c_void_p), ("fny", ctypes.c_void_p),
        ("flen", ctypes.c_void_p), ("vol", ctypes.c_void_p), ("b", ctypes.c_void_p),
        ("g", ctypes.c_double), ("c_slip", ctypes.c_double), ("nu", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("nquad", ctypes.c_int), ("qs", ctypes.c_void_p), ("qw", ctypes.c_void_p),
        ("M", ctypes.c_void_p), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
        ("K", ctypes.c_void_p), ("phi0", ctypes.c_void_p), ("implicit", ctypes.c_int),
    ]


def gauss01(n):
    """Gauss-Legendre nodes/weights mapped from [-1, 1] to [0, 1] (weights sum to 1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def nfields(level, dim):
    return level + 2 if dim == 1 else 2 * level + 3


class Oracle:
    """SME oracle bound to one mesh, level and parameter set."""

    def __init__(self, level, mesh, b=None, g=9.81, c_slip=0.0, nu=0.0, cfl=0.45, quad_points=3,
                 implicit_friction=0, order=1):
        if order not in (1, 2):
            raise ValueError("order must be 1 or 2")
        if order == 2 and mesh.maxf != 2 * mesh.dim:
            raise ValueError("the second-order scheme needs a 1D or structured grid")
        self.order = order
        self.level = level
        self.mesh = mesh
        self.dim = mesh.dim
        self.nf = nfields(level, mesh.dim)
        t = _tensors.tensors(level)
        self._keep = {
            "M": np.ascontiguousarray(t["M"]),
            "A": np.ascontiguousarray(t["A"].reshape(-1)),
            "B": np.ascontiguousarray(t["B"].reshape(-1)),
            "K": np.ascontiguousarray(t["K"].reshape(-1)),
            "phi0": np.ascontiguousarray(t["phi0"]),
        }
        qs, qw = gauss01(quad_points)
        self._keep["qs"] = np.ascontiguousarray(qs)
        self._keep["qw"] = np.ascontiguousarray(qw)
        bb = np.zeros(mesh.ncells) if b is None else np.ascontiguousarray(b, dtype=np.float64)
        self._keep["b"] = bb
        self.b = bb
        self.params = dict(g=g, c_slip=c_slip, nu=nu, cfl=cfl, quad_points=quad_points,
                           implicit_friction=int(implicit_friction), order=order)
        k = self._keep
        self._o = _OMesh(level, mesh.dim, mesh.ncells, mesh.maxf,
                         _p(mesh.nbr), _p(mesh.nx), _p(mesh.ny), _p(mesh.flen), _p(mesh.vol),
                         _p(bb), g, c_slip, nu, cfl, quad_points, _p(k["qs"]), _p(k["qw"]),
                         _p(k["M"]), _p(k["A"]), _p(k["B"]), _p(k["K"]), _p(k["phi0"]),
                         int(implicit_friction))
        self._lib = lib()

    # --- pointwise pieces --------------------------------------------------
    def flux(self, q, nx, ny=0.0):
        q = np.ascontiguousarray(q, dtype=np.float64)
        out = np.zeros(self.nf)
        self._lib.oracle_flux(ctypes.byref(self._o), _p(q), nx, ny, _p(out))
        return out

    def ncmat(self, q, nx, ny=0.0):
        """B(Q).n as an nf x (nf+1) matrix; last column multiplies the bed."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        out = np.zeros((self.nf, self.nf + 1))
        self._lib.oracle_ncmat(ctypes.byref(self._o), _p(q), nx, ny, _p(out))
        return out

    def lam(self, q, nx, ny=0.0):
        q = np.ascontiguousarray(q, dtype=np.float64)
        return self._lib.oracle_lambda(ctypes.byref(self._o), _p(q), nx, ny)

    def source(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        out = np.zeros(self.nf)
        self._lib.oracle_source(ctypes.byref(self._o), _p(q), _p(out))
        return out

    def friction_step(self, qstar, dt):
        """The friction ODE over one step from the predicted state of one cell
        (explicit or implicit as the oracle was built)."""
        q = np.ascontiguousarray(qstar, dtype=np.float64)
        out = np.zeros(self.nf)
        self._lib.oracle_friction_step(ctypes.byref(self._o), _p(q), float(dt), _p(out))
        return out

    # --- whole-mesh operations --------------------------------------------
    def _state(self, Q):
        Q = np.ascontiguousarray(Q, dtype=np.float64)
        if Q.shape != (self.nf, self.mesh.ncells):
            raise ValueError(f"state must be ({self.nf}, {self.mesh.ncells})")
        return Q

    def cfl_dt(self, Q):
        Q = self._state(Q)
        lam = ctypes.c_double(0.0)
        dt = self._lib.oracle_cfl_dt(ctypes.byref(self._o), _p(Q), ctypes.byref(lam))
        return dt, lam.value

    def step(self, Q, dt=None, cells=None):
        """Q^{n+1} for all cells, or for the cell indices ``cells`` (shape (nf, len))."""
        Q = self._state(Q)
        if dt is None:
            dt = self.cfl_dt(Q)[0]
        if self.order == 2:
            out = np.empty_like(Q)
            self._lib.oracle_step2(ctypes.byref(self._o), _p(Q), dt, _p(out))
            return (out if cells is None else out[:, np.asarray(cells)]), dt
        if cells is None:
            out = np.empty_like(Q)
            self._lib.oracle_step_cells(ctypes.byref(self._o), _p(Q), dt, None, 0, _p(out))
        else:
            idx = np.ascontiguousarray(cells, dtype=np.int64)
            out = np.empty((self.nf, idx.size))
            self._lib.oracle_step_cells(ctypes.byref(self._o), _p(Q), dt, _p(idx), idx.size, _p(out))
        return out, dt

    def rhs2(self, Q):
        """dQ/dt of the second-order hyperbolic operator."""
        Q = self._state(Q)
        out = np.empty_like(Q)
        self._lib.oracle_rhs2(ctypes.byref(self._o), _p(Q), _p(out))
        return out

    def predict(self, Q, dt):
        """Hyperbolic predictor Q* only (no friction)."""
        Q = self._state(Q)
        out = np.empty_like(Q)
        self._lib.oracle_predict_cells(ctypes.byref(self._o), _p(Q), dt, None, 0, _p(out))
        return out

    def run(self, Q, n_steps, dt_fixed=0.0):
        """n_steps steps from Q; returns (Q_end, t_end)."""
        Q = self._state(Q).copy()
        work = np.empty_like(Q)
        run = self._lib.oracle_run2 if self.order == 2 else self._lib.oracle_run
        t = run(ctypes.byref(self._o), _p(Q), _p(work), int(n_steps), float(dt_fixed))
        return Q, t


def max_threads():
    return lib().oracle_max_threads()


def mesh_of(problem):
    """Oracle mesh for a workload description (dict from the workload generators)."""
    from . import mesh as _mesh

    k = problem["kind"]
    if k == "1d":
        return _mesh.mesh_1d(problem["nx"], problem["x0"], problem["x1"], problem["bc"][:2])
    if k == "2d":
        return _mesh.mesh_2d_struct(problem["nx"], problem["ny"], problem["x0"], problem["x1"],
                                    problem["y0"], problem["y1"], problem["bc"])
    if k == "tri":
        return _mesh.mesh_tri(problem["vert"], problem["tri"])
    raise ValueError(k)


def from_problem(problem, **overrides):
    p = dict(problem["params"])
    p.update(overrides)
    return Oracle(problem["level"], mesh_of(problem), problem["b"], **p)
