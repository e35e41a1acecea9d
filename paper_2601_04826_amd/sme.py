"""Python binding of the SME HIP library (``libsme.so``, C ABI in include/sme.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  The functions carry the C names.  Device buffers may be torch CUDA
tensors (torch provides device memory and streams); host buffers are numpy
arrays.  ``torch`` is imported before the library is loaded so that both use the
one HIP runtime torch ships with.

If ``libsme.so`` has not been built, importing this module raises ImportError:
there is no fallback path.
"""
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (must precede loading libsme.so: one HIP runtime per process)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsme.so")

SME_OK, SME_EINVAL, SME_ENOMEM, SME_EHIP, SME_ENONPHYS, SME_EMESH = 0, -1, -2, -3, -4, -5
SME_MESH_1D, SME_MESH_2D_STRUCT, SME_MESH_2D_TRI = 1, 2, 3
SME_BC_PERIODIC, SME_BC_EXTRAP, SME_BC_WALL = 0, 1, 2
BC = {"periodic": SME_BC_PERIODIC, "extrap": SME_BC_EXTRAP, "wall": SME_BC_WALL}
MAX_LEVEL = 8
CLOSURE_PRECISIONS = {"fp32": 0, "fp16": 1}  # SME_CLOSURE_FP32, SME_CLOSURE_FP16_MFMA

EXPORTS = [
    "sme_layout", "sme_workspace_size", "sme_init", "sme_set_state", "sme_get_state", "sme_eigmax", "sme_step",
    "sme_run", "sme_time", "sme_interpolate_3d", "sme_current", "sme_nfields", "sme_ncells", "sme_level", "sme_state_device",
    "sme_field_stride", "sme_step_static",
    "sme_basis_tensors", "sme_strerror", "sme_last_error", "sme_destroy",
    "sme_batch_init", "sme_batch_set_state", "sme_batch_get_state", "sme_batch_run", "sme_batch_time",
    "sme_batch_cells", "sme_batch_rows", "sme_batch_set_rows", "sme_batch_autotune",
    "sme_batch_last_error", "sme_batch_destroy",
    "sme_mlp_create", "sme_mlp_init", "sme_mlp_set_params", "sme_mlp_get_params", "sme_mlp_set_scaling", "sme_mlp_fit_scaling",
    "sme_mlp_get_scaling", "sme_mlp_forward",
    "sme_mlp_loss_grad", "sme_mlp_train_step", "sme_mlp_reset_optimizer", "sme_mlp_last_error", "sme_mlp_destroy",
    "sme_closure_samples", "sme_closure_attach", "sme_closure_attach_ex", "sme_closure_out_of_range",
    "sme_closure_train", "sme_closure_run",
    "sme_vam_layout", "sme_vam_workspace_size", "sme_vam_init", "sme_vam_set_state", "sme_vam_get_state",
    "sme_vam_pressure", "sme_vam_step", "sme_vam_run", "sme_vam_time", "sme_vam_current", "sme_vam_field_stride",
    "sme_vam_last_error", "sme_vam_destroy",
]


class sme_params(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("c_slip", ctypes.c_double), ("nu", ctypes.c_double),
                ("cfl", ctypes.c_double), ("quad_points", ctypes.c_int), ("implicit_friction", ctypes.c_int),
                ("order", ctypes.c_int)]


class sme_mesh(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double), ("bc", ctypes.c_int * 4), ("n_vert", ctypes.c_int64),
                ("n_tri", ctypes.c_int64), ("vert_xy", ctypes.c_void_p), ("tri", ctypes.c_void_p)]


class SmeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2601_04826_amd.build.build() "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, d, i = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "sme_layout": (i, [i, vp, P(i), P(i64), P(i64)]),
        "sme_workspace_size": (i, [i, vp, vp, P(ctypes.c_size_t)]),
        "sme_init": (i, [P(vp), i, vp, vp, P(vp), vp, i, vp]),
        "sme_set_state": (i, [vp, vp, i]),
        "sme_get_state": (i, [vp, vp, i]),
        "sme_eigmax": (i, [vp, P(d), P(d)]),
        "sme_step": (i, [vp, d, P(d)]),
        "sme_run": (i, [vp, i64, d, P(d), P(i64)]),
        "sme_time": (i, [vp, P(d), P(i64)]),
        "sme_current": (i, [vp]),
        "sme_interpolate_3d": (i, [vp, i, vp, d, vp]),
        "sme_nfields": (i, [vp]),
        "sme_ncells": (i64, [vp]),
        "sme_level": (i, [vp]),
        "sme_state_device": (vp, [vp]),
        "sme_field_stride": (i64, [vp]),
        "sme_step_static": (i, [i, vp, vp, vp, vp, i64, vp, d, P(d), vp]),
        "sme_basis_tensors": (i, [i, vp, vp, vp, vp]),
        "sme_strerror": (ctypes.c_char_p, [i]),
        "sme_last_error": (ctypes.c_char_p, [vp]),
        "sme_destroy": (None, [vp]),
        "sme_batch_init": (i, [P(vp), i, vp, vp, vp, vp, vp]),
        "sme_batch_set_state": (i, [vp, i, vp, i]),
        "sme_batch_get_state": (i, [vp, i, vp, i]),
        "sme_batch_run": (i, [vp, i64]),
        "sme_batch_time": (i, [vp, i, P(d), P(i64)]),
        "sme_batch_cells": (i64, [vp]),
        "sme_batch_rows": (i, [vp, i]),
        "sme_batch_set_rows": (i, [vp, i, i]),
        "sme_batch_autotune": (i, [vp, ctypes.c_char_p]),
        "sme_batch_last_error": (ctypes.c_char_p, [vp]),
        "sme_batch_destroy": (None, [vp]),
        "sme_mlp_create": (i, [P(vp), vp]),
        "sme_mlp_init": (i, [vp, ctypes.c_uint64]),
        "sme_mlp_set_params": (i, [vp, vp, i]),
        "sme_mlp_get_params": (i, [vp, vp, i]),
        "sme_mlp_set_scaling": (i, [vp, vp, vp, vp, vp, vp]),
        "sme_mlp_forward": (i, [vp, vp, i64, vp]),
        "sme_mlp_fit_scaling": (i, [vp, vp, vp, i64, d]),
        "sme_mlp_get_scaling": (i, [vp, vp, vp, vp, vp, vp]),
        "sme_mlp_loss_grad": (i, [vp, vp, vp, vp, i64, vp, vp]),
        "sme_mlp_train_step": (i, [vp, vp, vp, vp, i64, ctypes.c_float, vp]),
        "sme_mlp_reset_optimizer": (i, [vp]),
        "sme_mlp_last_error": (ctypes.c_char_p, [vp]),
        "sme_mlp_destroy": (None, [vp]),
        "sme_closure_samples": (i, [vp, i64, vp, i64, vp, i64, i64, d, vp, i64, vp, vp, vp]),
        "sme_closure_attach": (i, [vp, vp]),
        "sme_closure_attach_ex": (i, [vp, vp, i]),
        "sme_closure_out_of_range": (i, [vp, P(i64)]),
        "sme_closure_train": (i, [vp, vp, vp, i64, i, i64, ctypes.c_float, ctypes.c_float, ctypes.c_uint64, d, vp]),
        "sme_closure_run": (i, [vp, vp, d, i64, i64, d, P(d), P(i64), P(d)]),
        "sme_vam_layout": (i, [i64, P(i64)]),
        "sme_vam_workspace_size": (i, [i64, P(ctypes.c_size_t)]),
        "sme_vam_init": (i, [P(vp), i64, d, d, d, d, i, P(vp), vp, i, vp]),
        "sme_vam_set_state": (i, [vp, vp, i]),
        "sme_vam_get_state": (i, [vp, vp, i]),
        "sme_vam_pressure": (i, [vp, vp, i]),
        "sme_vam_step": (i, [vp, d, P(d)]),
        "sme_vam_run": (i, [vp, i64, d, P(d), P(i64)]),
        "sme_vam_time": (i, [vp, P(d), P(i64)]),
        "sme_vam_current": (i, [vp]),
        "sme_vam_field_stride": (i64, [vp]),
        "sme_vam_last_error": (ctypes.c_char_p, [vp]),
        "sme_vam_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def _check(code, ctx=None):
    if code != SME_OK:
        msg = _lib.sme_strerror(code).decode()
        if ctx:
            detail = _lib.sme_last_error(ctx).decode()
            if detail:
                msg = f"{msg}: {detail}"
        raise SmeError(code, msg)


def _ptr(a):
    if isinstance(a, torch.Tensor):
        return ctypes.c_void_p(a.data_ptr()), bool(a.is_cuda)
    return a.ctypes.data_as(ctypes.c_void_p), False


def make_params(g=9.81, c_slip=0.0, nu=0.0, cfl=0.45, quad_points=3, implicit_friction=0, order=1):
    return sme_params(g, c_slip, nu, cfl, quad_points, int(implicit_friction), int(order))


def make_mesh(problem):
    """sme_mesh for a workload description (see ``workloads``); returns (mesh, keepalive)."""
    m = sme_mesh()
    k = problem["kind"]
    keep = []
    if k in ("1d", "2d"):
        m.kind = SME_MESH_1D if k == "1d" else SME_MESH_2D_STRUCT
        m.nx, m.ny = problem["nx"], problem.get("ny", 1)
        m.x0, m.x1 = problem["x0"], problem["x1"]
        m.y0, m.y1 = problem.get("y0", 0.0), problem.get("y1", 1.0)
        bc = list(problem["bc"]) + ["periodic"] * (4 - len(problem["bc"]))
        for s in range(4):
            m.bc[s] = BC[bc[s]]
    elif k == "tri":
        vert = np.ascontiguousarray(problem["vert"], dtype=np.float64)
        tri = np.ascontiguousarray(problem["tri"], dtype=np.int32)
        keep = [vert, tri]
        m.kind = SME_MESH_2D_TRI
        m.n_vert, m.n_tri = vert.shape[0], tri.shape[0]
        m.vert_xy = vert.ctypes.data_as(ctypes.c_void_p)
        m.tri = tri.ctypes.data_as(ctypes.c_void_p)
    else:
        raise ValueError(k)
    return m, keep


def sme_layout(level, mesh):
    """(nfields, ncells, field_stride) of a level on a mesh."""
    nf, nc, st = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.sme_layout(level, ctypes.byref(mesh), ctypes.byref(nf), ctypes.byref(nc), ctypes.byref(st)))
    return nf.value, nc.value, st.value


def sme_workspace_size(level, mesh, params=None):
    n = ctypes.c_size_t()
    _check(_lib.sme_workspace_size(level, ctypes.byref(mesh), ctypes.byref(params) if params is not None else None,
                                   ctypes.byref(n)))
    return n.value


def state_buffers(level, mesh, device=None):
    """Two caller-owned device buffers [nfields, field_stride] (float64) for sme_init."""
    nf, _, st = sme_layout(level, mesh)
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    return [torch.empty((nf, st), dtype=torch.float64, device=dev) for _ in range(2)]


def sme_init(level, mesh, params, q_dev, b=None, stream=None):
    """Context bound to the two device buffers q_dev (torch CUDA tensors)."""
    if len(q_dev) != 2 or not all(isinstance(x, torch.Tensor) and x.is_cuda for x in q_dev):
        raise TypeError("q_dev must be two torch CUDA tensors")
    qp = (ctypes.c_void_p * 2)(q_dev[0].data_ptr(), q_dev[1].data_ptr())
    ctx = ctypes.c_void_p()
    if b is not None:
        if not isinstance(b, torch.Tensor):
            b = np.ascontiguousarray(b, dtype=np.float64)
        bp, bdev = _ptr(b)
    else:
        bp, bdev = None, False
    if stream is None and torch.cuda.is_available():
        stream = torch.cuda.current_stream().cuda_stream
    code = _lib.sme_init(ctypes.byref(ctx), level, ctypes.byref(mesh), ctypes.byref(params), qp, bp,
                         int(bdev), ctypes.c_void_p(stream or 0))
    _check(code)
    return ctx


def sme_set_state(ctx, q):
    if isinstance(q, torch.Tensor):
        q = q.contiguous()
        if q.dtype != torch.float64:
            raise TypeError("state must be float64")
    else:
        q = np.ascontiguousarray(q, dtype=np.float64)
    p, dev = _ptr(q)
    _check(_lib.sme_set_state(ctx, p, int(dev)), ctx)


def sme_get_state(ctx, out=None):
    nf, nc = _lib.sme_nfields(ctx), _lib.sme_ncells(ctx)
    if out is None:
        out = np.empty((nf, nc))
    p, dev = _ptr(out)
    _check(_lib.sme_get_state(ctx, p, int(dev)), ctx)
    return out


def sme_eigmax(ctx):
    lam, dt = ctypes.c_double(), ctypes.c_double()
    _check(_lib.sme_eigmax(ctx, ctypes.byref(lam), ctypes.byref(dt)), ctx)
    return lam.value, dt.value


def sme_step(ctx, dt=0.0, sync=False):
    used = ctypes.c_double()
    _check(_lib.sme_step(ctx, float(dt), ctypes.byref(used) if sync else None), ctx)
    return used.value if sync else None


def sme_run(ctx, n_steps, t_end=0.0, sync=True):
    t, s = ctypes.c_double(), ctypes.c_int64()
    if sync:
        _check(_lib.sme_run(ctx, int(n_steps), float(t_end), ctypes.byref(t), ctypes.byref(s)), ctx)
        return t.value, s.value
    _check(_lib.sme_run(ctx, int(n_steps), float(t_end), None, None), ctx)
    return None


def sme_time(ctx):
    t, s = ctypes.c_double(), ctypes.c_int64()
    _check(_lib.sme_time(ctx, ctypes.byref(t), ctypes.byref(s)), ctx)
    return t.value, s.value


def sme_destroy(ctx):
    _lib.sme_destroy(ctx)


def sme_step_static(level, mesh, params, q, q_next, b, dt=0.0, stream=None):
    """One step from q to q_next (torch CUDA float64 [nfields, field_stride]) over
    b (torch CUDA float64, 256-byte aligned) with no allocation; returns dt."""
    for x in (q, q_next, b):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
            raise TypeError("q, q_next and b must be contiguous float64 CUDA tensors")
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    used = ctypes.c_double()
    _check(_lib.sme_step_static(level, ctypes.byref(mesh), ctypes.byref(params), ctypes.c_void_p(q.data_ptr()),
                                ctypes.c_void_p(q_next.data_ptr()), q.shape[1], ctypes.c_void_p(b.data_ptr()),
                                float(dt), ctypes.byref(used), ctypes.c_void_p(stream or 0)))
    return used.value


def sme_basis_tensors(level):
    n = level + 1
    M, A, B, K = np.zeros(n), np.zeros(n ** 3), np.zeros(n ** 3), np.zeros(n * n)
    _check(_lib.sme_basis_tensors(level, *(x.ctypes.data_as(ctypes.c_void_p) for x in (M, A, B, K))))
    return {"M": M, "A": A.reshape(n, n, n), "B": B.reshape(n, n, n), "K": K.reshape(n, n)}


class Solver:
    """One SME context: ``Solver(problem)`` builds it from a workload description."""

    def __init__(self, problem, stream=None, **param_overrides):
        p = dict(problem["params"])
        p.update(param_overrides)
        self.problem = problem
        self.level = problem["level"]
        self.params = make_params(**p)
        self.mesh, keep = make_mesh(problem)
        self.ctx = None
        # the state buffers belong to this object (torch memory), bound to the context
        self.q_dev = state_buffers(self.level, self.mesh)
        self.ctx = sme_init(self.level, self.mesh, self.params, self.q_dev, problem.get("b"), stream)
        del keep
        self.nf = _lib.sme_nfields(self.ctx)
        self.ncells = _lib.sme_ncells(self.ctx)

    def set_state(self, q):
        sme_set_state(self.ctx, q)

    def get_state(self, out=None):
        return sme_get_state(self.ctx, out)

    def eigmax(self):
        return sme_eigmax(self.ctx)

    def step(self, dt=0.0, sync=False):
        return sme_step(self.ctx, dt, sync)

    def run(self, n_steps, t_end=0.0, sync=True):
        return sme_run(self.ctx, n_steps, t_end, sync)

    def time(self):
        return sme_time(self.ctx)

    def attach_closure(self, mlp, precision="fp32"):
        """Attach a trained network (an MLP); None detaches.  precision "fp32"
        (FP32 network) or "fp16" (matrix cores, FP16 operands, FP32 accumulation)."""
        mode = CLOSURE_PRECISIONS[precision]
        rc = _lib.sme_closure_attach_ex(self.ctx, mlp.ctx if mlp is not None else None, mode)
        if rc != 0 and mlp is not None and mlp.ctx:
            msg = (_lib.sme_mlp_last_error(mlp.ctx) or b"").decode()
            if msg:
                raise SmeError(rc, msg)
        _check(rc, self.ctx)

    def out_of_range(self):
        n = ctypes.c_int64()
        _check(_lib.sme_closure_out_of_range(self.ctx, ctypes.byref(n)), self.ctx)
        return n.value

    def state_device(self):
        """(pointer, field stride) of the current state in the internal order."""
        return _lib.sme_state_device(self.ctx), _lib.sme_field_stride(self.ctx)

    def interpolate_3d(self, zeta, rho=1.0):
        """3D lifting of the current state at sigma levels zeta: dict of z, u,
        v, w, p as numpy arrays [len(zeta), ncells] (caller cell order)."""
        z = np.ascontiguousarray(zeta, dtype=np.float64)
        out = torch.empty((5, z.size, self.ncells), dtype=torch.float64, device=self.q_dev[0].device)
        _check(_lib.sme_interpolate_3d(self.ctx, int(z.size), z.ctypes.data_as(ctypes.c_void_p), float(rho),
                                       ctypes.c_void_p(out.data_ptr())), self.ctx)
        o = out.cpu().numpy()
        return dict(z=o[0], u=o[1], v=o[2], w=o[3], p=o[4])

    def interpolate_3d_into(self, zeta, out, rho=1.0):
        """The same lifting into a caller tensor out (torch CUDA float64,
        contiguous, [5, len(zeta), ncells]), queued on the solver's stream."""
        z = np.ascontiguousarray(zeta, dtype=np.float64)
        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64 and out.is_contiguous()
                and tuple(out.shape) == (5, z.size, self.ncells)):
            raise TypeError("out must be a contiguous float64 CUDA tensor [5, len(zeta), ncells]")
        _check(_lib.sme_interpolate_3d(self.ctx, int(z.size), z.ctypes.data_as(ctypes.c_void_p), float(rho),
                                       ctypes.c_void_p(out.data_ptr())), self.ctx)

    def current(self):
        """The bound buffer (torch tensor [nfields, field_stride]) holding the state."""
        return self.q_dev[_lib.sme_current(self.ctx)]

    def close(self):
        if self.ctx:
            sme_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _bcheck(code, bt):
    if code != SME_OK:
        msg = _lib.sme_strerror(code).decode()
        detail = _lib.sme_batch_last_error(bt).decode() if bt else ""
        raise SmeError(code, f"{msg}: {detail}" if detail else msg)


class Batch:
    """Batched ensemble of structured grids (levels 0..4) advanced together by
    one persistent launch per step, each grid with its own CFL step."""

    def __init__(self, problems, stream=None, **param_overrides):
        p = dict(problems[0]["params"])
        p.update(param_overrides)
        self.params = make_params(**p)
        n = len(problems)
        self.n = n
        meshes = (sme_mesh * n)()
        for k, pr in enumerate(problems):
            if pr["kind"] != "2d":
                raise ValueError("batched grids must be structured 2D")
            m, _ = make_mesh(pr)
            meshes[k] = m
        levels = (ctypes.c_int * n)(*[pr["level"] for pr in problems])
        self._b = [np.ascontiguousarray(pr["b"], dtype=np.float64) if pr.get("b") is not None else None
                   for pr in problems]
        bptr = (ctypes.c_void_p * n)(*[x.ctypes.data if x is not None else None for x in self._b])
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream().cuda_stream
        self.ctx = ctypes.c_void_p()
        _bcheck(_lib.sme_batch_init(ctypes.byref(self.ctx), n, levels, meshes, bptr, ctypes.byref(self.params),
                                    ctypes.c_void_p(stream or 0)), None)
        self.shapes = [(pr["q"].shape[0], pr["ncells"]) for pr in problems]
        self.cells = _lib.sme_batch_cells(self.ctx)

    def set_state(self, i, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        if q.shape != self.shapes[i]:
            raise ValueError(f"grid {i} state must have shape {self.shapes[i]}")
        _bcheck(_lib.sme_batch_set_state(self.ctx, i, q.ctypes.data_as(ctypes.c_void_p), 0), self.ctx)

    def get_state(self, i):
        out = np.empty(self.shapes[i])
        _bcheck(_lib.sme_batch_get_state(self.ctx, i, out.ctypes.data_as(ctypes.c_void_p), 0), self.ctx)
        return out

    def run(self, n_steps):
        _bcheck(_lib.sme_batch_run(self.ctx, int(n_steps)), self.ctx)

    def time(self, i):
        t, s = ctypes.c_double(), ctypes.c_int64()
        _bcheck(_lib.sme_batch_time(self.ctx, i, ctypes.byref(t), ctypes.byref(s)), self.ctx)
        return t.value, s.value

    def rows(self, level):
        return _lib.sme_batch_rows(self.ctx, level)

    def set_rows(self, level, rows):
        _bcheck(_lib.sme_batch_set_rows(self.ctx, level, rows), self.ctx)

    def autotune(self, cache_path=None):
        _bcheck(_lib.sme_batch_autotune(self.ctx, cache_path.encode() if cache_path else None), self.ctx)

    def close(self):
        if self.ctx:
            _lib.sme_batch_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NPARAM = 4930


def _mcheck(code, m):
    if code != SME_OK:
        msg = _lib.sme_strerror(code).decode()
        detail = _lib.sme_mlp_last_error(m).decode() if m else ""
        raise SmeError(code, f"{msg}: {detail}" if detail else msg)


def _fptr(a, dtype=np.float32):
    """(pointer, keepalive) of a torch CUDA tensor or a host numpy array."""
    if isinstance(a, torch.Tensor):
        return ctypes.c_void_p(a.data_ptr()), a
    a = np.ascontiguousarray(a, dtype=dtype)
    return a.ctypes.data_as(ctypes.c_void_p), a


class MLP:
    """The closure network (9 -> 64 -> 64 -> 2, tanh, FP32) on the device."""

    def __init__(self, params=None, stream=None):
        if stream is None and torch.cuda.is_available():
            stream = torch.cuda.current_stream().cuda_stream
        self.ctx = ctypes.c_void_p()
        _mcheck(_lib.sme_mlp_create(ctypes.byref(self.ctx), ctypes.c_void_p(stream or 0)), None)
        if params is not None:
            self.set_params(params)

    def init(self, seed):
        """Glorot-uniform weights from a seeded stream, zero biases (library call)."""
        _mcheck(_lib.sme_mlp_init(self.ctx, int(seed)), self.ctx)

    def train(self, feat, targ, epochs, batch, lr, lr_end, seed, margin=0.1):
        """sme_closure_train on raw samples (CUDA float32 [n, 9], [n, 2]);
        returns the last-batch loss of every epoch."""
        hist = np.zeros(epochs, dtype=np.float32)
        _mcheck(_lib.sme_closure_train(self.ctx, ctypes.c_void_p(feat.data_ptr()), ctypes.c_void_p(targ.data_ptr()),
                                       feat.shape[0], int(epochs), int(batch), ctypes.c_float(lr),
                                       ctypes.c_float(lr_end), int(seed), float(margin),
                                       hist.ctypes.data_as(ctypes.c_void_p)), self.ctx)
        return [float(x) for x in hist]

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == NPARAM
        _mcheck(_lib.sme_mlp_set_params(self.ctx, p.ctypes.data_as(ctypes.c_void_p), 0), self.ctx)

    def get_params(self):
        p = np.empty(NPARAM, dtype=np.float32)
        _mcheck(_lib.sme_mlp_get_params(self.ctx, p.ctypes.data_as(ctypes.c_void_p), 0), self.ctx)
        return p

    def set_scaling(self, mu, sigma, out_scale, box_lo, box_hi):
        a = [np.ascontiguousarray(v, dtype=np.float32) for v in (mu, sigma, out_scale)]
        b = [np.ascontiguousarray(v, dtype=np.float64) for v in (box_lo, box_hi)]
        _mcheck(_lib.sme_mlp_set_scaling(self.ctx, *(x.ctypes.data_as(ctypes.c_void_p) for x in a + b)), self.ctx)

    def fit_scaling(self, feat, targ, margin=0.1):
        """Scaling and training box from raw samples (CUDA float32 [n, 9], [n, 2])."""
        _mcheck(_lib.sme_mlp_fit_scaling(self.ctx, ctypes.c_void_p(feat.data_ptr()), ctypes.c_void_p(targ.data_ptr()),
                                         feat.shape[0], float(margin)), self.ctx)
        return self.get_scaling()

    def get_scaling(self):
        """dict of mu, sigma, out_scale (float32) and box_lo, box_hi (float64)."""
        out = dict(mu=np.empty(9, np.float32), sigma=np.empty(9, np.float32), out_scale=np.empty(2, np.float32),
                   box_lo=np.empty(9), box_hi=np.empty(9))
        _mcheck(_lib.sme_mlp_get_scaling(self.ctx, *(out[k].ctypes.data_as(ctypes.c_void_p)
                                                     for k in ("mu", "sigma", "out_scale", "box_lo", "box_hi"))),
                self.ctx)
        return out

    def forward(self, x):
        """x: torch CUDA float32 [B, 9] raw features -> normalised outputs [B, 2]."""
        y = torch.empty((x.shape[0], 2), dtype=torch.float32, device=x.device)
        _mcheck(_lib.sme_mlp_forward(self.ctx, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                     ctypes.c_void_p(y.data_ptr())), self.ctx)
        return y

    @staticmethod
    def _rows(x, idx):
        if idx is None:
            return None, x.shape[0]
        assert idx.dtype == torch.int64 and idx.is_cuda and idx.is_contiguous()
        return ctypes.c_void_p(idx.data_ptr()), idx.shape[0]

    def loss_grad(self, x, t, idx=None):
        """Loss and gradient on rows idx (CUDA int64; None: all rows) of raw samples x, t."""
        g = torch.empty(NPARAM, dtype=torch.float32, device=x.device)
        loss = ctypes.c_float()
        ip, nb = self._rows(x, idx)
        _mcheck(_lib.sme_mlp_loss_grad(self.ctx, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()), ip,
                                       nb, ctypes.byref(loss), ctypes.c_void_p(g.data_ptr())), self.ctx)
        return loss.value, g

    def train_step(self, x, t, lr, idx=None, want_loss=False):
        loss = ctypes.c_float()
        ip, nb = self._rows(x, idx)
        _mcheck(_lib.sme_mlp_train_step(self.ctx, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()), ip,
                                        nb, ctypes.c_float(lr), ctypes.byref(loss) if want_loss else None), self.ctx)
        return loss.value if want_loss else None

    def reset_optimizer(self):
        _mcheck(_lib.sme_mlp_reset_optimizer(self.ctx), self.ctx)

    def close(self):
        if self.ctx:
            _lib.sme_mlp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def closure_samples(q8, q8_next, q1_step, dt, cells, stream=None, out=None):
    """Training samples (features [S, 9], targets [S, 2], FP32 torch CUDA) from
    torch CUDA float64 states [nf, n] of a periodic 1D row; out = (feat, targ)
    writes them into given contiguous tensors."""
    n = q8.shape[1]
    ns = cells.shape[0]
    if out is None:
        feat = torch.empty((ns, 9), dtype=torch.float32, device=q8.device)
        targ = torch.empty((ns, 2), dtype=torch.float32, device=q8.device)
    else:
        feat, targ = out
        assert feat.shape == (ns, 9) and targ.shape == (ns, 2) and feat.is_contiguous() and targ.is_contiguous()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    code = _lib.sme_closure_samples(ctypes.c_void_p(q8.data_ptr()), q8.stride(0), ctypes.c_void_p(q8_next.data_ptr()),
                                    q8_next.stride(0), ctypes.c_void_p(q1_step.data_ptr()), q1_step.stride(0), n,
                                    float(dt), ctypes.c_void_p(cells.data_ptr()), ns, ctypes.c_void_p(feat.data_ptr()),
                                    ctypes.c_void_p(targ.data_ptr()), ctypes.c_void_p(stream or 0))
    _check(code)
    return feat, targ


def closure_run(s1, s8, t_end, chunk, max_steps, max_out_of_range):
    """sme_closure_run on two Solvers; returns (t, steps, fallback_at or None)."""
    t, n, fb = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _check(_lib.sme_closure_run(s1.ctx, s8.ctx, float(t_end), int(chunk), int(max_steps), float(max_out_of_range),
                                ctypes.byref(t), ctypes.byref(n), ctypes.byref(fb)), s1.ctx)
    return t.value, n.value, (fb.value if fb.value >= 0 else None)


# ---------------------------------------------------------------------------
# Non-hydrostatic VAM channel (include/sme.h, sme_vam_*)
def _vcheck(code, ctx=None):
    if code != SME_OK:
        msg = (_lib.sme_vam_last_error(ctx) or b"").decode() if ctx else ""
        raise SmeError(code, msg or _lib.sme_strerror(code).decode())


def sme_vam_layout(nx):
    st = ctypes.c_int64()
    _vcheck(_lib.sme_vam_layout(int(nx), ctypes.byref(st)))
    return st.value


def sme_vam_workspace_size(nx):
    n = ctypes.c_size_t()
    _vcheck(_lib.sme_vam_workspace_size(int(nx), ctypes.byref(n)))
    return n.value


class Vam:
    """A VAM channel bound to two torch state tensors [5, field_stride]
    (fields h, h u0, h u1, h w0, h w1), problem dict from workloads.vam_1d."""

    def __init__(self, problem, stream=None, **overrides):
        prm = dict(problem["params"])
        prm.update(overrides)
        self.nx = int(problem["nx"])
        st = sme_vam_layout(self.nx)
        self.q_dev = [torch.zeros((5, st), dtype=torch.float64, device="cuda") for _ in range(2)]
        qp = (ctypes.c_void_p * 2)(self.q_dev[0].data_ptr(), self.q_dev[1].data_ptr())
        b = np.ascontiguousarray(problem["b"], dtype=np.float64)
        self.ctx = ctypes.c_void_p()
        torch.cuda.synchronize()
        _vcheck(_lib.sme_vam_init(ctypes.byref(self.ctx), self.nx, float(problem["x0"]), float(problem["x1"]),
                                  float(prm["g"]), float(prm["cfl"]), int(prm["quad_points"]), qp,
                                  b.ctypes.data_as(ctypes.c_void_p), 0, stream))

    def set_state(self, q):
        if isinstance(q, torch.Tensor):
            q = q.contiguous()
            torch.cuda.synchronize()
            _vcheck(_lib.sme_vam_set_state(self.ctx, ctypes.c_void_p(q.data_ptr()), 1), self.ctx)
        else:
            q = np.ascontiguousarray(q, dtype=np.float64)
            _vcheck(_lib.sme_vam_set_state(self.ctx, q.ctypes.data_as(ctypes.c_void_p), 0), self.ctx)

    def get_state(self):
        out = np.empty((5, self.nx))
        _vcheck(_lib.sme_vam_get_state(self.ctx, out.ctypes.data_as(ctypes.c_void_p), 0), self.ctx)
        return out

    def pressure(self):
        out = np.empty((2, self.nx))
        _vcheck(_lib.sme_vam_pressure(self.ctx, out.ctypes.data_as(ctypes.c_void_p), 0), self.ctx)
        return out

    def step(self, dt=0.0):
        used = ctypes.c_double()
        _vcheck(_lib.sme_vam_step(self.ctx, float(dt), ctypes.byref(used)), self.ctx)
        return used.value

    def run(self, n_steps, t_end=0.0):
        t, k = ctypes.c_double(), ctypes.c_int64()
        _vcheck(_lib.sme_vam_run(self.ctx, int(n_steps), float(t_end), ctypes.byref(t), ctypes.byref(k)), self.ctx)
        return t.value, k.value

    def time(self):
        t, k = ctypes.c_double(), ctypes.c_int64()
        _vcheck(_lib.sme_vam_time(self.ctx, ctypes.byref(t), ctypes.byref(k)), self.ctx)
        return t.value, k.value

    def current(self):
        return _lib.sme_vam_current(self.ctx)

    def close(self):
        if self.ctx:
            _lib.sme_vam_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()
