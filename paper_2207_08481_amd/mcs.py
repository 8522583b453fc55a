"""ctypes binding of libmcs.so (the C ABI declared in include/mcs.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  PyTorch provides device memory (the workspace and vectors) and the
stream.  The binding refuses to run when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcs.so")

# status codes (mcs_status)
OK = 0
STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_MESH", -3: "ERR_WORKSPACE", -4: "ERR_NOT_SPD",
          -5: "ERR_NOT_CONVERGED", -6: "ERR_BREAKDOWN", -7: "ERR_NONFINITE", -8: "ERR_STATE",
          -9: "ERR_HIP", -10: "ERR_UNSUPPORTED"}
STATUS_NOT_CONVERGED = -5
F64, F32 = 0, 1
OP = {"K": 0, "A": 1, "ADELTA": 2, "B": 3, "BT": 4}
PC = {"KHAT": 0, "AEXT": 1, "ADELTA_MULT": 2, "SMOOTH_FWD": 3, "SMOOTH_BWD": 4, "AUX": 5,
      "EDELTA": 6, "EDELTA_T": 7, "MG": 8, "MP_INV": 9}

# exported symbols of include/mcs.h
SYMBOLS = ["mcs_plan", "mcs_bind", "mcs_condense", "mcs_load", "mcs_apply", "mcs_precond_apply",
           "mcs_solve", "mcs_solve_rhs", "mcs_solve_rhs_noalloc", "mcs_normalize_pressure", "mcs_eval", "mcs_eval_stress", "mcs_set_dirichlet",
                 "mcs_get_array",
           "mcs_get_topology", "mcs_get_full_colouring", "mcs_timer_enable", "mcs_timer_read", "mcs_get_launch_config",
           "mcs_set_launch_config", "mcs_get_apply_config", "mcs_set_apply_config", "mcs_set_solve_options",
           "mcs_destroy",
           "mcs_status_string", "mcs_last_error",
           "mcs_batch_plan", "mcs_batch_member_info", "mcs_batch_bind", "mcs_batch_condense",
           "mcs_batch_solve", "mcs_batch_solve_async", "mcs_batch_poll", "mcs_batch_wait",
           "mcs_batch_set_mode", "mcs_batch_launch_config", "mcs_batch_timer_enable",
           "mcs_batch_timer_read",
           "mcs_batch_destroy", "mcs_server_create", "mcs_server_submit", "mcs_server_poll",
           "mcs_server_wait", "mcs_server_stats", "mcs_server_destroy"]


class MCSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_vertices", C.c_int32), ("vertices_host", C.c_void_p),
                ("n_elements", C.c_int32), ("elements_host", C.c_void_p), ("lattice", C.c_int32 * 3),
                ("face_bc", C.c_int32 * 6)]


class Options(C.Structure):
    _fields_ = [("order", C.c_int32), ("precision", C.c_int32), ("smoothing_steps", C.c_int32),
                ("max_it", C.c_int32), ("tol", C.c_double), ("inner_tol", C.c_double),
                ("max_outer", C.c_int32), ("coarse_max", C.c_int32), ("autotune", C.c_int32),
                ("smoother", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("n_dof", C.c_int64), ("n_bubble_dofs", C.c_int64), ("n_facet_dofs", C.c_int64),
                ("n_pressure_dofs", C.c_int64), ("n_p1_dofs", C.c_int64), ("off_facet", C.c_int64),
                ("off_pressure", C.c_int64), ("n_bub", C.c_int32), ("n_F", C.c_int32),
                ("n_hat", C.c_int32), ("n_fb", C.c_int32), ("n_p", C.c_int32), ("n_lat", C.c_int32),
                ("n_free_facets", C.c_int32), ("n_colours", C.c_int32), ("n_mg_levels", C.c_int32),
                ("workspace_bytes", C.c_size_t)]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("outer_steps", C.c_int32),
                ("rel_precond_residual", C.c_double), ("rel_residual", C.c_double),
                ("t_solve_ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class RequestInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("outer_steps", C.c_int32),
                ("batch_size", C.c_int32), ("rel_residual", C.c_double), ("rel_precond_residual", C.c_double),
                ("queue_ms", C.c_double), ("solve_ms", C.c_double), ("latency_ms", C.c_double),
                ("message", C.c_char * 160)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["message"] = d["message"].decode(errors="replace")
        return d


class ServerStats(C.Structure):
    _fields_ = [("arena_bytes", C.c_size_t), ("arena_used", C.c_size_t), ("arena_peak", C.c_size_t),
                ("batches", C.c_int64), ("solved", C.c_int64), ("waiting", C.c_int64), ("inflight", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BatchInfo(C.Structure):
    _fields_ = [("n_problems", C.c_int32), ("n_groups", C.c_int32), ("n_dof_total", C.c_int64),
                ("workspace_bytes", C.c_size_t)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmcs.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} not found: build it with paper_2207_08481_amd/build.py")
    lib = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.mcs_plan.argtypes = [C.POINTER(Mesh), C.POINTER(Options), C.POINTER(vp), C.POINTER(Info)]
    lib.mcs_bind.argtypes = [vp, vp, C.c_size_t, vp]
    lib.mcs_condense.argtypes = [vp, vp]
    lib.mcs_load.argtypes = [vp, vp, vp]
    lib.mcs_apply.argtypes = [vp, i32, i32, vp, vp]
    lib.mcs_precond_apply.argtypes = [vp, i32, i32, vp, vp]
    lib.mcs_solve.argtypes = [vp, vp, vp, C.POINTER(SolveInfo)]
    lib.mcs_solve_rhs.argtypes = [vp, vp, vp, C.POINTER(SolveInfo)]
    lib.mcs_solve_rhs_noalloc.argtypes = [vp, vp, vp, C.POINTER(SolveInfo)]
    lib.mcs_normalize_pressure.argtypes = [vp, vp]
    lib.mcs_eval.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.mcs_eval_stress.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.mcs_set_dirichlet.argtypes = [vp, vp]
    lib.mcs_get_array.argtypes = [vp, C.c_char_p, C.POINTER(vp), C.POINTER(i64)]
    lib.mcs_get_topology.argtypes = [vp, vp, vp]
    lib.mcs_get_full_colouring.argtypes = [vp, C.POINTER(i64), vp]
    lib.mcs_timer_enable.argtypes = [vp, i32]
    lib.mcs_timer_read.argtypes = [vp, i32, C.POINTER(C.c_double), C.POINTER(i64), C.POINTER(C.c_double)]
    lib.mcs_get_launch_config.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i64), C.POINTER(C.c_double)]
    lib.mcs_set_launch_config.argtypes = [vp, i32, i32, i64]
    lib.mcs_get_apply_config.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(C.c_double)]
    lib.mcs_set_apply_config.argtypes = [vp, i32, i32]
    lib.mcs_set_solve_options.argtypes = [vp, C.c_double, i32, C.c_double, i32]
    lib.mcs_batch_launch_config.argtypes = [vp, i32, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                            C.POINTER(i64), C.POINTER(C.c_double)]
    lib.mcs_destroy.argtypes = [vp]
    lib.mcs_destroy.restype = None
    lib.mcs_status_string.argtypes = [i32]
    lib.mcs_status_string.restype = C.c_char_p
    lib.mcs_last_error.argtypes = []
    lib.mcs_last_error.restype = C.c_char_p
    lib.mcs_batch_plan.argtypes = [C.POINTER(Mesh), vp, i32, C.POINTER(Options), C.POINTER(vp),
                                   C.POINTER(BatchInfo)]
    lib.mcs_batch_member_info.argtypes = [vp, i32, C.POINTER(Info)]
    lib.mcs_batch_bind.argtypes = [vp, vp, C.c_size_t, vp]
    lib.mcs_batch_condense.argtypes = [vp, vp]
    lib.mcs_batch_solve.argtypes = [vp, vp, vp, vp]
    lib.mcs_batch_solve_async.argtypes = [vp, vp, vp]
    lib.mcs_batch_poll.argtypes = [vp, C.POINTER(i32)]
    lib.mcs_batch_wait.argtypes = [vp, vp]
    lib.mcs_batch_set_mode.argtypes = [vp, i32, i32]
    lib.mcs_batch_timer_enable.argtypes = [vp, i32]
    lib.mcs_batch_timer_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i64), C.POINTER(C.c_double)]
    lib.mcs_batch_destroy.argtypes = [vp]
    lib.mcs_batch_destroy.restype = None
    lib.mcs_server_create.argtypes = [C.POINTER(Options), vp, C.c_size_t, i32, i32, C.POINTER(vp)]
    lib.mcs_server_submit.argtypes = [vp, C.POINTER(Mesh), i32, vp, vp, C.POINTER(i64)]
    lib.mcs_server_poll.argtypes = [vp, i64, C.POINTER(i32)]
    lib.mcs_server_wait.argtypes = [vp, i64, vp, C.POINTER(RequestInfo)]
    lib.mcs_server_stats.argtypes = [vp, C.POINTER(ServerStats)]
    lib.mcs_server_destroy.argtypes = [vp]
    lib.mcs_server_destroy.restype = None
    for name in ("mcs_plan", "mcs_bind", "mcs_condense", "mcs_load", "mcs_apply", "mcs_precond_apply",
                 "mcs_solve", "mcs_solve_rhs", "mcs_solve_rhs_noalloc", "mcs_normalize_pressure", "mcs_eval", "mcs_eval_stress", "mcs_set_dirichlet",
                 "mcs_get_array",
                 "mcs_get_topology", "mcs_get_full_colouring", "mcs_timer_enable", "mcs_timer_read", "mcs_get_launch_config", "mcs_set_launch_config", "mcs_get_apply_config", "mcs_set_apply_config", "mcs_set_solve_options", "mcs_batch_plan",
                 "mcs_batch_member_info", "mcs_batch_bind", "mcs_batch_condense", "mcs_batch_solve",
                 "mcs_batch_solve_async", "mcs_batch_poll", "mcs_batch_wait", "mcs_batch_set_mode", "mcs_batch_launch_config", "mcs_batch_timer_enable", "mcs_batch_timer_read",
                 "mcs_server_create",
                 "mcs_server_submit", "mcs_server_poll", "mcs_server_wait", "mcs_server_stats"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(rc):
    if rc != OK:
        raise MCSError(rc, _lib.mcs_last_error().decode())


class _CudaArray:
    """Minimal __cuda_array_interface__ wrapper around a device pointer."""

    def __init__(self, ptr, n, typestr):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False),
                                         "version": 3, "strides": None}


@dataclass
class ProblemSpec:
    vertices: np.ndarray
    elements: np.ndarray
    lattice: tuple
    order: int


class Problem:
    """One MCS Stokes problem: plan (host), bind (device workspace), condense,
    solve.  Names follow the C ABI."""

    def __init__(self, vertices, elements, lattice, order, precision=0, smoothing_steps=2,
                 tol=1e-10, max_it=2000, inner_tol=1e-5, max_outer=10, coarse_max=512, autotune=0,
                 smoother=0, face_bc=None):
        lib = load_library()
        self._lib = lib
        v = np.ascontiguousarray(vertices, dtype=np.float64)
        e = np.ascontiguousarray(elements, dtype=np.int32)
        self.dim = v.shape[1]
        self._v, self._e = v, e
        lat = list(lattice) + [1] * (3 - len(lattice))
        fb = list(face_bc) if face_bc is not None else []
        self._mesh = Mesh(self.dim, v.shape[0], v.ctypes.data, e.shape[0], e.ctypes.data,
                          (C.c_int32 * 3)(*lat), (C.c_int32 * 6)(*(fb + [0] * (6 - len(fb)))))
        self._opt = Options(order, precision, smoothing_steps, max_it, tol, inner_tol, max_outer,
                            coarse_max, autotune, smoother)
        self.info = Info()
        h = C.c_void_p()
        _check(lib.mcs_plan(C.byref(self._mesh), C.byref(self._opt), C.byref(h), C.byref(self.info)))
        self._h = h
        self.workspace = None
        self.order = order
        self.n_elements = e.shape[0]

    # ------------------------------------------------------------------ host
    @property
    def n_dof(self):
        return self.info.n_dof

    def topology(self):
        colour = np.zeros(self.info.n_free_facets, dtype=np.int32)
        eff = np.zeros(self.n_elements * (self.dim + 1), dtype=np.int32)
        _check(self._lib.mcs_get_topology(self._h, colour.ctypes.data, eff.ctypes.data))
        return colour, eff.reshape(self.n_elements, self.dim + 1)

    # ---------------------------------------------------------------- device
    def bind(self, device="cuda:0"):
        import torch
        dev = torch.device(device)
        torch.cuda.set_device(dev)
        self.device = dev
        self.workspace = torch.empty(self.info.workspace_bytes, dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.current_stream(dev)
        _check(self._lib.mcs_bind(self._h, self.workspace.data_ptr(), self.info.workspace_bytes,
                                  self.stream.cuda_stream))
        return self

    def condense(self, nu):
        import torch
        nu = torch.as_tensor(nu, dtype=torch.float64, device=self.device).contiguous()
        if nu.numel() == 1:
            nu = nu.expand(self.n_elements).contiguous()
        self._nu = nu
        _check(self._lib.mcs_condense(self._h, nu.data_ptr()))

    def vector(self, dtype=None):
        import torch
        return torch.zeros(self.n_dof, dtype=dtype or torch.float64, device=self.device)

    def load(self, f_lattice):
        import torch
        f = torch.as_tensor(f_lattice, dtype=torch.float64, device=self.device).contiguous()
        b = self.vector()
        _check(self._lib.mcs_load(self._h, f.data_ptr(), b.data_ptr()))
        return b

    @staticmethod
    def _dt(t):
        import torch
        return F64 if t.dtype == torch.float64 else F32

    def apply(self, op, x, y=None):
        if y is None:
            y = x.new_zeros(self.n_dof)
        _check(self._lib.mcs_apply(self._h, OP[op], self._dt(x), x.data_ptr(), y.data_ptr()))
        return y

    def precond_apply(self, op, r, z=None, out_len=None):
        if z is None:
            n = out_len if out_len is not None else (
                self.info.n_p1_dofs if op in ("EDELTA_T", "MG") else self.n_dof)
            z = r.new_zeros(n)
        _check(self._lib.mcs_precond_apply(self._h, PC[op], self._dt(r), r.data_ptr(), z.data_ptr()))
        return z

    def solve(self, f_lattice, allow_max_it=False):
        """(x, info).  With allow_max_it, a solve that stops at max_it
        (MCS_ERR_NOT_CONVERGED) returns its last iterate instead of raising."""
        import torch
        f = torch.as_tensor(f_lattice, dtype=torch.float64, device=self.device).contiguous()
        x = self.vector()
        si = SolveInfo()
        rc = self._lib.mcs_solve(self._h, f.data_ptr(), x.data_ptr(), C.byref(si))
        if not (allow_max_it and rc == STATUS_NOT_CONVERGED):
            _check(rc)
        return x, si.as_dict()

    def solve_rhs(self, b, allow_max_it=False):
        """(x, info) for right-hand side b; allow_max_it as for solve()."""
        x = self.vector()
        si = SolveInfo()
        rc = self._lib.mcs_solve_rhs(self._h, b.data_ptr(), x.data_ptr(), C.byref(si))
        if not (allow_max_it and rc == STATUS_NOT_CONVERGED):
            _check(rc)
        return x, si.as_dict()

    def solve_rhs_noalloc(self, b, x, allow_max_it=False):
        """mcs_solve_rhs_noalloc into the caller's x (nothing is allocated by
        the library; x must be a device double vector of n_dof).  Returns info."""
        si = SolveInfo()
        rc = self._lib.mcs_solve_rhs_noalloc(self._h, b.data_ptr(), x.data_ptr(), C.byref(si))
        if not (allow_max_it and rc == STATUS_NOT_CONVERGED):
            _check(rc)
        return si.as_dict()

    def eval(self, x, ref_pts):
        """(u [n_e, n_pts, dim], p [n_e, n_pts]) of x at barycentric points
        ref_pts [n_pts, dim+1] w.r.t. each element's vertices in caller order."""
        import torch
        pts = np.ascontiguousarray(ref_pts, dtype=np.float64)
        npts = pts.shape[0]
        u = torch.zeros((self.n_elements, npts, self.dim), dtype=torch.float64, device=self.device)
        p = torch.zeros((self.n_elements, npts), dtype=torch.float64, device=self.device)
        _check(self._lib.mcs_eval(self._h, x.data_ptr(), npts, pts.ctypes.data, u.data_ptr(), p.data_ptr()))
        return u, p

    def set_dirichlet(self, g_lattice):
        """Dirichlet data g on the element lattices ([n_e, n_lat, dim], host
        array like f's values), or None for homogeneous data."""
        if g_lattice is None:
            _check(self._lib.mcs_set_dirichlet(self._h, None))
            return
        g = np.ascontiguousarray(g_lattice, dtype=np.float64)
        _check(self._lib.mcs_set_dirichlet(self._h, g.ctypes.data))

    def eval_stress(self, x, ref_pts):
        """(sigma, omega), each [n_e, n_pts, dim, dim]: the stress and vorticity
        recovered from x (local problems of the condensation) at barycentric
        points ref_pts [n_pts, dim+1] w.r.t. each element's vertices in caller
        order."""
        import torch
        pts = np.ascontiguousarray(ref_pts, dtype=np.float64)
        npts = pts.shape[0]
        shape = (self.n_elements, npts, self.dim, self.dim)
        sig = torch.zeros(shape, dtype=torch.float64, device=self.device)
        om = torch.zeros(shape, dtype=torch.float64, device=self.device)
        _check(self._lib.mcs_eval_stress(self._h, x.data_ptr(), npts, pts.ctypes.data, sig.data_ptr(),
                                         om.data_ptr()))
        return sig, om

    def normalize_pressure(self, x):
        _check(self._lib.mcs_normalize_pressure(self._h, x.data_ptr()))
        return x

    def get_array(self, name):
        """torch view of an internal workspace array (float64 unless '32')."""
        import torch
        p = C.c_void_p()
        n = C.c_int64()
        _check(self._lib.mcs_get_array(self._h, name.encode(), C.byref(p), C.byref(n)))
        if name in ("colour_desc", "elem_ff"):
            typestr = "<i4"
        elif name.endswith("32"):
            typestr = "<f4"
        else:
            typestr = "<f8"
        return torch.as_tensor(_CudaArray(p.value, n.value, typestr), device=self.device)

    def full_colouring(self):
        """Colour of every block of the full-system variant (canonical facet order)."""
        n = C.c_int64()
        _check(self._lib.mcs_get_full_colouring(self._h, C.byref(n), None))
        col = np.zeros(n.value, dtype=np.int32)
        _check(self._lib.mcs_get_full_colouring(self._h, C.byref(n), col.ctypes.data))
        return col

    def launch_config(self, dt=F64):
        f, c, us = C.c_int32(), C.c_int64(), C.c_double()
        _check(self._lib.mcs_get_launch_config(self._h, dt, C.byref(f), C.byref(c), C.byref(us)))
        return {"facets_per_block": f.value, "grid_cap": c.value, "us_per_launch": us.value}

    def set_launch_config(self, facets_per_block, grid_cap=0, dt=F64):
        """Fixes the colour phase's launch shape for precision slot dt; the
        autotuner leaves a slot set here alone.  dt=F64 on a precision 1
        problem (no FP64 smoother) raises."""
        _check(self._lib.mcs_set_launch_config(self._h, dt, facets_per_block, grid_cap))

    def apply_config(self, dt=F64):
        """Rows of A^d per thread of the operator apply for precision slot dt
        (0: the default choice) and the tuner's time per K x in us."""
        r, us = C.c_int32(), C.c_double()
        _check(self._lib.mcs_get_apply_config(self._h, dt, C.byref(r), C.byref(us)))
        return {"rows_per_thread": r.value, "us_per_apply": us.value}

    def set_apply_config(self, rows_per_thread, dt=F64):
        """Fixes the apply's rows of A^d per thread (0, 1, 2, or 4 in FP32);
        the autotuner leaves a slot set here alone."""
        _check(self._lib.mcs_set_apply_config(self._h, dt, rows_per_thread))

    def set_solve_options(self, tol, max_it, inner_tol=None, max_outer=None):
        """Stopping rules of later solves (tol, max_it, inner_tol, max_outer)."""
        o = self._opt
        inner = o.inner_tol if inner_tol is None else inner_tol
        outer = o.max_outer if max_outer is None else max_outer
        _check(self._lib.mcs_set_solve_options(self._h, tol, max_it, inner, outer))
        o.tol, o.max_it, o.inner_tol, o.max_outer = tol, max_it, inner, outer

    def timer_enable(self, on=True, period=1):
        """Kernel timer on (one call in `period` is timed) or off."""
        _check(self._lib.mcs_timer_enable(self._h, int(period) if on else 0))

    def timer_read(self, kernel="smooth"):
        """(total kernel ms, launches, algorithmic bytes) of the timed launches of
        one kernel: "smooth" (block Gauss-Seidel colour phase) or "kapply"
        (operator apply K x)."""
        ms = C.c_double()
        n = C.c_int64()
        b = C.c_double()
        kid = {"smooth": 0, "kapply": 1}[kernel]
        _check(self._lib.mcs_timer_read(self._h, kid, C.byref(ms), C.byref(n), C.byref(b)))
        return ms.value, n.value, b.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mcs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr_array(tensors):
    arr = (C.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])
    return arr


class Batch:
    """Many independent problems solved together (mcs_batch_*): members with
    the same dimension and order share every kernel launch; MINRES runs per
    member.  meshes: list of (vertices, elements, lattice); orders: list of k."""

    def __init__(self, meshes, orders, precision=1, smoothing_steps=2, tol=1e-8, max_it=2000,
                 inner_tol=1e-5, max_outer=10, coarse_max=512, autotune=1, smoother=0, face_bcs=None):
        lib = load_library()
        self._lib = lib
        self._keep = []
        arr = (Mesh * len(meshes))()
        self.dims, self.n_elements = [], []
        for i, (v, e, lat) in enumerate(meshes):
            v = np.ascontiguousarray(v, dtype=np.float64)
            e = np.ascontiguousarray(e, dtype=np.int32)
            self._keep += [v, e]
            lat = list(lat) + [1] * (3 - len(lat))
            fb = list(face_bcs[i]) if face_bcs is not None else []
            arr[i] = Mesh(v.shape[1], v.shape[0], v.ctypes.data, e.shape[0], e.ctypes.data, (C.c_int32 * 3)(*lat),
                          (C.c_int32 * 6)(*(fb + [0] * (6 - len(fb)))))
            self.dims.append(v.shape[1])
            self.n_elements.append(e.shape[0])
        self._meshes = arr
        self.orders = [int(k) for k in orders]
        ords = np.asarray(self.orders, dtype=np.int32)
        self._keep.append(ords)
        self._opt = Options(0, precision, smoothing_steps, max_it, tol, inner_tol, max_outer, coarse_max, autotune,
                            smoother)
        self.info = BatchInfo()
        h = C.c_void_p()
        _check(lib.mcs_batch_plan(arr, ords.ctypes.data, len(meshes), C.byref(self._opt), C.byref(h),
                                  C.byref(self.info)))
        self._h = h
        self.n = len(meshes)
        self.members = []
        for i in range(self.n):
            mi = Info()
            _check(lib.mcs_batch_member_info(h, i, C.byref(mi)))
            self.members.append(mi)

    def bind(self, device="cuda:0"):
        import torch
        dev = torch.device(device)
        torch.cuda.set_device(dev)
        self.device = dev
        self.workspace = torch.empty(self.info.workspace_bytes, dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.current_stream(dev)
        _check(self._lib.mcs_batch_bind(self._h, self.workspace.data_ptr(), self.info.workspace_bytes,
                                        self.stream.cuda_stream))
        return self

    def set_mode(self, use_graph=True, chunk=6):
        _check(self._lib.mcs_batch_set_mode(self._h, 1 if use_graph else 0, chunk))

    def launch_configs(self, dt=F32):
        """Per group: dimension, order and the smoother launch shape chosen by the tuner."""
        out = []
        for g in range(self.info.n_groups):
            d, k, f = C.c_int32(), C.c_int32(), C.c_int32()
            c, us = C.c_int64(), C.c_double()
            _check(self._lib.mcs_batch_launch_config(self._h, g, dt, C.byref(d), C.byref(k), C.byref(f), C.byref(c),
                                                     C.byref(us)))
            out.append({"dim": d.value, "order": k.value, "facets_per_block": f.value, "grid_cap": c.value,
                        "us_per_launch": us.value})
        return out

    def timer_enable(self, on=True):
        _check(self._lib.mcs_batch_timer_enable(self._h, 1 if on else 0))

    def timer_read(self):
        ms = C.c_double()
        n = C.c_int64()
        b = C.c_double()
        _check(self._lib.mcs_batch_timer_read(self._h, C.byref(ms), C.byref(n), C.byref(b)))
        return ms.value, n.value, b.value

    def condense(self, nus):
        import torch
        ts = []
        for i, nu in enumerate(nus):
            t = torch.as_tensor(nu, dtype=torch.float64, device=self.device).contiguous()
            if t.numel() == 1:
                t = t.expand(self.n_elements[i]).contiguous()
            ts.append(t)
        self._nus = ts
        _check(self._lib.mcs_batch_condense(self._h, _ptr_array(ts)))

    def solve(self, forces):
        """Returns (list of solution tensors in each member's own layout, list of info dicts)."""
        import torch
        fs = [torch.as_tensor(f, dtype=torch.float64, device=self.device).contiguous() for f in forces]
        xs = [torch.zeros(m.n_dof, dtype=torch.float64, device=self.device) for m in self.members]
        infos = (SolveInfo * self.n)()
        rc = self._lib.mcs_batch_solve(self._h, _ptr_array(fs), _ptr_array(xs), infos)
        out = [infos[i].as_dict() for i in range(self.n)]
        if rc != OK and rc != -5:
            _check(rc)
        return xs, out

    def solve_async(self, forces):
        """Starts the solve on a library thread (mcs_batch_solve_async) and
        returns at once; poll() tells whether it finished, wait() returns what
        solve() would."""
        import torch
        fs = [torch.as_tensor(f, dtype=torch.float64, device=self.device).contiguous() for f in forces]
        xs = [torch.zeros(m.n_dof, dtype=torch.float64, device=self.device) for m in self.members]
        _check(self._lib.mcs_batch_solve_async(self._h, _ptr_array(fs), _ptr_array(xs)))
        self._async = (fs, xs)   # the device memory stays alive until wait()

    def poll(self):
        d = C.c_int32()
        _check(self._lib.mcs_batch_poll(self._h, C.byref(d)))
        return bool(d.value)

    def wait(self):
        infos = (SolveInfo * self.n)()
        rc = self._lib.mcs_batch_wait(self._h, infos)
        fs, xs = getattr(self, "_async", (None, None))
        self._async = None
        out = [infos[i].as_dict() for i in range(self.n)]
        if rc != OK and rc != -5:
            _check(rc)
        return xs, out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mcs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching solve server (mcs_server_*): requests are queued,
    admitted in micro-batches against a device arena of `arena_bytes` (the HBM
    budget) and solved by the batch solver on library threads; up to
    max_inflight micro-batches run at once.  The calls release the GIL."""

    def __init__(self, arena_bytes, device="cuda:0", max_inflight=2, max_batch=64, precision=1,
                 smoothing_steps=2, tol=1e-8, max_it=5000, inner_tol=1e-5, max_outer=10, coarse_max=512,
                 autotune=0, smoother=0):
        import torch
        lib = load_library()
        self._lib = lib
        dev = torch.device(device)
        torch.cuda.set_device(dev)
        self.device = dev
        self._arena = torch.empty(arena_bytes + 4096, dtype=torch.uint8, device=dev)
        base = self._arena.data_ptr()
        aligned = (base + 4095) // 4096 * 4096
        self._opt = Options(0, precision, smoothing_steps, max_it, tol, inner_tol, max_outer, coarse_max, autotune,
                            smoother)
        torch.cuda.synchronize()
        h = C.c_void_p()
        _check(lib.mcs_server_create(C.byref(self._opt), aligned, arena_bytes, max_inflight, max_batch,
                                     C.byref(h)))
        self._h = h

    def submit(self, vertices, elements, lattice, order, nu, f_lattice):
        v = np.ascontiguousarray(vertices, dtype=np.float64)
        e = np.ascontiguousarray(elements, dtype=np.int32)
        nu = np.ascontiguousarray(np.broadcast_to(np.asarray(nu, dtype=np.float64), (e.shape[0],)))
        f = np.ascontiguousarray(f_lattice, dtype=np.float64)
        lat = list(lattice) + [1] * (3 - len(lattice))
        mesh = Mesh(v.shape[1], v.shape[0], v.ctypes.data, e.shape[0], e.ctypes.data, (C.c_int32 * 3)(*lat))
        rid = C.c_int64()
        _check(self._lib.mcs_server_submit(self._h, C.byref(mesh), order, nu.ctypes.data, f.ctypes.data,
                                           C.byref(rid)))
        return rid.value

    def poll(self, rid):
        d = C.c_int32()
        _check(self._lib.mcs_server_poll(self._h, rid, C.byref(d)))
        return bool(d.value)

    def wait(self, rid, n_dof):
        """Blocks until request rid is done; returns (solution numpy array, info dict)."""
        x = np.zeros(n_dof, dtype=np.float64)
        info = RequestInfo()
        self._lib.mcs_server_wait(self._h, rid, x.ctypes.data, C.byref(info))
        return x, info.as_dict()

    def stats(self):
        st = ServerStats()
        _check(self._lib.mcs_server_stats(self._h, C.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mcs_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
