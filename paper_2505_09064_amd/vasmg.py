"""ctypes binding of libvasmg (the C ABI declared in include/vasmg.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels. Device vectors are torch tensors on a HIP device (torch is used for
device memory and streams only). The library must have been built
(``python -m paper_2505_09064_amd.build``); importing this module fails loudly
otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvasmg.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, EBREAKDOWN, EDEGENERATE = range(7)
FP64, FP32_PRECOND = 0, 1
TREE_ALL, TREE_FREE = 0, 1
PRECOND_VASMG, PRECOND_JACOBI, PRECOND_NONE = 0, 1, 2
CYCLE_V, CYCLE_W, CYCLE_ADDITIVE = 0, 1, 2
SMOOTHER_GS, SMOOTHER_JACOBI = 0, 1

STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENOTCONV",
                5: "EBREAKDOWN", 6: "EDEGENERATE"}

EXPORTED = [
    "vasmg_default_options", "vasmg_setup", "vasmg_solve", "vasmg_solve_device", "vasmg_free",
    "vasmg_last_error", "vasmg_hierarchy_info", "vasmg_level_info", "vasmg_export_level",
    "vasmg_tree_info", "vasmg_spmv_device", "vasmg_gs_sweep_device", "vasmg_restrict_device",
    "vasmg_prolong_device", "vasmg_apply_precond_device", "vasmg_profile_iteration",
    "vasmg_upload", "vasmg_device_bytes", "vasmg_server_default_config", "vasmg_server_create",
    "vasmg_server_submit", "vasmg_server_wait", "vasmg_server_stats", "vasmg_server_destroy",
    "vasmg_set_galerkin_window", "vasmg_solve_noalloc", "vasmg_setup_phases", "vasmg_pack",
    "vasmg_packed_info", "vasmg_solve_packed_device", "vasmg_solve_packed",
]


class VasmgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_vertices", C.c_int64), ("coords", C.c_void_p),
                ("n_elements", C.c_int64), ("elems", C.c_void_p), ("E", C.c_void_p),
                ("nu", C.c_void_p), ("fixed", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("leaf_capacity", C.c_int32), ("n_pre", C.c_int32), ("n_post", C.c_int32),
                ("precision", C.c_int32), ("tree_vertices", C.c_int32),
                ("coarsest_max_dofs", C.c_int64), ("max_iters", C.c_int32),
                ("preconditioner", C.c_int32), ("profile", C.c_int32),
                ("host_only", C.c_int32), ("verbose", C.c_int32), ("autotune", C.c_int32),
                ("block_rhs", C.c_int32), ("cycle", C.c_int32), ("smoother", C.c_int32),
                ("setup_device", C.c_int32), ("color_blocks", C.c_int32),
                ("block_lanes", C.c_int32)]


class PhaseStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("level", C.c_int32), ("launches", C.c_int32),
                ("ms", C.c_double), ("bytes", C.c_double)]


class SetupPhase(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("ms", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("rel_res", C.c_double),
                ("rel_res_true", C.c_double), ("t_solve_ms", C.c_double),
                ("t_spmv_ms", C.c_double), ("t_precond_ms", C.c_double),
                ("t_vector_ms", C.c_double), ("bytes_model", C.c_double),
                ("status", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(C.Structure):
    _fields_ = [("slots", C.c_int32), ("setup_workers", C.c_int32),
                ("hbm_budget_bytes", C.c_int64), ("options", Options),
                ("pack_max_dofs", C.c_int32), ("pack_max_parts", C.c_int32),
                ("pack_wait_ms", C.c_int32), ("host_setup_max_dofs_2d", C.c_int32),
                ("host_setup_max_dofs_3d", C.c_int32), ("reserved", C.c_int32)]


class RequestResult(C.Structure):
    _fields_ = [("id", C.c_int64), ("status", C.c_int32), ("slot", C.c_int32),
                ("pack_size", C.c_int32), ("setup_device", C.c_int32), ("device_bytes", C.c_int64), ("t_submit_ms", C.c_double),
                ("t_setup_start_ms", C.c_double), ("t_setup_end_ms", C.c_double),
                ("t_admit_ms", C.c_double), ("t_done_ms", C.c_double), ("info", SolveInfo),
                ("message", C.c_char * 128)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("info", "message")}
        d["info"] = self.info.as_dict()
        d["message"] = self.message.decode(errors="replace")
        return d


class ServerCounters(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64),
                ("waiting_setup", C.c_int64), ("waiting_admission", C.c_int64),
                ("running", C.c_int64), ("bytes_in_use", C.c_int64), ("peak_bytes", C.c_int64),
                ("budget_bytes", C.c_int64), ("t_now_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libvasmg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with "
                              "`python -m paper_2505_09064_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "vasmg_default_options": (i32, [i32, C.POINTER(Options)]),
            "vasmg_setup": (i32, [C.POINTER(Mesh), C.POINTER(Options), C.POINTER(vp)]),
            "vasmg_solve": (i32, [vp, vp, vp, vp, i32, dbl, C.POINTER(SolveInfo)]),
            "vasmg_solve_device": (i32, [vp, vp, vp, vp, i32, dbl, vp, C.POINTER(SolveInfo)]),
            "vasmg_solve_noalloc": (i32, [vp, vp, vp, vp, i32, dbl, C.POINTER(SolveInfo)]),
            "vasmg_free": (None, [vp]),
            "vasmg_last_error": (C.c_char_p, []),
            "vasmg_hierarchy_info": (i32, [vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(i32)]),
            "vasmg_level_info": (i32, [vp, i32, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32),
                                       C.POINTER(i64)]),
            "vasmg_export_level": (i32, [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
            "vasmg_tree_info": (i32, [vp, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(i32)]),
            "vasmg_setup_phases": (i32, [vp, vp, i32, C.POINTER(i32)]),
            "vasmg_pack": (i32, [vp, i32, C.POINTER(vp)]),
            "vasmg_packed_info": (i32, [vp, C.POINTER(i32), vp]),
            "vasmg_solve_packed_device": (i32, [vp, vp, vp, dbl, vp, vp]),
            "vasmg_solve_packed": (i32, [vp, vp, vp, dbl, vp]),
            "vasmg_spmv_device": (i32, [vp, i32, i32, vp, vp, vp]),
            "vasmg_gs_sweep_device": (i32, [vp, i32, i32, i32, vp, vp, vp]),
            "vasmg_restrict_device": (i32, [vp, i32, i32, vp, vp, vp]),
            "vasmg_prolong_device": (i32, [vp, i32, i32, vp, vp, vp]),
            "vasmg_apply_precond_device": (i32, [vp, vp, vp, vp]),
            "vasmg_profile_iteration": (i32, [vp, i32, vp, C.POINTER(PhaseStat), i32,
                                              C.POINTER(i32)]),
            "vasmg_upload": (i32, [vp, vp]),
            "vasmg_device_bytes": (i32, [vp, C.POINTER(i64)]),
            "vasmg_server_default_config": (i32, [C.POINTER(ServerConfig)]),
            "vasmg_server_create": (i32, [C.POINTER(ServerConfig), C.POINTER(vp)]),
            "vasmg_server_submit": (i32, [vp, C.POINTER(Mesh), vp, dbl, C.POINTER(i64)]),
            "vasmg_server_wait": (i32, [vp, i64, vp, C.POINTER(RequestResult)]),
            "vasmg_server_stats": (i32, [vp, C.POINTER(ServerCounters)]),
            "vasmg_server_destroy": (None, [vp]),
            "vasmg_set_galerkin_window": (i32, [i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().vasmg_last_error().decode()


def _check(status: int):
    if status != OK:
        raise VasmgError(status, last_error())


def default_options(dim: int) -> Options:
    o = Options()
    _check(lib().vasmg_default_options(dim, C.byref(o)))
    return o


def _ptr(a) -> int:
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _check_tensor(t, shape, name, device=None):
    """Raises ValueError unless t is a contiguous float64 tensor on a HIP device
    (the handle's, when known) with exactly `shape`: the kernels index these
    arrays by the handle's sizes and cannot check them."""
    if t is None or not hasattr(t, "data_ptr") or not hasattr(t, "is_contiguous"):
        raise ValueError(f"{name}: expected a torch tensor on a HIP device")
    import torch
    if t.device.type != "cuda":
        raise ValueError(f"{name}: tensor is on {t.device}, not on a HIP device")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name}: tensor is on device {t.device.index}, the handle on {device}")
    if t.dtype != torch.float64:
        raise ValueError(f"{name}: dtype {t.dtype}, expected torch.float64")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor is not contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")


def _stream_ptr(stream):
    if stream is None:
        return None
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


class Solver:
    """Owns one vasmg handle (vasmg_setup ... vasmg_free)."""

    def __init__(self, coords, elems, E, nu, fixed, options: Options | None = None, **kw):
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        elems = np.ascontiguousarray(elems, dtype=np.int32)
        nv, dim = coords.shape
        ne = elems.shape[0]
        self._arrays = (
            coords, elems,
            np.ascontiguousarray(np.broadcast_to(np.asarray(E, dtype=np.float64), (ne,))),
            np.ascontiguousarray(np.broadcast_to(np.asarray(nu, dtype=np.float64), (ne,))),
            np.ascontiguousarray(fixed, dtype=np.uint8).reshape(nv, dim),
        )
        c, el, Ea, nua, fx = self._arrays
        m = Mesh(dim, nv, _ptr(c), ne, _ptr(el), _ptr(Ea), _ptr(nua), _ptr(fx))
        opt = options if options is not None else default_options(dim)
        for k, v in kw.items():
            setattr(opt, k, v)
        self.options = opt
        self.dim = dim
        self.n_vertices = nv
        h = C.c_void_p()
        _check(lib().vasmg_setup(C.byref(m), C.byref(opt), C.byref(h)))
        self._h = h
        self._arrays = None          # the library deep-copied the mesh
        self.device = None           # HIP device the handle's memory lives on
        if not opt.host_only:
            import torch
            if torch.cuda.is_available():
                self.device = torch.cuda.current_device()

    @classmethod
    def from_mesh(cls, mesh, options: Options | None = None, **kw):
        return cls(mesh.coords, mesh.elems, mesh.E, mesh.nu, mesh.fixed, options, **kw)

    # -- lifetime -------------------------------------------------------
    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().vasmg_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.free()

    @property
    def handle(self):
        return self._h

    # -- solves -----------------------------------------------------------
    def solve(self, rhs, rtol: float = 1e-6, x0=None, check: bool = True):
        """Host arrays [n_vertices, dim] or [n_rhs, n_vertices, dim]."""
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        single = rhs.ndim == 2
        R = rhs[None] if single else rhs
        n_rhs = R.shape[0]
        x = np.zeros_like(R)
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64).reshape(R.shape)
        infos = (SolveInfo * n_rhs)()
        st = lib().vasmg_solve(self._h, _ptr(R), _ptr(x0a), _ptr(x), n_rhs, rtol, infos)
        if check and st not in (OK, ENOTCONV):
            _check(st)
        out = [i.as_dict() for i in infos]
        for o in out:
            o["status"] = st
        return (x[0], out[0]) if single else (x, out)

    def solve_noalloc(self, rhs, rtol: float = 1e-6, x0=None, check: bool = True):
        """As solve(), through vasmg_solve_noalloc (device staging in the
        library's fixed array, no device allocation during the call)."""
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        single = rhs.ndim == 2
        R = rhs[None] if single else rhs
        n_rhs = R.shape[0]
        if R.shape[1:] != (self.n_vertices, self.dim):
            raise ValueError(f"rhs: shape {rhs.shape}, expected [n_rhs?, {self.n_vertices}, {self.dim}]")
        x = np.zeros_like(R)
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64).reshape(R.shape)
        infos = (SolveInfo * n_rhs)()
        st = lib().vasmg_solve_noalloc(self._h, _ptr(R), _ptr(x0a), _ptr(x), n_rhs, rtol, infos)
        if check and st not in (OK, ENOTCONV):
            _check(st)
        out = [i.as_dict() for i in infos]
        for o in out:
            o["status"] = st
        return (x[0], out[0]) if single else (x, out)

    def solve_device(self, d_rhs, d_x, rtol: float = 1e-6, d_x0=None, stream=None,
                     check: bool = True):
        """torch FP64 device tensors [n_rhs?, n_vertices, dim] (contiguous)."""
        if not hasattr(d_rhs, "dim") or d_rhs.dim() not in (2, 3):
            raise ValueError("d_rhs: expected a tensor [n_rhs?, n_vertices, dim]")
        shape = ((self.n_vertices, self.dim) if d_rhs.dim() == 2
                 else (d_rhs.shape[0], self.n_vertices, self.dim))
        if d_rhs.dim() == 3 and d_rhs.shape[0] < 1:
            raise ValueError("d_rhs: n_rhs must be >= 1")
        _check_tensor(d_rhs, shape, "d_rhs", self.device)
        _check_tensor(d_x, shape, "d_x", self.device)
        if d_x0 is not None:
            _check_tensor(d_x0, shape, "d_x0", self.device)
        n_rhs = 1 if d_rhs.dim() == 2 else d_rhs.shape[0]
        infos = (SolveInfo * n_rhs)()
        st = lib().vasmg_solve_device(self._h, _ptr(d_rhs), _ptr(d_x0), _ptr(d_x), n_rhs, rtol,
                                      _stream_ptr(stream), infos)
        if check and st not in (OK, ENOTCONV):
            _check(st)
        out = [i.as_dict() for i in infos]
        for o in out:
            o["status"] = st
        return out[0] if n_rhs == 1 else out

    # -- introspection ------------------------------------------------------
    def hierarchy_info(self):
        nl, nd, dim = C.c_int32(), C.c_int64(), C.c_int32()
        _check(lib().vasmg_hierarchy_info(self._h, C.byref(nl), C.byref(nd), C.byref(dim)))
        return nl.value, nd.value, dim.value

    def level_info(self, level: int):
        nv, nb, nc, pn = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int64()
        _check(lib().vasmg_level_info(self._h, level, C.byref(nv), C.byref(nb), C.byref(nc),
                                      C.byref(pn)))
        return dict(n_vertices=nv.value, n_blocks=nb.value, n_colors=nc.value, p_nnz=pn.value)

    def export_level(self, level: int):
        info = self.level_info(level)
        d = self.dim
        n, nb, pn = info["n_vertices"], info["n_blocks"], info["p_nnz"]
        keys = np.empty((n, d), dtype=np.int64)
        cell = np.empty(n, dtype=np.int32)
        color = np.empty(n, dtype=np.int32)
        rowptr = np.empty(n + 1, dtype=np.int64)
        cols = np.empty(nb, dtype=np.int32)
        vals = np.empty((nb, d, d), dtype=np.float64)
        prow = np.empty(n + 1, dtype=np.int64)
        pcol = np.empty(pn, dtype=np.int32)
        pval = np.empty(pn, dtype=np.float64)
        block = np.empty(n, dtype=np.int32)
        fixed = np.empty(n, dtype=np.uint8)
        _check(lib().vasmg_export_level(self._h, level, _ptr(keys), _ptr(cell), _ptr(color),
                                        _ptr(rowptr), _ptr(cols), _ptr(vals), _ptr(prow),
                                        _ptr(pcol), _ptr(pval), _ptr(block), _ptr(fixed)))
        return dict(keys=keys, cell=cell, color=color, rowptr=rowptr, cols=cols, vals=vals,
                    p_rowptr=prow, p_cols=pcol, p_vals=pval, block=block, fixed=fixed, **info)

    def tree_info(self):
        m, M, dep = C.c_double(), C.c_double(), C.c_int32()
        _check(lib().vasmg_tree_info(self._h, C.byref(m), C.byref(M), C.byref(dep)))
        return m.value, M.value, dep.value

    def setup_phases(self):
        """[(name, ms)] of the setup phases, in the order they ran."""
        n = C.c_int32()
        _check(lib().vasmg_setup_phases(self._h, None, 0, C.byref(n)))
        buf = (SetupPhase * max(n.value, 1))()
        _check(lib().vasmg_setup_phases(self._h, buf, n.value, C.byref(n)))
        return [(buf[i].name.decode(), buf[i].ms) for i in range(n.value)]

    # -- single-step device entry points -----------------------------------
    def _level_shape(self, level):
        nl, _, _ = self.hierarchy_info()
        if not 0 <= level < nl:
            raise ValueError(f"level {level} out of range [0, {nl})")
        return (self.level_info(level)["n_vertices"], self.dim)

    def spmv_device(self, level, precision, d_x, d_y, stream=None):
        sh = self._level_shape(level)
        _check_tensor(d_x, sh, "d_x", self.device)
        _check_tensor(d_y, sh, "d_y", self.device)
        _check(lib().vasmg_spmv_device(self._h, level, precision, _ptr(d_x), _ptr(d_y),
                                       _stream_ptr(stream)))

    def gs_sweep_device(self, level, precision, backward, d_b, d_x, stream=None):
        sh = self._level_shape(level)
        _check_tensor(d_b, sh, "d_b", self.device)
        _check_tensor(d_x, sh, "d_x", self.device)
        _check(lib().vasmg_gs_sweep_device(self._h, level, precision, int(backward), _ptr(d_b),
                                           _ptr(d_x), _stream_ptr(stream)))

    def restrict_device(self, level, precision, d_r, d_bc, stream=None):
        _check_tensor(d_r, self._level_shape(level), "d_r", self.device)
        _check_tensor(d_bc, self._level_shape(level + 1), "d_bc", self.device)
        _check(lib().vasmg_restrict_device(self._h, level, precision, _ptr(d_r), _ptr(d_bc),
                                           _stream_ptr(stream)))

    def prolong_device(self, level, precision, d_e, d_x, stream=None):
        _check_tensor(d_e, self._level_shape(level + 1), "d_e", self.device)
        _check_tensor(d_x, self._level_shape(level), "d_x", self.device)
        _check(lib().vasmg_prolong_device(self._h, level, precision, _ptr(d_e), _ptr(d_x),
                                          _stream_ptr(stream)))

    def profile_iteration(self, reps: int = 3, stream=None):
        """Per-phase device time and algorithmic bytes of one PCG iteration."""
        out = (PhaseStat * 128)()
        n = C.c_int32()
        _check(lib().vasmg_profile_iteration(self._h, reps, _stream_ptr(stream), out, 128,
                                             C.byref(n)))
        return [dict(name=o.name.decode(), level=o.level, launches=o.launches, ms=o.ms,
                     bytes=o.bytes) for o in out[:n.value]]

    def apply_precond_device(self, d_r, d_z, stream=None):
        sh = self._level_shape(0)
        _check_tensor(d_r, sh, "d_r", self.device)
        _check_tensor(d_z, sh, "d_z", self.device)
        _check(lib().vasmg_apply_precond_device(self._h, _ptr(d_r), _ptr(d_z),
                                                _stream_ptr(stream)))


class PackedSolver(Solver):
    """Owns a packed handle (vasmg_pack): several small problems solved as one,
    each with its own PCG recurrence. `parts` are Solver objects (host-only or
    uploaded); they stay valid and owned by the caller."""

    def __init__(self, parts, upload: bool = True):
        if not parts:
            raise ValueError("nothing to pack")
        arr = (C.c_void_p * len(parts))(*[p.handle.value for p in parts])
        h = C.c_void_p()
        _check(lib().vasmg_pack(arr, len(parts), C.byref(h)))
        self._h = h
        self._arrays = None
        self.dim = parts[0].dim
        self.options = parts[0].options
        n = C.c_int32()
        offs = np.zeros(len(parts) + 1, dtype=np.int64)
        _check(lib().vasmg_packed_info(h, C.byref(n), _ptr(offs)))
        self.n_parts = n.value
        self.offsets = offs
        self.n_vertices = int(offs[-1])
        self.device = None
        if upload:
            _check(lib().vasmg_upload(h, None))
            import torch
            self.device = torch.cuda.current_device()

    def solve_packed(self, rhs_list, rtol: float = 1e-6, check: bool = True):
        """Host arrays [n_vertices_i, dim], one per part -> ([x_i], [info_i])."""
        if len(rhs_list) != self.n_parts:
            raise ValueError(f"expected {self.n_parts} right-hand sides")
        R = np.concatenate([np.ascontiguousarray(r, dtype=np.float64).reshape(-1, self.dim)
                            for r in rhs_list])
        if R.shape[0] != self.n_vertices:
            raise ValueError("right-hand sides do not match the parts' vertex counts")
        X = np.zeros_like(R)
        infos = (SolveInfo * self.n_parts)()
        st = lib().vasmg_solve_packed(self._h, _ptr(R), _ptr(X), rtol, infos)
        if check and st not in (OK, ENOTCONV):
            _check(st)
        out = [i.as_dict() for i in infos]      # "status": each part's own
        o = self.offsets
        return [X[o[i]:o[i + 1]].copy() for i in range(self.n_parts)], out

    def solve_packed_device(self, d_rhs, d_x, rtol: float = 1e-6, stream=None, check: bool = True):
        """Packed torch FP64 device tensors [sum n_vertices_i, dim] -> [info_i]."""
        shape = (self.n_vertices, self.dim)
        _check_tensor(d_rhs, shape, "d_rhs", self.device)
        _check_tensor(d_x, shape, "d_x", self.device)
        infos = (SolveInfo * self.n_parts)()
        st = lib().vasmg_solve_packed_device(self._h, _ptr(d_rhs), _ptr(d_x), rtol,
                                             _stream_ptr(stream), infos)
        if check and st not in (OK, ENOTCONV):
            _check(st)
        return [i.as_dict() for i in infos]      # "status": each part's own


class Server:
    """Continuous-batching solve server (vasmg_server_*): requests are set up on
    host threads, admitted to device slots by HBM footprint, solved on the
    slots' own streams, and collected with wait()."""

    def __init__(self, slots: int = 4, setup_workers: int = 4, hbm_budget_bytes: int = 0,
                 pack_max_dofs: int = 0, pack_max_parts: int = 16, pack_wait_ms: int = 0,
                 host_setup_max_dofs=None, **opts):
        """host_setup_max_dofs: (2D, 3D) DOF limits up to which a request is set
        up on the host even with setup_device = 1; None: the library's defaults."""
        cfg = ServerConfig()
        _check(lib().vasmg_server_default_config(C.byref(cfg)))
        cfg.slots, cfg.setup_workers, cfg.hbm_budget_bytes = slots, setup_workers, hbm_budget_bytes
        cfg.pack_max_dofs, cfg.pack_max_parts = pack_max_dofs, pack_max_parts
        cfg.pack_wait_ms = pack_wait_ms
        if host_setup_max_dofs is not None:
            cfg.host_setup_max_dofs_2d, cfg.host_setup_max_dofs_3d = host_setup_max_dofs
        for k, v in opts.items():
            setattr(cfg.options, k, v)
        h = C.c_void_p()
        _check(lib().vasmg_server_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self._shapes = {}

    def submit(self, mesh, rhs, rtol: float = 1e-6) -> int:
        coords = np.ascontiguousarray(mesh.coords, dtype=np.float64)
        elems = np.ascontiguousarray(mesh.elems, dtype=np.int32)
        nv, dim = coords.shape
        ne = elems.shape[0]
        E = np.ascontiguousarray(np.broadcast_to(np.asarray(mesh.E, dtype=np.float64), (ne,)))
        nu = np.ascontiguousarray(np.broadcast_to(np.asarray(mesh.nu, dtype=np.float64), (ne,)))
        fixed = np.ascontiguousarray(mesh.fixed, dtype=np.uint8).reshape(nv, dim)
        F = np.ascontiguousarray(rhs, dtype=np.float64).reshape(nv, dim)
        m = Mesh(dim, nv, _ptr(coords), ne, _ptr(elems), _ptr(E), _ptr(nu), _ptr(fixed))
        rid = C.c_int64()
        _check(lib().vasmg_server_submit(self._h, C.byref(m), _ptr(F), rtol, C.byref(rid)))
        self._shapes[rid.value] = (nv, dim)     # the library copied every input
        return rid.value

    def wait(self, rid: int):
        """(x [n_vertices, dim], result dict) of request rid; x is None on failure."""
        nv, dim = self._shapes.pop(rid)
        x = np.zeros((nv, dim))
        res = RequestResult()
        st = lib().vasmg_server_wait(self._h, rid, _ptr(x), C.byref(res))
        return (x if st == OK else None), res.as_dict()

    def stats(self) -> dict:
        c = ServerCounters()
        _check(lib().vasmg_server_stats(self._h, C.byref(c)))
        return c.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().vasmg_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_galerkin_window(cols: int) -> None:
    """Test hook: caps the columns of one symbolic pass of the device Galerkin
    product (0 = the LDS maximum) for setups that start afterwards."""
    _check(lib().vasmg_set_galerkin_window(int(cols)))
