"""ctypes declarations mirroring include/gabp.h and argument marshalling.

Device arrays are torch tensors on the GPU; their ``data_ptr()`` is passed as
the C pointer.  The HIP stream is torch's current stream unless one is given.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgabp.so")

GABP_OK = 0
GABP_NOT_CONVERGED = 1
GABP_ERR_ARG = -1
GABP_ERR_NOT_SYMMETRIC = -2
GABP_ERR_ZERO_DIAG = -3
GABP_ERR_BREAKDOWN = -4
GABP_ERR_DIVERGED = -5
GABP_ERR_HIP = -6
GABP_ERR_NOMEM = -7
GABP_ERR_UNSUPPORTED = -8
GABP_LAYOUT_PAIR = 0
GABP_LAYOUT_GATHER = 1
GABP_SCHEDULE_SYNC = 0
GABP_SCHEDULE_COLORED = 1
GABP_BATCH_BIPARTITE = 0
GABP_BATCH_DENSE = 1
GABP_BATCH_CSR = 2
GABP_ACCEL_NONE = 0
GABP_ACCEL_AITKEN = 1
GABP_ACCEL_STEFFENSEN = 2

_NAMES = {v: k for k, v in dict(globals()).items()
          if k.startswith("GABP_")
          and not k.startswith(("GABP_LAYOUT", "GABP_BATCH", "GABP_SCHEDULE"))
          and isinstance(v, int)}


def status_name(code: int) -> str:
    return _NAMES.get(int(code), f"UNKNOWN({code})")


class GabpError(RuntimeError):
    def __init__(self, where: str, code: int):
        super().__init__(f"{where} failed: {status_name(code)}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
# torch ships its own HIP runtime under the same soname as the system one that
# libgabp.so is linked against.  Loading torch first makes the library bind to
# that same runtime; loading the library first would put two runtimes in the
# process and the library would then see no device.
import torch  # noqa: E402,F401

lib = C.CDLL(LIB_PATH)


class _Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class _Rect(C.Structure):
    _fields_ = [("m", C.c_int32), ("k", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("msg_fp32", C.c_int32), ("tol", C.c_double), ("max_sweeps", C.c_int32),
                ("check_every", C.c_int32), ("damping", C.c_double), ("inner_tol", C.c_double),
                ("max_restarts", C.c_int32), ("group", C.c_int32), ("layout", C.c_int32),
                ("grid_blocks", C.c_int32), ("freeze", C.c_int32), ("batch_waves", C.c_int32),
                ("freeze_tol", C.c_double), ("adapt_damping", C.c_int32),
                ("schedule", C.c_int32), ("col_blocks", C.c_int32), ("accel", C.c_int32),
                ("accel_stride", C.c_int32), ("accel_cycle", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("sweeps", C.c_int32), ("frozen_sweeps", C.c_int32),
                ("restarts", C.c_int32),
                ("checks", C.c_int32), ("rel_residual", C.c_double),
                ("residual_per_eq", C.c_double), ("seconds", C.c_double),
                ("sweep_ms", C.c_double), ("frozen_sweep_ms", C.c_double), ("edges", C.c_int64),
                ("edge_updates_per_s", C.c_double), ("damping", C.c_double),
                ("batch_waves", C.c_int32), ("batch_groups", C.c_int32),
                ("warm_start", C.c_int32), ("sweep_launches", C.c_int32),
                ("warm_rel0", C.c_double), ("mean_sweeps", C.c_double),
                ("mean_frozen_sweeps", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp, _i32 = C.c_void_p, C.c_int32
_sig = {
    "gabp_default_opts": (None, [C.POINTER(Opts)]),
    "gabp_solve": (C.c_int, [C.POINTER(_Csr), _vp, _vp, _vp, C.POINTER(Opts), C.POINTER(Stats), _vp]),
    "gabp_residual": (C.c_int, [C.POINTER(_Csr), _vp, _vp, _vp, C.POINTER(C.c_double), _vp]),
    "gabp_residual_noalloc": (C.c_int, [C.POINTER(_Csr), _vp, _vp, _vp, C.POINTER(C.c_double),
                                        _vp]),
    "gabp_plan_create": (C.c_int, [C.POINTER(_Csr), C.POINTER(Opts), C.POINTER(_vp), _vp]),
    "gabp_plan_colors": (C.c_int, [_vp, _vp, C.POINTER(C.c_int32), _vp]),
    "gabp_plan_workspace_bytes": (C.c_int, [_vp, C.POINTER(C.c_size_t)]),
    "gabp_plan_create_lsq": (C.c_int, [C.POINTER(_Rect), C.c_double, C.POINTER(Opts),
                                       C.POINTER(_vp), _vp]),
    "gabp_plan_solve_lsq": (C.c_int, [_vp, _vp, _vp, C.POINTER(Stats), _vp]),
    "gabp_solve_lsq": (C.c_int, [C.POINTER(_Rect), C.c_double, _vp, _vp, C.POINTER(Opts),
                                 C.POINTER(Stats), _vp]),
    "gabp_plan_residual_lsq": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double), _vp]),
    "gabp_plan_destroy": (C.c_int, [_vp]),
    "gabp_plan_solve": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(Stats), _vp]),
    "gabp_plan_reset": (C.c_int, [_vp, _vp, _vp]),
    "gabp_plan_sweeps": (C.c_int, [_vp, _i32, _vp]),
    "gabp_plan_marginals": (C.c_int, [_vp, _vp, _vp, _vp]),
    "gabp_plan_get_messages": (C.c_int, [_vp, _vp, _vp, _vp]),
    "gabp_plan_set_messages": (C.c_int, [_vp, _vp, _vp, _vp]),
    "gabp_version": (C.c_char_p, []),
    "gabp_plan_create_grid": (C.c_int, [C.c_void_p, C.POINTER(Opts), C.POINTER(_vp), _vp]),
    "gabp_solve_grid": (C.c_int, [C.c_void_p, _vp, _vp, _vp, C.POINTER(Opts), C.POINTER(Stats), _vp]),
    "gabp_residual_grid": (C.c_int, [C.c_void_p, _vp, _vp, _vp, C.POINTER(C.c_double), _vp]),
    "gabp_plan_create_batched": (C.c_int, [C.c_void_p, C.POINTER(Opts), C.POINTER(_vp), _vp]),
    "gabp_plan_solve_batched": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(Stats), _vp]),
    "gabp_solve_batched": (C.c_int, [C.c_void_p, _vp, _vp, C.POINTER(Opts), _vp, C.POINTER(Stats),
                                     _vp]),
    "gabp_model_create": (C.c_int, [C.c_uint64, C.POINTER(_vp), _vp]),
    "gabp_model_destroy": (C.c_int, [_vp]),
    "gabp_model_get_params": (C.c_int, [_vp, _vp, _vp]),
    "gabp_model_set_params": (C.c_int, [_vp, _vp, _vp]),
    "gabp_model_forward": (C.c_int, [_vp, _vp, C.c_int64, _vp, _vp]),
    "gabp_model_grad": (C.c_int, [_vp, _vp, _vp, C.c_int64, _vp, C.POINTER(C.c_double), _vp]),
    "gabp_model_train_step": (C.c_int, [_vp, _vp, _vp, C.c_int64, C.c_double,
                                        C.POINTER(C.c_double), _vp]),
    "gabp_model_grid_features": (C.c_int, [C.c_void_p, _vp, _vp, C.c_int64, _vp, _vp]),
    "gabp_model_grid_targets": (C.c_int, [C.c_void_p, _vp, _vp, _vp, C.c_int64, _vp, _vp]),
    "gabp_plan_solve_warm": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.POINTER(Stats), _vp]),
    "gabp_plan_solve_coarse": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(Stats), _vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _check_f64(t, n, name):
    import torch
    if t is None:
        return
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: expected a contiguous float64 CUDA tensor of {n} elements")


@dataclass
class DeviceCSR:
    """Full symmetric CSR matrix resident on the GPU (int64 row_ptr, int32 col,
    float64 val), and the gabp_csr view of it."""
    n: int
    row_ptr: object
    col: object
    val: object

    @classmethod
    def from_host(cls, m, device="cuda"):
        import numpy as np
        import torch
        rp = torch.from_numpy(np.ascontiguousarray(m.row_ptr, dtype=np.int64)).to(device)
        col = torch.from_numpy(np.ascontiguousarray(m.col, dtype=np.int32)).to(device)
        val = torch.from_numpy(np.ascontiguousarray(m.val, dtype=np.float64)).to(device)
        return cls(int(m.n), rp, col, val)

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def c(self) -> _Csr:
        return _Csr(self.n, self.nnz, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.val))


@dataclass
class DeviceRect:
    """Any sparse m x k matrix S resident on the GPU in CSR form (int64
    row_ptr, int32 col, float64 val), for the section VII least-squares plans."""
    m: int
    k: int
    row_ptr: object
    col: object
    val: object

    @classmethod
    def from_host(cls, row_ptr, col, val, shape, device="cuda"):
        import numpy as np
        import torch
        rp = torch.from_numpy(np.ascontiguousarray(row_ptr, dtype=np.int64)).to(device)
        cc = torch.from_numpy(np.ascontiguousarray(col, dtype=np.int32)).to(device)
        vv = torch.from_numpy(np.ascontiguousarray(val, dtype=np.float64)).to(device)
        return cls(int(shape[0]), int(shape[1]), rp, cc, vv)

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def c(self) -> _Rect:
        return _Rect(self.m, self.k, self.nnz, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.val))


@dataclass
class _LsqShape:
    """Array lengths of an lsq plan's assembled system (unknowns x then z)."""
    S: DeviceRect

    @property
    def n(self) -> int:
        return self.S.k + self.S.m

    @property
    def nnz(self) -> int:
        return 2 * self.S.nnz + self.S.k + self.S.m


def gabp_default_opts(**overrides) -> Opts:
    o = Opts()
    lib.gabp_default_opts(C.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def gabp_version() -> str:
    return lib.gabp_version().decode()


def gabp_solve(A: DeviceCSR, b, x, marg_prec=None, opts: Opts | None = None, stream=None):
    """Returns (status, Stats)."""
    _check_f64(b, A.n, "b"); _check_f64(x, A.n, "x"); _check_f64(marg_prec, A.n, "marg_prec")
    st = Stats()
    a = A.c()
    rc = lib.gabp_solve(C.byref(a), _ptr(b), _ptr(x), _ptr(marg_prec),
                        C.byref(opts) if opts is not None else None, C.byref(st), _stream(stream))
    return rc, st


def gabp_residual(A: DeviceCSR, b, x, r=None, stream=None):
    """Returns (status, ||b - A x|| / ||b||)."""
    _check_f64(b, A.n, "b"); _check_f64(x, A.n, "x"); _check_f64(r, A.n, "r")
    rel = C.c_double(0.0)
    a = A.c()
    rc = lib.gabp_residual(C.byref(a), _ptr(b), _ptr(x), _ptr(r), C.byref(rel), _stream(stream))
    return rc, rel.value


def gabp_residual_noalloc(A: DeviceCSR, b, x, r=None, stream=None):
    """gabp_residual through the allocation-free entry point: (status, rel)."""
    _check_f64(b, A.n, "b"); _check_f64(x, A.n, "x"); _check_f64(r, A.n, "r")
    rel = C.c_double(0.0)
    a = A.c()
    rc = lib.gabp_residual_noalloc(C.byref(a), _ptr(b), _ptr(x), _ptr(r), C.byref(rel),
                                   _stream(stream))
    return rc, rel.value


def gabp_plan_create(A: DeviceCSR, opts: Opts | None = None, stream=None):
    """Returns (status, plan handle).  The handle keeps A alive."""
    h = C.c_void_p()
    a = A.c()
    rc = lib.gabp_plan_create(C.byref(a), C.byref(opts) if opts is not None else None,
                              C.byref(h), _stream(stream))
    return rc, (_PlanHandle(h.value, A) if rc == GABP_OK else None)


class _PlanHandle:
    def __init__(self, ptr, A):
        self.ptr, self.A = ptr, A


def gabp_plan_destroy(plan) -> int:
    if plan is None or plan.ptr is None:
        return GABP_ERR_ARG
    rc = lib.gabp_plan_destroy(plan.ptr)
    plan.ptr = None
    return rc


def _lens(plan):
    """(right-hand side, unknowns, node values) lengths of a plan's arrays."""
    A = plan.A
    if isinstance(A, DeviceBatch):
        return A.rhslen, A.xlen, A.nodes
    return A.n, A.n, A.n


def gabp_plan_solve(plan, b, x, marg_prec=None, stream=None):
    nb, nx, _ = _lens(plan)
    _check_f64(b, nb, "b"); _check_f64(x, nx, "x"); _check_f64(marg_prec, nx, "marg_prec")
    st = Stats()
    rc = lib.gabp_plan_solve(plan.ptr, _ptr(b), _ptr(x), _ptr(marg_prec), C.byref(st),
                             _stream(stream))
    return rc, st


def gabp_plan_reset(plan, b, stream=None) -> int:
    _check_f64(b, _lens(plan)[0], "b")
    return lib.gabp_plan_reset(plan.ptr, _ptr(b), _stream(stream))


def gabp_plan_sweeps(plan, count: int, stream=None) -> int:
    return lib.gabp_plan_sweeps(plan.ptr, int(count), _stream(stream))


def gabp_plan_marginals(plan, mean, prec=None, stream=None) -> int:
    nn = _lens(plan)[2]
    _check_f64(mean, nn, "mean"); _check_f64(prec, nn, "prec")
    return lib.gabp_plan_marginals(plan.ptr, _ptr(mean), _ptr(prec), _stream(stream))


def gabp_plan_get_messages(plan, P, h, stream=None) -> int:
    _check_f64(P, plan.A.nnz, "P"); _check_f64(h, plan.A.nnz, "h")
    return lib.gabp_plan_get_messages(plan.ptr, _ptr(P), _ptr(h), _stream(stream))


def gabp_plan_set_messages(plan, P, h, stream=None) -> int:
    _check_f64(P, plan.A.nnz, "P"); _check_f64(h, plan.A.nnz, "h")
    return lib.gabp_plan_set_messages(plan.ptr, _ptr(P), _ptr(h), _stream(stream))


def gabp_plan_colors(plan, stream=None):
    """Returns (status, int32 CUDA tensor of node colours or None, colour count)."""
    import torch
    n = _lens(plan)[2]
    colors = torch.empty(n, dtype=torch.int32, device="cuda")
    nc = C.c_int32(0)
    rc = lib.gabp_plan_colors(plan.ptr, _ptr(colors), C.byref(nc), _stream(stream))
    return rc, (colors if rc == GABP_OK else None), nc.value


def gabp_plan_workspace_bytes(plan):
    """Returns (status, bytes of device memory the plan holds)."""
    nb = C.c_size_t(0)
    rc = lib.gabp_plan_workspace_bytes(plan.ptr, C.byref(nb))
    return rc, nb.value


def gabp_plan_create_lsq(S: DeviceRect, psi: float, opts: Opts | None = None, stream=None):
    """Returns (status, plan handle) of the section VII system of S."""
    h = C.c_void_p()
    a = S.c()
    rc = lib.gabp_plan_create_lsq(C.byref(a), float(psi),
                                  C.byref(opts) if opts is not None else None, C.byref(h),
                                  _stream(stream))
    return rc, (_PlanHandle(h.value, _LsqShape(S)) if rc == GABP_OK else None)


def gabp_plan_solve_lsq(plan, y, x, stream=None):
    S = plan.A.S
    _check_f64(y, S.m, "y"); _check_f64(x, S.k, "x")
    st = Stats()
    rc = lib.gabp_plan_solve_lsq(plan.ptr, _ptr(y), _ptr(x), C.byref(st), _stream(stream))
    return rc, st


def gabp_solve_lsq(S: DeviceRect, psi: float, y, x, opts: Opts | None = None, stream=None):
    _check_f64(y, S.m, "y"); _check_f64(x, S.k, "x")
    st = Stats()
    a = S.c()
    rc = lib.gabp_solve_lsq(C.byref(a), float(psi), _ptr(y), _ptr(x),
                            C.byref(opts) if opts is not None else None, C.byref(st),
                            _stream(stream))
    return rc, st


def gabp_plan_residual_lsq(plan, y, x, r=None, stream=None):
    """Returns (status, ||S^T y - (S^T S + psi I) x|| / ||S^T y||)."""
    S = plan.A.S
    _check_f64(y, S.m, "y"); _check_f64(x, S.k, "x"); _check_f64(r, S.k, "r")
    rel = C.c_double(0.0)
    rc = lib.gabp_plan_residual_lsq(plan.ptr, _ptr(y), _ptr(x), _ptr(r), C.byref(rel),
                                    _stream(stream))
    return rc, rel.value


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("batch", C.c_int32),
                ("diag", C.c_void_p), ("diag_value", C.c_double), ("cx", C.c_void_p),
                ("cy", C.c_void_p), ("cz", C.c_void_p), ("off_value", C.c_double)]


@dataclass
class DeviceGrid:
    """Stack of `batch` grids (nx x ny x nz each, natural node order) with the
    5/7-point operator: constant (diag_value, off_value) or per-node diagonal
    and per-face couplings cx, cy, cz (float64 CUDA tensors of batch*n)."""
    nx: int
    ny: int
    nz: int = 1
    batch: int = 1
    diag: object = None
    diag_value: float = 0.0
    cx: object = None
    cy: object = None
    cz: object = None
    off_value: float = 0.0

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz * self.batch

    @property
    def nnz(self) -> int:  # message slots of a grid plan: 6 directions per node
        return 6 * self.n

    def c(self) -> _Grid:
        return _Grid(self.nx, self.ny, self.nz, self.batch, _ptr(self.diag), self.diag_value,
                     _ptr(self.cx), _ptr(self.cy), _ptr(self.cz), self.off_value)


def gabp_plan_create_grid(A: DeviceGrid, opts: Opts | None = None, stream=None):
    h = C.c_void_p()
    a = A.c()
    rc = lib.gabp_plan_create_grid(C.byref(a), C.byref(opts) if opts is not None else None,
                                   C.byref(h), _stream(stream))
    return rc, (_PlanHandle(h.value, A) if rc == GABP_OK else None)


def gabp_solve_grid(A: DeviceGrid, b, x, marg_prec=None, opts: Opts | None = None, stream=None):
    _check_f64(b, A.n, "b"); _check_f64(x, A.n, "x"); _check_f64(marg_prec, A.n, "marg_prec")
    st = Stats()
    a = A.c()
    rc = lib.gabp_solve_grid(C.byref(a), _ptr(b), _ptr(x), _ptr(marg_prec),
                             C.byref(opts) if opts is not None else None, C.byref(st), _stream(stream))
    return rc, st


def gabp_residual_grid(A: DeviceGrid, b, x, r=None, stream=None):
    _check_f64(b, A.n, "b"); _check_f64(x, A.n, "x"); _check_f64(r, A.n, "r")
    rel = C.c_double(0.0)
    a = A.c()
    rc = lib.gabp_residual_grid(C.byref(a), _ptr(b), _ptr(x), _ptr(r), C.byref(rel), _stream(stream))
    return rc, rel.value


class _Batch(C.Structure):
    _fields_ = [("kind", C.c_int32), ("count", C.c_int32), ("k", C.c_void_p), ("m", C.c_void_p),
                ("sigma2", C.c_void_p), ("mat", C.c_void_p), ("csr", C.c_void_p)]


@dataclass
class DeviceBatch:
    """A batch of instances for gabp_solve_batched: per-instance sizes and
    noise variances on the host, the matrices on the device.  Bipartite: S_t
    (N_t x K_t, packed row-major float64), right-hand sides y_t; dense: A_t
    (K_t x K_t), right-hand sides b_t; CSR: the instances as the diagonal
    blocks of one sparse symmetric matrix (a DeviceCSR), right-hand sides and
    solutions packed like its rows."""
    kind: int
    k: object
    m: object = None
    sigma2: object = None
    mat: object = None
    csr: object = None

    @classmethod
    def sparse(cls, K, A, device="cuda"):
        """K: rows of each instance; A: host CSR (workloads.CSR) of the
        block-diagonal matrix, or a DeviceCSR."""
        import numpy as np
        K = np.ascontiguousarray(K, dtype=np.int32)
        if not isinstance(A, DeviceCSR):
            A = DeviceCSR.from_host(A, device)
        return cls(GABP_BATCH_CSR, K, None, None, None, A)

    @classmethod
    def bipartite(cls, K, N, sigma2, S, device="cuda"):
        import numpy as np
        import torch
        K = np.ascontiguousarray(K, dtype=np.int32)
        N = np.ascontiguousarray(N, dtype=np.int32)
        s2 = np.ascontiguousarray(sigma2, dtype=np.float64)
        mat = torch.from_numpy(np.ascontiguousarray(S, dtype=np.float64)).to(device)
        return cls(GABP_BATCH_BIPARTITE, K, N, s2, mat)

    @classmethod
    def dense(cls, K, A, device="cuda"):
        import numpy as np
        import torch
        K = np.ascontiguousarray(K, dtype=np.int32)
        mat = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float64)).to(device)
        return cls(GABP_BATCH_DENSE, K, None, None, mat)

    @property
    def count(self) -> int:
        return int(len(self.k))

    @property
    def xlen(self) -> int:
        return int(sum(int(v) for v in self.k))

    @property
    def n(self) -> int:  # rows of the batch (trajectory calls)
        return self.nodes

    @property
    def nnz(self) -> int:  # CSR kind: stored entries (get/set_messages)
        return self.csr.nnz if self.csr is not None else 0

    @property
    def rhslen(self) -> int:
        return int(sum(int(v) for v in (self.m if self.kind == GABP_BATCH_BIPARTITE else self.k)))

    @property
    def nodes(self) -> int:
        extra = sum(int(v) for v in self.m) if self.kind == GABP_BATCH_BIPARTITE else 0
        return self.xlen + int(extra)

    def c(self) -> _Batch:
        def p(a):
            return None if a is None else a.ctypes.data_as(C.c_void_p)
        if self.csr is not None:
            self._csr_c = self.csr.c()  # kept alive with the batch struct
            cp = C.cast(C.pointer(self._csr_c), C.c_void_p)
        else:
            cp = None
        return _Batch(self.kind, self.count, p(self.k), p(self.m), p(self.sigma2), _ptr(self.mat), cp)


def _batch_stats(per_instance: bool, count: int):
    return (Stats * max(1, count))() if per_instance else None


def gabp_plan_create_batched(B: DeviceBatch, opts: Opts | None = None, stream=None):
    h = C.c_void_p()
    b = B.c()
    rc = lib.gabp_plan_create_batched(C.byref(b), C.byref(opts) if opts is not None else None,
                                      C.byref(h), _stream(stream))
    return rc, (_PlanHandle(h.value, B) if rc == GABP_OK else None)


def gabp_plan_solve_batched(plan, b, x, per_instance: bool = True, stream=None):
    """Returns (status, per-instance Stats list or None, summary Stats)."""
    B = plan.A
    _check_f64(b, B.rhslen, "b"); _check_f64(x, B.xlen, "x")
    per = _batch_stats(per_instance, B.count)
    summary = Stats()
    rc = lib.gabp_plan_solve_batched(plan.ptr, _ptr(b), _ptr(x), per, C.byref(summary),
                                     _stream(stream))
    return rc, (list(per)[:B.count] if per is not None else None), summary


def gabp_solve_batched(B: DeviceBatch, b, x, opts: Opts | None = None, per_instance: bool = True,
                       stream=None):
    """Returns (status, per-instance Stats list or None, summary Stats)."""
    _check_f64(b, B.rhslen, "b"); _check_f64(x, B.xlen, "x")
    per = _batch_stats(per_instance, B.count)
    summary = Stats()
    bb = B.c()
    rc = lib.gabp_solve_batched(C.byref(bb), _ptr(b), _ptr(x),
                                C.byref(opts) if opts is not None else None, per,
                                C.byref(summary), _stream(stream))
    return rc, (list(per)[:B.count] if per is not None else None), summary


# ---------------------------------------------------------------------------
# learned warm start (grid plans)
# ---------------------------------------------------------------------------
GABP_MODEL_INPUTS = 8
GABP_MODEL_OUTPUTS = 12
GABP_MODEL_PARAMS = 5516


def _check_f32(t, n, name):
    import torch
    if t is None:
        return
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: expected a contiguous float32 CUDA tensor of {n} elements")


class Model:
    """Handle of a gabp_model (the warm-start network on the device)."""

    def __init__(self, ptr):
        self.ptr = ptr

    def __del__(self):
        if getattr(self, "ptr", None):
            lib.gabp_model_destroy(self.ptr)
            self.ptr = None


def gabp_model_create(seed: int = 0, stream=None):
    h = C.c_void_p()
    rc = lib.gabp_model_create(int(seed), C.byref(h), _stream(stream))
    return rc, (Model(h.value) if rc == GABP_OK else None)


def gabp_model_get_params(model: Model, stream=None):
    import numpy as np
    out = np.empty(GABP_MODEL_PARAMS, dtype=np.float32)
    rc = lib.gabp_model_get_params(model.ptr, out.ctypes.data_as(C.c_void_p), _stream(stream))
    return rc, out


def gabp_model_set_params(model: Model, params, stream=None) -> int:
    import numpy as np
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.size != GABP_MODEL_PARAMS:
        raise ValueError("params: expected 5516 values")
    return lib.gabp_model_set_params(model.ptr, p.ctypes.data_as(C.c_void_p), _stream(stream))


def gabp_model_forward(model: Model, U, out, stream=None) -> int:
    n = U.numel() // GABP_MODEL_INPUTS
    _check_f32(U, n * GABP_MODEL_INPUTS, "U"); _check_f32(out, n * GABP_MODEL_OUTPUTS, "out")
    return lib.gabp_model_forward(model.ptr, _ptr(U), n, _ptr(out), _stream(stream))


def gabp_model_grad(model: Model, U, T, grad=None, stream=None):
    """Returns (status, loss); the gradient goes to `grad` (float32 CUDA, 5516)."""
    n = U.numel() // GABP_MODEL_INPUTS
    _check_f32(U, n * GABP_MODEL_INPUTS, "U"); _check_f32(T, n * GABP_MODEL_OUTPUTS, "T")
    _check_f32(grad, GABP_MODEL_PARAMS, "grad")
    loss = C.c_double(0.0)
    rc = lib.gabp_model_grad(model.ptr, _ptr(U), _ptr(T), n, _ptr(grad), C.byref(loss),
                             _stream(stream))
    return rc, loss.value


def gabp_model_train_step(model: Model, U, T, lr: float, stream=None):
    """One Adam step; returns (status, loss before the step)."""
    n = U.numel() // GABP_MODEL_INPUTS
    _check_f32(U, n * GABP_MODEL_INPUTS, "U"); _check_f32(T, n * GABP_MODEL_OUTPUTS, "T")
    loss = C.c_double(0.0)
    rc = lib.gabp_model_train_step(model.ptr, _ptr(U), _ptr(T), n, float(lr), C.byref(loss),
                                   _stream(stream))
    return rc, loss.value


def _check_i64(t, n, name):
    import torch
    if t is None:
        return
    if t.dtype != torch.int64 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name}: expected a contiguous int64 CUDA tensor of {n} elements")


def gabp_model_grid_features(A: DeviceGrid, b, U, nodes=None, stream=None) -> int:
    count = A.n if nodes is None else nodes.numel()
    _check_f64(b, A.n, "b"); _check_f32(U, count * GABP_MODEL_INPUTS, "U")
    _check_i64(nodes, count, "nodes")
    a = A.c()
    return lib.gabp_model_grid_features(C.byref(a), _ptr(b), _ptr(nodes), count, _ptr(U),
                                        _stream(stream))


def gabp_model_grid_targets(A: DeviceGrid, P, h, T, nodes=None, stream=None) -> int:
    count = A.n if nodes is None else nodes.numel()
    _check_f64(P, 6 * A.n, "P"); _check_f64(h, 6 * A.n, "h")
    _check_f32(T, count * GABP_MODEL_OUTPUTS, "T"); _check_i64(nodes, count, "nodes")
    a = A.c()
    return lib.gabp_model_grid_targets(C.byref(a), _ptr(P), _ptr(h), _ptr(nodes), count, _ptr(T),
                                       _stream(stream))


def gabp_plan_solve_warm(plan, model: Model, b, x, marg_prec=None, stream=None):
    nb, nx, _ = _lens(plan)
    _check_f64(b, nb, "b"); _check_f64(x, nx, "x"); _check_f64(marg_prec, nx, "marg_prec")
    st = Stats()
    rc = lib.gabp_plan_solve_warm(plan.ptr, model.ptr, _ptr(b), _ptr(x), _ptr(marg_prec),
                                  C.byref(st), _stream(stream))
    return rc, st


def gabp_plan_solve_coarse(plan, b, x, marg_prec=None, stream=None):
    """Grid plans: the solve with coarse-grid predicted corrections.
    Returns (status, Stats)."""
    nb, nx, _ = _lens(plan)
    _check_f64(b, nb, "b"); _check_f64(x, nx, "x"); _check_f64(marg_prec, nx, "marg_prec")
    st = Stats()
    rc = lib.gabp_plan_solve_coarse(plan.ptr, _ptr(b), _ptr(x), _ptr(marg_prec), C.byref(st),
                                    _stream(stream))
    return rc, st
