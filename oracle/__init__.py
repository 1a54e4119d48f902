"""FP64 CPU oracle for GaBP -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path
(``paper_0810_1119_amd``) and never imports it.

The arithmetic lives in ``gabp_oracle.c`` (plain C, FP64, optional OpenMP over
rows); this module compiles it with gcc, loads it with ctypes and adds thin
array wrappers plus the section VII bipartite construction.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gabp_oracle.c")
_LIB = os.path.join(_HERE, "libgabp_oracle.so")

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_NOT_SYMMETRIC, ERR_ZERO_DIAG, ERR_BREAKDOWN, ERR_DIVERGED = -1, -2, -3, -4, -5
STOP_RESIDUAL, STOP_MESSAGES, STOP_MEANS = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (-O2, IEEE arithmetic, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("algorithm", C.c_int32), ("stop", C.c_int32), ("tol", C.c_double),
                ("max_rounds", C.c_int32), ("damping", C.c_double), ("nthreads", C.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = C.CDLL(build())
        vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        lib.orc_build_reverse.argtypes = [C.POINTER(_Csr), vp, vp]
        lib.orc_alg1_round.argtypes = [C.POINTER(_Csr), vp, vp, vp, vp, vp, vp, vp, f64, C.c_int]
        lib.orc_alg1_round.restype = i64
        lib.orc_alg2_round.argtypes = lib.orc_alg1_round.argtypes
        lib.orc_alg2_round.restype = i64
        lib.orc_alg2_color_round.argtypes = [C.POINTER(_Csr), vp, vp, vp, vp, vp, vp, C.c_int,
                                             f64, C.c_int]
        lib.orc_alg2_color_round.restype = i64
        lib.orc_marginals.argtypes = [C.POINTER(_Csr), vp, vp, vp, vp, vp, vp, vp, C.c_int]
        lib.orc_residual.argtypes = [C.POINTER(_Csr), vp, vp, vp]
        lib.orc_residual.restype = f64
        lib.orc_jacobi_variant_round.argtypes = [C.POINTER(_Csr), vp, vp, vp, vp, vp, vp]
        lib.orc_solve.argtypes = [C.POINTER(_Csr), vp, C.POINTER(_Opts), vp, vp, vp, vp,
                                  C.POINTER(i32), vp]
        lib.orc_refine_solve.argtypes = [C.POINTER(_Csr), vp, f64, f64, i32, i32, f64, i32,
                                         vp, vp, vp, C.POINTER(i32), C.POINTER(i32),
                                         C.POINTER(f64)]
        lib.orc_max_threads.restype = C.c_int
        lib.orc_residual_grid.argtypes = [i32, i32, i32, i32, vp, f64, vp, vp, vp, f64, vp, vp, vp]
        lib.orc_residual_grid.restype = f64
        lib.orc_aitken.argtypes = [i64, vp, vp, vp, vp]
        lib.orc_solve_aitken.argtypes = [C.POINTER(_Csr), vp, i32, f64, i32, f64, i32, vp,
                                         C.POINTER(i32)]
        lib.orc_solve_steffensen.argtypes = [C.POINTER(_Csr), vp, i32, i32, f64, i32, f64, i32,
                                             vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(f64)]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class Matrix:
    """Holds contiguous CSR arrays and the C view of them."""

    def __init__(self, m):
        self.n = int(m.n)
        self.row_ptr = np.ascontiguousarray(m.row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(m.col, dtype=np.int32)
        self.val = np.ascontiguousarray(m.val, dtype=np.float64)
        self.nnz = int(self.row_ptr[-1])
        self.c = _Csr(self.n, _p(self.row_ptr), _p(self.col), _p(self.val))


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError("length mismatch")
    return a


def max_threads() -> int:
    return int(_load().orc_max_threads())


def reverse(m):
    """(status, rev[nnz], diag[n]) -- rev of a diagonal slot is -1."""
    M = Matrix(m)
    rev = np.empty(M.nnz, dtype=np.int64)
    diag = np.empty(M.n)
    st = _load().orc_build_reverse(C.byref(M.c), _p(rev), _p(diag))
    return st, rev, diag


def is_proper_colouring(m, colors) -> bool:
    """True when no off-diagonal nonzero joins two nodes of the same colour."""
    colors = np.asarray(colors)
    rows = np.repeat(np.arange(m.n), np.diff(np.asarray(m.row_ptr)))
    cols = np.asarray(m.col)
    off = rows != cols
    return bool(np.all(colors[rows[off]] != colors[cols[off]]))


class Rounds:
    """Round-by-round access for trajectory comparisons (P, mu per CSR slot).

    colors=None: the synchronous schedule of Algorithm 1 / 2 (one step = one
    round).  colors = a proper node colouring 0..C-1: the coloured schedule
    (one step = every class sending once, class 0 first)."""

    def __init__(self, m, b, algorithm: int = 2, damping: float = 0.0, nthreads: int = 0,
                 colors=None):
        self.M = Matrix(m)
        self.b = _f64(b, self.M.n)
        st, self.rev, self.diag = reverse(m)
        if st != OK:
            raise ValueError(f"oracle rejected the matrix: status {st}")
        self.algorithm, self.damping, self.nthreads = algorithm, damping, nthreads
        self.colors = None
        if colors is not None:
            if not is_proper_colouring(m, colors):
                raise ValueError("the colouring puts both ends of an edge in one class")
            self.colors = np.ascontiguousarray(colors, dtype=np.int8)
        self.P = np.zeros(self.M.nnz)
        self.Mu = np.zeros(self.M.nnz)
        self.zero_cavities = 0

    def step(self, count: int = 1):
        lib = _load()
        if self.colors is not None:
            ncol = int(self.colors.max()) + 1 if self.colors.size else 0
            for _ in range(count):
                for c in range(ncol):
                    self.zero_cavities += lib.orc_alg2_color_round(
                        C.byref(self.M.c), _p(self.b), _p(self.rev), _p(self.diag), _p(self.P),
                        _p(self.Mu), _p(self.colors), c, self.damping, self.nthreads)
            return self
        fn = lib.orc_alg1_round if self.algorithm == 1 else lib.orc_alg2_round
        for _ in range(count):
            P2, M2 = np.empty_like(self.P), np.empty_like(self.Mu)
            self.zero_cavities += fn(C.byref(self.M.c), _p(self.b), _p(self.rev), _p(self.diag),
                                     _p(self.P), _p(self.Mu), _p(P2), _p(M2),
                                     self.damping, self.nthreads)
            self.P, self.Mu = P2, M2
        return self

    def marginals(self):
        mean, prec = np.empty(self.M.n), np.empty(self.M.n)
        _load().orc_marginals(C.byref(self.M.c), _p(self.b), _p(self.rev), _p(self.diag),
                              _p(self.P), _p(self.Mu), _p(mean), _p(prec), self.nthreads)
        return mean, prec

    def information(self):
        """h = P * mu per slot (zero on the diagonal)."""
        return self.P * self.Mu


@dataclass
class Result:
    status: int
    x: np.ndarray
    prec: np.ndarray
    rounds: int
    trace: np.ndarray
    P: np.ndarray
    Mu: np.ndarray


def solve(m, b, algorithm=2, stop=STOP_RESIDUAL, tol=1e-10, max_rounds=10000,
          damping=0.0, nthreads=0, P0=None, Mu0=None) -> Result:
    """Synchronous GaBP from zero messages (Algorithm 1 step 1) or from P0/Mu0."""
    M = Matrix(m)
    b = _f64(b, M.n)
    P = np.zeros(M.nnz) if P0 is None else _f64(P0, M.nnz).copy()
    Mu = np.zeros(M.nnz) if Mu0 is None else _f64(Mu0, M.nnz).copy()
    x, prec = np.empty(M.n), np.empty(M.n)
    trace = np.full(max_rounds + 1, np.nan)
    rounds = C.c_int32(0)
    o = _Opts(algorithm, stop, tol, max_rounds, damping, nthreads)
    st = _load().orc_solve(C.byref(M.c), _p(b), C.byref(o), _p(P), _p(Mu), _p(x), _p(prec),
                           C.byref(rounds), _p(trace))
    t = int(rounds.value)
    return Result(st, x, prec, t, trace[:t + 1], P, Mu)


def refine_solve(m, b, tol=1e-8, inner_tol=1e-5, inner_max=100000, max_restarts=50,
                 damping=0.0, nthreads=0):
    """Refinement loop around GaBP (see orc_refine_solve).  Returns
    (status, x, rounds, restarts, rel_residual)."""
    M = Matrix(m)
    b = _f64(b, M.n)
    x = np.empty(M.n)
    P, Mu = np.zeros(M.nnz), np.zeros(M.nnz)
    rounds, restarts, rel = C.c_int32(0), C.c_int32(0), C.c_double(0)
    st = _load().orc_refine_solve(C.byref(M.c), _p(b), tol, inner_tol, inner_max, max_restarts,
                                  damping, nthreads, _p(x), _p(P), _p(Mu), C.byref(rounds),
                                  C.byref(restarts), C.byref(rel))
    return st, x, int(rounds.value), int(restarts.value), float(rel.value)


def aitken(x0, x1, x2):
    """Section IV-A, Aitken's method per component (see orc_aitken): y from
    three consecutive members of a sequence; a zero second difference keeps x2."""
    x0, x1, x2 = (np.ascontiguousarray(a, dtype=np.float64) for a in (x0, x1, x2))
    if not (x0.shape == x1.shape == x2.shape):
        raise ValueError("shape mismatch")
    y = np.empty_like(x0)
    _load().orc_aitken(x0.size, _p(x0), _p(x1), _p(x2), _p(y))
    return y


def solve_aitken(m, b, stride=2, tol=1e-10, max_rounds=100000, damping=0.0, nthreads=0):
    """Parallel GaBP + Aitken (orc_solve_aitken): returns (status, y, rounds)."""
    M = Matrix(m)
    b = _f64(b, M.n)
    y = np.empty(M.n)
    rounds = C.c_int32(0)
    st = _load().orc_solve_aitken(C.byref(M.c), _p(b), stride, tol, max_rounds, damping,
                                  nthreads, _p(y), C.byref(rounds))
    return st, y, int(rounds.value)


def solve_steffensen(m, b, stride=2, cycle=100, tol=1e-10, max_cycles=1000, damping=0.0,
                     nthreads=0):
    """GaBP + Steffensen (orc_solve_steffensen): returns
    (status, x, rounds, cycles, rel_residual)."""
    M = Matrix(m)
    b = _f64(b, M.n)
    x = np.empty(M.n)
    rounds, cycles, rel = C.c_int32(0), C.c_int32(0), C.c_double(0)
    st = _load().orc_solve_steffensen(C.byref(M.c), _p(b), stride, cycle, tol, max_cycles,
                                      damping, nthreads, _p(x), C.byref(rounds),
                                      C.byref(cycles), C.byref(rel))
    return st, x, int(rounds.value), int(cycles.value), float(rel.value)


def residual(m, b, x):
    """(r = b - A x, ||r||_2)."""
    M = Matrix(m)
    b, x = _f64(b, M.n), _f64(x, M.n)
    r = np.empty(M.n)
    nrm = _load().orc_residual(C.byref(M.c), _p(b), _p(x), _p(r))
    return r, float(nrm)


def residual_grid(nx, ny, nz, batch, b, x, diag=None, dval=0.0, cx=None, cy=None, cz=None,
                  off=0.0):
    """(r = b - A x, ||r||_2) for a stack of 5/7-point grids (see orc_residual_grid)."""
    n = nx * ny * nz * batch
    b, x = _f64(b, n), _f64(x, n)
    arr = [None if a is None else _f64(a, n) for a in (diag, cx, cy, cz)]
    r = np.empty(n)
    nrm = _load().orc_residual_grid(nx, ny, nz, batch, _p(arr[0]), dval, _p(arr[1]), _p(arr[2]),
                                    _p(arr[3]), off, _p(b), _p(x), _p(r))
    return r, float(nrm)


def jacobi_variant(m, b, rounds: int):
    """Proposition GaBPJ: GaBP with zero precision messages and no exclusion of
    the target; returns the marginal means after each round (list of arrays)."""
    M = Matrix(m)
    b = _f64(b, M.n)
    st, rev, diag = reverse(m)
    if st != OK:
        raise ValueError(st)
    h = np.zeros(M.nnz)
    out = []
    for _ in range(rounds):
        h2, mean = np.empty(M.nnz), np.empty(M.n)
        _load().orc_jacobi_variant_round(C.byref(M.c), _p(b), _p(rev), _p(diag), _p(h), _p(h2),
                                         _p(mean))
        h = h2
        out.append(mean)
    return out


# ---------------------------------------------------------------------------
# Section VII: symmetric (K+N) x (K+N) system [[I_K, S^T], [S, -Psi]] with
# right-hand side [0; y]; its first K unknowns solve (S^T S + Psi) x = S^T y
# for Psi = sigma^2 I_N (the reading taken where the printed dimensions clash).
# ---------------------------------------------------------------------------
class _CSRLike:
    def __init__(self, n, row_ptr, col, val):
        self.n, self.row_ptr, self.col, self.val = n, row_ptr, col, val


def bipartite_system_sparse(m: int, k: int, row_ptr, col, val, y, sigma2: float):
    """The same system for S given in CSR form (m x k, no explicit zeros), for
    sizes where S cannot be dense: rows of x first (diagonal 1, then column i
    of S), then rows of z (row j of S, then the diagonal -sigma2)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    srow = np.repeat(np.arange(m, dtype=np.int64), np.diff(row_ptr))
    n = k + m
    rows = np.concatenate([np.arange(k), srow + k, col, np.arange(k, n)])
    cols = np.concatenate([np.arange(k), col, srow + k, np.arange(k, n)])
    vals = np.concatenate([np.ones(k), val, val, np.full(m, -float(sigma2))])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr_b = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr_b[1:])
    rhs = np.concatenate([np.zeros(k), np.asarray(y, dtype=np.float64)])
    return _CSRLike(n, row_ptr_b, cols.astype(np.int32), vals), rhs


def bipartite_system(S: np.ndarray, y: np.ndarray, sigma2: float):
    """CSR of [[I_K, S^T], [S, -sigma2 I_N]] (zero entries of S dropped) and [0; y]."""
    S = np.asarray(S, dtype=np.float64)
    N, K = S.shape
    n = K + N
    dense = np.zeros((n, n))
    dense[:K, :K] = np.eye(K)
    dense[:K, K:] = S.T
    dense[K:, :K] = S
    dense[K:, K:] = -sigma2 * np.eye(N)
    r, c = np.nonzero(dense)
    counts = np.bincount(r, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    rhs = np.concatenate([np.zeros(K), np.asarray(y, dtype=np.float64)])
    return _CSRLike(n, row_ptr, c.astype(np.int32), dense[r, c]), rhs
