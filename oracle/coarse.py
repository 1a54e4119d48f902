"""FP64 oracle of coarse-grid predicted corrections for stacks of grids --
TEST INFRASTRUCTURE (only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it; it never imports the HIP package).

Not a method of the paper: the paper's GaBP iterations, run as a smoother,
with a correction predicted on coarser grids for the smooth error that GaBP
removes slowly.  Written plainly from the definitions below:

* aggregation: cell (x, y, z) of a grid belongs to the coarse cell
  (x // 2, y // 2, z // 2) (a dimension of extent 1 is not halved); P is the
  indicator matrix of that map, and the coarse operator is the Galerkin
  product A_c = P^T A P (a sparse matrix product), again a 5/7-point stencil;
  the coarse hierarchy stops at the first level below the finest with at
  most `coarsest` cells per grid (512 by default; a finest grid of at most
  64 cells is its own coarsest level);
* smoothing on a level with right-hand side v: coloured GaBP rounds (the
  serial scheme in checkerboard order, colour (x + y + z) & 1 with z counted
  over the whole stack, colour 0 first; or synchronous rounds) from zero
  information messages, the
  precision messages of that level's previous smoothing kept (zero at the
  start of a solve), and the marginal means of the final messages;
* a cycle on level l with right-hand side v: on the coarsest level below
  the finest, the exact solution of its Galerkin system (a dense solve per
  grid); on a finest level that is already the coarsest, nu_coarse GaBP
  sweeps; otherwise d = smooth(v, nu_pre), and with rc = P^T (v - A d),
  e = cycle(l + 1, rc) and then, unless the next level is the exactly solved
  coarsest one or has at most `v_cells` cells per grid (4096 by default),
  gamma - 1 more times e += cycle(l + 1, rc - A_c e) (gamma = 2: a W-cycle
  into the larger levels, a V-cycle into the small ones), d += scale * P e,
  and d += smooth(v - A d, nu_post);
* the solve: x = 0, then x += cycle(0, b - A x) until every grid's
  ||b_t - A_t x_t|| / ||b_t|| <= tol;
* with accel=True (the default) each grid's corrections are combined by the
  generalized conjugate residual method truncated to the previous direction
  (GCR(1)): with c = cycle(0, r), w = A c and (pc, pw) the previous step's
  direction and its image, c' = c - beta pc and w' = w - beta pw with
  beta = (w, pw) / (pw, pw), so that w' is orthogonal to pw, then
  x += alpha c' with alpha = (r, w') / (w', w'), the step that minimises
  ||r - alpha w'||; inner products over the grid's own cells.  A direction
  whose w' keeps less than 1e-10 of ||w||^2 after the orthogonalisation is
  used as it came (beta = 0).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import Rounds, residual

MAX_COARSE_CELLS = 512   # the coarsest level below the finest: at most this many cells per grid
MAX_FINEST_ALONE = 64    # a finest grid of at most this many cells is its own coarsest level
V_CELLS = 4096           # a level of at most this many cells per grid is cycled once


def grid_matrix(nx, ny, nz, batch, diag, cx, cy, cz):
    """The stack's operator as a scipy CSR matrix (node x + nx (y + ny z) of
    grid t at t nx ny nz; cx/cy/cz: coupling with the +x/+y/+z neighbour,
    ignored on a grid's last plane in that direction)."""
    n = nx * ny * nz
    N = n * batch
    i = np.arange(N)
    x, y, z = i % nx, (i // nx) % ny, (i // (nx * ny)) % nz
    rows, cols, vals = [i], [i], [np.asarray(diag, dtype=np.float64)]
    for c, ok, step in ((cx, x < nx - 1, 1), (cy, y < ny - 1, nx), (cz, z < nz - 1, nx * ny)):
        if c is None:
            continue
        c = np.asarray(c, dtype=np.float64)
        sel = ok & (c != 0.0)
        rows += [i[sel], i[sel] + step]
        cols += [i[sel] + step, i[sel]]
        vals += [c[sel], c[sel]]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def coarse_dims(nx, ny, nz):
    return tuple((d + 1) // 2 if d > 1 else 1 for d in (nx, ny, nz))


def aggregation(nx, ny, nz, batch):
    """P: fine nodes x coarse nodes indicator of the 2 x 2 x 2 blocks."""
    ncx, ncy, ncz = coarse_dims(nx, ny, nz)
    n = nx * ny * nz
    i = np.arange(n * batch)
    t = i // n
    x, y, z = i % nx, (i // nx) % ny, (i // (nx * ny)) % nz
    sx, sy, sz = (2 if d > 1 else 1 for d in (nx, ny, nz))
    I = (x // sx) + ncx * ((y // sy) + ncy * (z // sz)) + t * (ncx * ncy * ncz)
    return sp.csr_matrix((np.ones(n * batch), (i, I)), shape=(n * batch, ncx * ncy * ncz * batch))


def coefficients(A, nx, ny, nz, batch):
    """(diag, cx, cy, cz) arrays of a stencil matrix in the grid layout."""
    N = nx * ny * nz * batch
    i = np.arange(N)
    x, y, z = i % nx, (i // nx) % ny, (i // (nx * ny)) % nz
    A = sp.csr_matrix(A)
    diag = A.diagonal().copy()
    out = []
    for ok, step in ((x < nx - 1, 1), (y < ny - 1, nx), (z < nz - 1, nx * ny)):
        c = np.zeros(N)
        j = np.nonzero(ok)[0]
        c[j] = np.asarray(A[j, j + step]).ravel()
        out.append(c)
    return diag, out[0], out[1], out[2]


def checkerboard(nx, ny, nz, batch):
    i = np.arange(nx * ny * nz * batch)
    x, y, zg = i % nx, (i // nx) % ny, i // (nx * ny)
    return ((x + y + zg) & 1).astype(np.int8)


def _csr(A):
    from types import SimpleNamespace
    A = sp.csr_matrix(A)
    A.sort_indices()
    return SimpleNamespace(n=A.shape[0], row_ptr=A.indptr.astype(np.int64),
                           col=A.indices.astype(np.int32), val=A.data.astype(np.float64),
                           nnz=int(A.nnz))


class Hierarchy:
    """The levels of a stack: operator, its CSR for the oracle's rounds, the
    checkerboard colouring, the aggregation to the next level."""

    def __init__(self, nx, ny, nz, batch, diag, cx, cy, cz, colored=True, damping=0.0,
                 coarsest=MAX_COARSE_CELLS):
        self.levels = []
        self.damping = damping
        A = grid_matrix(nx, ny, nz, batch, diag, cx, cy, cz)
        dims = (nx, ny, nz)
        while True:
            lev = {"dims": dims, "A": A, "csr": _csr(A),
                   "colors": checkerboard(*dims, batch) if colored else None, "P_msg": None,
                   "damping": damping}
            self.levels.append(lev)
            if dims[0] * dims[1] * dims[2] <= (MAX_FINEST_ALONE if len(self.levels) == 1
                                               else coarsest):
                break
            P = aggregation(*dims, batch)
            lev["P"] = P
            A = (P.T @ A @ P).tocsr()
            dims = coarse_dims(*dims)
        self.batch = batch


def smooth(lev, v, sweeps):
    """Coloured GaBP rounds on right-hand side v from zero information
    messages, precisions of this level's previous smoothing kept; the means."""
    R = Rounds(lev["csr"], v, algorithm=2, colors=lev["colors"], damping=lev["damping"])
    if lev["P_msg"] is not None:
        R.P = lev["P_msg"].copy()
    R.step(sweeps)
    lev["P_msg"] = R.P.copy()
    return R.marginals()[0]


def cycle(H, l, v, nu_pre, nu_post, nu_coarse, scale, gamma=2, v_cells=V_CELLS):
    lev = H.levels[l]
    if "P" not in lev:
        if l == 0:  # the grid is its own coarsest level: GaBP sweeps alone
            return smooth(lev, v, nu_coarse)
        return spla.spsolve(lev["A"].tocsc(), v)
    d = smooth(lev, v, nu_pre)
    r = v - lev["A"] @ d
    rc = lev["P"].T @ r
    # the coarse system P^T A P e = rc: gamma cycles of the next level (one of
    # a small level), each on the residual the previous ones left
    e = cycle(H, l + 1, rc, nu_pre, nu_post, nu_coarse, scale, gamma, v_cells)
    nxt = H.levels[l + 1]
    exact = "P" not in nxt  # the coarsest: e is already the exact solution
    once = exact or nxt["dims"][0] * nxt["dims"][1] * nxt["dims"][2] <= v_cells
    for _ in range(0 if once else gamma - 1):
        e = e + cycle(H, l + 1, rc - nxt["A"] @ e, nu_pre, nu_post, nu_coarse, scale, gamma,
                      v_cells)
    d = d + scale * (lev["P"] @ e)
    if nu_post:
        d = d + smooth(lev, v - lev["A"] @ d, nu_post)
    return d


GCR_PARALLEL = 1e-10  # (w', w') <= this * (w, w): beta = 0


def gcr_step(r, c, w, prev, n, batch):
    """One GCR(1) step per grid (n cells each): returns (dx, (c', w')) for
    x += dx, given the residual r, the correction c, w = A c and the previous
    step's (c', w') (None on the first step)."""
    dx, cn, wn = np.empty_like(c), np.empty_like(c), np.empty_like(w)
    for t in range(batch):
        sl = slice(t * n, (t + 1) * n)
        ct, wt = c[sl], w[sl]
        if prev is not None:
            pc, pw = prev[0][sl], prev[1][sl]
            pp = float(pw @ pw)
            if pp > 0.0:
                beta = float(wt @ pw) / pp
                wo = wt - beta * pw
                if float(wo @ wo) > GCR_PARALLEL * float(wt @ wt):
                    ct, wt = ct - beta * pc, wo
        ww = float(wt @ wt)
        alpha = float(r[sl] @ wt) / ww if ww > 0.0 else 0.0
        dx[sl], cn[sl], wn[sl] = alpha * ct, ct, wt
    return dx, (cn, wn)


def solve(nx, ny, nz, batch, diag, cx, cy, cz, b, tol=1e-8, nu_pre=3, nu_post=3, nu_coarse=24,
          scale=1.8, max_cycles=100, colored=True, damping=0.0, gamma=2, accel=True,
          coarsest=MAX_COARSE_CELLS, v_cells=V_CELLS):
    """Returns (x, cycles, worst per-grid relative residual, list of the x
    after each cycle).  colored=False smooths with synchronous rounds; damping
    as in the rounds (section VI-D reading); accel: the GCR(1) combination of
    the corrections (above); v_cells=0: a W-cycle into every level."""
    H = Hierarchy(nx, ny, nz, batch, diag, cx, cy, cz, colored, damping, coarsest)
    A = H.levels[0]["A"]
    b = np.asarray(b, dtype=np.float64)
    n = nx * ny * nz
    bn = np.array([np.linalg.norm(b[t * n:(t + 1) * n]) for t in range(batch)])
    bn = np.where(bn > 0, bn, max(np.linalg.norm(b), 1e-300))
    x = np.zeros_like(b)
    trail = []
    worst = np.inf
    prev = None
    for k in range(max_cycles + 1):
        r = b - A @ x
        worst = max(np.linalg.norm(r[t * n:(t + 1) * n]) / bn[t] for t in range(batch))
        if worst <= tol or k == max_cycles:
            return x, k, worst, trail
        c = cycle(H, 0, r, nu_pre, nu_post, nu_coarse, scale, gamma, v_cells)
        if accel:
            dx, prev = gcr_step(r, c, A @ c, prev, n, batch)
            x = x + dx
        else:
            x = x + c
        trail.append(x.copy())
    return x, max_cycles, worst, trail


__all__ = ["grid_matrix", "aggregation", "coefficients", "coarse_dims", "checkerboard",
           "Hierarchy", "smooth", "cycle", "gcr_step", "solve", "residual"]
