"""Seeded synthetic inputs for the GaBP solver (Shental, Bickson et al.,
"Gaussian Belief Propagation for Solving Systems of Linear Equations").

This module builds linear systems ``A x = b`` shaped like the paper's
workloads and holds none of the method's arithmetic: no message, cavity,
marginal or residual is computed here.  Both the FP64 CPU oracle and the HIP
path receive their inputs from these functions, so the two sides see the same
numbers without sharing any solver code.

Matrices are returned in CSR form with the full symmetric pattern including
the diagonal: ``row_ptr`` int64 (n+1), ``col`` int32 (nnz, sorted within each
row), ``val`` float64 (nnz).  Random numbers come from ``numpy.random.Generator``
(PCG64) keyed by an explicit seed, so every input is reproducible.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "csr_from_coo", "csr_from_dense", "dense_from_csr",
    "poisson2d", "poisson3d", "poisson3d_varcoef", "grf_field",
    "sdd_random", "random_tree", "detection_batch", "DetectionBatch",
    "uniform_b", "normal_b", "tree_diameter", "grid_stack", "block_diag_csr",
]


@dataclass
class CSR:
    """Full symmetric CSR matrix (diagonal stored explicitly)."""
    n: int
    row_ptr: np.ndarray  # int64 [n+1]
    col: np.ndarray      # int32 [nnz]
    val: np.ndarray      # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def directed_edges(self) -> int:
        """Number of off-diagonal stored entries = directed messages per sweep."""
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        return int(np.count_nonzero(rows != self.col))


def csr_from_coo(n: int, rows, cols, vals) -> CSR:
    """Sort (row, col) pairs and pack them as CSR.  Duplicates are an error."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size > 1 and np.any(key[1:] == key[:-1]):
        raise ValueError("duplicate (row, col) entry")
    rows = rows[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n, row_ptr, cols[order].astype(np.int32), vals[order])


def csr_from_dense(a: np.ndarray) -> CSR:
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    r, c = np.nonzero(a)
    return csr_from_coo(n, r, c, a[r, c])


def dense_from_csr(m: CSR) -> np.ndarray:
    a = np.zeros((m.n, m.n))
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    a[rows, m.col] = m.val
    return a


def uniform_b(n: int, seed: int) -> np.ndarray:
    """b ~ U[-1, 1]."""
    return np.random.default_rng([seed, 0xB]).uniform(-1.0, 1.0, n)


def normal_b(n: int, seed: int) -> np.ndarray:
    """b ~ N(0, 1)."""
    return np.random.default_rng([seed, 0xB]).standard_normal(n)


# ---------------------------------------------------------------------------
# Poisson discretisations (section IX: 5-point stencil, Dirichlet 0, natural
# row ordering left->right then bottom->up; extended to 7 points in 3-D).
# ---------------------------------------------------------------------------
def poisson2d(p: int, diag: float = 4.0, off: float = -1.0) -> CSR:
    """p x p interior grid; unknown U(i, j) has index (i-1) + (j-1) p."""
    idx = np.arange(p * p).reshape(p, p)  # [j, i]
    rows, cols = [idx.ravel()], [idx.ravel()]
    vals = [np.full(p * p, diag)]
    for a, b in ((idx[:, :-1], idx[:, 1:]), (idx[:-1, :], idx[1:, :])):
        for u, v in ((a, b), (b, a)):
            rows.append(u.ravel()); cols.append(v.ravel())
            vals.append(np.full(u.size, off))
    return csr_from_coo(p * p, np.concatenate(rows), np.concatenate(cols),
                        np.concatenate(vals))


def _grid_faces(nx: int, ny: int, nz: int):
    """Interior faces of an nx x ny x nz grid as (u, v, axis) index arrays,
    with node index x + nx (y + ny z)."""
    idx = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    out = []
    for axis, (a, b) in enumerate(((idx[:, :, :-1], idx[:, :, 1:]),
                                   (idx[:, :-1, :], idx[:, 1:, :]),
                                   (idx[:-1, :, :], idx[1:, :, :]))):
        out.append((a.ravel(), b.ravel(), axis))
    return out


def poisson3d(nx: int, ny: int, nz: int, shift: float = 0.0) -> CSR:
    """Constant-coefficient 7-point Laplacian, Dirichlet 0: A_ii = 6 + shift,
    A_ij = -1 for face neighbours.  Built directly in row order (columns of a
    row are -z, -y, -x, diagonal, +x, +y, +z, already sorted), so large grids
    need no sort."""
    n = nx * ny * nz
    i = np.arange(n, dtype=np.int64)
    x, y, z = i % nx, (i // nx) % ny, i // (nx * ny)
    nxy = nx * ny
    cand = [(z > 0, i - nxy), (y > 0, i - nx), (x > 0, i - 1), (None, i),
            (x < nx - 1, i + 1), (y < ny - 1, i + nx), (z < nz - 1, i + nxy)]
    mask = np.stack([np.ones(n, bool) if ok is None else ok for ok, _ in cand], axis=1)
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.stack([j for _, j in cand], axis=1)[mask].astype(np.int32)
    val = np.where(np.arange(7) == 3, 6.0 + shift, -1.0)[None, :].repeat(n, 0)[mask]
    return CSR(n, row_ptr, col, val)


def grf_field(nx: int, ny: int, nz: int, seed: int, ell: float = 8.0,
              std: float = 1.0) -> np.ndarray:
    """Smooth Gaussian random field G[z, y, x]: white noise convolved
    (periodically, by FFT) with a Gaussian kernel of width ell / sqrt(2), which
    gives correlation exp(-r^2 / (2 ell^2)); standardised to mean 0, std ``std``."""
    rng = np.random.default_rng([seed, 0x6F])
    w = rng.standard_normal((nz, ny, nx))
    sk = ell / np.sqrt(2.0)
    freqs = [np.fft.fftfreq(m) for m in (nz, ny, nx)]
    kz, ky, kx = np.meshgrid(*freqs, indexing="ij")
    # Fourier transform of a unit-sum Gaussian kernel with std sk (cells)
    g = np.exp(-2.0 * np.pi ** 2 * sk ** 2 * (kx ** 2 + ky ** 2 + kz ** 2))
    f = np.fft.ifftn(np.fft.fftn(w) * g).real
    f -= f.mean()
    return f * (std / f.std())


def poisson3d_varcoef(nx: int, ny: int, nz: int, seed: int, ell: float = 8.0,
                      std: float = 1.0):
    """Variable-coefficient 7-point operator -div(k grad u), Dirichlet 0.

    k = exp(G) per cell with G = ``grf_field``; an interior face carries the
    harmonic mean 2 k_i k_j / (k_i + k_j); a boundary face (to the Dirichlet
    ghost) carries k_i.  A_ij = -k_face, A_ii = sum of the node's 6 face values.

    Returns (CSR, faces) where faces = dict with float64 arrays
    ``diag`` [n] and ``cx``, ``cy``, ``cz`` holding the coupling A_ij between
    node i and its +x / +y / +z neighbour (0 on the last plane of each axis).
    """
    k = np.exp(grf_field(nx, ny, nz, seed, ell, std))  # [z, y, x]
    diag = np.zeros((nz, ny, nx))
    cpl = []
    for axis in (2, 1, 0):  # x, y, z in array-axis terms
        lo = [slice(None)] * 3; hi = [slice(None)] * 3
        lo[axis] = slice(0, -1); hi[axis] = slice(1, None)
        ka, kb = k[tuple(lo)], k[tuple(hi)]
        kf = 2.0 * ka * kb / (ka + kb)
        c = np.zeros_like(k)
        c[tuple(lo)] = -kf
        cpl.append(c)
        diag[tuple(lo)] += kf
        diag[tuple(hi)] += kf
        # boundary faces on both ends of this axis
        first = [slice(None)] * 3; last = [slice(None)] * 3
        first[axis] = 0; last[axis] = -1
        diag[tuple(first)] += k[tuple(first)]
        diag[tuple(last)] += k[tuple(last)]
    n = nx * ny * nz
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [diag.ravel()]
    for (u, v, axis), c in zip(_grid_faces(nx, ny, nz), cpl):
        cv = c.ravel()[u]
        rows += [u, v]; cols += [v, u]; vals += [cv, cv]
    m = csr_from_coo(n, np.concatenate(rows), np.concatenate(cols),
                     np.concatenate(vals))
    faces = {"diag": diag.ravel().copy(), "cx": cpl[0].ravel().copy(),
             "cy": cpl[1].ravel().copy(), "cz": cpl[2].ravel().copy()}
    return m, faces


# ---------------------------------------------------------------------------
# Random sparse symmetric strictly diagonally dominant matrix.
# ---------------------------------------------------------------------------
def sdd_random(n: int, seed: int, partners: int = 4, factor: float = 1.1) -> CSR:
    """Each node draws ``partners`` distinct partners j != i uniformly; the
    union with the transpose gives the pattern (about 2 * partners off-diagonal
    entries per row, at least ``partners``).  One N(0, 1) value per undirected
    pair; A_ii = factor * sum_j |A_ij|."""
    rng = np.random.default_rng([seed, 0x5DD])
    i = np.repeat(np.arange(n, dtype=np.int64), partners)
    j = rng.integers(0, n - 1, size=n * partners, dtype=np.int64)
    j += (j >= i)  # skip the node itself
    # redraw partners repeated within a row until each row's draws are distinct
    while True:
        jj = j.reshape(n, partners)
        s = np.sort(jj, axis=1)
        dup_rows = np.nonzero(np.any(s[:, 1:] == s[:, :-1], axis=1))[0]
        if dup_rows.size == 0:
            break
        for r in dup_rows:
            row = jj[r]
            seen = set()
            for t in range(partners):
                while row[t] in seen:
                    v = int(rng.integers(0, n - 1))
                    row[t] = v + (v >= r)
                seen.add(int(row[t]))
        j = jj.ravel()
    lo = np.minimum(i, j); hi = np.maximum(i, j)
    pairs = np.unique(lo * n + hi)
    u = pairs // n; v = pairs % n
    w = rng.standard_normal(pairs.size)
    absum = np.bincount(u, np.abs(w), minlength=n) + np.bincount(v, np.abs(w), minlength=n)
    rows = np.concatenate([u, v, np.arange(n)])
    cols = np.concatenate([v, u, np.arange(n)])
    vals = np.concatenate([w, w, factor * absum])
    return csr_from_coo(n, rows, cols, vals)


# ---------------------------------------------------------------------------
# Random trees (Pruefer sequences) with nonzero elimination pivots.
# ---------------------------------------------------------------------------
def random_tree(n: int, seed: int, dominant: bool = True) -> CSR:
    """Random labelled tree on n >= 2 nodes from a Pruefer sequence.

    Off-diagonals ~ N(0, 1).  ``dominant``: A_ii = +-(1 + sum|A_ij|) U[0.5, 1.5]
    with random signs (indefinite, usually diagonally dominant); otherwise
    A_ii = +-U[0.5, 1.5] (not walk-summable in general)."""
    rng = np.random.default_rng([seed, 0x7EE])
    if n == 2:
        edges = [(0, 1)]
    else:
        seq = rng.integers(0, n, size=n - 2)
        degree = np.ones(n, dtype=np.int64)
        np.add.at(degree, seq, 1)
        import heapq
        leaves = [k for k in range(n) if degree[k] == 1]
        heapq.heapify(leaves)
        edges = []
        for s in seq:
            leaf = heapq.heappop(leaves)
            edges.append((leaf, int(s)))
            degree[s] -= 1
            if degree[s] == 1:
                heapq.heappush(leaves, int(s))
        a, b = heapq.heappop(leaves), heapq.heappop(leaves)
        edges.append((a, b))
    e = np.array(edges, dtype=np.int64)
    w = rng.standard_normal(len(edges))
    absum = np.bincount(e[:, 0], np.abs(w), minlength=n) + np.bincount(e[:, 1], np.abs(w), minlength=n)
    sign = rng.choice([-1.0, 1.0], size=n)
    mag = rng.uniform(0.5, 1.5, size=n)
    d = sign * mag * ((1.0 + absum) if dominant else 1.0)
    rows = np.concatenate([e[:, 0], e[:, 1], np.arange(n)])
    cols = np.concatenate([e[:, 1], e[:, 0], np.arange(n)])
    return csr_from_coo(n, rows, cols, np.concatenate([w, w, d]))


def tree_diameter(m: CSR) -> int:
    """Longest shortest path (in edges) of a tree, by two breadth-first searches."""
    def bfs(src):
        dist = np.full(m.n, -1); dist[src] = 0; q = [src]
        for u in q:
            for v in m.col[m.row_ptr[u]:m.row_ptr[u + 1]]:
                if v != u and dist[v] < 0:
                    dist[v] = dist[u] + 1; q.append(int(v))
        far = int(np.argmax(dist))
        return far, int(dist[far])
    far, _ = bfs(0)
    return bfs(far)[1]


# ---------------------------------------------------------------------------
# Linear detection (section VIII-B): synchronous CDMA with random spreading.
# ---------------------------------------------------------------------------
@dataclass
class DetectionBatch:
    """Packed detection instances.  Instance t has K[t] users and N[t] chips;
    its spreading matrix S_t (N x K, row-major) sits at S[s_off[t]:s_off[t+1]],
    its chip observations y_t (N) at y[y_off[t]:y_off[t+1]], its transmitted
    symbols x_t (K, +-1) at x[x_off[t]:x_off[t+1]]."""
    K: np.ndarray
    N: np.ndarray
    sigma2: np.ndarray
    S: np.ndarray
    y: np.ndarray
    x: np.ndarray
    s_off: np.ndarray
    y_off: np.ndarray
    x_off: np.ndarray

    @property
    def batch(self) -> int:
        return int(self.K.size)

    def instance(self, t: int):
        K, N = int(self.K[t]), int(self.N[t])
        S = self.S[self.s_off[t]:self.s_off[t + 1]].reshape(N, K)
        return (S, self.y[self.y_off[t]:self.y_off[t + 1]],
                self.x[self.x_off[t]:self.x_off[t + 1]], float(self.sigma2[t]))

    def mmse_system(self, t: int):
        """Dense MMSE detector system: A = S^T S + sigma^2 I, b = S^T y."""
        S, y, _, s2 = self.instance(t)
        return S.T @ S + s2 * np.eye(S.shape[1]), S.T @ y


def detection_subset(batch: int, seed: int, ids, kmin: int = 16, kmax: int = 256,
                     load: float = 0.5, snr_db: float = 10.0) -> DetectionBatch:
    """Instances ids of detection_batch(batch, seed, ...), drawn alone."""
    rng = np.random.default_rng([seed, 0xDE7])
    K = rng.integers(kmin, kmax + 1, size=batch).astype(np.int64)
    N = np.ceil(K / load).astype(np.int64)
    ids = np.asarray(ids, dtype=np.int64)
    return detection_sizes(K[ids], N[ids], seed, snr_db, ids=ids)


def detection_batch(batch: int, seed: int, kmin: int = 16, kmax: int = 256,
                    load: float = 0.5, snr_db: float = 10.0) -> DetectionBatch:
    """K ~ U{kmin..kmax}, N = K / load chips, S entries +-1/sqrt(N) iid (unit-norm
    codes), x in {+-1}^K, y = S x + n with n ~ N(0, sigma^2 I),
    sigma^2 = 10^(-snr_db/10)."""
    rng = np.random.default_rng([seed, 0xDE7])
    K = rng.integers(kmin, kmax + 1, size=batch).astype(np.int64)
    N = np.ceil(K / load).astype(np.int64)
    return detection_sizes(K, N, seed, snr_db)


def detection_sizes(K, N, seed: int, snr_db: float = 10.0, ids=None) -> DetectionBatch:
    """Detection instances of the given users K[t] and chips N[t] (the recipe
    of detection_batch with explicit sizes).  Instance t draws from its own
    stream, number ids[t] (default t), so sizes and ids taken from a
    detection_batch reproduce any of its instances."""
    K = np.asarray(K, dtype=np.int64)
    N = np.asarray(N, dtype=np.int64)
    batch = int(K.size)
    ids = np.arange(batch) if ids is None else np.asarray(ids, dtype=np.int64)
    s2 = np.full(batch, 10.0 ** (-snr_db / 10.0))
    s_off = np.zeros(batch + 1, dtype=np.int64); np.cumsum(N * K, out=s_off[1:])
    y_off = np.zeros(batch + 1, dtype=np.int64); np.cumsum(N, out=y_off[1:])
    x_off = np.zeros(batch + 1, dtype=np.int64); np.cumsum(K, out=x_off[1:])
    S = np.empty(int(s_off[-1])); y = np.empty(int(y_off[-1])); x = np.empty(int(x_off[-1]))
    for t in range(batch):
        r = np.random.default_rng([seed, 0xDE7, int(ids[t])])
        k, nn = int(K[t]), int(N[t])
        St = r.choice([-1.0, 1.0], size=(nn, k)) / np.sqrt(max(nn, 1))
        xt = r.choice([-1.0, 1.0], size=k)
        yt = St @ xt + np.sqrt(s2[t]) * r.standard_normal(nn)
        S[s_off[t]:s_off[t + 1]] = St.ravel()
        y[y_off[t]:y_off[t + 1]] = yt
        x[x_off[t]:x_off[t + 1]] = xt
    return DetectionBatch(K, N, s2, S, y, x, s_off, y_off, x_off)


@dataclass
class DenseBatch:
    """Packed dense symmetric instances: A_t (K[t] x K[t], row-major) at
    A[a_off[t]:a_off[t+1]], right-hand side b_t at b[b_off[t]:b_off[t+1]]."""
    K: np.ndarray
    A: np.ndarray
    b: np.ndarray
    a_off: np.ndarray
    b_off: np.ndarray

    @property
    def batch(self) -> int:
        return int(self.K.size)

    def instance(self, t: int):
        k = int(self.K[t])
        return (self.A[self.a_off[t]:self.a_off[t + 1]].reshape(k, k),
                self.b[self.b_off[t]:self.b_off[t + 1]])


def pack_dense(mats, rhs) -> DenseBatch:
    """Packs square matrices and right-hand sides back to back."""
    K = np.array([m.shape[0] for m in mats], dtype=np.int64)
    a_off = np.zeros(K.size + 1, dtype=np.int64); np.cumsum(K * K, out=a_off[1:])
    b_off = np.zeros(K.size + 1, dtype=np.int64); np.cumsum(K, out=b_off[1:])
    A = np.concatenate([np.ascontiguousarray(m, dtype=np.float64).ravel() for m in mats]) \
        if len(mats) else np.zeros(0)
    b = np.concatenate([np.asarray(v, dtype=np.float64) for v in rhs]) if len(rhs) else np.zeros(0)
    return DenseBatch(K, A, b, a_off, b_off)


def dense_sdd_batch(batch: int, seed: int, kmin: int = 4, kmax: int = 96, density: float = 1.0,
                    factor: float = 1.2) -> DenseBatch:
    """K ~ U{kmin..kmax}; symmetric off-diagonals N(0,1) kept with probability
    `density`, A_ii = factor * sum_j |A_ij| (strictly diagonally dominant; an
    empty row gets A_ii = 1); b ~ N(0,1)."""
    rng = np.random.default_rng([seed, 0xD5D])
    K = rng.integers(kmin, kmax + 1, size=batch)
    mats, rhs = [], []
    for t in range(batch):
        r = np.random.default_rng([seed, 0xD5D, t])
        k = int(K[t])
        a = np.triu(r.standard_normal((k, k)), 1)
        a *= np.triu(r.random((k, k)) < density, 1)
        a = a + a.T
        d = factor * np.abs(a).sum(axis=1)
        d[d == 0] = 1.0
        mats.append(a + np.diag(d))
        rhs.append(r.standard_normal(k))
    return pack_dense(mats, rhs)


def block_diag_csr(blocks) -> CSR:
    """Block-diagonal CSR of independent systems (node offsets accumulate)."""
    rows, cols, vals, off = [], [], [], 0
    for m in blocks:
        r = np.repeat(np.arange(m.n, dtype=np.int64), np.diff(m.row_ptr))
        rows.append(r + off); cols.append(m.col.astype(np.int64) + off); vals.append(m.val)
        off += m.n
    return csr_from_coo(off, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def grid_stack(nx: int, ny: int, nz: int, batch: int = 1, varcoef: bool = False,
               shift: float = 0.0, seed: int = 0, ell: float = 8.0, with_csr: bool = True):
    """A stack of `batch` independent grids with the 5-point (nz = 1) or
    7-point operator.  Constant coefficients: A_ii = 2 dim + shift, A_ij = -1.
    Variable: grid t uses poisson3d_varcoef(seed + t).  Returns (csr or None,
    coefficients dict: diag, cx, cy, cz arrays of batch * n, or None with
    dval/off constants)."""
    n = nx * ny * nz
    if not varcoef:
        dim = 3 if nz > 1 else 2
        coef = {"diag": None, "cx": None, "cy": None, "cz": None,
                "dval": 2.0 * dim + shift, "off": -1.0}
        csr = None
        if with_csr:
            one = poisson3d(nx, ny, nz, shift) if nz > 1 else poisson2d_rect(nx, ny, shift)
            csr = block_diag_csr([one] * batch) if batch > 1 else one
        return csr, coef
    mats, faces = [], []
    for t in range(batch):
        m, f = poisson3d_varcoef(nx, ny, nz, seed + t, ell=ell)
        mats.append(m); faces.append(f)
    coef = {k: np.concatenate([f[k] for f in faces]) for k in ("diag", "cx", "cy", "cz")}
    coef.update(dval=0.0, off=0.0)
    csr = (block_diag_csr(mats) if batch > 1 else mats[0]) if with_csr else None
    return csr, coef


def poisson2d_rect(nx: int, ny: int, shift: float = 0.0) -> CSR:
    """nx x ny 5-point Laplacian, Dirichlet 0, index x + nx y."""
    n = nx * ny
    idx = np.arange(n).reshape(ny, nx)
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [np.full(n, 4.0 + shift)]
    for a, b in ((idx[:, :-1], idx[:, 1:]), (idx[:-1, :], idx[1:, :])):
        for u, v in ((a, b), (b, a)):
            rows.append(u.ravel()); cols.append(v.ravel()); vals.append(np.full(u.size, -1.0))
    return csr_from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def mlp_params(seed: int, n_in: int = 8, n_hid: int = 64, n_out: int = 12, scale: float = 1.0):
    """Random parameters of the 8-64-64-12 warm-start network, flat in the
    order W1 (n_hid x n_in, row-major), b1, W2, b2, W3, b3: He-uniform
    weights (bound sqrt(6 / fan_in)) times `scale`, biases U(-0.1, 0.1)."""
    rng = np.random.default_rng([seed, 0x31F])
    parts = []
    for rows, cols in ((n_hid, n_in), (n_hid, n_hid), (n_out, n_hid)):
        bound = scale * np.sqrt(6.0 / cols)
        parts.append(rng.uniform(-bound, bound, size=rows * cols))
        parts.append(rng.uniform(-0.1, 0.1, size=rows))
    return np.concatenate(parts)


def mlp_batch(count: int, seed: int, n_in: int = 8, n_out: int = 12, p_mask: float = 0.8):
    """Random training batch: features N(0, 1), targets N(0, 1), output mask
    Bernoulli(p_mask) per sample and direction (pairs of outputs)."""
    rng = np.random.default_rng([seed, 0xB7C])
    U = rng.standard_normal((count, n_in))
    T = rng.standard_normal((count, n_out))
    on = rng.random((count, n_out // 2)) < p_mask
    U[:, 1:1 + n_out // 2] *= on  # a direction without a neighbour has coupling 0
    M = np.repeat(on, 2, axis=1).astype(np.float64)
    return U, T * M, M


class SparseRect:
    """A sparse m x k matrix (any shape) in CSR form: int64 row_ptr, int32
    col (strictly increasing within a row), float64 val (no explicit zeros)."""

    def __init__(self, m, k, row_ptr, col, val):
        self.m, self.k = int(m), int(k)
        self.row_ptr, self.col, self.val = row_ptr, col, val

    @property
    def nnz(self) -> int:
        return int(self.col.size)

    def dense(self) -> np.ndarray:
        a = np.zeros((self.m, self.k))
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        a[rows, self.col] = self.val
        return a


def sparse_rect(m: int, k: int, per_row: int, seed: int, signs: bool = False,
                empty_rows=(), empty_cols=()) -> SparseRect:
    """Row j holds min(per_row, k) distinct random columns with N(0,1) values
    (or +-1 when `signs`) scaled by 1/sqrt(per_row); rows in `empty_rows` are
    empty and no entry falls in a column of `empty_cols`."""
    rng = np.random.default_rng([seed, 0x5EC7])
    allowed = np.setdiff1d(np.arange(k), np.asarray(empty_cols, dtype=np.int64))
    p = min(per_row, allowed.size)
    keep = np.ones(m, dtype=bool)
    keep[np.asarray(list(empty_rows), dtype=np.int64)] = False
    if p == 0:
        keep[:] = False
    if p == allowed.size:
        idx = np.tile(np.arange(p), (m, 1))
    else:
        idx = np.sort(rng.integers(0, allowed.size, size=(m, p)), axis=1)
        bad = np.nonzero((np.diff(idx, axis=1) == 0).any(axis=1))[0] if p > 1 else np.zeros(0, int)
        while bad.size:  # redraw rows with a repeated column
            idx[bad] = np.sort(rng.integers(0, allowed.size, size=(bad.size, p)), axis=1)
            sub = (np.diff(idx[bad], axis=1) == 0).any(axis=1)
            bad = bad[sub]
    v = rng.choice([-1.0, 1.0], size=(m, p)) if signs else rng.standard_normal((m, p))
    v = np.where(v == 0.0, 1.0, v) / np.sqrt(max(per_row, 1))
    counts = np.where(keep, p, 0)
    rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    col = allowed[idx[keep]].reshape(-1).astype(np.int32)
    val = v[keep].reshape(-1)
    return SparseRect(m, k, rp, col, val)
