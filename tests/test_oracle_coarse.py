"""Pins of the coarse-grid corrections oracle (oracle/coarse.py), CPU only.

The Galerkin coarse operator against a brute-force sum over the fine matrix's
entries (pure Python on tiny grids with odd extents), its row sums and
stencil shape (closed forms), the adjointness of restriction and
prolongation, the level count, the coarsest correction as the exact solution
of its system (its residual at rounding level), and the solve against a
direct sparse solve."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle import coarse as OC
import workloads as W


def _stack(nx, ny, nz, batch, seed):
    _, coef = W.grid_stack(nx, ny, nz, batch, varcoef=True, seed=seed, ell=3.0, with_csr=False)
    return coef


@pytest.mark.parametrize("dims", [(3, 5, 4), (5, 3, 1), (2, 2, 2), (1, 4, 3)])
def test_galerkin_operator_by_brute_force(dims):
    nx, ny, nz = dims
    batch = 2
    if nz == 1:
        m, coef = W.poisson2d_rect(nx, ny), None
        A = OC.grid_matrix(nx, ny, 1, 1, *OC.coefficients(
            __import__("scipy.sparse", fromlist=["csr_matrix"]).csr_matrix(
                (m.val, m.col, m.row_ptr), shape=(m.n, m.n)), nx, ny, 1, 1))
        batch = 1
    else:
        coef = _stack(nx, ny, nz, batch, 4)
        A = OC.grid_matrix(nx, ny, nz, batch, coef["diag"], coef["cx"], coef["cy"], coef["cz"])
    cx_, cy_, cz_ = OC.coarse_dims(nx, ny, nz)
    n, nc = nx * ny * nz, cx_ * cy_ * cz_

    def coarse_of(i):
        t, j = divmod(i, n)
        x, y, z = j % nx, (j // nx) % ny, j // (nx * ny)
        sx, sy, sz = (2 if d > 1 else 1 for d in (nx, ny, nz))
        return t * nc + (x // sx) + cx_ * ((y // sy) + cy_ * (z // sz))

    Ad = A.toarray()
    brute = np.zeros((nc * batch, nc * batch))
    for i in range(Ad.shape[0]):
        for j in range(Ad.shape[1]):
            if Ad[i, j] != 0.0:
                brute[coarse_of(i), coarse_of(j)] += Ad[i, j]
    P = OC.aggregation(nx, ny, nz, batch)
    Ac = (P.T @ A @ P).toarray()
    np.testing.assert_allclose(Ac, brute, rtol=1e-14, atol=1e-14)
    # the coarse operator is again a stencil of the coarse grid: rebuilt from
    # its own coefficient arrays it is the same matrix
    d, a, b, c = OC.coefficients(Ac, cx_, cy_, cz_, batch)
    again = OC.grid_matrix(cx_, cy_, cz_, batch, d, a, b, c).toarray()
    np.testing.assert_allclose(again, Ac, rtol=0, atol=0)


def test_row_sums_and_adjointness():
    nx, ny, nz, batch = 7, 6, 5, 3
    coef = _stack(nx, ny, nz, batch, 5)
    A = OC.grid_matrix(nx, ny, nz, batch, coef["diag"], coef["cx"], coef["cy"], coef["cz"])
    P = OC.aggregation(nx, ny, nz, batch)
    Ac = P.T @ A @ P
    one_c = np.ones(Ac.shape[0])
    # interior aggregates of a Dirichlet problem have row sums near zero: an
    # absolute floor at the size of the diagonal's rounding
    np.testing.assert_allclose(Ac @ one_c, P.T @ (A @ np.ones(A.shape[0])), rtol=1e-13,
                               atol=1e-13 * np.abs(Ac.diagonal()).max())
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal(Ac.shape[0]), rng.standard_normal(A.shape[0])
    assert (P @ u) @ v == pytest.approx(u @ (P.T @ v), rel=1e-13)
    # every fine cell belongs to exactly one coarse cell
    assert np.array_equal(np.asarray(P.sum(axis=1)).ravel(), np.ones(A.shape[0]))


@pytest.mark.parametrize("dims,levels512,levels64",
                         [((64, 64, 64), 4, 5), ((32, 32, 1), 2, 3), ((8, 8, 8), 2, 2),
                          ((5, 5, 5), 2, 2), ((4, 4, 4), 1, 1)])
def test_level_count(dims, levels512, levels64):
    """Levels down to the first one below the finest with at most 512 (or 64)
    cells per grid; a finest grid of at most 64 cells is its own coarsest."""
    nx, ny, nz = dims
    n = nx * ny * nz
    one = np.ones(n)
    for coarsest, levels in ((512, levels512), (64, levels64)):
        H = OC.Hierarchy(nx, ny, nz, 1, 6.5 * one, -one, -one, -one if nz > 1 else None,
                         coarsest=coarsest)
        assert len(H.levels) == levels, (dims, coarsest)
        sizes = [int(np.prod(L["dims"])) for L in H.levels]
        assert all(s > coarsest for s in sizes[1:-1]) and (len(sizes) == 1 or sizes[-1] <= coarsest)


def test_solve_matches_direct_solution():
    nx, ny, nz, batch = 16, 16, 16, 2
    coef = _stack(nx, ny, nz, batch, 6)
    b = W.normal_b(nx * ny * nz * batch, 6)
    A = OC.grid_matrix(nx, ny, nz, batch, coef["diag"], coef["cx"], coef["cy"], coef["cz"])
    x, cycles, worst, trail = OC.solve(nx, ny, nz, batch, coef["diag"], coef["cx"], coef["cy"],
                                       coef["cz"], b, tol=1e-10)
    assert worst <= 1e-10 and cycles < 30
    ref = spl.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-8
    # each cycle contracts the residual: a predicted correction, not a restart
    res = [np.linalg.norm(b - A @ xk) for xk in trail]
    assert all(r1 < 0.5 * r0 for r0, r1 in zip(res, res[1:]))


@pytest.mark.parametrize("coarsest", [512, 64])
def test_coarsest_correction_is_exact(coarsest):
    """Below the finest level the coarsest correction solves its Galerkin
    system exactly: A_c e = rc to rounding, on every grid of the stack."""
    nx, ny, nz, batch = (16, 14, 12, 2) if coarsest == 512 else (9, 7, 6, 3)
    coef = _stack(nx, ny, nz, batch, 8)
    H = OC.Hierarchy(nx, ny, nz, batch, coef["diag"], coef["cx"], coef["cy"], coef["cz"],
                     coarsest=coarsest)
    assert len(H.levels) == 2 and np.prod(H.levels[-1]["dims"]) > coarsest // 8
    last = H.levels[-1]
    rc = np.random.default_rng(3).standard_normal(last["A"].shape[0])
    e = OC.cycle(H, 1, rc, 4, 4, 24, 1.8)
    r = rc - last["A"] @ e
    assert np.abs(r).max() <= 1e-12 * np.abs(rc).max()
    # while 24 GaBP sweeps on the same system leave a visible residual
    g = OC.smooth(dict(last, P_msg=None), rc, 24)
    assert np.abs(rc - last["A"] @ g).max() > 1e3 * np.abs(r).max()


def _gcr_system(seed):
    nx, ny, nz, batch = 6, 5, 4, 3
    coef = _stack(nx, ny, nz, batch, seed)
    A = OC.grid_matrix(nx, ny, nz, batch, coef["diag"], coef["cx"], coef["cy"], coef["cz"])
    return A, nx * ny * nz, batch, np.random.default_rng(seed)


def _per_grid(u, v, n, batch):
    return np.array([float(u[t * n:(t + 1) * n] @ v[t * n:(t + 1) * n]) for t in range(batch)])


def test_gcr_step_minimises_and_orthogonalises():
    """Two GCR(1) steps with arbitrary corrections: each step's new residual
    is orthogonal, grid by grid, to the step's direction image w' and to the
    previous one (so it is the least-squares residual over both), the images
    stay A times the directions (c' and w' updated together), and no step
    raises a grid's residual."""
    A, n, batch, rng = _gcr_system(11)
    r0 = rng.standard_normal(A.shape[0])
    c1 = rng.standard_normal(A.shape[0])
    dx1, p1 = OC.gcr_step(r0, c1, A @ c1, None, n, batch)
    r1 = r0 - A @ dx1
    scale = np.sqrt(_per_grid(r0, r0, n, batch) * _per_grid(p1[1], p1[1], n, batch))
    assert np.all(np.abs(_per_grid(r1, p1[1], n, batch)) <= 1e-12 * scale)
    assert np.all(_per_grid(r1, r1, n, batch) <= _per_grid(r0, r0, n, batch))
    np.testing.assert_allclose(A @ p1[0], p1[1], rtol=0, atol=1e-12 * np.abs(p1[1]).max())
    c2 = rng.standard_normal(A.shape[0]) + 0.5 * c1
    dx2, p2 = OC.gcr_step(r1, c2, A @ c2, p1, n, batch)
    r2 = r1 - A @ dx2
    np.testing.assert_allclose(A @ p2[0], p2[1], rtol=0, atol=1e-12 * np.abs(p2[1]).max())
    for w in (p1[1], p2[1]):
        s2 = np.sqrt(_per_grid(r1, r1, n, batch) * _per_grid(w, w, n, batch))
        assert np.all(np.abs(_per_grid(r2, w, n, batch)) <= 1e-11 * s2)
    # the least-squares residual over span(w1', w2') on each grid, by lstsq
    for t in range(batch):
        sl = slice(t * n, (t + 1) * n)
        M = np.stack([p1[1][sl], p2[1][sl]], axis=1)
        coef, *_ = np.linalg.lstsq(M, r1[sl], rcond=None)
        best = r1[sl] - M @ coef
        assert np.linalg.norm(r2[sl]) <= np.linalg.norm(best) * (1 + 1e-10)


def test_gcr_step_exact_and_parallel_directions():
    """A correction that solves A c = r exactly is taken whole (alpha = 1,
    residual zero); a direction parallel to the previous one (nothing new)
    falls back to beta = 0 and, the residual being orthogonal to it already,
    moves nothing -- no division by a vanishing norm."""
    A, n, batch, rng = _gcr_system(12)
    r0 = rng.standard_normal(A.shape[0])
    c = spl.spsolve(A.tocsc(), r0)
    dx, prev = OC.gcr_step(r0, c, A @ c, None, n, batch)
    assert np.abs(r0 - A @ dx).max() <= 1e-12 * np.abs(r0).max()
    c1 = rng.standard_normal(A.shape[0])
    dx1, p1 = OC.gcr_step(r0, c1, A @ c1, None, n, batch)
    r1 = r0 - A @ dx1
    dx2, p2 = OC.gcr_step(r1, 2.0 * c1, A @ (2.0 * c1), p1, n, batch)
    assert np.all(np.isfinite(dx2))
    assert np.abs(dx2).max() <= 1e-10 * np.abs(dx1).max()


@pytest.mark.parametrize("varcoef", [True, False])
def test_accelerated_solve_needs_no_more_corrections(varcoef):
    """The GCR(1) combination reaches the tolerance on every grid in no more
    corrections than the plain sum (fewer on the shifted Poisson grid)."""
    nx = ny = nz = 24
    batch = 2
    _, coef = W.grid_stack(nx, ny, nz, batch, varcoef=varcoef, seed=9, shift=0.01,
                           with_csr=False)
    N = nx * ny * nz * batch
    if varcoef:
        arrs = (coef["diag"], coef["cx"], coef["cy"], coef["cz"])
    else:
        arrs = (np.full(N, coef["dval"]),) + (np.full(N, coef["off"]),) * 3
    b = W.normal_b(N, 10)
    runs = {acc: OC.solve(nx, ny, nz, batch, *arrs, b, tol=1e-8, accel=acc) for acc in (False, True)}
    assert runs[True][2] <= 1e-8
    assert runs[True][1] <= runs[False][1]
    if not varcoef:
        assert runs[True][1] < runs[False][1]


@pytest.mark.parametrize("v_cells, visits", [(4096, {32768: 1, 4096: 1, 512: 1}),
                                             (512, {32768: 1, 4096: 2, 512: 2}),
                                             (0, {32768: 1, 4096: 2, 512: 4})])
def test_small_levels_are_cycled_once(monkeypatch, v_cells, visits):
    """The visits of each level in one cycle of a 32^3 grid (levels 32^3,
    16^3, 8^3 and an exact 4^3): a level of at most v_cells cells per grid is
    cycled once by the level above, a larger one twice; each visit smooths
    twice (before and after the coarse prediction)."""
    n = 32
    coef = _stack(n, n, n, 1, 12)
    H = OC.Hierarchy(n, n, n, 1, coef["diag"], coef["cx"], coef["cy"], coef["cz"], coarsest=64)
    assert [int(np.prod(L["dims"])) for L in H.levels] == [32768, 4096, 512, 64]
    calls = {}
    smooth = OC.smooth

    def counting(lev, v, sweeps):
        k = int(np.prod(lev["dims"]))
        calls[k] = calls.get(k, 0) + 1
        return smooth(lev, v, sweeps)

    monkeypatch.setattr(OC, "smooth", counting)
    r = W.normal_b(n ** 3, 13)
    OC.cycle(H, 0, r, 3, 3, 24, 1.8, 2, v_cells)
    assert calls == {k: 2 * v for k, v in visits.items()}


def test_v_cycle_into_small_levels_keeps_the_corrections():
    """On a 32^3 variable-coefficient grid (levels down to an exact 4^3) the
    V-cycle into the levels of at most 4096 cells needs no more corrections
    to 1e-8 than W-cycles into every level, within one."""
    n = 32
    coef = _stack(n, n, n, 1, 14)
    b = W.normal_b(n ** 3, 15)
    args = (n, n, n, 1, coef["diag"], coef["cx"], coef["cy"], coef["cz"], b)
    _, cv, wv, _ = OC.solve(*args, tol=1e-8, coarsest=64)
    _, cw, ww, _ = OC.solve(*args, tol=1e-8, coarsest=64, v_cells=0)
    assert wv <= 1e-8 and ww <= 1e-8
    assert cv <= cw + 1, (cv, cw)
