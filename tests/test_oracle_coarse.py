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


@pytest.mark.parametrize("dims,levels", [((64, 64, 64), 5), ((32, 32, 1), 3), ((5, 5, 5), 2),
                                         ((4, 4, 4), 1)])
def test_level_count(dims, levels):
    nx, ny, nz = dims
    got = [dims]
    while got[-1][0] * got[-1][1] * got[-1][2] > OC.MAX_COARSE_CELLS:
        got.append(OC.coarse_dims(*got[-1]))
    assert len(got) == levels


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


def test_coarsest_correction_is_exact():
    """Below the finest level the coarsest correction solves its Galerkin
    system exactly: A_c e = rc to rounding, on every grid of the stack."""
    nx, ny, nz, batch = 9, 7, 6, 3
    coef = _stack(nx, ny, nz, batch, 8)
    H = OC.Hierarchy(nx, ny, nz, batch, coef["diag"], coef["cx"], coef["cy"], coef["cz"])
    assert len(H.levels) == 2
    last = H.levels[-1]
    rc = np.random.default_rng(3).standard_normal(last["A"].shape[0])
    e = OC.cycle(H, 1, rc, 4, 4, 24, 1.8)
    r = rc - last["A"] @ e
    assert np.abs(r).max() <= 1e-12 * np.abs(rc).max()
    # while 24 GaBP sweeps on the same system leave a visible residual
    g = OC.smooth(dict(last, P_msg=None), rc, 24)
    assert np.abs(rc - last["A"] @ g).max() > 1e3 * np.abs(r).max()
