"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them compares the oracle with
itself: the expected values come from the paper's printed tables
(tests/golden), closed forms, LAPACK solves, textbook iterations or brute
force on tiny inputs.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from golden_io import lines, num, read_matrix


def _slot(m, i, j):
    for e in range(m.row_ptr[i], m.row_ptr[i + 1]):
        if m.col[e] == j:
            return e
    raise KeyError((i, j))


def _toy():
    it = lines("toy_tree.txt")
    tok = next(it)
    assert tok[0] == "matrix"
    A = read_matrix(it, int(tok[1]))
    rec = {"msg": [], "mean": [], "prec": []}
    for t in it:
        if t[0] in ("b", "solution", "inverse"):
            rec[t[0]] = np.array([num(v) for v in t[1:]])
        else:
            rec[t[0]].append(t[1:])
    return A, rec


@pytest.mark.parametrize("algorithm", [1, 2])
def test_toy_tree_message_table(algorithm):
    """Section VIII-A, table of message evolution and table of tentative means:
    every message and tentative mean for t = 0..3 (exact rationals)."""
    A, rec = _toy()
    m = W.csr_from_dense(A)
    R = oracle.Rounds(m, rec["b"], algorithm=algorithm)
    for t in range(4):
        if t:
            R.step()
        for kind, i, j, *vals in rec["msg"]:
            e = _slot(m, int(i), int(j))
            got = (R.P if kind == "P" else R.Mu)[e]
            assert got == pytest.approx(num(vals[t]), rel=1e-15, abs=1e-15), (kind, i, j, t)
        mean, _ = R.marginals()
        for i, *vals in rec["mean"]:
            assert mean[int(i)] == pytest.approx(num(vals[t]), rel=1e-15, abs=1e-15), (i, t)
    _, prec = R.marginals()
    for i, v in rec["prec"]:
        assert prec[int(i)] == pytest.approx(num(v), rel=1e-15)
    # the exact precisions are the inverse diagonal of A^{-1} (printed inverse)
    inv = rec["inverse"].reshape(3, 3)
    np.testing.assert_allclose(1.0 / prec, np.diag(inv), rtol=1e-15)
    np.testing.assert_allclose(inv @ rec["b"], rec["solution"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(np.linalg.inv(A), inv, atol=1e-15)


@pytest.mark.parametrize("n,seed,dominant", [(2, 0, True), (5, 1, True), (17, 2, False),
                                             (60, 3, True), (200, 4, False), (200, 5, True)])
def test_tree_exact_within_diameter(n, seed, dominant):
    """Section IV (trees: exact means and variances) and Proposition GaBPGE
    (GaBP = Gaussian elimination on a tree): after diameter rounds the means
    equal the LU solve and the precisions equal 1 / (A^{-1})_ii; one more round
    changes nothing; one round fewer is not yet exact (checked on short,
    non-dominant trees, where distant influence stays above rounding)."""
    m = W.random_tree(n, seed, dominant=dominant)
    A = W.dense_from_csr(m)
    b = W.normal_b(n, seed)
    diam = W.tree_diameter(m)
    x_lu = np.linalg.solve(A, b)
    ainv = np.linalg.inv(A)
    R = oracle.Rounds(m, b, algorithm=1).step(diam)
    assert R.zero_cavities == 0
    mean, prec = R.marginals()
    np.testing.assert_allclose(mean, x_lu, rtol=1e-9, atol=1e-9 * np.abs(x_lu).max())
    np.testing.assert_allclose(1.0 / prec, np.diag(ainv), rtol=1e-9,
                               atol=1e-9 * np.abs(np.diag(ainv)).max())
    P, Mu = R.P.copy(), R.Mu.copy()
    R.step()
    assert np.array_equal(R.P, P) and np.array_equal(R.Mu, Mu)
    if 2 <= diam <= 8 and not dominant:
        # on long or dominant paths the far leaf's influence falls below rounding
        early = oracle.Rounds(m, b, algorithm=1).step(diam - 1).marginals()[0]
        assert np.max(np.abs(early - x_lu)) > 1e-6 * np.abs(x_lu).max()


@pytest.mark.parametrize("make", [
    lambda: W.sdd_random(300, 7),
    lambda: W.poisson2d(12),
    lambda: W.poisson3d(5, 4, 3, 0.01),
    lambda: W.poisson3d_varcoef(6, 5, 4, 3)[0],
])
def test_alg2_equals_alg1_each_round(make):
    """Section V: Algorithm 2 (aggregate, then subtract the reverse message)
    computes the same messages as Algorithm 1, round by round."""
    m = make()
    b = W.uniform_b(m.n, 11)
    r1 = oracle.Rounds(m, b, algorithm=1)
    r2 = oracle.Rounds(m, b, algorithm=2)
    for _ in range(12):
        r1.step(); r2.step()
        np.testing.assert_allclose(r2.P, r1.P, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(r2.information(), r1.information(), rtol=1e-11,
                                   atol=1e-12 * np.abs(r1.information()).max())


@pytest.mark.parametrize("algorithm", [1, 2])
def test_converged_means_equal_lu_on_sdd(algorithm):
    """Theorem 1 (strict diagonal dominance => convergence to the true means)."""
    m = W.sdd_random(400, 3)
    A = W.dense_from_csr(m)
    assert np.all(np.abs(np.diag(A)) > np.abs(A - np.diag(np.diag(A))).sum(1))
    b = W.normal_b(m.n, 3)
    res = oracle.solve(m, b, algorithm=algorithm, tol=1e-14, max_rounds=500)
    assert res.status == oracle.OK
    x = np.linalg.solve(A, b)
    np.testing.assert_allclose(res.x, x, rtol=1e-11, atol=1e-12 * np.abs(x).max())
    # residual decreases overall: last trace entry far below the first
    assert res.trace[-1] < 1e-12 * res.trace[0]


def test_poisson_32_fp64_matches_lu():
    """2-D Poisson (section IX) at p = 32, b ~ U[-1, 1], to relative residual
    1e-10: the means equal the LU solve."""
    m = W.poisson2d(32)
    b = W.uniform_b(m.n, 0)
    res = oracle.solve(m, b, algorithm=2, tol=1e-10, max_rounds=20000)
    assert res.status == oracle.OK
    x = np.linalg.solve(W.dense_from_csr(m), b)
    assert np.linalg.norm(res.x - x) / np.linalg.norm(x) < 1e-8
    assert res.trace[-1] <= 1e-10


def test_jacobi_special_case():
    """Proposition GaBPJ: zero precision messages and no exclusion of the
    target give exactly the textbook Jacobi iteration x <- D^{-1}(b - (A-D) x)."""
    m = W.sdd_random(150, 9)
    A = W.dense_from_csr(m)
    b = W.normal_b(m.n, 9)
    D = np.diag(A)
    R = A - np.diag(D)
    x = np.zeros(m.n)
    for t, mean in enumerate(oracle.jacobi_variant(m, b, 25)):
        x = (b - R @ x) / D
        np.testing.assert_allclose(mean, x, rtol=1e-13, atol=1e-14), t


def test_gold_code_matrices_walk_summable():
    """Section VIII-B: R3, R4 are not strictly diagonally dominant, their
    stated spectral radii rho(|I - R|) are 0.9008 and 0.8747 (Theorem 2), and
    GaBP converges to R^{-1} 1.  The iteration counts of the paper's table are
    context only (initial guess and ordering unspecified): a +-50% band."""
    it = lines("gold_codes.txt")
    mats, rho, iters = {}, {}, {}
    for t in it:
        if t[0] in ("R3", "R4"):
            scale, k = float(t[1]), int(t[2])
            mats[t[0]] = read_matrix(it, k) / scale
        elif t[0] == "rho":
            rho[t[1]] = float(t[2])
        elif t[0] == "iters":
            iters[t[1]] = int(t[3])
    for name, A in mats.items():
        offsum = np.abs(A - np.diag(np.diag(A))).sum(1)
        assert not np.all(np.abs(np.diag(A)) > offsum)
        r = np.max(np.abs(np.linalg.eigvals(np.abs(np.eye(len(A)) - A))))
        assert round(r, 4) == rho[name]
        b = np.ones(len(A))
        m = W.csr_from_dense(A)
        res = oracle.solve(m, b, algorithm=1, stop=oracle.STOP_MESSAGES, tol=1e-6, max_rounds=1000)
        assert res.status == oracle.OK
        np.testing.assert_allclose(res.x, np.linalg.solve(A, b), atol=1e-5)
        assert 0.5 * iters[name] <= res.rounds <= 1.5 * iters[name]


def test_nonpsd_example_converges():
    """Section VIII-C and the remark of section III-A: the derivation does not
    need positive definiteness; parallel GaBP converges on the indefinite 3x3
    example to A^{-1} 1 (iteration count +-50% of the printed 38)."""
    it = lines("nonpsd.txt")
    tok = next(it)
    A = read_matrix(it, int(tok[1]))
    printed = int(next(it)[2])
    assert np.linalg.eigvalsh(A).min() < 0
    b = np.ones(3)
    m = W.csr_from_dense(A)
    res = oracle.solve(m, b, algorithm=1, stop=oracle.STOP_MESSAGES, tol=1e-6, max_rounds=1000)
    assert res.status == oracle.OK
    np.testing.assert_allclose(res.x, np.linalg.solve(A, b), atol=1e-5)
    assert 0.5 * printed <= res.rounds <= 1.5 * printed
    # Jacobi (the classical iteration the paper compares) diverges here
    D = np.diag(A)
    x = np.zeros(3)
    for _ in range(60):
        x = (b - (A - np.diag(D)) @ x) / D
    assert np.abs(x).max() > 1e3


def test_poisson_generator_matches_printed_matrix():
    """Section IX: the natural-ordering 9x9 matrix printed for p = 3."""
    it = lines("poisson_p3.txt")
    tok = next(it)
    A = read_matrix(it, int(tok[1]))
    np.testing.assert_array_equal(W.dense_from_csr(W.poisson2d(3)), A)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bipartite_construction_is_mmse(seed):
    """Section VII: GaBP on [[I, S^T], [S, -sigma^2 I]] x = [0; y] yields, in
    its first K unknowns, (S^T S + sigma^2 I)^{-1} S^T y."""
    db = W.detection_batch(3, seed, kmin=6, kmax=24)
    for t in range(db.batch):
        S, y, _, s2 = db.instance(t)
        m, rhs = oracle.bipartite_system(S, y, s2)
        res = oracle.solve(m, rhs, algorithm=2, tol=1e-13, max_rounds=5000)
        assert res.status == oracle.OK, res.status
        A, b = db.mmse_system(t)
        np.testing.assert_allclose(res.x[:S.shape[1]], np.linalg.solve(A, b), rtol=1e-9, atol=1e-10)


def test_literal_dense_detection_diverges():
    """Dense MMSE matrices at load K/N = 1/2 and sigma^2 = 0.1 are far from
    walk-summable (Theorem 2 fails); synchronous GaBP does not converge on them."""
    db = W.detection_batch(1, 4, kmin=64, kmax=64)
    A, b = db.mmse_system(0)
    Dm = np.diag(1 / np.sqrt(np.diag(A)))
    An = Dm @ A @ Dm
    assert np.max(np.abs(np.linalg.eigvals(np.abs(np.eye(64) - An)))) > 1.0
    res = oracle.solve(W.csr_from_dense(A), b, algorithm=2, tol=1e-8, max_rounds=400)
    assert res.status in (oracle.ERR_DIVERGED, oracle.NOT_CONVERGED, oracle.ERR_BREAKDOWN)


def test_damping_keeps_fixed_point():
    """Damping (section VI-D moving average) changes the trajectory but not the
    fixed point: the damped run still reaches the LU solution."""
    m = W.poisson2d(10)
    b = W.uniform_b(m.n, 2)
    x = np.linalg.solve(W.dense_from_csr(m), b)
    und = oracle.solve(m, b, tol=1e-12, max_rounds=5000)
    dmp = oracle.solve(m, b, tol=1e-12, max_rounds=10000, damping=0.5)
    assert und.status == dmp.status == oracle.OK
    assert dmp.rounds > und.rounds
    np.testing.assert_allclose(dmp.x, x, rtol=1e-10, atol=1e-11)


def _toy_damped():
    alpha, msgs, means = None, [], []
    for t in lines("toy_tree_damped.txt"):
        if t[0] == "alpha":
            alpha = num(t[1])
        elif t[0] == "dmsg":
            msgs.append((t[1], int(t[2]), int(t[3]), int(t[4]), num(t[5]), num(t[6])))
        elif t[0] == "dmean":
            means.append((t[1], int(t[2]), np.array([num(v) for v in t[3:6]])))
    return alpha, msgs, means


@pytest.mark.parametrize("algorithm", [1, 2])
def test_damped_rounds_on_the_toy_tree(algorithm):
    """Section VI-D damping as read for GaBP (every message's P and h = P mu
    mixed as alpha old + (1 - alpha) new): two damped rounds from zero
    messages and one from the printed t = 1 messages of section VIII-A,
    against values derived by hand (tests/golden/toy_tree_damped.txt) at
    alpha = 3/10, where swapping alpha and 1 - alpha or damping mu instead of
    h gives different numbers."""
    A, rec = _toy()
    alpha, msgs, means = _toy_damped()
    m = W.csr_from_dense(A)
    for case, rounds in (("zero", 2), ("t1", 1)):
        R = oracle.Rounds(m, rec["b"], algorithm=algorithm, damping=alpha)
        if case == "t1":
            for kind, i, j, *vals in rec["msg"]:
                e = _slot(m, int(i), int(j))
                (R.P if kind == "P" else R.Mu)[e] = num(vals[1])
        for t in range(1, rounds + 1):
            R.step()
            for c, tt, i, j, P, h in msgs:
                if c != case or tt != t:
                    continue
                e = _slot(m, i, j)
                assert R.P[e] == pytest.approx(P, rel=1e-14, abs=1e-15), (case, t, i, j)
                assert R.information()[e] == pytest.approx(h, rel=1e-14, abs=1e-14), (case, t, i, j)
            mean, _ = R.marginals()
            exp = [v for c, tt, v in means if c == case and tt == t]
            assert len(exp) == 1
            np.testing.assert_allclose(mean, exp[0], rtol=1e-14)


@pytest.mark.parametrize("tol,rounds", [(10.0, 1), (5.0, 2), (1.0, 3), (1e-300, 3)])
def test_stop_on_the_change_of_the_means(tol, rounds):
    """The marginal-mean criterion (stop at the first round whose largest
    change of a tentative mean is below tol) on the printed table of tentative
    means of section VIII-A: changes 7, 2 and 0 at t = 1, 2, 3 (the tree is
    exact after its diameter, 2 rounds, so round 3 repeats round 2)."""
    A, rec = _toy()
    r = oracle.solve(W.csr_from_dense(A), rec["b"], stop=oracle.STOP_MEANS, tol=tol,
                     max_rounds=10)
    assert r.status == oracle.OK and r.rounds == rounds
    printed = np.array([[num(v) for v in row[1:]] for row in rec["mean"]])  # node x t
    np.testing.assert_allclose(r.x, printed[:, rounds], rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("tol,rounds", [(10.0, 1), (13.0, 1), (5.0, 3)])
def test_stop_on_the_change_of_the_messages(tol, rounds):
    """The criterion of section VIII (largest absolute change of any message,
    precision or mean) on the printed message table of section VIII-A: changes
    9, 12 and 0 at t = 1, 2, 3."""
    A, rec = _toy()
    r = oracle.solve(W.csr_from_dense(A), rec["b"], stop=oracle.STOP_MESSAGES, tol=tol,
                     max_rounds=10)
    assert r.status == oracle.OK and r.rounds == rounds


def test_residual_definition():
    """Section II-A residual: r = b - A x (norm as the paper's Frobenius norm)."""
    m = W.sdd_random(500, 1)
    A = W.dense_from_csr(m)
    rng = np.random.default_rng(5)
    x, b = rng.standard_normal(m.n), rng.standard_normal(m.n)
    r, nrm = oracle.residual(m, b, x)
    np.testing.assert_allclose(r, b - A @ x, rtol=1e-13, atol=1e-13)
    assert nrm == pytest.approx(np.linalg.norm(b - A @ x), rel=1e-13)


def test_refinement_loop_reaches_tolerance():
    """Refinement (x += d, r = b - A x, restart the mean messages, keep the
    precisions): reaches 1e-12 with several restarts and the LU answer."""
    m = W.poisson2d(16)
    b = W.uniform_b(m.n, 4)
    st, x, rounds, restarts, rel = oracle.refine_solve(m, b, tol=1e-12, inner_tol=1e-3)
    assert st == oracle.OK and rel <= 1e-12 and restarts >= 2
    xs = np.linalg.solve(W.dense_from_csr(m), b)
    np.testing.assert_allclose(x, xs, rtol=1e-10, atol=1e-11)


def test_error_paths():
    """Zero diagonal, asymmetric values and a zero elimination pivot."""
    A = np.array([[0.0, 1.0], [1.0, 2.0]])
    assert oracle.solve(W.csr_from_dense(A), np.ones(2)).status == oracle.ERR_ZERO_DIAG
    A = np.array([[2.0, 1.0], [1.5, 2.0]])
    assert oracle.solve(W.csr_from_dense(A), np.ones(2)).status == oracle.ERR_NOT_SYMMETRIC
    # path x - y - z with A_yy + P_xy = 0: the cavity precision of y toward z
    # vanishes (a zero Gaussian-elimination pivot) although A is nonsingular
    A = np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 1.0], [0.0, 1.0, 1.0]])
    assert abs(np.linalg.det(A)) > 0.5
    assert oracle.solve(W.csr_from_dense(A), np.ones(3)).status == oracle.ERR_BREAKDOWN


def test_thread_count_bitwise_identical():
    """Synchronous rounds read only the previous buffers: 1 and 4 threads agree bitwise."""
    m = W.sdd_random(5000, 2)
    b = W.normal_b(m.n, 2)
    a = oracle.Rounds(m, b, algorithm=2, nthreads=1).step(7)
    c = oracle.Rounds(m, b, algorithm=2, nthreads=4).step(7)
    assert np.array_equal(a.P, c.P) and np.array_equal(a.Mu, c.Mu)


@pytest.mark.parametrize("shape", [(5, 4, 3, 2, False, 0.01), (6, 5, 4, 3, True, 0.0),
                                   (7, 6, 1, 2, False, 0.0), (6, 5, 1, 2, True, 0.0)])
def test_structured_residual_matches_csr_residual(shape):
    """The oracle's stencil residual (used where a CSR of the full grid is too
    large) equals its CSR residual on the same operator."""
    nx, ny, nz, bt, vc, sh = shape
    m, c = W.grid_stack(nx, ny, nz, bt, varcoef=vc, shift=sh, seed=3)
    rng = np.random.default_rng(1)
    x, b = rng.standard_normal(m.n), rng.standard_normal(m.n)
    r1, n1 = oracle.residual(m, b, x)
    r2, n2 = oracle.residual_grid(nx, ny, nz, bt, b, x, c["diag"], c["dval"], c["cx"], c["cy"],
                                  c["cz"], c["off"])
    np.testing.assert_allclose(r2, r1, rtol=0, atol=1e-13 * np.abs(r1).max())
    assert n2 == pytest.approx(n1, rel=1e-14)


def test_poisson3d_row_order_construction():
    """The sort-free 7-point construction equals the face-list construction."""
    for dims in [(5, 4, 3), (1, 6, 2), (7, 1, 1), (3, 3, 3)]:
        a = W.poisson3d(*dims, shift=0.01)
        nx, ny, nz = dims
        n = nx * ny * nz
        rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.full(n, 6.01)]
        for u, v, _ in W._grid_faces(nx, ny, nz):
            rows += [u, v]; cols += [v, u]; vals += [np.full(u.size, -1.0)] * 2
        b = W.csr_from_coo(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))
        assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
        assert np.array_equal(a.val, b.val)


# ---------------------------------------------------------------------------
# Coloured (serial-like) schedule.  On a bipartite graph the synchronous
# rounds split into two independent chains (messages of one class at odd
# rounds feed the other class at even rounds), and a two-colour schedule runs
# one of them: after k coloured sweeps class 0 holds the synchronous messages
# of round 2k - 1 and class 1 those of round 2k, exactly.
# ---------------------------------------------------------------------------
def _grid_colours(nx, ny, nz=1):
    i = np.arange(nx * ny * nz)
    return ((i % nx) + (i // nx) % ny + i // (nx * ny)) % 2


def _class_slots(m, colors, c):
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    return (colors[rows] == c) & (rows != m.col)


@pytest.mark.parametrize("case", ["grid2d", "grid3d", "tree", "bipartite"])
def test_two_colour_schedule_runs_one_synchronous_chain(case):
    if case == "grid2d":
        m = W.poisson2d_rect(7, 5, 0.1); col = _grid_colours(7, 5)
    elif case == "grid3d":
        m = W.poisson3d(4, 3, 5, 0.2); col = _grid_colours(4, 3, 5)
    elif case == "tree":
        m = W.random_tree(40, 3)
        # two-colour a tree by depth parity
        A = W.dense_from_csr(m) != 0
        col = -np.ones(m.n, dtype=int); col[0] = 0; todo = [0]
        while todo:
            i = todo.pop()
            for j in np.nonzero(A[i])[0]:
                if j != i and col[j] < 0:
                    col[j] = 1 - col[i]; todo.append(j)
    else:
        db = W.detection_sizes([6], [12], seed=4)
        S, y, _, s2 = db.instance(0)
        m, b = oracle.bipartite_system(S, y, s2)
        col = np.r_[np.ones(6, dtype=int), np.zeros(12, dtype=int)]  # chips send first
    b = W.uniform_b(m.n, 7) if case != "bipartite" else b
    assert oracle.is_proper_colouring(m, col)
    sync = oracle.Rounds(m, b)
    colr = oracle.Rounds(m, b, colors=col)
    s0, s1 = _class_slots(m, col, 0), _class_slots(m, col, 1)
    hist = {}
    for t in range(1, 13):
        sync.step()
        hist[t] = (sync.P.copy(), sync.Mu.copy())
    for k in range(1, 7):
        colr.step()
        P1, M1 = hist[2 * k - 1]
        P2, M2 = hist[2 * k]
        assert np.array_equal(colr.P[s0], P1[s0]) and np.array_equal(colr.Mu[s0], M1[s0])
        assert np.array_equal(colr.P[s1], P2[s1]) and np.array_equal(colr.Mu[s1], M2[s1])


def test_coloured_schedule_reaches_the_solution_in_about_half_the_sweeps():
    m = W.poisson2d(16)
    b = W.uniform_b(m.n, 3)
    x = np.linalg.solve(W.dense_from_csr(m), b)
    def sweeps(colors):
        R = oracle.Rounds(m, b, colors=colors)
        for t in range(1, 5000):
            R.step()
            mean, _ = R.marginals()
            if np.abs(mean - x).max() <= 1e-10 * np.abs(x).max():
                return t
        raise AssertionError("no convergence")
    s_sync, s_col = sweeps(None), sweeps(_grid_colours(16, 16))
    assert s_col <= 0.6 * s_sync, (s_sync, s_col)


def test_colouring_must_be_proper():
    m = W.poisson2d(4)
    with pytest.raises(ValueError):
        oracle.Rounds(m, np.ones(m.n), colors=np.zeros(m.n, dtype=int))


# ---------------------------------------------------------------------------
# Section VII for any sparse matrix: the first k unknowns of the symmetric
# bipartite system are the regularised least-squares solution, for tall,
# wide and square nonsymmetric S (pinned against a direct solve of the normal
# equations, an independent route).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,k,per_row,psi", [(120, 40, 5, 0.1), (40, 90, 6, 0.5), (60, 60, 4, 0.3)])
def test_bipartite_system_gives_regularised_least_squares(m, k, per_row, psi):
    S = W.sparse_rect(m, k, per_row, seed=m + k).dense()
    assert not np.allclose(S[:min(m, k), :min(m, k)], S[:min(m, k), :min(m, k)].T)
    y = W.normal_b(m, 3)
    mb, rhs = oracle.bipartite_system(S, y, psi)
    r = oracle.solve(mb, rhs, tol=1e-12, max_rounds=20000)
    assert r.status == oracle.OK
    x = np.linalg.solve(S.T @ S + psi * np.eye(k), S.T @ y)
    np.testing.assert_allclose(r.x[:k], x, rtol=0, atol=1e-9 * np.abs(x).max())
    # the auxiliary unknowns are the scaled residual z = (S x - y) / psi
    np.testing.assert_allclose(r.x[k:], (S @ x - y) / psi, rtol=0, atol=1e-8 * np.abs(y).max() / psi)


def test_sparse_bipartite_construction_equals_the_dense_one():
    S = W.sparse_rect(37, 23, 4, seed=5, empty_rows=[3], empty_cols=[7])
    y = W.normal_b(37, 2)
    a, ra = oracle.bipartite_system(S.dense(), y, 0.25)
    b, rb = oracle.bipartite_system_sparse(S.m, S.k, S.row_ptr, S.col, S.val, y, 0.25)
    assert a.n == b.n
    np.testing.assert_array_equal(a.row_ptr, b.row_ptr)
    np.testing.assert_array_equal(a.col, b.col)
    np.testing.assert_array_equal(a.val, b.val)
    np.testing.assert_array_equal(ra, rb)


@pytest.mark.parametrize("m,k,per_row", [(50, 10, 8), (64, 3, 5), (30, 200, 7), (0, 5, 2), (9, 0, 3)])
def test_sparse_rect_generator_structure(m, k, per_row):
    # rows hold distinct sorted columns in range, nothing lands in an empty
    # row or column, and the values are finite and nonzero
    er = [r for r in (0, 4) if r < m]
    ec = [c for c in (1,) if c < k]
    S = W.sparse_rect(m, k, per_row, seed=11, empty_rows=er, empty_cols=ec)
    assert S.row_ptr[0] == 0 and S.row_ptr[-1] == S.col.size == S.val.size
    allowed = max(k - len(ec), 0)
    for j in range(m):
        c = S.col[S.row_ptr[j]:S.row_ptr[j + 1]]
        want = 0 if j in er else min(per_row, allowed)
        assert c.size == want
        assert np.all(np.diff(c) > 0)
        assert np.all((c >= 0) & (c < k))
        assert not np.isin(c, ec).any()
    assert np.all(np.isfinite(S.val)) and np.all(S.val != 0.0)
