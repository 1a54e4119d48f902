"""GPU parity of the section VII least-squares plans for any sparse S against
the FP64 CPU oracle run on oracle.bipartite_system(S, y, psi) (unknowns x
first, then z, the same node order and row ordering as the assembled system),
and solves checked against a direct solve of the regularised normal equations.

Tolerances as in test_gpu_csr.py: trajectories 1e-11 / 1e-10 relative in FP64;
solutions within what the requested residual allows."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import paper_0810_1119_amd as G
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return G


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def _rect(G, S):
    return G.DeviceRect.from_host(S.row_ptr, S.col, S.val, (S.m, S.k))


def _normal_solution(S, y, psi):
    A = S.dense()
    return np.linalg.solve(A.T @ A + psi * np.eye(S.k), A.T @ y)


SHAPES = {
    "tall_240x80": (240, 80, 5, 0.1),
    "wide_70x150": (70, 150, 6, 0.5),
    "square_nonsym_130": (130, 130, 4, 0.3),
    "ragged_1x3": (1, 3, 2, 0.2),
}


@pytest.mark.parametrize("case", sorted(SHAPES))
@pytest.mark.parametrize("col_blocks", [1, 2])
def test_lsq_fp64_trajectory_matches_oracle(G, case, col_blocks):
    """Synchronous rounds of the assembled system against the oracle, with one
    and with two column ranges of the pair layout."""
    m, k, pr, psi = SHAPES[case]
    S = W.sparse_rect(m, k, pr, seed=m * 7 + k)
    y = W.normal_b(m, 5)
    rc, plan = G.gabp_plan_create_lsq(_rect(G, S), psi, G.gabp_default_opts(
        msg_fp32=0, freeze=0, col_blocks=col_blocks))
    assert rc == G.GABP_OK, G.status_name(rc)
    try:
        mb, rhs = oracle.bipartite_system(S.dense(), y, psi)
        assert mb.row_ptr[-1] == 2 * S.nnz + m + k
        assert G.gabp_plan_reset(plan, dev(rhs)) == G.GABP_OK
        R = oracle.Rounds(mb, rhs)
        n, nnz = m + k, 2 * S.nnz + m + k
        for t in range(1, 7):
            R.step()
            assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
            P = torch.zeros(nnz, dtype=torch.float64, device="cuda")
            h = torch.zeros(nnz, dtype=torch.float64, device="cuda")
            assert G.gabp_plan_get_messages(plan, P, h) == G.GABP_OK
            np.testing.assert_allclose(host(P), R.P, rtol=1e-11, atol=1e-13 * np.abs(R.P).max())
            ho = R.information()
            np.testing.assert_allclose(host(h), ho, rtol=1e-10, atol=1e-12 * np.abs(ho).max())
            mean = torch.zeros(n, dtype=torch.float64, device="cuda")
            prec = torch.zeros(n, dtype=torch.float64, device="cuda")
            assert G.gabp_plan_marginals(plan, mean, prec) == G.GABP_OK
            mo, po = R.marginals()
            np.testing.assert_allclose(host(mean), mo, rtol=1e-10, atol=1e-12 * np.abs(mo).max())
            np.testing.assert_allclose(host(prec), po, rtol=1e-10)
    finally:
        G.gabp_plan_destroy(plan)


@pytest.mark.parametrize("case", sorted(SHAPES))
@pytest.mark.parametrize("damping", [0.0, 0.4])
def test_lsq_colored_fp64_trajectory_matches_oracle(G, case, damping):
    """Two-colour schedule: the x rows send, then the z rows; oracle coloured
    rounds with colour 0 on x."""
    m, k, pr, psi = SHAPES[case]
    S = W.sparse_rect(m, k, pr, seed=m * 7 + k)
    y = W.normal_b(m, 5)
    rc, plan = G.gabp_plan_create_lsq(_rect(G, S), psi, G.gabp_default_opts(
        msg_fp32=0, freeze=0, damping=damping, schedule=G.GABP_SCHEDULE_COLORED))
    assert rc == G.GABP_OK, G.status_name(rc)
    try:
        mb, rhs = oracle.bipartite_system(S.dense(), y, psi)
        assert G.gabp_plan_reset(plan, dev(rhs)) == G.GABP_OK
        R = oracle.Rounds(mb, rhs, damping=damping, colors=np.r_[np.zeros(k, int), np.ones(m, int)])
        n, nnz = m + k, 2 * S.nnz + m + k
        for t in range(1, 7):
            R.step()
            assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
            P = torch.zeros(nnz, dtype=torch.float64, device="cuda")
            h = torch.zeros(nnz, dtype=torch.float64, device="cuda")
            assert G.gabp_plan_get_messages(plan, P, h) == G.GABP_OK
            np.testing.assert_allclose(host(P), R.P, rtol=1e-11, atol=1e-13 * np.abs(R.P).max())
            ho = R.information()
            np.testing.assert_allclose(host(h), ho, rtol=1e-10, atol=1e-12 * np.abs(ho).max())
            mean = torch.zeros(n, dtype=torch.float64, device="cuda")
            prec = torch.zeros(n, dtype=torch.float64, device="cuda")
            assert G.gabp_plan_marginals(plan, mean, prec) == G.GABP_OK
            mo, po = R.marginals()
            np.testing.assert_allclose(host(mean), mo, rtol=1e-10, atol=1e-12 * np.abs(mo).max())
            np.testing.assert_allclose(host(prec), po, rtol=1e-10)
    finally:
        G.gabp_plan_destroy(plan)


@pytest.mark.parametrize("fp32,tol", [(1, 1e-8), (0, 1e-11)])
def test_lsq_colored_solve_in_about_half_the_sweeps(G, fp32, tol):
    m, k, pr, psi = SHAPES["tall_240x80"]
    S = W.sparse_rect(m, k, pr, seed=13)
    y = dev(W.normal_b(m, 14))
    res = {}
    for sched in (G.GABP_SCHEDULE_SYNC, G.GABP_SCHEDULE_COLORED):
        x = torch.zeros(k, dtype=torch.float64, device="cuda")
        rc, st = G.gabp_solve_lsq(_rect(G, S), psi, y, x,
                                  G.gabp_default_opts(msg_fp32=fp32, tol=tol, schedule=sched))
        assert rc == G.GABP_OK, G.status_name(rc)
        assert st.rel_residual <= tol
        res[sched] = (host(x), st.sweeps)
    ref = _normal_solution(S, host(y), psi)
    for xs, _ in res.values():
        np.testing.assert_allclose(xs, ref, rtol=0, atol=100 * tol * np.abs(ref).max())
    s_sync, s_col = res[G.GABP_SCHEDULE_SYNC][1], res[G.GABP_SCHEDULE_COLORED][1]
    print(f"sweeps: synchronous {s_sync}, coloured {s_col}", flush=True)
    assert s_col <= 0.65 * s_sync


@pytest.mark.parametrize("case", ["tall_240x80", "wide_70x150", "square_nonsym_130"])
@pytest.mark.parametrize("fp32,tol", [(1, 1e-8), (0, 1e-11)])
def test_lsq_solve_matches_the_normal_equations(G, case, fp32, tol):
    m, k, pr, psi = SHAPES[case]
    S = W.sparse_rect(m, k, pr, seed=m * 7 + k, signs=(case == "tall_240x80"))
    y = W.normal_b(m, 6)
    rc, plan = G.gabp_plan_create_lsq(_rect(G, S), psi, G.gabp_default_opts(msg_fp32=fp32, tol=tol))
    assert rc == G.GABP_OK
    try:
        x = torch.zeros(k, dtype=torch.float64, device="cuda")
        rc, st = G.gabp_plan_solve_lsq(plan, dev(y), x)
        assert rc == G.GABP_OK, G.status_name(rc)
        assert st.rel_residual <= tol
        ref = _normal_solution(S, y, psi)
        # the assembled system's residual bounds the normal-equations residual
        # by about (psi + ||S||) times it, relative to ||S^T y|| <= ||S|| ||y||
        np.testing.assert_allclose(host(x), ref, rtol=0, atol=100 * tol * np.abs(ref).max())
        r = torch.zeros(k, dtype=torch.float64, device="cuda")
        rc, rel = G.gabp_plan_residual_lsq(plan, dev(y), x, r)
        assert rc == G.GABP_OK
        A = S.dense()
        r_ref = A.T @ y - (A.T @ A + psi * np.eye(k)) @ host(x)
        np.testing.assert_allclose(host(r), r_ref, rtol=1e-9, atol=1e-12 * np.abs(A.T @ y).max())
        assert rel == pytest.approx(np.linalg.norm(r_ref) / np.linalg.norm(A.T @ y), rel=1e-9)
        assert rel <= 100 * tol
    finally:
        G.gabp_plan_destroy(plan)


def test_lsq_empty_rows_and_columns(G):
    """A column of S with no entry leaves x_i = 0 (its row of the normal
    equations is psi x_i = 0); an empty row of S leaves z_j = -y_j / psi."""
    m, k, psi = 50, 30, 0.4
    S = W.sparse_rect(m, k, 4, seed=3, empty_rows=[0, 17, 49], empty_cols=[5, 29])
    y = W.normal_b(m, 7)
    x = torch.full((k,), 7.0, dtype=torch.float64, device="cuda")
    rc, st = G.gabp_solve_lsq(_rect(G, S), psi, dev(y), x, G.gabp_default_opts(msg_fp32=0, tol=1e-12))
    assert rc == G.GABP_OK
    xs = host(x)
    assert xs[5] == 0.0 and xs[29] == 0.0
    np.testing.assert_allclose(xs, _normal_solution(S, y, psi), rtol=0, atol=1e-10)


def test_lsq_solve_is_deterministic(G):
    m, k, pr, psi = SHAPES["tall_240x80"]
    S = W.sparse_rect(m, k, pr, seed=9)
    y = dev(W.normal_b(m, 8))
    out = []
    for _ in range(2):
        x = torch.zeros(k, dtype=torch.float64, device="cuda")
        rc, _ = G.gabp_solve_lsq(_rect(G, S), psi, y, x)
        assert rc == G.GABP_OK
        out.append(host(x))
    assert np.array_equal(out[0], out[1])


def test_lsq_error_paths(G):
    S = W.sparse_rect(20, 10, 3, seed=4)
    R = _rect(G, S)
    y = dev(W.normal_b(20, 1))
    x = torch.zeros(10, dtype=torch.float64, device="cuda")
    for psi in (0.0, -1.0, float("nan"), float("inf")):
        assert G.gabp_solve_lsq(R, psi, y, x)[0] == G.GABP_ERR_ARG
    bad = W.sparse_rect(20, 10, 3, seed=4)
    bad.col = bad.col.copy()
    bad.col[1], bad.col[2] = bad.col[2], bad.col[1]  # row 0 no longer sorted
    assert G.gabp_solve_lsq(_rect(G, bad), 0.5, y, x)[0] == G.GABP_ERR_ARG
    bad = W.sparse_rect(20, 10, 3, seed=4)
    bad.col = bad.col.copy()
    bad.col[-1] = 10  # out of range
    assert G.gabp_solve_lsq(_rect(G, bad), 0.5, y, x)[0] == G.GABP_ERR_ARG
    bad = W.sparse_rect(20, 10, 3, seed=4)
    bad.val = bad.val.copy()
    bad.val[4] = np.nan
    assert G.gabp_solve_lsq(_rect(G, bad), 0.5, y, x)[0] == G.GABP_ERR_ARG
    bad = W.sparse_rect(20, 10, 3, seed=4)
    bad.row_ptr = bad.row_ptr.copy()
    bad.row_ptr[-1] -= 1  # last entry not covered
    assert G.gabp_solve_lsq(_rect(G, bad), 0.5, y, x)[0] == G.GABP_ERR_ARG
    rc, plan = G.gabp_plan_create_lsq(R, 0.5, G.gabp_default_opts(
        schedule=G.GABP_SCHEDULE_COLORED, layout=G.GABP_LAYOUT_GATHER))
    assert rc == G.GABP_ERR_UNSUPPORTED and plan is None
    # a CSR plan is not an lsq plan
    rc, csr = G.gabp_plan_create(G.DeviceCSR.from_host(W.sdd_random(16, 1)))
    r = G.lib.gabp_plan_solve_lsq(csr.ptr, G._abi._ptr(y), G._abi._ptr(x), None, None)
    assert r == G.GABP_ERR_ARG
    G.gabp_plan_destroy(csr)


@pytest.mark.slow
def test_lsq_large_sparse_tall(G):
    """2^18 x 2^16 with 6 nonzeros per row: every step on the device, checked
    by the normal-equations residual (FP64, recomputed by the library and on
    the CPU)."""
    m, k, pr, psi = 1 << 18, 1 << 16, 6, 0.2
    S = W.sparse_rect(m, k, pr, seed=21)
    y = W.normal_b(m, 9)
    rc, plan = G.gabp_plan_create_lsq(_rect(G, S), psi)
    assert rc == G.GABP_OK
    try:
        x = torch.zeros(k, dtype=torch.float64, device="cuda")
        rc, st = G.gabp_plan_solve_lsq(plan, dev(y), x)
        assert rc == G.GABP_OK, G.status_name(rc)
        rc, rel = G.gabp_plan_residual_lsq(plan, dev(y), x)
        rows = np.repeat(np.arange(m), np.diff(S.row_ptr))
        xs = host(x)
        u = y - np.bincount(rows, weights=S.val * xs[S.col], minlength=m)
        r = np.bincount(S.col, weights=S.val * u[rows], minlength=k) - psi * xs
        aty = np.bincount(S.col, weights=S.val * y[rows], minlength=k)
        rel_cpu = np.linalg.norm(r) / np.linalg.norm(aty)
        assert rel == pytest.approx(rel_cpu, rel=1e-6)
        assert rel <= 1e-6
        print(f"lsq 2^18 x 2^16: {st.sweeps} sweeps, {st.seconds * 1e3:.1f} ms, "
              f"normal-equations residual {rel:.1e}", flush=True)
    finally:
        G.gabp_plan_destroy(plan)


def test_coloured_settled_phase_stays_consistent(G):
    """Regression: the coloured schedule rebuilds in-messages from the senders'
    broadcasts, which is exact only while every rebuilt value rounds like the
    sent one; an inconsistency (the settled-phase coefficients once rounded
    differently from the full sweeps' factors) is not damped by the iteration
    and grew from FP32 rounding to overflow within ~30 settled sweeps.  One
    long FP32 pass must stay at the message precision's floor."""
    m, k = 1 << 18, 1 << 16
    S = W.sparse_rect(m, k, 8, seed=0)
    y = dev(W.normal_b(m, 0))
    R = _rect(G, S)
    for sweeps in (24, 64):
        x = torch.zeros(k, dtype=torch.float64, device="cuda")
        rc, st = G.gabp_solve_lsq(R, 0.1, y, x, G.gabp_default_opts(
            schedule=G.GABP_SCHEDULE_COLORED, max_restarts=0, max_sweeps=sweeps, inner_tol=1e-30))
        assert rc in (G.GABP_OK, G.GABP_NOT_CONVERGED), G.status_name(rc)
        assert st.frozen_sweeps > 0 and st.rel_residual < 1e-5, (sweeps, st.rel_residual)
