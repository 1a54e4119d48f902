"""GPU parity of the general-CSR path (HIP kernels through the C ABI) against
the FP64 CPU oracle.

Tolerances:
  * FP64 messages: each message is a handful of FP64 operations on values of
    the previous round; the GPU (information form, tree-shaped lane sums) and
    the oracle ((P, mu) form, sequential sums) round differently, so per-round
    agreement is held to 1e-11 relative over the first rounds.
  * FP32 messages: one rounding of 2^-24 per operation, about deg + 6 operations
    per message and a few rounds of propagation: 2e-5 relative after 4 rounds
    (entries near zero use an absolute floor of the same size times the scale).
  * Solves: the FP64 relative residual ||b - A x|| / ||b|| is recomputed on the
    CPU by the oracle and must meet the requested tolerance; the error against
    the oracle's own converged solution is reported and bounded by
    cond-based slack (checked loosely).
"""
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


def _plan(G, m, fp32, **kw):
    A = G.DeviceCSR.from_host(m)
    rc, plan = G.gabp_plan_create(A, G.gabp_default_opts(msg_fp32=int(fp32), **kw))
    assert rc == G.GABP_OK, G.status_name(rc)
    return A, plan


def _messages(G, plan, nnz):
    P = torch.zeros(nnz, dtype=torch.float64, device="cuda")
    h = torch.zeros(nnz, dtype=torch.float64, device="cuda")
    assert G.gabp_plan_get_messages(plan, P, h) == G.GABP_OK
    return host(P), host(h)


def _marginals(G, plan, n):
    mean = torch.empty(n, dtype=torch.float64, device="cuda")
    prec = torch.empty(n, dtype=torch.float64, device="cuda")
    assert G.gabp_plan_marginals(plan, mean, prec) == G.GABP_OK
    return host(mean), host(prec)


def test_toy_tree_table_on_gpu(G):
    """Section VIII-A message table, FP64 on the GPU (h = P * mu)."""
    from golden_io import lines, num, read_matrix
    it = lines("toy_tree.txt")
    tok = next(it)
    A = read_matrix(it, int(tok[1]))
    rec = {"msg": [], "mean": []}
    b = None
    for t in it:
        if t[0] == "b":
            b = np.array([num(v) for v in t[1:]])
        elif t[0] in rec:
            rec[t[0]].append(t[1:])
    m = W.csr_from_dense(A)
    Ad, plan = _plan(G, m, fp32=False)
    assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
    slot = {(i, int(m.col[e])): e for i in range(3) for e in range(m.row_ptr[i], m.row_ptr[i + 1])}
    for t in range(4):
        if t:
            assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
        P, h = _messages(G, plan, m.nnz)
        exp = {}
        for kind, i, j, *vals in rec["msg"]:
            exp[(kind, int(i), int(j))] = num(vals[t])
        for (i, j), e in slot.items():
            if i == j:
                continue
            Pe, mue = exp[("P", i, j)], exp[("mu", i, j)]
            assert P[e] == pytest.approx(Pe, abs=1e-14), (i, j, t)
            assert h[e] == pytest.approx(Pe * mue, abs=1e-13), (i, j, t)
        mean, _ = _marginals(G, plan, 3)
        for i, *vals in rec["mean"]:
            assert mean[int(i)] == pytest.approx(num(vals[t]), abs=1e-13), (i, t)
    G.gabp_plan_destroy(plan)


LAYOUT = {"pair": 0, "gather": 1}

CASES = {
    "sdd_ragged": lambda: W.sdd_random(3001, 5),
    "poisson2d_33": lambda: W.poisson2d(33),
    "poisson3d_13x11x7": lambda: W.poisson3d(13, 11, 7, 0.01),
    "varcoef_9x7x5": lambda: W.poisson3d_varcoef(9, 7, 5, 2)[0],
    "tree_777": lambda: W.random_tree(777, 3, dominant=False),
    "dense_rows_60": lambda: W.csr_from_dense(
        (lambda a: a + a.T + np.diag(2 * np.abs(a).sum(1) + 1))(
            np.random.default_rng(1).standard_normal((60, 60)))),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("layout,group", [("pair", 0), ("gather", 0), ("gather", 4),
                                          ("gather", 16), ("gather", 64)])
def test_fp64_trajectory_matches_oracle(G, case, group, layout):
    """Round-by-round FP64 messages and means against Algorithm 2 of the oracle,
    for both message layouts and, in the gather layout (the only one with
    lane groups), several lanes-per-row choices (each covers several blocks
    and a ragged last block)."""
    m = CASES[case]()
    b = W.uniform_b(m.n, 1)
    Ad, plan = _plan(G, m, fp32=False, group=group, layout=LAYOUT[layout])
    assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
    R = oracle.Rounds(m, b, algorithm=2)
    for t in range(1, 7):
        R.step()
        assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
        P, h = _messages(G, plan, m.nnz)
        Po, ho = R.P, R.information()
        sP, sh = np.abs(Po).max(), np.abs(ho).max() + 1e-300
        np.testing.assert_allclose(P, Po, rtol=1e-11, atol=1e-13 * sP, err_msg=f"P round {t}")
        np.testing.assert_allclose(h, ho, rtol=1e-10, atol=1e-12 * sh, err_msg=f"h round {t}")
        mean, prec = _marginals(G, plan, m.n)
        mo, po = R.marginals()
        np.testing.assert_allclose(mean, mo, rtol=1e-10, atol=1e-12 * np.abs(mo).max())
        # P_i sums terms much larger than itself on non-dominant graphs: the
        # rounding scales with sum |P_ki|, hence 1e-10 rather than 1e-12
        np.testing.assert_allclose(prec, po, rtol=1e-10, atol=1e-13 * np.abs(po).max())
    G.gabp_plan_destroy(plan)


@pytest.mark.parametrize("case", ["sdd_ragged", "poisson3d_13x11x7", "varcoef_9x7x5"])
@pytest.mark.parametrize("layout", ["pair", "gather"])
def test_fp32_trajectory_matches_oracle(G, case, layout):
    m = CASES[case]()
    b = W.uniform_b(m.n, 2)
    Ad, plan = _plan(G, m, fp32=True, layout=LAYOUT[layout])
    assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
    R = oracle.Rounds(m, b, algorithm=2)
    for t in range(1, 5):
        R.step()
        assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
        P, h = _messages(G, plan, m.nnz)
        np.testing.assert_allclose(P, R.P, rtol=2e-5, atol=2e-6 * np.abs(R.P).max())
        ho = R.information()
        np.testing.assert_allclose(h, ho, rtol=2e-5, atol=2e-5 * np.abs(ho).max())
    G.gabp_plan_destroy(plan)


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.7])
@pytest.mark.parametrize("layout", ["pair", "gather"])
def test_damped_trajectory_matches_oracle(G, layout, alpha):
    """Damping of section VI-D as the oracle reads it (P and h = P mu mixed as
    alpha old + (1 - alpha) new); alpha != 1/2 tells alpha from 1 - alpha."""
    m = W.poisson3d(10, 9, 8, 0.01)
    b = W.uniform_b(m.n, 3)
    Ad, plan = _plan(G, m, fp32=False, damping=alpha, layout=LAYOUT[layout])
    assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
    R = oracle.Rounds(m, b, algorithm=2, damping=alpha)
    for t in range(1, 6):
        R.step()
        assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
        P, h = _messages(G, plan, m.nnz)
        np.testing.assert_allclose(P, R.P, rtol=1e-12, atol=1e-14)
        ho = R.information()
        np.testing.assert_allclose(h, ho, rtol=1e-10, atol=1e-12 * np.abs(ho).max())
    G.gabp_plan_destroy(plan)


def _hub_chain(leaves, seed):
    """A hub joined to every leaf and the leaves joined in a chain, diagonally
    dominant: the hub's row holds more slots than two chunks of a row block
    (1024 slots each) of the pair sweeps."""
    rng = np.random.default_rng(seed)
    r = np.concatenate([np.zeros(leaves, dtype=np.int64), np.arange(1, leaves)])
    c = np.concatenate([np.arange(1, leaves + 1), np.arange(2, leaves + 1)])
    v = rng.standard_normal(r.size)
    n = leaves + 1
    rows, cols, vals = np.concatenate([r, c]), np.concatenate([c, r]), np.concatenate([v, v])
    d = np.zeros(n)
    np.add.at(d, rows, np.abs(vals))
    return W.csr_from_coo(n, np.concatenate([rows, np.arange(n)]),
                          np.concatenate([cols, np.arange(n)]),
                          np.concatenate([vals, 1.1 * d + 0.1]))


@pytest.mark.parametrize("case", ["hub_2600", "sdd_ragged"])
@pytest.mark.parametrize("fp32", [False, True])
def test_pair_row_blocks_long_rows_and_grid_stride(G, case, fp32):
    """Synchronous pair sweeps with a two-block grid, so every block walks many
    row blocks, and (hub) one row spread over three slot chunks: the messages
    follow Algorithm 2 of the oracle round by round."""
    m = _hub_chain(2600, 4) if case == "hub_2600" else CASES[case]()
    b = W.uniform_b(m.n, 6)
    Ad, plan = _plan(G, m, fp32=fp32, grid_blocks=2)
    assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
    R = oracle.Rounds(m, b, algorithm=2)
    # FP32: the hub sums 2600 in-messages in sequence; the worst-case bound of
    # such a sum is about count * 2^-24 = 1.5e-4 of the summed magnitudes
    rtol = (1e-4 if case == "hub_2600" else 2e-5) if fp32 else 1e-10
    for t in range(1, 5):
        R.step()
        assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
        P, h = _messages(G, plan, m.nnz)
        ho = R.information()
        np.testing.assert_allclose(P, R.P, rtol=rtol, atol=rtol * 0.1 * np.abs(R.P).max(),
                                   err_msg=f"P round {t}")
        np.testing.assert_allclose(h, ho, rtol=rtol, atol=rtol * np.abs(ho).max(),
                                   err_msg=f"h round {t}")
        mean, prec = _marginals(G, plan, m.n)
        mo, po = R.marginals()
        np.testing.assert_allclose(prec, po, rtol=rtol, atol=rtol * 0.1 * np.abs(po).max())
        np.testing.assert_allclose(mean, mo, rtol=rtol, atol=rtol * np.abs(mo).max())
    G.gabp_plan_destroy(plan)


# FP32 on the diagonally dominant cases only, as for one range: the trees and
# dense rows here are not dominant, and their small cavities amplify FP32
# rounding beyond a fixed tolerance
@pytest.mark.parametrize("case,fp32", [(c, False) for c in sorted(CASES)] +
                         [(c, True) for c in ("sdd_ragged", "poisson3d_13x11x7", "varcoef_9x7x5")])
def test_two_column_ranges_trajectory_matches_oracle(G, case, fp32):
    """Pair layout with two column ranges (each sweep one launch per range,
    node sums carried from the first to the second): round-by-round messages
    and marginals follow Algorithm 2 of the oracle."""
    m = CASES[case]()
    b = W.uniform_b(m.n, 7)
    Ad, plan = _plan(G, m, fp32=fp32, col_blocks=2)
    assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
    R = oracle.Rounds(m, b, algorithm=2)
    rtol = 2e-5 if fp32 else 1e-10
    for t in range(1, 5):
        R.step()
        assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
        P, h = _messages(G, plan, m.nnz)
        ho = R.information()
        np.testing.assert_allclose(P, R.P, rtol=rtol, atol=rtol * 0.1 * np.abs(R.P).max(),
                                   err_msg=f"P round {t}")
        np.testing.assert_allclose(h, ho, rtol=rtol, atol=rtol * np.abs(ho).max(),
                                   err_msg=f"h round {t}")
        mean, prec = _marginals(G, plan, m.n)
        mo, po = R.marginals()
        np.testing.assert_allclose(prec, po, rtol=rtol, atol=rtol * 0.1 * np.abs(po).max())
        np.testing.assert_allclose(mean, mo, rtol=rtol, atol=rtol * np.abs(mo).max())
    G.gabp_plan_destroy(plan)


def test_two_column_ranges_damped_and_resumed_bitwise(G):
    """Two column ranges: damped rounds follow the oracle, and exported
    messages resume a plan bit for bit (5 + 5 sweeps == 10 sweeps)."""
    m = W.poisson3d(10, 9, 8, 0.01)
    b = W.uniform_b(m.n, 3)
    Ad, plan = _plan(G, m, fp32=False, damping=0.3, col_blocks=2)
    assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
    R = oracle.Rounds(m, b, algorithm=2, damping=0.3)
    for t in range(1, 5):
        R.step()
        assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
        P, h = _messages(G, plan, m.nnz)
        np.testing.assert_allclose(P, R.P, rtol=1e-12, atol=1e-14)
        ho = R.information()
        np.testing.assert_allclose(h, ho, rtol=1e-10, atol=1e-12 * np.abs(ho).max())
    G.gabp_plan_destroy(plan)
    m = W.sdd_random(4001, 9)
    b = W.normal_b(m.n, 9)
    _, p1 = _plan(G, m, fp32=True, col_blocks=2)
    G.gabp_plan_reset(p1, dev(b)); G.gabp_plan_sweeps(p1, 10)
    P10, h10 = _messages(G, p1, m.nnz)
    _, p2 = _plan(G, m, fp32=True, col_blocks=2)
    G.gabp_plan_reset(p2, dev(b)); G.gabp_plan_sweeps(p2, 5)
    P5, h5 = _messages(G, p2, m.nnz)
    _, p3 = _plan(G, m, fp32=True, col_blocks=2)
    G.gabp_plan_reset(p3, dev(b))
    assert G.gabp_plan_set_messages(p3, dev(P5), dev(h5)) == G.GABP_OK
    G.gabp_plan_sweeps(p3, 5)
    P, h = _messages(G, p3, m.nnz)
    assert np.array_equal(P, P10) and np.array_equal(h, h10)
    for p in (p1, p2, p3):
        G.gabp_plan_destroy(p)


@pytest.mark.parametrize("col_blocks", [1, 2])
def test_column_ranges_solve_refined_with_settled_phase(G, col_blocks):
    """FP32 + FP64 refinement to 1e-8 with one or two column ranges, through
    the settled-precision phase; the plan reports its launches per sweep."""
    m = W.sdd_random(20011, 4)
    b = W.normal_b(m.n, 4)
    rc, st, x = _solve(G, m, b, msg_fp32=1, tol=1e-8, col_blocks=col_blocks)
    assert rc == G.GABP_OK, G.status_name(rc)
    assert st.frozen_sweeps > 0 and st.sweep_launches == col_blocks
    _, rn = oracle.residual(m, b, x)
    assert rn / np.linalg.norm(b) <= 1e-8


def test_column_ranges_automatic_choice(G):
    """Default choice: two ranges for a random graph whose FP32 node table
    exceeds 4 MiB, one for a naturally ordered grid of the same size (its
    edges join nearby indices) and for small graphs; either way the solve
    meets 1e-8."""
    for m, want in ((W.sdd_random(600_000, 2), 2), (W.poisson3d(90, 90, 80, 0.01), 1),
                    (W.sdd_random(3001, 5), 1)):
        b = W.normal_b(m.n, 1)
        rc, st, x = _solve(G, m, b, msg_fp32=1, tol=1e-8)
        assert rc == G.GABP_OK, G.status_name(rc)
        assert st.sweep_launches == want, (m.n, st.sweep_launches)
        _, rn = oracle.residual(m, b, x)
        assert rn / np.linalg.norm(b) <= 1e-8


def test_column_ranges_option_checks(G):
    m = W.sdd_random(200, 1)
    A = G.DeviceCSR.from_host(m)
    rc, plan = G.gabp_plan_create(A, G.gabp_default_opts(col_blocks=3))
    assert rc == G.GABP_ERR_ARG and plan is None
    rc, plan = G.gabp_plan_create(A, G.gabp_default_opts(col_blocks=2, layout=1))
    assert rc == G.GABP_ERR_UNSUPPORTED and plan is None
    rc, plan = G.gabp_plan_create(A, G.gabp_default_opts(col_blocks=2,
                                                         schedule=G.GABP_SCHEDULE_COLORED))
    assert rc == G.GABP_ERR_UNSUPPORTED and plan is None


def test_pair_hub_solve_settled_phase_small_grid(G):
    """FP32 solve of the hub graph to 1e-8 with a two-block grid: the check
    sweeps' block maxima and the settled-precision kernel walk many row
    blocks, the hub's row spans several chunks."""
    m = _hub_chain(2600, 5)
    b = W.normal_b(m.n, 5)
    rc, st, x = _solve(G, m, b, msg_fp32=1, tol=1e-8, grid_blocks=2)
    assert rc == G.GABP_OK, G.status_name(rc)
    assert st.frozen_sweeps > 0
    _, rn = oracle.residual(m, b, x)
    assert rn / np.linalg.norm(b) <= 1e-8


def test_tree_exact_after_diameter_on_gpu(G):
    """Trees: exact means and precisions after diameter sweeps (section IV)."""
    m = W.random_tree(300, 8, dominant=False)
    b = W.normal_b(m.n, 8)
    A = W.dense_from_csr(m)
    Ad, plan = _plan(G, m, fp32=False)
    assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
    assert G.gabp_plan_sweeps(plan, W.tree_diameter(m)) == G.GABP_OK
    mean, prec = _marginals(G, plan, m.n)
    x = np.linalg.solve(A, b)
    np.testing.assert_allclose(mean, x, rtol=1e-8, atol=1e-9 * np.abs(x).max())
    np.testing.assert_allclose(1 / prec, np.diag(np.linalg.inv(A)), rtol=1e-8, atol=1e-12)
    G.gabp_plan_destroy(plan)


def _solve(G, m, b, **kw):
    A = G.DeviceCSR.from_host(m)
    bd = dev(b)
    x = torch.zeros(m.n, dtype=torch.float64, device="cuda")
    rc, st = G.gabp_solve(A, bd, x, opts=G.gabp_default_opts(**kw))
    return rc, st, host(x)


def test_poisson32_fp64_to_1e10(G):
    """2-D Poisson 32 x 32, FP64 messages, to relative residual 1e-10."""
    m = W.poisson2d(32)
    b = W.uniform_b(m.n, 0)
    rc, st, x = _solve(G, m, b, msg_fp32=0, tol=1e-10)
    assert rc == G.GABP_OK, G.status_name(rc)
    _, rn = oracle.residual(m, b, x)
    assert rn / np.linalg.norm(b) <= 1e-10
    assert st.rel_residual == pytest.approx(rn / np.linalg.norm(b), rel=1e-6)
    ref = oracle.solve(m, b, tol=1e-12, max_rounds=50000)
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) < 1e-8


@pytest.mark.parametrize("n,seed", [(20011, 1), (257, 2)])
@pytest.mark.parametrize("variant", [dict(layout=0, freeze=1), dict(layout=0, freeze=0),
                                     dict(layout=1)])
def test_sdd_fp32_refined_to_1e8(G, n, seed, variant):
    """Random SDD, FP32 messages + FP64 refinement to 1e-8 (Theorem 1 class),
    pair layout with and without the settled-precision phase, gather layout."""
    m = W.sdd_random(n, seed)
    b = W.normal_b(n, seed)
    rc, st, x = _solve(G, m, b, msg_fp32=1, tol=1e-8, **variant)
    if variant.get("layout") == 0 and variant.get("freeze"):
        assert st.frozen_sweeps > 0
    else:
        assert st.frozen_sweeps == 0
    assert rc == G.GABP_OK, G.status_name(rc)
    _, rn = oracle.residual(m, b, x)
    assert rn / np.linalg.norm(b) <= 1e-8
    ref = oracle.solve(m, b, tol=1e-13, max_rounds=2000)
    err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    assert err < 1e-7, err
    assert st.restarts >= 1  # FP32 alone stalls near 1e-7: refinement must have run


def test_poisson3d_fp32_damped_refined(G):
    m = W.poisson3d(12, 10, 9, 0.01)
    b = W.uniform_b(m.n, 5)
    rc, st, x = _solve(G, m, b, msg_fp32=1, tol=1e-8, damping=0.5)
    assert rc == G.GABP_OK, G.status_name(rc)
    _, rn = oracle.residual(m, b, x)
    assert rn / np.linalg.norm(b) <= 1e-8


def test_nonpsd_and_gold_codes_on_gpu(G):
    from golden_io import lines, read_matrix
    it = lines("nonpsd.txt")
    tok = next(it)
    A = read_matrix(it, int(tok[1]))
    rc, st, x = _solve(G, W.csr_from_dense(A), np.ones(3), msg_fp32=0, tol=1e-12)
    assert rc == G.GABP_OK
    np.testing.assert_allclose(x, np.linalg.solve(A, np.ones(3)), rtol=1e-10)


def test_residual_entry_point(G):
    m = W.sdd_random(5003, 4)
    rng = np.random.default_rng(0)
    b, x = rng.standard_normal(m.n), rng.standard_normal(m.n)
    A = G.DeviceCSR.from_host(m)
    r = torch.empty(m.n, dtype=torch.float64, device="cuda")
    rc, rel = G.gabp_residual(A, dev(b), dev(x), r)
    assert rc == G.GABP_OK
    ro, rn = oracle.residual(m, b, x)
    np.testing.assert_allclose(host(r), ro, rtol=1e-12, atol=1e-12)
    assert rel == pytest.approx(rn / np.linalg.norm(b), rel=1e-12)


def test_error_paths_on_gpu(G):
    def status(a, b):
        return _solve(G, W.csr_from_dense(a), b)[0]
    assert status(np.array([[0.0, 1.0], [1.0, 2.0]]), np.ones(2)) == G.GABP_ERR_ZERO_DIAG
    assert status(np.array([[2.0, 1.0], [1.5, 2.0]]), np.ones(2)) == G.GABP_ERR_NOT_SYMMETRIC
    A = np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 1.0], [0.0, 1.0, 1.0]])
    assert _solve(G, W.csr_from_dense(A), np.ones(3), msg_fp32=0)[0] == G.GABP_ERR_BREAKDOWN
    assert status(np.array([[2.0, 1.0], [1.0, 2.0]]), np.array([1.0, np.nan])) == G.GABP_ERR_ARG
    m = W.poisson2d(16)
    rc, st, _ = _solve(G, m, W.uniform_b(m.n, 0), max_sweeps=4, max_restarts=0)
    assert rc == G.GABP_NOT_CONVERGED and st.sweeps == 4
    # unsorted columns in a row
    bad = W.poisson2d(3)
    bad.col = bad.col.copy()
    bad.col[[0, 1]] = bad.col[[1, 0]]
    assert _solve(G, bad, np.ones(9))[0] == G.GABP_ERR_ARG
    # pattern asymmetry: drop one off-diagonal entry
    A = W.dense_from_csr(W.poisson2d(3))
    A[0, 1] = 0.0
    assert status(A, np.ones(9)) == G.GABP_ERR_NOT_SYMMETRIC


def test_edge_cases(G):
    # no off-diagonal entries: x = b / diag
    d = np.array([2.0, -4.0, 0.5])
    rc, st, x = _solve(G, W.csr_from_dense(np.diag(d)), np.array([1.0, 2.0, 3.0]))
    assert rc == G.GABP_OK
    np.testing.assert_allclose(x, [0.5, -0.5, 6.0], rtol=1e-7)
    # zero right-hand side
    m = W.poisson2d(5)
    rc, st, x = _solve(G, m, np.zeros(m.n))
    assert rc == G.GABP_OK and np.all(x == 0)
    # a 2-node system (single edge), FP64
    rc, st, x = _solve(G, W.csr_from_dense(np.array([[3.0, 1.0], [1.0, 2.0]])), np.array([1.0, 1.0]),
                       msg_fp32=0, tol=1e-14)
    assert rc == G.GABP_OK
    np.testing.assert_allclose(x, np.linalg.solve([[3, 1], [1, 2]], [1, 1]), rtol=1e-13)


@pytest.mark.parametrize("layout", ["pair", "gather"])
def test_checkpoint_resume_bitwise(G, layout):
    """Exported messages restore a plan exactly: 5 + 5 sweeps == 10 sweeps."""
    m = W.sdd_random(4001, 9)
    b = W.normal_b(m.n, 9)
    L = LAYOUT[layout]
    _, p1 = _plan(G, m, fp32=True, layout=L)
    G.gabp_plan_reset(p1, dev(b)); G.gabp_plan_sweeps(p1, 10)
    P10, h10 = _messages(G, p1, m.nnz)
    _, p2 = _plan(G, m, fp32=True, layout=L)
    G.gabp_plan_reset(p2, dev(b)); G.gabp_plan_sweeps(p2, 5)
    P5, h5 = _messages(G, p2, m.nnz)
    _, p3 = _plan(G, m, fp32=True, layout=L)
    G.gabp_plan_reset(p3, dev(b))
    assert G.gabp_plan_set_messages(p3, dev(P5), dev(h5)) == G.GABP_OK
    G.gabp_plan_sweeps(p3, 5)
    P, h = _messages(G, p3, m.nnz)
    assert np.array_equal(P, P10) and np.array_equal(h, h10)
    for p in (p1, p2, p3):
        G.gabp_plan_destroy(p)


def test_solve_is_deterministic(G):
    m = W.sdd_random(30011, 3)
    b = W.normal_b(m.n, 3)
    x1 = _solve(G, m, b)[2]
    x2 = _solve(G, m, b)[2]
    assert np.array_equal(x1, x2)


@pytest.mark.slow
def test_c2_full_size_fp32_refined(G):
    """The benchmark configuration: n = 2^20 random SDD, about 8 off-diagonals
    per row, FP32 messages + FP64 refinement to 1e-8, default launch shape.
    Checked with the oracle's FP64 residual on the whole system and against the
    oracle's converged solution."""
    n = 1 << 20
    m = W.sdd_random(n, 0)
    b = W.normal_b(n, 0)
    rc, st, x = _solve(G, m, b, msg_fp32=1, tol=1e-8)
    assert rc == G.GABP_OK, G.status_name(rc)
    _, rn = oracle.residual(m, b, x)
    rel = rn / np.linalg.norm(b)
    assert rel <= 1e-8 and st.rel_residual == pytest.approx(rel, rel=1e-6)
    ref = oracle.solve(m, b, tol=1e-12, max_rounds=500)
    assert ref.status == oracle.OK
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) < 1e-7
