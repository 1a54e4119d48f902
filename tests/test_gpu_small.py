"""GPU parity of batches of small sparse instances (GABP_BATCH_CSR: one
workgroup per instance, messages in LDS) and of Aitken's and Steffensen's
acceleration (section IV-A) against the FP64 CPU oracle.

A batch is the block-diagonal matrix of its instances; GaBP on a
block-diagonal matrix is GaBP on each block, so the oracle runs on the whole
matrix and every instance is compared with its own rows.

Tolerances: as for the general CSR path (per-sweep FP64 messages and means
1e-11 / 1e-10 relative, FP32 2e-5); stop sweeps and extrapolated answers
against the oracle's own run with the same stop rule (the FP64 residual
crosses the tolerance at the same sweep unless the two roundings straddle it:
one sweep, or one sample, of slack)."""
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


def _dense_sdd(n, seed):
    a = np.random.default_rng(seed).standard_normal((n, n))
    a = a + a.T
    np.fill_diagonal(a, 0.0)
    return W.csr_from_dense(a + np.diag(1.2 * np.abs(a).sum(1) + 0.5))


def _uneven_blocks():
    """Instances of different size, degree and structure: a 2-D grid, a tree
    (indefinite diagonal), a random SDD graph, a variable-coefficient 3-D grid,
    a dense row set (degree 39: slot data read from memory), a single node, an
    empty instance and a ragged 2-D grid."""
    return [W.poisson2d(7), W.random_tree(200, 4), W.sdd_random(301, 6),
            W.poisson3d_varcoef(5, 4, 3, 7)[0], _dense_sdd(40, 8),
            W.csr_from_dense(np.array([[2.5]])), W.csr_from_dense(np.zeros((0, 0))),
            W.poisson2d_rect(13, 5)]


def _batch(G, blocks, **kw):
    m = W.block_diag_csr(blocks)
    B = G.DeviceBatch.sparse([b.n for b in blocks], m)
    rc, plan = G.gabp_plan_create_batched(B, G.gabp_default_opts(**kw))
    assert rc == G.GABP_OK, G.status_name(rc)
    return m, B, plan


def _state(G, plan, m):
    P = torch.zeros(m.nnz, dtype=torch.float64, device="cuda")
    h = torch.zeros(m.nnz, dtype=torch.float64, device="cuda")
    assert G.gabp_plan_get_messages(plan, P, h) == G.GABP_OK
    mean = torch.empty(m.n, dtype=torch.float64, device="cuda")
    prec = torch.empty(m.n, dtype=torch.float64, device="cuda")
    assert G.gabp_plan_marginals(plan, mean, prec) == G.GABP_OK
    return host(P), host(h), host(mean), host(prec)


def _colors(G, plan, m):
    rc, col, nc = G.gabp_plan_colors(plan)
    assert rc == G.GABP_OK
    col = host(col)
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    off = rows != np.asarray(m.col)
    assert np.all(col[rows[off]] != col[np.asarray(m.col)[off]]), "colouring is not proper"
    assert col.max() < nc
    return col


@pytest.mark.parametrize("schedule", ["sync", "colored"])
@pytest.mark.parametrize("alpha", [0.0, 0.3])
def test_fp64_trajectory_matches_oracle(G, schedule, alpha):
    print(f"case: small batch FP64 trajectory {schedule} alpha={alpha}", flush=True)
    blocks = _uneven_blocks()
    sch = G.GABP_SCHEDULE_COLORED if schedule == "colored" else G.GABP_SCHEDULE_SYNC
    m, B, plan = _batch(G, blocks, msg_fp32=0, damping=alpha, schedule=sch)
    b = W.uniform_b(m.n, 11)
    colors = _colors(G, plan, m) if schedule == "colored" else None
    R = oracle.Rounds(m, b, algorithm=2, damping=alpha, colors=colors)
    assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
    for t in range(1, 7):
        R.step()
        assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
        P, h, mean, prec = _state(G, plan, m)
        Po, ho = R.P, R.information()
        np.testing.assert_allclose(P, Po, rtol=1e-11, atol=1e-13 * np.abs(Po).max(),
                                   err_msg=f"P sweep {t}")
        np.testing.assert_allclose(h, ho, rtol=1e-10, atol=1e-12 * np.abs(ho).max(),
                                   err_msg=f"h sweep {t}")
        mo, po = R.marginals()
        np.testing.assert_allclose(mean, mo, rtol=1e-10, atol=1e-12 * np.abs(mo).max())
        np.testing.assert_allclose(prec, po, rtol=1e-10, atol=1e-13 * np.abs(po).max())
    G.gabp_plan_destroy(plan)


def test_fp32_trajectory_matches_oracle(G):
    print("case: small batch FP32 trajectory", flush=True)
    blocks = [W.poisson2d(9), W.sdd_random(500, 2), W.poisson3d(6, 5, 4, 0.01)]
    m, B, plan = _batch(G, blocks, msg_fp32=1)
    b = W.uniform_b(m.n, 12)
    R = oracle.Rounds(m, b, algorithm=2)
    assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
    for t in range(1, 5):
        R.step()
        assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
        P, h, _, _ = _state(G, plan, m)
        np.testing.assert_allclose(P, R.P, rtol=2e-5, atol=2e-6 * np.abs(R.P).max())
        ho = R.information()
        np.testing.assert_allclose(h, ho, rtol=2e-5, atol=2e-5 * np.abs(ho).max())
    G.gabp_plan_destroy(plan)


def test_rows_beyond_one_per_thread(G):
    """Instances of 1025..4096 rows take up to four rows per thread."""
    print("case: small batch 4 rows per thread", flush=True)
    blocks = [W.poisson2d_rect(40, 30), W.sdd_random(1030, 3)]
    m, B, plan = _batch(G, blocks, msg_fp32=1)
    b = W.uniform_b(m.n, 13)
    R = oracle.Rounds(m, b, algorithm=2)
    assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
    for t in range(1, 4):
        R.step()
        assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
        P, h, mean, _ = _state(G, plan, m)
        np.testing.assert_allclose(P, R.P, rtol=2e-5, atol=2e-6 * np.abs(R.P).max())
        ho = R.information()
        np.testing.assert_allclose(h, ho, rtol=2e-5, atol=2e-5 * np.abs(ho).max())
    rc, per, summ = G.gabp_plan_solve_batched(plan, dev(b), torch.zeros(m.n, dtype=torch.float64,
                                                                         device="cuda"))
    assert rc == G.GABP_OK and all(p.rel_residual <= 1e-8 for p in per)
    G.gabp_plan_destroy(plan)


def _solve(G, blocks, b, **kw):
    m = W.block_diag_csr(blocks)
    B = G.DeviceBatch.sparse([q.n for q in blocks], m)
    x = torch.full((m.n,), np.nan, dtype=torch.float64, device="cuda")
    rc, per, summ = G.gabp_solve_batched(B, dev(b), x, G.gabp_default_opts(**kw))
    return rc, per, summ, host(x)


def test_poisson32_fp64_stops_where_the_oracle_does(G):
    """The 32 x 32 Poisson system in FP64 to 1e-10, checked every sweep: the
    solve stops at the oracle's round (same residual stop rule) with its x."""
    print("case: small batch Poisson 32^2 FP64 to 1e-10", flush=True)
    m = W.poisson2d(32)
    b = W.uniform_b(m.n, 0)
    ref = oracle.solve(m, b, tol=1e-10, max_rounds=20000)
    assert ref.status == oracle.OK
    rc, per, summ, x = _solve(G, [m], b, msg_fp32=0, tol=1e-10, check_every=1,
                              max_sweeps=50000)
    assert rc == G.GABP_OK
    assert abs(per[0].sweeps - ref.rounds) <= 1, (per[0].sweeps, ref.rounds)
    _, rn = oracle.residual(m, b, x)
    assert rn / np.linalg.norm(b) <= 1e-10
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) < 1e-9


@pytest.mark.parametrize("stride", [1, 2, 4])
def test_aitken_matches_oracle(G, stride):
    """Parallel GaBP + Aitken (section IV-A) as the oracle runs it: same
    samples, the same extrapolated y and the same stopping sample."""
    print(f"case: small batch Aitken sync stride {stride}", flush=True)
    m = W.poisson2d(32)
    b = W.uniform_b(m.n, 0)
    st, y, rounds = oracle.solve_aitken(m, b, stride=stride, tol=1e-10)
    assert st == oracle.OK
    rc, per, summ, x = _solve(G, [m], b, msg_fp32=0, tol=1e-10, accel=G.GABP_ACCEL_AITKEN,
                              accel_stride=stride, max_sweeps=50000)
    assert rc == G.GABP_OK
    assert abs(per[0].sweeps - rounds) <= stride, (per[0].sweeps, rounds)
    _, rn = oracle.residual(m, b, x)
    assert rn / np.linalg.norm(b) <= 1e-10
    assert np.linalg.norm(x - y) / np.linalg.norm(y) < 1e-8
    plain = oracle.solve(m, b, tol=1e-10, max_rounds=20000).rounds
    if stride > 1:
        assert per[0].sweeps < 0.5 * plain  # 898 against 2129 at stride 2


def _colored_aitken_oracle(m, b, colors, stride, tol, max_sweeps=20000):
    """The oracle's pieces composed: coloured rounds (Rounds with colors),
    means every `stride` sweeps, orc_aitken on the last three samples, stop on
    the residual of the extrapolation."""
    R = oracle.Rounds(m, b, algorithm=2, colors=colors)
    bn = np.linalg.norm(b)
    hist = [R.marginals()[0]]
    for t in range(1, max_sweeps + 1):
        R.step()
        if t % stride:
            continue
        hist = (hist + [R.marginals()[0]])[-3:]
        y = oracle.aitken(*hist) if len(hist) == 3 else hist[-1]
        if oracle.residual(m, b, y)[1] / bn <= tol:
            return t, y
    raise AssertionError("oracle did not converge")


def test_colored_aitken_latency_path(G):
    """The serial scheme in red-black order with Aitken: about a fifth of the
    synchronous sweeps on the 32 x 32 grid (459 against 2129)."""
    print("case: small batch coloured + Aitken Poisson 32^2", flush=True)
    m = W.poisson2d(32)
    b = W.uniform_b(m.n, 0)
    blocks = [m]
    mm = W.block_diag_csr(blocks)
    B = G.DeviceBatch.sparse([m.n], mm)
    o = G.gabp_default_opts(msg_fp32=0, tol=1e-10, schedule=G.GABP_SCHEDULE_COLORED,
                            accel=G.GABP_ACCEL_AITKEN, accel_stride=1, max_sweeps=50000)
    rc, plan = G.gabp_plan_create_batched(B, o)
    assert rc == G.GABP_OK
    colors = _colors(G, plan, m)
    assert colors.max() == 1  # the grid is bipartite: red-black
    x = torch.zeros(m.n, dtype=torch.float64, device="cuda")
    rc, per, summ = G.gabp_plan_solve_batched(plan, dev(b), x)
    G.gabp_plan_destroy(plan)
    assert rc == G.GABP_OK
    t_ref, y_ref = _colored_aitken_oracle(m, b, colors, 1, 1e-10)
    assert abs(per[0].sweeps - t_ref) <= 1, (per[0].sweeps, t_ref)
    xh = host(x)
    assert np.linalg.norm(xh - y_ref) / np.linalg.norm(y_ref) < 1e-8
    assert per[0].sweeps < 0.3 * oracle.solve(m, b, tol=1e-10, max_rounds=20000).rounds


def test_steffensen_matches_oracle(G):
    """GaBP + Steffensen (cycles of 100 sweeps, extrapolated correction, restart
    on the residual with the precisions kept) as the oracle runs it."""
    print("case: small batch Steffensen", flush=True)
    m = W.poisson2d(20)
    b = W.uniform_b(m.n, 3)
    st, xo, rounds, cycles, rel = oracle.solve_steffensen(m, b, stride=2, cycle=100, tol=1e-10)
    assert st == oracle.OK
    rc, per, summ, x = _solve(G, [m], b, msg_fp32=0, tol=1e-10, accel=G.GABP_ACCEL_STEFFENSEN,
                              accel_stride=2, accel_cycle=100, max_restarts=1000,
                              max_sweeps=200000)
    assert rc == G.GABP_OK
    assert per[0].restarts + 1 == cycles and per[0].sweeps == rounds
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) < 1e-8


def test_uneven_batch_each_instance_stops_on_its_own(G):
    """Every instance stops at its own oracle round and returns its own x."""
    print("case: small batch uneven, per-instance stop", flush=True)
    blocks = [W.poisson2d(6), W.sdd_random(301, 6), W.poisson2d(14), W.random_tree(150, 9),
              W.poisson3d_varcoef(5, 4, 3, 7)[0], W.csr_from_dense(np.array([[2.5]]))]
    m = W.block_diag_csr(blocks)
    b = W.uniform_b(m.n, 21)
    rc, per, summ, x = _solve(G, blocks, b, msg_fp32=0, tol=1e-10, check_every=1,
                              max_sweeps=50000)
    assert rc == G.GABP_OK
    off = 0
    sweeps = []
    for t, q in enumerate(blocks):
        bt = b[off:off + q.n]
        ref = oracle.solve(q, bt, tol=1e-10, max_rounds=50000)
        assert ref.status == oracle.OK
        assert abs(per[t].sweeps - ref.rounds) <= 1, (t, per[t].sweeps, ref.rounds)
        xt = x[off:off + q.n]
        assert np.linalg.norm(xt - ref.x) <= 1e-8 * max(np.linalg.norm(ref.x), 1e-300), t
        sweeps.append(per[t].sweeps)
        off += q.n
    assert len(set(sweeps)) > 3  # the instances really stopped at different sweeps
    assert summ.sweeps == max(sweeps)


def test_fp32_batch_refines_to_1e8(G):
    print("case: small batch FP32 + refinement to 1e-8", flush=True)
    rng = np.random.default_rng(5)
    blocks = []
    for k in range(40):
        kind = k % 4
        if kind == 0:
            blocks.append(W.poisson2d(int(rng.integers(4, 30))))
        elif kind == 1:
            blocks.append(W.sdd_random(int(rng.integers(10, 900)), k))
        elif kind == 2:
            blocks.append(W.poisson3d(*[int(v) for v in rng.integers(3, 10, size=3)], 0.01))
        else:
            blocks.append(W.random_tree(int(rng.integers(2, 600)), k))
    m = W.block_diag_csr(blocks)
    b = W.normal_b(m.n, 22)
    for sch in (0, 1):
        rc, per, summ, x = _solve(G, blocks, b, msg_fp32=1, tol=1e-8, schedule=sch,
                                  max_sweeps=100000)
        assert rc == G.GABP_OK, G.status_name(rc)
        off = 0
        for t, q in enumerate(blocks):
            bt = b[off:off + q.n]
            _, rn = oracle.residual(q, bt, x[off:off + q.n])
            assert rn / np.linalg.norm(bt) <= 1e-8, (sch, t)
            off += q.n
        assert summ.restarts >= 1  # FP32 messages alone stop near 1e-7


def test_errors_and_edge_cases(G):
    print("case: small batch errors and edge cases", flush=True)
    # an entry joining two instances
    m = W.poisson2d(4)
    B = G.DeviceBatch.sparse([8, 8], m)
    assert G.gabp_plan_create_batched(B, G.gabp_default_opts())[0] == G.GABP_ERR_ARG
    # sizes that do not add up
    B = G.DeviceBatch.sparse([8, 7], m)
    assert G.gabp_plan_create_batched(B, G.gabp_default_opts())[0] == G.GABP_ERR_ARG
    # more rows than one workgroup holds
    big = W.poisson2d_rect(65, 65)
    B = G.DeviceBatch.sparse([big.n], big)
    assert G.gabp_plan_create_batched(B, G.gabp_default_opts())[0] == G.GABP_ERR_UNSUPPORTED
    # messages beyond the LDS (FP64, two buffers): 3-D grid of 4000 rows
    g3 = W.poisson3d(20, 20, 10, 0.01)
    B = G.DeviceBatch.sparse([g3.n], g3)
    assert G.gabp_plan_create_batched(B, G.gabp_default_opts(msg_fp32=0))[0] == \
        G.GABP_ERR_UNSUPPORTED
    # asymmetric values
    A = W.dense_from_csr(W.poisson2d(3))
    A[0, 1] = -0.5
    B = G.DeviceBatch.sparse([9], W.csr_from_dense(A))
    assert G.gabp_plan_create_batched(B, G.gabp_default_opts())[0] == G.GABP_ERR_NOT_SYMMETRIC
    # acceleration on other plan kinds; a Steffensen cycle shorter than 2 strides
    o = G.gabp_default_opts(accel=G.GABP_ACCEL_AITKEN)
    assert G.gabp_plan_create(G.DeviceCSR.from_host(W.poisson2d(4)), o)[0] == G.GABP_ERR_UNSUPPORTED
    o = G.gabp_default_opts(accel=G.GABP_ACCEL_STEFFENSEN, accel_stride=3, accel_cycle=5)
    B = G.DeviceBatch.sparse([16], W.poisson2d(4))
    assert G.gabp_plan_create_batched(B, o)[0] == G.GABP_ERR_ARG
    # zero right-hand side in one instance, empty instance, diagonal instance
    blocks = [W.poisson2d(5), W.csr_from_dense(np.zeros((0, 0))),
              W.csr_from_dense(np.diag([2.0, -4.0])), W.poisson2d(3)]
    b = np.concatenate([np.zeros(25), [1.0, 2.0], W.uniform_b(9, 1)])
    rc, per, summ, x = _solve(G, blocks, b, msg_fp32=0, tol=1e-12)
    assert rc == G.GABP_OK
    assert np.all(x[:25] == 0) and per[0].sweeps == 0
    assert per[1].sweeps == 0
    np.testing.assert_allclose(x[25:27], [0.5, -0.5], rtol=1e-15)
    ref = np.linalg.solve(W.dense_from_csr(W.poisson2d(3)), b[27:])
    np.testing.assert_allclose(x[27:], ref, rtol=1e-10, atol=1e-11 * np.abs(ref).max())
    # the empty batch
    e = W.csr_from_dense(np.zeros((0, 0)))
    B = G.DeviceBatch.sparse(np.zeros(0, dtype=np.int32), e)
    rc, plan = G.gabp_plan_create_batched(B, G.gabp_default_opts())
    assert rc == G.GABP_OK
    rc, per, summ = G.gabp_plan_solve_batched(plan, dev(np.zeros(0)), dev(np.zeros(0)))
    assert rc == G.GABP_OK
    G.gabp_plan_destroy(plan)


def test_breakdown_is_reported(G):
    """A zero cavity precision (a zero elimination pivot) in one instance is
    GABP_ERR_BREAKDOWN for that instance; the others converge."""
    print("case: small batch breakdown", flush=True)
    bad = W.csr_from_dense(np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 1.0], [0.0, 1.0, 1.0]]))
    blocks = [W.poisson2d(5), bad, W.poisson2d(4)]
    b = W.uniform_b(25 + 3 + 16, 4)
    rc, per, summ, x = _solve(G, blocks, b, msg_fp32=0, tol=1e-10)
    assert rc == G.GABP_ERR_BREAKDOWN
    assert per[0].status == G.GABP_OK and per[2].status == G.GABP_OK
    assert per[1].status == G.GABP_ERR_BREAKDOWN
