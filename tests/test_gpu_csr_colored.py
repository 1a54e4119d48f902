"""GPU parity of coloured CSR plans (pair layout): the plan's own colouring
(checked proper and deterministic here), and the trajectory against the FP64
CPU oracle's coloured rounds with that colouring (oracle.Rounds(colors=...),
classes in increasing colour order): marginals and, through the plan's
renumbering, every message.  Tolerances as in test_gpu_csr.py."""
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


def opts(G, **kw):
    return G.gabp_default_opts(schedule=G.GABP_SCHEDULE_COLORED, **kw)


MATRICES = {
    "sdd_3000": lambda: W.sdd_random(3000, 2),
    "poisson2d_20": lambda: W.poisson2d(20),
    "tree_500": lambda: W.random_tree(500, 4),
    "poisson3d_9x8x7": lambda: W.poisson3d(9, 8, 7, 0.1),
}


def _plan(G, m, **kw):
    rc, plan = G.gabp_plan_create(G.DeviceCSR.from_host(m), opts(G, **kw))
    assert rc == G.GABP_OK, G.status_name(rc)
    return plan


def _colors(G, plan, m):
    rc, col, nc = G.gabp_plan_colors(plan)
    assert rc == G.GABP_OK
    col = host(col)
    assert col.min() >= 0 and col.max() == nc - 1
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    off = rows != np.asarray(m.col)
    assert np.all(col[rows[off]] != col[np.asarray(m.col)[off]]), "colouring is not proper"
    return col, nc


@pytest.mark.parametrize("name", sorted(MATRICES))
def test_colouring_is_proper_and_deterministic(G, name):
    m = MATRICES[name]()
    p1, p2 = _plan(G, m), _plan(G, m)
    try:
        c1, n1 = _colors(G, p1, m)
        c2, n2 = _colors(G, p2, m)
        assert n1 == n2 and np.array_equal(c1, c2)
        # first-fit never needs more than max degree + 1 colours (the row
        # length counts the diagonal)
        assert n1 <= np.diff(m.row_ptr).max()
    finally:
        G.gabp_plan_destroy(p1)
        G.gabp_plan_destroy(p2)


@pytest.mark.parametrize("name", sorted(MATRICES))
@pytest.mark.parametrize("damping", [0.0, 0.3, 0.5])
def test_colored_csr_fp64_trajectory_matches_oracle(G, name, damping):
    m = MATRICES[name]()
    b = W.uniform_b(m.n, 5)
    plan = _plan(G, m, msg_fp32=0, freeze=0, damping=damping)
    try:
        col, _ = _colors(G, plan, m)
        assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
        R = oracle.Rounds(m, b, damping=damping, colors=col)
        for t in range(1, 7):
            R.step()
            assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
            mean = torch.zeros(m.n, dtype=torch.float64, device="cuda")
            prec = torch.zeros(m.n, dtype=torch.float64, device="cuda")
            assert G.gabp_plan_marginals(plan, mean, prec) == G.GABP_OK
            mo, po = R.marginals()
            np.testing.assert_allclose(host(mean), mo, rtol=1e-10, atol=1e-12 * np.abs(mo).max(),
                                       err_msg=f"sweep {t}")
            np.testing.assert_allclose(host(prec), po, rtol=1e-10, err_msg=f"sweep {t}")
    finally:
        G.gabp_plan_destroy(plan)


def test_colored_csr_fp32_trajectory_matches_oracle(G):
    m = W.sdd_random(3000, 3)
    b = W.normal_b(m.n, 2)
    plan = _plan(G, m, msg_fp32=1, freeze=0)
    try:
        col, _ = _colors(G, plan, m)
        assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
        R = oracle.Rounds(m, b, colors=col)
        for t in range(1, 5):
            R.step()
            assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
            mean = torch.zeros(m.n, dtype=torch.float64, device="cuda")
            assert G.gabp_plan_marginals(plan, mean) == G.GABP_OK
            mo, _ = R.marginals()
            np.testing.assert_allclose(host(mean), mo, rtol=2e-5, atol=2e-5 * np.abs(mo).max())
    finally:
        G.gabp_plan_destroy(plan)


@pytest.mark.parametrize("fp32,tol", [(1, 1e-8), (0, 1e-11)])
@pytest.mark.parametrize("freeze", [1, 0])
def test_colored_csr_solve_in_fewer_sweeps(G, fp32, tol, freeze):
    m = W.sdd_random(20000, 7)
    b = W.normal_b(m.n, 7)
    A = G.DeviceCSR.from_host(m)
    res = {}
    for sched in (G.GABP_SCHEDULE_SYNC, G.GABP_SCHEDULE_COLORED):
        x = torch.zeros(m.n, dtype=torch.float64, device="cuda")
        pr = torch.zeros(m.n, dtype=torch.float64, device="cuda")
        rc, st = G.gabp_solve(A, dev(b), x, marg_prec=pr, opts=G.gabp_default_opts(
            msg_fp32=fp32, tol=tol, freeze=freeze, schedule=sched))
        assert rc == G.GABP_OK, G.status_name(rc)
        _, rn = oracle.residual(m, b, host(x))
        assert rn / np.linalg.norm(b) <= tol
        res[sched] = (host(x), host(pr), st.sweeps)
    ref = oracle.solve(m, b, tol=1e-13, max_rounds=2000)
    for xs, _, _ in res.values():
        np.testing.assert_allclose(xs, ref.x, rtol=0, atol=10 * tol * np.abs(ref.x).max())
    # both schedules converge to the same precision fixed point
    np.testing.assert_allclose(res[1][1], res[0][1], rtol=1e-5 if fp32 else 1e-10)
    s_sync, s_col = res[0][2], res[1][2]
    print(f"sweeps: synchronous {s_sync}, coloured {s_col}", flush=True)
    assert s_col < s_sync


def test_colored_csr_damped_and_deterministic(G):
    m = W.poisson2d(24)
    b = W.uniform_b(m.n, 1)
    A = G.DeviceCSR.from_host(m)
    xs = []
    for _ in range(2):
        x = torch.zeros(m.n, dtype=torch.float64, device="cuda")
        rc, st = G.gabp_solve(A, dev(b), x, opts=opts(G, damping=0.3))
        assert rc == G.GABP_OK
        xs.append(host(x))
    assert np.array_equal(xs[0], xs[1])
    _, rn = oracle.residual(m, b, xs[0])
    assert rn / np.linalg.norm(b) <= 1e-8


def _messages(G, plan, nnz):
    P = torch.zeros(nnz, dtype=torch.float64, device="cuda")
    h = torch.zeros(nnz, dtype=torch.float64, device="cuda")
    assert G.gabp_plan_get_messages(plan, P, h) == G.GABP_OK
    return host(P), host(h)


@pytest.mark.parametrize("name", ["sdd_3000", "poisson3d_9x8x7", "tree_500"])
def test_colored_csr_messages_match_oracle(G, name):
    """Per-message parity through the renumbering: after each coloured sweep
    the (P, h) of every directed message, read in the caller's CSR order,
    equal the oracle's coloured rounds; messages set from the oracle's
    resume its trajectory."""
    m = MATRICES[name]()
    b = W.uniform_b(m.n, 8)
    plan = _plan(G, m, msg_fp32=0, freeze=0)
    try:
        col, _ = _colors(G, plan, m)
        assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
        R = oracle.Rounds(m, b, colors=col)
        for t in range(1, 5):
            R.step()
            assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
            P, h = _messages(G, plan, m.nnz)
            Po, ho = R.P, R.information()
            np.testing.assert_allclose(P, Po, rtol=1e-10, atol=1e-12 * np.abs(Po).max(),
                                       err_msg=f"P, sweep {t}")
            np.testing.assert_allclose(h, ho, rtol=1e-10, atol=1e-12 * np.abs(ho).max(),
                                       err_msg=f"h, sweep {t}")
        # resume from the oracle's messages two rounds on
        R.step(2)
        assert G.gabp_plan_set_messages(plan, dev(R.P), dev(R.information())) == G.GABP_OK
        P, h = _messages(G, plan, m.nnz)
        np.testing.assert_allclose(P, R.P, rtol=1e-14, atol=0)
        R.step()
        assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
        mean = torch.zeros(m.n, dtype=torch.float64, device="cuda")
        assert G.gabp_plan_marginals(plan, mean) == G.GABP_OK
        mo, _ = R.marginals()
        np.testing.assert_allclose(host(mean), mo, rtol=1e-10, atol=1e-12 * np.abs(mo).max())
    finally:
        G.gabp_plan_destroy(plan)


def test_colored_csr_limits(G):
    m = W.sdd_random(64, 1)
    rc, plan = G.gabp_plan_create(G.DeviceCSR.from_host(m),
                                  opts(G, layout=G.GABP_LAYOUT_GATHER))
    assert rc == G.GABP_ERR_UNSUPPORTED
    # a complete graph on 257 nodes needs 257 colours
    k = 257
    a = -np.ones((k, k)) / k
    np.fill_diagonal(a, 2.0)
    rc, plan = G.gabp_plan_create(G.DeviceCSR.from_host(W.csr_from_dense(a)), opts(G))
    assert rc == G.GABP_ERR_UNSUPPORTED
    # a plan without a colouring has none to report
    rc, plan = G.gabp_plan_create(G.DeviceCSR.from_host(m))
    assert G.gabp_plan_colors(plan)[0] == G.GABP_ERR_UNSUPPORTED
    G.gabp_plan_destroy(plan)
