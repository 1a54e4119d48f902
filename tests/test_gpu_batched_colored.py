"""GPU parity of the two-colour schedule of batched bipartite (section VII)
instances against the FP64 CPU oracle's coloured rounds.

The chips (rows of S) form colour 0 and send first, then the users (columns)
send: oracle.Rounds on the bipartite system (users first, then chips in its
node order) with colours [1] * K + [0] * N.  Tolerances as in
test_gpu_batched.py."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from test_gpu_batched import (  # noqa: E402
    HARD, SIZES_K, SIZES_N, _bip, _check_bip_solution, _marginals, _mmse_rel, _node_slices,
    _trajectory, dev, host)


@pytest.fixture(scope="module")
def G():
    import paper_0810_1119_amd as G
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return G


def opts(G, **kw):
    return G.gabp_default_opts(schedule=G.GABP_SCHEDULE_COLORED, **kw)


def _plan(G, B, **kw):
    rc, plan = G.gabp_plan_create_batched(B, opts(G, **kw))
    assert rc == G.GABP_OK, G.status_name(rc)
    return plan


def _colored_rounds(db, t, damping=0.0):
    S, y, _, s2 = db.instance(t)
    m, rhs = oracle.bipartite_system(S, y, s2)
    K, N = S.shape[1], S.shape[0]
    return oracle.Rounds(m, rhs, damping=damping, colors=np.r_[np.ones(K, int), np.zeros(N, int)])


@pytest.mark.parametrize("fp32,checkpoints,rtol,floor", [
    (0, (1, 2, 3, 8, 20), 1e-10, 1e-12),
    (1, (1, 2, 3), 2e-5, 2e-5),
])
def test_colored_bipartite_trajectory(G, fp32, checkpoints, rtol, floor):
    db = W.detection_sizes(SIZES_K, SIZES_N, seed=11)
    B = _bip(G, db)
    plan = _plan(G, B, msg_fp32=fp32, freeze=0)
    try:
        assert G.gabp_plan_reset(plan, dev(db.y)) == G.GABP_OK
        rounds = [_colored_rounds(db, t) for t in range(db.batch)]
        _trajectory(G, plan, B, rounds, checkpoints, rtol, floor, _node_slices(db.K, db.N))
    finally:
        G.gabp_plan_destroy(plan)


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.7])
def test_colored_bipartite_trajectory_damped(G, alpha):
    db = W.detection_sizes([5, 70, 129], [10, 140, 258], seed=12)
    B = _bip(G, db)
    plan = _plan(G, B, msg_fp32=0, freeze=0, damping=alpha)
    try:
        assert G.gabp_plan_reset(plan, dev(db.y)) == G.GABP_OK
        rounds = [_colored_rounds(db, t, damping=alpha) for t in range(db.batch)]
        _trajectory(G, plan, B, rounds, (1, 2, 6), 1e-10, 1e-12, _node_slices(db.K, db.N))
    finally:
        G.gabp_plan_destroy(plan)


def test_colored_max_sweeps_returns_the_last_iterate(G):
    db = W.detection_sizes([9, 40], [18, 80], seed=14)
    B = _bip(G, db)
    x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
    rc, per, _ = G.gabp_solve_batched(B, dev(db.y), x, opts(G, msg_fp32=0, max_sweeps=3, freeze=0))
    assert rc == G.GABP_NOT_CONVERGED
    xs = host(x)
    for t in range(db.batch):
        assert per[t].status == G.GABP_NOT_CONVERGED and per[t].sweeps == 3
        mean, _ = _colored_rounds(db, t).step(3).marginals()
        k0 = int(db.x_off[t])
        np.testing.assert_allclose(xs[k0:k0 + int(db.K[t])], mean[:int(db.K[t])], rtol=1e-10,
                                   atol=1e-12)


def test_colored_bipartite_solve_fp32_half_the_sweeps(G):
    """Every instance to 1e-8 with the settled phase, in about half the
    sweeps of the synchronous schedule (which runs two independent copies of
    the coloured recursion on a bipartite graph)."""
    db = W.detection_batch(24, seed=21, kmin=1, kmax=256)
    B = _bip(G, db)
    x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
    rc, per, summ = G.gabp_solve_batched(B, dev(db.y), x, opts(G))
    assert rc == G.GABP_OK, G.status_name(rc)
    assert summ.edges == int(2 * np.sum(db.K * db.N))
    _check_bip_solution(G, db, x, per, 1e-8, 1e-6)
    assert max(p.frozen_sweeps for p in per) > 0
    x0 = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
    rc, per0, _ = G.gabp_solve_batched(B, dev(db.y), x0)
    assert rc == G.GABP_OK
    s_col, s_sync = sum(p.sweeps for p in per), sum(p.sweeps for p in per0)
    print(f"sweeps over the batch: synchronous {s_sync}, coloured {s_col}", flush=True)
    assert s_col <= 0.65 * s_sync


def test_colored_bipartite_solve_fp64_tight(G):
    db = W.detection_batch(6, seed=22, kmin=20, kmax=180)
    B = _bip(G, db)
    x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
    rc, per, _ = G.gabp_solve_batched(B, dev(db.y), x, opts(G, msg_fp32=0, tol=1e-12))
    assert rc == G.GABP_OK, G.status_name(rc)
    _check_bip_solution(G, db, x, per, 1e-12, 1e-10)


def test_colored_hard_instances_converge(G):
    """The instances on which the undamped iteration does not contract: the
    coloured schedule runs one of the two synchronous chains, so they need
    damping here too, and the escalation provides it."""
    db = W.detection_subset(4096, 1, HARD)
    B = _bip(G, db)
    x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
    rc, per, _ = G.gabp_solve_batched(B, dev(db.y), x, opts(G))
    assert rc == G.GABP_OK, G.status_name(rc)
    xs = host(x)
    for t in range(db.batch):
        k0, k = int(db.x_off[t]), int(db.K[t])
        assert per[t].status == G.GABP_OK and _mmse_rel(db, t, xs[k0:k0 + k]) <= 1e-8
        S, y, _, s2 = db.instance(t)
        m, rhs = oracle.bipartite_system(S, y, s2)
        ref = oracle.solve(m, rhs, tol=1e-13, max_rounds=20000, damping=0.3).x[:k]
        np.testing.assert_allclose(xs[k0:k0 + k], ref, rtol=0, atol=1e-6 * np.abs(ref).max())
    print("damping per instance:", [p.damping for p in per], flush=True)
    assert per[5].damping == 0.0


@pytest.mark.parametrize("waves", [4, 8, 16])
def test_colored_workgroup_shapes_and_determinism(G, waves):
    db = W.detection_batch(12, seed=27, kmin=1, kmax=256)
    B = _bip(G, db)
    rc, plan = G.gabp_plan_create_batched(B, opts(G, batch_waves=waves))
    assert rc == G.GABP_OK
    try:
        xs = []
        for _ in range(2):
            x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
            rc, per, _ = G.gabp_plan_solve_batched(plan, dev(db.y), x)
            assert rc == G.GABP_OK
            xs.append(host(x))
        assert np.array_equal(xs[0], xs[1])
        for t in range(db.batch):
            k0, k = int(db.x_off[t]), int(db.K[t])
            assert _mmse_rel(db, t, xs[0][k0:k0 + k]) <= 1e-8
    finally:
        G.gabp_plan_destroy(plan)


def test_colored_marginal_precisions_match_the_fixed_point(G):
    db = W.detection_sizes([12, 90], [24, 180], seed=28)
    B = _bip(G, db)
    plan = _plan(G, B, msg_fp32=0, tol=1e-12)
    try:
        x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
        rc, per, _ = G.gabp_plan_solve_batched(plan, dev(db.y), x)
        assert rc == G.GABP_OK
        _, prec = _marginals(G, plan, B)
        for t, sl in enumerate(_node_slices(db.K, db.N)):
            R = _colored_rounds(db, t).step(400)
            _, po = R.marginals()
            np.testing.assert_allclose(prec[sl], po, rtol=1e-9)
    finally:
        G.gabp_plan_destroy(plan)


def test_colored_schedule_needs_the_bipartite_kind(G):
    dbat = W.dense_sdd_batch(2, seed=13, kmin=3, kmax=9)
    B = G.DeviceBatch.dense(dbat.K, dbat.A)
    rc, plan = G.gabp_plan_create_batched(B, opts(G))
    assert rc == G.GABP_ERR_UNSUPPORTED
