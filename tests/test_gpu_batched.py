"""GPU parity of the batched dense path (one persistent launch through
gabp_solve_batched / batched plans) against the FP64 CPU oracle.

Bipartite instances (section VII): the oracle runs Algorithm 2 on the CSR form
of [[I, S^T], [S, -sigma2 I]] (oracle.bipartite_system); the GPU marginals of a
batched plan are packed per instance as K users then N chips, the oracle's
node order.  Dense instances: the oracle runs on the CSR form of A_t.

Tolerances (as for the single-system path):
  * FP64 messages: 1e-10 relative per sweep (different summation order:
    wavefront trees and per-wavefront column partials against sequential sums),
    with an absolute floor of 1e-12 times the largest value.
  * FP32 messages: 2e-5 relative after at most 4 sweeps (sums over up to 400
    terms, one rounding of 2^-24 each), same kind of floor.
  * Solves: the FP64 relative residual of the problem each instance states,
    ||S^T y - (S^T S + sigma2 I) x|| / ||S^T y|| (bipartite) or
    ||b - A x|| / ||b|| (dense), recomputed on the CPU by the oracle, must meet
    the requested tolerance; the solution must agree with the oracle's own
    converged solution within what that residual allows, and the detected
    symbols sign(x) must agree exactly.
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# ragged sizes: one lane, one partial wavefront, exactly one and just over one
# 64-column chunk, several chunks with a tail; and a chip count other than 2K
SIZES_K = [1, 7, 63, 64, 65, 130, 200, 50]
SIZES_N = [2, 14, 126, 128, 130, 260, 400, 53]


@pytest.fixture(scope="module")
def G():
    import paper_0810_1119_amd as G
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return G


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def _bip(G, db):
    return G.DeviceBatch.bipartite(db.K, db.N, db.sigma2, db.S)


def _dense(G, dbat):
    return G.DeviceBatch.dense(dbat.K, dbat.A)


def _plan(G, B, **kw):
    rc, plan = G.gabp_plan_create_batched(B, G.gabp_default_opts(**kw))
    assert rc == G.GABP_OK, G.status_name(rc)
    return plan


def _marginals(G, plan, B):
    mean = torch.empty(B.nodes, dtype=torch.float64, device="cuda")
    prec = torch.empty(B.nodes, dtype=torch.float64, device="cuda")
    assert G.gabp_plan_marginals(plan, mean, prec) == G.GABP_OK
    return host(mean), host(prec)


def _close(got, ref, rtol, floor):
    scale = max(1.0, float(np.max(np.abs(ref)))) if ref.size else 1.0
    np.testing.assert_allclose(got, ref, rtol=rtol, atol=floor * scale)


def _bip_oracle_rounds(db, t, damping=0.0):
    S, y, _, s2 = db.instance(t)
    m, rhs = oracle.bipartite_system(S, y, s2)
    return oracle.Rounds(m, rhs, damping=damping)


def _mmse_rel(db, t, x):
    """Oracle FP64 residual of (S^T S + sigma2 I) x = S^T y."""
    A, b = db.mmse_system(t)
    _, nr = oracle.residual(W.csr_from_dense(A), b, x)
    nb = np.linalg.norm(b)
    return nr / nb if nb > 0 else nr


def _bip_oracle_solution(db, t):
    S, y, _, s2 = db.instance(t)
    m, rhs = oracle.bipartite_system(S, y, s2)
    r = oracle.solve(m, rhs, tol=1e-13, max_rounds=20000)
    assert r.status == oracle.OK, r.status
    return r.x[:S.shape[1]]


def _trajectory(G, plan, B, rounds_list, checkpoints, rtol, floor, node_slices):
    done = 0
    for T in checkpoints:
        assert G.gabp_plan_sweeps(plan, T - done) == G.GABP_OK
        for R in rounds_list:
            R.step(T - done)
        done = T
        mean, prec = _marginals(G, plan, B)
        for R, sl in zip(rounds_list, node_slices):
            ref_mean, ref_prec = R.marginals()
            _close(mean[sl], ref_mean, rtol, floor)
            _close(prec[sl], ref_prec, rtol, floor)


def _node_slices(K, N=None):
    out, o = [], 0
    for t in range(len(K)):
        n = int(K[t]) + (int(N[t]) if N is not None else 0)
        out.append(slice(o, o + n))
        o += n
    return out


# ---------------------------------------------------------------------------
# sweep-by-sweep parity
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("fp32,checkpoints,rtol,floor", [
    (0, (1, 2, 3, 8, 25), 1e-10, 1e-12),
    (1, (1, 2, 4), 2e-5, 2e-5),
])
def test_bipartite_trajectory(G, fp32, checkpoints, rtol, floor):
    db = W.detection_sizes(SIZES_K, SIZES_N, seed=11)
    B = _bip(G, db)
    plan = _plan(G, B, msg_fp32=fp32, freeze=0)
    try:
        assert G.gabp_plan_reset(plan, dev(db.y)) == G.GABP_OK
        rounds = [_bip_oracle_rounds(db, t) for t in range(db.batch)]
        _trajectory(G, plan, B, rounds, checkpoints, rtol, floor, _node_slices(db.K, db.N))
    finally:
        G.gabp_plan_destroy(plan)


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.7])
def test_bipartite_trajectory_damped(G, alpha):
    db = W.detection_sizes([5, 70, 129], [10, 140, 258], seed=12)
    B = _bip(G, db)
    plan = _plan(G, B, msg_fp32=0, freeze=0, damping=alpha)
    try:
        assert G.gabp_plan_reset(plan, dev(db.y)) == G.GABP_OK
        rounds = [_bip_oracle_rounds(db, t, damping=alpha) for t in range(db.batch)]
        _trajectory(G, plan, B, rounds, (1, 2, 6), 1e-10, 1e-12, _node_slices(db.K, db.N))
    finally:
        G.gabp_plan_destroy(plan)


@pytest.mark.parametrize("density", [1.0, 0.3])
def test_dense_trajectory_fp64(G, density):
    dbat = W.dense_sdd_batch(7, seed=13, kmin=1, kmax=140, density=density)
    B = _dense(G, dbat)
    plan = _plan(G, B, msg_fp32=0, freeze=0)
    try:
        assert G.gabp_plan_reset(plan, dev(dbat.b)) == G.GABP_OK
        rounds = []
        for t in range(dbat.batch):
            A, b = dbat.instance(t)
            rounds.append(oracle.Rounds(W.csr_from_dense(A), b))
        _trajectory(G, plan, B, rounds, (1, 2, 5, 12), 1e-10, 1e-12, _node_slices(dbat.K))
    finally:
        G.gabp_plan_destroy(plan)


def test_max_sweeps_returns_the_last_iterate(G):
    """x holds the means after the sweep budget (first pass: x = 0 + H/S)."""
    db = W.detection_sizes([9, 40], [18, 80], seed=14)
    B = _bip(G, db)
    x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
    o = G.gabp_default_opts(msg_fp32=0, max_sweeps=3, freeze=0)
    rc, per, _ = G.gabp_solve_batched(B, dev(db.y), x, o)
    assert rc == G.GABP_NOT_CONVERGED
    xs = host(x)
    for t in range(db.batch):
        assert per[t].status == G.GABP_NOT_CONVERGED and per[t].sweeps == 3
        mean, _ = _bip_oracle_rounds(db, t).step(3).marginals()
        k0 = int(db.x_off[t])
        _close(xs[k0:k0 + int(db.K[t])], mean[:int(db.K[t])], 1e-10, 1e-12)


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------
def _check_bip_solution(G, db, x, per, tol, sol_rtol):
    xs = host(x)
    for t in range(db.batch):
        k = int(db.K[t])
        k0 = int(db.x_off[t])
        assert per[t].status == G.GABP_OK, (t, G.status_name(per[t].status))
        xt = xs[k0:k0 + k]
        rel = _mmse_rel(db, t, xt)
        assert rel <= tol, (t, rel)
        assert abs(per[t].rel_residual - rel) <= 0.05 * rel + 1e-15
        ref = _bip_oracle_solution(db, t)
        np.testing.assert_allclose(xt, ref, rtol=0, atol=sol_rtol * np.abs(ref).max())
        assert np.array_equal(np.sign(xt), np.sign(ref))


def test_bipartite_solve_fp32(G):
    db = W.detection_batch(24, seed=21, kmin=1, kmax=256)
    B = _bip(G, db)
    x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
    rc, per, summ = G.gabp_solve_batched(B, dev(db.y), x)
    assert rc == G.GABP_OK, G.status_name(rc)
    assert summ.status == G.GABP_OK and summ.edges == int(2 * np.sum(db.K * db.N))
    # residual 1e-8 of a system with condition number below ~30 (load 1/2,
    # sigma2 = 0.1): the solution error stays below 1e-6 of max|x|
    _check_bip_solution(G, db, x, per, 1e-8, 1e-6)
    assert max(p.frozen_sweeps for p in per) > 0  # the settled phase was used


def test_bipartite_solve_fp64_tight(G):
    db = W.detection_batch(6, seed=22, kmin=20, kmax=180)
    B = _bip(G, db)
    x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
    rc, per, _ = G.gabp_solve_batched(B, dev(db.y), x, G.gabp_default_opts(msg_fp32=0, tol=1e-12))
    assert rc == G.GABP_OK, G.status_name(rc)
    _check_bip_solution(G, db, x, per, 1e-12, 1e-10)


@pytest.mark.parametrize("fp32,damping", [(1, 0.0), (0, 0.0), (1, 0.5)])
def test_dense_solve(G, fp32, damping):
    dbat = W.dense_sdd_batch(9, seed=23, kmin=1, kmax=300, density=0.6)
    B = _dense(G, dbat)
    x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
    rc, per, _ = G.gabp_solve_batched(B, dev(dbat.b), x,
                                      G.gabp_default_opts(msg_fp32=fp32, damping=damping))
    assert rc == G.GABP_OK, G.status_name(rc)
    xs = host(x)
    o = 0
    for t in range(dbat.batch):
        A, b = dbat.instance(t)
        k = A.shape[0]
        _, nr = oracle.residual(W.csr_from_dense(A), b, xs[o:o + k])
        assert nr / np.linalg.norm(b) <= 1e-8 and per[t].status == G.GABP_OK
        ref = oracle.solve(W.csr_from_dense(A), b, tol=1e-13).x
        np.testing.assert_allclose(xs[o:o + k], ref, rtol=0, atol=1e-7 * np.abs(ref).max())
        o += k


def test_literal_dense_detection_diverges_alone(G):
    """The dense MMSE matrix S^T S + sigma2 I at load 1/2 is not walk-summable
    and synchronous GaBP diverges on it (the oracle shows the same); in the
    same launch a diagonally dominant instance still converges."""
    db = W.detection_sizes([64], [128], seed=24)
    A_bad, b_bad = db.mmse_system(0)
    good = W.dense_sdd_batch(1, seed=25, kmin=40, kmax=40)
    A_good, b_good = good.instance(0)
    pack = W.pack_dense([A_bad, A_good], [b_bad, b_good])
    B = _dense(G, pack)
    x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
    rc, per, _ = G.gabp_solve_batched(B, dev(pack.b), x)
    assert per[0].status == G.GABP_ERR_DIVERGED
    assert per[1].status == G.GABP_OK
    assert rc == G.GABP_ERR_DIVERGED
    _, nr = oracle.residual(W.csr_from_dense(A_good), b_good, host(x)[64:])
    assert nr / np.linalg.norm(b_good) <= 1e-8


# instances of the 4096-instance detection batch (seed 1) on which synchronous
# GaBP does not converge undamped; the oracle diverges on them too and
# converges with damping 0.3 (instance 5 is an ordinary one)
HARD = [3870, 2587, 1945, 2706, 2371, 5]


def test_adaptive_damping_rescues_non_contracting_instances(G):
    db = W.detection_subset(4096, 1, HARD)
    B = _bip(G, db)
    x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
    rc, per, summ = G.gabp_solve_batched(B, dev(db.y), x)
    assert rc == G.GABP_OK, G.status_name(rc)
    assert [p.damping for p in per[:4]] == [0.3] * 4 and per[5].damping == 0.0
    assert summ.damping == 0.3
    xs = host(x)
    for t in range(db.batch):
        k0, k = int(db.x_off[t]), int(db.K[t])
        assert per[t].status == G.GABP_OK and _mmse_rel(db, t, xs[k0:k0 + k]) <= 1e-8
        S, y, _, s2 = db.instance(t)
        m, rhs = oracle.bipartite_system(S, y, s2)
        ref = oracle.solve(m, rhs, tol=1e-13, max_rounds=20000, damping=0.3).x[:k]
        np.testing.assert_allclose(xs[k0:k0 + k], ref, rtol=0, atol=1e-6 * np.abs(ref).max())
    # without the remedy the first two diverge, as the undamped oracle does
    x.zero_()
    rc, per, _ = G.gabp_solve_batched(B, dev(db.y), x,
                                      G.gabp_default_opts(adapt_damping=0, max_sweeps=3000))
    assert per[0].status == G.GABP_ERR_DIVERGED and per[1].status == G.GABP_ERR_DIVERGED
    assert per[5].status == G.GABP_OK and rc == G.GABP_ERR_DIVERGED


def test_batched_solve_is_deterministic(G):
    db = W.detection_batch(40, seed=26, kmin=16, kmax=256)
    B = _bip(G, db)
    rc, plan = G.gabp_plan_create_batched(B, G.gabp_default_opts(batch_waves=8))
    assert rc == G.GABP_OK
    try:
        xs = []
        for _ in range(2):
            x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
            rc, per, _ = G.gabp_plan_solve_batched(plan, dev(db.y), x)
            assert rc == G.GABP_OK
            xs.append(host(x))
        assert np.array_equal(xs[0], xs[1])
    finally:
        G.gabp_plan_destroy(plan)


@pytest.mark.parametrize("waves", [4, 8, 16])
def test_workgroup_shapes(G, waves):
    db = W.detection_batch(12, seed=27, kmin=1, kmax=256)
    B = _bip(G, db)
    x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
    rc, per, _ = G.gabp_solve_batched(B, dev(db.y), x, G.gabp_default_opts(batch_waves=waves))
    assert rc == G.GABP_OK
    xs = host(x)
    for t in range(db.batch):
        k0, k = int(db.x_off[t]), int(db.K[t])
        assert _mmse_rel(db, t, xs[k0:k0 + k]) <= 1e-8


def test_plan_solve_marginal_precisions(G):
    """Converged marginal precisions of the users agree with the oracle's
    converged ones (FP32 messages settle to about 1e-6 relative)."""
    db = W.detection_sizes([12, 90], [24, 180], seed=28)
    B = _bip(G, db)
    plan = _plan(G, B)
    try:
        x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
        prec = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
        rc, st = G.gabp_plan_solve(plan, dev(db.y), x, prec)
        assert rc == G.GABP_OK and st.status == G.GABP_OK
        p = host(prec)
        for t in range(db.batch):
            S, y, _, s2 = db.instance(t)
            m, rhs = oracle.bipartite_system(S, y, s2)
            ref = oracle.solve(m, rhs, tol=1e-13, max_rounds=20000).prec[:S.shape[1]]
            k0 = int(db.x_off[t])
            np.testing.assert_allclose(p[k0:k0 + S.shape[1]], ref, rtol=1e-4)
    finally:
        G.gabp_plan_destroy(plan)


# ---------------------------------------------------------------------------
# edge cases and errors
# ---------------------------------------------------------------------------
def test_empty_and_degenerate_instances(G):
    # an instance without chips has S^T y = 0, so x = 0 exactly
    db = W.detection_sizes([3, 0, 5, 4], [6, 3, 0, 8], seed=31)
    B = _bip(G, db)
    x = torch.full((B.xlen,), 7.0, dtype=torch.float64, device="cuda")
    rc, per, _ = G.gabp_solve_batched(B, dev(db.y), x)
    assert rc == G.GABP_OK, G.status_name(rc)
    xs = host(x)
    assert np.all(xs[3:8] == 0.0)  # instance 2 (K = 5, N = 0)
    for t in (0, 3):
        k0, k = int(db.x_off[t]), int(db.K[t])
        assert _mmse_rel(db, t, xs[k0:k0 + k]) <= 1e-8
    # no instances at all
    B0 = G.DeviceBatch.bipartite(np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(1))
    rc, per, summ = G.gabp_solve_batched(B0, dev(np.zeros(1))[:0], dev(np.zeros(1))[:0])
    assert rc == G.GABP_OK and summ.edges == 0


def test_batched_errors(G):
    def solve(B, b):
        x = torch.zeros(max(B.xlen, 1), dtype=torch.float64, device="cuda")[:B.xlen]
        return G.gabp_solve_batched(B, dev(b), x)[0]

    good = W.dense_sdd_batch(2, seed=32, kmin=5, kmax=9)
    A0, b0 = good.instance(0)
    A1, b1 = good.instance(1)
    asym = A1.copy(); asym[0, 1] += 1e-3
    assert solve(_dense(G, W.pack_dense([A0, asym], [b0, b1])), np.r_[b0, b1]) == \
        G.GABP_ERR_NOT_SYMMETRIC
    zd = A1.copy(); zd[2, 2] = 0.0
    assert solve(_dense(G, W.pack_dense([A0, zd], [b0, b1])), np.r_[b0, b1]) == G.GABP_ERR_ZERO_DIAG
    nanm = A1.copy(); nanm[3, 3] = np.nan
    assert solve(_dense(G, W.pack_dense([A0, nanm], [b0, b1])), np.r_[b0, b1]) == G.GABP_ERR_ARG
    db = W.detection_sizes([4, 6], [8, 12], seed=33)
    bad = G.DeviceBatch.bipartite(db.K, db.N, np.array([0.1, 0.0]), db.S)
    assert solve(bad, db.y) == G.GABP_ERR_ARG
    big = G.DeviceBatch.bipartite(np.array([513]), np.array([2]), np.array([0.1]), np.zeros(1026))
    assert solve(big, np.zeros(2)) == G.GABP_ERR_UNSUPPORTED
    # trajectory calls need a reset first; messages are not exported for batches
    B = _bip(G, db)
    plan = _plan(G, B)
    try:
        assert G.gabp_plan_sweeps(plan, 1) == G.GABP_ERR_ARG
        P = torch.zeros(4, dtype=torch.float64, device="cuda")
        assert G.lib.gabp_plan_get_messages(plan.ptr, P.data_ptr(), P.data_ptr(), None) == \
            G.GABP_ERR_UNSUPPORTED
    finally:
        G.gabp_plan_destroy(plan)


# ---------------------------------------------------------------------------
# full-size detection batch: 4096 instances, K ~ U{16..256}, N = 2K
# ---------------------------------------------------------------------------
def test_detection_batch_full_size(G):
    db = W.detection_batch(4096, seed=1)
    B = _bip(G, db)
    x = torch.zeros(B.xlen, dtype=torch.float64, device="cuda")
    rc, per, summ = G.gabp_solve_batched(B, dev(db.y), x)
    print(f"detection 4096: {summ.seconds * 1e3:.1f} ms, max sweeps {summ.sweeps}, "
          f"{summ.edge_updates_per_s:.3e} edge-updates/s", flush=True)
    assert rc == G.GABP_OK, G.status_name(rc)
    xs = host(x)
    # every instance: FP64 residual (CPU, plain numpy of the stated system)
    worst = 0.0
    for t in range(db.batch):
        S, y, _, s2 = db.instance(t)
        k0, k = int(db.x_off[t]), int(db.K[t])
        xt = xs[k0:k0 + k]
        r = S.T @ y - S.T @ (S @ xt) - s2 * xt
        worst = max(worst, np.linalg.norm(r) / np.linalg.norm(S.T @ y))
    assert worst <= 1e-8, worst
    # sampled instances against the oracle's converged solution and symbols
    for t in np.random.default_rng(5).choice(db.batch, 12, replace=False):
        k0, k = int(db.x_off[t]), int(db.K[t])
        ref = _bip_oracle_solution(db, int(t))
        np.testing.assert_allclose(xs[k0:k0 + k], ref, rtol=0, atol=1e-6 * np.abs(ref).max())
        assert np.array_equal(np.sign(xs[k0:k0 + k]), np.sign(ref))
