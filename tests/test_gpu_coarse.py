"""GPU parity of the coarse-grid predicted corrections of grid solves
(gabp_plan_solve_coarse) against the FP64 oracle (oracle/coarse.py).

FP64 messages: the x after each of the first cycles equals the oracle's
(same levels, Galerkin operators, smoothing sweeps and scale) to 1e-9
relative -- the levels' GaBP rounds agree to ~1e-11 per sweep as on the plain
grid path, and a cycle adds a handful of FP64 sums.  The three ways of running the
smallest levels are checked: a coarsest level of up to 512 cells per grid
solved by its dense inverse (the default), a coarsest level of up to 64
cells with the levels between inside one LDS tail launch per visit
(GABP_COARSE_EXACT=64), and those levels as plans of their own
(GABP_COARSE_EXACT=64, GABP_COARSE_TAIL=0).  FP32 messages:
every grid of the stack meets the tolerance (its residual recomputed by the
oracle)."""
import os
from contextlib import contextmanager

import numpy as np
import pytest

import oracle
from oracle import coarse as OC
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


def _grid(G, nx, ny, nz, batch, seed, varcoef=True):
    _, coef = W.grid_stack(nx, ny, nz, batch, varcoef=varcoef, seed=seed, ell=4.0, shift=0.01,
                           with_csr=False)
    if varcoef:
        A = G.DeviceGrid(nx, ny, nz, batch, diag=dev(coef["diag"]), cx=dev(coef["cx"]),
                         cy=dev(coef["cy"]), cz=dev(coef["cz"]) if nz > 1 else None)
        arrs = (coef["diag"], coef["cx"], coef["cy"], coef["cz"] if nz > 1 else None)
    else:
        A = G.DeviceGrid(nx, ny, nz, batch, diag_value=coef["dval"], off_value=coef["off"])
        N = nx * ny * nz * batch
        arrs = (np.full(N, coef["dval"]), np.full(N, coef["off"]), np.full(N, coef["off"]),
                np.full(N, coef["off"]) if nz > 1 else None)
    return A, arrs


@contextmanager
def env(name, value):
    old = os.environ.get(name)
    if value is None:
        os.environ.pop(name, None)
    else:
        os.environ[name] = value
    try:
        yield
    finally:
        if old is None:
            os.environ.pop(name, None)
        else:
            os.environ[name] = old


CASES = {
    "varcoef_16cubed_x2": (16, 16, 16, 2, True),
    "varcoef_odd_13x9x7_x3": (13, 9, 7, 3, True),
    "poisson2d_20x17": (20, 17, 1, 1, False),
    # four levels below the finest one (500, 250, 125, 63 cells), the last
    # three in the tail (all four would not fit the LDS with the inverse)
    "varcoef_1d_1000_x2": (1000, 1, 1, 2, True),
}


# how the small levels run: "exact" (the default: the coarsest level below
# the finest has at most 512 cells per grid, its dense inverse), "tail" (the
# coarsest at most 64 cells, the levels between in the LDS tail launch),
# "plans" (at most 64 cells, every level above it a plan of its own); "_w":
# W-cycles into every level (GABP_COARSE_WCYCLE=1; the oracle's v_cells=0)
# instead of one cycle of a level of at most 4096 cells per grid
LEVEL_MODES = {"exact": (None, None, 512, None), "tail": ("64", None, 64, None),
               "plans": ("64", "0", 64, None), "tail_w": ("64", None, 64, "1"),
               "plans_w": ("64", "0", 64, "1")}


@contextmanager
def level_mode(mode):
    exact, tail, _, wcycle = LEVEL_MODES[mode]
    with env("GABP_COARSE_EXACT", exact), env("GABP_COARSE_TAIL", tail), \
            env("GABP_COARSE_WCYCLE", wcycle):
        yield


def oracle_mode(mode):
    """OC.solve keywords of a level mode"""
    _, _, coarsest, wcycle = LEVEL_MODES[mode]
    return dict(coarsest=coarsest, v_cells=0 if wcycle else OC.V_CELLS)


@pytest.mark.parametrize("tail", sorted(LEVEL_MODES))
@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("schedule", ["colored", "sync"])
def test_cycles_match_oracle_fp64(G, case, schedule, tail):
    nx, ny, nz, batch, varc = CASES[case]
    print(f"case: coarse-grid cycles FP64 {case} {schedule} {tail}", flush=True)
    A, arrs = _grid(G, nx, ny, nz, batch, 3, varc)
    b = W.normal_b(A.n, 4)
    colored = schedule == "colored"
    # an undamped synchronous plan smooths with damping 0.3 (the alternating
    # mode of a bipartite graph is not damped otherwise)
    ref_x, ref_c, ref_w, trail = OC.solve(nx, ny, nz, batch, *arrs, b, tol=0.0, max_cycles=3,
                                          colored=colored, damping=0.0 if colored else 0.3,
                                          **oracle_mode(tail))
    for k in (1, 2, 3):
        o = G.gabp_default_opts(msg_fp32=0, tol=0.0, max_restarts=k, freeze=0,
                                schedule=G.GABP_SCHEDULE_COLORED if colored
                                else G.GABP_SCHEDULE_SYNC)
        rc, plan = G.gabp_plan_create_grid(A, o)
        assert rc == G.GABP_OK
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        with level_mode(tail):
            rc, st = G.gabp_plan_solve_coarse(plan, dev(b), x)
        G.gabp_plan_destroy(plan)
        assert rc == G.GABP_NOT_CONVERGED and st.restarts == k, (rc, st.restarts)
        xh = x.cpu().numpy()
        err = np.linalg.norm(xh - trail[k - 1]) / np.linalg.norm(trail[k - 1])
        assert err < 1e-9, (k, err)


def test_damped_sync_cycles_match_oracle(G):
    print("case: coarse-grid cycles FP64, synchronous damped 0.5", flush=True)
    nx, ny, nz, batch = 12, 10, 9, 1
    A, arrs = _grid(G, nx, ny, nz, batch, 5, varcoef=False)
    b = W.uniform_b(A.n, 6)
    _, _, _, trail = OC.solve(nx, ny, nz, batch, *arrs, b, tol=0.0, max_cycles=2, colored=False,
                              damping=0.5)
    o = G.gabp_default_opts(msg_fp32=0, tol=0.0, max_restarts=2, freeze=0, damping=0.5)
    rc, plan = G.gabp_plan_create_grid(A, o)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rc, st = G.gabp_plan_solve_coarse(plan, dev(b), x)
    G.gabp_plan_destroy(plan)
    assert rc == G.GABP_NOT_CONVERGED
    xh = x.cpu().numpy()
    assert np.linalg.norm(xh - trail[1]) / np.linalg.norm(trail[1]) < 1e-9


def test_fp32_stack_reaches_1e8_in_few_cycles(G):
    print("case: coarse-grid solve FP32 to 1e-8, 4 grids of 32^3", flush=True)
    nx = ny = nz = 32
    batch = 4
    A, arrs = _grid(G, nx, ny, nz, batch, 7)
    b = W.normal_b(A.n, 8)
    o = G.gabp_default_opts(schedule=G.GABP_SCHEDULE_COLORED)
    rc, plan = G.gabp_plan_create_grid(A, o)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rc, st = G.gabp_plan_solve_coarse(plan, dev(b), x)
    xp = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rc2, st2 = G.gabp_plan_solve(plan, dev(b), xp)
    G.gabp_plan_destroy(plan)
    assert rc == G.GABP_OK and rc2 == G.GABP_OK
    n = nx * ny * nz
    xh = x.cpu().numpy()
    for t in range(batch):
        sl = slice(t * n, (t + 1) * n)
        _, rn = oracle.residual_grid(nx, ny, nz, 1, b[sl], xh[sl], diag=arrs[0][sl],
                                     cx=arrs[1][sl], cy=arrs[2][sl], cz=arrs[3][sl])
        assert rn / np.linalg.norm(b[sl]) <= 1e-8, t
    print(f"coarse: {st.restarts} corrections, {st.sweeps} sweeps, {st.seconds * 1e3:.1f} ms; "
          f"plain: {st2.sweeps} sweeps (slowest grid), {st2.seconds * 1e3:.1f} ms", flush=True)
    assert st.restarts <= 20
    assert st.sweeps < st2.mean_sweeps / 4
    np.testing.assert_allclose(xh, xp.cpu().numpy(), rtol=0, atol=1e-6 * np.abs(xh).max())


def test_zero_rhs_and_other_plans(G):
    print("case: coarse-grid solve edge cases", flush=True)
    A, arrs = _grid(G, 8, 8, 8, 1, 9)
    rc, plan = G.gabp_plan_create_grid(A)
    x = torch.full((A.n,), 5.0, dtype=torch.float64, device="cuda")
    rc, st = G.gabp_plan_solve_coarse(plan, dev(np.zeros(A.n)), x)
    assert rc == G.GABP_OK and float(x.abs().max()) == 0.0
    # a grid small enough to be its own coarsest level: GaBP sweeps alone
    A4, arrs4 = _grid(G, 4, 4, 4, 2, 10)
    rc, p4 = G.gabp_plan_create_grid(A4, G.gabp_default_opts(msg_fp32=0, tol=1e-10,
                                                              max_restarts=200))
    b4 = W.normal_b(A4.n, 11)
    x4 = torch.zeros(A4.n, dtype=torch.float64, device="cuda")
    rc, st = G.gabp_plan_solve_coarse(p4, dev(b4), x4)
    assert rc == G.GABP_OK
    G.gabp_plan_destroy(p4)
    G.gabp_plan_destroy(plan)
    m = W.poisson2d(6)
    rc, pc = G.gabp_plan_create(G.DeviceCSR.from_host(m))
    rc, st = G.gabp_plan_solve_coarse(pc, dev(np.ones(m.n)),
                                      torch.zeros(m.n, dtype=torch.float64, device="cuda"))
    assert rc == G.GABP_ERR_UNSUPPORTED
    G.gabp_plan_destroy(pc)


def test_tail_equals_plans_fp64(G):
    """The smallest levels inside one launch give the corrections of the same
    levels run as plans, to FP64 rounding, over a whole solve (freeze off:
    the tail never settles its precisions)."""
    print("case: coarse-grid tail vs plans, FP64 solve, 3 grids of 24^3", flush=True)
    A, arrs = _grid(G, 24, 24, 24, 3, 14)
    b = dev(W.normal_b(A.n, 15))
    o = G.gabp_default_opts(msg_fp32=0, freeze=0, tol=1e-10,
                            schedule=G.GABP_SCHEDULE_COLORED)
    out = {}
    for tail in ("tail", "plans", "tail_w", "plans_w"):
        rc, p = G.gabp_plan_create_grid(A, o)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        with level_mode(tail):
            rc, st = G.gabp_plan_solve_coarse(p, b, x)
        G.gabp_plan_destroy(p)
        assert rc == G.GABP_OK, (tail, G.status_name(rc))
        out[tail] = (x.cpu().numpy(), st)
        print(f"{tail}: {st.restarts} corrections, {st.seconds * 1e3:.1f} ms", flush=True)
    for w in ("", "_w"):
        assert out["tail" + w][1].restarts == out["plans" + w][1].restarts, w
        xt, xp = out["tail" + w][0], out["plans" + w][0]
        assert np.abs(xt - xp).max() <= 1e-9 * np.abs(xp).max(), w


def test_graph_replays_equal_eager_corrections(G):
    """Steady-state corrections run from a captured graph: repeated solves on
    one plan (the graph captured in the first, replayed in all) give bitwise
    the answer of a plan that runs every correction eagerly, with other work
    and synchronisations of the program between the replays."""
    import os
    print("case: coarse-grid corrections from a captured graph vs eager", flush=True)
    nx = ny = nz = 24
    batch = 3
    A, arrs = _grid(G, nx, ny, nz, batch, 12)
    b = dev(W.normal_b(A.n, 13))
    o = G.gabp_default_opts(schedule=G.GABP_SCHEDULE_COLORED)
    os.environ["GABP_COARSE_GRAPH"] = "0"
    try:
        rc, pe = G.gabp_plan_create_grid(A, o)
        xe = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        rc, ste = G.gabp_plan_solve_coarse(pe, b, xe)  # the hierarchy is built here
    finally:
        del os.environ["GABP_COARSE_GRAPH"]
    assert rc == G.GABP_OK and ste.restarts >= 5  # steady corrections exist
    rc, pg = G.gabp_plan_create_grid(A, o)
    for rep in range(3):
        xg = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        rc, stg = G.gabp_plan_solve_coarse(pg, b, xg)
        assert rc == G.GABP_OK and stg.restarts == ste.restarts
        assert torch.equal(xg, xe), rep
        # the program's own eager work between the replays
        xp = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        assert G.gabp_plan_solve(pg, b, xp)[0] == G.GABP_OK
        torch.cuda.synchronize()
    G.gabp_plan_destroy(pg)
    G.gabp_plan_destroy(pe)


def test_damped_colored_cycles_match_oracle(G):
    """The red-black schedule with damping (the plan's own factor smooths):
    x after each of the first two cycles equals the oracle's in FP64 (the
    last launch of every smoothing also writes its colour's means)."""
    print("case: coarse-grid cycles FP64, red-black damped 0.3", flush=True)
    nx, ny, nz, batch = 14, 12, 10, 2
    A, arrs = _grid(G, nx, ny, nz, batch, 17)
    b = W.normal_b(A.n, 18)
    _, _, _, trail = OC.solve(nx, ny, nz, batch, *arrs, b, tol=0.0, max_cycles=2, colored=True,
                              damping=0.3)
    for k in (1, 2):
        o = G.gabp_default_opts(msg_fp32=0, tol=0.0, max_restarts=k, freeze=0, damping=0.3,
                                schedule=G.GABP_SCHEDULE_COLORED)
        rc, plan = G.gabp_plan_create_grid(A, o)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        rc, st = G.gabp_plan_solve_coarse(plan, dev(b), x)
        G.gabp_plan_destroy(plan)
        assert rc == G.GABP_NOT_CONVERGED and st.restarts == k
        xh = x.cpu().numpy()
        assert np.linalg.norm(xh - trail[k - 1]) / np.linalg.norm(trail[k - 1]) < 1e-9, k


@pytest.mark.parametrize("kind", ["colored", "colored_damped", "sync_damped"])
def test_fp32_settled_levels_reach_tolerance(G, kind):
    """FP32 messages with the levels' precisions settled after their first
    smoothing (the informations dropped at the switch, not copied), for both
    engines: every grid's FP64 residual, recomputed by the oracle, meets the
    tolerance, and x agrees with the plain solve."""
    print(f"case: coarse-grid FP32 settled levels, {kind}", flush=True)
    if kind == "sync_damped":
        nx = ny = nz = 32
        batch, varc = 1, False
        o = G.gabp_default_opts(damping=0.5)
    else:
        nx = ny = nz = 24
        batch, varc = 3, True
        o = G.gabp_default_opts(schedule=G.GABP_SCHEDULE_COLORED,
                                damping=0.3 if kind == "colored_damped" else 0.0)
    A, arrs = _grid(G, nx, ny, nz, batch, 19, varc)
    b = W.normal_b(A.n, 20)
    rc, plan = G.gabp_plan_create_grid(A, o)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rc, st = G.gabp_plan_solve_coarse(plan, dev(b), x)
    xp = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rc2, st2 = G.gabp_plan_solve(plan, dev(b), xp)
    G.gabp_plan_destroy(plan)
    assert rc == G.GABP_OK and rc2 == G.GABP_OK, (G.status_name(rc), G.status_name(rc2))
    n = nx * ny * nz
    xh = x.cpu().numpy()
    for t in range(batch):
        sl = slice(t * n, (t + 1) * n)
        _, rn = oracle.residual_grid(nx, ny, nz, 1, b[sl], xh[sl], diag=arrs[0][sl],
                                     cx=arrs[1][sl], cy=arrs[2][sl], cz=arrs[3][sl])
        assert rn / np.linalg.norm(b[sl]) <= 1e-8, t
    print(f"{kind}: {st.restarts} corrections, plain {st2.sweeps} sweeps", flush=True)
    assert st.restarts <= 20
    np.testing.assert_allclose(xh, xp.cpu().numpy(), rtol=0, atol=1e-6 * np.abs(xh).max())


def test_plain_sum_of_corrections_matches_oracle(G):
    """GABP_COARSE_GCR=0 at plan time adds the corrections as they come: x
    after each of the first cycles equals the oracle's unaccelerated trail."""
    print("case: coarse-grid cycles FP64 without the GCR combination", flush=True)
    nx, ny, nz, batch = 16, 16, 16, 2
    A, arrs = _grid(G, nx, ny, nz, batch, 21)
    b = W.normal_b(A.n, 22)
    _, _, _, trail = OC.solve(nx, ny, nz, batch, *arrs, b, tol=0.0, max_cycles=3, accel=False)
    for k in (1, 3):
        o = G.gabp_default_opts(msg_fp32=0, tol=0.0, max_restarts=k, freeze=0,
                                schedule=G.GABP_SCHEDULE_COLORED)
        rc, plan = G.gabp_plan_create_grid(A, o)
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        with env("GABP_COARSE_GCR", "0"):
            rc, st = G.gabp_plan_solve_coarse(plan, dev(b), x)
        G.gabp_plan_destroy(plan)
        assert rc == G.GABP_NOT_CONVERGED and st.restarts == k
        xh = x.cpu().numpy()
        assert np.linalg.norm(xh - trail[k - 1]) / np.linalg.norm(trail[k - 1]) < 1e-9, k


@pytest.mark.parametrize("budget", [0, 2, None])
def test_reported_residual_is_that_of_x(G, budget):
    """The GCR step carries the residual along with x (r - alpha A c'); the
    residual a solve reports is still b - A x of the x it returns, the worst
    grid's, whether it stops at the tolerance or at the correction budget."""
    print(f"case: coarse-grid reported residual, budget {budget}, 3 grids of 24^3", flush=True)
    nx = ny = nz = 24
    batch = 3
    A, arrs = _grid(G, nx, ny, nz, batch, 31)
    b = W.normal_b(A.n, 32)
    kw = dict(msg_fp32=0, tol=1e-10, schedule=G.GABP_SCHEDULE_COLORED)
    if budget is not None:
        kw["max_restarts"] = budget
    rc, plan = G.gabp_plan_create_grid(A, G.gabp_default_opts(**kw))
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rc, st = G.gabp_plan_solve_coarse(plan, dev(b), x)
    G.gabp_plan_destroy(plan)
    if budget is None:
        assert rc == G.GABP_OK
    else:
        assert rc == G.GABP_NOT_CONVERGED and st.restarts == budget
    n = nx * ny * nz
    xh = x.cpu().numpy()
    worst = 0.0
    for t in range(batch):
        sl = slice(t * n, (t + 1) * n)
        _, rn = oracle.residual_grid(nx, ny, nz, 1, b[sl], xh[sl], diag=arrs[0][sl],
                                     cx=arrs[1][sl], cy=arrs[2][sl], cz=arrs[3][sl])
        worst = max(worst, rn / np.linalg.norm(b[sl]))
    print(f"reported {st.rel_residual:.6e}, b - A x {worst:.6e}, {st.restarts} corrections",
          flush=True)
    assert st.rel_residual == pytest.approx(worst, rel=1e-9)
    if budget is None:
        assert worst <= 1e-10
