"""GPU parity of the structured-grid path (5/7-point stencils, constant or
variable coefficients, stacked grids) against the FP64 CPU oracle run on the
CSR form of the same operator.  Tolerances as in test_gpu_csr.py."""
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


def device_grid(G, nx, ny, nz, bt, coef):
    kw = dict(nx=nx, ny=ny, nz=nz, batch=bt, diag_value=coef["dval"], off_value=coef["off"])
    for k in ("diag", "cx", "cy", "cz"):
        if coef[k] is not None:
            kw[k] = dev(coef[k])
    return G.DeviceGrid(**kw)


def direction_map(m, nx, ny, nz, bt):
    """For the direction-major layout [6][N]: CSR slot of the message node i
    sends toward d (or -1 where there is no edge)."""
    N = nx * ny * nz * bt
    i = np.arange(N)
    x, y, zl = i % nx, (i // nx) % ny, (i // (nx * ny)) % nz
    nxy = nx * ny
    nbr = [(x < nx - 1, i + 1), (x > 0, i - 1), (y < ny - 1, i + nx), (y > 0, i - nx),
           (zl < nz - 1, i + nxy), (zl > 0, i - nxy)]
    rows = np.repeat(np.arange(m.n, dtype=np.int64), np.diff(m.row_ptr))
    keys = rows * N + m.col
    out = np.full((6, N), -1, dtype=np.int64)
    for d, (ok, j) in enumerate(nbr):
        k = i[ok].astype(np.int64) * N + j[ok]
        pos = np.searchsorted(keys, k)
        assert np.all(keys[pos] == k)
        out[d, ok] = pos
    return out


def to_dirs(slot_vals, dmap):
    out = np.zeros(dmap.shape)
    ok = dmap >= 0
    out[ok] = slot_vals[dmap[ok]]
    return out.ravel()


CASES = {
    "c3d_13x11x7": (13, 11, 7, 1, False, 0.01),
    "var3d_9x7x5_b2": (9, 7, 5, 2, True, 0.0),
    "c2d_17x13": (17, 13, 1, 1, False, 0.0),
    "var2d_11x9_b3": (11, 9, 1, 3, True, 0.0),
}


def _plan(G, case, fp32, **kw):
    nx, ny, nz, bt, vc, sh = CASES[case]
    m, coef = W.grid_stack(nx, ny, nz, bt, varcoef=vc, shift=sh, seed=5)
    A = device_grid(G, nx, ny, nz, bt, coef)
    rc, plan = G.gabp_plan_create_grid(A, G.gabp_default_opts(msg_fp32=int(fp32), **kw))
    assert rc == G.GABP_OK, G.status_name(rc)
    return m, A, plan, direction_map(m, nx, ny, nz, bt)


def _msgs(G, plan, A):
    P = torch.zeros(A.nnz, dtype=torch.float64, device="cuda")
    h = torch.zeros(A.nnz, dtype=torch.float64, device="cuda")
    assert G.gabp_plan_get_messages(plan, P, h) == G.GABP_OK
    return host(P), host(h)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("damping", [0.0, 0.3, 0.5, 0.7])
def test_grid_fp64_trajectory_matches_oracle(G, case, damping):
    m, A, plan, dmap = _plan(G, case, fp32=False, damping=damping)
    b = W.uniform_b(m.n, 3)
    assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
    R = oracle.Rounds(m, b, algorithm=2, damping=damping)
    for t in range(1, 7):
        R.step()
        assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
        P, h = _msgs(G, plan, A)
        Po, ho = to_dirs(R.P, dmap), to_dirs(R.information(), dmap)
        np.testing.assert_allclose(P, Po, rtol=1e-11, atol=1e-13 * np.abs(Po).max(), err_msg=f"P {t}")
        np.testing.assert_allclose(h, ho, rtol=1e-10, atol=1e-12 * np.abs(ho).max(), err_msg=f"h {t}")
        mean = torch.zeros(m.n, dtype=torch.float64, device="cuda")
        prec = torch.zeros(m.n, dtype=torch.float64, device="cuda")
        assert G.gabp_plan_marginals(plan, mean, prec) == G.GABP_OK
        mo, po = R.marginals()
        np.testing.assert_allclose(host(mean), mo, rtol=1e-10, atol=1e-12 * np.abs(mo).max())
        np.testing.assert_allclose(host(prec), po, rtol=1e-10)
    G.gabp_plan_destroy(plan)


@pytest.mark.parametrize("case", sorted(CASES))
def test_grid_fp32_trajectory_matches_oracle(G, case):
    m, A, plan, dmap = _plan(G, case, fp32=True)
    b = W.uniform_b(m.n, 4)
    assert G.gabp_plan_reset(plan, dev(b)) == G.GABP_OK
    R = oracle.Rounds(m, b, algorithm=2)
    for t in range(1, 5):
        R.step()
        assert G.gabp_plan_sweeps(plan, 1) == G.GABP_OK
        P, h = _msgs(G, plan, A)
        Po, ho = to_dirs(R.P, dmap), to_dirs(R.information(), dmap)
        np.testing.assert_allclose(P, Po, rtol=2e-5, atol=2e-6 * np.abs(Po).max())
        np.testing.assert_allclose(h, ho, rtol=2e-5, atol=2e-5 * np.abs(ho).max())
    G.gabp_plan_destroy(plan)


def _solve(G, nx, ny, nz, bt, coef, b, **kw):
    A = device_grid(G, nx, ny, nz, bt, coef)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    rc, st = G.gabp_solve_grid(A, dev(b), x, opts=G.gabp_default_opts(**kw))
    return rc, st, host(x)


def _grid_rel(nx, ny, nz, bt, coef, b, x):
    _, rn = oracle.residual_grid(nx, ny, nz, bt, b, x, coef["diag"], coef["dval"], coef["cx"],
                                 coef["cy"], coef["cz"], coef["off"])
    return rn / np.linalg.norm(b)


@pytest.mark.parametrize("freeze", [1, 0])
def test_poisson3d_damped_fp32_refined(G, freeze):
    """3-D Poisson + 0.01 shift, FP32 messages, damping 0.5, FP64 refinement
    to 1e-8 (the large-grid configuration at a test size)."""
    nx, ny, nz = 24, 20, 18
    m, coef = W.grid_stack(nx, ny, nz, 1, shift=0.01)
    b = W.uniform_b(m.n, 1)
    rc, st, x = _solve(G, nx, ny, nz, 1, coef, b, damping=0.5, tol=1e-8, freeze=freeze)
    assert rc == G.GABP_OK, G.status_name(rc)
    assert _grid_rel(nx, ny, nz, 1, coef, b, x) <= 1e-8
    assert (st.frozen_sweeps > 0) == bool(freeze)
    ref = oracle.solve(m, b, tol=1e-12, max_rounds=100000)
    assert ref.status == oracle.OK
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) < 1e-6


def test_varcoef_batch_fp32_refined(G):
    nx, ny, nz, bt = 12, 11, 10, 3
    m, coef = W.grid_stack(nx, ny, nz, bt, varcoef=True, seed=7)
    b = W.normal_b(m.n, 2)
    rc, st, x = _solve(G, nx, ny, nz, bt, coef, b, tol=1e-8)
    assert rc == G.GABP_OK, G.status_name(rc)
    assert _grid_rel(nx, ny, nz, bt, coef, b, x) <= 1e-8
    ref = oracle.solve(m, b, tol=1e-12, max_rounds=100000)
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) < 1e-6


def test_grid_poisson2d_fp64(G):
    """The 32 x 32 configuration through the grid path (FP64, to 1e-10)."""
    m, coef = W.grid_stack(32, 32, 1, 1)
    b = W.uniform_b(m.n, 0)
    rc, st, x = _solve(G, 32, 32, 1, 1, coef, b, msg_fp32=0, tol=1e-10)
    assert rc == G.GABP_OK
    assert _grid_rel(32, 32, 1, 1, coef, b, x) <= 1e-10
    ref = oracle.solve(W.poisson2d(32), b, tol=1e-12, max_rounds=50000)
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) < 1e-8


def test_grid_residual_entry_point(G):
    nx, ny, nz, bt = 10, 9, 8, 2
    _, coef = W.grid_stack(nx, ny, nz, bt, varcoef=True, seed=2, with_csr=False)
    n = nx * ny * nz * bt
    rng = np.random.default_rng(3)
    b, x = rng.standard_normal(n), rng.standard_normal(n)
    A = device_grid(G, nx, ny, nz, bt, coef)
    r = torch.empty(n, dtype=torch.float64, device="cuda")
    rc, rel = G.gabp_residual_grid(A, dev(b), dev(x), r)
    assert rc == G.GABP_OK
    ro, rn = oracle.residual_grid(nx, ny, nz, bt, b, x, coef["diag"], 0.0, coef["cx"], coef["cy"],
                                  coef["cz"], 0.0)
    np.testing.assert_allclose(host(r), ro, rtol=1e-12, atol=1e-12)
    assert rel == pytest.approx(rn / np.linalg.norm(b), rel=1e-12)


def test_grid_error_paths(G):
    b = torch.ones(27, dtype=torch.float64, device="cuda")
    x = torch.zeros(27, dtype=torch.float64, device="cuda")
    rc, _ = G.gabp_solve_grid(G.DeviceGrid(3, 3, 3, 1, diag_value=0.0, off_value=-1.0), b, x)
    assert rc == G.GABP_ERR_ZERO_DIAG
    d = torch.full((27,), 6.0, dtype=torch.float64, device="cuda")
    d[5] = 0.0
    rc, _ = G.gabp_solve_grid(G.DeviceGrid(3, 3, 3, 1, diag=d, off_value=-1.0), b, x)
    assert rc == G.GABP_ERR_ZERO_DIAG
    d[5] = float("nan")
    rc, _ = G.gabp_solve_grid(G.DeviceGrid(3, 3, 3, 1, diag=d, off_value=-1.0), b, x)
    assert rc == G.GABP_ERR_ARG
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    rc, _ = G.gabp_solve_grid(G.DeviceGrid(0, 3, 3, 1, diag_value=6.0, off_value=-1.0), e, e)
    assert rc == G.GABP_ERR_ARG


def test_grid_single_node_and_line(G):
    # 1 x 1 x 1: no edges, x = b / A_ii
    b = torch.tensor([3.0], dtype=torch.float64, device="cuda")
    x = torch.zeros(1, dtype=torch.float64, device="cuda")
    rc, _ = G.gabp_solve_grid(G.DeviceGrid(1, 1, 1, 1, diag_value=2.0, off_value=-1.0), b, x,
                              opts=G.gabp_default_opts(msg_fp32=0))
    assert rc == G.GABP_OK and host(x)[0] == pytest.approx(1.5)
    # a 1-D chain (ny = nz = 1) is a tree: exact after diameter sweeps
    n = 40
    m, coef = W.grid_stack(n, 1, 1, 1, shift=0.5)
    bb = W.uniform_b(n, 1)
    rc, st, xs = _solve(G, n, 1, 1, 1, coef, bb, msg_fp32=0, tol=1e-13)
    assert rc == G.GABP_OK
    np.testing.assert_allclose(xs, np.linalg.solve(W.dense_from_csr(m), bb), rtol=1e-11, atol=1e-13)


@pytest.mark.slow
def test_c5_full_size_256cubed(G):
    """The large-grid configuration at full size: 256^3, shift 0.01, damping
    0.5, FP32 messages + FP64 refinement to 1e-8; checked with the oracle's
    FP64 stencil residual over all 16.7M unknowns."""
    nx = ny = nz = 256
    _, coef = W.grid_stack(nx, ny, nz, 1, shift=0.01, with_csr=False)
    b = W.uniform_b(nx * ny * nz, 0)
    rc, st, x = _solve(G, nx, ny, nz, 1, coef, b, damping=0.5, tol=1e-8)
    assert rc == G.GABP_OK, G.status_name(rc)
    rel = _grid_rel(nx, ny, nz, 1, coef, b, x)
    assert rel <= 1e-8 and st.rel_residual == pytest.approx(rel, rel=1e-6)


@pytest.mark.parametrize("schedule", [0, 1])
def test_stack_every_grid_meets_the_tolerance(G, schedule):
    """The grids of a stack are independent systems: the solve stops only when
    each one's own relative residual is at most tol, also when their
    right-hand sides differ by orders of magnitude; a grid with b_t = 0 gets
    x_t = 0."""
    nx, ny, nz, bt = 12, 11, 10, 4
    _, coef = W.grid_stack(nx, ny, nz, bt, varcoef=True, seed=9, with_csr=False)
    n1 = nx * ny * nz
    b = W.normal_b(n1 * bt, 4)
    b[n1:2 * n1] *= 1e-6
    b[2 * n1:3 * n1] = 0.0
    rc, st, x = _solve(G, nx, ny, nz, bt, coef, b, tol=1e-8, schedule=schedule)
    assert rc == G.GABP_OK, G.status_name(rc)
    rels = []
    for t in range(bt):
        sl = slice(t * n1, (t + 1) * n1)
        c1 = {k: (coef[k][sl] if coef[k] is not None else None) for k in ("diag", "cx", "cy", "cz")}
        c1.update(dval=coef["dval"], off=coef["off"])
        if t == 2:
            assert np.all(x[sl] == 0.0)
            continue
        rels.append(_grid_rel(nx, ny, nz, 1, c1, b[sl], x[sl]))
    assert max(rels) <= 1e-8, rels
    assert st.rel_residual == pytest.approx(max(rels), rel=1e-6)


def test_check_interval_grows_with_long_passes(G):
    """check_every 0 (default) checks every 2 sweeps early in a pass and every
    8 in long passes; an explicit 2 keeps one check per 2 sweeps.  Both meet
    the tolerance (the oracle's residual)."""
    nx, ny, nz = 32, 30, 28
    m, coef = W.grid_stack(nx, ny, nz, 1, shift=0.001, with_csr=False)
    b = W.uniform_b(nx * ny * nz, 3)
    rc, auto, x = _solve(G, nx, ny, nz, 1, coef, b, tol=1e-8)
    assert rc == G.GABP_OK, G.status_name(rc)
    assert _grid_rel(nx, ny, nz, 1, coef, b, x) <= 1e-8
    rc, fixed, x2 = _solve(G, nx, ny, nz, 1, coef, b, tol=1e-8, check_every=2)
    assert rc == G.GABP_OK
    assert _grid_rel(nx, ny, nz, 1, coef, b, x2) <= 1e-8
    print(f"sweeps/checks: automatic {auto.sweeps}/{auto.checks}, fixed {fixed.sweeps}/{fixed.checks}",
          flush=True)
    assert auto.sweeps > 400
    assert fixed.checks * 2 == fixed.sweeps
    assert auto.checks * 4 < auto.sweeps
