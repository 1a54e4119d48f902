"""gabp_plan_workspace_bytes: the device memory a plan holds.

A red-black grid plan holds at least its messages (P, h) and right-hand side;
a solve that settles the precisions adds the settled-phase buffers, a
coarse-grid solve its levels; plans count separately; and the count agrees
with the device's free-memory change when a large plan is made and
destroyed."""
import numpy as np
import pytest

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


def _grid(G, n, batch, seed):
    _, coef = W.grid_stack(n, n, n, batch, varcoef=True, seed=seed, ell=4.0, shift=0.01,
                           with_csr=False)
    return G.DeviceGrid(n, n, n, batch, diag=dev(coef["diag"]), cx=dev(coef["cx"]),
                        cy=dev(coef["cy"]), cz=dev(coef["cz"]))


def test_grid_plan_bytes_grow_with_what_solves_add(G):
    print("case: workspace bytes of a red-black grid plan, 2 grids of 32^3", flush=True)
    A = _grid(G, 32, 2, 1)
    N = A.n
    rc, plan = G.gabp_plan_create_grid(A, G.gabp_default_opts(schedule=G.GABP_SCHEDULE_COLORED))
    assert rc == G.GABP_OK
    rc, b0 = G.gabp_plan_workspace_bytes(plan)
    assert rc == G.GABP_OK
    # FP32 (P, h) on 6 slots per node + the right-hand side; bounded above by
    # a few times that (coefficient copies, controller state)
    assert 52 * N <= b0 < 200 * N, b0
    b = dev(W.normal_b(N, 2))
    x = torch.zeros(N, dtype=torch.float64, device="cuda")
    rc, st = G.gabp_plan_solve(plan, b, x)
    assert rc == G.GABP_OK and st.frozen_sweeps > 0
    rc, b1 = G.gabp_plan_workspace_bytes(plan)
    # settled coefficients and informations: 2 x 6 FP32 per node
    assert b1 >= b0 + 48 * N, (b0, b1)
    rc, st = G.gabp_plan_solve_coarse(plan, b, x)
    assert rc == G.GABP_OK
    rc, b2 = G.gabp_plan_workspace_bytes(plan)
    # at least the finest level's two FP64 vectors
    assert b2 >= b1 + 16 * N, (b1, b2)
    # another plan counts on its own and leaves this one's count alone
    rc, other = G.gabp_plan_create_grid(_grid(G, 16, 1, 3))
    rc, bo = G.gabp_plan_workspace_bytes(other)
    assert rc == G.GABP_OK and 0 < bo < b0
    G.gabp_plan_destroy(other)
    rc, again = G.gabp_plan_workspace_bytes(plan)
    assert again == b2
    G.gabp_plan_destroy(plan)


def test_csr_plan_bytes_and_device_free_memory(G):
    print("case: workspace bytes of a CSR plan vs free device memory, Poisson 1024^2", flush=True)
    m = W.poisson2d(1024)
    A = G.DeviceCSR.from_host(m)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    rc, plan = G.gabp_plan_create(A)
    assert rc == G.GABP_OK
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    rc, nb = G.gabp_plan_workspace_bytes(plan)
    assert rc == G.GABP_OK
    E = m.nnz - m.n
    assert nb >= 2 * E * 8, nb  # two FP32 (P, h) message buffers at least
    used = free0 - free1
    print(f"plan holds {nb / 2**20:.1f} MiB; free device memory fell by {used / 2**20:.1f} MiB",
          flush=True)
    # the runtime rounds large allocations up and may serve small ones from
    # memory it already holds: a few MiB either way
    assert nb <= used + (8 << 20) and used <= nb + (32 << 20), (nb, used)
    G.gabp_plan_destroy(plan)
