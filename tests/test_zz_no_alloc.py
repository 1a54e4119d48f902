"""The allocation-free residual (gabp_residual_noalloc) against gabp_residual
through the C ABI: the same kernels in the same order, so bitwise the same
r and relative norm, on consecutive calls that reuse the GPU's static scratch
array (a large system, then a smaller one, then a malformed matrix, then a
valid one again), and against the oracle's residual to 1e-12."""
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


def _both(G, m, b, x):
    A = G.DeviceCSR.from_host(m)
    bd, xd = dev(b), dev(x)
    r0 = torch.full((m.n,), np.nan, dtype=torch.float64, device="cuda")
    r1 = torch.full((m.n,), np.nan, dtype=torch.float64, device="cuda")
    rc0, rel0 = G.gabp_residual(A, bd, xd, r0)
    rc1, rel1 = G.gabp_residual_noalloc(A, bd, xd, r1)
    return (rc0, rel0, r0.cpu().numpy()), (rc1, rel1, r1.cpu().numpy())


def _check(G, m, seed):
    rng = np.random.default_rng(seed)
    b, x = rng.standard_normal(m.n), rng.standard_normal(m.n)
    (rc0, rel0, r0), (rc1, rel1, r1) = _both(G, m, b, x)
    assert rc0 == G.GABP_OK and rc1 == G.GABP_OK
    assert rel1 == rel0  # bitwise: same kernels, same block count, same order
    assert np.array_equal(r1, r0)
    ro, rn = oracle.residual(m, b, x)
    np.testing.assert_allclose(r1, ro, rtol=1e-12, atol=1e-12)
    assert rel1 == pytest.approx(rn / np.linalg.norm(b), rel=1e-12)


def test_noalloc_residual_consecutive_calls(G):
    print("case: no-alloc residual, random SDD n=300007 then n=1237", flush=True)
    # more rows than 2048 residual workgroups cover at once (grid-stride rows),
    # then a much smaller system whose partials overwrite only the first slots
    _check(G, W.sdd_random(300007, 11), 1)
    _check(G, W.sdd_random(1237, 12), 2)


def test_noalloc_residual_errors_and_recovery(G):
    print("case: no-alloc residual, malformed CSR then a valid call", flush=True)
    bad = W.poisson2d(5)
    bad.col = bad.col.copy()
    bad.col[[0, 1]] = bad.col[[1, 0]]  # unsorted columns in row 0
    A = G.DeviceCSR.from_host(bad)
    z = dev(np.ones(bad.n))
    assert G.gabp_residual_noalloc(A, z, z)[0] == G.GABP_ERR_ARG
    # the flags of the failed call do not leak into the next one
    _check(G, W.poisson2d(33), 3)
    # empty system and zero right-hand side
    e = W.csr_from_dense(np.zeros((0, 0)))
    rc, rel = G.gabp_residual_noalloc(G.DeviceCSR.from_host(e), dev(np.zeros(0)), dev(np.zeros(0)))
    assert rc == G.GABP_OK and rel == 0.0
    m = W.poisson2d(4)
    xb = np.linspace(-1.0, 1.0, m.n)
    rc, rel = G.gabp_residual_noalloc(G.DeviceCSR.from_host(m), dev(np.zeros(m.n)), dev(xb))
    _, rn = oracle.residual(m, np.zeros(m.n), xb)
    assert rc == G.GABP_OK and rel == pytest.approx(rn, rel=1e-12)  # ||r|| when b = 0
