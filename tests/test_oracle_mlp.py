"""Pins of the FP64 warm-start network oracle (oracle/mlp.py).

The network is not in the paper; what pins it is mathematics: central finite
differences of the loss against the analytic gradient, the affine map the
network reduces to when every unit is active, closed forms of Adam's first
steps, exact bfloat16 rounding cases, and the message layout of the grid
targets checked against the CSR oracle on a small grid.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import mlp


def test_parameter_count():
    assert mlp.N_PARAMS == 8 * 64 + 64 + 64 * 64 + 64 + 12 * 64 + 12 == 5516
    th = W.mlp_params(1)
    assert th.size == mlp.N_PARAMS
    assert np.array_equal(mlp.pack(mlp.unpack(th)), th)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    th = W.mlp_params(seed)
    U, T, M = W.mlp_batch(16, seed)
    L, g = mlp.grad(th, U, T, M)
    assert abs(L - mlp.loss(th, U, T, M)) <= 1e-14 * max(1.0, L)
    rng = np.random.default_rng(seed)
    # every layer: a few entries of each weight matrix and bias
    idx, o = [], 0
    for name, shape in mlp.SHAPES:
        n = int(np.prod(shape))
        idx.extend(o + rng.choice(n, size=min(n, 10), replace=False))
        o += n
    h = 1e-6
    for k in idx:
        e = np.zeros_like(th); e[k] = h
        fd = (mlp.loss(th + e, U, T, M) - mlp.loss(th - e, U, T, M)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])), (k, fd, g[k])


def test_masked_outputs_carry_no_gradient():
    th = W.mlp_params(3)
    U, T, M = W.mlp_batch(8, 3)
    M2 = M.copy(); M2[:, 4:6] = 0.0
    T2 = T.copy(); T2[:, 4:6] = 1e6  # masked targets must not matter
    _, g1 = mlp.grad(th, U, T2 * 0 + T, M2)
    _, g2 = mlp.grad(th, U, T2, M2)
    np.testing.assert_allclose(g1, g2, rtol=0, atol=0)
    W3 = mlp.unpack(g1)["W3"]
    assert np.all(W3[4:6] == 0.0)


def test_all_active_network_is_one_affine_map():
    """With positive inputs, weights and biases every ReLU is active and the
    network is W3 W2 W1 u + (W3 W2 b1 + W3 b2 + b3), a product taken in the
    other association order."""
    rng = np.random.default_rng(4)
    p = {name: rng.uniform(0.01, 0.2, size=shape) for name, shape in mlp.SHAPES}
    th = mlp.pack(p)
    U = rng.uniform(0.1, 1.0, size=(5, 8))
    o, _ = mlp.forward(th, U)
    Wc = p["W3"] @ (p["W2"] @ p["W1"])
    bc = p["W3"] @ (p["W2"] @ p["b1"] + p["b2"]) + p["b3"]
    np.testing.assert_allclose(o, U @ Wc.T + bc, rtol=1e-13)
    # and with W2 = 0 the output no longer depends on the input
    p["W2"][:] = 0.0
    o, _ = mlp.forward(mlp.pack(p), U)
    np.testing.assert_allclose(o, np.tile(p["W3"] @ p["b2"] + p["b3"], (5, 1)), rtol=1e-14)


def test_adam_first_steps_move_each_parameter_by_lr():
    """With bias correction the first update is lr * g / |g| (up to eps), and a
    constant gradient keeps that size on the second step."""
    rng = np.random.default_rng(5)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m = np.zeros(50); v = np.zeros(50)
    g = np.where(np.abs(g) < 0.1, 0.1 * np.sign(g), g)  # eps / |g| <= 1e-7
    t1, m, v = mlp.adam_step(th, m, v, g, 1, 1e-3)
    np.testing.assert_allclose(th - t1, 1e-3 * np.sign(g), rtol=1e-6)
    t2, m, v = mlp.adam_step(t1, m, v, g, 2, 1e-3)
    np.testing.assert_allclose(t1 - t2, 1e-3 * np.sign(g), rtol=1e-6)


def test_bf16_rounding_cases():
    one = 1.0
    cases = {
        one: one,
        one + 2.0 ** -8: one,                       # halfway: ties to even (1.0)
        one + 3 * 2.0 ** -8: one + 2.0 ** -6,       # halfway: ties to even (odd -> up)
        one + 2.0 ** -8 + 2.0 ** -20: one + 2.0 ** -7,  # just above halfway
        -2.5: -2.5,
    }
    for x, want in cases.items():
        assert mlp.bf16_round(np.float32(x)) == want, (x, mlp.bf16_round(np.float32(x)), want)
    # every result is representable in 8 mantissa bits and within half an ulp
    xs = np.random.default_rng(6).standard_normal(1000).astype(np.float32)
    r = mlp.bf16_round(xs)
    assert np.all((r.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)
    ulp = 2.0 ** (np.floor(np.log2(np.abs(xs.astype(np.float64)))) - 7)
    assert np.all(np.abs(r - xs) <= 0.5 * ulp + 1e-30)


def test_grid_targets_follow_the_message_layout():
    """On a 3 x 2 x 2 grid the [6][N] targets of converged messages equal the
    oracle's CSR messages of the same edges, scaled by A_ii."""
    nx, ny, nz = 3, 2, 2
    csr, coef = W.grid_stack(nx, ny, nz, 1, varcoef=True, seed=3, ell=2.0)
    b = W.normal_b(csr.n, 3)
    R = oracle.Rounds(csr, b).step(60)
    P, h = R.P, R.information()
    N = csr.n
    P6 = np.zeros((6, N)); h6 = np.zeros((6, N))
    step = {0: 1, 1: -1, 2: nx, 3: -nx, 4: nx * ny, 5: -nx * ny}
    for i in range(N):
        for e in range(csr.row_ptr[i], csr.row_ptr[i + 1]):
            j = csr.col[e]
            if j == i:
                continue
            d = [dd for dd, s in step.items() if j - i == s][0]
            P6[d, i] = P[e]; h6[d, i] = h[e]
    T, M = mlp.grid_targets(nx, ny, nz, 1, coef, P6, h6)
    diag, a = mlp.grid_couplings(nx, ny, nz, 1, coef)
    dense = W.dense_from_csr(csr)
    np.testing.assert_allclose(diag, np.diag(dense))
    for d in range(6):
        for i in range(N):
            j = i + step[d]
            inside = 0 <= j < N and a[d, i] != 0
            if inside:
                assert a[d, i] == dense[i, j]
                assert T[i, 2 * d] == P6[d, i] / diag[i] and M[i, 2 * d] == 1
            else:
                assert M[i, 2 * d] == 0 and T[i, 2 * d + 1] == 0
    U = mlp.grid_features(nx, ny, nz, 1, coef, b)
    np.testing.assert_allclose(U[:, 0], np.log(diag))
    np.testing.assert_allclose(U[:, 7], b / diag)
    assert np.count_nonzero(U[:, 1:7]) == csr.nnz - N
