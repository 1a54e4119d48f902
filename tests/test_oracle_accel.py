"""Pins of the oracle's convergence acceleration (section IV-A: Aitken's
method and Steffensen's iterations) against closed forms, the LAPACK solve
and the paper's printed Poisson iteration counts (a +-50% band: the paper's
initial guess, ordering and stopping rule are not fully specified)."""
import numpy as np
import pytest

import oracle
import workloads as W


@pytest.mark.parametrize("q", [0.9, 0.5, -0.3, -0.95, 1.7, -2.5])
def test_aitken_is_exact_on_geometric_sequences(q):
    """x_n = x* + c q^n: Aitken's y_n equals x* for any n (its defining
    property; also for |q| > 1, where the sequence diverges)."""
    rng = np.random.default_rng(3)
    xs, c = rng.standard_normal(50), rng.standard_normal(50)
    for n in (0, 3, 7):
        x0, x1, x2 = (xs + c * q ** k for k in (n, n + 1, n + 2))
        np.testing.assert_allclose(oracle.aitken(x0, x1, x2), xs, rtol=1e-10, atol=1e-10)


def test_aitken_per_component_uses_each_components_own_ratio():
    """Each node extrapolates its own history: components with different
    ratios are all exact at once."""
    q = np.array([0.2, -0.7, 0.99, 0.5])
    xs = np.array([1.0, -2.0, 3.0, 0.25])
    c = np.array([1.0, 1.0, -0.5, 1e-3])
    x = [xs + c * q ** k for k in (4, 5, 6)]
    np.testing.assert_allclose(oracle.aitken(*x), xs, rtol=1e-11)


def test_aitken_zero_second_difference_keeps_the_last_member():
    """A vanishing second difference (reading of the paper's open case): a
    sequence at rest or moving linearly keeps x_{n+2}."""
    x0 = np.array([1.0, 5.0, -3.0, 0.0])
    x1 = np.array([2.0, 5.0, -3.0, 1.0])
    x2 = np.array([3.0, 5.0, -3.0, 4.0])
    y = oracle.aitken(x0, x1, x2)
    assert y[0] == 3.0 and y[1] == 5.0 and y[2] == -3.0
    # the last component has a nonzero second difference: 0 - 1 / 2
    assert y[3] == pytest.approx(-0.5, rel=1e-15)


def test_parallel_gabp_with_aitken_accelerates_poisson():
    """The table of section IX on the 2-D Poisson system with p = 10: parallel
    GaBP 134 iterations, parallel GaBP + Aitken 25.  Same ratio class here
    (b = 1, relative residual 1e-6, stride 2): each count within +-50% of the
    printed one and at least 3x fewer rounds with the extrapolation; the
    extrapolated vector is the LAPACK solution to the tolerance."""
    m = W.poisson2d(10)
    b = np.ones(m.n)
    xs = np.linalg.solve(W.dense_from_csr(m), b)
    plain = oracle.solve(m, b, tol=1e-6, max_rounds=5000)
    st, y, rounds = oracle.solve_aitken(m, b, stride=2, tol=1e-6)
    assert plain.status == st == oracle.OK
    assert 0.5 * 134 <= plain.rounds <= 1.5 * 134
    assert 0.5 * 25 <= rounds <= 1.5 * 25
    assert plain.rounds >= 3 * rounds
    assert np.linalg.norm(b - W.dense_from_csr(m) @ y) / np.linalg.norm(b) <= 1e-6
    np.testing.assert_allclose(y, xs, rtol=0, atol=1e-5 * np.abs(xs).max())


def test_aitken_error_vanishes_relative_to_the_iterate():
    """Aitken's theorem (section IV-A): |x* - y_n| / |x* - x_n| -> 0.  On the
    32 x 32 Poisson system the extrapolated vector at the round where it meets
    1e-10 is far closer to the LAPACK solution than GaBP's own means there."""
    m = W.poisson2d(32)
    b = W.uniform_b(m.n, 0)
    xs = np.linalg.solve(W.dense_from_csr(m), b)
    st, y, rounds = oracle.solve_aitken(m, b, stride=2, tol=1e-10)
    assert st == oracle.OK and rounds % 2 == 0
    R = oracle.Rounds(m, b).step(rounds)
    x, _ = R.marginals()
    assert np.abs(y - xs).max() <= 1e-3 * np.abs(x - xs).max()
    assert np.linalg.norm(b - W.dense_from_csr(m) @ y) / np.linalg.norm(b) <= 1e-10


def test_steffensen_on_a_tree_stops_after_one_exact_cycle():
    """On a tree GaBP is exact after diameter rounds (section IV); once the
    means are at rest the second difference vanishes, the extrapolation keeps
    the last iterate, and a cycle longer than diameter + 2 strides returns
    the exact solution at its first residual test."""
    m = W.random_tree(60, 3, dominant=True)
    b = W.normal_b(m.n, 3)
    d = W.tree_diameter(m)
    xs = np.linalg.solve(W.dense_from_csr(m), b)
    st, x, rounds, cycles, rel = oracle.solve_steffensen(m, b, stride=1, cycle=d + 2, tol=1e-13)
    assert st == oracle.OK and cycles == 1 and rounds == d + 2
    np.testing.assert_allclose(x, xs, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("stride,cycle", [(8, 400), (8, 300), (16, 400)])
def test_steffensen_reaches_the_solution_in_fewer_rounds(stride, cycle):
    """Steffensen's iterations (re-injection as a restart of the information
    messages on the correction system, precisions kept) converge to the LAPACK
    solution and need fewer rounds than plain GaBP on 32 x 32 Poisson."""
    m = W.poisson2d(32)
    b = W.uniform_b(m.n, 0)
    xs = np.linalg.solve(W.dense_from_csr(m), b)
    plain = oracle.solve(m, b, tol=1e-10, max_rounds=10000)
    st, x, rounds, cycles, rel = oracle.solve_steffensen(m, b, stride=stride, cycle=cycle,
                                                         tol=1e-10)
    assert st == oracle.OK and rel <= 1e-10 and rounds == cycles * cycle
    assert rounds < plain.rounds
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-8 * np.abs(xs).max())


def test_accelerated_solvers_reject_bad_arguments():
    m = W.poisson2d(4)
    b = np.ones(m.n)
    assert oracle.solve_aitken(m, b, stride=0)[0] == oracle.ERR_ARG
    assert oracle.solve_steffensen(m, b, stride=2, cycle=3)[0] == oracle.ERR_ARG


def test_steffensen_cycles_compose_restarted_passes():
    """The cycle structure of the Steffensen reading, rebuilt from the pinned
    pieces (synchronous rounds, Aitken's formula, the residual): cycle 1 runs
    from zero messages on b; cycle 2 keeps cycle 1's precision messages, starts
    from zero information on r = b - A x1 and adds its extrapolated correction."""
    m = W.poisson2d(12)
    b = W.uniform_b(m.n, 4)
    A = W.dense_from_csr(m)
    s, L = 4, 40

    def cycle(rhs, P0):
        R = oracle.Rounds(m, rhs)
        if P0 is not None:
            R.P = P0.copy()
        samples = {}
        for t in range(1, L + 1):
            R.step()
            if t in (L - 2 * s, L - s, L):
                samples[t] = R.marginals()[0]
        return oracle.aitken(samples[L - 2 * s], samples[L - s], samples[L]), R.P

    d1, P1 = cycle(b, None)
    x1 = d1
    d2, _ = cycle(b - A @ x1, P1)
    x2 = x1 + d2
    st, x, rounds, cycles, rel = oracle.solve_steffensen(m, b, stride=s, cycle=L, tol=0.0,
                                                         max_cycles=2)
    assert st == oracle.NOT_CONVERGED and cycles == 2 and rounds == 2 * L
    np.testing.assert_allclose(x, x2, rtol=1e-12, atol=1e-13 * np.abs(x2).max())
    assert rel == pytest.approx(np.linalg.norm(b - A @ x2) / np.linalg.norm(b), rel=1e-9)
