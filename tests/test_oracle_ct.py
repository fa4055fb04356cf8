"""Pins of the continuous-time flowpipe oracle (``oracle/ct.py``).

What pins it: closed forms (constant dynamics: the exact translate of the box; linear
dynamics: the Picard polynomial equals the second-order Taylor expansion of exp(F s)
and every box contains the exact image exp(F t) X_0 with a first-step width within
O(h^2); the scalar Riccati equation x' = -x^2: the exact interval x_0 / (1 + x_0 t) of
a monotone flow, within twice its width over 20 steps), dense simulations (a high-accuracy ODE solver from sampled initial
states stays inside every time-point box and every segment box, and inside the TM
itself, p(y, s) + J, at sampled times of a step), and for the closed loop: a
controller with zero output weights reduces to the open-loop flowpipe with a constant
input, and simulated zero-order-hold closed loops stay inside every box.
"""
import numpy as np
import pytest

from oracle import ct, exact
from paper_2605_25346_amd.workloads import make_network

scipy = pytest.importorskip("scipy")
from scipy.integrate import solve_ivp  # noqa: E402
from scipy.linalg import expm  # noqa: E402


def _lv():
    Q = np.zeros((2, 2, 2)); Q[0, 0, 1] = -0.5; Q[1, 0, 1] = 0.25
    return ct.QuadDynamics(np.zeros(2), np.array([[1.0, 0.0], [0.0, -0.75]]), Q=Q)


def test_constant_dynamics_is_a_translate():
    f = ct.QuadDynamics(np.array([0.3, -0.2, 1.0]), np.zeros((3, 3)))
    xc, xr = np.array([1.0, 0.0, -1.0]), np.array([0.1, 0.2, 0.05])
    pts, segs, ok = ct.flowpipe(f, xc, xr, 0.1, 5)
    assert ok
    for i in range(6):
        np.testing.assert_allclose(pts[i, :, 0], xc + 0.1 * i * f.a - xr, atol=1e-7)
        np.testing.assert_allclose(pts[i, :, 1], xc + 0.1 * i * f.a + xr, atol=1e-7)


def test_linear_dynamics_taylor_polynomial_and_exact_image():
    F = np.array([[-0.5, 1.0], [-1.0, -0.5]])
    f = ct.QuadDynamics(np.zeros(2), F)
    xc, xr, h = np.array([1.0, 0.5]), np.array([0.1, 0.05]), 0.05
    S = np.diag(xr)
    X, ok = ct.picard_step(f, xc, S, np.zeros(2), np.zeros(2), h)
    assert ok
    np.testing.assert_allclose(X.l, F @ xc, rtol=1e-14)
    np.testing.assert_allclose(X.w, 0.5 * F @ F @ xc, rtol=1e-14)
    np.testing.assert_allclose(X.M, F @ S, rtol=1e-14)
    np.testing.assert_allclose(X.L, S, rtol=1e-14)
    pts, _, ok = ct.flowpipe(f, xc, xr, h, 20)
    assert ok
    for i in range(21):
        E = expm(F * h * i)
        lo, hi = E @ xc - np.abs(E) @ xr, E @ xc + np.abs(E) @ xr
        assert np.all(pts[i, :, 0] <= lo + 1e-12) and np.all(pts[i, :, 1] >= hi - 1e-12), i
        if i == 1:
            assert np.all((pts[1, :, 1] - pts[1, :, 0]) <= (hi - lo) * (1 + 10 * h * h))


def test_riccati_exact_interval():
    Q = np.zeros((1, 1, 1)); Q[0, 0, 0] = -1.0
    f = ct.QuadDynamics(np.zeros(1), np.zeros((1, 1)), Q=Q)
    pts, _, ok = ct.flowpipe(f, np.array([1.0]), np.array([0.1]), 0.05, 20)
    assert ok
    for i in range(21):
        t = 0.05 * i
        lo, hi = 0.9 / (1 + 0.9 * t), 1.1 / (1 + 1.1 * t)
        assert pts[i, 0, 0] <= lo + 1e-12 and pts[i, 0, 1] >= hi - 1e-12
        assert (pts[i, 0, 1] - pts[i, 0, 0]) <= 2.0 * (hi - lo)


def _simulate(f, x0, T, t_eval, u=None):
    sol = solve_ivp(lambda t, x: f(x, u), (0, T), x0, t_eval=t_eval, rtol=1e-11, atol=1e-13)
    return sol.y.T


def test_lotka_volterra_sampled_trajectories_inside():
    f = _lv()
    xc, xr, h, N = np.array([2.0, 1.0]), np.array([0.05, 0.05]), 0.02, 50
    pts, segs, ok = ct.flowpipe(f, xc, xr, h, N)
    assert ok
    rng = np.random.default_rng(0)
    X0 = exact.sample_points(rng, xc, xr, 60, corners=True)
    fine = np.linspace(0, h * N, 4 * N + 1)
    for x0 in X0:
        tr = _simulate(f, x0, h * N, fine)
        for q, x in enumerate(tr):
            i = q // 4
            if q % 4 == 0:
                assert np.all(x >= pts[i, :, 0] - 1e-10) and np.all(x <= pts[i, :, 1] + 1e-10), (q, x)
            seg = segs[min(i, N - 1)]
            assert np.all(x >= seg[:, 0] - 1e-10) and np.all(x <= seg[:, 1] + 1e-10), (q, x)


def test_flowpipe_model_contains_trajectories():
    """Inside one step the TM itself (not only its box) encloses the solution: for a
    sampled y the trajectory at sampled s lies in p(y, s) + J."""
    f = _lv()
    c, xr, h = np.array([2.0, 1.0]), np.array([0.05, 0.05]), 0.05
    S = np.diag(xr)
    X, ok = ct.picard_step(f, c, S, np.zeros(2), np.zeros(2), h)
    assert ok
    rng = np.random.default_rng(1)
    for _ in range(40):
        y = rng.uniform(-1, 1, 2)
        ss = np.linspace(0, h, 6)
        tr = _simulate(f, c + S @ y, h, ss)
        for s, x in zip(ss, tr):
            p = X.c + X.L @ y + X.l * s + s * (X.M @ y) + X.w * s * s
            assert np.all(x >= p + X.lo - 1e-12) and np.all(x <= p + X.hi + 1e-12)


def _ct_plant(rng, n=4, n_u=2):
    F = rng.normal(0, 0.5, (n, n)) - 1.0 * np.eye(n)
    G = rng.normal(0, 0.5, (n, n_u))
    Q = rng.normal(0, 0.1, (n, n, n))
    return ct.QuadDynamics(rng.normal(0, 0.1, n), F, G, Q)


def test_closed_loop_constant_controller_is_open_loop():
    rng = np.random.default_rng(3)
    f = _ct_plant(rng)
    net = make_network(rng, [4, 16, 16, 2], np.float64)
    net.Ws[-1] = np.zeros_like(net.Ws[-1])           # u = b_L for every state
    xc, xr = rng.uniform(-0.5, 0.5, 4), np.full(4, 0.05)
    pts, segs, ok = ct.closed_loop(f, net, xc, xr, 0.02, 5, 3)
    assert ok
    fc = ct.QuadDynamics(f.a + f.G @ net.bs[-1], f.F, None, f.Q)
    pts2, segs2, ok2 = ct.flowpipe(fc, xc, xr, 0.02, 15)
    np.testing.assert_allclose(pts, pts2, rtol=1e-12, atol=1e-12)


def test_closed_loop_sampled_zero_order_hold_inside():
    rng = np.random.default_rng(4)
    f = _ct_plant(rng)
    net = make_network(rng, [4, 16, 16, 2], np.float64)
    xc, xr, h, K, N = rng.uniform(-0.5, 0.5, 4), np.full(4, 0.05), 0.02, 5, 4
    pts, segs, ok = ct.closed_loop(f, net, xc, xr, h, K, N)
    assert ok
    X0 = exact.sample_points(rng, xc, xr, 40, corners=True)
    for x0 in X0:
        x = x0.copy()
        for i in range(N):
            y, _ = exact.forward(net, x[None, :])
            u = y[0]
            tr = _simulate(f, x, h * K, np.linspace(0, h * K, K + 1), u=u)
            for j in range(K + 1):
                b = pts[i * K + j]
                assert np.all(tr[j] >= b[:, 0] - 1e-10) and np.all(tr[j] <= b[:, 1] + 1e-10)
            x = tr[-1]
