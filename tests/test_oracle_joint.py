"""Pins of the oracle of CROWN through the unrolled closed loop (``oracle/joint.py``).

What pins it: two small systems worked by hand (rational arithmetic, both adaptive
lower slopes, intermediate rows at a later step that are tighter than interval
propagation from the state box), closed forms of linear loops (B = 0: matrix powers,
with and without exogenous inputs; every neuron stably active: an affine loop), the
exact trajectory of a point initial set, dense sampled rollouts, and agreement of the
first step with plain closed-loop CROWN.
"""
import numpy as np
import pytest

from oracle import crown, exact, joint
from paper_2605_25346_amd.workloads import Network, config_workload, make_network


def net_from(Ws, bs, A, B):
    return Network([np.asarray(W, float) for W in Ws], [np.asarray(b, float) for b in bs],
                   np.asarray(A, float), np.asarray(B, float))


@pytest.mark.parametrize("lo,hi", [(-1.0, 2.0), (-2.0, 1.0)])
def test_hand_case_one_dimensional(lo, hi):
    """x' = -x + 2 relu(x).  For x_0 in [-1, 2] (adaptive slope 1) and in [-2, 1]
    (slope 0 at step 0, the chord s = 1/3, t = 2/3) the bounds worked by hand are
    x_1, x_2 in [-1, 2]: the lower row of x_2 goes back with the coefficient 1 on x_1
    and then -1 on x_0; the upper row takes the chord of step 1 (s = 2/3, t = 2/3 from
    z_1 in [-1, 2]) and reaches x_0 with the coefficient 1/9 or -1/9 and the offset
    -16/9, i.e. an upper bound of 2."""
    net = net_from([[[1.0]], [[1.0]]], [[0.0], [0.0]], [[-1.0]], [[2.0]])
    boxes, info = joint.reach_joint(net, np.array([(lo + hi) / 2]), np.array([(hi - lo) / 2]), 2)
    np.testing.assert_allclose(boxes[1:, 0, 0], [-1.0, -1.0], atol=1e-14)
    np.testing.assert_allclose(boxes[1:, 0, 1], [2.0, 2.0], atol=1e-14)
    l1, u1 = info["bounds"][1][0]
    np.testing.assert_allclose([l1[0], u1[0]], [-1.0, 2.0], atol=1e-14)


def test_hand_case_intermediate_rows_of_a_later_step():
    """x = (a, b) in [-1, 1]^2, z = x_1 + x_2 + 3/2, y = relu(z),
    x' = [[1, 1], [1, -1]] x + [0, 1]^T y.  By hand: z_0 in [-1/2, 7/2] (s = 7/8,
    t = 7/16, slope 1); x_1 in [-2, 2] x [-1/2, 15/4].  At step 1 interval propagation
    from that box gives z_1 in [-1, 29/4] but the rows carried back to x_0 give
    [-1, 7] (coefficients (3, 1) with offset 3 and (-23/8, -7/8) with offset -13/4),
    so the chord of step 1 is s = t = 7/8 and x_2 in [-5/2, 11/2] x [-5/2, 11/2]."""
    net = net_from([[[1.0, 1.0]], [[1.0]]], [[1.5], [0.0]], [[1.0, 1.0], [1.0, -1.0]], [[0.0], [1.0]])
    boxes, info = joint.reach_joint(net, np.zeros(2), np.ones(2), 2)
    np.testing.assert_allclose(boxes[1], [[-2.0, 2.0], [-0.5, 3.75]], atol=1e-14)
    l1, u1 = info["bounds"][1][0]
    np.testing.assert_allclose([l1[0], u1[0]], [-1.0, 7.0], atol=1e-14)
    np.testing.assert_allclose(boxes[2], [[-2.5, 5.5], [-2.5, 5.5]], atol=1e-14)
    assert info["rows"][1][0] == 2 and info["rows"][0][0] == 0


@pytest.mark.parametrize("m", [0, 3])
def test_zero_B_matrix_powers(m):
    """B = 0: x_{t+1} = A_x x_t + A_u u_t exactly, so X_t = c_t -+ |A_x^t| r with
    c_t = A_x c_{t-1} + A_u u_{t-1}; intervalising each step would give |A_x|^t r."""
    rng = np.random.default_rng(11 + m)
    n = 4
    net = make_network(rng, [n + m, 16, 16, 2], np.float64)
    net.A = rng.normal(0, 0.5, (n, n + m)); net.B = np.zeros((n, 2))
    xc = rng.uniform(-1, 1, n); xr = np.full(n, 0.05)
    u = rng.uniform(-1, 1, (5, m)) if m else None
    boxes, _ = joint.reach_joint(net, xc, xr, 5, u)
    Ax, Au = net.A[:, :n], net.A[:, n:]
    c, P = xc.copy(), np.eye(n)
    for t in range(6):
        np.testing.assert_allclose(boxes[t, :, 0], c - np.abs(P) @ xr, atol=1e-12)
        np.testing.assert_allclose(boxes[t, :, 1], c + np.abs(P) @ xr, atol=1e-12)
        if t < 5:
            c = Ax @ c + (Au @ u[t] if m else 0.0)
            P = Ax @ P


def test_all_active_affine_loop():
    """Every neuron stably active: x' = (A + B M) x + B m is affine, and CROWN through
    the unrolled loop is exact: X_t = C^t xc + o_t -+ |C^t| r."""
    rng = np.random.default_rng(4)
    net = make_network(rng, [3, 8, 8, 2], np.float64)
    net.bs[0] += 30.0; net.bs[1] += 100.0
    net.A = rng.normal(0, 0.3, (3, 3)); net.B = rng.normal(0, 0.01, (3, 2))
    M = net.Ws[2] @ net.Ws[1] @ net.Ws[0]
    mm = net.Ws[2] @ (net.Ws[1] @ net.bs[0] + net.bs[1]) + net.bs[2]
    Cm = net.A + net.B @ M; o = net.B @ mm
    xc = rng.uniform(-1, 1, 3); xr = np.full(3, 0.02)
    boxes, info = joint.reach_joint(net, xc, xr, 5)
    for bounds in info["bounds"]:
        assert all(np.all(l > 0) for l, _ in bounds)
    Ct = np.eye(3); ot = np.zeros(3)
    for t in range(6):
        np.testing.assert_allclose(boxes[t, :, 0], Ct @ xc + ot - np.abs(Ct) @ xr, rtol=1e-10, atol=1e-9)
        np.testing.assert_allclose(boxes[t, :, 1], Ct @ xc + ot + np.abs(Ct) @ xr, rtol=1e-10, atol=1e-9)
        ot = Cm @ ot + o; Ct = Cm @ Ct


def test_zero_radius_is_the_trajectory():
    """A point initial set gives degenerate boxes on the simulated trajectory."""
    wl = config_workload(6, n_sub=2)
    net = wl.nets[0]
    n = net.A.shape[0]
    H = 4
    for s in range(2):
        xc = wl.batch.x_center[s][:n]
        u = wl.meta["u"][s][:H]
        boxes, _ = joint.reach_joint(net, xc, np.zeros(n), H, u)
        x = xc.copy()
        for t in range(H + 1):
            np.testing.assert_allclose(boxes[t, :, 0], x, rtol=1e-11, atol=1e-11)
            np.testing.assert_allclose(boxes[t, :, 1], x, rtol=1e-11, atol=1e-11)
            if t < H:
                v = np.concatenate([x, u[t]])
                y, _ = exact.forward(net, v[None, :])
                x = net.A @ v + net.B @ y[0]


def _rollouts_inside(net, xc, xr, u, boxes, H, seed):
    n = net.A.shape[0]
    rng = np.random.default_rng(seed)
    X = exact.sample_points(rng, xc, xr, 1000, corners=True)
    for t in range(H + 1):
        assert np.all(X >= boxes[t, :, 0] - 1e-12) and np.all(X <= boxes[t, :, 1] + 1e-12), t
        if t < H:
            V = np.hstack([X, np.repeat(u[t][None, :], X.shape[0], axis=0)]) if u is not None else X
            y, _ = exact.forward(net, V)
            X = V @ net.A.T + y @ net.B.T
        assert X.shape[1] == n


def test_soundness_rollouts_exogenous():
    wl = config_workload(6, n_sub=2)
    net = wl.nets[0]
    n = net.A.shape[0]
    H = 4
    for s in range(2):
        xc, xr, u = wl.batch.x_center[s][:n], wl.batch.x_radius[s][:n], wl.meta["u"][s][:H]
        boxes, _ = joint.reach_joint(net, xc, xr, H, u)
        _rollouts_inside(net, xc, xr, u, boxes, H, s)


def test_soundness_rollouts_unstable_controller():
    """A small controller loop with many unstable neurons at every step."""
    rng = np.random.default_rng(21)
    net = make_network(rng, [3, 16, 16, 2], np.float64)
    net.A = 0.9 * np.linalg.qr(rng.normal(size=(3, 3)))[0]
    net.B = rng.normal(0, 0.3, (3, 2))
    xc = rng.uniform(-1, 1, 3); xr = np.full(3, 0.3)
    boxes, info = joint.reach_joint(net, xc, xr, 5)
    assert sum(r[0] + r[1] for r in info["rows"][1:]) > 0
    _rollouts_inside(net, xc, xr, None, boxes, 5, 0)


def test_first_step_is_closed_loop_crown():
    """Horizon 1 is plain CROWN of the closed loop (state rows on x')."""
    wl = config_workload(1, n_sub=3)
    net = wl.nets[0]
    for s in range(3):
        xc, xr = wl.batch.x_center[s], wl.batch.x_radius[s]
        boxes, info = joint.reach_joint(net, xc, xr, 1)
        ref = crown.crown(net, xc, xr)
        np.testing.assert_allclose(boxes[1, :, 0], ref["lb"], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(boxes[1, :, 1], ref["ub"], rtol=1e-12, atol=1e-12)
        for (l, u), (lr, ur) in zip(info["bounds"][0], ref["bounds"]):
            np.testing.assert_allclose(l, lr, atol=1e-12); np.testing.assert_allclose(u, ur, atol=1e-12)
