"""Pins of the reference gradient of the reach-tube volume (``oracle/tm_grad.py``).

What pins it: its forward pass equals the independent numpy reach of ``oracle/tm.py``;
its gradient equals central finite differences of that numpy reach (actions, box centre
and radius, entries of A, B, every weight matrix and bias vector), where the one-sided
slopes agree (no kink inside the difference); and closed forms of the volume of linear
loops: with B = 0 the tube is P_t = A_x^t diag(r), so dV/dr_z = 2 sum_t sum_j |A_x^t|_jz
and V does not depend on the actions, the centre or the network; with every neuron
stably active the loop is affine, x' = C x + o, so dV/dr_z = 2 sum_t sum_j |C^t|_jz and
V does not depend on the actions or the centre.
"""
import numpy as np
import pytest

from oracle import tm, tm_grad
from paper_2605_25346_amd.workloads import config_workload, make_network

torch = pytest.importorskip("torch")


def _V(net, xc, xr, H, u):
    boxes, _ = tm.reach_dt(net, xc, xr, H, u)
    return tm.tube_volume(boxes)


def _fd_check(f, x0, g, idx, rel=2e-5, h=1e-6):
    checked = 0
    for i in idx:
        x = x0.copy()
        step = h * max(1.0, abs(x0.flat[i]))
        x.flat[i] = x0.flat[i] + step; fp = f(x)
        x.flat[i] = x0.flat[i] - step; fm = f(x)
        f0 = f(x0)
        right, left = (fp - f0) / step, (f0 - fm) / step
        if abs(right - left) > 1e-4 * max(1.0, abs(right)):
            continue       # a kink inside the difference: the one-sided slopes disagree
        fd = (fp - fm) / (2 * step)
        assert abs(fd - g.flat[i]) <= rel * max(1.0, abs(fd)), (i, fd, g.flat[i])
        checked += 1
    return checked


@pytest.mark.parametrize("cfg,H", [(6, 4), (4, 3)])
def test_forward_equals_numpy_reach(cfg, H):
    wl = config_workload(cfg, n_sub=2)
    net = wl.nets[0]
    for s in range(2):
        u = wl.meta["u"][s][:H] if "u" in wl.meta else None
        ob, _ = tm.reach_dt(net, wl.batch.x_center[s], wl.batch.x_radius[s], H, u)
        g = tm_grad.volume_gradient(net, wl.batch.x_center[s], wl.batch.x_radius[s], H, u)
        np.testing.assert_allclose(g["boxes"], ob, rtol=1e-13, atol=1e-13)
        assert abs(g["V"] - tm.tube_volume(ob)) <= 1e-12 * max(1, g["V"])


def test_gradient_against_finite_differences_exogenous():
    """The candidate-action network (state 8, actions 4), 4 steps."""
    wl = config_workload(6, n_sub=1)
    net = wl.nets[0]
    n = net.A.shape[0]
    H = 4
    xc, xr, u = wl.batch.x_center[0][:n].copy(), wl.batch.x_radius[0][:n].copy(), wl.meta["u"][0][:H].copy()
    g = tm_grad.volume_gradient(net, xc, xr, H, u)
    rng = np.random.default_rng(0)
    n_ok = 0
    n_ok += _fd_check(lambda x: _V(net, xc, xr, H, x), u, g["du"], range(u.size))
    n_ok += _fd_check(lambda x: _V(net, x, xr, H, u), xc, g["dxc"], range(n))
    n_ok += _fd_check(lambda x: _V(net, xc, x, H, u), xr, g["dxr"], range(n))
    for k in range(net.n_layers):
        W0 = net.Ws[k]

        def fW(x, k=k):
            Ws = list(net.Ws); Ws[k] = x
            return _V(type(net)(Ws, net.bs, net.A, net.B), xc, xr, H, u)
        n_ok += _fd_check(fW, W0, g["dW"][k], rng.choice(W0.size, 12, replace=False))

        def fb(x, k=k):
            bs = list(net.bs); bs[k] = x
            return _V(type(net)(net.Ws, bs, net.A, net.B), xc, xr, H, u)
        n_ok += _fd_check(fb, net.bs[k], g["db"][k], rng.choice(net.bs[k].size, min(6, net.bs[k].size), replace=False))
    n_ok += _fd_check(lambda x: _V(type(net)(net.Ws, net.bs, x, net.B), xc, xr, H, u), net.A, g["dA"],
                      rng.choice(net.A.size, 12, replace=False))
    n_ok += _fd_check(lambda x: _V(type(net)(net.Ws, net.bs, net.A, x), xc, xr, H, u), net.B, g["dB"],
                      rng.choice(net.B.size, 12, replace=False))
    assert n_ok >= 90, n_ok


def test_gradient_against_finite_differences_controller():
    """A 32-wide controller loop without exogenous inputs, 3 steps."""
    rng = np.random.default_rng(7)
    net = make_network(rng, [4, 32, 32, 2], np.float64)
    net.A = 0.9 * np.linalg.qr(rng.normal(size=(4, 4)))[0]
    net.B = rng.normal(0, 0.3, (4, 2))
    xc, xr = rng.uniform(-1, 1, 4), np.full(4, 0.1)
    H = 3
    g = tm_grad.volume_gradient(net, xc, xr, H)
    n_ok = _fd_check(lambda x: _V(net, x, xr, H, None), xc, g["dxc"], range(4))
    n_ok += _fd_check(lambda x: _V(net, xc, x, H, None), xr, g["dxr"], range(4))
    for k in range(net.n_layers):
        def fW(x, k=k):
            Ws = list(net.Ws); Ws[k] = x
            return _V(type(net)(Ws, net.bs, net.A, net.B), xc, xr, H, None)
        n_ok += _fd_check(fW, net.Ws[k], g["dW"][k], rng.choice(net.Ws[k].size, 10, replace=False))
    assert n_ok >= 30, n_ok


@pytest.mark.parametrize("m", [0, 3])
def test_zero_B_closed_form(m):
    rng = np.random.default_rng(30 + m)
    n = 4
    net = make_network(rng, [n + m, 16, 16, 2], np.float64)
    net.A = rng.normal(0, 0.5, (n, n + m)); net.B = np.zeros((n, 2))
    xc, xr = rng.uniform(-1, 1, n), rng.uniform(0.01, 0.1, n)
    u = rng.uniform(-1, 1, (5, m)) if m else None
    g = tm_grad.volume_gradient(net, xc, xr, 5, u)
    Ax = net.A[:, :n]
    want, At = np.zeros(n), np.eye(n)
    for _ in range(5):
        At = Ax @ At
        want += 2 * np.abs(At).sum(axis=0)
    np.testing.assert_allclose(g["dxr"], want, rtol=1e-12)
    assert np.all(g["dxc"] == 0) and all(np.all(d == 0) for d in g["dW"])
    if m:
        assert np.all(g["du"] == 0)


def test_all_active_affine_closed_form():
    rng = np.random.default_rng(4)
    n, m = 3, 2
    net = make_network(rng, [n + m, 8, 8, 2], np.float64)
    net.bs[0] += 30.0; net.bs[1] += 100.0
    net.A = rng.normal(0, 0.3, (n, n + m)); net.B = rng.normal(0, 0.01, (n, 2))
    Mv = net.Ws[2] @ net.Ws[1] @ net.Ws[0]
    Cm = net.A[:, :n] + net.B @ Mv[:, :n]
    xc, xr = rng.uniform(-1, 1, n), np.full(n, 0.02)
    u = rng.uniform(-1, 1, (5, m))
    g = tm_grad.volume_gradient(net, xc, xr, 5, u)
    want, Ct = np.zeros(n), np.eye(n)
    for _ in range(5):
        Ct = Cm @ Ct
        want += 2 * np.abs(Ct).sum(axis=0)
    np.testing.assert_allclose(g["dxr"], want, rtol=1e-10)
    np.testing.assert_allclose(g["du"], 0.0, atol=1e-12)
    np.testing.assert_allclose(g["dxc"], 0.0, atol=1e-12)
