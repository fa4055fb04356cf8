"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test names what pins it: closed forms of one-neuron and hand cases, exact
affine ranges, brute force by activation-pattern enumeration + LP, strong LP
duality, finite differences, matrix-power closed forms and dense sampling.
"""
import itertools

import numpy as np
import pytest

from oracle import crown, exact, tm
from paper_2605_25346_amd.workloads import Network, config_workload, make_network

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402


def net_from(Ws, bs, A=None, B=None):
    return Network([np.asarray(W, float) for W in Ws], [np.asarray(b, float) for b in bs],
                   None if A is None else np.asarray(A, float), None if B is None else np.asarray(B, float))


# ---------------------------------------------------------------------------- P1
def test_one_neuron_closed_form():
    """y = relu(x), x in [-1, 2]: adaptive alpha = 1 gives lb = -1 and the chord gives
    ub = 2 (both exact); alpha = 0 gives the exact lb = 0."""
    net = net_from([[[1.0]], [[1.0]]], [[0.0], [0.0]])
    xc, xr = np.array([0.5]), np.array([1.5])
    out = crown.crown(net, xc, xr)
    assert out["lb"][0] == pytest.approx(-1.0, abs=1e-15)
    assert out["ub"][0] == pytest.approx(2.0, abs=1e-15)
    bounds = out["bounds"]
    lb, dal, dbe, _ = crown.evaluate_duals(net, bounds, xc, xr, np.array([[0.0], [1.0]]), np.zeros((2, 0)))
    assert lb[0] == pytest.approx(0.0, abs=1e-15)
    # d lb / d alpha = l = -1 at alpha = 1
    lb1, dal1, _, _ = crown.evaluate_duals(net, bounds, xc, xr, np.array([[1.0], [1.0]]), np.zeros((2, 0)))
    assert dal1[0, 0] == pytest.approx(-1.0, abs=1e-15)


def test_one_neuron_pga_reaches_exact():
    """Projected ascent with lr 0.1 moves alpha from 1 to 0 in at most ~10 steps, where
    the bound is the exact minimum 0."""
    net = net_from([[[1.0]], [[1.0]]], [[0.0], [0.0]])
    xc, xr = np.array([0.5]), np.array([1.5])
    bounds, _, _ = crown.intermediate_bounds(net, xc, xr)
    res = crown.optimize_duals(net, bounds, xc, xr, iters=11, lr=0.1)
    assert res["alpha"][0, 0] == pytest.approx(0.0, abs=1e-12)
    assert res["best"][0] == pytest.approx(0.0, abs=1e-12)
    # monotone along the trajectory: lb_t = -alpha_t
    assert np.all(np.diff(res["traj"][:, 0]) >= -1e-15)


def test_tie_rule_and_split():
    """y = relu(x) - relu(x), x in [-1, 1]: the tie u = -l gives alpha = 0 and lb = -1;
    splitting both neurons active makes the relaxation exact (lb = 0)."""
    net = net_from([[[1.0], [1.0]], [[1.0, -1.0]]], [[0.0, 0.0], [0.0]])
    xc, xr = np.array([0.0]), np.array([1.0])
    out = crown.crown(net, xc, xr)
    assert out["lb"][0] == pytest.approx(-1.0, abs=1e-15)
    out2 = crown.crown(net, xc, xr, splits=[(1, 0, 1), (1, 1, 1)])
    assert out2["lb"][0] == pytest.approx(0.0, abs=1e-15)
    assert out2["ub"][0] == pytest.approx(0.0, abs=1e-15)


# ---------------------------------------------------------------------------- P2
def test_beta_hand_case():
    """y = relu(-x) - relu(x) = -x on x in [-1, 2] with the split x <= 0 and alpha of
    relu(-x) fixed at 1: lb(beta) = 2(beta - 1) for beta < 1 and -(beta - 1) after, so
    beta* = 1 and lb* = 0 (the exact minimum of -x on [-1, 0])."""
    net = net_from([[[-1.0], [1.0]], [[1.0, -1.0]]], [[0.0, 0.0], [0.0]])
    xc, xr = np.array([0.5]), np.array([1.5])
    splits = [(1, 1, -1)]
    bounds, _, st_ = crown.intermediate_bounds(net, xc, xr, splits)
    assert st_ == 0
    al = np.ones((2, 2))
    for beta in [0.0, 0.3, 0.7, 1.0, 1.4, 2.5]:
        lb, _, dbe, _ = crown.evaluate_duals(net, bounds, xc, xr, al, np.full((2, 1), beta), splits)
        expect = 2 * (beta - 1) if beta < 1 else -(beta - 1)
        assert lb[0] == pytest.approx(expect, abs=1e-14)
        if beta < 1:
            assert dbe[0, 0] == pytest.approx(2.0, abs=1e-14)
        elif beta > 1:
            assert dbe[0, 0] == pytest.approx(-1.0, abs=1e-14)
    res = crown.optimize_duals(net, bounds, xc, xr, splits, iters=8, lr=0.1, alpha_init=al, opt_alpha=False)
    # hand trace: beta_t = 0.2 t for t <= 5, lb_t = 2(beta_t - 1)
    assert res["traj"][:6, 0] == pytest.approx([2 * (0.2 * t - 1) for t in range(6)], abs=1e-12)
    assert res["best"][0] == pytest.approx(0.0, abs=1e-12)


# ---------------------------------------------------------------------------- P3 / P4
def test_all_active_network_is_exact():
    """With every neuron stably active the network is affine: CROWN must equal the exact
    range c M xc + c m -+ |c M| r."""
    rng = np.random.default_rng(0)
    net = make_network(rng, [5, 16, 16, 3], np.float64)
    net.bs[0] = net.bs[0] + 50.0
    net.bs[1] = net.bs[1] + 200.0
    xc = rng.uniform(-1, 1, 5); xr = np.full(5, 0.1)
    out = crown.crown(net, xc, xr)
    M = net.Ws[2] @ net.Ws[1] @ net.Ws[0]
    m = net.Ws[2] @ (net.Ws[1] @ net.bs[0] + net.bs[1]) + net.bs[2]
    np.testing.assert_allclose(out["lb"], M @ xc + m - np.abs(M) @ xr, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(out["ub"], M @ xc + m + np.abs(M) @ xr, rtol=1e-13, atol=1e-12)


def test_zero_radius_equals_forward():
    wl = config_workload(2, n_sub=6)
    net = wl.nets[0]
    for s in range(6):
        xc = wl.batch.x_center[s]
        out = crown.crown(net, xc, np.zeros_like(xc))
        y, _ = exact.forward(net, xc[None, :])
        np.testing.assert_allclose(out["lb"], y[0], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(out["ub"], y[0], rtol=1e-12, atol=1e-12)


def test_ibp_is_exact_range_of_one_layer():
    """For one affine layer over a box of h, IBP is the exact range: compare with corners."""
    rng = np.random.default_rng(1)
    W = rng.normal(size=(5, 4)); b = rng.normal(size=5)
    lp = rng.uniform(-1, 0.5, 4); up = lp + rng.uniform(0, 1, 4)
    lo, hi = crown.ibp_next(W, b, lp, up)
    H = np.array(list(itertools.product(*[(max(a, 0), max(c, 0)) for a, c in zip(lp, up)])))
    Z = H @ W.T + b
    np.testing.assert_allclose(lo, Z.min(0), atol=1e-14)
    np.testing.assert_allclose(hi, Z.max(0), atol=1e-14)


# ---------------------------------------------------------------------------- P5
def _tiny_net(seed, widths):
    rng = np.random.default_rng(seed)
    return make_network(rng, widths, np.float64), rng


@settings(max_examples=25, deadline=None)
@given(seed=st.integers(0, 10_000), h1=st.integers(1, 5), h2=st.integers(1, 5), closed=st.booleans())
def test_bruteforce_sandwich(seed, h1, h2, closed):
    """lb_CROWN <= lb_alpha-beta <= exact min <= sampled min (and mirrored for ub)."""
    net, rng = _tiny_net(seed, [2, h1, h2, 2])
    if closed:
        net.A = rng.normal(0, 0.5, (2, 2)); net.B = rng.normal(0, 0.5, (2, 2))
    xc = rng.uniform(-1, 1, 2); xr = rng.uniform(0.05, 0.6, 2)
    # a random feasible split from a sampled point
    x0 = xc + xr * rng.uniform(-1, 1, 2)
    _, zs = exact.forward(net, x0[None, :])
    k = int(rng.integers(1, 3)); j = int(rng.integers(0, (h1, h2)[k - 1]))
    splits = [(k, j, 1 if zs[k - 1][0, j] >= 0 else -1)] if rng.random() < 0.6 else []
    spec = np.eye(2)
    out = crown.crown(net, xc, xr, splits, spec)
    assert out["status"] == 0
    opt = crown.optimize_duals(net, out["bounds"], xc, xr, splits, spec, iters=15, lr=0.1)
    smin, smax = exact.sampled_extrema(net, xc, xr, spec, splits, n=3000, seed=seed)
    for i in range(2):
        emin = exact.exact_min(net, xc, xr, spec[i], splits)
        emax = -exact.exact_min(net, xc, xr, -spec[i], splits)
        assert out["lb"][i] <= opt["lb"][i] + 1e-12
        assert opt["lb"][i] <= emin + 1e-9
        assert emin <= smin[i] + 1e-9
        assert out["ub"][i] >= opt["ub"][i] - 1e-12
        assert opt["ub"][i] >= emax - 1e-9
        assert emax >= smax[i] - 1e-9


# ---------------------------------------------------------------------------- P6
def test_strong_duality_all_split():
    """One hidden layer with every neuron split: the network is affine on the
    subdomain, so the exact minimum is an LP.  LP duality says the bound at the LP's
    optimal multipliers of the split constraints equals the LP optimum, and every
    beta >= 0 gives a bound below it (all PGA iterates)."""
    from scipy.optimize import linprog
    for seed in range(4):
        net, rng = _tiny_net(100 + seed, [3, 6, 1])
        xc = rng.uniform(-1, 1, 3); xr = np.full(3, 0.7)
        x0 = xc + xr * rng.uniform(-1, 1, 3)
        _, zs = exact.forward(net, x0[None, :])
        sig = np.where(zs[0][0] >= 0, 1.0, -1.0)
        splits = [(1, j, int(sig[j])) for j in range(6)]
        c = np.array([[1.0]])
        bounds, _, status = crown.intermediate_bounds(net, xc, xr, splits)
        assert status == 0
        W1, b1, W2, b2 = net.Ws[0], net.bs[0], net.Ws[1], net.bs[1]
        D = (sig > 0).astype(float)
        obj = (W2[0] * D) @ W1
        const = (W2[0] * D) @ b1 + b2[0]
        A_ub = -sig[:, None] * W1           # sigma_j z_j(x) >= 0
        b_ub = sig * b1
        lp = linprog(obj, A_ub=A_ub, b_ub=b_ub, bounds=list(zip(xc - xr, xc + xr)), method="highs")
        assert lp.status == 0
        opt = lp.fun + const
        assert opt == pytest.approx(exact.exact_min(net, xc, xr, c[0], splits), abs=1e-9)
        beta_star = -lp.ineqlin.marginals
        assert np.all(beta_star >= -1e-12)
        R = 2
        al = crown.default_alpha(net, bounds, R)
        lb, _, _, _ = crown.evaluate_duals(net, bounds, xc, xr, al, np.tile(np.maximum(beta_star, 0), (R, 1)), splits, c)
        assert lb[0] == pytest.approx(opt, abs=1e-9)
        res = crown.optimize_duals(net, bounds, xc, xr, splits, c, iters=300, lr=0.02)
        assert np.all(res["traj"][:, 0] <= opt + 1e-9)
        assert res["best"][0] >= res["traj"][0, 0] - 1e-15


# ---------------------------------------------------------------------------- P7
def test_iteration_zero_is_crown():
    wl = config_workload(3, n_sub=3)
    for s in range(3):
        net = wl.nets[0]; xc, xr = wl.batch.x_center[s], wl.batch.x_radius[s]
        sp = wl.batch.splits_of(s)
        out = crown.crown(net, xc, xr, sp)
        res = crown.optimize_duals(net, out["bounds"], xc, xr, sp, iters=0)
        np.testing.assert_array_equal(res["best"][:4], out["lb"])
        np.testing.assert_array_equal(-res["best"][4:], out["ub"])


# ---------------------------------------------------------------------------- P8
def test_gradient_finite_differences():
    """Central differences (h = 1e-6) of the bound w.r.t. alpha and beta match the hand
    adjoint where no branch flips inside +-h."""
    wl = config_workload(3, n_sub=2)
    net = wl.nets[0]
    rng = np.random.default_rng(5)
    for s in range(2):
        xc, xr = wl.batch.x_center[s], wl.batch.x_radius[s]
        sp = wl.batch.splits_of(s)
        bounds, _, status = crown.intermediate_bounds(net, xc, xr, sp)
        assert status == 0
        R, H = 8, sum(net.hidden)
        al = rng.uniform(0, 1, (R, H)); be = rng.uniform(0, 0.5, (R, len(sp)))
        lb, dal, dbe, out0 = crown.evaluate_duals(net, bounds, xc, xr, al, be, sp)
        unst = np.nonzero(np.concatenate([crown.relu_relaxation(*b)[0] == crown.UNSTABLE for b in bounds]))[0]
        h = 1e-6
        checked = 0
        for j in rng.choice(unst, size=min(12, unst.size), replace=False):
            ap = al.copy(); am = al.copy(); ap[:, j] += h; am[:, j] -= h
            lp_, _, _, op = crown.evaluate_duals(net, bounds, xc, xr, ap, be, sp, grad=True)
            lm_, _, _, om = crown.evaluate_duals(net, bounds, xc, xr, am, be, sp, grad=True)
            same = [np.array_equal(np.sign(op["res"]["w"]), np.sign(om["res"]["w"]))]
            same += [np.array_equal(a["g"] >= 0, b["g"] >= 0) for a, b in zip(op["res"]["tape"], om["res"]["tape"])]
            if not all(same):
                continue
            fd = (lp_ - lm_) / (2 * h)
            np.testing.assert_allclose(dal[:, j], fd, rtol=1e-6, atol=1e-8)
            checked += 1
        for i in range(len(sp)):
            bp = be.copy(); bm = be.copy(); bp[:, i] += h; bm[:, i] -= h
            lp_, _, _, _ = crown.evaluate_duals(net, bounds, xc, xr, al, bp, sp, grad=False)
            lm_, _, _, _ = crown.evaluate_duals(net, bounds, xc, xr, al, bm, sp, grad=False)
            np.testing.assert_allclose(dbe[:, i], (lp_ - lm_) / (2 * h), rtol=1e-6, atol=1e-8)
        assert checked > 4


def test_gradient_matches_torch_autograd():
    """An independent differentiation route: the same bound written with torch FP64
    tensors and differentiated by autograd."""
    torch = pytest.importorskip("torch")
    wl = config_workload(2, n_sub=2)
    net = wl.nets[0]
    rng = np.random.default_rng(7)
    for s in range(2):
        xc, xr = wl.batch.x_center[s], wl.batch.x_radius[s]
        sp = wl.batch.splits_of(s)
        bounds, _, _ = crown.intermediate_bounds(net, xc, xr, sp)
        R, H = 6, sum(net.hidden)
        al = rng.uniform(0, 1, (R, H)); be = rng.uniform(0, 0.5, (R, len(sp)))
        lb, dal, dbe, _ = crown.evaluate_duals(net, bounds, xc, xr, al, be, sp)
        # torch: rebuild the bound from relaxation data
        A = torch.tensor(al, requires_grad=True); Bt = torch.tensor(be, requires_grad=True)
        relax = [crown.relu_relaxation(*b) for b in bounds]
        offs = crown.hidden_offsets(net)
        C = torch.tensor(np.vstack([np.eye(3), -np.eye(3)]))
        Ws = [torch.tensor(W) for W in net.Ws]; bs = [torch.tensor(b) for b in net.bs]
        a = C; acc = a @ bs[-1]; g = a @ Ws[-1]
        for k in range(len(net.hidden), 0, -1):
            kind, sl, t, a0 = [torch.tensor(v) for v in relax[k - 1]]
            uns = kind == crown.UNSTABLE
            lo = torch.where(uns, A[:, offs[k - 1]:offs[k]], a0)
            d = torch.where(g >= 0, lo, sl)
            acc = acc + torch.where(uns & (g < 0), g * t, torch.zeros_like(g)).sum(1)
            a = d * g
            for idx, (kk, j, sgn) in enumerate(sp):
                if kk == k:
                    a = a.clone(); a[:, j] = a[:, j] - Bt[:, idx] * sgn
            acc = acc + a @ bs[k - 1]
            g = a @ Ws[k - 1]
        val = acc + g @ torch.tensor(xc) - g.abs() @ torch.tensor(xr)
        np.testing.assert_allclose(val.detach().numpy(), lb, rtol=1e-12, atol=1e-12)
        val.sum().backward()
        unst = np.concatenate([r[0] == crown.UNSTABLE for r in relax])
        np.testing.assert_allclose(A.grad.numpy()[:, unst], dal[:, unst], rtol=1e-10, atol=1e-12)
        if len(sp):
            np.testing.assert_allclose(Bt.grad.numpy(), dbe, rtol=1e-10, atol=1e-12)


# ------------------------------------------------------- parameter gradient (fixed relaxation)
def _perturbed(net, k, i, j, h, bias=False):
    Ws = [W.copy() for W in net.Ws]; bs = [b.copy() for b in net.bs]
    if bias:
        bs[k][i] += h
    else:
        Ws[k][i, j] += h
    return Network(Ws, bs, net.A, net.B)


def _same_branches(op, om):
    same = np.array_equal(np.sign(op["res"]["w"]), np.sign(om["res"]["w"]))
    return same and all(np.array_equal(a["g"] >= 0, b["g"] >= 0) for a, b in zip(op["res"]["tape"], om["res"]["tape"]))


@pytest.mark.parametrize("cfg", [1, 3])
def test_param_gradient_finite_differences(cfg):
    """Central differences (h = 1e-6) of the weighted row bounds w.r.t. weights, biases
    and the box, with the intermediate bounds and alpha, beta held fixed, match the
    hand adjoint (cfg 1: closed loop, the rows enter through B and the skip A)."""
    wl = config_workload(cfg, n_sub=2)
    net = wl.nets[0]
    rng = np.random.default_rng(17)
    q = crown.default_spec(net).shape[0]
    R, H, h = 2 * q, sum(net.hidden), 1e-6
    checked = 0
    for s in range(2):
        xc, xr = wl.batch.x_center[s], wl.batch.x_radius[s]
        sp = wl.batch.splits_of(s)
        bounds, _, status = crown.intermediate_bounds(net, xc, xr, sp)
        assert status == 0
        al = rng.uniform(0, 1, (R, H)); be = rng.uniform(0, 0.5, (R, len(sp)))
        om = rng.normal(size=R)
        pg = crown.param_gradient(net, bounds, xc, xr, al, be, om, sp)
        alpha = crown._split_alpha(net, al); beta = crown._dense_beta(net, be, sp)

        def val(n, c=xc, r=xr):
            o = crown.final_bounds(n, bounds, c, r, alpha=alpha, beta=beta, splits=sp, tape=True)
            return om @ o["rowlb"], o

        for k in range(net.n_layers):
            W = net.Ws[k]
            for _ in range(6):
                i, j = rng.integers(W.shape[0]), rng.integers(W.shape[1])
                vp, op = val(_perturbed(net, k, i, j, h)); vm, omn = val(_perturbed(net, k, i, j, -h))
                if not _same_branches(op, omn):
                    continue
                fd = (vp - vm) / (2 * h)
                assert pg["dW"][k][i, j] == pytest.approx(fd, rel=1e-6, abs=1e-8), (k, i, j)
                checked += 1
            i = rng.integers(W.shape[0])
            vp, _ = val(_perturbed(net, k, i, 0, h, bias=True)); vm, _ = val(_perturbed(net, k, i, 0, -h, bias=True))
            assert pg["db"][k][i] == pytest.approx((vp - vm) / (2 * h), rel=1e-6, abs=1e-8)
        for m in range(len(xc)):
            dc = np.zeros_like(xc); dc[m] = h
            vp, _ = val(net, xc + dc); vm, _ = val(net, xc - dc)
            assert pg["dxc"][m] == pytest.approx((vp - vm) / (2 * h), rel=1e-6, abs=1e-8)
            vp, _ = val(net, xc, xr + dc); vm, _ = val(net, xc, xr - dc)
            assert pg["dxr"][m] == pytest.approx((vp - vm) / (2 * h), rel=1e-6, abs=1e-8)
        np.testing.assert_array_equal(pg["rowlb"], crown.evaluate_duals(net, bounds, xc, xr, al, be, sp, grad=False)[0])
    assert checked >= 6 * net.n_layers


def test_param_gradient_all_active_is_the_full_gradient():
    """On a network whose every neuron is active over the box the bound is the exact
    range of the affine map  M x + m  (M = W_L ... W_1): lb_r = c_r (M xc + m) - |c_r M| xr.
    There the relaxation carries no slope or intercept, so the fixed-relaxation gradient
    is the gradient of the full CROWN bound (intermediate bounds recomputed at every
    perturbation), and d lb_r / d b_1 = c_r W_L ... W_2 in closed form."""
    rng = np.random.default_rng(3)
    widths = [3, 5, 4, 2]
    Ws = [rng.uniform(0.1, 1.0, (widths[k + 1], widths[k])) for k in range(3)]
    bs = [rng.uniform(0.5, 1.0, widths[k + 1]) for k in range(3)]
    net = net_from(Ws, bs)
    xc, xr = np.array([1.0, 2.0, 1.5]), np.array([0.2, 0.1, 0.3])
    out = crown.crown(net, xc, xr)
    assert all(np.all(l > 0) for (l, u) in out["bounds"])
    R, H = 4, sum(net.hidden)
    om = np.array([0.7, -1.3, 0.4, 2.0])
    pg = crown.param_gradient(net, out["bounds"], xc, xr, crown.default_alpha(net, out["bounds"], R),
                              np.zeros((R, 0)), om)
    C = np.vstack([np.eye(2), -np.eye(2)])
    np.testing.assert_allclose(pg["db"][0], om @ (C @ Ws[2] @ Ws[1]), rtol=1e-13)
    M = Ws[2] @ Ws[1] @ Ws[0]
    np.testing.assert_allclose(pg["dxc"], om @ (C @ M), rtol=1e-13)
    np.testing.assert_allclose(pg["dxr"], -(om @ np.abs(C @ M)), rtol=1e-13)
    h = 1e-6

    def full(n):
        o = crown.crown(n, xc, xr)
        return om @ np.concatenate([o["lb"], -o["ub"]])

    for k in range(3):
        for i in range(Ws[k].shape[0]):
            for j in range(Ws[k].shape[1]):
                fd = (full(_perturbed(net, k, i, j, h)) - full(_perturbed(net, k, i, j, -h))) / (2 * h)
                assert pg["dW"][k][i, j] == pytest.approx(fd, rel=1e-6, abs=1e-9)
            fd = (full(_perturbed(net, k, i, 0, h, True)) - full(_perturbed(net, k, i, 0, -h, True))) / (2 * h)
            assert pg["db"][k][i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


# ---------------------------------------------------------------------------- P9
def test_closed_loop_zero_B():
    """x' = A x with B = 0: the bound is the exact range A xc -+ |A| r."""
    wl = config_workload(1, n_sub=4)
    net = wl.nets[0]
    net0 = Network(net.Ws, net.bs, net.A, np.zeros_like(net.B))
    for s in range(4):
        xc, xr = wl.batch.x_center[s], wl.batch.x_radius[s]
        out = crown.crown(net0, xc, xr)
        np.testing.assert_allclose(out["lb"], net.A @ xc - np.abs(net.A) @ xr, atol=1e-13)
        np.testing.assert_allclose(out["ub"], net.A @ xc + np.abs(net.A) @ xr, atol=1e-13)


def test_tm_zero_B_matrix_powers():
    """Stepwise TM reach with B = 0 keeps the exact linear TM: X_t = A^t xc -+ |A^t| r."""
    rng = np.random.default_rng(3)
    net = make_network(rng, [4, 16, 16, 2], np.float64)
    net.A = rng.normal(0, 0.5, (4, 4)); net.B = np.zeros((4, 2))
    xc = rng.uniform(-1, 1, 4); xr = np.full(4, 0.05)
    boxes, _ = tm.reach_dt(net, xc, xr, 6)
    At = np.eye(4)
    for t in range(7):
        np.testing.assert_allclose(boxes[t, :, 0], At @ xc - np.abs(At) @ xr, atol=1e-12)
        np.testing.assert_allclose(boxes[t, :, 1], At @ xc + np.abs(At) @ xr, atol=1e-12)
        At = net.A @ At


def test_tm_all_active_linear_closed_loop():
    """All neurons stably active: the closed loop is x' = (A + B M) x + B m, exactly a
    linear TM, so X_t = C^t xc + o_t -+ |C^t| r."""
    rng = np.random.default_rng(4)
    net = make_network(rng, [3, 8, 8, 2], np.float64)
    net.bs[0] += 30.0; net.bs[1] += 100.0
    net.A = rng.normal(0, 0.3, (3, 3)); net.B = rng.normal(0, 0.01, (3, 2))
    M = net.Ws[2] @ net.Ws[1] @ net.Ws[0]
    m = net.Ws[2] @ (net.Ws[1] @ net.bs[0] + net.bs[1]) + net.bs[2]
    Cm = net.A + net.B @ M; o = net.B @ m
    xc = rng.uniform(-1, 1, 3); xr = np.full(3, 0.02)
    boxes, _ = tm.reach_dt(net, xc, xr, 5)
    Ct = np.eye(3); ot = np.zeros(3)
    for t in range(6):
        np.testing.assert_allclose(boxes[t, :, 0], Ct @ xc + ot - np.abs(Ct) @ xr, rtol=1e-10, atol=1e-9)
        np.testing.assert_allclose(boxes[t, :, 1], Ct @ xc + ot + np.abs(Ct) @ xr, rtol=1e-10, atol=1e-9)
        ot = Cm @ ot + o; Ct = Cm @ Ct


def test_tm_exogenous_zero_B_closed_form():
    """Exogenous inputs with B = 0: x' = A_x x + A_u u_t exactly, so the TM stays
    c_t = A_x c_{t-1} + A_u u_{t-1}, P_t = A_x^t diag(r), I = 0."""
    rng = np.random.default_rng(5)
    n, m = 4, 3
    net = make_network(rng, [n + m, 16, 16, 2], np.float64)
    net.A = rng.normal(0, 0.5, (n, n + m)); net.B = np.zeros((n, 2))
    xc = rng.uniform(-1, 1, n); xr = np.full(n, 0.05)
    u = rng.uniform(-1, 1, (5, m))
    boxes, _ = tm.reach_dt(net, xc, xr, 5, u)
    Ax, Au = net.A[:, :n], net.A[:, n:]
    c, P = xc.copy(), np.diag(xr)
    for t in range(6):
        np.testing.assert_allclose(boxes[t, :, 0], c - np.abs(P).sum(axis=1), atol=1e-12)
        np.testing.assert_allclose(boxes[t, :, 1], c + np.abs(P).sum(axis=1), atol=1e-12)
        if t < 5:
            c, P = Ax @ c + Au @ u[t], Ax @ P


def test_tm_exogenous_zero_radius_is_the_trajectory():
    """A point initial set (and a network with no neuron at a kink) gives degenerate
    boxes on the exact simulated trajectory x_{t+1} = A [x; u] + B f([x; u])."""
    wl = config_workload(6, n_sub=3)
    net = wl.nets[0]
    n = net.A.shape[0]
    for s in range(3):
        xc = wl.batch.x_center[s][:n]
        u = wl.meta["u"][s]
        boxes, _ = tm.reach_dt(net, xc, np.zeros(n), wl.horizon, u)
        x = xc.copy()
        for t in range(wl.horizon + 1):
            np.testing.assert_allclose(boxes[t, :, 0], x, rtol=1e-11, atol=1e-11)
            np.testing.assert_allclose(boxes[t, :, 1], x, rtol=1e-11, atol=1e-11)
            if t < wl.horizon:
                v = np.concatenate([x, u[t]])
                y, _ = exact.forward(net, v[None, :])
                x = net.A @ v + net.B @ y[0]


def test_tm_exogenous_soundness_rollouts():
    """Sampled initial states rolled out under the given action sequence stay inside
    every box."""
    wl = config_workload(6, n_sub=2)
    net = wl.nets[0]
    n = net.A.shape[0]
    for s in range(2):
        xc, xr, u = wl.batch.x_center[s][:n], wl.batch.x_radius[s][:n], wl.meta["u"][s]
        boxes, _ = tm.reach_dt(net, xc, xr, wl.horizon, u)
        rng = np.random.default_rng(s)
        X = exact.sample_points(rng, xc, xr, 500, corners=True)
        for t in range(wl.horizon + 1):
            assert np.all(X >= boxes[t, :, 0] - 1e-12) and np.all(X <= boxes[t, :, 1] + 1e-12)
            if t < wl.horizon:
                V = np.hstack([X, np.repeat(u[t][None, :], X.shape[0], axis=0)])
                y, _ = exact.forward(net, V)
                X = V @ net.A.T + y @ net.B.T


# ---------------------------------------------------------------------------- P10
@pytest.mark.parametrize("cfg", [1, 2, 3, 5])
def test_soundness_sampling(cfg):
    """Sampled outputs (and sampled pre-activations) lie inside every bound."""
    wl = config_workload(cfg, n_sub=3)
    for s in range(3):
        net = wl.nets[int(wl.batch.net_id[s])]
        xc, xr = wl.batch.x_center[s], wl.batch.x_radius[s]
        sp = wl.batch.splits_of(s)
        out = crown.crown(net, xc, xr, sp)
        if out["status"]:
            continue
        spec = crown.default_spec(net)
        smin, smax = exact.sampled_extrema(net, xc, xr, spec, sp, n=4000, seed=s)
        if smin is None:
            continue
        assert np.all(out["lb"] <= smin + 1e-12) and np.all(out["ub"] >= smax - 1e-12)
        rng = np.random.default_rng(s)
        X = exact.sample_points(rng, xc, xr, 2000)
        _, zs = exact.forward(net, X)
        keep = np.ones(X.shape[0], bool)
        for (k, j, sg) in sp:
            keep &= sg * zs[k - 1][:, j] >= 0
        for (l, u), z in zip(out["bounds"], zs):
            assert np.all(z[keep] >= l - 1e-12) and np.all(z[keep] <= u + 1e-12)
        if wl.iters:
            opt = crown.optimize_duals(net, out["bounds"], xc, xr, sp, iters=5, lr=wl.lr)
            assert np.all(opt["lb"] <= smin + 1e-12) and np.all(opt["ub"] >= smax - 1e-12)
            assert np.all(opt["lb"] >= out["lb"] - 1e-12)


def test_tm_soundness_rollouts():
    wl = config_workload(4, n_sub=2)
    net = wl.nets[0]
    for s in range(2):
        xc, xr = wl.batch.x_center[s], wl.batch.x_radius[s]
        boxes, _ = tm.reach_dt(net, xc, xr, 4)
        rng = np.random.default_rng(s)
        X = exact.sample_points(rng, xc, xr, 500, corners=False)
        for t in range(5):
            assert np.all(X >= boxes[t, :, 0] - 1e-12) and np.all(X <= boxes[t, :, 1] + 1e-12)
            y, _ = exact.forward(net, X)
            X = X @ net.A.T + y @ net.B.T


# ---------------------------------------------------------------------------- P12
def test_status_infeasible_and_nonfinite():
    net = net_from([[[1.0], [1.0]], [[1.0, 1.0]]], [[0.0, 0.0], [0.0]])
    xc, xr = np.array([-1.5]), np.array([0.5])     # z in [-2, -1]
    out = crown.crown(net, xc, xr, splits=[(1, 0, 1)])  # z >= 0 is impossible
    assert out["status"] & crown.STATUS_INFEASIBLE
    assert np.isposinf(out["lb"][0]) and np.isneginf(out["ub"][0])
    out2 = crown.crown(net, np.array([np.nan]), xr)
    assert out2["status"] & crown.STATUS_NONFINITE
