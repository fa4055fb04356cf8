"""Parity of dr_reach_dt_grad (the gradient of the reach-tube volume through the
stepwise reach) with the autograd oracle ``oracle/tm_grad.py``, through the C-ABI.

J = sum_s g_V[s] V_s with g_V = 1 / (S (1 + V_s)), the gradient of the paper's
L_reach = mean log(1 + V), w.r.t. the actions, the box centre and radius, A, B and every
weight matrix and bias vector.  Tolerances, relative to max(1e-3, max |reference|) per
gradient: FP64 chains without margins 1e-8, with margins 1e-7 (the margins move the
bounds by ~1e-13 relative and are constants of the gradient); FP32 chains without
margins 2e-4 (FP32 forward and reverse chains).
"""
import numpy as np
import pytest

from oracle import tm, tm_grad
from paper_2605_25346_amd.workloads import config_workload, make_workload
from tests.gpu_helpers import require_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {("f64", False): 1e-8, ("f64", True): 1e-7, ("f32", False): 2e-4}


def _reference(wl, S, H, u):
    net = wl.nets[0]
    n = net.A.shape[0]
    refs = [tm_grad.volume_gradient(net, wl.batch.x_center[s][:n], wl.batch.x_radius[s][:n], H,
                                    None if u is None else u[s][:H]) for s in range(S)]
    V = np.array([r["V"] for r in refs])
    gV = 1.0 / (S * (1.0 + V))
    out = dict(V=V, gV=gV, dxc=np.array([gV[s] * refs[s]["dxc"] for s in range(S)]),
               dxr=np.array([gV[s] * refs[s]["dxr"] for s in range(S)]),
               dA=sum(gV[s] * refs[s]["dA"] for s in range(S)), dB=sum(gV[s] * refs[s]["dB"] for s in range(S)))
    L = len(wl.nets[0].Ws)
    for k in range(L):
        out[f"dW{k + 1}"] = sum(gV[s] * refs[s]["dW"][k] for s in range(S))
        out[f"db{k + 1}"] = sum(gV[s] * refs[s]["db"][k] for s in range(S))
    if u is not None:
        out["du"] = np.array([gV[s] * refs[s]["du"] for s in range(S)])
    return out


def _check(tag, wl, S, H, u, precisions=(("f64", False), ("f64", True), ("f32", False))):
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    ref = _reference(wl, S, H, u)
    for precision, margins in precisions:
        if precision == "f32" and not all(np.array_equal(W, W.astype(np.float32)) for W in wl.nets[0].Ws + wl.nets[0].bs):
            continue
        ctx = BoundContext(wl.nets, precision=precision, max_sub=S, max_splits=0, margins=margins)
        boxes, st, g = ctx.dr_reach_dt_grad(DeviceBatch(wl.batch), H, ref["gV"], u=None if u is None else u[:, :H])
        torch.cuda.synchronize()
        assert np.all(st.cpu().numpy() == 0)
        b = boxes.cpu().numpy()
        V = (b[:, 1:, :, 1] - b[:, 1:, :, 0]).sum(axis=(1, 2))
        assert np.all(np.abs(V - ref["V"]) <= 1e-4 * np.maximum(1, ref["V"])), (V, ref["V"])
        tol = TOL[(precision, margins)]
        L = len(wl.nets[0].Ws)
        keys = ["dxc", "dxr", "dA", "dB", "du"] + [f"dW{k + 1}" for k in range(L)] + [f"db{k + 1}" for k in range(L)]
        for key in keys:
            if key not in ref:
                continue
            if key.startswith("dW") or key.startswith("db"):
                got = g[key[:2]][int(key[2:]) - 1].cpu().numpy()
            else:
                got = g[key].cpu().numpy()
            want = ref[key]
            got = got.reshape(want.shape)
            scale = max(1e-3, float(np.abs(want).max()))
            err = float(np.abs(got - want).max()) / scale
            print(f"[reach grad {tag} {precision} margins={margins}] {key}: max rel err {err:.2e} (scale {scale:.2e})",
                  flush=True)
            assert err <= tol, (key, err)
        ctx.close()


def test_reach_grad_candidate_dynamics():
    """The 96-wide dynamics network with actions (8 + 4 inputs), 4 boxes x 4 steps."""
    require_gpu()
    wl = config_workload(6, n_sub=4)
    _check("mpc 8+4-96x3-8", wl, 4, 4, wl.meta["u"])


def test_reach_grad_full_size():
    """The benchmarked launch: 128 boxes x 10 steps of the 96-wide dynamics network with
    actions (one workgroup per box, the weight-gradient accumulators in LDS), every
    gradient against the oracle over all 128 boxes."""
    require_gpu()
    wl = config_workload(6, n_sub=128)
    _check("mpc 8+4-96x3-8 S128 H10", wl, 128, wl.horizon, wl.meta["u"], precisions=(("f64", True), ("f32", False)))


def test_reach_grad_controller_loops():
    """Closed-loop controllers: a 64-wide one whose output matters and the 256-wide one."""
    require_gpu()
    wl = make_workload("grad64", 91, [[6, 64, 64, 3]], 3, closed_loop=True, radius=0.05, horizon=4,
                       shared_slope=True, A_mode="signed_perm", rho=0.9, b_var=0.05)
    _check("cl 6-64-64-3", wl, 3, 4, None)
    wl = config_workload(4, n_sub=2)
    _check("cl 12-256x3-4", wl, 2, 3, None, precisions=(("f64", False), ("f32", False)))


def test_reach_grad_edge_cases():
    """An empty batch, and horizon 0 (V = 0: zero gradients)."""
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    require_gpu()
    wl = config_workload(6, n_sub=2)
    ctx = BoundContext(wl.nets, precision="f64", max_sub=2, max_splits=0)
    boxes, st, g = ctx.dr_reach_dt_grad(DeviceBatch(wl.batch), 0, np.ones(2), u=wl.meta["u"][:, :0])
    torch.cuda.synchronize()
    for k in ("dxc", "dxr", "dA", "dB"):
        assert np.all(g[k].cpu().numpy() == 0), k
    assert all(np.all(t.cpu().numpy() == 0) for t in g["dW"] + g["db"])
    ctx.close()


def test_reach_volume_autograd_training_and_refinement():
    """ReachVolume: autograd of mean log(1 + V) equals the oracle's gradient; five
    normalised gradient steps on the weights lower the loss (the certified-training
    signal), and five on the actions of one candidate lower its tube volume (the
    top-candidate refinement)."""
    from paper_2605_25346_amd.api import BoundContext, ReachVolume
    require_gpu()
    wl = config_workload(6, n_sub=4)
    net = wl.nets[0]
    S, H = 4, 4
    ctx = BoundContext(wl.nets, precision="f64", max_sub=S, max_splits=0, margins=False)
    dev = ctx.device
    Ws = [torch.tensor(W, dtype=torch.float64, device=dev, requires_grad=True) for W in net.Ws]
    bs = [torch.tensor(b, dtype=torch.float64, device=dev, requires_grad=True) for b in net.bs]
    xc = torch.tensor(wl.batch.x_center, device=dev, requires_grad=True)
    xr = torch.tensor(wl.batch.x_radius, device=dev, requires_grad=True)
    u = torch.tensor(wl.meta["u"][:, :H], device=dev, requires_grad=True)
    V = ReachVolume.apply(ctx, xc, xr, u, H, *Ws, *bs)
    loss = torch.log1p(V).mean()
    loss.backward()
    ref = _reference(wl, S, H, wl.meta["u"])
    n = net.A.shape[0]
    np.testing.assert_allclose(xr.grad.cpu().numpy()[:, :n], ref["dxr"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(u.grad.cpu().numpy(), ref["du"], rtol=1e-9, atol=1e-12)
    for k in range(net.n_layers):
        np.testing.assert_allclose(Ws[k].grad.cpu().numpy(), ref[f"dW{k + 1}"], rtol=1e-8, atol=1e-12)
    # training: normalised steps on the weights lower mean log(1 + V)
    losses = [float(loss)]
    for _ in range(5):
        with torch.no_grad():
            gn = torch.sqrt(sum((p.grad ** 2).sum() for p in Ws + bs))
            for p in Ws + bs:
                p -= 0.02 * p.grad / gn
                p.grad = None
        V = ReachVolume.apply(ctx, xc.detach(), xr.detach(), u.detach(), H, *Ws, *bs)
        loss = torch.log1p(V).mean()
        loss.backward()
        losses.append(float(loss))
    print("[reach volume training] mean log(1+V):", " ".join(f"{v:.4f}" for v in losses), flush=True)
    assert losses[-1] < losses[0]
    # refinement of one candidate's actions (projected to the action box [-1, 1])
    Ws0 = [torch.tensor(W, dtype=torch.float64, device=dev) for W in net.Ws]
    bs0 = [torch.tensor(b, dtype=torch.float64, device=dev) for b in net.bs]
    uc = torch.tensor(wl.meta["u"][:1, :H], device=dev, requires_grad=True)
    vols = []
    for _ in range(6):
        V = ReachVolume.apply(ctx, xc.detach()[:1], xr.detach()[:1], uc, H, *Ws0, *bs0)
        vols.append(float(V[0]))
        V.sum().backward()
        with torch.no_grad():
            uc -= 0.05 * uc.grad / uc.grad.abs().max()
            uc.clamp_(-1.0, 1.0)
            uc.grad = None
    print("[candidate refinement] V:", " ".join(f"{v:.4f}" for v in vols), flush=True)
    assert vols[-1] < vols[0]
    ctx.close()
