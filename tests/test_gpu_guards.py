"""GPU tests of the library's guards on caller input and on its own state.

* Duals outside their feasible sets (alpha > 1, NaN, beta < 0) are projected on read:
  the bound, its gradient and the ascent step are those of the projected point, so the
  bound stays valid (weak duality holds for every alpha in [0, 1] and beta >= 0, the
  reading of the split multipliers in the preamble's notation and of Theorem "CROWN
  linear bounds of NN").
* A CrownBounds backward after a later forward on the same context raises instead of
  differentiating the wrong relaxation.
* A subdomain whose network id is out of range in a several-network context carries
  the BADSPLIT status bit and gets NaN intermediate-bound rows.
"""
import numpy as np
import pytest

from oracle import crown, exact
from paper_2605_25346_amd.workloads import config_workload
from tests.gpu_helpers import near_tie, print_stats, rel_gap, require_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_duals_outside_their_sets_are_projected():
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    require_gpu()
    wl = config_workload(2, n_sub=16)
    net = wl.nets[0]
    S, q = wl.batch.n_sub, 3
    R, H = 2 * q, sum(net.hidden)
    ms = max(int(np.max(np.diff(wl.batch.split_ptr))), 1)
    ctx = BoundContext(wl.nets, precision="f64", max_sub=S, max_splits=ms)
    ctx.dr_bound_init(DeviceBatch(wl.batch))
    al = np.full((S, R, H), 1.5, np.float32)
    al[:, :, ::7] = np.nan
    be = np.full((S, R, ms), -1.0, np.float32)
    alpha = torch.tensor(al, device="cuda")
    beta = torch.tensor(be, device="cuda")
    lb, ub, st, ga, gb = ctx.dr_optimize_duals(0, 0.0, alpha, beta, init_duals=False, grads=True)
    torch.cuda.synchronize()
    lb, ub, st = lb.cpu().numpy(), ub.cpu().numpy(), st.cpu().numpy()
    # the projected point: alpha = 1 (0 where NaN), beta = 0
    al_p = np.where(np.isnan(al), 0.0, np.clip(al, 0.0, 1.0)).astype(np.float64)
    gaps, checked = [], 0
    for s in range(S):
        sp = wl.batch.splits_of(s)
        xc, xr = wl.batch.x_center[s], wl.batch.x_radius[s]
        bounds, _, status = crown.intermediate_bounds(net, xc, xr, sp)
        if status or near_tie(bounds, 1e-9, slope=False):
            continue
        rowlb = crown.evaluate_duals(net, bounds, xc, xr, al_p[s], np.zeros((R, len(sp))), sp, grad=False)[0]
        g = np.concatenate([rel_gap(lb[s], rowlb[:q]), rel_gap(-ub[s], rowlb[q:])])
        assert np.all(g <= 1e-9), (s, g.max())
        gaps.append(g)
        smin, smax = exact.sampled_extrema(net, xc, xr, np.eye(q), sp, n=4000, seed=s)
        if smin is not None:
            assert np.all(lb[s] <= smin) and np.all(ub[s] >= smax), s
        checked += 1
    assert checked >= S // 2
    print_stats("bound at projected duals vs oracle", gaps)
    assert np.all(np.isfinite(ga.cpu().numpy())) and np.all(np.isfinite(gb.cpu().numpy()))
    # an ascent started from the infeasible point keeps its iterates in the sets
    ctx.dr_optimize_duals(3, 0.1, alpha, beta, init_duals=False)
    l, u = ctx.dr_get_bounds()
    torch.cuda.synchronize()
    a2, b2, l, u = alpha.cpu().numpy(), beta.cpu().numpy(), l.cpu().numpy(), u.cpu().numpy()
    for s in range(S):
        if st[s] & 9:
            continue
        uns = (l[s] < 0) & (u[s] > 0)          # the entries the ascent updates (the GPU's own bounds)
        assert np.all((a2[s][:, uns] >= 0) & (a2[s][:, uns] <= 1)), s
        n_sp = len(wl.batch.splits_of(s))
        assert np.all(b2[s][:, :n_sp] >= 0), s
    ctx.close()


def test_crown_bounds_backward_after_a_later_forward_raises():
    from paper_2605_25346_amd.api import BoundContext, CrownBounds, DeviceBatch
    require_gpu()
    wl = config_workload(3, n_sub=24)
    net = wl.nets[0]
    ms = int(np.max(np.diff(wl.batch.split_ptr)))
    ctx = BoundContext(wl.nets, precision="f64", max_sub=24, max_splits=ms)
    params = [torch.tensor(W, dtype=torch.float64, device="cuda", requires_grad=True) for W in net.Ws] + \
             [torch.tensor(b, dtype=torch.float64, device="cuda", requires_grad=True) for b in net.bs]
    first = DeviceBatch(wl.batch.subset(np.arange(8)))
    second = DeviceBatch(wl.batch)                      # larger: the stale backward would index past it
    lb1, ub1 = CrownBounds.apply(ctx, first, *params)
    lb2, ub2 = CrownBounds.apply(ctx, second, *params)
    keep1 = torch.isfinite(lb1).all(dim=1)
    loss = lb1[keep1].sum() + lb2[torch.isfinite(lb2).all(dim=1)].sum()
    with pytest.raises(RuntimeError, match="state changed"):
        loss.backward()
    # the latest forward alone still differentiates
    for p in params:
        p.grad = None
    lb3, ub3 = CrownBounds.apply(ctx, first, *params)
    lb3[torch.isfinite(lb3).all(dim=1)].sum().backward()
    torch.cuda.synchronize()
    assert all(p.grad is not None and torch.isfinite(p.grad).all() for p in params)
    ctx.close()


def test_out_of_range_network_id_gives_status_and_nan_rows():
    from paper_2605_25346_amd import binding as B
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    require_gpu()
    wl = config_workload(5, n_sub=12)
    S = wl.batch.n_sub
    batch = wl.batch.subset(np.arange(S))
    batch.net_id = batch.net_id.copy()
    batch.net_id[5] = 7                      # three networks in the context: id 7 does not exist
    batch.net_id[9] = -1
    ms = int(np.max(np.diff(batch.split_ptr)))
    ctx = BoundContext(wl.nets, precision="f64", max_sub=S, max_splits=ms)
    lb, ub, status, _ = ctx.crown(DeviceBatch(batch))
    l, u = ctx.dr_get_bounds()
    torch.cuda.synchronize()
    st, l, u = status.cpu().numpy(), l.cpu().numpy(), u.cpu().numpy()
    lb, ub = lb.cpu().numpy(), ub.cpu().numpy()
    for s in (5, 9):
        assert st[s] & B.DR_RES_BADSPLIT, (s, st[s])
        assert np.all(np.isnan(l[s])) and np.all(np.isnan(u[s]))
        assert np.all(np.isposinf(lb[s])) and np.all(np.isneginf(ub[s]))
    for s in range(S):
        if s in (5, 9) or st[s] & 1:
            continue
        net = wl.nets[int(batch.net_id[s])]
        H = sum(net.hidden)
        assert np.all(np.isfinite(l[s, :H])) and np.all(np.isfinite(u[s, :H])), s
        o = crown.crown(net, batch.x_center[s], batch.x_radius[s], batch.splits_of(s))
        if o["status"] == 0 and not near_tie(o["bounds"], 1e-9):
            assert np.all(rel_gap(lb[s], o["lb"]) <= 1e-9) and np.all(rel_gap(ub[s], o["ub"]) <= 1e-9), s
    ctx.close()
