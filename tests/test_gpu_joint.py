"""Parity of dr_reach_dt_joint (CROWN through the closed loop unrolled over the horizon)
with the oracle ``oracle/joint.py``, through the C-ABI.

Tolerances: FP64 chains 1e-9 relative to max(1, |b|) (margins on or off); FP32 chains
without margins 1e-5 at every step; FP32 with rigorous margins: sampled rollouts inside
every box and the gap printed.  The CROWN row counts (integers decided by interval
bounds) are compared exactly in FP64.
"""
import numpy as np
import pytest

from oracle import exact, joint
from paper_2605_25346_amd.workloads import Network, config_workload, make_network, make_workload
from tests.gpu_helpers import rel_gap, require_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {("f64", True): 1e-9, ("f64", False): 1e-9, ("f32", False): 1e-5}


def _ctx(nets, precision, S, margins=True):
    from paper_2605_25346_amd.api import BoundContext
    return BoundContext(nets, precision=precision, max_sub=max(S, 1), max_splits=0, margins=margins)


def _run(wl, precision, margins, H, u=None):
    from paper_2605_25346_amd.api import DeviceBatch
    ctx = _ctx(wl.nets, precision, wl.batch.n_sub, margins)
    boxes, st, rows = ctx.dr_reach_dt_joint(DeviceBatch(wl.batch), H, u=u)
    torch.cuda.synchronize()
    out = boxes.cpu().numpy(), st.cpu().numpy(), rows.cpu().numpy()
    ctx.close()
    return out


def _rollouts_inside(net, xc, xr, u, boxes, H, seed, n=2000):
    rng = np.random.default_rng(seed)
    X = exact.sample_points(rng, xc, xr, n, corners=True)
    for t in range(H + 1):
        assert np.all(X >= boxes[t, :, 0] - 1e-12) and np.all(X <= boxes[t, :, 1] + 1e-12), t
        if t < H:
            V = np.hstack([X, np.repeat(u[t][None, :], X.shape[0], axis=0)]) if u is not None else X
            y, _ = exact.forward(net, V)
            X = V @ net.A.T + y @ net.B.T


def _check(tag, wl, H, u, S, sample=None):
    """The GPU over all S boxes; the oracle and the comparisons over `sample` (all boxes
    by default)."""
    net = wl.nets[0]
    n = net.A.shape[0]
    idx = list(range(S)) if sample is None else list(sample)
    ref = {s: joint.reach_joint(net, wl.batch.x_center[s][:n], wl.batch.x_radius[s][:n], H,
                                None if u is None else u[s][:H]) for s in idx}
    for precision, margins in (("f64", True), ("f64", False), ("f32", False), ("f32", True)):
        if precision == "f32" and not all(np.array_equal(W, W.astype(np.float32)) for W in net.Ws + net.bs):
            continue     # FP64 weights run FP64 chains only (the network is its weights)
        boxes, st, rows = _run(wl, precision, margins, H, None if u is None else u[:, :H])
        assert np.all(st == 0), st
        gaps = np.array([rel_gap(boxes[s], ref[s][0]) for s in idx])
        print(f"[joint {tag} {precision} margins={margins}] per-step max gap "
              + " ".join(f"{v:.1e}" for v in gaps.max(axis=(0, 2, 3))), flush=True)
        tol = TOL.get((precision, margins))
        if tol is not None:
            assert np.all(gaps <= tol), (precision, margins, gaps.max(axis=(0, 2, 3)))
        if precision == "f64":
            want = np.array([ref[s][1]["rows"] for s in idx])
            L = net.n_layers
            np.testing.assert_array_equal(rows[idx, :H, :L], want)
        if margins:
            for s in idx:
                _rollouts_inside(net, wl.batch.x_center[s][:n], wl.batch.x_radius[s][:n],
                                 None if u is None else u[s][:H], boxes[s], H, s)
        if precision == "f64" and margins:
            for s in idx:
                ob = ref[s][0]
                sl = 1e-9 * np.maximum(1, np.abs(ob))
                assert np.all(boxes[s, :, :, 0] <= ob[:, :, 0] + sl[:, :, 0])
                assert np.all(boxes[s, :, :, 1] >= ob[:, :, 1] - sl[:, :, 1])


def test_joint_candidate_dynamics():
    """The 96-wide dynamics network with exogenous actions (8 state + 4 action inputs)."""
    require_gpu()
    wl = config_workload(6, n_sub=6)
    _check("mpc 8+4-96x3-8", wl, 6, wl.meta["u"], 6)


def test_joint_full_size_sampled():
    """The benchmarked launch: 128 boxes x 10 steps of the 96-wide dynamics network with
    actions (one workgroup per box, the horizon's relaxations in LDS); six boxes spread
    over the batch against the oracle."""
    require_gpu()
    wl = config_workload(6, n_sub=128)
    _check("mpc 8+4-96x3-8 S128 H10", wl, wl.horizon, wl.meta["u"], 128, sample=(0, 1, 37, 64, 101, 127))


def test_joint_controller_loop():
    """Closed-loop controllers without exogenous inputs: 4-32-32-2 (configuration 1's
    shape) and a 64-wide one whose controller output matters."""
    require_gpu()
    wl = config_workload(1, n_sub=5)
    _check("cl 4-32-32-2", wl, 5, None, 5)
    wl = make_workload("joint64", 90, [[6, 64, 64, 3]], 5, closed_loop=True, radius=0.05, horizon=4,
                       shared_slope=True, A_mode="signed_perm", rho=0.9, b_var=0.05)
    _check("cl 6-64-64-3", wl, 4, None, 5)


def test_joint_wide_network():
    """256-wide hidden layers (LDS chain stages) over 3 steps."""
    require_gpu()
    wl = config_workload(4, n_sub=3)
    _check("cl 12-256x3-4", wl, 3, None, 3)


def test_joint_hand_case():
    """x' = -x + 2 relu(x), x_0 in [-1, 2]: x_1, x_2 in [-1, 2] (worked by hand)."""
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    from paper_2605_25346_amd.workloads import Batch
    require_gpu()
    net = Network([np.ones((1, 1)), np.ones((1, 1))], [np.zeros(1), np.zeros(1)], -np.ones((1, 1)), 2 * np.ones((1, 1)))
    batch = Batch(np.array([[0.5]]), np.array([[1.5]]), np.zeros(2, np.int32), np.zeros(0, np.int32),
                  np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(1, np.int32))
    ctx = BoundContext([net], precision="f64", max_sub=1, max_splits=0)
    boxes, st, rows = ctx.dr_reach_dt_joint(DeviceBatch(batch), 2)
    b = boxes.cpu().numpy()[0, :, 0]
    np.testing.assert_allclose(b[1:], [[-1.0, 2.0], [-1.0, 2.0]], atol=1e-12)
    ctx.close()


def test_joint_argument_errors():
    """Host-side checks: exogenous inputs required, a horizon beyond the on-chip
    relaxation store is a capacity error naming the limit."""
    from paper_2605_25346_amd import binding as B
    from paper_2605_25346_amd.api import DeviceBatch
    require_gpu()
    wl = config_workload(6, n_sub=2)
    ctx = _ctx(wl.nets, "f32", 2)
    db = DeviceBatch(wl.batch)
    with pytest.raises(B.DrError) as ei:
        ctx.dr_reach_dt_joint(db, 3)
    assert ei.value.status == B.DR_EINVAL
    with pytest.raises(B.DrError) as ei:
        ctx.dr_reach_dt_joint(db, 500, u=np.zeros((2, 500, 4)))
    assert ei.value.status == B.DR_ECAPACITY and "at most" in str(ei.value)
    ctx.close()
