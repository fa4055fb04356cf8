"""dr_param_grad_static (the entry point that allocates nothing: its tapes and partial
sums live in the library's static device scratch) against dr_param_grad with a
caller-owned workspace, through the C-ABI: two calls in a row on one context, the
second on a smaller batch, each identical to the workspace call on the same inputs;
a batch too large for the static scratch is refused before any launch."""
import numpy as np
import pytest

from paper_2605_25346_amd.workloads import config_workload, random_duals
from tests.gpu_helpers import require_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _grads(ctx, db, static, seed):
    S, R = db.n_sub, ctx.R
    ctx.dr_bound_init(db)
    al, be = random_duals(seed, S, R, max(ctx.H_max, 1), max(ctx.max_splits, 1), beta_scale=0.5)
    alpha = torch.tensor(al, dtype=torch.float32, device="cuda")
    beta = torch.tensor(be, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed)
    g_lb = torch.tensor(rng.normal(size=(S, ctx.q)), device="cuda")
    g_ub = torch.tensor(rng.normal(size=(S, ctx.q)), device="cuda")
    out, ws = ctx.param_grad_outputs()
    if static:
        res = ctx.dr_param_grad_static(alpha, beta, g_lb, g_ub, out=out)
    else:
        res = ctx.dr_param_grad(alpha, beta, g_lb, g_ub, out=out, workspace=ws)
    torch.cuda.synchronize()
    lb, ub, dW, db_, dxc, dxr, st = res
    flat = [lb, ub, *dW, *db_, dxc, dxr]
    return [t.cpu().numpy().copy() for t in flat], st.cpu().numpy().copy()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_static_scratch_entry_matches_workspace_entry(precision):
    from paper_2605_25346_amd import binding as B
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    require_gpu()
    wl = config_workload(3, n_sub=256)
    ms = int(np.max(np.diff(wl.batch.split_ptr)))
    ctx = BoundContext(wl.nets, precision=precision, max_sub=2048, max_splits=ms)
    print(f"[no-alloc] {precision}: calls on 256 then 96 subdomains", flush=True)
    for S in (256, 96):                      # the second call is smaller
        db = DeviceBatch(wl.batch.subset(np.arange(S)))
        ref, st_ref = _grads(ctx, db, False, seed=S)
        got, st_got = _grads(ctx, db, True, seed=S)
        assert np.array_equal(st_ref, st_got)
        for a, b in zip(ref, got):
            assert a.shape == b.shape
            np.testing.assert_array_equal(a, b)
        assert np.any([np.any(x != 0) for x in got[2:]])   # the gradients are not trivially zero
    # a batch whose tapes exceed the static scratch is refused before any launch
    big = DeviceBatch(config_workload(3).batch)
    need = int(ctx.lib.dr_param_grad_workspace(ctx.ctx, big.n_sub))
    assert need > (64 << 20)
    ctx.dr_bound_init(big)
    alpha, beta = ctx.new_duals()
    z = torch.zeros(big.n_sub, ctx.q, dtype=torch.float64, device="cuda")
    with pytest.raises(B.DrError) as ei:
        ctx.dr_param_grad_static(alpha, beta, z, z, init_duals=True)
    assert ei.value.status == B.DR_ECAPACITY
    torch.cuda.synchronize()
    ctx.close()
