"""Throughput of the bound-propagation hot path on one MI355X.

Default workload (the headline): batched plain CROWN on the 6-64x3-3 network, 4096
subdomains with 0-8 ReLU splits each, FP32 matrix-core chains with FP64 concretization
and rigorous rounding margins.  One step = dr_bound_init (layer-1 bounds, IBP, CROWN
intermediate bounds, relaxation) + dr_propagate_backward (spec rows) + dr_concretize,
replayed from a HIP graph with the inputs resident in HBM.

Also measured (reported under "extra", each with its own roofline figure):
  * alpha/beta projected gradient ascent (20 steps, lr 0.1) on 8-128x4-4, 2048 subdomains;
  * stepwise linear-TM closed-loop reachability, 12-256x3-4, 8192 boxes, horizon 10;
  * the mixed persistent batch: 16384 subdomains over three networks, 0-32 splits,
    plain CROWN + 10 dual steps in one graph;
  * the FP64-chain variant of the headline workload.
The FP64 reference is timed on the host on a bounded sample ("cpu_baseline").

Prints ONE JSON line.  Runs on one GPU: the path has no multi-GPU execution.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "bounded subdomains/sec + α/β-opt iters/sec vs plain CROWN at equal tightness"
# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE/WRITE_SIZE runs, scaled by a plain
# copy of known size (see profiles/); valid only for the kernel sources they were taken with.
TRAFFIC = {"src_sha": "e3daff8e5d07a394", "k_bound_init_bytes": 2.12e6 + 30.74e6}


def kernel_src_sha():
    """Hash of what the headline kernel is built from: its sources and the compile flags of
    its translation unit (FP32 chains, 64-wide layers)."""
    import hashlib
    from paper_2605_25346_amd import build as B
    h = hashlib.sha256()
    for f in ("bound_kernels.hpp", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2605_25346_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    for obj, _, extra in B._units():
        if os.path.basename(obj) == "inst_float_4.o":
            h.update(" ".join(B.HIPCC_FLAGS + extra).encode())
    return h.hexdigest()[:16]
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}     # MI355X dense FP32 / FP64 matrix peaks
PEAK_VALU_F64 = 78.6                          # MI355X FP64 vector peak (TFLOP/s)
PEAK_HBM_GBS = 8000.0


def chain_flops_per_row(widths, k):
    """Algorithmic FLOPs (2 per MAC) of one backward chain row that starts at hidden
    layer k (its first product is a gather of a weight row, 0 FLOPs): the products
    with W_{k-1} .. W_1."""
    return sum(2 * widths[j] * widths[j - 1] for j in range(1, k))


def final_flops_per_row(widths):
    """A final (spec) row: its first product a_L W_L is the same for every subdomain and
    is formed once per network (the seeds), so a row costs the products with
    W_{L-1} .. W_1."""
    L = len(widths) - 1
    return chain_flops_per_row(widths, L)


def bound_init_flops(nets, net_id, rows):
    """Intermediate-bound chains actually required: rows[s][k-1] rows at layer k."""
    tot = 0
    for s in range(rows.shape[0]):
        w = nets[int(net_id[s])].widths
        for k in range(2, len(w) - 1):
            tot += int(rows[s, k - 1]) * chain_flops_per_row(w, k)
    return tot


def dense_flops(nets, net_id, status, R):
    """Context count: every hidden neuron of layers 2..L-1 gets its two CROWN rows
    (not only the IBP-unstable unsplit ones), plus the spec rows."""
    tot = 0
    for s in range(len(net_id)):
        if status[s] & 9:
            continue
        w = nets[int(net_id[s])].widths
        tot += sum(2 * w[k] * chain_flops_per_row(w, k) for k in range(2, len(w) - 1)) + R * final_flops_per_row(w)
    return tot


def final_flops(nets, net_id, status, R):
    tot = 0
    for s in range(len(net_id)):
        if status[s] & 9:
            continue
        tot += R * final_flops_per_row(nets[int(net_id[s])].widths)
    return tot


class KernelTimer:
    """HIP events around launches on torch's current stream (the stream the library
    launches on).  An untimed launch of the same call goes first, so that the GPU is busy
    while the host records the start event and enqueues the timed launch: the start
    event then completes when the timed kernel can begin, and the interval holds the
    kernel, not the host's launch latency."""

    def __init__(self, torch):
        self.torch = torch
        self.ms = []

    def run(self, fn):
        ev0 = self.torch.cuda.Event(enable_timing=True)
        ev1 = self.torch.cuda.Event(enable_timing=True)
        fn()
        ev0.record()
        out = fn()
        ev1.record()
        self.pending = (ev0, ev1)
        return out

    def collect(self):
        ev0, ev1 = self.pending
        ev1.synchronize()
        self.ms.append(ev0.elapsed_time(ev1))


def time_graph(torch, step, steps, warmup):
    """Capture `step` into a HIP graph; replay warmup + steps times; return ms/step."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, g


def headline(torch, args, precision="f32"):
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    from paper_2605_25346_amd.workloads import config_workload
    wl = config_workload(2)
    S = wl.batch.n_sub
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S, max_splits=8, tile_cfg="auto")
    db = DeviceBatch(wl.batch)
    q, n0 = ctx.q, ctx.n0
    f = lambda *sh: torch.zeros(*sh, dtype=torch.float64, device="cuda")
    aff = (f(S, q, n0), f(S, q), f(S, q, n0), f(S, q))
    out = (f(S, q), f(S, q), torch.zeros(S, dtype=torch.int32, device="cuda"))
    st0 = torch.zeros(S, dtype=torch.int32, device="cuda")

    def step():
        ctx.dr_bound_init(db, status=st0)
        ctx.dr_propagate_backward(aff)
        ctx.dr_concretize(*aff, out=out)

    ms, graph = time_graph(torch, step, args.steps, args.warmup)
    # dominant kernel (k_bound_init) timed alone with HIP events on the same stream
    kt = KernelTimer(torch)
    for _ in range(max(args.steps, 5)):
        kt.run(lambda: ctx.dr_bound_init(db))
        kt.collect()
    bi_ms = float(np.mean(kt.ms[1:])) if len(kt.ms) > 1 else kt.ms[0]
    rows = ctx.dr_get_rows().cpu().numpy()
    status = out[2].cpu().numpy()
    bounds = dict(lb=out[0].cpu().numpy(), ub=out[1].cpu().numpy(), margin=ctx.dr_get_margins().cpu().numpy())
    flops_bi = bound_init_flops(wl.nets, wl.batch.net_id, rows)
    flops_fin = final_flops(wl.nets, wl.batch.net_id, status, ctx.R)
    # with the spec rows fused at the end of k_bound_init, its work is both
    if ctx.fuse_spec:
        flops_bi += flops_fin
    achieved = flops_bi / (bi_ms * 1e-3) / 1e12
    flops_dense = dense_flops(wl.nets, wl.batch.net_id, status, ctx.R) - (0 if ctx.fuse_spec else flops_fin)
    res = dict(ms=ms, S=S, bi_ms=bi_ms, flops_bi=flops_bi, flops_final=flops_fin, achieved=achieved,
               tile_cfg=ctx.tile_cfg, fuse_spec=ctx.fuse_spec,
               flops_dense=flops_dense, achieved_dense=flops_dense / (bi_ms * 1e-3) / 1e12,
               step_tflops=flops_bi / (ms * 1e-3) / 1e12, infeasible=int(np.sum(status & 1)))
    ctx.close()
    return res, wl, bounds


def s_sweep(torch, args, mults=(1, 4, 16)):
    """Steady-state throughput of the headline step at 1x, 4x and 16x the batch: the
    4096 subdomains of the headline batch tiled m times (identical work per
    subdomain), so larger launches fill the chip for more rounds."""
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    from paper_2605_25346_amd.workloads import config_workload
    wl = config_workload(2)
    S0 = wl.batch.n_sub
    out = []
    for m in mults:
        batch = wl.batch.subset(np.tile(np.arange(S0), m))
        S = batch.n_sub
        ctx = BoundContext(wl.nets, precision="f32", max_sub=S, max_splits=8, tile_cfg="auto")
        db = DeviceBatch(batch)
        q, n0 = ctx.q, ctx.n0
        f = lambda *sh: torch.zeros(*sh, dtype=torch.float64, device="cuda")
        aff = (f(S, q, n0), f(S, q), f(S, q, n0), f(S, q))
        res = (f(S, q), f(S, q), torch.zeros(S, dtype=torch.int32, device="cuda"))
        st0 = torch.zeros(S, dtype=torch.int32, device="cuda")

        def step():
            ctx.dr_bound_init(db, status=st0)
            ctx.dr_propagate_backward(aff)
            ctx.dr_concretize(*aff, out=res)

        ms, _ = time_graph(torch, step, max(5, args.steps // m), 2)
        out.append(dict(S=S, ms_per_step=ms, subdomains_per_s=S / (ms * 1e-3)))
        ctx.close()
        del db, aff, res, st0
    return out


def dual_ascent(torch, args, precision="f32"):
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    from paper_2605_25346_amd.workloads import config_workload
    wl = config_workload(3)
    S = wl.batch.n_sub
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S, max_splits=16, tile_cfg="auto")
    db = DeviceBatch(wl.batch)
    ctx.dr_bound_init(db)
    alpha, beta = ctx.new_duals()
    q = ctx.q
    out = (torch.zeros(S, q, dtype=torch.float64, device="cuda"), torch.zeros(S, q, dtype=torch.float64, device="cuda"),
           torch.zeros(S, dtype=torch.int32, device="cuda"))
    aff_lb = None

    def step():
        ctx.dr_optimize_duals(wl.iters, wl.lr, alpha, beta, init_duals=True, out=out)

    ms, _ = time_graph(torch, step, max(2, args.steps // 4), 1)
    status = out[2].cpu().numpy()
    live = int(np.sum((status & 9) == 0))
    # per evaluation: forward chain + adjoint chain (same products transposed)
    fpr = final_flops_per_row(wl.nets[0].widths)
    w = wl.nets[0].widths
    adj = sum(2 * w[j] * w[j - 1] for j in range(1, len(w) - 1))
    flops = live * ctx.R * ((wl.iters + 1) * fpr + wl.iters * adj)
    res = dict(ms=ms, S=S, iters=wl.iters, subdomain_iters_per_s=S * wl.iters / (ms * 1e-3),
               tflops=flops / (ms * 1e-3) / 1e12)
    ctx.close()
    return res


def param_grad(torch, args, precision="f32"):
    """Gradient of a weighted sum of the bounds w.r.t. every weight, bias and box of the
    8-128x4-4 network over its 2048-subdomain batch (plain-CROWN relaxation)."""
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    from paper_2605_25346_amd.workloads import config_workload
    wl = config_workload(3)
    S = wl.batch.n_sub
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S, max_splits=16, tile_cfg="auto")
    db = DeviceBatch(wl.batch)
    ctx.dr_bound_init(db)
    alpha, beta = ctx.new_duals()
    rng = np.random.default_rng(0)
    g_lb = torch.tensor(rng.normal(size=(S, ctx.q)), device="cuda")
    g_ub = torch.tensor(rng.normal(size=(S, ctx.q)), device="cuda")
    out, ws = ctx.param_grad_outputs()

    def step():
        ctx.dr_param_grad(alpha, beta, g_lb, g_ub, init_duals=True, out=out, workspace=ws)

    ms, _ = time_graph(torch, step, max(4, args.steps // 2), 2)
    status = out[6].cpu().numpy()
    live = int(np.sum((status & 9) == 0))
    w = wl.nets[0].widths
    L = len(w) - 1
    # forward chain + adjoint chain of every final row, then the per-layer contraction
    # over all rows (rows of infeasible subdomains are zero but still summed)
    adj = sum(2 * w[j] * w[j - 1] for j in range(1, L))
    contr = sum(2 * w[k] * (w[k - 1] + 1) for k in range(1, L + 1))
    flops = live * ctx.R * (final_flops_per_row(w) + adj) + S * ctx.R * contr
    res = dict(ms=ms, S=S, rows=S * ctx.R, tflops=flops / (ms * 1e-3) / 1e12,
               subdomains_per_s=S / (ms * 1e-3))
    ctx.close()
    return res


def tm_reach(torch, args, precision="f32", cfg=4):
    """Stepwise TM reach (cfg 4: closed-loop controller; cfg 6: candidate action
    sequences through a dynamics network with exogenous inputs)."""
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    from paper_2605_25346_amd.workloads import config_workload
    wl = config_workload(cfg)
    S = wl.batch.n_sub
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S, tile_cfg="auto")
    db = DeviceBatch(wl.batch)
    boxes = torch.zeros(S, wl.horizon + 1, ctx.n_state, 2, dtype=torch.float64, device="cuda")
    u = torch.as_tensor(wl.meta["u"], dtype=torch.float64, device="cuda") if "u" in wl.meta else None

    def step():
        ctx.dr_reach_dt(db, wl.horizon, boxes=boxes, u=u)

    ms, _ = time_graph(torch, step, max(2, args.steps // 4), 1)
    rows = ctx.dr_get_rows().cpu().numpy()
    w = wl.nets[0].widths
    L = len(w) - 1
    flops = 0
    for k in range(2, L):
        flops += int(rows[:, k - 1].sum()) * chain_flops_per_row(w, k)
    flops += int(rows[:, L - 1].sum()) * final_flops_per_row(w)
    res = dict(ms=ms, S=S, horizon=wl.horizon, box_steps_per_s=S * wl.horizon / (ms * 1e-3),
               tflops=flops / (ms * 1e-3) / 1e12)
    ctx.close()
    return res


def joint_flops(widths, n_state, rows):
    """Algorithmic FLOPs of CROWN through the unrolled loop for one box, from its rows
    (H x 8: rows[t][k-1] CROWN rows of hidden layer k at step t, rows[t][L-1] the state
    rows).  A row of layer k at step t runs the products with W_{k-1} .. W_1 of step t
    (its first product, W_k's row, is a gather), then t steps back; a state row of
    x_{t+1} runs t + 1 steps back, the first without the boundary products (lam is a
    unit vector there: they are gathers).  One step back = lam (B W_L) (n_state x
    n_{L-1}), lam A (n_state x n_0) and the network's chain W_{L-1} .. W_1."""
    L = len(widths) - 1
    boundary = 2 * n_state * widths[L - 1] + 2 * n_state * widths[0]
    per_step = boundary + chain_flops_per_row(widths, L)
    tot = 0
    for t in range(rows.shape[0]):
        for k in range(1, L):
            tot += int(rows[t, k - 1]) * (chain_flops_per_row(widths, k) + t * per_step)
        tot += int(rows[t, L - 1]) * ((t + 1) * per_step - boundary)
    return tot


def joint_reach(torch, args, precision="f32", n_boxes=128):
    """CROWN through the closed loop unrolled over the horizon against the stepwise TM
    reach on the same boxes (the paper's DT comparison: 128 initial sets, a dynamics
    network of three 96-wide layers, horizon 10): time, tube volume V (width sum over
    steps 1..H) and the achieved FLOP rate of the joint kernel."""
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    from paper_2605_25346_amd.workloads import config_workload
    wl = config_workload(6, n_sub=n_boxes)
    S, H = wl.batch.n_sub, wl.horizon
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S, tile_cfg="auto")
    db = DeviceBatch(wl.batch)
    u = torch.as_tensor(wl.meta["u"], dtype=torch.float64, device="cuda")
    bj = torch.zeros(S, H + 1, ctx.n_state, 2, dtype=torch.float64, device="cuda")
    bs = torch.zeros_like(bj)
    rows = torch.zeros(S, H, 8, dtype=torch.int32, device="cuda")
    reps = max(2, args.steps // 4)
    ms_j, _ = time_graph(torch, lambda: ctx.dr_reach_dt_joint(db, H, boxes=bj, u=u, rows=rows), reps, 1)
    ms_s, _ = time_graph(torch, lambda: ctx.dr_reach_dt(db, H, boxes=bs, u=u), reps, 1)
    torch.cuda.synchronize()
    rows_h = rows.cpu().numpy()
    w = wl.nets[0].widths
    flops = sum(joint_flops(w, ctx.n_state, rows_h[s]) for s in range(S))
    vol = lambda b: (b[:, 1:, :, 1] - b[:, 1:, :, 0]).sum(axis=(1, 2))
    vj, vs = vol(bj.cpu().numpy()), vol(bs.cpu().numpy())
    res = dict(S=S, horizon=H, ms_joint=ms_j, ms_stepwise=ms_s, time_ratio=ms_j / ms_s,
               box_steps_per_s=S * H / (ms_j * 1e-3), tflops=flops / (ms_j * 1e-3) / 1e12, flops=flops,
               V_joint_median=float(np.median(vj)), V_stepwise_median=float(np.median(vs)),
               V_ratio_median=float(np.median(vj / vs)), V_ratio_min=float((vj / vs).min()),
               V_ratio_max=float((vj / vs).max()))
    ctx.close()
    return res


def reach_gradient(torch, args, precision="f32", n_boxes=128):
    """Gradient of the tube volume through the stepwise reach (dr_reach_dt_grad: the
    forward reach with its record, then the reverse pass) for the training batch shape of
    the paper's DT comparison (128 initial sets of the 96-wide dynamics network with
    actions, horizon 10), w.r.t. actions, boxes, A, B and all weights and biases; timed
    against the forward reach alone.  Algorithmic FLOPs: three times the forward chain
    FLOPs (the forward chains, the chains in reverse, and the weight-gradient outer
    products, each of the size of the forward products)."""
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    from paper_2605_25346_amd.workloads import config_workload
    wl = config_workload(6, n_sub=n_boxes)
    S, H = wl.batch.n_sub, wl.horizon
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S, tile_cfg="auto")
    db = DeviceBatch(wl.batch)
    u = torch.as_tensor(wl.meta["u"], dtype=torch.float64, device="cuda")
    boxes = torch.zeros(S, H + 1, ctx.n_state, 2, dtype=torch.float64, device="cuda")
    gV = torch.full((S,), 1.0 / S, dtype=torch.float64, device="cuda")
    ws = torch.empty(int(ctx.lib.dr_reach_grad_workspace(ctx.ctx, S, H)), dtype=torch.uint8, device="cuda")
    reps = max(2, args.steps // 4)
    ms_f, _ = time_graph(torch, lambda: ctx.dr_reach_dt(db, H, boxes=boxes, u=u), reps, 1)
    rows = ctx.dr_get_rows().cpu().numpy()
    ms_g, _ = time_graph(torch, lambda: ctx.dr_reach_dt_grad(db, H, gV, u=u, boxes=boxes, workspace=ws), reps, 1)
    # the same without the weight and bias gradients (actions, boxes, A, B only: the MPC use)
    ms_u, _ = time_graph(torch, lambda: ctx.dr_reach_dt_grad(db, H, gV, u=u, boxes=boxes, workspace=ws,
                                                             want=("du", "dxc", "dxr", "dA", "dB")), reps, 1)
    w = wl.nets[0].widths
    L = len(w) - 1
    fwd = sum(int(rows[:, k - 1].sum()) * chain_flops_per_row(w, k) for k in range(2, L))
    fwd += int(rows[:, L - 1].sum()) * final_flops_per_row(w)
    res = dict(S=S, horizon=H, ms_gradient=ms_g, ms_gradient_without_weights=ms_u, ms_forward=ms_f, ratio=ms_g / ms_f,
               box_steps_per_s=S * H / (ms_g * 1e-3), flops=3 * fwd, tflops=3 * fwd / (ms_g * 1e-3) / 1e12,
               workspace_bytes=int(ws.numel()))
    ctx.close()
    return res


# FP64 operations of the quasi-quadratic TM arithmetic (hand count of the definitions;
# FMA = 2, min/max = 1, |.| free): the product of two scalar models truncated to the
# representation (kept monomials, the dropped ones and the interval parts bounded), and
# one model scaled and accumulated (its 35 coefficients and the interval part).
CT_PROD_FLOPS, CT_AXPY_FLOPS = 540, 74


def ct_step_flops(F, G, Q, rounds=3):
    """Algorithmic FP64 operations of one flowpipe step of one box (Theorem "TM flowpipe
    step via Picard iteration" with order 2): 2 Picard iterations, one validating image
    of the remainder and `rounds` refinements, each an evaluation of f over the models
    (every distinct quadratic product X_j X_k once, then the sums of F, G and Q terms
    per component), plus per image the subtraction of d/ds p and the range (84 per
    component), the step-end model, and the preconditioning (Gauss-Jordan inversion
    4 n^3, its check 2 n^3, the column scales and the input update)."""
    n = F.shape[0]
    n_u = G.shape[1] if G is not None else 0
    pairs = {(min(j, k), max(j, k)) for (_, j, k) in zip(*np.nonzero(Q))} if Q is not None else set()
    nnz = np.count_nonzero(F) + (np.count_nonzero(G) if G is not None else 0) + (np.count_nonzero(Q) if Q is not None else 0)
    f_eval = len(pairs) * CT_PROD_FLOPS + nnz * CT_AXPY_FLOPS
    images = 1 + rounds
    return ((2 + images) * f_eval + images * 84 * n + 2 * 35 * n + 35 * n
            + 6 * n ** 3 + 2 * n_u * n * n + 4 * n * n)


def ct_reach(torch, args, n_sub=4096):
    """The CT closed loop of the paper's quadrotor shape (12 states, 4 inputs, a 64x64
    controller certified every 5 flowpipe steps of 0.02, 100 steps) on a batch of
    initial boxes, and the open-loop flowpipe of the same field: box-steps per second
    and the achieved FP64 rate of the flowpipe arithmetic against the vector FP64 peak
    (the controller's CROWN chain FLOPs are counted separately)."""
    from paper_2605_25346_amd.api import BoundContext, CtField, DeviceBatch, dr_flowpipe_ct
    from paper_2605_25346_amd.workloads import Network, make_ct_workload
    wl = make_ct_workload(n_sub=n_sub)
    S, n, N = n_sub, wl.F.shape[0], wl.K * wl.N_ctl
    n_u = wl.G.shape[1]
    ctl = wl.controller
    loop = Network(ctl.Ws, ctl.bs, np.zeros((n_u, n)), np.eye(n_u))
    ctx = BoundContext([loop], precision="f32", max_sub=S)
    field = CtField(wl.a, wl.F, wl.G, wl.Q)
    field0 = CtField(wl.a, wl.F, None, wl.Q)
    xc = torch.as_tensor(wl.x_center, dtype=torch.float64, device="cuda")
    xr = torch.as_tensor(wl.x_radius, dtype=torch.float64, device="cuda")
    db = DeviceBatch.from_tensors(xc, xr)
    f64 = lambda *sh: torch.zeros(*sh, dtype=torch.float64, device="cuda")
    out = (f64(S, N + 1, n, 2), f64(S, N, n, 2), torch.zeros(S, dtype=torch.int32, device="cuda"))
    out0 = (f64(S, N + 1, n, 2), f64(S, N, n, 2), torch.zeros(S, dtype=torch.int32, device="cuda"))
    reps = max(2, args.steps // 10)
    ms_c, _ = time_graph(torch, lambda: ctx.dr_reach_ct(field, db, wl.h, wl.K, wl.N_ctl, out=out), reps, 1)
    rows = ctx.dr_get_rows().cpu().numpy()
    ms_f, _ = time_graph(torch, lambda: dr_flowpipe_ct(field0, xc, xr, wl.h, N, out=out0), reps, 1)
    torch.cuda.synchronize()
    st_c, st_f = out[2].cpu().numpy(), out0[2].cpu().numpy()
    w = ctl.widths
    L = len(w) - 1
    ctl_flops = sum(int(rows[:, k - 1].sum()) * chain_flops_per_row(w, k) for k in range(2, L))
    ctl_flops += int(rows[:, L - 1].sum()) * final_flops_per_row(w)
    flow_c = S * N * ct_step_flops(wl.F, wl.G, wl.Q)
    flow_f = S * N * ct_step_flops(wl.F, None, wl.Q)
    width = lambda b: float(np.median((b[:, -1, :, 1] - b[:, -1, :, 0]).sum(axis=1)))
    res = dict(S=S, steps=N, h=wl.h, K=wl.K, ms_closed_loop=ms_c, ms_flowpipe=ms_f,
               box_steps_per_s=S * N / (ms_c * 1e-3), flowpipe_box_steps_per_s=S * N / (ms_f * 1e-3),
               closed_loop_ok=int((st_c == 0).sum()), flowpipe_ok=int((st_f == 0).sum()),
               final_width_sum_median_closed=width(out[0].cpu().numpy()),
               final_width_sum_median_open=width(out0[0].cpu().numpy()),
               flow_flops_per_box_step=ct_step_flops(wl.F, wl.G, wl.Q),
               tflops_closed=(flow_c + ctl_flops) / (ms_c * 1e-3) / 1e12, ctl_chain_flops=ctl_flops,
               tflops_flowpipe=flow_f / (ms_f * 1e-3) / 1e12)
    ctx.close()
    return res


def mixed_batch(torch, args, precision="f32"):
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    from paper_2605_25346_amd.workloads import config_workload
    wl = config_workload(5)
    S = wl.batch.n_sub
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S, max_splits=32, tile_cfg="auto")
    db = DeviceBatch(wl.batch)
    ctx.dr_bound_init(db)
    alpha, beta = ctx.new_duals()
    q, n0 = ctx.q, ctx.n0
    f = lambda *sh: torch.zeros(*sh, dtype=torch.float64, device="cuda")
    aff = (f(S, q, n0), f(S, q), f(S, q, n0), f(S, q))
    cout = (f(S, q), f(S, q), torch.zeros(S, dtype=torch.int32, device="cuda"))
    dout = (f(S, q), f(S, q), torch.zeros(S, dtype=torch.int32, device="cuda"))

    def step():
        ctx.dr_bound_init(db)
        ctx.dr_propagate_backward(aff)
        ctx.dr_concretize(*aff, out=cout)
        ctx.dr_optimize_duals(wl.iters, wl.lr, alpha, beta, init_duals=True, out=dout)

    ms, _ = time_graph(torch, step, max(2, args.steps // 4), 1)
    # algorithmic FLOPs of the step: the intermediate-bound chains actually required and
    # the spec rows (plain CROWN), then per ascent evaluation the forward and adjoint chains
    rows = ctx.dr_get_rows().cpu().numpy()
    status = dout[2].cpu().numpy()
    flops = bound_init_flops(wl.nets, wl.batch.net_id, rows) + final_flops(wl.nets, wl.batch.net_id, status, ctx.R)
    for s_ in np.nonzero((status & 9) == 0)[0]:
        w = wl.nets[int(wl.batch.net_id[s_])].widths
        adj = sum(2 * w[j] * w[j - 1] for j in range(1, len(w) - 1))
        flops += ctx.R * ((wl.iters + 1) * final_flops_per_row(w) + wl.iters * adj)
    res = dict(ms=ms, S=S, iters=wl.iters, subdomains_per_s=S / (ms * 1e-3), flops=flops,
               tflops=flops / (ms * 1e-3) / 1e12)
    ctx.close()
    return res


def bisect_boxes(xc, xr, parent, chosen):
    """Bisect the chosen boxes along their widest input dimension (the others are kept):
    returns the new centres, radii and parent (original subdomain) of every box."""
    dim = np.argmax(xr, axis=1)
    rows = np.nonzero(chosen)[0]
    half = xr[rows, dim[rows]] / 2.0
    lo_c, hi_c = xc[rows].copy(), xc[rows].copy()
    lo_c[np.arange(rows.size), dim[rows]] -= half
    hi_c[np.arange(rows.size), dim[rows]] += half
    r2 = xr[rows].copy()
    r2[np.arange(rows.size), dim[rows]] = half
    keep = ~chosen
    return (np.concatenate([xc[keep], lo_c, hi_c]), np.concatenate([xr[keep], r2, r2]),
            np.concatenate([parent[keep], parent[rows], parent[rows]]))


def equal_tightness(torch, args, cfg=3, precision="f32", tol=0.02, max_levels=4):
    """Plain CROWN + input splitting vs alpha/beta ascent at equal tightness (the
    comparison of the table "Refinement strategies": input splitting against gradient
    refinement).  The target is the mean width-sum V = sum_j (ub_j - lb_j) over the
    subdomains (the paper's volume proxy) of the ascent's bounds.  Plain CROWN refines by
    input splitting in levels: at each level a fraction f of the current boxes, those of
    the subdomains with the widest current bounds first, is bisected along its widest
    input dimension (the sub-boxes inherit the splits; a subdomain's bound is the union
    over its boxes); f is found by bisection search until V is within tol of the target
    (a level with f = 1 that is still wider moves to the next level).  Both sides run the
    same kernels and are timed as graph replays with the inputs resident."""
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    from paper_2605_25346_amd.workloads import config_workload
    wl = config_workload(cfg)
    S = wl.batch.n_sub
    ms_ = int(np.max(np.diff(wl.batch.split_ptr)))
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S, max_splits=ms_, tile_cfg="auto")
    db = DeviceBatch(wl.batch)
    ctx.dr_bound_init(db)
    alpha, beta = ctx.new_duals()
    q = ctx.q
    f = lambda *sh: torch.zeros(*sh, dtype=torch.float64, device="cuda")
    dout = (f(S, q), f(S, q), torch.zeros(S, dtype=torch.int32, device="cuda"))

    def step_ab():
        ctx.dr_bound_init(db)
        ctx.dr_optimize_duals(wl.iters, wl.lr, alpha, beta, init_duals=True, out=dout)

    ms_ab, _ = time_graph(torch, step_ab, max(2, args.steps // 10), 1)
    lb, ub, st = (t.cpu().numpy() for t in dout)
    live = (st & 9) == 0
    V_ab = float(np.mean((ub - lb).sum(axis=1)[live]))
    ctx.close()
    cap = S * 2 ** max_levels
    ck = BoundContext(wl.nets, precision=precision, max_sub=cap, max_splits=ms_)   # plain CROWN: default kernels

    def crown_of(xc, xr, parent, timed=False):
        sub = wl.batch.subset(parent)
        sub.x_center, sub.x_radius = xc, xr
        Sk = sub.n_sub
        dk = DeviceBatch(sub)
        aff = (f(Sk, q, ck.n0), f(Sk, q), f(Sk, q, ck.n0), f(Sk, q))
        cout = (f(Sk, q), f(Sk, q), torch.zeros(Sk, dtype=torch.int32, device="cuda"))

        def step_crown():
            ck.dr_bound_init(dk)
            ck.dr_propagate_backward(aff)
            ck.dr_concretize(*aff, out=cout)

        if timed:
            ms_k, _ = time_graph(torch, step_crown, max(2, args.steps // 10), 1)
        else:
            step_crown()
            ms_k = None
        slb, sub_ub, sst = (t.cpu().numpy() for t in cout)
        ok = (sst & 9) == 0
        ulb = np.full((S, q), np.inf); uub = np.full((S, q), -np.inf)
        np.minimum.at(ulb, parent[ok], slb[ok]); np.maximum.at(uub, parent[ok], sub_ub[ok])
        feas = live & np.isfinite(ulb).all(axis=1)
        Vs = np.where(feas, (uub - ulb).sum(axis=1), 0.0)
        return float(np.mean(Vs[feas])), Vs, ms_k

    xc, xr, parent = wl.batch.x_center.copy(), wl.batch.x_radius.copy(), np.arange(S)
    V0, Vs, _ = crown_of(xc, xr, parent)
    curve = [dict(level=0, fraction=0.0, boxes=S, V=V0)]
    best = (xc, xr, parent, V0)
    for level in range(1, max_levels + 1):
        # boxes ordered by their subdomain's current width sum, widest first
        order = np.argsort(-Vs[parent], kind="stable")

        def refine(frac):
            chosen = np.zeros(parent.size, bool)
            chosen[order[:int(round(frac * parent.size))]] = True
            return bisect_boxes(xc, xr, parent, chosen)

        nxt = refine(1.0)
        Vf, Vs_f, _ = crown_of(*nxt)
        curve.append(dict(level=level, fraction=1.0, boxes=int(nxt[2].size), V=Vf))
        if Vf > V_ab * (1 + tol):
            xc, xr, parent, Vs = nxt[0], nxt[1], nxt[2], Vs_f
            best = (xc, xr, parent, Vf)
            continue
        lo, hi = 0.0, 1.0
        best = (*nxt, Vf)
        for _ in range(8):
            mid = 0.5 * (lo + hi)
            cand = refine(mid)
            Vm, _, _ = crown_of(*cand)
            curve.append(dict(level=level, fraction=mid, boxes=int(cand[2].size), V=Vm))
            if Vm <= V_ab:
                hi, best = mid, (*cand, Vm)
            else:
                lo = mid
            if abs(Vm - V_ab) <= tol * V_ab and Vm <= V_ab * (1 + tol):
                best = (*cand, Vm)
                break
        break
    V_eq, _, ms_eq = crown_of(best[0], best[1], best[2], timed=True)
    ck.close()
    reached = V_eq <= V_ab * (1 + tol)
    return dict(workload=wl.name, V_alpha_beta=V_ab, ms_alpha_beta=ms_ab, V_plain_crown_matched=V_eq,
                boxes_plain_crown=int(best[2].size), ms_plain_crown_matched=ms_eq, V_plain_crown_unsplit=V0,
                curve=curve, reached=bool(reached),
                speedup_alpha_beta_vs_plain_crown=(ms_eq / ms_ab) if reached else None)


# ---- CPU baseline: the FP64 oracle as it stands, timed on the host ---------------------
_ORACLE_NETS = None


def _oracle_init(nets):
    global _ORACLE_NETS
    _ORACLE_NETS = nets
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)          # one BLAS thread per worker process
    except Exception:  # pragma: no cover
        pass


def _near_decision(bounds, tol=1e-4):
    """True if a discrete choice taken in floating point is within tol (relative) of
    flipping in the oracle's intermediate bounds: an adaptive lower slope (u vs -l) or a
    stability test (l or u near 0, exact zeros of split clamping aside).  Either choice
    gives a valid bound there, so the GPU's may differ from the oracle's."""
    for (l, u) in bounds:
        sc = np.maximum(np.maximum(np.abs(l), np.abs(u)), 1e-300)
        uns = (l < 0) & (u > 0)
        if np.any(uns & (np.abs(u + l) <= tol * sc)):
            return True
        if np.any(((np.abs(l) <= tol * sc) & (l != 0)) | ((np.abs(u) <= tol * sc) & (u != 0))):
            return True
    return False


def _oracle_chunk(args):
    """Oracle bounds (plain CROWN) of a chunk of subdomains: (indices, lb, ub, status,
    near-decision flag)."""
    from oracle import crown
    idx, xc, xr, splits, net_id = args
    lb = np.zeros((len(idx), _ORACLE_NETS[0].widths[-1])); ub = np.zeros_like(lb)
    st = np.zeros(len(idx), np.int64)
    tie = np.zeros(len(idx), bool)
    for i in range(len(idx)):
        o = crown.crown(_ORACLE_NETS[int(net_id[i])], xc[i], xr[i], splits[i])
        lb[i], ub[i], st[i] = o["lb"], o["ub"], o["status"]
        tie[i] = _near_decision(o["bounds"])
    return idx, lb, ub, st, tie


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, budget_s=15.0, workers=None):
    """The FP64 reference, as it stands (one subdomain at a time), on the headline
    batch: the subdomains are independent, so the host's cores each take a contiguous
    share in their own process (one BLAS thread each).  One warm-up pass, then the
    median of 5 timed passes over a sample sized to about budget_s seconds of CPU work
    in total; a single-process figure on part of the sample.  Runs before the GPU is
    initialised (the worker processes are forked).  Returns the baseline record and the
    oracle bounds of the sample (for the GPU's per-result gap)."""
    import multiprocessing as mp
    S = wl.batch.n_sub
    P = workers or max(1, min(16, os.cpu_count() or 1))
    # single-process rate on a small prefix sets the sample size
    _oracle_init(wl.nets)
    n1 = min(S, 256)
    chunk = lambda idx: (idx, wl.batch.x_center[idx], wl.batch.x_radius[idx], [wl.batch.splits_of(s) for s in idx],
                         wl.batch.net_id[idx])
    _oracle_chunk(chunk(np.arange(16)))                        # warm-up
    t0 = time.perf_counter()
    _oracle_chunk(chunk(np.arange(n1)))
    single = n1 / (time.perf_counter() - t0)
    n = int(min(S, max(P * 32, budget_s / 6.0 * single)))       # 6 passes in the budget, at P x the rate at most
    sample = np.arange(n)
    parts = [chunk(a) for a in np.array_split(sample, P) if a.size]
    ctx = mp.get_context("fork")
    times = []
    with ctx.Pool(P, initializer=_oracle_init, initargs=(wl.nets,)) as pool:
        pool.map(_oracle_chunk, parts)                          # warm-up
        for _ in range(5):
            t0 = time.perf_counter()
            out = pool.map(_oracle_chunk, parts)
            times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    lb = np.zeros((n, wl.nets[0].widths[-1])); ub = np.zeros_like(lb); st = np.zeros(n, np.int64)
    tie = np.zeros(n, bool)
    for idx, a, b, c, d in out:
        lb[idx], ub[idx], st[idx], tie[idx] = a, b, c, d
    rec = dict(value=n / med, unit="subdomains/s", cores=P, kind="oracle",
               sample=f"first {n} of {S} subdomains of the headline batch (plain CROWN, numpy FP64, one subdomain "
                      f"at a time), {P} worker processes x 1 BLAS thread, median of 5 passes after a warm-up "
                      f"({med:.2f} s per pass)",
               single_thread=dict(value=single, unit="subdomains/s", sample=f"first {n1} subdomains, 1 process"),
               cpu_model=_cpu_model(), host_cpus=os.cpu_count())
    return rec, dict(idx=sample, lb=lb, ub=ub, status=st, tie=tie)


def gap_to_oracle(lb, ub, margin, ref):
    """Per-result gap of GPU bounds to the oracle on the oracle's sample:
    |b_gpu - b_oracle| / max(1, |b_oracle|), the share of results where the GPU bound is
    tighter than the oracle's, and for rigorous margins the reported margin (same scale).
    A tighter GPU bound is not a soundness violation: the GPU's intermediate bounds are
    the oracle's loosened by their rounding margins, and CROWN with adaptive slopes is
    not monotone in the intermediate bounds (soundness against the network's true range
    is what the tests check, on sampled points).  Subdomains whose oracle run is within
    floating-point reach of a discrete decision (adaptive slope, stability) are counted
    apart: either decision is valid there."""
    if ref is None:
        return None
    idx = ref["idx"]
    ok = (ref["status"] == 0) & ~ref["tie"]
    g_lb, g_ub = lb[idx][ok], ub[idx][ok]
    o_lb, o_ub = ref["lb"][ok], ref["ub"][ok]
    gap = np.concatenate([np.abs(g_lb - o_lb) / np.maximum(1, np.abs(o_lb)),
                          np.abs(g_ub - o_ub) / np.maximum(1, np.abs(o_ub))]).ravel()
    tighter = np.concatenate([g_lb > o_lb + 1e-9 * np.maximum(1, np.abs(o_lb)),
                              g_ub < o_ub - 1e-9 * np.maximum(1, np.abs(o_ub))]).ravel()
    out = dict(results=int(gap.size), max=float(gap.max()), median=float(np.median(gap)),
               within_1e_5=float(np.mean(gap <= 1e-5)), tighter_than_oracle=float(np.mean(tighter)),
               near_decision_subdomains=int(np.sum(ref["tie"] & (ref["status"] == 0))))
    if margin is not None:
        q = lb.shape[1]
        m = margin[idx][ok]
        mg = np.concatenate([m[:, :q], m[:, q:]]).ravel() / np.concatenate(
            [np.maximum(1, np.abs(o_lb)), np.maximum(1, np.abs(o_ub))]).ravel()
        out["margin_median"] = float(np.median(mg))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-extra", action="store_true", help="only the headline workload")
    ap.add_argument("--only", default="", help="comma-separated extra legs to run (for profiling one leg): "
                    "f64,sweep,ascent,pgrad,reach,candidates,joint,reachgrad,ct,tightness,mixed")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of host work for the cpu_baseline leg (0: skip it, for profiler runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the bound propagation has no multi-GPU execution",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    cb = ref = None
    if not args.copy_calibration and args.cpu_budget > 0:
        # the host baseline first: its worker processes are forked before the GPU is touched
        from paper_2605_25346_amd.workloads import config_workload
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        cb, ref = cpu_baseline(config_workload(2), args.cpu_budget)
        print(f"bench: cpu baseline {cb}", file=sys.stderr, flush=True)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))
        return
    print("bench: headline workload", file=sys.stderr, flush=True)
    hl, wl, hb = headline(torch, args, "f32")
    print(f"bench: headline {hl}", file=sys.stderr, flush=True)
    gap32 = gap_to_oracle(hb["lb"], hb["ub"], hb["margin"], ref)
    extra = {}
    only = set(filter(None, args.only.split(",")))
    leg = lambda name: not args.no_extra and (not only or name in only)
    if leg("f64"):
        print("bench: f64 headline", file=sys.stderr, flush=True)
        h64, _, hb64 = headline(torch, args, "f64")
        print(f"bench: f64 headline {h64}", file=sys.stderr, flush=True)
        extra["crown_6-64x3-3_S4096_f64"] = dict(
            subdomains_per_s=h64["S"] / (h64["ms"] * 1e-3), ms_per_step=h64["ms"],
            roofline=dict(bound="mfma", achieved=h64["achieved"], peak=PEAK_TFLOPS["f64"], unit="TFLOP/s",
                          frac=h64["achieved"] / PEAK_TFLOPS["f64"]),
            gap_to_oracle=gap_to_oracle(hb64["lb"], hb64["ub"], hb64["margin"], ref))
    if leg("sweep"):
        print("bench: S sweep", file=sys.stderr, flush=True)
        sw = s_sweep(torch, args)
        print(f"bench: S sweep {sw}", file=sys.stderr, flush=True)
        extra["crown_6-64x3-3_S_sweep_tiled_x1_x4_x16"] = sw
    if leg("ascent"):
        print("bench: dual ascent", file=sys.stderr, flush=True)
        da = dual_ascent(torch, args, "f32")
        print(f"bench: dual ascent {da}", file=sys.stderr, flush=True)
        extra["abcrown_8-128x4-4_S2048_20it"] = dict(
            subdomain_iters_per_s=da["subdomain_iters_per_s"], ms_per_call=da["ms"],
            roofline=dict(bound="mfma", achieved=da["tflops"], peak=PEAK_TFLOPS["f32"], unit="TFLOP/s",
                          frac=da["tflops"] / PEAK_TFLOPS["f32"]))
    if leg("pgrad"):
        print("bench: parameter gradient", file=sys.stderr, flush=True)
        pg = param_grad(torch, args, "f32")
        print(f"bench: parameter gradient {pg}", file=sys.stderr, flush=True)
        extra["param_grad_8-128x4-4_S2048"] = dict(
            subdomains_per_s=pg["subdomains_per_s"], ms_per_call=pg["ms"],
            roofline=dict(bound="mfma", achieved=pg["tflops"], peak=PEAK_TFLOPS["f32"], unit="TFLOP/s",
                          frac=pg["tflops"] / PEAK_TFLOPS["f32"]))
    if leg("reach"):
        print("bench: TM reach", file=sys.stderr, flush=True)
        tr = tm_reach(torch, args, "f32")
        print(f"bench: TM reach {tr}", file=sys.stderr, flush=True)
        extra["tmreach_12-256x3-4_S8192_H10"] = dict(
            box_steps_per_s=tr["box_steps_per_s"], ms_per_call=tr["ms"],
            roofline=dict(bound="mfma", achieved=tr["tflops"], peak=PEAK_TFLOPS["f32"], unit="TFLOP/s",
                          frac=tr["tflops"] / PEAK_TFLOPS["f32"]))
    if leg("candidates"):
        print("bench: candidate reach", file=sys.stderr, flush=True)
        cr = tm_reach(torch, args, "f32", cfg=6)
        print(f"bench: candidate reach {cr}", file=sys.stderr, flush=True)
        extra["mpc_candidates_8+4-96x3-8_S4096_H10"] = dict(
            box_steps_per_s=cr["box_steps_per_s"], ms_per_call=cr["ms"],
            roofline=dict(bound="mfma", achieved=cr["tflops"], peak=PEAK_TFLOPS["f32"], unit="TFLOP/s",
                          frac=cr["tflops"] / PEAK_TFLOPS["f32"]))
    if leg("joint"):
        print("bench: joint CROWN through the unrolled loop", file=sys.stderr, flush=True)
        jr = joint_reach(torch, args, "f32")
        print(f"bench: joint reach {jr}", file=sys.stderr, flush=True)
        extra["joint_crown_vs_stepwise_8+4-96x3-8_S128_H10"] = dict(
            jr, roofline=dict(bound="mfma", achieved=jr["tflops"], peak=PEAK_TFLOPS["f32"], unit="TFLOP/s",
                              frac=jr["tflops"] / PEAK_TFLOPS["f32"], kernel="k_reach_joint"))
    if leg("reachgrad"):
        print("bench: reach-tube gradient", file=sys.stderr, flush=True)
        rg = reach_gradient(torch, args, "f32")
        print(f"bench: reach gradient {rg}", file=sys.stderr, flush=True)
        extra["reach_volume_gradient_8+4-96x3-8_S128_H10"] = dict(
            rg, roofline=dict(bound="mfma", achieved=rg["tflops"], peak=PEAK_TFLOPS["f32"], unit="TFLOP/s",
                              frac=rg["tflops"] / PEAK_TFLOPS["f32"], kernel="k_reach_dt + k_reach_grad"))
    if leg("ct"):
        print("bench: CT closed loop and flowpipe", file=sys.stderr, flush=True)
        cr = ct_reach(torch, args)
        print(f"bench: CT {cr}", file=sys.stderr, flush=True)
        extra["ct_quadratic12+4-64x2-4_S4096_N100"] = dict(
            cr, roofline=dict(bound="alu", achieved=cr["tflops_flowpipe"], peak=PEAK_VALU_F64, unit="TFLOP/s",
                              frac=cr["tflops_flowpipe"] / PEAK_VALU_F64, kernel="k_flowpipe_ct",
                              note="FP64 peak (vector and matrix cores alike: the term sums run on the "
                                   "matrix cores); closed loop: tflops_closed over both parts"))
    if leg("tightness"):
        for cfg_i, key in ((3, "equal_tightness_abcrown_8-128x4-4_vs_crown_input_splitting"),
                           (5, "equal_tightness_mixed_S16384_vs_crown_input_splitting")):
            print(f"bench: equal tightness cfg {cfg_i}", file=sys.stderr, flush=True)
            extra[key] = equal_tightness(torch, args, cfg=cfg_i)
            print(f"bench: equal tightness {extra[key]}", file=sys.stderr, flush=True)
    if leg("mixed"):
        print("bench: mixed batch", file=sys.stderr, flush=True)
        mb = mixed_batch(torch, args, "f32")
        print(f"bench: mixed batch {mb}", file=sys.stderr, flush=True)
        extra["mixed_S16384_crown+10it"] = dict(
            subdomains_per_s=mb["subdomains_per_s"], ms_per_step=mb["ms"],
            roofline=dict(bound="mfma", achieved=mb["tflops"], peak=PEAK_TFLOPS["f32"], unit="TFLOP/s",
                          frac=mb["tflops"] / PEAK_TFLOPS["f32"], flops_per_step=mb["flops"],
                          note="whole graph-replayed step (all kernels of the three networks)"))
    value = hl["S"] / (hl["ms"] * 1e-3)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "subdomains/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hl["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "crown_6-64x3-3_S4096", "network": "6-64-64-64-3", "subdomains": hl["S"],
                   "splits_per_subdomain": "0-8", "spec": "lower+upper of 3 outputs",
                   "chain_precision": "f32", "concretize": "f64", "margins": "rigorous",
                   "parallelism": "single GPU", "tile_cfg": hl["tile_cfg"], "spec_rows_fused": hl["fuse_spec"]},
        "roofline": {"bound": "mfma", "achieved": hl["achieved"], "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                     "frac": hl["achieved"] / PEAK_TFLOPS["f32"],
                     "traffic": TRAFFIC["k_bound_init_bytes"] if kernel_src_sha() == TRAFFIC["src_sha"] else None,
                     "kernel": "k_bound_init", "kernel_ms": hl["bi_ms"], "flops_per_launch": hl["flops_bi"],
                     "flops_dense_rows_per_launch": hl["flops_dense"],
                     "frac_dense_rows": hl["achieved_dense"] / PEAK_TFLOPS["f32"]},
        "cpu_baseline": cb,
        # per-result gap of the headline's bounds (FP32 chains, rigorous margins) to the
        # FP64 oracle on the CPU baseline's sample; the FP64-chain row beside it in extra
        "gap_to_oracle": gap32,
        "extra": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
