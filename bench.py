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
TRAFFIC = {"src_sha": "4ff5e1f5bd6ff017", "k_bound_init_bytes": 2.16e6 + 30.93e6}


def kernel_src_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("bound_kernels.hpp", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2605_25346_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}     # MI355X dense FP32 / FP64 matrix peaks
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
    launches on)."""

    def __init__(self, torch):
        self.torch = torch
        self.ms = []

    def run(self, fn):
        ev0 = self.torch.cuda.Event(enable_timing=True)
        ev1 = self.torch.cuda.Event(enable_timing=True)
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
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S, max_splits=8)
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
    flops_bi = bound_init_flops(wl.nets, wl.batch.net_id, rows)
    flops_fin = final_flops(wl.nets, wl.batch.net_id, status, ctx.R)
    # the spec rows run fused at the end of k_bound_init: its work is both
    flops_bi += flops_fin
    achieved = flops_bi / (bi_ms * 1e-3) / 1e12
    flops_dense = dense_flops(wl.nets, wl.batch.net_id, status, ctx.R)
    res = dict(ms=ms, S=S, bi_ms=bi_ms, flops_bi=flops_bi, flops_final=flops_fin, achieved=achieved,
               flops_dense=flops_dense, achieved_dense=flops_dense / (bi_ms * 1e-3) / 1e12,
               step_tflops=flops_bi / (ms * 1e-3) / 1e12, infeasible=int(np.sum(status & 1)))
    ctx.close()
    return res, wl


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
        ctx = BoundContext(wl.nets, precision="f32", max_sub=S, max_splits=8)
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
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S, max_splits=16)
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
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S, max_splits=16)
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
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S)
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


def mixed_batch(torch, args, precision="f32"):
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    from paper_2605_25346_amd.workloads import config_workload
    wl = config_workload(5)
    S = wl.batch.n_sub
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S, max_splits=32)
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
    res = dict(ms=ms, S=S, iters=wl.iters, subdomains_per_s=S / (ms * 1e-3))
    ctx.close()
    return res


def split_boxes(batch, k):
    """Input splitting: bisect the k widest input dimensions of every box (round robin
    from the widest), 2^k sub-boxes per subdomain, each inheriting the split set."""
    from paper_2605_25346_amd.workloads import Batch
    S, n0 = batch.x_center.shape
    xc, xr = batch.x_center.copy(), batch.x_radius.copy()
    parent = np.arange(S)
    for j in range(k):
        dim = np.argsort(-xr, axis=1, kind="stable")[:, 0]
        half = xr[np.arange(xr.shape[0]), dim] / 2.0
        lo_c, hi_c = xc.copy(), xc.copy()
        lo_c[np.arange(xc.shape[0]), dim] -= half
        hi_c[np.arange(xc.shape[0]), dim] += half
        xr2 = xr.copy(); xr2[np.arange(xr.shape[0]), dim] = half
        xc = np.concatenate([lo_c, hi_c]); xr = np.concatenate([xr2, xr2]); parent = np.concatenate([parent, parent])
    sub = batch.subset(parent)
    sub.x_center, sub.x_radius = xc, xr
    return sub, parent


def equal_tightness(torch, args, precision="f32", max_k=8):
    """Plain CROWN + input splitting vs alpha/beta ascent at equal tightness: the mean
    width-sum volume proxy V = sum_j (ub_j - lb_j) (the paper's tube-volume proxy for one
    step) of the ascent's bounds is the target; the number of sub-boxes per subdomain is
    doubled until plain CROWN reaches it.  Both sides run the same kernels and are
    timed as graph replays with inputs resident."""
    from paper_2605_25346_amd.api import BoundContext, DeviceBatch
    from paper_2605_25346_amd.workloads import config_workload
    wl = config_workload(3)
    S = wl.batch.n_sub
    ctx = BoundContext(wl.nets, precision=precision, max_sub=S, max_splits=16)
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
    curve = []
    for k in range(0, max_k + 1):
        sub, parent = split_boxes(wl.batch, k)
        Sk = sub.n_sub
        ck = BoundContext(wl.nets, precision=precision, max_sub=Sk, max_splits=16)
        dk = DeviceBatch(sub)
        aff = (f(Sk, q, ctx.n0), f(Sk, q), f(Sk, q, ctx.n0), f(Sk, q))
        cout = (f(Sk, q), f(Sk, q), torch.zeros(Sk, dtype=torch.int32, device="cuda"))

        def step_crown():
            ck.dr_bound_init(dk)
            ck.dr_propagate_backward(aff)
            ck.dr_concretize(*aff, out=cout)

        ms_k, _ = time_graph(torch, step_crown, max(2, args.steps // 10), 1)
        slb, sub_ub, sst = (t.cpu().numpy() for t in cout)
        ok = (sst & 9) == 0
        ulb = np.full((S, q), np.inf); uub = np.full((S, q), -np.inf)
        np.minimum.at(ulb, parent[ok], slb[ok]); np.maximum.at(uub, parent[ok], sub_ub[ok])
        feas = live & np.isfinite(ulb).all(axis=1)
        V_k = float(np.mean((uub - ulb).sum(axis=1)[feas]))
        curve.append(dict(k=k, sub_boxes=2 ** k, V=V_k, ms=ms_k))
        ck.close()
        del dk, aff, cout
        torch.cuda.empty_cache()
        if V_k <= V_ab:
            break
    reached = curve[-1]["V"] <= V_ab
    return dict(V_alpha_beta=V_ab, ms_alpha_beta=ms_ab, curve=curve, reached=reached,
                speedup_vs_plain_crown=(curve[-1]["ms"] / ms_ab) if reached else None)


def cpu_baseline(wl, budget_s=15.0):
    """The FP64 reference, as it stands, on a bounded sample of the headline batch."""
    from oracle import crown
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    n = 0
    t0 = time.perf_counter()
    ctxm = threadpool_limits(limits=1) if threadpool_limits else None
    try:
        while time.perf_counter() - t0 < budget_s and n < wl.batch.n_sub:
            s = n
            net = wl.nets[int(wl.batch.net_id[s])]
            crown.crown(net, wl.batch.x_center[s], wl.batch.x_radius[s], wl.batch.splits_of(s))
            n += 1
    finally:
        if ctxm is not None:
            ctxm.__exit__(None, None, None)
    dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="subdomains/s", cores=1, kind="oracle",
                sample=f"first {n} of {wl.batch.n_sub} subdomains of the headline batch, "
                       f"{dt:.1f} s wall, one thread (numpy FP64)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-extra", action="store_true", help="only the headline workload")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the bound propagation has no multi-GPU execution",
                          "n_gpus": args.gpus}))
        sys.exit(2)
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
    hl, wl = headline(torch, args, "f32")
    print(f"bench: headline {hl}", file=sys.stderr, flush=True)
    extra = {}
    if not args.no_extra:
        print("bench: f64 headline", file=sys.stderr, flush=True)
        h64, _ = headline(torch, args, "f64")
        print(f"bench: f64 headline {h64}", file=sys.stderr, flush=True)
        extra["crown_6-64x3-3_S4096_f64"] = dict(
            subdomains_per_s=h64["S"] / (h64["ms"] * 1e-3), ms_per_step=h64["ms"],
            roofline=dict(bound="mfma", achieved=h64["achieved"], peak=PEAK_TFLOPS["f64"], unit="TFLOP/s",
                          frac=h64["achieved"] / PEAK_TFLOPS["f64"]))
        print("bench: S sweep", file=sys.stderr, flush=True)
        sw = s_sweep(torch, args)
        print(f"bench: S sweep {sw}", file=sys.stderr, flush=True)
        extra["crown_6-64x3-3_S_sweep_tiled_x1_x4_x16"] = sw
        print("bench: dual ascent", file=sys.stderr, flush=True)
        da = dual_ascent(torch, args, "f32")
        print(f"bench: dual ascent {da}", file=sys.stderr, flush=True)
        extra["abcrown_8-128x4-4_S2048_20it"] = dict(
            subdomain_iters_per_s=da["subdomain_iters_per_s"], ms_per_call=da["ms"],
            roofline=dict(bound="mfma", achieved=da["tflops"], peak=PEAK_TFLOPS["f32"], unit="TFLOP/s",
                          frac=da["tflops"] / PEAK_TFLOPS["f32"]))
        print("bench: parameter gradient", file=sys.stderr, flush=True)
        pg = param_grad(torch, args, "f32")
        print(f"bench: parameter gradient {pg}", file=sys.stderr, flush=True)
        extra["param_grad_8-128x4-4_S2048"] = dict(
            subdomains_per_s=pg["subdomains_per_s"], ms_per_call=pg["ms"],
            roofline=dict(bound="mfma", achieved=pg["tflops"], peak=PEAK_TFLOPS["f32"], unit="TFLOP/s",
                          frac=pg["tflops"] / PEAK_TFLOPS["f32"]))
        print("bench: TM reach", file=sys.stderr, flush=True)
        tr = tm_reach(torch, args, "f32")
        print(f"bench: TM reach {tr}", file=sys.stderr, flush=True)
        extra["tmreach_12-256x3-4_S8192_H10"] = dict(
            box_steps_per_s=tr["box_steps_per_s"], ms_per_call=tr["ms"],
            roofline=dict(bound="mfma", achieved=tr["tflops"], peak=PEAK_TFLOPS["f32"], unit="TFLOP/s",
                          frac=tr["tflops"] / PEAK_TFLOPS["f32"]))
        print("bench: candidate reach", file=sys.stderr, flush=True)
        cr = tm_reach(torch, args, "f32", cfg=6)
        print(f"bench: candidate reach {cr}", file=sys.stderr, flush=True)
        extra["mpc_candidates_8+4-96x3-8_S4096_H10"] = dict(
            box_steps_per_s=cr["box_steps_per_s"], ms_per_call=cr["ms"],
            roofline=dict(bound="mfma", achieved=cr["tflops"], peak=PEAK_TFLOPS["f32"], unit="TFLOP/s",
                          frac=cr["tflops"] / PEAK_TFLOPS["f32"]))
        print("bench: equal tightness", file=sys.stderr, flush=True)
        extra["equal_tightness_abcrown_vs_crown_input_splitting"] = equal_tightness(torch, args, "f32")
        print(f"bench: equal tightness {extra['equal_tightness_abcrown_vs_crown_input_splitting']}", file=sys.stderr,
              flush=True)
        print("bench: mixed batch", file=sys.stderr, flush=True)
        mb = mixed_batch(torch, args, "f32")
        print(f"bench: mixed batch {mb}", file=sys.stderr, flush=True)
        extra["mixed_S16384_crown+10it"] = dict(subdomains_per_s=mb["subdomains_per_s"], ms_per_step=mb["ms"])
    print("bench: cpu baseline", file=sys.stderr, flush=True)
    cb = cpu_baseline(wl, args.cpu_budget)
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
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": hl["achieved"], "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                     "frac": hl["achieved"] / PEAK_TFLOPS["f32"],
                     "traffic": TRAFFIC["k_bound_init_bytes"] if kernel_src_sha() == TRAFFIC["src_sha"] else None,
                     "kernel": "k_bound_init", "kernel_ms": hl["bi_ms"], "flops_per_launch": hl["flops_bi"],
                     "flops_dense_rows_per_launch": hl["flops_dense"],
                     "frac_dense_rows": hl["achieved_dense"] / PEAK_TFLOPS["f32"]},
        "cpu_baseline": cb,
        "extra": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
