"""Python front end of the C-ABI, with torch tensors as device memory.

Nothing here computes bounds: the class marshals tensors into the C structs and
calls the entry points of libdiffreach.so under the same names.  Every call is
asynchronous on torch's current stream.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import binding as B
from .workloads import Batch, Network, pack_splits


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class DeviceBatch:
    """A batch of subdomains resident in device memory."""

    def __init__(self, batch: Batch, device="cuda"):
        self.n_sub = batch.n_sub
        self.x_center = torch.as_tensor(batch.x_center, dtype=torch.float64, device=device).contiguous()
        self.x_radius = torch.as_tensor(batch.x_radius, dtype=torch.float64, device=device).contiguous()
        self.net_id = torch.as_tensor(batch.net_id, dtype=torch.int32, device=device).contiguous()
        if batch.split_layer.size > 0 or np.any(batch.split_ptr):
            self.split_ptr = torch.as_tensor(batch.split_ptr, dtype=torch.int32, device=device).contiguous()
            words = pack_splits(batch.split_layer, batch.split_neuron, batch.split_sign).astype(np.int64)
            self.split_packed = torch.as_tensor(words.astype(np.uint32).view(np.int32), device=device).contiguous()
        else:
            self.split_ptr = None
            self.split_packed = None
        self.max_splits = int(np.max(np.diff(batch.split_ptr))) if batch.n_sub else 0

    @classmethod
    def from_tensors(cls, x_center: torch.Tensor, x_radius: torch.Tensor):
        """A batch of boxes without splits from FP64 device tensors (S x n_0)."""
        self = cls.__new__(cls)
        self.n_sub = int(x_center.shape[0])
        self.x_center = x_center.detach().to(torch.float64).contiguous()
        self.x_radius = x_radius.detach().to(torch.float64).contiguous()
        self.net_id = torch.zeros(max(self.n_sub, 1), dtype=torch.int32, device=self.x_center.device)
        self.split_ptr = None
        self.split_packed = None
        self.max_splits = 0
        return self

    def struct(self) -> B.dr_batch:
        b = B.dr_batch()
        b.n_sub = self.n_sub
        b.net_id = self.net_id.data_ptr()
        b.x_center = self.x_center.data_ptr()
        b.x_radius = self.x_radius.data_ptr()
        b.split_ptr = self.split_ptr.data_ptr() if self.split_ptr is not None else None
        b.split_packed = self.split_packed.data_ptr() if self.split_packed is not None else None
        return b


class CtField:
    """A polynomial vector field f_i(x, u) = a_i + F_i x + G_i u + x^T Q_i x resident in
    device memory (FP64), for dr_flowpipe_ct and dr_reach_ct."""

    def __init__(self, a, F, G=None, Q=None, device="cuda"):
        f64 = lambda v: torch.as_tensor(np.asarray(v, np.float64), dtype=torch.float64, device=device).contiguous()
        self.a, self.F = f64(a), f64(F)
        self.n = int(self.F.shape[0])
        self.G = f64(G) if G is not None and np.asarray(G).size else None
        self.n_u = int(self.G.shape[1]) if self.G is not None else 0
        self.Q = f64(Q) if Q is not None and np.any(np.asarray(Q)) else None

    @classmethod
    def from_dynamics(cls, f, device="cuda"):
        """From an object with attributes a, F, G, Q (G n x n_u, Q n x n x n)."""
        return cls(f.a, f.F, getattr(f, "G", None), getattr(f, "Q", None), device=device)

    def struct(self) -> B.dr_ct_field:
        s = B.dr_ct_field()
        s.n, s.n_u = self.n, self.n_u
        s.a, s.F = self.a.data_ptr(), self.F.data_ptr()
        s.G = self.G.data_ptr() if self.G is not None else None
        s.Q = self.Q.data_ptr() if self.Q is not None else None
        return s


def ct_options(h, steps, intervals=1, tries=40, rounds=3, eps=1e-9) -> B.dr_ct_options:
    o = B.dr_ct_options()
    o.h, o.steps, o.intervals, o.tries, o.rounds, o.eps = float(h), int(steps), int(intervals), int(tries), int(rounds), float(eps)
    return o


def _ct_out(S, N, n, segments, dev, out):
    if out is not None:
        return out
    boxes = torch.empty(S, N + 1, n, 2, dtype=torch.float64, device=dev)
    segs = torch.empty(S, N, n, 2, dtype=torch.float64, device=dev) if segments else None
    return boxes, segs, torch.zeros(max(S, 1), dtype=torch.int32, device=dev)


def dr_flowpipe_ct(field: CtField, x_center, x_radius, h, steps, intervals=1, segments=True, out=None, **kw):
    """Flowpipe of x' = f(x) from the boxes [x_center - x_radius, x_center + x_radius]
    (S x n): returns (boxes S x (N K + 1) x n x 2, segments S x N K x n x 2 or None,
    status S); `out` may give those three tensors."""
    lib = B.load()
    dev = field.F.device
    xc = torch.as_tensor(x_center, dtype=torch.float64, device=dev).contiguous()
    xr = torch.as_tensor(x_radius, dtype=torch.float64, device=dev).contiguous()
    S, n = int(xc.shape[0]), field.n
    N = int(steps) * int(intervals)
    boxes, segs, status = _ct_out(S, N, n, segments, dev, out)
    fs, o = field.struct(), ct_options(h, steps, intervals, **kw)
    B.check(lib.dr_flowpipe_ct(ctypes.byref(fs), ctypes.byref(o), S, _ptr(xc), _ptr(xr), _ptr(boxes), _ptr(segs),
                               _ptr(status), _stream()), None)
    return boxes, segs, status[:S]


class BoundContext:
    """dr_create + the per-batch entry points, holding the device copies of the
    networks and the output tensors."""

    def __init__(self, nets: Sequence[Network], *, precision="f32", max_sub=1, max_splits=0,
                 intermediate="crown_ibp", tile_cfg=0, spec: Optional[np.ndarray] = None, device="cuda",
                 margins=True, fuse_spec=True):
        self.lib = B.load()
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.precision = precision
        wdt = torch.float32 if precision == "f32" else torch.float64
        self._keep = []
        structs = (B.dr_network * len(nets))()
        for i, net in enumerate(nets):
            L = net.n_layers
            widths = (ctypes.c_int * (L + 1))(*net.widths)
            Ws = [torch.as_tensor(W, dtype=wdt, device=self.device).contiguous() for W in net.Ws]
            bs = [torch.as_tensor(b, dtype=wdt, device=self.device).contiguous() for b in net.bs]
            Wp = (ctypes.c_void_p * L)(*[W.data_ptr() for W in Ws])
            bp = (ctypes.c_void_p * L)(*[b.data_ptr() for b in bs])
            nw = structs[i]
            nw.n_layers = L
            nw.widths = widths
            nw.wdtype = B.DR_DTYPE_F32 if precision == "f32" else B.DR_DTYPE_F64
            nw.W = Wp
            nw.b = bp
            keep = [widths, Ws, bs, Wp, bp]
            if net.closed_loop:
                A = torch.as_tensor(net.A, dtype=torch.float64, device=self.device).contiguous()
                Bm = torch.as_tensor(net.B, dtype=torch.float64, device=self.device).contiguous()
                nw.A, nw.B, nw.n_state = A.data_ptr(), Bm.data_ptr(), net.A.shape[0]
                keep += [A, Bm]
            if spec is not None:
                C = torch.as_tensor(np.asarray(spec), dtype=torch.float64, device=self.device).contiguous()
                nw.spec, nw.n_spec = C.data_ptr(), C.shape[0]
                keep.append(C)
            self._keep.append(keep)
        self._structs = structs
        opt = B.dr_options()
        opt.precision = B.DR_PREC_F32 if precision == "f32" else B.DR_PREC_F64
        opt.intermediate = B.DR_INTER_CROWN_IBP if intermediate == "crown_ibp" else B.DR_INTER_IBP
        opt.max_sub = max_sub
        opt.max_splits = max_splits
        if tile_cfg == "auto":
            # the autotuner's choice for these network shapes (defaults when not tuned)
            from .autotune import lookup
            tile_cfg, fuse_spec = lookup(nets, precision)
        opt.tile_cfg = int(tile_cfg)
        opt.margin_mode = B.DR_MARGIN_RIGOROUS if margins else B.DR_MARGIN_OFF
        opt.fuse_spec = 1 if fuse_spec else 0
        self.tile_cfg, self.fuse_spec = int(tile_cfg), bool(fuse_spec)
        ctx = ctypes.c_void_p()
        st = self.lib.dr_create(ctypes.byref(ctx), structs, len(nets), ctypes.byref(opt), _stream())
        B.check(st, None)
        self.ctx = ctx
        self.n0 = nets[0].widths[0]
        self.widths = list(nets[0].widths)
        self.n_state = nets[0].A.shape[0] if nets[0].closed_loop else 0
        self.R = self.lib.dr_spec_rows(ctx)
        self.q = self.R // 2
        self.H_max = self.lib.dr_hidden_max(ctx)
        self.max_splits = max_splits
        self.n_layers = max(n.n_layers for n in nets)
        self.batch: Optional[DeviceBatch] = None
        # bumped by every call that replaces the state later calls read (the batch, its
        # relaxation or the weights), so holders of that state can tell it is stale
        self.generation = 0

    def close(self):
        if getattr(self, "ctx", None) is not None:
            self.lib.dr_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        B.check(st, self.ctx)

    # ---- entry points ---------------------------------------------------------------
    def dr_bound_init(self, batch: DeviceBatch, status=None) -> torch.Tensor:
        """a1-a4 for the batch; returns the per-subdomain status (every entry is written)."""
        self.batch = batch
        self.generation += 1
        if status is None:
            status = torch.empty(max(batch.n_sub, 1), dtype=torch.int32, device=self.device)
        b = batch.struct()
        self._batch_struct = b
        self._check(self.lib.dr_bound_init(self.ctx, ctypes.byref(b), _ptr(status), _stream()))
        return status[: batch.n_sub]

    def dr_propagate_backward(self, out=None):
        S, q, n0 = self.batch.n_sub, self.q, self.n0
        if out is None:
            f = lambda *s: torch.empty(*s, dtype=torch.float64, device=self.device)
            out = (f(S, q, n0), f(S, q), f(S, q, n0), f(S, q))
        lam_lo, acc_lo, lam_hi, acc_hi = out
        self._check(self.lib.dr_propagate_backward(self.ctx, _ptr(lam_lo), _ptr(acc_lo), _ptr(lam_hi),
                                                   _ptr(acc_hi), _stream()))
        return out

    def dr_concretize(self, lam_lo, acc_lo, lam_hi, acc_hi, out=None):
        S, q = self.batch.n_sub, self.q
        if out is None:
            out = (torch.empty(S, q, dtype=torch.float64, device=self.device),
                   torch.empty(S, q, dtype=torch.float64, device=self.device),
                   torch.zeros(max(S, 1), dtype=torch.int32, device=self.device))
        lb, ub, status = out
        self._check(self.lib.dr_concretize(self.ctx, _ptr(lam_lo), _ptr(acc_lo), _ptr(lam_hi), _ptr(acc_hi),
                                           _ptr(lb), _ptr(ub), _ptr(status), _stream()))
        return lb, ub, status[:S]

    def new_duals(self):
        S, R = self.batch.n_sub, self.R
        alpha = torch.zeros(S, R, max(self.H_max, 1), dtype=torch.float32, device=self.device)
        beta = torch.zeros(S, R, max(self.max_splits, 1), dtype=torch.float32, device=self.device)
        return alpha, beta

    def _check_duals(self, alpha, beta):
        """alpha: S x R x max(H_max, 1), beta: S x R x max(max_splits, 1), both contiguous
        FP32 on this context's device (the kernels index them with these strides)."""
        if self.batch is None:
            raise RuntimeError("dr_bound_init has not been called")
        S, R = self.batch.n_sub, self.R
        for name, t, cols in (("alpha", alpha, max(self.H_max, 1)), ("beta", beta, max(self.max_splits, 1))):
            if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.device != self.device:
                raise ValueError(f"{name} must be a float32 tensor on {self.device}")
            if tuple(t.shape) != (S, R, cols) or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {S} x {R} x {cols} tensor, got {tuple(t.shape)}")

    def _check_rows(self, name, t):
        S, q = self.batch.n_sub, self.q
        if tuple(t.shape) != (S, q):
            raise ValueError(f"{name} must be {S} x {q}, got {tuple(t.shape)}")

    def dr_optimize_duals(self, iters, lr, alpha, beta, init_duals=True, grads=False, out=None):
        self._check_duals(alpha, beta)
        S, q = self.batch.n_sub, self.q
        if out is None:
            out = (torch.empty(S, q, dtype=torch.float64, device=self.device),
                   torch.empty(S, q, dtype=torch.float64, device=self.device),
                   torch.zeros(max(S, 1), dtype=torch.int32, device=self.device))
        lb, ub, status = out
        ga = torch.zeros_like(alpha) if grads else None
        gb = torch.zeros_like(beta) if grads else None
        self._check(self.lib.dr_optimize_duals(self.ctx, int(iters), float(lr), int(bool(init_duals)), _ptr(alpha),
                                               _ptr(beta), _ptr(lb), _ptr(ub), _ptr(ga), _ptr(gb), _ptr(status),
                                               _stream()))
        return lb, ub, status[:S], ga, gb

    def param_grad_outputs(self):
        """Output tensors of dr_param_grad for the current batch and its workspace."""
        S, q = self.batch.n_sub, self.q
        f = lambda *s: torch.empty(*s, dtype=torch.float64, device=self.device)
        dW = [f(n_out, n_in) for n_in, n_out in zip(self.widths[:-1], self.widths[1:])]
        db = [f(n_out) for n_out in self.widths[1:]]
        status = torch.zeros(max(S, 1), dtype=torch.int32, device=self.device)
        out = (f(S, q), f(S, q), dW, db, f(max(S, 1), self.n0), f(max(S, 1), self.n0), status)
        nbytes = int(self.lib.dr_param_grad_workspace(self.ctx, S))
        return out, torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)

    def dr_param_grad(self, alpha, beta, g_lb, g_ub, init_duals=False, out=None, workspace=None):
        """Weighted gradient of the bounds w.r.t. weights, biases and boxes at a fixed
        relaxation.  Returns (lb, ub, dW list, db list, dxc, dxr, status); dW[k-1] is
        n_k x n_{k-1} FP64."""
        self._check_duals(alpha, beta)
        S = self.batch.n_sub
        if out is None or workspace is None:
            out2, ws2 = self.param_grad_outputs()
            out = out if out is not None else out2
            workspace = workspace if workspace is not None else ws2
        lb, ub, dW, db, dxc, dxr, status = out
        g_lb = torch.as_tensor(g_lb, dtype=torch.float64, device=self.device).contiguous()
        g_ub = torch.as_tensor(g_ub, dtype=torch.float64, device=self.device).contiguous()
        self._check_rows("g_lb", g_lb)
        self._check_rows("g_ub", g_ub)
        self._pg_keep = (g_lb, g_ub)
        Wp = (ctypes.c_void_p * len(dW))(*[t.data_ptr() for t in dW])
        bp = (ctypes.c_void_p * len(db))(*[t.data_ptr() for t in db])
        self._check(self.lib.dr_param_grad(self.ctx, _ptr(alpha), _ptr(beta), int(bool(init_duals)), _ptr(g_lb),
                                           _ptr(g_ub), _ptr(lb), _ptr(ub), Wp, bp, _ptr(dxc), _ptr(dxr),
                                           _ptr(workspace), ctypes.c_size_t(workspace.numel()), _ptr(status),
                                           _stream()))
        return lb, ub, dW, db, dxc[:S], dxr[:S], status[:S]

    def dr_param_grad_static(self, alpha, beta, g_lb, g_ub, init_duals=False, out=None):
        """dr_param_grad with the library's static scratch instead of a workspace (the
        entry point that allocates nothing; the outputs are the caller's)."""
        self._check_duals(alpha, beta)
        S = self.batch.n_sub
        if out is None:
            out, _ = self.param_grad_outputs()
        lb, ub, dW, db, dxc, dxr, status = out
        g_lb = torch.as_tensor(g_lb, dtype=torch.float64, device=self.device).contiguous()
        g_ub = torch.as_tensor(g_ub, dtype=torch.float64, device=self.device).contiguous()
        self._check_rows("g_lb", g_lb)
        self._check_rows("g_ub", g_ub)
        self._pg_keep = (g_lb, g_ub)
        Wp = (ctypes.c_void_p * len(dW))(*[t.data_ptr() for t in dW])
        bp = (ctypes.c_void_p * len(db))(*[t.data_ptr() for t in db])
        self._check(self.lib.dr_param_grad_static(self.ctx, _ptr(alpha), _ptr(beta), int(bool(init_duals)),
                                                  _ptr(g_lb), _ptr(g_ub), _ptr(lb), _ptr(ub), Wp, bp, _ptr(dxc),
                                                  _ptr(dxr), _ptr(status), _stream()))
        return lb, ub, dW, db, dxc[:S], dxr[:S], status[:S]

    def dr_reach_dt(self, batch: DeviceBatch, horizon: int, boxes=None, u=None):
        """Stepwise reach; ``u`` (S x horizon x (n_0 - n_state), FP64 device) selects
        dr_reach_dt_exo for networks with exogenous inputs."""
        self.batch = batch
        self.generation += 1
        S = batch.n_sub
        if boxes is None:
            boxes = torch.empty(S, horizon + 1, max(self.n_state, 1), 2, dtype=torch.float64, device=self.device)
        status = torch.zeros(max(S, 1), dtype=torch.int32, device=self.device)
        b = batch.struct()
        self._batch_struct = b
        if u is None:
            self._check(self.lib.dr_reach_dt(self.ctx, ctypes.byref(b), int(horizon), _ptr(boxes), _ptr(status),
                                             _stream()))
        else:
            u = torch.as_tensor(u, dtype=torch.float64, device=self.device).contiguous()
            self._u = u
            self._check(self.lib.dr_reach_dt_exo(self.ctx, ctypes.byref(b), int(horizon), _ptr(u), _ptr(boxes),
                                                 _ptr(status), _stream()))
        return boxes, status[:S]

    def dr_reach_dt_joint(self, batch: DeviceBatch, horizon: int, boxes=None, u=None, rows=None):
        """CROWN through the closed loop unrolled over the horizon; returns (boxes,
        status, rows) with rows S x horizon x 8 (CROWN rows per hidden layer and step)."""
        self.batch = batch
        self.generation += 1
        S = batch.n_sub
        if boxes is None:
            boxes = torch.empty(S, horizon + 1, max(self.n_state, 1), 2, dtype=torch.float64, device=self.device)
        if rows is None:
            rows = torch.zeros(max(S, 1), max(horizon, 1), 8, dtype=torch.int32, device=self.device)
        status = torch.zeros(max(S, 1), dtype=torch.int32, device=self.device)
        if u is not None:
            u = torch.as_tensor(u, dtype=torch.float64, device=self.device).contiguous()
            self._u = u
        b = batch.struct()
        self._batch_struct = b
        self._check(self.lib.dr_reach_dt_joint(self.ctx, ctypes.byref(b), int(horizon), _ptr(u) if u is not None else None,
                                               _ptr(boxes), _ptr(rows), _ptr(status), _stream()))
        return boxes, status[:S], rows[:S]

    def dr_reach_dt_grad(self, batch: DeviceBatch, horizon: int, g_V, u=None, boxes=None, workspace=None,
                         want=("du", "dxc", "dxr", "dA", "dB", "dW", "db")):
        """Reach (boxes) and the gradient of J = sum_s g_V[s] V_s: returns (boxes, status,
        grads) with grads a dict of the requested FP64 device tensors among du, dxc, dxr,
        dA, dB, and the lists dW, db (one tensor per layer)."""
        self.batch = batch
        self.generation += 1
        S = batch.n_sub
        ns = max(self.n_state, 1)
        dev = self.device
        f64 = lambda *sh: torch.zeros(*sh, dtype=torch.float64, device=dev)
        if boxes is None:
            boxes = f64(S, horizon + 1, ns, 2)
        g_V = torch.as_tensor(g_V, dtype=torch.float64, device=dev).contiguous()
        if g_V.shape != (S,):
            raise ValueError(f"g_V must have shape ({S},)")
        if u is not None:
            u = torch.as_tensor(u, dtype=torch.float64, device=dev).contiguous()
            self._u = u
        nx = self.n0 - self.n_state
        shapes = dict(du=(max(S, 1), max(horizon, 1), max(nx, 1)), dxc=(max(S, 1), ns), dxr=(max(S, 1), ns),
                      dA=(ns, self.n0), dB=(ns, self.widths[-1]))
        grads = {k: f64(*shapes[k]) for k in want if k in shapes and not (k == "du" and nx == 0)}
        L = len(self.widths) - 1
        dWp = dbp = None
        if "dW" in want:
            grads["dW"] = [f64(self.widths[k + 1], self.widths[k]) for k in range(L)]
            dWp = (ctypes.c_void_p * L)(*[t.data_ptr() for t in grads["dW"]])
        if "db" in want:
            grads["db"] = [f64(self.widths[k + 1]) for k in range(L)]
            dbp = (ctypes.c_void_p * L)(*[t.data_ptr() for t in grads["db"]])
        self._wptrs = (dWp, dbp)
        need = int(self.lib.dr_reach_grad_workspace(self.ctx, S, int(horizon)))
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        self._ws = workspace
        status = torch.zeros(max(S, 1), dtype=torch.int32, device=dev)
        b = batch.struct()
        self._batch_struct = b
        self._check(self.lib.dr_reach_dt_grad(
            self.ctx, ctypes.byref(b), int(horizon), _ptr(u), _ptr(g_V), _ptr(boxes), _ptr(grads.get("du")),
            _ptr(grads.get("dxc")), _ptr(grads.get("dxr")), _ptr(grads.get("dA")), _ptr(grads.get("dB")),
            dWp, dbp, _ptr(workspace), ctypes.c_size_t(workspace.numel()), _ptr(status), _stream()))
        return boxes, status[:S], grads

    def dr_reach_ct(self, field: CtField, batch: DeviceBatch, h, steps, intervals, segments=True, out=None, **kw):
        """CT closed loop with this context's network as the controller (held over each
        control interval of `steps` flowpipe steps): returns (boxes, segments, status)
        as dr_flowpipe_ct."""
        self.batch = batch
        self.generation += 1
        S, n = batch.n_sub, field.n
        N = int(steps) * int(intervals)
        boxes, segs, status = _ct_out(S, N, n, segments, self.device, out)
        fs, o = field.struct(), ct_options(h, steps, intervals, **kw)
        b = batch.struct()
        self._batch_struct = b
        self._check(self.lib.dr_reach_ct(self.ctx, ctypes.byref(fs), ctypes.byref(o), ctypes.byref(b), _ptr(boxes),
                                         _ptr(segs), _ptr(status), _stream()))
        return boxes, segs, status[:S]

    def dr_get_bounds(self):
        S = self.batch.n_sub
        l = torch.empty(S, max(self.H_max, 1), dtype=torch.float64, device=self.device)
        u = torch.empty_like(l)
        self._check(self.lib.dr_get_bounds(self.ctx, _ptr(l), _ptr(u), _stream()))
        return l, u

    def dr_get_rows(self):
        rows = torch.zeros(self.batch.n_sub, 8, dtype=torch.int32, device=self.device)
        self._check(self.lib.dr_get_rows(self.ctx, _ptr(rows), _stream()))
        return rows

    def dr_get_margins(self):
        m = torch.zeros(self.batch.n_sub, self.R, dtype=torch.float64, device=self.device)
        self._check(self.lib.dr_get_margins(self.ctx, _ptr(m), _stream()))
        return m

    def dr_set_weights(self, net_index, Ws, bs):
        """Replace network ``net_index``'s weights and biases (device tensors of the same
        shapes, or arrays) in place; A, B and the spec stay those of creation."""
        wdt = torch.float32 if self.precision == "f32" else torch.float64
        Ws = [torch.as_tensor(W, device=self.device).to(wdt).contiguous() for W in Ws]
        bs = [torch.as_tensor(b, device=self.device).to(wdt).contiguous() for b in bs]
        old = self._structs[net_index]
        nw = B.dr_network()
        nw.n_layers = old.n_layers
        nw.widths = old.widths
        nw.wdtype = B.DR_DTYPE_F32 if self.precision == "f32" else B.DR_DTYPE_F64
        Wp = (ctypes.c_void_p * len(Ws))(*[W.data_ptr() for W in Ws])
        bp = (ctypes.c_void_p * len(bs))(*[b.data_ptr() for b in bs])
        nw.W, nw.b = Wp, bp
        self._keep_weights = (Ws, bs, Wp, bp)   # read by kernels queued on the stream
        self._check(self.lib.dr_set_weights(self.ctx, int(net_index), ctypes.byref(nw), _stream()))
        self.generation += 1

    # ---- conveniences ----------------------------------------------------------------
    def crown(self, batch: DeviceBatch):
        """a1-a6 for a batch: plain CROWN lower/upper bounds and status."""
        self.dr_bound_init(batch)
        aff = self.dr_propagate_backward()
        lb, ub, status = self.dr_concretize(*aff)
        return lb, ub, status, aff


class DualBound(torch.autograd.Function):
    """Bound of every spec row as a differentiable function of (alpha, beta).

    forward: lower and upper bounds (S x q each) at the given duals, via
    dr_optimize_duals with iters = 0; backward: the hand-written adjoint's
    gradients of each row, scaled by the incoming gradient (rows are separable:
    lower rows use alpha[:, :q], upper rows alpha[:, q:], and ub = -lb_row)."""

    @staticmethod
    def forward(ctx_, alpha, beta, bctx: BoundContext):
        a = alpha.detach().clone().contiguous()
        b = beta.detach().clone().contiguous()
        lb, ub, status, ga, gb = bctx.dr_optimize_duals(0, 0.0, a, b, init_duals=False, grads=True)
        ctx_.save_for_backward(ga, gb)
        ctx_.q = bctx.q
        return lb, ub

    @staticmethod
    def backward(ctx_, g_lb, g_ub):
        ga, gb = ctx_.saved_tensors
        q = ctx_.q
        w = torch.cat([g_lb, -g_ub], dim=1).to(ga.dtype)     # d ub = - d lb_row
        return ga * w[:, :, None], gb * w[:, :, None], None


class CrownBounds(torch.autograd.Function):
    """Plain-CROWN bounds of a batch (lb, ub: S x q) as a differentiable function of a
    single-network context's weights and biases.

    forward: dr_set_weights, dr_bound_init, and the bound at the adaptive slopes;
    backward: dr_param_grad with the incoming gradients as row weights, i.e. the
    gradient at a fixed relaxation (the intermediate bounds and slopes of the forward
    pass are constants).  The backward pass reads the context's state, so a context
    serves one pending forward at a time: a backward after a later forward (or any call
    that replaces the batch or the weights) on the same context raises RuntimeError."""

    @staticmethod
    def forward(ctx_, bctx: BoundContext, batch: DeviceBatch, *params):
        L = len(params) // 2
        Ws, bs = params[:L], params[L:]
        bctx.dr_set_weights(0, [W.detach() for W in Ws], [b.detach() for b in bs])
        bctx.dr_bound_init(batch)
        alpha, beta = bctx.new_duals()
        lb, ub, _, _, _ = bctx.dr_optimize_duals(0, 0.0, alpha, beta, init_duals=True)
        ctx_.bctx, ctx_.duals = bctx, (alpha, beta)
        ctx_.generation = bctx.generation
        ctx_.dtypes = [p.dtype for p in params]
        return lb, ub

    @staticmethod
    def backward(ctx_, g_lb, g_ub):
        bctx = ctx_.bctx
        if bctx.generation != ctx_.generation:
            # the backward pass differentiates the context's current relaxation and weights:
            # another forward (or a weight or batch change) on the same context replaced them
            raise RuntimeError("CrownBounds.backward: the context's state changed after this forward "
                               "(another forward, dr_bound_init, dr_set_weights or dr_reach_dt ran on it); "
                               "use one BoundContext per pending forward")
        alpha, beta = ctx_.duals
        g_lb = torch.zeros_like(g_lb) if g_lb is None else g_lb
        g_ub = torch.zeros_like(g_ub) if g_ub is None else g_ub
        _, _, dW, db, _, _, _ = bctx.dr_param_grad(alpha, beta, g_lb.contiguous(), g_ub.contiguous(),
                                                   init_duals=False)
        grads = [g.to(dt) for g, dt in zip(list(dW) + list(db), ctx_.dtypes)]
        return (None, None, *grads)


class ReachVolume(torch.autograd.Function):
    """Tube volume V_s (sum over steps 1..H and states of the widths of the reachable
    boxes of the stepwise reach) of every box, as a differentiable function of the box
    centres and radii (S x n_0: entries n_state.. of an exogenous network are ignored),
    the action sequences u (S x H x (n_0 - n_state), or None) and a single-network
    closed-loop context's weights and biases: the reachability-aware loss of the paper is
    mean(log(1 + V)).

    forward: dr_set_weights and the reach (dr_reach_dt / dr_reach_dt_exo);
    backward: dr_reach_dt_grad with g_V = the incoming gradient (the reverse pass
    through every step, intermediate bounds included).  The backward pass reruns the
    reach with the weights set at forward time; like CrownBounds it refuses a context
    whose state a later call replaced."""

    @staticmethod
    def forward(ctx_, bctx: BoundContext, x_center, x_radius, u, horizon: int, *params):
        L = len(params) // 2
        Ws, bs = params[:L], params[L:]
        bctx.dr_set_weights(0, [W.detach() for W in Ws], [b.detach() for b in bs])
        batch = DeviceBatch.from_tensors(x_center, x_radius)
        ud = u.detach().to(torch.float64).contiguous() if u is not None else None
        boxes, _ = bctx.dr_reach_dt(batch, horizon, u=ud)
        V = (boxes[:, 1:, :, 1] - boxes[:, 1:, :, 0]).sum(dim=(1, 2))
        ctx_.bctx, ctx_.batch, ctx_.u, ctx_.horizon = bctx, batch, ud, horizon
        ctx_.generation = bctx.generation
        ctx_.shapes = (x_center.shape, x_radius.shape, None if u is None else u.shape)
        ctx_.dtypes = [p.dtype for p in params]
        return V

    @staticmethod
    def backward(ctx_, g_V):
        bctx = ctx_.bctx
        if bctx.generation != ctx_.generation:
            raise RuntimeError("ReachVolume.backward: the context's state changed after this forward; "
                               "use one BoundContext per pending forward")
        _, _, g = bctx.dr_reach_dt_grad(ctx_.batch, ctx_.horizon, g_V.detach().contiguous(), u=ctx_.u,
                                        want=("du", "dxc", "dxr", "dW", "db"))
        bctx.generation = ctx_.generation      # the rerun reproduces the forward's state
        xs, rs, us = ctx_.shapes
        ns = bctx.n_state
        dxc = torch.zeros(xs, dtype=torch.float64, device=bctx.device)
        dxr = torch.zeros(rs, dtype=torch.float64, device=bctx.device)
        dxc[:, :ns] = g["dxc"][: xs[0]]
        dxr[:, :ns] = g["dxr"][: rs[0]]
        du = g["du"][: us[0], : us[1]].reshape(us) if us is not None else None
        grads = [t.to(dt) for t, dt in zip(list(g["dW"]) + list(g["db"]), ctx_.dtypes)]
        return (None, dxc, dxr, du, None, *grads)

