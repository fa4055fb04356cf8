"""FP64 reference gradient of the reach-tube volume through the stepwise TM reach.

TEST INFRASTRUCTURE ONLY (see ``oracle/crown.py``).

The paper trains with the reachability-aware loss of Section "Certified training of
neural dynamics and controllers" (and Algorithm "Training of DT Neural Dynamics"):
L_reach = mean over episodes of log(1 + V), with V the sum over steps t = 1..T_h and
state dimensions of the widths of the reachable boxes X_t computed by the DT engine
(Algorithm "Reachability of DT Dynamics"), and differentiates it with automatic
differentiation through that engine; the planner of Section "Reachability-aware MPC"
refines its top candidate by the gradient of the same kind of objective with respect to
the actions.  This module restates the stepwise TM reach of ``oracle/tm.py`` in plain
PyTorch (CPU, FP64) so that autograd gives that gradient: with respect to the network
weights and biases, the loop matrices A and B, the box centre and radius, and the
exogenous actions.  Every step follows ``oracle/tm.py`` (same readings: shared-slope
chord relaxation, CROWN rows of the IBP-unstable neurons intersected with IBP, layer 1
exact on the TM, EvalInt as the box of the TM).  Discrete choices (which neurons are
unstable, which side of an intersection or a min/max is taken, sgn at 0) are not
differentiated: the gradient is that of the piecewise-smooth bound on the piece that
contains the point, as autodiff of the engine gives it.
"""
from __future__ import annotations

import numpy as np
import torch

T64 = torch.float64


def _relax(l, u):
    """Shared-slope relaxation: slope s (chord for unstable, 1 active, 0 inactive) and
    intercept t (chord intercept -s l for unstable neurons, else 0)."""
    inactive = u <= 0
    active = (~inactive) & (l >= 0)
    uns = (~inactive) & (~active)
    den = torch.where(uns, u - l, torch.ones_like(u))
    s = torch.where(uns, u / den, torch.where(active, torch.ones_like(u), torch.zeros_like(u)))
    t = torch.where(uns, -s * l, torch.zeros_like(u))
    return s, t, uns


def _backward_shared(Ws, bs, relax, K, a):
    """Rows a on z_K back to the input with the shared-slope relaxation: (w, acc_lo, acc_hi)."""
    acc_lo = a @ bs[K - 1]
    acc_hi = acc_lo
    g = a @ Ws[K - 1]
    for k in range(K - 1, 0, -1):
        s, t, uns = relax[k - 1]
        gt = torch.where(uns, g * t, torch.zeros_like(g))
        zero = torch.zeros_like(gt)
        acc_lo = acc_lo + torch.where(gt < 0, gt, zero).sum(dim=1)
        acc_hi = acc_hi + torch.where(gt > 0, gt, zero).sum(dim=1)
        a = s * g
        acc_lo = acc_lo + a @ bs[k - 1]
        acc_hi = acc_hi + a @ bs[k - 1]
        g = a @ Ws[k - 1]
    return g, acc_lo, acc_hi


def _interval_dot(w, Ilo, Ihi):
    """Range of w . r over r in [Ilo, Ihi] (rows of w), the end chosen by the sign of w."""
    pos = w >= 0
    a, b = w * Ilo, w * Ihi
    return torch.where(pos, a, b).sum(dim=1), torch.where(pos, b, a).sum(dim=1)


def _tm_eval(w, acc_lo, acc_hi, c, P, Ilo, Ihi):
    base = w @ c
    rad = (w @ P).abs().sum(dim=1)
    rl, rh = _interval_dot(w, Ilo, Ihi)
    return acc_lo + base - rad + rl, acc_hi + base + rad + rh


def _ibp(W, b, l, u):
    zero = torch.zeros_like(l)
    lo, hi = torch.where(l > 0, l, zero), torch.where(u > 0, u, zero)
    c, r = 0.5 * (lo + hi), 0.5 * (hi - lo)
    zc = W @ c + b
    zr = W.abs() @ r
    return zc - zr, zc + zr


def _step(Ws, bs, A, B, c, P, Ilo, Ihi):
    L = len(Ws)
    l, u = _tm_eval(Ws[0], bs[0], bs[0], c, P, Ilo, Ihi)
    bounds = [(l, u)]
    for k in range(2, L):
        li, ui = _ibp(Ws[k - 1], bs[k - 1], *bounds[-1])
        U = torch.nonzero((li < 0) & (ui > 0)).flatten()
        l, u = li, ui
        if U.numel():
            relax = [_relax(*bk) for bk in bounds]
            E = torch.zeros(U.numel(), Ws[k - 1].shape[0], dtype=T64)
            E[torch.arange(U.numel()), U] = 1.0
            w, alo, ahi = _backward_shared(Ws, bs, relax, k, E)
            lo, hi = _tm_eval(w, alo, ahi, c, P, Ilo, Ihi)
            # the interval bound is kept on ties
            l = l.index_put((U,), torch.where(lo > li[U], lo, li[U]))
            u = u.index_put((U,), torch.where(hi < ui[U], hi, ui[U]))
        bounds.append((l, u))
    relax = [_relax(*bk) for bk in bounds]
    w, alo, ahi = _backward_shared(Ws, bs, relax, L, B)
    W = A + w
    rl, rh = _interval_dot(W, Ilo, Ihi)
    return W @ c, W @ P, rl + alo, rh + ahi


def reach_volume(Ws, bs, A, B, xc, xr, horizon, u=None):
    """Tube volume V = sum_{t=1..H} sum_j width(X_t) of the stepwise TM reach from the
    box [xc - xr, xc + xr] (torch FP64 tensors; gradients flow to every argument), and
    the boxes (H+1 x n x 2)."""
    n = A.shape[0]
    m = Ws[0].shape[1] - n
    c, P = xc[:n], torch.diag(xr[:n])
    Ilo = torch.zeros(n, dtype=T64)
    Ihi = torch.zeros(n, dtype=T64)
    boxes = [torch.stack([c - xr[:n], c + xr[:n]], dim=1)]
    V = torch.zeros((), dtype=T64)
    for t in range(horizon):
        if m:
            cv = torch.cat([c, u[t]])
            Pv = torch.cat([P, torch.zeros(m, n, dtype=T64)], dim=0)
            Iv_lo = torch.cat([Ilo, torch.zeros(m, dtype=T64)])
            Iv_hi = torch.cat([Ihi, torch.zeros(m, dtype=T64)])
        else:
            cv, Pv, Iv_lo, Iv_hi = c, P, Ilo, Ihi
        c, P, Ilo, Ihi = _step(Ws, bs, A, B, cv, Pv, Iv_lo, Iv_hi)
        rad = P.abs().sum(dim=1)
        lo, hi = c - rad + Ilo, c + rad + Ihi
        boxes.append(torch.stack([lo, hi], dim=1))
        V = V + (hi - lo).sum()
    return V, torch.stack(boxes)


def volume_gradient(net, xc, xr, horizon, u=None):
    """V and dV/d(W_k, b_k, A, B, xc, xr, u) (numpy FP64) for one box."""
    Ws = [torch.tensor(W, dtype=T64, requires_grad=True) for W in net.Ws]
    bs = [torch.tensor(b, dtype=T64, requires_grad=True) for b in net.bs]
    A = torch.tensor(net.A, dtype=T64, requires_grad=True)
    B = torch.tensor(net.B, dtype=T64, requires_grad=True)
    n = net.A.shape[0]
    xct = torch.tensor(np.asarray(xc, np.float64)[:n], requires_grad=True)
    xrt = torch.tensor(np.asarray(xr, np.float64)[:n], requires_grad=True)
    ut = torch.tensor(np.asarray(u, np.float64), requires_grad=True) if u is not None else None
    V, boxes = reach_volume(Ws, bs, A, B, xct, xrt, horizon, ut)
    params = Ws + bs + [A, B, xct, xrt] + ([ut] if ut is not None else [])
    grads = torch.autograd.grad(V, params, allow_unused=True)
    g = [np.zeros(p.shape) if gi is None else gi.numpy() for p, gi in zip(params, grads)]
    L = len(Ws)
    out = dict(V=float(V.detach()), boxes=boxes.detach().numpy(), dW=g[:L], db=g[L:2 * L], dA=g[2 * L], dB=g[2 * L + 1],
               dxc=g[2 * L + 2], dxr=g[2 * L + 3])
    out["du"] = g[2 * L + 4] if ut is not None else None
    return out
