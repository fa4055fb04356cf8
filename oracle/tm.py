"""FP64 reference for stepwise closed-loop reachability with linear Taylor models.

TEST INFRASTRUCTURE ONLY (see ``oracle/crown.py``).

Follows the paper's Algorithm "Reachability of DT Dynamics" with the TM--CROWN
interface of Theorem "CROWN bounds of NN with linear TM input" and its proof in
the appendix on CT neural dynamics:

* the initial box is normalised to a linear TM  x = c + P z (+ r),  z in [-1,1]^n,
  r in I,  with c the box centre, P = diag(half-width), I = [0, 0] (the
  normalisation step of the appendix algorithm for CT flowpipes);
* each step applies CROWN to the reparameterised network f(c + P z + r) over the
  box (z, r) in [-1,1]^n x I with the shared-slope constraint (the lower and upper
  affine bounds have one common linear term), so the controller output is again a
  linear TM;
* the closed loop x' = A x + B y is composed in TM arithmetic: the new linear part
  is W P with W = A + (B-weighted CROWN coefficients), the interval part collects
  the relaxation offsets plus the interval product W (x) I;
* EvalInt gives the box c +- |P| 1 + I of each step.

Shared slope (the paper enforces it without naming a mechanism) is read as the
parallel relaxation of an unstable neuron: h >= s z and h <= s z + t with the
chord slope s = u/(u-l), t = -s l.  The row multipliers are then identical for the
lower and upper bound and only the offset sums differ.  Intermediate bounds are
CROWN (shared slope, one row per neuron that IBP leaves unstable) intersected with
IBP; layer 1 is exact for the TM input.
"""
from __future__ import annotations

import numpy as np

from .crown import UNSTABLE, backward, ibp_next, relu_relaxation


def _interval_dot(w, lo, hi):
    """Range of w . r for r in [lo, hi] (rows of w)."""
    a = w * lo[None, :]; b = w * hi[None, :]
    return np.minimum(a, b).sum(axis=1), np.maximum(a, b).sum(axis=1)


def tm_eval(w, acc_lo, acc_hi, c, P, Ilo, Ihi):
    """Range of w . x + [acc_lo, acc_hi] for x = c + P z + r, z in [-1,1]^n, r in I."""
    base = w @ c
    rad = np.abs(w @ P).sum(axis=1)
    rl, rh = _interval_dot(w, Ilo, Ihi)
    return acc_lo + base - rad + rl, acc_hi + base + rad + rh


def tm_intermediate_bounds(net, c, P, Ilo, Ihi):
    """Hidden pre-activation bounds for the TM input (shared-slope CROWN n IBP)."""
    L = net.n_layers
    W1, b1 = net.Ws[0], net.bs[0]
    zero = np.zeros(W1.shape[0])
    l, u = tm_eval(W1, b1 + zero, b1 + zero, c, P, Ilo, Ihi)
    bounds = [(l, u)]
    rows = [0]
    for k in range(2, L):
        li, ui = ibp_next(net.Ws[k - 1], net.bs[k - 1], *bounds[-1])
        U = np.nonzero((li < 0) & (ui > 0))[0]
        l, u = li.copy(), ui.copy()
        if U.size:
            relax = [relu_relaxation(*bk) for bk in bounds]
            n = net.hidden[k - 1]
            E = np.zeros((U.size, n)); E[np.arange(U.size), U] = 1.0
            res = backward(net, relax, k, E, shared=True)
            lo, hi = tm_eval(res["w"], res["acc"], res["acc_hi"], c, P, Ilo, Ihi)
            l[U] = np.maximum(li[U], lo)
            u[U] = np.minimum(ui[U], hi)
        rows.append(int(U.size))
        bounds.append((l, u))
    return bounds, rows


def tm_step(net, c, P, Ilo, Ihi):
    """One closed-loop step: returns the next TM (c, P, Ilo, Ihi), its box and row counts."""
    bounds, rows = tm_intermediate_bounds(net, c, P, Ilo, Ihi)
    relax = [relu_relaxation(*bk) for bk in bounds]
    n = net.A.shape[0]
    res = backward(net, relax, net.n_layers, net.B, shared=True)   # rows e_i on x': a_L = B_i
    W = net.A + res["w"]
    c2 = W @ c
    P2 = W @ P
    rl, rh = _interval_dot(W, Ilo, Ihi)
    Ilo2 = rl + res["acc"]
    Ihi2 = rh + res["acc_hi"]
    rad = np.abs(P2).sum(axis=1)
    box = np.stack([c2 - rad + Ilo2, c2 + rad + Ihi2], axis=1)
    rows.append(n)
    return (c2, P2, Ilo2, Ihi2), box, rows


def reach_dt(net, xc, xr, horizon, u=None):
    """Boxes X_0 .. X_H (H+1 x n x 2) of the stepwise TM reachability from one box.

    With exogenous inputs (the batched reach of candidate action sequences in the
    paper's MPC section): the network input is v = [x; u_t] and the loop is
    x' = A v + B f(v), A of shape n x (n + m), with u (H x m) a given sequence.  The
    TM of v is the state's TM extended by the point u_t (zero linear part, zero
    interval), so every step is the same CROWN step on the extended TM."""
    n = net.A.shape[0]
    xc = np.asarray(xc, np.float64)[:n]; xr = np.asarray(xr, np.float64)[:n]
    m = net.widths[0] - n
    if m and (u is None or np.shape(u) != (horizon, m)):
        raise ValueError("the network has %d exogenous inputs: u must be horizon x %d" % (m, m))
    c = xc.copy(); P = np.diag(xr)
    Ilo = np.zeros(n); Ihi = np.zeros(n)
    boxes = [np.stack([c - xr, c + xr], axis=1)]
    rows = []
    for t in range(horizon):
        if m:
            uv = np.asarray(u[t], np.float64)
            cv, Pv = np.concatenate([c, uv]), np.vstack([P, np.zeros((m, n))])
            Iv_lo, Iv_hi = np.concatenate([Ilo, np.zeros(m)]), np.concatenate([Ihi, np.zeros(m)])
        else:
            cv, Pv, Iv_lo, Iv_hi = c, P, Ilo, Ihi
        (c, P, Ilo, Ihi), box, r = tm_step(net, cv, Pv, Iv_lo, Iv_hi)
        boxes.append(box)
        rows.append(r)
    return np.array(boxes), dict(c=c, P=P, Ilo=Ilo, Ihi=Ihi, rows=rows)


def tube_volume(boxes):
    """Width-sum volume proxy of the paper's reachability-aware loss: sum over steps
    t >= 1 and dimensions of the box widths."""
    b = np.asarray(boxes)
    return float((b[1:, :, 1] - b[1:, :, 0]).sum())
