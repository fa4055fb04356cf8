"""FP64 reference for CROWN through the closed loop unrolled over the horizon.

TEST INFRASTRUCTURE ONLY (see ``oracle/crown.py``).

The paper's DT comparison (Section "Reachability Tool Evaluations", the DT panel of the
figure that benchmarks the reachability tool) runs CROWN on the graph of the closed
loop unrolled over the whole horizon: it is tighter than the stepwise Algorithm
"Reachability of DT Dynamics" because bounds are propagated jointly across the steps
(no Taylor model is re-formed at each step) and much slower, since every hidden neuron
of step t is bounded by a backward pass through all earlier steps to the initial box.

The graph: v_t = [x_t; u_t] (u_t a given exogenous input, empty for a plain
controller), x_{t+1} = A v_t + B f(v_t), with f the ReLU network; x_0 is in the box.
Readings (the rules of plain CROWN in ``crown.py``, applied to the unrolled graph):
  * relaxation of an unstable neuron: upper chord, adaptive lower slope
    alpha = 1 iff u > -l; lower and upper bounds are separate rows;
  * a linear function lam . x_{s+1} + acc is carried back through step s as
      lam . x_{s+1} = (lam A) . v_s + (lam B) . f(v_s):
    the rows a_L = lam B run the CROWN backward pass of the network of step s (its
    own relaxation), whose input coefficients w add to lam A; the coefficients on
    the exogenous part of v_s multiply the known u_s and move into the offset;
  * intermediate bounds of step t: layer 1 of step 0 is exact on the box; every other
    hidden layer takes interval bounds (IBP) from its input node -- the state box of
    step t for layer 1, the previous layer's bounds otherwise -- and each neuron that
    IBP leaves unstable gets the CROWN bound of its rows +-e_j carried back to x_0,
    intersected with IBP; stable neurons keep their IBP bounds;
  * the state box of x_{t+1}: rows +-e_i on x_{t+1} carried back to x_0 and
    concretized on the initial box (lower bound of -x_i gives the upper bound).
"""
from __future__ import annotations

import numpy as np

from .crown import affine_box, backward, concretize_box, ibp_next, relu_relaxation


def _split_input(net):
    n = net.A.shape[0]
    return n, net.widths[0] - n


def back_through_step(net, relax_s, lam, acc, u_s):
    """Carry rows lam (R x n) on x_{s+1} (offsets acc) back through step s.

    Returns the coefficients on x_s and the new offsets."""
    n, m = _split_input(net)
    res = backward(net, relax_s, net.n_layers, lam @ net.B)     # rows on v_s
    wv = res["w"] + lam @ net.A                                   # coefficients on v_s
    acc = acc + res["acc"]
    if m:
        acc = acc + wv[:, n:] @ np.asarray(u_s, np.float64)
    return wv[:, :n], acc


def to_initial(net, relaxes, t, lam, acc, us):
    """Carry rows on x_t back to x_0 through steps t-1, ..., 0."""
    for s in range(t - 1, -1, -1):
        lam, acc = back_through_step(net, relaxes[s], lam, acc, us[s] if us is not None else None)
    return lam, acc


def reach_joint(net, xc, xr, horizon, u=None):
    """Boxes X_0 .. X_H (H+1 x n x 2) of CROWN on the unrolled closed loop, and a dict
    with the per-step hidden bounds and the CROWN row counts rows[t][k-1] of hidden
    layer k at step t (rows[t][L-1]: the 2n state rows)."""
    n, m = _split_input(net)
    L = net.n_layers
    xc = np.asarray(xc, np.float64)[:n]; xr = np.asarray(xr, np.float64)[:n]
    if m and (u is None or np.shape(u) != (horizon, m)):
        raise ValueError("the network has %d exogenous inputs: u must be horizon x %d" % (m, m))
    us = [np.asarray(u[t], np.float64) for t in range(horizon)] if m else None
    boxes = [np.stack([xc - xr, xc + xr], axis=1)]
    relaxes, all_bounds, rows = [], [], []
    E_state = np.vstack([np.eye(n), -np.eye(n)])
    for t in range(horizon):
        lo, hi = boxes[t][:, 0], boxes[t][:, 1]
        vc, vr = 0.5 * (lo + hi), 0.5 * (hi - lo)
        if m:
            vc, vr = np.concatenate([vc, us[t]]), np.concatenate([vr, np.zeros(m)])
        r_t = []
        # layer 1: the affine range over the state box (exact at t = 0), then CROWN
        # rows carried back to x_0 for the neurons it leaves unstable
        l, uu = affine_box(net.Ws[0], net.bs[0], vc, vr)
        U = np.nonzero((l < 0) & (uu > 0))[0] if t > 0 else np.zeros(0, np.int64)
        if U.size:
            Wv = np.vstack([net.Ws[0][U], -net.Ws[0][U]])
            acc = np.concatenate([net.bs[0][U], -net.bs[0][U]])
            if m:
                acc = acc + Wv[:, n:] @ us[t]
            lam0, acc = to_initial(net, relaxes, t, Wv[:, :n], acc, us)
            lb = concretize_box(lam0, acc, xc, xr)
            l[U] = np.maximum(l[U], lb[:U.size])
            uu[U] = np.minimum(uu[U], -lb[U.size:])
        r_t.append(2 * int(U.size))
        bounds = [(l, uu)]
        for k in range(2, L):
            li, ui = ibp_next(net.Ws[k - 1], net.bs[k - 1], *bounds[-1])
            U = np.nonzero((li < 0) & (ui > 0))[0]
            l, uu = li.copy(), ui.copy()
            if U.size:
                relax_t = [relu_relaxation(*bk) for bk in bounds]
                E = np.zeros((U.size, net.hidden[k - 1])); E[np.arange(U.size), U] = 1.0
                res = backward(net, relax_t, k, np.vstack([E, -E]))   # rows on v_t
                acc = res["acc"]
                if m:
                    acc = acc + res["w"][:, n:] @ us[t]
                lam0, acc = to_initial(net, relaxes, t, res["w"][:, :n], acc, us)
                lb = concretize_box(lam0, acc, xc, xr)
                l[U] = np.maximum(li[U], lb[:U.size])
                uu[U] = np.minimum(ui[U], -lb[U.size:])
            r_t.append(2 * int(U.size))
            bounds.append((l, uu))
        relaxes.append([relu_relaxation(*bk) for bk in bounds])
        all_bounds.append(bounds)
        # state box of x_{t+1}
        lam0, acc = to_initial(net, relaxes, t + 1, E_state, np.zeros(2 * n), us)
        lb = concretize_box(lam0, acc, xc, xr)
        boxes.append(np.stack([lb[:n], -lb[n:]], axis=1))
        r_t.append(2 * n)
        rows.append(r_t)
    return np.array(boxes), dict(bounds=all_bounds, rows=rows)
