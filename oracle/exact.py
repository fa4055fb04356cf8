"""Exact extrema and sampled under-approximations for tiny networks.

TEST INFRASTRUCTURE ONLY (see ``oracle/crown.py``).

* ``exact_min`` enumerates activation patterns: for a fixed pattern the network is
  affine in x, and the set of inputs realising the pattern (plus the split
  constraints) is a polytope inside the box, so each pattern is one linear program
  (scipy HiGHS).  The minimum over feasible patterns is the exact minimum of the
  spec over the subdomain.  Only for H <= ~14 hidden neurons.
* ``sampled_extrema`` evaluates the network in FP64 at uniform samples, the box
  corners (when few) and the centre, keeping only points that satisfy the split
  constraints; it under-approximates the range, so every sound bound must contain
  it (the paper's sampling baselines play the same role for reachable sets).
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import linprog


def forward(net, X):
    """Network output and hidden pre-activations at points X (N x n0)."""
    h = X
    zs = []
    for k in range(net.n_layers - 1):
        z = h @ net.Ws[k].T + net.bs[k]
        zs.append(z)
        h = np.maximum(z, 0.0)
    y = h @ net.Ws[-1].T + net.bs[-1]
    return y, zs


def target(net, X, y):
    """The spec target: the network output, or x' = A x + B y in the closed loop."""
    if net.closed_loop:
        return X @ net.A.T + y @ net.B.T
    return y


def _affine_maps(net, pattern):
    """For an activation pattern (list of 0/1 arrays), z_k = M_k x + m_k for every
    hidden layer and the output y = M x + m."""
    n0 = net.widths[0]
    M = np.eye(n0); m = np.zeros(n0)
    pre = []
    for k in range(net.n_layers - 1):
        Mz = net.Ws[k] @ M; mz = net.Ws[k] @ m + net.bs[k]
        pre.append((Mz, mz))
        D = pattern[k].astype(np.float64)
        M = D[:, None] * Mz; m = D * mz
    return pre, (net.Ws[-1] @ M, net.Ws[-1] @ m + net.bs[-1])


def exact_min(net, xc, xr, c, splits=()):
    """Exact minimum of c . target over the box with split constraints (None if the
    subdomain is empty)."""
    hidden = net.hidden
    H = sum(hidden)
    if H > 16:
        raise ValueError("pattern enumeration is only for tiny networks")
    sig = [np.zeros(n, np.int64) for n in hidden]
    for (k, j, s) in splits:
        sig[k - 1][j] = s
    best = None
    bounds = list(zip(xc - xr, xc + xr))
    offs = np.cumsum([0] + hidden)
    for bits in itertools.product((0, 1), repeat=H):
        bits = np.array(bits)
        pattern = [bits[offs[k]:offs[k + 1]] for k in range(len(hidden))]
        # a split forces the pattern bit (z >= 0 active / z <= 0 inactive)
        ok = True
        for k in range(len(hidden)):
            if np.any((sig[k] > 0) & (pattern[k] == 0)) or np.any((sig[k] < 0) & (pattern[k] == 1)):
                ok = False; break
        if not ok:
            continue
        pre, (My, my) = _affine_maps(net, pattern)
        A_ub, b_ub = [], []
        for k, (Mz, mz) in enumerate(pre):
            for j in range(hidden[k]):
                if pattern[k][j]:       # z >= 0  ->  -Mz x <= mz
                    A_ub.append(-Mz[j]); b_ub.append(mz[j])
                else:                   # z <= 0
                    A_ub.append(Mz[j]); b_ub.append(-mz[j])
        if net.closed_loop:
            obj = c @ net.A + (c @ net.B) @ My
            const = (c @ net.B) @ my
        else:
            obj = c @ My
            const = c @ my
        res = linprog(obj, A_ub=np.array(A_ub) if A_ub else None,
                      b_ub=np.array(b_ub) if b_ub else None, bounds=bounds, method="highs")
        if res.status == 0:
            v = res.fun + const
            best = v if best is None else min(best, v)
    return best


def sample_points(rng, xc, xr, n, corners=True):
    n0 = xc.shape[0]
    pts = [xc[None, :], xc + xr * rng.uniform(-1.0, 1.0, size=(n, n0))]
    if corners and n0 <= 12:
        C = np.array(list(itertools.product((-1.0, 1.0), repeat=n0)))
        pts.append(xc + xr * C)
    return np.vstack(pts)


def sampled_extrema(net, xc, xr, spec, splits=(), n=10000, seed=0):
    """(min, max) of spec . target over sampled points satisfying the splits."""
    rng = np.random.default_rng(seed)
    X = sample_points(rng, xc, xr, n)
    y, zs = forward(net, X)
    keep = np.ones(X.shape[0], bool)
    for (k, j, s) in splits:
        keep &= (s * zs[k - 1][:, j]) >= 0
    T = target(net, X[keep], y[keep])
    vals = T @ np.asarray(spec).T
    if vals.shape[0] == 0:
        return None, None
    return vals.min(axis=0), vals.max(axis=0)
