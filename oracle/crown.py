"""FP64 reference ("oracle") for CROWN-style linear bound propagation.

TEST INFRASTRUCTURE ONLY.  This package is imported by ``tests/``, by the smoke
check and by the CPU-baseline leg of the benchmark, and by nothing else.  It
shares no code with the GPU path and must never be used as a fallback for it.

What it computes follows the paper:
  * Theorem "CROWN linear bounds of NN" (Section "Neural Components via CROWN"):
    an affine lower and upper bound  W_lo x + b_lo <= f(x) <= W_hi x + b_hi
    of a ReLU network over an input box, obtained by backward bound propagation.
  * Algorithm "Reachability of DT Dynamics" uses CROWN followed by EvalInt, the
    box enclosure of the affine bounds (concretization).
  * The refinements of the table "Refinement strategies" (gradient refinement and
    input splitting) and the split/dual notation of the preamble
    (beta, alpha, Lambda, D, d) which the body of the paper never defines.

The paper leaves the ReLU relaxation, the slopes alpha, the split multipliers
beta and the intermediate-bound procedure to the cited CROWN / alpha-beta-CROWN
works.  They are fixed here from first principles (weak duality), with these
readings:
  * relaxation of an unstable neuron (l < 0 < u): upper chord h <= s z + t with
    s = u / (u - l), t = -s l; lower line h >= alpha z, alpha in [0, 1], with the
    adaptive default alpha = 1 iff u > -l (a tie gives 0);
  * stability is tested as u <= 0 (inactive) first, then l >= 0 (active);
  * intermediate bounds: layer 1 exact, then for every deeper hidden layer the
    CROWN bound of each neuron that interval propagation (IBP) leaves unstable
    and that is not split, intersected with IBP; stable or split neurons keep
    their IBP bounds; split neurons are clamped (s = +1: l <- max(l, 0);
    s = -1: u <- min(u, 0)) and l > u marks the subdomain infeasible;
  * a split (k, j, s) adds  -beta * s * z_k[j]  to the objective (valid because
    s z_k[j] >= 0 on the subdomain and beta >= 0), so every alpha in [0,1] and
    beta >= 0 gives a sound bound;
  * the bound of the spec direction c is the lower bound of c.y; the upper bound
    is minus the lower bound of -c.y.  In the closed loop x' = A x + B y the spec
    is on x': the row starts as c B on the network output and c A is added to the
    input coefficients before concretization.
"""
from __future__ import annotations

import numpy as np

INACTIVE, ACTIVE, UNSTABLE = 0, 1, 2
STATUS_OK, STATUS_INFEASIBLE, STATUS_NONFINITE = 0, 1, 2


# --------------------------------------------------------------------------------------
# Elementary steps
# --------------------------------------------------------------------------------------
def relu_relaxation(l, u):
    """Classify neurons and build the chord relaxation.

    Returns (kind, s, t, alpha0): kind in {INACTIVE, ACTIVE, UNSTABLE}; for unstable
    neurons the upper chord slope s = u/(u-l) and intercept t = -s*l, and the
    adaptive lower slope alpha0 = 1 iff u > -l.  Stable neurons have s = alpha0 =
    1 (active) or 0 (inactive) and t = 0.
    """
    l = np.asarray(l, np.float64); u = np.asarray(u, np.float64)
    kind = np.where(u <= 0, INACTIVE, np.where(l >= 0, ACTIVE, UNSTABLE))
    uns = kind == UNSTABLE
    s = np.where(kind == ACTIVE, 1.0, 0.0)
    t = np.zeros_like(l)
    with np.errstate(divide="ignore", invalid="ignore"):
        s_uns = u / (u - l)
    s = np.where(uns, s_uns, s)
    t = np.where(uns, -s_uns * l, t)
    alpha0 = np.where(kind == ACTIVE, 1.0, np.where(uns & (u > -l), 1.0, 0.0))
    return kind, s, t, alpha0


def ibp_next(W, b, l_prev, u_prev):
    """Interval bound of z = W relu(h) + b for h in [l_prev, u_prev], centre/radius form."""
    lo = np.maximum(l_prev, 0.0); hi = np.maximum(u_prev, 0.0)
    c = 0.5 * (lo + hi); r = 0.5 * (hi - lo)
    zc = W @ c + b
    zr = np.abs(W) @ r
    return zc - zr, zc + zr


def affine_box(W, b, xc, xr):
    """Exact range of W x + b over the box [xc - xr, xc + xr]."""
    zc = W @ xc + b
    zr = np.abs(W) @ xr
    return zc - zr, zc + zr


def concretize_box(w, acc, xc, xr):
    """Minimum of w.x + acc over the box (one value per row)."""
    return acc + w @ xc - np.abs(w) @ xr


def split_arrays(splits, hidden):
    """Dense per-layer split signs (0 = not split) and per-layer split slot ids."""
    sig = [np.zeros(n, np.int64) for n in hidden]
    slot = [np.full(n, -1, np.int64) for n in hidden]
    for idx, (k, j, s) in enumerate(splits):
        sig[k - 1][j] = s
        slot[k - 1][j] = idx
    return sig, slot


def clamp_splits(l, u, sig):
    l = np.where(sig > 0, np.maximum(l, 0.0), l)
    u = np.where(sig < 0, np.minimum(u, 0.0), u)
    return l, u


# --------------------------------------------------------------------------------------
# Backward bound propagation (one subdomain, many rows at once)
# --------------------------------------------------------------------------------------
def backward(net, relax, K, a_K, *, alpha=None, beta=None, sig=None, shared=False, tape=False):
    """Propagate row multipliers ``a_K`` (R x n_K) on z_K back to the input.

    ``K`` is the 1-based layer of the rows (K = L for the network output).
    ``relax[k-1]`` = (kind, s, t, alpha0) of hidden layer k.  ``alpha[k-1]`` (R x n_k)
    overrides the lower slope of unstable neurons; ``beta[k-1]`` (R x n_k, zero off
    split neurons) with ``sig[k-1]`` adds the split terms.  With ``shared`` the
    parallel relaxation (common slope s on both sides) is used and two offset
    sums are returned (lower, upper).

    Returns dict(w = R x n0 input coefficients, acc = offsets, [acc_hi], tape).
    """
    Ws, bs = net.Ws, net.bs
    a = np.asarray(a_K, np.float64)
    acc = a @ bs[K - 1]
    acc_hi = acc.copy() if shared else None
    g = a @ Ws[K - 1]
    rec = []
    for k in range(K - 1, 0, -1):
        kind, s, t, alpha0 = relax[k - 1]
        uns = kind == UNSTABLE
        if shared:
            d = np.broadcast_to(s, g.shape)
            gt = np.where(uns, g * t, 0.0)
            acc = acc + np.minimum(gt, 0.0).sum(axis=1)
            acc_hi = acc_hi + np.maximum(gt, 0.0).sum(axis=1)
        else:
            lo = np.broadcast_to(alpha0, g.shape) if alpha is None else np.where(uns, alpha[k - 1], alpha0)
            d = np.where(g >= 0, lo, s)
            acc = acc + np.where(uns & (g < 0), g * t, 0.0).sum(axis=1)
        a = d * g
        if beta is not None and sig is not None:
            a = a - beta[k - 1] * sig[k - 1]
        if tape:
            rec.append(dict(k=k, g=g, d=d))
        acc = acc + a @ bs[k - 1]
        if shared:
            acc_hi = acc_hi + a @ bs[k - 1]
        g = a @ Ws[k - 1]
    out = dict(w=g, acc=acc)
    if shared:
        out["acc_hi"] = acc_hi
    if tape:
        out["tape"] = rec[::-1]   # ordered by layer k = 1 .. K-1
    return out


def gradient(net, relax, K, res, xc, xr, *, sig=None):
    """Hand adjoint of lb = acc + w.xc - |w|.xr with respect to alpha and beta.

    Uses the tape of ``backward(..., tape=True)``; sgn(0) = 0 for |w|, and the
    g >= 0 branch at g = 0.  Returns (dalpha[k-1], dbeta[k-1]) per hidden layer,
    each R x n_k (zero where the parameter has no effect).
    """
    Ws, bs = net.Ws, net.bs
    w = res["w"]
    dw = xc[None, :] - np.sign(w) * xr[None, :]
    delta = dw @ Ws[0].T + bs[0]          # d lb / d a^(1)
    dalpha, dbeta = [], []
    for k in range(1, K):
        kind, s, t, alpha0 = relax[k - 1]
        uns = kind == UNSTABLE
        g = res["tape"][k - 1]["g"]; d = res["tape"][k - 1]["d"]
        dalpha.append(np.where(uns & (g >= 0), delta * g, 0.0))
        if sig is not None:
            dbeta.append(-sig[k - 1] * delta * (sig[k - 1] != 0))
        else:
            dbeta.append(np.zeros_like(delta))
        e = delta * d + np.where(uns & (g < 0), t, 0.0)       # d lb / d g^(k)
        if k < K - 1:
            delta = e @ Ws[k].T + bs[k]                        # d lb / d a^(k+1)
    return dalpha, dbeta


# --------------------------------------------------------------------------------------
# Spec rows
# --------------------------------------------------------------------------------------
def default_spec(net):
    n = net.A.shape[0] if net.closed_loop else net.widths[-1]
    return np.eye(n)


def spec_rows(net, spec):
    """Rows for lower bounds of c.target and of -c.target.  Returns (a_L, skip)
    with a_L the multipliers on the network output and skip the multipliers added
    on the input (closed loop), both for the 2q rows [c; -c]."""
    C = np.vstack([spec, -spec])
    if net.closed_loop:
        return C @ net.B, C @ net.A
    return C, None


# --------------------------------------------------------------------------------------
# Full CROWN for one subdomain
# --------------------------------------------------------------------------------------
def intermediate_bounds(net, xc, xr, splits=()):
    """Pre-activation bounds of every hidden layer (list of (l, u)), rows counts of
    the CROWN chains per layer, and the status of the subdomain."""
    L = net.n_layers
    hidden = net.hidden
    sig, _ = split_arrays(splits, hidden)
    status = STATUS_OK
    if not (np.all(np.isfinite(xc)) and np.all(np.isfinite(xr))):
        status |= STATUS_NONFINITE
    l, u = affine_box(net.Ws[0], net.bs[0], xc, xr)
    l, u = clamp_splits(l, u, sig[0])
    bounds = [(l, u)]
    rows = [0]
    if np.any(l > u):
        status |= STATUS_INFEASIBLE
    for k in range(2, L):
        li, ui = ibp_next(net.Ws[k - 1], net.bs[k - 1], *bounds[-1])
        U = np.nonzero((li < 0) & (ui > 0) & (sig[k - 1] == 0))[0]
        l, u = li.copy(), ui.copy()
        if U.size:
            relax = [relu_relaxation(*bk) for bk in bounds]
            n = hidden[k - 1]
            E = np.zeros((U.size, n)); E[np.arange(U.size), U] = 1.0
            res = backward(net, relax, k, np.vstack([E, -E]))
            lb = concretize_box(res["w"], res["acc"], xc, xr)
            l[U] = np.maximum(li[U], lb[:U.size])
            u[U] = np.minimum(ui[U], -lb[U.size:])
        rows.append(2 * int(U.size))
        l, u = clamp_splits(l, u, sig[k - 1])
        if np.any(l > u):
            status |= STATUS_INFEASIBLE
        bounds.append((l, u))
    for (l, u) in bounds:
        if not (np.all(np.isfinite(l)) and np.all(np.isfinite(u))):
            status |= STATUS_NONFINITE
    return bounds, rows, status


def final_bounds(net, bounds, xc, xr, spec=None, *, alpha=None, beta=None, splits=(), tape=False):
    """Lower/upper bounds of the spec directions given fixed intermediate bounds.

    Returns dict with lb, ub (q,), lam_lo/lam_hi (q x n0), acc_lo/acc_hi (q,), and
    the raw per-row results (2q rows: [c; -c])."""
    L = net.n_layers
    spec = default_spec(net) if spec is None else np.asarray(spec, np.float64)
    q = spec.shape[0]
    relax = [relu_relaxation(*bk) for bk in bounds]
    sig, _ = split_arrays(splits, net.hidden)
    a_L, skip = spec_rows(net, spec)
    res = backward(net, relax, L, a_L, alpha=alpha, beta=beta, sig=sig if beta is not None else None, tape=tape)
    w = res["w"] + (skip if skip is not None else 0.0)
    res["w"] = w
    rowlb = concretize_box(w, res["acc"], xc, xr)
    return dict(lb=rowlb[:q], ub=-rowlb[q:], lam_lo=w[:q], acc_lo=res["acc"][:q],
                lam_hi=-w[q:], acc_hi=-res["acc"][q:], rowlb=rowlb, res=res, relax=relax, sig=sig)


def crown(net, xc, xr, splits=(), spec=None):
    """Plain CROWN (adaptive slopes, beta = 0) for one subdomain."""
    bounds, rows, status = intermediate_bounds(net, xc, xr, splits)
    q = (default_spec(net) if spec is None else np.asarray(spec)).shape[0]
    if status & STATUS_INFEASIBLE:
        n0 = net.widths[0]
        return dict(lb=np.full(q, np.inf), ub=np.full(q, -np.inf), bounds=bounds, rows=rows,
                    status=status, lam_lo=np.zeros((q, n0)), lam_hi=np.zeros((q, n0)),
                    acc_lo=np.full(q, np.inf), acc_hi=np.full(q, -np.inf))
    out = final_bounds(net, bounds, xc, xr, spec)
    out.update(bounds=bounds, rows=rows, status=status)
    return out


def hidden_offsets(net):
    return np.concatenate([[0], np.cumsum(net.hidden)]).astype(np.int64)


def default_alpha(net, bounds, n_rows):
    """Adaptive slopes of every hidden neuron, repeated for each row (R x H)."""
    a0 = np.concatenate([relu_relaxation(*bk)[3] for bk in bounds])
    return np.repeat(a0[None, :], n_rows, axis=0)


def _split_alpha(net, alpha_flat):
    offs = hidden_offsets(net)
    return [alpha_flat[:, offs[k]:offs[k + 1]] for k in range(len(net.hidden))]


def _dense_beta(net, beta_flat, splits):
    """Per-layer dense beta (R x n_k) from per-split beta (R x n_splits)."""
    R = beta_flat.shape[0]
    out = [np.zeros((R, n)) for n in net.hidden]
    for idx, (k, j, s) in enumerate(splits):
        out[k - 1][:, j] = beta_flat[:, idx]
    return out


def evaluate_duals(net, bounds, xc, xr, alpha_flat, beta_flat, splits=(), spec=None, grad=True):
    """Bound of every row at given (alpha, beta) and, optionally, its gradient.

    alpha_flat: 2q x H, beta_flat: 2q x n_splits.  Returns (rowlb (2q,), dalpha (2q x H),
    dbeta (2q x n_splits), result dict)."""
    alpha = _split_alpha(net, alpha_flat)
    beta = _dense_beta(net, beta_flat, splits)
    out = final_bounds(net, bounds, xc, xr, spec, alpha=alpha, beta=beta, splits=splits, tape=grad)
    if not grad:
        return out["rowlb"], None, None, out
    dal, dbe = gradient(net, out["relax"], net.n_layers, out["res"], xc, xr, sig=out["sig"])
    dalpha = np.concatenate(dal, axis=1)
    dbeta = np.zeros_like(beta_flat)
    for idx, (k, j, s) in enumerate(splits):
        dbeta[:, idx] = dbe[k - 1][:, j]
    return out["rowlb"], dalpha, dbeta, out


def param_gradient(net, bounds, xc, xr, alpha_flat, beta_flat, omega, splits=(), spec=None):
    """Weighted gradient of the row bounds w.r.t. the network parameters and the box,
    with the relaxation held fixed.

    The bound of row r is lb_r = acc_r + w_r.xc - |w_r|.xr (Theorem "CROWN linear
    bounds of NN"), where the slopes, intercepts (from the fixed intermediate bounds)
    and alpha, beta are constants.  W_k enters only through g^(k-1) = a^(k) W_k and
    b_k only through acc += a^(k).b_k, so with e^(k) = d lb / d g^(k) (the adjoint
    of the alpha/beta gradient) and e^(0) = xc - sgn(w) xr:
        d lb_r / d W_k = a^(k)_r (outer) e^(k-1)_r,   d lb_r / d b_k = a^(k)_r,
        d lb_r / d xc = w_r,   d lb_r / d xr = -|w_r|.
    ``omega`` (2q,) weights the rows (the incoming gradient of each row bound).

    Returns dict(dW, db (per layer, natural shapes), dxc, dxr (n0,), absW (per layer:
    sum_r |omega_r| |a^(k)_r| (outer) |e^(k-1)_r|, the scale of the rounding error
    of any summation order), rowlb)."""
    alpha = _split_alpha(net, alpha_flat)
    beta = _dense_beta(net, beta_flat, splits)
    out = final_bounds(net, bounds, xc, xr, spec, alpha=alpha, beta=beta, splits=splits, tape=True)
    L = net.n_layers
    Ws, bs = net.Ws, net.bs
    relax, res, sig = out["relax"], out["res"], out["sig"]
    om = np.asarray(omega, np.float64)
    a_L, _ = spec_rows(net, default_spec(net) if spec is None else np.asarray(spec, np.float64))
    # multipliers a^(k) on z_k (k = 1..L) and adjoints e^(k) (k = 0..L-1)
    a = [None] * (L + 1)
    e = [None] * L
    a[L] = a_L
    for k in range(1, L):
        tp = res["tape"][k - 1]
        a[k] = tp["d"] * tp["g"] - beta[k - 1] * sig[k - 1]
    w = res["w"]
    e[0] = xc[None, :] - np.sign(w) * xr[None, :]
    delta = e[0] @ Ws[0].T + bs[0]
    for k in range(1, L):
        kind, s, t, _ = relax[k - 1]
        g = res["tape"][k - 1]["g"]
        d = res["tape"][k - 1]["d"]
        e[k] = delta * d + np.where((kind == UNSTABLE) & (g < 0), t, 0.0)
        if k < L - 1:
            delta = e[k] @ Ws[k].T + bs[k]
    dW, db, absW = [], [], []
    for k in range(1, L + 1):
        dW.append((om[:, None] * a[k]).T @ e[k - 1])
        db.append(om @ a[k])
        absW.append((np.abs(om)[:, None] * np.abs(a[k])).T @ np.abs(e[k - 1]))
    return dict(dW=dW, db=db, dxc=om @ w, dxr=-(om @ np.abs(w)), absW=absW, rowlb=out["rowlb"])


def optimize_duals(net, bounds, xc, xr, splits=(), spec=None, iters=20, lr=0.1,
                   alpha_init=None, beta_init=None, opt_alpha=True, opt_beta=True):
    """Projected gradient ascent on (alpha, beta) with fixed intermediate bounds.

    Iterates t = 0..T: evaluate lb_t and its gradient at (alpha_t, beta_t); for
    t < T update alpha <- clip(alpha + lr*dalpha, 0, 1) on unstable neurons and
    beta <- max(0, beta + lr*dbeta).  Returns the best-so-far row bounds, the
    final iterate's bounds, the final (alpha, beta), the gradient at the final
    iterate and the full trajectory of row bounds.
    """
    spec_m = default_spec(net) if spec is None else np.asarray(spec, np.float64)
    R = 2 * spec_m.shape[0]
    unstable = np.concatenate([relu_relaxation(*bk)[0] == UNSTABLE for bk in bounds])
    alpha = default_alpha(net, bounds, R) if alpha_init is None else np.array(alpha_init, np.float64)
    beta = np.zeros((R, len(splits))) if beta_init is None else np.array(beta_init, np.float64)
    best = np.full(R, -np.inf)
    traj = []
    for t in range(iters + 1):
        lb, dal, dbe, _ = evaluate_duals(net, bounds, xc, xr, alpha, beta, splits, spec_m, grad=True)
        traj.append(lb)
        best = np.maximum(best, lb)
        if t == iters:
            break
        if opt_alpha:
            alpha = np.where(unstable[None, :], np.clip(alpha + lr * dal, 0.0, 1.0), alpha)
        if opt_beta and beta.size:
            beta = np.maximum(0.0, beta + lr * dbe)
    q = spec_m.shape[0]
    return dict(best=best, final=lb, lb=best[:q], ub=-best[q:], alpha=alpha, beta=beta,
                dalpha=dal, dbeta=dbe, traj=np.array(traj))


def crown_batch(nets, batch, spec=None, subset=None):
    """Plain CROWN over (a subset of) a batch; returns lb, ub (S x q), status (S,),
    per-subdomain intermediate bounds and CROWN row counts."""
    idx = range(batch.n_sub) if subset is None else subset
    lbs, ubs, st, bnds, rows = [], [], [], [], []
    for s in idx:
        net = nets[int(batch.net_id[s])]
        out = crown(net, batch.x_center[s], batch.x_radius[s], batch.splits_of(s), spec)
        lbs.append(out["lb"]); ubs.append(out["ub"]); st.append(out["status"])
        bnds.append(out["bounds"]); rows.append(out["rows"])
    return dict(lb=np.array(lbs), ub=np.array(ubs), status=np.array(st), bounds=bnds, rows=rows)
