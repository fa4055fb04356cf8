"""FP64 reference for continuous-time reachability with Taylor-model flowpipes.

TEST INFRASTRUCTURE ONLY (see ``oracle/crown.py``).

Follows Section "Propagation under Continuous-Time Analytical Dynamics" with Theorem
"TM flowpipe step via Picard iteration", the appendix Algorithm "Reachability of CT
Dynamics with TM Flowpipe", the fixed-shape representation of Section "Representation
of Reachable Sets" and the alternating closed loop of Algorithm "Reachability of CT NN
Control Systems" (Section "Closed-Loop Reachability for Continuous-Time Systems").

Representation (the paper's quasi-quadratic fixed-shape TM): over the normalised
generators y in [-1, 1]^m of the step's initial set and the time s in [0, h],

    X(y, s) = c + L y + l s + s (M y) + w s^2  (+)  [I_lo, I_hi],

i.e. c + A z + B s z with z = (y, s).  Readings where the paper is silent:
  * dynamics: polynomial of degree <= 2 in the state and affine in the input,
    f_i(x, u) = a_i + F_i x + G_i u + x^T Q_i x (the TM arithmetic of a product is
    exact up to the monomials outside the representation, which are bounded); the
    quadratic form is taken over its monomials x_j x_k, j <= k (coefficients
    Q_ijk + Q_ikj off the diagonal), one TM product per monomial;
  * Picard (polynomial part, order k = 2): g_0 = c + S y, g_{j+1} = Trunc(x_0 +
    int_0^s f(g_j)); Trunc keeps the monomials {1, y, s, s y, s^2};
  * remainder (validation): with x_0 = c + S y + r_0, r_0 in I_0, the Picard image of
    p + J lies in p + J' with J' = I_0 + hull(0, h D), D the range over y, s in
    [0, h] and j in J of f(p + j) - d/ds p, computed in TM arithmetic so that the
    polynomial terms of f(p) cancel d/ds p before the remaining ones are bounded;
    J is valid once J' is inside J (starting from [-eps, eps] and widening to the
    image plus eps while it is not, at most `tries` times, and giving up once J is
    unbounded: the theorem asks for a bounded interval), then refined by R more images;
  * preconditioning (linear reparameterisation of the step-end model c + S y + r,
    r in J): the centre of J moves into c and the rest is absorbed into the linear part,
    S y + r = S D y' with D = diag(1 + |S^-1| rad J) and y' = D^-1 (y + S^-1 r) in
    [-1, 1]^n (the next seed has no remainder); when S is singular or too ill-conditioned
    (a column of S^-1 S off the identity by more than 1e-9) the interval is carried as
    the seed's remainder instead.  A held input u = c_u + P_u y (+) I_u follows the same
    change of generators: P_u <- P_u D and I_u grows by |P_u S^-1| rad J;
  * the box of a segment is the interval bound of X over y and s in [0, h]; the box
    of a time point i h that of the step-end model.
"""
from __future__ import annotations

import numpy as np

from . import tm as _tm


# ---------------------------------------------------------------------------------
# Quasi-quadratic TM arithmetic (vectors of n components over m generators)
# ---------------------------------------------------------------------------------
class QTM:
    __slots__ = ("c", "L", "l", "M", "w", "lo", "hi")

    def __init__(self, c, L, l, M, w, lo, hi):
        self.c, self.L, self.l, self.M, self.w, self.lo, self.hi = c, L, l, M, w, lo, hi

    @staticmethod
    def const(c, m):
        n = len(c)
        z = np.zeros(n)
        return QTM(np.asarray(c, float), np.zeros((n, m)), z.copy(), np.zeros((n, m)), z.copy(), z.copy(), z.copy())

    @staticmethod
    def linear(c, S, lo=None, hi=None):
        n, m = S.shape
        z = np.zeros(n)
        return QTM(np.asarray(c, float), np.asarray(S, float), z.copy(), np.zeros((n, m)), z.copy(),
                   z.copy() if lo is None else np.asarray(lo, float), z.copy() if hi is None else np.asarray(hi, float))

    def poly_range(self, h):
        """Interval of the polynomial part over y in [-1,1]^m, s in [0, h] (term by term)."""
        r = np.abs(self.L).sum(axis=1) + h * np.abs(self.M).sum(axis=1)
        ls_lo, ls_hi = np.minimum(0.0, self.l * h), np.maximum(0.0, self.l * h)
        ws_lo, ws_hi = np.minimum(0.0, self.w * h * h), np.maximum(0.0, self.w * h * h)
        return self.c - r + ls_lo + ws_lo, self.c + r + ls_hi + ws_hi

    def range(self, h):
        lo, hi = self.poly_range(h)
        return lo + self.lo, hi + self.hi

    def __add__(self, o):
        return QTM(self.c + o.c, self.L + o.L, self.l + o.l, self.M + o.M, self.w + o.w, self.lo + o.lo, self.hi + o.hi)

    def __sub__(self, o):
        return QTM(self.c - o.c, self.L - o.L, self.l - o.l, self.M - o.M, self.w - o.w, self.lo - o.hi, self.hi - o.lo)

    def scale_rows(self, a):
        """Multiply component i by the constant a_i."""
        lo, hi = a * self.lo, a * self.hi
        return QTM(a * self.c, a[:, None] * self.L, a * self.l, a[:, None] * self.M, a * self.w,
                   np.minimum(lo, hi), np.maximum(lo, hi))

    def linmap(self, F):
        """F X (a constant matrix acting on the components); the interval part by interval
        matrix-vector product."""
        Fp, Fn = np.maximum(F, 0.0), np.minimum(F, 0.0)
        return QTM(F @ self.c, F @ self.L, F @ self.l, F @ self.M, F @ self.w,
                   Fp @ self.lo + Fn @ self.hi, Fp @ self.hi + Fn @ self.lo)


def _iv_mul(alo, ahi, blo, bhi):
    p = np.stack([alo * blo, alo * bhi, ahi * blo, ahi * bhi])
    return p.min(axis=0), p.max(axis=0)


def qtm_mul(a: QTM, b: QTM, h):
    """Componentwise product a_i b_i (vectors of TMs): the monomials {1, y, s, s y, s^2}
    of the product of the polynomial parts are kept, every other monomial (y y, s y y,
    s^2 y, s^3, ...) is bounded over the domain into the interval part, and the interval
    parts multiply the ranges of the other factor."""
    c = a.c * b.c
    L = a.c[:, None] * b.L + b.c[:, None] * a.L
    l = a.c * b.l + b.c * a.l
    M = a.c[:, None] * b.M + b.c[:, None] * a.M + a.l[:, None] * b.L + b.l[:, None] * a.L
    w = a.c * b.w + b.c * a.w + a.l * b.l
    # dropped monomials: (L_a y)(L_b y), s (L_a y)(M_b y) + ..., bounded term by term
    lo = np.zeros_like(c); hi = np.zeros_like(c)

    def add(iv):
        nonlocal lo, hi
        lo = lo + iv[0]; hi = hi + iv[1]

    # (L_a y)(L_b y) = sum_jk La_j Lb_k y_j y_k: y_j^2 in [0, 1], y_j y_k in [-1, 1]
    P = a.L[:, :, None] * b.L[:, None, :]
    diag = np.einsum("ijj->ij", P)
    off = np.abs(P).sum(axis=(1, 2)) - np.abs(diag).sum(axis=1)
    add((np.minimum(diag, 0.0).sum(axis=1) - off, np.maximum(diag, 0.0).sum(axis=1) + off))
    # s y y terms: (L_a y)(M_b y) s + (M_a y)(L_b y) s, |y y| <= 1, s in [0, h]
    t1 = (np.abs(a.L)[:, :, None] * np.abs(b.M)[:, None, :]).sum(axis=(1, 2)) + \
         (np.abs(a.M)[:, :, None] * np.abs(b.L)[:, None, :]).sum(axis=(1, 2))
    add((-h * t1, h * t1))
    # s^2 y terms: l_a s (M_b y) s + l_b s (M_a y) s + w s^2 (L y) cross terms
    t2 = np.abs(a.l) * np.abs(b.M).sum(axis=1) + np.abs(b.l) * np.abs(a.M).sum(axis=1) + \
        np.abs(a.w) * np.abs(b.L).sum(axis=1) + np.abs(b.w) * np.abs(a.L).sum(axis=1)
    add((-h * h * t2, h * h * t2))
    # s^2 y y: (M_a y)(M_b y) s^2
    t3 = (np.abs(a.M)[:, :, None] * np.abs(b.M)[:, None, :]).sum(axis=(1, 2))
    add((-h * h * t3, h * h * t3))
    # s^3: l_a w_b + w_a l_b (s^3 in [0, h^3]); s^3 y: w_a M_b y + w_b M_a y; s^4: w_a w_b
    s3 = a.l * b.w + a.w * b.l
    add((np.minimum(0.0, s3 * h ** 3), np.maximum(0.0, s3 * h ** 3)))
    t4 = np.abs(a.w) * np.abs(b.M).sum(axis=1) + np.abs(b.w) * np.abs(a.M).sum(axis=1)
    add((-h ** 3 * t4, h ** 3 * t4))
    s4 = a.w * b.w
    add((np.minimum(0.0, s4 * h ** 4), np.maximum(0.0, s4 * h ** 4)))
    # interval parts: Ia * range(b) + Ib * range(a) (polynomial ranges) + Ia Ib
    alo, ahi = a.poly_range(h)
    blo, bhi = b.poly_range(h)
    add(_iv_mul(a.lo, a.hi, blo, bhi))
    add(_iv_mul(b.lo, b.hi, alo, ahi))
    add(_iv_mul(a.lo, a.hi, b.lo, b.hi))
    return QTM(c, L, l, M, w, lo, hi)


def integrate(X: QTM, h):
    """x0-free part of int_0^s X ds, truncated to the representation: c s, (L y) s,
    l s^2 / 2 are kept; (M y) s^2 / 2 and w s^3 / 3 are dropped (polynomial Picard only)."""
    n, m = X.L.shape
    z = np.zeros(n)
    return QTM(z.copy(), np.zeros((n, m)), X.c.copy(), X.L.copy(), 0.5 * X.l, z.copy(), z.copy())


# ---------------------------------------------------------------------------------
# Dynamics: f(x, u) = a + F x + G u + x^T Q x (per component)
# ---------------------------------------------------------------------------------
class QuadDynamics:
    def __init__(self, a, F, G=None, Q=None):
        self.a = np.asarray(a, float)
        self.F = np.asarray(F, float)
        n = self.F.shape[0]
        self.G = np.zeros((n, 0)) if G is None else np.asarray(G, float)
        self.Q = np.zeros((n, n, n)) if Q is None else np.asarray(Q, float)

    @property
    def n(self):
        return self.F.shape[0]

    def __call__(self, x, u=None):
        x = np.asarray(x, float)
        v = self.a + self.F @ x + np.einsum("ijk,j,k->i", self.Q, x, x)
        if self.G.shape[1]:
            v = v + self.G @ np.asarray(u, float)
        return v

    def tm(self, X: QTM, U: QTM | None, h):
        """TM of f over the state TM X and the input TM U (same generators)."""
        n = self.n
        m = X.L.shape[1]
        out = QTM.const(self.a, m) + X.linmap(self.F)
        if self.G.shape[1]:
            out = out + U.linmap(self.G)
        # quadratic terms: sum_jk Q_ijk x_j x_k = sum_{j <= k} Qs_ijk x_j x_k over the
        # monomials x_j x_k (Qs_ijk = Q_ijk + Q_ikj for j < k, Q_ijj on the diagonal),
        # each formed once as a product of component TMs
        for j in range(n):
            for k in range(j, n):
                q = self.Q[:, j, k] + (self.Q[:, k, j] if k != j else 0.0)
                if not (np.any(self.Q[:, j, k]) or np.any(self.Q[:, k, j])):
                    continue
                xj = _pick(X, j, n); xk = _pick(X, k, n)
                out = out + qtm_mul(xj, xk, h).scale_rows(q)
        return out


def _pick(X: QTM, j, n):
    """The TM whose every component is component j of X (broadcast)."""
    return QTM(np.full(n, X.c[j]), np.repeat(X.L[j:j + 1], n, axis=0), np.full(n, X.l[j]),
               np.repeat(X.M[j:j + 1], n, axis=0), np.full(n, X.w[j]), np.full(n, X.lo[j]), np.full(n, X.hi[j]))


# ---------------------------------------------------------------------------------
# One flowpipe step (Theorem "TM flowpipe step via Picard iteration")
# ---------------------------------------------------------------------------------
def picard_step(f: QuadDynamics, c, S, I0lo, I0hi, h, U=None, order=2, eps=1e-9, tries=40, rounds=3):
    """Flowpipe X(y, s) = p(y, s) + J over s in [0, h] from the seed c + S y + I0.

    Returns (QTM p with J as its interval part, ok).  ok is False when no contractive
    remainder was found (the caller reports an unbounded set)."""
    n, m = S.shape
    x0 = QTM.linear(c, S)
    g = QTM.linear(c, S)
    for _ in range(order):
        fg = f.tm(g, U, h)
        g = x0 + integrate(fg, h)
        g.lo[:] = 0.0; g.hi[:] = 0.0
    p = g
    dp = QTM(p.l.copy(), p.M.copy(), 2.0 * p.w, np.zeros((n, m)), np.zeros(n), np.zeros(n), np.zeros(n))

    def image(Jlo, Jhi):
        X = QTM(p.c, p.L, p.l, p.M, p.w, Jlo, Jhi)
        D = f.tm(X, U, h) - dp
        dlo, dhi = D.range(h)
        return I0lo + np.minimum(0.0, h * dlo), I0hi + np.maximum(0.0, h * dhi)

    Jlo, Jhi = I0lo - eps, I0hi + eps
    ok = False
    if not (np.all(np.isfinite(I0lo)) and np.all(np.isfinite(I0hi))):
        tries = 0   # an unbounded initial set has no bounded remainder
    for _ in range(tries):
        nlo, nhi = image(Jlo, Jhi)
        if np.all(nlo >= Jlo) and np.all(nhi <= Jhi):
            ok = True
            Jlo, Jhi = nlo, nhi
            break
        # widen to the image plus eps (and keep the old set inside)
        wid = np.maximum(nhi - nlo, eps)
        Jlo = np.minimum(Jlo, nlo) - 0.5 * wid
        Jhi = np.maximum(Jhi, nhi) + 0.5 * wid
        if not (np.all(np.isfinite(Jlo)) and np.all(np.isfinite(Jhi))):
            break   # an unbounded set is no remainder of the theorem
    if not ok:
        return QTM(p.c, p.L, p.l, p.M, p.w, np.full(n, -np.inf), np.full(n, np.inf)), False
    for _ in range(rounds):
        nlo, nhi = image(Jlo, Jhi)
        Jlo, Jhi = np.maximum(Jlo, nlo), np.minimum(Jhi, nhi)
    return QTM(p.c, p.L, p.l, p.M, p.w, Jlo, Jhi), True


def end_model(X: QTM, h):
    """The step-end model X(., h) (linear in y): (c, S, I_lo, I_hi)."""
    return X.c + X.l * h + X.w * h * h, X.L + h * X.M, X.lo.copy(), X.hi.copy()


def precondition(c, S, lo, hi, U=None):
    """Step (A): absorb the remainder into the linear part (see the module header).
    Returns (c, S, lo, hi, U) of the next seed."""
    n = S.shape[0]
    mid, rad = 0.5 * (lo + hi), 0.5 * (hi - lo)
    if not (np.all(np.isfinite(rad)) and np.all(np.isfinite(S))):
        return c, S, lo, hi, U
    try:
        Si = np.linalg.inv(S)
    except np.linalg.LinAlgError:
        return c, S, lo, hi, U
    if not np.all(np.isfinite(Si)) or np.abs(Si @ S - np.eye(n)).max() > 1e-9:
        return c, S, lo, hi, U
    delta = np.abs(Si) @ rad
    D = 1.0 + delta
    c2, S2 = c + mid, S * D[None, :]
    if U is not None:
        extra = np.abs(U.L @ Si) @ rad
        U = QTM.linear(U.c, U.L * D[None, :], U.lo - extra, U.hi + extra)
    return c2, S2, np.zeros(n), np.zeros(n), U


def flowpipe(f: QuadDynamics, xc, xr, h, N, **kw):
    """Boxes of the time points 0, h, .., N h (N+1 x n x 2) and of the segments (N x n x 2)
    of the flowpipe from the box [xc - xr, xc + xr] (Algorithm "Reachability of CT
    Dynamics with TM Flowpipe", identity preconditioning)."""
    n = f.n
    c, S = np.asarray(xc, float).copy(), np.diag(np.asarray(xr, float))
    lo, hi = np.zeros(n), np.zeros(n)
    points = [np.stack([c - np.abs(S).sum(axis=1), c + np.abs(S).sum(axis=1)], axis=1)]
    segs = []
    ok_all = True
    for _ in range(N):
        X, ok = picard_step(f, c, S, lo, hi, h, **kw)
        ok_all &= ok
        slo, shi = X.range(h)
        segs.append(np.stack([slo, shi], axis=1))
        c, S, lo, hi = end_model(X, h)
        r = np.abs(S).sum(axis=1)
        points.append(np.stack([c - r + lo, c + r + hi], axis=1))
        c, S, lo, hi, _ = precondition(c, S, lo, hi)
    return np.array(points), np.array(segs), ok_all


# ---------------------------------------------------------------------------------
# CT closed loop with an NN controller (Algorithm "Reachability of CT NN Control Systems")
# ---------------------------------------------------------------------------------
def controller_tm(net, c, S, lo, hi):
    """Linear TM of the controller output u = net(x) over x = c + S y + [lo, hi]
    (Theorem "CROWN bounds of NN with linear TM input", shared slope): the stepwise
    TM step of ``oracle/tm.py`` with the loop x' = 0 x + I y, the centre of its interval
    part moved into the constant."""
    n_u = net.widths[-1]
    ctl = type(net)(net.Ws, net.bs, np.zeros((n_u, net.widths[0])), np.eye(n_u))
    (cu, Pu, ulo, uhi), _, _ = _tm.tm_step(ctl, c, S, lo, hi)
    # the centre of the interval part belongs to the polynomial part (the Picard
    # polynomial then carries the input's constant drift)
    mid = 0.5 * (ulo + uhi)
    return cu + mid, Pu, ulo - mid, uhi - mid


def closed_loop(f: QuadDynamics, net, xc, xr, h, K, N_ctl, **kw):
    """Boxes of the time points (N_ctl K + 1 x n x 2) and of the segments of the CT
    closed loop: at every control boundary the controller is certified on the state's
    TM (a linear TM of u over the same generators), then K flowpipe steps of
    x' = f(x, u) with u held (zero-order hold)."""
    n = f.n
    c, S = np.asarray(xc, float).copy(), np.diag(np.asarray(xr, float))
    lo, hi = np.zeros(n), np.zeros(n)
    points = [np.stack([c - np.abs(S).sum(axis=1), c + np.abs(S).sum(axis=1)], axis=1)]
    segs = []
    ok_all = True
    for _ in range(N_ctl):
        cu, Pu, ulo, uhi = controller_tm(net, c, S, lo, hi)
        U = QTM.linear(cu, Pu, ulo, uhi)
        for _ in range(K):
            X, ok = picard_step(f, c, S, lo, hi, h, U=U, **kw)
            ok_all &= ok
            slo, shi = X.range(h)
            segs.append(np.stack([slo, shi], axis=1))
            c, S, lo, hi = end_model(X, h)
            r = np.abs(S).sum(axis=1)
            points.append(np.stack([c - r + lo, c + r + hi], axis=1))
            c, S, lo, hi, U = precondition(c, S, lo, hi, U)
    return np.array(points), np.array(segs), ok_all
