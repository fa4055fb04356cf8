"""Value pins of the oracle's intermediate bounds and of its shared-slope Taylor-model step.

Soundness sandwiches cannot tell a CROWN intermediate bound from a looser interval one,
nor the shared-slope offsets of Theorem "CROWN bounds of NN with linear TM input" from
a symmetric widening of them.  The pins here fix the values themselves:

* a network whose first hidden layer is stably active is affine up to its second hidden
  layer, so the CROWN bounds of that layer (Theorem "CROWN linear bounds of NN") are the
  exact range of the composed affine map, strictly inside the interval bounds; and the
  whole bound computation equals that of the network with the two affine layers merged;
* with one hidden layer below a row, CROWN with fixed relaxation lines is the optimum of
  the linear program over those lines (each neuron's line is picked by the sign of its
  coefficient, and the rest is a linear function over the box), so the second-layer
  bounds equal max(interval bound, LP optimum); deeper rows are bounded above by the LP
  over all relaxed layers and by the exact minimum;
* hand-worked shared-slope steps: y = relu(x) on [-1, 2] has the chord slope s = 2/3 on
  both sides, lower offset 0 and upper offset 2/3, which fixes the first step's box and
  Taylor model, and the second step's interval product.
"""
import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import crown, exact, tm
from paper_2605_25346_amd.workloads import Network, make_network


def net_from(Ws, bs, A=None, B=None):
    return Network([np.asarray(W, float) for W in Ws], [np.asarray(b, float) for b in bs],
                   None if A is None else np.asarray(A, float), None if B is None else np.asarray(B, float))


def _affine_range(M, m, xc, xr):
    """Exact range of M x + m over the box (the textbook closed form of an affine map)."""
    return M @ xc + m - np.abs(M) @ xr, M @ xc + m + np.abs(M) @ xr


# ------------------------------------------------------------------ (a) active first layer
def _active_first_layer_case(seed, widths, lift=40.0):
    rng = np.random.default_rng(seed)
    net = make_network(rng, widths, np.float64)
    net.bs[0] = net.bs[0] + lift          # every first-layer neuron is active over the box
    xc = rng.uniform(-1, 1, widths[0]); xr = np.full(widths[0], 0.3)
    l1, u1 = _affine_range(net.Ws[0], net.bs[0], xc, xr)
    assert np.all(l1 > 0)
    # centre the second layer on zero so that most of its neurons are unstable
    M = net.Ws[1] @ net.Ws[0]
    m = net.Ws[1] @ net.bs[0] + net.bs[1]
    net.bs[1] = net.bs[1] - (M @ xc + m)
    return net, xc, xr


@pytest.mark.parametrize("seed,widths", [(0, [3, 6, 5, 2]), (1, [4, 8, 8, 3]), (2, [2, 5, 6, 4, 2])])
def test_second_layer_bounds_are_exact_affine_range(seed, widths):
    """Layer 1 active: z_2 = W_2 (W_1 x + b_1) + b_2 is affine in x, so its CROWN bounds equal
    the exact range, which is strictly tighter than interval propagation here."""
    net, xc, xr = _active_first_layer_case(seed, widths)
    bounds, rows, status = crown.intermediate_bounds(net, xc, xr)
    assert status == 0
    M = net.Ws[1] @ net.Ws[0]
    m = net.Ws[1] @ net.bs[0] + net.bs[1]
    lo, hi = _affine_range(M, m, xc, xr)
    ibl, ibu = crown.ibp_next(net.Ws[1], net.bs[1], *bounds[0])
    uns = (ibl < 0) & (ibu > 0)
    assert uns.sum() >= 2
    # IBP-unstable neurons get the CROWN (= exact) range; the rest keep IBP
    np.testing.assert_allclose(bounds[1][0][uns], lo[uns], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(bounds[1][1][uns], hi[uns], rtol=1e-12, atol=1e-12)
    assert np.all(lo[uns] > ibl[uns] + 1e-6) and np.all(hi[uns] < ibu[uns] - 1e-6)
    assert rows[1] == 2 * int(uns.sum())


@pytest.mark.parametrize("seed,widths", [(0, [3, 6, 5, 2]), (1, [4, 8, 8, 3]), (2, [2, 5, 6, 4, 2])])
def test_active_first_layer_merges_into_the_second(seed, widths):
    """The same network with the two affine layers merged (W_2 W_1, W_2 b_1 + b_2) has the
    same bounds at every later layer and the same final bounds: the final bound depends on
    the second layer's bounds, which must be the exact range."""
    net, xc, xr = _active_first_layer_case(seed, widths)
    merged = net_from([net.Ws[1] @ net.Ws[0]] + net.Ws[2:], [net.Ws[1] @ net.bs[0] + net.bs[1]] + net.bs[2:])
    full = crown.crown(net, xc, xr)
    red = crown.crown(merged, xc, xr)
    for (l, u), (lr, ur) in zip(full["bounds"][1:], red["bounds"]):
        np.testing.assert_allclose(l, lr, rtol=1e-11, atol=1e-11)
        np.testing.assert_allclose(u, ur, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(full["lb"], red["lb"], rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(full["ub"], red["ub"], rtol=1e-11, atol=1e-11)
    # with the second layer's bounds replaced by interval bounds the final bound moves
    # (so this pin sees a dropped CROWN row)
    ibl, ibu = crown.ibp_next(net.Ws[1], net.bs[1], *full["bounds"][0])
    loose = [full["bounds"][0], (ibl, ibu)] + full["bounds"][2:]
    lf = crown.final_bounds(net, loose, xc, xr)
    assert np.max(np.abs(lf["lb"] - full["lb"])) > 1e-6 or np.max(np.abs(lf["ub"] - full["ub"])) > 1e-6


# ------------------------------------------------------------------ (c) LP over the relaxation
def _relaxation_lp(W1, b1, l1, u1, alpha_of, w_obj, xc, xr, shared=False):
    """min w_obj . h over x in the box and h in the relaxation of h = relu(W_1 x + b_1)
    with one lower line per unstable neuron (slope alpha, or the chord slope if shared)
    and the chord above; stable neurons are exact (h = z or h = 0)."""
    n0, n1 = W1.shape[1], W1.shape[0]
    kind, s, t, alpha0 = crown.relu_relaxation(l1, u1)
    nv = n0 + n1
    A_ub, b_ub, A_eq, b_eq = [], [], [], []
    bnds = [(c - r, c + r) for c, r in zip(xc, xr)] + [(None, None)] * n1
    for i in range(n1):
        row_z = np.zeros(nv); row_z[:n0] = W1[i]          # z_i = row_z . v + b1_i
        e_h = np.zeros(nv); e_h[n0 + i] = 1.0
        if kind[i] == crown.INACTIVE:
            bnds[n0 + i] = (0.0, 0.0)
        elif kind[i] == crown.ACTIVE:
            A_eq.append(e_h - row_z); b_eq.append(b1[i])
        else:
            a = s[i] if shared else alpha_of[i]
            A_ub.append(a * row_z - e_h); b_ub.append(-a * b1[i])                  # h >= a z
            A_ub.append(e_h - s[i] * row_z); b_ub.append(s[i] * b1[i] + t[i])      # h <= s z + t
    c = np.concatenate([np.zeros(n0), w_obj])
    res = linprog(c, A_ub=np.array(A_ub) if A_ub else None, b_ub=np.array(b_ub) if b_ub else None,
                  A_eq=np.array(A_eq) if A_eq else None, b_eq=np.array(b_eq) if b_eq else None,
                  bounds=bnds, method="highs")
    assert res.status == 0
    return res.fun


@pytest.mark.parametrize("seed", range(12))
def test_second_layer_bounds_equal_the_relaxation_lp(seed):
    """Plain CROWN (adaptive slopes): each IBP-unstable, unsplit neuron of layer 2 gets
    max(IBP, LP) as its bounds, LP = the optimum over layer 1's relaxation lines."""
    rng = np.random.default_rng(100 + seed)
    n0, n1, n2 = int(rng.integers(1, 4)), int(rng.integers(2, 7)), int(rng.integers(2, 7))
    net = make_network(rng, [n0, n1, n2, 2], np.float64)
    xc = rng.uniform(-1, 1, n0); xr = rng.uniform(0.2, 1.0, n0)
    splits = []
    if seed % 3 == 2:   # a split neuron of layer 1 is clamped and then exact in the rows
        l1, u1 = _affine_range(net.Ws[0], net.bs[0], xc, xr)
        cand = np.nonzero((l1 < 0) & (u1 > 0))[0]
        if cand.size:
            splits = [(1, int(cand[0]), 1 if seed % 2 else -1)]
    bounds, rows, status = crown.intermediate_bounds(net, xc, xr, splits)
    if status:
        pytest.skip("infeasible draw")
    l1, u1 = bounds[0]
    _, _, _, alpha0 = crown.relu_relaxation(l1, u1)
    ibl, ibu = crown.ibp_next(net.Ws[1], net.bs[1], l1, u1)
    sig = np.zeros(n2)
    checked = 0
    for j in range(n2):
        if not (ibl[j] < 0 < ibu[j]):
            assert bounds[1][0][j] == ibl[j] and bounds[1][1][j] == ibu[j]
            continue
        lo = _relaxation_lp(net.Ws[0], net.bs[0], l1, u1, alpha0, net.Ws[1][j], xc, xr) + net.bs[1][j]
        hi = -_relaxation_lp(net.Ws[0], net.bs[0], l1, u1, alpha0, -net.Ws[1][j], xc, xr) + net.bs[1][j]
        # the upper row -e_j takes the lower line where -W_2[j] >= 0: same LP, negated objective
        tol = 1e-8 * max(1.0, abs(lo), abs(hi))
        assert abs(bounds[1][0][j] - max(ibl[j], lo)) <= tol, (seed, j, bounds[1][0][j], ibl[j], lo)
        assert abs(bounds[1][1][j] - min(ibu[j], hi)) <= tol, (seed, j, bounds[1][1][j], ibu[j], hi)
        checked += 1
    assert rows[1] == 2 * checked


@pytest.mark.parametrize("seed", range(6))
def test_deeper_rows_below_the_relaxation_lp(seed):
    """A row through two relaxed layers is a feasible dual of the LP over both layers'
    relaxation lines: CROWN <= LP <= exact minimum (pattern enumeration)."""
    rng = np.random.default_rng(200 + seed)
    net = make_network(rng, [2, 4, 4, 3, 1], np.float64)
    xc = rng.uniform(-1, 1, 2); xr = np.full(2, 0.6)
    bounds, _, status = crown.intermediate_bounds(net, xc, xr)
    assert status == 0
    # LP over layers 1 and 2 for each neuron of layer 3 (objective W_3[j] h_2 + b_3[j])
    (l1, u1), (l2, u2) = bounds[0], bounds[1]
    k1, s1, t1, a1 = crown.relu_relaxation(l1, u1)
    k2, s2, t2, a2 = crown.relu_relaxation(l2, u2)
    n0, n1, n2 = 2, 4, 4
    nv = n0 + n1 + n2
    for j in range(3):
        for sgn in (1.0, -1.0):
            A_ub, b_ub, A_eq, b_eq = [], [], [], []
            bnds = [(c - r, c + r) for c, r in zip(xc, xr)] + [(None, None)] * (n1 + n2)
            for (kind, s, t, a, W, b, zoff, hoff, n, nin) in (
                    (k1, s1, t1, a1, net.Ws[0], net.bs[0], 0, n0, n1, n0),
                    (k2, s2, t2, a2, net.Ws[1], net.bs[1], n0, n0 + n1, n2, n1)):
                for i in range(n):
                    rz = np.zeros(nv); rz[zoff:zoff + nin] = W[i]
                    eh = np.zeros(nv); eh[hoff + i] = 1.0
                    if kind[i] == crown.INACTIVE:
                        bnds[hoff + i] = (0.0, 0.0)
                    elif kind[i] == crown.ACTIVE:
                        A_eq.append(eh - rz); b_eq.append(b[i])
                    else:
                        A_ub.append(a[i] * rz - eh); b_ub.append(-a[i] * b[i])
                        A_ub.append(eh - s[i] * rz); b_ub.append(s[i] * b[i] + t[i])
            cobj = np.zeros(nv); cobj[n0 + n1:] = sgn * net.Ws[2][j]
            res = linprog(cobj, A_ub=np.array(A_ub) if A_ub else None, b_ub=np.array(b_ub) if b_ub else None,
                          A_eq=np.array(A_eq) if A_eq else None, b_eq=np.array(b_eq) if b_eq else None,
                          bounds=bnds, method="highs")
            assert res.status == 0
            lp = res.fun + sgn * net.bs[2][j]
            relax = [crown.relu_relaxation(*bk) for bk in bounds[:2]]
            E = np.zeros((1, 3)); E[0, j] = sgn
            r = crown.backward(net, relax, 3, E)
            cr = crown.concretize_box(r["w"], r["acc"], xc, xr)[0]
            sub = Network(net.Ws[:3], net.bs[:3])
            ex = exact.exact_min(sub, xc, xr, np.array([1.0 if q == j else 0.0 for q in range(3)]) * sgn)
            assert cr <= lp + 1e-9 and lp <= ex + 1e-9, (seed, j, sgn, cr, lp, ex)


# ------------------------------------------------------------------ (b) shared-slope steps
def test_shared_slope_one_neuron_step():
    """x' = relu(x) (A = 0, B = 1) from x in [-1, 2]: chord slope s = 2/3 on both sides,
    lower offset 0 and upper offset t = -s l = 2/3, so the Taylor model after one step is
    c = s * 1/2 = 1/3, P = s * 3/2 = 1, I = [0, 2/3] and the box is [-2/3, 2]."""
    net = net_from([[[1.0]], [[1.0]]], [[0.0], [0.0]], A=[[0.0]], B=[[1.0]])
    boxes, st = tm.reach_dt(net, np.array([0.5]), np.array([1.5]), 1)
    np.testing.assert_allclose(st["c"], [1.0 / 3.0], atol=1e-15)
    np.testing.assert_allclose(st["P"], [[1.0]], atol=1e-15)
    np.testing.assert_allclose([st["Ilo"][0], st["Ihi"][0]], [0.0, 2.0 / 3.0], atol=1e-15)
    np.testing.assert_allclose(boxes[1, 0], [-2.0 / 3.0, 2.0], atol=1e-15)


def test_shared_slope_two_steps_interval_product():
    """Second step of x' = relu(x): the input TM 1/3 + z + [0, 2/3] has range [-2/3, 2], so
    s = 3/4, t = 1/2; the new TM is c = 1/4, P = 3/4, I = s [0, 2/3] + [0, 1/2] = [0, 1],
    box [-1/2, 2]."""
    net = net_from([[[1.0]], [[1.0]]], [[0.0], [0.0]], A=[[0.0]], B=[[1.0]])
    boxes, st = tm.reach_dt(net, np.array([0.5]), np.array([1.5]), 2)
    np.testing.assert_allclose(st["c"], [0.25], atol=1e-15)
    np.testing.assert_allclose(st["P"], [[0.75]], atol=1e-15)
    np.testing.assert_allclose([st["Ilo"][0], st["Ihi"][0]], [0.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(boxes[2, 0], [-0.5, 2.0], atol=1e-15)


def test_shared_slope_negative_output_weight():
    """x' = -relu(x) (B = -1): the row multiplier is g = -1, so the offsets swap sides:
    lower -2/3 (min(0, g t)), upper 0; box [-2, 2/3]."""
    net = net_from([[[1.0]], [[1.0]]], [[0.0], [0.0]], A=[[0.0]], B=[[-1.0]])
    boxes, st = tm.reach_dt(net, np.array([0.5]), np.array([1.5]), 1)
    np.testing.assert_allclose([st["Ilo"][0], st["Ihi"][0]], [-2.0 / 3.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(boxes[1, 0], [-2.0, 2.0 / 3.0], atol=1e-15)


def test_tm_intermediate_crown_rows_matter():
    """x' = x + relu(h_1 - h_2) with h = relu((x, x)) on x in [1, 3]: layer 1 is active, so
    z_2 = x - x = 0 exactly (CROWN on the TM input) and the neuron is inactive: the box is
    [1, 3].  Interval bounds alone would give z_2 in [-2, 2] and the box [1, 4]."""
    net = net_from([[[1.0], [1.0]], [[1.0, -1.0]], [[1.0]]], [[0.0, 0.0], [0.0], [0.0]], A=[[1.0]], B=[[1.0]])
    boxes, st = tm.reach_dt(net, np.array([2.0]), np.array([1.0]), 1)
    np.testing.assert_allclose(boxes[1, 0], [1.0, 3.0], atol=1e-14)
    bounds, rows = tm.tm_intermediate_bounds(net, np.array([2.0]), np.eye(1), np.zeros(1), np.zeros(1))
    np.testing.assert_allclose([bounds[1][0][0], bounds[1][1][0]], [0.0, 0.0], atol=1e-14)
    assert rows[1] == 1


@pytest.mark.parametrize("seed", range(8))
def test_tm_second_layer_bounds_equal_the_parallel_relaxation_lp(seed):
    """First step of the TM reach (the TM is the box): every IBP-unstable neuron of layer 2
    gets max(IBP, LP) with the LP over layer 1's parallel relaxation (chord slope below and
    above, offsets 0 and t)."""
    rng = np.random.default_rng(300 + seed)
    n0, n1, n2 = int(rng.integers(1, 4)), int(rng.integers(2, 7)), int(rng.integers(2, 7))
    net = make_network(rng, [n0, n1, n2, 2], np.float64)
    net.A = np.eye(n0); net.B = rng.normal(0, 0.5, (n0, 2))
    xc = rng.uniform(-1, 1, n0); xr = rng.uniform(0.2, 1.0, n0)
    bounds, rows = tm.tm_intermediate_bounds(net, xc, np.diag(xr), np.zeros(n0), np.zeros(n0))
    l1, u1 = bounds[0]
    ibl, ibu = crown.ibp_next(net.Ws[1], net.bs[1], l1, u1)
    checked = 0
    for j in range(n2):
        if not (ibl[j] < 0 < ibu[j]):
            continue
        lo = _relaxation_lp(net.Ws[0], net.bs[0], l1, u1, None, net.Ws[1][j], xc, xr, shared=True) + net.bs[1][j]
        hi = -_relaxation_lp(net.Ws[0], net.bs[0], l1, u1, None, -net.Ws[1][j], xc, xr, shared=True) + net.bs[1][j]
        tol = 1e-8 * max(1.0, abs(lo), abs(hi))
        assert abs(bounds[1][0][j] - max(ibl[j], lo)) <= tol, (seed, j, bounds[1][0][j], ibl[j], lo)
        assert abs(bounds[1][1][j] - min(ibu[j], hi)) <= tol, (seed, j, bounds[1][1][j], ibu[j], hi)
        checked += 1
    assert rows[1] == checked
