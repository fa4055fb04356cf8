"""Seeded synthetic workloads for batched bound propagation.

This module only draws random inputs: network weights and biases, closed-loop
matrices, input boxes and branch-and-bound split constraints.  It holds none of
the bounding method's arithmetic, so both the FP64 reference and the GPU path
consume exactly the same arrays.  The one piece of arithmetic here is a plain
forward evaluation of the ReLU network at a handful of sample points, used only
to pick split candidates among neurons whose sign provably changes inside a box
(a neuron that takes both signs at two sampled points is split, as a
branch-and-bound driver would split it).

Shapes follow the paper's controllers and dynamics models (hidden widths 64/96
in the appendix on experimental details, horizon 10 and batches of 128+ initial
sets in the reachability-tool evaluation, 8-way splitting and 20 gradient
iterations in the table of refinement strategies).  The paper's own trained
robot models and datasets are not used: random initialisation N(0, 2/fan_in)
stands in for them.

Conventions (documented once, used everywhere):
  * ``N(mu, s2)`` is read as mean/variance, so biases N(0, 0.01) have std 0.1.
  * A network is a list of (W_k, b_k), W_k of shape (n_k, n_{k-1}) row-major,
    z_1 = W_1 x + b_1, h_k = relu(z_k), z_{k+1} = W_{k+1} h_k + b_{k+1}.
  * Splits are (hidden layer k in 1..L-1, neuron j, sign s) with s = +1 meaning
    z_k[j] >= 0 and s = -1 meaning z_k[j] <= 0, stored as CSR per subdomain.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Network", "Batch", "Workload", "make_network", "make_workload",
    "CONFIGS", "config_workload", "pack_splits", "unpack_splits", "random_duals",
    "CtWorkload", "make_ct_workload",
]


@dataclass
class Network:
    """A ReLU MLP, optionally in a closed loop x' = A x + B y."""
    Ws: List[np.ndarray]
    bs: List[np.ndarray]
    A: Optional[np.ndarray] = None     # (n_state, n_0) float64, closed loop only
    B: Optional[np.ndarray] = None     # (n_state, n_L) float64, closed loop only

    @property
    def widths(self) -> List[int]:
        return [self.Ws[0].shape[1]] + [W.shape[0] for W in self.Ws]

    @property
    def n_layers(self) -> int:
        return len(self.Ws)

    @property
    def hidden(self) -> List[int]:
        return [W.shape[0] for W in self.Ws[:-1]]

    @property
    def closed_loop(self) -> bool:
        return self.A is not None


@dataclass
class Batch:
    """A batch of subdomains: boxes, split constraints and network ids."""
    x_center: np.ndarray               # (S, n0) float64
    x_radius: np.ndarray               # (S, n0) float64
    split_ptr: np.ndarray              # (S+1,) int32
    split_layer: np.ndarray            # (nnz,) int32, hidden layer 1..L-1
    split_neuron: np.ndarray           # (nnz,) int32
    split_sign: np.ndarray             # (nnz,) int32, +1 or -1
    net_id: np.ndarray                 # (S,) int32

    @property
    def n_sub(self) -> int:
        return self.x_center.shape[0]

    def splits_of(self, s: int):
        a, b = int(self.split_ptr[s]), int(self.split_ptr[s + 1])
        return [(int(self.split_layer[i]), int(self.split_neuron[i]), int(self.split_sign[i]))
                for i in range(a, b)]

    def subset(self, idx) -> "Batch":
        idx = np.asarray(idx, dtype=np.int64)
        ptr = [0]
        lay, neu, sg = [], [], []
        for s in idx:
            a, b = int(self.split_ptr[s]), int(self.split_ptr[s + 1])
            lay.append(self.split_layer[a:b]); neu.append(self.split_neuron[a:b]); sg.append(self.split_sign[a:b])
            ptr.append(ptr[-1] + (b - a))
        cat = lambda xs: (np.concatenate(xs) if xs else np.zeros(0)).astype(np.int32)
        return Batch(self.x_center[idx].copy(), self.x_radius[idx].copy(), np.asarray(ptr, np.int32),
                     cat(lay), cat(neu), cat(sg), self.net_id[idx].copy())


@dataclass
class Workload:
    name: str
    nets: List[Network]
    batch: Batch
    dtype: str = "f32"                 # arithmetic of the GPU path: "f32" or "f64"
    iters: int = 0                     # projected gradient-ascent steps (0 = plain CROWN)
    lr: float = 0.1
    horizon: int = 0                   # > 0: stepwise closed-loop reachability
    shared_slope: bool = False
    meta: dict = field(default_factory=dict)


def make_network(rng: np.random.Generator, widths, dtype=np.float32) -> Network:
    """Weights N(0, 2/fan_in), biases N(0, 0.01); drawn layer by layer (W then b)."""
    Ws, bs = [], []
    for k in range(1, len(widths)):
        fan_in = widths[k - 1]
        W = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(widths[k], fan_in))
        b = rng.normal(0.0, 0.1, size=(widths[k],))
        Ws.append(W.astype(dtype).astype(np.float64) if dtype == np.float32 else W)
        bs.append(b.astype(dtype).astype(np.float64) if dtype == np.float32 else b)
    # Values are stored in float64 holding exactly the representable numbers of
    # the GPU dtype: the network *is* its rounded weights.
    return Network(Ws, bs)


def _signed_permutation(rng, n, rho):
    """rho times a random signed permutation: spectral radius and infinity-norm rho."""
    A = np.zeros((n, n))
    A[np.arange(n), rng.permutation(n)] = rho * rng.choice([-1.0, 1.0], size=n)
    return A


def _forward_preacts(net: Network, X: np.ndarray):
    """Plain network evaluation at points X (..., n0): list of hidden pre-activations."""
    zs = []
    h = X
    for k in range(net.n_layers - 1):
        z = h @ net.Ws[k].T + net.bs[k]
        zs.append(z)
        h = np.maximum(z, 0.0)
    return zs


def _draw_splits(rng, nets, net_id, xc, xr, max_splits, n_samples=16):
    """Per subdomain: a uniform count in [0, max_splits], capped by the number of
    candidates, of distinct neurons that change sign among sampled points of the
    box; each gets a random sign with probability 1/2."""
    S = xc.shape[0]
    ptr = np.zeros(S + 1, np.int32)
    lay, neu, sg = [], [], []
    if max_splits <= 0:
        return ptr, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32)
    n0 = xc.shape[1]
    U = rng.uniform(-1.0, 1.0, size=(S, n_samples, n0))
    pts = np.concatenate([xc[:, None, :], xc[:, None, :] + U * xr[:, None, :]], axis=1)
    counts = rng.integers(0, max_splits + 1, size=S)
    cand = [None] * S
    for nid, net in enumerate(nets):
        sel = np.nonzero(net_id == nid)[0]
        if sel.size == 0:
            continue
        zs = _forward_preacts(net, pts[sel])
        pos = np.concatenate([(z > 0).any(axis=1) for z in zs], axis=1)
        neg = np.concatenate([(z < 0).any(axis=1) for z in zs], axis=1)
        flip = pos & neg
        offs = np.cumsum([0] + net.hidden)
        for ii, s in enumerate(sel):
            idx = np.nonzero(flip[ii])[0]
            cand[s] = (idx, offs)
    for s in range(S):
        idx, offs = cand[s]
        c = int(min(counts[s], idx.size))
        chosen = rng.choice(idx, size=c, replace=False) if c > 0 else np.zeros(0, np.int64)
        signs = np.where(rng.random(c) < 0.5, 1, -1)
        order = np.argsort(chosen, kind="stable")
        for g, sig in zip(chosen[order], signs[order]):
            k = int(np.searchsorted(offs, g, side="right"))  # 1-based hidden layer
            lay.append(k); neu.append(int(g - offs[k - 1])); sg.append(int(sig))
        ptr[s + 1] = ptr[s] + c
    return ptr, np.asarray(lay, np.int32), np.asarray(neu, np.int32), np.asarray(sg, np.int32)


def pack_splits(layer, neuron, sign) -> np.ndarray:
    """Pack split triples into 32-bit words: layer<<24 | (sign>0)<<16 | neuron."""
    layer = np.asarray(layer, np.uint32); neuron = np.asarray(neuron, np.uint32)
    pos = (np.asarray(sign) > 0).astype(np.uint32)
    return (layer << 24) | (pos << 16) | neuron


def unpack_splits(words):
    w = np.asarray(words, np.uint32)
    return ((w >> 24) & 0xFF).astype(np.int32), (w & 0xFFFF).astype(np.int32), np.where((w >> 16) & 1, 1, -1).astype(np.int32)


def make_workload(name, seed, net_widths, n_sub, *, closed_loop=None, radius=(0.01, 0.1),
                  center=(-1.0, 1.0), max_splits=0, dtype="f32", iters=0, lr=0.1,
                  horizon=0, shared_slope=False, n_state=None, rho=0.95, a_var=0.3, b_var=0.3,
                  A_mode="gauss", B_mode="gauss", b_gain=0.1, n_split_samples=16) -> Workload:
    """Draw a workload.  Draw order: weights then biases layer by layer (network by
    network), then A, B, then centres, radii, then split candidates, counts,
    neurons and signs, then (networks with exogenous inputs) the input sequences.

    A closed loop with n_state < n_0 takes the remaining n_0 - n_state network
    inputs as exogenous actions u_t (meta["u"], S x horizon x m, U[-1, 1]):
    x' = A [x; u] + B f([x; u]).  A_mode "residual": A = [I, 0]; B_mode
    "scaled_identity": B = b_gain I (the network predicts a scaled state increment)."""
    rng = np.random.default_rng(seed)
    npdt = np.float32 if dtype == "f32" else np.float64
    nets = [make_network(rng, w, npdt) for w in net_widths]
    n0 = net_widths[0][0]
    if closed_loop:
        nL = net_widths[0][-1]
        n_state = n0 if n_state is None else n_state
        if A_mode == "signed_perm":
            A = _signed_permutation(rng, n_state, rho)
        elif A_mode == "residual":
            A = np.eye(n_state, n0)
        else:
            A = rng.normal(0.0, np.sqrt(a_var), size=(n_state, n0))
        if B_mode == "scaled_identity":
            B = b_gain * np.eye(n_state, nL)
        else:
            B = rng.normal(0.0, np.sqrt(b_var), size=(n_state, nL))
        for net in nets:
            net.A, net.B = A, B
    net_id = (rng.integers(0, len(nets), size=n_sub).astype(np.int32) if len(nets) > 1
              else np.zeros(n_sub, np.int32))
    xc = rng.uniform(center[0], center[1], size=(n_sub, n0))
    if np.isscalar(radius):
        r = np.full(n_sub, float(radius))
    else:
        r = rng.uniform(radius[0], radius[1], size=n_sub)
    xr = np.repeat(r[:, None], n0, axis=1)
    ptr, lay, neu, sg = _draw_splits(rng, nets, net_id, xc, xr, max_splits, n_split_samples)
    batch = Batch(xc, xr, ptr, lay, neu, sg, net_id)
    meta = dict(seed=seed, max_splits=max_splits)
    if closed_loop and n_state < n0 and horizon > 0:
        meta["u"] = rng.uniform(-1.0, 1.0, size=(n_sub, horizon, n0 - n_state))
    return Workload(name, nets, batch, dtype, iters, lr, horizon, shared_slope, meta=meta)


# The five synthetic configurations.  Index 1 is the small FP64 closed-loop case the
# reference finishes in seconds; index 2 is the headline batched-CROWN workload.
CONFIGS = {
    1: dict(name="cl_4-32-32-2_fp64", net_widths=[[4, 32, 32, 2]], n_sub=64, closed_loop=True,
            radius=0.05, dtype="f64"),
    2: dict(name="crown_6-64x3-3_S4096", net_widths=[[6, 64, 64, 64, 3]], n_sub=4096,
            max_splits=8),
    3: dict(name="abcrown_8-128x4-4_S2048", net_widths=[[8, 128, 128, 128, 128, 4]], n_sub=2048,
            max_splits=16, iters=20, lr=0.1),
    4: dict(name="tmreach_12-256x3-4_S8192_H10", net_widths=[[12, 256, 256, 256, 4]], n_sub=8192,
            closed_loop=True, radius=0.02, horizon=10, shared_slope=True, A_mode="signed_perm", rho=0.95,
            b_var=3e-5),
    5: dict(name="mixed_12-{64x5,128x3,256x2}-4_S16384",
            net_widths=[[12] + [64] * 5 + [4], [12] + [128] * 3 + [4], [12] + [256] * 2 + [4]],
            n_sub=16384, max_splits=32, iters=10, lr=0.1),
    # Batched reach of candidate action sequences through a learned dynamics model (the
    # paper's MPC use; dynamics MLP of three 96-wide layers): state 8, action 4.
    6: dict(name="mpc_8+4-96x3-8_S4096_H10", net_widths=[[12, 96, 96, 96, 8]], n_sub=4096,
            closed_loop=True, n_state=8, radius=0.02, horizon=10, shared_slope=True, A_mode="residual",
            B_mode="scaled_identity", b_gain=0.1),
}


def config_workload(idx: int, n_sub: Optional[int] = None, seed: Optional[int] = None) -> Workload:
    """Workload of configuration ``idx`` (seed = idx unless given).  ``n_sub`` draws a
    smaller batch with the same recipe (the first draws are not shared with the full
    batch because the counts differ; use ``Batch.subset`` for an exact sample)."""
    cfg = dict(CONFIGS[idx])
    if n_sub is not None:
        cfg["n_sub"] = n_sub
    name = cfg.pop("name")
    return make_workload(name, idx if seed is None else seed, **cfg)


def random_duals(seed, n_sub, n_rows, n_hidden, n_beta, beta_scale=1.0):
    """Random relaxation slopes alpha in [0,1] and split multipliers beta >= 0, for
    evaluating the bound and its gradient at points other than the default."""
    rng = np.random.default_rng(seed)
    alpha = rng.uniform(0.0, 1.0, size=(n_sub, n_rows, n_hidden))
    beta = rng.uniform(0.0, beta_scale, size=(n_sub, n_rows, n_beta))
    # FP32-representable values, so an FP32 consumer sees the same numbers.
    return alpha.astype(np.float32).astype(np.float64), beta.astype(np.float32).astype(np.float64)


@dataclass
class CtWorkload:
    """A continuous-time closed loop: the vector field f_i(x, u) = a_i + F_i x + G_i u +
    x^T Q_i x as arrays, a network controller (plain MLP: state in, input out), the
    initial boxes and the flowpipe schedule (step h, K steps per control interval,
    N_ctl intervals)."""
    name: str
    a: np.ndarray
    F: np.ndarray
    G: np.ndarray
    Q: np.ndarray
    controller: Network
    x_center: np.ndarray
    x_radius: np.ndarray
    h: float
    K: int
    N_ctl: int


def make_ct_workload(seed=0, n_sub=4096, hidden=(64, 64), h=0.02, K=5, N_ctl=20, radius=(0.005, 0.02),
                     q_scale=0.05, out_scale=0.05, name=None) -> CtWorkload:
    """The 12-state, 4-input rigid-body shape of the paper's CT quadrotor (state:
    position, velocity, attitude angles, body rates; inputs: thrust and three torques;
    a 64x64 controller; 100 steps of 0.02) as a quadratic field: the kinematic chain
    position' = velocity, velocity' = gravity-tilt coupling of the angles (+ thrust on
    the vertical axis) with light drag, angles' = body rates, rates' = torques with
    damping, plus small random quadratic couplings (N(0, q_scale^2), on the velocity,
    angle and rate rows, over the angle and rate states) standing in for the
    trigonometric and gyroscopic terms.  Initial boxes: centres N(0, 0.1^2) per state,
    radii uniform in `radius`.  The controller is a random MLP (make_network) whose
    output layer is scaled by `out_scale`."""
    rng = np.random.default_rng(seed)
    n, n_u = 12, 4
    P, V, TH, W = slice(0, 3), slice(3, 6), slice(6, 9), slice(9, 12)
    F = np.zeros((n, n))
    F[P, V] = np.eye(3)
    F[V, V] = -0.1 * np.eye(3)
    F[3, 7], F[4, 6] = 0.981, -0.981            # tilt couples gravity into horizontal velocity
    F[TH, W] = np.eye(3)
    F[W, W] = -0.5 * np.eye(3)
    G = np.zeros((n, n_u))
    G[5, 0] = 1.0                               # thrust deviation on the vertical velocity
    G[W, 1:] = np.eye(3)                        # torques on the body rates
    Q = np.zeros((n, n, n))
    ang = list(range(6, 12))
    for i in range(3, 12):
        for j in ang:
            for k in ang:
                if k >= j:
                    Q[i, j, k] = rng.normal(0.0, q_scale)
    a = np.zeros(n)
    ctl = make_network(rng, [n, *hidden, n_u], np.float32)
    ctl.Ws[-1] = (ctl.Ws[-1] * out_scale).astype(np.float32).astype(np.float64)
    ctl.bs[-1] = (ctl.bs[-1] * out_scale).astype(np.float32).astype(np.float64)
    xc = rng.normal(0.0, 0.1, (n_sub, n))
    xr = rng.uniform(radius[0], radius[1], (n_sub, n))
    return CtWorkload(name or f"ct_quadratic12+4-{hidden[0]}x{len(hidden)}-4_S{n_sub}_N{K * N_ctl}", a, F, G, Q, ctl,
                      xc, xr, h, K, N_ctl)
