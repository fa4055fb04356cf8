"""Shared helpers of the GPU parity tests (oracle side runs on the host)."""
import numpy as np
import pytest

from oracle import crown

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2605_25346_amd import binding
    binding.load()   # a missing library is a failure, not a skip


def rel_gap(a, b):
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(1.0, np.abs(b))


def near_tie(bounds, tol=1e-4, slope=True):
    """True if some unstable neuron's adaptive-slope decision (u > -l, only when
    ``slope``) or stability decision (l < 0 < u) is within tol of flipping: those are
    decisions taken by floating point, where several results are valid."""
    for (l, u) in bounds:
        scale = np.maximum(np.maximum(np.abs(l), np.abs(u)), 1e-300)
        uns = (l < 0) & (u > 0)
        if slope and np.any(uns & (np.abs(u + l) <= tol * scale)):
            return True
        # exact zeros come from split clamping on both sides: not a floating-point decision
        if np.any(((np.abs(l) <= tol * scale) & (l != 0)) | ((np.abs(u) <= tol * scale) & (u != 0))):
            return True
    return False


def oracle_subset(wl, idx):
    out = []
    for s in idx:
        net = wl.nets[int(wl.batch.net_id[s])]
        out.append(crown.crown(net, wl.batch.x_center[s], wl.batch.x_radius[s], wl.batch.splits_of(s)))
    return out


def print_stats(tag, gaps):
    gaps = np.asarray(gaps).ravel()
    if gaps.size:
        print(f"[{tag}] n={gaps.size} max={gaps.max():.3e} median={np.median(gaps):.3e}", flush=True)
