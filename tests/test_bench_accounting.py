"""The benchmark's algorithmic FLOP counts against hand-computed values (CPU only)."""
import numpy as np

import bench


def test_chain_and_spec_row_flops():
    w = [6, 64, 64, 64, 3]                        # the headline network
    # an intermediate row of layer 2 multiplies by W_1 only; of layer 3 by W_2 and W_1
    assert bench.chain_flops_per_row(w, 2) == 2 * 64 * 6
    assert bench.chain_flops_per_row(w, 3) == 2 * 64 * 6 + 2 * 64 * 64
    # a spec row: W_3, W_2, W_1 (its product with W_4 is formed once per network)
    assert bench.final_flops_per_row(w) == 2 * 64 * 6 + 2 * 64 * 64 * 2


def test_dense_row_count_matches_the_closed_form():
    """Dense rows: two per neuron of layers 2..L-1 plus 2q spec rows; 1.348 MFLOP per
    subdomain of the headline network (6 spec rows)."""
    class Net:
        widths = [6, 64, 64, 64, 3]
    per = 128 * (2 * 64 * 6) + 128 * (2 * 64 * 6 + 2 * 64 * 64) + 6 * (2 * 64 * 6 + 2 * 64 * 64 * 2)
    assert per == 1_348_096
    status = np.array([0, 0, 1, 8, 0])            # infeasible and bad-split subdomains are not counted
    assert bench.dense_flops([Net()], np.zeros(5, np.int32), status, 6) == 3 * per


def test_needed_row_count_uses_the_chain_rows():
    class Net:
        widths = [6, 64, 64, 64, 3]
    rows = np.zeros((2, 8), np.int32)
    rows[0, 1], rows[0, 2] = 10, 20               # rows of hidden layers 2 and 3
    rows[1, 2] = 4
    got = bench.bound_init_flops([Net()], np.zeros(2, np.int32), rows)
    assert got == 10 * (2 * 64 * 6) + 20 * (2 * 64 * 6 + 2 * 64 * 64) + 4 * (2 * 64 * 6 + 2 * 64 * 64)


def test_joint_flops_hand_count():
    """widths 3-4-5-2 with a 2-dimensional state: a chain through one step's network is
    2*4*3 + 2*5*4 = 64 FLOPs, the step boundary 2*2*5 + 2*2*3 = 32.  Rows (H = 2):
    t=0: 6 rows at layer 2 (24 each), 4 state rows (one step back without the boundary:
    64); t=1: 2 rows at layer 1 (one step back: 96), 6 at layer 2 (24 + 96), 4 state
    rows (two steps back less one boundary: 160) -> 144 + 256 + 192 + 720 + 640."""
    import numpy as np
    rows = np.zeros((2, 8), np.int64)
    rows[0, :3] = [0, 6, 4]
    rows[1, :3] = [2, 6, 4]
    assert bench.joint_flops([3, 4, 5, 2], 2, rows) == 1952


def test_ct_step_flops_hand_count():
    """Two states, no input, F with two nonzero entries, one monomial x_0 x_1 that both
    components use (Q_001 = 1, Q_110 = 2): an evaluation of f is one product (540) and
    four scaled terms (4 x 74) = 836; a step makes 2 Picard + 1 validating + 3 refining
    evaluations (5016), four images of 84 per component (672), the Picard and step-end
    updates (140 + 70) and the preconditioning (6 n^3 + 4 n^2 = 48 + 16) -> 5962."""
    import numpy as np
    F = np.array([[0.0, 1.0], [-1.0, 0.0]])
    Q = np.zeros((2, 2, 2)); Q[0, 0, 1] = 1.0; Q[1, 1, 0] = 2.0
    assert bench.ct_step_flops(F, None, Q) == 5962
    # the same monomial written on either side counts once; an input adds its terms and
    # the update of the held input's model (2 n_u n^2)
    G = np.array([[1.0], [0.0]])
    assert bench.ct_step_flops(F, G, Q) == 5962 + 6 * 74 + 2 * 1 * 4
