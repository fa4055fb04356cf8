"""FP64 CPU reference ("oracle") for the bound-propagation hot path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark.  It shares no code with the GPU library and is never a
fallback for it.  Parity status per function:

* crown.relu_relaxation, ibp_next, affine_box, concretize_box, backward,
  intermediate_bounds, final_bounds, crown: pinned (closed forms, linear and
  all-stable networks, zero-radius boxes, brute force by pattern enumeration + LP,
  dense sampling).  The intermediate-bound values themselves: the exact affine
  range of the second layer behind a stably active first layer (and equality with
  the network whose two affine layers are merged), and equality of every
  second-layer CROWN bound with max(interval bound, LP optimum over the first
  layer's relaxation lines); deeper rows lie between CROWN and that LP.
* crown.gradient / evaluate_duals: pinned (central finite differences, and an
  independent torch-FP64 autograd of the same bound).
* crown.param_gradient: pinned (central finite differences of final_bounds at a
  fixed relaxation; on all-active networks, finite differences of the full crown
  with its intermediate bounds recomputed, and the closed form of the affine map).
* crown.optimize_duals: pinned (one-neuron and split hand cases, strong duality
  against the LP optimum, soundness against brute force).
* tm.reach_dt, tm.tm_intermediate_bounds: pinned (B = 0 closed form
  A^t x +- |A^t| r, all-stable linear closed loop, dense sampled rollouts; the
  hand-worked shared-slope steps of x' = +-relu(x) on [-1, 2] fixing the Taylor
  model, both offsets and the interval product; a network whose second layer is
  exactly zero over the TM; second-layer bounds = max(interval bound, LP over the
  parallel relaxation)).
* joint.reach_joint, back_through_step, to_initial: pinned (two systems worked by
  hand in rational arithmetic, including a later step's intermediate row tighter
  than interval propagation from the state box; B = 0 matrix powers with and
  without exogenous inputs; an all-active affine loop; point initial sets on the
  simulated trajectory; dense sampled rollouts; horizon 1 = closed-loop crown).
* tm_grad.reach_volume, volume_gradient: pinned (forward = tm.reach_dt to 1e-13;
  gradient = central finite differences of the independent numpy tm.reach_dt with
  respect to actions, box centre and radius, A, B, weights and biases; closed forms of
  dV/dr for B = 0 and for an all-active affine loop, and zero action/centre gradients
  there).
* ct.picard_step, flowpipe, precondition, controller_tm, closed_loop: pinned (constant
  fields: the exact translate of the box; linear fields: the Picard polynomial equals
  the second-order Taylor expansion of exp(F s) and every box contains the exact image
  exp(F t) X_0; the scalar Riccati equation x' = -x^2 against its exact interval;
  ODE-solver trajectories inside every time-point and segment box and inside the Taylor
  model itself; a controller with zero output weights reduces the closed loop to the
  open-loop flowpipe with a constant input; sampled zero-order-hold closed loops inside
  every box).
"""
from . import crown, ct, exact, joint, tm, tm_grad  # noqa: F401
