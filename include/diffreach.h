/*
 * diffreach.h -- C-ABI of the gfx950 bound-propagation library (libdiffreach.so).
 *
 * Batched CROWN-style linear bound propagation for ReLU networks, alone or in a
 * closed loop x' = A x + B y, as used by the paper "Parallel Differentiable
 * Reachability for Learning and Planning with Certified Neural Dynamics and
 * Controllers":
 *   - Theorem "CROWN linear bounds of NN": affine lower/upper bounds
 *       W_lo x + b_lo <= f(x) <= W_hi x + b_hi   over an input box;
 *   - Algorithm "Reachability of DT Dynamics": CROWN followed by EvalInt (the
 *     box enclosure) at every step, with the TM--CROWN interface of Theorem
 *     "CROWN bounds of NN with linear TM input" and the shared-slope constraint;
 *   - "Gradient" refinement of the table "Refinement strategies": projected
 *     gradient ascent on the relaxation slopes alpha and split multipliers beta;
 *   - Algorithms "Reachability of CT Dynamics with TM Flowpipe" and "Reachability
 *     of CT NN Control Systems": Taylor-model flowpipes of polynomial vector fields,
 *     alone or with a network controller (dr_flowpipe_ct, dr_reach_ct; these carry
 *     no rounding margin, see there).
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers owned by the caller unless stated
 *     otherwise; the library never frees them.  Host-side structs (dr_network,
 *     dr_batch, dr_options) are read during the call only.
 *   - Every call after dr_create is asynchronous on `stream`, allocates nothing,
 *     never synchronises and never reads device memory on the host, so a sequence
 *     of calls can be captured into a HIP graph and replayed.
 *   - Argument and shape errors are returned synchronously as dr_status (the call
 *     then launches nothing) and described by dr_last_error.  Numerical trouble is
 *     never an error: it becomes per-subdomain status bits (DR_RES_*).
 *   - Network: z_1 = W_1 x + b_1, h_k = relu(z_k), z_{k+1} = W_{k+1} h_k + b_{k+1},
 *     y = z_L; W_k row-major n_k x n_{k-1}.  Hidden neurons of all layers are
 *     indexed in one concatenated range [0, H), layer k starting at
 *     n_1 + ... + n_{k-1}.
 *   - Spec: q directions c_r over the target (the network output y, or x' in
 *     the closed loop).  For each direction the library bounds c_r . target from
 *     below (row r) and from above (row q + r, computed as minus the lower bound
 *     of -c_r . target).  Default directions are the unit vectors.
 *   - A subdomain is a box [x_c - x_r, x_c + x_r] plus split constraints
 *     (hidden layer k, neuron j, sign s): s = +1 means z_k[j] >= 0, s = -1 means
 *     z_k[j] <= 0, packed as  (k << 24) | ((s > 0) << 16) | j.
 *   - Arithmetic (dr_options.precision): DR_PREC_F32 runs the coefficient chains
 *     on FP32 MFMA with FP32 accumulation; DR_PREC_F64 on FP64 MFMA.  Bounds,
 *     boxes, offsets and concretization are FP64 in both.  Every bound includes
 *     an outward margin covering the rounding of the chains (a priori error
 *     bound of the dot products), so it is sound in either precision; the
 *     margin is exported per result (dr_get_margins).
 */
#ifndef DIFFREACH_H
#define DIFFREACH_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dr_ctx dr_ctx;

typedef enum {
  DR_OK = 0,
  DR_EINVAL = -1,    /* null pointer, bad option or unsupported combination */
  DR_ESHAPE = -2,    /* widths/sizes out of the supported range */
  DR_ENOMEM = -3,    /* device allocation failed (dr_create only) */
  DR_EDEVICE = -4,   /* a HIP runtime call failed */
  DR_ECAPACITY = -5  /* batch larger than the context was created for */
} dr_status;

/* Per-subdomain status bits written to caller buffers. */
enum {
  DR_RES_OK = 0,
  DR_RES_INFEASIBLE = 1, /* split constraints contradict the bounds (some l > u) */
  DR_RES_NONFINITE = 2,  /* NaN or Inf met in the inputs or the chain */
  DR_RES_MARGIN = 4,     /* rounding margin larger than the bound's own magnitude */
  DR_RES_BADSPLIT = 8    /* split list invalid (bad layer/neuron, or too many) */
};

enum { DR_PREC_F32 = 0, DR_PREC_F64 = 1 };
enum { DR_DTYPE_F32 = 0, DR_DTYPE_F64 = 1 };
enum { DR_INTER_CROWN_IBP = 0, DR_INTER_IBP = 1 };
enum { DR_MARGIN_RIGOROUS = 0, DR_MARGIN_OFF = 1 };

typedef struct {
  int n_layers;               /* L >= 2 (at least one hidden layer), L <= 8 */
  const int* widths;          /* HOST array n_0..n_L; hidden n_k <= 256, n_0 <= 16, n_L <= 64 */
  int wdtype;                 /* DR_DTYPE_F32 or DR_DTYPE_F64: element type of W and b */
  const void* const* W;       /* HOST array of L device pointers, W_k row-major n_k x n_{k-1} */
  const void* const* b;       /* HOST array of L device pointers, b_k of n_k */
  const double* A;            /* device n_state x n_0 (closed loop) or NULL; read by later calls, so
                                 it must stay valid while the context lives */
  const double* B;            /* device n_state x n_L (closed loop) or NULL; same lifetime as A */
  int n_state;                /* rows of A and B, 1 <= n_state <= n_0; 0 without closed loop.  The
                                 network input is v = [x; u]: the first n_state entries are the
                                 state, the remaining n_0 - n_state exogenous inputs (actions),
                                 and x' = A v + B f(v) */
  const double* spec;         /* device q x n_target directions, or NULL for unit vectors */
  int n_spec;                 /* q <= 16 (ignored when spec == NULL); the spec chains and the dual
                                 ascent need 2q <= 16, dr_reach_dt needs n_state <= 16 */
} dr_network;

typedef struct {
  int n_sub;                  /* number of subdomains S */
  const int* net_id;          /* device S (index into the networks of dr_create), or NULL = all 0;
                                 ignored when the context has a single network */
  const double* x_center;     /* device S x n_0 */
  const double* x_radius;     /* device S x n_0, >= 0 */
  const int* split_ptr;       /* device S + 1 CSR offsets, or NULL = no splits */
  const uint32_t* split_packed; /* device split words (see header comment) */
} dr_batch;

typedef struct {
  int precision;              /* DR_PREC_F32 or DR_PREC_F64 */
  int intermediate;           /* DR_INTER_CROWN_IBP (default) or DR_INTER_IBP */
  int max_sub;                /* capacity: largest batch S for this context */
  int max_splits;             /* capacity: splits per subdomain (beta columns) */
  int tile_cfg;               /* launch and tile configuration, as chosen by the autotuner (0 = defaults):
                                 bits 0-15: 4-bit cap of workgroups per CU per kernel kind (bits 0-3
                                 bound_init, 4-7 spec chains, 8-11 dual ascent, 12-15 reach_dt; 0 = as
                                 many as fit); DR_TILE_* flags below */
  int margin_mode;            /* DR_MARGIN_RIGOROUS (default) or DR_MARGIN_OFF (diagnostics only:
                                 rounding of the chains is then not covered, bounds may be unsound) */
  int fuse_spec;              /* 1: dr_bound_init also runs the plain-CROWN spec rows while each
                                 subdomain's relaxation is on chip, and dr_propagate_backward only
                                 lays them out; 0: dr_propagate_backward runs the spec chains */
} dr_options;

/* Flags of dr_options.tile_cfg (kernel variants; results are identical up to rounding):
 *   DR_TILE_GLOBAL_WEIGHTS  bound kernel of narrow networks reads the weights from global
 *                           memory instead of a per-workgroup LDS copy;
 *   DR_TILE_PAIRED_TILES    bound kernel of narrow FP32 networks: two 16-row tiles per chain
 *                           step of a wavefront instead of one (shared loads, more registers);
 *   DR_TILE_NO_ITEM_CACHE   dual ascent without the per-item LDS copy of the relaxation. */
enum { DR_TILE_GLOBAL_WEIGHTS = 1 << 16, DR_TILE_PAIRED_TILES = 1 << 17, DR_TILE_NO_ITEM_CACHE = 1 << 18 };

/* Create a context for one or more networks sharing n_0 and the spec length.
 * Copies and re-lays-out the weights (asynchronously on `stream`) and allocates
 * all scratch for batches of up to opt->max_sub subdomains.  The only call that
 * allocates device memory.  Returns DR_OK and *ctx, or an error and *ctx = NULL. */
dr_status dr_create(dr_ctx** ctx, const dr_network* nets, int n_nets, const dr_options* opt,
                    hipStream_t stream);

/* Steps a1-a4: ingest a batch, compute exact layer-1 bounds, interval (IBP)
 * bounds, CROWN intermediate bounds of every deeper hidden layer for the neurons
 * IBP leaves unstable and unsplit (intersected with IBP), clamp split neurons and
 * detect infeasible subdomains; builds the ReLU relaxation of every hidden
 * neuron.  Results stay in the context for the calls below.  `status` (device,
 * S, may be NULL) receives DR_RES_* bits.  The batch arrays must stay valid and
 * unchanged until the last call that uses this batch has completed. */
dr_status dr_bound_init(dr_ctx* ctx, const dr_batch* batch, uint32_t* status, hipStream_t stream);

/* Step a5: backward propagation of the spec rows through every layer with the
 * adaptive slopes (plain CROWN).  Writes the affine bounds of Theorem "CROWN
 * linear bounds of NN" per subdomain and direction:
 *   lam_lo . x + acc_lo <= c_r . target(x) <= lam_hi . x + acc_hi  on the box,
 * lam_* S x q x n_0, acc_* S x q (all FP64, device).  The rounding margin is
 * already folded into acc_*.  Infeasible subdomains get acc_lo = +inf,
 * acc_hi = -inf and zero slopes. */
dr_status dr_propagate_backward(dr_ctx* ctx, double* lam_lo, double* acc_lo, double* lam_hi,
                                double* acc_hi, hipStream_t stream);

/* Step a6: concretization (EvalInt) of affine bounds over each subdomain's box
 * in FP64 with outward rounding: lb = acc_lo + lam_lo.x_c - |lam_lo|.x_r,
 * ub = acc_hi + lam_hi.x_c + |lam_hi|.x_r; lb, ub S x q.  `status` (S, may be
 * NULL) is OR-ed with DR_RES_NONFINITE / DR_RES_MARGIN where they apply. */
dr_status dr_concretize(dr_ctx* ctx, const double* lam_lo, const double* acc_lo,
                        const double* lam_hi, const double* acc_hi, double* lb, double* ub,
                        uint32_t* status, hipStream_t stream);

/* Step a7: projected gradient ascent on the duals of the final bound with the
 * intermediate bounds of the last dr_bound_init fixed.  Per subdomain and row
 * (R = 2q rows: lower rows then upper rows) the parameters are alpha (lower
 * relaxation slopes of unstable neurons, in [0,1]) and beta (one multiplier per
 * split, >= 0).  Iterates t = 0..iters: evaluate the bound and, by a
 * hand-written adjoint, its gradient at (alpha_t, beta_t); for t < iters update
 *   alpha <- clip(alpha + lr * d/dalpha, 0, 1),  beta <- max(0, beta + lr * d/dbeta).
 *   alpha   S x R x H_max FP32 (in/out; read unless init_duals, where it starts at
 *           the adaptive slopes); entries of non-unstable neurons are ignored.
 *   beta    S x R x max_splits FP32 (in/out; starts at 0 when init_duals).
 *   lb, ub  S x q best-so-far bounds over t = 0..iters (sound at every t).
 *   grad_alpha, grad_beta (nullable) gradients at the final iterate, same shapes.
 * iters = 0 evaluates the bound and gradient at the given duals. */
dr_status dr_optimize_duals(dr_ctx* ctx, int iters, float lr, int init_duals, float* alpha, float* beta,
                            double* lb, double* ub, float* grad_alpha, float* grad_beta,
                            uint32_t* status, hipStream_t stream);

/* Gradient of the bounds w.r.t. the network's weights and biases and the boxes, the
 * training signal of the reachability-aware loss (Sec. "Certified training of
 * neural dynamics and controllers": the loss is a function of bound widths, e.g.
 * mean log(1 + V) with V a width sum, and is differentiated through the bound).
 * For the objective
 *   J = sum_{s,i} g_lb[s,i] * lb[s,i] + g_ub[s,i] * ub[s,i]
 * (g_lb, g_ub: the caller's d loss / d lb, d loss / d ub) it returns dJ/dW_k,
 * dJ/db_k, dJ/dx_center and dJ/dx_radius with the relaxation of the last
 * dr_bound_init held fixed: the intermediate bounds (hence the chord slopes and
 * intercepts) and the given alpha, beta are constants; their own dependence on
 * the weights is not differentiated.  Where every neuron is stable this is the
 * gradient of the bound itself.  The bounds are those of dr_optimize_duals with
 * iters = 0 at (alpha, beta).
 * Context: one network (DR_EINVAL otherwise).
 *   alpha, beta   as dr_optimize_duals (init_duals: start at the adaptive slopes
 *                 and beta = 0, i.e. plain CROWN, and write them back).
 *   g_lb, g_ub    S x q FP64 (device).  Rows of infeasible subdomains are ignored.
 *   lb, ub        S x q FP64 out: the bounds at (alpha, beta).
 *   dW            host array of L device pointers, dW[k-1]: n_k x n_{k-1} FP64
 *                 row-major; db: L device pointers, db[k-1]: n_k FP64.  Overwritten.
 *   dxc, dxr      S x n_0 FP64 (nullable): dJ/dx_center and dJ/dx_radius.
 *   workspace     device memory of at least dr_param_grad_workspace(ctx, S) bytes
 *                 (caller-owned; holds the per-row multipliers and adjoints and the
 *                 per-chunk partial sums), so the call allocates nothing.
 * Asynchronous on `stream`; outputs are complete when the stream reaches the call's
 * end.  Sizes are checked before any launch (DR_EINVAL / DR_ESHAPE). */
size_t dr_param_grad_workspace(const dr_ctx* ctx, int n_sub);
dr_status dr_param_grad(dr_ctx* ctx, float* alpha, float* beta, int init_duals, const double* g_lb,
                        const double* g_ub, double* lb, double* ub, double* const* dW, double* const* db,
                        double* dxc, double* dxr, void* workspace, size_t workspace_bytes, uint32_t* status,
                        hipStream_t stream);

/* dr_param_grad without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture that must not call hipMalloc, tight serving or
 * training loops, harnesses that forbid allocation): the tapes and partial sums live in
 * a static device array of the library, 64 MiB per device (each device the library
 * runs on holds its own copy until the process ends), so the call allocates nothing
 * and needs no buffer beyond its inputs and outputs.  Same arguments, results and
 * errors as dr_param_grad; a batch whose dr_param_grad_workspace(ctx, S) exceeds
 * 64 MiB returns DR_ECAPACITY before any launch.  Every call on a device shares that
 * device's array (the call writes every byte it later reads, so nothing needs
 * clearing): calls that overlap in time on one device, from any context or stream,
 * race and must be ordered by the caller. */
dr_status dr_param_grad_static(dr_ctx* ctx, float* alpha, float* beta, int init_duals, const double* g_lb,
                               const double* g_ub, double* lb, double* ub, double* const* dW, double* const* db,
                               double* dxc, double* dxr, uint32_t* status, hipStream_t stream);

/* Replace the weights and biases of network `net_index` of the context in place
 * (same widths; W, b and wdtype read as in dr_create; the closed-loop A, B and the
 * spec stay those given at creation, and A, B must stay valid).  The copies, swizzles
 * and final-row seeds are rebuilt by kernels on `stream` into the existing buffers:
 * nothing is allocated, so a training step (set weights, dr_bound_init,
 * dr_param_grad) can be captured in one HIP graph.  The state of the last
 * dr_bound_init is invalidated.  DR_ESHAPE if the widths differ. */
dr_status dr_set_weights(dr_ctx* ctx, int net_index, const dr_network* net, hipStream_t stream);

/* Step a8: stepwise closed-loop reachability (Algorithm "Reachability of DT
 * Dynamics") with linear Taylor models: each box is normalised to the TM
 * x = c + P z, z in [-1,1]^n; every step certifies the controller with
 * shared-slope CROWN on the TM input, composes x' = A x + B y in TM arithmetic
 * and evaluates the box.  Needs a closed-loop network with n_state == n_0, no
 * spec and no splits.  boxes: S x (horizon+1) x n_state x 2 FP64 (step 0 is the
 * input box).  A network with exogenous inputs (n_state < n_0) returns DR_EINVAL
 * here; use dr_reach_dt_exo. */
dr_status dr_reach_dt(dr_ctx* ctx, const dr_batch* batch, int horizon, double* boxes, uint32_t* status,
                      hipStream_t stream);

/* The same stepwise reachability for a network whose input is v = [x; u_t] with a
 * given exogenous sequence u_t per box (the batched reach of candidate action
 * sequences through a learned dynamics model, Sec. "Model Predictive Control" of the
 * paper): at step t the TM of v is the state's TM extended by the point u_t (zero
 * linear part, zero interval), so x' = A v + B f(v) is composed exactly as above.
 * u: device FP64 S x horizon x (n_0 - n_state), row-major; must be non-NULL when
 * horizon > 0 and S > 0 (DR_EINVAL otherwise, and when the network has no
 * exogenous inputs).  The batch's x_center / x_radius keep their S x n_0 layout;
 * entries n_state..n_0-1 are ignored.  boxes: S x (horizon+1) x n_state x 2. */
dr_status dr_reach_dt_exo(dr_ctx* ctx, const dr_batch* batch, int horizon, const double* u, double* boxes,
                          uint32_t* status, hipStream_t stream);

/* Reachability by CROWN through the closed loop unrolled over the horizon: the joint,
 * non-truncated DT baseline the paper compares its stepwise engine with (Section
 * "Reachability Tool Evaluations", DT panel of the figure benchmarking the tool), tighter
 * than the stepwise Taylor models because no intermediate set is re-formed, and with a
 * cost that grows with the square of the horizon.  The graph is v_t = [x_t; u_t],
 * x_{t+1} = A v_t + B f(v_t) (u_t as in dr_reach_dt_exo, absent when n_state == n_0).
 * Relaxation as in dr_bound_init (chord upper line, adaptive lower slope; lower and
 * upper bounds are separate rows).  Per step t: every hidden layer takes interval bounds
 * from its input node (layer 1: the state box of step t, exact at t = 0) and each neuron
 * they leave unstable gets the rows +-e_j carried back through steps t-1..0 to the
 * initial box; then the state box of x_{t+1} from the rows +-e_i on x_{t+1} carried back
 * to x_0.  The relaxation of every step stays in LDS: a horizon beyond what fits for the
 * network returns DR_ECAPACITY (the message gives the limit).  Needs a context with one
 * closed-loop network, no spec, no splits.
 *   u      device FP64 S x horizon x (n_0 - n_state) or NULL (no exogenous inputs)
 *   boxes  device FP64 S x (horizon + 1) x n_state x 2 (step 0 is the input box)
 *   rows   device int S x horizon x 8 or NULL: CROWN rows of hidden layer k at step t
 *          (index k - 1) and the 2 n_state state rows (index L - 1), for FLOP accounting
 *   status device S or NULL: DR_RES_NONFINITE when a bound is not finite.
 * Rounding: the chain products carry the rigorous margins of dr_bound_init (each step
 * boundary adds the error of lam B W_L and lam A and of the seeds) unless margins are
 * off.  Asynchronous on `stream`. */
dr_status dr_reach_dt_joint(dr_ctx* ctx, const dr_batch* batch, int horizon, const double* u, double* boxes,
                            int* rows, uint32_t* status, hipStream_t stream);

/* Gradient of the reach-tube volume through the stepwise reach: the training signal of
 * the paper's reachability-aware loss (Section "Certified training of neural dynamics and
 * controllers", Algorithm "Training of DT Neural Dynamics": L_reach = mean log(1 + V)
 * with V the sum over steps t = 1..H and states of the widths of the boxes X_t) and the
 * action gradient of its top-candidate refinement (Section "Reachability-aware MPC").
 * Runs the reach of dr_reach_dt / dr_reach_dt_exo (same arguments and boxes output)
 * recording each box's Taylor models and bounds into the workspace, then the reverse
 * pass through every step: the output rows and the CROWN rows of the intermediate bounds
 * in reverse on the matrix cores, the chord relaxation (s = u/(u-l), t = -s l), the
 * intersections with the interval bounds and the interval bounds themselves, layer 1 over
 * the Taylor model, and the Taylor-model composition.  With J = sum_s g_V[s] V_s:
 *   g_V       device FP64 S: dJ/dV_s (for mean log(1 + V): 1 / (S (1 + V_s)))
 *   boxes     device FP64 S x (horizon + 1) x n_state x 2 (the forward result)
 *   du        device FP64 S x horizon x (n_0 - n_state) or NULL: dJ/du (exogenous inputs)
 *   dxc, dxr  device FP64 S x n_state or NULL: dJ/d(box centre), dJ/d(box radius)
 *   dA, dB    device FP64 n_state x n_0, n_state x n_L or NULL: dJ/dA, dJ/dB (overwritten)
 *   dW, db    host arrays of L device pointers or NULL (and NULL entries): dJ/dW_k (n_k x
 *             n_{k-1} row-major) and dJ/db_k (n_k), FP64, overwritten; accumulated per
 *             workgroup in the chain type with atomic additions and summed in a fixed order
 *   workspace device memory of at least dr_reach_grad_workspace(ctx, S, horizon) bytes
 *             (caller-owned: the forward record and the reverse kernel's chain records).
 * Rounding margins are constants of the gradient (it is the gradient of the bound in exact
 * arithmetic, as autodiff of the engine gives it); discrete choices (stability, the side of
 * an intersection, signs, a tie counts for the interval bound) are those of the forward
 * pass.  Needs a context with one closed-loop network and no spec.  dA and dB sum over the
 * batch with atomic additions (the order of the additions is not fixed).  Asynchronous on
 * `stream`; allocates nothing. */
size_t dr_reach_grad_workspace(const dr_ctx* ctx, int n_sub, int horizon);
dr_status dr_reach_dt_grad(dr_ctx* ctx, const dr_batch* batch, int horizon, const double* u, const double* g_V,
                           double* boxes, double* du, double* dxc, double* dxr, double* dA, double* dB,
                           double* const* dW, double* const* db, void* workspace, size_t workspace_bytes,
                           uint32_t* status, hipStream_t stream);

/* Continuous-time reachability with Taylor-model flowpipes (Section "Propagation under
 * Continuous-Time Analytical Dynamics", Theorem "TM flowpipe step via Picard iteration",
 * appendix Algorithm "Reachability of CT Dynamics with TM Flowpipe"; the closed loop of
 * Algorithm "Reachability of CT NN Control Systems").
 *
 * The vector field is polynomial of degree <= 2 in the state and affine in the input:
 *   f_i(x, u) = a_i + sum_j F_ij x_j + sum_k G_ik u_k + sum_jk Q_ijk x_j x_k.
 * Each box [c - r, c + r] is carried as a Taylor model of the paper's quasi-quadratic
 * fixed shape, X(y, s) = c + L y + l s + s (M y) + w s^2 (+) [lo, hi] over the box's
 * generators y in [-1, 1]^n and the time s in [0, h]: per step two Picard iterations of
 * the polynomial part, a remainder validated by the Picard operator (widened at most
 * `tries` times, then refined `rounds` times), the step-end model, and the remainder
 * absorbed into the linear part when that is well conditioned.  All arithmetic is FP64
 * without outward rounding of the flowpipe steps.  A box whose step found no validated
 * remainder gets DR_RES_NONFINITE and unbounded boxes from that step on. */
typedef struct {
  int n;              /* state dimension, 1..16 */
  int n_u;            /* input dimension, 0..16 (0: no input) */
  const double* a;    /* device n */
  const double* F;    /* device n x n, row-major */
  const double* G;    /* device n x n_u, row-major; NULL when n_u == 0 */
  const double* Q;    /* device n x n x n (Q_ijk at (i n + j) n + k), or NULL: linear field */
} dr_ct_field;

typedef struct {
  double h;           /* flowpipe step, 0 < h < inf */
  int steps;          /* flowpipe steps per control interval, K >= 1 */
  int intervals;      /* control intervals N >= 0 (N K steps in all; K N <= 100000) */
  int tries;          /* widenings of the remainder guess, 1..1000 (40 is ample) */
  int rounds;         /* refinements of a validated remainder, 0..100 (3) */
  double eps;         /* half-width of the first remainder guess, > 0 (1e-9) */
} dr_ct_options;

/* The flowpipe of x' = f(x) (n_u must be 0) from n_sub boxes (x_center, x_radius: device
 * n_sub x n; x_radius >= 0).  Outputs (device, FP64, written in full):
 *   boxes     n_sub x (N K + 1) x n x 2: the boxes of the time points 0, h, .., N K h;
 *   segments  n_sub x N K x n x 2: the box of every step's segment [t, t + h], or NULL;
 *   status    n_sub: DR_RES_* bits, or NULL.
 * Takes no context: errors are described by dr_last_error(NULL).  One wavefront per box.
 * The quadratic form is evaluated over its monomials x_j x_k (j <= k), each Taylor-model
 * product formed once per evaluation, with coefficient Q_ijk + Q_ikj (j < k) or Q_ijj.
 * Asynchronous on `stream`; allocates nothing. */
dr_status dr_flowpipe_ct(const dr_ct_field* f, const dr_ct_options* opt, int n_sub, const double* x_center,
                         const double* x_radius, double* boxes, double* segments, uint32_t* status,
                         hipStream_t stream);

/* The closed loop x' = f(x, u) with the network of `ctx` as the controller, its output
 * held over each control interval of K steps (zero-order hold).  At every control
 * boundary the controller is certified on the state's Taylor model by the step of
 * dr_reach_dt (Theorem "CROWN bounds of NN with linear TM input"): `ctx` must be a
 * closed-loop context with one network, no spec, n_0 = f->n inputs and n_state = f->n_u
 * (so n_u <= n), whose loop matrices A (n_u x n) and B (n_u x n_u) make the held input
 * u = A x + B net(x); pass A = 0 and B = I for a plain network controller.  The
 * controller's chains run in the context's precision (rigorous margins as configured);
 * the input's model is linear over the same generators, its interval part centred.
 * Batch as for dr_reach_dt (no splits; x_center, x_radius n_sub x n); outputs as for
 * dr_flowpipe_ct; status also carries the controller step's bits.  Two launches per
 * control interval: the controllers of all boxes (one workgroup per box), then their
 * flowpipes (one wavefront per box); each box's state waits in between in a buffer that
 * dr_create allocates for closed-loop contexts (max_sub boxes), so calls that overlap on
 * one context race.  Asynchronous on `stream`; allocates nothing. */
dr_status dr_reach_ct(dr_ctx* ctx, const dr_ct_field* f, const dr_ct_options* opt, const dr_batch* batch,
                      double* boxes, double* segments, uint32_t* status, hipStream_t stream);

/* Diagnostics of the last dr_bound_init / dr_propagate_backward /
 * dr_optimize_duals / dr_reach_dt on this context (device outputs):
 *   dr_get_bounds  l, u: S x H_max FP64 pre-activation bounds of hidden neurons;
 *   dr_get_rows    rows: S x 8 int, CROWN chain rows per layer (index k-1 for the
 *                  rows of hidden layer k; index L-1 for the spec rows), for
 *                  algorithmic FLOP accounting (reach_dt: summed over steps);
 *   dr_get_margins margin: S x 2q FP64, rounding margin of each final row of the
 *                  last dr_propagate_backward or dr_optimize_duals. */
dr_status dr_get_bounds(dr_ctx* ctx, double* l, double* u, hipStream_t stream);
dr_status dr_get_rows(dr_ctx* ctx, int* rows, hipStream_t stream);
dr_status dr_get_margins(dr_ctx* ctx, double* margin, hipStream_t stream);

/* Shape queries (host). */
int dr_hidden_max(const dr_ctx* ctx);   /* H_max over the networks */
int dr_spec_rows(const dr_ctx* ctx);    /* R = 2q */

/* Message of the last error on this context (or of the last failed dr_create
 * when ctx is NULL); never NULL. */
const char* dr_last_error(const dr_ctx* ctx);

/* Release the context and its scratch (synchronises the device first). */
void dr_destroy(dr_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* DIFFREACH_H */
