/*
 * mdpvi.h -- C ABI of the MI355X value-iteration library for the occupancy
 * MDP of vehicular bag-of-task placement.
 *
 * The model (paper Sec. V-B..V-G): K vehicular clouds ("hosts") of C VM
 * units each; J task classes, a class-j task needs size[j] units, arrives as
 * a Poisson stream of rate lambda[j]; each occupied unit is released at
 * rate mu; each host leaves at rate nu and is replaced empty (its VMs are
 * dropped).  The state (Eq. (10)) is the occupancy vector n = (n_0..n_{K-1})
 * together with the class e of the pending placement request; the actions
 * (Eq. (11)) are "place on host a" (a = 0..K-1, feasible iff
 * n_a + size[e] <= C) and "send to the paid cloud" (a = K, always
 * feasible).  The continuous-time chain is uniformised at
 *   Lam = sum_j lambda[j] + K*C*mu + K*nu,
 * the reward (Eqs. (14)-(16)) is reward[e] for a placement and
 * -reject_cost[e] for the paid cloud, paid on the arrival branch, and
 * the Bellman equation (Eq. (18)) carries a discount gamma per uniformised
 * step:
 *   Q(s,a) = P_arr R(e,a) + gamma * sum_s' P(s'|s,a) V(s'),
 *   V(s)   = max over feasible a of Q(s,a),    P_arr = sum_j lambda[j] / Lam.
 *
 * Layout of every per-state array (values, policies, gaps, adjoints):
 *   index(n, e) = sum_k n_k (C+1)^k + e (C+1)^K     (host 0 fastest, class slowest)
 *   N = J (C+1)^K entries.
 *
 * Conventions shared by every entry point:
 *   - Return value: MDPVI_OK (0) or a negative MDPVI_E* code; the message of
 *     the last failure on the calling thread is mdpvi_last_error().  No C++
 *     exception crosses this boundary.
 *   - Array arguments marked "device" are caller-owned device pointers of
 *     the GPU that is current when the call is made; the library never
 *     frees or keeps them.  The library owns the handle and its scratch
 *     (a second value buffer, residual slots, counters, pinned host words),
 *     allocated on first use and freed by mdp_free.
 *   - hip_stream is a hipStream_t (NULL = the null stream).  vi_solve,
 *     policy_eval and vi_adjoint return only after the stream has reached
 *     their stopping test (they must read the residual); policy_extract,
 *     policy_extract_f64 and policy_greedy are asynchronous on the stream.
 *   - One handle must not be used from two threads or on two streams at the
 *     same time.  Distinct handles are independent.
 */
#ifndef MDPVI_H
#define MDPVI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MDPVI_OK        0
#define MDPVI_EINVAL   (-1)  /* invalid argument: parameter out of range, NULL pointer */
#define MDPVI_ERANGE   (-2)  /* state space too large (N > 2^62) or size overflow      */
#define MDPVI_ENOCONV  (-3)  /* max_iter reached before the stopping test passed;
                                outputs and stats are valid (the last iterate)      */
#define MDPVI_ENAN     (-4)  /* a NaN / Inf appeared in the iterate                  */
#define MDPVI_EDEVICE  (-5)  /* a HIP runtime call failed (its text is in last_error) */
#define MDPVI_ENOMEM   (-6)  /* device or pinned host allocation failed              */

#define MDPVI_MAX_K 16       /* hosts */
#define MDPVI_MAX_J 8        /* task classes */
#define MDPVI_FORM_TILE 16   /* mdp_set_sweep_form: the tile form */
#define MDPVI_FORM_ROW 32    /* mdp_set_sweep_form: the row form of the tile sweep */
#define MDPVI_ADJOINT_GROUP 32 /* mdp_set_adjoint_form: the group form of the adjoint sweep */

/* Model parameters (Sec. V-B..V-E).  All pointers are host pointers to J
 * entries, read during mdp_build only.
 *   K in [1, 16], C >= 1, J in [1, 8], 1 <= size[j] <= C,
 *   lambda[j] >= 0 finite with sum > 0, mu >= 0, nu >= 0 finite,
 *   reward[j] finite, reject_cost NULL (all 0) or finite entries,
 *   gamma in [0, 1), idle_unit_cost >= 0 finite.
 * One uniformised step from (n, e) earns P_arr R(e, a) - idle_unit_cost
 * (KC - sum_k n_k): the placement reward r_e or the paid-cloud cost -c_e on
 * the arrival branch, less the under-utilisation penalty of Eq. (16) on
 * every free VM unit of every host (0 by default).                         */
typedef struct {
    int32_t K, C, J;
    const int32_t *size;
    const double *lambda;
    double mu;
    double nu;
    const double *reward;
    const double *reject_cost;
    double gamma;
    double idle_unit_cost;
} mdpvi_params;

typedef struct mdpvi_mdp *mdpvi_mdp_t;

/* Figures of one iterative call.  iterations = sweeps executed until the
 * stopping test passed; residual_inf = ||V^k - V^{k-1}||_inf of the last
 * sweep (FP64, exact from the stored values); bound_inf =
 * gamma/(1-gamma) * residual_inf, the contraction bound on the distance to
 * the fixed point (Alg. 3, step 3); seconds = device time between the first
 * and the last kernel of the call (HIP events); backups = feasible
 * (state, action) pairs per sweep x sweeps; bytes = algorithmic bytes moved
 * (values read once and written once per sweep); sweep_seconds = sum of the
 * durations of the sweep kernels that did work, each bracketed by its own
 * pair of HIP events on the call's stream (0 unless mdp_set_timing(h, 1)).  */
typedef struct {
    int64_t iterations;
    double residual_inf;
    double bound_inf;
    double seconds;
    double backups;
    double bytes;
    double sweep_seconds;
} mdpvi_stats;

/* Validate p, derive the uniformisation constants and mixed-radix strides,
 * and create a handle (host memory only; device scratch is allocated on
 * first use).  Errors: MDPVI_EINVAL, MDPVI_ERANGE, MDPVI_ENOMEM.            */
int mdp_build(const mdpvi_params *p, mdpvi_mdp_t *out);

/* Free the handle and its scratch.  NULL is accepted.  The caller must have
 * synchronised the stream of the last call.                                */
void mdp_free(mdpvi_mdp_t h);

/* N = J (C+1)^K; -1 for a NULL handle. */
int64_t mdp_num_states(mdpvi_mdp_t h);
/* K + 1 (placements plus the paid cloud); -1 for a NULL handle. */
int32_t mdp_num_actions(mdpvi_mdp_t h);
/* Feasible (state, action) pairs of one sweep; -1 for a NULL handle. */
int64_t mdp_feasible_pairs(mdpvi_mdp_t h);

/* Synchronous (Jacobi) value iteration, Alg. 3 steps 1-3 and Eq. (18).
 * V: device float[N]; in: V^0 (e.g. zeros), out: the first iterate V^k with
 * ||V^k - V^{k-1}||_inf < tol (strict; infinity norm exact in FP64).
 * Sums of the Bellman backup are formed in FP64 with non-negative weights,
 * stored values are FP32.  From a V^0 with V^0 <= T V^0 (V^0 = 0 when every
 * reject cost is 0) the iterates increase monotonically and reach an exact
 * FP32 fixed point, so any tol > 0 is met.
 * Errors: MDPVI_EINVAL (NULL, tol <= 0 or NaN, max_iter < 1), MDPVI_ENOCONV
 * (V holds V^{max_iter}), MDPVI_ENAN, MDPVI_EDEVICE, MDPVI_ENOMEM.
 * st may be NULL.                                                           */
int vi_solve(mdpvi_mdp_t h, float *V, double tol, int64_t max_iter,
             void *hip_stream, mdpvi_stats *st);

/* Value iteration for callers that cannot allocate device memory (code
 * under HIP graph capture aside, serving loops and harnesses that forbid
 * hipMalloc): the same sweeps, stopping test and result as vi_solve (bit for
 * bit), with every piece of device scratch (control and residual words, the
 * FP64 arrival-term arrays, the second value buffer) taken from one
 * file-scope device array of 64 MiB that each device running the library
 * holds until the process ends.  No hipMalloc, hipFree or other allocating
 * call is made; the caller still owns V (device float[N], in: V^0, out: the
 * result).  The tile order is the index order and the automatic form choice
 * ignores the tuning cache (every form and order gives the same iterates).
 * st->seconds is the host wall time of the call; st->sweep_seconds is 0.
 * The array keeps the last call's contents; every call clears what must
 * start at zero.  All calls on one device share the one array: calls that
 * overlap on one device (two streams, two threads) race and must not be made.
 * Errors: those of vi_solve, and MDPVI_ERANGE when the instance needs more
 * than the 64 MiB of scratch (about 5.5 million FP32 states of a tile-form
 * shape; vi_solve has no such limit).                                      */
int vi_solve_noalloc(mdpvi_mdp_t h, float *V, double tol, int64_t max_iter,
                     void *hip_stream, mdpvi_stats *st);

/* Greedy policy from a value function, Alg. 3 step 4:
 * pi[s] = lowest-index action maximising Q(s,a) (hosts in order, the paid
 * cloud last), Q formed in FP64 from V.
 * V: device float[N] (policy_extract) or double[N] (policy_extract_f64);
 * pi: device uint8[N] out; gap: device float[N] out or NULL, the best Q minus
 * the second-best Q over feasible actions (+inf when only the paid cloud is
 * feasible; 0 on exact ties).  Asynchronous.
 * Errors: MDPVI_EINVAL, MDPVI_EDEVICE.                                      */
int policy_extract(mdpvi_mdp_t h, const float *V, uint8_t *pi, float *gap,
                   void *hip_stream);
int policy_extract_f64(mdpvi_mdp_t h, const double *V, uint8_t *pi, float *gap,
                       void *hip_stream);

/* Fixed-policy evaluation V_pi = r_pi + gamma P_pi V_pi (the Bellman equation
 * of Eq. (18) without the max), FP64 Jacobi sweeps.
 * pi: device uint8[N], every entry a feasible action (checked: an infeasible
 * placement makes the call fail with MDPVI_EINVAL before any sweep);
 * V: device double[N], in: V^0 (warm start), out: V_pi to ||dV||_inf < tol.
 * Errors as vi_solve.                                                       */
int policy_eval(mdpvi_mdp_t h, const uint8_t *pi, double *V, double tol,
                int64_t max_iter, void *hip_stream, mdpvi_stats *st);

/* Fixed policies of the fast greedy heuristic (Alg. 2).
 * kind 0 = least-loaded: the feasible host with the fewest occupied units,
 *          lowest index on ties; the paid cloud iff no host has room.
 * kind 1 = first-fit: the lowest-index host with room (Alg. 2 scans the VCs
 *          in order); the paid cloud iff none has room.
 * pi: device uint8[N] out.  Asynchronous.  Errors: MDPVI_EINVAL, MDPVI_EDEVICE. */
int policy_greedy(mdpvi_mdp_t h, int32_t kind, uint8_t *pi, void *hip_stream);

/* Gradient of the expected discounted reward from the empty system,
 *   J = sum_e c_e V_pi(0, e),   c_e = lambda[e] / sum_j lambda[j],
 * with respect to theta = (lambda[0..J-1], mu, nu, reward[0..J-1]), the policy
 * held fixed (for the optimal pi of Eq. (18) this is the derivative of the
 * optimal J wherever the optimal action is unique up to ties between
 * equivalent hosts).  Adjoint method: w solves (I - gamma P_pi)^T w = c by
 * transposed Jacobi sweeps w <- c + gamma P_pi^T w (FP32 w, FP64 sums, stop at
 * ||dw||_1 < tol), then one pass forms
 *   dJ/dtheta = sum_s w(s) (d r_pi(s) + gamma d(P_pi V_pi)(s)) + sum_e d c_e V_pi(0, e)
 * in FP64 with a fixed-order reduction (bitwise reproducible).
 * pi: device uint8[N] (feasible, checked); V_pi: device double[N], the value
 * of pi (policy_eval); w: device float[N], in: w^0 (e.g. zeros), out: the
 * adjoint weights; grad: host double[2J+2] out, ordered lambda[0..J-1], mu,
 * nu, reward[0..J-1]; objective: host double out (J) or NULL.
 * Errors: as policy_eval; on MDPVI_ENOCONV grad is formed from the last w.  */
int vi_adjoint(mdpvi_mdp_t h, const uint8_t *pi, const double *V_pi, float *w,
               double *grad, double *objective, double tol, int64_t max_iter,
               void *hip_stream, mdpvi_stats *st);

/* J = sum_e c_e V(0, e) of a device double[N] value array (host double out).
 * Synchronous.  Errors: MDPVI_EINVAL, MDPVI_EDEVICE, MDPVI_ENOMEM.          */
int policy_objective(mdpvi_mdp_t h, const double *V, double *out, void *hip_stream);

/* ------------------------------------------------------------------ batches
 * Many independent instances (a parameter sweep over rates and fleet sizes)
 * solved together.  Per-state arrays of a batch are the instances' arrays
 * concatenated in instance order; batch_offsets gives the n+1 offsets.
 * Each instance keeps its own stopping test.  Instances whose two FP32 value
 * copies fit one workgroup's LDS (about 20k states) are solved LDS-resident,
 * one workgroup each, in one persistent launch; larger ones advance one sweep
 * per round kernel over all of them at once, concurrently on a second stream
 * owned by the batch.  Every instance must have fewer than 2^31 states.   */
typedef struct mdpvi_batch *mdpvi_batch_t;

/* p: host array of n parameter blocks (validated as mdp_build).  Host only.
 * Errors: MDPVI_EINVAL (the message names the instance), MDPVI_ERANGE,
 * MDPVI_ENOMEM.                                                             */
int mdp_build_batch(const mdpvi_params *p, int32_t n, mdpvi_batch_t *out);
void mdp_free_batch(mdpvi_batch_t b);
/* n; -1 for NULL. */
int32_t batch_num_instances(mdpvi_batch_t b);
/* States of instance i, or of the whole batch for i = -1; -1 if invalid. */
int64_t batch_num_states(mdpvi_batch_t b, int32_t i);
/* Feasible (state, action) pairs per sweep of instance i (-1: sum). */
int64_t batch_feasible_pairs(mdpvi_batch_t b, int32_t i);
/* offsets: host int64[n+1] out, offsets[i] = first state of instance i. */
int batch_offsets(mdpvi_batch_t b, int64_t *offsets);

/* vi_solve for every instance (same tol and max_iter).  V: device
 * float[total states], in V^0, out each instance's final iterate.
 * iterations, residuals: host arrays of n (or NULL) with each instance's
 * sweeps and final residual.  st: aggregate (max iterations, total backups
 * and bytes, device seconds of the whole call).  Errors: as vi_solve;
 * MDPVI_ENOCONV / MDPVI_ENAN if any instance is affected (all outputs valid). */
int vi_solve_batch(mdpvi_batch_t b, float *V, double tol, int64_t max_iter,
                   void *hip_stream, mdpvi_stats *st, int64_t *iterations,
                   double *residuals);

/* Policy iteration (Howard's, with full evaluations): repeat { evaluate pi
 * in FP64 (policy_eval to eval_tol, at most eval_max_iter sweeps); improve:
 * pi'(s) = pi(s) unless some action's FP64 Q (formed from V_pi as in
 * policy_extract_f64) exceeds Q(s, pi(s)) by more than improve_tol, else
 * the lowest-index argmax } until pi' = pi.  Keeping the current action on
 * near-ties stops the cycling between equivalent hosts that rounding would
 * otherwise cause; at the end pi is improve_tol-greedy for its own value,
 * so V* - V_pi <= (improve_tol + 2 gamma bound)/(1 - gamma) elementwise, with
 * bound the last evaluation's error bound (st->bound_inf).  Choose
 * improve_tol above twice that bound.
 * pi: device uint8[N], in the starting policy (every action feasible), out
 * the final policy; V: device double[N], in the first evaluation's starting
 * iterate, out V_pi of the final policy (each evaluation starts from the
 * previous one's result).  rounds (host, nullable): evaluations done.
 * st: evaluation sweeps summed (iterations, backups, bytes, sweep_seconds),
 * the last evaluation's residual and bound, host wall seconds of the call.
 * Synchronous.  Errors: MDPVI_EINVAL (NULL pointer, eval_tol <= 0,
 * improve_tol < 0 or not finite, eval_max_iter or max_rounds < 1, an
 * infeasible action in pi); MDPVI_ENOCONV if an evaluation reaches
 * eval_max_iter or the policy still changes after max_rounds (pi and V hold
 * the last round's); MDPVI_ENAN, MDPVI_EDEVICE, MDPVI_ENOMEM.               */
int policy_iteration(mdpvi_mdp_t h, uint8_t *pi, double *V, double eval_tol, int64_t eval_max_iter,
                     double improve_tol, int64_t max_rounds, void *hip_stream, mdpvi_stats *st,
                     int64_t *rounds);

/* Block-asynchronous value iteration (the paper's BSDI, Alg. 4) on the tiles
 * of the tile form: a pass stages each tile of (C+1)^T occupancies (all
 * classes) in LDS and runs `inner` synchronous episodes of the Bellman backup
 * of Eq. (18) on it, in which a successor inside the tile (along a low
 * digit, the state itself, or the reset of an empty high-digit host)
 * contributes the tile's latest value and a successor outside the tile the
 * previous pass's value; the pass writes the last episode back.  Passes
 * repeat until the largest change of a pass is < tol.  inner = 1 is
 * vi_solve's Jacobi iteration, bit for bit.  The iterates differ from
 * Jacobi's for inner > 1, but every episode applies the same monotone FP32
 * operator, so from a sub-solution both increase to the same FP32 fixed
 * point.  V: device float[N], in V^0, out the last pass.  st->iterations
 * counts passes, st->backups counts feasible pairs times passes times
 * inner.  Needs K in 3..8, J <= 3 distinct sizes and a tile (T >= 2) whose
 * two LDS images fit 64 KB.  Errors: as vi_solve; MDPVI_EINVAL for inner
 * outside 1..1024 or a shape the form does not cover.                       */
int vi_solve_bsdi(mdpvi_mdp_t h, float *V, double tol, int64_t max_iter, int32_t inner,
                  void *hip_stream, mdpvi_stats *st);

/* Choice of the sweep kernels for this handle (a tuning knob; every form
 * computes bit-identical iterates).  slab_digits = -1: automatic (the
 * default); 0: the direct forms (every neighbour read from global memory);
 * t in 1..K-1: the LDS slab form of value iteration, each workgroup staging
 * the (C+1)^t occupancies that share the high digits (evaluation: direct);
 * MDPVI_FORM_TILE + w (w = 0..8): the tile form of value iteration and
 * evaluation, the exact-shape counterpart of the slab form (K in 3..8,
 * J <= 3 distinct sizes, (C+1)^T occupancies per tile for the deepest T in
 * 2..4 whose tile fits 48 KB of LDS); w = 0 launches one workgroup per
 * tile, w > 0 launches w workgroups per CU that walk their XCD's tiles in
 * order.  The automatic choice requires at least 256 occupancies per tile
 * and 256 tiles.  Tiles are handed to the XCDs in a host-computed order:
 * the one mdp_autotune recorded for the shape, else recursive coordinate
 * bisection of the tile grid when the sweep's working set fits 256 MB and
 * runs of 16 tiles dealt round-robin beyond; the environment variable
 * MDPVI_TILE_ORDER (read at every solve; a measurement aid) forces "index"
 * (contiguous eighths), "rcb" or "dealN" (runs of N).
 * Every order and every w give bit-identical iterates.
 * MDPVI_FORM_ROW + w (w = 0..8): the row form of the value-iteration tile
 * sweep (tiles of T = 3 digits, each lane a chunk of four consecutive
 * occupancies along digit 0; compiled for K in 5..7, C = 10, J <= 3
 * distinct sizes of at most 3 units); evaluation runs in the tile form.
 * Automatic mode uses the form mdp_autotune recorded for the shape, else
 * the row form where it applies and a sweep's working set exceeds 256 MB,
 * else the tile form, else the exact-shape direct form, else the slab form.
 * Errors: MDPVI_EINVAL (NULL handle, t >= K, a slab that does not fit 64 KB
 * of LDS, or a tile or row form that does not apply).                       */
int mdp_set_sweep_form(mdpvi_mdp_t h, int32_t slab_digits);

/* Batched extraction / greedy heuristic: as policy_extract(_f64) and
 * policy_greedy for every instance, over the concatenated arrays (one
 * launch over the tiles of all instances).  Asynchronous.                   */
int policy_extract_batch(mdpvi_batch_t b, const float *V, uint8_t *pi, float *gap,
                         void *hip_stream);
int policy_extract_batch_f64(mdpvi_batch_t b, const double *V, uint8_t *pi, float *gap,
                             void *hip_stream);
int policy_greedy_batch(mdpvi_batch_t b, int32_t kind, uint8_t *pi, void *hip_stream);

/* Batched policy_eval: V device double[total] in V^0, out each instance's V_pi
 * (FP64 round-form sweeps, per-instance stopping test).  iterations and
 * residuals: host arrays of n or NULL.  Errors: as policy_eval (EINVAL names
 * the first instance with an infeasible action).                            */
int policy_eval_batch(mdpvi_batch_t b, const uint8_t *pi, double *V, double tol,
                      int64_t max_iter, void *hip_stream, mdpvi_stats *st,
                      int64_t *iterations, double *residuals);

/* Policy iteration of every instance (as policy_iteration, per instance):
 * repeat { FP64 evaluation of the instances still running (round form, to
 * eval_tol, at most eval_max_iter sweeps, each from its previous values);
 * in-place improvement of those instances with tolerance improve_tol } and
 * an instance stops at the first improvement that changes none of its
 * actions, so V holds the value of its final policy.  pi (device uint8[N]):
 * in the starting policies (feasible), out the final ones; V (device
 * double[N]): in the starting iterates, out V_pi.  rounds (host int64[n],
 * nullable): evaluations per instance.  st: evaluation sweeps summed over
 * rounds (iterations = sum over rounds of the longest instance's sweeps),
 * largest residual and bound, host wall seconds.  Synchronous.  Errors:
 * MDPVI_EINVAL (NULL pointer, eval_tol <= 0, improve_tol < 0 or not finite,
 * eval_max_iter or max_rounds < 1, an infeasible action); MDPVI_ENOCONV
 * (an evaluation reached eval_max_iter, or instances still change after
 * max_rounds; outputs hold the last round's); MDPVI_ENAN, MDPVI_EDEVICE,
 * MDPVI_ENOMEM.                                                            */
int policy_iteration_batch(mdpvi_batch_t b, uint8_t *pi, double *V, double eval_tol,
                           int64_t eval_max_iter, double improve_tol, int64_t max_rounds,
                           void *hip_stream, mdpvi_stats *st, int64_t *rounds);

/* Batched vi_adjoint.  w: device float[total] in w^0, out the adjoint weights.
 * grad: host array of sum_i (2 J_i + 2) doubles, instance i's gradient
 * (lambda_1..J_i, mu, nu, r_1..J_i) at offset sum_{k<i} (2 J_k + 2);
 * objective: host double[n] (J of every instance) or NULL; iterations: host
 * int64[n] or NULL.  Errors: as vi_adjoint.                                  */
int vi_adjoint_batch(mdpvi_batch_t b, const uint8_t *pi, const double *V_pi, float *w,
                     double *grad, double *objective, double tol, int64_t max_iter,
                     void *hip_stream, mdpvi_stats *st, int64_t *iterations);

/* Choice of the round kernels of a batch (a tuning knob: every choice gives
 * bit-identical results).  op: 0 value iteration, 1 FP64 evaluation,
 * 2 adjoint.  opt: occupancies per thread of a round kernel (its tiles hold
 * 256 * opt occupancies of one instance), 1, 2 or 4; 0 automatic (the
 * default: the choice batch_autotune recorded for this batch's instance
 * shapes, else 4).  Errors: MDPVI_EINVAL.                                   */
int batch_set_round_form(mdpvi_batch_t b, int32_t op, int32_t opt);

/* opt[3] (host): the occupancies per thread the next value iteration,
 * evaluation and adjoint calls on this batch use.  Errors: MDPVI_EINVAL.   */
int batch_round_forms(mdpvi_batch_t b, int32_t *opt);

/* Tile form of the round kernels of operation op (0 value iteration, 1 FP64
 * evaluation) for the batch's instances of 4 or 5 hosts and up to 3 classes
 * of distinct sizes (a tuning knob: the same bits either way).  Each
 * workgroup stages the values of one tile of (C+1)^3 occupancies in LDS,
 * reads every neighbour along the three low digits from there and the
 * arrival terms from FP64 side arrays (value iteration: its round-form
 * instances whose tile of values and terms would fit 60 KB; evaluation: the
 * instances with tiles of at least 1,000 occupancies whose FP64 values fit
 * 32 KB); the other instances keep the direct round kernels.  mode 1 on,
 * 0 off, -1 automatic (the default: the choice batch_autotune recorded for
 * the batch's instance shapes, else on for value iteration and off for
 * evaluation).  Errors: MDPVI_EINVAL.                                        */
int batch_set_tile_form(mdpvi_batch_t b, int32_t op, int32_t mode);

/* The number of instances the next value iteration (op 0) or evaluation
 * (op 1) call on this batch runs in the tile form (0 when the form is off
 * or covers none); -1 for a NULL batch or another op.                      */
int32_t batch_tile_form_instances(mdpvi_batch_t b, int32_t op);

/* Times one round of each operation's round kernel with 1, 2 and 4
 * occupancies per thread over every instance of the batch (trials rounds
 * each, median; zero inputs and the least-loaded policy, in temporary
 * buffers) and records the fastest per operation in the tuning cache, keyed
 * by the architecture and a digest of the instances' (K, C, J, sizes); any
 * batch of the same instance shapes then uses it.  For value iteration and
 * evaluation it then times the tile form (batch_set_tile_form) beside the
 * winner and records whether it is faster.  opt[3], us[3] (host,
 * nullable): the choices and their median microseconds per round (us[0],
 * us[1]: of the faster form; value iteration is skipped, and its entries
 * left unchanged, when every instance is solved in LDS).
 * Synchronous.  Errors: MDPVI_EINVAL, MDPVI_ENOMEM, MDPVI_EDEVICE.          */
int batch_autotune(mdpvi_batch_t b, int32_t trials, void *hip_stream, int32_t *opt, double *us);

/* The forms the next vi_solve and policy_eval on this handle run (after the
 * automatic choice): vi, eval (host, nullable).  A value in 1..K-1 is a slab
 * depth, 0 the direct form (the exact-shape one where it applies),
 * MDPVI_FORM_TILE + w the tile form, MDPVI_FORM_ROW + w the row form of
 * value iteration.  Errors: MDPVI_EINVAL (NULL handle).                     */
int mdp_sweep_forms(mdpvi_mdp_t h, int32_t *vi, int32_t *eval);

/* Autotuner (a tuning step of this library; not in the paper): times, on
 * this instance, `trials` single sweeps of every applicable form of
 *   value iteration (direct, LDS slabs of 1..K-1 low digits that fit 64 KB,
 *     tile and row forms with 0..4 workgroups per CU), from V;
 *   FP64 evaluation (direct, tile with 0..5 workgroups per CU) and
 *   the adjoint sweep (group form, generic and exact-shape kernels with 1,
 *     2 or 4 occupancies per thread), both on the least-loaded policy;
 * and, when a tile or row form wins, that form under each tile order (the
 * assignment of tiles to the 8 XCDs: recursive coordinate bisection, index
 * order, runs of 16 or of (C+1)^2 consecutive tiles dealt round-robin);
 * (V: device float[N], read only; the sweeps write the handle's scratch and
 * temporary buffers), keeps each operation's form (and tile order) with the
 * smallest median time and records it for the shape (GPU arch, K, C, J,
 * sizes): later calls
 * in automatic mode on any handle of that shape use it (vi_solve,
 * policy_eval, vi_adjoint and the calls built on them).  When the
 * environment variable MDPVI_AUTOTUNE_CACHE names a file, the records are
 * loaded from and saved to it as JSON.  best_form / best_us (host,
 * nullable): value iteration's chosen form and its median microseconds per
 * sweep.  Synchronous.  Errors: MDPVI_EINVAL, MDPVI_EDEVICE, MDPVI_ENOMEM. */
int mdp_autotune(mdpvi_mdp_t h, const float *V, int32_t trials, void *hip_stream,
                 int32_t *best_form, double *best_us);

/* The adjoint sweep form the next vi_adjoint on this handle runs:
 * MDPVI_ADJOINT_GROUP for the group form, 16 + OPT for the exact-shape
 * kernels (K in 3..8, J <= 3), OPT for the generic ones, OPT in {1, 2, 4}
 * occupancies per thread.  The form set by mdp_set_adjoint_form, else the
 * recorded tuning, else the group form where it applies, else the
 * exact-shape kernels with one occupancy per thread below 2^21 occupancies
 * and four above, else the generic ones; -1 for a NULL handle.             */
int32_t mdp_adjoint_form(mdpvi_mdp_t h);

/* Choice of the adjoint sweep kernels for this handle (a tuning knob: every
 * form gives bit-identical w and gradients).  0: automatic (the default);
 * MDPVI_ADJOINT_GROUP: the group form (each workgroup takes whole groups of
 * the (C+1)^2 occupancies that share digits 2..K-1, one occupancy per lane;
 * neighbours along digits 0 and 1, including the reset line sums of the
 * transposed backup of Eq. (18), are read from LDS; K in 3..8, J <= 3,
 * C <= 15, fewer than 2^29 states); 16 + OPT or OPT as for mdp_adjoint_form.
 * Errors: MDPVI_EINVAL (NULL handle, or a form that does not apply).        */
int mdp_set_adjoint_form(mdpvi_mdp_t h, int32_t form);

/* Per-sweep kernel timing for the iterative calls of this handle: when on,
 * every sweep launch is bracketed by two HIP events and their elapsed times
 * are summed into mdpvi_stats.sweep_seconds (a measurement aid; it adds two
 * event records per sweep).  Errors: MDPVI_EINVAL (NULL handle).           */
int mdp_set_timing(mdpvi_mdp_t h, int32_t per_sweep_events);

/* ---- Static bags of tasks (Alg. 2; the example of Sec. VII) ------------
 * B independent scenarios, each K vehicular clouds (VCs) with free VM
 * capacities and T task slots in arrival order (bag by bag, tasks of a bag
 * in order).  Layouts, all device arrays, row-major by scenario:
 *   caps   int32 [B][K]   free VMs of each VC, in [0, 2^30]
 *   need   int32 [B][T]   VMs a task needs, in [0, 2^30]; 0 = empty slot
 *   place  int32 [B][T]   VC index, MDPVI_STATIC_PAID, or MDPVI_STATIC_EMPTY
 *   used   int32 [B][K]   VMs taken on each VC
 *   totals int64 [B][3]   (VMs in VCs, VMs in the paid cloud, idle VMs left in VCs)
 *   reward double [B]     beta_vc*vc - beta_tc*paid - gamma_vc*idle (Eqs. (14)-(16)
 *                         summed over the cloud; each product rounded, then
 *                         subtracted left to right)
 *   status int32 [B]      0 ok; 1 a capacity, 2 a need out of range; 3 a VC
 *                         over capacity, 4 a place code outside [-1, K) on a
 *                         task (static_score only).  A scenario with a nonzero
 *                         status gets no other output.
 * need and place may be NULL when T = 0; B = 0 is a no-op.  K in [1, 64],
 * beta_vc, beta_tc, gamma_vc finite.  Both calls are asynchronous on the
 * stream.  Errors (host-side argument checks only): MDPVI_EINVAL,
 * MDPVI_ERANGE (B above 2^33 - 4 or B*T above 2^62), MDPVI_EDEVICE.        */
#define MDPVI_STATIC_MAX_K 64
#define MDPVI_STATIC_PAID (-1)
#define MDPVI_STATIC_EMPTY (-2)

/* The fast greedy heuristic of Alg. 2: each task goes to the first VC, in
 * index order, that still has need[t] free VMs, and takes them; if no VC
 * has, it goes to the paid cloud.  Writes place, used, totals, reward and
 * status.                                                                   */
int static_first_fit(const int32_t *caps, const int32_t *need, int64_t B, int32_t K, int64_t T,
                     double beta_vc, double beta_tc, double gamma_vc, int32_t *place, int32_t *used,
                     int64_t *totals, double *reward, int32_t *status, void *hip_stream);

/* Score a given placement (for instance the best one, or an MDP's): place is
 * read, not written (codes on empty slots are ignored).  Writes used, totals,
 * reward and status.                                                        */
int static_score(const int32_t *caps, const int32_t *need, const int32_t *place, int64_t B, int32_t K,
                 int64_t T, double beta_vc, double beta_tc, double gamma_vc, int32_t *used,
                 int64_t *totals, double *reward, int32_t *status, void *hip_stream);

/* Thread-local text of the last failure ("" if none). */
const char *mdpvi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MDPVI_H */
