/*
 * pgo.h -- C ABI of the MI355X (gfx950) PRADMM sweep library.
 *
 * Problem (Model section, eq. 1): n poses (p_i unit quaternion, t_i in R^3)
 * and m directed edges e = (i -> j) carrying a relative rotation R~_ij, a
 * relative translation t~_ij and isotropic precisions kappa_ij (rotation)
 * and tau_ij (translation).  The library runs the Parallelizable Riemannian
 * ADMM of Alg. 1 on the split model (eq. 2): each sweep updates, for every
 * vertex in parallel, p (projection onto the unit sphere, App. B.1), q
 * (App. B.2), t (App. B.3), s (App. B.4), then the multipliers lambda and z
 * with relaxation step gamma in (0, 2) (eq. 3e-3f).
 *
 * Conventions
 *   - quaternions are [w, x, y, z] with the Hamilton product of App. A.2;
 *     rotation matrices are row-major 3x3, R v = Im(q [0, v] q^*).
 *   - Sigma1 = tau_e I, Sigma2 = kappa_e I per edge; one penalty
 *     beta = beta1 = beta2; proximal weights H_s = h_s I.
 *   - state of a vertex, as 21 doubles: p(4) q(4) t(3) s(3) lambda(4) z(3).
 *
 * Second model (pgo_options.model = PGO_MODEL_CHORDAL): the same splitting
 * and sweep applied to the chordal cost (chordal distance of App. A.4 on the
 * rotation measurements, model (1)'s translation term), rotations kept as
 * 3x3 matrices: P_i in SO(3) (a 3x3 polar factor per vertex and sweep),
 * Q_i and the multiplier Lambda_i free 3x3 blocks.  This is not the paper's
 * quaternion model; its state is 36 doubles per vertex:
 * P(9) Q(9) t(3) s(3) Lambda(9) z(3), matrices row-major.  Everything below
 * applies to both models unless it says otherwise.
 *
 * Ownership: host arrays passed to pgo_create* are read during the call and
 * copied; the caller keeps them.  A handle owns all of its device memory
 * until pgo_destroy.  Output buffers are caller-allocated.  Pointers named
 * *_dev are device pointers on the handle's device.
 *
 * Threading: a handle is not thread-safe.  All work of a handle is enqueued
 * on one HIP stream (its own, or the one given to pgo_set_stream); calls
 * that return host data synchronise that stream.
 *
 * Errors: every call returns a pgo_status; pgo_last_error() returns a
 * thread-local message describing the last failure.
 */
#ifndef PGO_H
#define PGO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pgo_graph pgo_graph;

typedef enum {
  PGO_OK = 0,
  PGO_EINVAL = 1,   /* invalid argument (message names the offending item) */
  PGO_ENOMEM = 2,   /* device or host allocation failed */
  PGO_EDEVICE = 3,  /* HIP runtime error (message carries hipGetErrorString) */
  PGO_ENUMERIC = 4, /* a reduction found a non-finite value in the state */
  PGO_ESTATE = 5    /* call not valid for this handle (e.g. wrong precision) */
} pgo_status;

typedef enum {
  PGO_FP64 = 0, /* state, edges and arithmetic in double */
  PGO_FP32 = 1  /* state, edges and accumulation in float; double for the
                   boundary preparation, the cost/residual reductions and a
                   p-update whose sum cancels (|v| < 1e-3 of the summed
                   magnitudes) */
} pgo_precision;

typedef enum {
  PGO_SCHED_AUTO = 0,  /* per graph for at least 256 graphs of at most 8192
                          poses, else per phase (or the autotuner's choice) */
  PGO_SCHED_PHASE = 1, /* one kernel launch per phase; any graph size */
  PGO_SCHED_GRAPH = 2, /* one persistent workgroup per graph runs all the
                          sweeps of one pgo_iterate call (graphs of at most
                          PGO_GRAPH_SCHED_MAX_N vertices) */
  PGO_SCHED_COOP = 3   /* one persistent cooperative launch runs all the
                          sweeps of one pgo_iterate call, every phase over
                          all vertices with a device-wide barrier between
                          phases; bitwise the state of PGO_SCHED_PHASE;
                          quaternion model (PGO_MODEL_QUAT) only.  The
                          barrier's wait is bounded (seconds): a launch
                          whose wait runs out ends anyway and writes NaN
                          into the first vertex's translation, so the next
                          cost or residual call reports PGO_ENUMERIC */
} pgo_schedule;

#define PGO_GRAPH_SCHED_MAX_N 65536

typedef enum {
  PGO_MODEL_QUAT = 0,    /* the paper's unit-quaternion model (eq. 1-2) */
  PGO_MODEL_CHORDAL = 1, /* rotation matrices, chordal rotation cost; FP32
                            takes the P update's 3x3 polar factor in double
                            when it is ill-conditioned (sigma_2 + sign(det)
                            sigma_3 below 1e-2 of the summed term sizes) */
  PGO_MODEL_QUAT_INFO = 2 /* the quaternion model with a full 3x3 translation
                            information matrix per edge (pgo_create_info);
                            at most 256 threads per workgroup (512 in the
                            per-graph schedule) */
} pgo_model;

typedef struct {
  double h1, h2, h3, h4; /* proximal weights H_1..H_4 (defaults 1, 1e-3, 1e-3,
                            1e-3: the experiment settings) */
  int32_t precision;     /* pgo_precision, default PGO_FP64 */
  int32_t schedule;      /* pgo_schedule, default PGO_SCHED_AUTO */
  int32_t block;         /* threads per workgroup; 0 = library default */
  int32_t device;        /* HIP device ordinal, default 0 */
  int32_t model;         /* pgo_model, default PGO_MODEL_QUAT */
} pgo_options;

/* Fill *opt with the defaults above. */
void pgo_default_options(pgo_options* opt);

/*
 * pgo_create -- build a handle for one pose graph (Alg. 1 input: the graph,
 * the measurements, the initial points).
 *   n         number of poses, >= 1
 *   R0, t0    initial rotations (n x 9, row-major) and translations (n x 3)
 *   m         number of edges, >= 0 (< 2^31)
 *   ei, ej    edge tails and heads (m each), 0 <= ei, ej < n, ei != ej
 *   Rm, tm    measured relative rotations (m x 9) and translations (m x 3)
 *   kappa,tau precisions (m each), finite and > 0
 *   opt       options, or NULL for the defaults
 * Every rotation must have det > 0 and ||R^T R - I||_F <= 1e-2; it is
 * projected onto SO(3) on the device (FP64 3x3 Jacobi SVD polar factor) and
 * converted to a unit quaternion.  A vertex quaternion's sign is chosen so
 * that its first component of magnitude > 1e-6 is positive; each edge
 * quaternion's sign so that <p_i^0 q~_e, p_j^0> >= 0 (the cost of model (1)
 * depends on that sign and a rotation matrix does not fix it).  Initial
 * state: q = p, s = t, lambda = z = 0.  Duplicate and reverse edges,
 * isolated vertices and disconnected graphs are allowed.
 * Returns PGO_EINVAL (bad input, message names it), PGO_ENOMEM, PGO_EDEVICE.
 */
pgo_status pgo_create(pgo_graph** out, int32_t n, const double* R0, const double* t0,
                      int64_t m, const int32_t* ei, const int32_t* ej, const double* Rm,
                      const double* tm, const double* kappa, const double* tau,
                      const pgo_options* opt);

/*
 * pgo_create_batched -- G independent pose graphs in one handle.  Graph g
 * owns poses voff[g]..voff[g+1]-1 and edges eoff[g]..eoff[g+1]-1 of the
 * concatenated arrays (same layouts as pgo_create); ei/ej are graph-local
 * (0 <= ei < voff[g+1]-voff[g]).  voff[0] = eoff[0] = 0, every graph has at
 * least one pose, offsets are nondecreasing.  Sweeps and gamma are shared
 * by all graphs; beta is shared (pgo_iterate) or per graph
 * (pgo_iterate_graphs); costs and residuals are reported per graph.
 */
pgo_status pgo_create_batched(pgo_graph** out, int32_t G, const int64_t* voff,
                              const int64_t* eoff, const double* R0, const double* t0,
                              const int32_t* ei, const int32_t* ej, const double* Rm,
                              const double* tm, const double* kappa, const double* tau,
                              const pgo_options* opt);

/*
 * pgo_create_info -- the quaternion model with a general translation weight
 * per edge (Model section: Sigma1 = diag(c, Omega1^{-1}), Sigma2 = kappa I):
 * info (m x 9, row-major) holds each edge's information matrix S_e =
 * Omega_e^{-1}, symmetric (to 1e-12 of its largest entry) and positive
 * definite; c_e = trace(S_e) / 3 (c is arbitrary in the paper; with S_e =
 * tau_e I this is the isotropic model with tau_e).  The blocks of App. B are
 * full matrices: the p update is the sphere-constrained quadratic of Lemma 1
 * (solved per vertex in FP64 by the secular equation of Lemma B.1, hard case
 * included), q a 4x4 and t, s 3x3 positive definite solves.  Other arrays
 * and offsets as pgo_create_batched (G >= 1); opt->model is set to
 * PGO_MODEL_QUAT_INFO.  The state is the quaternion model's (21 doubles).
 * pgo_chordal_init weighs translations by c_e.  No reverse mode.
 */
pgo_status pgo_create_info(pgo_graph** out, int32_t G, const int64_t* voff, const int64_t* eoff,
                           const double* R0, const double* t0, const int32_t* ei,
                           const int32_t* ej, const double* Rm, const double* tm,
                           const double* kappa, const double* info, const pgo_options* opt);

/* Use the given hipStream_t (e.g. torch.cuda.current_stream().cuda_stream)
 * for all later work of the handle; NULL returns to the handle's own stream. */
pgo_status pgo_set_stream(pgo_graph* g, void* hip_stream);

/*
 * pgo_iterate -- enqueue k PRADMM sweeps (Alg. 1 steps 2-6) with penalty
 * beta > 0 and relaxation gamma in (0, 2) (open interval).  k = 0 is a
 * no-op.  Asynchronous: returns once the work is enqueued.
 */
pgo_status pgo_iterate(pgo_graph* g, int32_t k, double beta, double gamma);

/*
 * pgo_iterate_graphs -- pgo_iterate with one penalty per graph of the handle:
 * beta is a host array of G values, each finite and > 0 (graph g runs with
 * beta[g]; the theory asks beta above a problem-dependent threshold, so a
 * batch of graphs with very different weight scales needs its own beta per
 * graph).  The residual e of pgo_residuals then uses each graph's beta.
 */
pgo_status pgo_iterate_graphs(pgo_graph* g, int32_t k, const double* beta, double gamma);

/* Cost of model (1) at (p, t), one double per graph, accumulated in FP64. */
pgo_status pgo_cost(pgo_graph* g, double* F);

/*
 * Residuals, 6 doubles per graph:
 *   [0] ||p - q||, [1] ||t - s||,
 *   [2] e = (||dlambda||^2 + ||dz||^2)/beta + beta(||dq||^2 + ||dt||^2)
 *       (iteration residual of App. E.1; d = change over the last sweep,
 *        the graph's beta of the last iterate call; 0 before any sweep),
 *   [3] beta ||dq||, [4] beta ||ds|| (dual residuals),
 *   [5] cost of model (1).
 * All sums in FP64.  PGO_ENUMERIC if any value is not finite.
 */
pgo_status pgo_residuals(pgo_graph* g, double* out);

/*
 * Merit values, 2 doubles per graph: [0] the augmented Lagrangian L_beta
 * (PRADMM section, beta1 = beta2 = the graph's beta) at the current state,
 * [1] Psi = L_beta + alpha1/(gamma beta) ||dlambda||^2, alpha1 =
 * |1-gamma|/(1-|1-gamma|): the Lyapunov function of Theorem 1 without its
 * proximal-difference terms (whose weights the paper leaves implicit).
 * Uses the beta and gamma of the last iterate/solve call.  FP64 sums.
 */
pgo_status pgo_merit(pgo_graph* g, double* out);

/*
 * pgo_evaluate -- pgo_cost, pgo_residuals and pgo_merit from one pass of the
 * FP64 reductions over the current state (the values are those of the
 * three calls; one device pass and one synchronisation instead of three).
 *   F      out, G doubles, or NULL
 *   res    out, G x 6 doubles (as pgo_residuals), or NULL
 *   merit  out, G x 2 doubles (as pgo_merit), or NULL
 * PGO_ENUMERIC if any value is not finite.
 */
pgo_status pgo_evaluate(pgo_graph* g, double* F, double* res, double* merit);

/*
 * pgo_evaluate_noalloc -- pgo_evaluate for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same FP64 reductions, with their
 * partial sums and per-graph values in a static device array of the library
 * (2 MiB on each device it runs on, held until the process ends) instead of
 * the handle's buffers, and every result written on the device.  No
 * allocation, no host transfer and no synchronisation: the work is enqueued
 * on the handle's stream.
 *   beta_dev  in, device, G doubles: each graph's penalty (pgo_evaluate uses
 *             those of the last iterate call)
 *   gamma     the relaxation step of the merit (pgo_evaluate uses the last
 *             iterate call's)
 *   out_dev   out, device, G x 8 doubles per graph: F, the five residuals of
 *             pgo_residuals [0..4], L_beta and Psi of pgo_merit -- equal bit
 *             for bit to what pgo_evaluate returns for the same penalties
 * Quaternion models (PGO_MODEL_QUAT, PGO_MODEL_QUAT_INFO) only
 * (PGO_ESTATE otherwise).  PGO_EINVAL when the handle's reductions need more
 * of the array than it holds (2 per edge chunk + 9 per vertex chunk + 11 per
 * graph doubles, chunks of up to 8192 items per graph; the 4096-graph batch
 * needs about a third of it).  The array is shared by every call on one
 * device and keeps the last call's contents (each call writes all it
 * reads); calls that overlap on one device race on it.  Non-finite values
 * are returned as they are (no PGO_ENUMERIC).
 */
pgo_status pgo_evaluate_noalloc(pgo_graph* g, const double* beta_dev, double gamma,
                                double* out_dev);

/*
 * pgo_iterate_until -- sweeps with the experiments' stopping rule and no
 * penalty control: every graph runs chunks of check_every sweeps at its
 * beta (host array, G values > 0) and stops after the first chunk whose
 * last sweep leaves the residual e of App. E.1 below tol (see
 * pgo_residuals [2]), or after max_sweeps sweeps (a multiple of
 * check_every).  For the quaternion model in the per-graph schedule the
 * whole call is one launch and each graph evaluates e inside it (FP64 sums
 * of the stored values), with no host round trip per chunk; otherwise the
 * chunks are separate launches checked on the host.  The state equals that
 * of the same chunks run by pgo_iterate_graphs calls.
 *   sweeps_done  out, G values: the sweeps each graph ran
 * Synchronises the stream.
 */
pgo_status pgo_iterate_until(pgo_graph* g, int32_t max_sweeps, int32_t check_every,
                             const double* beta, double gamma, double tol, int32_t* sweeps_done);

/*
 * pgo_solve -- the outer loop of Alg. 1 with the experiments' stopping rule
 * and penalty check, per graph.  Sweeps run in chunks of check_every (one
 * launch per chunk for all graphs still running).  After each chunk, for
 * every running graph:
 *   - if beta_growth > 1 and its merit Psi (see pgo_merit) rose over the
 *     chunk by more than the rounding noise of the state (1e-12 |Psi| +
 *     8 eps (beta + w) n, eps the unit roundoff of the precision, w the
 *     graph's mean vertex weight 2 sum_out (tau |t~|^2 + kappa) + 2 sum_in
 *     kappa, n its vertex count), or the chunk left a non-finite value in
 *     the graph, the chunk is undone for that graph (state restored on the
 *     device) and its beta multiplied by beta_growth (at most 40 times per
 *     call and never past 1e30; Theorem 1 asks beta above a threshold the
 *     paper does not give, and the experiments adjust beta by checking
 *     exactly this descent);
 *   - otherwise the chunk is accepted; the graph stops when its residual
 *     e (App. E.1) is below tol (tol <= 0: never) or after max_sweeps
 *     accepted sweeps.
 *   max_sweeps  accepted sweeps per graph, a multiple of check_every
 *   beta        in/out, G values > 0 (the penalties reached)
 *   sweeps_done out, G values (accepted sweeps), may be NULL
 *   converged   out, G values (1 where e < tol stopped the graph), may be NULL
 * PGO_ENUMERIC when a graph reaches a non-finite state that cannot be undone
 * (beta_growth == 1, or its beta can grow no further).
 * Synchronises the stream once per chunk.
 */
pgo_status pgo_solve(pgo_graph* g, int32_t max_sweeps, int32_t check_every, double gamma,
                     double tol, double beta_growth, double* beta, int32_t* sweeps_done,
                     int32_t* converged);

/* Current poses: R(p_i) (chordal model: P_i) (n x 9, row-major) and t_i
 * (n x 3); either may be NULL. */
pgo_status pgo_get_poses(pgo_graph* g, double* R, double* t);

/* Raw state, n x 21 doubles (chordal model: n x 36; see conventions);
 * set_state restarts the residual history (the next residuals report d = 0
 * until a sweep runs). */
pgo_status pgo_get_state(pgo_graph* g, double* state);
pgo_status pgo_set_state(pgo_graph* g, const double* state);

/* The prepared (projected, converted, sign-aligned) edge quaternions in the
 * caller's edge order (m x 4) and vertex quaternions p^0 (n x 4); either may
 * be NULL.  Chordal model: the projected measured rotations (m x 9) and
 * initial rotations P^0 (n x 9), row-major. */
pgo_status pgo_get_prepared(pgo_graph* g, double* edge_quat, double* vertex_quat0);

/* Sizes and settings of the handle; any pointer may be NULL.  lds = 1 when
 * the per-graph schedule keeps each graph's state in LDS for the whole
 * launch as far as it fits, by graph size (quaternion and information
 * models: p, q, t, s, then the multipliers; chordal model: s, P, t, Q, z,
 * Lambda; within 160 KiB per workgroup; chosen by default or by the
 * autotuner). */
pgo_status pgo_info(pgo_graph* g, int64_t* n, int64_t* m, int32_t* G, int32_t* precision,
                    int32_t* schedule, int32_t* block, int32_t* model, int32_t* lds);

/*
 * pgo_autotune -- time the candidate schedules, workgroup sizes and (per-
 * graph schedule) LDS residency of the state on this handle's own
 * graphs (sweeps sweeps each, beta, gamma), keep the fastest for later
 * pgo_iterate calls, and restore the state it found.  Reports the choice
 * through pgo_info.
 */
pgo_status pgo_autotune(pgo_graph* g, double beta, double gamma, int32_t sweeps);

/*
 * pgo_chordal_init -- chordal initialisation, the step before the path (the
 * experiments section starts every method from it; the paper cites it
 * without describing it).  Per graph and connected component, with the
 * component's lowest-index vertex held at its current initial pose:
 *   1. relaxed rotations: min sum_e kappa_e |R_i R~_e - R_j|_F^2 over free
 *      3x3 blocks (model (1)'s rotation term in chordal distance, App. A.4);
 *   2. each R_i projected onto SO(3) (3x3 polar factor);
 *   3. translations: min sum_e tau_e |t_j - t_i - R_i t~_e|^2.
 * Both least-squares problems are solved on the device in FP64 by
 * Jacobi-preconditioned conjugate gradients per graph, from the current
 * initial point, until <r, M^-1 r> <= tol^2 of its starting value or
 * max_iters iterations.  The result replaces the handle's initial point
 * (quaternion model: p^0, and each edge quaternion's sign aligned against
 * the new p^0 as at create) and the state is reset to it (as
 * pgo_reset_state).
 *   max_iters >= 1; tol in (0, 1)
 *   iters  out, G x 2 (iterations of the rotation and translation solves),
 *          may be NULL
 * Device scratch is allocated for the call and released before it returns.
 * Synchronises the stream.
 */
pgo_status pgo_chordal_init(pgo_graph* g, int32_t max_iters, double tol, int32_t* iters);

/*
 * Differentiation of K unrolled sweeps (reverse mode written by hand).
 * pgo_set_edge_params, pgo_forward_record and pgo_adjoint exist for the
 * isotropic quaternion model only (PGO_ESTATE on other handles).
 *
 * pgo_set_edge_params -- replace edge parameters in place (caller edge
 * order, device FP64 pointers; NULL keeps the current values): kappa (m),
 * tau (m), tm (m x 3), omega (m x 3).  omega is a right perturbation of each
 * measured rotation, R~_e Exp(omega_e), applied to the prepared quaternion
 * of pgo_create: q~_e = q~0_e [cos(|w|/2), sin(|w|/2) w/|w|].  Values are
 * checked (kappa, tau finite and > 0; tm, omega finite): PGO_EINVAL names
 * the first bad entry.  The graph structure is unchanged; a recorded
 * forward pass is discarded.  Synchronises the stream.
 */
pgo_status pgo_set_edge_params(pgo_graph* g, const double* kappa_dev, const double* tau_dev,
                               const double* tm_dev, const double* omega_dev);

/* Put the state back to the initial point of pgo_create (q = p^0, s = t^0,
 * lambda = z = 0; chordal: Q = P^0, Lambda = 0). */
pgo_status pgo_reset_state(pgo_graph* g);

/* The state (n x 21, chordal n x 36 doubles) written to a device buffer
 * (asynchronous). */
pgo_status pgo_get_state_dev(pgo_graph* g, double* state_dev);

/*
 * pgo_forward_record -- run K >= 1 sweeps (scalar beta, gamma in (0,2))
 * from the current state, keeping the state every C >= 1 sweeps (and at K)
 * so that pgo_adjoint can recompute the sweeps in between.  Device memory:
 * (ceil(K/C) + C + 2) state copies.
 */
pgo_status pgo_forward_record(pgo_graph* g, int32_t K, double beta, double gamma, int32_t C);

/*
 * pgo_record_id -- which forward pass the handle's recording is: the count
 * of pgo_forward_record calls on the handle, or -1 when there is no
 * recording (none made, or the edges or the state were replaced since:
 * pgo_set_edge_params, pgo_reset_state, pgo_chordal_init).  A caller that
 * keeps gradients of several forward passes compares it before pgo_adjoint,
 * which always uses the latest recording.
 */
pgo_status pgo_record_id(pgo_graph* g, int64_t* id);

/*
 * pgo_adjoint -- gradients of a scalar loss L(x^K) through the recorded
 * sweeps.  dL_dstate: device n x 21 FP64, dL/dx^K in the state layout.
 * Outputs (device FP64, caller edge order, any may be NULL): g_kappa (m),
 * g_tau (m), g_tm (m x 3), g_omega (m x 3, derivative with respect to the
 * omega of pgo_set_edge_params at its current value), dL_dstate0 (n x 21,
 * dL/dx^0).  Each graph segment of C sweeps is recomputed from its
 * checkpoint; the reverse sweep runs in the handle's precision and sums
 * edge gradients in FP64.  Leaves the state at x^K.  PGO_ESTATE if no
 * forward pass is recorded.  Synchronises the stream.
 */
pgo_status pgo_adjoint(pgo_graph* g, const double* dL_dstate, double* g_kappa, double* g_tau,
                       double* g_tm, double* g_omega, double* dL_dstate0);

/* Release the handle and its device memory.  NULL is ignored. */
void pgo_destroy(pgo_graph* g);

/* Message for the last error on the calling thread ("" if none). */
const char* pgo_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PGO_H */
