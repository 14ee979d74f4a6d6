/*
 * rh.h - reduced Hessians of the power-flow balance equations on MI355X.
 *
 * C ABI of librh.  The operations follow the paper "Batched Second-Order
 * Adjoint Sensitivity for Reduced Space Methods":
 *   - the network and its balance equations g(x, p) = 0 (Sec. 3.1,
 *     eq. (powerflow), eq. (powerflowvec));
 *   - Newton-Raphson projection onto g = 0 (Sec. 3.2);
 *   - the reduced gradient by the first-order adjoint (Sec. 3.3,
 *     eq. (lagrangian), eq. (reduced_gradient));
 *   - reduced-Hessian-vector products by the batched adjoint-adjoint
 *     reduction (Sec. 4.1 eq. (socadjoint), eq. (hessvecprod); Sec. 4.3
 *     Algorithm 2), and the full reduced Hessian assembled by blocks of
 *     directions (Sec. 5.3).
 *
 * Conventions (all entry points):
 *   - Every function returns an rh_status; nothing else crosses the ABI
 *     (no exceptions, no aborts).  rh_last_error() returns a message for the
 *     most recent failure on the calling thread.
 *   - Host matrices are column-major; a block of k directions W is n_p x k
 *     with leading dimension ldw >= n_p, and so is its product HW.
 *   - The caller owns every buffer it passes.  rh_network_create copies the
 *     description; handles returned through `out` are owned by the library
 *     and released with the matching destroy call.
 *   - A network handle is not re-entrant: calls on one handle must not
 *     overlap.  Distinct handles may be used from different threads.
 *   - State and parameter orderings (eq. (powerflowvec), parameter count of
 *     Table 1):
 *       x = [theta at PV buses; theta at PQ buses; v at PQ buses]
 *       p = [Pg at PV buses; v at the reference bus; v at PV buses]
 *     each block in ascending bus id.  rh_network_index_maps exports them.
 *   - Units are per-unit.  The cost is f = sum over generators of
 *     c2 Pg^2 + c1 Pg + c0, the reference generator's Pg being its bus
 *     balance P^inj_ref + Pd_ref (the paper leaves f unspecified beyond its
 *     dependence on the generation).
 */
#ifndef RH_H
#define RH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rh_context rh_context; /* opaque; one per GPU (or host-only) */
typedef struct rh_network rh_network; /* opaque; one network + operating point */

typedef enum {
  RH_OK = 0,
  RH_EINVAL = -1,    /* bad argument or network description (incl. NaN/Inf) */
  RH_ENOMEM = -2,    /* host or device allocation failed */
  RH_ENOCONV = -3,   /* Newton did not reach the tolerance */
  RH_ESINGULAR = -4, /* G_x is singular or numerically so (tiny pivot) */
  RH_ESTATE = -5,    /* call out of order, e.g. a product before a solve */
  RH_EDEVICE = -6,   /* HIP error, or a device call on a host-only context */
  RH_EBUSY = -7      /* reserved for callers that share a handle */
} rh_status;

typedef enum {
  RH_FP64 = 0,        /* every step in FP64 */
  RH_FP32_REFINED = 1 /* triangular sweeps in FP32 with FP64 residual refinement
                         (see rh_context_set_refinement): residuals, stored
                         vectors, tensor projection and G_p products in FP64;
                         LU factors computed in FP64 */
} rh_precision;

/* Network description (Sec. 3.1).  All arrays are read-only and copied.
 * Branch b joins br_from[b] and br_to[b] (0-based, distinct) with series
 * impedance br_r + j br_x and total line charging br_b, half at each end.
 * bus_type: 1 = PQ, 2 = PV, 3 = reference (exactly one).  gen_bus lists one
 * generator per PV bus and one at the reference bus (no other buses);
 * Pg is its active set-point (ignored for the reference generator), Vg its
 * voltage set-point, c2/c1/c0 its cost coefficients. */
typedef struct {
  int32_t n_bus, n_branch, n_gen;
  const int32_t *br_from, *br_to;
  const double *br_r, *br_x, *br_b;
  const int32_t *bus_type;
  const double *Pd, *Qd;
  const int32_t *gen_bus;
  const double *Pg, *Vg, *c2, *c1, *c0;
} rh_network_desc;

/* Launch shape of a network's products in one precision, chosen by
 * rh_autotune: the full Hessian's launch size (k directions per launch, the
 * block of Sec. 5.3), the directions one workgroup owns, and the two
 * parameters of the triangular-sweep schedule (the largest dense block of
 * merged narrow levels, and whether elimination-tree subtrees are walked by
 * single waves).  k = 0: not chosen yet (library defaults). */
typedef struct {
  int32_t k;
  int32_t dirs_per_group;  /* 1, 2 or 4 */
  int32_t block_rows;      /* 0 (no merged blocks) .. 64 */
  int32_t wave_steps;      /* 0 or 1 */
  double ms_per_hessian;   /* the tuner's estimate for the full Hessian */
  int32_t source;          /* 0 defaults, 1 measured, 2 read from the cache */
} rh_tile;

/* Figures of the last solve and the last Hessian call on a network. */
typedef struct {
  int32_t n_x, n_p;
  int64_t nnz_gx, nnz_l, nnz_u; /* G_x and its LU factors (unit diagonal of L not stored) */
  int32_t levels_l, levels_u;   /* dependency depth of the L and U sweeps */
  int32_t steps_l, steps_u;     /* barrier-separated steps of the device sweeps
                                   (narrow levels merged into dense-inverse blocks) */
  int32_t newton_iters;
  double newton_resid;          /* ||g||_inf at the accepted state */
  int32_t last_k;               /* directions in the last product call */
  int32_t last_launches;        /* kernel launches since the previous report */
  int32_t dirs_per_group;       /* directions owned by one workgroup (last launch) */
  double last_kernel_ms;        /* summed duration of those launches when timing was
                                   on (HIP events on the launch stream), else -1 */
  double phase_us[7];           /* timing level 2: mean time per workgroup of SpMul,
                                   L sweep, U sweep, tensor projection, U^T sweep,
                                   L^T sweep, SpMulAdd in the last timed launch */
  rh_tile tile[2];              /* launch shapes chosen so far, FP64 and refined */
} rh_report;

/* Create a context on HIP device `device`; device = -1 gives a host-only
 * context (network set-up, Newton and gradients work; products return
 * RH_EDEVICE). */
rh_status rh_context_create(int32_t device, rh_context **out);
rh_status rh_context_destroy(rh_context *ctx);
/* Timing: 0 off; 1 HIP events around every kernel launch
 * (rh_report.last_kernel_ms); 2 also in-kernel phase timestamps
 * (rh_report.phase_us), which add a little work per workgroup. */
rh_status rh_context_set_timing(rh_context *ctx, int32_t on);

/* Refined mode (RH_FP32_REFINED): each of the two sparse solves of a direction
 * (G_x z = b and G_x^T psi = b') is x = solve32(b), then corrections
 * x += solve32(r) with the FP64 residual r = b - A x, until
 * ||r||_inf <= tol ||A||_inf ||x||_inf (a backward-error test) or `steps`
 * corrections were made.  Each direction stops on its own.  Defaults: at most
 * 4 corrections, tol 1e-13; tol 0 makes every direction take all `steps`. */
rh_status rh_context_set_refinement(rh_context *ctx, int32_t steps);     /* 0 .. 16 */
rh_status rh_context_set_refinement_tol(rh_context *ctx, double tol);   /* finite, >= 0 */

/* Validate and copy a network; builds the index maps, the sparsity pattern of
 * G_x, a fill-reducing ordering, the symbolic LU and the level schedules.
 * The parameters start at the description's set-points. */
rh_status rh_network_create(rh_context *ctx, const rh_network_desc *desc, rh_network **out);
rh_status rh_network_destroy(rh_network *net);
rh_status rh_network_dims(const rh_network *net, int32_t *n_x, int32_t *n_p);
/* x_bus[n_x], x_kind[n_x], p_bus[n_p], p_kind[n_p]; kind 0 = angle,
 * 1 = voltage magnitude, 2 = generator active power.  Any pointer may be NULL. */
rh_status rh_network_index_maps(const rh_network *net, int32_t *x_bus, int32_t *x_kind,
                                int32_t *p_bus, int32_t *p_kind);

/* Replace p (n_p values) or the loads (n_bus values each).  Both invalidate
 * the solution: products and gradients return RH_ESTATE until the next
 * successful rh_solve_powerflow. */
rh_status rh_set_parameters(rh_network *net, const double *p);
rh_status rh_get_parameters(const rh_network *net, double *p);
rh_status rh_set_loads(rh_network *net, const double *Pd, const double *Qd);

/* Starting point of the next Newton solve: x0 (n_x values, the state
 * ordering), or NULL for a flat start (angles 0, PQ magnitudes 1).  Kept until
 * replaced; a good guess is the previous operating point's state. */
rh_status rh_set_initial_state(rh_network *net, const double *x0);

/* Newton-Raphson from the initial state (flat start by default) until
 * ||g||_inf <= tol or max_iter steps (Sec. 3.2); a residual below 1e-11 that
 * no longer halves after three steps counts as converged (rounding level of
 * a large grid, resid_inf reports it).  On success it factorises
 * G_x, forms the first-order adjoint and the per-branch second-order
 * coefficients, and (on a device context) uploads them.  iters/resid_inf may
 * be NULL.  Returns RH_ENOCONV or RH_ESINGULAR on failure. */
rh_status rh_solve_powerflow(rh_network *net, double tol, int32_t max_iter, int32_t *iters,
                             double *resid_inf);
/* As rh_solve_powerflow, with Newton on the device (Sec. 3.2) and the
 * numeric LU factorisation of G_x repeated on the device on the fixed pattern
 * and ordering analysed at rh_network_create (Sec. 5.2): per step the GPU
 * evaluates the mismatch and G_x on its pattern, refactorises and solves for
 * the step, and the host reads back only max |g|.  At convergence the state
 * and the factors are copied to the host, which forms the adjoint and the
 * branch coefficients from them without factorising, and the product path is
 * uploaded as after rh_solve_powerflow.  Needs a device context; rows of the
 * LU pattern wider than about 1,200 entries give RH_EINVAL.  Same statuses
 * as rh_solve_powerflow. */
rh_status rh_solve_powerflow_device(rh_network *net, double tol, int32_t max_iter, int32_t *iters,
                                    double *resid_inf);
/* Values of the LU factors of the solved operating point, P G_x P^T = L U
 * (Sec. 5.2), in the fixed pattern's row order: l receives nnz_l values (row
 * by row, the strictly lower entries in ascending column order), u nnz_u
 * values (row by row, diagonal first).  Either may be NULL. */
rh_status rh_get_factors(const rh_network *net, double *l, double *u);
/* Converged state x (n_x), objective F(p) = f(x(p), p), reduced gradient (n_p). */
rh_status rh_get_state(const rh_network *net, double *x);
rh_status rh_objective(const rh_network *net, double *F);
/* 1-norm condition estimate of G_x at the solved operating point,
 * ||G_x||_1 times an estimate of ||G_x^{-1}||_1 from a few solves with the
 * factors (Hager's method with Higham's refinements, the estimator of
 * LAPACK's xLACON): a lower bound, usually exact or within a small factor.
 * The pivots are static (diagonal), so a large value warns of an operating
 * point near the loading limit, where the factors lose accuracy.  Host-side,
 * synchronous. */
rh_status rh_condition_estimate(const rh_network *net, double *cond1);
rh_status rh_reduced_gradient(rh_network *net, double *grad);

/* k reduced-Hessian-vector products HW = (d2 F) W, host buffers (Algorithm 2:
 * SpMul, batched sparse solve, batched tensor projection, transposed batched
 * solve, SpMulAdd).  Synchronous. */
rh_status rh_hvp(rh_network *net, int32_t k, const double *W, int64_t ldw, double *HW,
                 int64_t ldhw, rh_precision prec);
/* As rh_hvp on device buffers (FP64, column-major), enqueued on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  Asynchronous: the buffers must
 * stay valid until the stream reaches this work. */
rh_status rh_hvp_device(rh_network *net, int32_t k, const void *dW, int64_t ldw, void *dHW,
                        int64_t ldhw, rh_precision prec, void *hip_stream);
/* For callers that cannot allocate device memory (work recorded under HIP
 * graph capture, serving loops and harnesses that forbid allocation):
 * rh_hvp_device without any allocation.  Same arguments and products, bitwise
 * equal to rh_hvp_device's.  Launch scratch comes from one fixed device array
 * of RH_NOALLOC_SCRATCH_BYTES per GPU, whose address rh_context_create takes
 * and which the GPU holds until the process ends; when a launch's full
 * scratch would exceed it, fewer workgroups run, each taking several chunks
 * of directions in turn.  No launch timing and no per-column refinement
 * figures are recorded.  RH_EINVAL when one workgroup's scratch alone exceeds
 * the array (with the vector in global memory, about 8 million states in FP64
 * and 6 million in the refined mode); RH_ESTATE if no context was created on
 * the network's device.  Every call on a GPU shares that GPU's array and
 * nothing in it needs to start at zero, but calls that overlap on one GPU
 * (other streams, threads or contexts) race: the caller serialises them. */
#define RH_NOALLOC_SCRATCH_BYTES (128ll << 20)
rh_status rh_hvp_device_noalloc(rh_network *net, int32_t k, const void *dW, int64_t ldw, void *dHW,
                                int64_t ldhw, rh_precision prec, void *hip_stream);
/* Choose the launch shape (rh_tile) of the network's products in precision
 * `prec` and apply it.  Unless flags has RH_TUNE_MEASURE, a shape cached for
 * the same grid topology (which fixes the LU pattern and the sweep
 * schedules), device and precision is taken from the cache file; otherwise
 * every candidate is timed on the device: sweep schedules with merged blocks
 * of at most 16, 32 or 64 rows and with or without wave steps (the
 * network's sweeps are re-planned and uploaded for each, so device data of
 * the network moves and recorded batches of it must be re-created), every
 * directions-per-workgroup count whose vectors fit, and launch sizes of 128,
 * 256, 512 and 1,024 directions (and n_p when smaller); one launch of
 * identity columns is timed per candidate (the best of two after one
 * untimed) and the full Hessian estimated as that time x the launches it
 * needs.  The fastest shape is applied, reported in rh_report.tile, and
 * (unless RH_TUNE_NO_CACHE) appended to the cache file: $RH_TUNE_CACHE, else
 * $HOME/.cache/librh/tiles.txt (a text file, one shape per line).  `out` may
 * be NULL.  The network must be solved; synchronises the device. */
#define RH_TUNE_MEASURE 1
#define RH_TUNE_NO_CACHE 2
rh_status rh_autotune(rh_network *net, rh_precision prec, int32_t flags, rh_tile *out);
/* The network's current shape in precision prec (k = 0: none chosen). */
rh_status rh_get_tile(const rh_network *net, rh_precision prec, rh_tile *out);

/* The dense reduced Hessian H (n_p x n_p, column-major, ldh >= n_p), computed
 * in ceil(n_p / k_block) blocks of identity columns (Sec. 5.3), consecutive
 * blocks sharing a launch when one block would leave CUs idle;
 * k_block = 0 lets the library choose: the network's tuned shape
 * (rh_autotune, run on the first such call, from the cache when it holds
 * one), whose k is then the number of directions per launch;
 * rh_report.last_k gives the size used.  Host output, synchronous. */
rh_status rh_reduced_hessian(rh_network *net, double *H, int64_t ldh, int32_t k_block,
                             rh_precision prec);
/* As rh_reduced_hessian into a device buffer, enqueued on `hip_stream` (the
 * first call with k_block = 0 synchronises the stream while it tunes). */
rh_status rh_reduced_hessian_device(rh_network *net, void *dH, int64_t ldh, int32_t k_block,
                                    rh_precision prec, void *hip_stream);

/* Batched instances (several networks, or operating points of one grid, in
 * one kernel launch; the direction blocks of Algorithm 2 are independent
 * across instances as they are across directions).  Item i: network nets[i]
 * (solved, created on ctx), k[i] directions in device buffers dW[i] /
 * dHW[i] (FP64, column-major, leading dimensions ldw[i], ldhw[i] >= its n_p).
 * identity_from may be NULL; where identity_from[i] >= 0, item i's directions
 * are the identity columns identity_from[i] .. + k[i] - 1 (dW[i] is not read;
 * a block of the full reduced Hessian).  Enqueued on hip_stream.  The context
 * keeps launch resources per stream: batched calls on different streams may
 * run concurrently (call from one host thread at a time). */
rh_status rh_hvp_batch_device(rh_context *ctx, int32_t n, rh_network *const *nets,
                              const int32_t *k, const void *const *dW, const int64_t *ldw,
                              void *const *dHW, const int64_t *ldhw,
                              const int32_t *identity_from, rh_precision prec,
                              void *hip_stream);

/* A batched launch recorded once and replayed (Sec. 4.3: the direction
 * blocks of Algorithm 2 are independent, across instances as across
 * directions; Sec. 6: many operating points of one grid).  rh_batch_create
 * takes the arguments of rh_hvp_batch_device, uploads the work list,
 * allocates the launch scratch and records the single batched kernel launch
 * as a HIP graph; rh_batch_launch replays it on hip_stream (one graph launch,
 * no host-side work list and no allocation).  The device buffers dW/dHW are
 * bound at creation: every replay reads their current contents and overwrites
 * the products.  A network re-solved or given new loads or parameters since
 * creation makes rh_batch_launch return RH_ESTATE (its device data moved);
 * create a new batch then.  No per-column refinement figures are recorded.
 * rh_batch_info gives the launch shape (directions per workgroup,
 * workgroups, directions).  rh_batch_destroy waits for the device. */
typedef struct rh_batch rh_batch; /* opaque, library-owned */
rh_status rh_batch_create(rh_context *ctx, int32_t n, rh_network *const *nets, const int32_t *k,
                          const void *const *dW, const int64_t *ldw, void *const *dHW, const int64_t *ldhw,
                          const int32_t *identity_from, rh_precision prec, rh_batch **out);
rh_status rh_batch_launch(rh_batch *b, void *hip_stream);
rh_status rh_batch_info(const rh_batch *b, int32_t *dirs_per_group, int32_t *workgroups, int32_t *directions);
rh_status rh_batch_destroy(rh_batch *b);

/* Per-column figures of the last RH_FP32_REFINED call of rh_hvp,
 * rh_hvp_device, rh_reduced_hessian or rh_reduced_hessian_device on the
 * network (batched calls record none).  For columns j < n (n at most that
 * call's column count, n_p for a full Hessian): the backward error of each
 * solve after its last correction, ||r||_inf / (||A||_inf ||x||_inf) with the
 * residual in FP64 (A = G_x for the state tangent z, G_x^T for the
 * second-order adjoint psi), and the corrections each solve took.  Any output
 * may be NULL.  Waits for the device.  RH_ESTATE before any refined call. */
rh_status rh_refinement_report(const rh_network *net, int32_t n, double *berr_z, int32_t *steps_z,
                               double *berr_psi, int32_t *steps_psi);

/* Device memory of a network, for admission control by callers that keep
 * several networks resident: `resident` = bytes the network holds now (LU
 * factors and sweep schedules in both precisions, branch coefficients, G_p,
 * G_x, descriptors, and its own launch scratch), `scratch_per_direction` =
 * launch scratch one direction of this network may take in precision `prec`
 * (a launch holds it for each direction it runs at once, up to the
 * workgroups it keeps resident).  Either output may be NULL. */
rh_status rh_network_device_bytes(const rh_network *net, rh_precision prec, int64_t *resident,
                                  int64_t *scratch_per_direction);

/* ---- Real-time tracking (Sec. 6.3) ---------------------------------------
 *
 * Reduced gradient grad F = grad_p f + G_p^T lambda (eq. (reduced_gradient))
 * of the solved operating point into the device buffer dgrad (n_p doubles),
 * enqueued on hip_stream.  lambda and grad_p f are resident since the solve.
 * RH_ESTATE if the network is not solved. */
rh_status rh_reduced_gradient_device(rh_network *net, void *dgrad, void *hip_stream);

/* Dense symmetric positive definite solve on the device, FP64: A = L L^T from
 * the lower triangle of the column-major n x n matrix dA (leading dimension
 * lda >= n; the strict upper triangle is neither read nor written), the lower
 * triangle then holding L; then L L^T X = B for the nrhs columns of dB
 * (ldb >= n), overwritten by X.  This is the dense system of eq. (qp_rto),
 * factorised by Cholesky as in Sec. 6.3; the trailing updates run on FP64
 * matrix cores.  Enqueued on hip_stream, then the stream is synchronised.  A
 * leading minor that is not positive definite gives RH_ESINGULAR with
 * *failed_col (may be NULL) = its last column (0-based; -1 on success); dA
 * and dB are then undefined.  The caller owns both buffers. */
rh_status rh_cholesky_solve_device(rh_context *ctx, int32_t n, void *dA, int64_t lda, void *dB, int64_t ldb,
                                   int32_t nrhs, void *hip_stream, int32_t *failed_col);

typedef struct {
  double tau;          /* shift on the diagonal of H_t: 0 is the step of eq. (qp_rto) */
  int32_t tries;       /* Cholesky factorisations attempted */
  int32_t pad;
  double grad_inf;     /* ||g_t||_inf */
  double step_inf;     /* ||d_t||_inf before the projection */
  double ms_gradient;  /* device time of g_t */
  double ms_hessian;   /* device time of H_t (Algorithm 2 over the identity) */
  double ms_solve;     /* device time of the factorisations and the two solves */
} rh_tracking_info;

/* One update of the real-time tracking algorithm (Sec. 6.3) on a network
 * solved at the current loads w_t and control p_t.  Step 1: g_t and H_t into
 * device workspace owned by the network (H_t in blocks of k_block directions,
 * 0 = the tuned launch size, FP64).  Step 2: (H_t + tau I) d_t = -g_t by the
 * dense Cholesky factorisation on the device, tau = shift (>= 0; 0 is the
 * paper's step) when that factorisation succeeds, else the first success of
 * tau_0 = -min_i H_ii + beta, tau <- max(2 tau, beta), beta = 1e-3 max_i |H_ii|
 * (Cholesky with an added multiple of the identity, Nocedal and Wright,
 * Numerical Optimization, Algorithm 3.3).  Then the network's parameters
 * become p_t + d_t clipped to |p_{t+1} - p_t| <= ramp, then to lo <= p <= hi
 * (each an n_p array or NULL), the next power-flow solve starts from the
 * current state, and the network is no longer solved (set the next loads and
 * solve again).  dd (device, n_p doubles, may be NULL) receives d_t on
 * hip_stream.  Synchronises the stream (the shift and d_t are read back);
 * info (may be NULL) receives the figures.  RH_ESTATE if not solved,
 * RH_ESINGULAR if no shift succeeds, RH_ENOCONV on non-finite values. */
rh_status rh_tracking_step_device(rh_network *net, int32_t k_block, double shift, const double *lo, const double *hi,
                                  const double *ramp, void *dd, void *hip_stream, rh_tracking_info *info);

/* Figures of the network; waits for the timed launches since the previous
 * report, sums their durations, then starts a new timing window. */
rh_status rh_last_report(const rh_network *net, rh_report *out);
/* Launch figures of the batched calls on ctx since the previous call (only
 * the launch, timing and phase fields are filled). */
rh_status rh_context_report(rh_context *ctx, rh_report *out);
const char *rh_status_string(rh_status s);
const char *rh_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RH_H */
