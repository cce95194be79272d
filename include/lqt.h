/*
 * lqt.h - C ABI of the MI355X (gfx950) parallel-in-time solver for the continuous-time linear
 * quadratic tracker (LQT) of Sarkka & Garcia-Fernandez, "Temporal parallelisation of the HJB
 * equation and continuous-time linear quadratic control".
 *
 * The solver works in three stages, each one entry point:
 *   lqt_build_elements  per-block conditional value function parameters (A, b, C, eta, J) by RK4
 *                       integration of the backward conditional LQT ODEs (Theorem 8, Sec. IV-B);
 *                       every block is independent.
 *   lqt_scan_value      the value function V(., t_k) = a_k (x) ... (x) a_T (Theorem 6, Sec. III-D)
 *                       with the LQT combination rule (Lemma 7, Sec. IV-A) and the terminal
 *                       element (Sec. IV-D); outputs S_k = J, v_k = eta at every block boundary.
 *   lqt_forward_traj    the optimal trajectory by composing the per-block closed-loop maps
 *                       x_{k+1} = Psi_k x_k + alpha_k (Method 1, Sec. IV-E; the per-block map is
 *                       the Method 2 formula applied to one block) and the control law of Sec.
 *                       II-B, u_k = -R^{-1} L(t_k)^T (S_k x_k - v_k).
 * plus lqt_solve (the three stages in one call) and lqt_backward (the adjoint:
 * gradients of a loss on the trajectory with respect to Q, R, r, x0, Qf and rf).
 *
 * Problem (Sec. II-B with H = I, so Q = H^T X H and the reference r is in state space):
 *     dx/dt = F(t) x + L(t) u + c(t),
 *     cost  = 1/2 (x(t_T) - rf)^T Qf (x(t_T) - rf) + int 1/2 (x-r)^T Q (x-r) + 1/2 u^T R u dt.
 * The horizon is split into T blocks [t_k, t_{k+1}], each integrated with n_steps classical RK4
 * steps of h_k = (t_{k+1} - t_k) / n_steps.  Time-varying inputs are sampled on the half-step grid:
 * sample j of block k is at t_k + j h_k / 2 (j = 0..2 n_steps) and has global index
 * 2 n_steps k + j, so there are NS = 2 n_steps T + 1 samples (block ends shared).
 *
 * Conventions for every entry point:
 *  - All array pointers are DEVICE pointers owned by the caller; the library never allocates,
 *    frees or retains user memory.  Scratch memory is a caller buffer of at least
 *    lqt_workspace_size() bytes, 256-byte aligned.
 *  - Arrays are dense, row-major, all of the dtype named in lqt_dims (double or float), and hold
 *    `batch` independent problems back to back (leading batch dimension), except F and L when
 *    they are constant, which are shared by the whole batch.
 *  - Calls are stream-ordered and non-blocking: they enqueue kernels on `stream` and return.
 *  - Arguments are validated on the host before anything is launched; on error nothing is
 *    launched and the status names the problem (lqt_last_error() gives a message).  Faults of the
 *    device itself surface at the caller's next synchronisation as HIP errors.
 *  - Q, R, Qf must be symmetric; R must be positive definite (its Cholesky factor is taken; a
 *    non-positive-definite R yields NaN outputs, not an error code).
 *  - Finite check: with the environment variable LQT_CHECK_FINITE set to a value other than "0",
 *    every single-problem entry point (lqt_build_elements*, lqt_scan_value, lqt_forward_traj*,
 *    lqt_dense_output, lqt_solve, lqt_backward) scans its outputs for NaN and Inf on `stream`
 *    after its kernels, waits for the stream, and returns LQT_ENONFINITE if any is found (the
 *    outputs are still written).  The (I + C J) systems of the combination rule are
 *    non-singular for symmetric positive semidefinite C, J (Lemma 10), so a breakdown of the
 *    pivoted elimination needs invalid inputs (e.g. an indefinite Q) and shows up as non-finite
 *    outputs, which this check reports.  The check costs one synchronisation per call; the
 *    batched calls and plans do not run it.  Unset, nothing is scanned and calls stay
 *    asynchronous.  The check uses a 256-byte slot of the workspace (included in
 *    lqt_workspace_size).
 *  - Supported sizes: 1 <= nu <= nx <= 16; T >= 1; 1 <= n_steps <= 4096; batch >= 1.
 */
#ifndef LQT_H
#define LQT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lqt_status {
  LQT_OK = 0,
  LQT_EINVAL = -1,       /* an argument is invalid (null pointer, size out of range, ...)        */
  LQT_EUNSUPPORTED = -2, /* a valid request outside what this library implements                 */
  LQT_EWORKSPACE = -3,   /* workspace pointer missing, misaligned or smaller than required       */
  LQT_EHIP = -4,         /* a HIP runtime call (kernel launch) failed                            */
  LQT_ENONFINITE = -5    /* an output holds NaN or Inf (only with LQT_CHECK_FINITE set, below)   */
} lqt_status;

typedef enum lqt_dtype { LQT_F64 = 0, LQT_F32 = 1 } lqt_dtype;

/* Which entry point a workspace is sized for. */
typedef enum lqt_call {
  LQT_CALL_BUILD = 0,
  LQT_CALL_SCAN_VALUE = 1,
  LQT_CALL_FORWARD_TRAJ = 2,
  LQT_CALL_SOLVE = 3,
  LQT_CALL_BACKWARD = 4,
  LQT_CALL_TRAJ_METHOD2 = 5
} lqt_call;

typedef struct lqt_dims {
  int32_t nx;        /* state dimension                                                         */
  int32_t nu;        /* control dimension                                                       */
  int32_t T;         /* number of blocks (sub-intervals)                                        */
  int32_t n_steps;   /* RK4 steps per block                                                     */
  int32_t batch;     /* independent problems of identical sizes in one call                     */
  int32_t dtype;     /* lqt_dtype                                                               */
  int32_t F_sampled; /* 0: F constant [nx*nx] shared by the batch; 1: F [batch][NS][nx*nx]      */
  int32_t L_sampled; /* 0: L constant [nx*nu] shared by the batch; 1: L [batch][NS][nx*nu]      */
  int32_t has_c;     /* 0: c = 0 (c may be NULL); 1: c [batch][NS][nx]                          */
  int32_t lti;       /* 1: the caller asserts a time-invariant problem on a uniform grid (F, L
                        constant, c = 0, t_k = t_0 + k (t_1 - t_0) for every problem).  The ODEs
                        of A, C, J (Theorem 8) then do not involve r and are the same for every
                        block, and b, eta are linear in the block's 2 n_steps + 1 reference
                        samples: the build integrates one block per problem with unit-impulse
                        references to tabulate those linear maps, and forms each block's b, eta
                        as weighted sums of its samples (same results as the general build up to
                        rounding).  Requires F_sampled = L_sampled = has_c = 0 (LQT_EINVAL
                        otherwise); used by lqt_build_elements and lqt_solve (every nx; the
                        batched solve uses the general build).  0: general path.                */
} lqt_dims;

typedef struct lqt_problem {
  const void *t;  /* [batch][T+1] block boundaries, strictly increasing                          */
  const void *F;  /* see lqt_dims.F_sampled                                                      */
  const void *L;  /* see lqt_dims.L_sampled                                                      */
  const void *c;  /* see lqt_dims.has_c                                                          */
  const void *Q;  /* [batch][nx*nx] running state weight, symmetric positive semi-definite      */
  const void *R;  /* [batch][nu*nu] control weight, symmetric positive definite                  */
  const void *r;  /* [batch][NS][nx] reference on the half-step grid                             */
  const void *Qf; /* [batch][nx*nx] terminal weight, symmetric positive semi-definite           */
  const void *rf; /* [batch][nx] terminal reference                                              */
  const void *x0; /* [batch][nx] initial state                                                   */
} lqt_problem;

/* Number of values per element: NE = 2 nx^2 + 3 nx.  Element storage is a tiled structure of
 * arrays, elts[batch][ceil(T/512)][NE][512]: value q of block k of problem p is
 *     elts[((p * ceil(T/512) + k / 512) * NE + q) * 512 + 64 * (k % 8) + (k % 512) / 8]
 * (512 consecutive blocks share a tile; when lane l of a wavefront handles blocks 8 l .. 8 l + 7
 * of a tile, "block j of every lane" is one contiguous 64-value row; the last tile is padded).
 * Values q:
 *   [0, nx^2)                A - I, row-major (the deviation from the identity is stored so that
 *                            short blocks keep full relative precision in FP32)
 *   [nx^2, nx^2+nx)          b
 *   next nx(nx+1)/2          C, upper triangle, row by row ((0,0),(0,1),..,(0,nx-1),(1,1),..)
 *   next nx                  eta
 *   next nx(nx+1)/2          J, upper triangle, row by row                                   */
size_t lqt_element_count(int32_t nx);

/* Bytes of scratch memory entry point `call` needs for these dims (0 if dims are invalid). */
size_t lqt_workspace_size(const lqt_dims *dims, lqt_call call);

/* Elements a_0..a_{T-1} (Theorem 8, Sec. IV-B): for each block independently, integrate
 * dA/ds = A G J - A F, db/ds = -A G eta - A c, dC/ds = -A G A^T,
 * deta/ds = -Q r - F^T eta + J c + J G eta, dJ/ds = -Q - J F - F^T J + J G J  (G = L R^{-1} L^T)
 * in s from s = t_{k+1}, where (A, b, C, eta, J) = (I, 0, 0, 0, 0), down to s = t_k with n_steps
 * classical RK4 steps.  elts: [batch][ceil(T/512)][NE][512] output (layout above).  ws:
 * LQT_CALL_BUILD bytes. */
lqt_status lqt_build_elements(const lqt_dims *dims, const lqt_problem *prob, void *elts, void *ws,
                              size_t ws_bytes, hipStream_t stream);

/* The same elements from the forward conditional ODEs (Theorem 9, Sec. IV-C), integrated in the
 * upper limit tau from tau = t_k, where (A, b, C, eta, J) = (I, 0, 0, 0, 0), up to t_{k+1} with
 * n_steps classical RK4 steps of +h_k:
 * dA/dtau = (F - C Q) A, db/dtau = (F - C Q) b + C Q r + c, dC/dtau = G + F C + C F^T - C Q C,
 * deta/dtau = A^T Q (r - b), dJ/dtau = A^T Q A.  Samples of step m: 2 n_steps k + 2m (stage 1),
 * + 1 (stages 2, 3), + 2 (stage 4).  Both theorems describe the same conditional value function,
 * so the two builds agree to the order of RK4 (O(h^4) per block), not to rounding.  Same
 * arguments and layout as lqt_build_elements (workspace LQT_CALL_BUILD; lqt_dims.lti ignored);
 * 1 <= nx <= 16 (per-lane kernels up to nx = 4, one wavefront per block above); a plain batch
 * (no ragged members). */
lqt_status lqt_build_elements_forward(const lqt_dims *dims, const lqt_problem *prob, void *elts,
                                      void *ws, size_t ws_bytes, hipStream_t stream);

/* The same elements with every block split in two (Sec. IV-D): with m = floor(n_steps / 2), the
 * forward ODEs of Theorem 9 over the first m RK4 steps give V(., t_k; ., tau), tau = t_k + m h_k
 * (the steps of lqt_build_elements_forward), the backward ODEs of Theorem 8 over the last
 * n_steps - m steps give V(., tau; ., t_{k+1}) (the steps of lqt_build_elements), and Lemma 7
 * joins them.  For nx <= 4 the two parts of a block are integrated at the same time by two
 * wavefronts, so the span of the build is about halved (useful when T is small); for nx 5 .. 16
 * one wavefront per block integrates them one after the other.  Agrees with lqt_build_elements
 * to the order of RK4; equal up to rounding for n_steps = 1.  Same arguments and layout as
 * lqt_build_elements (workspace LQT_CALL_BUILD; lqt_dims.lti ignored); 1 <= nx <= 16. */
lqt_status lqt_build_elements_split(const lqt_dims *dims, const lqt_problem *prob, void *elts,
                                    void *ws, size_t ws_bytes, hipStream_t stream);

/* Value functions (Theorem 6 with the terminal element A = b = C = 0, eta = Qf rf, J = Qf):
 * S [batch][T+1][nx*nx] (full symmetric) and v [batch][T+1][nx], V(x, t_k) = 1/2 x^T S_k x -
 * v_k^T x + const.  elts: as written by lqt_build_elements (any producer of the same layout). */
lqt_status lqt_scan_value(const lqt_dims *dims, const void *elts, const void *Qf, const void *rf,
                          void *S, void *v, void *ws, size_t ws_bytes, hipStream_t stream);

/* Trajectory and control at the block boundaries: x [batch][T+1][nx], u [batch][T+1][nu], with
 * x_{k+1} = (I + C_k S_{k+1})^{-1} (A_k x_k + b_k + C_k v_{k+1}) composed by a parallel scan
 * from x_0 = x0, and u_k = -R^{-1} L(t_k)^T (S_k x_k - v_k).  Reads prob->{L, R, x0} (L at sample
 * 2 n_steps k if sampled), elts, S, v.  u may be NULL. */
lqt_status lqt_forward_traj(const lqt_dims *dims, const lqt_problem *prob, const void *elts,
                            const void *S, const void *v, void *x, void *u, void *ws,
                            size_t ws_bytes, hipStream_t stream);

/* The same trajectory by Method 2 (Sec. IV-E): x_k minimises V(x0, t_0; x, t_k) + V(x, t_k), with the
 * conditional value function on [t_0, t_k] the prefix a_0 (x) ... (x) a_{k-1} (Lemma 7) and
 * V(., t_k) from S_k, v_k:  x_k = (I + C S_k)^{-1} (A x0 + b + C v_k) for the prefix's A, b, C,
 * computed by a forward parallel scan; u_k as in lqt_forward_traj.  Agrees with lqt_forward_traj
 * up to rounding.  Same arguments (workspace LQT_CALL_TRAJ_METHOD2); 1 <= nx <= 16 (per-lane
 * trees up to nx = 4, one wavefront per tree node above); a plain batch. */
lqt_status lqt_forward_traj_method2(const lqt_dims *dims, const lqt_problem *prob,
                                    const void *elts, const void *S, const void *v, void *x,
                                    void *u, void *ws, size_t ws_bytes, hipStream_t stream);

/* Values inside the blocks (Sec. VI-A): S, v, x, u at the n T + 1 nodes t_k + m h_k (block k,
 * 0 <= m < n_steps, node index n_steps k + m) and t_T (node n_steps T), from the block-boundary
 * solution S, v, x (as written by lqt_scan_value and lqt_forward_traj, [batch][T+1][...]).  Node
 * n_steps k takes S_k, v_k, x_k unchanged.  Inside block k, S and v come from classical RK4 on
 * dS/dt = -F^T S - S F - Q + S G S and dv/dt = -Q r - F^T v + S G v + S c (Sec. II-B), n_steps - 1
 * steps of -h_k from S_{k+1}, v_{k+1} (step mp: samples 2 n_steps k + 2(n_steps - mp) for stage
 * 1, - 1 for stages 2 and 3, - 2 for stage 4); x from the forward parts A, b, C of Theorem 9 on
 * [t_k, t_k + m h_k] (the RK4 steps of lqt_build_elements_forward) by the Method 2 formula
 * x = (I + C S)^{-1} (A x_k + b + C v) (Sec. IV-E); u = -R^{-1} L^T (S x - v) with L at sample 2 x
 * node.  Outputs (device, caller-allocated): Sd [batch][n T + 1][nx*nx] (full symmetric),
 * vd and xd [batch][n T + 1][nx], ud [batch][n T + 1][nu] (may be NULL).  Reads prob->{t, F, L,
 * c, Q, R, r}.  ws: LQT_CALL_BUILD bytes.  1 <= nx <= 16 (one lane per block up to nx = 4, one
 * wavefront per block above); a plain batch. */
lqt_status lqt_dense_output(const lqt_dims *dims, const lqt_problem *prob, const void *S,
                            const void *v, const void *x, void *Sd, void *vd, void *xd, void *ud,
                            void *ws, size_t ws_bytes, hipStream_t stream);

/* All three stages in one call (prep, element build, value scan, trajectory scan; the same
 * kernels and results as the stage calls).  elts may be NULL (then the elements live in the
 * workspace); S, v, x must be non-NULL; u may be NULL. */
lqt_status lqt_solve(const lqt_dims *dims, const lqt_problem *prob, void *elts, void *S, void *v,
                     void *x, void *u, void *ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): lqt_solve with its scratch memory in a fixed device array of the
 * library instead of a workspace argument.  The array holds LQT_NOALLOC_SCRATCH_BYTES bytes on
 * every device the library runs on, from the first call on that device until the process ends;
 * a problem whose scratch need (lqt_noalloc_scratch_size) exceeds it returns LQT_EWORKSPACE
 * before anything is launched.  Unlike lqt_solve, elts is required (the caller's output buffer,
 * layout above), so only per-problem constants and the scan records live in the scratch array
 * (about 2 MB for the 2^20-block point mass).  The call allocates and frees nothing.  All calls
 * on one device share its array, and each clears what must start at zero: calls that overlap on
 * one device (concurrent streams or threads) race and must not be issued.  `stream` must belong
 * to the current device.  Other arguments and errors as lqt_solve. */
#define LQT_NOALLOC_SCRATCH_BYTES (64u << 20)
size_t lqt_noalloc_scratch_size(const lqt_dims *dims);
lqt_status lqt_solve_noalloc(const lqt_dims *dims, const lqt_problem *prob, void *elts, void *S,
                             void *v, void *x, void *u, hipStream_t stream);

/* Adjoint of lqt_solve for a loss whose gradient with respect to the trajectory is dLdx
 * [batch][T+1][nx] (the exact adjoint of the discrete scheme, not of the continuous problem).
 * Overwrites (accumulates nothing):
 *   dQ [batch][nx*nx], dR [batch][nu*nu], dr [batch][NS][nx], dx0 [batch][nx],
 *   dQf [batch][nx*nx], drf [batch][nx]   (dQf, drf may be NULL).
 * dQ, dR, dQf are symmetric gradients: dL = <dQ, E> for every symmetric perturbation E of Q.
 * S, v, x are the outputs of lqt_solve for the same problem; the elements are rebuilt in the
 * workspace, not read.  Structure: a reverse affine scan for the state adjoint
 * lambda_k = dLdx_k + Psi_k^T lambda_{k+1}, a forward scan for the value adjoints (the linear
 * parts compose like the trajectory maps), per-block gradients of the combination rule
 * (Lemma 7) and the discrete adjoint of each block's RK4 steps.  FP64 or FP32, nx <= 4
 * (LQT_EUNSUPPORTED otherwise); F and L constant or sampled, with or without a drift c (F, L, c
 * are not differentiated; with sampled L, R enters through G(t) = L(t) R^{-1} L(t)^T at every
 * sample, and the workspace holds G at every sample). */
lqt_status lqt_backward(const lqt_dims *dims, const lqt_problem *prob, const void *S,
                        const void *v, const void *x, const void *dLdx, void *dQ, void *dR,
                        void *dr, void *dx0, void *dQf, void *drf, void *ws, size_t ws_bytes,
                        hipStream_t stream);

/* ---------------------------------------------------------------------------------------------
 * Batched solve: many problems with uneven horizons and several sizes in one call.
 *
 * Problems are grouped in classes that share nx, nu, n_steps, dtype and the sampling flags; a
 * call takes several classes.  Inside a class, problem i has T_i >= 1 blocks and the arrays of
 * all its problems are concatenated ("rows" = sum_i (T_i + 1)):
 *   start  [count + 1] DEVICE int64: start[0] = 0, start[i + 1] = start[i] + T_i + 1,
 *          start[count] = rows.  Row start[i] + k (k = 0..T_i) of t, S, v, x, u is boundary k
 *          of problem i.  The kernels trust these values (they only clamp problem indices).
 *   t      [rows]  block boundaries, strictly increasing within each problem
 *   r      the NS_i = 2 n_steps T_i + 1 half-step samples of each problem back to back:
 *          [2 n_steps (rows - count) + count][nx]; F, L, c when sampled likewise
 *   F, L   when constant: one per problem, [count][nx*nx] and [count][nx*nu]
 *   Q, R, Qf, rf, x0  [count][...] one per problem
 *   S [rows][nx*nx], v [rows][nx], x [rows][nx], u [rows][nu] (u may be NULL)
 * Results equal those of lqt_solve on each problem alone up to rounding.  Method: the problems
 * of a class form one horizon in which every problem is followed by a separator element
 * (A = 0, b = x0 of the next problem, C = 0, eta = Qf rf, J = Qf).  Folded into a value
 * function (Theorem 6, Lemma 7) the separator returns the problem's terminal value (Sec. IV-D)
 * whatever follows it, and its closed-loop map (Sec. IV-E) sends any state to the next x0, so
 * one scan of each kind solves every problem of the class.  Launches per class: problem
 * constants, elements, clearing of status words, and one launch for both scans, whose waves take
 * tiles (nx <= 4: value tiles in the value scan's order, then trajectory tiles) or tree nodes
 * (nx >= 5: every level of both trees, in dependency order) from a work queue; a wave only waits
 * for work taken before its own, so every wait ends.  The number of launches does not depend on
 * the number of problems.
 * ------------------------------------------------------------------------------------------- */
typedef struct lqt_ragged {
  int32_t nx, nu, n_steps, dtype; /* as in lqt_dims                                             */
  int32_t count;                  /* problems in the class (>= 1)                                */
  int32_t F_sampled, L_sampled, has_c;
  int64_t rows;                   /* sum over problems of (T_i + 1); at most 2^31 - 1            */
  const int64_t *start;           /* DEVICE [count + 1]                                          */
  lqt_problem prob;               /* concatenated problem arrays (above)                         */
  void *S, *v, *x, *u;            /* outputs (above); u may be NULL                              */
} lqt_ragged;

/* Bytes of workspace for lqt_solve_batched / lqt_plan_create on these classes (0 if invalid). */
size_t lqt_batched_workspace_size(const lqt_ragged *classes, int32_t nclasses);

/* All classes solved eagerly on `stream`, one after another, with the default configuration. */
lqt_status lqt_solve_batched(const lqt_ragged *classes, int32_t nclasses, void *ws,
                             size_t ws_bytes, hipStream_t stream);

/* A plan: the batched solve of fixed classes and buffers with a configuration fixed at creation,
 * replayed by lqt_plan_launch: every class on its own stream, forked from and joined back into
 * the launch stream (or one after another when tuning prefers that).  The arrays named in
 * `classes` and the workspace are bound to the plan: refill them in place between launches and
 * keep them alive until lqt_plan_destroy; launches of one plan must not overlap.
 * flags & LQT_PLAN_AUTOTUNE: time the candidate configurations (per class: the blocks per lane
 * of the value tiles on the per-lane path, two candidates chosen from the class's rows among 1,
 * 4 and 8; 4, 8 or 16 nodes per wave on the wave path; then concurrent or serial classes) by
 * running them on `stream` (outputs are overwritten)
 * and keep the fastest; choices are cached per class signature for the life of the process
 * (thread-safe).  Without the flag the default configuration is used.  flags & LQT_PLAN_GRAPH:
 * after tuning, the plan's launch sequence is captured once into a HIP graph (on a stream of the
 * plan's own; the tuner never captures) and lqt_plan_launch replays it with one hipGraphLaunch on
 * `stream`.  lqt_plan_create synchronises `stream`; lqt_plan_destroy waits for the plan's last
 * replay before it releases the graph. */
typedef struct lqt_plan_s *lqt_plan;
enum { LQT_PLAN_AUTOTUNE = 1, LQT_PLAN_GRAPH = 2 };
lqt_status lqt_plan_create(const lqt_ragged *classes, int32_t nclasses, void *ws,
                           size_t ws_bytes, int32_t flags, hipStream_t stream, lqt_plan *plan);
lqt_status lqt_plan_launch(lqt_plan plan, hipStream_t stream);
/* Human-readable description of the configuration a plan uses (valid until destroy). */
const char *lqt_plan_config(lqt_plan plan);
void lqt_plan_destroy(lqt_plan plan);

/* ---- Debugging aids (process-wide settings; not for calls that run concurrently) ----
 * lqt_debug_canary(mode): mode 1 places a 256-byte canary after every region of the workspace
 * layout (lqt_workspace_size grows accordingly: query it after changing the mode); every
 * single-problem call then fills the canaries before its first launch and, at its end,
 * synchronises its stream and checks them, returning LQT_EWORKSPACE ("workspace canary i of n
 * overwritten") if a kernel wrote past a region.  Mode 2 does the same and spoils canary 0
 * itself after filling it, so the check must fire (a test of the check).  0 turns it off.
 * Batched calls and lqt_solve_noalloc lay the canaries out but do not check them.  The
 * environment variable LQT_CANARY=1|2 sets the mode when the library loads.
 * lqt_debug_fail_launch(n): the n-th checked HIP call from now on (n >= 1; 0 disables) reports
 * hipErrorLaunchFailure: the call itself is made, and the entry point returns LQT_EHIP with a
 * message naming the simulation, as it would for a real failure (the error paths of callers
 * can be tested without a fault).  LQT_FAIL_LAUNCH=n sets it when the library loads.
 * Also read from the environment: LQT_CHECK_FINITE (above); LQT_AUTOTUNE=off|on|force
 * (lqt_plan_create: off never tunes, on tunes plans created with LQT_PLAN_AUTOTUNE unless the
 * cache holds their classes, force always tunes) and LQT_TUNE_CACHE=<file> (the tuner's choices
 * persist in that file, keyed by GPU architecture and class signature, read when the first plan
 * is created and rewritten after every tuning). */
void lqt_debug_canary(int32_t mode);
void lqt_debug_fail_launch(int32_t n);

/* Short description of a status code. */
const char *lqt_status_string(lqt_status status);

/* Detail message of the last error returned on the calling thread ("" if none). */
const char *lqt_last_error(void);

/* Library version: major * 10000 + minor * 100 + patch. */
int32_t lqt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LQT_H */
