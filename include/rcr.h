/*
 * rcr.h — C-ABI of the rake-compress tree-LQR solver for AMD MI355X (gfx950).
 *
 * The solver computes the unique saddle point of the branched
 * dual-regularised LQR problem of Sec. II-A (Lagrangian eq. (lagrangian),
 * saddle problem eq. (saddle); unique by Prop. 1) on a rooted tree, and the
 * Riccati data of its factorisation: it returns the KKT solution (x, u, y)
 * of eq. (kkt), the subtree Hessians P_i (Thm. 1) and the feedback gains
 * K_e (eq. (factor-local)).  It follows Algorithm 1 (Sec. VI): a reusable
 * topology plan (Sec. VII), local control condensation (eq. (edge-components)),
 * rake/compress contraction and reverse expansion of the conditional
 * quadratics (Sec. IV), local factors (eqs. (FW), (factor-local)), then the
 * affine solve and state recovery (Sec. V).
 *
 * Conventions (all calls):
 *  - Nodes are 0..N-1 in the caller's order; parent[root] = -1, exactly one
 *    root.  The edge e = (parent[j], j) lives in "edge slot j"; the root's
 *    edge slot is ignored on input and written as zero on output.
 *  - Problem and solution arrays are DEVICE pointers to float64, row-major,
 *    one contiguous block per node or edge slot:
 *      per node    Q[N][n][n]  q[N][n]  c[N][n]  Delta[N][n][n]
 *      per edge    R[N][m][m]  S[N][n][m]  r[N][m]  A[N][n][n]  B[N][n][m]
 *      outputs     K[N][m][n] (edge)  P[N][n][n]  x[N][n]  u[N][m] (edge)
 *                  lam[N][n]  (lam = the node multipliers y_i)
 *    S is the cross term M_e of eq. (lagrangian) (x_i^T M_e u_e); c_root is
 *    the root constraint of eq. (kkt-root), c_j the offset of the dynamics
 *    into j (eq. (kkt-dyn)); Delta_i is the dual regulariser of node i.
 *  - The caller owns every problem/solution buffer and the stream; inputs are
 *    never modified.  The library owns the plan, its device copy and (unless
 *    the caller supplies one) a workspace cached in the plan.
 *  - The caller guarantees the standing convexity assumptions of
 *    Definition 1 (R_e > 0, Delta_i >= 0, Q_i - sum_out M R^-1 M^T >= 0); the
 *    solver only reports pivot breakdowns it meets (RCR_SINGULAR, RCR_NOT_PD).
 *  - Return value: 0 on success, a negative RCR_* status otherwise.
 *    rcr_status_string() names it.  Calls are thread-safe.  One plan may
 *    serve concurrent solves on different streams when each passes its own
 *    workspace (the workspace also holds that solve's status words and
 *    residual accumulator); solves that share the plan-owned workspace must
 *    be ordered by the caller.
 */
#ifndef RCR_H
#define RCR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------------- status */
#define RCR_OK 0
#define RCR_INVALID_TREE (-1) /* no root, several roots, a cycle, an index out of range   */
#define RCR_BAD_DIMS (-2)     /* n or m < 1, or above RCR_MAX_DIM, or N < 1               */
#define RCR_NULL_ARG (-3)     /* a required pointer is NULL                                */
#define RCR_NOT_PD (-4)       /* Cholesky of R_e or G_e broke down                         */
#define RCR_SINGULAR (-5)     /* zero pivot in I + C U, S, or F (excluded by Definition 1) */
#define RCR_NONFINITE (-6)    /* a NaN or Inf reached an output                            */
#define RCR_OOM (-7)          /* host or device allocation failed                          */
#define RCR_HIP_ERROR (-8)    /* a HIP runtime call failed                                 */
#define RCR_BAD_OPTION (-9)   /* an option value is out of range                           */
#define RCR_SMALL_WORKSPACE (-10) /* caller workspace smaller than rcr_workspace_size()    */
#define RCR_NO_DEVICE (-11)   /* no usable GPU                                             */

#define RCR_MAX_DIM 16 /* largest n and m the kernels are compiled for */

/* ---------------------------------------------------------------- planning */
typedef struct rcr_plan rcr_plan; /* opaque, immutable after creation */

#define RCR_SELECT_GREEDY_INDEX 0 /* greedy in increasing node id (Sec. VII-A, as the paper) */
#define RCR_SELECT_LIST_RANK 1    /* alternate positions along each maximal unary path       */

typedef struct {
  int32_t selection;     /* RCR_SELECT_*; any maximal non-adjacent set is valid (Lemma 2) */
  int32_t single_thread; /* nonzero: build on the calling thread only (by default trees of
                            16384 nodes or more build their four pass schedules on four
                            threads); for callers that build many plans at once          */
  int32_t reserved[6];   /* zero */
} rcr_plan_options;

typedef struct {
  int64_t N;
  int32_t n, m;
  int64_t root;
  int64_t height;        /* longest root-to-leaf path, edges                             */
  int64_t leaves;
  int64_t max_degree;
  int64_t rounds;        /* structural rounds (Lemma 2: <= ceil(log_{3/2} N))            */
  int64_t levels;        /* nonempty dependency levels of the contraction (Lemma 4)     */
  int64_t expand_levels; /* levels of the reverse (expansion) graph                      */
  int64_t state_levels;  /* levels of the state-map contraction (compressions only)      */
  int64_t sexp_levels;   /* levels of the state expansion                                */
  int64_t n_rake, n_compress, n_combine, n_absorb;
  int64_t depth_bound;   /* D_N of eq. (dependency-level-bound)                          */
  int64_t crew_ok;       /* 1 if every datum has one writer and is read only at a later level */
  int64_t workspace_bytes_fp64;  /* device scratch of one FP64 solve                    */
  int64_t workspace_bytes_mixed; /* device scratch of one MIXED32 solve                 */
  int64_t n_trees;               /* 1, or the number of trees of a batched plan         */
  int64_t plan_device_bytes;     /* bytes of the plan's device copy (made by the first  */
                                 /* solve or rcr_plan_upload), whether made yet or not  */
  int64_t graph_cache_entries;   /* captured launch sequences the plan holds (at most   */
                                 /* RCR_GRAPH_CACHE_CAP of each of its two caches)      */
} rcr_plan_stats;

/* Captured launch sequences (RCR_EXEC_GRAPH) are cached per plan under the
 * buffer addresses they were captured with, at most this many per cache; the
 * least recently used is destroyed, once its own latest replay has completed,
 * to make room. */
#define RCR_GRAPH_CACHE_CAP 8

/* Build the topology plan of Sec. VII from a HOST parent array (int64, N
 * entries).  Host-only work: structural rounds, readiness-weighted sibling
 * reductions (eq. (readiness-code-data)), earliest-start dependency levels
 * (eq. (earliest-level)) and static slot indices.  n, m are the state and
 * control dimensions the plan's workspace is sized for (1..RCR_MAX_DIM).
 * The device copy is made lazily by the first solve.  *out receives the plan;
 * release it with rcr_plan_destroy.  Errors: RCR_NULL_ARG, RCR_BAD_DIMS,
 * RCR_INVALID_TREE, RCR_BAD_OPTION, RCR_OOM. */
int rcr_plan_create(const int64_t *parent, int64_t N, int32_t n, int32_t m,
                    const rcr_plan_options *opt, rcr_plan **out);

/* The same plan built on the GPU (the device-side planner, Sec. VII: the
 * structural rounds with list ranking for the compress selection, the
 * readiness-weighted sibling reductions of Lemma 3, earliest-start levels and
 * static slots, by one workgroup of one CU, so that solves keep the rest of
 * the device) from a DEVICE parent array (int64, N entries, root -1).  The
 * result is byte-identical to rcr_plan_create with RCR_SELECT_LIST_RANK: opt
 * may be NULL (meaning that selection); RCR_SELECT_GREEDY_INDEX, a sequential
 * choice in node-id order, is rejected with RCR_BAD_OPTION.  The planner runs
 * in the order of `stream` (a hipStream_t, NULL the default stream) and the
 * call returns when the plan's schedules are back on the host; its working
 * memory (about 0.65 KB per node) comes from the library's device pool and is
 * released in stream order.  single_thread is ignored.  Errors: RCR_NULL_ARG,
 * RCR_BAD_DIMS, RCR_INVALID_TREE, RCR_BAD_OPTION, RCR_OOM, RCR_NO_DEVICE,
 * RCR_HIP_ERROR. */
int rcr_plan_create_device(const int64_t *parent, int64_t N, int32_t n, int32_t m,
                           const rcr_plan_options *opt, void *stream, rcr_plan **out);

/* 64-bit FNV-1a hash of everything a plan holds (dimensions, statistics and
 * every schedule and offset array, each preceded by its length), for checking
 * that two plans are identical (tests, caches).  Host only.
 * Errors: RCR_NULL_ARG. */
int rcr_plan_digest(const rcr_plan *plan, uint64_t *digest);

/* Summary of a plan (host only).  Errors: RCR_NULL_ARG. */
int rcr_plan_info(const rcr_plan *plan, rcr_plan_stats *out);

/* Bytes of the plan's device copy (as rcr_plan_stats.plan_device_bytes,
 * without the plan's other statistics); 0 for NULL. */
int64_t rcr_plan_device_bytes(const rcr_plan *plan);

/* Copy the plan's primitive operations to HOST arrays, for inspection and
 * tests.  Each op is 8 int32 words:
 *   {kind, round, level, a, b, c, d, e}
 * kind 0 rake     a = node j, b = edge slot into j, c = contribution slot, d = parent
 * kind 1 combine  a, b = input contribution slots (left, right), c = output slot, d = parent
 * kind 2 absorb   a = node i, b = aggregate contribution slot
 * kind 3 compress a = node j, b = edge slot into j, c = edge slot out of j,
 *                 d = new edge slot, e = child node k
 * Ops are sorted by (level, kind).  With ops == NULL only *count is written.
 * Errors: RCR_NULL_ARG, RCR_SMALL_WORKSPACE (capacity < count). */
int rcr_plan_export(const rcr_plan *plan, int32_t *ops, int64_t capacity, int64_t *count);

/* Release a plan.  Its device memory is returned in stream order after the
 * latest rcr_solve that used it has completed; the host is not blocked.  The
 * caller must not destroy a plan while a solve issued before that latest one,
 * on another stream, is still running.  NULL is ignored. */
void rcr_plan_destroy(rcr_plan *plan);

/* Batched plan of k independent trees (their forest), for solving many trees
 * with one merged launch sequence.  The parts must share n and m; they are
 * only read.  Tree t occupies nodes [off_t, off_t + N_t) of the batched
 * problem, in part order (off_0 = 0), and edge slots likewise; per-node and
 * per-edge arrays of rcr_solve are the concatenation of the trees' arrays.
 * Dependency level t of the batch is the union of every tree's level t (the
 * trees share no data, so each datum keeps a unique writer); the launch count
 * is that of the deepest tree, not the sum over trees.  The batched plan is
 * independent of the parts afterwards.  Errors: RCR_NULL_ARG, RCR_BAD_DIMS
 * (different n or m, or too many slots), RCR_OOM. */
int rcr_batch_plan_create(const rcr_plan *const *plans, int32_t k, rcr_plan **out);

/* Make the plan's device copy now (on the current device, in the order of
 * `stream`, a hipStream_t or NULL), instead of at its first rcr_solve; waits
 * for the copy.  A no-op when the copy exists.  Lets a caller move the
 * host-to-device transfer of a fresh plan off its critical path (e.g. into a
 * worker thread).  Errors: RCR_NULL_ARG, RCR_OOM, RCR_HIP_ERROR,
 * RCR_NO_DEVICE. */
int rcr_plan_upload(const rcr_plan *plan, void *stream);

/* ------------------------------------------------------------------ solving */
typedef struct {
  const double *Q, *q, *c, *Delta; /* node data   */
  const double *R, *S, *r, *A, *B; /* edge data   */
} rcr_problem;

typedef struct {
  double *K, *P, *x, *u, *lam;
} rcr_solution;

#define RCR_FP64 0    /* all arithmetic in float64                                        */
#define RCR_MIXED32 1 /* float32 bulk, float64 R/G Cholesky and compress (I + C P) solve, */
                      /* float64 KKT residual and refinement_steps correction solves        */

#define RCR_EXEC_LEVELS 0 /* one launch per dependency level                              */
#define RCR_EXEC_GRAPH 1  /* the same launches captured once into a hipGraph and replayed */

typedef struct {
  int32_t precision;        /* RCR_FP64 (default) or RCR_MIXED32                           */
  int32_t refine_steps;     /* MIXED32: iterative-refinement steps (default 1 when < 0)    */
  int32_t executor;         /* RCR_EXEC_LEVELS or RCR_EXEC_GRAPH                           */
  int32_t check;            /* nonzero: synchronise the stream and report device flags     */
  void *workspace;          /* optional caller device workspace (NULL: plan-owned)         */
  int64_t workspace_bytes;  /* its size                                                    */
  double *kkt_residual;     /* optional HOST out: max-abs KKT residual of eq. (kkt) over   */
                            /* all four blocks (forces a synchronisation)                  */
  float *kernel_ms;         /* optional HOST out[RCR_NUM_KERNEL_CLASSES]: per kernel class, */
                            /* the device time of this call's launches from HIP events on  */
                            /* `stream` (synchronises).  RCR_EXEC_LEVELS: one span per      */
                            /* launch (boundary events shared by consecutive launches);    */
                            /* RCR_EXEC_GRAPH: the graph is captured with event-record     */
                            /* nodes where the kernel class changes, so a span covers a    */
                            /* run of back-to-back launches of one class                   */
  int32_t *kernel_launches; /* optional HOST out[RCR_NUM_KERNEL_CLASSES]: launch counts     */
  int32_t reserved[4];      /* zero */
} rcr_solve_options;

/* Kernel classes reported in rcr_solve_options.kernel_ms */
#define RCR_K_CONDENSE 0
#define RCR_K_QUAD_CONTRACT 1
#define RCR_K_QUAD_EXPAND 2
#define RCR_K_LOCAL_FACTOR 3
#define RCR_K_TCOMPOSE 4
#define RCR_K_RHS_INIT 5
#define RCR_K_AFF_CONTRACT 6
#define RCR_K_AFF_EXPAND 7
#define RCR_K_LOCAL_AFFINE 8
#define RCR_K_STATE_CONTRACT 9
#define RCR_K_STATE_EXPAND 10
#define RCR_K_RECOVER 11
#define RCR_K_RESIDUAL 12
#define RCR_K_QUAD_TAIL 13  /* narrow quadratic levels (contraction end + expansion start) */
#define RCR_K_AFF_TAIL 14   /* narrow affine levels                                         */
#define RCR_K_STATE_TAIL 15 /* narrow state levels                                          */
#define RCR_NUM_KERNEL_CLASSES 16

/* Device scratch one rcr_solve needs for this plan and precision (including
 * a 512-byte header for the solve's status words and residual).  This is the
 * request's HBM footprint beyond its inputs and outputs. */
int64_t rcr_workspace_size(const rcr_plan *plan, int32_t precision);

/* Factor and solve one tree-LQR instance (Algorithm 1, Steps 2-6) on
 * `stream` (a hipStream_t; NULL = the default stream).  Asynchronous and
 * stream-ordered unless options request a synchronisation.  opt may be NULL
 * (FP64, per-level executor, no check).  The first solve of a plan copies its
 * integer arrays to the device in the order of `stream` and waits for that
 * copy, so it must not be issued while `stream` is being captured.  Errors: RCR_NULL_ARG, RCR_BAD_OPTION,
 * RCR_SMALL_WORKSPACE, RCR_OOM, RCR_HIP_ERROR, RCR_NO_DEVICE and, when
 * opt->check is set, RCR_SINGULAR, RCR_NOT_PD, RCR_NONFINITE. */
int rcr_solve(const rcr_plan *plan, const rcr_problem *in, rcr_solution *out,
              const rcr_solve_options *opt, void *stream);

/* ------------------------------------------- factor once, solve many times */
/* The factor of Algorithm 1 (Steps 2-3: condensation, the quadratic
 * contraction and expansion of Sec. IV, the local factors of eqs. (FW),
 * (factor-local)) does not depend on the right-hand side (q, r, c); Steps 4-6
 * (the affine and state passes of Sec. V and the recovery eq. (recover)) are
 * matrix-vector passes on it.  rcr_factor runs Steps 2-3 once; rcr_solve_rhs
 * then solves any number of right-hand sides on the same matrices. */
typedef struct {
  const double *q, *r, *c; /* q[N][n]  r[N][m] (edge slots)  c[N][n]: device, float64 */
} rcr_rhs;

typedef struct {
  double *x, *u, *lam;     /* x[N][n]  u[N][m] (edge slots)  lam[N][n]: device, float64 */
} rcr_rhs_solution;

/* Factor the matrices of `in` (Q, Delta, R, S, A, B; q, r and c are not read)
 * on `stream`.  Writes out->K and out->P (out->x, u, lam are not touched) and
 * keeps the rest of the factor (W, F^-1, G^-1, A^cl and the composite
 * transitions of every compression) in the workspace: opt->workspace when
 * given (at least rcr_workspace_size(plan, precision) bytes), else the
 * plan-owned workspace of opt->precision.  The factor stays valid until the
 * next rcr_factor, rcr_solve or rcr_batch_solve that uses the same workspace.
 * Options as for rcr_solve (opt->kkt_residual is ignored: there is no iterate
 * yet).  Errors: those of rcr_solve. */
int rcr_factor(const rcr_plan *plan, const rcr_problem *in, rcr_solution *out, const rcr_solve_options *opt,
               void *stream);

/* Solve k >= 1 right-hand sides rhs[0..k) on the factor made by rcr_factor
 * (same plan, precision and workspace; factor->K, factor->P are its outputs;
 * rcr_solve leaves no factor for this: in float64 it does not store A^cl;
 * Delta and B of `in` are read, and in MIXED32 also Q, R, S, A for the
 * refinement's residual), writing sol[i] for rhs[i], one after the other on
 * `stream`.  MIXED32 refines each solution with opt->refine_steps correction
 * solves on the float64 KKT residual.  opt->kkt_residual receives the largest
 * residual over the k solutions.  Only the solve passes run: no factor-class
 * kernel is launched.  Errors: those of rcr_solve; RCR_BAD_OPTION when no
 * workspace is given and the plan-owned workspace of this precision holds no
 * factor (no rcr_factor yet, or an rcr_solve since). */
int rcr_solve_rhs(const rcr_plan *plan, const rcr_problem *in, const rcr_solution *factor, int32_t k,
                  const rcr_rhs *rhs, rcr_rhs_solution *sol, const rcr_solve_options *opt, void *stream);

/* Gradients of a scalar loss L(x, u, lam) of the solution with respect to the
 * problem data (sensitivity / reverse-mode differentiation through the solve;
 * the paper checks differentiation through a right-hand side, Sec. IX-A).
 * The KKT matrix of eq. (kkt) is symmetric, so the adjoint system is the same
 * system: with seed = (dL/dx, dL/du, dL/dlam) passed as (q, r, c) of an
 * rcr_rhs, rcr_adjoint solves it on the factor (as rcr_solve_rhs) and writes
 *   grad->q = dL/dq, grad->r = dL/dr, grad->c = dL/dc   (required)
 * and, for each of grad->Q, Delta, R, S, A, B that is not NULL, the gradient
 * with respect to that array (unsymmetrised outer products; the root's edge
 * slot is written as zero).  `fwd` holds the factor's K, P and the forward
 * solution x, u, lam of the same problem.  Arrays have the layouts of
 * rcr_problem.  Errors: those of rcr_solve_rhs. */
typedef struct {
  double *Q, *q, *c, *Delta, *R, *S, *r, *A, *B;
} rcr_gradient;

int rcr_adjoint(const rcr_plan *plan, const rcr_problem *in, const rcr_solution *fwd, const rcr_rhs *seed,
                rcr_gradient *grad, const rcr_solve_options *opt, void *stream);

/* Max-abs residual of eq. (kkt) over all four blocks for the iterate
 * (sol->x, u, lam) of problem `in` (float64, on `stream`; synchronises).  The
 * result goes to *opt->kkt_residual (required); a NaN anywhere in the rows
 * gives +Inf.  opt->workspace, when given, needs 512 bytes.  Errors:
 * RCR_NULL_ARG, RCR_OOM, RCR_HIP_ERROR, RCR_NO_DEVICE. */
int rcr_kkt_residual(const rcr_plan *plan, const rcr_problem *in, const rcr_solution *sol,
                     const rcr_solve_options *opt, void *stream);

/* ------------------------------------------------------- batched solves */
/* Solve k independent trees with one merged launch sequence (the forest plan
 * of rcr_batch_plan_create; Sec. VIII suggests batches of equal-shaped
 * operations).  plans[t] is tree t's plan (all with the same n and m), in[t]
 * and out[t] its own problem and solution buffers, laid out as for rcr_solve
 * with that tree's N.  The merged plan is built on the first call for this
 * sequence of plans (or by rcr_batch_prepare) and cached by the library
 * (least recently used of 32 dropped; entries holding a destroyed plan are
 * dropped with it).  The trees' inputs are gathered into staging arrays of
 * the workspace, solved together, and the outputs scattered back, one launch
 * each; results equal those of solving each tree alone, bit for bit.  A
 * caller workspace needs rcr_batch_workspace_size bytes.  Options and errors
 * as for rcr_solve (opt->kkt_residual: the largest over the trees). */
int rcr_batch_solve(const rcr_plan *const *plans, int32_t k, const rcr_problem *in, rcr_solution *out,
                    const rcr_solve_options *opt, void *stream);

/* Build, cache and upload (in the order of `stream`, waiting for the copy)
 * the merged plan rcr_batch_solve uses for these plans, ahead of the solve.
 * Errors: those of rcr_batch_plan_create and rcr_plan_upload. */
int rcr_batch_prepare(const rcr_plan *const *plans, int32_t k, void *stream);

/* Drop the cached merged plan of these plans, if any (its device copy is
 * released in stream order after its last solve).  For callers whose batches
 * rarely repeat.  NULL or unknown sequences are ignored. */
void rcr_batch_release(const rcr_plan *const *plans, int32_t k);

/* Device bytes one rcr_batch_solve of these plans needs in this precision:
 * the merged plan's solver workspace, the staged inputs and outputs, and the
 * copy table.  Builds and caches the merged plan if needed; 0 on error. */
int64_t rcr_batch_workspace_size(const rcr_plan *const *plans, int32_t k, int32_t precision);

/* ------------------------------------------------ solve without allocating */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rcr_solve
 * with its workspace in a static device array of the library, one per GPU,
 * rcr_noalloc_scratch_bytes() (64 MiB) large and held until the process
 * ends.  The call makes no allocation: the plan must have been prepared by
 * rcr_plan_upload on the current device (else RCR_BAD_OPTION), opt->executor
 * must be RCR_EXEC_LEVELS and opt->workspace, kernel_ms and kernel_launches
 * must be unset (else RCR_BAD_OPTION); a problem whose workspace
 * (rcr_workspace_size) exceeds the array is rejected with
 * RCR_SMALL_WORKSPACE.  All calls on one GPU share its array, which keeps the
 * last call's contents: calls that overlap on one GPU (other streams, other
 * threads) race and must be ordered by the caller.  Results equal those of
 * rcr_solve bit for bit.  Errors: those of rcr_solve. */
int rcr_solve_noalloc(const rcr_plan *plan, const rcr_problem *in, rcr_solution *out, const rcr_solve_options *opt,
                      void *stream);

/* Size in bytes of the per-GPU array of rcr_solve_noalloc. */
int64_t rcr_noalloc_scratch_bytes(void);

/* ------------------------------------------------- node-control problems */
/* Scenario MPC with one control v_i per non-leaf node, shared by all its
 * outgoing transitions x_j = A_j x_i + B_j v_i + c_j (Sec. II-B, eq.
 * (node-control), saddle function eq. (node-lagrangian)).  Device pointers,
 * float64, row-major, one block per node (native tree of N nodes, state n,
 * control m):
 *   per node    Q[N][n][n]  q[N][n]  c[N][n]  Delta[N][n][n]
 *               M[N][n][m]  R[N][m][m]  r[N][m]   (cost of v_i; rows of leaves
 *                                                  are not read)
 *   per edge    A[N][n][n]  B[N][n][m]            (slot j: edge parent[j] -> j;
 *                                                  root slot not read)
 *   outputs     x[N][n]  v[N][m] (zero rows at leaves)  lam[N][n]
 * The solve runs through the exact lifting of Prop. 2: an edge-control tree
 * with a predecision node i^- (id i) for every node and a decision node i^+
 * (id N + rank of i among the non-leaves) for every non-leaf, lifted state
 * (x, v) of dimension n + m, decision edges per eq. (decision-edge) and
 * uncertainty edges per eq. (uncertainty-edge) (dummy control cost I). */
typedef struct {
  const double *Q, *q, *c, *Delta; /* per node                  */
  const double *M, *R, *r;         /* per node (non-leaf rows)  */
  const double *A, *B;             /* per edge slot             */
} rcr_native_problem;

typedef struct {
  double *x, *v, *lam;
} rcr_native_solution;

/* Plan of the lifted tree of the HOST native parent array (N entries) for
 * state n and control m (n + m <= RCR_MAX_DIM).  The plan's rcr_plan_info
 * describes the lifted tree (N + #non-leaves nodes, state n + m); its
 * rcr_workspace_size includes the lifted problem and solution buffers.
 * Errors: RCR_NULL_ARG, RCR_BAD_DIMS, RCR_INVALID_TREE, RCR_BAD_OPTION,
 * RCR_OOM. */
int rcr_lift_plan_create(const int64_t *parent, int64_t N, int32_t n, int32_t m,
                         const rcr_plan_options *opt, rcr_plan **out);

/* Solve a node-control problem with a plan from rcr_lift_plan_create: device
 * kernels write the lifted data (eqs. (decision-edge), (uncertainty-edge)),
 * rcr_solve runs on the lifted tree, and device kernels project the lifted
 * solution back (x_i and lam_i = the first n entries of the lifted state and
 * multiplier of i^-, v_i = the control of i's decision edge).  Options as for
 * rcr_solve; a caller workspace must hold rcr_workspace_size(plan,
 * precision) bytes; opt->kkt_residual reports the residual of the lifted
 * system.  Errors: those of rcr_solve, and RCR_BAD_OPTION when the plan is not
 * a lifted plan. */
int rcr_lift_solve(const rcr_plan *plan, const rcr_native_problem *in, rcr_native_solution *out,
                   const rcr_solve_options *opt, void *stream);

/* ------------------------------------------- non-uniform dimensions */
/* Trees whose node v has its own state dimension n_v and whose edge into v
 * has its own control dimension m_v (uniform dimensions are a convenience of
 * the presentation, Sec. II-A; static-shape backends may pad, Sec. VIII).
 * Blocks are rectangular: for the edge e = (p, v), A_e is n_v x n_p, B_e
 * n_v x m_v, S_e (the cross term M_e) n_p x m_v, K_e m_v x n_p.  The arrays are
 * PACKED: field f holds the blocks of nodes (or edge slots) 0..N-1 one after
 * another, row-major, each block of its own size (the root's edge blocks are
 * empty); rcr_ragged_offsets gives where each block starts.  Fields, in the
 * order of the offsets (index f):
 *   0 Q (n_v^2)   1 q (n_v)   2 c (n_v)   3 Delta (n_v^2)   4 R (m_v^2)
 *   5 S (n_p m_v) 6 r (m_v)   7 A (n_v n_p)   8 B (n_v m_v)
 *   9 K (m_v n_p) 10 P (n_v^2) 11 x (n_v) 12 u (m_v) 13 lam (n_v)
 * The solve pads every block to the largest dimensions (zeros, and the
 * identity in the unused part of R): the padded coordinates decouple from the
 * rest and solve to zero, so the real blocks of the padded solution are the
 * solution. */
#define RCR_RAGGED_FIELDS 14

/* Plan of a tree with per-node state dimensions n_node[N] and per-edge control
 * dimensions m_edge[N] (HOST int32 arrays; m_edge[root] is ignored), each in
 * 1..RCR_MAX_DIM.  rcr_plan_info reports the padded n and m.  Errors: those of
 * rcr_plan_create. */
int rcr_ragged_plan_create(const int64_t *parent, int64_t N, const int32_t *n_node, const int32_t *m_edge,
                           const rcr_plan_options *opt, rcr_plan **out);

/* Element offsets of the blocks of a ragged plan: offsets[f * (N + 1) + v] is
 * where node (or edge slot) v's block of field f starts in the packed array,
 * offsets[f * (N + 1) + N] the array's length (HOST int64 array of
 * RCR_RAGGED_FIELDS * (N + 1) entries).  Errors: RCR_NULL_ARG, RCR_BAD_OPTION
 * (not a ragged plan). */
int rcr_ragged_offsets(const rcr_plan *plan, int64_t *offsets);

/* Factor and solve a ragged problem (packed DEVICE float64 arrays in the
 * rcr_problem / rcr_solution structs, layouts above) with a plan from
 * rcr_ragged_plan_create.  Options as for rcr_solve; a caller workspace must
 * hold rcr_workspace_size(plan, precision) bytes (it includes the padded
 * problem and solution); opt->kkt_residual reports the residual of the
 * padded system, whose real rows are those of eq. (kkt).  A field of length 0
 * (the edge arrays of a one-node tree) may be NULL.  Errors: those of
 * rcr_solve; RCR_BAD_OPTION when the plan is not a ragged plan. */
int rcr_ragged_solve(const rcr_plan *plan, const rcr_problem *in, rcr_solution *out, const rcr_solve_options *opt,
                     void *stream);

/* ------------------------------------------------------- launch mapping */
/* How a plan maps its narrow dependency levels onto single-workgroup tail
 * kernels (the levels near the root hold few primitives; running them inside
 * one workgroup separated by barriers avoids a launch and a device-wide
 * round trip per level).  A level runs in a tail kernel when its primitives
 * fit in the given number of rounds of the tail workgroup.  0 selects the
 * default of a field; quad_tail_rounds < 0 or vec_tail_rounds < 0 disables
 * that tail.  Results do not depend on the mapping (every primitive runs the
 * same arithmetic wherever it is launched); only the time does. */
typedef struct {
  int32_t quad_tail_rounds; /* quadratic contraction/expansion tail (default: 1 for n > 8,
                                off for n <= 8)                                            */
  int32_t vec_tail_rounds;  /* affine and state tails (default: 2 in FP64, 4 in float32)   */
  int32_t vec_tail_waves;   /* wavefronts of the vector tail workgroup, 1..16 (default 8)  */
  int32_t reserved[5];
} rcr_launch_config;

/* Set (NULL: reset to defaults) or read a plan's launch mapping.  Host only;
 * a change drops the plan's captured graphs.  Errors: RCR_NULL_ARG,
 * RCR_BAD_OPTION (vec_tail_waves outside 0..16). */
int rcr_plan_set_launch(rcr_plan *plan, const rcr_launch_config *cfg);
int rcr_plan_get_launch(const rcr_plan *plan, rcr_launch_config *cfg);

/* Autotune the launch mapping of a plan on a representative problem.  The
 * candidates are timed with HIP events on `stream` (one warm-up and three
 * timed solves each, with the options in opt; the per-level executor is used
 * for the timing).  The quadratic tail only changes the factor's launches and
 * the vector tails only the solve's, so they are tuned in turn: first
 * quad_tail_rounds in {-1 (off), 1, 2, 4, 8}, then, with the best of those,
 * vec_tail_rounds -1 (off) and {2, 4, 8} x vec_tail_waves {8, 16}.  The
 * fastest is kept in the plan and returned in *best (and its time in
 * *best_ms, if not NULL).  `out` receives the solution.  Synchronises the
 * stream.  Errors: those of rcr_solve. */
int rcr_plan_tune(rcr_plan *plan, const rcr_problem *in, rcr_solution *out, const rcr_solve_options *opt,
                  void *stream, rcr_launch_config *best, float *best_ms);

/* Static name of a status code. */
const char *rcr_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* RCR_H */
