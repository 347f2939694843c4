/*
 * hjb.h -- C ABI of the MI355X patchy semi-Lagrangian solver for the
 * minimum-time Hamilton-Jacobi-Bellman equation.
 *
 * Method: Cacace, Cristiani, Falcone, Picarelli, "A Patchy Dynamic
 * Programming Scheme for a Class of Hamilton-Jacobi-Bellman Equations".
 *   - Problem (Section 1, eq. HJB): find the minimal time T(x) to reach a
 *     target Omega_0 under x' = f(x, a), a in A, inside a box Omega with
 *     state constraints on the box boundary.
 *   - Scheme (Section 2.1, eqs. SLscheme and iterativeSLscheme), solved here in
 *     the Kruzkov variable v = 1 - exp(-T):
 *        v_p = min_k  beta * I[v](p + s (c_p a_k + w_p)) + (1 - beta)
 *     with v = 0 on target nodes, linear interpolation I, value iteration
 *     from v = 1 off the target.
 *   - Patchy Algorithm (Section 3): Step 1 coarse solve -> hjb_coarse_solve;
 *     Step 2 prolongation + discrete feedback and Step 3.1 patch creation ->
 *     hjb_build_patches; Step 3.2 independent per-patch iteration and Step 4
 *     merge -> hjb_solve_patches.  hjb_solve_global is the plain solve on the
 *     whole grid (the fixed point the patchy result approximates).
 *
 * Conventions
 *   - Nodes p = (x, y, z), flat index x + n0 (y + n1 z) (x fastest).  2D
 *     problems have dim = 2 and n[2] = 1.
 *   - Dynamics family f(x, a) = c(x) a + w(x), tabulated at the nodes; the
 *     controls a_k are given as vectors.  step[d] = h / k_d converts a
 *     velocity into a displacement in cells.  The per-node displacement
 *     |s_d (c a_kd + w_d)| must stay below 2 cells on every axis (the
 *     kernels' halo is two nodes wide); otherwise HJB_EINVAL.
 *   - beta = exp(-h) is computed by the caller (host libm) and passed in;
 *     one_minus_beta must equal 1 - beta exactly.  For FP32 solves beta
 *     should be FP32-representable so that both constants are exact.
 *   - All floating-point inputs are FP64.  FP32 solves round them to FP32
 *     on the device; FP64 solves use them as given.
 *   - Every call takes a stream (hjb_stream_t is a hipStream_t; NULL = the
 *     default stream), enqueues its device work there and synchronises
 *     that stream before returning (convergence needs host-visible flags).
 *
 * Ownership
 *   - Arrays reachable from an hjb_problem are borrowed for the duration of
 *     the call only and never written.  mem = HJB_MEM_HOST: host pointers
 *     (copied to the device by the call); HJB_MEM_DEVICE: device pointers.
 *   - Output buffers (v_out etc.) are owned by the caller; their memory
 *     kind is given by the call's `mem` argument or is device memory where
 *     stated.
 *   - Handles (hjb_coarse_t, hjb_patches_t, hjb_batch_t, hjb_server_t) are
 *     owned by the library and released only by the matching *_free, which
 *     accepts NULL.
 *
 * Errors
 *   - Every int-returning call returns an HJB_* status; HJB_OK = 0.
 *   - HJB_EINVAL is returned before any output is written when an argument
 *     is malformed (dimensions, beta, control count, target parts, non-finite
 *     data, displacement reach, precision, null pointers).
 *   - HJB_ENOCONV: max_sweeps was reached.  The output still holds the
 *     current iterate, which is an upper bound of the fixed point (value
 *     iteration from above is monotone).
 *   - HJB_EDEVICE / HJB_ENOMEM: a HIP runtime failure / allocation failure.
 *   - hjb_last_error() returns a description of the calling thread's last
 *     failure.  No C++ exception crosses this interface.
 *
 * Threading: calls on different handles may run on different threads; one
 * handle must not be used by two threads at the same time.
 */
#ifndef HJB_H
#define HJB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HJB_OK 0
#define HJB_EINVAL 1
#define HJB_EDEVICE 2
#define HJB_ENOMEM 3
#define HJB_ENOCONV 4
#define HJB_EAGAIN 5

#define HJB_MEM_HOST 0
#define HJB_MEM_DEVICE 1

#define HJB_F32 0
#define HJB_F64 1

/* Schedules of hjb_solve_global. */
#define HJB_SCHED_TILED 0  /* LDS tiles, in-tile sweeps, active-tile lists:
                              synchronous rounds, one launch per round */
#define HJB_SCHED_JACOBI 1 /* one full-grid Jacobi sweep per launch
                              (hjb_solve_global only) */
#define HJB_SCHED_ASYNC 2  /* the same tiles in one persistent launch that
                              drains a device work queue (no rounds; no
                              sweep cap: max_sweeps must be 0) */

/* Boundary of the patch problems in Step 3.2 (hjb_solve_opts.patch_bc). */
#define HJB_BC_STATE 0     /* state constraint: other patches' nodes are
                              ghosts of value 1 */
#define HJB_BC_DIRICHLET 1 /* eq. dbc: other patches' nodes (and unlabeled
                              ones) hold U^(0) of Step 2; the domain
                              boundary keeps the state constraint */

typedef void *hjb_stream_t; /* hipStream_t */

/* A tabulated minimum-time problem (Section 1, eq. HJB; Section 2.1). */
typedef struct {
  int32_t dim;                /* 2 or 3 */
  int32_t n[3];               /* nodes per axis, >= 2; n[2] = 1 in 2D */
  double step[3];             /* s_d = h / k_d (cells per unit velocity) */
  double beta;                /* exp(-h), in [0.5, 1) */
  double one_minus_beta;      /* exactly 1 - beta */
  int32_t n_controls;         /* N_c, 1..255 */
  const double *controls;     /* [N_c][dim] control vectors a_k */
  const double *speed;        /* [N] c(x_p) >= 0 */
  const double *drift;        /* [N][dim] w(x_p), or NULL for w = 0 */
  const int16_t *target_part; /* [N] -1 off the target, part j < n_parts on
                                 it, HJB_OBSTACLE inside an obstacle */
  int32_t n_parts;            /* R >= 1: parts of the target (Section 3) */
  int32_t mem;                /* HJB_MEM_HOST or HJB_MEM_DEVICE */
  const double *beta_node;    /* [N] or NULL.  Variable step (Section 2.1,
                                 h_i with the foot point one cell away):
                                 beta_i = exp(-h_i) in [0, 1) per node, used
                                 instead of beta in the scheme and in the
                                 colour transport, with 1 - beta_i formed in
                                 FP64.  beta_i = 0 freezes the node at 1.
                                 For f = c(x) a with unit controls the caller
                                 passes speed 1, step 1 and
                                 beta_i = exp(-k / c_i). */
  const double *foot;         /* [N_c][N][dim] or NULL.  Tabulated dynamics
                                 (any f, e.g. with the step rule of Section
                                 2.1 per node and control): the foot-point
                                 displacement of node p under control k, in
                                 cells, replacing s (c a_k + w); |foot| must
                                 stay below 2 cells.  Patch and global
                                 solves in rounds (not HJB_SCHED_ASYNC, not
                                 control_cone, not in batches or the
                                 server). */
  const double *beta_pk;      /* [N_c][N] or NULL: beta per control and node
                                 (exp(-h_{p,k})), in [0, 1), replacing beta /
                                 beta_node; 1 - beta formed in FP64.  Needs
                                 foot. */
} hjb_problem;

/* Per-call statistics. */
typedef struct {
  int64_t updates;         /* node-control updates executed (nodes x N_c per node sweep) */
  int64_t node_updates;    /* node updates executed */
  int64_t item_runs;       /* tile work-item activations */
  int32_t items;           /* tile work items of the solve */
  int32_t rounds;          /* sweep-kernel launches */
  double residual;         /* sup-norm decrease in the last round (FP64) */
  double ms_wall;          /* host wall time of the call */
  double ms_kernel;        /* summed HIP-event time of the sweep kernel (time_kernels) */
  int32_t kernel_launches; /* launches included in ms_kernel */
  int32_t status;          /* HJB_OK or HJB_ENOCONV */
  /* hjb_build_patches only: per-step wall times and colour-transport work */
  double ms_prolong_feedback;
  double ms_trace;
  int64_t trace_node_updates;
  int32_t unreached;       /* nodes no colour reached; they took their
                              neighbours' label (Remark 3.1) */
  int32_t sweeps;          /* HJB_SCHED_JACOBI: whole-grid sweeps executed */
  /* launch configuration of the sweep kernel that ran (tiled solves) */
  int32_t tile[3];
  int32_t threads;
  int32_t inner_sweeps;
  int32_t excluded;        /* hjb_build_patches_ex: nodes excluded as
                              unreachable after Step 1 */
  int32_t detached;        /* hjb_build_patches: nodes of pieces of a patch
                              that the projection cut off from their own
                              target part (no node of the piece, 8 / 26
                              neighbours, is a target node of its part);
                              they took their neighbours' label
                              (Remark 3.1) */
} hjb_stats;

/* target_part value of a node inside an obstacle (Section 4.5): a state
 * constraint inside the box.  Such a node is never updated, keeps the value
 * 1 (T = +inf), reads as the ghost value in every interpolation (1 for
 * values and U^(0), 0 for colours), gets feedback 255 and label
 * HJB_OBSTACLE, and is never given a label by the Remark 3.1 fill. */
#define HJB_OBSTACLE (-2)

/* Tuning options; NULL or zero fields select the defaults. */
typedef struct {
  int32_t tile[3];         /* tile shape in nodes; supported (tile, threads):
                              2D 16x16 and 32x8 with 256, 512 or 1024;
                              32x16 with 256, 512 or 1024; 64x8, 64x16 and
                              32x32 with 256 or 512;
                              3D 8x8x8 with 256 or 512, 16x8x8 with 256 or
                              512, 32x8x4 with 256.  More threads than tile
                              nodes split each node's controls into
                              threads / nodes slices (same results). */
  int32_t inner_sweeps;    /* max in-LDS sweeps per tile activation */
  int32_t rounds_per_poll; /* sweep rounds enqueued between host polls */
  int32_t schedule;        /* HJB_SCHED_* (JACOBI: hjb_solve_global only) */
  int32_t time_kernels;    /* 1: HIP events around each polled block of
                              sweep launches (kernel time in hjb_stats) */
  int32_t use_graph;       /* 1: replay the polled rounds as a hipGraph */
  int32_t threads;         /* workgroup size of the sweep kernel (see tile) */
  const uint8_t *patch_select; /* host [n_parts] 0/1, NULL = all patches
                                  (hjb_solve_patches only): nodes of
                                  unselected patches are left at 1 */
  double control_cone;     /* add-on AO3 (Section "Patchy method's add-ons"),
                              hjb_solve_patches only: r > 1 lets each node
                              minimise over the controls a_k with
                              a_k . a_ks >= cos(pi / r) only, a_ks = its
                              Step 2 feedback control (always kept); the dot
                              product is an FP64 sum over the axes in order,
                              no fused multiply-add.  0 (or <= 1) = every
                              control.  Needs HJB_SCHED_TILED and a tile
                              shape among 2D 32x8, 32x16, 3D 8x8x8 (256
                              threads); the tables (N_c rows of the
                              largest cone, padded to 4 bytes, plus the
                              controls) must fit 32 KiB of LDS.
                              hjb_stats.updates then counts the largest
                              cone per node update. */
  int32_t patch_bc;        /* HJB_BC_* (patch solves: hjb_solve_patches,
                              batches, the server); 0 = HJB_BC_STATE */
  double order_window;     /* add-on AO2 (Section "Patchy method's add-ons"),
                              patch solves (also batches and the server),
                              rounds schedule: > 0
                              runs the tiles in the order of their Step 2
                              values.  A tile's key is the smallest minimal
                              time -ln(1 - U^(0)) of its patch nodes; a
                              queued tile runs in a round only if its key is
                              at most the round's threshold, else it waits.
                              The threshold of a round is the larger of the
                              smallest queued key and the previous round's
                              threshold plus order_window time steps h
                              (h = -ln beta).  The fixed point (and so the
                              result, bit for bit) is the same; only the
                              order and the work change.  0 = off. */
  int32_t start_u0;        /* add-on AO1 (same section), patch solves (also
                              batches and the server, with their tol),
                              rounds schedule: 1 starts every patch
                              node at U^(0) of Step 2.  U^(0) is not above
                              the fixed point, so the iteration becomes
                              v <- F(v) (values may rise) and stops when no
                              node moves by more than tol, which must be at
                              least 1e-7 in FP32 and 1e-13 in FP64; the
                              result then lies within about
                              tol beta / (1 - beta) of the fixed point. */
} hjb_solve_opts;

typedef struct hjb_coarse_s hjb_coarse_t;
typedef struct hjb_patches_s hjb_patches_t;
typedef struct hjb_batch_s hjb_batch_t;
typedef struct hjb_server_s hjb_server_t;

/* Step 1 of the Patchy Algorithm (Section 3): value iteration of eq.
 * iterativeSLscheme on the coarse grid, every node active, FP64.  The
 * paper runs it with its domain-decomposition solver; both reach the fixed
 * point of the same operator (Section 2.2, F and F_SPLIT share it), which is
 * what is computed here.  tol = 0 iterates to the exact FP64 fixed point
 * (no node changes in a full pass); tol > 0 stops once no node decreases by
 * more than tol.  *out receives a new handle holding the coarse values. */
int hjb_coarse_solve(const hjb_problem *coarse, double tol, int32_t max_sweeps,
                     hjb_stream_t stream, hjb_coarse_t **out);

/* Copies the coarse values (FP64, [N coarse]) to out (host or device). */
int hjb_coarse_values(const hjb_coarse_t *c, double *out, int32_t mem);
void hjb_coarse_free(hjb_coarse_t *c);

/* Steps 2 and 3.1 of the Patchy Algorithm (Section 3), FP64:
 *   - U^(0) = linear interpolation of the coarse values at the fine nodes;
 *   - discrete feedback (eq. feedbackcontrol): at every non-target fine node
 *     the first control k minimising the scheme's right-hand side at the
 *     foot point, beta_k I_k + 1 - beta_k with I_k = I[U^(0)](p + s (c a_k
 *     + w)) (ghost 1 outside the box); when beta does not depend on the
 *     control (no beta_pk table) the raw I_k is compared; target nodes
 *     carry 255;
 *   - for every part j the colour transport with frozen feedback (eq.
 *     HJBridotta_discreta), phi^j = 1 on part j of the target, 0 on the rest
 *     of it, phi <- max(phi, beta I[phi](foot of the feedback)) from 0
 *     until no node changes (ghost 0 outside the box; colours below 1e-9
 *     count as 0);
 *   - labels (eq. proiezionecolore with Remark 3.1): target node -> its
 *     part; obstacle node -> HJB_OBSTACLE; otherwise the part of largest
 *     colour, the lowest index on ties, and where every colour is 0 the
 *     smallest label of the nearest labelled nodes (8 / 26 neighbours,
 *     layer by layer), -1 if there is none.
 * The coarse problem only fixes the coarse grid size; the handle carries its
 * values.  *out receives a new handle with labels, feedback and U^(0) on the
 * device.  st may be NULL. */
int hjb_build_patches(const hjb_problem *fine, const hjb_coarse_t *coarse, hjb_stream_t stream,
                      hjb_patches_t **out, hjb_stats *st);

/* Options of hjb_build_patches_ex; NULL or zero fields select the defaults. */
typedef struct {
  double exclude_at;       /* Section 4.6: > 0 excludes, after Step 1, the
                              unreachable regions: a fine node off the
                              target whose U^(0) is at least exclude_at
                              (in (0, 1]; 1 = the coarse solve never reached
                              any of its coarse corners) takes no part in
                              Steps 2 and 3 -- it is treated as an obstacle
                              node: no feedback (255), label -2, value 1,
                              a ghost of value 1 for the other nodes.
                              hjb_stats.excluded counts these nodes. */
} hjb_build_opts;

/* hjb_build_patches with options (NULL = hjb_build_patches). */
int hjb_build_patches_ex(const hjb_problem *fine, const hjb_coarse_t *coarse,
                         const hjb_build_opts *opts, hjb_stream_t stream, hjb_patches_t **out,
                         hjb_stats *st);

/* Accessors of a patches handle; `out` is host or device memory per mem. */
int hjb_patches_labels(const hjb_patches_t *p, int16_t *out, int32_t mem);     /* [N] */
int hjb_patches_feedback(const hjb_patches_t *p, uint8_t *out, int32_t mem);   /* [N] */
int hjb_patches_u0(const hjb_patches_t *p, double *out, int32_t mem);          /* [N] */
void hjb_patches_free(hjb_patches_t *p);

/* Steps 3.2 and 4 of the Patchy Algorithm (Section 3): value iteration of
 * eq. iterativeSLscheme independently in every patch j, with the
 * state-constraint patch boundary (non-target nodes of other patches and
 * nodes outside the box are ghosts of value 1; every target node is 0), then
 * the merge: v_out = value of the node's own patch, 0 on the target, 1 where
 * the label is -1.  precision HJB_F32: v stored and iterated in FP32, the
 * stopping residual in FP64; HJB_F64: FP64 throughout, bitwise equal to any
 * other exact-fixed-point schedule of the same operator.  tol as in
 * hjb_coarse_solve.  With tol = 0 every schedule (tile shape, sweeps per
 * round, graph replay, persistent launch) stops at the same bits, in FP32
 * too; with tol > 0 the point where the iteration stops depends on the
 * order in which workgroups ran, so two runs may differ in the last bits
 * (each within the tolerance bound of the fixed point).  v_out:
 * caller-owned DEVICE buffer of N floats or doubles.  opts and st may be
 * NULL. */
int hjb_solve_patches(const hjb_problem *fine, const hjb_patches_t *p, int32_t precision,
                      double tol, int32_t max_sweeps, void *v_out, const hjb_solve_opts *opts,
                      hjb_stats *st, hjb_stream_t stream);

/* Plain solve of eq. iterativeSLscheme on the whole grid (every box node an
 * unknown, ghost 1 outside the box), FP32 or FP64; schedule per opts
 * (default HJB_SCHED_TILED).  Arguments as hjb_solve_patches. */
int hjb_solve_global(const hjb_problem *fine, int32_t precision, double tol, int32_t max_sweeps,
                     void *v_out, const hjb_solve_opts *opts, hjb_stats *st,
                     hjb_stream_t stream);

/* ---------------------------------------------------------------- batching
 * Many independent patchy problems (2D and 3D, uneven sizes, control and
 * patch counts) solved together: every (problem, patch, tile) is one work
 * item of one sweep launch per round (replayed as a hipGraph with
 * solve.use_graph), or of one persistent launch that drains a device queue
 * of items (solve.schedule = HJB_SCHED_ASYNC), with a per-item device
 * convergence flag; a problem is finished when none of its items is active.
 * Independence of the patches (Section 3, parallelisation "Method 2") is
 * what makes the packing exact: each result is bitwise the one of a solve
 * alone. */
typedef struct {
  int32_t precision;       /* HJB_F32 (default) or HJB_F64 */
  double tol;              /* as hjb_solve_patches */
  int32_t max_sweeps;      /* per problem, in rounds x inner sweeps */
  hjb_solve_opts solve;    /* tile / inner sweeps / polling / graph /
                              schedule (HJB_SCHED_TILED rounds or
                              HJB_SCHED_ASYNC, the latter without
                              order_window, start_u0, use_graph and with
                              max_sweeps 0) */
  uint64_t prepare_bytes;  /* device bytes that the shared colour transport
                              of hjb_batch_create may hold at once (colour
                              fields and the rest of Steps 2-3.1); problems
                              beyond it go to the next chunk.  0 = 32 GiB. */
} hjb_batch_opts;

/* fine[i] and coarse[i] describe problem i; the call runs Steps 1-3.1 for
 * every problem and prepares the work items.  opts may be NULL. */
int hjb_batch_create(const hjb_problem *const *fine, const hjb_problem *const *coarse,
                     int32_t count, const hjb_batch_opts *opts, hjb_stream_t stream,
                     hjb_batch_t **out);
/* Runs Step 3.2 for every problem of the batch to convergence. */
int hjb_batch_run(hjb_batch_t *b, hjb_stream_t stream, hjb_stats *st);
/* Copies problem i's merged result (precision of the batch) to v_out (host
 * or device per mem). */
int hjb_batch_result(const hjb_batch_t *b, int32_t i, void *v_out, int32_t mem, hjb_stats *st);
void hjb_batch_free(hjb_batch_t *b);

/* ---------------------------------------------------------------- no allocation
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the plain
 * global solve of hjb_solve_global with HJB_SCHED_JACOBI, bitwise the same
 * values and statistics, with every buffer beyond the caller's inputs and
 * v_out in one static device array of the library (48 MiB per GPU, held
 * until the process ends).  It calls no hipMalloc, hipFree or other
 * allocating routine.
 *   - fine: device inputs (mem = HJB_MEM_DEVICE) of the family
 *     f = c(x) a + w(x) with one beta (no beta_node, foot or beta_pk);
 *     at most HJB_NOALLOC_MAX_NODES nodes; otherwise HJB_EINVAL before any
 *     device work.
 *   - v_out: device, N values of the precision; the stats as
 *     hjb_solve_global (no kernel timing).
 *   - Every call on a GPU uses that GPU's one array, which keeps the last
 *     call's contents: calls that overlap on one GPU (several host threads
 *     or streams) race and must be serialised by the caller. */
#define HJB_NOALLOC_MAX_NODES (1 << 21)
int hjb_solve_global_noalloc(const hjb_problem *fine, int32_t precision, double tol,
                             int32_t max_sweeps, void *v_out, hjb_stats *st,
                             hjb_stream_t stream);

/* ---------------------------------------------------------------- serving
 * Continuous batching of solve requests: a submitted request is admitted
 * when its HBM footprint fits the budget, goes through Steps 1-3.1, and its
 * work items join the live sweep rounds while other requests are running;
 * its value grid stays resident until it is collected. */
typedef struct {
  int32_t precision;       /* HJB_F32 (default) or HJB_F64 */
  double tol;
  int32_t max_sweeps;
  hjb_solve_opts solve;
} hjb_server_opts;

/* hbm_budget: bytes of device memory requests may hold at once.  The
 * server starts a pool of host threads (a HIP stream each, on the calling
 * thread's current device) that prepare admitted requests; they stop in
 * hjb_server_free.  The server runs in rounds, since requests join between
 * them (HJB_EINVAL for HJB_SCHED_ASYNC). */
int hjb_server_create(size_t hbm_budget, const hjb_server_opts *opts, hjb_stream_t stream,
                      hjb_server_t **out);
/* Queues a request (arrays are copied before returning); *ticket
 * identifies it.  HJB_EINVAL if it could never fit the budget. */
int hjb_server_submit(hjb_server_t *s, const hjb_problem *fine, const hjb_problem *coarse,
                      uint64_t *ticket);
/* Advances the server: admits queued requests that fit (their footprint is
 * reserved and the preparation pool runs their coarse solve and build steps
 * meanwhile), adds the requests whose preparation finished to the live set,
 * runs `rounds` sweep rounds over every live request and retires the
 * converged ones.  *live and *queued (may be NULL) receive the counts
 * (queued: waiting for admission or in preparation). */
int hjb_server_step(hjb_server_t *s, int32_t rounds, int32_t *live, int32_t *queued);
/* HJB_EAGAIN until the request is done; then copies its result (precision
 * of the server) to v_out (host or device per mem), fills st and releases
 * the request's memory.  A request whose preparation failed returns that
 * error here (and is released). */
int hjb_server_poll(hjb_server_t *s, uint64_t ticket, void *v_out, int32_t mem, hjb_stats *st);
void hjb_server_free(hjb_server_t *s);

/* Description of the calling thread's last error ("" if none). */
const char *hjb_last_error(void);

/* Library version string. */
const char *hjb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HJB_H */
