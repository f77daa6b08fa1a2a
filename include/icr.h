/*
 * icr.h -- C ABI of the MI355X constraint-matrix library.
 *
 * Implements the hot path of the implicit contact/friction scheme of
 * Zeng & Courtecuisse, "An efficient implicit constraint resolution scheme for
 * interactive FE simulations" (arXiv 2306.06946):
 *   per time step        W_H = H A^{-1} H^T         (Eq. 28, Algorithm 3)
 *   per Newton iteration W = C W_H C^T, projected Gauss-Seidel for lambda,
 *                        p_k = p_free + h^2 W_H C_k^T lambda_k  (Eq. 31)
 * for the backward-Euler system A = M + h B + h^2 K (Eq. 5) of a linear
 * tetrahedral mesh, with A factored once by a supernodal Cholesky on the GPU.
 *
 * Conventions (all entry points):
 *   - Every call returns an icr_status; no exception crosses the ABI.  On an
 *     error, icr_last_error() holds a message until the next call on that
 *     scene.  A scene is not thread-safe: one host thread at a time.
 *   - "host" pointers are read during the call and copied; "device" pointers
 *     are caller-owned GPU buffers (e.g. torch tensors) that the library never
 *     frees.  Library-owned device memory (mesh, factor, work arenas, state)
 *     lives until icr_destroy.
 *   - Device work is enqueued on the scene's stream (icr_create).  Calls that
 *     return host values (sweeps, eps, reports) synchronise that stream.
 *   - Arrays are row-major, float64 unless stated; node ids are int32,
 *     DOF index = 3 * node + axis.  A contact is a point mapped from mesh
 *     nodes (Eq. 6: a node, or a weighted sum of up to four nodes in
 *     icr_build_WH) with a frame of three rows (normal, tangent 1,
 *     tangent 2; Eq. 26) and three force components.
 */
#ifndef ICR_H
#define ICR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct icr_scene icr_scene;

typedef enum {
  ICR_OK = 0,
  ICR_WARN_NOT_CONVERGED = 1, /* PGS hit max_sweeps with eps > tol; results valid */
  ICR_E_ARG = -1,             /* invalid argument (message says which) */
  ICR_E_NOT_SPD = -2,         /* Cholesky met a non-positive pivot (column in message) */
  ICR_E_OOM = -3,             /* device allocation failed */
  ICR_E_HIP = -4,             /* HIP runtime error (message has the HIP error string) */
  ICR_E_STATE = -5            /* call order violated (e.g. build_WH before factor) */
} icr_status;

/* Arithmetic of a time step (icr_step_opts.precision). */
typedef enum {
  ICR_FP64 = 0,    /* every solve, product and store in FP64 */
  ICR_FP32_IR = 1  /* the multi-RHS forward solve of W_H in FP32 (FP32 MFMA) followed by
                      icr_step_opts.refine steps of iterative refinement whose residual
                      P H^T - L Z is formed in FP64 against the FP64 factor, W_H = Z^T Z summed
                      in FP64; W_H and W stored in FP32 for the Newton loop, every product
                      with them and the PGS local solves accumulated in FP64 */
} icr_precision;

/* Contact status codes written by icr_solve_contacts / icr_step. */
enum { ICR_SEPARATE = 0, ICR_STICK = 1, ICR_SLIP = 2 };

/* Create a scene bound to a HIP stream (hipStream_t passed as void*; NULL =
 * the null stream) on the current device.  *out is NULL on failure. */
icr_status icr_create(icr_scene **out, void *stream);

/* Free every library-owned buffer.  Safe on NULL. */
void icr_destroy(icr_scene *s);

/* Last error message of this scene ("" if none); valid until the next call. */
const char *icr_last_error(const icr_scene *s);

/* Rebind the scene to another stream (e.g. torch's current stream). */
icr_status icr_set_stream(icr_scene *s, void *stream);

/* enable = 1 (default): the multi-RHS solve of icr_build_WH / icr_step runs
 * the W_H products of each elimination-tree level on a second stream of the
 * scene, overlapping the next level's solve (joined before the call's later
 * work).  enable = 0: everything on the scene's stream -- what many scenes
 * stepped concurrently want, since every extra stream takes a place among
 * the process's few hardware queues.  Same results either way.
 * ICR_E_ARG unless enable is 0 or 1. */
icr_status icr_set_overlap(icr_scene *s, int32_t enable);

/*
 * Assemble the linear-elastic FE model (Sec. "Implicit time integration",
 * Eq. 4-5): per tetrahedron K_e = V B^T D B (isotropic D from E, nu), lumped
 * mass rho V / 4 per node, Rayleigh damping B = alpha M + beta K, and
 * A = M + h B + h^2 K.  DOFs of nodes with fixed[i] != 0 are clamped
 * (identity rows/columns of A, zero right-hand side).
 *   nodes [N*3] host, rest positions (also the initial state q, v = 0)
 *   tets  [T*4] host int32, positively oriented
 *   E, nu [T]   host, per element
 *   gravity[3] host; fixed [N] host uint8
 * Errors: ICR_E_ARG on bad sizes/ids, a non-positive volume, E <= 0 or
 * nu outside (0, 0.5).  Replaces any previous mesh (and drops the factor).
 */
icr_status icr_assemble(icr_scene *s, const double *nodes, int32_t N, const int32_t *tets, int32_t T,
                        const double *E, const double *nu, double rho, double alpha, double beta, double h,
                        const double *gravity, const uint8_t *fixed);

/*
 * Factor A = P^T L L^T P: nested-dissection ordering and supernodal symbolic
 * analysis on the host, numeric supernodal FP64 Cholesky on the device (the
 * factor the multi-RHS solves of W_H run against, Eq. 28).  Synchronises.
 * ICR_E_NOT_SPD names the first failing permuted column.
 */
icr_status icr_factor(icr_scene *s);

typedef struct {
  int64_t n;             /* DOFs */
  int64_t n_supernodes;
  int64_t n_levels;      /* height levels of the supernodal tree */
  int64_t nnz_L;         /* stored entries of the supernodal panels (lower, incl. zeros) */
  int64_t max_front;     /* largest front order (DOFs) */
  double factor_flops;   /* dense flops of the numeric factor (partial Choleskys) */
  double factor_ms;      /* device time of the numeric factor */
  int64_t device_bytes;  /* library-owned device memory */
} icr_factor_info;

icr_status icr_get_factor_info(icr_scene *s, icr_factor_info *out);

/*
 * Mapping compliance W_H = H A^{-1} H^T (Eq. 28), H the Jacobian of the
 * geometric mapping of the contact points (Eq. 6).  Computed as W_H = Z^T Z
 * with Z = L^{-1} P H^T: a sparse-RHS supernodal forward solve (each node's
 * three columns live only on the path from its supernode to the root)
 * followed by per-supernode SYRK updates.  The result is exactly symmetric.
 *   weights == NULL: nodal contacts, H selects the three DOFs of a node:
 *     node_ids [n_c] device int32, distinct, not clamped.
 *   weights != NULL: mapped contacts, point c = sum_k weights[4c+k] x(node_ids[4c+k]):
 *     node_ids [n_c*4] device int32, -1 marks an unused slot; weights
 *     [n_c*4] device, finite and non-zero on used slots.  A node may be
 *     shared by several contacts; a negative weight puts the node on the
 *     other side of the pair, so that with the nodes of body 1 weighted +w
 *     and those of body 2 -w, H = [H_1, -H_2] and H q = x_1 - x_2 (the two-
 *     body mapping of Eq. 16-17 on the block-diagonal A of two meshes).
 *     Computed from the nodal W_N of the distinct nodes (at most 8192):
 *     W_H = H_w W_N H_w^T, H_w the n_c x nodes weight matrix.
 *   WH [m*m] device, m = 3 n_c, row-major; row 3c+a = contact c, axis a
 * Errors: ICR_E_STATE before icr_factor; ICR_E_ARG if n_c < 1, n_c > 8192
 * or more distinct nodes than that, or a bad id or weight.  Nodal ids are
 * validated on the device, mapped ones on the host; the call synchronises
 * the stream.
 */
icr_status icr_build_WH(icr_scene *s, int32_t n_c, const int32_t *node_ids, const double *weights, double *WH);

/*
 * Fast update of the compliance matrix (Eq. 28, Algorithm 3 step 2):
 * W_ab = C_a (W_H)_ab C_b^T for all 3x3 blocks.
 *   WH [m*m] device; C [n_c*9] device, row-major 3x3 per contact (rows
 *   normal, t1, t2); W [m*m] device output (may not alias WH).
 */
icr_status icr_update_W(icr_scene *s, int32_t n_c, const double *WH, const double *C, double *W);

/*
 * Projected Gauss-Seidel on delta = d + h^2 W lambda with Signorini (Eq. 8)
 * and the Coulomb cone |lambda_t| <= mu lambda_n (Eq. 9), sweeping contacts in
 * index order (Eq. 19, Algorithm 1).  Per contact: separate if its gap
 * d_n >= 0; else the stick trial lambda = -(h^2 W_aa)^{-1} d if inside the
 * cone; else slip on the cone boundary (delta_n = 0, lambda_t opposite to the
 * tangential gap) by j_inner passes of a shifted fixed point.  After every
 * sweep eps = |lam_i - lam_{i-1}|_2 / |lam_i|_2; stop when eps <= tol or after
 * max_sweeps sweeps.
 *   W [m*m] device, exactly symmetric and positive semidefinite with
 *   positive definite 3x3 diagonal blocks, as icr_update_W writes it from a
 *   W_H of icr_build_WH (rows are read in place of columns, and contacts that
 *   cannot change in a sweep are settled by the Cauchy-Schwarz bound
 *   |W_cq| <= sqrt(W_cc W_qq) of a PSD matrix; an indefinite W gives iterates
 *   that may differ from the sequential sweep); d [m], mu [n_c] device;
 *   lambda [m] device in/out (warm start);
 *   status [n_c] device int8 (branch of the last sweep)
 *   sweeps_out, eps_out: host, may be NULL (then the call does not synchronise)
 * Returns ICR_WARN_NOT_CONVERGED (when eps_out/sweeps_out are given and
 * eps > tol).  ICR_E_ARG on n_c < 1 or n_c > 4096, max_sweeps < 1, j_inner < 0, h <= 0.
 */
icr_status icr_solve_contacts(icr_scene *s, int32_t n_c, const double *W, const double *d, const double *mu,
                              double h, double *lambda, int8_t *status, int32_t max_sweeps, double tol,
                              int32_t j_inner, int32_t *sweeps_out, double *eps_out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * icr_solve_contacts without a scene.  Same arguments, kernels and results;
 * the call allocates nothing and enqueues its work on `stream` (hipStream_t
 * as void*, NULL = the null stream) of the current device.  Its work buffers
 * live in one static device array of the library, about 32 MB per GPU, held
 * until the process ends; every call on a GPU shares that GPU's array, so
 * calls that overlap on one GPU (other streams, other host threads) race.
 * n_c <= 1024.  Errors are return codes only (no scene holds a message):
 * ICR_E_ARG on n_c outside [1, 1024], max_sweeps < 1, j_inner < 0,
 * h <= 0 or non-finite, a NULL device pointer; ICR_E_HIP on a runtime error.
 */
icr_status icr_solve_contacts_noalloc(void *stream, int32_t n_c, const double *W, const double *d, const double *mu,
                                      double h, double *lambda, int8_t *status, int32_t max_sweeps, double tol,
                                      int32_t j_inner, int32_t *sweeps_out, double *eps_out);

/*
 * Proximity update p = p_free + h^2 W_H f (Eq. 31 with the total force
 * f = C_k^T lambda_k in world frame, one 3-vector per contact).
 *   WH [m*m] device, exactly symmetric (as icr_build_WH writes it: rows are
 *   read in place of columns, and only those of contacts with a non-zero
 *   force); p_free [m], f [m] device; p [m] device output.
 * ICR_E_ARG on n_c < 1 or a non-finite or non-positive h.
 */
icr_status icr_proximity_update(icr_scene *s, int32_t n_c, const double *WH, const double *p_free,
                                const double *f, double h, double *p);

/* Kinematic rigid obstacle (stand-in for collision detection, Sec. "Contact
 * generation"): a sphere (kind 1, centre c(t) = c0 + vel t, radius) or a plane
 * (kind 0, point c(t), unit normal pointing towards the body). */
typedef struct {
  int32_t kind;
  double c0[3];
  double vel[3];
  double normal[3];
  double radius;
} icr_obstacle;

/* Contact candidates (surface nodes) and their friction coefficients, host
 * arrays, copied.  count in [1, 4096]; candidates must be distinct, in range
 * and not clamped, mu finite and >= 0 (else ICR_E_ARG).  Their order is
 * irrelevant: each step keeps the n_contacts candidates with the smallest
 * (signed distance, node id) and numbers its contacts by ascending node id. */
icr_status icr_set_candidates(icr_scene *s, int32_t count, const int32_t *nodes, const double *mu);

/*
 * Pair contacts between two deformable bodies meshed in one scene (two
 * components of the mesh: A is block diagonal).  A pair is a point of body 1
 * against the same point of body 2: p = H q = x_1 - x_2 with H = [H_1, -H_2]
 * (Eq. 6, 16-17), given as up to four (node, weight) slots with the body-2
 * weights negative, so that its force acts as +f on body 1 and -f on body 2
 * (c_2 = -J_2^T lambda).  Its normal n is the unit normal of body 2's
 * surface at the point, fixed over a time step; the normal gap is n . p
 * (0 for points that coincide at rest), the tangential gap the relative
 * tangential displacement over the step, tangents by the axis rule.  Every
 * step's contacts are the pairs, in the given order, followed by the
 * obstacle contacts (n_contacts - count closest candidates); a pair
 * warm-starts from its own force of the previous step.  Host arrays, copied:
 *   node_ids [count*4] int32 (-1 unused), weights [count*4], normals
 *   [count*3] (unit), mu [count] (>= 0).  count = 0 removes the pairs.
 * Pair nodes may not be clamped or contact candidates; at most 8192
 * distinct pair nodes; count <= 4096.  More pairs than the interface nodes
 * can carry (several points per node) make W rank deficient; PGS still runs
 * (its 3x3 diagonal blocks stay SPD), lambda is then not unique.
 * ICR_E_STATE before icr_assemble; ICR_E_ARG on a bad id, weight, normal or
 * friction.
 */
icr_status icr_set_pairs(icr_scene *s, int32_t count, const int32_t *node_ids, const double *weights,
                         const double *normals, const double *mu);

typedef struct {
  int32_t n_contacts;   /* contacts per step: the pairs (icr_set_pairs), then the closest candidates */
  int32_t n_newton;     /* Newton iterations (Algorithm 3), 1..256.  With max_sweeps = 1 the
                           directions are updated after every PGS sweep (the per-sweep update
                           the results section proposes) */
  int32_t max_sweeps;   /* PGS sweeps per Newton iteration */
  int32_t j_inner;      /* slip fixed-point passes */
  double tol;           /* PGS stopping tolerance */
  int32_t timing;       /* 1: record per-phase device times in the report */
  int32_t scheme;       /* 0: fast update (Algorithm 3); 1: standard rebuild (Algorithm 2);
                           2: directions updated before every local solve (the per-constraint
                           variant of the results section): each Newton iteration is one
                           Gauss-Seidel call on world-frame forces in which contact a's frame,
                           gap and block h^2 C_a W_H,aa C_a^T are taken at its current proximity
                           p_a = p_free,a + h^2 (W_H f)_a, followed by Eq. 31 */
  int32_t graph;        /* 1: capture the step's launch sequence once (per options) as a HIP graph
                           and replay it; 0: launch every kernel eagerly.  Same results. */
  int32_t precision;    /* icr_precision; ICR_FP32_IR needs scheme 0 */
  int32_t refine;       /* refinement steps of ICR_FP32_IR, 0..2 (0: the raw FP32 solve) */
} icr_step_opts;

typedef struct {
  double t;                 /* simulation time at the end of the step */
  double ms_total;          /* device time of the whole step (timing = 1) */
  double ms_free;           /* free motion: right-hand side + solve (Eq. 5, 12) */
  double ms_contacts;       /* signed distances + selection + mapping */
  double ms_build_WH;       /* W_H = H A^-1 H^T (Eq. 28) */
  double ms_newton;         /* all Newton iterations (directions, update_W, PGS, GEMV) */
  double ms_update_W;       /* sum over Newton iterations (standard scheme: J A^-1 J^T rebuild) */
  double ms_pgs;            /* sum over Newton iterations */
  double ms_correct;        /* corrective solve + integration (Eq. 20) */
  int32_t sweeps[16];       /* PGS sweeps per Newton iteration (first 16) */
  double eps[16];           /* final eps per Newton iteration (first 16) */
  int32_t n_separate, n_stick, n_slip;   /* status counts after the last iteration */
  double ms_corr;           /* sum over Newton iterations of the per-iteration correction:
                               proximity GEMV (fast) or A^-1 J^T lambda solve + H q (standard) */
} icr_step_report;

/*
 * One time step (Algorithm 1 with Algorithm 3 inside; opt->scheme = 1 runs
 * Algorithm 2 instead: per iteration W_k = J_k A^-1 J_k^T by the multi-RHS
 * solve with RHS J_k^T, PGS, q_k = q_free + h^2 A^-1 J_k^T lambda_k, p_k = H q_k):
 * free motion; contacts = the n_contacts candidates with the smallest signed
 * distance at q_free (ties by node id), ordered by node id; W_H; n_newton
 * iterations of {frames and gaps at p_{k-1}, W_k = C_k W_H C_k^T, PGS warm
 * started from the rotated previous force, p_k = p_free + h^2 W_H C_k^T
 * lambda_k}; corrective motion dv = dv_free + h A^-1 H^T f; v += dv;
 * q += h v.  rep (host, may be NULL) is filled after a synchronisation.
 */
icr_status icr_step(icr_scene *s, const icr_obstacle *obs, const icr_step_opts *opt, icr_step_report *rep);

/* Allocate now every device buffer that a time step (or icr_build_WH) with up
 * to max_contacts nodal contacts uses in the given icr_precision (ICR_FP32_IR
 * adds the FP32 copy of the factor and the FP32 solve buffers), so that such
 * calls allocate nothing later (serving admission charges these bytes).
 * ICR_E_STATE before icr_factor; ICR_E_ARG unless max_contacts is in
 * [1, 4096] and precision is an icr_precision; ICR_E_OOM. */
icr_status icr_reserve(icr_scene *s, int32_t max_contacts, int32_t precision);

/* Scene state, device buffers of n = 3N doubles (read / overwrite).
 * icr_set_state starts a new trajectory: it also clears the per-node contact
 * forces that warm-start the next step's PGS. */
icr_status icr_get_state(icr_scene *s, double *q, double *v, double *t_out);
icr_status icr_set_state(icr_scene *s, const double *q, const double *v, double t);

/*
 * Results of the last icr_step, device outputs (any may be NULL):
 *   node_ids [n_c] int32, q_free [n], p [m] final proximity, lambda [m] in
 *   the last frame, C [n_c*9], f [m] world force, status [n_c] int8, WH [m*m].
 */
icr_status icr_get_step_results(icr_scene *s, int32_t *node_ids, double *q_free, double *p, double *lambda,
                                double *C, double *f, int8_t *status, double *WH);

/*
 * Host-side analysis only (no device needed): nested-dissection ordering and
 * supernodal symbolic structure of the mesh graph, for inspection and tests.
 *   perm [N] out: perm[new] = old node id.
 *   sup  [nsup_cap*4] out: per supernode (postorder) {first permuted node,
 *        node count, parent (-1 root), first descendant}.
 *   rows [rows_cap] out: below-row permuted node ids, concatenated per
 *        supernode in postorder; rows_ptr [nsup_cap+1] out.
 *   *nsup_out, *nrows_out: sizes needed (arrays untouched if caps too small).
 */
icr_status icr_analyze(const double *nodes, int32_t N, const int32_t *tets, int32_t T, int32_t *perm,
                       int32_t *sup, int32_t nsup_cap, int32_t *rows_ptr, int32_t *rows, int32_t rows_cap,
                       int32_t *nsup_out, int32_t *nrows_out);

/* ---------------------------------------------------------------------------
 * Serving: many independent scenes stepped concurrently on one GPU.
 *
 * A server holds admitted scenes (each keeps its factor, W_H buffers and
 * warm start resident) and a FIFO of step requests.  icr_server_poll starts
 * queued requests on free slots (one HIP stream per slot) as soon as a slot
 * frees up (continuous admission), and returns the requests that completed.
 * The startable requests (the oldest queued ones whose scenes have nothing
 * in flight) are spread evenly over the free slots, at most `group` per slot
 * (icr_server_set_batching); a slot runs its group in its stream's order: the requests whose Newton loops allow it
 * (fast scheme, ICR_FP64, no pair contacts, at most 512 contacts, untimed)
 * run their steps up to the Newton loop, then all their Newton loops
 * (Algorithm 3, steps 1-4) in one persistent launch with one workgroup per
 * scene, then the rest of their steps; other requests run icr_step(scene,
 * obstacle, opts, NULL) whole.  The slot is free again when its whole group
 * completed.  Requests of one scene run in submission order; those of
 * different scenes overlap on the device.  Either way a request's results
 * are bit for bit those of the same step run alone.
 * Scenes are admitted against a device-memory budget: admission first
 * allocates every buffer the scene's steps use (icr_reserve for the contacts
 * reserved before, else for its candidate count) and charges the scene's
 * library-owned device bytes (icr_factor_info.device_bytes) after that, so
 * that served steps allocate nothing; the sum may not exceed the budget.
 * Not thread-safe; the server does not own the scenes (destroy them after
 * the server).
 * ------------------------------------------------------------------------- */
typedef struct icr_server icr_server;

typedef struct {
  uint64_t tag;        /* the caller's request id (icr_server_submit) */
  int32_t scene;       /* scene id (icr_server_admit) */
  int32_t status;      /* icr_status of the step: ICR_OK; ICR_WARN_NOT_CONVERGED when the request's
                          tol > 0 and a Newton iteration's PGS ended with eps > tol (tol = 0 asks for a
                          fixed sweep count); or the error of a launch that failed (the scene stays
                          admitted and later requests run) */
  double latency_ms;   /* submission -> completion seen by icr_server_poll (host clock) */
  double queue_ms;     /* submission -> launch */
} icr_completion;

/* slots in [1, 32]; hbm_budget in bytes (> 0).  HIP spreads streams over the
 * process's hardware queues (GPU_MAX_HW_QUEUES, 4 unless set): slots beyond
 * that count share a queue and their steps run one after another, so a
 * server with more than 4 slots wants the variable set to at least `slots`
 * before the process's first HIP call. */
icr_status icr_server_create(icr_server **out, int64_t hbm_budget, int32_t slots);
void icr_server_destroy(icr_server *srv); /* waits for the requests in flight */
const char *icr_server_last_error(const icr_server *srv);
/* group in [1, 64] (8 by default): requests a slot takes per round, their
 * Newton loops batched into one launch where the step allows it; group = 0:
 * one request per slot, run as icr_step whole (the Newton loop then runs as
 * the scene's own kernels, in a captured graph when opts.graph is set).  The
 * batched loop computes every value as the per-scene kernels do, in the same
 * order, so both forms give identical results.  With group > 1 and
 * max_wait_ms > 0 (0 by default: start at once), fewer startable requests
 * than `group` wait until the oldest of them has waited max_wait_ms, or until
 * no slot runs.  Applies to
 * the rounds that start after the call.  ICR_E_ARG for group outside
 * [0, 64] or a negative or non-finite max_wait_ms. */
icr_status icr_server_set_batching(icr_server *srv, int32_t group, double max_wait_ms);

/* Admit a factored scene with candidates set; *scene_id receives its id.
 * Synchronises the device once (the scene's set-up work must be complete
 * before its steps run on the slot streams).  ICR_E_OOM (nothing admitted;
 * the scene keeps the buffers reserved for it) when it would exceed the
 * budget.  A request runs on a slot's stream; when it completes (or its
 * launch fails) the scene is set back to the stream it had at admission, so
 * that direct calls on the scene after its requests have completed
 * (icr_destroy included) run on its own stream.  Admission also turns the
 * scene's second stream off (icr_set_overlap(scene, 0)). */
icr_status icr_server_admit(icr_server *srv, icr_scene *scene, int32_t *scene_id);
/* Remove an idle scene (no request queued or in flight: else ICR_E_STATE);
 * its bytes return to the budget.  The scene itself is not destroyed. */
icr_status icr_server_evict(icr_server *srv, int32_t scene_id);
/* Device bytes currently admitted (host out). */
icr_status icr_server_used(const icr_server *srv, int64_t *bytes);

/* Queue one time step of an admitted scene (obstacle and options copied).
 * The request is checked as icr_step checks it (same error codes) and
 * refused with ICR_E_ARG when n_contacts exceeds the contacts reserved at
 * admission, or when it asks for ICR_FP32_IR and the scene was not reserved
 * for that precision (icr_reserve) before admission. */
icr_status icr_server_submit(icr_server *srv, int32_t scene_id, const icr_obstacle *obs, const icr_step_opts *opt,
                             uint64_t tag);
/* Launch what fits on free slots, then collect completed requests into
 * out[0 .. cap); *n_out receives their count.  With wait != 0 it blocks until
 * at least one request completes (returns at once if nothing is queued or in
 * flight).  *pending_out (may be NULL) receives queued + in-flight requests. */
icr_status icr_server_poll(icr_server *srv, icr_completion *out, int32_t cap, int32_t *n_out, int32_t wait,
                           int32_t *pending_out);

#ifdef __cplusplus
}
#endif
#endif /* ICR_H */
