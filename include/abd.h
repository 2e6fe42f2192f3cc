/*
 * libabd -- one worker's local affine-body-dynamics subproblem of the
 * consensus-ADMM method (Sec. 4.1, Eq. 5), solved by projected Newton on
 * one gfx950 GPU.
 *
 * The problem (Eq. 5 with the local objective of Eq. 3 and the incremental
 * potential of Eq. 1):
 *
 *   q_i^{k+1} = argmin_q  sum_b (1/kappa_b) [ 1/2 |q_b - qt_b|^2_{M_b}
 *                                             + h^2 E_orth(q_b) ]
 *                        + h^2 sum_c (1/kappa_c) kappa b(d_c(q))
 *                        + sum_{b shared} rho_b/2 |q_b - z_b + u_b|^2
 *
 * with affine body DoFs q_b = [p (3), A row-major (9)], vertices
 * x = A xbar + p, prediction qt = q^t + h qdot + h^2 M^-1 f_ext, the
 * orthogonality energy E_orth = kappa_A V_b |A A^T - I|_F^2, and the IPC log
 * barrier b(d) = -(d - dhat)^2 ln(d/dhat) on the unsquared distance of
 * point-triangle, edge-edge (mollified) and point-ground pairs.  Every
 * Newton iterate stays penetration free: the step is bounded by additive
 * CCD and accepted by a backtracking line search on the energy.
 *
 * Conventions for every call:
 *  - return value: ABD_OK (0) or a negative ABD_E_* status; the message of
 *    the last failure is abd_last_error(ctx) (owned by the context, valid
 *    until the next call on it);
 *  - every input pointer is a HOST pointer owned by the caller and copied
 *    during the call; every output pointer is a caller-allocated HOST buffer
 *    of the documented size;
 *  - the library owns all device memory (allocated in abd_finalize and
 *    grown on demand), unless the caller binds a workspace of its own
 *    (abd_bind_workspace); work is issued on the bound stream (default: a
 *    stream the library creates) and every call returns after its results
 *    are on the host;
 *  - arrays are FP64 unless stated, array-of-structures: points [n][3],
 *    body states [n][12], 12x12 blocks [n][144] row-major in the DoF order
 *    [p0 p1 p2 A00 A01 A02 A10 A11 A12 A20 A21 A22];
 *  - body ids are dense int32 in insertion order; vertex, triangle and edge
 *    ids are global, in insertion order; a body's edges are its unique
 *    (lo, hi) local vertex pairs sorted lexicographically;
 *  - SI units, y up.
 * A context is not thread safe; distinct contexts are independent.
 */
#ifndef ABD_H
#define ABD_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define ABD_OK 0
#define ABD_E_INVALID_ARG (-1) /* bad argument or call order */
#define ABD_E_MESH (-2)        /* dynamic mesh not closed/oriented */
#define ABD_E_INFEASIBLE (-3)  /* initial state has distance <= 0 */
#define ABD_E_NOCONV (-4)      /* Newton hit max_newton (state = last iterate) */
#define ABD_E_LINESEARCH (-5)  /* line search exhausted */
#define ABD_E_CAPACITY (-6)    /* caller buffer too small (count still set) */
#define ABD_E_DEVICE (-7)      /* HIP runtime or kernel error */
#define ABD_E_OOM (-8)         /* device allocation failed */

/* body kinds */
#define ABD_DYNAMIC 0
#define ABD_STATIC 1

/* precision of the Newton linear algebra */
#define ABD_FP64 0  /* everything FP64 */
#define ABD_MIXED 1 /* Hessian blocks, assembly and the PCG matvec and
                       preconditioner in FP32 (FP32 accumulation); gradient,
                       distances, CCD, energies, PCG residual and dots FP64:
                       the FP64 gradient of every Newton iteration refines
                       the FP32-Hessian steps to the same solution.  A solve
                       in which a problem stops making progress this way
                       (eps_N not halving for 16 Newton iterations, or
                       mixed_switch iterations spent) continues from its
                       current iterate with FP64 Hessians
                       (abd_stats.fp64_fallback, newton_fp32) */

/* candidate kinds */
#define ABD_PT 0 /* point-triangle: (vertex, triangle) */
#define ABD_EE 1 /* edge-edge: (lo edge, hi edge) */
#define ABD_PG 2 /* point-ground: vertex */

/* pair replication rule for kappa_c (Eq. 3) */
#define ABD_PAIRS_ALL_ONE 0     /* kappa_c = 1 for every pair */
#define ABD_PAIRS_BY_SHARED 1   /* kappa_c = 2 if every dynamic body of the
                                   pair is shared, else 1 */

typedef struct abd_params {
  double dt;           /* time step h (s) */
  double dhat;         /* barrier activation distance (m) */
  double kappa;        /* barrier stiffness */
  double kappa_A;      /* orthogonality stiffness (Pa) */
  double gravity[3];   /* m/s^2 */
  double newton_theta; /* stop when |dq|_inf / (h l) < theta (Eq. 8 form) */
  double pcg_eta;      /* PCG stops at |r|_2 <= eta |g|_2 */
  double ground_y;     /* analytic ground plane height (if has_ground) */
  int32_t max_newton, max_pcg, max_ls;
  int32_t has_ground;  /* vertex-ground pairs against y = ground_y */
  int32_t mollify_ee;  /* edge-edge mollifier on |ea x eb|^2 */
  int32_t precision;   /* ABD_FP64 or ABD_MIXED */
  int64_t list_capacity; /* initial capacity of each pair and candidate list;
                            0: the default (64K entries, body pairs at least
                            4 per body).  Lists grow on overflow either way:
                            a small value exercises that growth, a large one
                            avoids it on scenes known to be contact-rich */
  int32_t mixed_switch;  /* ABD_MIXED: Newton iterations after which a solve
                            continues with FP64 Hessians in any case (0: a
                            third of max_newton); a stall (eps_N not halving
                            for 16 iterations) switches earlier */
  int32_t deterministic; /* 1: every local solve is bit-reproducible: the
                            barrier gradient and Hessian sums and the
                            line-search energy sums are accumulated exactly
                            (fixed point on the grid 2^-128, independent of
                            the order in which terms arrive) and rounded
                            once, block rows are in ascending neighbour
                            order and the PCG is the problem-local
                            one-exchange form (abd_finalize fails with
                            INVALID_ARG when a problem exceeds what that
                            form holds resident).  A barrier term of
                            magnitude 2^100 or more ends the solve with
                            DEVICE.  0 (default): FP64/FP32 atomics, last
                            bits may vary between runs.  Not available to
                            abd_local_solve_static (INVALID_ARG); the
                            consensus kernels keep their atomics */
} abd_params;

typedef struct abd_stats {
  int32_t newton_iters;    /* linear solves performed */
  int32_t pcg_iters_total;
  int32_t ls_halvings;
  int32_t status;
  double final_eps_N;      /* |dq|_inf / (h l) of the last direction */
  double min_alpha;        /* smallest accepted step */
  double min_dist;         /* smallest candidate distance seen */
  double scene_scale;      /* l: bounding-box diagonal at step start */
  int64_t n_cand_pt, n_cand_ee, n_cand_pg, n_active; /* last iteration */
  double t_solve_ms;       /* wall time of the call */
  /* broad-phase sizes of the last pass: body pairs and chunk pairs of the
   * static phase (at q) and of the swept phase (over q -> q + dq) */
  int64_t n_body_pairs, n_chunk_pairs, n_body_pairs_swept,
      n_chunk_pairs_swept;
  /* mixed precision: 1 if a problem stopped making progress with FP32
   * Hessians and the solve continued from its current iterate with FP64
   * Hessians (no work is repeated); newton_fp32 of the newton_iters were
   * taken with FP32 Hessians */
  int32_t fp64_fallback;
  int32_t newton_fp32;
} abd_stats;

typedef struct abd_ctx abd_ctx;

/* Create a context on the current HIP device. */
int abd_create(abd_ctx** out, const abd_params* p);
void abd_destroy(abd_ctx* ctx);
const char* abd_last_error(const abd_ctx* ctx);

/* Add a body before abd_finalize.  xbar: [nv][3] rest vertices; tris:
 * [nt][3] local vertex ids (outward oriented and closed for DYNAMIC);
 * density in kg/m^3; q0, qdot0: [12] initial state (qdot0 may be NULL);
 * kind: ABD_DYNAMIC or ABD_STATIC (no DoFs, fixed at q0).  Mass properties
 * (Mhat = int rho [1 xbar^T; xbar xbar xbar^T] dV and volume) come from the
 * mesh.  *body_id receives the dense id.  Errors: INVALID_ARG, MESH. */
int abd_add_body(abd_ctx* ctx, const double* xbar, int32_t nv,
                 const int32_t* tris, int32_t nt, double density,
                 const double* q0, const double* qdot0, int32_t kind,
                 int32_t* body_id);

/* Upload the scene to the device and check that the initial state is
 * feasible: every candidate distance > 0 and no edge of one body crossing a
 * triangle of another.  Errors: INVALID_ARG, INFEASIBLE, OOM, DEVICE. */
int abd_finalize(abd_ctx* ctx);

/* sizes[0..3] = bodies, vertices, triangles, edges */
int abd_sizes(const abd_ctx* ctx, int64_t* sizes);

/* Consensus data of the shared bodies B_{i,d} (Eq. 5): ids [n]; z, u
 * [n][12]; rho [n] >= 0; kappa_b [n] >= 1 (replica count, Eq. 3).  Replaces
 * the previous set; n = 0 gives the monolithic problem.  Callable every
 * ADMM iteration.  Errors: INVALID_ARG (bad id, non-finite z/u, rho < 0). */
int abd_set_shared(abd_ctx* ctx, const int32_t* ids, int32_t n,
                   const double* z, const double* u, const double* rho,
                   const int32_t* kappa_b);

/* kappa_c rule: ABD_PAIRS_ALL_ONE (default) or ABD_PAIRS_BY_SHARED. */
int abd_set_pair_replication(abd_ctx* ctx, int32_t mode);

/* Start a time step (Eq. 1): store q^t, form the prediction q-tilde and
 * the scene scale l (bounding-box diagonal of the dynamic vertices). */
int abd_begin_step(abd_ctx* ctx);

/* Solve Eq. 5 from the current q (warm start).  out may be NULL.
 * Errors: NOCONV, LINESEARCH, DEVICE, OOM. */
int abd_local_solve(abd_ctx* ctx, abd_stats* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as abd_local_solve, with the same results, that allocates nothing.
 * The per-pass lists of the solve (body pairs with their off-diagonal
 * blocks and block-row columns, chunk pairs, candidate and active pairs)
 * live in a static device array of the library (64 MiB on every GPU it
 * runs on, held until the process ends) instead of the context's buffers,
 * at fixed maximum sizes: 32768 body pairs, 262144 chunk pairs, 524288
 * point-triangle and 524288 edge-edge candidates, 262144 point-ground
 * candidates, 262144 active pairs and 16384 pairs whose CCD continues in
 * blocked steps.  A solve whose lists would exceed a
 * maximum stops with ABD_E_CAPACITY (abd_last_error names the list and
 * its maximum; q is the last accepted iterate, feasible like every
 * iterate) instead of growing them.  Passes are launched directly (no
 * graph replay) and stage timing is off during the call; no device memory
 * is allocated or freed.  The context's own buffers must exist
 * (abd_finalize).  The context's device must be current (INVALID_ARG
 * otherwise).  All calls on one GPU share its array: two such calls that
 * overlap in time on one GPU (from several threads, or on contexts whose
 * streams run concurrently) race and give undefined results.  Errors:
 * NOCONV, LINESEARCH, CAPACITY, DEVICE, INVALID_ARG. */
int abd_local_solve_static(abd_ctx* ctx, abd_stats* out);

/* Finish the step: qdot = (q - q^t) / h. */
int abd_end_step(abd_ctx* ctx);

/* State [B][12] (checkpoint / resume); either pointer may be NULL.
 * abd_set_state ignores static bodies. */
int abd_get_state(const abd_ctx* ctx, double* q, double* qdot);
int abd_set_state(abd_ctx* ctx, const double* q, const double* qdot);
/* q-tilde [B][12] of the current step */
int abd_get_qtilde(const abd_ctx* ctx, double* qtilde);
/* Prescribe the step-start data directly: q^t, q-tilde [B][12] and the
 * scene scale l (for lock-step comparisons from a shared start state). */
int abd_set_step(abd_ctx* ctx, const double* qt, const double* qtilde,
                 double scale);

/* Work on a caller stream (a hipStream_t; NULL = the legacy null stream,
 * on which Newton passes are launched directly instead of replayed from
 * captured graphs). */
int abd_set_stream(abd_ctx* ctx, void* hip_stream);

/* Caller-owned device memory for the context's buffers (the caller's
 * allocator, e.g. PyTorch's, owns the memory; the library sub-allocates).
 * dev_ptr: device memory of the current device, bytes >= 256; it must stay
 * valid and untouched by the caller until abd_destroy.  Bind once, after
 * abd_create and before abd_finalize: from then on every buffer of the
 * context (scene data, state, lists, Hessian blocks, PCG vectors, test-hook
 * and autotune temporaries) is taken from it, 256-byte aligned, as a stack;
 * lists grown during a solve take fresh space above the lists they replace,
 * whose space comes back only once nothing above it is live.  Pinned host
 * counters, events and graphs, and the objects of abd_batch_* and
 * abd_consensus_*, are allocated by the library as before.  When the
 * workspace runs out the call that needed memory fails with ABD_E_OOM and
 * abd_last_error names the size asked for; the context keeps its state.
 * Errors: INVALID_ARG (NULL context or pointer, bytes < 256, pointer not
 * device memory of the current device, context finalized or already
 * bound). */
int abd_bind_workspace(abd_ctx* ctx, void* dev_ptr, size_t bytes);

/* info[3]: usable workspace bytes (0 when none is bound), bytes in use
 * (top of the stack), and the most ever in use. */
int abd_workspace_info(const abd_ctx* ctx, int64_t* info);

/* ---- launch tuning ---- */
#define ABD_PCG_TWO_BARRIER 0 /* textbook PCG: two grid barriers per iteration */
#define ABD_PCG_PIPELINED 1   /* single-reduction PCG: one grid barrier */
#define ABD_PCG_LOCAL 2       /* textbook PCG, blocks wait only for the blocks
                                 of their own problems; deterministic dot
                                 products (one block per 16 bodies; scenes
                                 too large to keep every block resident use
                                 TWO_BARRIER) */
#define ABD_PCG_LOCAL1 3      /* as LOCAL, one exchange per iteration
                                 (Chronopoulos-Gear recurrences; u and w
                                 recomputed exactly every iteration) */
typedef struct abd_tuning {
  int32_t pcg_variant;     /* ABD_PCG_* (default LOCAL1; the pipelined
                              form carries u, s and t by recurrences, which
                              can stall short of a very tight tolerance such
                              as eta = 1e-12 on stiff contact systems) */
  int32_t pcg_blocks;      /* blocks of the persistent PCG launch, 16 bodies
                              each per pass; 0 = one block per 16 bodies up to
                              the co-resident limit */
  int32_t grid_blocks;     /* blocks of the grid-stride broad-phase, filter and
                              CCD kernels (default 2048) */
  int32_t assemble_blocks; /* blocks of the barrier assembly (default 2048) */
  int32_t use_graphs;      /* replay Newton passes from captured graphs (1)
                              or launch their kernels directly (0, default);
                              batches always launch directly */
  int32_t overlap_body;    /* body terms on a second stream, overlapping the
                              broad phase (1), or in line (0, default) */
  int32_t pcg_coop;        /* reserved, must be 0 (INVALID_ARG otherwise):
                              the PCG is always a plain launch whose grid
                              is at most what the device holds resident
                              at once; its waits are bounded and end in
                              DEVICE should the blocks not be resident
                              together (another process filling the GPU) */
  int32_t body_pairs;      /* body-pair broad phase, the same pairs either
                              way: ABD_BODY_PAIRS_AUTO (default: every pair
                              of each problem while those number at most
                              2^21, else sort and sweep), ABD_BODY_PAIRS_ALL
                              (INVALID_ARG beyond 2^27 pairs) or
                              ABD_BODY_PAIRS_SWEEP */
  int32_t pcg_launch_groups; /* problem-local PCG forms: at most this many
                              16-body groups per launch (0: as many as the
                              device holds resident at once); problems that
                              share no group may run in separate launches
                              one after another; a problem needing more
                              groups runs the two-barrier form */
  int32_t label_rows;      /* component labelling: at most this many bodies
                              per workgroup of whole problems (0: 12288,
                              also the largest value used); a scene of at
                              most this many bodies builds its block rows
                              and labels in one workgroup; a problem of
                              more bodies leaves every component to the PCG */
} abd_tuning;
#define ABD_BODY_PAIRS_AUTO 0
#define ABD_BODY_PAIRS_ALL 1
#define ABD_BODY_PAIRS_SWEEP 2

/* Read or replace the launch settings of a finalized context.  Settings
 * change launch shapes and the PCG recurrence, not the system solved:
 * any setting gives a solution within the stated tolerances.
 * INVALID_ARG for an unknown variant or negative sizes. */
int abd_get_tuning(abd_ctx* ctx, abd_tuning* out);
int abd_set_tuning(abd_ctx* ctx, const abd_tuning* t);

/* Autotuner: from the current state, run the next time step's local solve
 * (prediction, solve) once per candidate setting, each from the same saved
 * state and timed on the device, restore the state, and keep the fastest
 * setting that solved the step (returned in out, may be NULL).  The search
 * is coordinate-wise: PCG form and grid first (the pipelined form only for
 * pcg_eta >= 1e-6), then the grid-stride grid, then the assembly grid.
 * Costs about 2 x trials local solves. */
int abd_autotune(abd_ctx* ctx, abd_tuning* out);

/* ---- batching: many local problems in the same launches ---- */
typedef struct abd_batch abd_batch;

/* Merge n finalized contexts with identical parameters and pair
 * replication rule into one device scene (for instance the subdomains of
 * several workers, or independent small scenes).  Problems never interact:
 * no candidate pair joins two of them, and each keeps its own PCG
 * recurrence, Newton stop test (with its own scene scale) and line search,
 * so a batch solve gives what abd_local_solve would give on each context.
 * The contexts stay usable and keep their own state.  Errors: INVALID_ARG
 * (not finalized, parameters differ), OOM, DEVICE. */
int abd_batch_create(abd_ctx** ctxs, int32_t n, abd_batch** out);

/* Solve Eq. 5 for every problem of the batch in one device loop: the
 * current q, q^t, q-tilde, qdot, scene scale and shared-body data of each
 * context are gathered in, every Newton pass runs all problems in the same
 * kernel launches (direct launches; the batch takes the first context's
 * tuning except use_graphs, which it ignores), and the solutions are
 * scattered back to the contexts.  out: [n] stats (may be NULL).  Returns
 * ABD_OK or the first non-OK problem status. */
int abd_batch_run(abd_batch* batch, abd_stats* out);

/* One-call form: solve the contexts ctxs[0..n) together.  The merged
 * scene is built on the first call and kept by ctxs[0] for later calls with
 * the same contexts in the same order (rebuilt when the list or a pair
 * replication rule changes; released with ctxs[0]).  Same requirements and
 * results as abd_batch_create + abd_batch_run. */
int abd_batch_solve(abd_ctx** ctxs, int32_t n, abd_stats* out);
void abd_batch_destroy(abd_batch* batch);

/* ---- consensus ADMM over the subdomains of a batch ---- */
/* The problems of a batch are the workers of Sec. 4.1 (subdomains of one
 * scene, each a context holding its own copies of the shared bodies).  A
 * consensus object links the replicas of every shared body and runs the
 * consensus side on the device: the z-update (Eq. 6), the dual update
 * (Eq. 7), the residuals (Eqs. 9-10), the penalty rule (Eq. 12) with the
 * mass-aware start (Sec. 4.3) and the merge check and merge of Sec. 4.2.
 * Replica data moves between the problems through device memory. */
typedef struct abd_consensus abd_consensus;

typedef struct abd_admm_params {
  double beta;      /* rho0 = beta * m_b (Sec. 4.3); <= 0: rho0 = rho_fixed */
  double rho_fixed;
  double tau, mu;   /* Eq. 12 (2, 5) */
  double sigma_min, sigma_max; /* rho kept in [sigma_min, sigma_max] * rho0 */
  double scale;     /* l of Eq. 8; <= 0: the largest problem scene scale */
  int32_t adapt_rho;   /* apply Eq. 12 between iterations */
  int32_t merge_check; /* convergence also needs TOI = 1 toward the merge */
  int32_t max_iters;   /* ADMM iterations per time step (K of Alg. 1) */
} abd_admm_params;

typedef struct abd_admm_report {
  int32_t iters;       /* local solves per problem in this time step */
  int32_t converged;   /* the three tests of Eq. 8 held (and the merge check) */
  int32_t merge_ok;    /* every problem reached TOI = 1 toward its merge */
  int32_t newton_iters_total; /* over all problems and iterations */
  double eps_newton;   /* max over problems of |dq|_inf / (h l_p) */
  double r_inf, s_inf; /* Eqs. 9-10 divided by h l */
  double min_toi;      /* smallest merge-check TOI over problems */
} abd_admm_report;

/* Replica k is body rep_body[k] of problem rep_prob[k] (a dynamic body)
 * and a copy of shared body rep_group[k] in [0, n_groups); every group
 * needs a replica, and a problem holds at most one replica per group.
 * kappa_b of each replica is its group's replica count.  The batch keeps
 * using these as its shared data (abd_set_shared on its contexts no longer
 * reaches the batch).  Errors: INVALID_ARG, OOM, DEVICE. */
int abd_consensus_create(abd_batch* bt, const int32_t* rep_prob,
                         const int32_t* rep_body, const int32_t* rep_group,
                         int32_t n_rep, int32_t n_groups,
                         const abd_admm_params* ap, abd_consensus** out);
void abd_consensus_destroy(abd_consensus* c);

/* Alg. 1 start of a time step, after abd_begin_step on every context:
 * z = q-tilde of the replicas, u = 0 (rho keeps its adapted values). */
int abd_consensus_begin(abd_consensus* c);

/* After a batch local solve: Eqs. 6, 7, 9, 10 on the device, the merge
 * check if enabled (ACCD of every problem from its q to its merged state),
 * and the report (may be NULL). */
int abd_consensus_update(abd_consensus* c, abd_admm_report* rep);

/* Eq. 12 with the residuals of the last update. */
int abd_consensus_adapt(abd_consensus* c);

/* Sec. 4.2 merge: every replica takes its group's z; written back to the
 * contexts. */
int abd_consensus_merge(abd_consensus* c);

/* Copies out z [n_groups*12], u [n_rep*12], rho [n_rep] (any may be NULL). */
int abd_consensus_get(abd_consensus* c, double* z, double* u, double* rho);

/* One time step of Alg. 1 for every problem: begin_step on each context,
 * z = q-tilde and u = 0, then up to max_iters rounds of batch local solve
 * and consensus update (stopping when Eq. 8 and the merge check hold, and
 * adapting rho between rounds), the merge, and end_step on each context.
 * Returns ABD_OK, ABD_E_NOCONV (no convergence in max_iters; the replicas
 * keep their local solutions) or the first failing local solve's status. */
int abd_admm_step(abd_consensus* c, abd_admm_report* rep);

/* ---- inspection hooks (used for parity; not needed to simulate) ---- */

/* Vertex positions x = A xbar + p [V][3] at q (NULL = current q) and, if
 * dq and dx are given, the displacements dx = dA xbar + dp [V][3]; these
 * are exactly the values the broad phase and CCD use. */
int abd_get_vertices(abd_ctx* ctx, const double* q, const double* dq,
                     double* x, double* dx);

/* Candidate pairs at the current q: static boxes, or swept boxes over
 * [x, x + dx] when dq != NULL.  A pair (P, Q) of primitives of different
 * bodies, at least one dynamic, is a candidate iff on every axis
 * lo_P <= hi_Q + dhat and lo_Q <= hi_P + dhat, with exact min/max boxes.
 * Output sorted lexicographically: PT and EE write [count][2] int32, PG
 * writes [count].  If count > cap nothing is written and CAPACITY is
 * returned with *count set. */
int abd_export_candidates(abd_ctx* ctx, int32_t kind, const double* dq,
                          int32_t* out, int64_t cap, int64_t* count);

/* Energy, gradient [B][12] and Hessian blocks at q (static bodies get a
 * zero gradient and an identity block).  Off-diagonal blocks (a < b, rows
 * a's DoFs) for body pairs with at least one active contact, sorted by
 * (a, b): off_ij [n][2], Hoff [n][144]; CAPACITY if n > cap (n_off set). */
int abd_eval(abd_ctx* ctx, const double* q, double* E, double* g,
             double* Hdiag, int64_t cap, int64_t* n_off, int32_t* off_ij,
             double* Hoff, int64_t* n_active);

/* One Newton direction at the current q: dq [B][12] solving H dq = -g. */
int abd_direction(abd_ctx* ctx, double* dq, int32_t* pcg_iters);

/* alpha_max = min(1, min over swept candidates of the additive-CCD
 * time of impact) for the step dq [B][12] from the current q (the CCD
 * filter of the line search, Sec. 3 and Alg. 1).  toi (may be NULL): each
 * swept candidate's own time of impact in [0, 1] (1: no impact along the
 * step), in the order abd_export_candidates(kind, dq) lists the pairs: PT,
 * then EE, then PG, each sorted; cap is its capacity (CAPACITY when the
 * candidates do not fit) and *count (may be NULL) receives their number.
 * alpha_max equals min(1, min of toi). */
int abd_ccd(abd_ctx* ctx, const double* dq, double* alpha_max, double* toi,
            int64_t cap, int64_t* count);

/* Penetration check of the current state: *min_dist receives the smallest
 * distance over the candidate pairs at q (pairs whose d-hat inflated boxes
 * meet; +inf when there are none) and *n_cross the number of edges of one
 * body crossing a triangle of another (strictly, by signed volumes).  The
 * state is penetration free iff *n_cross == 0 and *min_dist > 0. */
int abd_check_penetration(abd_ctx* ctx, int64_t* n_cross, double* min_dist);

/* E(q + alpha dq) - E(q) at the current q, summed term by term. */
int abd_energy_delta(abd_ctx* ctx, const double* dq, double alpha,
                     double* dE);

/* Per-stage device timing with HIP events on the bound stream.  Stage ids:
 * 0 body terms, 1 broad phase, 2 barrier assembly (distance filter and
 * assembly), 3 PCG, 4 CCD, 5 line search, 6 other (block rows, block
 * inverses and the direct component solves), 7 the assembly kernel alone
 * (ABD_TIMING_ASM).  abd_get_timing returns the summed milliseconds,
 * the number of timed launches and the algorithmic bytes those launches
 * had to move (sizes as launched).  Modes: ABD_TIMING_OFF (default);
 * ABD_TIMING_ALL times every stage, which replaces the captured graphs by
 * direct launches; ABD_TIMING_PCG times the PCG launch of every fourth
 * pass of the device loop (those passes run as two captured halves around
 * it, the others as whole captured passes), so the solve keeps its normal
 * launch path.  Other values: INVALID_ARG. */
#define ABD_TIMING_OFF 0
#define ABD_TIMING_ALL 1
#define ABD_TIMING_PCG 2
#define ABD_TIMING_ASM 3 /* as ABD_TIMING_PCG for the assembly kernel (stage 7,
                            with its algorithmic bytes and flops); the
                            sampled passes launch their kernels directly */
int abd_set_timing(abd_ctx* ctx, int32_t on);
int abd_get_timing(abd_ctx* ctx, int32_t stage, double* ms,
                   int64_t* launches, double* bytes);
int abd_reset_timing(abd_ctx* ctx);
/* Algorithmic FP64 flops of the timed launches of a stage (counted for the
 * barrier stage 2 with ABD_TIMING_ALL and the assembly kernel, stage 7,
 * with ABD_TIMING_ASM; 0 for the others).  With the bytes
 * of abd_get_timing this places stage 2 against both the HBM and the FP64
 * roofline.  Per pass: about 100 flops per candidate distance and 22,300
 * per active point-triangle or edge-edge pair (distance derivatives, 9x9
 * PSD projection, mapping to three body blocks).  The stage's bytes count
 * each access once with no cache reuse: candidate entries and their four
 * vertices' rest positions and body ids, active-pair entries, three 12x12
 * blocks and two 12-gradients read and written per active pair, and the
 * off-diagonal block cleared per body pair. */
int abd_get_timing_flops(abd_ctx* ctx, int32_t stage, double* flops);

/* ---- load balancing of the plane between two workers (Sec. 5.2) ----
 * A discrete-time PD controller on the workers' smoothed frame times moves
 * the plane p_12 + s n_12 that separates worker 1 from worker 2 (n_12 from
 * 1 to 2): Eq. 13, T = (eta - 1) / (eta + 1) with eta = tau_1 / tau_2 (0
 * when balanced, > 0 when worker 1 is slower), and Eq. 14, the shift
 * dp = k_p T + k_d (T - T_prev), applied by the caller as p_12 += dp n_12.
 * The times are smoothed as tau = (1 - smooth) tau + smooth t, starting
 * from the first frame's times; the first frame has no derivative term.
 * As printed, a controller that shrinks the slower worker's side has
 * negative gains in this orientation.  Host-only: no device is used. */
typedef struct abd_balance {
  double k_p, k_d;  /* gains, in plane-shift length per unit imbalance */
  double smooth;    /* weight of the newest frame time, in (0, 1] */
  double tau[2];    /* state: smoothed times of workers 1 and 2 */
  double T_prev;    /* state: imbalance of the previous frame */
  int32_t frames;   /* state: frames seen; 0 starts the controller afresh */
  int32_t pad_;
} abd_balance;

/* One frame: the compute times t1, t2 > 0 of workers 1 and 2 update the
 * state of *b and *dp receives the plane shift of Eq. 14.  Errors:
 * INVALID_ARG (NULL pointer, a time not finite and positive, smooth outside
 * (0, 1], a gain not finite); the state is then left as it was. */
int abd_balance_update(abd_balance* b, double t1, double t2, double* dp);

#ifdef __cplusplus
}
#endif
#endif
