/*
 * adafac.h -- C ABI of the MI355X (gfx950) additively damped asynchronous FAC solver.
 *
 * The library solves  -div(eps grad u) = f  on the unit square (d = 2) or cube
 * (d = 3) with u = 0 on the boundary (problem statement, Sec. 1 of Murray &
 * Weinzierl, "Stabilised asynchronous fast adaptive composite multigrid using
 * additive damping", arXiv:1903.10367), discretised with d-linear finite
 * elements on the levels of a 3:1 spacetree (Sec. 2.1), and iterates the
 * additive adAFAC cycle of eq. (adaFACx) / Algorithm 1 (Sec. 3.1): every level
 * takes one damped Jacobi step, the coarse levels see the FAS right-hand side
 * of eq. (fas-with-htmg) (Sec. 2.4), and every level below the finest solves
 * the auxiliary damping equation with the smoothed restriction R~ (Sec. 3.2).
 *
 * Conventions shared by every entry point
 *  - Return value: ADAFAC_OK (0) or one of the ADAFAC_E* codes below.  No C++
 *    exception crosses the ABI.  adafac_last_error() gives a message for the
 *    last failing call on a context.
 *  - Host arrays are read (or written) during the call only; the caller keeps
 *    ownership and may free them afterwards.
 *  - Device memory: the caller allocates ONE workspace of at least
 *    adafac_workspace_bytes() bytes on the GPU (any allocator, 256-byte
 *    aligned), passes it to adafac_bind() and keeps it alive until
 *    adafac_destroy() or the next adafac_bind().  The library sub-allocates
 *    all level arrays inside it and never calls hipMalloc while cycling.
 *  - All GPU work is enqueued on the hipStream_t given to adafac_bind().
 *    adafac_cycle() returns without synchronising; adafac_residual(),
 *    adafac_solve(), adafac_get_solution() and adafac_get_level() synchronise
 *    that stream.
 *  - Lattice arrays are C order with x fastest: entry (x, y[, z]) of a level
 *    with n = 3^l cells per axis sits at x + (n+1)*(y + (n+1)*z).
 *  - A context is used by one host thread at a time.
 */
#ifndef ADAFAC_H
#define ADAFAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define ADAFAC_OK 0
#define ADAFAC_EINVAL 1      /* bad argument: dims, levels, sizes, eps <= 0, non-finite data */
#define ADAFAC_ESTATE 2      /* entry point called out of order */
#define ADAFAC_ENOMEM 3      /* workspace too small */
#define ADAFAC_EDEVICE 4     /* a HIP runtime call failed (message kept) */
#define ADAFAC_EDIVERGED 5   /* residual became NaN/Inf or grew beyond 1e3 x its initial value */
#define ADAFAC_EUNSUPPORTED 7/* option combination not implemented */

/* inter-grid transfers (Sec. 2.5; the switch of Sec. 3.2) */
#define ADAFAC_TRANSFER_DLINEAR 0
#define ADAFAC_TRANSFER_BOXMG 1
/* damping of the additive corrections (Sec. 3.2, Sec. 5.1) */
#define ADAFAC_DAMP_JAC 0    /* adAFAC-Jac: auxiliary equation with R~ one level coarser */
#define ADAFAC_DAMP_PI 1     /* adAFAC-PI: c~_l = P I c_l */
#define ADAFAC_DAMP_NONE 2   /* plain additive multigrid, eq. (additive-mg) */
#define ADAFAC_DAMP_EXP 3    /* exponential damping omega_hat^(L-l) */
/* the smoothed restriction R~ = omega R A M^-1 truncated to P's support (Sec. 3.2) */
#define ADAFAC_RTILDE_CONST_EPS1 0 /* from the eps = 1 operator, the same on every level */
#define ADAFAC_RTILDE_OPERATOR 1   /* omega trunc(P^T A_l D_l^-1) of the level's own operator and
                                      transfer, stored per coarse vertex (5^dim weights; the
                                      storage the paper's Sec. 4.1 notes); uniform trees only, and
                                      it runs the one-kernel-per-step form of the cycle */
/* arithmetic of the cycle (spec precision form) */
#define ADAFAC_PREC_FP64 0
#define ADAFAC_PREC_FP32_REFINED 1 /* FP32 cycles inside FP64 defect correction */

typedef struct adafac_ctx adafac_ctx;

typedef struct {
  int transfer;        /* ADAFAC_TRANSFER_* */
  int damping;         /* ADAFAC_DAMP_* */
  int rtilde;          /* ADAFAC_RTILDE_* */
  int precision;       /* ADAFAC_PREC_* */
  int inner_k;         /* FP32_REFINED: cycles per outer FP64 step (>= 1) */
  int fused;           /* 1: single-pass fine sweep with deferred prolongation (default),
                          0: one kernel per step (same iterates; used as a cross-check) */
  double omega;        /* Jacobi damping, 0.6 in Sec. 5 */
  double omega_tilde;  /* auxiliary Jacobi damping (the paper gives no value; default omega) */
  double omega_hat;    /* ADAFAC_DAMP_EXP base */
} adafac_opts;

/* Fill *o with the defaults: DLINEAR, JAC, CONST_EPS1, FP64, inner_k 4, fused,
 * omega = omega_tilde = 0.6, omega_hat = 0.5. */
void adafac_default_opts(adafac_opts* o);

/* Create a context for a d-dimensional (dim = 2 or 3) uniform spacetree whose
 * levels l_min..l_max carry degrees of freedom (Sec. 2.1: levels counted from
 * the root cell, l_max the finest, 1 <= l_min <= l_max; l_max <= 9 for d = 2,
 * l_max <= 6 for d = 3).  Level l has 3^l cells per axis.  *out receives a new
 * context owned by the caller (free with adafac_destroy).  EINVAL on bad
 * arguments. */
int adafac_create(adafac_ctx** out, int dim, int l_min, int l_max);

/* Coefficient eps of the PDE (Sec. 1), piecewise constant on the cells of
 * spacetree level k: blocks_per_axis = 3^k (1 <= 3^k <= 3^l_max), eps holds
 * blocks_per_axis^dim finite values > 0, C order with x fastest.  Default when
 * never called: eps = 1 (Poisson).  EINVAL on bad sizes or values. */
int adafac_set_coefficient_blocks(adafac_ctx* ctx, int blocks_per_axis, const double* eps);

/* Right-hand side f(x) = amplitude exp(-|x - centre|^2 / (2 sigma^2)), a Gaussian
 * source (centre: dim coordinates, x first), evaluated at every vertex where the
 * load is formed; replaces a lattice given with adafac_set_rhs_lattice.  EINVAL on
 * sigma <= 0 or non-finite values. */
int adafac_set_rhs_gaussian(adafac_ctx* ctx, const double* centre, double sigma, double amplitude);

/* Adaptive spacetree (Sec. 2.1): refinement flags of the cells of one level
 * l_min <= level < l_max, over the whole (3^level)^dim cell lattice (C order, x
 * fastest; nonzero = refine).  Flags of cells that do not exist are ignored.
 * Levels without flags refine every existing cell, unless adafac_refine_ball
 * covers them.  With any flags (or a ball) set, the context solves on the
 * adaptive tree: levels are ragged, vertices of a level that are not
 * surrounded by 2^dim cells of that level hang (d-linear interpolation of the
 * next coarser level), and the composite grid is formed by the finest dof of
 * every position.  The cycle works over the hierarchical generating system
 * (Sec. 2.3, eq. (adaFACx)).  Adaptive trees support d-linear transfers,
 * adAFAC-Jac and plain additive damping, in FP64 or FP32_REFINED (the FP64
 * defect of a step is the composite residual of the FP64 iterate; the inner
 * FP32 cycles take it, at the composite dofs, as their leaf loads and start
 * from zero values on every level).  The coefficient blocks must be
 * no finer than the first refined level.  Call build_operators again afterwards.
 * EINVAL on a bad level or size. */
int adafac_set_refinement(adafac_ctx* ctx, int level, const uint8_t* flags, size_t ncells);

/* Feature-based refinement of the Sec. 5 runs (dynamic AMR with a full-multigrid-like
 * start): the refinement flags of the next tree, for levels l_uniform .. l_cap-1 (l_cap >=
 * l_max), concatenated level by level, (3^l)^dim cells each in C order (x fastest); n must be
 * their total.  A flag marks a cell that the next tree refines:
 *  - every cell the current tree refines (levels below l_uniform must be complete and fully
 *    refined: they carry no flags);
 *  - while l_max < l_cap, every cell of level l_max with a face on which the Dirichlet data
 *    are nonzero at every corner (the boundary carrying u = 1);
 *  - the 2^dim cells around each composite dof of a level below l_cap that carries one of the
 *    (approximately) `fraction` largest directional second derivatives of the current iterate
 *    (max over the axes of |u(x + h e_i) - 2 u(x) + u(x - h e_i)| / h^2 on the dof's level):
 *    the values are sorted into 1024 equal bins over [0, their maximum] and whole bins are
 *    taken from the top until they hold at least that fraction of the dofs.
 * *l_new receives the depth of the next tree (1 + its finest refined level, at least l_max).
 * A uniform tree (no flags) needs l_uniform = l_max.  Synchronises.  EINVAL on bad
 * arguments; ESTATE before bind. */
int adafac_amr_mark(adafac_ctx* ctx, double fraction, int l_uniform, int l_cap, uint8_t* flags, size_t n,
                    int* l_new);

/* Start a deeper tree from a shallower one's solution (full-multigrid-like growth): u holds
 * n = (3^l_src + 1)^dim values of the composite function on the finest lattice of a tree of
 * depth l_src <= l_max (adafac_get_solution of that tree); they are interpolated d-linearly
 * onto this tree's finest lattice and set as with adafac_set_solution (boundary entries take
 * this context's Dirichlet data).  EINVAL on bad arguments; ESTATE before bind. */
int adafac_set_solution_coarse(adafac_ctx* ctx, const double* u, size_t n, int l_src);

/* Refine, on levels l_from .. l_max-1 without explicit flags, every existing cell
 * whose closure meets the closed ball |x - centre| <= radius (centre: dim
 * coordinates, x first).  Levels below l_from refine every cell.  radius 0
 * clears the ball.  EINVAL on non-finite values or l_from outside
 * l_min..l_max-1. */
int adafac_refine_ball(adafac_ctx* ctx, const double* centre, double radius, int l_from);

/* Regrid a bound adaptive context (the moving-source workload): prepare a tree
 * refined around the ball (centre, radius, l_from) as adafac_refine_ball, with the
 * right-hand side f (n = (3^l_max + 1)^dim; NULL keeps a Gaussian source and
 * moves its centre to the ball's), and report in *bytes the device workspace it
 * needs.  The bound tree keeps cycling unchanged until
 * adafac_regrid.  EINVAL on bad arguments, ESTATE on a context that is not a
 * bound adaptive one. */
int adafac_regrid_prepare(adafac_ctx* ctx, const double* centre, double radius, int l_from, const double* f,
                          size_t n, size_t* bytes);

/* Move onto the prepared tree.  Its operators and loads are uploaded into
 * dev_workspace (>= the prepared size, 256-byte aligned).  Every dof of the new
 * tree takes the old composite function at its position: kept vertices keep their
 * value, new ones get the d-linear interpolation, and dropped ones vanish.  The
 * residual history and the normalisation by the iterate-0 norm carry over.
 * Afterwards the previous workspace is no longer referenced (the caller may free
 * it).  Synchronises.  ENOMEM if the workspace is too small. */
int adafac_regrid(adafac_ctx* ctx, void* dev_workspace, size_t bytes);

/* Number of composite degrees of freedom of the built tree (0 before
 * build_operators). */
int64_t adafac_composite_dofs(const adafac_ctx* ctx);

/* Right-hand side f sampled at the vertices of the finest level: n must equal
 * (3^l_max + 1)^dim; boundary entries are ignored.  The load vector is
 * b_v = m_v f_v with the lumped mass m_v (h^d on a uniform level).  EINVAL on
 * a wrong n or non-finite values. */
int adafac_set_rhs_lattice(adafac_ctx* ctx, const double* f, size_t n);

/* Build operators and transfers on the host in FP64 (Sec. 2.2, 2.5, 3.2,
 * 4.1): Q1 element operators from eps, BoxMG or d-linear P and R = P^T,
 * Ritz-Galerkin coarse operators, Jacobi diagonals, R~.  opts may be NULL
 * (defaults).  Invalidates a previous bind.  EINVAL / EUNSUPPORTED on bad
 * options. */
int adafac_build_operators(adafac_ctx* ctx, const adafac_opts* opts);

/* Bytes of device workspace the bound context needs (after build_operators). */
int adafac_workspace_bytes(const adafac_ctx* ctx, size_t* bytes);

/* Bind device workspace and stream; uploads operators and the right-hand side
 * and sets u = 0 (iterate 0).  dev_workspace: device pointer, bytes >= the
 * value of adafac_workspace_bytes (else ENOMEM).  hip_stream: a hipStream_t
 * (NULL = the null stream).  EDEVICE if a copy fails. */
int adafac_bind(adafac_ctx* ctx, void* dev_workspace, size_t bytes, void* hip_stream);

/* Inhomogeneous Dirichlet data (the set-ups of Sec. 5: u = 1 on x_2 = 0, 0 on
 * the rest of the boundary): g holds n = (3^l_max + 1)^dim values on the finest
 * vertex lattice; its boundary entries are the values of u there, the interior
 * entries are ignored.  The iterate then carries these values on its boundary
 * vertices (adafac_set_solution keeps them, adafac_get_solution returns them),
 * and every residual sees them, which is the load -A G of the lift u = u_0 + G.
 * On adaptive trees every level's boundary vertices carry the data at their
 * positions (hanging vertices next to the boundary interpolate it; a regrid keeps
 * it), and the composite function's boundary traces are d-linear in the values at
 * the corners of the leaf cells.  FP32_REFINED inner cycles solve for corrections
 * with zero boundary values.  Takes effect at the next adafac_bind (or regrid).
 * EINVAL on a wrong n or a non-finite boundary value.  All-zero boundary values
 * restore the homogeneous problem. */
int adafac_set_dirichlet_lattice(adafac_ctx* ctx, const double* g, size_t n);

/* Size of the library's static device workspace (see adafac_bind_static). */
#define ADAFAC_STATIC_WORKSPACE_BYTES (32u << 20)

/* adafac_bind without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops or harnesses that
 * forbid hipMalloc).  The context is bound to the library's own device array of
 * ADAFAC_STATIC_WORKSPACE_BYTES (32 MiB) on the stream's device; each device
 * that binds holds one such array until the process ends.  Fits 2D hierarchies
 * up to l_max = 6 and 3D up to l_max = 4 (adafac_workspace_bytes tells);
 * ENOMEM, with the needed size in the message, if the hierarchy is larger.
 * Allocates no device memory and makes no allocating HIP or torch call; the
 * workspace is cleared by a kernel, not a memset.  Otherwise as adafac_bind:
 * uploads operators and the load, sets iterate 0, synchronises the stream.
 * The array holds ONE hierarchy per device: binding a second context to it
 * unbinds the first (its later calls return ESTATE), and calls on two contexts
 * that overlap on one device race.  The binding ends at adafac_destroy, the next
 * adafac_bind / adafac_bind_static, or adafac_regrid (which moves the context to
 * the workspace it is given).  EDEVICE if the stream's device cannot be told or
 * the array's address cannot be taken. */
int adafac_bind_static(adafac_ctx* ctx, void* hip_stream);

/* Enqueue ncycles adAFAC cycles.  Cycle n computes the residual norms of
 * iterate n and produces iterate n+1.  FP32_REFINED: ncycles outer steps of
 * FP64 defect correction, each the FP64 defect r = b - A u of the outer
 * iterate (its norms are recorded), inner_k FP32 cycles on A e = r from e = 0,
 * and u <- u + e in FP64 (applied at the start of the next step or when the
 * solution is read).  Non-blocking. */
int adafac_cycle(adafac_ctx* ctx, int ncycles);

/* Iterate until ||r^(n)||_h / ||r^(0)||_h <= rel_tol for the input iterate n
 * of the last cycle run, or max_cycles cycles (outer steps for FP32_REFINED)
 * have run; r^(0) is the residual of the iterate at bind / set_solution.
 * *cycles_done (may be NULL) receives the number of residual evaluations.  FP64
 * form: the cycle that measured iterate n also produced n+1, and the solution
 * afterwards is that iterate.  FP32_REFINED: an outer step measures the FP64
 * defect of its iterate and, unless it met the tolerance, runs inner_k FP32
 * cycles on A e = r; the solution afterwards is the last outer iterate (the one
 * whose FP64 residual met the tolerance when the solve converged).
 * FP64 (uniform hierarchies and adaptive trees) and the one-pass 3D FP32_REFINED
 * form: the cycles (outer steps with their inner cycles) are launched in batches without a host
 * wait (8 first, then as many as the observed contraction predicts, at most 64);
 * the stopping rule is applied on the device where each step's norms are formed,
 * and the launches after the step that met it do nothing, so the step count, the
 * norms and the solution are those of a check after every step.  The environment
 * variable ADAFAC_SOLVE_HOST_CHECK=1 (read at each call) makes the host check
 * after every step instead.
 * Synchronises.  EDIVERGED on NaN/Inf or growth beyond 1e3 x the initial norm. */
int adafac_solve(adafac_ctx* ctx, double rel_tol, int max_cycles, int* cycles_done);

/* Residual norms of iterate `cycle` (0-based, < cycles run since bind):
 * l2h = sqrt(sum_i h^d r_i^2) and linf = max_i |r_i| over the finest-level
 * dofs (Sec. 5, eq. (normalised-residual), before normalisation).  For
 * FP32_REFINED, `cycle` counts outer steps.  Synchronises.  EINVAL if the
 * cycle has not run. */
int adafac_residual(adafac_ctx* ctx, int cycle, double* l2h, double* linf);

/* Number of residual norms recorded so far. */
int adafac_cycles_run(const adafac_ctx* ctx);

/* Copy the current finest-level iterate (full lattice, n = (3^l_max+1)^dim,
 * boundary zero) to host memory u.  Synchronises.  EINVAL on a wrong n. */
int adafac_get_solution(adafac_ctx* ctx, double* u, size_t n);

/* Replace the current iterate (warm start / resume); boundary entries are
 * ignored.  Residual history is cleared.  Synchronises. */
int adafac_set_solution(adafac_ctx* ctx, const double* u, size_t n);

/* Adaptive trees: the finest-lattice values returned by adafac_get_solution are
 * the composite FE function at every finest vertex, and adafac_set_solution takes
 * the values at the dofs' positions from such a lattice.  adafac_get_level
 * returns which = 0 (nodal values u_l, hanging ones interpolated), 1 (b_l, the
 * level hats tested against the composite residual) or 4 (S_l, levels below
 * l_max only) for levels l_min..l_max, on the full level lattice, zero outside
 * the level's cells; under FP32_REFINED only which = 0 (ESTATE otherwise).
 * Under adAFAC-PI with the single-pass sweeps, S_{l_max-1} of a uniform tree
 * holds S_{l_max-1} - I c_{l_max} (the coarse part of the deferred correction).
 *
 * Copy a level array of the last cycle to host memory (inspection and
 * per-step parity checks).  which: 0 = u_l (FAS solution, injected),
 * 1 = b_l (FAS right-hand side), 2 = b~_l (auxiliary right-hand side),
 * 3 = r_l (level residual), 4 = S_l (accumulated correction P^{..}(c - c~)).
 * Levels l_min..l_max-1; n = (3^l+1)^dim.  FP64 form only.  Synchronises. */
int adafac_get_level(adafac_ctx* ctx, int level, int which, double* out, size_t n);

/* Copy a host-side FP64 operator built by adafac_build_operators (no GPU needed):
 * which 0 = the level's 3^dim stencil per vertex (slot index (ox+1) + 3 (oy+1) + 9 (oz+1),
 * n = 3^dim (3^l+1)^dim; Q1 rows from eps for levels whose cells lie inside one eps block,
 * Ritz-Galerkin rows below that, Sec. 2.2), 1 = its diagonal (n = (3^l+1)^dim),
 * 2 = prolongation weights from level l-1 into level l, 2^dim per fine vertex for the
 * corners of the coarse cell floor(x/3) clamped to the last cell (Sec. 2.5; d-linear or
 * BoxMG), n = 2^dim (3^l+1)^dim, l > l_min, 3 = the R~ weights times omega on the 5^dim
 * offsets (Sec. 3.2), n = 5^dim, level ignored, 4 = the OPERATOR R~ restricting level l+1
 * into level l (l_min <= l < l_max): 5^dim weights per level-l vertex, offset index
 * (ox+2) + 5 (oy+2) + 25 (oz+2) of the fine vertex 3v + o, n = 5^dim (3^l+1)^dim (ESTATE
 * unless built with ADAFAC_RTILDE_OPERATOR).  ESTATE before build_operators. */
int adafac_host_operator(const adafac_ctx* ctx, int level, int which, double* out, size_t n);

/* Sum over levels of the dofs (3^l - 1)^dim: the vertex updates of one cycle. */
int64_t adafac_dofs_per_cycle(const adafac_ctx* ctx);

/* Kernel timing of the dominant (finest-level) kernel: when enabled, every
 * launch of it is bracketed by HIP events on the bound stream.  Returns the
 * summed duration in ms and the number of launches since enabling.
 * Synchronises. */
int adafac_set_kernel_timing(adafac_ctx* ctx, int enable);
int adafac_kernel_time(adafac_ctx* ctx, double* total_ms, int* launches);

void adafac_destroy(adafac_ctx* ctx);
const char* adafac_last_error(const adafac_ctx* ctx);

/* Right-hand side given as a function (problem statement, Sec. 1): f(x, user) with x the
 * dim coordinates of a point of the unit square/cube (x first).  It is evaluated, on the
 * calling thread, at every vertex where the lumped load is formed, during adafac_bind (and
 * adafac_regrid when the prepared tree keeps this source); f and user must stay valid until
 * then.  Replaces a lattice or Gaussian source.  EINVAL on a null f. */
int adafac_set_rhs_fn(adafac_ctx* ctx, double (*f)(const double* x, void* user), void* user);

/* Residual norms of iterate `cycle` divided by those of iterate 0 (the iterate at bind or
 * set_solution): the normalised residual of Sec. 5, ||r^(n)||_h / ||r^(0)||_h and
 * max|r^(n)| / max|r^(0)| (0 when the initial norm is 0).  Synchronises.  EINVAL if the
 * cycle has not run. */
int adafac_residual_normalised(adafac_ctx* ctx, int cycle, double* l2h_rel, double* linf_rel);

/* Positions of the composite degrees of freedom (Sec. 2.1: every position's finest dof) in
 * the composite order used by adafac_get_composite / adafac_set_composite: uniform trees the
 * interior vertices of the finest level in lattice order (x fastest); adaptive trees level by
 * level from l_min, each level's composite dofs in lattice order.  xyz (may be NULL) receives
 * dim coordinates per dof (x first), level (may be NULL) the dof's level.  n must equal
 * adafac_composite_dofs.  No GPU involved.  ESTATE before build_operators. */
int adafac_dof_coords(const adafac_ctx* ctx, double* xyz, int* level, size_t n);

/* Current iterate at the composite dofs, in the order of adafac_dof_coords (n =
 * adafac_composite_dofs).  Synchronises.  EINVAL on a wrong n. */
int adafac_get_composite(adafac_ctx* ctx, double* u, size_t n);

/* Replace the iterate by composite dof values in that order (warm start); clears the
 * residual history as adafac_set_solution.  Synchronises.  EINVAL on a wrong n or
 * non-finite values. */
int adafac_set_composite(adafac_ctx* ctx, const double* u, size_t n);

/* Reference streaming copy for roofline context (not part of the method): copies
 * `bytes` from device memory src to device memory dst on `stream` (a hipStream_t;
 * NULL = default stream) with 16-byte non-temporal loads and stores, 1024
 * workgroups of 256 lanes striding over the buffers.  Its rate is the memory
 * rate a plain copy reaches on this GPU, reported beside the sweep's.  src and
 * dst: 16-byte aligned, non-overlapping, owned by the caller; bytes: a multiple
 * of 16.  Asynchronous.  ADAFAC_EINVAL on a null pointer, misalignment or a
 * size that is not a multiple of 16; ADAFAC_EDEVICE if the launch fails. */
int adafac_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

/* ------------------------------------------------------------------------
 * Request server: continuous batching of independent solves (the cycle of
 * Sec. 3.1 run to the stopping criterion of Sec. 5, one hierarchy per request).
 *
 * The caller hands over one device workspace.  A small header of it holds the
 * batched kernel's request table; the rest is a pool that holds the hierarchies
 * of the admitted requests.  Requests wait in a FIFO queue while their host-side
 * set-up (operators) runs on worker threads.  A set-up request is
 * admitted, in arrival order (a later request may pass one that does not fit
 * yet), when an active slot is free and its exact device footprint (the
 * adafac_workspace_bytes of its hierarchy) fits in the free pool.  Each
 * scheduling round (adafac_server_step) does three things:
 *  - harvests the oldest round in flight once it has completed;
 *  - admits, binding on worker threads while the device runs the rounds in
 *    flight;
 *  - enqueues rounds until three are in flight: each advances every active
 *    request by up to cycles_per_round cycles (outer steps for FP32_REFINED).
 *    A request admitted now joins the next round enqueued.
 * All active requests, of any depth and dimension, advance together in shared
 * launches.  A request's cycle is a chain of phases (finest-level residual and
 * Jacobi step, the residual norms and stopping rule, the FAS update of each
 * coarser level, the prolongations back up), each cut into work items of a few
 * thousand vertices; one launch runs the same phase slot of every request's
 * chain, so requests of every size share each launch and the launch count per
 * round (cycles_per_round x the longest chain, times at most three kernel
 * classes) does not grow with the number of requests.  Requests of at least
 * 2^18 finest vertices sweep their finest level in one pass instead, in a
 * launch of their own within the same slot.  A request stops exactly at the
 * first iterate that meets the tolerance (the stopping rule runs on the
 * device; the request's work in a round enqueued after that does nothing).
 * Requests above batch_max_vertices finest vertices (default: none) advance on
 * streams of their own instead and stop at the end of the round in which they
 * converged.  A finished request's solution is copied to host memory (on a
 * worker thread; it reads as running until then) and its device memory and
 * slot are freed (the slot once no round in flight can read it).  A request's
 * arithmetic does not depend on the other requests, so results are the same
 * served alone or in a mix.
 * A server is driven by one host thread.
 * ------------------------------------------------------------------------ */
typedef struct adafac_server adafac_server;

typedef struct {
  int max_active;             /* requests on the device at once, 1..4096 */
  int max_queued;             /* requests waiting for admission (EAGAIN beyond), >= 1 */
  int cycles_per_round;       /* cycles a request advances per round, >= 1 */
  int max_streams;            /* requests on streams of their own advancing concurrently, 1..16 */
  size_t batch_max_vertices;  /* finest-level vertex count up to which a request is batched */
} adafac_server_cfg;

typedef struct {
  int dim, l_min, l_max;      /* as adafac_create */
  int blocks_per_axis;        /* eps blocks per axis (3^k), 0: eps = 1 */
  const double* eps;          /* blocks_per_axis^dim values, copied by submit */
  const double* f;            /* (3^l_max + 1)^dim right-hand side samples, copied by submit */
  adafac_opts opts;           /* as adafac_build_operators */
  double rel_tol;             /* stop when ||r||_h / ||r^0||_h <= rel_tol */
  int max_cycles;             /* cycle (outer step) cap, >= 1 */
} adafac_request;

#define ADAFAC_REQ_QUEUED 0
#define ADAFAC_REQ_RUNNING 1
#define ADAFAC_REQ_CONVERGED 2
#define ADAFAC_REQ_DIVERGED 3
#define ADAFAC_REQ_CAPPED 4       /* max_cycles reached first */
#define ADAFAC_REQ_FAILED 5       /* set-up failed or the request can never fit */
#define ADAFAC_EAGAIN 6           /* queue full: submit again after a round */

typedef struct {
  int status;                 /* ADAFAC_REQ_* */
  int cycles;                 /* cycles (outer steps) run */
  int batched;                /* 1: served by the batched kernel */
  int error;                  /* ADAFAC_E* of a failed set-up, else 0 */
  double l2h0, l2h, linf;     /* ||r^0||_h, and ||r||_h, max |r| of the last measured iterate */
  double t_submit, t_admit, t_done;  /* seconds since adafac_server_create (host clock) */
  size_t footprint;           /* device bytes held while active */
} adafac_result;

/* Defaults: max_active 256, max_queued 4096, cycles_per_round 4, max_streams 4,
 * batch_max_vertices SIZE_MAX (every request batched). */
void adafac_server_default_cfg(adafac_server_cfg* cfg);

/* Create a server over the device workspace [dev_workspace, +bytes) (256-byte
 * aligned), with all work on hip_stream (and max_streams streams of its own for
 * requests above batch_max_vertices).  cfg may be NULL (defaults).  EINVAL on
 * bad values, ENOMEM when the workspace cannot hold the request table and work
 * list. */
int adafac_server_create(const adafac_server_cfg* cfg, void* dev_workspace, size_t bytes, void* hip_stream,
                         adafac_server** out);

/* Queue a request; inputs are copied.  *ticket identifies it.  EINVAL on bad
 * arguments (as adafac_create / set_* / build_operators would report),
 * ADAFAC_EAGAIN when max_queued requests wait already. */
int adafac_server_submit(adafac_server* srv, const adafac_request* req, uint64_t* ticket);

/* One scheduling round: wait (briefly) for the oldest round in flight, harvest
 * finished requests, admit, enqueue rounds up to three in flight.  *active (may
 * be NULL) receives the number of requests on the device after admission,
 * *queued (may be NULL) the number waiting.  Returns after enqueuing. */
int adafac_server_step(adafac_server* srv, int* active, int* queued);

/* State of a ticket (no GPU synchronisation).  EINVAL for an unknown ticket. */
int adafac_server_poll(const adafac_server* srv, uint64_t ticket, adafac_result* out);

/* Copy the solution of a finished request (full finest lattice, n = (3^l_max +
 * 1)^dim) and forget the ticket.  ESTATE while it is queued or running. */
int adafac_server_fetch(adafac_server* srv, uint64_t ticket, double* u, size_t n);

void adafac_server_destroy(adafac_server* srv);
const char* adafac_server_last_error(const adafac_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* ADAFAC_H */
