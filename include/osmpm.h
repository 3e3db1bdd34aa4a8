/*
 * osmpm.h -- C ABI of the MI355X (gfx950) OS-MPM library.
 *
 * The library implements the hot path of the overlapping Schwarz space-time
 * refinement method for the material point method (arXiv 2605.09097):
 * per-subdomain implicit MPM steps (APIC particle-to-grid transfer, the
 * backward-Euler incremental potential minimised by Newton's method whose
 * linear systems are solved by matrix-free conjugate gradients with
 * Hessian-vector products evaluated through the particles, APIC
 * grid-to-particle transfer with the deformation-gradient update and
 * advection) and the coupling of a coarse background domain B with a fine
 * refined domain S (boundary-grid selection, overlap arbitration,
 * mass-weighted projection Pi, interpolation I, temporal interpolation T and
 * the multiplicative Schwarz frame).
 *
 * Conventions (every entry point):
 *  - Pointers named *_host point to host memory; every other array pointer
 *    is a device pointer on the context's device.  Arrays are dense and
 *    row-major: per-particle vectors are [n][d], per-particle matrices
 *    [n][d][d], per-node vectors [n_nodes][d] with nodes numbered x fastest
 *    (i = ix + nx * (iy + ny * iz)).
 *  - The caller owns every buffer it passes; the library copies what it
 *    keeps and never frees caller memory.  Handles own their device storage
 *    until destroyed.
 *  - Work is enqueued on the context's stream and is asynchronous unless the
 *    call returns statistics (those synchronise).  Errors raised on the
 *    device (a particle outside its grid, an inverted particle at an accepted
 *    iterate) are reported by the next synchronising call and by
 *    osmpm_sync().
 *  - Every call returns an osmpm_status; nothing throws across the ABI.
 *    osmpm_last_error() gives a message for the last failure on a context.
 *  - Non-convergence of Newton, CG, the line search or the Schwarz loop is
 *    not an error: it is reported in the statistics with converged = 0.
 *  - A context is used by one host thread at a time.
 */
#ifndef OSMPM_H
#define OSMPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OSMPM_OK = 0,
  OSMPM_E_INVALID_ARG = 1, /* bad argument, detected before any work is queued */
  OSMPM_E_NO_MEMORY = 2,   /* device or pinned-host allocation failed */
  OSMPM_E_DEVICE = 3,      /* HIP runtime error */
  OSMPM_E_OUT_OF_GRID = 4, /* a particle's 3^d stencil left its grid */
  OSMPM_E_INVERTED = 5,    /* det F <= 0 at an iterate that had to be evaluated */
  OSMPM_E_NOT_CONVERGED = 6, /* an iteration with a required tolerance ran out of passes */
  OSMPM_E_STATE = 7        /* call out of order (e.g. solve before P2G) */
} osmpm_status;

typedef enum {
  OSMPM_FP64 = 0,  /* every quantity in double precision */
  OSMPM_MIXED = 1  /* FP32 bulk (P2G, stress blocks, Hessian-vector products, CG
                      iterates) with FP64 Newton residual, line-search energy,
                      CG dot products, Schwarz residuals and positions */
} osmpm_precision;

typedef enum { OSMPM_BC_FIX = 0, OSMPM_BC_TRANSLATE = 1, OSMPM_BC_ROTATE = 2 } osmpm_bc_kind;

/* Instrumented kernels (osmpm_profile_query). */
typedef enum {
  OSMPM_K_CG_ITER = 0,   /* one CG iteration: vector updates, Hessian-vector product
                             through the particles and the inner products */
  OSMPM_K_P2G = 1,       /* APIC particle-to-grid */
  OSMPM_K_G2P = 2,       /* APIC grid-to-particle, F update, advection */
  OSMPM_K_GRAD_HESS = 3, /* gradient and per-particle tangent build */
  OSMPM_K_COUNT = 4
} osmpm_kernel;

typedef struct osmpm_ctx osmpm_ctx;
typedef struct osmpm_domain osmpm_domain;
typedef struct osmpm_batch osmpm_batch;

/* Structured grid of one subdomain on an integer lattice of pitch h0:
 * node i sits at x_i = (origin_q + i * dx_q) * h0 (per axis), so nodes of
 * two domains coincide exactly when their lattice coordinates are equal
 * (the coincidence test of the overlap arbitration, Eq. overlap_donor). */
typedef struct {
  int32_t dim;         /* 2 or 3 */
  int32_t n_nodes[3];  /* nodes per axis; n_nodes[2] = 1 in 2D */
  double h0;           /* lattice pitch */
  int64_t origin_q[3]; /* origin in lattice units */
  int64_t dx_q;        /* grid spacing in lattice units */
} osmpm_grid;

/* Compressible Neo-Hookean material (Sec. 4): Young's modulus and Poisson
 * ratio; Psi = mu/2 (|F|^2 - d) - mu ln J + lam/2 (ln J)^2. */
typedef struct {
  double E, nu;
} osmpm_material;

/* Newton / CG / line-search controls of one implicit solve (Sec. 2.2.5).
 * Newton stops when |g_free| <= max(newton_rtol |g_free(u0)|,
 * newton_atol * sum_i m_i * dx / dt^2) or after max_newton steps; CG stops at
 * |r| <= cg_rtol |r0| or after max_cg iterations; the line search halves at
 * most max_ls times.  project_psd = 1 projects each particle's dP/dF onto the
 * PSD cone.  gravity is the body-force acceleration (f_ext = m_i g).
 * forcing > 0 (an extension; the paper fixes no CG tolerance) loosens CG per
 * Newton step by the Eisenstat-Walker rule (choice 2: eta_k = 0.9
 * (|g_k| / |g_k-1|)^2, safeguarded by 0.9 eta_k-1^2 when that exceeds 0.1,
 * at least 0.5 times the Newton tolerance over |g_k|, at most forcing; the
 * first step takes forcing), CG then stopping at |r| <= max(cg_rtol,
 * eta_k) |r0|; 0 keeps cg_rtol alone.  Newton's own test is unchanged, so a
 * converged solve meets the same tolerance.  Negative or NaN:
 * OSMPM_E_INVALID_ARG. */
typedef struct {
  double newton_rtol, newton_atol, cg_rtol;
  int32_t max_newton, max_cg, max_ls;
  int32_t project_psd;
  double gravity[3];
  double forcing;
} osmpm_solve_opts;

typedef struct {
  int32_t newton_iters, cg_iters, ls_halvings, converged, ls_failed;
  double gnorm0, gnorm;
} osmpm_solve_stats;

/* Multiplicative Schwarz controls (Alg. 1): sub-cycling ratio M = dT/dt,
 * iteration cap k_max, convergence tolerance eps_conv on the relative
 * interface-velocity changes r_B and r_S (Eq. convergence_criterion) and the
 * vacuum regulariser eps_tol of the projection (Eq. spatial_projection).
 * warm_start = 1: from the second Schwarz iteration of a frame on, every
 * implicit solve (the coarse solve, fine sub-step m) starts its free DOFs
 * from the same solve's solution in the previous iteration (on nodes that
 * were active then; dt v^n elsewhere) instead of dt v^n, and tests Newton
 * convergence against the initial gradient norm of that solve in the
 * frame's first iteration; the converged states agree with cold starts to
 * the solver tolerances (the paper does not state the initial iterate).
 * The reverse-mode entry points recompute frames with cold starts. */
typedef struct {
  int32_t M, k_max;
  double eps_conv, eps_tol;
  osmpm_solve_opts coarse, fine;
  int32_t warm_start;
} osmpm_schwarz_opts;

/* Statistics of one Schwarz frame: iterations and convergence of the
 * Schwarz loop, the last residuals, receiver and ambiguous-node counts, and
 * per side (B coarse, S fine) the Newton, CG and line-search halving counts
 * summed over the frame's implicit solves, the number of those solves that
 * ended unconverged (Newton cap reached or line search failed) and the
 * number whose line search failed. */
typedef struct {
  int32_t iters, converged;
  double r_B, r_S;
  int32_t n_recv_B, n_recv_S, n_amb;
  int32_t newton_B, newton_S, cg_B, cg_S, ls_B, ls_S;
  int32_t unconv_B, unconv_S, lsfail_B, lsfail_S;
} osmpm_schwarz_stats;

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device`.  `stream` is a hipStream_t
 * borrowed from the caller (e.g. torch.cuda.current_stream().cuda_stream) or
 * NULL for the default stream; the context never destroys it. */
osmpm_status osmpm_ctx_create(int32_t device, void *stream, osmpm_ctx **out);
osmpm_status osmpm_ctx_set_stream(osmpm_ctx *ctx, void *stream);
/* HIP graph replay.  enable = 1: solve cycles (a fixed sequence of CG,
 * line-search, Newton-step, gradient and Newton-test launches plus the copy
 * of the small status block) are replayed as HIP graphs, built once per
 * batch side and cycle shape and cached.  enable = 2: in addition, a whole
 * Schwarz iteration of a pair or batch frame (Alg. 1's loop body: the coarse
 * solve, the fine restart, interpolations and M sub-steps, the projection
 * and the residuals, then the status copy) is one graph, built once per
 * iteration class (the first iteration, later odd and even ones), frame
 * step and option set, when both solves have a fixed schedule: max_newton =
 * 1, max_ls = 0, cg_rtol = 0 (one Newton step of exactly max_cg CG
 * iterations, the step taken only if it lowers the energy).  Adaptive solves
 * decide Newton steps and halvings on the host between cycles and keep
 * cycle graphs (or direct launches).  enable = 0 enqueues every launch
 * individually.  Results are the same either way.  Default: 0 (cycle
 * replay measured about 2 % slower per frame than direct launches on the
 * refined inclusion: the cost is the GPU's dependent-dispatch latency, which
 * a graph does not remove).  Kernel timing (osmpm_profile_enable) always uses
 * individual launches.  OSMPM_E_INVALID_ARG for other values. */
osmpm_status osmpm_ctx_set_graphs(osmpm_ctx *ctx, int32_t enable);
/* How the CG scalars (stop test, step length, direction weight; Sec. 2.2.5's
 * linear solve) are formed.  mode 0: inside every CG launch, each workgroup
 * summing all workgroups' partial sums of the previous launch; mode 1: by an
 * extra one-workgroup-per-domain launch after each CG launch; mode -1
 * (default): mode 1 when the partial sums every workgroup would read exceed
 * 128 MB per launch (24 B x workgroups^2, summed over the batch side), else
 * mode 0.  Both sum in the same order, so results are identical.  Any
 * other value: OSMPM_E_INVALID_ARG. */
osmpm_status osmpm_ctx_set_cg_split(osmpm_ctx *ctx, int32_t mode);
/* Waits for all queued work and reports device-side errors. */
osmpm_status osmpm_sync(osmpm_ctx *ctx);
const char *osmpm_last_error(const osmpm_ctx *ctx);

/* Kernel timing with HIP events on the context stream.  enable = 1 clears the
 * counters and records an event pair around every launch of the
 * instrumented kernels (osmpm_kernel); enable = 0 stops.  CG launches that
 * only find the solve already finished are not counted.  Synchronises. */
osmpm_status osmpm_profile_enable(osmpm_ctx *ctx, int32_t enable);
/* Counted launches, their summed duration in milliseconds and their summed
 * algorithmic bytes (the bytes the operation must move once: particle arrays
 * read or written, node arrays gathered, atomic updates as read + write) for
 * kernel `which` since profiling was enabled.  Outputs may be NULL.
 * Synchronises. */
osmpm_status osmpm_profile_query(osmpm_ctx *ctx, int32_t which, int64_t *launches, double *total_ms,
                                 double *bytes);
void osmpm_ctx_destroy(osmpm_ctx *ctx);

/* ---------------------------------------------------------------- domain */

/* Creates a subdomain (Sec. 3.1) with room for `capacity` particles.  tile
 * gives the cells per axis of one workgroup tile of the particle/grid
 * kernels (0 = library default); the particle sort orders bins tile-major.
 * The capacity, the node count and the bin count (the cells of whole tiles)
 * are each limited to 2^28; beyond that, or with a tile too large for LDS:
 * OSMPM_E_INVALID_ARG. */
osmpm_status osmpm_domain_create(osmpm_ctx *ctx, const osmpm_grid *grid, int32_t precision,
                                 int64_t capacity, const int32_t *tile_host, osmpm_domain **out);
void osmpm_domain_destroy(osmpm_domain *dom);

/* Material table (host array of n_mat entries). */
osmpm_status osmpm_domain_set_materials(osmpm_domain *dom, const osmpm_material *mats_host,
                                        int32_t n_mat);
/* Elastoplastic extension (the paper keeps to elasticity and names
 * elastoplastic hinges as future work, Sec. 4.4 and Sec. 5): von Mises yield
 * stress per material (host array of n_mat entries, n_mat equal to the
 * material table's; n_mat = 0 makes every material elastic; an entry <= 0
 * or infinite: that material is elastic).  Reading: F = F^E F^P with the
 * particle holding F^E; the implicit solve sees the elastic energy only;
 * after G2P's deformation-gradient update F^E is projected onto
 * |dev eps| <= tau_y / (2 mu), eps the logarithms of its singular values
 * (the closest point in eps: det F^E, the polar rotation and the principal
 * directions are kept).  The reverse-mode entry points return
 * OSMPM_E_INVALID_ARG for domains with a finite yield stress.  NaN entries
 * or a length mismatch: OSMPM_E_INVALID_ARG.  Synchronises. */
osmpm_status osmpm_domain_set_yield(osmpm_domain *dom, int32_t n_mat, const double *tau_y_host);

/* Copies n particles in: positions x [n][d], velocities v [n][d], affine
 * matrices B [n][d][d], deformation gradients F [n][d][d], masses m_p and
 * initial volumes V_p^0 [n], material indices [n] and flags [n] (bit 0: the
 * particle belongs to the boundary layer P^partial of Sec. 3.2.1; bit 1+g:
 * member of scene boundary-condition group g).  The library may reorder
 * particles (binning); osmpm_get_particles returns each one's input index. */
osmpm_status osmpm_domain_set_particles(osmpm_domain *dom, int64_t n, const double *x,
                                        const double *v, const double *B, const double *F,
                                        const double *mass, const double *vol, const int32_t *mat,
                                        const uint8_t *flags);

/* Node selection by particle mass (Eq. boundary_grid_set): node masses are
 * summed in fixed point with unit m_ref / 2^32 (per contribution
 * rint(N_ip * m_p * 2^32 / m_ref)), and a node is selected when its sum
 * exceeds rint(tau * 2^32 / m_ref).  Both domains of a pair must use the same
 * m_ref. */
osmpm_status osmpm_domain_set_selection(osmpm_domain *dom, double m_ref, double tau);

/* Scene Dirichlet groups (host arrays of n_groups <= 4 entries): kind
 * (osmpm_bc_kind), component mask and 8 parameters each.  FIX: u = 0.
 * TRANSLATE: u = dt * params[0..d-1] (a velocity).  ROTATE (3D): incremental
 * rigid rotation about the axis through params[0..2] with unit direction
 * params[3..5] at angular velocity params[6].  A node is constrained by the
 * lowest group whose selected mass (as above) exceeds tau; scene groups take
 * precedence over Schwarz data on the same DOF. */
osmpm_status osmpm_domain_set_scene_bc(osmpm_domain *dom, int32_t n_groups, const int32_t *kind_host,
                                       const int32_t *mask_host, const double *params_host);

/* Particle-to-grid transfer (Eq. p2g_transfer): bins particles by the cell of
 * their base node with a stable counting sort, then accumulates
 * m_i = sum m_p N_ip and (mv)_i = sum m_p N_ip (v_p + B_p D_p^-1 (x_i - x_p)),
 * D_p = dx^2/4 I, sets v_i = (mv)_i / m_i on active nodes (m_i > 0) and
 * selects the scene-BC nodes. */
osmpm_status osmpm_p2g(osmpm_domain *dom);

/* One implicit backward-Euler solve over dt (Eq. discrete_energy, Sec. 2.2.5)
 * on the grid of the last P2G: the displacement u = x_hat - x^n minimising
 * E_h over the free DOFs.  use_schwarz_bc = 1 also prescribes
 * u = dt * v_bc on the receiver nodes (osmpm_set_schwarz_bc).  Synchronises;
 * stats may be NULL. */
osmpm_status osmpm_implicit_solve(osmpm_domain *dom, double dt, int32_t use_schwarz_bc,
                                  const osmpm_solve_opts *opts, osmpm_solve_stats *stats_host);

/* Grid-to-particle transfer with v_i = u_i / dt (Eqs. g2p_v, g2p_B), the
 * deformation-gradient update (Eq. F_update) and advection (Eq. advection),
 * from the displacement u of the implicit solve of the current grid: returns
 * OSMPM_E_STATE when no osmpm_implicit_solve (or frame) has run on this
 * domain since its last P2G. */
osmpm_status osmpm_g2p(osmpm_domain *dom, double dt);

/* Boundary sets Gamma_B, Gamma_S from the boundary-layer particles (Eq.
 * boundary_grid_set) and the receiver sets after the mass arbitration of
 * coincident boundary nodes (Eq. overlap_donor, ties to B).  Uses the grids
 * of the last P2G of each domain.  n_amb_host (may be NULL) receives the
 * number of ambiguous node pairs; synchronises when it is not NULL. */
osmpm_status osmpm_interface_build(osmpm_domain *B, osmpm_domain *S, int32_t *n_amb_host);

/* Pi_{S->B} (Eq. spatial_projection) of the fine field vS ([nS][d]; NULL =
 * S's P2G velocity) over S's active nodes onto B's receivers:
 * out_I = sum m_j v_j N_I(x_j) / (sum m_j N_I(x_j) + eps_tol); 0 elsewhere. */
osmpm_status osmpm_project_S_to_B(osmpm_domain *S, osmpm_domain *B, double eps_tol,
                                  const double *vS, double *out);

/* I_{B->S} (Eq. interp_BtoS) of the coarse field vB ([nB][d]; NULL = B's P2G
 * velocity) at S's receivers: out_j = sum_I v_I N_I(x_j), inactive coarse
 * nodes contributing zero; 0 on non-receivers. */
osmpm_status osmpm_interp_B_to_S(osmpm_domain *B, const double *vB, osmpm_domain *S, double *out);

/* T_m (Eq. temporal_interp): out = (1 - m/M) vn + (m/M) vn1 over n values. */
osmpm_status osmpm_temporal_interp(osmpm_ctx *ctx, int64_t n, int32_t m, int32_t M, const double *vn,
                                   const double *vn1, double *out);

/* Receiver velocities ([n_nodes][d]) prescribed by the next solve with
 * use_schwarz_bc = 1. */
osmpm_status osmpm_set_schwarz_bc(osmpm_domain *dom, const double *vbc);

/* One global frame t_n -> t_n + dT of Alg. 1 on the pair (B, S): store the
 * fine state, P2G on both, boundary sets and arbitration, then Schwarz
 * iterations (Pi -> coarse solve -> restore fine state, P2G, I at both
 * endpoints -> M fine sub-steps of T_m, solve, G2P, P2G -> residuals) until
 * r_B <= eps_conv and r_S <= eps_conv or k_max, then the coarse G2P and
 * advection.  Synchronises; stats may be NULL. */
osmpm_status osmpm_schwarz_frame(osmpm_domain *B, osmpm_domain *S, double dT,
                                 const osmpm_schwarz_opts *opts, osmpm_schwarz_stats *stats_host);

/* One single-domain step: P2G, implicit solve, G2P.  Synchronises. */
osmpm_status osmpm_single_frame(osmpm_domain *dom, double dt, const osmpm_solve_opts *opts,
                                osmpm_solve_stats *stats_host);

/* ---------------------------------------------------------------- batches */

/* A batch runs many independent scenes in shared launches: every stage of
 * the frame is one launch over all scenes (one launch dimension indexes the
 * scene), domains of uneven size included.  Each scene keeps its own Newton,
 * CG, line-search and Schwarz decisions, taken on the device, so its results
 * are those of running it alone; a scene whose Schwarz loop has converged
 * leaves the remaining iterations' launches.  All members share the batch's
 * dT, M and solver options (Alg. 1 per scene).
 *
 * osmpm_batch_create: n scenes (1 <= n <= 1024); coarse[i] (host array of
 * handles) and, for Schwarz batches, fine[i] form pair i; fine = NULL makes a
 * batch of single domains.  Members must share the context, dimension and
 * precision, and no domain may appear twice.  The batch references the
 * domains (it does not own them): destroy it before them; a batch whose
 * member was destroyed returns OSMPM_E_STATE.  Per-scene settings
 * (materials, particles, selection, scene BC parameters) are changed on the
 * domains between frames as usual. */
osmpm_status osmpm_batch_create(osmpm_ctx *ctx, int32_t n, osmpm_domain *const *coarse_host,
                                osmpm_domain *const *fine_host, osmpm_batch **out);
/* One global frame of Alg. 1 for every pair of a Schwarz batch (the steps of
 * osmpm_schwarz_frame); stats_host[n] receives each pair's statistics (may be
 * NULL).  Synchronises. */
osmpm_status osmpm_batch_schwarz_frame(osmpm_batch *batch, double dT, const osmpm_schwarz_opts *opts,
                                       osmpm_schwarz_stats *stats_host);
/* One single-domain step (P2G, implicit solve, G2P) for every member of a
 * batch created with fine = NULL; stats_host[n] may be NULL.  Synchronises. */
osmpm_status osmpm_batch_single_frame(osmpm_batch *batch, double dt, const osmpm_solve_opts *opts,
                                      osmpm_solve_stats *stats_host);
/* A multi-frame run of a Schwarz batch and its reverse mode (Alg. 1 frame
 * after frame; the gradient of a loss of the end-of-run particle positions
 * with respect to every material's Young's modulus).
 *
 * osmpm_batch_run: n_frames >= 1 frames of osmpm_batch_schwarz_frame from the
 * domains' current states.  bc_host is NULL (scene-BC parameters left as set
 * on the domains) or [n_frames][n][2][4][8] doubles: at frame f, pair i's
 * coarse (0) and fine (1) domain take parameters [f][i][side][g][0..7] for
 * its scene groups g (as osmpm_domain_set_scene_bc; rows past a domain's
 * group count are ignored).  The batch keeps, for osmpm_batch_backward,
 * every pair's Schwarz iteration count per frame, a device copy of every
 * domain's particle state at the start of frames 0, c, 2c, ...
 * (c = checkpoint_every >= 1) and at the end, replacing the previous run's.
 * stats_host (may be NULL) receives [n_frames][n] frame statistics.
 * Synchronises. */
osmpm_status osmpm_batch_run(osmpm_batch *batch, int32_t n_frames, double dT, const osmpm_schwarz_opts *opts,
                             int32_t checkpoint_every, const double *bc_host, osmpm_schwarz_stats *stats_host);
/* Reverse mode over the last osmpm_batch_run: xbar_B_host / xbar_S_host are
 * host arrays of n device pointers (either array, or any entry, may be NULL
 * for zero), entry i the adjoint dL/dx of pair i's end-of-run coarse / fine
 * particle positions, FP64 [np][d] in the order of the last
 * osmpm_domain_set_particles.  Each checkpointed segment is restored and
 * rerun to recover its frame start states; the frames are then swept from
 * last to first through each pair's frame adjoint (mode 0: that of
 * osmpm_schwarz_frame_adjoint with the run's iteration count; mode 1: the
 * implicit one of osmpm_schwarz_frame_adjoint_implicit with fp_tol, fp_max),
 * with adjoint CG tolerance adj_cg_rtol, carrying the particle adjoints.
 * The Lame-parameter derivatives are mapped to Young's moduli by the chain
 * rule of mu = E / (2 (1 + nu)), lam = E nu / ((1 + nu) (1 - 2 nu)).
 * dL_dE_host receives, pair after pair, dL/dE of each material of the coarse
 * domain followed by each material of the fine domain (sum over pairs of
 * n_mat_B + n_mat_S values; a material present in both domains appears
 * twice and the two entries add).  The domains hold the end-of-run state
 * afterwards.  OSMPM_E_STATE without a run.  Synchronises. */
osmpm_status osmpm_batch_backward(osmpm_batch *batch, const double *const *xbar_B_host,
                                  const double *const *xbar_S_host, double adj_cg_rtol, int32_t mode, double fp_tol,
                                  int32_t fp_max, double *dL_dE_host);
void osmpm_batch_destroy(osmpm_batch *batch);

/* Several refined regions (named as future work in the conclusion; the
 * paper gives no algorithm, so these are readings): one coarse domain and k
 * fine domains that overlap the coarse domain and possibly each other.
 * Boundary sets as for a pair; each fine domain is arbitrated against the
 * coarse one by the rule of Eq. overlap_donor, and fine domains against each
 * other pairwise by the same rule (ties: the lower index donates); Pi (Eq.
 * spatial_projection) takes the union of the fine point masses (sums over
 * all fine domains, divided on the coarse receivers); each Schwarz iteration
 * solves the coarse domain, then sub-cycles every fine domain from the same
 * coarse solution.  A fine receiver that lies in another fine domain's
 * material (the coincident lattice node active with a fixed-point mass above
 * that domain's threshold; the largest such mass wins, ties to the lower
 * index) takes, at sub-step m, that domain's grid velocity u/dt of sub-step
 * m of the previous Schwarz iteration (the first iteration uses the coarse
 * data); r_S (Eq. convergence_residuals) runs over the receivers of all fine
 * domains together, a linked receiver's datum being its donor's sub-step-M
 * velocity, and the frame ends when r_B and r_S pass.  Disjoint fine
 * domains have no links; with k = 1 the frame is that of
 * osmpm_schwarz_frame.  The group holds the coarse
 * domain k times internally; every fine domain must pair with it as for
 * osmpm_schwarz_frame (same context, dimension, precision, lattice and
 * reference mass), each at most once.  k <= 1024. */
osmpm_status osmpm_multi_create(osmpm_ctx *ctx, osmpm_domain *coarse, int32_t k, osmpm_domain *const *fine_host,
                                osmpm_batch **out);
/* One global frame of Alg. 1 on a group from osmpm_multi_create (only that
 * kind: other groups return OSMPM_E_INVALID_ARG, and osmpm_batch_schwarz_frame
 * refuses this one); *stats_host (may be NULL) receives the frame's
 * statistics, fine-domain counts summed.  Synchronises.  Destroy the group
 * with osmpm_batch_destroy. */
osmpm_status osmpm_multi_schwarz_frame(osmpm_batch *batch, double dT, const osmpm_schwarz_opts *opts,
                                       osmpm_schwarz_stats *stats_host);

/* ---------------------------------------------------------------- reverse mode */

/* Adjoints (reverse-mode derivatives) of a frame.  The frame is recomputed
 * from the domains' current states with its intermediates stored, then swept
 * in reverse.  Discrete decisions (bins, active nodes, boundary and receiver
 * sets, the Schwarz iteration count) are held at their forward values; each
 * implicit solve (Sec. 2.2.5) is differentiated at its minimiser by the
 * implicit-function theorem (the adjoint system H_ff lambda = ubar_f with the
 * Hessian of Eq. discrete_energy, not PSD-projected, solved on the forward CG
 * kernels to adj_cg_rtol); P2G (Eq. p2g_transfer), G2P (Eqs. g2p_v .. advection),
 * Pi_{S->B} (Eq. spatial_projection), I_{B->S} (Eq. interp_BtoS) and T_m
 * (Eq. temporal_interp) are transposed exactly, including the dependence of
 * the weights on particle positions.
 *
 * Adjoint arrays are device FP64 in the caller's layout and particle order of
 * the last osmpm_domain_set_particles: x, v [n][d], B, F [n][d][d].  Inputs:
 * the adjoint of the end-of-frame state; outputs (overwritten): the adjoint of
 * the start-of-frame state.  mubar / lambar (host, [n_mat] of each domain) ACCUMULATE
 * the derivative with respect to the Lame parameters of each material.  On
 * return the domains hold the end-of-frame state (as after the forward call).
 * Synchronises.  All arithmetic of the reverse sweep is FP64; in the mixed
 * path the stored forward states and the adjoint CG vectors are FP32. */
osmpm_status osmpm_single_frame_adjoint(osmpm_domain *dom, double dt, const osmpm_solve_opts *opts,
                                        double adj_cg_rtol, const double *xbar, const double *vbar,
                                        const double *Bbar, const double *Fbar, double *xbar_out,
                                        double *vbar_out, double *Bbar_out, double *Fbar_out,
                                        double *mubar_host, double *lambar_host);
/* osmpm_single_frame_adjoint without any device or pinned-host allocation,
 * for callers that cannot allocate (code under HIP graph capture, tight
 * serving or training loops, harnesses that forbid allocation).  Its work
 * arrays (the frame's two stored forward points, the particle adjoints
 * entering and leaving, node adjoints) are carved out of one fixed 64 MiB
 * device region per device, looked up when the first context on the device
 * is created and held until the process ends.  They take, each array
 * rounded up to 256 bytes, 2 (cap (8 d + tb (d + 2 d^2) + 25) + 4 (n_keys + 1)
 * + nodes (8 + 25 d)) + 32 np d (1 + d) + nodes (24 d + 8) + 1024 bytes
 * (cap: particle capacity, tb: 8 FP64 / 4 mixed); a domain that needs more
 * returns OSMPM_E_INVALID_ARG before any work is queued.  Every call on a
 * device shares its region, and the region keeps the last call's contents
 * (each work array is written before it is read): calls that overlap on one
 * device (from several contexts or threads) race and must be serialised by
 * the caller.  HIP graph replay and kernel timing are suspended for the
 * call.  Arguments, results, accumulation and end state as
 * osmpm_single_frame_adjoint. */
osmpm_status osmpm_single_frame_adjoint_noalloc(osmpm_domain *dom, double dt, const osmpm_solve_opts *opts,
                                                double adj_cg_rtol, const double *xbar, const double *vbar,
                                                const double *Bbar, const double *Fbar, double *xbar_out,
                                                double *vbar_out, double *Bbar_out, double *Fbar_out,
                                                double *mubar_host, double *lambar_host);
/* The frame of osmpm_schwarz_frame on the pair (B, S) with exactly `iters`
 * Schwarz iterations (the forward call's stats.iters). */
osmpm_status osmpm_schwarz_frame_adjoint(osmpm_domain *B, osmpm_domain *S, double dT,
                                         const osmpm_schwarz_opts *opts, int32_t iters, double adj_cg_rtol,
                                         const double *xbar_B, const double *vbar_B, const double *Bbar_B,
                                         const double *Fbar_B, const double *xbar_S, const double *vbar_S,
                                         const double *Bbar_S, const double *Fbar_S, double *xbar_B_out,
                                         double *vbar_B_out, double *Bbar_B_out, double *Fbar_B_out,
                                         double *xbar_S_out, double *vbar_S_out, double *Bbar_S_out,
                                         double *Fbar_S_out, double *mubar_B_host, double *lambar_B_host,
                                         double *mubar_S_host, double *lambar_S_host);

/* Implicit (fixed-point) adjoint of the same frame.  Alg. 1 iterates
 * z -> Phi(z), z the projected Dirichlet data of the coarse solve (Eq.
 * spatial_projection), and the Schwarz iteration contracts for coercive
 * problems (Sec. 2.3); at its fixed point z* the derivative of the
 * end-of-frame states is that of psi(z*) (the coarse solve with data z*, its
 * G2P and the fine sub-steps it drives) plus Phi's own inputs weighted by
 * mu = sum_j (Phi_z^T)^j w, w = psi_z^T times the output adjoint.  The series
 * is summed pass by pass, each pass one reverse Schwarz iteration (Steps 1
 * and 2 transposed), all linearised at the forward's last iterate: only that
 * iteration's intermediates are stored (the unrolled call stores all
 * `iters`), and the first iterate's data (the Step-0 projection) carries no
 * derivative.  The frame is recomputed with exactly `iters` iterations.
 * fp_tol > 0: stop once the 2-norm of (Phi_z^T)^j w (all coarse node
 * components) is at most fp_tol times that of w, or return
 * OSMPM_E_NOT_CONVERGED after fp_max passes; fp_tol <= 0: exactly fp_max
 * passes.  fp_max >= 1.  *fp_used_host (may be NULL) receives the number of
 * passes j.  Arrays, accumulation and end state as osmpm_schwarz_frame_adjoint. */
osmpm_status osmpm_schwarz_frame_adjoint_implicit(
    osmpm_domain *B, osmpm_domain *S, double dT, const osmpm_schwarz_opts *opts, int32_t iters,
    double adj_cg_rtol, double fp_tol, int32_t fp_max, int32_t *fp_used_host, const double *xbar_B,
    const double *vbar_B, const double *Bbar_B, const double *Fbar_B, const double *xbar_S,
    const double *vbar_S, const double *Bbar_S, const double *Fbar_S, double *xbar_B_out, double *vbar_B_out,
    double *Bbar_B_out, double *Fbar_B_out, double *xbar_S_out, double *vbar_S_out, double *Bbar_S_out,
    double *Fbar_S_out, double *mubar_B_host, double *lambar_B_host, double *mubar_S_host,
    double *lambar_S_host);

/* ---------------------------------------------------------------- readback */

/* Particle state in the library's current order; id receives each
 * particle's index in the last osmpm_domain_set_particles input.  Any output
 * may be NULL. */
osmpm_status osmpm_get_particles(osmpm_domain *dom, double *x, double *v, double *B, double *F,
                                 int32_t *id);
/* Grid of the last P2G / solve: node mass m [n_nodes], P2G velocity vn and
 * displacement u [n_nodes][d].  Any output may be NULL. */
osmpm_status osmpm_get_grid(osmpm_domain *dom, double *m, double *vn, double *u);
/* Interface sets: gamma and recv flags [n_nodes] (uint8) and the fixed-point
 * node mass of all particles q_all [n_nodes] (int64).  Any may be NULL. */
osmpm_status osmpm_get_sets(osmpm_domain *dom, uint8_t *gamma, uint8_t *recv, int64_t *q_all);
/* The stable counting sort of the last binning: perm[i] = position before
 * the sort of the i-th particle in stable bin order, and the bin offsets
 * cell_start [n_keys + 1] of that order.  The particle arrays store each
 * tile's particles slot-major (the first particle of every non-empty cell of
 * the tile in cell order, then the second, ...), so a tile occupies the same
 * range [cell_start[t * tile_volume], cell_start[(t + 1) * tile_volume]) in
 * both orders; osmpm_get_particles returns the storage order with ids. */
osmpm_status osmpm_get_sort(osmpm_domain *dom, int32_t *perm, int32_t *cell_start);
/* Sizes: particles, nodes, sort keys (host outputs, any may be NULL). */
osmpm_status osmpm_domain_info(osmpm_domain *dom, int64_t *n_particles, int64_t *n_nodes,
                               int64_t *n_keys);

#ifdef __cplusplus
}
#endif

#endif /* OSMPM_H */
