/*
 * npfem.h -- C ABI of the batched npFEM red-blood-cell step on AMD Instinct MI355X
 * (gfx950).
 *
 * The library advances membranes by one implicit time step of the nodal projective
 * FEM of Kotsalos, Latt & Chopard (arXiv:1903.06479), Algorithm 1 (section 2.1.5):
 *
 *   minimise g(x) = 1/(2h^2) (x - y_n)^T M~ (x - y_n) + sum_i E_i(x)
 *       (eqs. genericOptimizationNewton / GeneralizedObjectiveFunction)
 *   with the local-area, bending and global-volume projective-dynamics energies of
 *   section 2.1.2 and the modified Skalak material of section 2.1.3, by L-BFGS whose
 *   initial Hessian is the constant H~ = M~/h^2 + L (section 2.1.1), with a halving
 *   line search; then v_{n+1} = (x_{n+1} - x_n)/h and the post-convergence
 *   dissipation of section 2.1.4.
 *
 * Units: any consistent set (the workloads use um, us, pN, fg).
 *
 * Conventions
 *  - Every call returns npfem_status (0 = success, < 0 = error); nothing throws across
 *    the ABI.  npfem_last_error() returns a message describing the last failure of
 *    the calling thread.
 *  - Host pointers are read during the call only.  Device pointers are owned by the
 *    caller, must stay valid until the stream work that uses them has completed, and
 *    are never freed or retained by the library.
 *  - Library objects (mesh, plan, batch) are owned by the library; destroy them only
 *    after the stream work that uses them has completed.  One batch serves one stream
 *    at a time (its workspace is reused by every step).
 *  - Device arrays of positions, velocities and forces are array-of-structures
 *    [V_total][3] in the plan's precision (float for NPFEM_FP32, double for
 *    NPFEM_FP64); the cells of a batch are stored one after another, each cell's n
 *    vertices contiguous, in the order given to npfem_batch_create.
 *  - Positions are cell-local (each cell expressed relative to an origin near it;
 *    the step is translation invariant, so the world origin never enters).
 *  - Per-cell numerical trouble never fails a step: it is reported in the per-cell
 *    status bits of npfem_cell_stats.
 */
#ifndef NPFEM_H
#define NPFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NPFEM_OK = 0,
  NPFEM_E_INVALID = -1,      /* bad argument */
  NPFEM_E_MESH = -2,         /* mesh not a closed, consistently oriented, outward 2-manifold */
  NPFEM_E_NOT_SPD = -3,      /* M~ or H~ not symmetric positive definite */
  NPFEM_E_HIP = -4,          /* HIP runtime failure */
  NPFEM_E_OOM = -5,          /* device or host allocation failed */
  NPFEM_E_UNSUPPORTED = -6   /* valid request the library does not support */
} npfem_status;

typedef enum { NPFEM_FP32 = 0, NPFEM_FP64 = 1 } npfem_precision;

/* Per-cell status bits. */
#define NPFEM_CONVERGED 1u   /* residual <= tol */
#define NPFEM_MAXITER 2u     /* max_iter reached */
#define NPFEM_LS_FAIL 4u     /* line search failed even with the plain preconditioned gradient */
#define NPFEM_NONFINITE 8u   /* non-finite objective or gradient at the first guess; x, v unchanged */
#define NPFEM_DEGENERATE_TRI 16u  /* a triangle of x_{n+1} is collapsed (area below 1e-6 of its rest
                                     area): its in-plane direction normal to the collapse is
                                     undefined and carries no force */
#define NPFEM_START_FALLBACK 32u  /* npfem_step_learned: the learned start y_n + delta did not lower
                                     the objective below its value at y_n, so the cell started
                                     from y_n (as npfem_step does) */

typedef struct npfem_mesh npfem_mesh;
typedef struct npfem_plan npfem_plan;
typedef struct npfem_batch npfem_batch;

/* Membrane material (Table 1 and sections 2.1.2-2.1.4). */
typedef struct {
  double B;         /* Skalak B of the modified Skalak law (section 2.1.3) */
  double C;         /* local-area PD stiffness k of w = A_t k (section 2.1.2) */
  double D;         /* Skalak correction D (section 2.1.3) */
  double k_bend;    /* bending stiffness (eq. BendingDiscretizedPotential) */
  double k_volume;  /* global-volume PD weight (section 2.1.2) */
  double beta;      /* Rayleigh beta_D in units of the time step: C = beta h L' (section 2.1.4) */
  double kappa;     /* post-convergence dissipation factor in [0, 1] (section 2.1.4) */
  double density;   /* total mass = density * rest volume, lumped by vertex area (section 2.1) */
  double k_mat;     /* material stiffness added to H~ only (section 2.1.1); < 0 means B */
  double k_area_global;  /* weight of the optional global-area PD term (section 2.1.2: the
                            paper notes it could be built like the volume term and does not
                            use it): E = (k/2)(A - A0)^2 / |grad A(x_n)|^2, and k I in L and
                            H~; 0 (default) = off */
} npfem_material;

/* Normaliser of the global-volume term (section 2.1.2). */
#define NPFEM_VOLUME_STEP_FROZEN 0    /* |grad V|^2 taken at x_n for the whole step: the energy
                                         (k/2) C^2 / G_n and its gradient k C grad V / G_n agree,
                                         and the gradient equals the paper's PD force at x_n */
#define NPFEM_VOLUME_PAPER_LITERAL 1  /* |grad V(x)|^2 at the current x, force k (x - p(x)) as
                                         printed; that force is not the derivative of the
                                         energy once C != 0, so near convergence the line
                                         search may stop on it (LS_FAIL) */

/* Solver controls.  The paper fixes none of these (section 2.1.5). */
typedef struct {
  int32_t precision;        /* npfem_precision */
  int32_t lbfgs_m;          /* L-BFGS history length, 0..8 */
  int32_t max_iter;         /* quasi-Newton iterations per step */
  int32_t max_halvings;     /* line-search halvings before the plain-gradient retry */
  double tol;               /* residual tolerance */
  double c1;                /* sufficient-decrease constant */
  double noise_factor;      /* line search accepts increases below noise_factor*eps*sum|terms| */
  int32_t cells_per_tile;   /* cells sharing one H~^-1 product (1..21); 0 = automatic */
  int32_t grid_blocks;      /* persistent workgroups; 0 = automatic */
  int32_t inverse_bf16;     /* FP32 plans: 1 = apply H~^-1 and h^2 M~^-1 as an exact FP32
                               diagonal plus a BF16 off-diagonal part on the matrix cores
                               (they only precondition and start the iteration, so the
                               solution is unchanged); 2 = the same with the off-diagonal
                               part banded: stored in a reverse Cuthill-McKee order of the
                               mesh, each 16-column block applied over the k range that holds
                               its entries above 1e-4 sqrt(A_ii A_jj) (smaller entries outside
                               that range are dropped; the inverses decay fast away from the
                               diagonal); 0 = FP32 matrix cores */
  int32_t volume_normaliser;  /* NPFEM_VOLUME_STEP_FROZEN (default) or NPFEM_VOLUME_PAPER_LITERAL */
} npfem_solver_params;

/* Per-cell result of a step (device array filled by npfem_step). */
typedef struct {
  int32_t iterations;   /* accepted quasi-Newton iterations */
  int32_t evaluations;  /* objective/gradient evaluations, first guess included */
  uint32_t status;      /* NPFEM_CONVERGED | NPFEM_MAXITER | ... */
  int32_t halvings;     /* line-search halvings over the step */
  double residual;      /* final residual */
  double objective;     /* final g (up to the constant dropped from the inertial term) */
  double volume;        /* enclosed volume at x_{n+1} (FP64 reduction) */
  double area;          /* total membrane area at x_{n+1} (FP64 reduction) */
} npfem_cell_stats;

/* Totals of per-cell results over one or more steps (device struct, see
 * npfem_stats_accumulate).  status_count[k] counts cells with status bit 1 << (k + 1)
 * set: MAXITER, LS_FAIL, NONFINITE, DEGENERATE_TRI. */
typedef struct {
  int64_t cell_steps;       /* cells counted */
  int64_t iterations;       /* sum of iterations */
  int64_t evaluations;      /* sum of evaluations */
  int64_t halvings;         /* sum of line-search halvings */
  int64_t not_converged;    /* cells without NPFEM_CONVERGED */
  int64_t status_count[4];
  int32_t max_iterations;
  int32_t start_fallback;   /* cells with NPFEM_START_FALLBACK */
  double max_residual;
} npfem_stats_total;

const char *npfem_status_string(npfem_status s);
const char *npfem_last_error(void);

/* Defaults: the material reading used by the workloads and the solver controls above. */
void npfem_material_default(npfem_material *m);
void npfem_solver_params_default(npfem_solver_params *p);

/*
 * Rest mesh of one membrane type.  rest_xyz: host [n_verts][3]; tris: host
 * [n_tris][3], counter-clockwise seen from outside.  Validates that the surface is a
 * closed, consistently oriented 2-manifold enclosing a positive volume
 * (NPFEM_E_MESH otherwise) and computes the rest data: per triangle D_m^-1 in the
 * triangle's own 2D frame with the third vertex as reference (Appendix B) and the rest
 * area; per vertex the mixed Voronoi area, cotangent weights and |l0| of the
 * Laplace-Beltrami operator (eq. BendingDiscretizedPotential); the rest volume
 * (section 2.1.2).
 */
npfem_status npfem_mesh_create(int32_t n_verts, const double *rest_xyz, int32_t n_tris,
                               const int32_t *tris, npfem_mesh **out);
void npfem_mesh_destroy(npfem_mesh *mesh);
/* Any output pointer may be NULL. */
npfem_status npfem_mesh_query(const npfem_mesh *mesh, int32_t *n_verts, int32_t *n_tris,
                              int32_t *n_edges, double *rest_volume, double *rest_area);

/*
 * Rest data computed by npfem_mesh_create (host outputs, each may be NULL):
 * vor_area [n_verts] mixed Voronoi areas, ell0 [n_verts] |l0_i| (the rest
 * Laplace-Beltrami vector's length), tri_area [n_tris], dminv [n_tris][4] (D_m^-1
 * row-major).  Host-only; for inspection and tests.
 */
npfem_status npfem_mesh_rest_data(const npfem_mesh *mesh, double *vor_area, double *ell0,
                                  double *tri_area, double *dminv);

/*
 * Plan: one or more mesh types, one material, one time step.  Builds in FP64 on the
 * host the lumped mass M, L' (area + bending PD terms), L = L' + k_volume I
 * (eq. fullyDeveloped_g), M~ = M + beta h^2 L' (eq. preOptimizationNewton with Rayleigh
 * damping) and H~ = M~/h^2 + L + K_mat (section 2.1.1), Cholesky-factors M~ and H~
 * (NPFEM_E_NOT_SPD on failure), and uploads the dense inverses h^2 M~^-1 and H~^-1
 * in the plan's precision, zero-padded to a multiple of 32.  A new dt needs a new plan.
 * meshes: host array of n_meshes handles, which must outlive the plan.
 */
npfem_status npfem_plan_create(int32_t hip_device, const npfem_mesh *const *meshes,
                               int32_t n_meshes, const npfem_material *mat, double dt,
                               const npfem_solver_params *params, npfem_plan **out);
void npfem_plan_destroy(npfem_plan *plan);
/* Lumped masses of mesh type mesh_index: host output [n_verts]. */
npfem_status npfem_plan_masses(const npfem_plan *plan, int32_t mesh_index, double *mass_out);

/*
 * Batch: the cell list of a plan.  cell_mesh: host [n_cells] mesh indices into the
 * plan's mesh list.  Groups cells of one mesh type into tiles of cells_per_tile, orders
 * tiles by cost, uploads the schedule and allocates the step workspace.
 * n_vertices_total (may be NULL) receives the length V_total of the vertex arrays.
 */
npfem_status npfem_batch_create(npfem_plan *plan, int64_t n_cells, const int32_t *cell_mesh,
                                npfem_batch **out, int64_t *n_vertices_total);
void npfem_batch_destroy(npfem_batch *batch);

/*
 * Schedule of a batch: cells_per_tile (1..21) cells share one product with H~^-1 on the
 * matrix cores and one workgroup; lbfgs_m (0..8) is the L-BFGS history length used by
 * this batch (the solution does not depend on either, only the time to reach it).
 * npfem_batch_schedule rebuilds the tile queue and workspace (synchronously; no step of
 * this batch may be in flight); npfem_batch_get_schedule reports the current one
 * (outputs may be NULL).
 */
npfem_status npfem_batch_schedule(npfem_batch *batch, int32_t cells_per_tile, int32_t lbfgs_m);
npfem_status npfem_batch_get_schedule(const npfem_batch *batch, int32_t *cells_per_tile,
                                      int32_t *lbfgs_m, int32_t *grid_blocks, int32_t *n_tiles);

/*
 * Autotuner: times one step of the batch on the caller's inputs for each candidate
 * schedule (cells_per_tile in {5, 10, 16, 21}, and also 2 and 3 when the batch has fewer
 * than 10 cells per compute unit, so that its tiles can occupy every workgroup slot;
 * lbfgs_m in {2, 3, 5, 8} up to max_lbfgs_m) and keeps the fastest.  x, v, f_ext: device inputs as for npfem_step;
 * x_scratch, v_scratch: device [V_total][3] outputs it may overwrite.  Synchronous.
 * best_ms (may be NULL) receives the best step time in milliseconds.
 */
npfem_status npfem_batch_autotune(npfem_batch *batch, const void *x, const void *v, const void *f_ext,
                                  void *x_scratch, void *v_scratch, int32_t max_lbfgs_m, void *stream,
                                  double *best_ms);

/*
 * use_graph = 1: npfem_step and npfem_step_learned capture their launches into a HIP
 * graph on the first call with a given set of buffers, stream and network, and replay
 * that graph on later calls with the same arguments.  Up to four argument sets are kept
 * (the least recently used is dropped), so a caller alternating between two buffer
 * sets replays both.  The NULL stream cannot be captured: calls on it launch directly.
 * use_graph = 0 (default): launches directly, and the kept graphs are released.
 * Rescheduling the batch releases them too.
 */
npfem_status npfem_batch_set_graph(npfem_batch *batch, int32_t use_graph);

/* Number of graph captures and graph replays performed by the batch's steps so far
 * (host outputs, each may be NULL).  For tests and measurement. */
npfem_status npfem_batch_graph_counts(const npfem_batch *batch, int64_t *captures, int64_t *replays);

/*
 * One time step of every cell of the batch (Algorithm 1), asynchronous on `stream`
 * (a hipStream_t; NULL = default stream).
 *   x, v, f_ext : device [V_total][3] inputs x_n, v_n, F_ext(x_n)
 *   x_out, v_out: device [V_total][3] outputs x_{n+1}, v_{n+1}; may alias x, v
 *   u_guess     : device [V_total][3] or NULL: first guess of the displacement
 *                 x^(1) - x_n, replacing h^2 M~^-1 (M v_n / h + F_ext) (Algorithm 1,
 *                 first line); the solution does not depend on it
 *   stats       : device [n_cells] or NULL
 * Errors (NPFEM_E_INVALID for NULL required pointers, NPFEM_E_HIP for launch
 * failures) are returned synchronously; per-cell results are valid once the stream
 * has completed.
 */
npfem_status npfem_step(npfem_batch *batch, const void *x, const void *v, const void *f_ext,
                        void *x_out, void *v_out, const void *u_guess, npfem_cell_stats *stats,
                        void *stream);

/*
 * Adds the per-cell results `stats` (device [n_cells], as written by npfem_step) to the
 * device totals `total`, asynchronously on `stream`, so that a caller can count every
 * step of a run without copying per-cell results to the host.  npfem_stats_reset
 * zeroes `total` with a kernel (no memset node, so both may be captured in a graph).
 * NPFEM_E_INVALID for NULL pointers or n_cells < 0.
 */
npfem_status npfem_stats_accumulate(const npfem_cell_stats *stats, int64_t n_cells, npfem_stats_total *total,
                                    void *stream);
npfem_status npfem_stats_reset(npfem_stats_total *total, void *stream);

/*
 * Collision term between cells (section 4.7: a non-PD spring energy on colliding
 * vertices, dropped at every iteration where the vertex no longer penetrates, with no
 * share of H~).  npfem_collisions_detect finds, from the positions at the start of the
 * step, for every vertex the nearest vertex of another cell closer than `cutoff`
 * (ties: the smaller batch-wide vertex index), with a uniform grid of cell size
 * `cutoff` hashed into a table of at least twice the vertex count:
 *   cell_origin : device double [n_cells][3], world origin of each cell's local frame
 *   x           : device [V_total][3] cell-local positions (plan precision)
 *   contact_q   : device [V_total][3] out: the partner's position in the searching
 *                 vertex's cell frame (plan precision; zero without a contact)
 *   contact_n   : device [V_total][3] out: the partner's unit area-weighted vertex
 *                 normal (zero without a contact)
 *   n_contacts  : host, may be NULL: number of vertices with a contact (the call then
 *                 synchronises the stream)
 * The grid's buffers are allocated by the batch on the first call.
 * npfem_step_contacts is npfem_step with the collision energy
 *   (w_col/2) sum_i min((x_i - q_i) . n_i, 0)^2
 * added to g, so that a vertex behind its partner's tangent plane is pushed out along
 * the partner's normal (p_i = x_i - d_i n_i is its desired position) and the term
 * vanishes once it is out.  Launched directly (not through the batch's graphs).
 */
npfem_status npfem_collisions_detect(npfem_batch *batch, const double *cell_origin, const void *x, double cutoff,
                                     void *contact_q, void *contact_n, int64_t *n_contacts, void *stream);
npfem_status npfem_step_contacts(npfem_batch *batch, const void *x, const void *v, const void *f_ext,
                                 const void *contact_q, const void *contact_n, double w_col, void *x_out,
                                 void *v_out, npfem_cell_stats *stats, void *stream);

/*
 * npfem_step without any allocation, for callers that cannot allocate device memory
 * while they run: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and per-cell statistics as npfem_step
 * (bit for bit), launched directly on `stream` (never through the batch's graphs).
 * The tile counter, the cell states and the persistent workgroups' workspace live in a
 * static device array of 64 MiB per GPU, allocated when the library's code is loaded on
 * that GPU and held until the process ends; its address is looked up when the first
 * plan on the GPU is created.  The persistent grid is reduced to the workgroups whose
 * workspace fits the array (a 642-vertex FP32 batch at 5 cells per tile and history 2
 * keeps about 180 workgroups).  NPFEM_E_UNSUPPORTED if a single workgroup's workspace
 * exceeds 64 MiB.  Every call on a GPU shares that GPU's array: calls that overlap on
 * one GPU (on different streams, or from several threads) race and must not be issued.
 */
npfem_status npfem_step_noalloc(npfem_batch *batch, const void *x, const void *v, const void *f_ext,
                                void *x_out, void *v_out, const void *u_guess, npfem_cell_stats *stats,
                                void *stream);

/*
 * Objective and gradient of every cell at x = x_n + u (section 2.1.1,
 * eq. GeneralizedObjectiveFunctionDerivative), without iterating: the kernel that
 * evaluates the trial points of the line search, exposed for testing and measurement.
 *   x, v, f_ext, u: device [V_total][3]; grad_out: device [V_total][3]
 *   terms_out     : device double [n_cells][11] = { g, inertial part, area PD, Skalak,
 *                   bending (incl. its Rayleigh part), volume PD, triangle Rayleigh
 *                   part, residual, global-area PD, total area, collapsed triangles }
 * The volume normaliser |grad V|^2 is taken at x_n (at x_n + u with
 * NPFEM_VOLUME_PAPER_LITERAL), the global-area one at x_n.
 */
npfem_status npfem_eval(npfem_batch *batch, const void *x, const void *v, const void *f_ext,
                        const void *u, void *grad_out, double *terms_out, void *stream);

/*
 * out[r][:] = A in[r][:] for r < rows, with A = H~^-1 (which = 0) or h^2 M~^-1
 * (which = 1) of mesh type mesh_index: the MFMA product the step applies once per
 * iteration (section 2.1.1).  in, out: device [rows][n_pad] row-major in the plan's
 * precision, n_pad = n_verts rounded up to 32 (padding entries of `in` must be zero).
 * n_pad_out (may be NULL) receives n_pad.  Exposed for testing and measurement.
 */
npfem_status npfem_apply_inverse(npfem_plan *plan, int32_t mesh_index, int32_t which,
                                 const void *in, void *out, int32_t rows, int32_t *n_pad_out,
                                 void *stream);

/*
 * The paper's own route to the same products (section 2.1.1: H~ is factored once and
 * each iteration solves with the factor).  A = H~ (which = 0) or M~/h^2 (which = 1) is
 * factored at plan creation as P A P^T = L L^T, with P the reverse Cuthill-McKee order
 * of the mesh's vertex graph, so that L is banded (half bandwidth b); out[r] = A^-1 in[r]
 * is then solved by forward and back substitution with L, 64 right-hand sides per GPU
 * wave, in the plan's precision (FP32 on the matrix cores, in blocks of 16 positions;
 * FP64 on the vector units).  The result equals npfem_apply_inverse's up to rounding.
 *   in, out  : device [rows][n_pad] row-major, as for npfem_apply_inverse (padding
 *              entries of `in` must be zero; those of `out` are written as zero)
 *   work     : device workspace owned by the caller, at least
 *              npfem_solve_factor_workspace(plan, mesh_index, rows) bytes (work_bytes);
 *              calls that share a workspace must not overlap
 *   bandwidth_out (may be NULL): receives b, the larger of the two factors' half
 *              bandwidths
 * NPFEM_E_INVALID for bad arguments or a short workspace; NPFEM_E_UNSUPPORTED when
 * the band is too wide for the kernel's LDS ring (b above about 500 in FP32, 250 in
 * FP64).  Exposed to measure the factor route against the products with the inverses;
 * the step applies the inverses.
 */
int64_t npfem_solve_factor_workspace(const npfem_plan *plan, int32_t mesh_index, int32_t rows);  /* -1: bad args */
npfem_status npfem_solve_factor(npfem_plan *plan, int32_t mesh_index, int32_t which, const void *in,
                                void *out, int32_t rows, void *work, int64_t work_bytes,
                                int32_t *bandwidth_out, void *stream);

/*
 * First guess of the step (Algorithm 1, first line): u_out = y_n - x_n = h^2 M~^-1 b
 * with b = M v_n / h + f_ext, for every cell.  x, v, f_ext, u_out: device [V_total][3]
 * in the plan's precision.  Used to form the training targets of the learned warm start.
 */
npfem_status npfem_first_guess(npfem_batch *batch, const void *x, const void *v, const void *f_ext,
                               void *u_out, void *stream);

/*
 * Learned warm start.  The paper starts every step from y_n; this network predicts the
 * correction delta = x_{n+1} - y_n per vertex so that the iteration starts closer to its
 * fixed point (the fixed point itself does not depend on the start).  Per cell, the
 * inputs are expressed in the cell's best-fit rest frame R (mass-weighted Kabsch fit of
 * the rest mesh to x_n), as 12 features per vertex: shape deviation
 * (R^T (x_i - x_c) - (X_i - X_c)) / shape_scale, velocity R^T (v_i - v_c) h / s, force
 * R^T (f_i - m_i a_c) h^2 / (m_i s) and rest position (X_i - X_c) / max|X - X_c|, with the
 * displacement scale s = h^2 (rms_i |f_i - m_i a_c| + force_floor) / mean(m).  The network
 * is a residual GraphSAGE: h = relu(W_e feat + b_e), then `layers` times
 * h <- h + relu(W_s h + W_n mean_{mesh neighbours}(h) + b), then o = W_d h + b_d and
 * delta_i = s R o_i.  Hidden width 64.  Weights are applied as BF16 on the matrix cores
 * with FP32 accumulation; activations are stored in BF16; frame and sums in FP64.
 *
 * Parameters: one FP32 vector, row-major blocks in this order: W_e [64][12], b_e [64],
 * per layer W_s [64][64], W_n [64][64], b [64], then W_d [3][64], b_d [3].
 * A network belongs to one plan (its mesh types) and one device.
 */
typedef struct npfem_net npfem_net;
typedef struct {
  int32_t hidden;        /* must be 64 */
  int32_t layers;        /* message-passing layers, 1..8 */
  double force_floor;    /* force floor of the displacement scale (force units) */
  double shape_scale;    /* length scale of the shape-deviation features */
} npfem_net_config;

void npfem_net_config_default(npfem_net_config *cfg);  /* 64, 4, 1.0, 0.1 */
int64_t npfem_net_param_count(const npfem_net_config *cfg);   /* -1 for an invalid config */
/* theta: host FP32 [param_count] initial parameters (copied). */
npfem_status npfem_net_create(npfem_plan *plan, const npfem_net_config *cfg, const float *theta,
                              npfem_net **out);
void npfem_net_destroy(npfem_net *net);
npfem_status npfem_net_set_params(npfem_net *net, const float *theta);   /* host FP32; resets Adam */
npfem_status npfem_net_get_params(const npfem_net *net, float *theta);   /* host FP32 */

/*
 * Inference: delta_out (device [V_total][3], plan precision) = predicted correction of
 * every cell of the batch, world frame.
 */
npfem_status npfem_net_infer(npfem_net *net, npfem_batch *batch, const void *x, const void *v,
                             const void *f_ext, void *delta_out, void *stream);

/*
 * One step that starts from y_n + delta (delta from the network) instead of y_n; otherwise
 * identical to npfem_step (same outputs, statistics and convergence test).  The objective
 * g (eq. GeneralizedObjectiveFunction) is evaluated at y_n and at y_n + delta, and each
 * cell starts from y_n + delta only if g(y_n + delta) <= g(y_n); otherwise it starts from
 * y_n and its status carries NPFEM_START_FALLBACK (the quasi-Newton iterations and their
 * convergence test judge the result either way).  Both evaluations count in the cell's
 * `evaluations`.  Honours the batch's graph setting (the network and the step are
 * captured together).
 */
npfem_status npfem_step_learned(npfem_batch *batch, npfem_net *net, const void *x, const void *v,
                                const void *f_ext, void *x_out, void *v_out,
                                npfem_cell_stats *stats, void *stream);

/*
 * Training.  For the cells listed in `cells` (device int32 [n_cells] batch cell indices,
 * or NULL for cells 0..n_cells-1), with inputs x, v, f_ext, the converged x_next and the
 * first guess u0 (all device [V_total][3], plan precision), the loss is the mean over
 * the listed cells, their vertices and the 3 components of (o_i - t_i)^2 with target
 * t_i = R^T (x_next_i - x_i - u0_i) / s.  loss_out (host, may be NULL) receives the loss
 * (the call then synchronises the stream); grad_out (device FP32 [param_count]) the
 * gradient with respect to the parameters, summed in a fixed order (deterministic).
 */
npfem_status npfem_net_loss_grad(npfem_net *net, npfem_batch *batch, const int32_t *cells,
                                 int32_t n_cells, const void *x, const void *v, const void *f_ext,
                                 const void *x_next, const void *u0, double *loss_out,
                                 float *grad_out, void *stream);
/* Adam (Kingma & Ba) on the FP32 parameters with a device FP32 gradient; t counts
 * the updates since creation or the last set_params, from 1. */
npfem_status npfem_net_adam_step(npfem_net *net, const float *grad, double lr, double beta1,
                                 double beta2, double eps, void *stream);

/*
 * Stand-in for the fluid (not part of the method): per-vertex Stokes drag towards an
 * analytic flow, f = zeta_c (u(x) - v) with u = [rate_c * z + u_P] e_x, where
 * u_P = umax (1 - rho^2/R^2) for rho < R, rho^2 = (oy_c + y - axis_y)^2 + (oz_c + z - axis_z)^2.
 *   x, v, f_out: device [V_total][3]; cell_zeta, cell_rate: device double [n_cells];
 *   cell_origin: device double [n_cells][3]; umax = 0 disables the Poiseuille term.
 */
npfem_status npfem_drag_forces(npfem_batch *batch, const void *x, const void *v,
                               const double *cell_zeta, const double *cell_rate,
                               const double *cell_origin, double umax, double radius,
                               double axis_y, double axis_z, void *f_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* NPFEM_H */
