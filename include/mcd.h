/*
 * mcd.h - C ABI of libmcd, the MI355X (gfx950) hot path of the
 * mesh-constrained discrete point (MCD) method for incompressible flow with
 * moving boundaries (Matsuda & Ii, arXiv 2404.17542).
 *
 * Conventions shared by every call
 * --------------------------------
 * - One discrete point (DP) per background-mesh cell (Sec. 2.2).  Cell
 *   c = i + n0*(j + n1*k) (x fastest); Nc = n0*n1*(n2).
 * - Per-DP vectors are structure-of-arrays: a "[d][Nc]" argument is d
 *   consecutive planes of Nc values.
 * - Every pointer argument is a DEVICE pointer owned by the caller unless its
 *   comment says "host".  The library never frees caller memory.
 * - role is int8: -1 inner (Omega_I), 0 void, >= 1 boundary id (mask
 *   equation of Sec. 2.2).  When the mesh has walls, the outer ring (2D) or
 *   shell (3D) of cells carries the role mesh.wall_id.
 * - All work is enqueued on the context's HIP stream and is asynchronous
 *   unless a call says it synchronises.  Errors detected on the device
 *   (singular moment matrix, forbidden role transition) are latched in the
 *   context and returned by the next mcd_sync().
 * - No call throws; every call returns an mcd_status.  mcd_last_error()
 *   returns a human-readable message of the last failure.
 * - The context allocates all workspaces in mcd_create(); later calls do not
 *   allocate device memory.
 */
#ifndef MCD_H
#define MCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MCD_OK = 0,
    MCD_ERR_ARG = 1,           /* invalid argument (null pointer, bad size, NaN input ...) */
    MCD_ERR_SINGULAR = 2,      /* an inner DP's MLS moment matrix is singular */
    MCD_ERR_NOT_CONVERGED = 3, /* PPE not converged in max_iter; p holds the last iterate */
    MCD_ERR_BREAKDOWN = 4,     /* Bi-CGSTAB breakdown that restarts could not cure */
    MCD_ERR_ROLE = 5,          /* forbidden role transition (void <-> inner in one step) */
    MCD_ERR_HIP = 6,           /* a HIP runtime call failed */
    MCD_ERR_OOM = 7            /* device allocation failed in mcd_create */
} mcd_status;

enum { MCD_ROLE_INNER = -1, MCD_ROLE_VOID = 0 };
enum { MCD_BC_DIRICHLET = 0, MCD_BC_NEUMANN = 1 };
enum { MCD_WEIGHT_COS2 = 0, MCD_WEIGHT_GAUSS = 1 };
/* Arithmetic of the PPE solve (the tolerance is checked on the FP64 operator
 * in every mode):
 *   FP64         FP64 matrix, vectors and dots.
 *   FP32_REFINE  FP64 iterative refinement around an FP32 Bi-CGSTAB (FP32
 *                matrix and vectors, FP64 dots).
 *   FP32_MATRIX  FP64 Bi-CGSTAB whose matrix products read the FP32-stored
 *                matrix, with the residual periodically recomputed with the
 *                FP64 matrix and replaced (Krylov space kept). */
enum { MCD_PREC_FP64 = 0, MCD_PREC_FP32_REFINE = 1, MCD_PREC_FP32_MATRIX = 2 };
enum { MCD_GUESS_ZERO = 0, MCD_GUESS_CALLER = 1 };
enum { MCD_PRECOND_NONE = 0, MCD_PRECOND_JACOBI = 1, MCD_PRECOND_MG = 2 };

#define MCD_MAX_IDS 16      /* boundary ids 1 .. 15 */
#define MCD_MAX_BODIES 8
#define MCD_MAX_SETS 4      /* stencil-set slots held by a context */
#define MCD_MAX_GRAPHS 4    /* captured-sequence slots held by a context */

/* Background mesh (Sec. 2.2): uniform spacing l0, dim in {2, 3}. */
typedef struct {
    int dim;
    int n[3];            /* cells per axis (n[2] ignored in 2D) */
    double origin[3];    /* coordinates of vertex (0,0,0) */
    double l0;           /* mesh spacing */
    int periodic[3];     /* 1: axis is periodic */
    int walls;           /* 1: outer ring/shell of cells are wall DPs */
    int wall_id;         /* role id of wall DPs (1 .. 15) */
} mcd_mesh_desc;

/* Method constants (Sec. 2.3, 2.4, 3.2).  Paper values in brackets. */
typedef struct {
    int weight_kind;       /* MCD_WEIGHT_COS2 [paper] or MCD_WEIGHT_GAUSS (exp(-4 r^2/re^2)) */
    double re_over_l0;     /* MLS influence radius r_e / l0 [2.5] */
    double rs_over_l0;     /* MLS scaling length r_s / l0 [1] */
    double kappa;          /* relaxation coefficient [1/5] */
    double band_over_l0;   /* DPs re-positioned within this distance of a body [5] */
    double eps_relax;      /* relaxation stops when max |dx| <= eps_relax * l0 */
    double fit_alpha;      /* boundary-fitted arrangement (Sec. 4, Eqs. dp_arrng_boundary-fit_x**,
                              dp_arrng_beta): inner DPs of the band move by beta psi towards the
                              nearest body, beta = fit_alpha/2 (1 + cos(pi psi / r_e)) for psi < r_e;
                              0 = the original arrangement [0; the paper's example 0.03], in [0, 1] */
    double fit_re_over_l0; /* its r_e / l0 [5]; > 0 when fit_alpha > 0 */
} mcd_params;

/* Rigid circle (2D) / sphere (3D) at one time level; host memory.
 * psi = |x - centre| - radius (> 0 in the fluid, Sec. 2.5).
 * Velocity of a body point x (Eq. velocity_moving_boundary):
 *   V(x) = velocity + omega x r,  r = x - centre;
 * its time derivative (Eq. dvdt_moving_boundary, backward differences
 * supplied by the caller):
 *   dV/dt(x) = dvdt + domega_dt x r + omega x (omega x r).
 * In 2D only the z components omega[2], domega_dt[2] may be non-zero
 * (MCD_ERR_ARG otherwise).
 *
 * Discrete-SDF body (Sec. 2.5; 2D as in the paper, 3D by the same rule),
 * sdf != NULL: a device array [sdf_n[1]][sdf_n[0]] (2D) or
 * [sdf_n[2]][sdf_n[1]][sdf_n[0]] (3D), x fastest, caller-owned, read by the
 * calls that take the body in stream order, of psi at the body-frame nodes
 * xi = sdf_origin + (i, j[, k]) sdf_h.  A point x maps to
 * xi = R^T (x - centre), R the posture: the rotation by theta about z (2D)
 * or about the unit vector `axis` (3D).  psi(x) and grad psi are the
 * chi_c = 1 quadratic MLS reconstruction (Sec. 3.2, with the weight and
 * r_e / l0 of mcd_params taken in units of sdf_h) over the 3^d nodes around
 * the node nearest to xi, rotated back by R.  `radius` is then the radius
 * of a ball about `centre` that contains the body: beyond
 * rho = radius + (band_over_l0 + 2) l0 psi is |x - centre| - radius (those
 * points lie outside the body's band, where only the sign of psi is used).
 * The nodes 1 .. sdf_n[a] - 2 must span [-rho, rho] along each body axis
 * and sdf_n >= 3, sdf_h > 0, |axis| = 1 in 3D (MCD_ERR_ARG otherwise, also
 * when r_e does not reach the diagonal nodes).  mcd_fluid_force (2D) orders
 * a body's boundary DPs by their polar angle about `centre`: the body must
 * be star-shaped about it. */
typedef struct {
    int id;              /* role id of its boundary DPs (1 .. 15), != wall_id, distinct
                            within one body list (MCD_ERR_ARG otherwise) */
    double centre[3];
    double radius;
    double velocity[3];  /* V_trans of Eq. (velocity_moving_boundary) */
    double dvdt[3];      /* (V_trans^{k+1} - V_trans^k) / dt, Eq. (dvdt_moving_boundary) */
    double omega[3];     /* angular velocity omega^{k+1} */
    double domega_dt[3]; /* (omega^{k+1} - omega^k) / dt */
    double theta;        /* posture angle of a discrete-SDF body's frame */
    double axis[3];      /* its rotation axis (3D; unit length); 2D: z, not read */
    const double* sdf;   /* NULL: the circle/sphere psi above; else a discrete SDF (above) */
    int sdf_n[3];        /* nodes along the body-frame axes (sdf_n[2] unused in 2D) */
    double sdf_origin[3];/* body-frame position of node 0 */
    double sdf_h;        /* node spacing */
} mcd_body;

/* Boundary condition of one field per role id (Eq. set: Dirichlet DPs are
 * value rows, Neumann DPs are normal-derivative rows of the MLS fit). */
typedef struct {
    int type[MCD_MAX_IDS];   /* index = role id; MCD_BC_DIRICHLET / MCD_BC_NEUMANN */
    int pin_first;           /* 1: DP 0 is a known value (periodic PPE) */
} mcd_bc_table;

typedef struct mcd_ctx mcd_ctx;

/* ---------------------------------------------------------------------
 * Context
 * ------------------------------------------------------------------- */

/* Creates a context for one mesh on the current HIP device.  hip_stream is a
 * hipStream_t (NULL = default stream).  Allocates all workspaces: stencil
 * storage for MCD_MAX_SETS sets, Krylov vectors and reduction scratch.
 * Errors: MCD_ERR_ARG for an invalid mesh/params, MCD_ERR_OOM. */
mcd_status mcd_create(const mcd_mesh_desc* mesh, const mcd_params* prm, void* hip_stream,
                      mcd_ctx** out);
/* Releases ctx: waits for its stream, then frees its device memory.  An open
 * recording of ctx itself is abandoned.  While any context of the process
 * has a recording open (mcd_graph_begin .. mcd_graph_end), the release is
 * deferred until the last such recording ends, because freeing memory or
 * waiting for a stream during a recording can make the runtime invalidate
 * it; the caller must not use ctx after this call either way. */
void mcd_destroy(mcd_ctx* ctx);
/* Contexts and models whose release is deferred (see mcd_destroy). */
int mcd_pending_destroys(void);
mcd_status mcd_set_stream(mcd_ctx* ctx, void* hip_stream);
/* Waits for the context's stream and returns latched device errors
 * (MCD_ERR_SINGULAR, MCD_ERR_ROLE), clearing them. */
mcd_status mcd_sync(mcd_ctx* ctx);
const char* mcd_last_error(const mcd_ctx* ctx);

/* ---------------------------------------------------------------------
 * DP rearrangement and role reassignment (Sec. 2.2 - 2.4)
 * ------------------------------------------------------------------- */

typedef struct {
    int sweeps;             /* relaxation sweeps executed */
    int band_cells;         /* cells in the re-positioned band */
    int counts[9];          /* transition codes: 3*cls(old)+cls(new), cls: void 0, inner 1, boundary 2 */
    int role_errors;        /* void->inner plus inner->void transitions */
} mcd_update_info;

/* One rearrangement at the bodies' new state t^{k+1}:
 *  1. pos_prev := pos, role_prev := role;
 *  2. role := mask of each cell from the number of its vertices with
 *     psi >= 0 (2D: 4 inner, 2-3 boundary, 0-1 void; 3D: 8 / 4-7 / <= 3),
 *     the boundary id being the body of smallest |psi| at the centroid;
 *     wall DPs are moved onto the walls; trans := transition code;
 *  3. up to max_sweeps Jacobi sweeps over the band (non-void, non-wall cells
 *     whose centroid has min |psi| < band): spring relaxation (Eqs.
 *     resultant_force .. 1st_intermed_position), SDF projection of body DPs
 *     (Eq. 2nd_intermed_position) and the mesh-constraint clamp; stops after
 *     the first sweep whose max |dx| <= eps_relax l0;
 *  4. normal := unit normal pointing into the fluid at boundary DPs, 0
 *     elsewhere.
 * Arrays: pos, pos_prev, normal [dim][Nc] f64; role, role_prev [Nc] i8;
 * trans [Nc] u8.  bodies: host array of n_bodies (<= MCD_MAX_BODIES).
 * Bit-exact contract: only + - * / sqrt min max, no contraction.
 * info (host, nullable): when given the call synchronises and fills it;
 * role errors are then returned directly as MCD_ERR_ROLE. */
mcd_status mcd_update_dps(mcd_ctx* ctx, const mcd_body* bodies, int n_bodies, int max_sweeps,
                          double* pos, int8_t* role, double* pos_prev, int8_t* role_prev,
                          uint8_t* trans, double* normal, mcd_update_info* info);

/* ---------------------------------------------------------------------
 * MLS stencils (Sec. 3.2, chi_c = 1)
 * ------------------------------------------------------------------- */

/* Builds the quadratic MLS weights of every non-void DP into context slot
 * `set` (0 .. MCD_MAX_SETS-1), minimising J of Eq. (obj_func) with
 * phi_c fixed: value rows from inner and Dirichlet neighbours of the 3x3
 * (3x3x3) block, normal-derivative rows from Neumann neighbours (and the DP
 * itself when it is Neumann), weight cos^2(pi r / 2 r_e) (r <= r_e).
 * Also builds the PPE matrix of the set (Laplacian weights over unknown
 * rows/columns: inner and Neumann DPs minus the pinned DP) in FP64 and FP32.
 * normal: [dim][Nc] (read at Neumann DPs).  bc: host.
 * Singular inner DPs latch MCD_ERR_SINGULAR (weights set to 0); singular
 * boundary DPs are counted only. */
mcd_status mcd_build_stencils(mcd_ctx* ctx, int set, const double* pos, const int8_t* role,
                              const double* normal, const mcd_bc_table* bc);

/* Copies the weights of a set into caller memory (for inspection / tests):
 * phi [nb][S+1][Nc] f64 with nb = 5 (2D) / 9 (3D), S = 9 / 27 slots in
 * lexicographic order (x fastest), slot (S-1)/2 = -sum of value weights,
 * slot S = the DP's own Neumann row; masks [2][Nc] u32 (bit s of masks[0]:
 * slot s is a value row; bit s of masks[1]: slot s is a Neumann row, bit S:
 * own Neumann row); amat [S][Nc] f64 PPE matrix over the unknown rows and
 * columns (nullable; the library's own copy also keeps the weights of known
 * value neighbours, which the export sets to 0). */
mcd_status mcd_get_stencils(mcd_ctx* ctx, int set, double* phi, uint32_t* masks, double* amat);

typedef enum {
    MCD_OP_PHI = 0,    /* out[nb][Nc]: polynomial coefficients Phi (ncomp must be 1) */
    MCD_OP_GRAD = 1,   /* out[dim][Nc] = grad in (ncomp 1) */
    MCD_OP_LAP = 2,    /* out[ncomp][Nc] = laplacian of each component */
    MCD_OP_DIV = 3,    /* out[1][Nc] = div in (ncomp = dim) */
    MCD_OP_SHIFT = 4   /* out[ncomp][Nc] = in_c + p(shift/r_s) . Phi (Eq. intrp_chi_1) */
} mcd_op;

/* Applies set weights to a field: Phi = sum_value W_j (in_j - in_c) +
 * sum_Neumann W^N_j f_j; derivatives d/dx_a = Phi_a / r_s, laplacian =
 * sum of the pure second-derivative components / r_s^2.
 * in [ncomp][Nc]; neumann_f [ncomp][Nc] Neumann data (NULL = 0);
 * shift [dim][Nc] (MCD_OP_SHIFT only); out as listed per op.
 * Void DPs get 0. */
mcd_status mcd_apply(mcd_ctx* ctx, int set, int op, const double* in, int ncomp,
                     const double* neumann_f, const double* shift, double* out);

/* ---------------------------------------------------------------------
 * Fractional-step glue (Sec. 3.3, Appendix A)
 * ------------------------------------------------------------------- */

/* u~ = u^k(x^{k+1}) (Eq. ale_vel, second order = chi_c = 1 Taylor shift)
 * with the step-k weights of set_prev:
 *  inner->inner: Eq. (A.1) at the DP itself;
 *  boundary/void->inner: Eq. (A.2) centred on c' = cell(c + s), s_a =
 *   sign of (x^k_c - centre^k)_a of its step-k body (support shifted into
 *   the fluid, Sec. 3.4); if c' was not inner at step k the DP's own step-k
 *   weights are used;
 *  -> body boundary: the body's velocity V(x) at x = pos; -> wall or void: 0.
 * u, out [dim][Nc]; bodies_prev / bodies_new: host arrays (same order). */
mcd_status mcd_remap(mcd_ctx* ctx, int set_prev, const double* u, const double* pos_prev,
                     const double* pos, const int8_t* role_prev, const int8_t* role,
                     const mcd_body* bodies_prev, const mcd_body* bodies_new, int n_bodies,
                     double* out);

/* u* = F_MOC + nu dt lap u~ at inner DPs (Eq. intermed_vel); F_MOC is the
 * chi_c = 1 Taylor value of u~ at x - u~ dt with the weights of `set`.
 * Body DPs take the body velocity V(x) at their position, walls and void 0.
 * ut, ustar [dim][Nc]; pos [dim][Nc] (nullable when no body rotates:
 * omega = 0; MCD_ERR_ARG otherwise).  rhs [Nc] (nullable) := div u* / dt
 * with the same set (Eq. pressure_poisson); it is computed in a second pass
 * after u* is complete. */
mcd_status mcd_advect_diffuse(mcd_ctx* ctx, int set, const double* ut, double dt, double nu,
                              const double* pos, const int8_t* role, const mcd_body* bodies, int n_bodies,
                              double* ustar, double* rhs);

/* f = -dV/dt(x) . n at body DPs (Eqs. neumann_moving_boundary,
 * dvdt_moving_boundary), 0 elsewhere.  pos [dim][Nc] as above (nullable when
 * omega = domega_dt = 0 for every body). */
mcd_status mcd_neumann_pressure(mcd_ctx* ctx, const double* pos, const int8_t* role, const double* normal,
                                const mcd_body* bodies, int n_bodies, double* f);

/* u^{k+1} = u* - dt grad P at inner DPs (Eq. projection) with the weights of
 * pressure set `set` and Neumann data f; body DPs take the body velocity
 * V(x); pos as for mcd_advect_diffuse. */
mcd_status mcd_project(mcd_ctx* ctx, int set, const double* P, const double* f,
                       const double* ustar, double dt, const double* pos, const int8_t* role,
                       const mcd_body* bodies, int n_bodies, double* u);

/* Fluid force on each body (Sec. 3.4, evaluation of fluid forces acting on
 * moving boundaries), 2D meshes: F = sum over the body's boundary DPs i of
 * t_i dGamma_i, t = (-P I + mu (grad u + grad u^T)) . n, n = normal[.][i]
 * (the unit normal into the fluid, as written by mcd_update_dps).  dGamma_i
 * is the mean distance from x_i to its two neighbouring boundary DPs, the
 * neighbours being the predecessor and successor in the order of the polar
 * angle about the body centre (ties by cell index).  P and grad u at x_i are
 * the chi_c = 1 reconstruction (Eq. intrp_chi_1 and its derivative) of the
 * support shifted into the fluid: the fit of the cell one step along
 * sign(n_x), sign(n_y) (no step for a zero component), evaluated at x_i;
 * when that cell is not an inner DP the DP's own fit is used (counted).
 * set_u: velocity weights (body DPs Dirichlet, holding the body velocity in
 * u [2][Nc]); set_p: pressure weights with their Neumann data neumann_f
 * [Nc] (NULL = 0) and p [Nc].  mu: dynamic viscosity.  force: host
 * [n_bodies][2], in the order of `bodies`; counts: host [n_bodies][2] or
 * NULL: boundary DPs and fallbacks.  At most 4096 boundary DPs per body
 * (MCD_ERR_ARG beyond).  Synchronises. */
mcd_status mcd_fluid_force(mcd_ctx* ctx, int set_u, int set_p, const double* u, const double* p,
                           const double* neumann_f, const double* pos, const int8_t* role, const double* normal,
                           const mcd_body* bodies, int n_bodies, double mu, double* force, int* counts);

/* ---------------------------------------------------------------------
 * Pressure Poisson solve (Eq. pressure_poisson, Bi-CGSTAB)
 * ------------------------------------------------------------------- */

typedef struct {
    double tol;          /* stop when ||b - A x||_2 <= tol ||b||_2 over unknown rows */
    int max_iter;        /* total Bi-CGSTAB iterations (all restarts/refinements) */
    int precision;       /* MCD_PREC_FP64, MCD_PREC_FP32_REFINE or MCD_PREC_FP32_MATRIX */
    int guess;           /* MCD_GUESS_ZERO or MCD_GUESS_CALLER (p on entry) */
    double inner_tol;    /* FP32_REFINE: relative recurrence residual of each FP32 inner solve
                            (about 1e-2: FP32 Krylov stalls near cond(A) u_32);
                            FP32_MATRIX: the residual is replaced once the recursive residual is
                            below inner_tol times its largest value since the last
                            replacement (about 0.03) */
    int max_outer;       /* FP32_REFINE: refinement steps; FP32_MATRIX: replacements before plain
                            FP64 Bi-CGSTAB takes over */
    int check_every;     /* iterations between host convergence checks (16 = graph chunk) */
    int max_inner;       /* FP32_REFINE: cap on inner iterations per refinement step (0 = none) */
    double fp64_below;   /* FP32_MATRIX: once the residual is below fp64_below times ||b||, the
                            products read the FP64 matrix and replacements stop (0 = never;
                            about 1e-2: the FP32 products' error on smooth modes costs
                            iterations near the tolerance) */
    int precond;         /* MCD_PRECOND_NONE (the plain method) or MCD_PRECOND_JACOBI: right
                            preconditioning with the diagonal D of the PPE matrix, done by
                            solving (A D^-1) y = b and returning x = D^-1 y; the scaled matrix
                            is formed once per solve in the workspace (FP64, plus its FP32 copy
                            for the FP32 modes), the residual and the stopping rule stay those
                            of A x = b, and the tolerance is confirmed on A (a miss is finished
                            by unpreconditioned FP64 Bi-CGSTAB within max_iter).  Columns with
                            a zero or non-finite diagonal are not scaled.
                            MCD_PRECOND_MG (precision FP64 or FP32_MATRIX; FP32_REFINE is
                            refused with MCD_ERR_ARG): Bi-CGSTAB with FP64 vectors and inner
                            products, its matrix products with the FP64 matrix (FP64) or with
                            the FP32 copy in difference form (FP32_MATRIX; fp64_below and the
                            inner options are not used), right-preconditioned by one
                            multigrid V-cycle in FP32
                            (geometric coarsening by 2 per axis down to at most 64 cells,
                            multilinear prolongation, averaging restriction, Galerkin coarse
                            operators R A P built for every solve, one damped-Jacobi sweep
                            (0.8) before and after each coarse correction, dense solve on the
                            coarsest level); the tolerance is confirmed with the FP64 matrix,
                            and a run that misses it restarts from that residual; MCD_ERR_ARG
                            when the mesh cannot be coarsened that far (an odd periodic axis or
                            an axis below 6 cells). */
} mcd_solve_opts;

typedef struct {
    int iterations;           /* Bi-CGSTAB iterations executed */
    int restarts;             /* restarts of the recursion (true-residual check failed,
                                 breakdown, stall, hand-over to FP64) */
    int refinements;          /* refinement steps (FP32_REFINE) or residual replacements
                                 (FP32_MATRIX) */
    int converged;
    double true_rel_residual; /* ||b - A64 x|| / ||b|| in FP64 at exit */
    double rhs_norm;          /* ||b|| of the effective right-hand side */
} mcd_solve_info;

/* Solves the PPE of set `set`: unknown rows are inner DPs and Neumann DPs
 * (collocated with their own Neumann row), Dirichlet DPs (and the pinned DP)
 * are known.  rhs [Nc]: right-hand side at unknown rows; neumann_f [Nc]:
 * Neumann data (NULL = 0); p [Nc]: on entry the known values at known DPs
 * (and the initial guess at unknown DPs for MCD_GUESS_CALLER); on exit the
 * solution at unknown DPs (known DPs unchanged).  Synchronises; info is host
 * memory.  Returns MCD_ERR_NOT_CONVERGED if the tolerance was not met. */
mcd_status mcd_solve_ppe(mcd_ctx* ctx, int set, const double* rhs, const double* neumann_f,
                         double* p, const mcd_solve_opts* opts, mcd_solve_info* info);

/* One V-cycle of the multigrid preconditioner (MCD_PRECOND_MG) of set's PPE
 * matrix: out ~ A^-1 in, with the hierarchy built from the set (not from
 * the paper: the preconditioner of the mixed form).  in: [Nc] f64 device,
 * read at unknown cells; out: [Nc] f64 device, zero at other cells;
 * levels: host int, the number of levels.  Synchronises.  MCD_ERR_ARG for
 * an unbuilt set or a mesh that cannot be coarsened to 64 cells. */
mcd_status mcd_mg_apply(mcd_ctx* ctx, int set, const double* in, double* out, int* levels);

/* Residual of the PPE of set `set` at p (Sec. 3.3, the pressure Poisson
 * equation as assembled for mcd_solve_ppe): r = b_eff - A p on unknown rows,
 * where b_eff is rhs with the Dirichlet columns (values of p at known DPs)
 * and the Neumann data moved over; r = 0 at other cells.  rhs, neumann_f
 * (nullable), p, r: [Nc] f64 device.  norms: host [2] = (||r||_2,
 * ||b_eff||_2): then the call synchronises and returns MCD_ERR_ARG for a
 * non-finite right-hand side.  norms NULL: the call only enqueues r on the
 * context's stream and returns at once, without checking the right-hand
 * side (a non-finite value reaches r; mcd_solve_ppe on the same right-hand
 * side reports it).  MCD_ERR_ARG for an unbuilt set or a null array. */
mcd_status mcd_ppe_residual(mcd_ctx* ctx, int set, const double* rhs, const double* neumann_f, const double* p,
                            double* r, double* norms);

/* For callers that cannot allocate device memory at call time (a tight
 * serving loop, a harness that forbids hipMalloc): mcd_ppe_residual with the
 * same arguments, results and errors (r and norms equal to its own, bit for
 * bit), that allocates nothing and touches no workspace of ctx.  Its scratch
 * (per-block partial sums, the two norms, a counter) is a fixed device array
 * of mcd_noalloc_scratch_bytes() bytes (about 16 KB) per device, held from
 * the first mcd_create on that device until the process ends; it does not
 * grow with the mesh (the residual runs at most 1024 blocks), so no mesh
 * size is beyond it.  Every call on a device shares that array: calls that
 * overlap on one device (other threads, other streams) race and must be
 * serialised by the caller.  Synchronises the context's stream. */
mcd_status mcd_ppe_residual_noalloc(mcd_ctx* ctx, int set, const double* rhs, const double* neumann_f,
                                    const double* p, double* r, double* norms);
/* Size in bytes of the per-device scratch of mcd_ppe_residual_noalloc. */
size_t mcd_noalloc_scratch_bytes(void);

/* ---------------------------------------------------------------------
 * Learned PPE initial guess (2D and 3D): a U-Net on the background mesh.
 * Not part of the MCD method: a network that corrects the warm start of the
 * solve.  One DP per cell makes the DP arrays channels-last images: (y, x)
 * in 2D, (z, y, x) in 3D, x fastest.
 * Inputs: r / rms(r), where r is the PPE residual of the warm start p_prev
 * (mcd_ppe_residual), p_prev / rms(p_prev), one-hot roles (inner, body,
 * wall); output h; guess = p_prev + s rms(r) h at unknown cells (FP64), s =
 * the model's output scale.  rms over unknown cells (1 where it is 0).
 * Levels L: per level two 3x3 (3x3x3) convolutions with ReLU, 2x2 (2x2x2)
 * mean pooling down, nearest 2x upsampling and concatenation with the skip
 * up, a 3x3 (3x3x3) head to one channel.  BF16 weights and activations, FP32 accumulation on the matrix
 * cores; FP32 master weights trained with Adam.
 * Parameters: flat FP32 vector, convolutions in the order enc0a, enc0b, ...,
 * enc(L-1)b, dec(L-2)a, dec(L-2)b, ..., dec0a, dec0b, head, each W[T][cin][cout]
 * then b[cout]; T = 9 taps in 2D (tap t = 3 dy + dx, offset (dx - 1, dy - 1)),
 * 27 in 3D (t = 9 dz + 3 dy + dx, offset (dx - 1, dy - 1, dz - 1)).
 * ------------------------------------------------------------------- */

typedef struct mcd_model mcd_model;

/* channels: host array of `levels` (2..5) widths, multiples of 16 in
 * [16, 256]; every mesh axis must be divisible by 2^(levels-1).  body_id: role id
 * of the body for the one-hot input.  Weights start at zero (set them). */
mcd_status mcd_model_create(mcd_ctx* ctx, int levels, const int* channels, int body_id, mcd_model** out);
/* Releases a model (deferred like mcd_destroy while a recording is open). */
void mcd_model_destroy(mcd_model* model);
size_t mcd_model_num_params(const mcd_model* model);
/* host arrays of mcd_model_num_params floats; set resets the optimiser */
mcd_status mcd_model_set_params(mcd_model* model, const float* theta, size_t n);
mcd_status mcd_model_get_params(mcd_model* model, float* theta, size_t n);
/* gradient of the loss of the last training step (host array) */
mcd_status mcd_model_get_grads(mcd_model* model, float* grad, size_t n);
/* copy of the head output h [Nc] of the last forward pass (device, FP32) */
mcd_status mcd_model_output(mcd_model* model, float* h);
/* output scale s > 0 (default 1): the typical size of the correction in
 * units of rms(r); a training set fixes it once */
mcd_status mcd_model_set_output_scale(mcd_model* model, double s);
/* p_out := p_prev + s rms(resid) h at unknown cells (rows of bc); other cells
 * of p_out untouched.  resid = mcd_ppe_residual of p_prev; resid, p_prev,
 * p_out [Nc] f64, role [Nc] i8 (device); bc host.  p_out may alias p_prev. */
mcd_status mcd_model_infer(mcd_model* model, const double* resid, const double* p_prev, const int8_t* role,
                           const mcd_bc_table* bc, double* p_out);
/* One Adam step (lr > 0; lr = 0 computes the gradient only) on the loss
 * sum_unknown (h - t)^2 / sum_unknown t^2, t = (p_target - p_prev) / (s rms(resid)).
 * loss: host, nullable (synchronises when given). */
mcd_status mcd_model_train_step(mcd_model* model, const double* resid, const double* p_prev, const double* p_target,
                                const int8_t* role, const mcd_bc_table* bc, double lr, double* loss);

/* ---------------------------------------------------------------------
 * Launch shape of the Krylov stage kernels and its autotuner
 *
 * The stage kernels of mcd_solve_ppe (Bi-CGSTAB, Sec. 3.3) give each block
 * of 512 threads a contiguous run of 64 x 8-cell tiles (2D) or of
 * 64 x 8 x depth-cell bricks marched plane by plane (3D).  The shape is the
 * block count `grid` (1..512; clipped to the number of tiles) and, in 3D, the
 * brick depth in planes (1..n_z; 1 in 2D).  Default: grid 512, depth 8.  The
 * shape changes the summation order of the dot products (results stay
 * within the solve's tolerance; for one shape they are run-to-run
 * bit-identical).
 * ------------------------------------------------------------------- */

#define MCD_TUNE_MAX 32
typedef struct {
    int n;                           /* candidates timed */
    int grid[MCD_TUNE_MAX];          /* block count asked for */
    int depth[MCD_TUNE_MAX];         /* 3D brick depth (1 in 2D) */
    double us_per_iter[MCD_TUNE_MAX];/* FP64 P- + S-stage microseconds per iteration (best of two
                                        runs); < 0: rejected (the timing recursion stopped early) */
    int chosen;                      /* index now in use (-1: none usable, shape unchanged) */
} mcd_tuning;

/* Times every candidate shape on the FP64 operator of built set `set`
 * (iters >= 1 iterations of a problem with b = 1 at the unknown rows, after
 * two untimed ones, each candidate twice), then applies the fastest; the
 * default shape is kept when it is within 2 % of the fastest.  Uses the
 * solver workspace (the next solve overwrites it) and synchronises.  out:
 * host. */
mcd_status mcd_autotune(mcd_ctx* ctx, int set, int iters, mcd_tuning* out);
/* Applies a shape (e.g. one found earlier by mcd_autotune); MCD_ERR_ARG when
 * outside the limits above. */
mcd_status mcd_set_shape(mcd_ctx* ctx, int grid, int depth);
/* The shape in use: block count asked for, brick depth, and the blocks
 * launched (grid clipped to the tiles).  Host pointers. */
mcd_status mcd_get_shape(mcd_ctx* ctx, int* grid, int* depth, int* blocks);

/* ---------------------------------------------------------------------
 * Kernel timing (measurement aid)
 * ------------------------------------------------------------------- */

/* enable = 1: every P-stage and S-stage kernel launch of later
 * mcd_solve_ppe calls is bracketed by HIP events on the context's stream
 * (the events are created on the first enable; at most 4096 iterations are
 * timed per restart cycle).  Launches that only observed convergence and
 * returned are excluded.  enable = 0 stops recording. */
mcd_status mcd_profile(mcd_ctx* ctx, int enable);
/* Accumulated milliseconds and launch counts of the working P- and S-stage
 * launches since the last reset (all host pointers). */
mcd_status mcd_profile_read(mcd_ctx* ctx, double* ms_p, long long* n_p, double* ms_s, long long* n_s,
                            int reset);
/* The same split by the matrix copy the launches read, so that their bytes
 * can be counted from the matrix they actually read: ms[4] and n[4] (host)
 * receive, in this order, P-stage and S-stage launches on the FP64 matrix,
 * then P-stage and S-stage launches on the FP32 matrix (FP32_MATRIX and
 * FP32_REFINE solves). */
mcd_status mcd_profile_read_split(mcd_ctx* ctx, double* ms, long long* n, int reset);

/* ---------------------------------------------------------------------
 * PPE on a wider MLS support (comparison path, 2D)
 * ------------------------------------------------------------------- */

typedef struct {
    int iterations;            /* Bi-CGSTAB iterations */
    int converged;             /* true residual <= tol */
    int singular;              /* unknown DPs whose fit was singular (weights zero) */
    double true_rel_residual;  /* ||b - A x|| / ||b|| over unknown rows */
    double build_ms;           /* GPU time of the weight build and assembly */
    double solve_ms;           /* GPU time of the solve */
} mcd_wide_info;

/* Sec. 4 (flow past stationary cylinders) compares the 3x3 MLS support with
 * an expanded 9x9 one (r_e = 3.5 l0).  This call builds the chi_c = 1
 * quadratic fit of Sec. 3.2 over the (2 half + 1)^2 block of cells around
 * every DP (half 1 .. 4; weight kind and r_s of the context, r_e =
 * re_over_l0 l0), assembles its Laplacian weights into the PPE over the
 * unknown DPs exactly as the sets of mcd_build_stencils do (Dirichlet values
 * taken from p, Neumann data neumann_f, nullable), and solves it with a plain
 * Bi-CGSTAB from p (unknown rows) to ||b - A x|| <= tol ||b||; p receives
 * the solution at unknown rows.  One code path serves every half width (one
 * thread per DP, host-formed scalars each iteration), so 3x3 and 9x9 are
 * compared on equal terms; the production solve is mcd_solve_ppe.  2D only.
 * Synchronises.  Errors: MCD_ERR_ARG, MCD_ERR_SINGULAR (a singular fit at an
 * unknown DP; info still filled; known DPs such as wall corners may be
 * singular and get zero weights), MCD_ERR_NOT_CONVERGED, MCD_ERR_OOM/HIP (the work arrays,
 * (2 half + 1)^2 + 1 planes of Nc doubles and more, are allocated on first
 * use and kept by the context). */
mcd_status mcd_ppe_wide(mcd_ctx* ctx, int half, double re_over_l0, const double* pos, const int8_t* role,
                        const double* normal, const mcd_bc_table* bc, const double* rhs, const double* neumann_f,
                        double* p, double tol, int max_iter, mcd_wide_info* info);
/* Copies the last assembled wide PPE matrix: (2 half + 1)^2 slot planes of
 * Nc doubles (slot s = the cell at offset (s % W - half, s / W - half),
 * W = 2 half + 1; the centre slot holds the diagonal; rows of known DPs are
 * the identity) into the device array A.  Synchronises. */
mcd_status mcd_ppe_wide_matrix(mcd_ctx* ctx, double* A);

/* ---------------------------------------------------------------------
 * Captured call sequences (HIP graphs): the parts of a time step around
 * the PPE solve as one graph launch each
 * ------------------------------------------------------------------- */

/* Starts recording into graph slot `slot` (0 .. MCD_MAX_GRAPHS-1): the
 * calls on this context that follow are recorded on a private stream, not
 * run, until mcd_graph_end.  Recordable are the calls that only enqueue
 * device work: mcd_update_dps with info = NULL, mcd_build_stencils,
 * mcd_get_stencils, mcd_apply, mcd_remap, mcd_advect_diffuse,
 * mcd_neumann_pressure, mcd_project.  The others return MCD_ERR_ARG while a
 * capture is open (mcd_sync, mcd_solve_ppe, mcd_ppe_residual,
 * mcd_fluid_force, mcd_autotune, mcd_set_shape, mcd_profile*, the model
 * calls, mcd_set_stream, mcd_update_dps with info, mcd_ppe_wide*).  Host arguments
 * (bodies, boundary tables, scalars) are copied when a call is recorded;
 * device arrays are referenced and must stay valid until the graph has run.
 * A context records one slot at a time and is used from one thread.  Errors:
 * MCD_ERR_ARG (bad slot, a capture already open), MCD_ERR_HIP. */
mcd_status mcd_graph_begin(mcd_ctx* ctx, int slot);
/* Ends the recording of `slot` and, with launch != 0, launches it on the
 * context's stream.  The first recording of a slot is instantiated; a later
 * one with the same sequence of calls (arguments may differ) updates that
 * executable graph in place, any other replaces it; a slot must not be
 * re-recorded while its previous launch may still be running (alternate
 * slots for work recorded ahead).  If a recorded call failed, nothing runs
 * and MCD_ERR_ARG is returned (with that call's message).  Device-side
 * results are those of the same calls made directly, bit for bit. */
mcd_status mcd_graph_end(mcd_ctx* ctx, int slot, int launch);
/* Launches slot's executable graph (as last recorded) on the context's
 * stream; MCD_ERR_ARG if the slot holds none. */
mcd_status mcd_graph_launch(mcd_ctx* ctx, int slot);
/* How often slot's graph was instantiated and updated in place (host ints). */
mcd_status mcd_graph_stats(mcd_ctx* ctx, int slot, int* instantiated, int* updated);

#ifdef __cplusplus
}
#endif

#endif /* MCD_H */
