/*
 * hpmg.h - C ABI of the MI355X (gfx950) matrix-free Neo-Hookean operator and its
 * p-multigrid solver (arXiv:2204.01722, "Performance-Portable Solid Mechanics via
 * Matrix-Free p-Multigrid").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function is extern "C", returns an hpmg_status (0 = HPMG_OK), never throws
 *   and never exits.  On failure hpmg_last_error() (thread-local) holds a message.
 * - Device buffers are owned by the caller (the Python layer allocates them with
 *   PyTorch); the library performs no device allocation.  Handles own host metadata
 *   only and borrow every device pointer passed to them, which must outlive the handle.
 * - All device work is enqueued on the hipStream_t passed as `stream` (NULL = default
 *   stream) and is asynchronous unless a function says it synchronises.
 * - L-vectors are [n_nodes][3] with the three displacement components interleaved.
 *   Element-to-node maps are int32 [n_elem][P^3], element-local nodes lexicographic
 *   with xi_1 fastest.  Pointers must be 8-byte aligned (PyTorch allocations are).
 * - Argument and shape errors are detected on the host before any launch.  Errors
 *   found on the device (non-positive Jacobian determinant, non-finite values) set
 *   bits in a per-operator flag word read by hpmg_op_query_flags.
 * - Dirichlet mask (uint8 [n_nodes][3], 1 = constrained component): the residual's
 *   constrained rows are zero; the Jacobian apply is M J M + (I - M) with
 *   M = diag(1 - mask) (constrained rows are the identity); the diagonal is 1 there.
 * - Outputs are overwritten, not accumulated, unless the name says "add".
 * - Handles are not thread-safe; distinct handles may be used from distinct threads.
 */
#ifndef HPMG_H
#define HPMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HPMG_OK = 0,
  HPMG_ERR_ARG = 1,           /* null pointer, bad enum, bad scalar */
  HPMG_ERR_SHAPE = 2,         /* sizes inconsistent with the handle */
  HPMG_ERR_UNSUPPORTED = 3,   /* (P, Q) pair or mode not compiled */
  HPMG_ERR_WORKSPACE = 4,     /* workspace missing or too small */
  HPMG_ERR_HIP = 5,           /* a HIP runtime call failed */
  HPMG_ERR_NONPOSITIVE_J = 6, /* a determinant <= 0 was found on the device */
  HPMG_ERR_NONFINITE = 7,     /* NaN/Inf found on the device */
  HPMG_ERR_BREAKDOWN = 8,     /* Krylov breakdown (p^T A p <= 0 or 0/0) */
  HPMG_ERR_NOT_CONVERGED = 9  /* iteration limit reached */
} hpmg_status;

typedef enum { HPMG_F64 = 0, HPMG_F32 = 1 } hpmg_precision;
typedef enum {
  HPMG_STORED = 0,         /* the current-configuration state (Section III-B), 16 scalars */
  HPMG_RECOMPUTE = 1,      /* rebuilt from u and the geometric factors */
  HPMG_INITIAL_NATIVE = 2, /* initial configuration, 19 scalars: W, grad_X xi; grad_X u */
  HPMG_INITIAL_TUNED = 3,  /* initial configuration, 26 scalars: + C^-1, lambda log J */
  HPMG_CURRENT_20 = 4      /* current configuration, 20 scalars: dxi/dx, J, grad_X u, W */
} hpmg_mode;

/* Device flag bits reported by hpmg_op_query_flags. */
#define HPMG_FLAG_NONPOSITIVE_J 1u
#define HPMG_FLAG_NONFINITE 2u
#define HPMG_FLAG_BAD_INDEX 4u

typedef struct hpmg_op_s *hpmg_op;
typedef struct hpmg_mg_s *hpmg_mg;

/* ---------------------------------------------------------------------------------
 * Diagnostics
 * --------------------------------------------------------------------------------- */
const char *hpmg_status_string(int status);
/* Message of the last failing call on this thread ("" if none). */
const char *hpmg_last_error(void);
/* Library version string and the HIP device architecture it was compiled for. */
const char *hpmg_version(void);

/* ---------------------------------------------------------------------------------
 * Reference-element tables (Section II-B, eq. tensorDense; host only, no GPU needed).
 * P = p + 1 Gauss-Lobatto nodes, Q Gauss-Legendre points on [-1, 1].
 *   interp [Q][P]  B_I[q][i]  = l_i(x_q)
 *   grad   [Q][P]  B_xi[q][i] = l_i'(x_q)
 *   colloc [Q][Q]  collocated derivative B_xi B_I^+ (requires Q >= P, Section II-B)
 *   qref [Q], qweight [Q], gll [P]
 * Any output pointer may be NULL.  Returns HPMG_ERR_ARG for P < 2, Q < P or Q > 16.
 * --------------------------------------------------------------------------------- */
int hpmg_basis_tabulate(int P, int Q, double *interp, double *grad, double *colloc,
                        double *qref, double *qweight, double *gll);
/* Coarse-to-fine interpolation table [Pf][Pc]: coarse Lagrange basis (Pc GLL nodes)
 * evaluated at the Pf GLL nodes (the 1D factor of B_ctof in eq. mg_prolong). */
int hpmg_basis_ctof(int Pf, int Pc, double *ctof);

/* ---------------------------------------------------------------------------------
 * Operator handles (one per multigrid level; eq. libceed_representation restricted
 * to one device: E^T B^T D B E).
 * --------------------------------------------------------------------------------- */
/* Fine operator: order P-1 elements with Q^3 Gauss points.  elem_nodes: device int32
 * [n_elem][P^3] with ids in [0, n_nodes); mask: device uint8 [n_nodes][3] or NULL.
 * Supported (P, Q): 2 <= P <= 5, P <= Q <= 5 (and (5, 6)). */
int hpmg_op_create(int P, int Q, int64_t n_elem, int64_t n_nodes, const int32_t *elem_nodes,
                   const uint8_t *mask, hpmg_op *out);
/* Coarse operator on the same elements and the same quadrature points as `fine`,
 * with basis order Pc - 1 (Pc < fine P).  It reuses the fine operator's geometric
 * factors and stored linearisation, which makes it the exact Galerkin coarse operator
 * (Section III-B).  `fine` must outlive it. */
int hpmg_op_create_coarse(hpmg_op fine, int Pc, int64_t n_nodes, const int32_t *elem_nodes,
                          const uint8_t *mask, hpmg_op *out);
void hpmg_op_destroy(hpmg_op op);
/* Lame parameters: scalars, or per-element device arrays [n_elem] (used when non-NULL;
 * both must then be given).  Copied to the coarse operators that share the state. */
int hpmg_op_set_material(hpmg_op op, double mu, double lambda, const double *mu_e,
                         const double *lambda_e);
/* Device workspace needed by the operator (tables, geometric factors, stored
 * linearisation in FP64 and FP32, element records and node incidence lists for the
 * assembly, reduction scratch, flags). */
int hpmg_op_workspace_bytes(hpmg_op op, size_t *bytes);
/* Binds a caller-owned device buffer of at least the queried size (256-byte aligned)
 * and uploads the reference tables; enqueued on `stream`. */
int hpmg_op_bind_workspace(hpmg_op op, void *workspace, size_t bytes, void *stream);
/* info[0..7] = P, Q, n_elem, n_nodes, elements per tile, tiles, threads per block,
 * quadrature-array stride per field. */
int hpmg_op_info(hpmg_op op, int64_t *info);
/* Version of the stored linearisation that `op` applies (the fine operator's, for a
 * coarse operator that shares it): a counter bumped by every call that overwrites it
 * (hpmg_residual with store_state, multigrid setups and the Newton and L-BFGS drivers).
 * Lets a caller detect that the state it linearised at has since been replaced. */
int hpmg_op_state_version(hpmg_op op, uint64_t *version);
/* Reads and clears the device flag word (synchronises `stream`). */
int hpmg_op_query_flags(hpmg_op op, void *stream, unsigned *flags);

/* a1: geometric factors (Section II-B: W = w_hat det(dX/dxi), and dxi/dX) from node
 * coordinates, device double [n_nodes][3] (fine operators only).  Sets
 * HPMG_FLAG_NONPOSITIVE_J if an element is inverted. */
int hpmg_qdata_setup(hpmg_op op, const double *coords, void *stream);
/* Copies the geometric factors out as double [n_elem][10][Q^3] (W, then dxi_k/dX_J
 * row-major), for inspection and tests. */
int hpmg_qdata_export(hpmg_op op, double *out, void *stream);

/* a2-a7: residual F(u) of eq. residual-discrete-ref with f_1 = Kirchhoff stress
 * (eq. Kirchhoff-stress) pulled back to reference coordinates.  u, r: device double
 * [n_nodes][3].  With store_state != 0 it also stores the linearisation of the
 * current-configuration form (Section III-B, Table different-storage: dxi/dx, tau,
 * lambda log J and the weight W, 17 scalars) as 16: sqrt(W) dxi/dx, tau, lambda log J
 * (every use is W times a form bilinear in dxi/dx), used by stored-mode Jacobian
 * applies, the diagonal, the element matrices and the adjoint of this operator and its
 * coarse operators. */
int hpmg_residual(hpmg_op op, const double *u, double *r, int store_state, void *stream);

/* a5/a5': Jacobian action y = J(u) du (eqs. Jacobian, dtau, Jacobian-discrete-ref).
 *   precision HPMG_F64: du, y double; HPMG_F32: du, y float (FP32 state and FP32
 *   accumulation; requires hpmg_state_cast_f32 after the last state update).
 *   mode HPMG_STORED reads the stored linearisation (u unused, may be NULL);
 *   HPMG_RECOMPUTE rebuilds it from u (double [n_nodes][3]) and the geometric
 *   factors (fine operators only, precision HPMG_F64 or HPMG_F32);
 *   HPMG_INITIAL_NATIVE / HPMG_INITIAL_TUNED apply the same operator written in the
 *   initial configuration (S(E) form, Table different-storage) from the geometric
 *   factors and the linearisation stored by hpmg_state_initial; HPMG_CURRENT_20 applies
 *   the current-configuration form from dxi/dx, J, grad_X u and W (tau and lambda log J
 *   rebuilt per point) from the same buffer (fine operators, HPMG_F64 only). */
int hpmg_jacobian_apply(hpmg_op op, int precision, int mode, const double *u, const void *du,
                        void *y, void *stream);
/* Order-1 operators only (P = 2): builds the dense 24 x 24 element matrices of the
 * operator from its stored linearisation (the element-level triple product B^T D B of
 * Section III-D), in `precision`: for a Galerkin coarse operator the fine operator's
 * linearisation on the fine quadrature, for a stand-alone one its own.  While that
 * linearisation is unchanged, stored-mode applies of this operator in that
 * precision then read the element matrices (symmetric: 300 scalars per element;
 * HPMG_F32 builds them in FP32 from the FP32 state, after hpmg_state_cast_f32)
 * instead of the quadrature-point linearisation.  A new stored linearisation makes them
 * stale; applies fall back to the quadrature form until they are rebuilt. */
int hpmg_op_assemble_elements(hpmg_op op, int precision, void *stream);

/* External dead loads (eq. variational-form, right-hand side): f_ext = int phi rho0 g dV
 * + int phi t dA over the listed element faces, constant per unit reference volume and
 * area.  rho_g (host double[3]) may be NULL (no body force); faces are given by element
 * (device int32 [n_faces]) and local face (device int32 [n_faces]: 0..5 = xi_1 = -1, +1,
 * xi_2 = -1, +1, xi_3 = -1, +1) with coords (device double [n_nodes][3]) and traction
 * (host double[3]).  Constrained components of f_ext are 0.  Sums are in a fixed order.
 * The workspace (hpmg_external_load_workspace_bytes, 256-byte aligned) is needed only
 * when n_faces > 0.  Fine operators; synchronises `stream`. */
int hpmg_external_load_workspace_bytes(hpmg_op op, int64_t n_faces, size_t *bytes);
int hpmg_external_load(hpmg_op op, const double *rho_g, const double *coords, int64_t n_faces,
                       const int32_t *face_elem, const int32_t *face_id, const double *traction,
                       void *workspace, size_t bytes, double *f_ext, void *stream);

/* Alternative linearisations (Table different-storage) at u: grad_X u (9), C^-1 (6,
 * symmetric xx yy zz yz xz xy), lambda log J (1), dxi/dx (9), J - 1 (1) per point,
 * written to a caller-owned device buffer of hpmg_state_initial_bytes() bytes (FP64,
 * [tile][26][ET*Q^3], 256-byte aligned) that the operator then reads in the
 * HPMG_INITIAL_NATIVE, HPMG_INITIAL_TUNED and HPMG_CURRENT_20 Jacobian modes (each
 * reads only its own fields); the buffer must stay allocated while they are used and
 * is not refreshed by hpmg_residual.  Fine operators only. */
int hpmg_state_initial_bytes(hpmg_op op, size_t *bytes);
int hpmg_state_initial(hpmg_op op, const double *u, void *buffer, size_t bytes, void *stream);

/* Casts the stored FP64 linearisation to the FP32 copy used by FP32 applies. */
int hpmg_state_cast_f32(hpmg_op op, void *stream);

/* a8: diagonal of this level's Jacobian (stored linearisation, this level's basis on
 * the shared quadrature), device [n_nodes][3] in `precision`; 1 on constrained rows. */
int hpmg_diagonal(hpmg_op op, int precision, void *diag, void *stream);

/* a11: p-transfer between a coarse operator and its fine operator (eq. mg_prolong):
 *   hpmg_prolong_add: yf += M_f P xc   (P = sum_e E_f^T O_e B_ctof E_c)
 *   hpmg_restrict:    rc  = M_c P^T rf (restriction is the transpose, Section III-B)
 * O_e selects the fine nodes owned by element e (each node has exactly one owner, its
 * first element), which equals the paper's averaging diag(1/m_f) over the m_f elements
 * sharing a node because every element interpolates the same continuous coarse field
 * there.  M masks constrained components.  Deterministic (no atomics).  Vectors in
 * `precision` (double or float). */
int hpmg_prolong_add(hpmg_op coarse, hpmg_op fine, int precision, const void *xc, void *yf,
                     void *stream);
int hpmg_restrict(hpmg_op fine, hpmg_op coarse, int precision, const void *rf, void *rc,
                  void *stream);

/* Strain energy Psi(u) = sum W psi (eq. strain-energy) into a device double scalar. */
int hpmg_energy(hpmg_op op, const double *u, double *psi, void *stream);

/* a16: vector-Jacobian product of the (masked) residual r(u; mu_e, lambda_e):
 *   u_bar = (dr/du)^T w, written as the transposed pointwise map (adjoint kernel),
 *   mu_bar[e] = dr/dmu_e^T w, lambda_bar[e] = dr/dlambda_e^T w  (per element).
 * mode HPMG_STORED uses the linearisation stored by the last hpmg_residual at this u
 * (parameter gradients then need mu_e, lambda_e > 0; FP32 needs hpmg_state_cast_f32);
 * HPMG_RECOMPUTE rebuilds it from u (double).  precision HPMG_F64: w, u_bar double;
 * HPMG_F32: w, u_bar float, FP32 arithmetic (J - 1 and log J in double).  mu_bar /
 * lambda_bar (double [n_elem]) may be NULL. */
int hpmg_residual_vjp(hpmg_op op, int precision, int mode, const double *u, const void *w, void *u_bar,
                      double *mu_bar, double *lambda_bar, void *stream);

/* ---------------------------------------------------------------------------------
 * Vector kernels used by the solvers (deterministic FP64 reductions).
 * n counts scalars (x and y may be NULL when n = 0).  Reductions write a device double
 * and do not synchronise.
 * --------------------------------------------------------------------------------- */
/* scratch: device double buffer of at least HPMG_REDUCE_SCRATCH entries. */
#define HPMG_REDUCE_SCRATCH 2048
int hpmg_vec_dot(int precision, int64_t n, const void *x, const void *y, double *out,
                 double *scratch, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): hpmg_vec_dot without the scratch
 * argument.  Its partial sums live in a library-owned static device array of
 * HPMG_NOALLOC_SCRATCH_DOUBLES doubles (4 KiB) that each GPU holds until the process
 * ends; it allocates nothing and makes no allocating call.  The reduction's grid is
 * fixed, so any n >= 0 fits (no size is too large).  Same kernels, same summation order:
 * the result equals hpmg_vec_dot's bit for bit.  The current device must be the one
 * `stream` belongs to.  Every call on one GPU shares that array: calls that overlap on
 * one GPU (different streams or threads without ordering) race and give wrong sums. */
#define HPMG_NOALLOC_SCRATCH_DOUBLES 512
int hpmg_vec_dot_noalloc(int precision, int64_t n, const void *x, const void *y, double *out,
                         void *stream);
int hpmg_vec_axpby(int precision, int64_t n, double alpha, const void *x, double beta, void *y,
                   void *stream); /* y = alpha x + beta y */
int hpmg_vec_cast(int64_t n, int to_precision, const void *x, void *y, void *stream);

/* ---------------------------------------------------------------------------------
 * p-multigrid preconditioner (Section III-B, Fig. multigrid_algorithm) and solvers.
 * --------------------------------------------------------------------------------- */
typedef struct {
  int cheb_degree;      /* operator applications per smoothing sweep (default 3) */
  double cheb_lo;       /* interval [lo, hi] * lambda_max (defaults 0.1, 1.1) */
  double cheb_hi;
  int lanczos_its;      /* CG/Lanczos iterations for lambda_max (default 10, at most 64) */
  double coarse_rtol;   /* coarsest-level Jacobi-PCG relative tolerance (1e-3) */
  int coarse_maxit;     /* its cap (default 10000) */
  int coarse_fixed_its; /* > 0: run exactly this many coarse iterations (tests) */
  int precision;        /* HPMG_F32: smoothing/transfer/coarse solve in FP32 */
  int coarse_element_matrices; /* 1: order-1 Galerkin coarsest level from element matrices,
                                  assembled into 3 x 3 node blocks for its Jacobi-PCG */
  int coarse_block_layout; /* those blocks: -1 (default) by size, node-major from 65,536
                              coarse nodes; 0: a node's rows contiguous, a thread per row
                              (faster on small coarse levels); 1: each block entry
                              contiguous over the nodes, a thread per node (faster once the
                              blocks stream from HBM).  Same arithmetic either way */
} hpmg_mg_params;

void hpmg_mg_default_params(hpmg_mg_params *p);
/* levels[0] is the fine operator; the coarse levels, of decreasing order, are either
 * all coarse operators of levels[0] (Galerkin: they share its quadrature and state,
 * Section III-B) or all stand-alone operators on the same elements with their own
 * order, quadrature and geometry ("rediscretised": their linearisations are stored at
 * the injected field by hpmg_mg_set_state; needs nested node sets: order 1, or order 2
 * below an even order).  The last level is solved by Jacobi-PCG.  Handles are
 * borrowed. */
int hpmg_mg_create(const hpmg_op *levels, int n_levels, const hpmg_mg_params *params,
                   hpmg_mg *out);
void hpmg_mg_destroy(hpmg_mg mg);
int hpmg_mg_workspace_bytes(hpmg_mg mg, size_t *bytes);
int hpmg_mg_bind_workspace(hpmg_mg mg, void *workspace, size_t bytes);
/* Rediscretised levels only (a no-op otherwise): injects u (device double
 * [n_nodes][3] of levels[0]) level by level and stores each level's linearisation
 * there (a residual evaluation per level).  Call before hpmg_mg_setup whenever the
 * fine linearisation changes; the Newton and L-BFGS drivers do it themselves. */
int hpmg_mg_set_state(hpmg_mg mg, const double *u, void *stream);
/* Per-linearisation setup: FP32 cast of the state (mixed precision), level diagonals
 * and lambda_max of D^{-1}A per smoothed level from `lanczos_its` Jacobi-PCG
 * iterations on the caller's rough vectors seeds[l] (device double [n_nodes_l][3],
 * l = 0 .. n_levels-2).  Synchronises `stream` (reads CG coefficients). */
int hpmg_mg_setup(hpmg_mg mg, const double *const *seeds, void *stream);
/* z = M^{-1} r (one V-cycle, zero initial guess), double in and out.
 * The coarse solve's stopping test runs on the device; the host queues its iterations
 * in batches (the first as long as the previous coarse solve) and synchronises once per
 * batch to read the outcome, or never with coarse_fixed_its. */
int hpmg_mg_vcycle(hpmg_mg mg, const double *r, double *z, void *stream);
/* lambda_max estimate of a level and the last coarse-solve iteration count. */
int hpmg_mg_info(hpmg_mg mg, int level, double *lambda_max, int *last_coarse_its);

/* Counters since creation (host only): out[0] V-cycles, out[1] coarse-solve
 * iterations, out[2] setups, out[3 + l] stored-mode operator applies on level l
 * (l < 8; smoothing, residuals, coarse iterations and eigenvalue estimates). */
int hpmg_mg_stats(hpmg_mg mg, int64_t *out);

/* a14: flexible CG (FP64) on the fine operator, preconditioned by one V-cycle of
 * `mg`.  Solves J x = b from the x passed in; stops at ||b - Jx|| <= rtol ||b - J x0||.
 * A direction of non-positive curvature (p^T J p <= 0, possible when the tangent is
 * indefinite) stops it with HPMG_ERR_BREAKDOWN and x at the iterate reached (x plus the
 * preconditioned residual if it happens before the first step).  Step lengths are
 * formed on the device; synchronises once per iteration. */
int hpmg_fcg_solve(hpmg_op fine, hpmg_mg mg, const double *b, double *x, double rtol, int maxit,
                   int *its, double *relres, void *stream);

/* a15: Newton with load stepping and the critical-point line search (Section III-A).
 * Step k = 1..n_steps adds lift / n_steps to u (lift holds the full imposed displacement
 * on constrained components and an extension elsewhere) and iterates on
 * F(u) = r(u) - (k / n_steps) f_ext (f_ext: external dead load from hpmg_external_load,
 * or NULL) until ||F(u)|| <= rtol ||F(u_start)||.  An increment starts from the secant
 * extrapolation of the last two converged load levels when there are two (predictor = 1),
 * else from the previous converged state plus the lifted increment, whose first
 * correction uses the tangent of that previous state (an Euler predictor); later
 * corrections use the tangent at the current iterate.  Linear solves: FCG + V-cycle to lin_rtol (a negative-
 * curvature breakdown truncates the solve and the line search takes the direction found
 * so far).  A step length whose point has an inverted element or a non-finite residual
 * is halved (at most 6 times).  A load increment whose Newton solve fails (iteration
 * limit, no admissible step, no descent direction) is retried from the previous
 * converged state in halves, at most 6 times in a row; after a converged increment the
 * increment doubles again up to the full step.  When the whole solve has spent
 * max_total_newton Newton or max_total_krylov FCG iterations it stops with
 * HPMG_ERR_NOT_CONVERGED and u at the last converged load level, so a solve that
 * stalls returns in bounded time.  Statistics (host):
 *   stats[0] = total Newton iterations, stats[1] = total FCG iterations,
 *   stats[2] = final relative residual of the last increment, stats[3] = halvings,
 *   stats[4 + k] = Newton iterations spent in load step k (k < n_steps, at most 60). */
typedef struct {
  double rtol;      /* Newton relative residual tolerance (1e-8) */
  int max_newton;   /* per load step (20) */
  double lin_rtol;  /* FCG relative tolerance (1e-3) */
  int lin_maxit;    /* (500) */
  int line_search;  /* 1: critical-point secant step, clipped to [0.1, 1.5] */
  int monitor;      /* (0) 1: one line per Newton iteration on stderr: load, iteration,
                       relative residual, FCG iterations and outcome, step length */
  int max_total_newton; /* (200) Newton iterations of the whole solve, retries included */
  int max_total_krylov; /* (20000) FCG iterations of the whole solve, retries included */
  int predictor;        /* (1) 1: once two load levels have converged, an increment starts
                           from their secant extrapolation (tangent at that start); it falls
                           back to the lifted start when that point has an inverted element.
                           0: always the lifted start with the Euler predictor */
  int lin_norm;         /* (0) norm of the FCG stopping test: 0: ||r||_2 <= lin_rtol ||r0||_2;
                           1: the natural norm of the preconditioned system (Section III-A),
                           sqrt(r^T M^-1 r) <= lin_rtol sqrt(r0^T M^-1 r0), M^-1 one V-cycle;
                           any other value: HPMG_ERR_ARG */
} hpmg_newton_params;
void hpmg_newton_default_params(hpmg_newton_params *p);
int hpmg_newton_solve(hpmg_op fine, hpmg_mg mg, double *u, const double *lift, const double *f_ext,
                      int n_steps, const hpmg_newton_params *params, const double *const *seeds,
                      double *stats, void *stream);

/* L-BFGS with the V-cycle as the initial inverse Hessian and the critical-point line
 * search (Section III-A; the residual F(u) is the gradient of the strain energy).
 * Load stepping as in hpmg_newton_solve (step k adds lift / n_steps to u and k / n_steps
 * of the external load f_ext, which may be NULL).  At the
 * start of every load step the state is stored at the lifted point and the V-cycle is
 * set up there; it then serves as H0 for all iterations of that step (residuals of
 * the iterations do not overwrite the stored state).  Direction by the two-loop
 * recursion over the last `memory` pairs s = u_new - u, y = F(u_new) - F(u) (pairs with
 * y^T s <= 0 are skipped; a non-descent direction drops all pairs).  A step length
 * whose point has an inverted element is halved (at most 6 times).  Stops when
 * ||F(u)|| <= rtol ||F(u_start)|| in every load step.  The caller provides a device
 * workspace of hpmg_lbfgs_workspace_bytes() (256-byte aligned), private to the call.
 * Statistics (host): stats[0] = total iterations, stats[1] = V-cycles, stats[2] = final
 * relative residual of the last load step, stats[3] = memory restarts,
 * stats[4 + k] = iterations of load step k (k < n_steps, at most 60). */
typedef struct {
  double rtol;     /* (1e-8) */
  int max_its;     /* (200) per load step */
  int memory;      /* (5) stored pairs, 1..32 */
  int line_search; /* 1: critical-point secant step, clipped to [0.1, 1.5] */
  int monitor;     /* (0) 1: one line per iteration on stderr */
} hpmg_lbfgs_params;
void hpmg_lbfgs_default_params(hpmg_lbfgs_params *p);
int hpmg_lbfgs_workspace_bytes(hpmg_mg mg, int memory, size_t *bytes);
int hpmg_lbfgs_solve(hpmg_op fine, hpmg_mg mg, double *u, const double *lift, const double *f_ext,
                     int n_steps, const hpmg_lbfgs_params *params, const double *const *seeds,
                     void *workspace, size_t workspace_bytes, double *stats, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HPMG_H */
