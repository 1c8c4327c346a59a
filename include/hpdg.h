/*
 * hpdg: matrix-free SIPG hp-DG elliptic operator and its multigrid-preconditioned
 * Krylov solve on one AMD MI355X (gfx950).  C ABI.
 *
 * The problem follows arXiv:1907.01572:
 *   - domain: a macro-mesh of mapped cubes refined by octrees with at most 2:1 face
 *     balance, per-element polynomial degree p (Sec. II.A.1, II.A.2);
 *   - discrete problem: find u_h in V_h with L_h(u_h, v) = F_h(v) for all v
 *     (Eqs. lh2, Fh2), written as the linear system L u = F (Eq. semidiscrete) in the
 *     nodal LGL basis (Eq. Lagrange_Basis), integrals by GL quadrature (Sec. II.A.5);
 *   - solver: flexible CG (Alg. 2) preconditioned by a multigrid V-cycle (Alg. 3) with
 *     Chebyshev smoothing (Alg. 4) and spectral bounds from CG (Alg. 5).
 * The model equation is read as -div(k grad u) + c u = g, u = g_D on Dirichlet faces.
 *
 * Conventions shared by every call:
 *   - Every function returns an int status: HPDG_OK (0) or a negative HPDG_ERR_* code;
 *     hpdg_last_error() then describes the failure.  No C++ exception crosses the ABI.
 *   - Device pointers are HIP device addresses (e.g. torch CUDA tensors on ROCm).  The
 *     caller owns every pointer it passes; the library never frees or retains them
 *     beyond the call.  Host arrays passed in are copied.
 *   - ``stream`` is a hipStream_t passed as void* (NULL = the default stream).  Calls
 *     that take a stream are enqueued on it and return without synchronising, unless
 *     stated otherwise.
 *   - Vector layout (a "level vector"): contiguous; elements in the level's element
 *     order; element e occupies (p_e+1)^3 consecutive entries starting at its dof
 *     offset (prefix sum of (p+1)^3); inside an element the LGL nodes are ordered
 *     i + n j + n^2 k (reference axis 0 fastest).  Level 0 is the uploaded mesh, in
 *     the caller's element order; coarser multigrid levels are 1, 2, ...
 *   - Precision: HPDG_F64 vectors are double, HPDG_F32 vectors are float.
 *   - A context is used by one host thread at a time; different contexts are
 *     independent.
 */
#ifndef HPDG_H
#define HPDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HPDG_OK = 0,
  HPDG_ERR_INVALID_ARG = -1,   /* a NULL or out-of-range argument */
  HPDG_ERR_INVALID_MESH = -2,  /* unmatched face, 4:1 face, J <= 0, p outside [1, 15] */
  HPDG_ERR_OOM = -3,           /* device allocation failed or the HBM budget is exceeded */
  HPDG_ERR_NOT_CONVERGED = -4, /* iteration cap reached before the tolerance */
  HPDG_ERR_BREAKDOWN = -5,     /* non-positive curvature or a non-finite dot product */
  HPDG_ERR_HIP = -6,           /* a HIP runtime call failed */
  HPDG_ERR_UNSUPPORTED = -7    /* a feature not built into this library */
};

enum { HPDG_F64 = 0, HPDG_F32 = 1 };                 /* vector precision of a call */
/* solve precision: FP64 throughout; FP32 V-cycle; FP32 V-cycle whose block-Jacobi smoother
 * reads bf16 inverse blocks (FP32 arithmetic; the outer FCG stays FP64 in every mode) */
enum { HPDG_PREC_F64 = 0, HPDG_PREC_MIXED = 1, HPDG_PREC_MIXED_BF16 = 2 };
enum { HPDG_MAP_AFFINE = 0, HPDG_MAP_SHELL = 1, HPDG_MAP_CUBE_SPHERE = 2 };
/* boundary kinds (Sec. II.A.1, Eqs. NeumannBC, RobinBC): Dirichlet u = g_D; Neumann
 * k n.grad u = g_N; Robin k n.grad u + gamma u = g_R (gamma from hpdg_disc_params) */
enum { HPDG_BC_INTERIOR = 0, HPDG_BC_DIRICHLET = 1, HPDG_BC_NEUMANN = 2, HPDG_BC_ROBIN = 3 };
enum { HPDG_COEF_CONSTANT = 0, HPDG_COEF_RADIAL_STEP = 1 };
enum { HPDG_RHS_SINSINSIN = 0, HPDG_RHS_SHELL_HARMONIC = 1, HPDG_RHS_RADIAL_STEP = 2,
       HPDG_RHS_POLYNOMIAL = 3, HPDG_RHS_GAUSSIANS = 4, HPDG_RHS_POLYNOMIAL_DIRICHLET = 5,
       HPDG_RHS_STAR = 6 };
enum { HPDG_NL_PUNCTURE = 0, HPDG_NL_QUADRATIC = 1, HPDG_NL_STAR = 2 };
/* Outer Krylov solvers, each preconditioned by one V-cycle per iteration: flexible CG
 * (Alg. 2), textbook PCG, and restarted flexible GMRES (right preconditioned: the
 * preconditioned directions are kept, so the V-cycle may vary between iterations, e.g. in
 * FP32; modified Gram-Schmidt, Givens rotations; the residual is recomputed as b - A u at
 * every restart and at exit). */
enum { HPDG_SOLVER_FCG = 0, HPDG_SOLVER_PCG = 1, HPDG_SOLVER_FGMRES = 2 };

typedef struct hpdg_ctx hpdg_ctx;
typedef struct hpdg_mesh hpdg_mesh;

/*
 * Macro-mesh + refinement + degrees (Sec. II.A.1: macro-elements are images of
 * [-1,1]^3 under analytic maps; fine elements are octree cells of their macro).
 *   macro_kind[m]        HPDG_MAP_*; macro_params[16 m + i] its parameters:
 *     AFFINE       x = o + sum_i (xi_i + 1)/2 a_i; params o(3), a0(3), a1(3), a2(3).
 *     SHELL        cubed-sphere patch; params[0..8] = R (row-major, det +1), [9] radial
 *                  kind (0 linear, 1 inverse (Eq. inverse_mapping), 2 linear up to
 *                  zeta_break then inverse), [10] r_in, [11] r_out, [12] zeta_break,
 *                  [13] r_break; direction v = R (tan(pi xi0/4), tan(pi xi1/4), 1),
 *                  x = r(xi2) v / |v|.
 *     CUBE_SPHERE  blend in xi2 of a R (xi0, xi1, 1) (a = params[10]) and the sphere
 *                  point params[11] v/|v| (R as for SHELL).
 *   macro_nbr[6 m + f], macro_nbr_face, macro_nbr_orient: neighbour macro across face f
 *     (f = 2 d + s, axis d, s = 0 at xi_d = -1) or -1 on the boundary; the face it
 *     meets; orientation o mapping face coordinates (a, b) (tangential axes in
 *     increasing order) to the neighbour's: (s, t) = o & 1 ? (b, a) : (a, b),
 *     a' = o & 2 ? -s : s, b' = o & 4 ? -t : t.
 *   macro_bc[6 m + f]    HPDG_BC_* on boundary faces.
 *   elem_macro, elem_level, elem_anchor[3 e + d], elem_p: octree cells; the cell
 *     covers macro coordinates [-1 + 2 a/2^l, -1 + 2 (a+1)/2^l] per axis.
 */
typedef struct {
  int32_t n_macro;
  const int32_t* macro_kind;
  const double* macro_params;
  const int32_t* macro_nbr;
  const int32_t* macro_nbr_face;
  const int32_t* macro_nbr_orient;
  const int32_t* macro_bc;
  int64_t n_elem;
  const int32_t* elem_macro;
  const int32_t* elem_level;
  const int32_t* elem_anchor;
  const int32_t* elem_p;
} hpdg_mesh_desc;

/*
 * Discretisation parameters.
 *   penalty_C   C of Eq. penaltyparameter: sigma = C p_m^2 / h_m (default 10).
 *   quad_extra  extra GL points per axis on curved elements or with a variable
 *               coefficient (Sec. II.A.5 leaves the GL grid size open; default 1).
 *   coef_kind   HPDG_COEF_*: k = 1, or k = coef_params[1] for |x| < coef_params[0]
 *               and coef_params[2] otherwise.
 *   max_levels  cap on the number of multigrid levels (0 = until the macro-mesh). The last
 *               level is solved exactly through a dense FP64 inverse (N_c^2 scalars), formed by
 *               hpdg_setup_smoother: N_c^2 must stay below 2^31, else that call fails with
 *               HPDG_ERR_UNSUPPORTED (a mesh used only for applies never forms it).
 *   build_f32   also build FP32 copies of every level (needed by HPDG_F32 calls and
 *               mixed-precision solves).
 *   mass_term   1: every level carries a mass form  sum_sigma w det J c u v  with c set per
 *               volume GL point by hpdg_nonlinear_linearize / hpdg_newton_solve (zero
 *               until then); the volume rule then has p + 1 + quad_extra points on every
 *               element.  Needed by the nonlinear calls.
 *   robin_gamma gamma of the Robin faces (macro face kind HPDG_BC_ROBIN): the operator gains
 *               int gamma u v on them (Eq. lh) and the right-hand side int g_R v.
 *   ec_mode     element-centric apply (elements with an affine axis-aligned map, constant k and
 *               no mass term): HPDG_EC_AUTO on levels with at least 4096 such elements (one
 *               degree) or 16384 (several degrees; below these the launches are latency bound),
 *               HPDG_EC_ALWAYS wherever an element qualifies, HPDG_EC_NEVER nowhere.  The
 *               operator is the same up to rounding either way.
 */
enum { HPDG_EC_AUTO = 0, HPDG_EC_ALWAYS = 1, HPDG_EC_NEVER = 2 };
typedef struct {
  double penalty_C;
  int32_t quad_extra;
  int32_t coef_kind;
  double coef_params[4];
  int32_t max_levels;
  int32_t build_f32;
  int32_t mass_term;
  double robin_gamma;
  int32_t ec_mode;
} hpdg_disc_params;

typedef struct {
  int32_t n_levels;
  int64_t n_elem[32];
  int64_t n_dof[32];
  int64_t n_mortar[32];
  int64_t vgeo_scalars[32];  /* volume metric values stored per level */
  int64_t mgeo_scalars[32];  /* mortar metric values stored per level */
  int64_t table_bytes[32];   /* element + mortar records and face lists per level */
  size_t device_bytes;   /* resident device memory of this mesh */
  /* setup factorisations repeated after a failed attempt (the element-block Cholesky of the
   * block-Jacobi smoother, the coarsest operator's Cholesky): a failure on an SPD operator that
   * does not repeat on a fresh assembly is retried once; both stay 0 in a healthy run */
  int32_t block_retries;
  int32_t coarse_retries;
  /* operator apply per level: elements evaluated element-centrically (affine, axis-aligned,
   * constant k, no mass term, p <= 7: volume and conforming faces from the 1-D mass and
   * stiffness matrices, neighbours read directly) and mortars left to the mortar kernel */
  int64_t n_elem_centric[32];
  int64_t n_mortar_tasks[32];
  /* FP64 (or FP32) operations of one apply per level as its kernels compute it (an FMA counts
   * two): element-centric elements 8 n^4 FMAs of the 1-D passes plus n^2 (3n + 6) per face;
   * the others the sum-factorised passes through the q GL points and the metric contraction,
   * plus the mortar interpolations and lifts of their faces */
  double apply_flops[32];
  /* a posteriori estimate (hpdg_estimate) of the last problem estimated, 0 before the first:
   * algorithmic bytes of one call (u, the point data, the volume and mortar metric read once,
   * h_e^2 p_e^2 and eta2; the face traces in between not counted) and the element volume
   * points and mortar points it evaluates */
  int64_t est_alg_bytes;
  int64_t est_volume_points;
  int64_t est_mortar_points;
} hpdg_mesh_info;

/* Chebyshev smoother (Alg. 4) and CG spectral bound (Alg. 5) parameters.
 * ``scaling`` preconditions the smoother's residual, r = M^-1 (b - A x):
 *   HPDG_SMOOTH_NONE   M = I (the printed form of Alg. 4);
 *   HPDG_SMOOTH_POINT  M = diag(A) (point Jacobi);
 *   HPDG_SMOOTH_BLOCK  M = the element-diagonal blocks A_ee (element-block Jacobi; their
 *                      inverses are formed on the device at setup and kept as packed lower
 *                      triangles, N (N + 1) / 2 values per element and level, N = (p+1)^3).
 * The bound of Alg. 5 is then taken for M^-1 A (preconditioned CG with the same M).
 *   HPDG_SMOOTH_SCHWARZ  the additive Schwarz smoother of Sec. II.D instead of Chebyshev
 *                      (Alg. schwarz_smoother, Eq. schwarz_weight): n_cheb (n_cheb_coarse below
 *                      the finest level) cycles x += sum_s R_s^T W_s A_ss^-1 R_s (b - A x) over
 *                      element-centred subdomains of schwarz_overlap = N_overlap layers of
 *                      points beyond the centre element (N_overlap >= 1; a level of degree
 *                      p < N_overlap uses N_overlap = p).  The local
 *                      problems are solved exactly (their inverses, restricted to the rows of
 *                      non-zero weight, are formed at setup on the device and kept: m_w m
 *                      values per subdomain, m = (p + 1 + 2 N_overlap)^3 points inside the
 *                      mesh, m_w = (p + 3)^3 weighted ones for N_overlap >= 2).  Neighbours'
 *                      points are placed in the centre's reference frame through the maps of the
 *                      faces crossed to reach them (any macro maps and face orientations).  On a
 *                      side of the centre element that lies on the domain boundary the weight
 *                      keeps its plateau; where three cells meet around an edge (the six-patch
 *                      shell) the weights covering a point are divided by their sum; so they
 *                      sum to one at every point.  Where degrees differ across a face the
 *                      subdomains are ragged: each face takes the narrower of its two cells'
 *                      overlap widths.  Levels with 2:1 faces need axis-aligned affine cells:
 *                      there the extended coordinate is the offset from the centre cell in units
 *                      of its half-widths, and a cell's width is scaled by its half-width.  Scope:
 *                      every smoothed level has one refinement level and faces that meet 1:1,
 *                      or axis-aligned affine cells; subdomains of at most 8190 points and 64
 *                      cells (HPDG_ERR_UNSUPPORTED at setup otherwise).  On meshes with FP32
 *                      levels the stored rows are also kept rounded to FP32, for FP32 smoothing
 *                      and the FP32 V-cycle of mixed-precision solves.  Not rebuilt for Newton
 *                      linearisations (HPDG_ERR_UNSUPPORTED).  No spectral bound is computed
 *                      (lambda_max 0). */
enum { HPDG_SMOOTH_NONE = 0, HPDG_SMOOTH_POINT = 1, HPDG_SMOOTH_BLOCK = 2, HPDG_SMOOTH_SCHWARZ = 3 };
typedef struct {
  int32_t n_cheb;        /* Chebyshev steps per smoothing call (default 4) */
  int32_t n_eigs;        /* CG steps for the bound (default 15) */
  double Lambda;         /* lambda_min = lambda_max / Lambda (default 20) */
  int32_t scaling;       /* HPDG_SMOOTH_* (default HPDG_SMOOTH_POINT) */
  uint64_t seed;         /* SplitMix64 seed of the CG start vector */
  int32_t n_cheb_coarse; /* Chebyshev steps per smoothing call on the levels below the finest
                            (0: n_cheb) */
  int32_t unfused;       /* HPDG_SMOOTH_POINT, or HPDG_SMOOTH_BLOCK with FP64 / FP32 blocks,
                            on a level of degrees p <= 7: 0 runs each Chebyshev step that needs
                            A x as the mortar kernel and then one fused kernel per element
                            (volume term and face sums, r = b - A x, z = M^-1 r and the update;
                            the same arithmetic); 1 keeps the apply and the scaling step apart */
  int32_t schwarz_overlap; /* HPDG_SMOOTH_SCHWARZ: N_overlap (the paper's runs use 2) */
} hpdg_smoother_params;

typedef struct {
  int32_t solver;        /* HPDG_SOLVER_FCG (Alg. 2), HPDG_SOLVER_PCG or HPDG_SOLVER_FGMRES */
  int32_t precision;     /* HPDG_PREC_F64 or HPDG_PREC_MIXED (FP32 V-cycle) */
  double tol_rel;        /* stop when |b - A u|_2 <= tol_rel |b|_2 */
  int32_t max_iter;      /* iterations (one V-cycle and one apply each) */
  int32_t restart;       /* FGMRES: Krylov vectors per cycle (0: 30); the 2 restart + 1
                            level-0 vectors are allocated on the first FGMRES solve of a mesh */
} hpdg_solve_params;

typedef struct {
  int32_t iterations;
  double rel_residual;   /* |b - A u| / |b| of the recurrence residual at exit */
  double solve_ms;       /* wall time of the Krylov loop (host clock, synchronised) */
  int32_t status;        /* the return code */
} hpdg_solve_stats;

/* RHS descriptor: analytic source / Dirichlet data (ids as HPDG_RHS_*).  HPDG_RHS_STAR
 * [rho0, r0]: no source, Dirichlet data the closed-form conformal factor of the
 * constant-density star (Sec. III.B): psi = C u_alpha(r) inside r0, beta / r + 1 outside,
 * C = (2 pi rho0 / 3)^(-1/4), alpha >= sqrt(5) from
 * rho0 r0^2 = (3 / (2 pi)) alpha^10 / (1 + alpha^2)^6 (the continuity of psi and its slope),
 * beta = r0 (C u_alpha(r0) - 1). */
typedef struct {
  int32_t kind;
  int32_t n_params;
  const double* params;
} hpdg_rhs_desc;

/* Semilinear source N: -lap u = beta(x) (1 + alpha(x) u)^-7  (the puncture equation of
 * Sec. III.D, Eq. Two_Punctures_PDE, for the regular part u, with psi = (1 + alpha u) /
 * alpha), or -lap psi = 2 pi rho psi^5 (the constant-density star of Sec. III.B,
 * Eq. Constant_Density_Star_PDE).  Parameters (copied):
 *   HPDG_NL_PUNCTURE   [s, then rows (cx, cy, cz, m, a)]:
 *                      alpha = 1 / (1 + sum_I m_I / (2 |x - c_I|)),
 *                      beta = sum_I a_I exp(-|x - c_I|^2 / (2 s^2)) / (1 + |x|^2)^2;
 *   HPDG_NL_QUADRATIC  [alpha, C[a][b][c] (27 values, x^a y^b z^c, a, b, c <= 2)]:
 *                      constant alpha, beta = (-lap u*) (1 + alpha u*)^7 for the quadratic
 *                      u* (a manufactured problem whose exact solution is u*);
 *   HPDG_NL_STAR       [rho0, r0]: N(psi) = 2 pi rho psi^5, rho = rho0 for |x| <= r0 and 0
 *                      outside (with HPDG_RHS_STAR Dirichlet data). */
typedef struct {
  int32_t kind;
  int32_t n_params;
  const double* params;
} hpdg_nonlinear_desc;

/* Newton-Krylov parameters (Alg. 1 with FCG, Alg. 2, as the linear solver). */
typedef struct {
  double tol_rel;        /* stop when |R(u_k)|_2 <= tol_rel |R(u_0)|_2 */
  double lin_tol_rel;    /* FCG tolerance of each correction, relative to |R(u_k)|_2 */
  int32_t max_newton;
  int32_t max_lin_iter;  /* FCG iteration cap per Newton step */
  int32_t precision;     /* HPDG_PREC_F64 or HPDG_PREC_MIXED V-cycle */
} hpdg_newton_params;

typedef struct {
  int32_t newton_steps;
  int32_t linear_iterations;  /* FCG iterations summed over the Newton steps */
  double rel_residual;        /* |R(u)| / |R(u_0)| at exit */
  double solve_ms;            /* wall time (host clock, synchronised) */
  int32_t status;             /* the return code */
} hpdg_newton_stats;

/* Create a context on HIP device ``hip_device``; device memory of all its meshes is
 * limited to ``hbm_budget_bytes`` (0 = no limit). */
int hpdg_create(hpdg_ctx** out, int hip_device, size_t hbm_budget_bytes);
/* Free the context and every mesh it still owns. */
int hpdg_destroy(hpdg_ctx* ctx);
/* Message of the last failed call made by the calling thread (thread-local: calls on other
 * threads, e.g. the solve server's workers, do not overwrite it); never NULL.  The pointer stays
 * valid until the calling thread's next failing call. */
const char* hpdg_last_error(const hpdg_ctx* ctx);

/* Build the level hierarchy (Sec. II.D.3: surrogate coarsening + 2:1 restoration,
 * coarse degree = min over children), the mortar tables (Sec. II.A.1), FP64 geometry
 * at GL points (Eqs. Jacobian, Surface-Jacobian), penalties (Eq. penaltyparameter),
 * operator tables and transfer maps, and upload them.  Synchronises ``stream``. */
int hpdg_mesh_upload(hpdg_ctx* ctx, const hpdg_mesh_desc* desc, const hpdg_disc_params* disc,
                     hpdg_mesh** out, void* stream);
int hpdg_mesh_info_get(const hpdg_mesh* mesh, hpdg_mesh_info* out);
/* Cells of a level (host arrays of n_elem[level] entries each; anchor has 3 per cell). */
int hpdg_level_cells(const hpdg_mesh* mesh, int level, int32_t* macro, int32_t* lvl,
                     int32_t* anchor, int32_t* p);
int hpdg_mesh_free(hpdg_mesh* mesh);

/* Coefficients of the model -div(k grad u) + c u = g (Sec. II.A.2, Eq. Laplacian: c is the
 * f u term, read with the sign of the bilinear form of Eq. lh; k is this library's variable
 * coefficient, folded into the metric as k J^-1 J^-T).  ``kind``: HPDG_COEF_DIFFUSION (k > 0)
 * or HPDG_COEF_MASS (c; needs a mesh uploaded with mass_term = 1; replaced by the nonlinear
 * calls' own mass terms when those are used).  ``where``:
 *   HPDG_WHERE_ELEMENT   host_vals[n_elem[0]]: one value per level-0 element;
 *   HPDG_WHERE_NODE      host_vals[n_dof[0]]: values at the LGL nodes in the level-vector layout;
 *                        the coefficient at any point of an element is their interpolant there;
 *   HPDG_WHERE_ANALYTIC  params: diffusion [HPDG_COEF_* kind, its 4 parameters] (as
 *                        hpdg_disc_params); mass [c] (constant).
 * Values are copied (FP64 master; the FP32 levels take its rounding).  Coarser levels take the
 * mean over the level-0 cells inside each cell (per element) or the injection of the nodal
 * field (each coarse node takes the value of the finer polynomial of the child containing it).
 * A tabulated k may jump across a face: each side of a mortar uses its own value in
 * {{k grad u}} and the penalty takes max(k-, k+).  The call rebuilds every level's tables and
 * device data (the mesh handle stays valid; device vectors of the previous tables are not
 * touched) and, when the smoother was set up, sets it up again (bounds recomputed by Alg. 5).
 * Synchronises ``stream``.  Errors: HPDG_ERR_INVALID_ARG (unknown kind / placement, missing,
 * non-finite or non-positive k values), HPDG_ERR_UNSUPPORTED (mass without mass_term). */
enum { HPDG_COEF_DIFFUSION = 0, HPDG_COEF_MASS = 1 };
enum { HPDG_WHERE_ELEMENT = 0, HPDG_WHERE_NODE = 1, HPDG_WHERE_ANALYTIC = 2 };
int hpdg_set_coefficient(hpdg_mesh* mesh, int kind, int where, const double* host_vals, const double* params,
                         void* stream);

/* F = F_h(psi) (Eq. Fh2) for an analytic source g and Dirichlet data g_D = u, written
 * to the device FP64 vector F_dev of level 0.  Faces marked Neumann in the mesh (macro
 * face kind 2) add int g_N psi with g_N = k n.grad u (Eq. NeumannBC, n the outward normal)
 * for HPDG_RHS_SINSINSIN, HPDG_RHS_POLYNOMIAL and HPDG_RHS_POLYNOMIAL_DIRICHLET, and
 * g_N = 0 for HPDG_RHS_GAUSSIANS; Robin faces (kind 3) add int g_R psi with
 * g_R = k n.grad u + gamma u (Eq. RobinBC with the sign of Eq. lh; 0 for the Gaussians);
 * other kinds with Neumann or Robin faces return HPDG_ERR_UNSUPPORTED.
 * Every face integral uses the face's own rule.  The face terms are computed on the host in
 * FP64 and copied; the volume term int g psi runs on the device in FP64 (the GL points mapped
 * by the macro maps there, one workgroup per element) and is added.  Synchronises ``stream``.
 * HPDG_ERR_INVALID_ARG also for a polynomial of degree above 15. */
int hpdg_assemble_rhs(hpdg_mesh* mesh, const hpdg_rhs_desc* rhs, double* F_dev, void* stream);

/* A posteriori error estimate of u_dev (a level-0 FP64 vector) for the problem of ``rhs``
 * (Sec. II.E, Eqs. Eta2_Ingredients, Eta2_Integrals, Eta2_Local), per level-0 element, into the
 * device FP64 array eta2_dev[n_elem[0]]:
 *   eta2(e) = h_e^2 p_e^2 int_e R^2 + sum over the interior mortars of e of
 *             int_m ((h_m / p_m) [[k grad u]]^2 + sigma [[u]]^2) + sum over its Dirichlet mortars of
 *             int_m sigma (u - g_D)^2,
 * R = g + div(k grad u) - c u (c: the mass coefficient the operator applies, so after
 * hpdg_nonlinear_linearize the Jacobian's mass term); sigma the operator's penalty
 * (Eq. penaltyparameter, with max(k-, k+)) and h_m, p_m as there, pointwise on the mortar
 * rule; h_e the largest distance
 * between two vertices of e; div(k grad u) by the collocation derivative on the element's GL
 * points (exact on affine elements with a constant k); Neumann and Robin faces add no term.
 * eta2_vol_dev (may be NULL): the volume parts h_e^2 p_e^2 int_e R^2.  Runs on the device in
 * FP64 (face traces, one kernel per element for the volume part, one wavefront per mortar for
 * the face parts, one sum per element); the point data of the problem are built on the host on
 * the first call for a (kind, params) and kept with the mesh.  Stream-ordered; the first call
 * for a problem synchronises ``stream``.  Errors: HPDG_ERR_INVALID_ARG (unknown rhs kind,
 * missing arguments, eta2_dev == eta2_vol_dev), HPDG_ERR_UNSUPPORTED (degree above 8). */
int hpdg_estimate(hpdg_mesh* mesh, const hpdg_rhs_desc* rhs, const double* u_dev, double* eta2_dev,
                  double* eta2_vol_dev, void* stream);
/* The grid the estimator's integrals are taken on (Sec. II.E, the fiducial grid; Sec. III.C uses
 * an unstretched twin of a compactified shell): the macro maps of ``grid`` (its macro fields;
 * its cells are ignored) with the mesh's cells.  The integrands (R and the jumps) stay on the
 * physical grid; W det J, w S, h_e and h_m (and with it sigma) come from ``grid`` at the same
 * reference points.  NULL restores the physical grid.  Takes effect at the next hpdg_estimate.
 * Errors: HPDG_ERR_INVALID_MESH (another macro count or connectivity; a fiducial cell with
 * det J <= 0 is reported by hpdg_estimate). */
int hpdg_set_estimator_grid(hpdg_mesh* mesh, const hpdg_mesh_desc* grid);

/* hp-adaptation (Sec. II.E, Alg. hpamr), host-side steps between solves.
 *
 * hpdg_amr_mark: marked[e] = 1 for the elements to refine, from eta2[n] (host arrays):
 *   HPDG_MARK_FRACTION  the ceil(param n) elements of largest eta2 (0 <= param <= 1; ties: lower
 *                       index first; the product param n is taken with a guard of 1e-9 against
 *                       its representation error);
 *   HPDG_MARK_MEAN      the elements with eta2 > param * mean(eta2).
 * hpdg_amr_smooth_pred: the smooth-pred decision for every marked element (host arrays of n):
 *   eta2 > eta2_pred[e]  -> action 1 (h-refine); its children predict
 *                           gamma_h (1/2)^3 (1/2)^(2 p_e) eta2(e);
 *   otherwise            -> action 2 (p-refine); it predicts gamma_p eta2(e).
 *   An element without a prediction carries eta2_pred = +inf (every element at the start), so it
 *   is p-refined first.  Unmarked elements: action 0, prediction unchanged.  pred_out[e] is the
 *   prediction element e (or each of its children) carries to the next step; typical
 *   gamma_h = 0.25, gamma_p = 0.1.
 * hpdg_amr_adapt: apply action[e] (0 keep, 1 h-refine: 8 children of the same degree, 2 p-refine:
 *   degree + 1, at most max_degree <= 15) to the cells of ``mesh`` (its macro fields describe the
 *   macro-mesh, which the new mesh shares), then refine where 2:1 face balance is violated
 *   (Sec. II.A.1; those children keep the degree).  Each old cell is replaced in place by the
 *   cells inside it, children ordered by their bits (x fastest); origin[i] is the old cell that
 *   new cell i lies in.  Output host arrays hold ``capacity`` cells (anchor 3 per cell; 8 n
 *   always suffice); *n_out is the new count (also when the capacity is too small, which returns
 *   HPDG_ERR_INVALID_ARG).  HPDG_ERR_INVALID_MESH: the input is not a valid 2:1-balanced mesh or
 *   a cell would pass level 14.
 * These three calls need no context and no device; their errors are reported by
 * hpdg_last_error(NULL). */
enum { HPDG_MARK_FRACTION = 0, HPDG_MARK_MEAN = 1 };
int hpdg_amr_mark(const double* eta2, int64_t n, int mode, double param, uint8_t* marked);
int hpdg_amr_smooth_pred(const double* eta2, const double* eta2_pred, const int32_t* p, const uint8_t* marked,
                         int64_t n, double gamma_h, double gamma_p, int8_t* action, double* pred_out);
int hpdg_amr_adapt(const hpdg_mesh_desc* mesh, const int8_t* action, int32_t max_degree, int64_t capacity,
                   int32_t* macro, int32_t* level, int32_t* anchor, int32_t* p, int64_t* origin, int64_t* n_out);
/* u_to_dev = u_from_dev carried from mesh ``from`` onto mesh ``to`` (level-0 FP64 vectors): both
 * meshes have the same macro-mesh and every cell of ``to`` is a cell of ``from`` or a child of
 * one (one level finer), of equal or higher degree -- the output of hpdg_amr_adapt.  Each new
 * cell takes the interpolant of its old cell's polynomial at its LGL nodes (child-half and
 * degree interpolation as in the multigrid prolongation, Sec. II.D), which is exact for these
 * pairs.  Synchronises ``stream``.  Errors: HPDG_ERR_INVALID_ARG (other meshes, other
 * contexts, u_from_dev == u_to_dev). */
int hpdg_transfer(const hpdg_mesh* from, hpdg_mesh* to, const double* u_from_dev, double* u_to_dev,
                  void* stream);

/* y = A_level x (Eq. lh2 applied matrix-free): volume stiffness by sum factorisation,
 * SIPG fluxes on every mortar with hp-mortar projections (Fig. mortar).  Three stream-ordered
 * launches: the face traces of x, the mortar kernel (both sides of each mortar, into per-face
 * slots of the mesh), the element kernel (volume term plus the element's face slots).  x, y:
 * level vectors of precision ``prec``; x != y. */
int hpdg_apply(hpdg_mesh* mesh, int level, int prec, const void* x_dev, void* y_dev, void* stream);

/* y = A_level x as hpdg_apply, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the face traces and the
 * face slots go to a fixed device array of the library (64 MiB per GPU, held until the process
 * ends; its address is taken when the context is created) instead of the mesh's buffers, and
 * the call makes no allocation of any kind.  Same kernels and result as hpdg_apply.  A level
 * whose traces and slots need more than 64 MiB (12 (p+1)^2 trace scalars per element and
 * 2 (p+1)^2 slot scalars per face-mortar pair) returns HPDG_ERR_INVALID_ARG.  Every call
 * on a GPU shares that GPU's array: calls that overlap on one GPU (other streams, other
 * threads, other contexts) race and must be serialised by the caller. */
int hpdg_apply_noalloc(hpdg_mesh* mesh, int level, int prec, const void* x_dev, void* y_dev, void* stream);

/* Solver setup: the exact coarse solve (the coarsest operator assembled on the device,
 * Cholesky and explicit inverse; once per mesh), the smoother's scaling data, and the spectral
 * bounds of every smoothed level.  With lambda_max[l] > 0 on entry the value
 * is used as given (frozen); otherwise it is computed by Alg. 5 and written back.
 * ``lambda_max`` is a host array of n_levels - 1 entries.  Synchronises ``stream``. */
int hpdg_setup_smoother(hpdg_mesh* mesh, const hpdg_smoother_params* params, double* lambda_max,
                        void* stream);
/* x <- Chebyshev(x, b) on ``level`` with n_iter steps (Alg. 4, update p = alpha r + beta p). */
int hpdg_smooth(hpdg_mesh* mesh, int level, int prec, const void* b_dev, void* x_dev, int n_iter,
                void* stream);
/* z = V(r): one V-cycle (Alg. 3) from zero initial guesses; level-0 vectors of ``prec``;
 * coarsest level solved exactly through the FP64 inverse formed at setup (Cholesky); an FP32
 * V-cycle widens the coarse right-hand side to FP64 for that solve and rounds the result. */
int hpdg_vcycle(hpdg_mesh* mesh, int prec, const void* r_dev, void* z_dev, void* stream);
/* Solve A u = b (FP64 level-0 vectors).  u is the initial guess on entry (Alg. 2,
 * r0 = b - A u0) and the solution on exit.  ``stats`` is filled even on failure;
 * HPDG_ERR_NOT_CONVERGED leaves the last iterate in u.  Synchronises ``stream``. */
int hpdg_solve(hpdg_mesh* mesh, const hpdg_solve_params* params, const double* b_dev,
               double* u_dev, hpdg_solve_stats* stats, void* stream);

/* Nonlinear residual R(u) = A u - N(u) - F (Eq. Ru=0 discretised):
 * N(u)_psi = sum_sigma w det J beta (1 + alpha u)^-7 psi at the volume GL points (star:
 * w det J 2 pi rho u^5 psi); F_dev may
 * be NULL (F = 0), else the level-0 F (e.g. from hpdg_assemble_rhs).  FP64 level-0
 * vectors; R_dev must differ from u_dev and F_dev.  Needs a mesh uploaded with
 * mass_term = 1.  Returns HPDG_ERR_BREAKDOWN when 1 + alpha u <= 0 at a GL point. */
int hpdg_nonlinear_residual(hpdg_mesh* mesh, const hpdg_nonlinear_desc* nl, const double* F_dev,
                            const double* u_dev, double* R_dev, void* stream);
/* Linearise at u (Eq. newtoncorrectionsystem): every level's mass coefficient becomes
 * w det J 7 alpha beta (1 + alpha u_l)^-8 (star: -5 w det J 2 pi rho u_l^4; the Jacobian
 * must stay positive definite, which holds on the weak-field branch) with u_0 = u and
 * u_{l+1} injected from u_l (each
 * coarse LGL node takes the value of the finer child containing it; nodes on the cut
 * belong to the lower child); then the point-Jacobi scaling, the spectral bounds (Alg. 5)
 * and the coarsest inverse are recomputed.  Afterwards hpdg_apply on level l applies the
 * Jacobian J_l = A_l + M_l(u_l).  Needs hpdg_setup_smoother first (scaling NONE or POINT;
 * BLOCK returns HPDG_ERR_UNSUPPORTED).  Synchronises ``stream``. */
int hpdg_nonlinear_linearize(hpdg_mesh* mesh, const hpdg_nonlinear_desc* nl, const double* u_dev,
                             void* stream);
/* Newton-Krylov (Alg. 1): u_{k+1} = u_k + delta, J(u_k) delta = -R(u_k) solved by FCG
 * with the V-cycle of the linearised levels, until |R(u_k)| <= tol_rel |R(u_0)| or
 * max_newton steps.  u_dev: initial guess on entry, solution on exit (FP64 level 0).
 * ``stats`` is filled even on failure; HPDG_ERR_NOT_CONVERGED leaves the last iterate. */
int hpdg_newton_solve(hpdg_mesh* mesh, const hpdg_newton_params* params, const hpdg_nonlinear_desc* nl,
                      const double* F_dev, double* u_dev, hpdg_newton_stats* stats, void* stream);

/* ---- solve server: continuous batching of independent linear solves ----------------
 * Requests (mesh + discretisation + analytic right-hand side) are queued on submit.  Up to
 * ``max_active`` worker threads, each with its own HIP stream, take requests as slots and
 * device memory free up: a request is admitted when its device footprint (its level
 * tables, Krylov state and smoother data, computed from its host-side tables before any
 * device allocation) fits in ``hbm_budget_bytes`` minus the footprint of the requests in
 * flight; the first queued request that fits is taken, and the head of the queue is not
 * passed over more than 2 max_active times.  Each request's element data and solver
 * state stay on the device from upload to its last iteration; requests in flight share
 * the GPU concurrently.  The result is copied to the caller's host buffer.  The request's
 * mesh then stays uploaded, with its smoother set up, as long as device memory allows: a
 * later request with the same mesh and discretisation (byte-identical descriptions) takes
 * it and only assembles its right-hand side (host faces, device volume) and solves.  Such
 * idle meshes count against hbm_budget_bytes with their requests' footprint; the least
 * recently used are freed when a queued request needs the room, or beyond 64 GiB; all are
 * freed by hpdg_server_destroy.  Results do not depend on the mix or on the reuse: every
 * kernel and reduction of a solve is deterministic and private to its request. */
typedef struct hpdg_server hpdg_server;
typedef struct {
  int32_t max_active;          /* requests in flight (worker threads / streams), >= 1 */
  size_t hbm_budget_bytes;     /* device memory for requests in flight (0: no limit) */
  int32_t precision;           /* HPDG_PREC_F64 or HPDG_PREC_MIXED */
  hpdg_smoother_params smoother;
  double tol_rel;              /* |b - A u| <= tol_rel |b| */
  int32_t max_iter;
} hpdg_server_params;

typedef struct {
  hpdg_mesh_desc mesh;         /* copied at submit */
  hpdg_disc_params disc;       /* build_f32 is set by the server for mixed precision */
  hpdg_rhs_desc rhs;           /* copied at submit */
  double* u_out;               /* host buffer of n_dof doubles, written before DONE; the caller
                                  keeps it alive until the request is DONE or FAILED */
} hpdg_request;

enum { HPDG_REQ_QUEUED = 0, HPDG_REQ_RUNNING = 1, HPDG_REQ_DONE = 2, HPDG_REQ_FAILED = 3 };
typedef struct {
  int32_t state;               /* HPDG_REQ_* */
  int32_t status;              /* return code of the solve (HPDG_OK when DONE) */
  int32_t iterations;
  double rel_residual;
  double submit_ms, start_ms, end_ms;  /* host clock, ms since the server was created */
  size_t device_bytes;         /* admitted footprint */
  int64_t n_dof;
  char message[200];           /* FAILED: the error text (NUL-terminated, possibly cut) */
} hpdg_request_status;

int hpdg_server_create(hpdg_ctx* ctx, const hpdg_server_params* params, hpdg_server** out);
/* Queue a request; its ticket (> 0) identifies it in poll / wait. */
int hpdg_server_submit(hpdg_server* server, const hpdg_request* request, uint64_t* ticket);
int hpdg_server_poll(hpdg_server* server, uint64_t ticket, hpdg_request_status* status);
/* Wait until the request is DONE or FAILED, or timeout_ms passes (< 0: no limit; the
 * status is returned either way). */
int hpdg_server_wait(hpdg_server* server, uint64_t ticket, int64_t timeout_ms, hpdg_request_status* status);
/* Stop taking requests, finish those in flight, mark the queued ones FAILED, free.  No other
 * thread may be inside a call on this server (e.g. hpdg_server_wait) when it is destroyed. */
int hpdg_server_destroy(hpdg_server* server);

/* Kernel timing for measurement.  While enabled (every = k > 0), every k-th operator
 * application of each (kind, level, precision) (HPDG_TIMING_APPLY: hpdg_apply and the
 * applies inside hpdg_smooth, hpdg_vcycle and hpdg_solve), every k-th block-Jacobi
 * Chebyshev step (HPDG_TIMING_BLOCK), every k-th fused apply + Jacobi-scaled Chebyshev step
 * (HPDG_TIMING_SMOOTH, see hpdg_smoother_params.unfused) and every k-th launch of the Schwarz
 * smoother's local solves (HPDG_TIMING_SCHWARZ) is bracketed by two HIP events on
 * its stream, and the algorithmic bytes of the launch are recorded (every = 0 disables):
 *   apply: 2 s N (x read, y written) + s (volume + mortar metric scalars) + record bytes;
 *   block step: s sum_e N_e (N_e + 1) / 2 (packed inverse blocks, N_e = n_e^3) + s N per
 *   vector read or written;
 *   fused step (the mortar kernel and the fused element kernels; the face-trace launch before
 *   the first step is not timed): the
 *   apply's bytes without the y write, plus the packed blocks (point Jacobi: s N, the inverse
 *   diagonal) and s N per vector (b, p, x written, p read after the first step);
 *   Schwarz local solves: s sum_s m_w,s m_s (the stored rows) + (s + 4) sum_s m_s (gathered
 *   residual and its indices) + s sum_s m_w,s (corrections written) + 24 per subdomain (its
 *   offsets).
 * (s = 8 for HPDG_F64, 4 for HPDG_F32; N = level DOF.)  hpdg_kernel_timing() waits for
 * the recorded events and returns, for one (kind, level, prec), the summed event time in
 * ms, the number of launches and the summed algorithmic bytes since the previous read of
 * that entry, then resets the entry.  Recording costs two event records per launch. */
enum { HPDG_TIMING_APPLY = 0, HPDG_TIMING_BLOCK = 1, HPDG_TIMING_SMOOTH = 2, HPDG_TIMING_SCHWARZ = 3,
       HPDG_TIMING_KINDS = 4 };
int hpdg_timing_enable(hpdg_mesh* mesh, int every);
int hpdg_kernel_timing(hpdg_mesh* mesh, int kind, int level, int prec, double* total_ms, int64_t* launches,
                       double* alg_bytes);

#ifdef __cplusplus
}
#endif
#endif
