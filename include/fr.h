/*
 * fr.h -- C ABI of the MI355X (gfx950) implementation of the hot path of the
 * p-adaptive implicit high-order flux reconstruction method of Wang, Gobbert
 * & Yu, "A dynamically load-balanced parallel p-adaptive implicit high-order
 * flux reconstruction method for under-resolved turbulence simulation"
 * (arXiv 1910.03693).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - State layout (device, float64 unless stated): U[var][sp], var = (rho,
 *    rho u, rho v, rho w, rho E); the (p+1)^3 solution points of every element
 *    are contiguous, elements in mesh order, xi index fastest, then eta, zeta.
 *    The solution points are the tensor Gauss-Legendre points of the element's
 *    trilinear map.  fr_layout() returns the offsets.
 *  - Array arguments of the compute calls are DEVICE pointers owned by the
 *    caller; the library never frees them.  The mesh descriptor and the
 *    stats structs are HOST memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  fr_residual,
 *    fr_jvp, fr_vjp and spectral_decay_indicator only enqueue work.
 *    gmres_stage_solve and esdirk_step synchronise the stream to read their
 *    convergence scalars.
 *  - The library owns its workspace.  fr_create allocates the mesh data and
 *    the residual's face buffers; fr_reserve allocates the Krylov and
 *    time-step workspace and instantiates the captured Arnoldi graphs.  No
 *    compute call allocates device memory: a solver call that needs more than
 *    was reserved returns FR_E_INVALID.
 *  - Errors: argument errors return at once; a failed HIP call returns
 *    FR_E_HIP; a density or pressure <= 0 met by a residual kernel raises a
 *    device flag that the next synchronising call reports as FR_E_NONPHYSICAL.
 *    fr_last_error() describes the last error of a context.  No call aborts
 *    the process or lets a C++ exception escape.
 *  - A context may be used by one host thread and one stream at a time.
 *  - Output arrays must not overlap the call's inputs or each other ("must not
 *    alias" below means any overlap, not only the same start address); the
 *    calls that can check it return FR_E_INVALID.
 */
#ifndef FR_H
#define FR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fr_ctx_s* fr_ctx;

typedef enum {
  FR_OK = 0,
  FR_E_INVALID = -1,       /* bad argument or mesh description */
  FR_E_NOMEM = -2,         /* device allocation failed */
  FR_E_HIP = -3,           /* a HIP runtime call failed */
  FR_E_NOTCONVERGED = -4,  /* solver stopped by its iteration budget */
  FR_E_NONPHYSICAL = -5,   /* rho <= 0, p <= 0 or a NaN of either was met */
  FR_E_UNSUPPORTED = -6
} fr_status;

enum { FR_EULER = 0, FR_NAVIER_STOKES = 1 };
enum { FR_ROE = 0, FR_RUSANOV = 1 };
enum { FR_BC_WALL = -1, FR_BC_FARFIELD = -2 };
typedef enum { FR_F64 = 0, FR_F32 = 1 } fr_prec;
/* Jacobian-vector product: exact tangent, or the finite difference of
 * section 2.3 with the step eps taken along the unit direction (FR_JV_FD, the
 * paper's fixed eps = 1e-6), or with the step scaled to the state as
 * eps sqrt(1 + ||U||_2) (FR_JV_FD_SCALED, Walker and Pernice's choice for
 * matrix-free Newton-Krylov; a reading, the paper fixes no scaling). */
typedef enum { FR_JV_EXACT = 0, FR_JV_FD = 1, FR_JV_FD_SCALED = 2 } fr_jv_mode;

/*
 * Mesh and physics (section 2.1 and 2.2 of the paper).  Conforming hexahedra:
 * element vertex v = a + 2b + 4c sits at reference (xi, eta, zeta) =
 * (2a-1, 2b-1, 2c-1) of a trilinear map.  Faces are numbered (-xi, +xi, -eta,
 * +eta, -zeta, +zeta).  elem_nbr[e][2d+1] = e' >= 0 requires
 * elem_nbr[e'][2d] = e, with e's +d face equal to e''s -d face up to a
 * translation (periodic images allowed) and the same tangential orientation.
 * A negative entry is a boundary: FR_BC_WALL (no-slip adiabatic wall) or
 * FR_BC_FARFIELD (far-field state `farfield`).  Degrees elem_p in 1..5 may
 * differ by any amount across a face.  Non-dimensional gas with gas constant
 * 1: T = p / rho, cp = gamma / (gamma - 1), constant mu and Prandtl number.
 */
typedef struct {
  int32_t n_elem;
  const double* elem_xyz;   /* host [n_elem][8][3] */
  const int32_t* elem_nbr;  /* host [n_elem][6] */
  const int8_t* elem_p;     /* host [n_elem], 1..5 */
  int32_t physics;          /* FR_EULER or FR_NAVIER_STOKES */
  int32_t flux;             /* FR_ROE (eq. invis_com) or FR_RUSANOV */
  double gamma, mu, prandtl;
  double farfield[5];       /* conservative far-field state */
} fr_mesh_desc;

/* Restarted GMRES (section 2.3: matrix-free PETSc GMRES in the paper). */
typedef struct {
  int32_t restart;    /* Krylov basis size m per cycle (paper: 60) */
  int32_t max_iter;   /* operator products per solve (paper: 100) */
  double tol;         /* stop when ||r|| <= tol ||F|| (paper: 1e-1) */
  int32_t jv_mode;    /* FR_JV_EXACT (dual-number tangent), FR_JV_FD or FR_JV_FD_SCALED */
  int32_t precision;  /* FR_F64, or FR_F32 (exact Jv and Krylov basis in
                         float32; Hessenberg, rotations, dots and the update
                         stay float64) */
  double fd_eps;      /* finite-difference step along the unit direction (1e-6) */
  int32_t use_graph;  /* replay each Arnoldi cycle from the graphs that fr_reserve
                         captured for this (jv_mode, precision) */
  int32_t precond;    /* 1: left preconditioning by the element-Jacobi
                         preconditioner (section 2.3) built in this precision;
                         2: the same with its inverse kept in float16
                         (FR_PC_F16 build, float32 GMRES only); the stop test
                         and rel_res are then those of the preconditioned
                         system; 0: none */
  int32_t orthog;     /* Gram-Schmidt of the Arnoldi step: FR_ORTHO_CGS2 (0,
                         classical, twice) or FR_ORTHO_CGS (classical, once:
                         the default of the PETSc GMRES the paper uses; needs
                         restart <= 32) */
} fr_gmres_opts;

enum { FR_ORTHO_CGS2 = 0, FR_ORTHO_CGS = 1 };

typedef struct {
  int32_t iterations;  /* operator products */
  int32_t cycles;
  double rel_res;      /* final residual estimate / ||F|| */
  int32_t converged;
} fr_gmres_stats;

/* ESDIRK schemes of section 2.3: the three-stage, second-order ESDIRK2 and
 * the six-stage, fourth-order ESDIRK4 (the implicit tableau of Kennedy and
 * Carpenter's ARK4(3)6L[2]SA, which the paper takes from Bijl et al.). */
enum { FR_ESDIRK2 = 0, FR_ESDIRK4 = 1 };

/* Pseudo-transient continuation inside an ESDIRK step (section 2.3). */
typedef struct {
  double dtau_init, dtau_max, dtau_min;  /* SER bounds (eq. ser); halving floor: need
                                            0 < dtau_min <= dtau_init <= dtau_max */
  double tol_pseudo;                     /* ||F|| / ||F^0|| stop (paper: 1e-4) */
  int32_t max_ptc_iter;
  int32_t last_stage;                    /* 0 (or the stage count): full step; 2..s-1: return
                                            that stage's solution */
  fr_gmres_opts gmres;
  int32_t scheme;                        /* FR_ESDIRK2 (default, 0) or FR_ESDIRK4 */
} fr_step_opts;

typedef struct {
  int32_t ptc_iterations;
  int32_t gmres_iterations;
  int32_t halvings;    /* dtau halvings after a GMRES failure */
  int32_t stages;      /* implicit stages solved */
  double final_rel_F;  /* ||F|| / ||F^0|| of the last stage */
} fr_step_stats;

/* Builds the device mesh (geometry, degree buckets, face lists) and the
 * residual workspace.  Returns FR_E_INVALID for a non-conforming or
 * inconsistent description. */
fr_status fr_create(const fr_mesh_desc* desc, fr_ctx* out);
/* Releases a context.  Its device blocks and pinned host buffers go back to a
 * per-device cache of the library, which later fr_create / fr_reserve calls
 * reuse (a p-adaptation replaces a context by one of nearly the same sizes);
 * fr_trim frees the cached blocks of every device. */
fr_status fr_destroy(fr_ctx ctx);
fr_status fr_trim(void);

/* Number of degrees of freedom (5 x solution points) and, if sp_offset is not
 * NULL, the first solution point of every element (host [n_elem + 1]). */
fr_status fr_layout(fr_ctx ctx, int64_t* n_dof, int64_t* sp_offset);

/* Graph sets of fr_reserve: the Arnoldi iteration (section 2.3, the GMRES
 * inner loop) captured per (jv_mode, precision). */
enum {
  FR_GRAPHS_F64_EXACT = 1,
  FR_GRAPHS_F32_EXACT = 2,
  FR_GRAPHS_F64_FD = 4,
  FR_GRAPHS_F64_FD_SCALED = 8,
  FR_GRAPHS_ALL = 15,
  /* storage of the element-Jacobi preconditioner (one of the two): sum over
   * elements of N_e^2 float64 or float32 entries (each block rounded up to a
   * multiple of 32 entries), N_e = 5 (p_e + 1)^3 */
  FR_RESERVE_PRECOND_F64 = 16,
  FR_RESERVE_PRECOND_F32 = 32
};

/* Allocates the workspace of gmres_stage_solve and esdirk_step (section
 * 2.3): a Krylov basis of max_restart + 1 vectors of n_dof float64 entries
 * (float32 bases use half of it), the Hessenberg system and 11 n_dof float64
 * vectors of ESDIRK stages, and captures the Arnoldi graphs of every set in
 * graph_sets (or-ed FR_GRAPHS_* bits; sets reserved earlier are kept) and,
 * with FR_RESERVE_PRECOND_F64 or _F32, the element-Jacobi blocks.  It
 * synchronises the device.  Later solver calls with restart <= max_restart
 * and use_graph on a reserved set allocate nothing; a larger restart, an
 * unreserved graph set or an esdirk_step before any fr_reserve returns
 * FR_E_INVALID.  Calling it again with a larger max_restart reallocates;
 * fr_set_launch and fr_autotune capture the reserved graphs again.
 * FR_E_INVALID for max_restart outside 1..200 or unknown bits. */
fr_status fr_reserve(fr_ctx ctx, int32_t max_restart, int32_t graph_sets);

/* R = -(P(div f) + delta) of eq. FR_diff (with R = -div f of eq. ESDIRK_ns).
 * U, R: device [5][n_sp] float64.  R must not alias U. */
fr_status fr_residual(fr_ctx ctx, const double* U, double* R, void* stream);

/* fr_residual for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernels and result, with the face-slot buffers of the residual stages
 * in a static device array of 64 MiB that the library holds on every GPU it
 * runs on until the process ends, instead of the context's workspace.  The
 * call allocates nothing.  Limit: 30 x 8 bytes per own face point, i.e.
 * 240 * 6 * sum_e (p_e + 1)^2 <= 64 MiB (a 32x32x4 mesh of degrees 1..4 fits,
 * 128x128x8 does not); a larger mesh returns FR_E_INVALID with the size it
 * needs.  Every call on one GPU shares that GPU's array and overwrites what
 * the last call left there (each call writes every entry it reads, so nothing
 * needs clearing); calls that overlap in time on one GPU, from any context or
 * stream, race.  The context's device must be current (else FR_E_INVALID).
 * U, R: device [5][n_sp] float64, R must not alias U. */
fr_status fr_residual_noalloc(fr_ctx ctx, const double* U, double* R, void* stream);

/* R(U) and the exact tangent J(U) v in float64 from one forward-mode pass:
 * the dual-number residual kernels carry the residual in their value part and
 * the tangent in their derivative part (as a forward-mode derivative returns
 * the primal with the tangent).  U, v, R, Jv: device [5][n_sp] float64; R and
 * Jv must be distinct and alias neither input. */
fr_status fr_residual_jvp(fr_ctx ctx, const double* U, const double* v, double* R, double* Jv, void* stream);

/* Jv = dR/dU(U) v.  FR_JV_EXACT: forward-mode (dual-number) residual kernels;
 * precision FR_F64: v, Jv float64; FR_F32: v, Jv float32, computed from a
 * float32 copy of U.  FR_JV_FD: the finite difference of section 2.3,
 * (R(U + h v/|v|) - R(U)) |v| / h with h = fd_eps (0 selects 1e-6);
 * FR_JV_FD_SCALED: the same with h = fd_eps sqrt(1 + ||U||_2); float64 only.
 * Jv must not alias v; fd_eps < 0 is FR_E_INVALID. */
fr_status fr_jvp(fr_ctx ctx, const double* U, const void* v, void* Jv, int32_t precision, int32_t jv_mode,
                 double fd_eps, void* stream);

/* JTw = (dR/dU(U))^T w, float64 (reverse mode; face-flux intermediates are
 * recomputed inside the call).  JTw must not alias w. */
fr_status fr_vjp(fr_ctx ctx, const double* U, const double* w, double* JTw, void* stream);

/* Solves (shift I - dR/dU(U)) dU = F (eq. linearized_pseudo_transient_final
 * with shift = 1/(omega dt) + 1/dtau) by restarted GMRES from dU = 0.
 * U, F, dU: device float64 [5][n_sp].  Returns FR_E_NOTCONVERGED (dU and
 * stats still written) if the budget ran out. */
fr_status gmres_stage_solve(fr_ctx ctx, const double* U, double shift, const double* F, double* dU,
                            const fr_gmres_opts* opts, fr_gmres_stats* stats, void* stream);

/* One step of ESDIRK2 or ESDIRK4 (eq. ESDIRK_ns, opts->scheme): stages
 * 2..s are solved by pseudo-transient continuation with SER (eqs.
 * pseudo_transient, ser) and GMRES; a GMRES failure halves dtau and redoes
 * the iterate, until dtau would fall below dtau_min (then FR_E_NOTCONVERGED);
 * each stage starts from the previous stage's solution.  U: device float64,
 * in/out.  FR_E_INVALID for an unknown scheme, a last_stage outside
 * {0, 2..s}, dtau bounds that are not 0 < dtau_min <= dtau_init <= dtau_max,
 * or a context without fr_reserve. */
fr_status esdirk_step(fr_ctx ctx, double* U, double dt, const fr_step_opts* opts, fr_step_stats* stats,
                      void* stream);

/* Preconditioner forms of fr_precond_build beside FR_F64 and FR_F32:
 * FR_PC_F16 builds in float32 (float32 storage) and keeps sigma times the
 * inverse of every block as float16 in place, which halves the bytes each
 * application streams; it serves float32 GMRES with precond = 2. */
enum { FR_PC_F16 = 2 };

/* The element-Jacobi preconditioner of section 2.3: the diagonal blocks of
 * (sigma I - dR/dq(U)), one dense block of order N_e = 5 (p_e + 1)^3 per
 * element, assembled from exact tangent products over a colouring of the
 * elements (no two face neighbours share a colour; seeding one DOF of every
 * element of a colour gives a column of each of their blocks), in the
 * storage precision fr_reserve made (FR_F64: float64 tangents on U; FR_F32:
 * float32 tangents on a float32 copy of U), then LU-factored with partial
 * pivoting and inverted through the factors (as the paper does), in place.
 * The paper evaluates it once at the start of each physical step
 * with sigma = 1/(omega dt) + 1/dtau_max (esdirk_step does so when
 * opts->gmres.precond is set).  U: device float64 [5][n_sp].  Synchronises the
 * stream.  FR_E_INVALID for sigma <= 0 or a precision without storage;
 * FR_E_NONPHYSICAL if a block is singular. */
fr_status fr_precond_build(fr_ctx ctx, const double* U, double sigma, int32_t precision, void* stream);

/* y = P^{-1} x with the preconditioner last built (per element: the row
 * permutation of the factorisation, then the product with the stored
 * inverse).  x, y: device float64 [5][n_sp]; y may
 * be x (in place), else they must not overlap.  FR_E_INVALID if none was
 * built. */
fr_status fr_precond_apply(fr_ctx ctx, const double* x, double* y, void* stream);

/* Spectral-decay smoothness indicator of section 3.1 for variable `var`
 * (the paper uses 1 = rho u): eta[e] = ||s_p - s_{p-1}|| / ||s_p|| in the
 * paper's |J|-weighted Gauss norm (ratio of weighted sums of squares),
 * *eta_max = max_e eta[e].  eta: device [n_elem], eta_max: device scalar. */
fr_status spectral_decay_indicator(fr_ctx ctx, const double* U, int32_t var, double* eta, double* eta_max,
                                   void* stream);

/* Degree selection of section 3.1 on the device: the indicator of variable
 * `var` as above, then per element p + 1 where eta > nu_max * eta_max and
 * p - 1 where eta < nu_min * eta_max (the paper: nu_max = 0.1,
 * nu_min = 0.001; decisions in float64), clamped to [p_min, p_max]; then
 * the lower side of every face whose degrees differ by more than one is
 * raised until no face does.  The paper's eta_{k,max} is not defined beyond
 * its name; eta_max_scope selects the reading: FR_ETA_MAX_ALL, the maximum
 * over all elements, or FR_ETA_MAX_SAME_DEGREE, the maximum over the
 * elements of the same degree as the element (so that elements are ranked
 * among those whose indicator measures the same modes).  p_new: device int8
 * [n_elem], written in mesh order.  FR_E_INVALID for 1 <= p_min <= p_max <= 5
 * violated, var outside 0..4, nu_max < nu_min or an unknown scope.  To
 * adapt, create a context for p_new and move the state with fr_project. */
enum { FR_ETA_MAX_ALL = 0, FR_ETA_MAX_SAME_DEGREE = 1 };
fr_status fr_select_degrees(fr_ctx ctx, const double* U, int32_t var, double nu_max, double nu_min, int32_t p_min,
                            int32_t p_max, int32_t eta_max_scope, int8_t* p_new, void* stream);

/* Moves a state between two contexts of the same mesh with different degree
 * fields (section 3.1: a lower degree takes the projection of the solution
 * onto the lower-degree space).  Element by element in reference coordinates:
 * to a lower degree the L2 projection onto the tensor space of that degree
 * (Legendre modes truncated); to an equal or higher degree the element
 * polynomial evaluated at the new solution points (exact).  U_src: device
 * float64 in src's layout; U_dst: device float64 in dst's layout (distinct
 * buffers).  FR_E_INVALID if the element counts or devices differ. */
fr_status fr_project(fr_ctx src, const double* U_src, fr_ctx dst, double* U_dst, void* stream);

/* Nodal polynomial filter (section 4.2, the SD7003 runs with p^3 elements;
 * the method of Fischer and Mullen): in every element of degree p >= p_from
 * (the paper filters p > 2, i.e. p_from = 3, with alpha = 0.2),
 *   q <- (1 - alpha) q + alpha P q,
 * P the projection onto the degree p - 1 space taken as in fr_project
 * (reference-space L2 projection onto the tensor polynomials of degree
 * p - 1, the highest Legendre mode of each direction removed) and evaluated
 * at the element's solution points; all five variables.  Elements of lower
 * degree keep their values.  U, U_out: device float64 [5][n_sp]; U_out may
 * be U (in place), otherwise U is copied to U_out first on the stream.
 * FR_E_INVALID for alpha outside [0, 1], p_from outside 1..5 or a U_out
 * that overlaps U without being U.  The paper
 * does not say when in the step the filter acts; the caller applies it (for
 * example after each time step). */
fr_status fr_filter(fr_ctx ctx, const double* U, double* U_out, double alpha, int32_t p_from, void* stream);

/* Picks, per scalar kind, the launch shapes of the residual kernels by timing
 * the candidates on U (device float64): elements (faces) per block of every
 * degree bucket in the per-bucket mode; items per tile of every stage and
 * degree (degree pair) in the fused plans; the one- or two-pass face stage.
 * It synchronises the stream and captures the reserved Arnoldi graphs again
 * with the chosen shapes. */
fr_status fr_autotune(fr_ctx ctx, const double* U, void* stream);

/* Items per tile of the fused (degree-bucketed) plans of one scalar kind
 * (0: float64, 1: float64 dual numbers, 2: float32 dual numbers), as chosen by
 * fr_autotune or the default: out[3 i .. 3 i + 2] = (stage: 0 traces, 1
 * interior faces, 2 divergence; code: n = p + 1 of an element bucket, or
 * 8 n_low + n_high of a face bucket; items per 256-thread tile), host memory,
 * for up to max_out entries; *n_out = entries written. */
fr_status fr_launch_shapes(fr_ctx ctx, int32_t kind, int32_t* out, int32_t max_out, int32_t* n_out);

/* Per-launch timing of one operator's kernels (op 0: residual float64,
 * 1: exact tangent float64, 2: exact tangent float32, 3: residual and
 * float64 tangent from one pass as fr_residual_jvp; U doubles as the
 * direction).  Each launch is bracketed by HIP events on `stream`; out[i]
 * receives the stage ("k_trace", "k_face", "k_bface", "k_div"), the degree
 * sizes n = p + 1 of its bucket, the elements or faces it processes and the
 * average duration over `reps` runs.  Synchronises the stream. */
typedef struct {
  char stage[16];
  int32_t n_lo, n_hi;
  int64_t units;
  double ms;
} fr_kernel_time;
fr_status fr_profile(fr_ctx ctx, const double* U, int32_t op, int32_t reps, fr_kernel_time* out, int32_t max_out,
                     int32_t* n_out, void* stream);

/* Launch mode of the residual, tangent and Krylov operators of a context.
 * FR_LAUNCH_PER_BUCKET (default): each stage (traces, faces, divergence) is
 * launched once per degree bucket (per degree pair for faces).
 * FR_LAUNCH_FUSED: each stage is one launch over all buckets, its blocks
 * ordered by decreasing work (the degree-bucketed work queue). */
enum { FR_LAUNCH_PER_BUCKET = 0, FR_LAUNCH_FUSED = 1 };
/* Optional flags or-ed into the mode (Navier-Stokes only; without either,
 * the current choice for that launch mode is kept, which fr_autotune makes
 * per scalar kind by timing):
 * FR_LAUNCH_FACES_TWO_PASS: the interior-face stage runs as two kernels, the
 * inviscid common flux and then the viscous correction (each needs about half
 * the registers of the one-pass face kernel);
 * FR_LAUNCH_FACES_ONE_PASS: one kernel for both (the default). */
enum { FR_LAUNCH_FACES_TWO_PASS = 4, FR_LAUNCH_FACES_ONE_PASS = 8 };
fr_status fr_set_launch(fr_ctx ctx, int32_t mode);

/* Reads and clears the non-physical-state flag (synchronises the stream). */
fr_status fr_check(fr_ctx ctx, int32_t* nonphysical, void* stream);

/* Text of the last error on this context (or of the last failed fr_create
 * if ctx is NULL).  Valid until the next call on the same context. */
const char* fr_last_error(fr_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* FR_H */
