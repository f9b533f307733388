/*
 * yasps.h -- C ABI of the MI355X (gfx950) library for one Newton iteration of
 * Incremental Potential Contact,
 *
 *     E(x) = 1/2 |x - x_tilde|_M^2 + h^2 sum_t Psi_t(x) + sum_s kappa b(d_s(x)),
 *
 * where the elastic sum runs over tets and, for cloth, over StVK membrane
 * triangles and dihedral bending hinges (the paper's cloth examples,
 * section "Examples").
 * after "YASPS: A Symbolic Framework for Extensible, High-Performance IPC
 * Simulation" (ACM TOG 45(4), 2026).  The library evaluates per-stencil
 * energy, gradient and PSD-projected local Hessians (stable Neo-Hookean tets,
 * Eq. snh; log-barrier contact stencils, section "Eigendecomposition:
 * Automatic Optimization"), assembles them without atomics into a 3x3
 * block-sparse upper-triangular Hessian (appendix "Global Hessian
 * Compression"), and solves H p = b with block-Jacobi preconditioned CG
 * (section "Solver", appendices "SpMV" and "Preconditioner").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array pointers in yasps_problem / yasps_contacts and every x / b / p
 *   argument are DEVICE pointers on the device that is current when
 *   yasps_create is called.  They stay owned by the caller and must outlive
 *   the context (problem arrays) or the call (x, b, p).
 * - Vertex ids: 0 <= i < n_free is a free vertex (3 DoF); n_free <= i <
 *   n_free + n_fixed is fixed vertex i - n_free (no DoF; the paper's
 *   "special primitive whose degrees of freedom are excluded from
 *   differentiation", Table 1 caption); -1 marks an unused stencil entry.
 * - Positions and vectors are (n_rows, 3) row-major f64 over the rows of degrees
 *   of freedom: the free vertices, then four rows per affine body (n_rows =
 *   n_free + 4 n_bodies; n_rows = n_free without bodies).
 * - Per-stencil arrays are structure-of-arrays: tet_idx is [4][n_tets]
 *   (entry k of tet t at tet_idx[k * n_tets + t]), dm_inv is [9][n_tets]
 *   (row-major 3x3 components), contact idx is [4][n_contacts].
 * - Work is enqueued on the stream given to yasps_create; calls return after
 *   their host-visible scalars (energies, solver info) are final.
 * - Every call returns a yasps_status; no C++ exception crosses the ABI.
 *   yasps_last_error() describes the last failure of a context.
 * - A context is not thread safe; distinct contexts are independent.
 */
#ifndef YASPS_H
#define YASPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t yasps_status;
#define YASPS_OK 0
#define YASPS_E_ARG (-1)        /* invalid argument, index out of range, repeated vertex in a stencil */
#define YASPS_E_HIP (-2)        /* a HIP runtime call failed */
#define YASPS_E_DOMAIN (-3)     /* a contact stencil has squared distance d <= 0 */
#define YASPS_E_NONFINITE (-4)  /* NaN/Inf in positions or in an evaluated quantity */
#define YASPS_E_NOCONV (-5)     /* PCG hit max_iter; the last iterate is still returned */
#define YASPS_E_BREAKDOWN (-6)  /* PCG met p^T H p <= 0 (matrix not positive definite) */
#define YASPS_E_UNIMPL (-7)     /* option not implemented */
#define YASPS_E_LINESEARCH (-8) /* no admissible step after the maximum number of halvings */

/* contact stencil types and their vertex order */
#define YASPS_PT 0 /* (p, t0, t1, t2): squared distance from p to the plane of the triangle */
#define YASPS_EE 1 /* (a0, a1, b0, b1): squared distance between the two edge lines */
#define YASPS_PE 2 /* (p, e0, e1, -1): squared distance from p to the edge line */
#define YASPS_PP 3 /* (p, q, -1, -1): squared distance between the points */

/* yasps_params.precision */
#define YASPS_FP64 0  /* everything in float64 */
#define YASPS_MIXED 1 /* float32 element Hessians, BSR values and PCG inner vectors; contact
                         geometry, barrier, contact projection, energies, gradient and the
                         Newton residual stay float64 */
/* yasps_params.proj: where the Neo-Hookean Hessian is projected */
#define YASPS_F_SPACE 0 /* h^2 J_F^T Proj(d2Psi/dF2) J_F (9x9 eigenproblem), section
                           "Eigendecomposition: Manual Optimization" */
#define YASPS_X_SPACE 1 /* Proj(h^2 d2Psi/dx2) over the tet's free vertices */
/* yasps_newton_params.hessian and the `flags` argument of yasps_eval_stencils */
#define YASPS_PROJECTED 0 /* local Hessians projected to the PSD cone (negative eigenvalues -> 0) */
#define YASPS_EXACT 1     /* unprojected local Hessians (adjoint solves) */
/* yasps_params.barrier */
#define YASPS_SQLOG 0       /* kappa (d - dhat)^2 log(d/dhat)^2, as printed in the paper */
#define YASPS_IPC_CLASSIC 1 /* -kappa (d - dhat)^2 log(d/dhat) */
/* yasps_params.index_build: where yasps_set_contacts builds the dynamic part's
   pattern, slot map, staging layout and SpMV rows (identical results; the paper
   rebuilds only this part when the contacts change, section "Implementation") */
#define YASPS_INDEX_DEVICE 0 /* on the GPU: a stable counting sort, a stable radix sort and scans */
#define YASPS_INDEX_HOST 1   /* on the host (reference) */

typedef struct yasps_ctx yasps_ctx;

typedef struct {
  int32_t n_free;          /* free vertices */
  int32_t n_fixed;         /* fixed vertices */
  const double* x_fixed;   /* (n_fixed, 3) positions of fixed vertices; may be NULL if n_fixed == 0 */
  const double* mass;      /* (n_free) lumped masses */
  const double* x_tilde;   /* (n_rows, 3) inertial target x0 + h v0 + h^2 g (a body's rows: its q~);
                              ignored if is_static */
  int32_t n_tets;
  const int32_t* tet_idx;  /* [4][n_tets] vertex ids, positively oriented at rest */
  const double* dm_inv;    /* [9][n_tets] inverse rest edge matrices Dm^-1, row-major components */
  const double* vol;       /* [n_tets] rest volumes */
  const double* mu_lambda; /* [2][n_tets] per-tet Lame parameters, or NULL to use mu / lambda */
  double mu, lambda;       /* global Lame parameters when mu_lambda is NULL */
  double h;                /* time step; the elastic term is scaled by h^2 */
  double kappa;            /* barrier stiffness */
  double dhat;             /* barrier activation, a SQUARED distance; d >= dhat contributes 0 */
  double gravity[3];       /* used only when is_static: adds -sum_v m_v gravity . x_v */
  int32_t is_static;       /* 1: static equilibrium (no inertia term), 0: implicit Euler step */
  /* Cloth (all optional; n_tris = n_hinges = 0 for volumetric scenes), the
   * membrane and bending terms of the paper's cloth examples (section
   * "Examples"; StVK membrane, discrete-shells dihedral bending).  Both are
   * elastic energies and are scaled by h^2 like the tets'.  The membrane
   * Hessian is projected in F-space (6x6); the hinge Hessian on its free
   * vertices (section "Eigendecomposition (EVD) and PSD Projection"). */
  int32_t n_tris;           /* StVK membrane triangles */
  const int32_t* tri_idx;   /* [3][n_tris] vertex ids, counter-clockwise in the rest frame */
  const double* tri_dm_inv; /* [4][n_tris] inverse 2x2 rest edge matrices [X1 - X0, X2 - X0]^-1 in a
                               2-D frame of the rest triangle, row-major components */
  const double* tri_area;   /* [n_tris] rest areas */
  double mu_c, lambda_c;    /* membrane Lame parameters: Psi = A t [mu tr(G^2) + lambda/2 (tr G)^2],
                               G = (F^T F - I) / 2 */
  double thickness;         /* t */
  int32_t n_hinges;         /* dihedral bending hinges */
  const int32_t* hinge_idx; /* [4][n_hinges]: shared edge (x0, x1), then the wing x2 of the triangle
                               (x0, x1, x2) and the wing x3 of the triangle (x1, x0, x3); at least one
                               free vertex each */
  const double* hinge_rest; /* [2][n_hinges]: rest angle theta_bar, stiffness k (E = k (theta -
                               theta_bar)^2, k = k_b 3 |e_bar|^2 / (A1 + A2) for discrete shells) */
  /* Affine bodies (all optional; n_bodies = 0 without): a body vertex sits at
   * p = A r + t (the paper's mixed parameterisation, section "UNION").  Each
   * body adds four rows of degrees of freedom after the free vertices: the
   * columns a_1, a_2, a_3 of A, then t; so x, x_tilde and every vector are
   * (n_free + 4 n_bodies, 3).  Energies per body: inertia 1/2 (q - q~)^T
   * (M4 (x) I3) (q - q~) and the orthogonality regulariser
   * h^2 k_b 1/2 |A^T A - I|_F^2 (the paper's E_affine), its 9x9 Hessian
   * projected.  Body vertices have ids n_free + n_fixed + k and appear only in
   * the stencils given to yasps_set_body_contacts. */
  int32_t n_bodies;
  const double* body_mass;  /* [n_bodies][16] row-major 4x4 M4 = sum_v m_v w_v w_v^T, w = (r, 1) */
  const double* body_k;     /* [n_bodies] orthogonality stiffness k_b */
  int32_t n_body_verts;
  const int32_t* body_of;   /* [n_body_verts] body of each body vertex */
  const double* body_rest;  /* [n_body_verts][3] rest position r */
} yasps_problem;

typedef struct {
  int32_t n_contacts;
  const int32_t* type; /* [n_contacts] YASPS_PT / EE / PE / PP */
  const int32_t* idx;  /* [4][n_contacts] vertex ids in the order given for the type */
  const double* ee_eps; /* [n_contacts] or NULL: edge-edge mollifier thresholds eps_x (IPC's
                           1e-3 |a1 - a0|^2 |b1 - b0|^2 from rest edge lengths).  An EE stencil
                           with eps_x > 0 and c = |(a1 - a0) x (b1 - b0)|^2 < eps_x has the
                           barrier m(c) kappa b(d), m = (c / eps_x)(2 - c / eps_x) (near-parallel
                           edges; m = 1 above eps_x).  Ignored for the other types; NULL or
                           eps_x <= 0: no mollifier. */
} yasps_contacts;

typedef struct {
  int32_t precision; /* YASPS_FP64 or YASPS_MIXED */
  int32_t proj;      /* YASPS_F_SPACE or YASPS_X_SPACE */
  int32_t barrier;   /* YASPS_SQLOG or YASPS_IPC_CLASSIC */
  int32_t index_build; /* YASPS_INDEX_DEVICE or YASPS_INDEX_HOST */
} yasps_params;

typedef struct {
  double energy;    /* total E(x), summed in float64 in a fixed order */
  double e_inertia; /* 1/2 |x - x_tilde|_M^2, or -sum m g.x when static */
  double e_elastic; /* h^2 sum of the tet, membrane and hinge energies */
  double e_contact; /* sum kappa b(d_s) */
  double min_d;     /* smallest contact squared distance (+inf without contacts) */
  int32_t n_active; /* contact stencils with d < dhat */
} yasps_eval_info;

/* Device views of context-owned storage, valid until the next yasps_set_contacts,
 * yasps_set_body_contacts or yasps_destroy.  Upper-triangular BSR with row-major
 * 3x3 blocks over n_rows = n_free + 4 n_bodies rows; the diagonal block is the
 * first block of every static row.  H = H_static + H_dynamic + H_body. */
typedef struct {
  int32_t n_rows;       /* n_free + 4 n_bodies */
  int32_t nnzb_static;  /* elastic pairs, body blocks and every diagonal */
  int32_t nnzb_dynamic; /* contact pairs */
  const int32_t* row_ptr_s; const int32_t* col_idx_s; const void* values_s;
  const int32_t* row_ptr_d; const int32_t* col_idx_d; const void* values_d;
  int32_t values_are_f32; /* 1 in the MIXED precision form, else float64 */
  const double* grad;     /* (n_rows, 3) float64 gradient */
  const double* block_inv;/* (n_rows, 9) float64 inverses of the diagonal blocks of H */
  int32_t nnzb_body;      /* pairs of the stencils touching bodies (third part) */
  const int32_t* row_ptr_b; const int32_t* col_idx_b; const void* values_b;
} yasps_bsr_view;

typedef struct {
  int32_t iters;       /* matrix-vector products performed */
  double rel_residual; /* |b - H x| / |b| of the recurrence residual at exit */
  int32_t status;      /* YASPS_OK, YASPS_E_NOCONV or YASPS_E_BREAKDOWN */
} yasps_pcg_info;

typedef struct {
  double rtol;          /* PCG relative tolerance (default 1e-8) */
  int32_t max_iter;     /* PCG iteration cap (default 20000) */
  int32_t max_halvings; /* line-search halvings (default 40) */
  double armijo;        /* sufficient-decrease constant (default 1e-4) */
  double tie_rtol;      /* a trial with |E - E(x)| <= tie_rtol |E(x)| also counts as a decrease
                           (for solves driven to the rounding floor of E); 0 = plain Armijo */
  int32_t hessian;      /* YASPS_PROJECTED (default, 0): projected Newton; YASPS_EXACT: solve with the
                           unprojected Hessian (near a minimum where it is positive definite; returns
                           YASPS_E_BREAKDOWN when PCG meets p^T H p <= 0) */
  double shift;         /* >= 0: the solve uses H + shift diag(m_v I) (Levenberg-Marquardt damping with
                           the lumped masses; the assembled BSR holds the shifted matrix until the next
                           assembly); the line search still uses E itself.  0 = plain Newton */
} yasps_newton_params;

typedef struct {
  double e0, e1;       /* energy before / after the step */
  double alpha;        /* accepted step length (0 if none) */
  double alpha0;       /* initial step bound min(1, 0.4 min sqrt(d) / max |p_v|) */
  double grad_dot_p;   /* g . p (< 0 for a descent direction) */
  double grad_max;     /* max_v |g_v| at the start of the step (stop rules) */
  double step_max;     /* max_v |alpha p_v| of the accepted step */
  int32_t cg_iters;
  double cg_rel_residual;
  int32_t cg_status;
  int32_t ls_trials;
  /* phase times measured with HIP events on the context stream (ms) */
  float ms_eval, ms_assemble, ms_pcg, ms_linesearch;
} yasps_newton_info;

/* Creates a context bound to the current device and `hip_stream` (a hipStream_t,
 * NULL = default stream).  Validates the tets, triangles and hinges (ids in
 * range, distinct vertices, every hinge with a free vertex), builds the static
 * pattern and slot map over tets, then triangles, then hinges (appendix
 * "Global Hessian Compression"), and allocates the workspace.  `opt` may be
 * NULL for defaults.
 * Errors: YASPS_E_ARG, YASPS_E_UNIMPL, YASPS_E_HIP.  *out is NULL on failure. */
yasps_status yasps_create(yasps_ctx** out, void* hip_stream, const yasps_problem* P,
                          const yasps_params* opt);

/* Replaces the contact stencil list (the paper's dynamic primitives, section
 * "Index Generator" and the static/dynamic split of the index-computation
 * evaluation) and rebuilds the dynamic pattern, slot map, staging layout and
 * SpMV rows: on the GPU by default (YASPS_INDEX_DEVICE), on the host with
 * YASPS_INDEX_HOST; both give the same arrays.  `type` and `idx` are device
 * arrays; they are copied, and the caller may free them after the call.  The
 * call synchronises the context stream.  Errors: YASPS_E_ARG (the first
 * stencil with an unknown type, an id out of range, a repeated or misplaced
 * vertex, or no free vertex; the context is then left without contacts),
 * YASPS_E_HIP. */
yasps_status yasps_set_contacts(yasps_ctx* ctx, const yasps_contacts* C);

/* Replaces the list of contact stencils that touch affine bodies (vertex ids
 * as in yasps_contacts, body vertices allowed; each side of a stencil should
 * come from one body or from free / fixed vertices: a stencil may reach at
 * most 8 rows of degrees of freedom).  Their derivatives follow the chain
 * rule through the union of free, fixed and body vertices (section
 * "Differentiation of Unioned Attributes"); the local Hessian is projected
 * over the stencil's movable positions and mapped to the degrees of freedom,
 * J^T Proj(H_p) J (the reduced-coordinate projection of section
 * "Eigendecomposition (EVD) and PSD Projection": 6x6 for a point-point
 * stencil whatever the bodies).  They form a third part of the matrix, built
 * on the host.  Arrays are device arrays, copied.  Errors: YASPS_E_ARG (bad
 * type or id, a repeated vertex, no movable vertex, more than 8 rows; the
 * context is then left without body contacts), YASPS_E_HIP. */
yasps_status yasps_set_body_contacts(yasps_ctx* ctx, const yasps_contacts* C);

/* Evaluates every stencil at positions x (n_rows, 3): energies, gradients and
 * local Hessians (flags: YASPS_PROJECTED or YASPS_EXACT), staged for assembly.
 * Fills *info (may be NULL).  Errors: YASPS_E_DOMAIN (some contact d <= 0),
 * YASPS_E_NONFINITE, YASPS_E_HIP. */
yasps_status yasps_eval_stencils(yasps_ctx* ctx, const double* x, int32_t flags,
                                 yasps_eval_info* info);

/* Sums the staged contributions of the last yasps_eval_stencils into the BSR
 * values, the gradient and the inverted diagonal blocks (block-Jacobi M^-1),
 * without atomics and in a fixed order (bitwise reproducible).  *view (may be
 * NULL) receives device pointers to the result.  Errors: YASPS_E_HIP,
 * YASPS_E_ARG if called before any evaluation. */
yasps_status yasps_assemble_bsr(yasps_ctx* ctx, yasps_bsr_view* view);

/* Solves H x = b with block-Jacobi preconditioned CG on the assembled H
 * (x0 = 0, stop when |r| <= rtol |b| or after max_iter products).  b and x
 * are (n_rows, 3) device arrays; x is overwritten.  The system is solved as
 * given (the paper's convention, section "Solution Extraction").
 * Errors: YASPS_E_NOCONV (x holds the last iterate), YASPS_E_BREAKDOWN,
 * YASPS_E_ARG, YASPS_E_HIP. */
yasps_status yasps_pcg(yasps_ctx* ctx, const double* b, double* x, double rtol, int32_t max_iter,
                       yasps_pcg_info* info);

/* yasps_pcg for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, bit for bit, with the solver's workspace (Krylov vectors,
 * per-workgroup partials, device scalars) in one fixed array per GPU instead of
 * the context's.  The call makes no hipMalloc / hipFree and no allocating
 * library call.  The array is 32 MiB; a solve needs 96 bytes per free vertex
 * plus 24 bytes per SpMV slot (one per chunk of stored blocks and row it
 * reaches: about 3 per vertex on tet meshes) plus 25 KiB, so the 40^3-cell
 * block (68,921 free vertices) fits with room to spare; larger systems are
 * rejected with YASPS_E_ARG before anything is launched.  Each GPU the library runs on
 * holds its own array until the process ends; every call on one GPU shares
 * it and leaves the last solve's contents there (no call reads what an earlier
 * one left: the solver writes its state and vectors before reading them), so
 * calls that overlap on one GPU (contexts on different streams or host
 * threads) race.  Arguments, results and the other errors are yasps_pcg's. */
yasps_status yasps_pcg_noalloc(yasps_ctx* ctx, const double* b, double* x, double rtol, int32_t max_iter,
                               yasps_pcg_info* info);

/* One Newton step on the current stencil set (projected local Hessians unless
 * prm->hessian = YASPS_EXACT): evaluate, assemble, solve H p = -g, then
 * backtrack from alpha0 = min(1, 0.4 min_s sqrt(d_s) /
 * max_v |p_v|) by halving until every contact d > 0, every PT/EE stencil keeps
 * its side of the plane/line, and E(x + alpha p) <= E(x) + armijo alpha g.p.
 * x (n_rows, 3) is updated in place.  `prm` may be NULL for defaults.
 * Errors: as eval / pcg, plus YASPS_E_LINESEARCH (x unchanged). */
yasps_status yasps_newton_step(yasps_ctx* ctx, double* x, const yasps_newton_params* prm,
                               yasps_newton_info* info);

/* Copies one part of the pattern to HOST arrays for inspection (bit-exact tests):
 * part 0 = static, 1 = dynamic, 2 = body contacts.  row_ptr has n_rows + 1
 * entries (n_rows = n_free + 4 n_bodies), col_idx nnzb, slot [n_stencils][10]
 * (part 0: tets, then triangles, then hinges, then bodies (their 4 rows), each
 * in the order given at create; part 1: contacts in the order given; local
 * pair (a, b), a <= b, enumerated row by row over the stencil's used vertices;
 * -1 = no block), for part 2 [n_stencils][36] over each stencil's row list
 * (its vertices' rows in vertex order, a body's four rows once).
 * Any output pointer may be NULL.  Errors: YASPS_E_ARG. */
yasps_status yasps_get_pattern(yasps_ctx* ctx, int32_t part, int32_t* row_ptr, int32_t* col_idx,
                               int32_t* slot);

/* Adjoint of the static-equilibrium solve with per-tet Young's modulus theta_t
 * (mu_t, lambda_t proportional to theta_t): for every tet writes
 * grad_theta[t] = -lambda_t^T d/dx (Psi_t(x) / theta_t), the mixed partial
 * d2E/dx dtheta_t contracted with the adjoint vector lambda (x, lambda: (n_rows, 3)).
 * theta (n_tets) and grad_theta (n_tets) are device arrays.
 * Errors: YASPS_E_ARG, YASPS_E_HIP. */
yasps_status yasps_theta_adjoint(yasps_ctx* ctx, const double* x, const double* lambda,
                                 const double* theta, double* grad_theta);

/* Levenberg-Marquardt damping scale for the damped Newton steps of the static
 * equilibrium of the differentiation form (yasps_newton_params.shift; the
 * paper's own solver, section "Solver", takes plain projected Newton steps):
 * *out = frac * median over the free vertices v of |tr(H_vv)| / (3 m_v), with
 * H_vv the diagonal block (all matrix parts) of the last assembly,
 * including any shift that assembly added, and m_v the lumped masses.  For an
 * even vertex count the median is the mean of the two middle values.
 * Errors: YASPS_E_ARG (before any assembly, frac < 0), YASPS_E_HIP. */
yasps_status yasps_lm_shift(yasps_ctx* ctx, double frac, double* out);

/* ---- Time stepping with contact (IPC's frame loop; the paper takes its
 * collision detection and CCD from an external module, section "Limitations")
 * ---- */

/* Collision surface: the primitives whose pairs can touch.  Vertex ids as in
 * yasps_contacts (free or fixed).  Device arrays, copied. */
typedef struct {
  int32_t n_points;
  const int32_t* points;        /* [n_points] vertex ids */
  int32_t n_edges;
  const int32_t* edges;         /* [2][n_edges] */
  int32_t n_tris;
  const int32_t* tris;          /* [3][n_tris] */
  const double* edge_rest_len2; /* [n_edges] squared rest lengths, or NULL: the edge-edge stencils found
                                   get the mollifier threshold 1e-3 |a|^2 |b|^2 (none when NULL) */
  double cell;                  /* cell size of the search grid (> 0; about the longest edge).  A search
                                   counts its entries per cell over the box of cells the primitives
                                   span (up to 2^22 cells, else it sorts them by cell: slower); a
                                   primitive whose box covers more than 2^16 cells is an error */
} yasps_surface;

typedef struct {
  double tol;           /* stop when max_v |p_v| / h < tol (m/s; the paper's examples use 1e-2) */
  int32_t max_newton;   /* Newton iterations at most (default 50) */
  double rtol;          /* PCG relative tolerance (default 1e-8) */
  int32_t max_iter;     /* PCG iteration cap (default 20000) */
  double armijo;        /* sufficient-decrease constant (default 1e-4) */
  int32_t max_halvings; /* line-search halvings (default 40) */
  double ccd_s;         /* additive CCD: stop once the distance falls below ccd_s times its start (0.1) */
} yasps_frame_params;

typedef struct {
  int32_t newton_iters;   /* steps taken */
  int32_t cg_iters;       /* PCG iterations of all solves */
  int32_t ls_trials;      /* line-search energy evaluations */
  int32_t n_contacts_max; /* most stencils found by one proximity search */
  double e_begin, e_end;  /* incremental potential at the first and the last iterate */
  double alpha_min;       /* smallest accepted step */
  int32_t converged;      /* 1 if the stop rule was met */
  float ms_detect, ms_newton, ms_ccd, ms_linesearch; /* device time per phase (HIP events) */
} yasps_frame_info;

/* Sets the collision surface (replaces the previous one).  Errors:
 * YASPS_E_ARG (ids out of range, a degenerate edge or triangle, cell <= 0),
 * YASPS_E_HIP. */
yasps_status yasps_set_surface(yasps_ctx* ctx, const yasps_surface* S);

/* Proximity search at positions x (n_rows, 3): every point-triangle and
 * edge-edge pair of the surface (no shared vertex, at least one free or
 * affine-body vertex, not all its vertices on one body; a body vertex at
 * r_1 a_1 + r_2 a_2 + r_3 a_3 + t) whose squared distance is below dhat
 * becomes one contact stencil, typed by
 * where its closest points lie (point-triangle: face / edge / vertex -> PT /
 * PE / PP; edge-edge: both interiors / one endpoint / two endpoints -> EE / PE
 * / PP; Ericson, Real-Time Collision Detection, 5.1.5 and 5.1.9).  Pairs are
 * not merged, so the barrier sum is IPC's sum over primitive pairs.  The
 * stencils replace the contact set (as yasps_set_contacts with the device
 * index build; those that reach a body vertex replace the body contacts, as
 * yasps_set_body_contacts); order: point-triangle pairs by (point,
 * triangle), then edge-edge pairs by (edge, edge).  *n_contacts (may be NULL) receives their
 * number.  Errors: YASPS_E_ARG (no surface; a primitive's box over more than
 * 2^16 grid cells: a non-finite position or a cell size far below the
 * primitives), YASPS_E_HIP. */
yasps_status yasps_detect(yasps_ctx* ctx, const double* x, int32_t* n_contacts);

/* Copies the stencils of the last yasps_detect to HOST arrays (any may be
 * NULL): type [n], idx [4][n], ee_eps [n] (0 for non-EE stencils).
 * Errors: YASPS_E_HIP. */
yasps_status yasps_get_detected(yasps_ctx* ctx, int32_t* type, int32_t* idx, double* ee_eps);

/* Largest conservative step along x + t p, t <= t_max: the minimum over the
 * point-triangle and edge-edge pairs whose swept boxes (inflated by
 * sqrt(dhat) / 2) overlap of additive CCD (Li, Kaufman, Jiang 2021), which
 * stops a pair once its distance falls below s times its start value.  A
 * body vertex moves by the affine map of its body's row motion (linear, so
 * its trajectory is a straight line).  x, p: (n_rows, 3) device arrays.
 * Errors: YASPS_E_ARG, YASPS_E_HIP. */
yasps_status yasps_ccd(yasps_ctx* ctx, const double* x, const double* p, double t_max, double s, double* t_out);

/* One implicit-Euler time step with contact (IPC): x_tilde = x + h v + h^2 g
 * (the problem's h and gravity, on the free rows and the bodies' t rows —
 * M4^-1 of a body's gravity force moves t only; the problem's x_tilde is not
 * used), then
 * Newton iterations, each: proximity search at x (yasps_detect), projected
 * Newton direction p by PCG, stop when max_v |p_v| / h < tol, step bound by
 * CCD, Armijo backtracking on E with the contacts found at each trial; at the
 * end v = (x - x_start) / h.  x and v (n_rows, 3) device arrays, updated in
 * place.  `prm` may be NULL for defaults.  Needs the dynamic form and a
 * surface.  Errors: YASPS_E_ARG, YASPS_E_NOCONV (max_newton reached; x, v
 * hold the last iterate),
 * YASPS_E_LINESEARCH, YASPS_E_BREAKDOWN, YASPS_E_HIP. */
yasps_status yasps_frame(yasps_ctx* ctx, double* x, double* v, const yasps_frame_params* prm,
                         yasps_frame_info* info);

/* Kernel classes timed by the opt-in profiler (yasps_profile_*). */
#define YASPS_K_INERTIA 0       /* inertia / gravity term per vertex */
#define YASPS_K_SNH 1           /* Neo-Hookean tet evaluation (energy, gradient, projected Hessian) */
#define YASPS_K_CONTACT 2       /* contact stencil evaluation (all groups) */
#define YASPS_K_ASSEMBLE 3      /* segmented sums of the staged blocks and gradient */
#define YASPS_K_BLOCKINV 4      /* block-Jacobi inverse */
#define YASPS_K_SPMV 5          /* PCG: w = H u with the u.w partials */
#define YASPS_K_PCG_UPDATE 6    /* PCG: recurrences, vector updates, preconditioning */
#define YASPS_K_LINESEARCH 7    /* line-search energy and feasibility kernels */
#define YASPS_K_CLOTH 8         /* membrane and hinge evaluation */
#define YASPS_K_COUNT 9

/* Opt-in per-kernel timing with HIP events recorded on the context stream
 * around every launch of each class (adds a little launch overhead; off by
 * default).  enable = 1 turns it on and clears the totals, 0 turns it off.
 * yasps_profile_query returns the launches and the summed device time (ms)
 * of one class since it was enabled.  Errors: YASPS_E_ARG, YASPS_E_HIP. */
yasps_status yasps_profile_enable(yasps_ctx* ctx, int32_t enable);
yasps_status yasps_profile_query(yasps_ctx* ctx, int32_t kernel_class, int32_t* launches, double* total_ms);

/* y = H x with the assembled H (both parts), through the same SpMV kernel the
 * solver uses (appendix "SpMV"); x, y (n_rows, 3) device arrays.
 * Errors: YASPS_E_ARG (before assembly), YASPS_E_HIP. */
yasps_status yasps_spmv(yasps_ctx* ctx, const double* x, double* y);

/* Frees the context and everything it owns.  NULL is accepted. */
void yasps_destroy(yasps_ctx* ctx);

/* Message describing the last error of ctx (or of the last failed create when
 * ctx is NULL).  The string is owned by the library. */
const char* yasps_last_error(const yasps_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* YASPS_H */
