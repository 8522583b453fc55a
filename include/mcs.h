/*
 * mcs.h -- C ABI of the MI355X solver for the hybridised mass conserving mixed
 * stress (MCS) discretisation of the Stokes problem with its conforming
 * auxiliary-space preconditioner.
 *
 * Method: Kogler, Lederer, Schoeberl, "A conforming auxiliary space
 * preconditioner for the mass conserving mixed stress method"
 * (arXiv 2207.08481).  Problem statement: Sec. 1, eq. (stokes):
 *     -div(nu eps(u)) + grad p = f,  div u = 0  in Omega,   u = 0 on dOmega,
 * discretised by eq. (discrmixedstressstokesweak) with the spaces of Sec. 3
 * (order k >= 2), sigma and omega statically condensed (Sec. 4.2), or, for
 * k = 1 in 3D, by the method of Sec. 7, the lowest order case (omega in the
 * lowest-order Raviart-Thomas space entering through kappa(omega), one flux
 * dof per facet beside the velocity dofs, only sigma condensed, the
 * stabilisation nu |T|^(2/3) (div omega, div eta)_T, E u = (u, Pi^0 u_t,
 * curl u)), and solved
 * by MINRES preconditioned with the block factorisation eq. (mhatinvfactor)
 * whose velocity block is the multiplicative auxiliary-space preconditioner
 * of the double Schur complement (Sec. 6.1, Theorem aux_pc_schur, Corollary
 * aux_pc_mult) applied through the bubble factorisation eq. (factorSsigma).
 *
 * Conventions
 * -----------
 * Ownership: every pointer argument is owned by the caller.  Pointers named
 * *_host are host memory; all other data pointers are device memory of the
 * device the problem is bound to.  The library never allocates device memory:
 * all of its device state lives in the caller's workspace (mcs_bind).
 *
 * Mesh: dim in {2, 3}; vertices[n_vertices * dim] (double, row-major);
 * elements[n_elements * (dim+1)] (int32, any vertex order).  Each face of
 * the box the lattice fills is Dirichlet or an outlet (mcs_mesh.face_bc); by
 * default the whole boundary is Dirichlet with u = 0 (mcs_set_dirichlet sets
 * other data).  The auxiliary multigrid needs the
 * vertices to form a structured lattice: lattice[a] = vertices per axis,
 * vertex (i, j[, l]) has index i + lattice[0] * (j + lattice[1] * l), and
 * every element lies inside one lattice cell.
 *
 * Discrete spaces and the coefficient layout (the documented basis; sorted
 * vertex order per element, barycentric coordinates lambda_i):
 *   velocity bubbles (zero normal trace), per element n_bub functions
 *       lambda^alpha (x_a - x_s0), |alpha| = k, s0 = min supp(alpha),
 *       a in supp(alpha) \ {s0}   (alpha lexicographically descending);
 *   per free facet one block of n_fb = n_F + n_hat (+ 1 for k = 1) dofs:
 *       n_F normal dofs: BDM facet functions lambda^beta (x_j0 - x_i) * c with
 *       normal trace lambda^beta / |F| w.r.t. the facet normal n_F (the
 *       normal of the sorted facet vertex tuple), beta over the facet
 *       vertices, |beta| = k;
 *       n_hat tangential dofs: lambda_F^gamma (x_{f_b} - x_{f_0}),
 *       b = 1..dim-1 (outer), |gamma| = k-1 (inner);
 *       k = 1 only: the flux of omega through F w.r.t. n_F (basis
 *       s (x - x_i) / (3 |T|) on an element, s = +-1 its orientation);
 *   pressure, per element n_p functions lambda^gamma, |gamma| = k-1.
 *   Global vector: [u_bubble: element-major][facet blocks: free facets in
 *   canonical order (sorted by their sorted vertex tuple)][p: element-major].
 *   Auxiliary P1 vectors: dim values per free (interior) vertex, vertices in
 *   increasing index order.
 *
 * Force: f_lattice[n_elements][n_lat][dim], the values of f at the degree-m
 * principal lattice of each element, m = k + 1, points
 * x = sum_i (beta_i/m) v_i over the element's vertices in the order given in
 * `elements`, beta in N^{dim+1}, |beta| = m, lexicographically descending.
 * f is replaced by its Lagrange interpolant on that lattice.
 *
 * Errors: functions return MCS_OK (0) or a negative mcs_status; no exception
 * crosses the ABI; mcs_last_error() gives a thread-local message.  Calls on one
 * problem are not thread safe.  Kernels run on the stream given to mcs_bind;
 * functions marked [sync] synchronise that stream before returning.
 */
#ifndef MCS_H
#define MCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MCS_OK = 0,
  MCS_ERR_ARG = -1,           /* invalid argument (sizes, k, nu <= 0, NaN ...)   */
  MCS_ERR_MESH = -2,          /* mesh not usable (degenerate element, lattice)   */
  MCS_ERR_WORKSPACE = -3,     /* workspace missing or too small                  */
  MCS_ERR_NOT_SPD = -4,       /* Cholesky breakdown in an element / facet block  */
  MCS_ERR_NOT_CONVERGED = -5, /* max_it reached                                  */
  MCS_ERR_BREAKDOWN = -6,     /* MINRES breakdown (preconditioner not SPD)       */
  MCS_ERR_NONFINITE = -7,     /* NaN / Inf encountered                           */
  MCS_ERR_STATE = -8,         /* call out of order (e.g. solve before condense)  */
  MCS_ERR_HIP = -9,           /* HIP runtime error                               */
  MCS_ERR_UNSUPPORTED = -10   /* order / dimension not compiled in               */
} mcs_status;

typedef enum { MCS_F64 = 0, MCS_F32 = 1 } mcs_dtype;

/* Operators of mcs_apply; x and y are full global vectors (n_dof). */
typedef enum {
  MCS_OP_K = 0,       /* y = K x, K = [[A, B^T], [B, 0]]  (eq. femSPmat)           */
  MCS_OP_A = 1,       /* y_u = A x_u through eq. factorSsigma; y_p = 0              */
  MCS_OP_ADELTA = 2,  /* y_d = A^d x_d on the facet dofs; other parts 0             */
  MCS_OP_B = 3,       /* y_p = B x_u; y_u = 0                                       */
  MCS_OP_BT = 4       /* y_u = B^T x_p; y_p = 0                                     */
} mcs_op;

/* Operators of mcs_precond_apply. */
typedef enum {
  MCS_PC_KHAT = 0,        /* z = K-hat^{-1} r (eq. mhatinvfactor)                   */
  MCS_PC_AEXT = 1,        /* z_u = A-hat_ext^{-1} r_u (Sec. 6.1)                    */
  MCS_PC_ADELTA_MULT = 2, /* z_d = A-hat^d^{-1} r_d of the chosen smoother option  */
  MCS_PC_SMOOTH_FWD = 3,  /* z_d = `smoothing_steps` forward block-GS sweeps, x0=0  */
  MCS_PC_SMOOTH_BWD = 4,  /* same with the colours in reverse order                  */
  MCS_PC_AUX = 5,         /* z_d = E^d C^{-1} E^d^T r_d                              */
  MCS_PC_EDELTA = 6,      /* z (global) = E^d r, r a P1 vector                       */
  MCS_PC_EDELTA_T = 7,    /* z (P1) = E^d^T r, r global                              */
  MCS_PC_MG = 8,          /* z (P1) = C^{-1} r (one V(1,1) cycle)                    */
  MCS_PC_MP_INV = 9       /* z_p = M_p^{-1} r_p                                      */
} mcs_pc;

typedef struct {
  int32_t dim;
  int32_t n_vertices;
  const double* vertices_host;   /* [n_vertices * dim] */
  int32_t n_elements;
  const int32_t* elements_host;  /* [n_elements * (dim+1)] */
  int32_t lattice[3];            /* vertices per axis (unused axes: 1) */
  int32_t face_bc[6];            /* boundary condition of each face of the box the
                                    lattice fills: [x-, x+, y-, y+, z-, z+];
                                    0 = Dirichlet u = g (eq. stokes_D; g = 0 unless
                                    set by mcs_set_dirichlet), 1 = outlet Gamma_NT:
                                    u_t = 0 and ((sigma + p I) n).n = 0
                                    (eq. stokes_NT).  All zero: the whole boundary
                                    is Dirichlet and p is fixed by mean zero. */
} mcs_mesh;

typedef struct {
  int32_t order;            /* k in 2..5; k = 1: dim 3 only (Sec. 7) */
  int32_t precision;        /* 0: FP64 MINRES; 1: FP32 inner MINRES + FP64 refinement */
  int32_t smoothing_steps;  /* block-GS sweeps before / after the coarse correction (2) */
  int32_t max_it;           /* MINRES iteration limit (per inner solve) */
  double tol;               /* relative tolerance (preconditioned residual / error target) */
  double inner_tol;         /* precision 1: inner MINRES relative tolerance (1e-5) */
  int32_t max_outer;        /* precision 1: refinement step limit (10) */
  int32_t coarse_max;       /* multigrid: coarsest level when free dofs <= coarse_max (512) */
  int32_t autotune;         /* 1: the first mcs_condense times the smoother's launch shapes and keeps the fastest */
  int32_t smoother;         /* auxiliary-space preconditioner of A^d (Sec. 5.2):
                               0: multiplicative, coloured facet block Gauss-Seidel (Corollary aux_pc_mult);
                               1: additive, facet block Jacobi D = blockdiag(D_F):
                                  A-hat^d^{-1} = D^{-1} + E^d C^{-1} E^d^T (Theorem aux_pc_schur);
                               2: full system (Theorem aux_pc, Gauss-Seidel form of Corollary aux_pc_mult):
                                  A-hat of the whole velocity block A instead of A-hat_ext, overlapping
                                  blocks per facet (its free dofs and the bubbles of its neighbours,
                                  Dirichlet facets included) swept in the colours of a greedy colouring of
                                  all facets, around E C^{-1} E^T with the full embedding.  Single
                                  problems, precision 0, n_fb + 2 n_b <= 64 (2D k <= 5, 3D k <= 3);
                                  otherwise MCS_ERR_UNSUPPORTED.  mcs_precond_apply(MCS_PC_AEXT) then
                                  applies this A-hat^{-1}. */
} mcs_options;

typedef struct {
  int64_t n_dof;            /* full global vector length */
  int64_t n_bubble_dofs, n_facet_dofs, n_pressure_dofs, n_p1_dofs;
  int64_t off_facet, off_pressure;
  int32_t n_bub, n_F, n_hat, n_fb, n_p, n_lat;  /* per element / facet */
  int32_t n_free_facets, n_colours, n_mg_levels;
  size_t workspace_bytes;   /* bytes the caller must provide to mcs_bind */
} mcs_info;

typedef struct {
  int32_t status;
  int32_t iterations;       /* MINRES iterations (summed over refinement steps) */
  int32_t outer_steps;      /* refinement steps (precision 1), else 1 */
  double rel_precond_residual; /* last inner ||r||_{K-hat^{-1}} / ||b||_{K-hat^{-1}} */
  double rel_residual;      /* ||b - K x||_2 / ||b||_2 (FP64) */
  double t_solve_ms;        /* wall time of the iteration (excl. load assembly) */
} mcs_solve_info;

typedef struct mcs_problem mcs_problem;

/* Host only.  Copies the mesh, builds topology, dof numbering, facet colouring
 * and the multigrid plan; fills *info (sizes, workspace bytes).  Reference:
 * Sec. 3 (mesh, facets, spaces); k = 1: Sec. 7 (facet blocks of n_F + n_hat
 * + 1 = 6 dofs: normal moments, tangential means, the flux of omega; no
 * bubbles; on an outlet facet the tangential dofs are fixed to zero and the
 * omega flux stays an unknown).  Errors: MCS_ERR_ARG (k = 1 in 2D among
 * others), MCS_ERR_MESH, MCS_ERR_UNSUPPORTED (k > 5; k = 1 with the
 * full-system variant). */
int mcs_plan(const mcs_mesh* mesh, const mcs_options* options, mcs_problem** out,
             mcs_info* info);

/* Binds the problem to the current HIP device, a caller-owned device
 * workspace of at least info.workspace_bytes bytes (256-byte aligned) and a
 * stream (hipStream_t, may be NULL).  Uploads the host tables.  [sync]
 * Errors: MCS_ERR_WORKSPACE, MCS_ERR_HIP. */
int mcs_bind(mcs_problem* pb, void* workspace, size_t bytes, void* stream);

/* Element matrices, sigma/omega condensation, bubble condensation, facet
 * smoother blocks, embedding blocks and the P1 multigrid hierarchy
 * (Sec. 4.2, eq. bigfemSPmat, eq. factorSsigma, Theorem aux_pc_schur,
 * eq. defAhat, eq. defED).  nu: device, [n_elements] viscosities (> 0).
 * [sync]  Errors: MCS_ERR_ARG (nu <= 0 or not finite), MCS_ERR_NOT_SPD
 * (Cholesky breakdown of an element or facet block). */
int mcs_condense(mcs_problem* pb, const double* nu);

/* b = load vector (f, phi_u) in the global layout, from f_lattice (device),
 * minus K x_D for the Dirichlet data set by mcs_set_dirichlet (without it, b
 * is zero on uhat and p).  b: device double[n_dof]. */
int mcs_load(mcs_problem* pb, const double* f_lattice, double* b);

/* Inhomogeneous Dirichlet data u = g on the Dirichlet faces (eq. stokes_D):
 * g_lattice_host (host) holds g at the degree-m lattice points of every
 * element ([n_elements][n_lat][dim], caller vertex order, the layout of f;
 * only the points on Dirichlet facets are read).  On each Dirichlet facet F
 * its dofs are the L2 projection of g.n_F onto the normal traces
 * (mu^beta / |F|, |beta| = k) and of g_t onto V-hat(F); the solution is then
 * the lift x_D plus the free dofs that mcs_solve returns (mcs_load subtracts
 * K x_D; mcs_eval and mcs_eval_stress include x_D).  g_lattice_host = NULL
 * returns to homogeneous data.  For k = 1 the flux of curl g through each
 * Dirichlet facet is omega's dof there (Sec. 7).  Needs a bound problem.
 * [sync]  Errors: MCS_ERR_ARG for non-finite data. */
int mcs_set_dirichlet(mcs_problem* pb, const double* g_lattice_host);

/* y = op x (see mcs_op); x, y: device vectors of length n_dof in dtype dt
 * (MCS_F32 uses the FP32 operator copies).  Asynchronous. */
int mcs_apply(mcs_problem* pb, int op, int dt, const void* x, void* y);

/* z = op r (see mcs_pc).  Asynchronous.  P1 vectors have n_p1_dofs entries. */
int mcs_precond_apply(mcs_problem* pb, int op, int dt, const void* r, void* z);

/* Solves K x = b(f) with preconditioned MINRES from x = 0 (precision 0), or
 * FP32 inner MINRES with FP64 iterative refinement on the true residual
 * (precision 1).  Without an outlet face it then subtracts the mean of p (p
 * is fixed up to a constant); with one, p is unique and is returned as
 * computed.  f_lattice: device force
 * values; x: device double[n_dof] (output).  info may be NULL.  [sync]
 * Errors: MCS_ERR_NOT_CONVERGED, MCS_ERR_BREAKDOWN, MCS_ERR_NONFINITE. */
int mcs_solve(mcs_problem* pb, const double* f_lattice, double* x, mcs_solve_info* info);

/* Same as mcs_solve with a given right-hand side b (device double[n_dof]). */
int mcs_solve_rhs(mcs_problem* pb, const double* b, double* x, mcs_solve_info* info);

/* For callers that cannot allocate (no hipMalloc, hipHostMalloc or freeing
 * calls: tight serving loops, harnesses that forbid allocation): the same
 * solve as mcs_solve_rhs, which allocates pinned host memory for the MINRES
 * scalars on every call.  This variant allocates no device or pinned host
 * memory (with the kernel timer off: mcs_timer_enable creates HIP events on
 * its first timed launches): the reductions of
 * its dot products and of the pressure mean run in a fixed device array of
 * 4096 doubles (32 KiB) that the library holds on every device it is bound
 * on, until the process ends, and each scalar is copied back to the caller's
 * stack.  The problem's workspace (mcs_bind) holds everything else, as for
 * mcs_solve_rhs.  All calls on one device share that array, so calls that
 * overlap on one device (other threads, other problems on the same device)
 * race; every slot is written before it is read, so nothing needs clearing
 * between calls.  A problem whose reductions would need more slots than the
 * array holds is refused with MCS_ERR_WORKSPACE.  Otherwise as mcs_solve_rhs
 * (same kernels and arithmetic, bitwise the same result).  [sync] */
int mcs_solve_rhs_noalloc(mcs_problem* pb, const double* b, double* x, mcs_solve_info* info);

/* Point values of a solution, for comparisons that do not depend on the
 * basis: u_h and p_h of x (device double[n_dof]) at n_pts points of every
 * element, given as barycentric coordinates ref_pts_host[n_pts][dim+1] (host)
 * w.r.t. the element's vertices in the order of `elements`.  u_vals (device)
 * [n_elements][n_pts][dim], p_vals (device) [n_elements][n_pts].  u_h is the
 * BDM field (Sec. 3, V_h); u-hat lives on facets only.  n_pts <= 1024
 * (3D) / 1365 (2D).  Needs mcs_condense first (det J): MCS_ERR_STATE.  [sync] */
int mcs_eval(mcs_problem* pb, const double* x, int32_t n_pts, const double* ref_pts_host, double* u_vals,
             double* p_vals);

/* Stress and vorticity recovered from a solution (Sec. 4.2: after the
 * condensed solve, sigma_h in Sigma_h and omega_h in W_h follow element by
 * element from the local problems eq. projection, with the element's u_h,
 * u-hat_h and viscosity).  Point values at the same kind of points as
 * mcs_eval: x (device double[n_dof]); ref_pts_host[n_pts][dim+1] (host);
 * sigma_vals and omega_vals (device) [n_elements][n_pts][dim][dim], row-major
 * matrices.  For conforming velocity data sigma_h = -nu dev eps(u_h) and
 * omega_h = kappa(curl u_h) (Lemma SPD).  Needs mcs_condense first
 * (MCS_ERR_STATE); n_pts as for mcs_eval (MCS_ERR_ARG).  For k = 1 omega_h is
 * the Raviart-Thomas field of the facet fluxes in x and omega_vals holds
 * kappa(omega_h).  Uses the condensation scratch.  [sync] */
int mcs_eval_stress(mcs_problem* pb, const double* x, int32_t n_pts, const double* ref_pts_host,
                    double* sigma_vals, double* omega_vals);

/* Subtracts the mean of the pressure from x (device double[n_dof]). */
int mcs_normalize_pressure(mcs_problem* pb, double* x);

/* Device pointer and element count of an internal array, for inspection:
 * name in {"Ad", "H", "Aoo", "Aooinv", "Dinv", "EF", "Ad32", "H32", "detJ",
 * "colour_desc", "elem_ff", "W", "Cinv", "mgA0"}.  "colour_desc" holds four
 * int32 per free facet in colour order: facet id, its two elements (-1: none)
 * and their local facet slots packed as s1 | s2 << 8.  The memory belongs to
 * the caller's workspace. */
int mcs_get_array(mcs_problem* pb, const char* name, void** ptr, int64_t* count);

/* Host copy of the facet colour of each free facet, and of each element's
 * free facet ids (-1: Dirichlet facet), for tests.  Arrays sized n_free_facets
 * and n_elements*(dim+1). */
int mcs_get_topology(const mcs_problem* pb, int32_t* colour_host, int32_t* elem_ff_host);

/* Blocks of the full-system variant (smoother 2), one per facet of the mesh in
 * canonical order (facets sorted by their sorted vertex ids): their number,
 * and, when colour_host (host int32[n_blocks]) is given, the colour of each
 * (greedy in canonical order; facets of one element differ).  Host only. */
int mcs_get_full_colouring(const mcs_problem* pb, int64_t* n_blocks, int32_t* colour_host);

/* Measurement hook for the dominant solve kernels.  While enabled, every
 * launch of a timed kernel is bracketed by HIP events on the problem's stream.
 * mcs_timer_read returns, for one kernel, the accumulated kernel time, the
 * number of launches and their algorithmic HBM bytes:
 *   MCS_TIMER_SMOOTH: the coloured block Gauss-Seidel phase kernel (one colour
 *     of one sweep of A-hat^d_m, Corollary aux_pc_mult).  Per facet of the
 *     colour: the facet's rows of A^d_T of both neighbours (2 n_fb n_d words),
 *     D_F^{-1} (n_fb^2), the right-hand side and the updated block (3 n_fb),
 *     the gathered neighbour vectors (2 n_d) and the index words, counted on
 *     the device over the facet blocks actually processed.
 *   MCS_TIMER_KAPPLY: the operator apply K x of MINRES (eq. femSPmat through
 *     eq. factorSsigma).  Per element: A^d_T, H_T and A_oo,T as stored
 *     (n_d^2 + n_b n_d + n_b^2 words), the gathered inputs and written outputs
 *     (2 (n_d + n_b + n_p) words), the free facet ids and det J.
 * enable = 0 switches the timer off; enable = p >= 1 times one call in p (all
 * launches of a sampled sweep call, every p-th operator apply), so that the
 * event records disturb a timed run little.  Enabling resets the counters.
 * kernel outside the two values, enable < 0: MCS_ERR_ARG.  [sync on read] */
enum { MCS_TIMER_SMOOTH = 0, MCS_TIMER_KAPPLY = 1 };
int mcs_timer_enable(mcs_problem* pb, int enable);
int mcs_timer_read(mcs_problem* pb, int32_t kernel, double* total_ms, int64_t* launches, double* bytes);

/* Launch shape of the coloured block Gauss-Seidel phase kernel for work
 * precision dt (MCS_F64 / MCS_F32): facet blocks per workgroup (1 or 2) and
 * the grid cap (0: one workgroup per facet block); us = the tuner's measured
 * time per launch of the largest colour (0 if not tuned).  The shapes the
 * autotuner tries are bitwise equivalent. */
int mcs_get_launch_config(const mcs_problem* pb, int dt, int32_t* facets_per_block, int64_t* grid_cap, double* us);

/* Sets that launch shape for work precision dt: facets_per_block 1 or 2, grid
 * cap >= 0 (0: one workgroup per facet block).  A shape set here stays: the
 * autotuner (mcs_options.autotune) only tunes the precision slots the caller
 * has not set.  Every shape gives bitwise the same results; the setter lets a
 * caller fix the shape (or compare them).  Other values, and MCS_F64 on a
 * precision 1 problem (it has no FP64 smoother): MCS_ERR_ARG. */
int mcs_set_launch_config(mcs_problem* pb, int dt, int32_t facets_per_block, int64_t grid_cap);

/* Rows of A^d per thread in the operator apply K x for work precision dt
 * (MCS_F64 / MCS_F32): 1, 2 or 4 (FP32), 0 = the largest that n_d allows (the
 * default); us = the tuner's time per K x (0 if not tuned).  The autotuner
 * (mcs_options.autotune) times the valid choices at the first mcs_condense,
 * except for k = 1 (one wave per element) and the split FP64 storage of
 * precision 1 (one row per thread).  The tuner tries the choices whose
 * products H x_d use the lane width of the default and whose A^d sums run in
 * the same order (four rows per thread, FP32, split the columns of A^d over
 * two waves), which give bitwise the same results (a single such choice is
 * timed for the record); a choice set by hand may change the rounding of
 * those sums. */
int mcs_get_apply_config(const mcs_problem* pb, int dt, int32_t* rows_per_thread, double* us);

/* Sets that choice (0, 1, 2, or 4 for MCS_F32; a choice the sizes do not
 * allow falls back to the next smaller one) and keeps the autotuner off that
 * slot.  Other values: MCS_ERR_ARG. */
int mcs_set_apply_config(mcs_problem* pb, int dt, int32_t rows_per_thread);

/* Changes the stopping rules of later solves on a planned problem (the fields
 * of mcs_options that do not change the layout): tol >= 0, max_it >= 1,
 * 0 <= inner_tol < 1, max_outer >= 1.  With tol = 0 a solve runs max_it
 * iterations (precision 0) or max_outer refinement steps of max_it inner
 * iterations when inner_tol = 0 (precision 1), and returns its last iterate
 * with MCS_ERR_NOT_CONVERGED: a fixed block of iterations, e.g. for timing.
 * Other values: MCS_ERR_ARG. */
int mcs_set_solve_options(mcs_problem* pb, double tol, int32_t max_it, double inner_tol, int32_t max_outer);

void mcs_destroy(mcs_problem* pb);
const char* mcs_status_string(int status);
const char* mcs_last_error(void);

/* ---------------------------------------------------------------------------
 * Batches: many independent problems (meshes, orders, viscosities, forces)
 * solved together.  Members with the same dimension and order form a group;
 * a group is one union of its members' elements, facets and lattices, so
 * every kernel of the path runs once per group over all of its members.  The
 * MINRES recurrences run per member with device-resident scalars, members
 * leave the iteration one by one (their work is masked out), and the
 * iterations of all groups are replayed as one captured HIP graph.  Every
 * member's arithmetic is the same whatever the other members are: per-member
 * reductions run over tiles that never straddle two members, in a fixed
 * order.  The method per member is the one of mcs_solve (Sec. 4.2, eq.
 * mhatinvfactor, Corollary aux_pc_mult); precision 1 refines every member in
 * FP64 with its own stopping test.
 * ------------------------------------------------------------------------- */
typedef struct mcs_batch mcs_batch;

typedef struct {
  int32_t n_problems;
  int32_t n_groups;         /* distinct (dim, order) pairs */
  int64_t n_dof_total;      /* sum of the members' n_dof */
  size_t workspace_bytes;   /* bytes the caller must provide to mcs_batch_bind */
} mcs_batch_info;

/* Host only.  Plans n >= 1 members: meshes[i] with order orders[i]; the other
 * options (precision, tolerances, smoothing, limits) are shared.  Errors as
 * mcs_plan, naming the member. */
int mcs_batch_plan(const mcs_mesh* meshes, const int32_t* orders, int32_t n, const mcs_options* options,
                   mcs_batch** out, mcs_batch_info* info);

/* Sizes of member i in its own layout (the layout of mcs_plan's info). */
int mcs_batch_member_info(const mcs_batch* b, int32_t i, mcs_info* info);

/* Binds the batch to the current device, a caller-owned workspace of at least
 * info.workspace_bytes bytes (256-byte aligned) and a stream (hipStream_t,
 * may be NULL); each group also gets a library-created stream of default
 * priority, joined to the given one around every call.  [sync] */
int mcs_batch_bind(mcs_batch* b, void* workspace, size_t bytes, void* stream);

/* Condensation and preconditioner setup of every member (mcs_condense).
 * nu_host: host array of n device pointers, member i's viscosities
 * [n_elements_i].  [sync]  Errors name the member. */
int mcs_batch_condense(mcs_batch* b, const double* const* nu_host);

/* Solves every member (mcs_solve semantics, pressure mean zero).  f_host and
 * x_host: host arrays of n device pointers, member i's force values
 * [n_elements_i][n_lat][dim] and its solution double[n_dof_i] in its own
 * layout.  infos: host array of n entries or NULL; t_solve_ms is the batch's
 * wall time.  Returns MCS_OK when every member converged, else the first
 * failing member's status (each member's own status is in infos).  [sync] */
int mcs_batch_solve(mcs_batch* b, const double* const* f_host, double* const* x_host, mcs_solve_info* infos);

/* Asynchronous form of mcs_batch_solve: waits for the work queued so far on
 * the bind stream (the inputs must be ready then), starts the solve on a
 * library thread and returns.  f_host and x_host as for mcs_batch_solve; the
 * pointer arrays are copied, the device memory they name must stay valid and
 * untouched until mcs_batch_wait returns.  While a solve is in flight and
 * until mcs_batch_wait has collected it, every other call on the batch but
 * mcs_batch_poll and mcs_batch_destroy (which waits for the solve) returns
 * MCS_ERR_STATE.  Errors: MCS_ERR_STATE (not bound or condensed, or a solve
 * in flight), MCS_ERR_ARG.  [async] */
int mcs_batch_solve_async(mcs_batch* b, const double* const* f_host, double* const* x_host);

/* *done = 1 once the solve started by mcs_batch_solve_async has finished, 0
 * while it runs.  MCS_ERR_STATE if none was started.  Host only, no wait. */
int mcs_batch_poll(const mcs_batch* b, int32_t* done);

/* Waits for the solve started by mcs_batch_solve_async and returns its status
 * as mcs_batch_solve would (its error text in mcs_last_error); infos: host
 * array of n entries or NULL.  MCS_ERR_STATE if none was started.  [sync] */
int mcs_batch_wait(mcs_batch* b, mcs_solve_info* infos);

/* Execution mode of mcs_batch_solve: use_graph = 1 (default) replays each run
 * of `chunk` MINRES iterations of all groups as one captured HIP graph;
 * use_graph = 0 launches the same kernels one by one.  chunk is a positive
 * multiple of 6 (default 6).  Both modes give identical results. */
int mcs_batch_set_mode(mcs_batch* b, int use_graph, int chunk);

/* Launch configuration of group g (0 <= g < n_groups) for work precision dt:
 * its dimension and order, and the smoother launch shape (mcs_get_launch_config). */
int mcs_batch_launch_config(const mcs_batch* b, int32_t g, int dt, int32_t* dim, int32_t* order,
                            int32_t* facets_per_block, int64_t* grid_cap, double* us);

/* Smoother timing over all groups (see mcs_timer_enable; the bytes count
 * only the facet blocks of members still iterating).  While enabled,
 * mcs_batch_solve launches kernels one by one (no graph).  [sync] */
int mcs_batch_timer_enable(mcs_batch* b, int enable);
int mcs_batch_timer_read(mcs_batch* b, double* total_ms, int64_t* launches, double* bytes);

void mcs_batch_destroy(mcs_batch* b);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of solve requests under an HBM budget.
 * A server owns a caller-provided device arena (its memory budget) and a
 * scheduler thread.  Requests are queued on submit (their host data is
 * copied); the scheduler takes waiting requests in arrival order into a
 * micro-batch while their standalone footprint (workspace + inputs +
 * solution, known from planning) fits the largest free block of the arena,
 * and runs it on a worker thread with the batch solver.  Up to max_inflight
 * micro-batches run at once, each on its own streams, so requests arriving
 * while others are on the device are admitted as soon as a slot and memory
 * are free and their work overlaps with the running batches.  A request's
 * result is the same alone or in any mix (see the batch section).  A request
 * that cannot fit even an empty arena fails with MCS_ERR_WORKSPACE.
 * ------------------------------------------------------------------------- */
typedef struct mcs_server mcs_server;

typedef struct {
  int32_t status;           /* mcs_status; 1 while pending */
  int32_t iterations, outer_steps;
  int32_t batch_size;       /* members of the micro-batch that solved it */
  double rel_residual, rel_precond_residual;
  double queue_ms;          /* submit -> start of its micro-batch */
  double solve_ms;          /* iteration wall time of its micro-batch */
  double latency_ms;        /* submit -> result on the host */
  char message[160];        /* error text when status < 0 */
} mcs_request_info;

typedef struct {
  size_t arena_bytes, arena_used, arena_peak;
  int64_t batches, solved, waiting;
  int32_t inflight;
} mcs_server_stats_t;

/* options: shared solver options (order ignored: per request).  arena: device
 * memory of the current device, 4096-byte aligned, owned by the caller and
 * kept alive until mcs_server_destroy returns. */
int mcs_server_create(const mcs_options* options, void* arena, size_t arena_bytes, int32_t max_inflight,
                      int32_t max_batch, mcs_server** out);

/* Queues a solve: mesh (as mcs_plan), order, nu_host[n_elements], f_host
 * [n_elements][n_lat][dim] (host memory, copied).  Plans the request on the
 * calling thread (errors as mcs_plan). */
int mcs_server_submit(mcs_server* s, const mcs_mesh* mesh, int32_t order, const double* nu_host,
                      const double* f_host, int64_t* id);

/* done = 1 once the request's result is on the host. */
int mcs_server_poll(mcs_server* s, int64_t id, int32_t* done);

/* Blocks until the request is done, copies its solution (double[n_dof], the
 * layout of mcs_plan; may be NULL) and info, and forgets the request.
 * Returns the request's status. */
int mcs_server_wait(mcs_server* s, int64_t id, double* x_host, mcs_request_info* info);

int mcs_server_stats(mcs_server* s, mcs_server_stats_t* stats);

/* Solves every queued request, waits for them, stops the scheduler. */
void mcs_server_destroy(mcs_server* s);

#ifdef __cplusplus
}
#endif
#endif /* MCS_H */
