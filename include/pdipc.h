/*
 * pdipc.h -- C ABI of the MI355X PD+IPC quasi-static solver.
 *
 * The library solves the actuated soft-body problem of "Efficient Incremental
 * Potential Contact for Actuated Face Simulation" (Li, Yang, Solenthaler,
 * SIGGRAPH Asia 2023 Technical Communications): given an equilibrium x_t and a
 * per-element symmetric actuation A_i, it returns x_{t+1} by Algorithm 1
 * (projective-dynamics local step, IPC constraint set and barrier, global step
 * of Eq. (4) via the Schur complement of Eq. (6)-(8) and the low-rank update
 * of Eq. (9)-(11), CCD step bound, back-tracking line search).
 *
 * Conventions
 *  - All functions are extern "C", never throw, and return int32_t status:
 *    0 = OK, < 0 = error (nothing written), > 0 = warning (result written).
 *  - "device" pointers are HIP device addresses on the solver's device (for
 *    example torch.cuda tensors' data_ptr()); "host" pointers are CPU memory.
 *  - Vertex arrays are n x 3 row-major float64 (x, y, z per vertex).
 *  - Work is ordered on the stream given in pdipc_options.stream (NULL = the
 *    default stream); every call returns after its work has completed.
 *  - A solver handle is not re-entrant: calls on one handle must not overlap.
 *    Different handles are independent.
 *  - The library owns every device buffer it allocates; the caller owns every
 *    buffer it passes in.  Mesh data is copied at pdipc_init_mesh.
 */
#ifndef PDIPC_H
#define PDIPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PDIPC_OK = 0,
  PDIPC_E_INVALID = -1,      /* bad argument, index out of range, NaN input   */
  PDIPC_E_DEGENERATE = -2,   /* a tet with rest volume <= 0                   */
  PDIPC_E_NOT_SPD = -3,      /* PD matrix or reduced contact system not SPD   */
  PDIPC_E_NOMEM = -4,        /* device or host allocation failed              */
  PDIPC_E_INTERSECTING = -5, /* input state has a contact pair at distance 0  */
  PDIPC_E_HIP = -6,          /* a HIP runtime call failed                     */
  PDIPC_W_LS_FAILED = 1,     /* some line search found no decrease (alpha=0)  */
  PDIPC_W_NOT_CONVERGED = 2  /* tolerance mode hit the iteration cap          */
};

enum { PDIPC_FP64 = 0, PDIPC_MIXED_FP32 = 1 };

/* Global step (Table 1 configurations with collision):
 *  PDIPC_GSTEP_SCHUR_WOODBURY  the constant factor, the Schur complement of
 *                              Eq. (6)-(8) and the low-rank update of Eq. (11)
 *                              (the method; default)
 *  PDIPC_GSTEP_PCG             conjugate gradients on (H + kappa B) dx = -g
 *                              preconditioned by the constant factor L L^T = H
 *                              (Eq. 5, the paper's baseline); FP64 only
 *  PDIPC_GSTEP_SCHUR           the Schur complement alone (Section 3.1): the
 *                              dense Sigma + B_22 (3 n2 unknowns) factored every
 *                              iteration; FP64 only
 * All three solve the same system; they differ in cost. */
enum { PDIPC_GSTEP_SCHUR_WOODBURY = 0, PDIPC_GSTEP_PCG = 1, PDIPC_GSTEP_SCHUR = 2 };

/*
 * Mesh description (Section 2 of the paper: tetrahedral simulation mesh,
 * embedded collision proxy s = W x of Section 3.1, manually marked collision
 * region x2 of Eq. 6).  All pointers are host memory and are only read during
 * pdipc_init_mesh; the library copies what it keeps.
 *  rest_pos    n_verts x 3   rest positions X [m]
 *  tets        n_tets x 4    vertex ids; every tet must have det[X1-X0,
 *                            X2-X0, X3-X0] > 0 (else PDIPC_E_DEGENERATE)
 *  dirichlet   n_verts       1 = vertex fixed at its rest position; at least
 *                            one is needed (else PDIPC_E_NOT_SPD: the PD
 *                            matrix of Eq. 2 would be singular)
 *  n_surf_verts, W_rowptr, W_col, W_val
 *                            the proxy vertices s = W x as a CSR matrix of
 *                            n_surf_verts rows over the n_verts simulation
 *                            vertices (W_rowptr: n_surf_verts + 1 entries,
 *                            W_col: column ids, W_val: weights, NULL = every
 *                            row has one entry of weight 1).  Rows must have
 *                            non-negative weights that sum to 1 within 1e-12,
 *                            distinct columns and at most 4 entries (else
 *                            PDIPC_E_INVALID).  Rows may interpolate (a proxy
 *                            finer than the simulation surface): the contact
 *                            terms then live on s = W x, and the barrier
 *                            gradient and Hessian reach x as W^T grad and
 *                            W^T H W.  The adjoint (pdipc_solve_frame_backward)
 *                            supports a selection only (every row one weight
 *                            of 1).  W_rowptr = NULL: no W; surf_tris then
 *                            holds simulation vertex ids directly.
 *  n_surf_tris, surf_tris    proxy triangles, n_surf_tris x 3 ids of proxy
 *                            vertices (rows of W), or of simulation vertices
 *                            when W_rowptr is NULL
 *  region      n_verts or NULL  1 = collision-aware vertex (block x2 of Eq. 6);
 *                            NULL = the free simulation vertices the proxy
 *                            moves with (the columns W uses).  Every such
 *                            vertex must be marked (else PDIPC_E_INVALID).
 *  youngs, poisson           element weight w_i = 2 mu V_i, mu = E/(2(1+nu))
 */
typedef struct {
  int32_t n_verts, n_tets;
  const double* rest_pos;
  const int32_t* tets;
  const uint8_t* dirichlet;
  int32_t n_surf_tris;
  const int32_t* surf_tris;
  const uint8_t* region;
  double youngs, poisson;
  int32_t n_surf_verts;
  const int32_t* W_rowptr;
  const int32_t* W_col;
  const double* W_val;
} pdipc_mesh_desc;

/*
 * Solver options.
 *  dhat, kappa     barrier threshold d_0 and stiffness (Eq. 3)
 *  iters           iterations per frame (fixed mode) or cap (tolerance mode)
 *  tol             > 0: stop when max |alpha dx| <= tol; <= 0: fixed iters
 *  precision       PDIPC_FP64 or PDIPC_MIXED_FP32 (FP32 local/barrier passes and,
 *                  from fp32_reduced_min unknowns on, an FP32 factor of the
 *                  reduced system refined against FP64 residuals)
 *  ccd_eta         CCD target gap as a fraction of the current distance
 *  ccd_steps       conservative-advancement steps per pair
 *  ls_max_halvings line-search halvings before giving up (alpha = 0)
 *  cinv_updates_max  when at most 32 vertices leave and 32 enter the contact
 *                  set, C^-1 is updated in place of rebuilt, up to this many
 *                  times in a row (0 = always rebuild)
 *  hinv_rows_mb    device memory (MiB) allowed for the rows x2 of H_s^-1
 *                  (n2 x (n1 + n2) FP64, built at init with one backward sweep
 *                  per three rows).  With them the contact correction of the
 *                  global step is one product over all rows, and the backward
 *                  sweep runs on the uncorrected step while the reduced system
 *                  is factored; 0 = off (correct x2, then sweep)
 *  fp32_reduced_min  mixed precision: smallest reduced system (3 n_c unknowns)
 *                  solved with the refined FP32 factor (default 8192); smaller
 *                  ones use the FP64 factor.  Up to a few thousand unknowns
 *                  the factorisation is bound by its sequence of block steps,
 *                  not by arithmetic, so the FP32 factor saves little there
 *                  and its refinement (and FP64 refactorisation when FP32
 *                  breaks down) costs more
 *  stream          hipStream_t to order work on (NULL = default stream)
 *  global_method   PDIPC_GSTEP_* (above)
 *  cg_tol, cg_max_iters  PDIPC_GSTEP_PCG: stop when |r| <= cg_tol |g| over the
 *                  free DOFs, or after cg_max_iters products
 *  barrier_form    0: IPC's b(d) = -(d - dhat)^2 ln(d / dhat) on the distance
 *                  d (Eq. 3 as read); 1: the same function of the squared
 *                  distance d^2 with threshold dhat^2.  Both select the same
 *                  pairs (d < dhat)
 *  kappa_adapt     0: kappa fixed; 1: IPC-style adaptive stiffness (Section 4
 *                  mentions it): at the start of a frame with pairs, kappa =
 *                  -(g_E . g_b) / (g_b . g_b) clamped to [kappa, 100 kappa] (g_E
 *                  the elastic gradient, g_b that of the unit barrier); later,
 *                  kappa doubles (up to 100 kappa) at an iteration whose
 *                  smallest squared pair distance is below 1e-9 l^2 (l: rest
 *                  bounding-box diagonal) and below the previous iteration's.
 *                  The adjoint uses the last iteration's kappa.
 */
typedef struct {
  double dhat, kappa;
  int32_t iters;
  double tol;
  int32_t precision;
  double ccd_eta;
  int32_t ccd_steps, ls_max_halvings, cinv_updates_max, fp32_reduced_min, hinv_rows_mb;
  void* stream;
  int32_t global_method;
  double cg_tol;
  int32_t cg_max_iters;
  int32_t barrier_form, kappa_adapt;
} pdipc_options;

/* Per-frame statistics (host).  Stage times follow the paper's Table 1
 * columns, measured with HIP events at the stage boundaries of every
 * iteration on the solver's stream (the reduced system's second stream is
 * inside G-Step, which waits for it): IPC (constraint set, barrier
 * derivatives and their incidence), Misc (local step, gradient assembly, and
 * the frame's own copies and checks), G-Step (global solve), CCD (swept
 * candidates and the step bound), LS (line search and update).
 * near_ties: candidates whose distance was within 1e-10 dhat of dhat when the
 * constraint set was formed (membership there can follow rounding).
 * refine_steps / refine_fallbacks: mixed-precision refinement solves and the
 * iterations whose reduced system fell back to the FP64 factor.
 * cinv_rebuilds: iterations whose contact set c differed from the previous
 * one (C^-1 recomputed); c_delta_max / c_delta_sum: vertices that entered or
 * left c at those iterations (largest, total); cinv_updates: those of them
 * served by the incremental update of C^-1.  pcg_iters: products of the
 * conjugate-gradient global step over the frame (PDIPC_GSTEP_PCG). */
typedef struct {
  int32_t iters, n_pt, n_ee, n_c, ls_halvings, ls_failures, refine_steps;
  int32_t n_candidates, refine_fallbacks, cinv_rebuilds, c_delta_max, c_delta_sum, cinv_updates;
  int32_t near_ties, pcg_iters;
  double alpha_m_min, alpha_min, energy, grad_inf;
  double ms_ipc, ms_gstep, ms_ccd, ms_ls, ms_misc, ms_total;
} pdipc_frame_stats;

/* Fill *opt with defaults: dhat 5e-4, kappa 1e3, 30 iters, fixed mode, FP64,
 * eta 0.1, 16 CCD steps, 20 halvings, default stream, the Schur-complement and
 * low-rank-update global step (CG: tolerance 1e-12, at most 2000 products),
 * barrier form 0, fixed kappa. */
void pdipc_default_options(pdipc_options* opt);

/* Build a solver: validate the mesh, precompute per-tet data, assemble the
 * constant PD matrix H of Eq. (2), order the x1 block by nested dissection,
 * factor H11 = L1 L1^T (Section 3.1) and form the inverse Schur complement
 * Sigma^-1 (Section 3.2).  On success *out owns all device state. */
int32_t pdipc_init_mesh(const pdipc_mesh_desc* mesh, const pdipc_options* opt, void** out);

/* Set per-element actuation A_i (Eq. 1) from its 6 symmetric entries.
 * A: device, n_tets x 6 float64, (xx, yy, zz, xy, yz, zx) per tet. */
int32_t pdipc_set_actuation(void* solver, const double* A);

/* Set A_i = R_i diag(1 - a_i, 1 + a_i/2, 1 + a_i/2) R_i^T.
 * a: device n_tets float64; R: device n_tets x 9 float64 row-major, or NULL
 * to keep the frames from the previous call.  The backward pass
 * differentiates with respect to a. */
int32_t pdipc_set_actuation_scalar(void* solver, const double* a, const double* R);

/* One frame of Algorithm 1: x_out = x_{t+1} from x_in = x_t.
 * x_in, x_out: device n_verts x 3 float64 (may alias).  Fixed vertices are
 * taken from x_in.  stats: host, may be NULL.
 * Errors: PDIPC_E_INTERSECTING if x_in has a pair at distance 0;
 * PDIPC_E_NOT_SPD if the reduced system fails to factor. */
int32_t pdipc_solve_frame(void* solver, const double* x_in, double* x_out, pdipc_frame_stats* stats);

/* Adjoint of the last converged frame with respect to the per-tet actuation
 * scalars (set through pdipc_set_actuation_scalar): given dL/dx* (device,
 * n_verts x 3), writes dL/da (device, n_tets).  Solves K lambda = dL/dx* with
 * K the Hessian of the total energy at x* (Eq. 1 and Eq. 3 terms). */
int32_t pdipc_solve_frame_backward(void* solver, const double* dL_dx, double* dL_da);

/* Device memory currently held by the solver, in bytes (host out). */
int32_t pdipc_device_bytes(const void* solver, int64_t* bytes);

/* Sizes of the blocks after init: n1, n2 of Eq. (6) and nnz of the factor. */
int32_t pdipc_get_sizes(const void* solver, int64_t* n1, int64_t* n2, int64_t* factor_nnz);

/* Release everything the solver owns. NULL is allowed. */
void pdipc_destroy(void* solver);

/* Last error message of a handle (or, for NULL, of the last failed
 * pdipc_init_mesh or pdipc_dense_spd_noalloc call of this thread). */
const char* pdipc_last_error(const void* solver);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call the allocator): the dense SPD
 * factorisation, solve and inverse of the reduced contact system, on caller
 * data, with no allocation of any kind.  Every work buffer lives in one
 * file-scope device array of the library (about 26 MB per device, held until
 * the process ends), which limits the order to n <= 1024.
 *  A       device, n x n float64 row-major, symmetric positive definite
 *          (lower triangle read); not modified
 *  b       device, n x nrhs float64 row-major, solved in place (A x = b);
 *          may be NULL when nrhs = 0.  0 <= nrhs <= 4
 *  Ainv    device, n x n float64, receives A^-1 (full); may be NULL
 *  precision  PDIPC_FP64, or PDIPC_MIXED_FP32 (factor, solve and inverse in
 *          FP32 on a rounded copy; results widened to float64)
 *  info    device int32 (caller-owned): 0, or 1 + the first column whose
 *          pivot was not positive (the outputs are then not meaningful)
 *  stream  hipStream_t the work is queued on (NULL = default stream)
 * The call only queues work: it returns without waiting, and info is valid
 * once the stream has reached it.  All calls on one device share the array,
 * which keeps the last call's contents: calls that overlap on one device (on
 * different streams or host threads) race and must be serialised by the
 * caller.  Errors: PDIPC_E_INVALID for n < 1 or n > 1024, a bad nrhs,
 * precision or NULL pointer (nothing queued); PDIPC_E_HIP when the array's
 * address or a launch fails.  Same results as pdipc_debug_dense.
 */
int32_t pdipc_dense_spd_noalloc(const double* A, int64_t n, double* b, int32_t nrhs, double* Ainv,
                                int32_t precision, int32_t* info, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PDIPC_H */
