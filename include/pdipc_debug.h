/*
 * pdipc_debug.h -- parity and measurement taps of the PD+IPC solver library.
 *
 * These entry points exist for tests and benchmarks: they expose intermediate
 * results of one iteration of Algorithm 1 (local step, constraint set, global
 * step), per-iteration traces, kernel timers and the dense SPD kernels on
 * caller data.  A user of the method needs only pdipc.h.  Conventions (status
 * codes, device and host pointers, streams) are those of pdipc.h.
 */
#ifndef PDIPC_DEBUG_H
#define PDIPC_DEBUG_H

#include "pdipc.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One iteration of the last pdipc_solve_frame call (Algorithm 1 loop body):
 * pair counts of the constraint set, affected vertices n_c (Eq. 9), swept
 * candidates of the CCD step, line-search halvings and outcome, near ties of
 * the constraint set, refinement solves of the reduced system, and the step
 * bound alpha_m and accepted step alpha; cg_iters: products of the conjugate-gradient
 * global step (PDIPC_GSTEP_PCG); kappa: the barrier stiffness of the
 * iteration. */
typedef struct {
  int32_t n_pt, n_ee, n_c, n_candidates, ls_halvings, ls_ok, near_ties, refine_steps, cg_iters;
  double alpha_m, alpha, kappa;
} pdipc_iter_trace;

/* Copy up to cap iteration records of the last frame into out (host); the
 * number of iterations of that frame is written to *count (host). */
int32_t pdipc_debug_trace(const void* solver, pdipc_iter_trace* out, int32_t cap, int32_t* count);

/* Measurement tap: read and reset the HIP-event timer, then arm it for the
 * kernel family `which` (-1 = off): 0 local step, 1 Sigma^-1 GEMV, 2 lower
 * sweep, 3 upper sweep, 4 barrier, 5 line-search energies, 6 reduced
 * Cholesky, 8 CCD, 9 incremental C^-1 update, 10 full C^-1
 * rebuild (Cholesky and inverse of the contact block).  Events are recorded on the solver's stream around every
 * launch of that family during pdipc_solve_frame; *total_ms and *launches
 * (host, nullable) return what was accumulated since the previous call. */
int32_t pdipc_kernel_timer(void* solver, int32_t which, double* total_ms, int64_t* launches);


/* ---- debug / parity taps (device pointers, sizes from pdipc_get_sizes) ----
 * pdipc_debug_local: run only the local step at x (device n x 3): writes
 *   R (device m x 9 row-major) and element energies (device m), and the PD
 *   gradient sum_i w_i G_i^T (G_i x - p_i) (device n x 3, zero at fixed).
 * pdipc_debug_contacts: constraint set at x: writes up to cap pairs as
 *   (type, i, j) int32 triples into pairs (device), returns the count in
 *   *count (host).  type 0 = point-triangle (proxy vertex, proxy triangle),
 *   type 1 = edge-edge (edge, edge) with edges sorted (lo, hi).  Proxy
 *   vertices are simulation vertex ids for a proxy embedded by selection,
 *   else rows of W.
 * pdipc_debug_step: one full iteration from x; writes dx (device n x 3) and
 *   the host scalars alpha_m, alpha. */
int32_t pdipc_debug_local(void* solver, const double* x, double* R, double* energies, double* grad);
int32_t pdipc_debug_contacts(void* solver, const double* x, int32_t* pairs, int32_t cap, int32_t* count);
int32_t pdipc_debug_step(void* solver, const double* x, double* dx, double* alpha_m, double* alpha);

/* Dense SPD kernels on caller data (test tap, default stream): factor the
 * device matrix A (n x n row-major, symmetric positive definite; not
 * modified), solve A x = b in place for b (device n x nrhs, nrhs <= 4, may
 * be NULL) and write A^-1 to Ainv (device n x n, may be NULL).  precision 1
 * runs the FP32 kernels on a rounded copy.  PDIPC_E_NOT_SPD on a non-positive
 * pivot. */
int32_t pdipc_debug_dense(const double* A, int64_t n, double* b, int32_t nrhs, double* Ainv, int32_t precision);

/* Host-only check of the set-up factorization (no device work, usable
 * without a GPU).  Input: the scalar PD matrix over free vertices in
 * extended order (x1 block [0, n1) with coordinates coords1 (n1 x 3), then
 * x2 block) as full-pattern CSR (ptr: n1 + n2 + 1 int64, col int32, val);
 * leaf = nested-dissection leaf size.  Solves H x = b (host vectors of
 * n1 + n2) through the supernodal factor and a dense host Cholesky of the
 * Schur complement, writes Sigma_s (n2 x n2 row-major, host) and the factor
 * size.  b/x/sigma_out/nnz_out may be NULL to skip. */
int32_t pdipc_debug_host_factor(int32_t n1, int32_t n2, const double* coords1, const int64_t* ptr,
                                const int32_t* col, const double* val, int32_t leaf, const double* b, double* x,
                                double* sigma_out, int64_t* nnz_out);


#ifdef __cplusplus
}
#endif
#endif /* PDIPC_DEBUG_H */
