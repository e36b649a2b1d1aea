// Launchers of the gfx950 kernels.  All pointers are device memory unless a
// name says host; every launcher enqueues on the given stream and returns.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace pdipc {

// ---------------------------------------------------------------- local step
struct LocalArgs {
  int64_t m;
  const int32_t* tets;  // 4 x m
  const double* B;      // 9 x m
  const double* w;      // m
  const double* A;      // 6 x m
};
// Rwarm (optional, may alias Rout): rotations at a nearby state to start from;
// tetg: per-tet gradient shares, m x 12 (entry 3a + r: local vertex a, coordinate r)
// ev_start / ev_stop (optional): events stamped at the kernel's start and end
void launch_local_step(const LocalArgs& la, const double* x, const double* Rwarm, double* Rout, double* energy,
                       double* tetg, bool fp32, hipStream_t st, hipEvent_t ev_start = nullptr,
                       hipEvent_t ev_stop = nullptr);
void launch_identity_rotations(int64_t m, double* R, hipStream_t st);
void launch_trial_energy(const LocalArgs& la, const double* x, const double* dx, const double* ls, const double* Rwarm,
                         const double* E0, double* dE, bool fp32, hipStream_t st);
void launch_gather_vertex_grad(int32_t n, int64_t m, const int32_t* vt_ptr, const int32_t* vt_ent,
                               const double* tetg, const uint8_t* fixed, double* g, hipStream_t st);
void launch_actuation_scalar(int64_t m, const double* a, const double* R, double* A, hipStream_t st);
void launch_actuation_transpose(int64_t m, const double* Ain, double* A, hipStream_t st);

// ------------------------------------------------------------------- utility
// exclusive scan of n int32 into out (out may alias in); total -> *d_total.
// A job may also write a copy of the output and hand over the scanned value
// at index pick; two jobs share one pair of launches (temp sized by
// scan_temp_bytes of the larger n).
struct ScanJob {
  const int32_t* in;
  int32_t* out;
  int64_t n;
  int32_t* d_total;
  int32_t* copy;       // optional second output
  int64_t pick;        // index whose scanned value goes to *pick_out (optional)
  int32_t* pick_out;
};
struct ScanJobs {
  ScanJob j[2];
  int64_t nb0;         // tiles of the first job
};
size_t scan_temp_bytes(int64_t n);
void launch_exclusive_scans(const ScanJob* jobs, int njobs, void* temp, hipStream_t st);
void launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* d_total, void* temp,
                           hipStream_t st);
// deterministic sum of n doubles into *d_out (fixed blocked order)
size_t sum_temp_bytes(int64_t n);
void launch_sum(const double* in, int64_t n, double* d_out, void* temp, hipStream_t st);
void launch_sum2(const double* a, int64_t na, const double* b, int64_t nb, double* d_out, void* temp,
                 hipStream_t st, const double* ls = nullptr);
// Device line-search state: a few doubles, indexed as below.  Trial kernels
// read alpha from it and do nothing once the state is decided (1 accepted,
// -1 failed), so several trials can be queued without reading anything back.
enum { LS_ALPHA = 0, LS_STATE = 1, LS_HALVINGS = 2, LS_ALPHA_M = 3, LS_DE = 4, LS_SIZE = 8 };
// alpha_m = min(1, the CCD blocks' minima); starts the search
void launch_ls_init(double* ls, const double* part, int nparts, hipStream_t st);
// dE of a trial = the deterministic sum of a (elements) and b (pairs), as
// launch_sum2; then accept / halve / give up
void launch_sum2_decide(const double* a, int64_t na, const double* b, int64_t nb, double* ls, void* temp,
                        int32_t max_halvings, hipStream_t st);
void launch_axpy_ls(int64_t n3, const double* ls, const double* dx, double* x, hipStream_t st);
// min of n doubles (>= 0 entries) into *d_out, 1.0 if n == 0 (exact: min is order-free)
void launch_min_clamp1(const double* in, int64_t n, double* d_out, void* temp, hipStream_t st);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st);
// two int32 arrays filled with v in one launch
void launch_fill2_i32(int32_t* a, int64_t na, int32_t* b, int64_t nb, int32_t v, hipStream_t st);
void launch_fill_f64(double* p, int64_t n, double v, hipStream_t st);
void launch_axpy_positions(int64_t n3, double alpha, const double* dx, double* x, hipStream_t st);
void launch_max_abs(const double* in, int64_t n, double* d_out, void* temp, hipStream_t st);
// number of non-finite entries -> *d_out
void launch_count_nonfinite(const double* x, int64_t n, int32_t* d_out, hipStream_t st);
// ------------------------------------------------------------------- contact
struct ProxyDev {
  int32_t nsv, nst, nse;
  const int32_t* sv;    // nsv sim ids, ascending
  const int32_t* st;    // 3 x nst (AoS triples of sim ids)
  const int32_t* se;    // 2 x nse (AoS (lo, hi) sim ids), sorted
};

// Partners a query keeps from its counting pass; the broad phase walks the
// grid a second time only when some query has more.
constexpr int32_t kQueryKeep = 64;
struct BroadPhaseBuffers {
  // boxes: 6 doubles per primitive (lo xyz, hi xyz)
  double* vbox;         // nsv
  double* tbox;         // nst
  double* ebox;         // nse
  double* params;       // [0..2] origin, [3] cell size, [4..] scratch
  int32_t table_bits;   // table size = 1 << bits
  int32_t* t_count;     // triangle table: table + 1
  int32_t* t_cursor;
  int32_t* t_id;        // entries
  uint64_t* t_key;
  int32_t* e_count;
  int32_t* e_cursor;
  int32_t* e_id;
  uint64_t* e_key;
  int64_t ent_cap;      // capacity of each entry array
  int32_t* q_count;     // nsv + nse + 1 per-query counts / offsets
  int32_t* qbuf;        // (nsv + nse) x kQueryKeep: each query's first partners, in discovery order
  int32_t* tmpj;        // unsorted partner ids (queries with more than kQueryKeep partners)
  int64_t tmp_cap;
  int32_t* d_totals;    // [0] pairs total, [7] largest partner count above kQueryKeep (else 0)
  int32_t* h_totals;    // pinned host copy of d_totals (4 entries)
  void* scan_temp;
  void* red_temp;
};

// Candidate (swept == true: boxes over x and x + dx) or constraint-set pairs.
// Pairs are written sorted: point-triangle (query = proxy vertex, ascending
// sim id, then triangle id), then edge-edge (e < e').  Returns via host the
// two counts (point-triangle, edge-edge) after a synchronising read.
struct PairList {
  int32_t* type;        // 0 = PT, 1 = EE
  int32_t* i;           // PT: sim vertex id; EE: edge id
  int32_t* j;           // PT: triangle id;  EE: edge id (> i)
  int32_t* v4;          // 4 sim ids per pair in local order
  int64_t cap;
};
int find_pairs(const ProxyDev& px, const BroadPhaseBuffers& bb, const double* x, const double* dx, double dhat,
               bool distance_filter, PairList& out, int32_t* n_pt, int32_t* n_ee, hipStream_t st,
               int64_t* needed);

// Constraint set at x as the pairs of a (sorted) candidate list with squared
// distance below dhat^2; order preserved.  flag, pos: ncand + 1 ints.
// h_tot: pinned host memory for the two counts read back
int filter_active(const PairList& cand, int32_t ncand, int32_t cand_pt, const double* x, double dhat, PairList& out,
                  int32_t* flag, int32_t* pos, int32_t* d_tot, int32_t* h_tot, void* scan_temp, int32_t* n_pt,
                  int32_t* n_ee, hipStream_t st, int64_t* needed, int32_t* near_ties);

// CCD: t_k per candidate pair (conservative advancement), then alpha_m.
// per-candidate bounds t_out and per-block minima part; returns the blocks.
// With e0, also each candidate's barrier energy at x (kappa b, 0 beyond dhat;
// barrier form as barrier_of_D).
int launch_ccd(const PairList& pl, int32_t npairs, int32_t n_pt, const double* x, const double* dx, double eta,
               int32_t steps, double* t_out, double* part, hipStream_t st, double dhat = 0.0, double kappa = 0.0,
               int form = 0, double* e0 = nullptr);
// kappa * b per candidate at x + alpha dx (alpha = 0 allowed); pairs at
// d >= dhat give 0.
void launch_pair_barrier_energy(const PairList& pl, int32_t npairs, int32_t n_pt, const double* x, const double* dx,
                                const double* ls, double dhat, double kappa, int form, const double* E0, double* out,
                                hipStream_t st);
// smallest pair distance (for the intersection check); -> d_out
void launch_pair_min_dist2(const PairList& pl, int32_t npairs, int32_t n_pt, const double* x, double* d2_out,
                           hipStream_t st);

// ------------------------------------------------------------------- barrier
// Per active pair: energy, gradient (12), PSD Hessian factor U (12 x 5, row
// r = 3 * local point + coord), so that the projected Hessian is U U^T.
struct BarrierOut {
  double* energy;       // npairs
  double* grad;         // 12 x npairs (SoA)
  double* U;            // 60 x npairs (SoA, entry 5 r + k)
};
void launch_barrier(const PairList& pl, int32_t npairs, int32_t n_pt, const double* x, double dhat, double kappa,
                    int form, bool fp32, BarrierOut& bo, hipStream_t st);

// Per-pair terms over simulation vertices ("slots"): S slots per pair, the
// simulation vertex of each (v: S x npairs, -1 = unused), the barrier gradient
// rows (grad: 3 S x npairs SoA, row 3 slot + coordinate) and the rows of the
// PSD factor (U: 15 S x npairs SoA, entry 5 (3 slot + coordinate) + column).
// With the proxy embedded by selection these are the barrier outputs
// themselves (S = 4, v = the pair's four vertices); with an interpolating
// embedding s = W x they are W^T applied to them (S = 16: the distinct
// simulation vertices of the pair's four proxy points).
struct PairSlots {
  int32_t S;
  const int32_t* v;
  const double* grad;
  const double* U;
};

// Proxy embedding s = W x (CSR over the proxy vertices, at most 4 entries
// per row).
struct EmbedDev {
  int32_t ns;
  const int32_t* ptr;
  const int32_t* col;
  const double* val;
};
// s (ns x 3) = W x
void launch_embed_positions(const EmbedDev& W, const double* x, double* s, hipStream_t st);
// Slots of every pair (S = 16): each proxy point's W entries, merged per
// simulation vertex in the order they occur; grad and U rows weighted.
void launch_expand_pairs(const EmbedDev& W, const int32_t* v4, int32_t npairs, const BarrierOut& bo,
                         int32_t* slot_v, double* slot_grad, double* slot_U, hipStream_t st);

// vertex -> (pair, slot) incidence (sorted), per-vertex gradient add,
// affected-set map.  inc_ptr: n + 1, inc_ent: S * npairs (entry S k + slot).
struct Incidence {
  int32_t* cnt;         // n + 1
  int32_t* ptr;         // n + 1
  int32_t* cursor;      // n
  int32_t* raw;         // 4 * cap pairs, unsorted fill
  int32_t* ent;         // 4 * cap pairs, sorted per vertex
  int32_t* cflag;       // n + 1: 1 if free and touched
  int32_t* cidx;        // n + 1: exclusive scan of cflag (c index if flagged)
  int32_t* clist;       // n: c index -> sim vertex
  int32_t* d_nc;        // 5: n_c, then the change of c (any, left, entered), then the entry total
  const int32_t* verts; // the simulation vertices that slots can name, ascending
  int32_t nverts;
};
// Incidence lists, contact flags, ranks and list of c.  With prev_cflag (the
// flags of an earlier c, n + 1 entries), d_nc[1..3] also receive the change
// of c (any flag differs, vertices that left, vertices that entered) and, with
// ids, up to cap of the leaving / entering vertices go to rem_ids / add_ids.
void build_incidence(const PairSlots& ps, int32_t npairs, int32_t n, const uint8_t* fixed, Incidence& inc,
                     void* scan_temp, hipStream_t st, const int32_t* prev_cflag = nullptr,
                     int32_t* rem_ids = nullptr, int32_t* add_ids = nullptr, int32_t cap = 0);
void launch_add_barrier_grad(const Incidence& inc, const PairSlots& ps, int32_t npairs, const uint8_t* fixed,
                             double* g, hipStream_t st);

// ---------------------------------------------------------- global (Eq. 7)
struct FactorDev {
  int32_t n1, n2, nnodes, nlevels;
  const int32_t* node_c0;
  const int32_t* node_s;
  const int32_t* node_r;
  const int64_t* node_rows_off;
  const int64_t* node_panel_off;
  const int64_t* node_dinv_off;
  const int32_t* level_nodes;      // node ids grouped by level
  const int32_t* h_level_ptr;      // HOST: nlevels + 1
  const int32_t* h_level_maxs;     // HOST: max s in each level
  const int32_t* h_level_maxr;     // HOST: max r in each level
  const int32_t* h_lvl_row_ptr;    // HOST: nlevels + 1 offsets into lvl_rows
  const int32_t* lvl_rows;         // extended index of every x1 column, by level
  const int32_t* lvl_row_node;     // its supernode
  const int32_t* rows;
  const double* panelT;            // s x r row-major per node: L[R(J), cols(J)]^T
  const double* dinv;              // s x s row-major per node
  const double* dinvT;             // s x s row-major per node of Dinv^T
  const int64_t* fwd_ptr;          // n1 + n2 + 1
  const int32_t* fwd_col;
  const double* fwd_val;
  const double* sigma_inv;         // n2 x n2 row-major
  const double* hinv_x2;           // n2 x (n1 + n2) row-major: rows x2 of H_s^-1 (extended order), or null
  const int32_t* ext2vert;         // n1 + n2: sim vertex of each extended index
};
// b (ext, 3) = -g at ext2vert
void launch_pack_rhs(const FactorDev& f, const double* g, double* b, hipStream_t st);
// W_J = L[R(J), cols(J)] Dinv_J per supernode, in the panel layout (init)
void launch_panel_times_dinv(int32_t nnodes, const int32_t* node_s, const int32_t* node_r, const int64_t* poff,
                             const int64_t* doff, const double* P, const double* D, double* W, hipStream_t st);
// forward sweep: y (ext, 3); rows of x2 get r2 - L21 y1 (no diagonal solve).
// The sweeps read W (f.fwd_val by rows, f.panelT transposed) in place of the
// panels; levels carry t, and the diagonal blocks go in one launch.
// (levels [level_begin, level_end) of the x1 sweep; level_end < 0: to the end,
// then the x2 rows)
void launch_forward_sweep(const FactorDev& f, const double* b, double* y, hipStream_t st, int level_begin = 0,
                          int level_end = -1);
// z = Sigma^-1 r (n2 x 3)
void launch_sigma_gemv(const FactorDev& f, const double* r, double* z, hipStream_t st);
// backward sweep: sol[0, n1) from y and sol[n1, n1 + n2) (already set)
void launch_backward_sweep(const FactorDev& f, const double* y, double* sol, hipStream_t st);
// dx (n x 3) from sol (ext) at the free vertices; the fixed vertices' entries
// are not written (the caller keeps them zero)
void launch_unpack(const FactorDev& f, int32_t n, const double* sol, double* dx, hipStream_t st);
// Rows [j0, j1) of the extended order only.
void launch_unpack_range(const FactorDev& f, int32_t j0, int32_t j1, const double* sol, double* dx, hipStream_t st);

// ------------------------------------------------- reduced contact system
// C_s = Sigma^-1[c, c] (nc x nc), using x2 index of each c vertex
void launch_gather_cc(const FactorDev& f, int32_t nc, const int32_t* c_x2, double* Cs, hipStream_t st);
// M = Cinv (x) I3 + sum_k U_k U_k^T blocks (3nc x 3nc row-major, full)
void launch_assemble_reduced(int32_t nc, const double* Cinv, const Incidence& inc, const PairSlots& ps,
                             int32_t npairs, double* M, hipStream_t st);
// out (nc x 3) = (Cinv (x) I3) z_c, z_c gathered from z (n2 x 3) by c_x2
void launch_cinv_times_zc(int32_t nc, const double* Cinv, const int32_t* c_x2, const double* z, double* out,
                          hipStream_t st);
// v (nc x 3) = Bcheck u
void launch_bcheck_apply(int32_t nc, const Incidence& inc, const PairSlots& ps, int32_t npairs, const uint8_t* fixed,
                         const double* u, double* wtmp, double* v, hipStream_t st);
// z -= Sigma^-1[:, c] v   (n2 x 3)
void launch_sigma_cols_update(const FactorDev& f, int32_t nc, const int32_t* c_x2, const double* v, double* z,
                              hipStream_t st);
// sol -= H_s^-1[:, c] v over all n1 + n2 extended rows (3 RHS), from the
// stored rows x2 of H_s^-1 (f.hinv_x2)
void launch_hinv_cols_update(const FactorDev& f, int32_t nc, const int32_t* c_x2, const double* v, double* sol,
                             hipStream_t st);
// The same for rows [j0, j1) of the extended order (x1 rows first, then x2).
void launch_hinv_cols_update_range(const FactorDev& f, int32_t nc, const int32_t* c_x2, const double* v, double* sol,
                                   int64_t j0, int64_t j1, hipStream_t st);
// Rows x2 of H_s^-1 into K (n2 x (n1 + n2)): column q of Sigma^-1 is the x2
// part of H_s^-1 e_q, and the backward sweep with y1 = 0 gives its x1 part,
// -H11^-1 H12 Sigma^-1 e_q; three columns per sweep.  y and sol are the
// sweep's work vectors (3 (n1 + n2) and 6 (n1 + n2)); y is left zero.
void launch_build_hinv_rows(const FactorDev& f, double* y, double* sol, double* K, hipStream_t st);
// c index -> x2 index
void launch_c_to_x2(int32_t nc, const int32_t* clist, const int32_t* vert2x2, int32_t* c_x2, hipStream_t st);

// ---------------------------------------- comparison global steps (Table 1)
// out = H v (per-tet shares into tetg, m x 12, gathered per free vertex)
void launch_pd_matvec(const LocalArgs& la, int32_t n, const int32_t* vt_ptr, const int32_t* vt_ent,
                      const uint8_t* fixed, const double* v, double* tetg, double* out, hipStream_t st);
// vc (nc x 3) = v at the contact vertices; out at the contact vertices += vc
void launch_gather_c(int32_t nc, const int32_t* clist, const double* v, double* vc, hipStream_t st);
void launch_scatter_add_c(int32_t nc, const int32_t* clist, const double* vc, double* out, hipStream_t st);
// CG updates with device scalars: x += a p, r -= a q (a = sc[num] / sc[den]);
// p = z + b p (b = sc[num] / sc[den])
void launch_cg_step(int64_t n3, const double* sc, int num, int den, const double* p, const double* q, double* x,
                    double* r, hipStream_t st);
void launch_cg_dir(int64_t n3, const double* sc, int num, int den, const double* z, double* p, hipStream_t st);
// out (3 n2 square, vertex-major) = S (x) I3; out[x2 rows/cols of c] += Bc (3 nc square)
void launch_kron_i3(int32_t n2, const double* S, double* out, hipStream_t st);
void launch_scatter_block(int32_t nc, const int32_t* c_x2, const double* Bc, int32_t n2, double* out,
                          hipStream_t st);

// Message returned by pdipc_last_error(NULL) (this thread).
void set_last_error(const char* msg);

// ---------------------------------------------------------------- dense SPD
// Lower Cholesky of an n x n row-major SPD matrix A (destroyed: lower tiles by
// the factorisation, strictly upper blocks as workspace), 32-wide blocks up to
// 2048 unknowns and 64-wide above.  F receives L^-1 (lower triangle,
// row-major) and aux its transpose; aux (dense_aux_size(n) entries) then holds
// 1 / diag(L) (n), the inverses of the diagonal blocks and solve scratch
// (4 n).  The factor L itself is not kept, and the strict upper part of F is
// not written.  *d_info <- 0 ok, else 1 + the first failing column (the
// outputs are then NaN from that column on).
constexpr int64_t dense_blocks_size(int64_t n) { return ((n + 63) / 64) * 64 * 64; }
constexpr int64_t dense_tmp_offset(int64_t n) { return n * n + n + dense_blocks_size(n); }
constexpr int64_t dense_aux_size(int64_t n) { return dense_tmp_offset(n) + 4 * n + 64; }
template <typename T>
void dense_cholesky(T* A, int64_t n, T* F, T* aux, int32_t* d_info, hipStream_t st);
// The same factorisation queued in parts: its launches are numbered
// 0 .. dense_cholesky_launches(n) - 1 and dense_cholesky_range queues
// [p0, p1) of them, so that a caller can interleave other streams' launches.
int64_t dense_cholesky_launches(int64_t n);
template <typename T>
void dense_cholesky_range(T* A, int64_t n, T* F, T* aux, int32_t* d_info, hipStream_t st, int64_t p0, int64_t p1);
// Solve L L^T x = b in place (b: n x nrhs row-major, nrhs <= 4).
template <typename T>
void dense_chol_solve(const T* F, T* aux, int64_t n, T* b, int32_t nrhs, hipStream_t st);
// Single right-hand side, b -> x (no aliasing).
template <typename T>
void dense_chol_solve_into(const T* F, T* aux, int64_t n, const T* b, T* x, hipStream_t st);
// Iterative refinement of M u = rhs with the FP32 inverse factor (F, aux) of
// S M S, S = diag(sc): step s computes r_s = rhs - M u_s (u_0 = 0) in FP64,
// res[s] = max |r_s| and r32 = float(S r_s) (launch_refine_residual), then
// u += S Y^T Y r32 (launch_refine_correct).  Kernels of a step do nothing once
// an earlier res met res <= tol res[0]; res (>= steps + 1 entries) starts at 0.
void launch_refine_residual(const double* M, int64_t n, const double* rhs, const double* u, const double* sc,
                            float* r32, double* res, int s, double tol, hipStream_t st);
void launch_refine_correct(const float* F, float* aux, int64_t n, const float* r32, const double* sc, double* u,
                           const double* res, int s, double tol, hipStream_t st);
// Ainv = (L L^T)^-1 (full symmetric, row-major), work: n x n scratch
template <typename T>
void dense_chol_inverse(const T* F, const T* aux, int64_t n, T* Ainv, T* work, hipStream_t st);
// C^-1 after a small change of the contact set c (at most 32 vertices leave and
// at most 32 enter; at least one is kept): the previous inverse Ci (order of
// the previous c, nold x nold) is downdated for the leaving vertices and
// bordered with the entering ones (Schur complement against Sigma^-1), giving
// out (nc x nc, order of the new c).  rem_ids / add_ids hold the r leaving and
// a entering vertices in any order (build_incidence's lists); pflag/pidx are
// the previous contact flags and ranks, cflag/cidx the current ones.  A
// non-positive pivot of the two small SPD inverses sets *info (zeroed first).
struct CinvLists {
  int32_t* kept_old;   // nk: previous index of the k-th kept vertex
  int32_t* kept_x2;    // nk: its index among the rows of Sigma^-1
  int32_t* rem_old;    // r: previous index of the leaving vertices (by id)
  int32_t* add_x2;     // a: Sigma^-1 index of the entering vertices (by id)
  int32_t* kind;       // nc: k >= 0 kept rank k, -1 - q entering vertex q
};
struct CinvUpdateArgs {
  int32_t n, nold, nc, r, a, n2;
  const int32_t *cflag, *cidx, *pflag, *pidx, *vert2x2;
  const int32_t *rem_ids, *add_ids;
  int32_t* info;
  CinvLists L;
  const double* Ci;                  // previous inverse
  const double* Si;                  // Sigma^-1 (n2 x n2)
  double *Sm, *Sinv;                 // a x a, 32 x 32
  double *T, *W, *V;                 // nk x r, nk x a, nk x a
  double* G;                         // r x nk: G[q][i] = Ci[kept i][removed q]
  double* CK;                        // nk x nk
  double* out;                       // nc x nc
};
void launch_cinv_update(const CinvUpdateArgs& u, hipStream_t st);
void launch_convert_f64_f32(const double* in, float* out, int64_t n, hipStream_t st);
void launch_convert_f32_f64(const float* in, double* out, int64_t n, hipStream_t st);
// Jacobi scaling sc_i = 1/sqrt(M_ii); FP32 copies of S M S and S r; u += S y
void launch_jacobi_scaling(const double* M, int64_t n, double* sc, hipStream_t st);
void launch_scale_convert_matrix(const double* M, int64_t n, const double* sc, float* out, hipStream_t st);
void launch_scale_convert_vec(const double* r, int64_t n, const double* sc, float* out, hipStream_t st);
void launch_scaled_accumulate(const float* y, int64_t n, const double* sc, double* u, hipStream_t st);
// r = b - M u  (dense, n x n row-major FP64), all vectors n
void launch_dense_residual(const double* M, int64_t n, const double* b, const double* u, double* r, hipStream_t st);

// ------------------------------------------------------------------ adjoint
// out = K v on the free DOFs (true energy Hessian: PD term with the rotation
// derivative + unprojected barrier Hessian); tetg: 12 x m scratch, pairbuf:
// 12 x npairs scratch.
void launch_hessvec(const LocalArgs& la, int32_t n, const int32_t* vt_ptr, const int32_t* vt_ent,
                    const uint8_t* fixed, const double* x, const double* Rrot, const double* v, double* tetg,
                    const PairList& pl, int32_t npairs, int32_t n_pt, const Incidence& inc, const ProxyDev& px,
                    double dhat, double kappa, int form, double* pairbuf, double* out, hipStream_t st);
// dL/da per tet from the adjoint state lambda (n x 3)
void launch_actuation_grad(const LocalArgs& la, const double* x, const double* Rrot, const double* R0,
                           const double* lam, double* out, hipStream_t st);
void launch_masked_mul(int64_t n, const double* a, const double* b, const uint8_t* fixed, double* out,
                       hipStream_t st);
// y = alpha x + beta y
void launch_axpby(int64_t n3, double alpha, const double* x, double beta, double* y, hipStream_t st);

}  // namespace pdipc
