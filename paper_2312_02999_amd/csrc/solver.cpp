// Solver runtime and the C ABI of include/pdipc.h.
//
// One iteration of Algorithm 1 (quasi-static PD with IPC contact):
//   local step            per-tet rotation fit and PD gradient     (Eq. 1)
//   constraint set        spatial hash + exact distances < dhat   (Section 2.2)
//   barrier               gradient + PSD Hessian factors          (Eq. 3)
//   global step           Eq. (7) sweeps + Eq. (11) reduced system (Section 3)
//   CCD                   swept candidates + conservative advancement
//   line search           back-tracking on the total energy difference
// All state stays in device memory; the host reads back only the pair
// counts, n_c, the factorization status, alpha_m and the line-search sign.
#include "../../include/pdipc.h"
#include "../../include/pdipc_debug.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "host_factor.h"
#include "kernels.h"

namespace pdipc {

static thread_local std::string g_last_init_error;

void set_last_error(const char* msg) { g_last_init_error = msg; }

#define HIPCHK(expr)                                                   \
  do {                                                                 \
    hipError_t e_ = (expr);                                            \
    if (e_ != hipSuccess) {                                            \
      throw HipFailure(std::string(#expr) + ": " + hipGetErrorString(e_)); \
    }                                                                  \
  } while (0)

struct HipFailure {
  std::string msg;
  explicit HipFailure(std::string m) : msg(std::move(m)) {}
};
struct SolverError {
  int code;
  std::string msg;
};

// device bytes held by all DBufs of the calling thread's current solver
static thread_local int64_t* g_bytes_counter = nullptr;

template <typename T>
struct DBuf {
  T* p = nullptr;
  int64_t cap = 0;
  int64_t* counter = nullptr;
  void ensure(int64_t count) {
    if (count <= cap) return;
    if (!counter) counter = g_bytes_counter;
    if (p) {
      HIPCHK(hipFree(p));
      if (counter) *counter -= static_cast<int64_t>(sizeof(T)) * cap;
    }
    p = nullptr;
    // regrowth is geometric: sizes that creep up over a frame (contact counts)
    // would otherwise free and reallocate, and hipFree waits for the device
    int64_t c = std::max<int64_t>(count, cap > 0 ? cap + cap / 2 : 1);
    if (hipMalloc(&p, sizeof(T) * c) != hipSuccess) {
      p = nullptr;
      cap = 0;
      throw SolverError{PDIPC_E_NOMEM, "device allocation failed"};
    }
    cap = c;
    if (counter) *counter += static_cast<int64_t>(sizeof(T)) * c;
  }
  void upload(const T* h, int64_t count, hipStream_t st) {
    ensure(count);
    if (count > 0) HIPCHK(hipMemcpyAsync(p, h, sizeof(T) * count, hipMemcpyHostToDevice, st));
  }
  void release() {
    if (p) {
      (void)hipFree(p);
      if (counter) *counter -= static_cast<int64_t>(sizeof(T)) * cap;
    }
    p = nullptr;
    cap = 0;
  }
};

struct BytesScope {
  int64_t* prev;
  explicit BytesScope(int64_t* c) : prev(g_bytes_counter) { g_bytes_counter = c; }
  ~BytesScope() { g_bytes_counter = prev; }
};

struct Solver {
  std::string err;
  int64_t device_bytes = 0;
  pdipc_options opt{};
  hipStream_t st = nullptr;
  int32_t n = 0, m = 0, nsv = 0, nst = 0, nse = 0, n1 = 0, n2 = 0;
  int64_t factor_nnz = 0;
  bool have_actuation = false, have_scalar = false, have_solution = false;

  // mesh
  DBuf<int32_t> tets, vt_ptr, vt_ent, sv, stri, sedge;
  DBuf<double> Bm, w, A, a_s, R0, X;
  DBuf<uint8_t> fixed;
  // per-iteration vectors
  DBuf<double> x, g, dx, tetg, E0, dE, Rtet, tpair, bE0, bdE, scal;
  // factor
  DBuf<int32_t> node_c0, node_s, node_r, level_nodes, frows, fcol, ext2vert, vert2x2, lvl_rows, lvl_row_node;
  DBuf<int64_t> node_roff, node_poff, node_doff, fptr;
  DBuf<double> panelT, dinv, dinvT, fval, sigma_inv, hinv_x2;
  std::vector<int32_t> h_level_ptr, h_level_maxs, h_level_maxr, h_lvl_row_ptr;
  FactorDev fd{};
  DBuf<double> bvec, yvec, solvec;
  // contact
  ProxyDev px{};
  BroadPhaseBuffers bb{};
  DBuf<double> vbox, tbox, ebox, params;
  DBuf<int32_t> t_count, t_cursor, t_id, e_count, e_cursor, e_id, q_count, qbuf, totals, tmpj;
  DBuf<uint64_t> t_key, e_key;
  DBuf<char> scan_tmp, red_tmp;
  DBuf<int32_t> act_type, act_i, act_j, act_v4, cand_type, cand_i, cand_j, cand_v4;
  PairList act{}, cand{};
  DBuf<double> b_energy, b_grad, b_U;
  BarrierOut bo{};
  DBuf<int32_t> inc_cnt, inc_ptr, inc_cursor, inc_ent, inc_raw, inc_cflag, inc_cidx, inc_clist, inc_nc;
  Incidence inc{};
  // reduced system
  DBuf<int32_t> c_x2, info;
  DBuf<double> Cs, Cinv, work, Mred, rhs, u, vvec, wtmp, resid, CsL, CsLi, ML, MLi, scl;
  int32_t refine_steps = 0, refine_fallbacks = 0;
  int32_t cinv_rebuilds = 0, c_delta_max = 0, c_delta_sum = 0, cinv_updates = 0;
  DBuf<float> Mf, uf, MLf, MLif;
  // swept candidates of the last step (x_prev -> x_prev + dx), valid for x on that path
  bool cand_valid = false;
  int32_t cand_n = 0, cand_pt = 0;
  DBuf<int32_t> cflagbuf, cposbuf;
  // C^-1 = ((Sigma_s^-1)_cc)^-1 depends only on the contact set c (Sigma_s^-1 is
  // constant): it is kept while the flags of c are unchanged
  DBuf<int32_t> prev_cflag;
  bool cinv_valid = false;
  // incremental update of C^-1: ranks of the previous c, its size, updates
  // since the last full rebuild, and the work buffers
  DBuf<int32_t> prev_cidx, cupd_i, cset_ids;
  DBuf<double> Cinv_next, cupd_d;
  int32_t nc_prev = 0, cinv_since_full = 0;
  bool cinv_incr_ok = false;
  // device line-search state; factor statuses still to be checked
  DBuf<double> lsbuf;
  DBuf<double> refres;        // refinement residual maxima
  DBuf<double> ccd_part;      // per-block minima of the CCD bounds
  bool check_info_m = false, check_info_cs = false;
  // adjoint work vectors
  DBuf<double> lam, res, zvec, pvec, kp, prod, pairbuf;
  // comparison global steps: CG vectors and device scalars; the dense
  // Sigma-hat, its factor and Sigma_s (kept only for the Schur-only step)
  DBuf<double> cg_r, cg_z, cg_p, cg_q, cg_t, cg_sc, cg_pc, cg_vc;
  DBuf<double> shat, shat_L, shat_aux, sigma_s;
  // barrier stiffness of the current iteration (kappa_0, or the adaptive
  // value); smallest squared pair distance of the previous iteration and the
  // threshold 1e-9 l^2 (l: rest bounding-box diagonal) of the adaptive rule;
  // work arrays of the balancing gradients
  double kappa = 0.0, d2min_prev = 0.0, eps_d2 = 0.0;
  DBuf<double> ka_gE, ka_gb, ka_R;
  // proxy embedding s = W x (Section 3.1) when a row of W interpolates:
  // collision primitives index proxy vertices, positions s and steps W dx
  // feed the contact kernels, and each pair's terms go to its simulation
  // vertices through W (slots); otherwise the proxy selects simulation
  // vertices and the pairs' own terms are used
  bool embed = false;
  int32_t n_inc_verts = 0;
  EmbedDev W{};
  DBuf<int32_t> w_ptr, w_col, inc_verts, slot_v;
  DBuf<double> w_val, spos, sdx, slot_g, slot_U;
  int32_t adjoint_iters = 0;

  // host helpers
  double* h_scal = nullptr;   // pinned readback
  int32_t* h_counts = nullptr;   // pinned readback of pair counts (8)
  // optional HIP-event timer around every launch of one kernel family
  int32_t timer_which = -1;
  // second stream (default priority) for the reduced contact system, which
  // runs concurrently with the sweeps of the global step
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_cinv = nullptr;
  // the x1 rows of the contact correction run on the second stream beside the
  // CCD (which reads proxy vertices, all in x2); the line search waits for them
  hipEvent_t ev_rows = nullptr, ev_x1 = nullptr;
  bool x1_pending = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  double timer_ms = 0.0;
  int64_t timer_count = 0;
  // Table 1 stage boundaries of one iteration on the main stream (recorded
  // while a frame collects statistics): start, IPC done (constraint set,
  // barrier, incidence), local step and gradient done (Misc), global step
  // done, CCD done, line search done
  hipEvent_t sev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  bool stage_on = false;
  // per-iteration record of the last frame (pdipc_debug_trace)
  std::vector<pdipc_iter_trace> trace;

  ~Solver() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : sev)
      if (e) (void)hipEventDestroy(e);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_cinv) (void)hipEventDestroy(ev_cinv);
    if (ev_rows) (void)hipEventDestroy(ev_rows);
    if (ev_x1) (void)hipEventDestroy(ev_x1);
    if (side) (void)hipStreamDestroy(side);
    if (h_scal) (void)hipHostFree(h_scal);
    if (h_counts) (void)hipHostFree(h_counts);
    if (st) (void)hipStreamSynchronize(st);
  }
};

// ----------------------------------------------------------------- init
static void fail(int code, const std::string& msg) { throw SolverError{code, msg}; }

// Kernel families that the event timer can bracket.
enum TimerKernel { TK_LOCAL = 0, TK_SIGMA_GEMV = 1, TK_FWD = 2, TK_BWD = 3, TK_BARRIER = 4, TK_TRIAL = 5,
                   TK_REDUCED_CHOL = 6, TK_PAIRS = 7, TK_CCD = 8, TK_CINV_UPDATE = 9, TK_CINV_FULL = 10 };

struct ScopedTimer {
  Solver* S;
  bool on;
  hipStream_t stream;
  ScopedTimer(Solver* s, int which, hipStream_t sx = nullptr)
      : S(s), on(s->timer_which == which), stream(sx ? sx : s->st) {
    if (on) record();
  }
  ~ScopedTimer() {
    if (on) record();
  }
  void record() {
    if (S->ev_used >= S->ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
      S->ev_pool.push_back(e);
    }
    (void)hipEventRecord(S->ev_pool[S->ev_used++], stream);
  }
};

// A start/stop event pair for a launch that stamps them itself (extended
// launch): the elapsed time is the kernel's own duration.
static bool timer_events(Solver* S, int which, hipEvent_t* e0, hipEvent_t* e1) {
  if (S->timer_which != which) return false;
  while (S->ev_pool.size() < S->ev_used + 2) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return false;
    S->ev_pool.push_back(e);
  }
  *e0 = S->ev_pool[S->ev_used];
  *e1 = S->ev_pool[S->ev_used + 1];
  S->ev_used += 2;
  return true;
}

static void stage_mark(Solver* S, int k) {
  if (S->stage_on) HIPCHK(hipEventRecord(S->sev[k], S->st));
}

static void harvest_timer(Solver* S) {
  for (size_t k = 0; k + 1 < S->ev_used; k += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, S->ev_pool[k], S->ev_pool[k + 1]) == hipSuccess) {
      S->timer_ms += ms;
      S->timer_count += 1;
    }
  }
  S->ev_used = 0;
}

static int32_t do_init(const pdipc_mesh_desc* md, const pdipc_options* op, Solver* S) {
  if (!md || !op) fail(PDIPC_E_INVALID, "null mesh or options");
  S->opt = *op;
  S->st = static_cast<hipStream_t>(op->stream);
  hipStream_t st = S->st;
  const int32_t n = md->n_verts, m = md->n_tets;
  if (n <= 0 || m <= 0 || !md->rest_pos || !md->tets || !md->dirichlet) fail(PDIPC_E_INVALID, "empty mesh");
  if (!(op->dhat > 0) || !(op->kappa > 0) || op->iters <= 0 || op->ccd_steps <= 0 || op->ls_max_halvings < 0 ||
      op->cinv_updates_max < 0 || op->fp32_reduced_min < 0 || op->hinv_rows_mb < 0 ||
      !(op->ccd_eta > 0 && op->ccd_eta < 1))
    fail(PDIPC_E_INVALID, "bad options");
  if (op->precision != PDIPC_FP64 && op->precision != PDIPC_MIXED_FP32) fail(PDIPC_E_INVALID, "bad precision");
  if (op->global_method != PDIPC_GSTEP_SCHUR_WOODBURY && op->global_method != PDIPC_GSTEP_PCG &&
      op->global_method != PDIPC_GSTEP_SCHUR)
    fail(PDIPC_E_INVALID, "bad global_method");
  if (op->global_method != PDIPC_GSTEP_SCHUR_WOODBURY && op->precision != PDIPC_FP64)
    fail(PDIPC_E_INVALID, "the comparison global steps run in FP64 only");
  if (op->global_method == PDIPC_GSTEP_PCG && (!(op->cg_tol > 0) || op->cg_max_iters <= 0))
    fail(PDIPC_E_INVALID, "bad CG options");
  if (op->barrier_form != 0 && op->barrier_form != 1) fail(PDIPC_E_INVALID, "bad barrier_form");
  if (op->kappa_adapt != 0 && op->kappa_adapt != 1) fail(PDIPC_E_INVALID, "bad kappa_adapt");
  S->kappa = op->kappa;
  if (!(md->youngs > 0) || !(md->poisson > -1 && md->poisson < 0.5)) fail(PDIPC_E_INVALID, "bad material");
  S->n = n;
  S->m = m;
  const double* X = md->rest_pos;
  for (int64_t i = 0; i < 3LL * n; ++i)
    if (!std::isfinite(X[i])) fail(PDIPC_E_INVALID, "non-finite rest position");
  {
    // squared rest bounding-box diagonal, for the adaptive-stiffness threshold
    double lo[3] = {X[0], X[1], X[2]}, hi[3] = {X[0], X[1], X[2]};
    for (int32_t v = 0; v < n; ++v)
      for (int r = 0; r < 3; ++r) {
        lo[r] = std::min(lo[r], X[3 * v + r]);
        hi[r] = std::max(hi[r], X[3 * v + r]);
      }
    double l2 = 0.0;
    for (int r = 0; r < 3; ++r) l2 += (hi[r] - lo[r]) * (hi[r] - lo[r]);
    S->eps_d2 = 1e-9 * l2;
  }
  for (int64_t i = 0; i < 4LL * m; ++i)
    if (md->tets[i] < 0 || md->tets[i] >= n) fail(PDIPC_E_INVALID, "tet index out of range");
  int nfixed = 0;
  for (int32_t v = 0; v < n; ++v) nfixed += md->dirichlet[v] ? 1 : 0;
  if (nfixed == 0) fail(PDIPC_E_NOT_SPD, "no fixed vertex: the PD matrix is singular");

  // ---- per-tet rest data (Eq. 1, 2): B = D_m^-1, w = 2 mu V -----------------
  const double mu = md->youngs / (2.0 * (1.0 + md->poisson));
  std::vector<int32_t> tsoa(4LL * m);
  std::vector<double> bsoa(9LL * m), wv(m);
  std::vector<double> g4(12LL * m);   // shape gradients per tet (host use)
  for (int64_t i = 0; i < m; ++i) {
    const int32_t* t = md->tets + 4 * i;
    double D[3][3];
    for (int k = 0; k < 3; ++k)
      for (int r = 0; r < 3; ++r) D[r][k] = X[3 * t[k + 1] + r] - X[3 * t[0] + r];
    double det = D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1]) - D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0]) +
                 D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0]);
    if (!(det > 0)) fail(PDIPC_E_DEGENERATE, "tet " + std::to_string(i) + " has non-positive rest volume");
    double inv[3][3];
    inv[0][0] = (D[1][1] * D[2][2] - D[1][2] * D[2][1]) / det;
    inv[0][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) / det;
    inv[0][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) / det;
    inv[1][0] = (D[1][2] * D[2][0] - D[1][0] * D[2][2]) / det;
    inv[1][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) / det;
    inv[1][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) / det;
    inv[2][0] = (D[1][0] * D[2][1] - D[1][1] * D[2][0]) / det;
    inv[2][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) / det;
    inv[2][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) / det;
    for (int k = 0; k < 4; ++k) tsoa[k * m + i] = t[k];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) bsoa[(3 * r + c) * m + i] = inv[r][c];
    wv[i] = 2.0 * mu * det / 6.0;
    for (int c = 0; c < 3; ++c) {
      g4[12 * i + 3 + c] = inv[0][c];
      g4[12 * i + 6 + c] = inv[1][c];
      g4[12 * i + 9 + c] = inv[2][c];
      g4[12 * i + c] = -(inv[0][c] + inv[1][c] + inv[2][c]);
    }
  }
  // vertex -> (tet, local) incidence, tet-ascending
  std::vector<int32_t> vptr(n + 1, 0), vent(4LL * m);
  for (int64_t i = 0; i < m; ++i)
    for (int k = 0; k < 4; ++k) vptr[md->tets[4 * i + k] + 1]++;
  for (int32_t v = 0; v < n; ++v) vptr[v + 1] += vptr[v];
  {
    std::vector<int32_t> cur(vptr.begin(), vptr.end() - 1);
    for (int64_t i = 0; i < m; ++i)
      for (int k = 0; k < 4; ++k) vent[cur[md->tets[4 * i + k]]++] = static_cast<int32_t>(4 * i + k);
  }

  // ---- proxy (embedded by selection) ------------------------------------------
  const int32_t F = md->n_surf_tris;
  if (F < 0 || (F > 0 && !md->surf_tris)) fail(PDIPC_E_INVALID, "bad proxy triangles");
  std::vector<int32_t> tris(md->surf_tris, md->surf_tris + 3LL * std::max(F, 0));
  if (md->W_rowptr) {
    // s = W x (Section 3.1): validate the CSR rows, then resolve the
    // triangles' proxy-vertex ids to the simulation vertices W selects
    const int32_t ns = md->n_surf_verts;
    if (ns <= 0 || !md->W_col || md->W_rowptr[0] != 0) fail(PDIPC_E_INVALID, "bad proxy embedding W");
    std::vector<int32_t> pick(ns), seen(n, -1);
    for (int32_t r = 0; r < ns; ++r) {
      const int32_t b = md->W_rowptr[r], e = md->W_rowptr[r + 1];
      if (e <= b) fail(PDIPC_E_INVALID, "empty row in the proxy embedding W");
      double sum = 0.0;
      for (int32_t k = b; k < e; ++k) {
        const int32_t c = md->W_col[k];
        const double wv = md->W_val ? md->W_val[k] : 1.0;
        if (c < 0 || c >= n) fail(PDIPC_E_INVALID, "proxy embedding W column out of range");
        if (!(wv >= 0.0) || !std::isfinite(wv)) fail(PDIPC_E_INVALID, "negative or non-finite weight in W");
        for (int32_t k2 = b; k2 < k; ++k2)
          if (md->W_col[k2] == c) fail(PDIPC_E_INVALID, "repeated column in a row of W");
        sum += wv;
      }
      if (!(std::fabs(sum - 1.0) <= 1e-12)) fail(PDIPC_E_INVALID, "a row of W does not sum to 1");
      if (e - b > 4) fail(PDIPC_E_INVALID, "a row of W has more than 4 entries");
      const int32_t c = md->W_col[b];
      const bool picks = e - b == 1 && (md->W_val ? md->W_val[b] : 1.0) == 1.0 && seen[c] < 0;
      if (picks) seen[c] = r;
      pick[r] = picks ? c : -1;
      if (!picks) S->embed = true;
    }
    for (int32_t v : tris)
      if (v < 0 || v >= ns) fail(PDIPC_E_INVALID, "proxy triangle index out of range");
    if (!S->embed) {
      // every row selects its own vertex: resolve the triangles to those
      for (int32_t& v : tris) v = pick[v];
    } else {
      std::vector<int32_t> wp(md->W_rowptr, md->W_rowptr + ns + 1), wc(md->W_col, md->W_col + md->W_rowptr[ns]);
      std::vector<double> wv(wc.size(), 1.0);
      if (md->W_val) wv.assign(md->W_val, md->W_val + md->W_rowptr[ns]);
      S->w_ptr.upload(wp.data(), ns + 1LL, st);
      S->w_col.upload(wc.data(), static_cast<int64_t>(wc.size()), st);
      S->w_val.upload(wv.data(), static_cast<int64_t>(wv.size()), st);
      S->W = EmbedDev{ns, S->w_ptr.p, S->w_col.p, S->w_val.p};
      S->spos.ensure(3LL * ns);
      S->sdx.ensure(3LL * ns);
    }
  }
  const int32_t nproxy = S->embed ? md->n_surf_verts : n;
  for (int32_t v : tris)
    if (v < 0 || v >= nproxy) fail(PDIPC_E_INVALID, "proxy triangle index out of range");
  for (int32_t f = 0; f < F; ++f)
    if (tris[3 * f] == tris[3 * f + 1] || tris[3 * f + 1] == tris[3 * f + 2] || tris[3 * f] == tris[3 * f + 2])
      fail(PDIPC_E_INVALID, "proxy triangle with repeated vertex");
  std::vector<int32_t> svv(tris.begin(), tris.end());
  std::sort(svv.begin(), svv.end());
  svv.erase(std::unique(svv.begin(), svv.end()), svv.end());
  std::vector<std::pair<int32_t, int32_t>> ev;
  ev.reserve(3LL * F);
  for (int32_t f = 0; f < F; ++f)
    for (int k = 0; k < 3; ++k) {
      int32_t a = tris[3 * f + k], b = tris[3 * f + (k + 1) % 3];
      ev.emplace_back(std::min(a, b), std::max(a, b));
    }
  std::sort(ev.begin(), ev.end());
  ev.erase(std::unique(ev.begin(), ev.end()), ev.end());
  std::vector<int32_t> sev(2 * ev.size());
  for (size_t e = 0; e < ev.size(); ++e) {
    sev[2 * e] = ev[e].first;
    sev[2 * e + 1] = ev[e].second;
  }
  S->nsv = static_cast<int32_t>(svv.size());
  S->nst = F;
  S->nse = static_cast<int32_t>(ev.size());
  // the simulation vertices the proxy moves with: the proxy vertices
  // themselves, or the columns of their rows of W
  std::vector<int32_t> wsupp = svv;
  if (S->embed) {
    wsupp.clear();
    for (int32_t p : svv)
      for (int32_t e = md->W_rowptr[p]; e < md->W_rowptr[p + 1]; ++e) wsupp.push_back(md->W_col[e]);
    std::sort(wsupp.begin(), wsupp.end());
    wsupp.erase(std::unique(wsupp.begin(), wsupp.end()), wsupp.end());
  }
  S->inc_verts.upload(wsupp.data(), static_cast<int64_t>(wsupp.size()), st);
  S->n_inc_verts = static_cast<int32_t>(wsupp.size());

  // ---- DOF split (Eq. 6) -----------------------------------------------------------
  std::vector<uint8_t> reg(n, 0);
  if (md->region) {
    for (int32_t v = 0; v < n; ++v) reg[v] = md->region[v] && !md->dirichlet[v];
    for (int32_t v : wsupp)
      if (!md->dirichlet[v] && !reg[v]) fail(PDIPC_E_INVALID, "a free proxy vertex is outside the marked region");
  } else {
    for (int32_t v : wsupp) reg[v] = md->dirichlet[v] ? 0 : 1;
  }
  std::vector<int32_t> x1, x2, vblock(n, -1), vlocal(n, -1);
  for (int32_t v = 0; v < n; ++v) {
    if (md->dirichlet[v]) continue;
    if (reg[v]) { vblock[v] = 2; vlocal[v] = static_cast<int32_t>(x2.size()); x2.push_back(v); }
    else { vblock[v] = 1; vlocal[v] = static_cast<int32_t>(x1.size()); x1.push_back(v); }
  }
  S->n1 = static_cast<int32_t>(x1.size());
  S->n2 = static_cast<int32_t>(x2.size());
  const int32_t n1 = S->n1, n2 = S->n2, N = n1 + n2;

  // ---- scalar PD matrix H_s over free vertices in extended input order ---------------
  auto ext_in = [&](int32_t v) { return vblock[v] == 1 ? vlocal[v] : n1 + vlocal[v]; };
  ScalarCSR H;
  H.n = N;
  {
    std::vector<int64_t> cnt(N + 1, 0);
    for (int64_t i = 0; i < m; ++i)
      for (int a = 0; a < 4; ++a) {
        int32_t va = md->tets[4 * i + a];
        if (vblock[va] < 0) continue;
        for (int b = 0; b < 4; ++b)
          if (vblock[md->tets[4 * i + b]] >= 0) cnt[ext_in(va) + 1]++;
      }
    for (int32_t r = 0; r < N; ++r) cnt[r + 1] += cnt[r];
    std::vector<int32_t> tc(cnt[N]);
    std::vector<double> tv(cnt[N]);
    std::vector<int64_t> cur(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < m; ++i)
      for (int a = 0; a < 4; ++a) {
        int32_t va = md->tets[4 * i + a];
        if (vblock[va] < 0) continue;
        const double* ga = &g4[12 * i + 3 * a];
        for (int b = 0; b < 4; ++b) {
          int32_t vb = md->tets[4 * i + b];
          if (vblock[vb] < 0) continue;
          const double* gb = &g4[12 * i + 3 * b];
          int64_t c = cur[ext_in(va)]++;
          tc[c] = ext_in(vb);
          tv[c] = wv[i] * (ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]);
        }
      }
    H.ptr.assign(N + 1, 0);
    std::vector<std::pair<int32_t, double>> rowbuf;
    for (int32_t r = 0; r < N; ++r) {
      rowbuf.clear();
      for (int64_t e = cnt[r]; e < cnt[r + 1]; ++e) rowbuf.emplace_back(tc[e], tv[e]);
      std::sort(rowbuf.begin(), rowbuf.end(),
                [](const std::pair<int32_t, double>& p, const std::pair<int32_t, double>& q) { return p.first < q.first; });
      for (size_t k = 0; k < rowbuf.size(); ++k) {
        if (k > 0 && rowbuf[k].first == H.col.back()) H.val.back() += rowbuf[k].second;
        else { H.col.push_back(rowbuf[k].first); H.val.push_back(rowbuf[k].second); }
      }
      H.ptr[r + 1] = static_cast<int64_t>(H.col.size());
    }
  }
  std::vector<double> coords1(3LL * n1);
  for (int32_t p = 0; p < n1; ++p)
    for (int r = 0; r < 3; ++r) coords1[3 * p + r] = X[3 * x1[p] + r];
  HostFactor hf;
  std::string ferr;
  int frc = build_host_factor(n1, n2, coords1.data(), H, 96, hf, ferr);
  if (frc != 0) fail(PDIPC_E_NOT_SPD, ferr);
  S->factor_nnz = hf.factor_nnz;

  // ---- upload mesh data -----------------------------------------------------------------
  S->tets.upload(tsoa.data(), 4LL * m, st);
  S->Bm.upload(bsoa.data(), 9LL * m, st);
  S->w.upload(wv.data(), m, st);
  S->A.ensure(6LL * m);
  S->a_s.ensure(m);
  S->R0.ensure(9LL * m);
  S->X.upload(X, 3LL * n, st);
  S->fixed.upload(md->dirichlet, n, st);
  S->vt_ptr.upload(vptr.data(), n + 1, st);
  S->vt_ent.upload(vent.data(), 4LL * m, st);
  S->sv.upload(svv.data(), S->nsv, st);
  S->stri.upload(tris.data(), 3LL * F, st);
  S->sedge.upload(sev.data(), static_cast<int64_t>(sev.size()), st);
  for (auto* b : {&S->x, &S->g, &S->dx}) b->ensure(3LL * n);
  launch_fill_f64(S->dx.p, 3LL * n, 0.0, st);      // the fixed vertices' entries stay zero
  S->tetg.ensure(12LL * m);
  S->E0.ensure(m);
  S->dE.ensure(m);
  S->Rtet.ensure(9LL * m);
  launch_identity_rotations(m, S->Rtet.p, st);
  S->scal.ensure(16);
  S->lsbuf.ensure(LS_SIZE);
  HIPCHK(hipStreamCreateWithFlags(&S->side, hipStreamNonBlocking));
  HIPCHK(hipEventCreateWithFlags(&S->ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&S->ev_join, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&S->ev_cinv, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&S->ev_rows, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&S->ev_x1, hipEventDisableTiming));
  for (hipEvent_t& e : S->sev) HIPCHK(hipEventCreate(&e));
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&S->h_scal), 16 * sizeof(double), hipHostMallocDefault));
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&S->h_counts), 8 * sizeof(int32_t), hipHostMallocDefault));

  // ---- factor upload ---------------------------------------------------------------------------
  const int32_t nn = static_cast<int32_t>(hf.nodes.size());
  std::vector<int32_t> c0(nn), ss(nn), rr(nn), lev_nodes;
  std::vector<int64_t> ro(nn), po(nn), dof(nn);
  for (int32_t J = 0; J < nn; ++J) {
    c0[J] = hf.nodes[J].c0; ss[J] = hf.nodes[J].s; rr[J] = hf.nodes[J].r;
    ro[J] = hf.nodes[J].rows_off; po[J] = hf.nodes[J].panel_off; dof[J] = hf.nodes[J].dinv_off;
  }
  S->h_level_ptr.assign(hf.nlevels + 1, 0);
  S->h_level_maxs.assign(std::max(hf.nlevels, 1), 0);
  S->h_level_maxr.assign(std::max(hf.nlevels, 1), 0);
  for (int32_t J = 0; J < nn; ++J) S->h_level_ptr[hf.nodes[J].level + 1]++;
  for (int32_t L = 0; L < hf.nlevels; ++L) S->h_level_ptr[L + 1] += S->h_level_ptr[L];
  lev_nodes.resize(nn);
  {
    std::vector<int32_t> cur(S->h_level_ptr.begin(), S->h_level_ptr.end() - 1);
    for (int32_t J = 0; J < nn; ++J) {
      int L = hf.nodes[J].level;
      lev_nodes[cur[L]++] = J;
      S->h_level_maxs[L] = std::max(S->h_level_maxs[L], ss[J]);
      S->h_level_maxr[L] = std::max(S->h_level_maxr[L], rr[J]);
    }
  }
  // rows of each level (columns of its supernodes), for wave-per-row sweeps
  S->h_lvl_row_ptr.assign(hf.nlevels + 1, 0);
  std::vector<int32_t> lrows, lnode;
  lrows.reserve(n1);
  lnode.reserve(n1);
  for (int32_t L = 0; L < hf.nlevels; ++L) {
    for (int32_t k = S->h_level_ptr[L]; k < S->h_level_ptr[L + 1]; ++k) {
      const int32_t J = lev_nodes[k];
      for (int32_t c = 0; c < ss[J]; ++c) {
        lrows.push_back(c0[J] + c);
        lnode.push_back(J);
      }
    }
    S->h_lvl_row_ptr[L + 1] = static_cast<int32_t>(lrows.size());
  }
  std::vector<double> dT(hf.dinv.size());
  for (int32_t J = 0; J < nn; ++J) {
    const int s = ss[J];
    const double* D = hf.dinv.data() + dof[J];
    double* T = dT.data() + dof[J];
    for (int r = 0; r < s; ++r)
      for (int c = 0; c < s; ++c) T[static_cast<int64_t>(c) * s + r] = D[static_cast<int64_t>(r) * s + c];
  }
  std::vector<int32_t> e2v(N), v2x2(n, -1);
  for (int32_t p = 0; p < n1; ++p) e2v[p] = x1[hf.perm[p]];
  for (int32_t q = 0; q < n2; ++q) { e2v[n1 + q] = x2[q]; v2x2[x2[q]] = q; }
  S->node_c0.upload(c0.data(), nn, st);
  S->node_s.upload(ss.data(), nn, st);
  S->node_r.upload(rr.data(), nn, st);
  S->node_roff.upload(ro.data(), nn, st);
  S->node_poff.upload(po.data(), nn, st);
  S->node_doff.upload(dof.data(), nn, st);
  S->level_nodes.upload(lev_nodes.data(), nn, st);
  S->frows.upload(hf.rows.data(), static_cast<int64_t>(hf.rows.size()), st);
  S->lvl_rows.upload(lrows.data(), static_cast<int64_t>(lrows.size()), st);
  S->lvl_row_node.upload(lnode.data(), static_cast<int64_t>(lnode.size()), st);
  S->dinv.upload(hf.dinv.data(), static_cast<int64_t>(hf.dinv.size()), st);
  S->dinvT.upload(dT.data(), static_cast<int64_t>(dT.size()), st);
  S->fptr.upload(hf.fwd_ptr.data(), static_cast<int64_t>(hf.fwd_ptr.size()), st);
  S->fcol.upload(hf.fwd_col.data(), static_cast<int64_t>(hf.fwd_col.size()), st);
  {
    // The sweeps use W_J = L_{R(J),J} Dinv_J in place of the panels: the lower
    // sweep then carries t (before the diagonal blocks) from level to level,
    // t_J = b_J - sum over descendants K of W_K[J rows] t_K, and applies every
    // Dinv_J in one launch at the end; the upper sweep applies every Dinv_J^T
    // first and then needs one launch per level, x_J = z_J - W_J^T x_R.
    std::vector<double> pw(hf.panel.size());
    if (!pw.empty()) {
      DBuf<double> pan, out;
      pan.upload(hf.panel.data(), static_cast<int64_t>(pw.size()), st);
      out.ensure(static_cast<int64_t>(pw.size()));
      launch_panel_times_dinv(nn, S->node_s.p, S->node_r.p, S->node_poff.p, S->node_doff.p, pan.p, S->dinv.p, out.p,
                              st);
      HIPCHK(hipMemcpyAsync(pw.data(), out.p, sizeof(double) * pw.size(), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      pan.release();
      out.release();
    }
    // transposed (s x r row-major per node) for the upper sweep
    std::vector<double> pT(pw.size());
    for (int32_t J = 0; J < nn; ++J) {
      const int s_ = ss[J], r_ = rr[J];
      const double* P = pw.data() + po[J];
      double* Q = pT.data() + po[J];
      for (int i = 0; i < r_; ++i)
        for (int c = 0; c < s_; ++c) Q[static_cast<int64_t>(c) * r_ + i] = P[static_cast<int64_t>(i) * s_ + c];
    }
    S->panelT.upload(pT.data(), static_cast<int64_t>(pT.size()), st);
    // by rows for the lower sweep, in the order of the row copy of the panels
    std::vector<double> fv(hf.fwd_val.size());
    std::vector<int64_t> cur(hf.fwd_ptr.begin(), hf.fwd_ptr.end() - 1);
    for (int32_t J = 0; J < nn; ++J) {
      const int s_ = ss[J], r_ = rr[J];
      const double* P = pw.data() + po[J];
      const int32_t* R = hf.rows.data() + ro[J];
      for (int i = 0; i < r_; ++i) {
        int64_t& q = cur[R[i]];
        for (int k = 0; k < s_; ++k) fv[q++] = P[static_cast<int64_t>(i) * s_ + k];
      }
    }
    S->fval.upload(fv.data(), static_cast<int64_t>(fv.size()), st);
    HIPCHK(hipStreamSynchronize(st));
  }
  S->ext2vert.upload(e2v.data(), N, st);
  S->vert2x2.upload(v2x2.data(), n, st);
  S->bvec.ensure(3LL * std::max(N, 1));
  S->yvec.ensure(6LL * std::max(N, 1));
  S->solvec.ensure(6LL * std::max(N, 1));
  S->info.ensure(8);

  // ---- Sigma^-1 on the device: Cholesky of Sigma_s, then L^-T L^-1 ---------------------------
  S->sigma_inv.ensure(std::max<int64_t>(1, static_cast<int64_t>(n2) * n2));
  if (n2 > 0) {
    DBuf<double> sig, wk, sl, sli;
    sig.upload(hf.sigma.data(), static_cast<int64_t>(n2) * n2, st);
    if (op->global_method == PDIPC_GSTEP_SCHUR) S->sigma_s.upload(hf.sigma.data(), static_cast<int64_t>(n2) * n2, st);
    wk.ensure(static_cast<int64_t>(n2) * n2);
    sl.ensure(static_cast<int64_t>(n2) * n2);
    sli.ensure(dense_aux_size(n2));
    dense_cholesky<double>(sig.p, n2, sl.p, sli.p, S->info.p, st);
    int32_t hinfo = 0;
    HIPCHK(hipMemcpyAsync(&hinfo, S->info.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hinfo != 0) {
      sig.release(); wk.release(); sl.release(); sli.release();
      fail(PDIPC_E_NOT_SPD, "Schur complement Sigma is not positive definite");
    }
    dense_chol_inverse<double>(sl.p, sli.p, n2, S->sigma_inv.p, wk.p, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    sig.release();
    wk.release();
    sl.release();
    sli.release();
  }
  FactorDev& f = S->fd;
  f.n1 = n1; f.n2 = n2; f.nnodes = nn; f.nlevels = hf.nlevels;
  f.node_c0 = S->node_c0.p; f.node_s = S->node_s.p; f.node_r = S->node_r.p;
  f.node_rows_off = S->node_roff.p; f.node_panel_off = S->node_poff.p; f.node_dinv_off = S->node_doff.p;
  f.level_nodes = S->level_nodes.p;
  f.h_level_ptr = S->h_level_ptr.data(); f.h_level_maxs = S->h_level_maxs.data(); f.h_level_maxr = S->h_level_maxr.data();
  f.h_lvl_row_ptr = S->h_lvl_row_ptr.data(); f.lvl_rows = S->lvl_rows.p; f.lvl_row_node = S->lvl_row_node.p;
  f.rows = S->frows.p; f.panelT = S->panelT.p; f.dinv = S->dinv.p; f.dinvT = S->dinvT.p;
  f.fwd_ptr = S->fptr.p; f.fwd_col = S->fcol.p; f.fwd_val = S->fval.p;
  f.sigma_inv = S->sigma_inv.p; f.ext2vert = S->ext2vert.p;
  f.hinv_x2 = nullptr;
  // rows x2 of H_s^-1 (contact correction as one product), within the budget
  if (n2 > 0 && static_cast<int64_t>(n2) * N * 8 <= static_cast<int64_t>(op->hinv_rows_mb) << 20) {
    S->hinv_x2.ensure(static_cast<int64_t>(n2) * N);
    launch_build_hinv_rows(f, S->yvec.p, S->solvec.p, S->hinv_x2.p, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    f.hinv_x2 = S->hinv_x2.p;
  }

  // ---- contact buffers ---------------------------------------------------------------------------------
  S->px = ProxyDev{S->nsv, S->nst, S->nse, S->sv.p, S->stri.p, S->sedge.p};
  S->vbox.ensure(6LL * std::max(S->nsv, 1));
  S->tbox.ensure(6LL * std::max(S->nst, 1));
  S->ebox.ensure(6LL * std::max(S->nse, 1));
  S->params.ensure(8 + 4 * 64);
  int bits = 10;
  while ((1LL << bits) < 4LL * (S->nst + S->nse) && bits < 28) ++bits;
  const int64_t T = 1LL << bits;
  const int64_t ent = 8LL * std::max(S->nst, S->nse) + 64;
  for (auto* b : {&S->t_count, &S->t_cursor, &S->e_count, &S->e_cursor}) b->ensure(T + 1);
  S->t_id.ensure(ent); S->e_id.ensure(ent); S->t_key.ensure(ent); S->e_key.ensure(ent);
  S->q_count.ensure(8LL * (static_cast<int64_t>(S->nsv) + S->nse) + 1);
  S->qbuf.ensure(static_cast<int64_t>(kQueryKeep) * (static_cast<int64_t>(S->nsv) + S->nse) + 1);
  S->totals.ensure(8);
  const int64_t scan_n = std::max<int64_t>({T + 1, 8LL * (static_cast<int64_t>(S->nsv) + S->nse) + 1,
                                            static_cast<int64_t>(n) + 1});
  S->scan_tmp.ensure(static_cast<int64_t>(scan_temp_bytes(scan_n)));
  S->red_tmp.ensure(static_cast<int64_t>(sum_temp_bytes(0)) + 4096);
  BroadPhaseBuffers& bb = S->bb;
  bb.vbox = S->vbox.p; bb.tbox = S->tbox.p; bb.ebox = S->ebox.p; bb.params = S->params.p;
  bb.table_bits = bits;
  bb.t_count = S->t_count.p; bb.t_cursor = S->t_cursor.p; bb.t_id = S->t_id.p; bb.t_key = S->t_key.p;
  bb.e_count = S->e_count.p; bb.e_cursor = S->e_cursor.p; bb.e_id = S->e_id.p; bb.e_key = S->e_key.p;
  bb.ent_cap = ent; bb.q_count = S->q_count.p; bb.qbuf = S->qbuf.p; bb.d_totals = S->totals.p;
  bb.h_totals = S->h_counts;
  S->tmpj.ensure(4LL * S->nsv + 1024);
  bb.tmpj = S->tmpj.p;
  bb.tmp_cap = S->tmpj.cap;
  bb.scan_temp = S->scan_tmp.p; bb.red_temp = S->red_tmp.p;
  for (auto* b : {&S->inc_cnt, &S->inc_ptr, &S->inc_cflag, &S->inc_cidx}) b->ensure(n + 1);
  S->inc_cursor.ensure(n + 1);
  S->inc_clist.ensure(n);
  S->inc_nc.ensure(8);
  HIPCHK(hipStreamSynchronize(st));
  return PDIPC_OK;
}

// Positions the contact kernels read: s = W x (computed by
// update_proxy_positions), or x itself.
static const double* proxy_x(Solver* S) { return S->embed ? S->spos.p : S->x.p; }
static const double* proxy_dx(Solver* S) { return S->embed ? S->sdx.p : S->dx.p; }
static void update_proxy_positions(Solver* S, const double* x) {
  if (S->embed) launch_embed_positions(S->W, x, S->spos.p, S->st);
}
static void update_proxy_step(Solver* S) {
  if (S->embed) launch_embed_positions(S->W, S->dx.p, S->sdx.p, S->st);
}
static void grow_pairs(Solver* S, PairList& pl, DBuf<int32_t>& ty, DBuf<int32_t>& ii, DBuf<int32_t>& jj,
                       DBuf<int32_t>& v4, int64_t need) {
  int64_t cap = std::max<int64_t>(need + need / 2 + 256, pl.cap);
  ty.ensure(cap); ii.ensure(cap); jj.ensure(cap); v4.ensure(4 * cap);
  pl.type = ty.p; pl.i = ii.p; pl.j = jj.p; pl.v4 = v4.p; pl.cap = cap;
}

// constraint set (dist) or swept candidates (dx != null)
static void pairs(Solver* S, bool active, const double* xx, const double* dxx, int32_t* npt, int32_t* nee) {
  PairList& pl = active ? S->act : S->cand;
  auto& ty = active ? S->act_type : S->cand_type;
  auto& ii = active ? S->act_i : S->cand_i;
  auto& jj = active ? S->act_j : S->cand_j;
  auto& v4 = active ? S->act_v4 : S->cand_v4;
  if (pl.cap == 0) grow_pairs(S, pl, ty, ii, jj, v4, 4LL * S->nsv + 1024);
  for (int attempt = 0; attempt < 3; ++attempt) {
    int64_t need = 0;
    int rc = find_pairs(S->px, S->bb, xx, dxx, S->opt.dhat, active, pl, npt, nee, S->st, &need);
    if (rc == 0) return;
    if (rc < 0) fail(PDIPC_E_HIP, "broad phase overflow");
    if (need > pl.cap) grow_pairs(S, pl, ty, ii, jj, v4, need);
    if (need > S->bb.tmp_cap) {
      S->tmpj.ensure(need + need / 2 + 256);
      S->bb.tmpj = S->tmpj.p;
      S->bb.tmp_cap = S->tmpj.cap;
    }
  }
  fail(PDIPC_E_NOMEM, "pair list growth failed");
}

// Constraint set from the previous step's swept candidates (same sorted set as
// a fresh broad phase at any point of that step).
static void pairs_from_candidates(Solver* S, int32_t* npt, int32_t* nee, int32_t* near_ties) {
  PairList& pl = S->act;
  if (pl.cap == 0) grow_pairs(S, pl, S->act_type, S->act_i, S->act_j, S->act_v4, 4LL * S->nsv + 1024);
  S->cflagbuf.ensure(S->cand_n + 1);
  S->cposbuf.ensure(S->cand_n + 1);
  S->scan_tmp.ensure(static_cast<int64_t>(scan_temp_bytes(S->cand_n + 1)));
  S->bb.scan_temp = S->scan_tmp.p;
  for (int attempt = 0; attempt < 3; ++attempt) {
    int64_t need = 0;
    int rc = filter_active(S->cand, S->cand_n, S->cand_pt, proxy_x(S), S->opt.dhat, pl, S->cflagbuf.p, S->cposbuf.p,
                           S->totals.p + 4, S->h_counts + 4, S->scan_tmp.p, npt, nee, S->st, &need, near_ties);
    if (rc == 0) return;
    grow_pairs(S, pl, S->act_type, S->act_i, S->act_j, S->act_v4, need);
  }
  fail(PDIPC_E_NOMEM, "pair list growth failed");
}

static constexpr int kEmbedSlots = 16;   // slots per pair with an interpolating W

static void ensure_pair_arrays(Solver* S, int64_t np) {
  int64_t cap = std::max<int64_t>(np, 1);
  const int64_t slots = S->embed ? kEmbedSlots : 4;
  if (S->b_energy.cap < cap) {
    int64_t c = cap + cap / 2 + 256;
    S->b_energy.ensure(c); S->b_grad.ensure(12 * c); S->b_U.ensure(60 * c); S->inc_ent.ensure(slots * c);
    S->inc_raw.ensure(slots * c);
    S->wtmp.ensure(5 * c);
    if (S->embed) {
      S->slot_v.ensure(slots * c);
      S->slot_g.ensure(3 * slots * c);
      S->slot_U.ensure(15 * slots * c);
    }
  }
  S->bo = BarrierOut{S->b_energy.p, S->b_grad.p, S->b_U.p};
  S->inc = Incidence{S->inc_cnt.p, S->inc_ptr.p, S->inc_cursor.p, S->inc_raw.p, S->inc_ent.p, S->inc_cflag.p,
                     S->inc_cidx.p, S->inc_clist.p, S->inc_nc.p, S->inc_verts.p, S->n_inc_verts};
}

// The active pairs' terms over simulation vertices.
static PairSlots pair_slots(Solver* S) {
  if (!S->embed) return PairSlots{4, S->act.v4, S->bo.grad, S->bo.U};
  return PairSlots{kEmbedSlots, S->slot_v.p, S->slot_g.p, S->slot_U.p};
}

// The barrier terms of the np active pairs over simulation vertices.
static void expand_pair_terms(Solver* S, int32_t np) {
  if (S->embed) launch_expand_pairs(S->W, S->act.v4, np, S->bo, S->slot_v.p, S->slot_g.p, S->slot_U.p, S->st);
}

static LocalArgs local_args(Solver* S) { return LocalArgs{S->m, S->tets.p, S->Bm.p, S->w.p, S->A.p}; }

static double read_scalar_d(Solver* S, const double* dptr) {
  HIPCHK(hipMemcpyAsync(S->h_scal, dptr, sizeof(double), hipMemcpyDeviceToHost, S->st));
  HIPCHK(hipStreamSynchronize(S->st));
  return S->h_scal[0];
}
static int32_t read_scalar_i(Solver* S, const int32_t* dptr) {
  int32_t v = 0;
  HIPCHK(hipMemcpyAsync(S->h_scal, dptr, sizeof(int32_t), hipMemcpyDeviceToHost, S->st));
  HIPCHK(hipStreamSynchronize(S->st));
  std::memcpy(&v, S->h_scal, sizeof(int32_t));
  return v;
}

struct IterOut;
static void finish_readback(Solver* S, IterOut& io);

struct IterOut {
  int32_t npt = 0, nee = 0, nc = 0, ncand = 0, halvings = 0, near_ties = 0;
  bool ls_ok = true;
  bool c_same = false;          // contact set equal to the one C^-1 was built for
  bool nc_pending = false;      // n_c (and c_same) still in flight to h_scal
  bool nc_with_same = false;    // the readback carries the c_same flag
  int32_t c_removed = 0, c_added = 0;   // vertices that left / entered c
  int32_t cg_iters = 0;                 // products of the CG baseline's step
  double alpha_m = 1.0, alpha = 0.0;
  double kappa = 0.0;                   // barrier stiffness of the iteration
};

static void finish_readback(Solver* S, IterOut& io) {
  if (!io.nc_pending) return;
  HIPCHK(hipEventSynchronize(S->ev_fork));
  int32_t h4[4] = {0, 1, 0, 0};
  std::memcpy(h4, S->h_scal, sizeof(int32_t) * (io.nc_with_same ? 4 : 1));
  io.nc = h4[0];
  io.c_same = io.nc_with_same && h4[1] == 0;
  io.c_removed = io.nc_with_same ? h4[2] : 0;
  io.c_added = io.nc_with_same ? h4[3] : h4[0];
  io.nc_pending = false;
}

// Largest product (bytes of H_s^-1 rows read) for the contact correction by
// the stored rows; beyond it the backward sweep after the x2 correction is
// cheaper.
static constexpr int64_t kHinvColsBytes = 512LL << 20;

// Launches of the reduced factorisation queued before the rest of the main
// stream's forward sweep.
static constexpr int64_t kFactorLaunchesFirst = 10;

// Levels of the lower sweep queued before the host waits for n_c.
static constexpr int kFwdLevelsBeforeFork = 3;

// Most vertices that may leave (and, separately, enter) c for an incremental
// update of C^-1 in place of a rebuild.
static constexpr int32_t kCinvMaxDelta = 32;

// Start of a frame (or of another pass over one state): C^-1 is kept only if
// it came from a full rebuild, a function of its contact set alone, and the
// first change of the set is a full rebuild too, so that what a pass computes
// does not depend on earlier calls.
static void cinv_begin_pass(Solver* S) {
  if (S->cinv_since_full > 0) S->cinv_valid = false;
  S->cinv_incr_ok = false;
}

// Adaptive barrier stiffness (IPC's scheme as read here).  At the start of a
// frame with active pairs, kappa = argmin_k |g_E + k g_b|^2 = -(g_E . g_b) /
// (g_b . g_b) over the free DOFs (g_E: PD gradient, g_b: gradient of the
// unit-stiffness barrier), clamped to [kappa_0, 100 kappa_0]; kappa_0
// without pairs.  At later iterations kappa doubles (up to 100 kappa_0) when
// the smallest squared pair distance is below 1e-9 l^2 and below its value
// at the previous iteration.
static double balanced_kappa(Solver* S, int32_t npt, int32_t np) {
  hipStream_t st = S->st;
  const int64_t n3 = 3LL * S->n;
  S->ka_gE.ensure(n3);
  S->ka_gb.ensure(n3);
  S->ka_R.ensure(9LL * S->m);
  S->prod.ensure(n3);
  launch_barrier(S->act, np, npt, proxy_x(S), S->opt.dhat, 1.0, S->opt.barrier_form, false, S->bo, st);
  expand_pair_terms(S, np);
  build_incidence(pair_slots(S), np, S->n, S->fixed.p, S->inc, S->scan_tmp.p, st);
  launch_fill_f64(S->ka_gb.p, n3, 0.0, st);
  launch_add_barrier_grad(S->inc, pair_slots(S), np, S->fixed.p, S->ka_gb.p, st);
  // PD gradient at x from the frame's starting rotations (kept unchanged)
  launch_local_step(local_args(S), S->x.p, S->Rtet.p, S->ka_R.p, S->E0.p, S->tetg.p, false, st);
  launch_gather_vertex_grad(S->n, S->m, S->vt_ptr.p, S->vt_ent.p, S->tetg.p, S->fixed.p, S->ka_gE.p, st);
  launch_masked_mul(S->n, S->ka_gE.p, S->ka_gb.p, S->fixed.p, S->prod.p, st);
  launch_sum(S->prod.p, n3, S->scal.p + 5, S->red_tmp.p, st);
  launch_masked_mul(S->n, S->ka_gb.p, S->ka_gb.p, S->fixed.p, S->prod.p, st);
  launch_sum(S->prod.p, n3, S->scal.p + 6, S->red_tmp.p, st);
  HIPCHK(hipMemcpyAsync(S->h_scal, S->scal.p + 5, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double eb = S->h_scal[0], bb = S->h_scal[1];
  const double k = bb > 0.0 ? -eb / bb : S->opt.kappa;
  return std::min(std::max(k, S->opt.kappa), 100.0 * S->opt.kappa);
}

static void adapt_kappa(Solver* S, bool frame_start, int32_t npt, int32_t np) {
  double d2min = INFINITY;
  if (np > 0) {
    S->tpair.ensure(np);
    launch_pair_min_dist2(S->act, np, npt, proxy_x(S), S->tpair.p, S->st);
    launch_min_clamp1(S->tpair.p, np, S->scal.p, S->red_tmp.p, S->st);
    d2min = read_scalar_d(S, S->scal.p);
  }
  if (frame_start) S->kappa = np > 0 ? balanced_kappa(S, npt, np) : S->opt.kappa;
  else if (d2min < S->eps_d2 && d2min < S->d2min_prev) S->kappa = std::min(2.0 * S->kappa, 100.0 * S->opt.kappa);
  S->d2min_prev = d2min;
}

// Constraint set + barrier + local step + gradient; returns pair counts, n_c.
// The contact terms go first: the fork event follows them, so the reduced
// system (second stream) builds while the local step runs.  With defer, n_c
// is left in flight (the fork event marks its copy) and global_step collects
// it after queueing the first sweep levels, which need only g.
static void assemble_gradient(Solver* S, bool first_check, IterOut& io, bool defer = false) {
  const bool fp32 = S->opt.precision == PDIPC_MIXED_FP32;
  hipStream_t st = S->st;
  update_proxy_positions(S, S->x.p);
  if (S->cand_valid && !first_check) pairs_from_candidates(S, &io.npt, &io.nee, &io.near_ties);
  else pairs(S, true, proxy_x(S), nullptr, &io.npt, &io.nee);
  const int32_t np = io.npt + io.nee;
  ensure_pair_arrays(S, np);
  if (first_check && np > 0) {
    S->tpair.ensure(np);
    launch_pair_min_dist2(S->act, np, io.npt, proxy_x(S), S->tpair.p, st);
    launch_min_clamp1(S->tpair.p, np, S->scal.p, S->red_tmp.p, st);
    double dmin2 = read_scalar_d(S, S->scal.p);
    if (!(dmin2 > 0.0)) fail(PDIPC_E_INTERSECTING, "input state has a contact pair at distance 0");
  }
  if (S->opt.kappa_adapt) adapt_kappa(S, first_check, io.npt, np);
  io.kappa = S->kappa;
  {
    ScopedTimer tm(S, TK_BARRIER);
    launch_barrier(S->act, np, io.npt, proxy_x(S), S->opt.dhat, S->kappa, S->opt.barrier_form, fp32, S->bo, st);
  }
  expand_pair_terms(S, np);
  {
    // against the c of the current C^-1: the change of c, and the vertices
    // that left / entered it listed for the incremental update
    int32_t* ids = nullptr;
    if (S->cinv_valid && S->opt.cinv_updates_max > 0) {
      S->cset_ids.ensure(2 * kCinvMaxDelta);
      ids = S->cset_ids.p;
    }
    build_incidence(pair_slots(S), np, S->n, S->fixed.p, S->inc, S->scan_tmp.p, st,
                    S->cinv_valid ? S->prev_cflag.p : nullptr, ids, ids ? ids + kCinvMaxDelta : nullptr,
                    kCinvMaxDelta);
  }
  io.nc_with_same = S->cinv_valid;
  HIPCHK(hipMemcpyAsync(S->h_scal, S->inc.d_nc, sizeof(int32_t) * (io.nc_with_same ? 4 : 1), hipMemcpyDeviceToHost,
                        st));
  HIPCHK(hipEventRecord(S->ev_fork, st));
  io.nc_pending = true;
  stage_mark(S, 1);
  {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    timer_events(S, TK_LOCAL, &e0, &e1);
    launch_local_step(local_args(S), S->x.p, S->Rtet.p, S->Rtet.p, S->E0.p, S->tetg.p, fp32, st, e0, e1);
  }
  launch_gather_vertex_grad(S->n, S->m, S->vt_ptr.p, S->vt_ent.p, S->tetg.p, S->fixed.p, S->g.p, st);
  launch_add_barrier_grad(S->inc, pair_slots(S), np, S->fixed.p, S->g.p, st);
  stage_mark(S, 2);
  if (!defer) finish_readback(S, io);
}

// Mixed path: M u = rhs by iterative refinement with the FP32 factor of the
// Jacobi-scaled M against FP64 residuals, to max|r| <= 1e-13 max|rhs|; false
// if the FP32 factor failed or the steps ran out (then the FP64 factor is
// used).  With the FP32 inverse factor, three steps and the following residual
// are queued and read back once; steps after convergence do nothing.
static constexpr double kRefineTol = 1e-13;
static constexpr int kRefineMaxSteps = 10;

static bool refine_on_inverse(Solver* S, int64_t N3) {
  hipStream_t st = S->st;
  constexpr int kQueued = 3;
  S->refres.ensure(kRefineMaxSteps + 2);
  launch_fill_f64(S->refres.p, kRefineMaxSteps + 2, 0.0, st);
  launch_fill_f64(S->u.p, N3, 0.0, st);
  auto residual = [&](int s) {
    launch_refine_residual(S->Mred.p, N3, S->rhs.p, S->u.p, S->scl.p, S->uf.p, S->refres.p, s, kRefineTol, st);
  };
  auto correct = [&](int s) {
    launch_refine_correct(S->MLf.p, S->MLif.p, N3, S->uf.p, S->scl.p, S->u.p, S->refres.p, s, kRefineTol, st);
  };
  for (int s = 0; s < kQueued; ++s) {
    residual(s);
    correct(s);
  }
  int s = kQueued;
  residual(s);
  while (true) {
    HIPCHK(hipMemcpyAsync(S->h_scal, S->refres.p, sizeof(double) * (s + 1), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(S->h_scal + 12, S->info.p + 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int32_t finfo = 0;
    std::memcpy(&finfo, S->h_scal + 12, sizeof(int32_t));
    if (finfo != 0) return false;
    for (int i = 0; i <= s; ++i)
      if (S->h_scal[i] <= kRefineTol * S->h_scal[0]) {
        S->refine_steps += i;
        return true;
      }
    if (s >= kRefineMaxSteps) {
      S->refine_steps += s;
      return false;
    }
    correct(s);
    ++s;
    residual(s);
  }
}

// Global step of Eq. (4) via Eq. (7) and (11): dx from g.
static void global_step(Solver* S, IterOut& io) {
  hipStream_t st = S->st;
  FactorDev& f = S->fd;
  const int64_t n1x3 = 3LL * f.n1;
  const bool mixed_prec = S->opt.precision == PDIPC_MIXED_FP32;
  // the side stream below starts from the fork event: everything queued on
  // the main stream before this step (the contact terms, C^-1's last users)
  if (!io.nc_pending) HIPCHK(hipEventRecord(S->ev_fork, st));
  // Eq. (7) forward part needs only g.  Its first levels are queued before
  // waiting for n_c, so that the main stream stays busy while the host queues
  // the side stream's work; the rest follows that.
  launch_pack_rhs(f, S->g.p, S->bvec.p, st);
  const int split = std::min(kFwdLevelsBeforeFork, f.nlevels);
  {
    ScopedTimer tm(S, TK_FWD);
    launch_forward_sweep(f, S->bvec.p, S->yvec.p, st, 0, split);
  }
  auto rest_of_forward = [&]() {
    {
      ScopedTimer tm(S, TK_FWD);
      launch_forward_sweep(f, S->bvec.p, S->yvec.p, st, split, -1);
    }
    ScopedTimer tm(S, TK_SIGMA_GEMV);
    launch_sigma_gemv(f, S->yvec.p + n1x3, S->solvec.p + n1x3, st);
  };
  finish_readback(S, io);
  const int32_t np = io.npt + io.nee, nc = io.nc;
  const int64_t N3 = 3LL * nc;
  // FP32 factor of the reduced system with FP64 refinement, or the FP64 factor
  const bool mixed = mixed_prec && N3 >= S->opt.fp32_reduced_min;
  // Contact correction from the stored rows of H_s^-1: the backward sweep then
  // runs on the uncorrected step, before the join, and the correction of all
  // rows is one product after it (taken while that product reads less than
  // kHinvColsBytes; else x2 is corrected first and the sweep follows).
  const int64_t Next = static_cast<int64_t>(f.n1) + f.n2;
  const bool hinv_path = f.hinv_x2 && nc > 0 && static_cast<int64_t>(nc) * Next * 8 <= kHinvColsBytes;
  if (nc > 0) {
    S->c_x2.ensure(nc);
    S->Cs.ensure(static_cast<int64_t>(nc) * nc);
    S->work.ensure(static_cast<int64_t>(nc) * nc);
    S->Mred.ensure(N3 * N3);
    S->CsL.ensure(static_cast<int64_t>(nc) * nc);
    S->CsLi.ensure(dense_aux_size(nc));
    S->ML.ensure(N3 * N3);
    S->MLi.ensure(dense_aux_size(N3));
    S->rhs.ensure(N3);
    S->u.ensure(N3);
    S->vvec.ensure(N3);
    if (mixed) {
      S->Mf.ensure(N3 * N3);
      S->MLf.ensure(N3 * N3);
      S->MLif.ensure(dense_aux_size(N3));
      S->uf.ensure(N3);
      S->resid.ensure(N3);
      S->scl.ensure(N3);
    }
    // The reduced system depends only on the contact terms and C^-1: build and
    // factor it on the side stream while the sweeps run on the main stream.
    hipStream_t sd = S->side;
    bool keep_flags = false;
    HIPCHK(hipStreamWaitEvent(sd, S->ev_fork, 0));
    if (!io.c_same) {
      const int32_t nk = nc - io.c_added;
      const bool incremental = io.nc_with_same && S->cinv_incr_ok && S->cinv_since_full < S->opt.cinv_updates_max &&
                               io.c_removed <= kCinvMaxDelta && io.c_added <= kCinvMaxDelta && nk >= 1 &&
                               nk == S->nc_prev - io.c_removed;
      if (io.nc_with_same) {
        const int32_t delta = io.c_removed + io.c_added;
        S->cinv_rebuilds++;
        S->c_delta_sum += delta;
        S->c_delta_max = std::max(S->c_delta_max, delta);
      }
      // c -> rows of Sigma^-1: on the main stream when only the main stream
      // reads them (the update takes its indices from the vertex map itself)
      launch_c_to_x2(nc, S->inc.clist, S->vert2x2.p, S->c_x2.p, incremental ? st : sd);
      if (incremental) {
        ScopedTimer tm(S, TK_CINV_UPDATE, sd);
        const int32_t r = io.c_removed, a = io.c_added;
        S->cupd_i.ensure(2LL * nk + 2 * kCinvMaxDelta + nc);
        S->cupd_d.ensure(32 * 32 + a * a + static_cast<int64_t>(nk) * (2 * r + 2 * a + nk));
        S->Cinv_next.ensure(static_cast<int64_t>(nc) * nc);
        CinvUpdateArgs u{};
        u.n = S->n; u.nold = S->nc_prev; u.nc = nc; u.r = r; u.a = a; u.n2 = f.n2;
        u.cflag = S->inc.cflag; u.cidx = S->inc.cidx; u.pflag = S->prev_cflag.p; u.pidx = S->prev_cidx.p;
        u.vert2x2 = S->vert2x2.p;
        u.rem_ids = S->cset_ids.p;
        u.add_ids = S->cset_ids.p + kCinvMaxDelta;
        int32_t* ip = S->cupd_i.p;
        u.L.kept_old = ip; ip += nk;
        u.L.kept_x2 = ip; ip += nk;
        u.L.rem_old = ip; ip += kCinvMaxDelta;
        u.L.add_x2 = ip; ip += kCinvMaxDelta;
        u.L.kind = ip;
        u.info = S->info.p + 3;
        u.Ci = S->Cinv.p;
        u.Si = f.sigma_inv;
        double* dp = S->cupd_d.p;
        u.Sinv = dp; dp += 32 * 32;
        u.Sm = dp; dp += a * a;
        u.T = dp; dp += static_cast<int64_t>(nk) * r;
        u.G = dp; dp += static_cast<int64_t>(nk) * r;
        u.W = dp; dp += static_cast<int64_t>(nk) * a;
        u.V = dp; dp += static_cast<int64_t>(nk) * a;
        u.CK = dp;
        u.out = S->Cinv_next.p;
        launch_cinv_update(u, sd);
        std::swap(S->Cinv, S->Cinv_next);
        S->cinv_updates++;
        S->cinv_since_full++;
      } else {
        ScopedTimer tm(S, TK_CINV_FULL, sd);
        S->Cinv.ensure(static_cast<int64_t>(nc) * nc);
        launch_gather_cc(f, nc, S->c_x2.p, S->Cs.p, sd);
        dense_cholesky<double>(S->Cs.p, nc, S->CsL.p, S->CsLi.p, S->info.p + 3, sd);
        dense_chol_inverse<double>(S->CsL.p, S->CsLi.p, nc, S->Cinv.p, S->work.p, sd);
        S->cinv_since_full = 0;
      }
      S->check_info_cs = true;
      S->prev_cflag.ensure(S->n + 1LL);
      S->prev_cidx.ensure(S->n + 1LL);
      keep_flags = true;                // copied on the main stream once C^-1 is ready
      S->nc_prev = nc;
      S->cinv_valid = true;
      io.c_same = true;                 // later solves with this io reuse it
    }
    S->cinv_incr_ok = true;
    HIPCHK(hipEventRecord(S->ev_cinv, sd));          // C^-1 and c_x2 ready
    launch_assemble_reduced(nc, S->Cinv.p, S->inc, pair_slots(S), np, S->Mred.p, sd);
    // The factorisation is queued in two parts with the rest of the main
    // stream's sweep between them, so that neither stream waits for the host.
    const int64_t nlaunch = dense_cholesky_launches(N3);
    const int64_t first_part = std::min<int64_t>(nlaunch, kFactorLaunchesFirst);
    if (mixed) {
      // Jacobi-scaled FP32 copy and its factor (refined against FP64 below)
      launch_jacobi_scaling(S->Mred.p, N3, S->scl.p, sd);
      launch_scale_convert_matrix(S->Mred.p, N3, S->scl.p, S->Mf.p, sd);
      ScopedTimer tm(S, TK_REDUCED_CHOL, sd);
      dense_cholesky_range<float>(S->Mf.p, N3, S->MLf.p, S->MLif.p, S->info.p + 1, sd, 0, first_part);
      rest_of_forward();
      dense_cholesky_range<float>(S->Mf.p, N3, S->MLf.p, S->MLif.p, S->info.p + 1, sd, first_part, nlaunch);
    } else {
      ScopedTimer tm(S, TK_REDUCED_CHOL, sd);
      dense_cholesky_range<double>(S->Mred.p, N3, S->ML.p, S->MLi.p, S->info.p, sd, 0, first_part);
      rest_of_forward();
      dense_cholesky_range<double>(S->Mred.p, N3, S->ML.p, S->MLi.p, S->info.p, sd, first_part, nlaunch);
      S->check_info_m = true;           // read back with the line-search state
    }
    HIPCHK(hipEventRecord(S->ev_join, sd));
    if (hinv_path) {
      ScopedTimer tm(S, TK_BWD);
      launch_backward_sweep(f, S->yvec.p, S->solvec.p, st);
    }
    HIPCHK(hipStreamWaitEvent(st, S->ev_cinv, 0));
    launch_cinv_times_zc(nc, S->Cinv.p, S->c_x2.p, S->solvec.p + n1x3, S->rhs.p, st);
    if (keep_flags) {
      // the flags and ranks of the c that C^-1 now belongs to (the update has
      // read the previous ones: it precedes the C^-1 event)
      HIPCHK(hipMemcpyAsync(S->prev_cflag.p, S->inc.cflag, sizeof(int32_t) * (S->n + 1LL), hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(S->prev_cidx.p, S->inc.cidx, sizeof(int32_t) * (S->n + 1LL), hipMemcpyDeviceToDevice, st));
    }
    HIPCHK(hipStreamWaitEvent(st, S->ev_join, 0));
    bool fallback = false;
    if (mixed) {
      const bool solved = refine_on_inverse(S, N3);
      if (!solved) {
        S->refine_fallbacks++;
        fallback = true;
        {
          ScopedTimer tm(S, TK_REDUCED_CHOL);
          dense_cholesky<double>(S->Mred.p, N3, S->ML.p, S->MLi.p, S->info.p, st);
        }
        S->check_info_m = true;
      }
    }
    if (!mixed || fallback) dense_chol_solve_into<double>(S->ML.p, S->MLi.p, N3, S->rhs.p, S->u.p, st);
    launch_bcheck_apply(nc, S->inc, pair_slots(S), np, S->fixed.p, S->u.p, S->wtmp.p, S->vvec.p, st);
    if (hinv_path) {
      // the x2 rows now; the x1 rows (all but n2 of them) and their unpacking
      // on the second stream, which the line search joins (the CCD before it
      // reads proxy vertices only, all in x2)
      HIPCHK(hipEventRecord(S->ev_rows, st));
      launch_hinv_cols_update_range(f, nc, S->c_x2.p, S->vvec.p, S->solvec.p, f.n1, Next, st);
      HIPCHK(hipStreamWaitEvent(S->side, S->ev_rows, 0));
      launch_hinv_cols_update_range(f, nc, S->c_x2.p, S->vvec.p, S->solvec.p, 0, f.n1, S->side);
      launch_unpack_range(f, 0, f.n1, S->solvec.p, S->dx.p, S->side);
      HIPCHK(hipEventRecord(S->ev_x1, S->side));
      S->x1_pending = true;
      launch_unpack_range(f, f.n1, f.n1 + f.n2, S->solvec.p, S->dx.p, st);
      return;
    }
    launch_sigma_cols_update(f, nc, S->c_x2.p, S->vvec.p, S->solvec.p + n1x3, st);
  } else {
    rest_of_forward();
  }
  if (!hinv_path) {
    ScopedTimer tm(S, TK_BWD);
    launch_backward_sweep(f, S->yvec.p, S->solvec.p, st);
  }
  launch_unpack(f, S->n, S->solvec.p, S->dx.p, st);
}

// The main stream takes the x1 rows of dx from the second stream (queued by a
// global step that corrected them there).
static void join_x1(Solver* S) {
  if (!S->x1_pending) return;
  HIPCHK(hipStreamWaitEvent(S->st, S->ev_x1, 0));
  S->x1_pending = false;
}

// ---- comparison configurations of Table 1 -------------------------------------
// z = H^-1 r through the constant factor with no contact (Eq. 7 with c empty):
// lower sweep, Sigma^-1, upper sweep.  z is written at the free vertices only.
static void pd_factor_solve(Solver* S, const double* r, double* z) {
  hipStream_t st = S->st;
  FactorDev& f = S->fd;
  const int64_t n3 = 3LL * S->n;
  // the right-hand side of the factor solve is -g: pass g = -r
  launch_axpby(n3, -1.0, r, 0.0, S->cg_t.p, st);
  launch_pack_rhs(f, S->cg_t.p, S->bvec.p, st);
  {
    ScopedTimer tm(S, TK_FWD);
    launch_forward_sweep(f, S->bvec.p, S->yvec.p, st);
  }
  {
    ScopedTimer tm(S, TK_SIGMA_GEMV);
    launch_sigma_gemv(f, S->yvec.p + 3LL * f.n1, S->solvec.p + 3LL * f.n1, st);
  }
  {
    ScopedTimer tm(S, TK_BWD);
    launch_backward_sweep(f, S->yvec.p, S->solvec.p, st);
  }
  launch_unpack(f, S->n, S->solvec.p, z, st);
}

// Global step of the conjugate-gradient baseline (Eq. 5): CG on
// (H + kappa B) dx = -g, preconditioned by L L^T = H.  Stops when
// |r| <= cg_tol |g| (free DOFs) or after cg_max_iters products.
static void global_step_pcg(Solver* S, IterOut& io) {
  hipStream_t st = S->st;
  finish_readback(S, io);
  const int32_t np = io.npt + io.nee, nc = io.nc;
  const int64_t n3 = 3LL * S->n;
  for (DBuf<double>* b : {&S->cg_r, &S->cg_z, &S->cg_p, &S->cg_q, &S->cg_t}) b->ensure(n3);
  S->cg_sc.ensure(8);
  if (nc > 0) {
    S->cg_pc.ensure(3LL * nc);
    S->cg_vc.ensure(3LL * nc);
  }
  // the preconditioner writes z at the free vertices only: the rest stays 0
  launch_fill_f64(S->cg_z.p, n3, 0.0, st);
  launch_fill_f64(S->dx.p, n3, 0.0, st);
  launch_axpby(n3, -1.0, S->g.p, 0.0, S->cg_r.p, st);            // r = b = -g
  auto dot = [&](const double* a, const double* b, int slot) {
    launch_masked_mul(S->n, a, b, S->fixed.p, S->prod.p, st);
    launch_sum(S->prod.p, n3, S->cg_sc.p + slot, S->red_tmp.p, st);
  };
  auto apply = [&](const double* p, double* q) {                 // q = (H + kappa B) p
    launch_pd_matvec(local_args(S), S->n, S->vt_ptr.p, S->vt_ent.p, S->fixed.p, p, S->tetg.p, q, st);
    if (nc > 0 && np > 0) {
      launch_gather_c(nc, S->inc.clist, p, S->cg_pc.p, st);
      launch_bcheck_apply(nc, S->inc, pair_slots(S), np, S->fixed.p, S->cg_pc.p, S->wtmp.p, S->cg_vc.p, st);
      launch_scatter_add_c(nc, S->inc.clist, S->cg_vc.p, q, st);
    }
  };
  S->prod.ensure(n3);
  dot(S->cg_r.p, S->cg_r.p, 0);
  const double bn = std::sqrt(read_scalar_d(S, S->cg_sc.p + 0));
  int it = 0;
  if (bn > 0.0) {
    const double tol = S->opt.cg_tol * bn;
    pd_factor_solve(S, S->cg_r.p, S->cg_z.p);
    HIPCHK(hipMemcpyAsync(S->cg_p.p, S->cg_z.p, sizeof(double) * n3, hipMemcpyDeviceToDevice, st));
    int rz = 1, rz_new = 4;
    dot(S->cg_r.p, S->cg_z.p, rz);
    while (it < S->opt.cg_max_iters) {
      apply(S->cg_p.p, S->cg_q.p);
      dot(S->cg_p.p, S->cg_q.p, 2);
      launch_cg_step(n3, S->cg_sc.p, rz, 2, S->cg_p.p, S->cg_q.p, S->dx.p, S->cg_r.p, st);
      ++it;
      dot(S->cg_r.p, S->cg_r.p, 3);
      if (std::sqrt(read_scalar_d(S, S->cg_sc.p + 3)) <= tol) break;
      pd_factor_solve(S, S->cg_r.p, S->cg_z.p);
      dot(S->cg_r.p, S->cg_z.p, rz_new);
      launch_cg_dir(n3, S->cg_sc.p, rz_new, rz, S->cg_z.p, S->cg_p.p, st);
      std::swap(rz, rz_new);
    }
  }
  io.cg_iters = it;
}

// Global step with the Schur complement only (Section 3.1): the lower sweep
// gives y1 and r2, the dense Sigma-hat = Sigma_s (x) I3 + kappa B_22 (3 n2
// unknowns) is assembled and factored every iteration, dx2 = Sigma-hat^-1 r2,
// and the upper sweep gives dx1 (Eq. 7 with Sigma-hat in place of Sigma).
static void global_step_schur(Solver* S, IterOut& io) {
  hipStream_t st = S->st;
  FactorDev& f = S->fd;
  finish_readback(S, io);
  const int32_t np = io.npt + io.nee, nc = io.nc;
  const int64_t n1x3 = 3LL * f.n1, N2 = 3LL * f.n2;
  launch_pack_rhs(f, S->g.p, S->bvec.p, st);
  {
    ScopedTimer tm(S, TK_FWD);
    launch_forward_sweep(f, S->bvec.p, S->yvec.p, st);
  }
  if (N2 > 0) {
    S->shat.ensure(N2 * N2);
    S->shat_L.ensure(N2 * N2);
    S->shat_aux.ensure(dense_aux_size(N2));
    launch_kron_i3(f.n2, S->sigma_s.p, S->shat.p, st);
    if (nc > 0 && np > 0) {
      // kappa B on the contact vertices (3 n_c square, from the pair factors),
      // added at their x2 rows and columns
      S->Cs.ensure(static_cast<int64_t>(nc) * nc);
      S->Mred.ensure(9LL * nc * nc);
      S->c_x2.ensure(nc);
      launch_fill_f64(S->Cs.p, static_cast<int64_t>(nc) * nc, 0.0, st);
      launch_assemble_reduced(nc, S->Cs.p, S->inc, pair_slots(S), np, S->Mred.p, st);
      launch_c_to_x2(nc, S->inc.clist, S->vert2x2.p, S->c_x2.p, st);
      launch_scatter_block(nc, S->c_x2.p, S->Mred.p, f.n2, S->shat.p, st);
    }
    {
      ScopedTimer tm(S, TK_REDUCED_CHOL);
      dense_cholesky<double>(S->shat.p, N2, S->shat_L.p, S->shat_aux.p, S->info.p + 4, st);
    }
    if (read_scalar_i(S, S->info.p + 4) != 0) fail(PDIPC_E_NOT_SPD, "Schur complement with contact not SPD");
    // r2 (n2 x 3, vertex-major) -> dx2 in the x2 part of the solution
    HIPCHK(hipMemcpyAsync(S->solvec.p + n1x3, S->yvec.p + n1x3, sizeof(double) * N2, hipMemcpyDeviceToDevice, st));
    dense_chol_solve<double>(S->shat_L.p, S->shat_aux.p, N2, S->solvec.p + n1x3, 1, st);
  }
  {
    ScopedTimer tm(S, TK_BWD);
    launch_backward_sweep(f, S->yvec.p, S->solvec.p, st);
  }
  launch_unpack(f, S->n, S->solvec.p, S->dx.p, st);
}

static void global_step_method(Solver* S, IterOut& io) {
  switch (S->opt.global_method) {
    case PDIPC_GSTEP_PCG: global_step_pcg(S, io); break;
    case PDIPC_GSTEP_SCHUR: global_step_schur(S, io); break;
    default: global_step(S, io); break;
  }
}

// Statuses of the reduced factorisations queued since the last check.
static void check_factor_status(Solver* S) {
  if (!S->check_info_m && !S->check_info_cs) return;
  int32_t hinfo[4] = {0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(S->h_scal, S->info.p, sizeof(int32_t) * 4, hipMemcpyDeviceToHost, S->st));
  HIPCHK(hipStreamSynchronize(S->st));
  std::memcpy(hinfo, S->h_scal, sizeof(hinfo));
  const bool bad_m = S->check_info_m && hinfo[0] != 0, bad_cs = S->check_info_cs && hinfo[3] != 0;
  S->check_info_m = S->check_info_cs = false;
  if (bad_m) fail(PDIPC_E_NOT_SPD, "reduced contact system not SPD");
  if (bad_cs) fail(PDIPC_E_NOT_SPD, "contact block of the inverse Schur complement not SPD");
}

// CCD bound and back-tracking line search; updates x.
static void step_and_search(Solver* S, IterOut& io, bool apply) {
  hipStream_t st = S->st;
  const bool fp32 = S->opt.precision == PDIPC_MIXED_FP32;
  int32_t cpt = 0, cee = 0;
  update_proxy_step(S);
  pairs(S, false, proxy_x(S), proxy_dx(S), &cpt, &cee);
  const int32_t ncand = cpt + cee;
  io.ncand = ncand;
  S->cand_n = ncand;
  S->cand_pt = cpt;
  S->cand_valid = apply;
  S->tpair.ensure(std::max(ncand, 1));
  S->bE0.ensure(std::max(ncand, 1));
  S->bdE.ensure(std::max(ncand, 1));
  S->ccd_part.ensure(std::max<int64_t>((ncand + 255) / 256, 1));
  int nccd = 0;
  {
    ScopedTimer tm(S, TK_CCD);
    // with the candidates' barrier energies at x, the line search's reference
    nccd = launch_ccd(S->cand, ncand, cpt, proxy_x(S), proxy_dx(S), S->opt.ccd_eta, S->opt.ccd_steps, S->tpair.p,
                      S->ccd_part.p, st, S->opt.dhat, S->kappa, S->opt.barrier_form, S->bE0.p);
  }
  // back-tracking line search on the device: trials read alpha from the state
  // and become no-ops once it is decided; one is queued, then one readback
  // (the first trial is accepted in nearly every iteration: 4 halvings in 240
  // on the 50k face, so a second queued trial costs more than its round trip)
  stage_mark(S, 4);
  join_x1(S);                          // the trials read dx everywhere
  double* ls = S->lsbuf.p;
  launch_ls_init(ls, S->ccd_part.p, nccd, st);
  auto trial = [&]() {
    {
      ScopedTimer tm(S, TK_TRIAL);
      launch_trial_energy(local_args(S), S->x.p, S->dx.p, ls, S->Rtet.p, S->E0.p, S->dE.p, fp32, st);
    }
    launch_pair_barrier_energy(S->cand, ncand, cpt, proxy_x(S), proxy_dx(S), ls, S->opt.dhat, S->kappa,
                               S->opt.barrier_form,
                               S->bE0.p, S->bdE.p, st);
    launch_sum2_decide(S->dE.p, S->m, S->bdE.p, ncand, ls, S->red_tmp.p, S->opt.ls_max_halvings, st);
  };
  const int queued = 1;
  for (int h = 0; h < queued; ++h) trial();
  // x += alpha dx is applied by the device once the search has accepted, so it
  // is queued before the readback; a search still open repeats it below
  if (apply) launch_axpy_ls(3LL * S->n, ls, S->dx.p, S->x.p, st);
  double hls[LS_SIZE];
  int32_t hinfo[4] = {0, 0, 0, 0};
  auto readback = [&]() {
    HIPCHK(hipMemcpyAsync(S->h_scal, ls, sizeof(double) * LS_SIZE, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(S->h_scal + LS_SIZE, S->info.p, sizeof(int32_t) * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::memcpy(hls, S->h_scal, sizeof(double) * LS_SIZE);
    std::memcpy(hinfo, S->h_scal + LS_SIZE, sizeof(int32_t) * 4);
  };
  stage_mark(S, 5);
  readback();
  if (S->check_info_m && hinfo[0] != 0) fail(PDIPC_E_NOT_SPD, "reduced contact system not SPD");
  if (S->check_info_cs && hinfo[3] != 0) fail(PDIPC_E_NOT_SPD, "contact block of the inverse Schur complement not SPD");
  S->check_info_m = S->check_info_cs = false;
  bool reopened = false;
  while (hls[LS_STATE] == 0.0) {
    reopened = true;
    trial();
    readback();
  }
  io.alpha_m = hls[LS_ALPHA_M];
  io.halvings = static_cast<int32_t>(hls[LS_HALVINGS]);
  io.ls_ok = hls[LS_STATE] == 1.0;
  io.alpha = io.ls_ok ? hls[LS_ALPHA] : 0.0;
  if (apply && reopened && io.alpha > 0.0) launch_axpy_ls(3LL * S->n, ls, S->dx.p, S->x.p, st);
  if (reopened && S->stage_on) {
    stage_mark(S, 5);
    HIPCHK(hipEventSynchronize(S->sev[5]));
  }
}

static int32_t do_solve_frame(Solver* S, const double* x_in, double* x_out, pdipc_frame_stats* stats) {
  if (!S->have_actuation) fail(PDIPC_E_INVALID, "no actuation set");
  if (!x_in || !x_out) fail(PDIPC_E_INVALID, "null state pointer");
  hipStream_t st = S->st;
  auto t0 = std::chrono::steady_clock::now();
  HIPCHK(hipMemcpyAsync(S->x.p, x_in, sizeof(double) * 3 * S->n, hipMemcpyDeviceToDevice, st));
  S->cand_valid = false;
  S->check_info_m = S->check_info_cs = false;
  // the local steps of a frame start from the identity, so a frame does not
  // depend on earlier calls
  launch_identity_rotations(S->m, S->Rtet.p, st);
  cinv_begin_pass(S);
  launch_count_nonfinite(S->x.p, 3LL * S->n, S->info.p + 2, st);
  if (read_scalar_i(S, S->info.p + 2) != 0) fail(PDIPC_E_INVALID, "non-finite input state");
  pdipc_frame_stats fs{};
  fs.alpha_m_min = 1.0;
  fs.alpha_min = 1.0;
  int32_t rc = PDIPC_OK;
  const bool tol_mode = S->opt.tol > 0;
  double tms[5] = {0, 0, 0, 0, 0};
  S->stage_on = stats != nullptr;
  S->trace.clear();
  S->refine_steps = 0;
  S->refine_fallbacks = 0;
  S->cinv_rebuilds = S->c_delta_max = S->c_delta_sum = S->cinv_updates = 0;
  int it = 0;
  for (; it < S->opt.iters; ++it) {
    IterOut io;
    const int32_t refine_before = S->refine_steps;
    stage_mark(S, 0);
    assemble_gradient(S, it == 0, io, /*defer=*/true);
    global_step_method(S, io);
    stage_mark(S, 3);
    step_and_search(S, io, true);
    if (S->stage_on) {
      // the line-search readback has synchronised past every stage event
      for (int k = 0; k < 5; ++k) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, S->sev[k], S->sev[k + 1]));
        tms[k] += ms;
      }
    }
    HIPCHK(hipGetLastError());
    {
      pdipc_iter_trace tr{};
      tr.n_pt = io.npt; tr.n_ee = io.nee; tr.n_c = io.nc; tr.n_candidates = io.ncand;
      tr.ls_halvings = io.halvings; tr.ls_ok = io.ls_ok ? 1 : 0; tr.near_ties = io.near_ties;
      tr.refine_steps = S->refine_steps - refine_before;
      tr.cg_iters = io.cg_iters;
      tr.alpha_m = io.alpha_m; tr.alpha = io.alpha; tr.kappa = io.kappa;
      S->trace.push_back(tr);
    }
    fs.near_ties += io.near_ties;
    fs.pcg_iters += io.cg_iters;
    if (S->timer_which >= 0) {
      HIPCHK(hipStreamSynchronize(st));
      harvest_timer(S);
    }
    fs.n_pt = io.npt;
    fs.n_ee = io.nee;
    fs.n_c = std::max(fs.n_c, io.nc);
    fs.n_candidates = io.ncand;
    fs.ls_halvings += io.halvings;
    if (!io.ls_ok) { fs.ls_failures++; rc = PDIPC_W_LS_FAILED; }
    fs.alpha_m_min = std::min(fs.alpha_m_min, io.alpha_m);
    fs.alpha_min = std::min(fs.alpha_min, io.alpha);
    if (tol_mode) {
      launch_max_abs(S->dx.p, 3LL * S->n, S->scal.p + 2, S->red_tmp.p, st);
      // converged when the full direction (before the line search) is small
      double step = read_scalar_d(S, S->scal.p + 2);
      if (step <= S->opt.tol) { ++it; break; }
    }
  }
  fs.iters = it;
  fs.refine_steps = S->refine_steps;
  fs.refine_fallbacks = S->refine_fallbacks;
  fs.cinv_rebuilds = S->cinv_rebuilds;
  fs.c_delta_max = S->c_delta_max;
  fs.c_delta_sum = S->c_delta_sum;
  fs.cinv_updates = S->cinv_updates;
  if (tol_mode && it >= S->opt.iters && rc == PDIPC_OK) rc = PDIPC_W_NOT_CONVERGED;
  HIPCHK(hipMemcpyAsync(x_out, S->x.p, sizeof(double) * 3 * S->n, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  S->have_solution = true;
  auto t1 = std::chrono::steady_clock::now();
  S->stage_on = false;
  if (stats) {
    // Table 1 columns: IPC, Misc (local step, gradient assembly and the
    // frame's own copies and checks), G-Step, CCD, LS
    fs.ms_total = std::chrono::duration<double, std::milli>(t1 - t0).count();
    fs.ms_ipc = tms[0];
    fs.ms_gstep = tms[2];
    fs.ms_ccd = tms[3];
    fs.ms_ls = tms[4];
    fs.ms_misc = fs.ms_total - tms[0] - tms[2] - tms[3] - tms[4];
    *stats = fs;
  }
  return rc;
}

// Adjoint of the last frame: K lambda = dL/dx by conjugate gradients
// preconditioned with the forward global step (H + projected barrier Hessian,
// Eq. 7 and 11), then dL/da from lambda.
static int32_t do_backward(Solver* S, const double* dLdx, double* dLda) {
  if (!S->have_solution) fail(PDIPC_E_INVALID, "no converged frame to differentiate");
  if (S->embed) fail(PDIPC_E_INVALID, "the adjoint supports a proxy embedded by selection only");
  if (!S->have_scalar) fail(PDIPC_E_INVALID, "the actuation was not set through pdipc_set_actuation_scalar");
  hipStream_t st = S->st;
  const int64_t n3 = 3LL * S->n;
  IterOut io;
  S->cand_valid = false;
  launch_identity_rotations(S->m, S->Rtet.p, st);   // same rotations whatever ran before
  cinv_begin_pass(S);
  // the energy of the last frame: its final barrier stiffness, not a new balance
  const int32_t adapt = S->opt.kappa_adapt;
  S->opt.kappa_adapt = 0;
  assemble_gradient(S, true, io);                   // rotations, pairs, barrier factors at x*
  S->opt.kappa_adapt = adapt;
  const int32_t np = io.npt + io.nee;
  S->lam.ensure(n3); S->res.ensure(n3); S->zvec.ensure(n3); S->pvec.ensure(n3); S->kp.ensure(n3);
  S->prod.ensure(n3);
  S->pairbuf.ensure(12LL * std::max(np, 1));
  launch_fill_f64(S->lam.p, n3, 0.0, st);
  launch_masked_mul(S->n, dLdx, dLdx, S->fixed.p, S->prod.p, st);   // |b|^2
  launch_sum(S->prod.p, n3, S->scal.p + 3, S->red_tmp.p, st);
  const double bn = std::sqrt(read_scalar_d(S, S->scal.p + 3));
  if (bn == 0.0) {
    launch_fill_f64(dLda, S->m, 0.0, st);
    HIPCHK(hipStreamSynchronize(st));
    return PDIPC_OK;
  }
  // r = b (free DOFs only)
  HIPCHK(hipMemcpyAsync(S->res.p, dLdx, sizeof(double) * n3, hipMemcpyDeviceToDevice, st));
  launch_masked_mul(S->n, S->res.p, S->res.p, S->fixed.p, S->prod.p, st);
  auto precond = [&](const double* r, double* z) {
    launch_axpby(n3, -1.0, r, 0.0, S->g.p, st);     // g = -r  =>  dx = Hhat^-1 r
    global_step(S, io);
    join_x1(S);
    HIPCHK(hipMemcpyAsync(z, S->dx.p, sizeof(double) * n3, hipMemcpyDeviceToDevice, st));
  };
  auto dot = [&](const double* a, const double* b) {
    launch_masked_mul(S->n, a, b, S->fixed.p, S->prod.p, st);
    launch_sum(S->prod.p, n3, S->scal.p + 4, S->red_tmp.p, st);
    return read_scalar_d(S, S->scal.p + 4);
  };
  auto kvec = [&](const double* v, double* out) {
    launch_hessvec(local_args(S), S->n, S->vt_ptr.p, S->vt_ent.p, S->fixed.p, S->x.p, S->Rtet.p, v, S->tetg.p,
                   S->act, np, io.npt, S->inc, S->px, S->opt.dhat, S->kappa, S->opt.barrier_form, S->pairbuf.p,
                   out, st);
  };
  precond(S->res.p, S->zvec.p);
  HIPCHK(hipMemcpyAsync(S->pvec.p, S->zvec.p, sizeof(double) * n3, hipMemcpyDeviceToDevice, st));
  double rz = dot(S->res.p, S->zvec.p);
  int it = 0;
  const int max_it = 500;
  const double tol = 1e-12;
  for (; it < max_it; ++it) {
    kvec(S->pvec.p, S->kp.p);
    const double pkp = dot(S->pvec.p, S->kp.p);
    if (!(pkp > 0.0)) fail(PDIPC_E_NOT_SPD, "energy Hessian is not positive definite at the frame's state");
    const double alpha = rz / pkp;
    launch_axpby(n3, alpha, S->pvec.p, 1.0, S->lam.p, st);
    launch_axpby(n3, -alpha, S->kp.p, 1.0, S->res.p, st);
    const double rn = std::sqrt(dot(S->res.p, S->res.p));
    if (rn <= tol * bn) { ++it; break; }
    precond(S->res.p, S->zvec.p);
    const double rz2 = dot(S->res.p, S->zvec.p);
    launch_axpby(n3, 1.0, S->zvec.p, rz2 / rz, S->pvec.p, st);
    rz = rz2;
  }
  S->adjoint_iters = it;
  check_factor_status(S);
  launch_actuation_grad(local_args(S), S->x.p, S->Rtet.p, S->R0.p, S->lam.p, dLda, st);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return it >= max_it ? PDIPC_W_NOT_CONVERGED : PDIPC_OK;
}

}  // namespace pdipc

using namespace pdipc;

template <typename F>
static int32_t guarded(Solver* S, F&& fn) {
  BytesScope scope(S ? &S->device_bytes : nullptr);
  try {
    return fn();
  } catch (const SolverError& e) {
    if (S) S->err = e.msg;
    return e.code;
  } catch (const HipFailure& e) {
    if (S) S->err = e.msg;
    return PDIPC_E_HIP;
  } catch (const std::bad_alloc&) {
    if (S) S->err = "host allocation failed";
    return PDIPC_E_NOMEM;
  } catch (...) {
    if (S) S->err = "unexpected exception";
    return PDIPC_E_INVALID;
  }
}

extern "C" {

void pdipc_default_options(pdipc_options* o) {
  if (!o) return;
  o->dhat = 5e-4;
  o->kappa = 1e3;
  o->iters = 30;
  o->tol = 0.0;
  o->precision = PDIPC_FP64;
  o->ccd_eta = 0.1;
  o->ccd_steps = 16;
  o->ls_max_halvings = 20;
  o->cinv_updates_max = 16;
  o->fp32_reduced_min = 8192;
  o->hinv_rows_mb = 4096;
  o->stream = nullptr;
  o->global_method = PDIPC_GSTEP_SCHUR_WOODBURY;
  o->cg_tol = 1e-12;
  o->cg_max_iters = 2000;
  o->barrier_form = 0;
  o->kappa_adapt = 0;
}

int32_t pdipc_init_mesh(const pdipc_mesh_desc* mesh, const pdipc_options* opt, void** out) {
  if (!out) return PDIPC_E_INVALID;
  *out = nullptr;
  Solver* S = nullptr;
  try {
    S = new Solver();
  } catch (...) {
    g_last_init_error = "host allocation failed";
    return PDIPC_E_NOMEM;
  }
  int32_t rc = guarded(S, [&] { return do_init(mesh, opt, S); });
  if (rc != PDIPC_OK) {
    g_last_init_error = S->err;
    delete S;
    return rc;
  }
  *out = S;
  return PDIPC_OK;
}

int32_t pdipc_set_actuation(void* h, const double* A) {
  Solver* S = static_cast<Solver*>(h);
  if (!S || !A) return PDIPC_E_INVALID;
  return guarded(S, [&] {
    launch_count_nonfinite(A, 6LL * S->m, S->info.p + 2, S->st);
    if (read_scalar_i(S, S->info.p + 2) != 0) fail(PDIPC_E_INVALID, "non-finite actuation");
    launch_actuation_transpose(S->m, A, S->A.p, S->st);
    HIPCHK(hipStreamSynchronize(S->st));
    S->have_actuation = true;
    S->have_scalar = false;
    return PDIPC_OK;
  });
}

int32_t pdipc_set_actuation_scalar(void* h, const double* a, const double* R) {
  Solver* S = static_cast<Solver*>(h);
  if (!S || !a) return PDIPC_E_INVALID;
  return guarded(S, [&] {
    if (!R && !S->have_scalar) fail(PDIPC_E_INVALID, "no actuation frames given yet");
    launch_count_nonfinite(a, S->m, S->info.p + 2, S->st);
    if (read_scalar_i(S, S->info.p + 2) != 0) fail(PDIPC_E_INVALID, "non-finite actuation strength");
    if (R) {
      launch_count_nonfinite(R, 9LL * S->m, S->info.p + 2, S->st);
      if (read_scalar_i(S, S->info.p + 2) != 0) fail(PDIPC_E_INVALID, "non-finite actuation frame");
    }
    HIPCHK(hipMemcpyAsync(S->a_s.p, a, sizeof(double) * S->m, hipMemcpyDeviceToDevice, S->st));
    if (R) HIPCHK(hipMemcpyAsync(S->R0.p, R, sizeof(double) * 9 * S->m, hipMemcpyDeviceToDevice, S->st));
    launch_actuation_scalar(S->m, S->a_s.p, S->R0.p, S->A.p, S->st);
    HIPCHK(hipStreamSynchronize(S->st));
    S->have_actuation = true;
    S->have_scalar = true;
    return PDIPC_OK;
  });
}

int32_t pdipc_solve_frame(void* h, const double* x_in, double* x_out, pdipc_frame_stats* stats) {
  Solver* S = static_cast<Solver*>(h);
  if (!S) return PDIPC_E_INVALID;
  return guarded(S, [&] { return do_solve_frame(S, x_in, x_out, stats); });
}

int32_t pdipc_solve_frame_backward(void* h, const double* dL_dx, double* dL_da) {
  Solver* S = static_cast<Solver*>(h);
  if (!S || !dL_dx || !dL_da) return PDIPC_E_INVALID;
  return guarded(S, [&] { return do_backward(S, dL_dx, dL_da); });
}

int32_t pdipc_device_bytes(const void* h, int64_t* bytes) {
  const Solver* S = static_cast<const Solver*>(h);
  if (!S || !bytes) return PDIPC_E_INVALID;
  *bytes = S->device_bytes;
  return PDIPC_OK;
}

int32_t pdipc_get_sizes(const void* h, int64_t* n1, int64_t* n2, int64_t* nnz) {
  const Solver* S = static_cast<const Solver*>(h);
  if (!S) return PDIPC_E_INVALID;
  if (n1) *n1 = S->n1;
  if (n2) *n2 = S->n2;
  if (nnz) *nnz = S->factor_nnz;
  return PDIPC_OK;
}

void pdipc_destroy(void* h) {
  Solver* S = static_cast<Solver*>(h);
  if (!S) return;
  if (S->st) (void)hipStreamSynchronize(S->st);
  DBuf<int32_t>* bi[] = {&S->tets, &S->vt_ptr, &S->vt_ent, &S->sv, &S->stri, &S->sedge, &S->node_c0, &S->node_s,
                         &S->node_r, &S->level_nodes, &S->frows, &S->fcol, &S->ext2vert, &S->vert2x2, &S->lvl_rows, &S->lvl_row_node, &S->t_count,
                         &S->t_cursor, &S->t_id, &S->e_count, &S->e_cursor, &S->e_id, &S->q_count, &S->qbuf, &S->totals, &S->tmpj,
                         &S->act_type, &S->act_i, &S->act_j, &S->act_v4, &S->cand_type, &S->cand_i, &S->cand_j,
                         &S->cand_v4, &S->inc_cnt, &S->inc_ptr, &S->inc_cursor, &S->inc_ent, &S->inc_raw, &S->inc_cflag,
                         &S->inc_cidx, &S->inc_clist, &S->inc_nc, &S->c_x2, &S->info, &S->cflagbuf, &S->cposbuf};
  for (auto* b : bi) b->release();
  DBuf<double>* bd[] = {&S->Bm, &S->w, &S->A, &S->a_s, &S->R0, &S->X, &S->x, &S->g, &S->dx, &S->tetg, &S->E0,
                        &S->dE, &S->Rtet, &S->tpair, &S->bE0, &S->bdE, &S->scal, &S->panelT, &S->dinv, &S->dinvT,
                        &S->fval, &S->sigma_inv, &S->hinv_x2, &S->bvec, &S->yvec, &S->solvec, &S->vbox, &S->tbox, &S->ebox,
                        &S->params, &S->b_energy, &S->b_grad, &S->b_U, &S->Cs, &S->Cinv, &S->work, &S->Mred,
                        &S->rhs, &S->u, &S->vvec, &S->wtmp, &S->resid};
  for (auto* b : bd) b->release();
  S->fixed.release();
  S->node_roff.release(); S->node_poff.release(); S->node_doff.release(); S->fptr.release();
  S->t_key.release(); S->e_key.release(); S->scan_tmp.release(); S->red_tmp.release();
  S->Mf.release(); S->uf.release(); S->MLf.release(); S->MLif.release();
  S->lam.release(); S->res.release(); S->zvec.release(); S->pvec.release(); S->kp.release(); S->prod.release();
  S->pairbuf.release();
  S->CsL.release(); S->CsLi.release(); S->ML.release(); S->MLi.release(); S->scl.release();
  S->prev_cflag.release();
  S->prev_cidx.release(); S->cupd_i.release(); S->Cinv_next.release(); S->cupd_d.release(); S->cset_ids.release();
  S->lsbuf.release();
  S->refres.release();
  S->ccd_part.release();
  delete S;
}

int32_t pdipc_kernel_timer(void* h, int32_t which, double* total_ms, int64_t* launches) {
  Solver* S = static_cast<Solver*>(h);
  if (!S) return PDIPC_E_INVALID;
  if (total_ms) *total_ms = S->timer_ms;
  if (launches) *launches = S->timer_count;
  S->timer_which = which;
  S->timer_ms = 0.0;
  S->timer_count = 0;
  S->ev_used = 0;
  return PDIPC_OK;
}

int32_t pdipc_debug_trace(const void* h, pdipc_iter_trace* out, int32_t cap, int32_t* count) {
  const Solver* S = static_cast<const Solver*>(h);
  if (!S || cap < 0 || (cap > 0 && !out)) return PDIPC_E_INVALID;
  const int32_t k = static_cast<int32_t>(S->trace.size());
  for (int32_t i = 0; i < std::min(k, cap); ++i) out[i] = S->trace[i];
  if (count) *count = k;
  return PDIPC_OK;
}

const char* pdipc_last_error(const void* h) {
  const Solver* S = static_cast<const Solver*>(h);
  return S ? S->err.c_str() : g_last_init_error.c_str();
}

int32_t pdipc_debug_local(void* h, const double* x, double* R, double* energies, double* grad) {
  Solver* S = static_cast<Solver*>(h);
  if (!S || !x) return PDIPC_E_INVALID;
  return guarded(S, [&] {
    if (!S->have_actuation) fail(PDIPC_E_INVALID, "no actuation set");
    const bool fp32 = S->opt.precision == PDIPC_MIXED_FP32;
    launch_identity_rotations(S->m, S->Rtet.p, S->st);
    launch_local_step(local_args(S), x, S->Rtet.p, S->Rtet.p, S->E0.p, S->tetg.p, fp32, S->st);
    launch_gather_vertex_grad(S->n, S->m, S->vt_ptr.p, S->vt_ent.p, S->tetg.p, S->fixed.p, S->g.p, S->st);
    if (R) {
      // SoA 9 x m -> m x 9 through the host (debug path)
      std::vector<double> h9(9LL * S->m), o9(9LL * S->m);
      HIPCHK(hipMemcpyAsync(h9.data(), S->Rtet.p, sizeof(double) * 9 * S->m, hipMemcpyDeviceToHost, S->st));
      HIPCHK(hipStreamSynchronize(S->st));
      for (int64_t i = 0; i < S->m; ++i)
        for (int e = 0; e < 9; ++e) o9[9 * i + e] = h9[e * S->m + i];
      HIPCHK(hipMemcpyAsync(R, o9.data(), sizeof(double) * 9 * S->m, hipMemcpyHostToDevice, S->st));
    }
    if (energies) HIPCHK(hipMemcpyAsync(energies, S->E0.p, sizeof(double) * S->m, hipMemcpyDeviceToDevice, S->st));
    if (grad) HIPCHK(hipMemcpyAsync(grad, S->g.p, sizeof(double) * 3 * S->n, hipMemcpyDeviceToDevice, S->st));
    HIPCHK(hipStreamSynchronize(S->st));
    return PDIPC_OK;
  });
}

int32_t pdipc_debug_contacts(void* h, const double* x, int32_t* out, int32_t cap, int32_t* count) {
  Solver* S = static_cast<Solver*>(h);
  if (!S || !x || !count) return PDIPC_E_INVALID;
  return guarded(S, [&] {
    int32_t npt = 0, nee = 0;
    S->cand_valid = false;
    update_proxy_positions(S, x);
    pairs(S, true, S->embed ? S->spos.p : x, nullptr, &npt, &nee);
    const int32_t np = npt + nee;
    *count = np;
    if (out && np > 0) {
      std::vector<int32_t> ty(np), ii(np), jj(np), o(3LL * np);
      HIPCHK(hipMemcpyAsync(ty.data(), S->act.type, sizeof(int32_t) * np, hipMemcpyDeviceToHost, S->st));
      HIPCHK(hipMemcpyAsync(ii.data(), S->act.i, sizeof(int32_t) * np, hipMemcpyDeviceToHost, S->st));
      HIPCHK(hipMemcpyAsync(jj.data(), S->act.j, sizeof(int32_t) * np, hipMemcpyDeviceToHost, S->st));
      HIPCHK(hipStreamSynchronize(S->st));
      const int32_t k = std::min(np, cap);
      for (int32_t p = 0; p < k; ++p) { o[3 * p] = ty[p]; o[3 * p + 1] = ii[p]; o[3 * p + 2] = jj[p]; }
      if (k > 0) HIPCHK(hipMemcpyAsync(out, o.data(), sizeof(int32_t) * 3 * k, hipMemcpyHostToDevice, S->st));
      HIPCHK(hipStreamSynchronize(S->st));
    }
    return PDIPC_OK;
  });
}

int32_t pdipc_debug_step(void* h, const double* x, double* dx, double* alpha_m, double* alpha) {
  Solver* S = static_cast<Solver*>(h);
  if (!S || !x) return PDIPC_E_INVALID;
  return guarded(S, [&] {
    if (!S->have_actuation) fail(PDIPC_E_INVALID, "no actuation set");
    HIPCHK(hipMemcpyAsync(S->x.p, x, sizeof(double) * 3 * S->n, hipMemcpyDeviceToDevice, S->st));
    S->cand_valid = false;
    launch_identity_rotations(S->m, S->Rtet.p, S->st);
    cinv_begin_pass(S);
    IterOut io;
    assemble_gradient(S, true, io);
    global_step_method(S, io);
    step_and_search(S, io, false);
    if (dx) HIPCHK(hipMemcpyAsync(dx, S->dx.p, sizeof(double) * 3 * S->n, hipMemcpyDeviceToDevice, S->st));
    HIPCHK(hipStreamSynchronize(S->st));
    if (alpha_m) *alpha_m = io.alpha_m;
    if (alpha) *alpha = io.alpha;
    return PDIPC_OK;
  });
}

// Dense SPD kernels on caller data (device): factor A (n x n, preserved), solve
// A x = b in place (b: n x nrhs), and write A^-1 if Ainv is not NULL.
// precision 1 runs the FP32 kernels on a rounded copy.  Test tap.
int32_t pdipc_debug_dense(const double* A, int64_t n, double* b, int32_t nrhs, double* Ainv, int32_t precision) {
  if (!A || n <= 0 || nrhs < 0 || nrhs > 4) return PDIPC_E_INVALID;
  try {
    hipStream_t st = nullptr;
    const int64_t nn = n * n;
    DBuf<int32_t> info;
    info.ensure(1);
    int32_t hinfo = 0;
    if (precision == 0) {
      DBuf<double> W, L, Li, wk;
      W.ensure(nn); L.ensure(nn); Li.ensure(dense_aux_size(n)); wk.ensure(nn);
      HIPCHK(hipMemcpyAsync(W.p, A, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
      dense_cholesky<double>(W.p, n, L.p, Li.p, info.p, st);
      if (b && nrhs > 0) dense_chol_solve<double>(L.p, Li.p, n, b, nrhs, st);
      if (Ainv) dense_chol_inverse<double>(L.p, Li.p, n, Ainv, wk.p, st);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(&hinfo, info.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      W.release(); L.release(); Li.release(); wk.release();
    } else {
      DBuf<float> W, L, Li, wk, bf, invf;
      W.ensure(nn); L.ensure(nn); Li.ensure(dense_aux_size(n)); wk.ensure(nn);
      launch_convert_f64_f32(A, W.p, nn, st);
      dense_cholesky<float>(W.p, n, L.p, Li.p, info.p, st);
      if (b && nrhs > 0) {
        bf.ensure(n * nrhs);
        launch_convert_f64_f32(b, bf.p, n * nrhs, st);
        dense_chol_solve<float>(L.p, Li.p, n, bf.p, nrhs, st);
        launch_convert_f32_f64(bf.p, b, n * nrhs, st);
      }
      if (Ainv) {
        invf.ensure(nn);
        dense_chol_inverse<float>(L.p, Li.p, n, invf.p, wk.p, st);
        launch_convert_f32_f64(invf.p, Ainv, nn, st);
      }
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(&hinfo, info.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      W.release(); L.release(); Li.release(); wk.release(); bf.release(); invf.release();
    }
    info.release();
    return hinfo == 0 ? PDIPC_OK : PDIPC_E_NOT_SPD;
  } catch (const SolverError& e) {
    return e.code;
  } catch (const HipFailure& e) {
    g_last_init_error = e.msg;
    return PDIPC_E_HIP;
  }
}

// Host-only check of the set-up factorization (no device work): solves
// H x = b over the free block with the supernodal factor and a dense
// Cholesky of Sigma_s on the host, and returns Sigma_s.  Test tap.
int32_t pdipc_debug_host_factor(int32_t n1, int32_t n2, const double* coords1, const int64_t* ptr,
                                const int32_t* col, const double* val, int32_t leaf, const double* b, double* x,
                                double* sigma_out, int64_t* nnz_out) {
  try {
    ScalarCSR H;
    const int32_t N = n1 + n2;
    H.n = N;
    H.ptr.assign(ptr, ptr + N + 1);
    H.col.assign(col, col + ptr[N]);
    H.val.assign(val, val + ptr[N]);
    HostFactor hf;
    std::string e;
    int rc = build_host_factor(n1, n2, coords1, H, leaf, hf, e);
    if (rc) return PDIPC_E_NOT_SPD;
    if (nnz_out) *nnz_out = hf.factor_nnz;
    if (sigma_out) std::copy(hf.sigma.begin(), hf.sigma.end(), sigma_out);
    if (!b || !x) return PDIPC_OK;
    // extended rhs: x1 in dissection order, x2 unchanged
    std::vector<double> be(N), y(N), sol(N);
    for (int32_t p = 0; p < n1; ++p) be[p] = b[hf.perm[p]];
    for (int32_t q = 0; q < n2; ++q) be[n1 + q] = b[n1 + q];
    const int nn = static_cast<int>(hf.nodes.size());
    std::vector<int> order(nn);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return hf.nodes[a].level < hf.nodes[c].level; });
    for (int J : order) {
      const FactorNode& nd = hf.nodes[J];
      std::vector<double> t(nd.s);
      for (int r = 0; r < nd.s; ++r) {
        int64_t row = nd.c0 + r;
        double acc = 0;
        for (int64_t q = hf.fwd_ptr[row]; q < hf.fwd_ptr[row + 1]; ++q) acc += hf.fwd_val[q] * y[hf.fwd_col[q]];
        t[r] = be[row] - acc;
      }
      const double* D = hf.dinv.data() + nd.dinv_off;
      for (int r = 0; r < nd.s; ++r) {
        double acc = 0;
        for (int c = 0; c <= r; ++c) acc += D[static_cast<int64_t>(r) * nd.s + c] * t[c];
        y[nd.c0 + r] = acc;
      }
    }
    for (int32_t q = 0; q < n2; ++q) {
      int64_t row = n1 + q;
      double acc = 0;
      for (int64_t e2 = hf.fwd_ptr[row]; e2 < hf.fwd_ptr[row + 1]; ++e2) acc += hf.fwd_val[e2] * y[hf.fwd_col[e2]];
      y[row] = be[row] - acc;
    }
    // dense Sigma_s solve on the host (Cholesky, test only)
    std::vector<double> Lc(hf.sigma);
    for (int32_t j = 0; j < n2; ++j) {
      double d = Lc[static_cast<size_t>(j) * n2 + j];
      for (int32_t k = 0; k < j; ++k) d -= Lc[static_cast<size_t>(j) * n2 + k] * Lc[static_cast<size_t>(j) * n2 + k];
      if (!(d > 0)) return PDIPC_E_NOT_SPD;
      d = std::sqrt(d);
      Lc[static_cast<size_t>(j) * n2 + j] = d;
      for (int32_t i = j + 1; i < n2; ++i) {
        double s = Lc[static_cast<size_t>(i) * n2 + j];
        for (int32_t k = 0; k < j; ++k) s -= Lc[static_cast<size_t>(i) * n2 + k] * Lc[static_cast<size_t>(j) * n2 + k];
        Lc[static_cast<size_t>(i) * n2 + j] = s / d;
      }
    }
    std::vector<double> z(n2);
    for (int32_t i = 0; i < n2; ++i) {
      double s = y[n1 + i];
      for (int32_t k = 0; k < i; ++k) s -= Lc[static_cast<size_t>(i) * n2 + k] * z[k];
      z[i] = s / Lc[static_cast<size_t>(i) * n2 + i];
    }
    for (int32_t i = n2 - 1; i >= 0; --i) {
      double s = z[i];
      for (int32_t k = i + 1; k < n2; ++k) s -= Lc[static_cast<size_t>(k) * n2 + i] * sol[n1 + k];
      sol[n1 + i] = s / Lc[static_cast<size_t>(i) * n2 + i];
    }
    for (int oi = nn - 1; oi >= 0; --oi) {
      const FactorNode& nd = hf.nodes[order[oi]];
      const int32_t* R = hf.rows.data() + nd.rows_off;
      const double* P = hf.panel.data() + nd.panel_off;
      std::vector<double> t(nd.s);
      for (int c = 0; c < nd.s; ++c) {
        double acc = y[nd.c0 + c];
        for (int i = 0; i < nd.r; ++i) acc -= P[static_cast<int64_t>(i) * nd.s + c] * sol[R[i]];
        t[c] = acc;
      }
      const double* D = hf.dinv.data() + nd.dinv_off;
      for (int c = 0; c < nd.s; ++c) {
        double acc = 0;
        for (int r = c; r < nd.s; ++r) acc += D[static_cast<int64_t>(r) * nd.s + c] * t[r];
        sol[nd.c0 + c] = acc;
      }
    }
    for (int32_t p = 0; p < n1; ++p) x[hf.perm[p]] = sol[p];
    for (int32_t q = 0; q < n2; ++q) x[n1 + q] = sol[n1 + q];
    return PDIPC_OK;
  } catch (...) {
    return PDIPC_E_INVALID;
  }
}

}  // extern "C"
