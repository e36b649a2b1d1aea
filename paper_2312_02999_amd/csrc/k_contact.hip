// Contact detection on the GPU: spatial-hash broad phase, exact box filter,
// narrow phase (constraint set of Algorithm 1), conservative-advancement CCD
// and line-search barrier energies.
//
// Broad phase.  Every stored primitive (triangle or edge) is inserted into
// the uniform-grid cells its box covers; a query (proxy vertex or edge) box,
// widened by dhat, visits its cells.  Each (query, primitive) pair is reported
// only from its "home" cell (the componentwise max of the two cell ranges'
// lower corners), and table entries carry their cell key, so hash collisions
// and multi-cell overlaps never duplicate a pair.  The final test is the
// exact box predicate lo_a <= hi_b + dhat and lo_b <= hi_a + dhat.
//
// Output order is canonical without a global sort: a count pass, an
// exclusive scan over queries, a fill pass, and a per-query insertion sort.
#include "common.h"
#include "geom.h"
#include "kernels.h"

namespace pdipc {

namespace {
constexpr int BT = 256;

__device__ __forceinline__ uint32_t cell_hash(int32_t ix, int32_t iy, int32_t iz, uint32_t mask) {
  uint32_t h = static_cast<uint32_t>(ix) * 73856093u ^ static_cast<uint32_t>(iy) * 19349663u ^
               static_cast<uint32_t>(iz) * 83492791u;
  return h & mask;
}
__device__ __forceinline__ uint64_t cell_key(int32_t ix, int32_t iy, int32_t iz) {
  return (static_cast<uint64_t>(ix) & 0x1FFFFF) | ((static_cast<uint64_t>(iy) & 0x1FFFFF) << 21) |
         ((static_cast<uint64_t>(iz) & 0x1FFFFF) << 42);
}
__device__ __forceinline__ int32_t cell_of(double c, double o, double h) {
  double f = floor((c - o) / h);
  // non-finite or absurd coordinates map to cell 0 (ranges are clamped below)
  return (f >= 0.0 && f < 1.0e9) ? static_cast<int32_t>(f) : 0;
}
// A box never spans more than 3 cells per axis (cell size >= largest extent
// gives at most 2); the clamp bounds every loop even for corrupt input.
// The cell size exceeds every (padded) box extent, so a finite box spans at
// most two cells per axis; the clamp only bounds non-finite input.
__device__ __forceinline__ int32_t clamp_hi(int32_t lo, int32_t hi) {
  return hi < lo ? lo : (hi > lo + 1 ? lo + 1 : hi);
}
}  // namespace

// ---- boxes --------------------------------------------------------------------
__global__ void __launch_bounds__(BT) boxes_kernel(ProxyDev px, const double* __restrict__ x,
                                                   const double* __restrict__ dx, double* __restrict__ vbox,
                                                   double* __restrict__ tbox, double* __restrict__ ebox) {
  int64_t gid = static_cast<int64_t>(blockIdx.x) * BT + threadIdx.x;
  const int64_t total = static_cast<int64_t>(px.nsv) + px.nst + px.nse;
  if (gid >= total) return;
  int32_t vs[3];
  int nv;
  double* out;
  if (gid < px.nsv) {
    vs[0] = px.sv[gid]; nv = 1; out = vbox + 6 * gid;
  } else if (gid < px.nsv + px.nst) {
    int64_t f = gid - px.nsv;
    vs[0] = px.st[3 * f]; vs[1] = px.st[3 * f + 1]; vs[2] = px.st[3 * f + 2]; nv = 3; out = tbox + 6 * f;
  } else {
    int64_t e = gid - px.nsv - px.nst;
    vs[0] = px.se[2 * e]; vs[1] = px.se[2 * e + 1]; nv = 2; out = ebox + 6 * e;
  }
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int k = 0; k < nv; ++k)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      double p = x[3 * vs[k] + r];
      lo[r] = fmin(lo[r], p);
      hi[r] = fmax(hi[r], p);
      if (dx) {
        double q = p + dx[3 * vs[k] + r];
        lo[r] = fmin(lo[r], q);
        hi[r] = fmax(hi[r], q);
      }
    }
#pragma unroll
  for (int r = 0; r < 3; ++r) { out[r] = lo[r]; out[3 + r] = hi[r]; }
}

// params[0..2] = grid origin, params[3] = cell size, params[4] = query pad.
__global__ void __launch_bounds__(BT) grid_params_partial(ProxyDev px, const double* __restrict__ vbox,
                                                          const double* __restrict__ tbox,
                                                          const double* __restrict__ ebox, double pad,
                                                          double* __restrict__ part) {
  double mn[3] = {INFINITY, INFINITY, INFINITY}, ext = 0.0;
  const int64_t total = static_cast<int64_t>(px.nsv) + px.nst + px.nse;
  for (int64_t gid = static_cast<int64_t>(blockIdx.x) * BT + threadIdx.x; gid < total;
       gid += static_cast<int64_t>(gridDim.x) * BT) {
    const double* b;
    double pd = 0.0;
    if (gid < px.nsv) { b = vbox + 6 * gid; pd = pad; }
    else if (gid < px.nsv + px.nst) b = tbox + 6 * (gid - px.nsv);
    else { b = ebox + 6 * (gid - px.nsv - px.nst); pd = pad; }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      mn[r] = fmin(mn[r], b[r] - pd);
      ext = fmax(ext, b[3 + r] - b[r] + 2.0 * pd);
    }
  }
  __shared__ double sh[4][BT / PDIPC_WAVE];
  double vals[4] = {mn[0], mn[1], mn[2], ext};
#pragma unroll
  for (int k = 0; k < 4; ++k) vals[k] = k < 3 ? wave_min(vals[k]) : wave_max(vals[k]);
  int lane = threadIdx.x % PDIPC_WAVE, wid = threadIdx.x / PDIPC_WAVE;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[k][wid] = vals[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k) {
      double r = sh[k][0];
      for (int w = 1; w < BT / PDIPC_WAVE; ++w) r = k < 3 ? fmin(r, sh[k][w]) : fmax(r, sh[k][w]);
      part[4 * blockIdx.x + k] = r;
    }
  }
}

__global__ void __launch_bounds__(64) grid_params_final(const double* __restrict__ part, int nparts, double pad,
                                                        double* params) {
  // one wave: lane i folds partials i, i + 64, ...
  double mn[3] = {INFINITY, INFINITY, INFINITY}, ext = 0.0;
  for (int i = threadIdx.x; i < nparts; i += PDIPC_WAVE) {
#pragma unroll
    for (int r = 0; r < 3; ++r) mn[r] = fmin(mn[r], part[4 * i + r]);
    ext = fmax(ext, part[4 * i + 3]);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) mn[r] = wave_min(mn[r]);
  ext = wave_max(ext);
  if (threadIdx.x != 0) return;
  const double h = ext * (1.0 + 1e-6) + 1e-12;
  for (int r = 0; r < 3; ++r) params[r] = mn[r] - h;
  params[3] = h;
  params[4] = pad;
}

// ---- table build ---------------------------------------------------------------
// Triangles (g < nt) and edges in one launch: each primitive goes into the
// hash bucket of every cell its box spans (at most 2 x 2 x 2).
template <bool FILL>
__global__ void __launch_bounds__(BT) insert_kernel(int32_t nt, int32_t ne, const double* __restrict__ tbox,
                                                    const double* __restrict__ ebox,
                                                    const double* __restrict__ params, uint32_t mask,
                                                    int32_t* __restrict__ tcount, int32_t* __restrict__ tids,
                                                    uint64_t* __restrict__ tkeys, int32_t* __restrict__ ecount,
                                                    int32_t* __restrict__ eids, uint64_t* __restrict__ ekeys) {
  const int32_t g = blockIdx.x * BT + threadIdx.x;
  if (g >= nt + ne) return;
  const bool tri = g < nt;
  const int32_t p = tri ? g : g - nt;
  int32_t* count = tri ? tcount : ecount;
  int32_t* ids = tri ? tids : eids;
  uint64_t* keys = tri ? tkeys : ekeys;
  const double o0 = params[0], o1 = params[1], o2 = params[2], h = params[3];
  const double* b = (tri ? tbox : ebox) + 6 * static_cast<int64_t>(p);
  int32_t l0 = cell_of(b[0], o0, h), l1 = cell_of(b[1], o1, h), l2 = cell_of(b[2], o2, h);
  int32_t u0 = clamp_hi(l0, cell_of(b[3], o0, h)), u1 = clamp_hi(l1, cell_of(b[4], o1, h)),
          u2 = clamp_hi(l2, cell_of(b[5], o2, h));
  for (int32_t k = l2; k <= u2; ++k)
    for (int32_t j = l1; j <= u1; ++j)
      for (int32_t i = l0; i <= u0; ++i) {
        uint32_t hh = cell_hash(i, j, k, mask);
        int32_t slot = atomicAdd(&count[hh], 1);
        if (FILL) {
          ids[slot] = p;
          keys[slot] = cell_key(i, j, k);
        }
      }
}

// ---- queries --------------------------------------------------------------------
struct QueryArgs {
  ProxyDev px;
  const double* x;
  const double* vbox;
  const double* tbox;
  const double* ebox;
  const double* params;
  uint32_t mask;
  const int32_t* t_start;
  const int32_t* t_id;
  const uint64_t* t_key;
  const int32_t* e_start;
  const int32_t* e_id;
  const uint64_t* e_key;
  double dhat;
  bool dist;
};

__device__ __forceinline__ bool box_overlap(const double* a, const double* b, double dhat) {
  return a[0] <= b[3] + dhat && b[0] <= a[3] + dhat && a[1] <= b[4] + dhat && b[1] <= a[4] + dhat &&
         a[2] <= b[5] + dhat && b[2] <= a[5] + dhat;
}

// One wave per query.  The query's box spans at most 2 x 2 x 2 cells; the
// bucket ranges of all of them are read at once, and the lanes test their
// entries as one range, 64 at a time (buckets are short but several dozen
// long where the mesh is dense, so a serial scan would be a long chain of
// dependent loads).  A pair is reported only in the first cell both boxes
// share, so each appears once.
struct QueryCtx {
  bool is_pt;
  double qb[6];
  int32_t qv[2];
  int32_t ql[3], qu[3];
  double o[3], h;
};

__device__ __forceinline__ QueryCtx query_ctx(const QueryArgs& qa, int64_t q) {
  const ProxyDev& px = qa.px;
  QueryCtx c;
  c.is_pt = q < px.nsv;
  c.qv[0] = c.qv[1] = 0;
  const double* qb;
  if (c.is_pt) {
    qb = qa.vbox + 6 * q;
    c.qv[0] = px.sv[q];
  } else {
    const int64_t e = q - px.nsv;
    qb = qa.ebox + 6 * e;
    c.qv[0] = px.se[2 * e];
    c.qv[1] = px.se[2 * e + 1];
  }
#pragma unroll
  for (int r = 0; r < 6; ++r) c.qb[r] = qb[r];
  c.o[0] = qa.params[0]; c.o[1] = qa.params[1]; c.o[2] = qa.params[2];
  c.h = qa.params[3];
  const double pad = qa.params[4];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    c.ql[r] = cell_of(c.qb[r] - pad, c.o[r], c.h);
    c.qu[r] = clamp_hi(c.ql[r], cell_of(c.qb[3 + r] + pad, c.o[r], c.h));
  }
  return c;
}

// Partner of bucket entry s in cell (i, j, k) if the pair is accepted, else -1.
__device__ __forceinline__ int32_t query_test(const QueryArgs& qa, const QueryCtx& c, int64_t q, int32_t s,
                                              uint64_t key, int32_t i, int32_t j, int32_t k) {
  const ProxyDev& px = qa.px;
  const int32_t* ids = c.is_pt ? qa.t_id : qa.e_id;
  const uint64_t* keys = c.is_pt ? qa.t_key : qa.e_key;
  const double* pbox = c.is_pt ? qa.tbox : qa.ebox;
  // the entry's key and id, then the partner's box and vertices, each group
  // loaded at once (a valid entry's id indexes both, whatever its key)
  const uint64_t ks = keys[s];
  const int32_t p = ids[s];
  const double* bp = pbox + 6 * static_cast<int64_t>(p);
  double b[6];
#pragma unroll
  for (int r = 0; r < 6; ++r) b[r] = bp[r];
  int32_t w0, w1, w2 = -1;
  if (c.is_pt) {
    w0 = px.st[3 * p]; w1 = px.st[3 * p + 1]; w2 = px.st[3 * p + 2];
  } else {
    w0 = px.se[2 * p]; w1 = px.se[2 * p + 1];
  }
  if (ks != key) return -1;
  if (!c.is_pt && p <= q - px.nsv) return -1;
  const int32_t pl0 = cell_of(b[0], c.o[0], c.h), pl1 = cell_of(b[1], c.o[1], c.h), pl2 = cell_of(b[2], c.o[2], c.h);
  if (max(c.ql[0], pl0) != i || max(c.ql[1], pl1) != j || max(c.ql[2], pl2) != k) return -1;
  if (!box_overlap(c.qb, b, qa.dhat)) return -1;
  int32_t v4[4];
  if (c.is_pt) {
    if (c.qv[0] == w0 || c.qv[0] == w1 || c.qv[0] == w2) return -1;
    v4[0] = c.qv[0]; v4[1] = w0; v4[2] = w1; v4[3] = w2;
  } else {
    if (c.qv[0] == w0 || c.qv[0] == w1 || c.qv[1] == w0 || c.qv[1] == w1) return -1;
    v4[0] = c.qv[0]; v4[1] = c.qv[1]; v4[2] = w0; v4[3] = w1;
  }
  if (qa.dist) {
    double P[4][3];
    load_pair_abs(v4, qa.x, P);
    const double d2 = pair_dist2<double>(c.is_pt, P);
    if (!(d2 < qa.dhat * qa.dhat)) return -1;
  }
  return p;
}

// Walk the query's cells with the whole wave; emit(partner, rank) for every
// accepted partner (rank: its position among the wave's accepted partners so
// far); returns the count.
template <typename Emit>
__device__ __forceinline__ int32_t query_wave(const QueryArgs& qa, int64_t q, Emit emit) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const QueryCtx c = query_ctx(qa, q);
  const int32_t* start = c.is_pt ? qa.t_start : qa.e_start;
  // lane l < 8 reads the bucket range of cell slot l (empty outside the box)
  int32_t s0 = 0, len = 0;
  if (lane < 8) {
    const int32_t i = c.ql[0] + (lane & 1), j = c.ql[1] + ((lane >> 1) & 1), k = c.ql[2] + (lane >> 2);
    if (i <= c.qu[0] && j <= c.qu[1] && k <= c.qu[2]) {
      const uint32_t hh = cell_hash(i, j, k, qa.mask);
      s0 = start[hh];
      len = start[hh + 1] - s0;
    }
  }
  // the slots' entries one after another: slot l covers [off[l], off[l + 1])
  int32_t off[9], sb[8];
  off[0] = 0;
#pragma unroll
  for (int l = 0; l < 8; ++l) {
    sb[l] = __builtin_amdgcn_readlane(s0, l);
    off[l + 1] = off[l] + __builtin_amdgcn_readlane(len, l);
  }
  int32_t total = 0;
  for (int32_t f0 = 0; f0 < off[8]; f0 += PDIPC_WAVE) {
    const int32_t f = f0 + lane;
    int slot = 0;
#pragma unroll
    for (int l = 1; l < 8; ++l) slot += f >= off[l] ? 1 : 0;
    int32_t s = 0, base = 0;
#pragma unroll
    for (int l = 0; l < 8; ++l)
      if (slot == l) { s = sb[l]; base = off[l]; }
    s += f - base;
    const int32_t i = c.ql[0] + (slot & 1), j = c.ql[1] + ((slot >> 1) & 1), k = c.ql[2] + (slot >> 2);
    const int32_t p = f < off[8] ? query_test(qa, c, q, s, cell_key(i, j, k), i, j, k) : -1;
    const uint64_t m = __ballot(p >= 0);
    if (p >= 0) {
      const int32_t below = static_cast<int32_t>(
          __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u)));
      emit(p, total + below);
    }
    total += static_cast<int32_t>(__popcll(m));
  }
  return total;
}

constexpr int QT = 256;
constexpr int QW = QT / PDIPC_WAVE;   // queries per workgroup

// Counts each query's partners and keeps the first kQueryKeep of them; the
// largest count above kQueryKeep goes to *over (zero before the launch).
__global__ void __launch_bounds__(QT) query_count_kernel(QueryArgs qa, int32_t* __restrict__ qcount,
                                                         int32_t* __restrict__ qbuf, int32_t* __restrict__ over) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * QW + threadIdx.x / PDIPC_WAVE;
  const int64_t nq = static_cast<int64_t>(qa.px.nsv) + qa.px.nse;
  if (blockIdx.x == 0 && threadIdx.x == 0) qcount[nq] = 0;     // sentinel of the scan
  if (q >= nq) return;
  int32_t* keep = qbuf + q * kQueryKeep;
  const int32_t c = query_wave(qa, q, [&](int32_t p, int32_t r) {
    if (r < kQueryKeep) keep[r] = p;
  });
  if (threadIdx.x % PDIPC_WAVE == 0) {
    qcount[q] = c;
    if (c > kQueryKeep) atomicMax(over, c);
  }
}

__global__ void __launch_bounds__(QT) query_fill_kernel(QueryArgs qa, const int32_t* __restrict__ qoff,
                                                        int32_t* __restrict__ tmpj) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * QW + threadIdx.x / PDIPC_WAVE;
  const int64_t nq = static_cast<int64_t>(qa.px.nsv) + qa.px.nse;
  if (q >= nq) return;
  const int32_t b = qoff[q];
  query_wave(qa, q, [&](int32_t p, int32_t r) { tmpj[b + r] = p; });
}

// one wave per query: rank its partners (unique ids) and emit sorted pairs;
// the partners are read from src + q * stride (the counting pass's kept
// ones), or, with stride 0, from src + qoff[q] (the second pass's)
__global__ void __launch_bounds__(256) query_emit_kernel(ProxyDev px, const int32_t* __restrict__ qoff,
                                                         const int32_t* __restrict__ src, int64_t stride,
                                                         int32_t* __restrict__ ptype, int32_t* __restrict__ pi,
                                                         int32_t* __restrict__ pj, int32_t* __restrict__ pv4) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const int64_t q = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / PDIPC_WAVE;
  const int64_t nq = static_cast<int64_t>(px.nsv) + px.nse;
  if (q >= nq) return;
  const int32_t b = qoff[q], e = qoff[q + 1], cnt = e - b;
  const int64_t base = stride > 0 ? q * stride : b;                  // partner a at src[base + a]
  const bool is_pt = q < px.nsv;
  const int32_t qi = is_pt ? px.sv[q] : static_cast<int32_t>(q - px.nsv);
  for (int32_t a = lane; a < cnt; a += PDIPC_WAVE) {
    const int32_t key = src[base + a];
    int32_t rank = 0;
    for (int32_t j = 0; j < cnt; ++j) rank += src[base + j] < key ? 1 : 0;
    const int32_t o = b + rank;
    ptype[o] = is_pt ? 0 : 1;
    pi[o] = qi;
    pj[o] = key;
    if (is_pt) {
      pv4[4 * o] = qi;
      pv4[4 * o + 1] = px.st[3 * key];
      pv4[4 * o + 2] = px.st[3 * key + 1];
      pv4[4 * o + 3] = px.st[3 * key + 2];
    } else {
      pv4[4 * o] = px.se[2 * qi];
      pv4[4 * o + 1] = px.se[2 * qi + 1];
      pv4[4 * o + 2] = px.se[2 * key];
      pv4[4 * o + 3] = px.se[2 * key + 1];
    }
  }
}

int find_pairs(const ProxyDev& px, const BroadPhaseBuffers& bb, const double* x, const double* dx, double dhat,
               bool distance_filter, PairList& out, int32_t* n_pt, int32_t* n_ee, hipStream_t st,
               int64_t* needed) {
  const int64_t total = static_cast<int64_t>(px.nsv) + px.nst + px.nse;
  const int64_t nq = static_cast<int64_t>(px.nsv) + px.nse;

  *needed = 0;
  if (px.nsv == 0 || (px.nst == 0 && px.nse == 0)) {
    *n_pt = 0;
    *n_ee = 0;
    return 0;
  }
  const double pad = dhat * (1.0 + 1e-9) + 1e-15;
  boxes_kernel<<<grid_for(total, BT), BT, 0, st>>>(px, x, dx, bb.vbox, bb.tbox, bb.ebox);
  double* part = bb.params + 8;
  grid_params_partial<<<64, BT, 0, st>>>(px, bb.vbox, bb.tbox, bb.ebox, pad, part);
  grid_params_final<<<1, 64, 0, st>>>(part, 64, pad, bb.params);
  const uint32_t T = 1u << bb.table_bits;
  const uint32_t mask = T - 1;
  launch_fill2_i32(bb.t_count, T + 1, bb.e_count, T + 1, 0, st);
  const int32_t nte = px.nst + px.nse;
  insert_kernel<false><<<grid_for(nte, BT), BT, 0, st>>>(px.nst, px.nse, bb.tbox, bb.ebox, bb.params, mask, bb.t_count,
                                                         nullptr, nullptr, bb.e_count, nullptr, nullptr);
  {
    // bucket starts, with copies as the fill cursors
    const ScanJob jobs[2] = {{bb.t_count, bb.t_count, T + 1, bb.d_totals + 2, bb.t_cursor, -1, nullptr},
                             {bb.e_count, bb.e_count, T + 1, bb.d_totals + 3, bb.e_cursor, -1, nullptr}};
    launch_exclusive_scans(jobs, 2, bb.scan_temp, st);
  }
  insert_kernel<true><<<grid_for(nte, BT), BT, 0, st>>>(px.nst, px.nse, bb.tbox, bb.ebox, bb.params, mask, bb.t_cursor,
                                                        bb.t_id, bb.t_key, bb.e_cursor, bb.e_id, bb.e_key);

  QueryArgs qa{px, x, bb.vbox, bb.tbox, bb.ebox, bb.params, mask, bb.t_count, bb.t_id, bb.t_key,
               bb.e_count, bb.e_id, bb.e_key, dhat, distance_filter};
  launch_fill_i32(bb.d_totals + 7, 1, 0, st);
  query_count_kernel<<<grid_for(nq, QW), QT, 0, st>>>(qa, bb.q_count, bb.qbuf, bb.d_totals + 7);
  {
    // per-query offsets; the offset of the first edge query is the PT count
    const ScanJob job{bb.q_count, bb.q_count, nq + 1, bb.d_totals, nullptr, px.nsv, bb.d_totals + 1};
    launch_exclusive_scans(&job, 1, bb.scan_temp, st);
  }
  int32_t* h_tot = bb.h_totals;
  hipMemcpyAsync(h_tot, bb.d_totals, sizeof(int32_t) * 4, hipMemcpyDeviceToHost, st);
  hipMemcpyAsync(h_tot + 7, bb.d_totals + 7, sizeof(int32_t), hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  const int32_t npairs = h_tot[0];
  if (h_tot[2] > bb.ent_cap || h_tot[3] > bb.ent_cap) return -1;   // grid sizing broke
  const bool kept = h_tot[7] == 0;        // every query's partners are in qbuf
  if (npairs > out.cap || (!kept && npairs > bb.tmp_cap)) {
    *needed = npairs;
    return 1;
  }
  *n_pt = h_tot[1];
  *n_ee = npairs - h_tot[1];
  if (npairs > 0) {
    if (!kept) query_fill_kernel<<<grid_for(nq, QW), QT, 0, st>>>(qa, bb.q_count, bb.tmpj);
    query_emit_kernel<<<grid_for(nq, 4), 256, 0, st>>>(px, bb.q_count, kept ? bb.qbuf : bb.tmpj,
                                                       kept ? kQueryKeep : 0, out.type, out.i, out.j, out.v4);
  }
  return 0;
}

// ---- constraint set as the active subset of a candidate list -------------------
// Candidates swept over x_prev -> x_prev + dx contain every pair within dhat at
// any x_prev + alpha dx, alpha in [0, 1]; filtering them by the exact distance
// at the new iterate gives the same sorted set as a fresh broad phase.
// Near ties: candidates with |d - dhat| below kNearTie dhat, where a rounding
// difference in the positions could flip membership (|d^2 - dhat^2| is about
// 2 dhat |d - dhat|); counted with integer atomics for the frame statistics.
constexpr double kNearTie = 1e-10;

__global__ void __launch_bounds__(BT) active_flag_kernel(const int32_t* __restrict__ v4all, int32_t npairs,
                                                         int32_t n_pt, const double* __restrict__ x, double dhat,
                                                         int32_t* __restrict__ flag, int32_t* __restrict__ near) {
  int32_t k = blockIdx.x * BT + threadIdx.x;
  if (k > npairs) return;
  if (k == npairs) { flag[k] = 0; return; }
  int32_t v4[4] = {v4all[4 * k], v4all[4 * k + 1], v4all[4 * k + 2], v4all[4 * k + 3]};
  double P[4][3];
  load_pair_abs(v4, x, P);
  double d2 = pair_dist2<double>(k < n_pt, P);
  const double dh2 = dhat * dhat;
  flag[k] = d2 < dh2 ? 1 : 0;
  if (fabs(d2 - dh2) < 2.0 * kNearTie * dh2) atomicAdd(near, 1);
}

__global__ void __launch_bounds__(BT) compact_pairs_kernel(PairList src, int32_t npairs, const int32_t* __restrict__ flag,
                                                           const int32_t* __restrict__ pos, PairList dst) {
  int32_t k = blockIdx.x * BT + threadIdx.x;
  if (k >= npairs || !flag[k]) return;
  int32_t o = pos[k];
  dst.type[o] = src.type[k];
  dst.i[o] = src.i[k];
  dst.j[o] = src.j[k];
#pragma unroll
  for (int a = 0; a < 4; ++a) dst.v4[4 * o + a] = src.v4[4 * k + a];
}

int filter_active(const PairList& cand, int32_t ncand, int32_t cand_pt, const double* x, double dhat, PairList& out,
                  int32_t* flag, int32_t* pos, int32_t* d_tot, int32_t* h_tot, void* scan_temp, int32_t* n_pt,
                  int32_t* n_ee, hipStream_t st, int64_t* needed, int32_t* near_ties) {
  *needed = 0;
  if (near_ties) *near_ties = 0;
  if (ncand <= 0) {
    *n_pt = 0;
    *n_ee = 0;
    return 0;
  }
  launch_fill_i32(d_tot + 2, 1, 0, st);
  active_flag_kernel<<<grid_for(ncand + 1, BT), BT, 0, st>>>(cand.v4, ncand, cand_pt, x, dhat, flag, d_tot + 2);
  {
    // active positions; the position of the first EE candidate is the PT count
    const ScanJob job{flag, pos, ncand + 1, d_tot, nullptr, cand_pt, d_tot + 1};
    launch_exclusive_scans(&job, 1, scan_temp, st);
  }
  int32_t* h = h_tot;
  hipMemcpyAsync(h, d_tot, sizeof(int32_t) * 3, hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  if (h[0] > out.cap) {
    *needed = h[0];
    return 1;
  }
  *n_pt = h[1];
  *n_ee = h[0] - h[1];
  if (near_ties) *near_ties = h[2];
  if (h[0] > 0) compact_pairs_kernel<<<grid_for(ncand, BT), BT, 0, st>>>(cand, ncand, flag, pos, out);
  return 0;
}

// ---- CCD: conservative advancement ---------------------------------------------
// Conservative bound of one swept candidate.
__device__ __forceinline__ double ccd_pair(const int32_t* __restrict__ v4all, int32_t k, int32_t n_pt,
                                           const double* __restrict__ x, const double* __restrict__ dx, double eta,
                                           int32_t steps) {
  const bool is_pt = k < n_pt;
  int32_t v4[4] = {v4all[4 * k], v4all[4 * k + 1], v4all[4 * k + 2], v4all[4 * k + 3]};
  double P[4][3];
  load_pair_rel(v4, x, P);
  double d0 = sqrt(pair_dist2<double>(is_pt, P));
  double g = eta * d0;
  double D[4][3], m[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      D[a][r] = dx[3 * v4[a] + r];
      m[r] += D[a][r];
    }
  double nr[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double c[3] = {D[a][0] - 0.25 * m[0], D[a][1] - 0.25 * m[1], D[a][2] - 0.25 * m[2]};
    nr[a] = sqrt(dot3(c, c));
  }
  double l = is_pt ? nr[0] + fmax(nr[1], fmax(nr[2], nr[3])) : fmax(nr[0], nr[1]) + fmax(nr[2], nr[3]);
  double t = 0.0;
  if (!(l > 0.0)) {
    t = 1.0;
  } else {
    for (int it = 0; it < steps; ++it) {
      double Q[4][3];
      load_pair_rel_step(v4, x, dx, t, Q);
      double dt = sqrt(pair_dist2<double>(is_pt, Q));
      t = fmin(1.0, t + fmax(0.0, dt - g) / l);
    }
  }
  return t;
}

// One thread per candidate; each block also writes the minimum of its bounds
// (the step bound alpha_m is the minimum over the blocks).
__device__ __forceinline__ double pair_energy_at(const int32_t* __restrict__ v4all, int32_t k, int32_t n_pt,
                                                  const double* __restrict__ x, const double* __restrict__ dx,
                                                  double alpha, double dhat, double kappa, int form);

// With e0 (optional), each candidate's barrier energy at x as well (the line
// search's reference values).
__global__ void __launch_bounds__(BT) ccd_kernel(const int32_t* __restrict__ v4all, int32_t npairs, int32_t n_pt,
                                                 const double* __restrict__ x, const double* __restrict__ dx,
                                                 double eta, int32_t steps, double* __restrict__ tout,
                                                 double* __restrict__ part, double dhat, double kappa,
                                                 int form, double* __restrict__ e0) {
  __shared__ double sh4[4];
  const int32_t k = blockIdx.x * BT + threadIdx.x;
  const double t = k < npairs ? ccd_pair(v4all, k, n_pt, x, dx, eta, steps) : 1.0;
  if (k < npairs) {
    tout[k] = t;
    if (e0) e0[k] = pair_energy_at(v4all, k, n_pt, x, nullptr, 0.0, dhat, kappa, form);
  }
  const double mn = block256_min(t, sh4);
  if (threadIdx.x == 0) part[blockIdx.x] = mn;
}

int launch_ccd(const PairList& pl, int32_t npairs, int32_t n_pt, const double* x, const double* dx, double eta,
               int32_t steps, double* t_out, double* part, hipStream_t st, double dhat, double kappa, int form,
               double* e0) {
  if (npairs <= 0) return 0;
  const unsigned g = grid_for(npairs, BT);
  ccd_kernel<<<g, BT, 0, st>>>(pl.v4, npairs, n_pt, x, dx, eta, steps, t_out, part, dhat, kappa, form, e0);
  return static_cast<int>(g);
}

// ---- line-search barrier energies -------------------------------------------------
// Barrier energy of every candidate at x (dx == nullptr) or at x + alpha dx with
// alpha = ls[LS_ALPHA] (no-op once the line search is decided), optionally as
// a difference from E0.
__global__ void __launch_bounds__(BT) pair_energy_kernel(const int32_t* __restrict__ v4all, int32_t npairs,
                                                         int32_t n_pt, const double* __restrict__ x,
                                                         const double* __restrict__ dx,
                                                         const double* __restrict__ ls, double dhat, double kappa,
                                                         int form, const double* __restrict__ E0,
                                                         double* __restrict__ out) {
  double alpha = 0.0;
  if (ls) {
    if (ls[LS_STATE] != 0.0) return;
    alpha = ls[LS_ALPHA];
  }
  int32_t k = blockIdx.x * BT + threadIdx.x;
  if (k >= npairs) return;
  const double e = pair_energy_at(v4all, k, n_pt, x, dx, alpha, dhat, kappa, form);
  out[k] = E0 ? e - E0[k] : e;
}

__device__ __forceinline__ double pair_energy_at(const int32_t* __restrict__ v4all, int32_t k, int32_t n_pt,
                                                  const double* __restrict__ x, const double* __restrict__ dx,
                                                  double alpha, double dhat, double kappa, int form) {
  int32_t v4[4] = {v4all[4 * k], v4all[4 * k + 1], v4all[4 * k + 2], v4all[4 * k + 3]};
  double P[4][3];
  if (dx) load_pair_rel_step(v4, x, dx, alpha, P);
  else load_pair_rel(v4, x, P);
  double d2 = pair_dist2<double>(k < n_pt, P);
  if (!(d2 > 0.0)) return INFINITY;
  return kappa * barrier_b_of_D(d2, dhat, form);
}

void launch_pair_barrier_energy(const PairList& pl, int32_t npairs, int32_t n_pt, const double* x, const double* dx,
                                const double* ls, double dhat, double kappa, int form, const double* E0, double* out,
                                hipStream_t st) {
  if (npairs <= 0) return;
  pair_energy_kernel<<<grid_for(npairs, BT), BT, 0, st>>>(pl.v4, npairs, n_pt, x, dx, ls, dhat, kappa, form, E0,
                                                          out);
}

__global__ void __launch_bounds__(BT) pair_d2_kernel(const int32_t* __restrict__ v4all, int32_t npairs, int32_t n_pt,
                                                     const double* __restrict__ x, double* __restrict__ out) {
  int32_t k = blockIdx.x * BT + threadIdx.x;
  if (k >= npairs) return;
  int32_t v4[4] = {v4all[4 * k], v4all[4 * k + 1], v4all[4 * k + 2], v4all[4 * k + 3]};
  double P[4][3];
  load_pair_abs(v4, x, P);
  out[k] = pair_dist2<double>(k < n_pt, P);
}

void launch_pair_min_dist2(const PairList& pl, int32_t npairs, int32_t n_pt, const double* x, double* d2_out,
                           hipStream_t st) {
  if (npairs <= 0) return;
  pair_d2_kernel<<<grid_for(npairs, BT), BT, 0, st>>>(pl.v4, npairs, n_pt, x, d2_out);
}

}  // namespace pdipc
