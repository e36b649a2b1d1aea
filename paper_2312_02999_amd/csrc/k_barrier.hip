// Barrier energy, gradient and positive-semidefinite Hessian per active pair
// (Eq. 3 and the PositiveDefinite step of Algorithm 1).
//
// Derivatives of the squared distance D come from the closest-feature form
// D(x) = min_beta |q(x, beta)|^2, q = sum_j c_j(beta) P_j with c affine in
// beta.  At the minimiser (envelope and implicit-function theorems):
//   grad D  = f_x = 2 C^T q
//   hess D  = f_xx - f_xb f_bb^-1 f_bx,  f_xx = 2 C^T C,  f_bb = 2 D_k.D_l,
//   f_xb_k  = 2 (dC/dbeta_k)^T q + 2 C^T D_k,   D_k = sum_j dc_j/dbeta_k P_j.
// The barrier Hessian kappa (phi'' gradD gradD^T + phi' hessD), with
// phi(D) = b(sqrt D), has its range inside span{C^T e_r, f_xb_k} (at most 5
// dimensions), so the clamp of negative eigenvalues is done exactly on the
// projection onto an orthonormal basis of that span: a <= 5x5 Jacobi
// eigen-problem instead of 12x12.  Output is the factor U (12 x 5) with
// projected Hessian U U^T.
#include "common.h"
#include "geom.h"
#include "kernels.h"

namespace pdipc {

namespace {
constexpr int BT = 64;
}

// Cyclic Jacobi on a symmetric 5x5 (fixed size: fully unrolled, no scratch).
template <typename T>
__device__ __forceinline__ void sym_eig_jacobi5(T A[5][5], T V[5][5]) {
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) V[i][j] = i == j ? T(1) : T(0);
  for (int sweep = 0; sweep < 12; ++sweep) {
    T off = T(0), dia = T(0);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      dia += A[i][i] * A[i][i];
#pragma unroll
      for (int j = i + 1; j < 5; ++j) off += A[i][j] * A[i][j];
    }
    if (off == T(0) || off <= T(sizeof(T) == 8 ? 1e-32 : 1e-18) * dia) break;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = p + 1; q < 5; ++q) {
        T apq = A[p][q];
        if (apq != T(0)) {
          T theta = (A[q][q] - A[p][p]) / (T(2) * apq);
          T t = (theta >= T(0) ? T(1) : T(-1)) / (fabs(theta) + sqrt(theta * theta + T(1)));
          T c = T(1) / sqrt(t * t + T(1));
          T s = t * c;
#pragma unroll
          for (int k = 0; k < 5; ++k) {
            T akp = A[k][p], akq = A[k][q];
            A[k][p] = c * akp - s * akq;
            A[k][q] = s * akp + c * akq;
          }
#pragma unroll
          for (int k = 0; k < 5; ++k) {
            T apk = A[p][k], aqk = A[q][k];
            A[p][k] = c * apk - s * aqk;
            A[q][k] = s * apk + c * aqk;
          }
#pragma unroll
          for (int k = 0; k < 5; ++k) {
            T vkp = V[k][p], vkq = V[k][q];
            V[k][p] = c * vkp - s * vkq;
            V[k][q] = s * vkp + c * vkq;
          }
        }
      }
  }
}

// Barrier energy, gradient and the factor U (12 x 5) of the projected
// Hessian, H+ = U U^T.  Geometry, derivatives and the projected 5 x 5 matrix
// are formed in T; the 5 x 5 eigen-decomposition runs in TE (FP32 in the
// mixed path: the cancellation-prone geometry, e.g. nearly parallel edges,
// stays in FP64).
template <typename T, typename TE = T>
__device__ void pair_barrier(const double Pd[4][3], bool is_pt, double dhat, double kappa, int form, double& energy,
                             double grad[12], double U[12][5]) {
  T P[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 3; ++r) P[a][r] = static_cast<T>(Pd[a][r]);
  Feature<T> f;
  pair_feature<T>(is_pt, P, f);
  T q[3] = {T(0), T(0), T(0)}, Dk[2][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      q[r] += f.c[j] * P[j][r];
      Dk[0][r] += f.dcdb[0][j] * P[j][r];
      Dk[1][r] += f.dcdb[1][j] * P[j][r];
    }
  const T D = dot3(q, q);
  T eb, phi1, phi2;
  barrier_of_D<T>(D, static_cast<T>(dhat), static_cast<T>(kappa), form, eb, phi1, phi2);
  energy = static_cast<double>(eb);
  T gD[12];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 3; ++r) gD[3 * j + r] = T(2) * f.c[j] * q[r];
#pragma unroll
  for (int i = 0; i < 12; ++i) grad[i] = static_cast<double>(phi1 * gD[i]);
  // f_xb columns (zero for missing parameters) and f_bb^-1
  const T use0 = f.nb >= 1 ? T(1) : T(0), use1 = f.nb >= 2 ? T(1) : T(0);
  T fxb[2][12];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      fxb[0][3 * j + r] = use0 * (T(2) * f.dcdb[0][j] * q[r] + T(2) * f.c[j] * Dk[0][r]);
      fxb[1][3 * j + r] = use1 * (T(2) * f.dcdb[1][j] * q[r] + T(2) * f.c[j] * Dk[1][r]);
    }
  T fbbi[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
  {
    T b00 = T(2) * dot3(Dk[0], Dk[0]), b01 = T(2) * dot3(Dk[0], Dk[1]), b11 = T(2) * dot3(Dk[1], Dk[1]);
    if (f.nb == 1) {
      fbbi[0][0] = T(1) / b00;
    } else if (f.nb == 2) {
      T det = b00 * b11 - b01 * b01;
      fbbi[0][0] = b11 / det;
      fbbi[1][1] = b00 / det;
      fbbi[0][1] = fbbi[1][0] = -b01 / det;
    }
  }
  // orthonormal basis Q of span{C^T e_r, f_xb_k}: three C columns, then up to two more
  T Q[5][12];
  const T cn = sqrt(f.c[0] * f.c[0] + f.c[1] * f.c[1] + f.c[2] * f.c[2] + f.c[3] * f.c[3]);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int rr = 0; rr < 3; ++rr) Q[r][3 * j + rr] = rr == r ? f.c[j] / cn : T(0);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    T v[12], n0 = T(0);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      v[i] = fxb[k][i];
      n0 += v[i] * v[i];
    }
#pragma unroll
    for (int pass = 0; pass < 2; ++pass)
#pragma unroll
      for (int b = 0; b < 3 + k; ++b) {
        T pr = T(0);
#pragma unroll
        for (int i = 0; i < 12; ++i) pr += Q[b][i] * v[i];
#pragma unroll
        for (int i = 0; i < 12; ++i) v[i] -= pr * Q[b][i];
      }
    T nv = T(0);
#pragma unroll
    for (int i = 0; i < 12; ++i) nv += v[i] * v[i];
    const bool keep = nv > T(sizeof(T) == 8 ? 1e-28 : 1e-12) * n0 && nv > T(0);
    const T inv = keep ? T(1) / sqrt(nv) : T(0);
#pragma unroll
    for (int i = 0; i < 12; ++i) Q[3 + k][i] = v[i] * inv;
  }
  // Ht = Q^T H Q with H = phi2 gD gD^T + phi1 (2 C^T C - f_xb f_bb^-1 f_bx)
  T qg[5], qf[5][2], cq[5][3];
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      s0 += Q[a][i] * gD[i];
      s1 += Q[a][i] * fxb[0][i];
      s2 += Q[a][i] * fxb[1][i];
    }
    qg[a] = s0;
    qf[a][0] = s1;
    qf[a][1] = s2;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      T t = T(0);
#pragma unroll
      for (int j = 0; j < 4; ++j) t += f.c[j] * Q[a][3 * j + r];
      cq[a][r] = t;
    }
  }
  T Ht[5][5], V[5][5];
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      T hd = T(2) * dot3(cq[a], cq[b]);
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int l = 0; l < 2; ++l) hd -= qf[a][k] * fbbi[k][l] * qf[b][l];
      Ht[a][b] = phi2 * qg[a] * qg[b] + phi1 * hd;
    }
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int b = a + 1; b < 5; ++b) {
      T sm = T(0.5) * (Ht[a][b] + Ht[b][a]);
      Ht[a][b] = sm;
      Ht[b][a] = sm;
    }
  TE He[5][5], Ve[5][5];
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b) He[a][b] = static_cast<TE>(Ht[a][b]);
  sym_eig_jacobi5<TE>(He, Ve);
  T sq[5];
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    sq[a] = He[a][a] > TE(0) ? sqrt(static_cast<T>(He[a][a])) : T(0);
#pragma unroll
    for (int b = 0; b < 5; ++b) V[a][b] = static_cast<T>(Ve[a][b]);
  }
#pragma unroll
  for (int i = 0; i < 12; ++i)
#pragma unroll
    for (int e2 = 0; e2 < 5; ++e2) {
      T sm = T(0);
#pragma unroll
      for (int a = 0; a < 5; ++a) sm += Q[a][i] * V[a][e2];
      U[i][e2] = static_cast<double>(sm * sq[e2]);
    }
}


__global__ void __launch_bounds__(BT) barrier_kernel(const int32_t* __restrict__ v4all, int32_t npairs, int32_t n_pt,
                                                     const double* __restrict__ x, double dhat, double kappa,
                                                     int form, bool fp32, double* __restrict__ energy,
                                                     double* __restrict__ grad, double* __restrict__ U) {
  int32_t k = blockIdx.x * BT + threadIdx.x;
  if (k >= npairs) return;
  int32_t v4[4] = {v4all[4 * k], v4all[4 * k + 1], v4all[4 * k + 2], v4all[4 * k + 3]};
  double P[4][3];
  load_pair_rel(v4, x, P);
  double e, g[12], u[12][5];
  if (fp32) {
    // FP32 eigen-decomposition of the projected Hessian; everything else,
    // including the energy and gradient that fix the equilibrium, in FP64
    pair_barrier<double, float>(P, k < n_pt, dhat, kappa, form, e, g, u);
  } else {
    pair_barrier<double>(P, k < n_pt, dhat, kappa, form, e, g, u);
  }
  energy[k] = e;
#pragma unroll
  for (int i = 0; i < 12; ++i) grad[static_cast<int64_t>(i) * npairs + k] = g[i];
#pragma unroll
  for (int i = 0; i < 12; ++i)
#pragma unroll
    for (int c = 0; c < 5; ++c) U[static_cast<int64_t>(5 * i + c) * npairs + k] = u[i][c];
}

void launch_barrier(const PairList& pl, int32_t npairs, int32_t n_pt, const double* x, double dhat, double kappa,
                    int form, bool fp32, BarrierOut& bo, hipStream_t st) {
  if (npairs <= 0) return;
  barrier_kernel<<<grid_for(npairs, BT), BT, 0, st>>>(pl.v4, npairs, n_pt, x, dhat, kappa, form, fp32, bo.energy,
                                                       bo.grad, bo.U);
}

// ---- embedding s = W x and the pairs' slots over simulation vertices --------------
__global__ void __launch_bounds__(256) embed_positions_kernel(EmbedDev W, const double* __restrict__ x,
                                                              double* __restrict__ s) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (t >= 3LL * W.ns) return;
  const int64_t p = t / 3;
  const int r = static_cast<int>(t % 3);
  double acc = 0.0;
  for (int32_t e = W.ptr[p]; e < W.ptr[p + 1]; ++e) acc += W.val[e] * x[3LL * W.col[e] + r];
  s[t] = acc;
}

void launch_embed_positions(const EmbedDev& W, const double* x, double* s, hipStream_t st) {
  if (W.ns > 0) embed_positions_kernel<<<grid_for(3LL * W.ns, 256), 256, 0, st>>>(W, x, s);
}

// One thread per pair: the W entries of its four proxy points in order
// (point, entry); an entry whose simulation vertex already has a slot adds
// to it, otherwise it opens the next slot.  Slot rows are the weighted sums
// of the points' gradient and factor rows.
constexpr int kSlotsW = 16;
__global__ void __launch_bounds__(128) expand_pairs_kernel(EmbedDev W, const int32_t* __restrict__ v4,
                                                           int32_t npairs, const double* __restrict__ grad,
                                                           const double* __restrict__ U, int32_t* __restrict__ sv,
                                                           double* __restrict__ sg, double* __restrict__ sU) {
  const int32_t k = blockIdx.x * 128 + threadIdx.x;
  if (k >= npairs) return;
  int32_t vert[kSlotsW];
  int nslot = 0;
  for (int q = 0; q < kSlotsW; ++q) {
    vert[q] = -1;
    for (int r = 0; r < 3; ++r) sg[static_cast<int64_t>(3 * q + r) * npairs + k] = 0.0;
    for (int e = 0; e < 15; ++e) sU[static_cast<int64_t>(15 * q + e) * npairs + k] = 0.0;
  }
  for (int a = 0; a < 4; ++a) {
    const int32_t p = v4[4 * k + a];
    for (int32_t e = W.ptr[p]; e < W.ptr[p + 1]; ++e) {
      const int32_t j = W.col[e];
      const double w = W.val[e];
      int q = 0;
      while (q < nslot && vert[q] != j) ++q;
      if (q == nslot) vert[nslot++] = j;
      for (int r = 0; r < 3; ++r) {
        sg[static_cast<int64_t>(3 * q + r) * npairs + k] += w * grad[static_cast<int64_t>(3 * a + r) * npairs + k];
        for (int c = 0; c < 5; ++c)
          sU[static_cast<int64_t>(5 * (3 * q + r) + c) * npairs + k] +=
              w * U[static_cast<int64_t>(5 * (3 * a + r) + c) * npairs + k];
      }
    }
  }
  for (int q = 0; q < kSlotsW; ++q) sv[kSlotsW * k + q] = vert[q];
}

void launch_expand_pairs(const EmbedDev& W, const int32_t* v4, int32_t npairs, const BarrierOut& bo,
                         int32_t* slot_v, double* slot_grad, double* slot_U, hipStream_t st) {
  if (npairs > 0)
    expand_pairs_kernel<<<grid_for(npairs, 128), 128, 0, st>>>(W, v4, npairs, bo.grad, bo.U, slot_v, slot_grad,
                                                                slot_U);
}

// ---- vertex incidence ------------------------------------------------------------
template <int S>
__global__ void inc_count_kernel(const int32_t* __restrict__ v, int32_t npairs, int32_t* __restrict__ cnt) {
  int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npairs) return;
#pragma unroll
  for (int a = 0; a < S; ++a) {
    const int32_t j = v[S * k + a];
    if (j >= 0) atomicAdd(&cnt[j], 1);
  }
}

template <int S>
__global__ void inc_fill_kernel(const int32_t* __restrict__ v, int32_t npairs, int32_t* __restrict__ cursor,
                                int32_t* __restrict__ ent) {
  int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npairs) return;
#pragma unroll
  for (int a = 0; a < S; ++a) {
    const int32_t j = v[S * k + a];
    if (j < 0) continue;
    int32_t s = atomicAdd(&cursor[j], 1);
    ent[s] = S * k + a;
  }
}

// Sort each vertex's incidence list (keys are unique: S * pair + slot) into
// a second array, one wave per vertex: each lane ranks its keys against the
// whole list (any length), then scatters them to their rank.
__global__ void __launch_bounds__(256) inc_sort_kernel(int32_t nverts, const int32_t* __restrict__ verts,
                                                       const int32_t* __restrict__ ptr, const int32_t* __restrict__ ent,
                                                       int32_t* __restrict__ out) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const int64_t w = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / PDIPC_WAVE;
  if (w >= nverts) return;
  const int32_t v = verts[w];
  const int32_t b = ptr[v], e = ptr[v + 1], cnt = e - b;
  for (int32_t i = lane; i < cnt; i += PDIPC_WAVE) {
    const int32_t key = ent[b + i];
    int32_t rank = 0;
    for (int32_t j = 0; j < cnt; ++j) rank += ent[b + j] < key ? 1 : 0;
    out[b + rank] = key;
  }
}

// cflag[v] = 1 for a free vertex touched by at least one pair (from the
// entry counts).  With prev, the change against prev as well: out[0] = 1 if
// any flag differs, out[1] / out[2] = vertices that left / entered (wave
// ballots, one integer atomic per wave), and the first cap of each kind listed
// (in no particular order).
__global__ void __launch_bounds__(256) cflag_kernel(int32_t n, const int32_t* __restrict__ cnt,
                                                    const uint8_t* __restrict__ fixed, int32_t* __restrict__ cflag,
                                                    const int32_t* __restrict__ prev, int32_t* __restrict__ out,
                                                    int32_t* __restrict__ rem_ids, int32_t* __restrict__ add_ids,
                                                    int32_t cap) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool c = v < n && cnt[v] > 0 && !fixed[v];
  if (v <= n) cflag[v] = c ? 1 : 0;
  if (!prev) return;
  const bool p = v <= n && prev[v] != 0;
  const uint64_t mr = __ballot(p && !c), ma = __ballot(c && !p);
  if ((mr | ma) == 0) return;
  int32_t br = 0, ba = 0;
  if (threadIdx.x % PDIPC_WAVE == 0) {
    out[0] = 1;
    if (mr) br = atomicAdd(out + 1, static_cast<int32_t>(__popcll(mr)));
    if (ma) ba = atomicAdd(out + 2, static_cast<int32_t>(__popcll(ma)));
  }
  if (!rem_ids) return;
  br = __shfl(br, 0, PDIPC_WAVE);
  ba = __shfl(ba, 0, PDIPC_WAVE);
  if (p && !c) {
    const int32_t slot = br + lanes_below(mr);
    if (slot < cap) rem_ids[slot] = static_cast<int32_t>(v);
  } else if (c && !p) {
    const int32_t slot = ba + lanes_below(ma);
    if (slot < cap) add_ids[slot] = static_cast<int32_t>(v);
  }
}

__global__ void clist_kernel(int32_t n, const int32_t* __restrict__ cflag, const int32_t* __restrict__ cidx,
                             int32_t* __restrict__ clist) {
  int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (cflag[v]) clist[cidx[v]] = v;
}

void build_incidence(const PairSlots& ps, int32_t npairs, int32_t n, const uint8_t* fixed, Incidence& inc,
                     void* scan_temp, hipStream_t st, const int32_t* prev_cflag, int32_t* rem_ids, int32_t* add_ids,
                     int32_t cap) {
  // counts and (with prev_cflag) the three change counters start at zero
  launch_fill2_i32(inc.cnt, n + 1LL, inc.d_nc + 1, prev_cflag ? 3 : 0, 0, st);
  if (npairs > 0) {
    if (ps.S == 4) inc_count_kernel<4><<<grid_for(npairs, 256), 256, 0, st>>>(ps.v, npairs, inc.cnt);
    else inc_count_kernel<kSlotsW><<<grid_for(npairs, 256), 256, 0, st>>>(ps.v, npairs, inc.cnt);
  }
  cflag_kernel<<<grid_for(n + 1LL, 256), 256, 0, st>>>(n, inc.cnt, fixed, inc.cflag, prev_cflag, inc.d_nc + 1,
                                                        rem_ids, add_ids, cap);
  {
    // entry offsets (cursor: a copy of them) and c ranks in the same two launches
    const ScanJob jobs[2] = {{inc.cnt, inc.ptr, n + 1LL, inc.d_nc + 4, inc.cursor, -1, nullptr},
                             {inc.cflag, inc.cidx, n + 1LL, inc.d_nc, nullptr, -1, nullptr}};
    launch_exclusive_scans(jobs, 2, scan_temp, st);
  }
  if (npairs > 0) {
    if (ps.S == 4) inc_fill_kernel<4><<<grid_for(npairs, 256), 256, 0, st>>>(ps.v, npairs, inc.cursor, inc.raw);
    else inc_fill_kernel<kSlotsW><<<grid_for(npairs, 256), 256, 0, st>>>(ps.v, npairs, inc.cursor, inc.raw);
    inc_sort_kernel<<<grid_for(inc.nverts, 4), 256, 0, st>>>(inc.nverts, inc.verts, inc.ptr, inc.raw, inc.ent);
  }
  clist_kernel<<<grid_for(n, 256), 256, 0, st>>>(n, inc.cflag, inc.cidx, inc.clist);
}

// g[v] += sum of the pair gradient rows at v over its incidence entries (free
// vertices only): one wave per vertex, lanes over entries, then a fixed-order
// wave sum.
template <int S>
__global__ void __launch_bounds__(256) add_barrier_grad_kernel(int32_t nverts, const int32_t* __restrict__ verts,
                                                               const int32_t* __restrict__ ptr,
                                                               const int32_t* __restrict__ ent,
                                                               const double* __restrict__ grad, int32_t npairs,
                                                               const uint8_t* __restrict__ fixed,
                                                               double* __restrict__ g) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * (256 / PDIPC_WAVE) + threadIdx.x / PDIPC_WAVE;
  if (i >= nverts) return;
  const int32_t v = verts[i];
  const int32_t b = ptr[v], e = ptr[v + 1];
  if (fixed[v] || e == b) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 4
  for (int32_t t = b + lane; t < e; t += PDIPC_WAVE) {
    const int32_t k = ent[t] / S, a = ent[t] % S;
    s0 += grad[static_cast<int64_t>(3 * a) * npairs + k];
    s1 += grad[static_cast<int64_t>(3 * a + 1) * npairs + k];
    s2 += grad[static_cast<int64_t>(3 * a + 2) * npairs + k];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) {
    g[3 * v] += s0;
    g[3 * v + 1] += s1;
    g[3 * v + 2] += s2;
  }
}

void launch_add_barrier_grad(const Incidence& inc, const PairSlots& ps, int32_t npairs, const uint8_t* fixed,
                             double* g, hipStream_t st) {
  if (npairs <= 0) return;
  const unsigned grid = grid_for(inc.nverts, 256 / PDIPC_WAVE);
  if (ps.S == 4)
    add_barrier_grad_kernel<4><<<grid, 256, 0, st>>>(inc.nverts, inc.verts, inc.ptr, inc.ent, ps.grad, npairs, fixed,
                                                     g);
  else
    add_barrier_grad_kernel<kSlotsW><<<grid, 256, 0, st>>>(inc.nverts, inc.verts, inc.ptr, inc.ent, ps.grad, npairs,
                                                           fixed, g);
}

// ---- reduced contact system ----------------------------------------------------------
__global__ void c_to_x2_kernel(int32_t nc, const int32_t* __restrict__ clist, const int32_t* __restrict__ vert2x2,
                               int32_t* __restrict__ c_x2) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc) c_x2[i] = vert2x2[clist[i]];
}
void launch_c_to_x2(int32_t nc, const int32_t* clist, const int32_t* vert2x2, int32_t* c_x2, hipStream_t st) {
  if (nc > 0) c_to_x2_kernel<<<grid_for(nc, 256), 256, 0, st>>>(nc, clist, vert2x2, c_x2);
}

// Row block a of M = C^-1 + B_check in one pass: one workgroup per contact
// vertex and block of up to RB_LDS_N columns (grid y), so that the block's
// three rows fit in LDS.  The 9 S products of
// each incidence entry (3 rows x S slots x 3 columns) are formed by all
// threads, RB_GROUPS x (256 / 9 S) entries at a time with every thread's loads
// for its RB_GROUPS entries issued together, and staged in LDS with their
// target column; the first 9 S threads then add those in the block to the
// three rows (LDS) entry by entry in incidence order (deterministic: the slots
// of one pair name distinct vertices), and the rows are written with the
// C^-1 = C_s^-1 (x) I3 part added.
constexpr int RB_LDS_N = 2048;
constexpr int RB_GROUPS = 4;
template <int S>
__global__ void __launch_bounds__(256) assemble_rows_kernel(int32_t nc, const double* __restrict__ Cinv,
                                                            const int32_t* __restrict__ clist,
                                                            const int32_t* __restrict__ ptr,
                                                            const int32_t* __restrict__ ent,
                                                            const int32_t* __restrict__ vslot,
                                                            const int32_t* __restrict__ cflag,
                                                            const int32_t* __restrict__ cidx,
                                                            const double* __restrict__ U, int32_t npairs,
                                                            double* __restrict__ M) {
  constexpr int NP = 9 * S;                   // products per incidence entry
  constexpr int CHUNK = 256 / NP;             // entries per group of 256 threads
  constexpr int PASS = RB_GROUPS * CHUNK;     // entries per pass
  extern __shared__ unsigned char smem_raw[];
  double* R = reinterpret_cast<double*>(smem_raw);     // 3 x Wc
  __shared__ double P[PASS * NP];
  __shared__ int32_t Q[PASS * NP];
  const int tid = threadIdx.x;
  const int64_t ca = blockIdx.x;
  const int64_t N = 3 * static_cast<int64_t>(nc);
  const int64_t c0 = static_cast<int64_t>(blockIdx.y) * RB_LDS_N;
  const int64_t Wc = N - c0 < RB_LDS_N ? N - c0 : RB_LDS_N;
  for (int64_t i = tid; i < 3 * Wc; i += blockDim.x) R[i] = 0.0;
  const int32_t va = clist[ca];
  const int32_t t0 = ptr[va], t1 = ptr[va + 1];
  const int e = tid / NP, lp = tid % NP;
  const int lb = lp / 9, r = (lp % 9) / 3, sc = lp % 3;
  for (int32_t tc = t0; tc < t1; tc += PASS) {
    if (e < CHUNK) {
      // entry g of this thread: tc + e + CHUNK g; an entry past the end, or a
      // slot that is not in c, reads pair 0 and slot vertex 0 and adds nothing
      int32_t k[RB_GROUPS], la[RB_GROUPS], vb[RB_GROUPS];
      bool ok[RB_GROUPS];
#pragma unroll
      for (int g = 0; g < RB_GROUPS; ++g) {
        const int32_t t = tc + e + CHUNK * g;
        ok[g] = t < t1;
        const int32_t en = ent[ok[g] ? t : t0];
        k[g] = en / S;
        la[g] = en % S;
      }
      double ua[RB_GROUPS][5], ub[RB_GROUPS][5];
#pragma unroll
      for (int g = 0; g < RB_GROUPS; ++g) {
        vb[g] = vslot[S * k[g] + lb];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          ua[g][c] = U[static_cast<int64_t>(5 * (3 * la[g] + r) + c) * npairs + k[g]];
          ub[g][c] = U[static_cast<int64_t>(5 * (3 * lb + sc) + c) * npairs + k[g]];
        }
      }
      int32_t fl[RB_GROUPS], ci[RB_GROUPS];
#pragma unroll
      for (int g = 0; g < RB_GROUPS; ++g) {
        const int32_t v = vb[g] >= 0 ? vb[g] : 0;
        fl[g] = cflag[v];
        ci[g] = cidx[v];
      }
#pragma unroll
      for (int g = 0; g < RB_GROUPS; ++g) {
        double acc = 0.0;
        int32_t q = -1;
        const int64_t col = 3 * static_cast<int64_t>(ci[g]) + sc - c0;
        if (ok[g] && vb[g] >= 0 && fl[g] && col >= 0 && col < Wc) {
#pragma unroll
          for (int c = 0; c < 5; ++c) acc += ua[g][c] * ub[g][c];
          q = static_cast<int32_t>(r * Wc + col);
        }
        P[(g * CHUNK + e) * NP + lp] = acc;
        Q[(g * CHUNK + e) * NP + lp] = q;
      }
    }
    __syncthreads();
    if (tid < NP) {
      const int ne = min(PASS, t1 - tc);
      for (int ee = 0; ee < ne; ++ee) {
        const int32_t q = Q[ee * NP + tid];
        if (q >= 0) R[q] += P[ee * NP + tid];
      }
    }
    __syncthreads();
  }
  if (t0 >= t1) __syncthreads();               // R zeroed by every thread
  for (int rr = 0; rr < 3; ++rr)
    for (int64_t cl = tid; cl < Wc; cl += blockDim.x) {
      const int64_t col = c0 + cl;
      const double kron = (col % 3 == rr) ? Cinv[ca * nc + col / 3] : 0.0;
      M[(3 * ca + rr) * N + col] = kron + R[rr * Wc + cl];
    }
}

void launch_assemble_reduced(int32_t nc, const double* Cinv, const Incidence& inc, const PairSlots& ps,
                             int32_t npairs, double* M, hipStream_t st) {
  const int64_t N = 3 * static_cast<int64_t>(nc);
  if (nc <= 0) return;
  const size_t shm = sizeof(double) * 3 * (N < RB_LDS_N ? N : RB_LDS_N);
  const dim3 grid(static_cast<unsigned>(nc), static_cast<unsigned>((N + RB_LDS_N - 1) / RB_LDS_N));
  if (ps.S == 4)
    assemble_rows_kernel<4><<<grid, 256, shm, st>>>(nc, Cinv, inc.clist, inc.ptr, inc.ent, ps.v, inc.cflag, inc.cidx,
                                                    ps.U, npairs, M);
  else
    assemble_rows_kernel<kSlotsW><<<grid, 256, shm, st>>>(nc, Cinv, inc.clist, inc.ptr, inc.ent, ps.v, inc.cflag,
                                                          inc.cidx, ps.U, npairs, M);
}

// w_k = U_k^T u_local (5 per pair), u indexed by the c index of each free slot
template <int S>
__global__ void pair_ut_kernel(int32_t npairs, const int32_t* __restrict__ vslot, const int32_t* __restrict__ cflag,
                               const int32_t* __restrict__ cidx, const double* __restrict__ U,
                               const double* __restrict__ u, double* __restrict__ w) {
  int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npairs) return;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int lb = 0; lb < S; ++lb) {
    int32_t vb = vslot[S * k + lb];
    if (vb < 0 || !cflag[vb]) continue;
    int64_t cb = cidx[vb];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      double us = u[3 * cb + s];
#pragma unroll
      for (int c = 0; c < 5; ++c) acc[c] += U[static_cast<int64_t>(5 * (3 * lb + s) + c) * npairs + k] * us;
    }
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) w[static_cast<int64_t>(c) * npairs + k] = acc[c];
}

// v_a = sum over incident (pair k, slot l) of U_{k,l} w_k: one wave per c
// vertex, lanes over its incidence entries, then a fixed-order wave sum.
template <int S>
__global__ void __launch_bounds__(256) bu_gather_kernel(int32_t nc, const int32_t* __restrict__ clist,
                                                        const int32_t* __restrict__ ptr, const int32_t* __restrict__ ent,
                                                        const double* __restrict__ U, const double* __restrict__ w,
                                                        int32_t npairs, double* __restrict__ v) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const int64_t ca = static_cast<int64_t>(blockIdx.x) * (256 / PDIPC_WAVE) + threadIdx.x / PDIPC_WAVE;
  if (ca >= nc) return;
  const int32_t va = clist[ca];
  double s[3] = {0, 0, 0};
#pragma unroll 4
  for (int32_t t = ptr[va] + lane; t < ptr[va + 1]; t += PDIPC_WAVE) {
    const int32_t k = ent[t] / S, la = ent[t] % S;
    double wk[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) wk[c] = w[static_cast<int64_t>(c) * npairs + k];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 5; ++c) s[r] += U[static_cast<int64_t>(5 * (3 * la + r) + c) * npairs + k] * wk[c];
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) s[r] = wave_sum(s[r]);
  if (lane == 0)
#pragma unroll
    for (int r = 0; r < 3; ++r) v[3 * ca + r] = s[r];
}

void launch_bcheck_apply(int32_t nc, const Incidence& inc, const PairSlots& ps, int32_t npairs, const uint8_t* fixed,
                         const double* u, double* wtmp, double* v, hipStream_t st) {
  (void)fixed;
  if (nc <= 0) return;
  const unsigned gp = grid_for(npairs, 256), gc = grid_for(nc, 256 / PDIPC_WAVE);
  if (ps.S == 4) {
    pair_ut_kernel<4><<<gp, 256, 0, st>>>(npairs, ps.v, inc.cflag, inc.cidx, ps.U, u, wtmp);
    bu_gather_kernel<4><<<gc, 256, 0, st>>>(nc, inc.clist, inc.ptr, inc.ent, ps.U, wtmp, npairs, v);
  } else {
    pair_ut_kernel<kSlotsW><<<gp, 256, 0, st>>>(npairs, ps.v, inc.cflag, inc.cidx, ps.U, u, wtmp);
    bu_gather_kernel<kSlotsW><<<gc, 256, 0, st>>>(nc, inc.clist, inc.ptr, inc.ent, ps.U, wtmp, npairs, v);
  }
}

}  // namespace pdipc
