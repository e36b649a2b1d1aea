// Dense symmetric-positive-definite kernels for the reduced contact system of
// Eq. (11) and the inverse Schur complement Sigma^-1 (Section 3.2): blocked
// right-looking Cholesky (64-wide blocks, trailing updates on the matrix
// cores), triangular solves, and the inverse through L^-1 and a Gram product.
// Row-major, lower triangle.
#include "common.h"
#include "kernels.h"

namespace pdipc {

namespace {
constexpr int NB = 64;
}

// ---- Cholesky -----------------------------------------------------------------
// Right-looking, blocked (NB = 32 or 64).  Outputs: L (lower, row-major), its
// transpose Lt (upper, row-major), the reciprocals of the diagonal, dinv, and
// the inverses of the diagonal blocks L_kk^-1 (for the panels and the solves);
// Lt, dinv and the block inverses share the auxiliary buffer (dense_aux_size
// entries).  A is the workspace (its lower tiles are destroyed).  Per block
// step k: one launch, one workgroup per trailing tile (i, j), k < j <= i: the
// panels L_ik = A_ik (L_kk^-1)^T and L_jk, then A_ij -= L_ik L_jk^T, both on the
// matrix cores; the workgroups of column k+1 store the panels, and the
// workgroup of tile (k+1, k+1) factors and inverts it.
// Diagonal tiles are factored by one wave: lane r keeps row r in registers,
// step j broadcasts the pivot by readlane and column j through LDS.  Ragged
// last blocks are padded with the identity.

template <typename T>
struct MfmaVec;
template <>
struct MfmaVec<double> {
  typedef double type __attribute__((ext_vector_type(4)));
};
template <>
struct MfmaVec<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};

// D (16x16) += A (16x4) B (4x16); lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds column l % 16 of D.  Element q of its result is
// row 4 (l / 16) + q for the FP32 instruction and row l / 16 + 4 q for the
// FP64 one (both checked on the device).
template <typename T>
__device__ __forceinline__ int mfma_row(int lk, int q) {
  return sizeof(T) == 8 ? lk + 4 * q : 4 * lk + q;
}
__device__ __forceinline__ MfmaVec<double>::type mfma16x16x4(double a, double b, MfmaVec<double>::type c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ MfmaVec<float>::type mfma16x16x4(float a, float b, MfmaVec<float>::type c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double read_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ float read_lane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// 1/sqrt(d) for d > 0: hardware estimate, then Newton steps y <- y (3 - d y^2) / 2
// (two for FP64, one for FP32; each squares the relative error).
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
  y = y * (1.5 - h * y * y);
  y = y * (1.5 - h * y * y);
  return y;
}
__device__ __forceinline__ float rsqrt_nr(float d) {
  float y = __builtin_amdgcn_rsqf(d);
  return y * (1.5f - 0.5f * d * y * y);
}

// Factor and invert the 16 x 16 block W[o..o+16)[o..o+16) of a 32-wide
// diagonal tile with one wave.  Lanes 0-15 hold its rows; lanes 32-47 carry
// the identity through the same steps and so forward-substitute it, ending
// with column c of the block's inverse in lane 32 + c.  Per pivot the next
// column is updated first (one readlane), so the chain from one pivot to the
// next is rsqrt -> mul -> fma -> readlane; the other columns take the column of
// L from LDS.  The inverse goes to Xs, 1 / diag to dk[o..o+16).  Pivots are
// kept as they come: a non-positive one turns the rest of the factor into
// NaN, and the first such column (tile index + 1, below kb) goes to first_bad
// from one ballot at the end.  The unrolled loop is free of branches, so the
// row stays in registers.
template <typename T, int LD = 33>
__device__ __forceinline__ void factor_invert16(const T (*W)[LD], int o, T (*Xs)[17], T* dk, int kb,
                                                int& first_bad) {
  __shared__ T bc[PDIPC_WAVE];
  __shared__ T piv[16];
  const int lane = threadIdx.x;
  const int rr = lane & 15;
  const bool rowlane = lane < 16;
  T a[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) a[c] = rowlane ? W[o + rr][o + c] : (c == rr ? T(1) : T(0));
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const T d = read_lane(a[j], j);
    piv[j] = d;
    const T isd = rsqrt_nr(d);
    dk[o + j] = isd;
    const T l = a[j] * isd;             // lane j: d / sqrt(d)
    a[j] = l;
    if (j + 1 < 16) {
      const T ln = read_lane(l, j + 1);
      a[j + 1] -= l * ln;
    }
    if (j + 2 < 16) {
      bc[lane] = l;
#pragma unroll
      for (int c = j + 2; c < 16; ++c) a[c] -= l * bc[c];
    }
  }
  if (lane >= 32 && lane < 48) {
#pragma unroll
    for (int r = 0; r < 16; ++r) Xs[r][rr] = a[r];
  }
  const bool bad = rowlane && o + rr < kb && !(piv[rr] > T(0));
  const unsigned long long m = __ballot(bad);
  if (m != 0 && first_bad == 0) first_bad = o + __ffsll(m);
  __builtin_amdgcn_wave_barrier();
}

// NB = 32 diagonal tile, factored and inverted by one wave as 2 x 2 blocks of
// 16: L11 (and L11^-1) as above, L21 = A21 L11^-T and A22 -= L21 L21^T on the
// matrix cores, L22 (and L22^-1), then (L^-1)_21 = -L22^-1 L21 L11^-1.  The
// tile W is overwritten; X receives L_kk^-1 (32 x 33), dk 1 / diag(L_kk);
// S is scratch for three 16 x 17 blocks.  The factor itself is not kept.
template <typename T, int LD = 33>
__device__ __forceinline__ void factor_invert_wave32(T (*W)[LD], T (*X)[LD], int kb, int64_t k0,
                                                     int32_t* __restrict__ info, T (*S)[17], T* dk) {
  const int lane = threadIdx.x, lr = lane & 15, lk = lane >> 4;
  T (*X11)[17] = S;
  T (*X22)[17] = S + 16;
  T (*Tm)[17] = S + 32;
  typedef typename MfmaVec<T>::type V;
  int first_bad = 0;
  factor_invert16<T, LD>(W, 0, X11, dk, kb, first_bad);
  V acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int q0 = 0; q0 < 16; q0 += 4) acc = mfma16x16x4(W[16 + lr][q0 + lk], X11[lr][q0 + lk], acc);
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int q = 0; q < 4; ++q) W[16 + mfma_row<T>(lk, q)][lr] = acc[q];        // L21
  __builtin_amdgcn_wave_barrier();
  V upd = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int p0 = 0; p0 < 16; p0 += 4) {
    const T v = W[16 + lr][p0 + lk];
    upd = mfma16x16x4(v, v, upd);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) W[16 + mfma_row<T>(lk, q)][16 + lr] -= upd[q];
  __builtin_amdgcn_wave_barrier();
  factor_invert16<T, LD>(W, 16, X22, dk, kb, first_bad);
  V t = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int p0 = 0; p0 < 16; p0 += 4) t = mfma16x16x4(W[16 + lr][p0 + lk], X11[p0 + lk][lr], t);
#pragma unroll
  for (int q = 0; q < 4; ++q) Tm[mfma_row<T>(lk, q)][lr] = t[q];
  __builtin_amdgcn_wave_barrier();
  V x21 = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int p0 = 0; p0 < 16; p0 += 4) x21 = mfma16x16x4(X22[lr][p0 + lk], Tm[p0 + lk][lr], x21);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = mfma_row<T>(lk, q);
    X[16 + r][lr] = -x21[q];
    X[r][lr] = X11[r][lr];
    X[r][16 + lr] = T(0);
    X[16 + r][16 + lr] = X22[r][lr];
  }
  if (first_bad != 0 && lane == 0 && *info == 0) *info = static_cast<int32_t>(k0 + first_bad);
}

// Stores 1 / diag(L_kk) and the inverse D of a factored 32 x 32 diagonal block
// with the whole workgroup (coalesced).
template <typename T>
__device__ __forceinline__ void store_diag32(const T (*X)[33], const T* dk, int kb, int64_t k0,
                                             T* __restrict__ dinv, T* __restrict__ D) {
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int idx = threadIdx.x + 256 * it;
    D[idx] = X[idx / 32][idx % 32];
  }
  if (threadIdx.x < kb) dinv[k0 + threadIdx.x] = dk[threadIdx.x];
}

// p[idx] if ok, else 0, with the load issued either way (from p[0] when not
// ok), so that a run of such loads has no branches and stays in flight.
template <typename T>
__device__ __forceinline__ T load_if(const T* __restrict__ p, int64_t idx, bool ok) {
  const T v = p[ok ? idx : 0];
  return ok ? v : T(0);
}

// ---- L^-1 along the factorisation (NB = 32) ----------------------------------
// The substitution L Y = I runs block by block with the factor: Y_kj =
// L_kk^-1 B_kj, then B_ij -= L_ik Y_kj for i > k, starting from B = I.  The
// working blocks B_ij (i > j) live in the strictly upper blocks of A, which the
// factorisation never touches: B_ij[r][c] at A[(j0 + c) n + i0 + r].  Block
// step k adds one workgroup per tile (i, j), i > k >= j: it forms L_ik =
// A_ik (L_kk^-1)^T as the trailing tiles do, Y_kj (B_kk = I, so Y_kk = L_kk^-1
// and B_ik starts from zero), and the update, all on the matrix cores; the
// tiles of block row k + 1 store Y_kj to F (row-major) and Yt (transposed).
// The last block row follows in a launch of its own.
template <typename T>
__device__ __forceinline__ void rhs_tile_step(T* __restrict__ A, int64_t n, int64_t k, int64_t t,
                                              T* __restrict__ F, T* __restrict__ Yt,
                                              const T* __restrict__ Dinv, unsigned char* smem_raw) {
  constexpr int NB = 32;
  T (*Ds)[NB + 1] = reinterpret_cast<T (*)[NB + 1]>(smem_raw);  // L_kk^-1
  T (*Ai)[NB + 1] = Ds + NB;                                     // A_ik, then Ta[p][r] = L_ik[r][p]
  T (*Bk)[NB + 1] = Ai + NB;                                     // B_kj, then Y_kj
  T (*Ta)[NB + 1] = Ai;
  T (*Yl)[NB + 1] = Bk;
  const int64_t bi = k + 1 + t / (k + 1), bj = t % (k + 1);
  const int64_t k0 = k * NB, i0 = bi * NB, j0 = bj * NB;
  const bool diag = bj == k;
  const int lane = threadIdx.x % PDIPC_WAVE, w = threadIdx.x / PDIPC_WAVE;
  const int rb = 16 * (w / 2), cb = 16 * (w % 2);
  const int lr = lane % 16, lk = lane / 16;
  const T* D = Dinv + k * NB * NB;
  // every load in flight before the first LDS write (B_kj is read for the
  // diagonal tile too, from block (k, k), and not used there)
  T vd[4], vi[4], vb[4], pre[4];
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int idx = threadIdx.x + 256 * it;
    const int r = idx / NB, c = idx % NB;
    vd[it] = D[idx];
    vi[it] = load_if(A, (i0 + r) * n + k0 + c, i0 + r < n);
    vb[it] = A[(j0 + r) * n + k0 + c];                    // block k is full
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = rb + mfma_row<T>(lk, q), c = cb + lr;
    pre[q] = load_if(A, (j0 + c) * n + i0 + r, !diag && i0 + r < n);
  }
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int idx = threadIdx.x + 256 * it;
    const int r = idx / NB, c = idx % NB;
    Ds[r][c] = vd[it];
    Ai[r][c] = vi[it];
    Bk[c][r] = vb[it];                                    // B_kj[c][r]
  }
  __syncthreads();
  typename MfmaVec<T>::type pm = {T(0), T(0), T(0), T(0)}, ym = {T(0), T(0), T(0), T(0)};
  {
    T a[NB / 4], d[NB / 4];
#pragma unroll
    for (int s = 0; s < NB / 4; ++s) {
      a[s] = Ai[rb + lr][4 * s + lk];
      d[s] = Ds[cb + lr][4 * s + lk];
    }
#pragma unroll
    for (int s = 0; s < NB / 4; ++s) pm = mfma16x16x4(a[s], d[s], pm);
  }
  if (!diag) {
    T d[NB / 4], b[NB / 4];
#pragma unroll
    for (int s = 0; s < NB / 4; ++s) {
      d[s] = Ds[rb + lr][4 * s + lk];
      b[s] = Bk[4 * s + lk][cb + lr];
    }
#pragma unroll
    for (int s = 0; s < NB / 4; ++s) ym = mfma16x16x4(d[s], b[s], ym);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = rb + mfma_row<T>(lk, q);
    Ta[cb + lr][r] = pm[q];
    if (!diag) Yl[r][cb + lr] = ym[q];
  }
  __syncthreads();
  T (*Yk)[NB + 1] = diag ? Ds : Yl;
  if (bi == k + 1) {
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int idx = threadIdx.x + 256 * it;
      F[(k0 + idx / NB) * n + j0 + idx % NB] = Yk[idx / NB][idx % NB];
      Yt[(j0 + idx / NB) * n + k0 + idx % NB] = Yk[idx % NB][idx / NB];
    }
  }
  typename MfmaVec<T>::type acc = {T(0), T(0), T(0), T(0)};
  {
    T a[NB / 4], b[NB / 4];
#pragma unroll
    for (int s = 0; s < NB / 4; ++s) {
      a[s] = Ta[4 * s + lk][rb + lr];
      b[s] = Yk[4 * s + lk][cb + lr];
    }
#pragma unroll
    for (int s = 0; s < NB / 4; ++s) acc = mfma16x16x4(a[s], b[s], acc);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = rb + mfma_row<T>(lk, q), c = cb + lr;
    if (i0 + r < n) A[(j0 + c) * n + i0 + r] = pre[q] - acc[q];
  }
}

// Last block row of L^-1: Y_lj = L_ll^-1 B_lj (Y_ll = L_ll^-1), one workgroup
// per block column j.
template <typename T>
__global__ void __launch_bounds__(256) chol_lastrow_kernel(const T* __restrict__ A, int64_t n, T* __restrict__ F,
                                                           T* __restrict__ Yt, const T* __restrict__ Dinv) {
  constexpr int NB = 32;
  __shared__ T Ds[NB][NB + 1];
  __shared__ T Bl[NB][NB + 1];
  __shared__ T Yl[NB][NB + 1];
  const int64_t nblk = (n + NB - 1) / NB, last = nblk - 1;
  const int64_t bj = blockIdx.x, i0 = last * NB, j0 = bj * NB;
  const int kb = static_cast<int>(n - i0);
  const bool diag = bj == last;
  const T* D = Dinv + last * NB * NB;
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int idx = threadIdx.x + 256 * it;
    Ds[idx / NB][idx % NB] = D[idx];
    const int r = idx % NB, c = idx / NB;
    Bl[r][c] = load_if(A, (j0 + c) * n + i0 + r, !diag && r < kb);
  }
  __syncthreads();
  if (!diag) {
    const int lane = threadIdx.x % PDIPC_WAVE, w = threadIdx.x / PDIPC_WAVE;
    const int rb = 16 * (w / 2), cb = 16 * (w % 2);
    const int lr = lane % 16, lk = lane / 16;
    typename MfmaVec<T>::type ym = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int q0 = 0; q0 < NB; q0 += 4) ym = mfma16x16x4(Ds[rb + lr][q0 + lk], Bl[q0 + lk][cb + lr], ym);
#pragma unroll
    for (int q = 0; q < 4; ++q) Yl[rb + mfma_row<T>(lk, q)][cb + lr] = ym[q];
  }
  __syncthreads();
  T (*Yk)[NB + 1] = diag ? Ds : Yl;
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int idx = threadIdx.x + 256 * it;
    const int p = idx / NB, c = idx % NB;
    if (p < kb && (!diag || c < kb)) F[(i0 + p) * n + j0 + c] = Yk[p][c];
    const int c2 = idx / NB, p2 = idx % NB;
    if (p2 < kb && (!diag || c2 < kb)) Yt[(j0 + c2) * n + i0 + p2] = Yk[p2][c2];
  }
}

template <typename T, int NB>
__global__ void __launch_bounds__(256) chol_first_kernel(const T* __restrict__ A, int64_t n, T* __restrict__ L,
                                                         T* __restrict__ Lt, T* __restrict__ dinv,
                                                         T* __restrict__ Dinv, int32_t* __restrict__ info) {
  static_assert(NB == 32, "32-wide blocks");
  __shared__ T W[NB][NB + 1];
  __shared__ T X[32][33];
  __shared__ T Sc[48][17];
  __shared__ T dk[NB];
  const int kb = static_cast<int>(n < NB ? n : NB);
  if (threadIdx.x == 0) *info = 0;
#pragma unroll
  for (int it = 0; it < NB * NB / 256; ++it) {
    const int idx = threadIdx.x + 256 * it;
    const int r = idx / NB, c = idx % NB;
    const bool in = r < kb && c < kb;
    W[r][c] = in ? load_if(A, r * n + c, in) : (r == c ? T(1) : T(0));
  }
  __syncthreads();
  if (threadIdx.x < PDIPC_WAVE) factor_invert_wave32<T>(W, X, kb, 0, info, Sc, dk);
  __syncthreads();
  store_diag32<T>(X, dk, kb, 0, dinv, Dinv);
}

// Block step k for tile (bi, bj), k < bj <= bi.  The panels L_bk = A_bk
// L_kk^-T are products with the stored inverse of the diagonal block (matrix
// cores), the trailing update A_ij -= L_ik L_jk^T too; the workgroups of the
// first trailing column store the panels (coalesced), and the workgroup of
// tile (k+1, k+1) factors and inverts it afterwards.  The tile to update is
// loaded together with the panel operands.
template <typename T, int NB>
__global__ void __launch_bounds__(256) chol_update_kernel(T* __restrict__ A, int64_t n, int64_t k,
                                                          T* __restrict__ L, T* __restrict__ Lt,
                                                          T* __restrict__ dinv, T* __restrict__ Dinv,
                                                          int32_t* __restrict__ info) {
  extern __shared__ unsigned char smem_raw[];
  T (*Ds)[NB + 1] = reinterpret_cast<T (*)[NB + 1]>(smem_raw);  // Ds[p][q] = (L_kk^-1)[p][q]
  T (*Ai)[NB + 1] = Ds + NB;                                     // Ai[r][q] = A[i0 + r][k0 + q]
  T (*Aj)[NB + 1] = Ai + NB;
  T (*Ta)[NB + 1] = Ai;   // then Ta[p][r] = L[i0 + r][k0 + p]
  T (*Tb)[NB + 1] = Aj;
  T (*W)[NB + 1] = Ds;    // then the tile to factor
  __shared__ T dk[NB];
  const int64_t nblk = (n + NB - 1) / NB;
  const int64_t m = nblk - k - 1;
  int64_t t = blockIdx.x, ii = 0;
  static_assert(NB == 32, "32-wide blocks");
  if (t >= m * (m + 1) / 2) {
    rhs_tile_step<T>(A, n, k, t - m * (m + 1) / 2, L, Lt, Dinv, smem_raw);
    return;
  }
  while (t >= m - ii) { t -= m - ii; ++ii; }
  const int64_t bj = k + 1 + ii, bi = bj + t;
  const int64_t k0 = k * NB, i0 = bi * NB, j0 = bj * NB;
  const bool same = bi == bj;
  const bool last = (bi == k + 1) && same;
  const int lane = threadIdx.x % PDIPC_WAVE, w = threadIdx.x / PDIPC_WAVE;
  const int rb = (NB / 2) * (w / 2), cb = (NB / 2) * (w % 2);
  const int lr = lane % 16, lk = lane / 16;
  T pre[4];
  {
    // every load in flight before the first LDS write (A_jk is read for the
    // diagonal tiles too, and not used there)
    const T* D = Dinv + k * NB * NB;
    T vd[4], vi[4], vj[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int idx = threadIdx.x + 256 * it;
      const int r = idx / NB, c = idx % NB;
      vd[it] = D[idx];
      vi[it] = load_if(A, (i0 + r) * n + k0 + c, i0 + r < n);
      vj[it] = load_if(A, (j0 + r) * n + k0 + c, j0 + r < n);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t gr = i0 + rb + mfma_row<T>(lk, q), gc = j0 + cb + lr;
      pre[q] = load_if(A, gr * n + gc, gr < n && gc < n);
    }
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int idx = threadIdx.x + 256 * it;
      const int r = idx / NB, c = idx % NB;
      Ds[r][c] = vd[it];
      Ai[r][c] = vi[it];
      Aj[r][c] = vj[it];
    }
  }
  __syncthreads();
  // panels on the matrix cores: wave w owns a 16 x 16 quadrant; a diagonal
  // tile forms one panel
  typename MfmaVec<T>::type pi = {T(0), T(0), T(0), T(0)}, pj = pi;
  {
    T ai[NB / 4], aj[NB / 4], bd[NB / 4];
#pragma unroll
    for (int s = 0; s < NB / 4; ++s) {
      ai[s] = Ai[rb + lr][4 * s + lk];
      bd[s] = Ds[cb + lr][4 * s + lk];
    }
    if (same) {
#pragma unroll
      for (int s = 0; s < NB / 4; ++s) pi = mfma16x16x4(ai[s], bd[s], pi);
    } else {
#pragma unroll
      for (int s = 0; s < NB / 4; ++s) aj[s] = Aj[rb + lr][4 * s + lk];
#pragma unroll
      for (int s = 0; s < NB / 4; ++s) {
        pi = mfma16x16x4(ai[s], bd[s], pi);
        pj = mfma16x16x4(aj[s], bd[s], pj);
      }
    }
  }
  __syncthreads();      // Ai/Aj become the transposed panels
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = rb + mfma_row<T>(lk, q), p = cb + lr;
    Ta[p][r] = pi[q];
    Tb[p][r] = pj[q];     // unused by a diagonal tile
  }
  __syncthreads();
  T (*Tbs)[NB + 1] = same ? Ta : Tb;
  {
    typename MfmaVec<T>::type acc = {T(0), T(0), T(0), T(0)};
    T av[NB / 4], bv[NB / 4];
#pragma unroll
    for (int s = 0; s < NB / 4; ++s) {
      av[s] = Ta[4 * s + lk][rb + lr];
      bv[s] = Tbs[4 * s + lk][cb + lr];
    }
#pragma unroll
    for (int s = 0; s < NB / 4; ++s) acc = mfma16x16x4(av[s], bv[s], acc);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = rb + mfma_row<T>(lk, q), c = cb + lr;
      const int64_t gr = i0 + r, gc = j0 + c;
      const T v = pre[q] - acc[q];
      if (last) W[r][c] = (gr < n && gc < n) ? v : (r == c ? T(1) : T(0));
      else if (gr < n && gc < n) A[gr * n + gc] = v;
    }
  }
  if (!last) return;
  __syncthreads();
  const int kb = static_cast<int>(n - i0 < NB ? n - i0 : NB);
  T (*X)[33] = Ai;      // the panels are consumed
  T (*Sc)[17] = reinterpret_cast<T (*)[17]>(&Aj[0][0]);
  if (threadIdx.x < PDIPC_WAVE) factor_invert_wave32<T>(W, X, kb, i0, info, Sc, dk);
  __syncthreads();
  store_diag32<T>(X, dk, kb, i0, dinv, Dinv + (k + 1) * NB * NB);
}


// ---- 64-wide blocked Cholesky with L^-1, two launches per block step ---------
// For the reduced systems of a few thousand unknowns.  Block step k:
//  panel launch: L_ik = A_ik (L_kk^-1)^T for every row block i > k (each panel
//    once, on the matrix cores, stored over A_ik), and the row k of
//    Y = L^-1: Y_kj = L_kk^-1 B_kj (Y_kk = L_kk^-1), stored to F and Yt;
//  update launch: A_ij -= L_ik L_jk^T for the trailing tiles and
//    B_ij -= L_ik Y_kj for i > k >= j (the substitution L Y = I, B = I at the
//    start, B_ij kept transposed in the strictly upper block (j, i) of A);
//    the workgroup of tile (k+1, k+1) then factors and inverts it.
// The 64 x 64 diagonal blocks are factored and inverted by one workgroup as
// 2 x 2 blocks of 32 (each by one wave, as above), the coupling blocks on the
// matrix cores.  Outputs as the 32-wide path: F = Y (lower), aux = Yt, then
// 1 / diag(L), the diagonal-block inverses (64 x 64 each) and solve scratch.
namespace {
constexpr int NB6 = 64;
constexpr int LD6 = NB6 + 1;
}

// Each wave owns a 32 x 32 quadrant (2 x 2 MFMA blocks of 16) of a 64 x 64
// product acc += op(As) op(Bs) over 64 terms: element (r, p) of the left
// operand is As[r][p] (As[p][r] when TA), element (p, c) of the right one is
// Bs[c][p] when TB, else Bs[p][c].
template <typename T, bool TA, bool TB>
__device__ __forceinline__ void tile_gemm64(const T (*As)[LD6], const T (*Bs)[LD6],
                                            typename MfmaVec<T>::type acc[2][2]) {
  const int lane = threadIdx.x % PDIPC_WAVE, w = threadIdx.x / PDIPC_WAVE;
  const int rb = 32 * (w / 2), cb = 32 * (w % 2), lr = lane % 16, lk = lane / 16;
#pragma unroll 4
  for (int p0 = 0; p0 < NB6; p0 += 4) {
    const int p = p0 + lk;
    T a[2], b[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const int r = rb + 16 * x + lr, c = cb + 16 * x + lr;
      a[x] = TA ? As[p][r] : As[r][p];
      b[x] = TB ? Bs[c][p] : Bs[p][c];
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[x][y] = mfma16x16x4(a[x], b[y], acc[x][y]);
  }
}

template <typename T>
__device__ __forceinline__ void zero_acc(typename MfmaVec<T>::type acc[2][2]) {
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = typename MfmaVec<T>::type{T(0), T(0), T(0), T(0)};
}

// Row and column of element q of block (x, y) of the calling lane's quadrant.
template <typename T>
__device__ __forceinline__ void quad_pos(int x, int y, int q, int& r, int& c) {
  const int lane = threadIdx.x % PDIPC_WAVE, w = threadIdx.x / PDIPC_WAVE;
  r = 32 * (w / 2) + 16 * x + mfma_row<T>(lane / 16, q);
  c = 32 * (w % 2) + 16 * y + lane % 16;
}

// 32 x 32 x 32 product on the matrix cores by all four waves (one 16 x 16
// block each): out[r][c] = s * sum_p a(r, p) b(p, c) with a(r, p) = A[r][p]
// and b(p, c) = Bt[c][p] (BT) or B[p][c]; operands and result are 32 x 32
// sub-blocks of LDS arrays with row stride LD6.
template <typename T, bool BT>
__device__ __forceinline__ void gemm32_lds(const T (*A)[LD6], const T (*B)[LD6], T (*out)[LD6], T s, bool accumulate) {
  const int lane = threadIdx.x % PDIPC_WAVE, w = threadIdx.x / PDIPC_WAVE;
  const int rb = 16 * (w / 2), cb = 16 * (w % 2), lr = lane % 16, lk = lane / 16;
  typename MfmaVec<T>::type acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int p0 = 0; p0 < 32; p0 += 4) {
    const int p = p0 + lk;
    acc = mfma16x16x4(A[rb + lr][p], BT ? B[cb + lr][p] : B[p][cb + lr], acc);
  }
  __syncthreads();     // operands may alias the output
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = rb + mfma_row<T>(lk, q), c = cb + lr;
    out[r][c] = (accumulate ? out[r][c] : T(0)) + s * acc[q];
  }
  __syncthreads();
}

// Factor and invert the 64 x 64 tile W (LDS, symmetric, identity beyond kb)
// with a workgroup of four waves: L11 and L11^-1 (wave 0), L21 = A21 L11^-T,
// A22 -= L21 L21^T, L22 and L22^-1 (wave 0), (L^-1)_21 = -L22^-1 L21 L11^-1.
// X receives L^-1 (64 x 64, zero above the diagonal), dk 1 / diag(L); W is
// destroyed.  The 32-wide factorisations take their scratch from parts of W
// and X that are free at the time, and L21 X11 goes where A22 was.
template <typename T>
__device__ void factor_invert_wg64(T (*W)[LD6], T (*X)[LD6], int kb, int64_t k0, int32_t* __restrict__ info,
                                   T* dk) {
  const int kb1 = kb < 32 ? kb : 32, kb2 = kb > 32 ? kb - 32 : 0;
  T (*W21)[LD6] = reinterpret_cast<T (*)[LD6]>(&W[32][0]);
  T (*W22)[LD6] = reinterpret_cast<T (*)[LD6]>(&W[32][32]);
  T (*X22)[LD6] = reinterpret_cast<T (*)[LD6]>(&X[32][32]);
  T (*X21)[LD6] = reinterpret_cast<T (*)[LD6]>(&X[32][0]);
  // scratch of the first 32-wide factorisation: rows 32.. of X (still free)
  if (threadIdx.x < PDIPC_WAVE)
    factor_invert_wave32<T, LD6>(W, X, kb1, k0, info, reinterpret_cast<T (*)[17]>(&X[32][0]), dk);
  __syncthreads();
  gemm32_lds<T, true>(W21, X, W21, T(1), false);            // L21 = A21 X11^T
  gemm32_lds<T, true>(W21, W21, W22, T(-1), true);          // A22 -= L21 L21^T
  // scratch of the second: the first block of W (consumed)
  if (threadIdx.x < PDIPC_WAVE)
    factor_invert_wave32<T, LD6>(W22, X22, kb2, k0 + 32, info, reinterpret_cast<T (*)[17]>(&W[0][0]), dk + 32);
  __syncthreads();
  gemm32_lds<T, false>(W21, X, W22, T(1), false);           // L21 X11 (where A22 was)
  gemm32_lds<T, false>(X22, W22, X21, T(-1), false);        // X21 = -X22 L21 X11
  for (int idx = threadIdx.x; idx < 32 * 32; idx += blockDim.x) X[idx / 32][32 + idx % 32] = T(0);
  __syncthreads();
}

// Each thread's 16 elements of a 64 x 64 tile, all loads in flight before the
// first LDS write (a loop with the write inside waits on every load in turn):
// S[r][c] = get(r, c), or S[c][r] when TR.
template <typename T, bool TR, typename G>
__device__ __forceinline__ void stage_tile64(T (*S)[LD6], G get) {
  T v[16];
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int idx = threadIdx.x + 256 * it;
    v[it] = get(idx / NB6, idx % NB6);
  }
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int idx = threadIdx.x + 256 * it;
    if (TR) S[idx % NB6][idx / NB6] = v[it];
    else S[idx / NB6][idx % NB6] = v[it];
  }
}

// Two tiles at once (32 loads in flight).
template <typename T, bool TR1, bool TR2, typename G1, typename G2>
__device__ __forceinline__ void stage_tiles64(T (*S1)[LD6], G1 get1, T (*S2)[LD6], G2 get2) {
  T v[16], u[16];
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int idx = threadIdx.x + 256 * it;
    v[it] = get1(idx / NB6, idx % NB6);
    u[it] = get2(idx / NB6, idx % NB6);
  }
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int idx = threadIdx.x + 256 * it, r = idx / NB6, c = idx % NB6;
    if (TR1) S1[c][r] = v[it];
    else S1[r][c] = v[it];
    if (TR2) S2[c][r] = u[it];
    else S2[r][c] = u[it];
  }
}

// Each thread's 16 elements of a 64 x 64 LDS tile to memory: put(r, c, S[r][c]).
template <typename T, typename P>
__device__ __forceinline__ void flush_tile64(const T (*S)[LD6], P put) {
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int idx = threadIdx.x + 256 * it;
    put(idx / NB6, idx % NB6, S[idx / NB6][idx % NB6]);
  }
}

// Block 0: factor and invert the first diagonal block.
template <typename T>
__global__ void __launch_bounds__(256) chol64_first_kernel(const T* __restrict__ A, int64_t n, T* __restrict__ dinv,
                                                           T* __restrict__ Dinv, int32_t* __restrict__ info) {
  __shared__ T W[NB6][LD6];
  __shared__ T X[NB6][LD6];
  __shared__ T dk[NB6];
  const int kb = static_cast<int>(n < NB6 ? n : NB6);
  if (threadIdx.x == 0) *info = 0;
  stage_tile64<T, false>(W, [&](int r, int c) {
    const bool in = r < kb && c < kb;
    return in ? load_if(A, r * n + c, in) : (r == c ? T(1) : T(0));
  });
  __syncthreads();
  factor_invert_wg64<T>(W, X, kb, 0, info, dk);
  flush_tile64<T>(X, [&](int r, int c, T v) { Dinv[r * NB6 + c] = v; });
  if (threadIdx.x < kb) dinv[threadIdx.x] = dk[threadIdx.x];
}

// Panel launch of block step k: workgroups t < m form L_ik (i = k + 1 + t);
// the others form Y_kj, j = t - m.
template <typename T>
__global__ void __launch_bounds__(256) chol64_panel_kernel(T* __restrict__ A, int64_t n, int64_t k,
                                                           T* __restrict__ F, T* __restrict__ Yt,
                                                           const T* __restrict__ Dinv) {
  __shared__ T Ds[NB6][LD6];
  __shared__ T Bs[NB6][LD6];
  const int64_t nblk = (n + NB6 - 1) / NB6, m = nblk - k - 1;
  const int64_t t = blockIdx.x, k0 = k * NB6;
  const int kb = static_cast<int>(n - k0 < NB6 ? n - k0 : NB6);
  const T* D = Dinv + k * NB6 * NB6;
  typename MfmaVec<T>::type acc[2][2];
  zero_acc<T>(acc);
  if (t < m) {
    const int64_t i0 = (k + 1 + t) * NB6;
    stage_tiles64<T, false, false>(
        Ds, [&](int r, int c) { return D[r * NB6 + c]; },
        Bs, [&](int r, int c) { return load_if(A, (i0 + r) * n + k0 + c, i0 + r < n && c < kb); });
    __syncthreads();
    tile_gemm64<T, false, true>(Bs, Ds, acc);        // L_ik[r][c] = sum_p A_ik[r][p] D[c][p]
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int r, c;
          quad_pos<T>(x, y, q, r, c);
          if (i0 + r < n && c < kb) A[(i0 + r) * n + k0 + c] = acc[x][y][q];
        }
    return;
  }
  const int64_t j = t - m, j0 = j * NB6;
  if (j == k) {
    // Y_kk = L_kk^-1
    stage_tile64<T, false>(Ds, [&](int r, int c) { return D[r * NB6 + c]; });
    __syncthreads();
    flush_tile64<T>(Ds, [&](int r, int c, T v) {
      if (r < kb && c < kb) F[(k0 + r) * n + k0 + c] = v;
    });
    flush_tile64<T>(Ds, [&](int c, int r, T) {
      if (r < kb && c < kb) Yt[(k0 + c) * n + k0 + r] = Ds[r][c];
    });
    return;
  }
  // Y_kj = L_kk^-1 B_kj, B_kj[p][c] kept at A[(j0 + c) n + k0 + p]
  // Bs[c][p] = B_kj[p][c], read along rows of A (coalesced)
  stage_tiles64<T, false, false>(
      Ds, [&](int r, int c) { return D[r * NB6 + c]; },
      Bs, [&](int c, int p) { return load_if(A, (j0 + c) * n + k0 + p, p < kb); });
  __syncthreads();
  tile_gemm64<T, false, true>(Ds, Bs, acc);          // Y[r][c] = sum_p D[r][p] B[p][c]
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int r, c;
        quad_pos<T>(x, y, q, r, c);
        if (r < kb) {
          F[(k0 + r) * n + j0 + c] = acc[x][y][q];
          Yt[(j0 + c) * n + k0 + r] = acc[x][y][q];
        }
      }
}

// Update launch of block step k: trailing tiles (bi, bj), k < bj <= bi,
// then the tiles (bi, bj), bi > k >= bj, of the substitution.
template <typename T>
__global__ void __launch_bounds__(256) chol64_update_kernel(T* __restrict__ A, int64_t n, int64_t k,
                                                            const T* __restrict__ F, T* __restrict__ dinv,
                                                            T* __restrict__ Dinv, int32_t* __restrict__ info) {
  __shared__ T Li[NB6][LD6];
  __shared__ T Lj[NB6][LD6];
  __shared__ T dk[NB6];
  const int64_t nblk = (n + NB6 - 1) / NB6, m = nblk - k - 1;
  const int64_t k0 = k * NB6;
  int64_t t = blockIdx.x;
  typename MfmaVec<T>::type acc[2][2];
  zero_acc<T>(acc);
  T pre[2][2][4];
  if (t < m * (m + 1) / 2) {
    int64_t ii = 0;
    while (t >= m - ii) { t -= m - ii; ++ii; }
    const int64_t bj = k + 1 + ii, bi = bj + t, i0 = bi * NB6, j0 = bj * NB6;
    const bool diag_next = bi == k + 1 && bj == k + 1;
    stage_tiles64<T, false, false>(
        Li, [&](int r, int c) { return load_if(A, (i0 + r) * n + k0 + c, i0 + r < n); },
        Lj, [&](int r, int c) { return load_if(A, (j0 + r) * n + k0 + c, j0 + r < n); });
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int r, c;
          quad_pos<T>(x, y, q, r, c);
          pre[x][y][q] = load_if(A, (i0 + r) * n + j0 + c, i0 + r < n && j0 + c < n);
        }
    __syncthreads();
    tile_gemm64<T, false, true>(Li, Lj, acc);        // sum_p L_ik[r][p] L_jk[c][p]
    if (!diag_next) {
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            int r, c;
            quad_pos<T>(x, y, q, r, c);
            if (i0 + r < n && j0 + c < n) A[(i0 + r) * n + j0 + c] = pre[x][y][q] - acc[x][y][q];
          }
      return;
    }
    // the next diagonal block: factor and invert it (identity beyond n)
    __syncthreads();
    T (*W)[LD6] = Li;
    T (*X)[LD6] = Lj;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int r, c;
          quad_pos<T>(x, y, q, r, c);
          W[r][c] = (i0 + r < n && j0 + c < n) ? pre[x][y][q] - acc[x][y][q] : (r == c ? T(1) : T(0));
        }
    __syncthreads();
    const int kb = static_cast<int>(n - i0 < NB6 ? n - i0 : NB6);
    factor_invert_wg64<T>(W, X, kb, i0, info, dk);
    T* D = Dinv + (k + 1) * NB6 * NB6;
    flush_tile64<T>(X, [&](int r, int c, T v) { D[r * NB6 + c] = v; });
    if (threadIdx.x < kb) dinv[i0 + threadIdx.x] = dk[threadIdx.x];
    return;
  }
  // B_ij -= L_ik Y_kj, B_ij[r][c] kept at A[(j0 + c) n + i0 + r]; B_ik starts at 0
  t -= m * (m + 1) / 2;
  const int64_t bi = k + 1 + t / (k + 1), bj = t % (k + 1), i0 = bi * NB6, j0 = bj * NB6;
  const int kb = static_cast<int>(n - k0 < NB6 ? n - k0 : NB6);     // k < bi, so block k is full
  stage_tiles64<T, false, false>(
      Li, [&](int r, int c) { return load_if(A, (i0 + r) * n + k0 + c, i0 + r < n); },       // L_ik
      Lj, [&](int r, int c) { return load_if(F, (k0 + r) * n + j0 + c, r < kb); });         // Y_kj[p = r][c]
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int r, c;
        quad_pos<T>(x, y, q, r, c);
        pre[x][y][q] = load_if(A, (j0 + c) * n + i0 + r, bj < k && i0 + r < n);
      }
  __syncthreads();
  tile_gemm64<T, false, false>(Li, Lj, acc);         // sum_p L_ik[r][p] Y_kj[p][c]
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int r, c;
        quad_pos<T>(x, y, q, r, c);
        if (i0 + r < n) A[(j0 + c) * n + i0 + r] = pre[x][y][q] - acc[x][y][q];
      }
}

// Block size: 32 below kDense64Min unknowns, where the chain of block steps
// is short and one launch per step wins; 64 above, where each panel is formed
// once and the trailing tiles need a single product (two launches per step).
// Both leave L^-1 (F) and its transpose (aux), so solves and the inverse are
// the same products.
static constexpr int64_t kDense64Min = 2049;
static int dense_block(int64_t n) { return n < kDense64Min ? 32 : 64; }

// Launches [p0, p1) of the 32-wide factorisation: launch 0 is the first
// diagonal block, launch 1 + k the block step k, the last one forms the last
// block row of L^-1.
template <typename T>
static void dense_cholesky_32(T* A, int64_t n, T* L, T* aux, int32_t* d_info, hipStream_t st, int64_t p0,
                              int64_t p1) {
  constexpr int NB = 32;
  T* Lt = aux;
  T* dinv = aux + n * n;
  T* Dinv = aux + n * n + n;
  const int64_t nblk = (n + NB - 1) / NB;
  if (p0 <= 0 && p1 > 0) chol_first_kernel<T, NB><<<1, 256, 0, st>>>(A, n, L, Lt, dinv, Dinv, d_info);
  const size_t shm = sizeof(T) * 3 * NB * (NB + 1);
  for (int64_t k = 0; k + 1 < nblk; ++k) {
    if (1 + k < p0 || 1 + k >= p1) continue;
    const int64_t m = nblk - k - 1;
    const int64_t tiles = m * (m + 1) / 2 + m * (k + 1);
    chol_update_kernel<T, NB><<<static_cast<unsigned>(tiles), 256, shm, st>>>(A, n, k, L, Lt, dinv, Dinv, d_info);
  }
  if (nblk >= p0 && nblk < p1)
    chol_lastrow_kernel<T><<<static_cast<unsigned>(nblk), 256, 0, st>>>(A, n, L, Lt, Dinv);
}

// Launches [p0, p1) of the 64-wide factorisation: launch 0 is the first
// diagonal block, then per block step k the panel launch (1 + 2k) and, but
// for the last step, the update launch (2 + 2k).
template <typename T>
static void dense_cholesky_64(T* A, int64_t n, T* F, T* aux, int32_t* d_info, hipStream_t st, int64_t p0,
                              int64_t p1) {
  T* Yt = aux;
  T* dinv = aux + n * n;
  T* Dinv = aux + n * n + n;
  const int64_t nblk = (n + NB6 - 1) / NB6;
  auto in = [&](int64_t l) { return l >= p0 && l < p1; };
  if (in(0)) chol64_first_kernel<T><<<1, 256, 0, st>>>(A, n, dinv, Dinv, d_info);
  for (int64_t k = 0; k < nblk; ++k) {
    const int64_t m = nblk - k - 1;
    if (in(1 + 2 * k))
      chol64_panel_kernel<T><<<static_cast<unsigned>(m + k + 1), 256, 0, st>>>(A, n, k, F, Yt, Dinv);
    if (m > 0 && in(2 + 2 * k))
      chol64_update_kernel<T><<<static_cast<unsigned>(m * (m + 1) / 2 + m * (k + 1)), 256, 0, st>>>(
          A, n, k, F, dinv, Dinv, d_info);
  }
}

int64_t dense_cholesky_launches(int64_t n) {
  if (n <= 0) return 0;
  if (dense_block(n) == 32) return (n + 31) / 32 + 1;
  return 2 * ((n + NB6 - 1) / NB6);
}

template <typename T>
void dense_cholesky_range(T* A, int64_t n, T* L, T* aux, int32_t* d_info, hipStream_t st, int64_t p0, int64_t p1) {
  if (n <= 0) return;
  if (dense_block(n) == 32) dense_cholesky_32<T>(A, n, L, aux, d_info, st, p0, p1);
  else dense_cholesky_64<T>(A, n, L, aux, d_info, st, p0, p1);
}

template <typename T>
void dense_cholesky(T* A, int64_t n, T* L, T* aux, int32_t* d_info, hipStream_t st) {
  dense_cholesky_range<T>(A, n, L, aux, d_info, st, 0, dense_cholesky_launches(n));
}

// Row-major triangular matrix times nrhs <= 4 vectors (n x nrhs row-major):
// y_r = sum over the columns c <= r (LOWER) or c >= r of M[r][c] x_c.  One
// wave per row, coalesced along the row.
template <typename T, bool LOWER>
__global__ void __launch_bounds__(256) tri_gemv_kernel(const T* __restrict__ M, int64_t n, const T* __restrict__ x,
                                                       T* __restrict__ y, int nrhs) {
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / PDIPC_WAVE;
  const int lane = threadIdx.x % PDIPC_WAVE;
  if (row >= n) return;
  const int64_t c0 = LOWER ? 0 : row, c1 = LOWER ? row + 1 : n;
  const T* Mr = M + row * n;
  T s[4] = {T(0), T(0), T(0), T(0)};
  if (nrhs == 1) {
    // four partial sums, so that each lane has eight loads in flight
    T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
    int64_t c = c0 + lane;
    for (; c + 3 * PDIPC_WAVE < c1; c += 4 * PDIPC_WAVE) {
      const T m0 = Mr[c], m1 = Mr[c + PDIPC_WAVE], m2 = Mr[c + 2 * PDIPC_WAVE], m3 = Mr[c + 3 * PDIPC_WAVE];
      const T x0 = x[c], x1 = x[c + PDIPC_WAVE], x2 = x[c + 2 * PDIPC_WAVE], x3 = x[c + 3 * PDIPC_WAVE];
      a0 += m0 * x0;
      a1 += m1 * x1;
      a2 += m2 * x2;
      a3 += m3 * x3;
    }
    for (; c < c1; c += PDIPC_WAVE) a0 += Mr[c] * x[c];
    s[0] = (a0 + a1) + (a2 + a3);
  } else {
    for (int64_t c = c0 + lane; c < c1; c += PDIPC_WAVE) {
      const T m = Mr[c];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < nrhs) s[q] += m * x[c * nrhs + q];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int off = PDIPC_WAVE / 2; off > 0; off /= 2) s[q] += __shfl_xor(s[q], off, PDIPC_WAVE);
  }
  if (lane < nrhs) {
    T v = s[0];
#pragma unroll
    for (int q = 1; q < 4; ++q) v = (lane == q) ? s[q] : v;
    y[row * nrhs + lane] = v;
  }
}

// x = Y^T (Y b) with Y = L^-1 (F, row-major) and Y^T (aux): two triangular
// products over all workgroups, for either block size.
template <typename T>
void dense_chol_solve(const T* L, T* aux, int64_t n, T* b, int32_t nrhs, hipStream_t st) {
  if (n <= 0) return;
  T* z = aux + dense_tmp_offset(n);
  const unsigned g = static_cast<unsigned>((n + 3) / 4);
  tri_gemv_kernel<T, true><<<g, 256, 0, st>>>(L, n, b, z, nrhs);
  tri_gemv_kernel<T, false><<<g, 256, 0, st>>>(aux, n, z, b, nrhs);
}

// Single right-hand side into a separate output.
template <typename T>
void dense_chol_solve_into(const T* F, T* aux, int64_t n, const T* b, T* x, hipStream_t st) {
  if (n <= 0) return;
  T* z = aux + dense_tmp_offset(n);
  const unsigned g = static_cast<unsigned>((n + 3) / 4);
  tri_gemv_kernel<T, true><<<g, 256, 0, st>>>(F, n, b, z, 1);
  tri_gemv_kernel<T, false><<<g, 256, 0, st>>>(aux, n, z, x, 1);
}

// ---- iterative refinement on an FP32 inverse factor (32-wide blocks) ---------
// Step s: r_s = rhs - M u_s in FP64 (u_0 = 0), res[s] = max |r_s|; unless
// res[s] <= tol res[0], u_{s+1} = u_s + S Y^T Y S r_s with the FP32 factor of
// S M S.  Every kernel of a step returns at once when the previous residual
// already met the tolerance, so several steps are queued without a readback
// (res must start at zero).
__device__ __forceinline__ bool refined(const double* res, int s, double tol) {
  return res[s] <= tol * res[0];
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = PDIPC_WAVE / 2; off > 0; off /= 2) v += __shfl_xor(v, off, PDIPC_WAVE);
  return v;
}
__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = PDIPC_WAVE / 2; off > 0; off /= 2) v += __shfl_xor(v, off, PDIPC_WAVE);
  return v;
}

__global__ void __launch_bounds__(256) refine_residual_kernel(const double* __restrict__ M, int64_t n,
                                                              const double* __restrict__ rhs,
                                                              const double* __restrict__ u,
                                                              const double* __restrict__ sc, float* __restrict__ out,
                                                              double* __restrict__ res, int s, double tol) {
  if (s > 0 && refined(res, s - 1, tol)) return;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / PDIPC_WAVE;
  const int lane = threadIdx.x % PDIPC_WAVE;
  if (row >= n) return;
  double acc = 0.0;
  if (s > 0) {
    const double* Mr = M + row * n;
    for (int64_t c = lane; c < n; c += PDIPC_WAVE) acc += Mr[c] * u[c];
    acc = wave_sum_d(acc);
  }
  if (lane == 0) {
    const double r = rhs[row] - acc;
    out[row] = static_cast<float>(sc[row] * r);
    atomicMax(reinterpret_cast<unsigned long long*>(res + s), static_cast<unsigned long long>(__double_as_longlong(fabs(r))));
  }
}

__global__ void __launch_bounds__(256) refine_lower_kernel(const float* __restrict__ Y, int64_t n,
                                                           const float* __restrict__ r, float* __restrict__ z,
                                                           const double* __restrict__ res, int s, double tol) {
  if (refined(res, s, tol)) return;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / PDIPC_WAVE;
  const int lane = threadIdx.x % PDIPC_WAVE;
  if (row >= n) return;
  const float* Yr = Y + row * n;
  float acc = 0.0f;
  for (int64_t c = lane; c <= row; c += PDIPC_WAVE) acc += Yr[c] * r[c];
  acc = wave_sum_f(acc);
  if (lane == 0) z[row] = acc;
}

__global__ void __launch_bounds__(256) refine_upper_kernel(const float* __restrict__ Yt, int64_t n,
                                                           const float* __restrict__ z, const double* __restrict__ sc,
                                                           double* __restrict__ u, const double* __restrict__ res,
                                                           int s, double tol) {
  if (refined(res, s, tol)) return;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / PDIPC_WAVE;
  const int lane = threadIdx.x % PDIPC_WAVE;
  if (row >= n) return;
  const float* Yr = Yt + row * n;
  float acc = 0.0f;
  for (int64_t c = row + lane; c < n; c += PDIPC_WAVE) acc += Yr[c] * z[c];
  acc = wave_sum_f(acc);
  if (lane == 0) u[row] += sc[row] * static_cast<double>(acc);
}

void launch_refine_residual(const double* M, int64_t n, const double* rhs, const double* u, const double* sc,
                            float* r32, double* res, int s, double tol, hipStream_t st) {
  if (n > 0)
    refine_residual_kernel<<<static_cast<unsigned>((n + 3) / 4), 256, 0, st>>>(M, n, rhs, u, sc, r32, res, s, tol);
}
void launch_refine_correct(const float* F, float* aux, int64_t n, const float* r32, const double* sc, double* u,
                           const double* res, int s, double tol, hipStream_t st) {
  if (n <= 0) return;
  float* z = aux + dense_tmp_offset(n);
  const unsigned g = static_cast<unsigned>((n + 3) / 4);
  refine_lower_kernel<<<g, 256, 0, st>>>(F, n, r32, z, res, s, tol);
  refine_upper_kernel<<<g, 256, 0, st>>>(aux, n, z, sc, u, res, s, tol);
}

// (L L^T)^-1 = Y^T Y = Yt Yt^T with Yt = Y^T (row-major, upper triangle and
// diagonal blocks valid) for 32-wide blocks: one workgroup per 32 x 32 tile
// (i, j), i >= j, summing over the column blocks p >= i of Yt on the matrix
// cores, and writing the tile and its mirror.
template <typename T>
__global__ void __launch_bounds__(256) yty_kernel(const T* __restrict__ Yt, int64_t n, T* __restrict__ C) {
  constexpr int NB = 32;
  __shared__ T As[NB][NB + 1];
  __shared__ T Bs[NB][NB + 1];
  __shared__ T Cs[NB][NB + 1];
  const int64_t nblk = (n + NB - 1) / NB;
  int64_t t = blockIdx.x, bi = 0;
  while (t > bi) { t -= bi + 1; ++bi; }
  const int64_t bj = t, i0 = bi * NB, j0 = bj * NB;
  const int lane = threadIdx.x % PDIPC_WAVE, w = threadIdx.x / PDIPC_WAVE;
  const int rb = 16 * (w / 2), cb = 16 * (w % 2);
  const int lr = lane % 16, lk = lane / 16;
  typename MfmaVec<T>::type acc = {T(0), T(0), T(0), T(0)};
  for (int64_t pb = bi; pb < nblk; ++pb) {
    const int64_t p0 = pb * NB;
#pragma unroll
    for (int it = 0; it < 4; ++it) {
      const int idx = threadIdx.x + 256 * it;
      const int r = idx / NB, c = idx % NB;
      As[r][c] = (i0 + r < n && p0 + c < n) ? Yt[(i0 + r) * n + p0 + c] : T(0);
      Bs[r][c] = (j0 + r < n && p0 + c < n) ? Yt[(j0 + r) * n + p0 + c] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int q0 = 0; q0 < NB; q0 += 4) acc = mfma16x16x4(As[rb + lr][q0 + lk], Bs[cb + lr][q0 + lk], acc);
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) Cs[rb + mfma_row<T>(lk, q)][cb + lr] = acc[q];
  __syncthreads();
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int idx = threadIdx.x + 256 * it;
    const int r = idx / NB, c = idx % NB;
    if (i0 + r < n && j0 + c < n) C[(i0 + r) * n + j0 + c] = Cs[r][c];
    if (bi != bj && j0 + r < n && i0 + c < n) C[(j0 + r) * n + i0 + c] = Cs[c][r];
  }
}

template <typename T>
void dense_chol_inverse(const T* L, const T* aux, int64_t n, T* Ainv, T* work, hipStream_t st) {
  (void)L;
  (void)work;
  if (n <= 0) return;
  const int64_t nb = (n + 31) / 32;
  yty_kernel<T><<<static_cast<unsigned>(nb * (nb + 1) / 2), 256, 0, st>>>(aux, n, Ainv);
}

// ---- conversions and residuals -------------------------------------------------------
__global__ void f64_to_f32_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = static_cast<float>(in[i]);
}
__global__ void f32_to_f64_kernel(const float* __restrict__ in, double* __restrict__ out, int64_t n) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = static_cast<double>(in[i]);
}
void launch_convert_f64_f32(const double* in, float* out, int64_t n, hipStream_t st) {
  if (n > 0) f64_to_f32_kernel<<<grid_for(n, 256), 256, 0, st>>>(in, out, n);
}
void launch_convert_f32_f64(const float* in, double* out, int64_t n, hipStream_t st) {
  if (n > 0) f32_to_f64_kernel<<<grid_for(n, 256), 256, 0, st>>>(in, out, n);
}

__global__ void __launch_bounds__(256) dense_residual_kernel(const double* __restrict__ M, int64_t n,
                                                             const double* __restrict__ b,
                                                             const double* __restrict__ u, double* __restrict__ r) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / PDIPC_WAVE;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += PDIPC_WAVE) s += M[i * n + j] * u[j];
  s = wave_sum(s);
  if (lane == 0) r[i] = b[i] - s;
}
void launch_dense_residual(const double* M, int64_t n, const double* b, const double* u, double* r, hipStream_t st) {
  if (n > 0) dense_residual_kernel<<<grid_for(n, 4), 256, 0, st>>>(M, n, b, u, r);
}

// ---- Jacobi-scaled FP32 copies for mixed-precision refinement --------------------
__global__ void diag_scale_kernel(const double* __restrict__ M, int64_t n, double* __restrict__ sc) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    double d = M[i * n + i];
    sc[i] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
  }
}
__global__ void scale_convert_matrix_kernel(const double* __restrict__ M, int64_t n, const double* __restrict__ sc,
                                            float* __restrict__ out) {
  int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx < n * n) out[idx] = static_cast<float>(sc[idx / n] * M[idx] * sc[idx % n]);
}
__global__ void scale_convert_vec_kernel(const double* __restrict__ r, int64_t n, const double* __restrict__ sc,
                                         float* __restrict__ out) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = static_cast<float>(sc[i] * r[i]);
}
__global__ void scaled_accumulate_kernel(const float* __restrict__ y, int64_t n, const double* __restrict__ sc,
                                         double* __restrict__ u) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) u[i] += sc[i] * static_cast<double>(y[i]);
}

void launch_jacobi_scaling(const double* M, int64_t n, double* sc, hipStream_t st) {
  if (n > 0) diag_scale_kernel<<<grid_for(n, 256), 256, 0, st>>>(M, n, sc);
}
void launch_scale_convert_matrix(const double* M, int64_t n, const double* sc, float* out, hipStream_t st) {
  if (n > 0) scale_convert_matrix_kernel<<<grid_for(n * n, 256), 256, 0, st>>>(M, n, sc, out);
}
void launch_scale_convert_vec(const double* r, int64_t n, const double* sc, float* out, hipStream_t st) {
  if (n > 0) scale_convert_vec_kernel<<<grid_for(n, 256), 256, 0, st>>>(r, n, sc, out);
}
void launch_scaled_accumulate(const float* y, int64_t n, const double* sc, double* u, hipStream_t st) {
  if (n > 0) scaled_accumulate_kernel<<<grid_for(n, 256), 256, 0, st>>>(y, n, sc, u);
}

template void dense_cholesky<double>(double*, int64_t, double*, double*, int32_t*, hipStream_t);
template void dense_cholesky<float>(float*, int64_t, float*, float*, int32_t*, hipStream_t);
template void dense_cholesky_range<double>(double*, int64_t, double*, double*, int32_t*, hipStream_t, int64_t,
                                           int64_t);
template void dense_cholesky_range<float>(float*, int64_t, float*, float*, int32_t*, hipStream_t, int64_t, int64_t);
template void dense_chol_solve<double>(const double*, double*, int64_t, double*, int32_t, hipStream_t);
template void dense_chol_solve<float>(const float*, float*, int64_t, float*, int32_t, hipStream_t);
template void dense_chol_solve_into<double>(const double*, double*, int64_t, const double*, double*, hipStream_t);
template void dense_chol_solve_into<float>(const float*, float*, int64_t, const float*, float*, hipStream_t);
template void dense_chol_inverse<double>(const double*, const double*, int64_t, double*, double*, hipStream_t);
template void dense_chol_inverse<float>(const float*, const float*, int64_t, float*, float*, hipStream_t);

}  // namespace pdipc
