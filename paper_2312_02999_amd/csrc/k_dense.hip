// Dense symmetric-positive-definite kernels for the reduced contact system of
// Eq. (11) and the inverse Schur complement Sigma^-1 (Section 3.2): blocked
// right-looking Cholesky (64-wide panels), triangular solves, and the inverse
// through L^-1 and a Gram product.  Row-major, lower triangle.
#include "common.h"
#include "kernels.h"

namespace pdipc {

namespace {
constexpr int NB = 64;
}

// ---- tiled GEMM: C = beta C + alpha op(A) op(B), 64x64 tiles, K chunks of 16 ----
template <typename T, bool TA, bool TB>
__global__ void __launch_bounds__(256) gemm_kernel(int64_t M, int64_t N, int64_t K, T alpha, const T* __restrict__ A,
                                                   int64_t lda, const T* __restrict__ B, int64_t ldb, T beta,
                                                   T* __restrict__ C, int64_t ldc, int lower_only) {
  const int64_t ti = blockIdx.y, tj = blockIdx.x;
  if (lower_only && tj > ti) return;
  __shared__ T As[16][64 + 1];
  __shared__ T Bs[16][64 + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = T(0);
  const int64_t i0 = ti * 64, j0 = tj * 64;
  T pa[4], pb[4];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int idx = threadIdx.x + 256 * u;
      int kk = idx / 64, r = idx % 64;
      int64_t gi = i0 + r, gk = k0 + kk, gj = j0 + r;
      pa[u] = (gi < M && gk < K) ? (TA ? A[gk * lda + gi] : A[gi * lda + gk]) : T(0);
      pb[u] = (gj < N && gk < K) ? (TB ? B[gj * ldb + gk] : B[gk * ldb + gj]) : T(0);
    }
  };
  fetch(0);
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int idx = threadIdx.x + 256 * u;
      As[idx / 64][idx % 64] = pa[u];
      Bs[idx / 64][idx % 64] = pb[u];
    }
    __syncthreads();
    if (k0 + 16 < K) fetch(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ty + 16 * q];
        b[q] = Bs[kk][tx + 16 * q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int64_t gi = i0 + ty + 16 * p, gj = j0 + tx + 16 * q;
      if (gi < M && gj < N && (!lower_only || gj <= gi)) {
        T old = beta == T(0) ? T(0) : C[gi * ldc + gj];
        C[gi * ldc + gj] = beta * old + alpha * acc[p][q];
      }
    }
}

// ---- Cholesky -----------------------------------------------------------------
// Right-looking with 64-wide blocks, one launch per block step.  Step k (k >= 0)
// handles the trailing lower tiles (i, j), k < j <= i:
//   P_i = A_ik Linv_k^T          (panel solve via the stored inverse of L_kk)
//   A_ij -= P_i P_j^T            (trailing update)
// the diagonal tile (i, i) also writes P_i into L, and tile (k+1, k+1), after
// its last update, factors itself and stores the inverse of L_{k+1,k+1}.
// A is the workspace (destroyed); the off-diagonal blocks of L and the
// diagonal-block inverses are the outputs (the solves never need L_kk).
// Ragged last blocks are padded with the identity.

// Factor the 64x64 tile held in LDS (lower part; rows and columns beyond kb
// are the identity) and write the inverse of its Cholesky factor to Linv
// (global, 64 x 64 row-major).  256 threads; thread (ty, tx) keeps rows
// 4ty..4ty+3 x columns 4tx..4tx+3 of the tile and of the inverse in
// registers.  Step j broadcasts column j of the tile and row j of the
// inverse through double-buffered LDS vectors:
//   L[:, j] = T[:, j] / sqrt(T[j][j]);  T[i][l] -= L[i][j] L[l][j]  (i, l > j)
//   X[j, :] /= L[j][j];                 X[i, :] -= L[i][j] X[j, :]  (i > j)
// starting from X = I, which leaves X = L^-1 (forward elimination on I).
template <typename T>
__device__ void tile_factor_inverse(const T (*Tl)[NB + 1], T* __restrict__ Linv, int kb, int64_t k0,
                                    int32_t* info, T (*colbuf)[NB], T (*rowbuf)[NB]) {
  const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
  const int r0 = 4 * ty, c0 = 4 * tx;
  T tr[4][4], xr[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      tr[a][b] = Tl[r0 + a][c0 + b];
      xr[a][b] = (r0 + a == c0 + b) ? T(1) : T(0);
    }
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    const int buf = j & 1;
    if (j >= c0 && j < c0 + 4) {
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (c0 + b == j)
#pragma unroll
          for (int a = 0; a < 4; ++a) colbuf[buf][r0 + a] = tr[a][b];
    }
    __syncthreads();
    T d = colbuf[buf][j];
    if (!(d > T(0))) {
      if (j < kb && threadIdx.x == 0 && *info == 0) *info = static_cast<int32_t>(k0 + j + 1);
      d = T(1);
    }
    const T sd = sqrt(d), isd = T(1) / sd;
    T lr[4], lc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      lr[a] = colbuf[buf][r0 + a] * isd;
      lc[a] = colbuf[buf][c0 + a] * isd;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = r0 + a, l = c0 + b;
        if (i > j && l > j && l <= i) tr[a][b] -= lr[a] * lc[b];
      }
    if (j >= r0 && j < r0 + 4) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (r0 + a == j)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            xr[a][b] *= isd;
            rowbuf[buf][c0 + b] = xr[a][b];
          }
    }
    __syncthreads();
    T xj[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) xj[b] = rowbuf[buf][c0 + b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      if (r0 + a > j)
#pragma unroll
        for (int b = 0; b < 4; ++b) xr[a][b] -= lr[a] * xj[b];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) Linv[(r0 + a) * NB + c0 + b] = xr[a][b];
}

template <typename T>
__global__ void __launch_bounds__(256) chol_first_kernel(const T* __restrict__ A, int64_t n, T* __restrict__ L,
                                                         T* __restrict__ Linv, int32_t* __restrict__ info) {
  __shared__ T Tl[NB][NB + 1];
  __shared__ T colbuf[2][NB];
  __shared__ T rowbuf[2][NB];
  const int kb = static_cast<int>(n < NB ? n : NB);
  if (threadIdx.x == 0) *info = 0;
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
    int r = idx / NB, c = idx % NB;
    Tl[r][c] = (r < kb && c < kb) ? A[r * n + c] : (r == c ? T(1) : T(0));
  }
  __syncthreads();
  tile_factor_inverse<T>(Tl, Linv, kb, 0, info, colbuf, rowbuf);
  (void)L;
}

// P = Araw Linv^T into LDS (rows beyond the matrix are zero)
template <typename T>
__device__ void panel_times_linvT(const T* __restrict__ A, int64_t n, int64_t r0, int64_t k0, const T (*Li)[NB + 1],
                                  T (*Raw)[NB + 1], T (*P)[NB + 1]) {
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
    int r = idx / NB, c = idx % NB;
    int64_t gr = r0 + r, gc = k0 + c;
    Raw[r][c] = (gr < n && gc < n) ? A[gr * n + gc] : T(0);
  }
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = T(0);
  for (int p = 0; p < NB; ++p) {
    T x[4], y[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      x[q] = Raw[ty + 16 * q][p];
      y[q] = Li[tx + 16 * q][p];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) P[ty + 16 * a][tx + 16 * b] = acc[a][b];
  __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(256) chol_step_kernel(T* __restrict__ A, int64_t n, int64_t k, T* __restrict__ L,
                                                        T* __restrict__ Linv, int32_t* __restrict__ info) {
  extern __shared__ unsigned char smem_raw[];
  T (*Li)[NB + 1] = reinterpret_cast<T (*)[NB + 1]>(smem_raw);
  T (*Pi)[NB + 1] = Li + NB;
  T (*Pj)[NB + 1] = Pi + NB;
  T (*Wk)[NB + 1] = Pj + NB;            // scratch: raw panel, then the tile
  const int64_t nblk = (n + NB - 1) / NB;
  // tile index -> (i, j) with k < j <= i < nblk
  const int64_t m = nblk - k - 1;
  int64_t t = blockIdx.x, ii = 0;
  while (t >= m - ii) { t -= m - ii; ++ii; }
  const int64_t bj = k + 1 + ii, bi = bj + t;
  const int64_t k0 = k * NB, i0 = bi * NB, j0 = bj * NB;
  const T* Lk = Linv + k * NB * NB;
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) Li[idx / NB][idx % NB] = Lk[idx];
  __syncthreads();
  panel_times_linvT<T>(A, n, i0, k0, Li, Wk, Pi);
  if (bi != bj) panel_times_linvT<T>(A, n, j0, k0, Li, Wk, Pj);
  T (*Q)[NB + 1] = (bi != bj) ? Pj : Pi;
  if (bi == bj) {
    for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
      int r = idx / NB, c = idx % NB;
      int64_t gr = i0 + r, gc = k0 + c;
      if (gr < n && gc < n) L[gr * n + gc] = Pi[r][c];
    }
  }
  // trailing update of tile (bi, bj), kept in Wk
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = T(0);
  for (int p = 0; p < NB; ++p) {
    T x[4], y[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      x[q] = Pi[ty + 16 * q][p];
      y[q] = Q[tx + 16 * q][p];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
  }
  __syncthreads();
  const bool last = (bi == k + 1) && (bj == k + 1);
  const int kb = static_cast<int>(n - i0 < NB ? n - i0 : NB);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int r = ty + 16 * a, c = tx + 16 * b;
      int64_t gr = i0 + r, gc = j0 + c;
      T v;
      if (gr < n && gc < n) {
        v = A[gr * n + gc] - acc[a][b];
        if (!last) A[gr * n + gc] = v;
      } else {
        v = (r == c) ? T(1) : T(0);
      }
      Wk[r][c] = v;
    }
  __syncthreads();
  if (!last) return;
  // factor the next diagonal tile and store the inverse of its factor
  T (*colbuf)[NB] = reinterpret_cast<T (*)[NB]>(&Pi[0][0]);
  T (*rowbuf)[NB] = reinterpret_cast<T (*)[NB]>(&Pj[0][0]);
  tile_factor_inverse<T>(Wk, Linv + (k + 1) * NB * NB, kb, i0, info, colbuf, rowbuf);
}

template <typename T>
void dense_cholesky(T* A, int64_t n, T* L, T* Linv, int32_t* d_info, hipStream_t st) {
  if (n <= 0) return;
  const int64_t nblk = (n + NB - 1) / NB;
  launch_fill_i32(d_info, 1, 0, st);
  // only the lower blocks of L are ever read: the upper part is left as is
  chol_first_kernel<T><<<1, 256, 0, st>>>(A, n, L, Linv, d_info);
  const size_t shm = sizeof(T) * 4 * NB * (NB + 1);
  for (int64_t k = 0; k + 1 < nblk; ++k) {
    const int64_t m = nblk - k - 1;
    chol_step_kernel<T><<<static_cast<unsigned>(m * (m + 1) / 2), 256, shm, st>>>(A, n, k, L, Linv, d_info);
  }
}

// ---- solves: one workgroup, blocked with the stored diagonal inverses ----------
template <typename T>
__global__ void __launch_bounds__(1024) chol_solve_kernel(const T* __restrict__ L, const T* __restrict__ Linv,
                                                          int64_t n, T* __restrict__ b, int nrhs) {
  __shared__ T t[NB][4];
  __shared__ T red[16][NB][4];
  __shared__ T Ls[NB][NB + 1];
  const int lane = threadIdx.x % PDIPC_WAVE, wave = threadIdx.x / PDIPC_WAVE;
  const int64_t nblk = (n + NB - 1) / NB;
  // forward: L y = b
  for (int64_t bk = 0; bk < nblk; ++bk) {
    const int64_t k0 = bk * NB;
    const int kb = static_cast<int>(n - k0 < NB ? n - k0 : NB);
    for (int r = wave; r < NB; r += 16) {
      T s[4] = {T(0), T(0), T(0), T(0)};
      if (r < kb) {
        const T* Lr = L + (k0 + r) * n;
        for (int64_t c = lane; c < k0; c += PDIPC_WAVE) {
          T v = Lr[c];
          for (int q = 0; q < nrhs; ++q) s[q] += v * b[c * nrhs + q];
        }
      }
      for (int q = 0; q < nrhs; ++q) {
        T w = s[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, PDIPC_WAVE);
        s[q] = w;
      }
      if (lane == 0)
        for (int q = 0; q < 4; ++q) t[r][q] = (r < kb && q < nrhs) ? b[(k0 + r) * nrhs + q] - s[q] : T(0);
    }
    for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) Ls[idx / NB][idx % NB] = Linv[bk * NB * NB + idx];
    __syncthreads();
    if (threadIdx.x < NB * 4) {
      const int r = threadIdx.x / 4, q = threadIdx.x % 4;
      T acc = T(0);
      for (int c = 0; c <= r; ++c) acc += Ls[r][c] * t[c][q];
      if (r < kb && q < nrhs) b[(k0 + r) * nrhs + q] = acc;
    }
    __syncthreads();
  }
  // backward: L^T x = y
  for (int64_t bk = nblk - 1; bk >= 0; --bk) {
    const int64_t k0 = bk * NB;
    const int kb = static_cast<int>(n - k0 < NB ? n - k0 : NB);
    {
      T s[4] = {T(0), T(0), T(0), T(0)};
      if (lane < kb)
        for (int64_t i = k0 + kb + wave; i < n; i += 16) {
          T v = L[i * n + k0 + lane];
          for (int q = 0; q < nrhs; ++q) s[q] += v * b[i * nrhs + q];
        }
      for (int q = 0; q < 4; ++q) red[wave][lane][q] = s[q];
    }
    __syncthreads();
    if (threadIdx.x < NB * 4) {
      const int c = threadIdx.x / 4, q = threadIdx.x % 4;
      T acc = T(0);
      for (int w = 0; w < 16; ++w) acc += red[w][c][q];
      t[c][q] = (c < kb && q < nrhs) ? b[(k0 + c) * nrhs + q] - acc : T(0);
    }
    for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) Ls[idx / NB][idx % NB] = Linv[bk * NB * NB + idx];
    __syncthreads();
    if (threadIdx.x < NB * 4) {
      const int c = threadIdx.x / 4, q = threadIdx.x % 4;
      T acc = T(0);
      for (int r = c; r < NB; ++r) acc += Ls[r][c] * t[r][q];
      if (c < kb && q < nrhs) b[(k0 + c) * nrhs + q] = acc;
    }
    __syncthreads();
  }
}

template <typename T>
void dense_chol_solve(const T* L, const T* Linv, int64_t n, T* b, int32_t nrhs, hipStream_t st) {
  if (n <= 0) return;
  chol_solve_kernel<T><<<1, 1024, 0, st>>>(L, Linv, n, b, nrhs);
}

// ---- Y = L^-1 by block diagonals ------------------------------------------------
// Y_ii = Linv_i; for i - j = d >= 1: Y_ij = -Linv_i sum_{j <= p < i} L_ip Y_pj.
// Launch d computes every block of diagonal d (one workgroup each) from the
// diagonals already done; the strict upper blocks are zeroed by launch 0.
template <typename T>
__global__ void __launch_bounds__(256) inv_diag_kernel(const T* __restrict__ L, const T* __restrict__ Linv, int64_t n,
                                                       int64_t dd, T* __restrict__ Y) {
  extern __shared__ unsigned char smem_raw[];
  T (*Lt)[NB + 1] = reinterpret_cast<T (*)[NB + 1]>(smem_raw);
  T (*Yp)[NB + 1] = Lt + NB;
  T (*Acc)[NB + 1] = Yp + NB;
  const int64_t nblk = (n + NB - 1) / NB;
  const int64_t bj = blockIdx.x, bi = bj + dd;
  const int64_t i0 = bi * NB, j0 = bj * NB;
  const int ib = static_cast<int>(n - i0 < NB ? n - i0 : NB);
  const int jb = static_cast<int>(n - j0 < NB ? n - j0 : NB);
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  if (dd == 0) {
    // diagonal block and the zero block-row above it
    for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
      int r = idx / NB, c = idx % NB;
      if (r < ib && c < ib) Y[(i0 + r) * n + i0 + c] = Linv[bi * NB * NB + idx];
    }
    for (int64_t bq = bi + 1; bq < nblk; ++bq) {
      const int64_t q0 = bq * NB;
      const int qb = static_cast<int>(n - q0 < NB ? n - q0 : NB);
      for (int idx = threadIdx.x; idx < ib * qb; idx += blockDim.x) Y[(i0 + idx / qb) * n + q0 + idx % qb] = T(0);
    }
    return;
  }
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = T(0);
  for (int64_t bp = bj; bp < bi; ++bp) {
    const int64_t p0 = bp * NB;
    for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
      int r = idx / NB, c = idx % NB;
      Lt[r][c] = (r < ib && p0 + c < n) ? L[(i0 + r) * n + p0 + c] : T(0);
      Yp[r][c] = (p0 + r < n && c < jb) ? Y[(p0 + r) * n + j0 + c] : T(0);
    }
    __syncthreads();
    for (int p = 0; p < NB; ++p) {
      T x[4], y[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        x[q] = Lt[ty + 16 * q][p];
        y[q] = Yp[p][tx + 16 * q];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) Acc[ty + 16 * a][tx + 16 * b] = -acc[a][b];
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) Lt[idx / NB][idx % NB] = Linv[bi * NB * NB + idx];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = T(0);
  for (int p = 0; p < NB; ++p) {
    T x[4], y[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      x[q] = Lt[ty + 16 * q][p];
      y[q] = Acc[p][tx + 16 * q];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int r = ty + 16 * a, c = tx + 16 * b;
      if (r < ib && c < jb) Y[(i0 + r) * n + j0 + c] = acc[a][b];
    }
}

template <typename T>
void dense_chol_inverse(const T* L, const T* Linv, int64_t n, T* Ainv, T* work, hipStream_t st) {
  if (n <= 0) return;
  const unsigned nblk = grid_for(n, NB);
  const size_t shm = sizeof(T) * 3 * NB * (NB + 1);
  for (unsigned dd = 0; dd < nblk; ++dd)
    inv_diag_kernel<T><<<nblk - dd, 256, shm, st>>>(L, Linv, n, dd, work);
  dim3 grid(nblk, nblk);
  gemm_kernel<T, true, false><<<grid, 256, 0, st>>>(n, n, n, T(1), work, n, work, n, T(0), Ainv, n, 0);
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
template void dense_chol_solve<double>(const double*, const double*, int64_t, double*, int32_t, hipStream_t);
template void dense_chol_solve<float>(const float*, const float*, int64_t, float*, int32_t, hipStream_t);
template void dense_chol_inverse<double>(const double*, const double*, int64_t, double*, double*, hipStream_t);
template void dense_chol_inverse<float>(const float*, const float*, int64_t, float*, float*, hipStream_t);

}  // namespace pdipc
