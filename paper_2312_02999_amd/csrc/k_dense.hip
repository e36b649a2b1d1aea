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

// ---- diagonal block: unblocked Cholesky in LDS --------------------------------
template <typename T>
__global__ void __launch_bounds__(256) potrf_diag_kernel(T* __restrict__ A, int64_t n, int64_t k, int kb,
                                                         int32_t* __restrict__ info) {
  __shared__ T L[NB][NB + 1];
  for (int idx = threadIdx.x; idx < kb * kb; idx += blockDim.x) {
    int i = idx / kb, j = idx % kb;
    L[i][j] = A[(k + i) * n + k + j];
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    if (threadIdx.x == 0) {
      T d = L[j][j];
      if (!(d > T(0))) {
        if (*info == 0) *info = static_cast<int32_t>(k + j + 1);
        d = T(1);
      }
      L[j][j] = sqrt(d);
    }
    __syncthreads();
    T djj = L[j][j];
    for (int i = j + 1 + threadIdx.x; i < kb; i += blockDim.x) L[i][j] /= djj;
    __syncthreads();
    const int m = kb - j - 1;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      int i = j + 1 + idx / m, l = j + 1 + idx % m;
      if (l <= i) L[i][l] -= L[i][j] * L[l][j];
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < kb * kb; idx += blockDim.x) {
    int i = idx / kb, j = idx % kb;
    if (j <= i) A[(k + i) * n + k + j] = L[i][j];
  }
}

// ---- panel below the diagonal: X L_kk^T = A_ik, one row per thread --------------
template <typename T>
__global__ void __launch_bounds__(64) trsm_panel_kernel(T* __restrict__ A, int64_t n, int64_t k, int kb) {
  __shared__ T L[NB][NB + 1];
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
    int i = idx / NB, j = idx % NB;
    T v;
    if (i < kb && j < kb) v = j <= i ? A[(k + i) * n + k + j] : T(0);
    else v = (i == j) ? T(1) : T(0);
    L[i][j] = v;
  }
  __syncthreads();
  const int64_t row = k + kb + static_cast<int64_t>(blockIdx.x) * 64 + threadIdx.x;
  if (row >= n) return;
  T x[NB];
#pragma unroll
  for (int l = 0; l < NB; ++l) x[l] = l < kb ? A[row * n + k + l] : T(0);
#pragma unroll
  for (int l = 0; l < NB; ++l) {
    T s = x[l];
#pragma unroll
    for (int p = 0; p < l; ++p) s -= x[p] * L[l][p];
    x[l] = s / L[l][l];
  }
#pragma unroll
  for (int l = 0; l < NB; ++l)
    if (l < kb) A[row * n + k + l] = x[l];
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
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
    for (int idx = threadIdx.x; idx < 16 * 64; idx += 256) {
      int kk = idx / 64, r = idx % 64;
      int64_t gi = i0 + r, gk = k0 + kk;
      T va = T(0);
      if (gi < M && gk < K) va = TA ? A[gk * lda + gi] : A[gi * lda + gk];
      As[kk][r] = va;
      int64_t gj = j0 + r;
      T vb = T(0);
      if (gj < N && gk < K) vb = TB ? B[gj * ldb + gk] : B[gk * ldb + gj];
      Bs[kk][r] = vb;
    }
    __syncthreads();
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

template <typename T>
void dense_cholesky(T* A, int64_t n, int32_t* d_info, hipStream_t st) {
  launch_fill_i32(d_info, 1, 0, st);
  for (int64_t k = 0; k < n; k += NB) {
    int kb = static_cast<int>(n - k < NB ? n - k : NB);
    potrf_diag_kernel<T><<<1, 256, 0, st>>>(A, n, k, kb, d_info);
    int64_t rem = n - k - kb;
    if (rem > 0) {
      trsm_panel_kernel<T><<<grid_for(rem, 64), 64, 0, st>>>(A, n, k, kb);
      unsigned tiles = grid_for(rem, 64);
      dim3 grid(tiles, tiles);
      const T* P = A + (k + kb) * n + k;
      T* C = A + (k + kb) * n + k + kb;
      gemm_kernel<T, false, true><<<grid, 256, 0, st>>>(rem, rem, kb, T(-1), P, n, P, n, T(1), C, n, 1);
    }
  }
}

// ---- solves: one workgroup, blocked forward then backward substitution -------
template <typename T>
__global__ void __launch_bounds__(1024) chol_solve_kernel(const T* __restrict__ L, int64_t n, T* __restrict__ b,
                                                          int nrhs) {
  __shared__ T t[NB][4];
  __shared__ T red[16][NB][4];
  const int lane = threadIdx.x % PDIPC_WAVE, wave = threadIdx.x / PDIPC_WAVE;
  // forward: L y = b
  for (int64_t k0 = 0; k0 < n; k0 += NB) {
    const int kb = static_cast<int>(n - k0 < NB ? n - k0 : NB);
    for (int r = wave; r < kb; r += 16) {
      T s[4] = {T(0), T(0), T(0), T(0)};
      const T* Lr = L + (k0 + r) * n;
      for (int64_t c = lane; c < k0; c += PDIPC_WAVE) {
        T v = Lr[c];
        for (int q = 0; q < nrhs; ++q) s[q] += v * b[c * nrhs + q];
      }
      for (int q = 0; q < nrhs; ++q) {
        T w = s[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, PDIPC_WAVE);
        s[q] = w;
      }
      if (lane == 0)
        for (int q = 0; q < nrhs; ++q) t[r][q] = b[(k0 + r) * nrhs + q] - s[q];
    }
    __syncthreads();
    if (threadIdx.x < nrhs) {
      const int q = threadIdx.x;
      for (int r = 0; r < kb; ++r) {
        T s = t[r][q];
        const T* Lr = L + (k0 + r) * n + k0;
        for (int p = 0; p < r; ++p) s -= Lr[p] * t[p][q];
        t[r][q] = s / Lr[r];
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kb * nrhs; idx += blockDim.x) b[(k0 + idx / nrhs) * nrhs + idx % nrhs] = t[idx / nrhs][idx % nrhs];
    __syncthreads();
  }
  // backward: L^T x = y
  const int64_t nblk = (n + NB - 1) / NB;
  for (int64_t bi = nblk - 1; bi >= 0; --bi) {
    const int64_t k0 = bi * NB;
    const int kb = static_cast<int>(n - k0 < NB ? n - k0 : NB);
    // partial sums over rows i >= k0 + kb of L[i][k0 + c] x_i, split over waves
    for (int c = lane; c < NB; c += PDIPC_WAVE) {
      T s[4] = {T(0), T(0), T(0), T(0)};
      if (c < kb)
        for (int64_t i = k0 + kb + wave; i < n; i += 16) {
          T v = L[i * n + k0 + c];
          for (int q = 0; q < nrhs; ++q) s[q] += v * b[i * nrhs + q];
        }
      for (int q = 0; q < 4; ++q) red[wave][c][q] = s[q];
    }
    __syncthreads();
    if (threadIdx.x < kb)
      for (int q = 0; q < nrhs; ++q) {
        T s = T(0);
        for (int w = 0; w < 16; ++w) s += red[w][threadIdx.x][q];
        t[threadIdx.x][q] = b[(k0 + threadIdx.x) * nrhs + q] - s;
      }
    __syncthreads();
    if (threadIdx.x < nrhs) {
      const int q = threadIdx.x;
      for (int r = kb - 1; r >= 0; --r) {
        T s = t[r][q];
        for (int p = r + 1; p < kb; ++p) s -= L[(k0 + p) * n + k0 + r] * t[p][q];
        t[r][q] = s / L[(k0 + r) * n + k0 + r];
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kb * nrhs; idx += blockDim.x) b[(k0 + idx / nrhs) * nrhs + idx % nrhs] = t[idx / nrhs][idx % nrhs];
    __syncthreads();
  }
}

template <typename T>
void dense_chol_solve(const T* L, int64_t n, T* b, int32_t nrhs, hipStream_t st) {
  if (n <= 0) return;
  chol_solve_kernel<T><<<1, 1024, 0, st>>>(L, n, b, nrhs);
}

// ---- inverse of the lower factor, one block column per workgroup --------------
// Y = L^-1: for block column j, Y_jj = L_jj^-1 and for i > j
// Y_ij = -L_ii^-1 sum_{j <= p < i} L_ip Y_pj.
template <typename T>
__global__ void __launch_bounds__(256) lower_inverse_kernel(const T* __restrict__ L, int64_t n, T* __restrict__ Y) {
  __shared__ T Lt[NB][NB + 1];
  __shared__ T Acc[NB][NB + 1];
  __shared__ T Yp[NB][NB + 1];
  const int64_t j0 = static_cast<int64_t>(blockIdx.x) * NB;
  const int jb = static_cast<int>(n - j0 < NB ? n - j0 : NB);
  const int64_t nblk = (n + NB - 1) / NB;
  // zero the strictly upper part of this block column
  for (int64_t idx = threadIdx.x; idx < j0 * jb; idx += blockDim.x) Y[(idx / jb) * n + j0 + idx % jb] = T(0);
  for (int64_t bi = blockIdx.x; bi < nblk; ++bi) {
    const int64_t i0 = bi * NB;
    const int ib = static_cast<int>(n - i0 < NB ? n - i0 : NB);
    // Acc = (i == j ? I : 0) - sum_p L_ip Y_pj
    for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
      int r = idx / NB, c = idx % NB;
      Acc[r][c] = (bi == blockIdx.x && r == c) ? T(1) : T(0);
    }
    __syncthreads();
    for (int64_t bp = blockIdx.x; bp < bi; ++bp) {
      const int64_t p0 = bp * NB;
      for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
        int r = idx / NB, c = idx % NB;
        Lt[r][c] = (r < ib) ? L[(i0 + r) * n + p0 + c] : T(0);
        Yp[r][c] = (c < jb) ? Y[(p0 + r) * n + j0 + c] : T(0);
      }
      __syncthreads();
      for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
        int r = idx / NB, c = idx % NB;
        T s = T(0);
#pragma unroll 8
        for (int p = 0; p < NB; ++p) s += Lt[r][p] * Yp[p][c];
        Acc[r][c] -= s;
      }
      __syncthreads();
    }
    // solve L_ii X = Acc (column per thread)
    for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
      int r = idx / NB, c = idx % NB;
      Lt[r][c] = (r < ib && c < ib) ? (c <= r ? L[(i0 + r) * n + i0 + c] : T(0)) : (r == c ? T(1) : T(0));
    }
    __syncthreads();
    if (threadIdx.x < NB) {
      const int c = threadIdx.x;
      for (int r = 0; r < NB; ++r) {
        T s = Acc[r][c];
        for (int p = 0; p < r; ++p) s -= Lt[r][p] * Acc[p][c];
        Acc[r][c] = s / Lt[r][r];
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < ib * jb; idx += blockDim.x) {
      int r = idx / jb, c = idx % jb;
      Y[(i0 + r) * n + j0 + c] = Acc[r][c];
    }
    __syncthreads();
  }
}

template <typename T>
void dense_chol_inverse(const T* L, int64_t n, T* Ainv, T* work, hipStream_t st) {
  if (n <= 0) return;
  const unsigned nblk = grid_for(n, NB);
  lower_inverse_kernel<T><<<nblk, 256, 0, st>>>(L, n, work);
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

template void dense_cholesky<double>(double*, int64_t, int32_t*, hipStream_t);
template void dense_cholesky<float>(float*, int64_t, int32_t*, hipStream_t);
template void dense_chol_solve<double>(const double*, int64_t, double*, int32_t, hipStream_t);
template void dense_chol_solve<float>(const float*, int64_t, float*, int32_t, hipStream_t);
template void dense_chol_inverse<double>(const double*, int64_t, double*, double*, hipStream_t);
template void dense_chol_inverse<float>(const float*, int64_t, float*, float*, hipStream_t);

}  // namespace pdipc
