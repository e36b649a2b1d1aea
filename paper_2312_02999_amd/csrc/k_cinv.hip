// Update of C^-1 = ((Sigma^-1)_cc)^-1 when a few vertices leave or enter the
// contact set c between iterations (Section 3.2: the reduced system of
// Eq. 11 needs C^-1; a rebuild factors C_s and inverts it with the dense
// kernels instead).  Row-major FP64.
#include "common.h"
#include "kernels.h"

namespace pdipc {

// ---- C^-1 after a small change of the contact set ---------------------------
// C = (Sigma^-1)_cc changes by a few rows/columns when a few vertices enter or
// leave c.  With the previous inverse Ci (old order), kept vertices K,
// removed R and added A:
//   leaving R:  (C_KK)^-1 = Ci_KK - Ci_KR (Ci_RR)^-1 Ci_RK   (Ci_RR is SPD)
//   entering A: with B = Sigma^-1[K, A], D = Sigma^-1[A, A], W = (C_KK)^-1 B
//               and the Schur complement S = D - B^T W (SPD),
//               C^-1 = [[(C_KK)^-1 + W S^-1 W^T, -W S^-1], [-S^-1 W^T, S^-1]]
// written in the new order (c sorted by vertex id).  At most 32 vertices may
// leave and 32 enter; the two small inverses use the sweep operator below.

// Sorts the (at most 32) unordered entries of ids into out by value, in LDS.
__device__ __forceinline__ void sort_small_ids(const int32_t* __restrict__ ids, int m, int32_t* out) {
  __shared__ int32_t tmp[32];
  if (threadIdx.x < m) tmp[threadIdx.x] = ids[threadIdx.x];
  __syncthreads();
  if (threadIdx.x < m) {
    const int32_t v = tmp[threadIdx.x];
    int rank = 0;
    for (int q = 0; q < m; ++q) rank += tmp[q] < v ? 1 : 0;
    out[rank] = v;
  }
  __syncthreads();
}

// Kept vertices in the order of the new c (rank = new index - entering
// vertices before it), leaving / entering vertices by id, and kind[] of every
// new index.  Also zeroes *info.
__global__ void __launch_bounds__(256) cinv_lists_kernel(int32_t n, int32_t r, int32_t a,
                                                         const int32_t* __restrict__ cflag,
                                                         const int32_t* __restrict__ cidx,
                                                         const int32_t* __restrict__ pflag,
                                                         const int32_t* __restrict__ pidx,
                                                         const int32_t* __restrict__ vert2x2,
                                                         const int32_t* __restrict__ rem_ids,
                                                         const int32_t* __restrict__ add_ids, CinvLists L,
                                                         int32_t* __restrict__ info) {
  __shared__ int32_t add_s[32];
  __shared__ int32_t rem_s[32];
  sort_small_ids(add_ids, a, add_s);
  if (blockIdx.x == 0) {
    sort_small_ids(rem_ids, r, rem_s);
    if (threadIdx.x < r) L.rem_old[threadIdx.x] = pidx[rem_s[threadIdx.x]];
    if (threadIdx.x < a) {
      const int32_t v = add_s[threadIdx.x];
      L.add_x2[threadIdx.x] = vert2x2[v];
      L.kind[cidx[v]] = -1 - static_cast<int32_t>(threadIdx.x);
    }
    if (threadIdx.x == 0) *info = 0;
  }
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || !cflag[v] || !pflag[v]) return;
  int32_t before = 0;
  for (int q = 0; q < a; ++q) before += add_s[q] < v ? 1 : 0;
  const int32_t kr = cidx[v] - before;
  L.kept_old[kr] = pidx[v];
  L.kept_x2[kr] = vert2x2[v];
  L.kind[cidx[v]] = kr;
}

// In-place inverse of the SPD m x m matrix in A (m <= 32) by the sweep
// operator over every pivot (Gauss-Jordan without pivoting, stable for SPD),
// which leaves -A^-1; the sign is folded into the final copy by the caller.
// A non-positive pivot is replaced by 1 and sets *info.
__device__ __forceinline__ void sweep_all(double (*A)[33], int m, int32_t* info) {
  for (int k = 0; k < m; ++k) {
    const double d = A[k][k];
    const bool ok = d > 0.0;
    const double id = ok ? 1.0 / d : 1.0;
    double nv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int e = threadIdx.x + 256 * s;
      const int i = e / 32, j = e % 32;
      double v = 0.0;
      if (i < m && j < m) {
        if (i == k && j == k) v = -id;
        else if (i == k) v = A[k][j] * id;
        else if (j == k) v = A[i][k] * id;
        else v = A[i][j] - A[i][k] * A[k][j] * id;
      }
      nv[s] = v;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int e = threadIdx.x + 256 * s;
      const int i = e / 32, j = e % 32;
      if (i < m && j < m) A[i][j] = nv[s];
    }
    __syncthreads();
    if (!ok && threadIdx.x == 0) *info = 1;
  }
}

// T = Ci_KR (Ci_RR)^-1 (nk x r); every workgroup inverts Ci_RR itself
__global__ void __launch_bounds__(256) cinv_t_kernel(const double* __restrict__ Ci, int32_t nold, CinvLists L,
                                                     int32_t nk, int32_t r, double* __restrict__ T,
                                                     double* __restrict__ G, int32_t* info) {
  __shared__ double Ri[32][33];
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
    const int i = e / r, j = e % r;
    Ri[i][j] = Ci[static_cast<int64_t>(L.rem_old[i]) * nold + L.rem_old[j]];
  }
  __syncthreads();
  sweep_all(Ri, r, info);                                           // Ri = -(Ci_RR)^-1
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(nk) * r) return;
  const int64_t i = idx / r;
  const int q = static_cast<int>(idx % r);
  const double* row = Ci + static_cast<int64_t>(L.kept_old[i]) * nold;
  double acc = 0.0;
  for (int p = 0; p < r; ++p) acc -= row[L.rem_old[p]] * Ri[p][q];
  T[idx] = acc;
  G[static_cast<int64_t>(q) * nk + i] = row[L.rem_old[q]];       // Ci_KR, transposed for the next kernel
}

// CK = Ci_KK - T Ci_RK (nk x nk); Ci_RK[p][j] = Ci[kept j][removed p] comes
// from G, row p of which neighbouring threads read contiguously
__global__ void cinv_keep_kernel(const double* __restrict__ Ci, int32_t nold, CinvLists L, int32_t nk, int32_t r,
                                 const double* __restrict__ T, const double* __restrict__ G,
                                 double* __restrict__ CK) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(nk) * nk) return;
  const int64_t i = idx / nk, j = idx % nk;
  double v = Ci[static_cast<int64_t>(L.kept_old[i]) * nold + L.kept_old[j]];
  for (int p = 0; p < r; ++p) v -= T[i * r + p] * G[static_cast<int64_t>(p) * nk + j];
  CK[idx] = v;
}

// W = CK B with B = Sigma^-1[K, A] (nk x a, a <= 32); one wave per row of
// CK, all a columns in one pass over the row
__global__ void __launch_bounds__(256) cinv_w_kernel(const double* __restrict__ CK, int32_t nk, CinvLists L,
                                                     int32_t a, const double* __restrict__ Si, int32_t n2,
                                                     double* __restrict__ W) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / PDIPC_WAVE;
  const int lane = threadIdx.x % PDIPC_WAVE;
  if (i >= nk) return;
  double acc[32];
  const double* sq[32];                                                  // Sigma^-1 is symmetric
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    acc[q] = 0.0;
    sq[q] = Si + static_cast<int64_t>(L.add_x2[q < a ? q : 0]) * n2;
  }
  for (int64_t j = lane; j < nk; j += PDIPC_WAVE) {
    const double c = CK[i * nk + j];
    const int32_t kx = L.kept_x2[j];
#pragma unroll
    for (int q = 0; q < 32; ++q)
      if (q < a) acc[q] += c * sq[q][kx];
  }
#pragma unroll
  for (int q = 0; q < 32; ++q)
    if (q < a) {
      const double s = wave_sum(acc[q]);
      if (lane == 0) W[i * a + q] = s;
    }
}

// Sm = D - B^T W (a x a); one wave per entry
__global__ void __launch_bounds__(256) cinv_schur_kernel(const double* __restrict__ Si, int32_t n2, CinvLists L,
                                                         int32_t nk, int32_t a, const double* __restrict__ W,
                                                         double* __restrict__ Sm) {
  const int e = blockIdx.x * 4 + threadIdx.x / PDIPC_WAVE;
  const int lane = threadIdx.x % PDIPC_WAVE;
  if (e >= a * a) return;
  const int p = e / a, q = e % a;
  const double* sp = Si + static_cast<int64_t>(L.add_x2[p]) * n2;
  double acc = 0.0;
  for (int64_t i = lane; i < nk; i += PDIPC_WAVE) acc += sp[L.kept_x2[i]] * W[i * a + q];
  acc = wave_sum(acc);
  if (lane == 0) Sm[e] = sp[L.add_x2[q]] - acc;
}

// V = W Sm^-1 (nk x a), Sm symmetrised; every workgroup inverts Sm itself and
// the first one stores the inverse to Sinv (32 x 32)
__global__ void __launch_bounds__(256) cinv_v_kernel(int32_t nk, int32_t a, const double* __restrict__ W,
                                                     const double* __restrict__ Sm, double* __restrict__ Sinv,
                                                     double* __restrict__ V, int32_t* info) {
  __shared__ double Si_[32][33];
  for (int e = threadIdx.x; e < a * a; e += blockDim.x) {
    const int i = e / a, j = e % a;
    Si_[i][j] = 0.5 * (Sm[i * a + j] + Sm[j * a + i]);
  }
  __syncthreads();
  sweep_all(Si_, a, info);                                          // Si_ = -Sm^-1
  if (blockIdx.x == 0)
    for (int e = threadIdx.x; e < a * a; e += blockDim.x) Sinv[(e / a) * 32 + e % a] = -Si_[e / a][e % a];
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(nk) * a) return;
  const int64_t i = idx / a;
  const int q = static_cast<int>(idx % a);
  double acc = 0.0;
  for (int p = 0; p < a; ++p) acc -= W[i * a + p] * Si_[p][q];
  V[idx] = acc;
}

// C^-1 in the new order from CK, W, V, Sinv
__global__ void __launch_bounds__(256) cinv_assemble_kernel(int32_t nc, int32_t nk, int32_t a, CinvLists L,
                                                            const double* __restrict__ CK,
                                                            const double* __restrict__ W,
                                                            const double* __restrict__ V,
                                                            const double* __restrict__ Sinv,
                                                            double* __restrict__ out) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(nc) * nc) return;
  const int32_t ki = L.kind[idx / nc], kj = L.kind[idx % nc];
  double v;
  if (ki >= 0 && kj >= 0) {
    v = CK[static_cast<int64_t>(ki) * nk + kj];
    for (int q = 0; q < a; ++q) v += V[static_cast<int64_t>(ki) * a + q] * W[static_cast<int64_t>(kj) * a + q];
  } else if (ki >= 0) {
    v = -V[static_cast<int64_t>(ki) * a + (-1 - kj)];
  } else if (kj >= 0) {
    v = -V[static_cast<int64_t>(kj) * a + (-1 - ki)];
  } else {
    v = Sinv[(-1 - ki) * 32 + (-1 - kj)];
  }
  out[idx] = v;
}

void launch_cinv_update(const CinvUpdateArgs& u, hipStream_t st) {
  const int32_t nk = u.nold - u.r;
  cinv_lists_kernel<<<grid_for(u.n, 256), 256, 0, st>>>(u.n, u.r, u.a, u.cflag, u.cidx, u.pflag, u.pidx, u.vert2x2,
                                                         u.rem_ids, u.add_ids, u.L, u.info);
  if (u.r > 0)
    cinv_t_kernel<<<grid_for(static_cast<int64_t>(nk) * u.r, 256), 256, 0, st>>>(u.Ci, u.nold, u.L, nk, u.r, u.T,
                                                                                 u.G, u.info);
  cinv_keep_kernel<<<grid_for(static_cast<int64_t>(nk) * nk, 256), 256, 0, st>>>(u.Ci, u.nold, u.L, nk, u.r, u.T,
                                                                                 u.G, u.CK);
  if (u.a > 0) {
    cinv_w_kernel<<<static_cast<unsigned>((nk + 3) / 4), 256, 0, st>>>(u.CK, nk, u.L, u.a, u.Si, u.n2, u.W);
    cinv_schur_kernel<<<static_cast<unsigned>((u.a * u.a + 3) / 4), 256, 0, st>>>(u.Si, u.n2, u.L, nk, u.a, u.W,
                                                                                 u.Sm);
    cinv_v_kernel<<<grid_for(static_cast<int64_t>(nk) * u.a, 256), 256, 0, st>>>(nk, u.a, u.W, u.Sm, u.Sinv, u.V,
                                                                                 u.info);
  }
  cinv_assemble_kernel<<<grid_for(static_cast<int64_t>(u.nc) * u.nc, 256), 256, 0, st>>>(u.nc, nk, u.a, u.L, u.CK,
                                                                                         u.W, u.V, u.Sinv, u.out);
}

}  // namespace pdipc
