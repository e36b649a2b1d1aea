// Global step of Eq. (4) in the factored form of Eq. (7):
//   lower sweep   [L1 0; H21 L1^-T I] y = -g          (level-scheduled)
//   middle        Sigma_hat dx2 = y2  via Eq. (11)     (dense GEMV + reduced system)
//   upper sweep   [L1^T L1^-1 H12; 0 I] dx = [y1; dx2] (level-scheduled)
// The factor is a tree of dense supernodes (one per nested-dissection node).
// Every sum is a gather in a fixed order: the result is bitwise repeatable.
#include "common.h"
#include "kernels.h"

namespace pdipc {

namespace {
constexpr int FT = 256;
}

__global__ void pack_rhs_kernel(int32_t N, const int32_t* __restrict__ ext2vert, const double* __restrict__ g,
                                double* __restrict__ b) {
  int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  int32_t v = ext2vert[k];
  b[3 * k] = -g[3 * v];
  b[3 * k + 1] = -g[3 * v + 1];
  b[3 * k + 2] = -g[3 * v + 2];
}

void launch_pack_rhs(const FactorDev& f, const double* g, double* b, hipStream_t st) {
  int32_t N = f.n1 + f.n2;
  if (N > 0) pack_rhs_kernel<<<grid_for(N, 256), 256, 0, st>>>(N, f.ext2vert, g, b);
}

// Level-scheduled sweeps with W_J = L[R(J), cols(J)] Dinv_J in place of the
// panels, so that a level is one launch: one wavefront per row (lower sweep)
// or column (upper sweep) of that level's supernodes, lanes over the
// reduction dimension (coalesced):
//   lower  t_rho = b_rho - sum_e W[rho, e] t_e     (CSR rows of W), per level
//          y_J   = Dinv_J t_J                      (all blocks, one launch)
//   upper  z_J   = Dinv_J^T y_J                    (all blocks, one launch)
//          x_c   = z_c - sum_i W[R_i, c] x_{R_i}   (transposed W), per level
namespace {
constexpr int WPB = FT / PDIPC_WAVE;   // waves per block
}

__device__ __forceinline__ void wave_sum3(double& a0, double& a1, double& a2) {
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
}

__global__ void __launch_bounds__(FT) fwd_gather_kernel(FactorDev f, int32_t row0, int32_t nrows,
                                                        const double* __restrict__ b, double* t) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * WPB + threadIdx.x / PDIPC_WAVE;
  if (k >= nrows) return;
  const int64_t row = f.lvl_rows[row0 + k];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 4
  for (int64_t e = f.fwd_ptr[row] + lane; e < f.fwd_ptr[row + 1]; e += PDIPC_WAVE) {
    int32_t c = f.fwd_col[e];
    double v = f.fwd_val[e];
    a0 += v * t[3 * c];
    a1 += v * t[3 * c + 1];
    a2 += v * t[3 * c + 2];
  }
  wave_sum3(a0, a1, a2);
  if (lane == 0) {
    t[3 * row] = b[3 * row] - a0;
    t[3 * row + 1] = b[3 * row + 1] - a1;
    t[3 * row + 2] = b[3 * row + 2] - a2;
  }
}

// y_rho = sum_{c <= r} Dinv_J[r][c] t_{c0 + c}
__global__ void __launch_bounds__(FT) fwd_diag_kernel(FactorDev f, int32_t row0, int32_t nrows,
                                                      const double* __restrict__ t, double* __restrict__ y) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * WPB + threadIdx.x / PDIPC_WAVE;
  if (k >= nrows) return;
  const int64_t row = f.lvl_rows[row0 + k];
  const int32_t J = f.lvl_row_node[row0 + k];
  const int32_t c0 = f.node_c0[J], s = f.node_s[J];
  const int32_t r = static_cast<int32_t>(row - c0);
  const double* D = f.dinv + f.node_dinv_off[J] + static_cast<int64_t>(r) * s;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 4
  for (int32_t c = lane; c <= r; c += PDIPC_WAVE) {
    double d = D[c];
    a0 += d * t[3 * (c0 + c)];
    a1 += d * t[3 * (c0 + c) + 1];
    a2 += d * t[3 * (c0 + c) + 2];
  }
  wave_sum3(a0, a1, a2);
  if (lane == 0) {
    y[3 * row] = a0;
    y[3 * row + 1] = a1;
    y[3 * row + 2] = a2;
  }
}

// rows of x2: y2 = r2 - L21 y1 = r2 - sum over x1 nodes of W_J[x2 rows] t_J
__global__ void __launch_bounds__(FT) fwd_x2_kernel(FactorDev f, const double* __restrict__ b,
                                                    const double* __restrict__ t, double* __restrict__ y) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const int64_t q = static_cast<int64_t>(blockIdx.x) * WPB + threadIdx.x / PDIPC_WAVE;
  if (q >= f.n2) return;
  const int64_t row = f.n1 + q;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 4
  for (int64_t e = f.fwd_ptr[row] + lane; e < f.fwd_ptr[row + 1]; e += PDIPC_WAVE) {
    int32_t c = f.fwd_col[e];
    double v = f.fwd_val[e];
    a0 += v * t[3 * c];
    a1 += v * t[3 * c + 1];
    a2 += v * t[3 * c + 2];
  }
  wave_sum3(a0, a1, a2);
  if (lane == 0) {
    y[3 * row] = b[3 * row] - a0;
    y[3 * row + 1] = b[3 * row + 1] - a1;
    y[3 * row + 2] = b[3 * row + 2] - a2;
  }
}

void launch_forward_sweep(const FactorDev& f, const double* b, double* y, hipStream_t st, int level_begin,
                          int level_end) {
  // t lives after y in the same allocation (caller provides 2 * 3 * N)
  double* tbuf = y + 3 * static_cast<int64_t>(f.n1 + f.n2);
  const bool to_end = level_end < 0;
  if (to_end || level_end > f.nlevels) level_end = f.nlevels;
  for (int L = level_begin > 0 ? level_begin : 0; L < level_end; ++L) {
    const int32_t r0 = f.h_lvl_row_ptr[L], nr = f.h_lvl_row_ptr[L + 1] - r0;
    if (nr <= 0) continue;
    fwd_gather_kernel<<<grid_for(nr, WPB), FT, 0, st>>>(f, r0, nr, b, tbuf);
  }
  if (!to_end) return;
  // every diagonal block at once: y_J = Dinv_J t_J, then the x2 rows from t
  if (f.n1 > 0) fwd_diag_kernel<<<grid_for(f.n1, WPB), FT, 0, st>>>(f, 0, f.n1, tbuf, y);
  if (f.n2 > 0) fwd_x2_kernel<<<grid_for(f.n2, WPB), FT, 0, st>>>(f, b, tbuf, y);
}

// z = Sigma^-1 r, r and z are n2 x 3 (x2 part of the extended vectors).  One
// workgroup per two rows, its four waves over interleaved quarters of the
// columns: two row streams per lane and four waves per row pair keep enough
// loads in flight to stream the matrix, and each r entry serves both rows.
// The four wave partials are added in wave order (deterministic).
__global__ void __launch_bounds__(FT) sigma_gemv_kernel(int32_t n2, const double* __restrict__ S,
                                                        const double* __restrict__ r, double* __restrict__ z) {
  __shared__ double part[WPB][6];
  const int lane = threadIdx.x % PDIPC_WAVE, w = threadIdx.x / PDIPC_WAVE;
  const int64_t i0 = 2 * static_cast<int64_t>(blockIdx.x);
  const bool two = i0 + 1 < n2;
  const double* S0 = S + i0 * n2;
  const double* S1 = two ? S0 + n2 : S0;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0;
#pragma unroll 4
  for (int64_t j = w * PDIPC_WAVE + lane; j < n2; j += FT) {
    const double v0 = S0[j], v1 = S1[j];
    const double r0 = r[3 * j], r1 = r[3 * j + 1], r2 = r[3 * j + 2];
    a0 += v0 * r0;
    a1 += v0 * r1;
    a2 += v0 * r2;
    b0 += v1 * r0;
    b1 += v1 * r1;
    b2 += v1 * r2;
  }
  wave_sum3(a0, a1, a2);
  wave_sum3(b0, b1, b2);
  if (lane == 0) {
    part[w][0] = a0; part[w][1] = a1; part[w][2] = a2;
    part[w][3] = b0; part[w][4] = b1; part[w][5] = b2;
  }
  __syncthreads();
  if (threadIdx.x < 6 && (threadIdx.x < 3 || two)) {
    double acc = 0.0;
    for (int q = 0; q < WPB; ++q) acc += part[q][threadIdx.x];
    z[3 * i0 + threadIdx.x] = acc;
  }
}

void launch_sigma_gemv(const FactorDev& f, const double* r, double* z, hipStream_t st) {
  if (f.n2 > 0) sigma_gemv_kernel<<<static_cast<unsigned>((f.n2 + 1) / 2), FT, 0, st>>>(f.n2, f.sigma_inv, r, z);
}

// x_c = z_c - sum_i W_J^T[c][i] x[R_J[i]], z_c in sol already (z = Dinv^T y)
__global__ void __launch_bounds__(FT) bwd_gather_kernel(FactorDev f, int32_t row0, int32_t nrows, double* sol) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * WPB + threadIdx.x / PDIPC_WAVE;
  if (k >= nrows) return;
  const int64_t col = f.lvl_rows[row0 + k];
  const int32_t J = f.lvl_row_node[row0 + k];
  const int32_t c0 = f.node_c0[J], r = f.node_r[J];
  const int32_t c = static_cast<int32_t>(col - c0);
  const double* P = f.panelT + f.node_panel_off[J] + static_cast<int64_t>(c) * r;
  const int32_t* R = f.rows + f.node_rows_off[J];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 4
  for (int32_t i = lane; i < r; i += PDIPC_WAVE) {
    double v = P[i];
    int64_t q = R[i];
    a0 += v * sol[3 * q];
    a1 += v * sol[3 * q + 1];
    a2 += v * sol[3 * q + 2];
  }
  wave_sum3(a0, a1, a2);
  if (lane == 0) {
    sol[3 * col] -= a0;
    sol[3 * col + 1] -= a1;
    sol[3 * col + 2] -= a2;
  }
}

__global__ void __launch_bounds__(FT) bwd_diag_kernel(FactorDev f, int32_t row0, int32_t nrows,
                                                      const double* __restrict__ t, double* __restrict__ sol) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * WPB + threadIdx.x / PDIPC_WAVE;
  if (k >= nrows) return;
  const int64_t col = f.lvl_rows[row0 + k];
  const int32_t J = f.lvl_row_node[row0 + k];
  const int32_t c0 = f.node_c0[J], s = f.node_s[J];
  const int32_t c = static_cast<int32_t>(col - c0);
  const double* DT = f.dinvT + f.node_dinv_off[J] + static_cast<int64_t>(c) * s;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll 4
  for (int32_t rr = c + lane; rr < s; rr += PDIPC_WAVE) {
    double d = DT[rr];
    a0 += d * t[3 * (c0 + rr)];
    a1 += d * t[3 * (c0 + rr) + 1];
    a2 += d * t[3 * (c0 + rr) + 2];
  }
  wave_sum3(a0, a1, a2);
  if (lane == 0) {
    sol[3 * col] = a0;
    sol[3 * col + 1] = a1;
    sol[3 * col + 2] = a2;
  }
}

void launch_backward_sweep(const FactorDev& f, const double* y, double* sol, hipStream_t st) {
  // every diagonal block first: z_J = Dinv_J^T y_J into the x1 rows of sol
  if (f.n1 > 0) bwd_diag_kernel<<<grid_for(f.n1, WPB), FT, 0, st>>>(f, 0, f.n1, y, sol);
  for (int L = f.nlevels - 1; L >= 0; --L) {
    const int32_t r0 = f.h_lvl_row_ptr[L], nr = f.h_lvl_row_ptr[L + 1] - r0;
    if (nr <= 0) continue;
    bwd_gather_kernel<<<grid_for(nr, WPB), FT, 0, st>>>(f, r0, nr, sol);
  }
}

__global__ void unpack_kernel(int32_t N, const int32_t* __restrict__ ext2vert, const double* __restrict__ sol,
                              double* __restrict__ dx) {
  int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  int32_t v = ext2vert[k];
  dx[3 * v] = sol[3 * k];
  dx[3 * v + 1] = sol[3 * k + 1];
  dx[3 * v + 2] = sol[3 * k + 2];
}

void launch_unpack(const FactorDev& f, int32_t n, const double* sol, double* dx, hipStream_t st) {
  (void)n;
  int32_t N = f.n1 + f.n2;
  if (N > 0) unpack_kernel<<<grid_for(N, 256), 256, 0, st>>>(N, f.ext2vert, sol, dx);
}

void launch_unpack_range(const FactorDev& f, int32_t j0, int32_t j1, const double* sol, double* dx, hipStream_t st) {
  if (j1 > j0) unpack_kernel<<<grid_for(j1 - j0, 256), 256, 0, st>>>(j1 - j0, f.ext2vert + j0, sol + 3LL * j0, dx);
}

// W_J = P_J Dinv_J per supernode (P_J = L[R(J), cols(J)], r x s row-major;
// Dinv_J lower triangular, s x s row-major): one workgroup per node.
__global__ void __launch_bounds__(256) panel_dinv_kernel(const int32_t* __restrict__ node_s,
                                                         const int32_t* __restrict__ node_r,
                                                         const int64_t* __restrict__ poff,
                                                         const int64_t* __restrict__ doff,
                                                         const double* __restrict__ P,
                                                         const double* __restrict__ D, double* __restrict__ W) {
  const int32_t J = blockIdx.x;
  const int32_t s = node_s[J], r = node_r[J];
  const double* PJ = P + poff[J];
  const double* DJ = D + doff[J];
  double* WJ = W + poff[J];
  for (int64_t e = threadIdx.x; e < static_cast<int64_t>(r) * s; e += blockDim.x) {
    const int64_t i = e / s;
    const int32_t c = static_cast<int32_t>(e % s);
    double acc = 0.0;
    for (int32_t k = c; k < s; ++k) acc += PJ[i * s + k] * DJ[static_cast<int64_t>(k) * s + c];
    WJ[e] = acc;
  }
}

void launch_panel_times_dinv(int32_t nnodes, const int32_t* node_s, const int32_t* node_r, const int64_t* poff,
                             const int64_t* doff, const double* P, const double* D, double* W, hipStream_t st) {
  if (nnodes > 0) panel_dinv_kernel<<<static_cast<unsigned>(nnodes), 256, 0, st>>>(node_s, node_r, poff, doff, P, D, W);
}

// ---- reduced contact system helpers ---------------------------------------------
__global__ void gather_cc_kernel(int32_t n2, int32_t nc, const int32_t* __restrict__ c_x2,
                                 const double* __restrict__ S, double* __restrict__ Cs) {
  int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(nc) * nc) return;
  int64_t a = idx / nc, b = idx % nc;
  Cs[idx] = S[static_cast<int64_t>(c_x2[a]) * n2 + c_x2[b]];
}

void launch_gather_cc(const FactorDev& f, int32_t nc, const int32_t* c_x2, double* Cs, hipStream_t st) {
  if (nc > 0)
    gather_cc_kernel<<<grid_for(static_cast<int64_t>(nc) * nc, 256), 256, 0, st>>>(f.n2, nc, c_x2, f.sigma_inv, Cs);
}

// out[a] = sum_b Cinv[a][b] z[c_x2[b]]   (3 RHS), one wave per a
__global__ void __launch_bounds__(FT) cinv_zc_kernel(int32_t nc, const double* __restrict__ Cinv,
                                                     const int32_t* __restrict__ c_x2, const double* __restrict__ z,
                                                     double* __restrict__ out) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const int64_t a = static_cast<int64_t>(blockIdx.x) * (FT / PDIPC_WAVE) + threadIdx.x / PDIPC_WAVE;
  if (a >= nc) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t b = lane; b < nc; b += PDIPC_WAVE) {
    double c = Cinv[a * nc + b];
    int64_t q = c_x2[b];
    s0 += c * z[3 * q];
    s1 += c * z[3 * q + 1];
    s2 += c * z[3 * q + 2];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) {
    out[3 * a] = s0;
    out[3 * a + 1] = s1;
    out[3 * a + 2] = s2;
  }
}

void launch_cinv_times_zc(int32_t nc, const double* Cinv, const int32_t* c_x2, const double* z, double* out,
                          hipStream_t st) {
  if (nc > 0) cinv_zc_kernel<<<grid_for(nc, FT / PDIPC_WAVE), FT, 0, st>>>(nc, Cinv, c_x2, z, out);
}

// z_j -= sum_i S[c_i][j] v_i over n_out outputs, S row-major with leading
// dimension ld (for Sigma^-1, symmetric, the rows of c are its columns; for
// the stored rows x2 of H_s^-1 they are those columns by symmetry of H_s^-1).
// Rows are read coalesced along j.  Block: 64 consecutive j (one per lane) x
// 16 waves, wave g takes i = g, g + 16, ...; the 16 partial sums are added in
// wave order, so the result does not depend on scheduling.
constexpr int SC_WAVES = 16;
__global__ void __launch_bounds__(SC_WAVES * PDIPC_WAVE) rows_update_kernel(int64_t n_out, int64_t ld, int32_t nc,
                                                                         const int32_t* __restrict__ c_x2,
                                                                         const double* __restrict__ S,
                                                                         const double* __restrict__ v,
                                                                         double* __restrict__ z) {
  __shared__ double part[SC_WAVES][3][PDIPC_WAVE];
  const int lane = threadIdx.x % PDIPC_WAVE, g = threadIdx.x / PDIPC_WAVE;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * PDIPC_WAVE + lane;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (j < n_out) {
#pragma unroll 4
    for (int32_t i = g; i < nc; i += SC_WAVES) {
      const double c = S[static_cast<int64_t>(c_x2[i]) * ld + j];
      s0 += c * v[3 * i];
      s1 += c * v[3 * i + 1];
      s2 += c * v[3 * i + 2];
    }
  }
  part[g][0][lane] = s0;
  part[g][1][lane] = s1;
  part[g][2][lane] = s2;
  __syncthreads();
  if (g < 3 && j < n_out) {
    double acc = 0.0;
    for (int w = 0; w < SC_WAVES; ++w) acc += part[w][g][lane];
    z[3 * j + g] -= acc;
  }
}

void launch_sigma_cols_update(const FactorDev& f, int32_t nc, const int32_t* c_x2, const double* v, double* z,
                              hipStream_t st) {
  if (nc > 0 && f.n2 > 0)
    rows_update_kernel<<<grid_for(f.n2, PDIPC_WAVE), SC_WAVES * PDIPC_WAVE, 0, st>>>(f.n2, f.n2, nc, c_x2,
                                                                                     f.sigma_inv, v, z);
}

void launch_hinv_cols_update(const FactorDev& f, int32_t nc, const int32_t* c_x2, const double* v, double* sol,
                             hipStream_t st) {
  const int64_t N = static_cast<int64_t>(f.n1) + f.n2;
  launch_hinv_cols_update_range(f, nc, c_x2, v, sol, 0, N, st);
}

void launch_hinv_cols_update_range(const FactorDev& f, int32_t nc, const int32_t* c_x2, const double* v, double* sol,
                                   int64_t j0, int64_t j1, hipStream_t st) {
  const int64_t N = static_cast<int64_t>(f.n1) + f.n2;
  if (nc > 0 && f.n2 > 0 && j1 > j0)
    rows_update_kernel<<<grid_for(j1 - j0, PDIPC_WAVE), SC_WAVES * PDIPC_WAVE, 0, st>>>(
        j1 - j0, N, nc, c_x2, f.hinv_x2 + j0, v, sol + 3 * j0);
}

// sol's x2 rows = columns q0, q0 + 1, q0 + 2 of Sigma^-1 (one per right-hand side)
__global__ void hinv_fill_x2_kernel(int32_t n1, int32_t n2, int32_t q0, const double* __restrict__ Si,
                                    double* __restrict__ sol) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= 3LL * n2) return;
  const int64_t j = idx / 3;
  const int r = static_cast<int>(idx % 3);
  const int32_t q = q0 + r;
  sol[3 * (n1 + j) + r] = q < n2 ? Si[static_cast<int64_t>(q) * n2 + j] : 0.0;
}

// K[q][p] for the three columns of the batch: x1 part from the sweep, x2 part
// from Sigma^-1 (row q, by symmetry)
__global__ void hinv_store_rows_kernel(int32_t n1, int32_t n2, int32_t q0, const double* __restrict__ sol,
                                       const double* __restrict__ Si, double* __restrict__ K) {
  const int64_t N = static_cast<int64_t>(n1) + n2;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= 3 * N) return;
  const int r = static_cast<int>(idx / N);
  const int64_t p = idx % N;
  const int32_t q = q0 + r;
  if (q >= n2) return;
  K[static_cast<int64_t>(q) * N + p] = p < n1 ? sol[3 * p + r] : Si[static_cast<int64_t>(q) * n2 + (p - n1)];
}

void launch_build_hinv_rows(const FactorDev& f, double* y, double* sol, double* K, hipStream_t st) {
  const int64_t N = static_cast<int64_t>(f.n1) + f.n2;
  if (f.n2 <= 0) return;
  launch_fill_f64(y, 3 * N, 0.0, st);
  for (int32_t q0 = 0; q0 < f.n2; q0 += 3) {
    hinv_fill_x2_kernel<<<grid_for(3LL * f.n2, 256), 256, 0, st>>>(f.n1, f.n2, q0, f.sigma_inv, sol);
    launch_backward_sweep(f, y, sol, st);
    hinv_store_rows_kernel<<<grid_for(3 * N, 256), 256, 0, st>>>(f.n1, f.n2, q0, sol, f.sigma_inv, K);
  }
}

}  // namespace pdipc
