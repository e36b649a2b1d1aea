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

// t_row = b_row - sum_e val_e y_col(e), one wave per row
__device__ __forceinline__ void row_gather(const FactorDev& f, int64_t row, const double* __restrict__ b,
                                           const double* __restrict__ y, int lane, double out[3]) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int64_t e = f.fwd_ptr[row] + lane; e < f.fwd_ptr[row + 1]; e += PDIPC_WAVE) {
    int32_t c = f.fwd_col[e];
    double v = f.fwd_val[e];
    a0 += v * y[3 * c];
    a1 += v * y[3 * c + 1];
    a2 += v * y[3 * c + 2];
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  out[0] = b[3 * row] - a0;
  out[1] = b[3 * row + 1] - a1;
  out[2] = b[3 * row + 2] - a2;
}

__global__ void __launch_bounds__(FT) fwd_level_kernel(FactorDev f, const int32_t* __restrict__ nodes,
                                                       const double* __restrict__ b, double* __restrict__ y,
                                                       double* __restrict__ tbuf) {
  const int32_t J = nodes[blockIdx.x];
  const int32_t c0 = f.node_c0[J], s = f.node_s[J];
  const int lane = threadIdx.x % PDIPC_WAVE, wave = threadIdx.x / PDIPC_WAVE;
  const int nw = blockDim.x / PDIPC_WAVE;
  for (int r = wave; r < s; r += nw) {
    double t[3];
    row_gather(f, c0 + r, b, y, lane, t);
    if (lane == 0) {
      tbuf[3 * (c0 + r)] = t[0];
      tbuf[3 * (c0 + r) + 1] = t[1];
      tbuf[3 * (c0 + r) + 2] = t[2];
    }
  }
  __syncthreads();
  const double* DT = f.dinvT + f.node_dinv_off[J];   // DT[c * s + r] = Dinv[r][c]
  for (int r = threadIdx.x; r < s; r += blockDim.x) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int c = 0; c <= r; ++c) {
      double d = DT[static_cast<int64_t>(c) * s + r];
      a0 += d * tbuf[3 * (c0 + c)];
      a1 += d * tbuf[3 * (c0 + c) + 1];
      a2 += d * tbuf[3 * (c0 + c) + 2];
    }
    y[3 * (c0 + r)] = a0;
    y[3 * (c0 + r) + 1] = a1;
    y[3 * (c0 + r) + 2] = a2;
  }
}

// rows of x2: y2 = r2 - L21 y1
__global__ void __launch_bounds__(FT) fwd_x2_kernel(FactorDev f, const double* __restrict__ b, double* __restrict__ y) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const int64_t q = static_cast<int64_t>(blockIdx.x) * (FT / PDIPC_WAVE) + threadIdx.x / PDIPC_WAVE;
  if (q >= f.n2) return;
  const int64_t row = f.n1 + q;
  double t[3];
  row_gather(f, row, b, y, lane, t);
  if (lane == 0) {
    y[3 * row] = t[0];
    y[3 * row + 1] = t[1];
    y[3 * row + 2] = t[2];
  }
}

void launch_forward_sweep(const FactorDev& f, const double* b, double* y, hipStream_t st) {
  // tbuf lives after y in the same allocation (caller provides 2 * 3 * N)
  double* tbuf = y + 3 * static_cast<int64_t>(f.n1 + f.n2);
  for (int L = 0; L < f.nlevels; ++L) {
    int32_t cnt = f.h_level_ptr[L + 1] - f.h_level_ptr[L];
    if (cnt > 0)
      fwd_level_kernel<<<cnt, FT, 0, st>>>(f, f.level_nodes + f.h_level_ptr[L], b, y, tbuf);
  }
  if (f.n2 > 0) fwd_x2_kernel<<<grid_for(f.n2, FT / PDIPC_WAVE), FT, 0, st>>>(f, b, y);
}

// z = Sigma^-1 r, r and z are n2 x 3 (x2 part of the extended vectors)
__global__ void __launch_bounds__(FT) sigma_gemv_kernel(int32_t n2, const double* __restrict__ S,
                                                        const double* __restrict__ r, double* __restrict__ z) {
  const int lane = threadIdx.x % PDIPC_WAVE;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * (FT / PDIPC_WAVE) + threadIdx.x / PDIPC_WAVE;
  if (i >= n2) return;
  const double* Si = S + i * n2;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int64_t j = lane; j < n2; j += PDIPC_WAVE) {
    double v = Si[j];
    a0 += v * r[3 * j];
    a1 += v * r[3 * j + 1];
    a2 += v * r[3 * j + 2];
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  if (lane == 0) {
    z[3 * i] = a0;
    z[3 * i + 1] = a1;
    z[3 * i + 2] = a2;
  }
}

void launch_sigma_gemv(const FactorDev& f, const double* r, double* z, hipStream_t st) {
  if (f.n2 > 0) sigma_gemv_kernel<<<grid_for(f.n2, FT / PDIPC_WAVE), FT, 0, st>>>(f.n2, f.sigma_inv, r, z);
}

__global__ void __launch_bounds__(FT) bwd_level_kernel(FactorDev f, const int32_t* __restrict__ nodes,
                                                       const double* __restrict__ y, double* __restrict__ sol,
                                                       double* __restrict__ tbuf) {
  const int32_t J = nodes[blockIdx.x];
  const int32_t c0 = f.node_c0[J], s = f.node_s[J], r = f.node_r[J];
  const int32_t* R = f.rows + f.node_rows_off[J];
  const double* Pn = f.panel + f.node_panel_off[J];     // r x s row-major
  for (int c = threadIdx.x; c < s; c += blockDim.x) {
    double a0 = y[3 * (c0 + c)], a1 = y[3 * (c0 + c) + 1], a2 = y[3 * (c0 + c) + 2];
    for (int i = 0; i < r; ++i) {
      double v = Pn[static_cast<int64_t>(i) * s + c];
      int32_t k = R[i];
      a0 -= v * sol[3 * k];
      a1 -= v * sol[3 * k + 1];
      a2 -= v * sol[3 * k + 2];
    }
    tbuf[3 * (c0 + c)] = a0;
    tbuf[3 * (c0 + c) + 1] = a1;
    tbuf[3 * (c0 + c) + 2] = a2;
  }
  __syncthreads();
  const double* D = f.dinv + f.node_dinv_off[J];        // row-major Dinv
  for (int c = threadIdx.x; c < s; c += blockDim.x) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int rr = c; rr < s; ++rr) {
      double d = D[static_cast<int64_t>(rr) * s + c];
      a0 += d * tbuf[3 * (c0 + rr)];
      a1 += d * tbuf[3 * (c0 + rr) + 1];
      a2 += d * tbuf[3 * (c0 + rr) + 2];
    }
    sol[3 * (c0 + c)] = a0;
    sol[3 * (c0 + c) + 1] = a1;
    sol[3 * (c0 + c) + 2] = a2;
  }
}

void launch_backward_sweep(const FactorDev& f, const double* y, double* sol, hipStream_t st) {
  double* tbuf = sol + 3 * static_cast<int64_t>(f.n1 + f.n2);
  for (int L = f.nlevels - 1; L >= 0; --L) {
    int32_t cnt = f.h_level_ptr[L + 1] - f.h_level_ptr[L];
    if (cnt > 0)
      bwd_level_kernel<<<cnt, FT, 0, st>>>(f, f.level_nodes + f.h_level_ptr[L], y, sol, tbuf);
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
  launch_fill_f64(dx, 3 * static_cast<int64_t>(n), 0.0, st);
  int32_t N = f.n1 + f.n2;
  if (N > 0) unpack_kernel<<<grid_for(N, 256), 256, 0, st>>>(N, f.ext2vert, sol, dx);
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

// z[j] -= sum_i S[c_x2[i]][j] v[i]   (S symmetric: the rows of c are its columns)
__global__ void __launch_bounds__(FT) sigma_cols_kernel(int32_t n2, int32_t nc, const int32_t* __restrict__ c_x2,
                                                        const double* __restrict__ S, const double* __restrict__ v,
                                                        double* __restrict__ z) {
  int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n2) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int32_t i = 0; i < nc; ++i) {
    double c = S[static_cast<int64_t>(c_x2[i]) * n2 + j];
    s0 += c * v[3 * i];
    s1 += c * v[3 * i + 1];
    s2 += c * v[3 * i + 2];
  }
  z[3 * j] -= s0;
  z[3 * j + 1] -= s1;
  z[3 * j + 2] -= s2;
}

void launch_sigma_cols_update(const FactorDev& f, int32_t nc, const int32_t* c_x2, const double* v, double* z,
                              hipStream_t st) {
  if (nc > 0 && f.n2 > 0)
    sigma_cols_kernel<<<grid_for(f.n2, FT), FT, 0, st>>>(f.n2, nc, c_x2, f.sigma_inv, v, z);
}

}  // namespace pdipc
