// Kernels of the two comparison configurations of the paper's Table 1 that
// share the frame loop with the main global step:
//  - the preconditioned conjugate-gradient baseline of Eq. (5) (Section 3):
//    CG on (H + kappa B) dx = -g with the constant factor L L^T = H as the
//    preconditioner; products with H (per-tet, gathered per vertex) and with
//    the projected barrier Hessian (per-pair rank-5 factors on the contact
//    vertices), and the CG vector updates with their scalars kept on the
//    device;
//  - the Schur-complement-only global step of Section 3.1: the dense
//    Sigma-hat = Sigma + B_22 (3 n2 unknowns), assembled from Sigma_s (x) I3
//    and the barrier blocks of the contact vertices.
#include "common.h"
#include "kernels.h"

namespace pdipc {

namespace {
constexpr int VT = 256;
}

// Per tet: the share w G^T vec(D_s(v) B) of H v (m x 12 records, as the local
// step's gradient shares, so that the same per-vertex gather sums them).
__global__ void __launch_bounds__(VT) pd_matvec_kernel(LocalArgs la, const double* __restrict__ v,
                                                       double* __restrict__ tetg) {
  const int64_t m = la.m;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * VT + threadIdx.x;
  if (i >= m) return;
  int32_t vt[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) vt[k] = la.tets[k * m + i];
  double B[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) B[e] = la.B[e * m + i];
  // dF = D_s(v) B with D_s(v) = [v1 - v0, v2 - v0, v3 - v0]
  double Ds[3][3];
#pragma unroll
  for (int k = 1; k < 4; ++k)
#pragma unroll
    for (int r = 0; r < 3; ++r) Ds[r][k - 1] = v[3 * vt[k] + r] - v[3 * vt[0] + r];
  double dF[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) dF[r][c] = Ds[r][0] * B[c] + Ds[r][1] * B[3 + c] + Ds[r][2] * B[6 + c];
  // G^T: corner a > 0 takes row a - 1 of B, corner 0 minus their sum
  double g[4][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    g[1][c] = B[c];
    g[2][c] = B[3 + c];
    g[3][c] = B[6 + c];
    g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
  }
  const double w = la.w[i];
  double sh[12];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 3; ++r) sh[3 * a + r] = w * (dF[r][0] * g[a][0] + dF[r][1] * g[a][1] + dF[r][2] * g[a][2]);
  double2* out = reinterpret_cast<double2*>(tetg + 12 * i);
#pragma unroll
  for (int q = 0; q < 6; ++q) out[q] = make_double2(sh[2 * q], sh[2 * q + 1]);
}

// vc (nc x 3) = v at the contact vertices
__global__ void __launch_bounds__(VT) gather_c_kernel(int32_t nc, const int32_t* __restrict__ clist,
                                                      const double* __restrict__ v, double* __restrict__ vc) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * VT + threadIdx.x;
  if (t >= 3LL * nc) return;
  vc[t] = v[3LL * clist[t / 3] + t % 3];
}

// out at the contact vertices += vc (nc x 3); each vertex appears once in c
__global__ void __launch_bounds__(VT) scatter_add_c_kernel(int32_t nc, const int32_t* __restrict__ clist,
                                                           const double* __restrict__ vc, double* __restrict__ out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * VT + threadIdx.x;
  if (t >= 3LL * nc) return;
  out[3LL * clist[t / 3] + t % 3] += vc[t];
}

// x += (sc[num] / sc[den]) p ;  r -= (sc[num] / sc[den]) q
__global__ void __launch_bounds__(VT) cg_step_kernel(int64_t n3, const double* __restrict__ sc, int num, int den,
                                                     const double* __restrict__ p, const double* __restrict__ q,
                                                     double* __restrict__ x, double* __restrict__ r) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * VT + threadIdx.x;
  if (i >= n3) return;
  const double a = sc[num] / sc[den];
  x[i] += a * p[i];
  r[i] -= a * q[i];
}

// p = z + (sc[num] / sc[den]) p
__global__ void __launch_bounds__(VT) cg_dir_kernel(int64_t n3, const double* __restrict__ sc, int num, int den,
                                                    const double* __restrict__ z, double* __restrict__ p) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * VT + threadIdx.x;
  if (i >= n3) return;
  p[i] = z[i] + (sc[num] / sc[den]) * p[i];
}

// Out (3 n2 x 3 n2, row-major, vertex-major unknowns 3 a + r) = S (x) I3
__global__ void __launch_bounds__(VT) kron_i3_kernel(int32_t n2, const double* __restrict__ S,
                                                     double* __restrict__ out) {
  const int64_t N = 3LL * n2;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * VT + threadIdx.x;
  if (t >= N * N) return;
  const int64_t row = t / N, col = t % N;
  out[t] = (row % 3 == col % 3) ? S[(row / 3) * n2 + col / 3] : 0.0;
}

// out[3 x2(a) + r][3 x2(b) + s] += Bc[3 a + r][3 b + s] for the contact
// vertices a, b (x2 index c_x2 of each; distinct per vertex)
__global__ void __launch_bounds__(VT) scatter_block_kernel(int32_t nc, const int32_t* __restrict__ c_x2,
                                                           const double* __restrict__ Bc, int32_t n2,
                                                           double* __restrict__ out) {
  const int64_t Nc = 3LL * nc, N = 3LL * n2;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * VT + threadIdx.x;
  if (t >= Nc * Nc) return;
  const int64_t i = t / Nc, j = t % Nc;
  const int64_t gi = 3LL * c_x2[i / 3] + i % 3, gj = 3LL * c_x2[j / 3] + j % 3;
  out[gi * N + gj] += Bc[t];
}

void launch_pd_matvec(const LocalArgs& la, int32_t n, const int32_t* vt_ptr, const int32_t* vt_ent,
                      const uint8_t* fixed, const double* v, double* tetg, double* out, hipStream_t st) {
  pd_matvec_kernel<<<grid_for(la.m, VT), VT, 0, st>>>(la, v, tetg);
  launch_gather_vertex_grad(n, la.m, vt_ptr, vt_ent, tetg, fixed, out, st);
}

void launch_gather_c(int32_t nc, const int32_t* clist, const double* v, double* vc, hipStream_t st) {
  if (nc > 0) gather_c_kernel<<<grid_for(3LL * nc, VT), VT, 0, st>>>(nc, clist, v, vc);
}

void launch_scatter_add_c(int32_t nc, const int32_t* clist, const double* vc, double* out, hipStream_t st) {
  if (nc > 0) scatter_add_c_kernel<<<grid_for(3LL * nc, VT), VT, 0, st>>>(nc, clist, vc, out);
}

void launch_cg_step(int64_t n3, const double* sc, int num, int den, const double* p, const double* q, double* x,
                    double* r, hipStream_t st) {
  cg_step_kernel<<<grid_for(n3, VT), VT, 0, st>>>(n3, sc, num, den, p, q, x, r);
}

void launch_cg_dir(int64_t n3, const double* sc, int num, int den, const double* z, double* p, hipStream_t st) {
  cg_dir_kernel<<<grid_for(n3, VT), VT, 0, st>>>(n3, sc, num, den, z, p);
}

void launch_kron_i3(int32_t n2, const double* S, double* out, hipStream_t st) {
  const int64_t N = 3LL * n2;
  if (n2 > 0) kron_i3_kernel<<<grid_for(N * N, VT), VT, 0, st>>>(n2, S, out);
}

void launch_scatter_block(int32_t nc, const int32_t* c_x2, const double* Bc, int32_t n2, double* out,
                          hipStream_t st) {
  const int64_t Nc = 3LL * nc;
  if (nc > 0) scatter_block_kernel<<<grid_for(Nc * Nc, VT), VT, 0, st>>>(nc, c_x2, Bc, n2, out);
}

}  // namespace pdipc
