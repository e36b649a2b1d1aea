// Adjoint of a converged frame with respect to the per-tet actuation scalars.
//
// At the equilibrium x* the total-energy gradient g(x*, a) vanishes, so
// dL/da = -lambda^T dg/da with K lambda = dL/dx and K the true Hessian of the
// energy (PD term of Eq. 1 with the rotation's derivative, plus the barrier
// Hessian of Eq. 3 without the positive-definite projection).
//
// Rotation derivative: with M = F A = R S (S = R^T M symmetric), a change dM
// gives dR = R [w]_x, w = (tr(S) I - S)^-1 a(R^T dM), where
// a(X) = (X32 - X23, X13 - X31, X21 - X12).
#include "common.h"
#include "geom.h"
#include "kernels.h"

namespace pdipc {

namespace {
constexpr int AT = 256;

__device__ __forceinline__ void load_ds(const int32_t v[4], const double* __restrict__ x, M3<double>& Ds) {
#pragma unroll
  for (int k = 1; k < 4; ++k)
#pragma unroll
    for (int r = 0; r < 3; ++r) Ds(r, k - 1) = x[3 * v[k] + r] - x[3 * v[0] + r];
}

// dR for the rotation R of M = R S when M changes by dM
__device__ void rotation_derivative(const M3<double>& R, const M3<double>& M, const M3<double>& dM, M3<double>& dR) {
  M3<double> Rt;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Rt(r, c) = R(c, r);
  M3<double> S = mul(Rt, M);
  M3<double> X = mul(Rt, dM);
  double av[3] = {X(2, 1) - X(1, 2), X(0, 2) - X(2, 0), X(1, 0) - X(0, 1)};
  // symmetrise S (it is symmetric up to rounding)
  double s01 = 0.5 * (S(0, 1) + S(1, 0)), s02 = 0.5 * (S(0, 2) + S(2, 0)), s12 = 0.5 * (S(1, 2) + S(2, 1));
  double tr = S(0, 0) + S(1, 1) + S(2, 2);
  // B = tr I - S, solve B w = av (3x3, Cramer)
  double b00 = tr - S(0, 0), b11 = tr - S(1, 1), b22 = tr - S(2, 2);
  double b01 = -s01, b02 = -s02, b12 = -s12;
  double c00 = b11 * b22 - b12 * b12, c01 = b02 * b12 - b01 * b22, c02 = b01 * b12 - b02 * b11;
  double c11 = b00 * b22 - b02 * b02, c12 = b01 * b02 - b00 * b12, c22 = b00 * b11 - b01 * b01;
  double det = b00 * c00 + b01 * c01 + b02 * c02;
  double w[3] = {0.0, 0.0, 0.0};
  if (det != 0.0) {
    w[0] = (c00 * av[0] + c01 * av[1] + c02 * av[2]) / det;
    w[1] = (c01 * av[0] + c11 * av[1] + c12 * av[2]) / det;
    w[2] = (c02 * av[0] + c12 * av[1] + c22 * av[2]) / det;
  }
  M3<double> W;
  W(0, 0) = 0.0; W(0, 1) = -w[2]; W(0, 2) = w[1];
  W(1, 0) = w[2]; W(1, 1) = 0.0; W(1, 2) = -w[0];
  W(2, 0) = -w[1]; W(2, 1) = w[0]; W(2, 2) = 0.0;
  dR = mul(R, W);
}

__device__ __forceinline__ void load_sym(const double* __restrict__ A, int64_t m, int64_t i, M3<double>& Am) {
  double a6[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) a6[e] = A[e * m + i];
  Am(0, 0) = a6[0]; Am(1, 1) = a6[1]; Am(2, 2) = a6[2];
  Am(0, 1) = Am(1, 0) = a6[3];
  Am(1, 2) = Am(2, 1) = a6[4];
  Am(2, 0) = Am(0, 2) = a6[5];
}
}  // namespace

// Per tet: share of K_PD v = w G^T vec(dF - dR A), dF = D_s(v) B.
__global__ void __launch_bounds__(AT) pd_hessvec_kernel(LocalArgs la, const double* __restrict__ x,
                                                        const double* __restrict__ Rrot, const double* __restrict__ v,
                                                        double* __restrict__ tetg) {
  const int64_t m = la.m;
  int64_t i = static_cast<int64_t>(blockIdx.x) * AT + threadIdx.x;
  if (i >= m) return;
  int32_t vt[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) vt[k] = la.tets[k * m + i];
  M3<double> Bm, Ds, dDs, A, R;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    Bm.a[e] = la.B[e * m + i];
    R.a[e] = Rrot[e * m + i];
  }
  load_ds(vt, x, Ds);
  load_ds(vt, v, dDs);
  load_sym(la.A, m, i, A);
  M3<double> F = mul(Ds, Bm), dF = mul(dDs, Bm);
  M3<double> M = mul(F, A), dM = mul(dF, A), dR;
  rotation_derivative(R, M, dM, dR);
  M3<double> dRA = mul(dR, A);
  const double w = la.w[i];
  double res[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) res[e] = dF.a[e] - dRA.a[e];
  double g[4][3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    g[1][c] = Bm(0, c);
    g[2][c] = Bm(1, c);
    g[3][c] = Bm(2, c);
    g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
  }
  double sh[12];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 3; ++r)
      sh[3 * a + r] = w * (res[3 * r] * g[a][0] + res[3 * r + 1] * g[a][1] + res[3 * r + 2] * g[a][2]);
  double2* out = reinterpret_cast<double2*>(tetg + 12 * i);      // m x 12 records, as the local step
#pragma unroll
  for (int q = 0; q < 6; ++q) out[q] = make_double2(sh[2 * q], sh[2 * q + 1]);
}

// Per pair: true barrier Hessian times the pair's local 12-vector of v.
__global__ void __launch_bounds__(64) barrier_hessvec_kernel(const int32_t* __restrict__ v4all, int32_t npairs,
                                                             int32_t n_pt, const double* __restrict__ x,
                                                             const double* __restrict__ v, double dhat, double kappa,
                                                             int form, double* __restrict__ out) {
  int32_t k = blockIdx.x * 64 + threadIdx.x;
  if (k >= npairs) return;
  int32_t v4[4] = {v4all[4 * k], v4all[4 * k + 1], v4all[4 * k + 2], v4all[4 * k + 3]};
  double P[4][3];
  load_pair_rel(v4, x, P);
  Feature<double> f;
  pair_feature<double>(k < n_pt, P, f);
  double q[3] = {0, 0, 0}, Dk[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      q[r] += f.c[j] * P[j][r];
      Dk[0][r] += f.dcdb[0][j] * P[j][r];
      Dk[1][r] += f.dcdb[1][j] * P[j][r];
    }
  const double D = dot3(q, q);
  double eb, phi1, phi2;
  barrier_of_D<double>(D, dhat, kappa, form, eb, phi1, phi2);
  double vl[12];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 3; ++r) vl[3 * j + r] = v[3 * v4[j] + r];
  // C v (3-vector), grad D . v
  double Cv[3] = {0, 0, 0};
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 3; ++r) Cv[r] += f.c[j] * vl[3 * j + r];
  const double gDv = 2.0 * dot3(q, Cv);
  // f_bx v for each parameter
  double fbv[2] = {0, 0};
  for (int kk = 0; kk < f.nb; ++kk) {
    double dcv[3] = {0, 0, 0};
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 3; ++r) dcv[r] += f.dcdb[kk][j] * vl[3 * j + r];
    fbv[kk] = 2.0 * dot3(q, dcv) + 2.0 * dot3(Dk[kk], Cv);
  }
  double fbbi[2][2] = {{0, 0}, {0, 0}};
  {
    double b00 = 2.0 * dot3(Dk[0], Dk[0]), b01 = 2.0 * dot3(Dk[0], Dk[1]), b11 = 2.0 * dot3(Dk[1], Dk[1]);
    if (f.nb == 1) {
      fbbi[0][0] = 1.0 / b00;
    } else if (f.nb == 2) {
      double det = b00 * b11 - b01 * b01;
      fbbi[0][0] = b11 / det;
      fbbi[1][1] = b00 / det;
      fbbi[0][1] = fbbi[1][0] = -b01 / det;
    }
  }
  double y[2] = {fbbi[0][0] * fbv[0] + fbbi[0][1] * fbv[1], fbbi[1][0] * fbv[0] + fbbi[1][1] * fbv[1]};
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double gD = 2.0 * f.c[j] * q[r];
      double hD = 2.0 * f.c[j] * Cv[r];
      for (int kk = 0; kk < f.nb; ++kk) hD -= (2.0 * f.dcdb[kk][j] * q[r] + 2.0 * f.c[j] * Dk[kk][r]) * y[kk];
      out[static_cast<int64_t>(3 * j + r) * npairs + k] = phi2 * gD * gDv + phi1 * hD;
    }
}

// dL/da_i = w_i < D_s(lambda) B_i , dR A + R dA >,  dA = R0 diag(-1, 1/2, 1/2) R0^T, dM = F dA
__global__ void __launch_bounds__(AT) actuation_grad_kernel(LocalArgs la, const double* __restrict__ x,
                                                            const double* __restrict__ Rrot,
                                                            const double* __restrict__ R0,
                                                            const double* __restrict__ lam, double* __restrict__ out) {
  const int64_t m = la.m;
  int64_t i = static_cast<int64_t>(blockIdx.x) * AT + threadIdx.x;
  if (i >= m) return;
  int32_t vt[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) vt[k] = la.tets[k * m + i];
  M3<double> Bm, Ds, Dl, A, R, Q;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    Bm.a[e] = la.B[e * m + i];
    R.a[e] = Rrot[e * m + i];
    Q.a[e] = R0[9 * i + e];
  }
  load_ds(vt, x, Ds);
  load_ds(vt, lam, Dl);
  load_sym(la.A, m, i, A);
  M3<double> F = mul(Ds, Bm), Lm = mul(Dl, Bm);
  const double dd[3] = {-1.0, 0.5, 0.5};
  M3<double> dA;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) dA(r, c) = Q(r, 0) * dd[0] * Q(c, 0) + Q(r, 1) * dd[1] * Q(c, 1) + Q(r, 2) * dd[2] * Q(c, 2);
  M3<double> M = mul(F, A), dM = mul(F, dA), dR;
  rotation_derivative(R, M, dM, dR);
  M3<double> t1 = mul(dR, A), t2 = mul(R, dA);
  double s = 0.0;
#pragma unroll
  for (int e = 0; e < 9; ++e) s += Lm.a[e] * (t1.a[e] + t2.a[e]);
  out[i] = la.w[i] * s;
}

// deterministic dot product of two 3n vectors restricted to free vertices
__global__ void __launch_bounds__(256) masked_mul_kernel(int64_t n, const double* __restrict__ a,
                                                         const double* __restrict__ b, const uint8_t* __restrict__ fixed,
                                                         double* __restrict__ out) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= 3 * n) return;
  out[i] = fixed[i / 3] ? 0.0 : a[i] * b[i];
}

__global__ void __launch_bounds__(256) axpby_kernel(int64_t n3, double alpha, const double* __restrict__ x, double beta,
                                                    double* __restrict__ y) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i < n3) y[i] = alpha * x[i] + beta * y[i];
}

__global__ void __launch_bounds__(256) add_pair_vec_kernel(int32_t nsv, const int32_t* __restrict__ sv,
                                                           const int32_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ ent,
                                                           const double* __restrict__ pv, int32_t npairs,
                                                           const uint8_t* __restrict__ fixed, double* __restrict__ g) {
  int32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nsv) return;
  int32_t v = sv[i];
  if (fixed[v]) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 4
  for (int32_t t = ptr[v]; t < ptr[v + 1]; ++t) {
    int32_t k = ent[t] >> 2, a = ent[t] & 3;
    s0 += pv[static_cast<int64_t>(3 * a) * npairs + k];
    s1 += pv[static_cast<int64_t>(3 * a + 1) * npairs + k];
    s2 += pv[static_cast<int64_t>(3 * a + 2) * npairs + k];
  }
  g[3 * v] += s0;
  g[3 * v + 1] += s1;
  g[3 * v + 2] += s2;
}

void launch_hessvec(const LocalArgs& la, int32_t n, const int32_t* vt_ptr, const int32_t* vt_ent,
                    const uint8_t* fixed, const double* x, const double* Rrot, const double* v, double* tetg,
                    const PairList& pl, int32_t npairs, int32_t n_pt, const Incidence& inc, const ProxyDev& px,
                    double dhat, double kappa, int form, double* pairbuf, double* out, hipStream_t st) {
  pd_hessvec_kernel<<<grid_for(la.m, AT), AT, 0, st>>>(la, x, Rrot, v, tetg);
  launch_gather_vertex_grad(n, la.m, vt_ptr, vt_ent, tetg, fixed, out, st);
  if (npairs > 0) {
    barrier_hessvec_kernel<<<grid_for(npairs, 64), 64, 0, st>>>(pl.v4, npairs, n_pt, x, v, dhat, kappa, form,
                                                                  pairbuf);
    add_pair_vec_kernel<<<grid_for(px.nsv, 256), 256, 0, st>>>(px.nsv, px.sv, inc.ptr, inc.ent, pairbuf, npairs,
                                                              fixed, out);
  }
}

void launch_actuation_grad(const LocalArgs& la, const double* x, const double* Rrot, const double* R0,
                           const double* lam, double* out, hipStream_t st) {
  actuation_grad_kernel<<<grid_for(la.m, AT), AT, 0, st>>>(la, x, Rrot, R0, lam, out);
}

void launch_masked_mul(int64_t n, const double* a, const double* b, const uint8_t* fixed, double* out,
                       hipStream_t st) {
  masked_mul_kernel<<<grid_for(3 * n, 256), 256, 0, st>>>(n, a, b, fixed, out);
}

void launch_axpby(int64_t n3, double alpha, const double* x, double beta, double* y, hipStream_t st) {
  axpby_kernel<<<grid_for(n3, 256), 256, 0, st>>>(n3, alpha, x, beta, y);
}

}  // namespace pdipc
