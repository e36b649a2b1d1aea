// Local step of projective dynamics (Eq. 1): per tet, the rotation R_i that
// minimises ||F_i - R A_i||_F, the projection p_i = vec(R_i A_i), the element
// energy (w_i/2)||F_i - R_i A_i||^2 and the element's share of
// sum_i w_i G_i^T (G_i x - p_i).  One thread per tet; per-tet data are SoA
// streams (coalesced), vertex positions are gathered as xyz triples.
#include <hip/hip_ext.h>

#include "common.h"
#include "kernels.h"

namespace pdipc {

// Nearest rotation to M (row-major 3x3) in SO(3).  Symmetric Jacobi on M^T M
// gives V and the squared singular values; u_k = M v_k / sigma_k for the two
// largest, and R = [u1, u2, u1 x u2] [v1, v2, v1 x v2]^T, which equals
// U diag(1, 1, det(U V^T)) V^T of the SVD M = U S V^T.
template <typename T>
__device__ void nearest_rotation(const M3<T>& M, M3<T>& R) {
  T S[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) S[i][j] = M(0, i) * M(0, j) + M(1, i) * M(1, j) + M(2, i) * M(2, j);
  T V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  const T tiny = sizeof(T) == 8 ? T(1e-30) : T(1e-20);
  for (int sweep = 0; sweep < 12; ++sweep) {
    T off = S[0][1] * S[0][1] + S[0][2] * S[0][2] + S[1][2] * S[1][2];
    T dia = S[0][0] * S[0][0] + S[1][1] * S[1][1] + S[2][2] * S[2][2];
    if (off <= tiny * dia || off == T(0)) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0;
      const int q = pq == 0 ? 1 : 2;
      T apq = S[p][q];
      if (apq == T(0)) continue;
      T theta = (S[q][q] - S[p][p]) / (T(2) * apq);
      T t = (theta >= T(0) ? T(1) : T(-1)) / (fabs(theta) + sqrt(theta * theta + T(1)));
      T c = T(1) / sqrt(t * t + T(1));
      T s = t * c;
#pragma unroll
      for (int k = 0; k < 3; ++k) {          // S <- S J (columns p, q)
        T skp = S[k][p], skq = S[k][q];
        S[k][p] = c * skp - s * skq;
        S[k][q] = s * skp + c * skq;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {          // S <- J^T S (rows p, q)
        T spk = S[p][k], sqk = S[q][k];
        S[p][k] = c * spk - s * sqk;
        S[q][k] = s * spk + c * sqk;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {          // V <- V J
        T vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - s * vkq;
        V[k][q] = s * vkp + c * vkq;
      }
    }
  }
  // order eigenvalues descending
  int o0 = 0, o1 = 1, o2 = 2;
  T l0 = S[0][0], l1 = S[1][1], l2 = S[2][2];
  if (l1 > l0) { T t = l0; l0 = l1; l1 = t; int ti = o0; o0 = o1; o1 = ti; }
  if (l2 > l1) { T t = l1; l1 = l2; l2 = t; int ti = o1; o1 = o2; o2 = ti; }
  if (l1 > l0) { T t = l0; l0 = l1; l1 = t; int ti = o0; o0 = o1; o1 = ti; }
  T v1[3] = {V[0][o0], V[1][o0], V[2][o0]};
  T v2[3] = {V[0][o1], V[1][o1], V[2][o1]};
  T v3[3];
  cross3(v1, v2, v3);
  T u1[3], u2[3], u3[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    u1[r] = M(r, 0) * v1[0] + M(r, 1) * v1[1] + M(r, 2) * v1[2];
    u2[r] = M(r, 0) * v2[0] + M(r, 1) * v2[1] + M(r, 2) * v2[2];
  }
  T n1 = sqrt(dot3(u1, u1));
  if (n1 > T(0)) {
#pragma unroll
    for (int r = 0; r < 3; ++r) u1[r] /= n1;
  } else {
    u1[0] = T(1); u1[1] = T(0); u1[2] = T(0);
  }
  T pr = dot3(u1, u2);
#pragma unroll
  for (int r = 0; r < 3; ++r) u2[r] -= pr * u1[r];
  T n2 = sqrt(dot3(u2, u2));
  if (n2 > T(0)) {
#pragma unroll
    for (int r = 0; r < 3; ++r) u2[r] /= n2;
  } else {                                   // any unit vector orthogonal to u1
    T e[3] = {T(0), T(0), T(0)};
    e[fabs(u1[0]) < T(0.6) ? 0 : 1] = T(1);
    T pe = dot3(u1, e);
#pragma unroll
    for (int r = 0; r < 3; ++r) u2[r] = e[r] - pe * u1[r];
    T ne = sqrt(dot3(u2, u2));
#pragma unroll
    for (int r = 0; r < 3; ++r) u2[r] /= ne;
  }
  cross3(u1, u2, u3);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) R(r, c) = u1[r] * v1[c] + u2[r] * v2[c] + u3[r] * v3[c];
}

// One FP64 Newton step on SO(3) toward the rotation maximising tr(R^T M):
// with S0 = R0^T M, the optimum R0 Q has Q^T S0 symmetric; to first order
// Q = exp([w]_x) with (tr(Sym) I - Sym) w = a(S0), Sym = sym(S0),
// a(X) = (X32 - X23, X13 - X31, X21 - X12).  Convergence is quadratic, so an
// FP32 rotation becomes FP64-accurate in one step.
__device__ void refine_rotation(const M3<double>& M, M3<double>& R) {
  M3<double> Rt;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Rt(r, c) = R(c, r);
  M3<double> S = mul(Rt, M);
  double av[3] = {S(2, 1) - S(1, 2), S(0, 2) - S(2, 0), S(1, 0) - S(0, 1)};
  double s01 = 0.5 * (S(0, 1) + S(1, 0)), s02 = 0.5 * (S(0, 2) + S(2, 0)), s12 = 0.5 * (S(1, 2) + S(2, 1));
  double tr = S(0, 0) + S(1, 1) + S(2, 2);
  double b00 = tr - S(0, 0), b11 = tr - S(1, 1), b22 = tr - S(2, 2);
  double b01 = -s01, b02 = -s02, b12 = -s12;
  double c00 = b11 * b22 - b12 * b12, c01 = b02 * b12 - b01 * b22, c02 = b01 * b12 - b02 * b11;
  double c11 = b00 * b22 - b02 * b02, c12 = b01 * b02 - b00 * b12, c22 = b00 * b11 - b01 * b01;
  double det = b00 * c00 + b01 * c01 + b02 * c02;
  if (!(fabs(det) > 0.0)) return;
  double w[3] = {(c00 * av[0] + c01 * av[1] + c02 * av[2]) / det, (c01 * av[0] + c11 * av[1] + c12 * av[2]) / det,
                 (c02 * av[0] + c12 * av[1] + c22 * av[2]) / det};
  // Q = exp([w]_x) by Rodrigues' formula (exactly orthogonal in exact arithmetic)
  double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  double th = sqrt(th2);
  double A1, B1;
  if (th < 1e-4) {
    A1 = 1.0 - th2 / 6.0;
    B1 = 0.5 - th2 / 24.0;
  } else {
    A1 = sin(th) / th;
    B1 = (1.0 - cos(th)) / th2;
  }
  M3<double> K, K2, Q;
  K(0, 0) = 0.0; K(0, 1) = -w[2]; K(0, 2) = w[1];
  K(1, 0) = w[2]; K(1, 1) = 0.0; K(1, 2) = -w[0];
  K(2, 0) = -w[1]; K(2, 1) = w[0]; K(2, 2) = 0.0;
  K2 = mul(K, K);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Q(r, c) = (r == c ? 1.0 : 0.0) + A1 * K(r, c) + B1 * K2(r, c);
  R = mul(R, Q);
}

// Warm-started nearest rotation in FP64: Newton steps on SO(3) from R (the
// rotation of the same tet at a nearby state).  With S = R^T M, the update
// solves (tr(S) I - sym(S)) w = a(S) and applies R <- R cay(w), where the
// Cayley map cay(w) = I + 2 ([v]x + [v]x^2) / (1 + |v|^2), v = w / 2, is
// orthogonal and agrees with exp([w]x) to second order, so convergence stays
// quadratic.  Returns false (R unusable) unless the iteration converged to the
// maximiser of tr(R^T M): there tr(S) I - sym(S) is positive definite.
__device__ __forceinline__ bool polar_warm(const M3<double>& M, M3<double>& R) {
  // one Newton-Schulz step removes drift from orthogonality: R (3 I - R^T R) / 2
  {
    M3<double> RtR;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) RtR(i, j) = R(0, i) * R(0, j) + R(1, i) * R(1, j) + R(2, i) * R(2, j);
    M3<double> Rn;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        Rn(i, j) = 1.5 * R(i, j) - 0.5 * (R(i, 0) * RtR(0, j) + R(i, 1) * RtR(1, j) + R(i, 2) * RtR(2, j));
    // the start must already be a rotation up to rounding drift
    double dev = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) dev = fmax(dev, fabs(RtR(i, j) - (i == j ? 1.0 : 0.0)));
    if (!(dev < 1e-6) || !(det3(Rn) > 0.0)) return false;
    R = Rn;
  }
  const double scale = fabs(M(0, 0)) + fabs(M(1, 1)) + fabs(M(2, 2)) + fabs(M(0, 1)) + fabs(M(1, 0)) +
                       fabs(M(0, 2)) + fabs(M(2, 0)) + fabs(M(1, 2)) + fabs(M(2, 1));
  if (!(scale > 0.0)) return false;
  bool conv = false;
  double b00 = 0, b11 = 0, b22 = 0, b01 = 0, b02 = 0, b12 = 0;
#pragma unroll 1
  for (int it = 0; it < 5; ++it) {
    double S[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) S[i][j] = R(0, i) * M(0, j) + R(1, i) * M(1, j) + R(2, i) * M(2, j);
    const double av[3] = {S[2][1] - S[1][2], S[0][2] - S[2][0], S[1][0] - S[0][1]};
    const double tr = S[0][0] + S[1][1] + S[2][2];
    b00 = tr - S[0][0]; b11 = tr - S[1][1]; b22 = tr - S[2][2];
    b01 = -0.5 * (S[0][1] + S[1][0]); b02 = -0.5 * (S[0][2] + S[2][0]); b12 = -0.5 * (S[1][2] + S[2][1]);
    const double c00 = b11 * b22 - b12 * b12, c01 = b02 * b12 - b01 * b22, c02 = b01 * b12 - b02 * b11;
    const double c11 = b00 * b22 - b02 * b02, c12 = b01 * b02 - b00 * b12, c22 = b00 * b11 - b01 * b01;
    const double det = b00 * c00 + b01 * c01 + b02 * c02;
    if (!(det > 0.0)) return false;
    const double id = 1.0 / det;
    const double w0 = (c00 * av[0] + c01 * av[1] + c02 * av[2]) * id;
    const double w1 = (c01 * av[0] + c11 * av[1] + c12 * av[2]) * id;
    const double w2 = (c02 * av[0] + c12 * av[1] + c22 * av[2]) * id;
    const double wn = fabs(w0) + fabs(w1) + fabs(w2);
    if (!(wn < 1.0)) return false;                 // too far from the basin
    const double v0 = 0.5 * w0, v1 = 0.5 * w1, v2 = 0.5 * w2;
    const double f = 2.0 / (1.0 + v0 * v0 + v1 * v1 + v2 * v2);
    M3<double> K, Q;
    K(0, 0) = 0.0; K(0, 1) = -v2; K(0, 2) = v1;
    K(1, 0) = v2; K(1, 1) = 0.0; K(1, 2) = -v0;
    K(2, 0) = -v1; K(2, 1) = v0; K(2, 2) = 0.0;
    M3<double> K2 = mul(K, K);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Q(i, j) = (i == j ? 1.0 : 0.0) + f * (K(i, j) + K2(i, j));
    R = mul(R, Q);
    if (wn < 1e-9) { conv = true; break; }         // the step just taken is below 1e-18 next
  }
  if (!conv || !(det3(R) > 0.5)) return false;
  // maximiser test on the last system matrix: leading minors positive
  return b00 > 0.0 && b00 * b11 - b01 * b01 > 0.0;
}

struct TetStreams {
  const int32_t* tets;   // 4 x m
  const double* B;       // 9 x m, D_m^-1 row-major entries
  const double* w;       // m
  const double* A;       // 6 x m: xx yy zz xy yz zx
};

__device__ __forceinline__ void load_tet(const TetStreams& ts, int64_t m, int64_t i, const double* __restrict__ x,
                                         M3<double>& F, M3<double>& A, double& w, int32_t v[4], M3<double>& Bm) {
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = ts.tets[k * m + i];
  double p0[3] = {x[3 * v[0]], x[3 * v[0] + 1], x[3 * v[0] + 2]};
  M3<double> Ds;
#pragma unroll
  for (int k = 1; k < 4; ++k) {
#pragma unroll
    for (int r = 0; r < 3; ++r) Ds(r, k - 1) = x[3 * v[k] + r] - p0[r];
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) Bm.a[e] = ts.B[e * m + i];
  F = mul(Ds, Bm);
  double a6[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) a6[e] = ts.A[e * m + i];
  A(0, 0) = a6[0]; A(1, 1) = a6[1]; A(2, 2) = a6[2];
  A(0, 1) = A(1, 0) = a6[3];
  A(1, 2) = A(2, 1) = a6[4];
  A(2, 0) = A(0, 2) = a6[5];
  w = ts.w[i];
}

// Writes per tet: R (9 x m, optional), energy (m), gradient share (m x 12,
// one 96-byte record per tet, entry 3a + r for local vertex a, coordinate r,
// so that the per-vertex gather reads one cache line per incident corner).
// Rotation of tet i at deformation M: warm-started FP64 Newton from Rwarm
// (if given), else (or if that fails) Jacobi in TP, refined in FP64 when TP
// is FP32.
template <typename TP>
__device__ __forceinline__ void tet_rotation(const M3<double>& M, const double* __restrict__ Rwarm, int64_t m,
                                             int64_t i, M3<double>& R) {
  if (Rwarm) {
#pragma unroll
    for (int e = 0; e < 9; ++e) R.a[e] = Rwarm[e * m + i];
    if (polar_warm(M, R)) return;
  }
  M3<TP> Mt, Rt;
#pragma unroll
  for (int e = 0; e < 9; ++e) Mt.a[e] = static_cast<TP>(M.a[e]);
  nearest_rotation<TP>(Mt, Rt);
#pragma unroll
  for (int e = 0; e < 9; ++e) R.a[e] = static_cast<double>(Rt.a[e]);
  if (sizeof(TP) < sizeof(double)) refine_rotation(M, R);
}

// Rwarm may alias Rout (each thread reads its own tet before writing it).
template <typename TP>
__global__ void __launch_bounds__(256) local_step_kernel(TetStreams ts, int64_t m, const double* __restrict__ x,
                                                         const double* Rwarm, double* Rout,
                                                         double* __restrict__ energy, double* __restrict__ tetg) {
  const int64_t blk = xcd_block();
  const int64_t i = blk * blockDim.x + threadIdx.x;
  double sh[12];
  if (i < m) {
    M3<double> F, A, Bm;
    double w;
    int32_t v[4];
    load_tet(ts, m, i, x, F, A, w, v, Bm);
    M3<double> M = mul(F, A);
    M3<double> R;
    tet_rotation<TP>(M, Rwarm, m, i, R);
    M3<double> P = mul(R, A);
    double res[9];
    double e2 = 0.0;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      res[e] = F.a[e] - P.a[e];
      e2 += res[e] * res[e];
    }
    energy[i] = 0.5 * w * e2;
    if (Rout) {
#pragma unroll
      for (int e = 0; e < 9; ++e) Rout[e * m + i] = R.a[e];
    }
    // g_a = row (a-1) of B for a >= 1, g_0 = -(sum of rows); share_a = w * res * g_a
    double g[4][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      g[1][c] = Bm(0, c);
      g[2][c] = Bm(1, c);
      g[3][c] = Bm(2, c);
      g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 3; ++r)
        sh[3 * a + r] = w * (res[3 * r] * g[a][0] + res[3 * r + 1] * g[a][1] + res[3 * r + 2] * g[a][2]);
  }
  if (tetg) {
    // the block's 256 records are contiguous: stage them in LDS (row pitch 13
    // against bank conflicts) and store them with consecutive lanes on
    // consecutive words
    __shared__ double stage[256 * 13];
    if (i < m) {
#pragma unroll
      for (int q = 0; q < 12; ++q) stage[threadIdx.x * 13 + q] = sh[q];
    }
    __syncthreads();
    const int64_t base = blk * blockDim.x;
    const int64_t nval = 12 * (m - base < 256 ? m - base : 256);
    double* out = tetg + 12 * base;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const int e = k * 256 + threadIdx.x;
      if (e < nval) out[e] = stage[(e / 12) * 13 + e % 12];
    }
  }
}

// Element energies at x + alpha dx (line-search trial), as differences from
// the energies at x: out[i] = E_i(x + alpha dx) - E0[i].  alpha is ls[LS_ALPHA]
// of the device line-search state; a decided search (ls[LS_STATE] != 0)
// makes the launch a no-op.
template <typename TP>
__global__ void __launch_bounds__(256) trial_energy_kernel(TetStreams ts, int64_t m, const double* __restrict__ x,
                                                           const double* __restrict__ dx,
                                                           const double* __restrict__ ls,
                                                           const double* __restrict__ Rwarm,
                                                           const double* __restrict__ E0, double* __restrict__ dE) {
  if (ls[LS_STATE] != 0.0) return;
  const double alpha = ls[LS_ALPHA];
  int64_t i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int32_t v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = ts.tets[k * m + i];
  double p[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int r = 0; r < 3; ++r) p[k][r] = x[3 * v[k] + r] + alpha * dx[3 * v[k] + r];
  M3<double> Ds, Bm, A;
#pragma unroll
  for (int k = 1; k < 4; ++k)
#pragma unroll
    for (int r = 0; r < 3; ++r) Ds(r, k - 1) = p[k][r] - p[0][r];
#pragma unroll
  for (int e = 0; e < 9; ++e) Bm.a[e] = ts.B[e * m + i];
  M3<double> F = mul(Ds, Bm);
  double a6[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) a6[e] = ts.A[e * m + i];
  A(0, 0) = a6[0]; A(1, 1) = a6[1]; A(2, 2) = a6[2];
  A(0, 1) = A(1, 0) = a6[3];
  A(1, 2) = A(2, 1) = a6[4];
  A(2, 0) = A(0, 2) = a6[5];
  M3<double> M = mul(F, A);
  M3<double> R;
  tet_rotation<TP>(M, Rwarm, m, i, R);
  M3<double> P = mul(R, A);
  double e2 = 0.0;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    double d = F.a[e] - P.a[e];
    e2 += d * d;
  }
  dE[i] = 0.5 * ts.w[i] * e2 - E0[i];
}

// Per-vertex sum of tet shares in a fixed (tet-ascending) order; fixed
// vertices get zero.  Optionally adds an extra per-vertex term (barrier).
__global__ void __launch_bounds__(256) gather_vertex_grad_kernel(int32_t n, int64_t m, const int32_t* __restrict__ vt_ptr,
                                                                 const int32_t* __restrict__ vt_ent,
                                                                 const double* __restrict__ tetg,
                                                                 const uint8_t* __restrict__ fixed,
                                                                 double* __restrict__ g) {
  const int64_t vv = xcd_block() * blockDim.x + threadIdx.x;
  if (vv >= n) return;
  const int32_t v = static_cast<int32_t>(vv);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (!fixed[v]) {
#pragma unroll 4
    for (int32_t e = vt_ptr[v]; e < vt_ptr[v + 1]; ++e) {
      int32_t ent = vt_ent[e];
      const double* sh = tetg + 12 * static_cast<int64_t>(ent >> 2) + 3 * (ent & 3);
      s0 += sh[0];
      s1 += sh[1];
      s2 += sh[2];
    }
  }
  g[3 * v] = s0;
  g[3 * v + 1] = s1;
  g[3 * v + 2] = s2;
}

// A_i from (a_i, R_i): R diag(1-a, 1+a/2, 1+a/2) R^T, stored as 6 SoA entries.
__global__ void actuation_from_scalar_kernel(int64_t m, const double* __restrict__ a, const double* __restrict__ R,
                                             double* __restrict__ A) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double ai = a[i];
  double d[3] = {1.0 - ai, 1.0 + 0.5 * ai, 1.0 + 0.5 * ai};
  double Rm[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) Rm[e] = R[9 * i + e];
  auto ent = [&](int r, int c) {
    return Rm[3 * r] * d[0] * Rm[3 * c] + Rm[3 * r + 1] * d[1] * Rm[3 * c + 1] + Rm[3 * r + 2] * d[2] * Rm[3 * c + 2];
  };
  A[0 * m + i] = ent(0, 0);
  A[1 * m + i] = ent(1, 1);
  A[2 * m + i] = ent(2, 2);
  A[3 * m + i] = ent(0, 1);
  A[4 * m + i] = ent(1, 2);
  A[5 * m + i] = ent(2, 0);
}

// caller layout (m x 6 row-major) -> SoA 6 x m
__global__ void actuation_transpose_kernel(int64_t m, const double* __restrict__ Ain, double* __restrict__ A) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
#pragma unroll
  for (int e = 0; e < 6; ++e) A[e * m + i] = Ain[6 * i + e];
}

// ---- launchers --------------------------------------------------------------
void launch_local_step(const LocalArgs& la, const double* x, const double* Rwarm, double* Rout, double* energy,
                       double* tetg, bool fp32, hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop) {
  TetStreams ts{la.tets, la.B, la.w, la.A};
  const dim3 g(grid_for(la.m, 256)), b(256);
  // with events: the runtime stamps them at the dispatch's own start and end
  if (fp32)
    hipExtLaunchKernelGGL(local_step_kernel<float>, g, b, 0, st, ev_start, ev_stop, 0, ts, la.m, x, Rwarm, Rout,
                          energy, tetg);
  else
    hipExtLaunchKernelGGL(local_step_kernel<double>, g, b, 0, st, ev_start, ev_stop, 0, ts, la.m, x, Rwarm, Rout,
                          energy, tetg);
}

void launch_trial_energy(const LocalArgs& la, const double* x, const double* dx, const double* ls,
                         const double* Rwarm, const double* E0, double* dE, bool fp32, hipStream_t st) {
  TetStreams ts{la.tets, la.B, la.w, la.A};
  unsigned g = grid_for(la.m, 256);
  if (fp32)
    trial_energy_kernel<float><<<g, 256, 0, st>>>(ts, la.m, x, dx, ls, Rwarm, E0, dE);
  else
    trial_energy_kernel<double><<<g, 256, 0, st>>>(ts, la.m, x, dx, ls, Rwarm, E0, dE);
}

__global__ void identity_rotations_kernel(int64_t m, double* __restrict__ R) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
#pragma unroll
  for (int e = 0; e < 9; ++e) R[e * m + i] = (e % 4 == 0) ? 1.0 : 0.0;
}
void launch_identity_rotations(int64_t m, double* R, hipStream_t st) {
  if (m > 0) identity_rotations_kernel<<<grid_for(m, 256), 256, 0, st>>>(m, R);
}

void launch_gather_vertex_grad(int32_t n, int64_t m, const int32_t* vt_ptr, const int32_t* vt_ent,
                               const double* tetg, const uint8_t* fixed, double* g, hipStream_t st) {
  gather_vertex_grad_kernel<<<grid_for(n, 256), 256, 0, st>>>(n, m, vt_ptr, vt_ent, tetg, fixed, g);
}

void launch_actuation_scalar(int64_t m, const double* a, const double* R, double* A, hipStream_t st) {
  actuation_from_scalar_kernel<<<grid_for(m, 256), 256, 0, st>>>(m, a, R, A);
}

void launch_actuation_transpose(int64_t m, const double* Ain, double* A, hipStream_t st) {
  actuation_transpose_kernel<<<grid_for(m, 256), 256, 0, st>>>(m, Ain, A);
}

}  // namespace pdipc
