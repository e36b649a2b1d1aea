// Unsigned distances between closed primitives (point-triangle, edge-edge)
// with the closest-feature label used by the barrier derivatives.
//
// The distance is the minimum over smooth candidates, scanned in a fixed
// order with the first minimum kept:
//   point-triangle (p, t0, t1, t2): plane foot inside the closed triangle,
//     then the segments (t0 t1), (t1 t2), (t2 t0);
//   edge-edge (a0, a1, b0, b1): line-line closest points with both
//     parameters in [0, 1] (edges not parallel), then a0, a1 against
//     segment b and b0, b1 against segment a.
// Degenerate systems (|n|^2 <= 1e-12 |e1|^2 |e2|^2) skip the interior
// candidate; for parallel segments the minimum is at an endpoint anyway.
//
// Decisions (d^2 < dhat^2 for the constraint set, the intersection check)
// take the points in absolute FP64 coordinates (load_pair_abs) and evaluate
// every product and sum separately rounded, in the order written here (the
// files that hold them are built without floating-point contraction), so
// that the same positions give the same squared distance, bit for bit, as a
// plain evaluation of these formulas.  The barrier derivatives take points
// relative to the pair's first point (load_pair_rel), which keeps the
// relative accuracy of FP32 evaluations.
#pragma once
#include "common.h"

namespace pdipc {

enum FeatureKind { KPP = 0, KPE = 1, KPT = 2, KEE = 3 };

// Squared distance as a function of the closest-point parameters beta:
// q(beta) = sum_j c_j(beta) P_j, c affine in beta; dcdb[k][j] = dc_j/dbeta_k.
template <typename T>
struct Feature {
  int kind;
  int nb;            // number of parameters (0, 1, 2)
  T c[4];
  T dcdb[2][4];
  T d2;
};

// Closest point of the closed segment [a, b] to p: q = a + t (b - a) with t
// clamped to [0, 1]; d2 = |p - q|^2.
template <typename T>
__device__ __forceinline__ T seg_param(const T* p, const T* a, const T* b, T& d2) {
  T ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  T ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
  T L2 = dot3(ab, ab);
  T t = L2 > T(0) ? dot3(ap, ab) / L2 : T(0);
  t = fmin(fmax(t, T(0)), T(1));
  T q[3] = {a[0] + t * ab[0], a[1] + t * ab[1], a[2] + t * ab[2]};
  T r[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
  d2 = dot3(r, r);
  return t;
}

// Point-segment candidate -> feature on local indices (ip; ia, ib).
template <typename T>
__device__ __forceinline__ void ps_feature(T t, int ip, int ia, int ib, T d2, Feature<T>& f) {
  f.d2 = d2;
#pragma unroll
  for (int j = 0; j < 4; ++j) { f.c[j] = T(0); f.dcdb[0][j] = T(0); f.dcdb[1][j] = T(0); }
  f.c[ip] = T(1);
  if (t <= T(0)) {
    f.kind = KPP; f.nb = 0; f.c[ia] = T(-1);
  } else if (t >= T(1)) {
    f.kind = KPP; f.nb = 0; f.c[ib] = T(-1);
  } else {
    f.kind = KPE; f.nb = 1;
    f.c[ia] = -(T(1) - t);
    f.c[ib] = -t;
    f.dcdb[0][ia] = T(1);
    f.dcdb[0][ib] = T(-1);
  }
}

template <typename T>
__device__ void point_triangle_feature(const T P[4][3], Feature<T>& f) {
  const T* p = P[0];
  const T* a = P[1];
  const T* b = P[2];
  const T* c = P[3];
  T e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  T e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  T ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
  T m11 = dot3(e1, e1), m12 = dot3(e1, e2), m22 = dot3(e2, e2);
  T r1 = dot3(ap, e1), r2 = dot3(ap, e2);
  T det = m11 * m22 - m12 * m12;
  T best = T(INFINITY);
  int which = -1;
  T u = T(0), v = T(0);
  if (det > T(1e-12) * m11 * m22) {
    u = (m22 * r1 - m12 * r2) / det;
    v = (m11 * r2 - m12 * r1) / det;
    if (u >= T(0) && v >= T(0) && u + v <= T(1)) {
      T ft[3] = {ap[0] - u * e1[0] - v * e2[0], ap[1] - u * e1[1] - v * e2[1], ap[2] - u * e1[2] - v * e2[2]};
      best = dot3(ft, ft);
      which = 0;
    }
  }
  T dab, dbc, dca;
  T tab = seg_param(p, a, b, dab);
  T tbc = seg_param(p, b, c, dbc);
  T tca = seg_param(p, c, a, dca);
  if (dab < best) { best = dab; which = 1; }
  if (dbc < best) { best = dbc; which = 2; }
  if (dca < best) { best = dca; which = 3; }
  if (which == 0) {
    f.kind = KPT; f.nb = 2; f.d2 = best;
    f.c[0] = T(1); f.c[1] = -(T(1) - u - v); f.c[2] = -u; f.c[3] = -v;
    f.dcdb[0][0] = T(0); f.dcdb[0][1] = T(1); f.dcdb[0][2] = T(-1); f.dcdb[0][3] = T(0);
    f.dcdb[1][0] = T(0); f.dcdb[1][1] = T(1); f.dcdb[1][2] = T(0); f.dcdb[1][3] = T(-1);
  } else if (which == 1) {
    ps_feature(tab, 0, 1, 2, best, f);
  } else if (which == 2) {
    ps_feature(tbc, 0, 2, 3, best, f);
  } else {
    ps_feature(tca, 0, 3, 1, best, f);
  }
}

template <typename T>
__device__ void edge_edge_feature(const T P[4][3], Feature<T>& f) {
  const T* a0 = P[0];
  const T* a1 = P[1];
  const T* b0 = P[2];
  const T* b1 = P[3];
  T ea[3] = {a1[0] - a0[0], a1[1] - a0[1], a1[2] - a0[2]};
  T eb[3] = {b1[0] - b0[0], b1[1] - b0[1], b1[2] - b0[2]};
  T w0[3] = {a0[0] - b0[0], a0[1] - b0[1], a0[2] - b0[2]};
  T aa = dot3(ea, ea), bb = dot3(eb, eb), ab = dot3(ea, eb);
  T aw = dot3(ea, w0), bw = dot3(eb, w0);
  T det = aa * bb - ab * ab;
  T best = T(INFINITY);
  int which = -1;
  T s = T(0), t = T(0);
  if (det > T(1e-12) * aa * bb) {
    s = (ab * bw - bb * aw) / det;
    t = (aa * bw - ab * aw) / det;
    if (s >= T(0) && s <= T(1) && t >= T(0) && t <= T(1)) {
      T q[3] = {w0[0] + s * ea[0] - t * eb[0], w0[1] + s * ea[1] - t * eb[1], w0[2] + s * ea[2] - t * eb[2]};
      best = dot3(q, q);
      which = 0;
    }
  }
  T d0, d1, d2, d3;
  T t0 = seg_param(a0, b0, b1, d0);
  T t1 = seg_param(a1, b0, b1, d1);
  T t2 = seg_param(b0, a0, a1, d2);
  T t3 = seg_param(b1, a0, a1, d3);
  if (d0 < best) { best = d0; which = 1; }
  if (d1 < best) { best = d1; which = 2; }
  if (d2 < best) { best = d2; which = 3; }
  if (d3 < best) { best = d3; which = 4; }
  if (which == 0) {
    f.kind = KEE; f.nb = 2; f.d2 = best;
    f.c[0] = T(1) - s; f.c[1] = s; f.c[2] = -(T(1) - t); f.c[3] = -t;
    f.dcdb[0][0] = T(-1); f.dcdb[0][1] = T(1); f.dcdb[0][2] = T(0); f.dcdb[0][3] = T(0);
    f.dcdb[1][0] = T(0); f.dcdb[1][1] = T(0); f.dcdb[1][2] = T(1); f.dcdb[1][3] = T(-1);
  } else if (which == 1) {
    ps_feature(t0, 0, 2, 3, best, f);
  } else if (which == 2) {
    ps_feature(t1, 1, 2, 3, best, f);
  } else if (which == 3) {
    ps_feature(t2, 2, 0, 1, best, f);
  } else {
    ps_feature(t3, 3, 0, 1, best, f);
  }
}

template <typename T>
__device__ __forceinline__ void pair_feature(bool is_pt, const T P[4][3], Feature<T>& f) {
  if (is_pt) point_triangle_feature(P, f);
  else edge_edge_feature(P, f);
}

// Only the squared distance (no feature bookkeeping).
template <typename T>
__device__ __forceinline__ T pair_dist2(bool is_pt, const T P[4][3]) {
  Feature<T> f;
  pair_feature(is_pt, P, f);
  return f.d2;
}

// Load the 4 points of a pair in absolute coordinates (decisions).
__device__ __forceinline__ void load_pair_abs(const int32_t* v4, const double* __restrict__ x, double P[4][3]) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int r = 0; r < 3; ++r) P[k][r] = x[3 * v4[k] + r];
}

// Load the 4 points of a pair relative to its first point (FP64 difference).
__device__ __forceinline__ void load_pair_rel(const int32_t* v4, const double* __restrict__ x, double P[4][3]) {
  double o[3] = {x[3 * v4[0]], x[3 * v4[0] + 1], x[3 * v4[0] + 2]};
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int r = 0; r < 3; ++r) P[k][r] = x[3 * v4[k] + r] - o[r];
}

// Same at x + alpha dx (positions formed first, then differenced).
__device__ __forceinline__ void load_pair_rel_step(const int32_t* v4, const double* __restrict__ x,
                                                   const double* __restrict__ dx, double alpha, double P[4][3]) {
  double q[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int r = 0; r < 3; ++r) q[k][r] = x[3 * v4[k] + r] + alpha * dx[3 * v4[k] + r];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int r = 0; r < 3; ++r) P[k][r] = q[k][r] - q[0][r];
}

// Barrier of a pair at squared distance D (0 < D < dhat^2), the energy
// kappa b and its first two derivatives in D (phi1 = dE/dD, phi2 = d2E/dD2):
// form 0 is IPC's b(d) = -(d - dhat)^2 ln(d / dhat) on d = sqrt(D); form 1 is
// the same function of D with threshold dhat^2, -(D - dhat^2)^2 ln(D / dhat^2).
template <typename T>
__device__ __forceinline__ void barrier_of_D(T D, T dhat, T kappa, int form, T& e, T& phi1, T& phi2) {
  if (form == 0) {
    const T d = sqrt(D);
    const T u = d - dhat, lg = log(d / dhat);
    const T b1 = -T(2) * u * lg - u * u / d;
    const T b2 = -T(2) * lg - T(4) * u / d + u * u / (d * d);
    e = -kappa * u * u * lg;
    phi1 = kappa * b1 / (T(2) * d);
    phi2 = kappa * (b2 - b1 / d) / (T(4) * D);
  } else {
    const T Dh = dhat * dhat;
    const T u = D - Dh, lg = log(D / Dh);
    e = -kappa * u * u * lg;
    phi1 = kappa * (-T(2) * u * lg - u * u / D);
    phi2 = kappa * (-T(2) * lg - T(4) * u / D + u * u / (D * D));
  }
}

// b at squared distance D (0 < D), zero from the threshold on.
__device__ __forceinline__ double barrier_b_of_D(double D, double dhat, int form) {
  if (!(D < dhat * dhat)) return 0.0;
  if (form == 0) {
    const double d = sqrt(D), u = d - dhat;
    return -u * u * log(d / dhat);
  }
  const double Dh = dhat * dhat, u = D - Dh;
  return -u * u * log(D / Dh);
}

}  // namespace pdipc
