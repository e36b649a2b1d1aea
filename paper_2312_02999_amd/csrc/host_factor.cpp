// Nested-dissection ordering and multifrontal factorization of the constant
// PD matrix (host, FP64).  See host_factor.h for the layout.
#include "host_factor.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>

namespace pdipc {
namespace {

struct Dissector {
  const double* xyz;
  const ScalarCSR* H;
  int32_t n1;
  int32_t leaf;
  std::vector<char> mark;                 // scratch flags over x1
  std::vector<int32_t> order;             // emitted columns (x1 input ids)
  std::vector<FactorNode> nodes;
  std::vector<std::vector<int32_t>> node_cols;
  std::vector<std::vector<int32_t>> node_kids;

  int emit(std::vector<int32_t>& cols, const std::vector<int32_t>& kids) {
    FactorNode nd{};
    nd.c0 = static_cast<int32_t>(order.size());
    nd.s = static_cast<int32_t>(cols.size());
    nd.parent = -1;
    order.insert(order.end(), cols.begin(), cols.end());
    nodes.push_back(nd);
    node_cols.push_back(cols);
    node_kids.push_back(kids);
    int id = static_cast<int>(nodes.size()) - 1;
    for (int k : kids) nodes[k].parent = id;
    return id;
  }

  // Returns the roots of the sub-forest built on S (post-order emission).
  std::vector<int> build(std::vector<int32_t>& S) {
    if (static_cast<int32_t>(S.size()) <= leaf) {
      if (S.empty()) return {};
      return {emit(S, {})};
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t v : S)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], xyz[3 * v + d]);
        hi[d] = std::max(hi[d], xyz[3 * v + d]);
      }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
      if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
    size_t half = S.size() / 2;
    std::nth_element(S.begin(), S.begin() + half, S.end(), [&](int32_t a, int32_t b) {
      double ca = xyz[3 * a + ax], cb = xyz[3 * b + ax];
      return ca < cb || (ca == cb && a < b);
    });
    std::vector<int32_t> left(S.begin(), S.begin() + half), right(S.begin() + half, S.end());
    for (int32_t v : left) mark[v] = 1;
    std::vector<int32_t> sep, rest;
    for (int32_t v : right) {
      bool touches = false;
      for (int64_t e = H->ptr[v]; e < H->ptr[v + 1]; ++e) {
        int32_t u = H->col[e];
        if (u < n1 && mark[u]) { touches = true; break; }
      }
      (touches ? sep : rest).push_back(v);
    }
    for (int32_t v : left) mark[v] = 0;
    if (rest.empty() || left.empty()) {       // no useful split: dense node
      return {emit(S, {})};
    }
    std::sort(sep.begin(), sep.end());
    std::vector<int> kids = build(left);
    std::vector<int> kr = build(rest);
    kids.insert(kids.end(), kr.begin(), kr.end());
    if (sep.empty()) return kids;             // disconnected halves: a forest
    return {emit(sep, kids)};
  }
};

// Dense in-place partial Cholesky of an m x m column-major front on its first
// s columns; the trailing (m-s) x (m-s) block becomes the update matrix.
bool partial_cholesky(double* F, int m, int s, double tiny) {
  for (int k = 0; k < s; ++k) {
    double* ck = F + static_cast<int64_t>(k) * m;
    double d = ck[k];
    if (!(d > tiny)) return false;
    d = std::sqrt(d);
    ck[k] = d;
    double inv = 1.0 / d;
    for (int i = k + 1; i < m; ++i) ck[i] *= inv;
    for (int j = k + 1; j < m; ++j) {
      double f = ck[j];
      if (f == 0.0) continue;
      double* cj = F + static_cast<int64_t>(j) * m;
      for (int i = j; i < m; ++i) cj[i] -= ck[i] * f;
    }
  }
  return true;
}

// Inverse of a lower-triangular s x s block (column-major input, ld m) into
// a row-major s x s output (upper part zero).
void lower_inverse(const double* L, int ld, int s, double* out) {
  std::fill(out, out + static_cast<int64_t>(s) * s, 0.0);
  std::vector<double> col(s);
  for (int j = 0; j < s; ++j) {
    // solve L x = e_j by forward substitution
    std::fill(col.begin(), col.end(), 0.0);
    col[j] = 1.0 / L[static_cast<int64_t>(j) * ld + j];
    for (int i = j + 1; i < s; ++i) {
      double acc = 0.0;
      for (int k = j; k < i; ++k) acc += L[static_cast<int64_t>(k) * ld + i] * col[k];
      col[i] = -acc / L[static_cast<int64_t>(i) * ld + i];
    }
    for (int i = j; i < s; ++i) out[static_cast<int64_t>(i) * s + j] = col[i];
  }
}

}  // namespace

int build_host_factor(int32_t n1, int32_t n2, const double* coords1, const ScalarCSR& H,
                      int32_t leaf_size, HostFactor& out, std::string& err) {
  out = HostFactor{};
  out.n1 = n1;
  out.n2 = n2;
  const int32_t N = n1 + n2;

  // ---- ordering -----------------------------------------------------------
  Dissector D;
  D.xyz = coords1;
  D.H = &H;
  D.n1 = n1;
  D.leaf = std::max<int32_t>(8, leaf_size);
  D.mark.assign(n1, 0);
  std::vector<int32_t> all(n1);
  std::iota(all.begin(), all.end(), 0);
  std::vector<int> roots = D.build(all);
  const int nn = static_cast<int>(D.nodes.size());
  out.perm = D.order;
  std::vector<int32_t> ext(N);                 // input extended index -> new
  for (int32_t p = 0; p < n1; ++p) ext[out.perm[p]] = p;
  for (int32_t q = 0; q < n2; ++q) ext[n1 + q] = n1 + q;

  // ---- symbolic: row sets R(J) in post-order --------------------------------
  std::vector<std::vector<int32_t>> R(nn);
  std::vector<int32_t> stamp(N, -1);
  for (int J = 0; J < nn; ++J) {
    FactorNode& nd = D.nodes[J];
    const int32_t c1 = nd.c0 + nd.s;
    std::vector<int32_t>& rj = R[J];
    for (int32_t p = nd.c0; p < c1; ++p) {
      int32_t v = out.perm[p];
      for (int64_t e = H.ptr[v]; e < H.ptr[v + 1]; ++e) {
        int32_t u = ext[H.col[e]];
        if (u >= c1 && stamp[u] != J) { stamp[u] = J; rj.push_back(u); }
      }
    }
    for (int K : D.node_kids[J])
      for (int32_t u : R[K])
        if (u >= c1 && stamp[u] != J) { stamp[u] = J; rj.push_back(u); }
    std::sort(rj.begin(), rj.end());
    nd.r = static_cast<int32_t>(rj.size());
  }
  // levels (height) for the level-scheduled sweeps
  int maxlev = 0;
  for (int J = 0; J < nn; ++J) {
    int lev = 0;
    for (int K : D.node_kids[J]) lev = std::max(lev, D.nodes[K].level + 1);
    D.nodes[J].level = lev;
    maxlev = std::max(maxlev, lev);
  }
  out.nlevels = nn ? maxlev + 1 : 0;

  // offsets
  int64_t roff = 0, poff = 0, doff = 0;
  for (int J = 0; J < nn; ++J) {
    FactorNode& nd = D.nodes[J];
    nd.rows_off = roff;
    nd.panel_off = poff;
    nd.dinv_off = doff;
    roff += nd.r;
    poff += static_cast<int64_t>(nd.r) * nd.s;
    doff += static_cast<int64_t>(nd.s) * nd.s;
  }
  out.rows.resize(roff);
  out.panel.resize(poff);
  out.dinv.resize(doff);
  for (int J = 0; J < nn; ++J)
    std::copy(R[J].begin(), R[J].end(), out.rows.begin() + D.nodes[J].rows_off);

  // ---- numeric multifrontal -------------------------------------------------
  // pivots below 1e-13 of the largest diagonal entry mean a singular matrix
  double maxdiag = 0.0;
  for (int32_t v = 0; v < N; ++v)
    for (int64_t e = H.ptr[v]; e < H.ptr[v + 1]; ++e)
      if (H.col[e] == v) maxdiag = std::max(maxdiag, std::fabs(H.val[e]));
  const double tiny = 1e-13 * maxdiag;
  std::vector<std::vector<double>> update(nn);   // pending child updates
  std::vector<int32_t> loc(N, -1);
  std::vector<double> sigma(static_cast<size_t>(n2) * n2, 0.0);
  int64_t nnz = 0;
  for (int J = 0; J < nn; ++J) {
    FactorNode& nd = D.nodes[J];
    const int s = nd.s, r = nd.r, m = s + r;
    std::vector<double> F(static_cast<size_t>(m) * m, 0.0);
    for (int i = 0; i < s; ++i) loc[nd.c0 + i] = i;
    for (int i = 0; i < r; ++i) loc[R[J][i]] = s + i;
    for (int i = 0; i < s; ++i) {
      const int32_t c = nd.c0 + i;
      const int32_t v = out.perm[c];
      for (int64_t e = H.ptr[v]; e < H.ptr[v + 1]; ++e) {
        int32_t u = ext[H.col[e]];
        if (u < c) continue;
        F[static_cast<size_t>(i) * m + loc[u]] += H.val[e];
      }
    }
    for (int K : D.node_kids[J]) {
      const std::vector<double>& U = update[K];
      const std::vector<int32_t>& RK = R[K];
      const int rk = static_cast<int>(RK.size());
      for (int b = 0; b < rk; ++b) {
        const int lb = loc[RK[b]];
        for (int a = b; a < rk; ++a) F[static_cast<size_t>(lb) * m + loc[RK[a]]] += U[static_cast<size_t>(b) * rk + a];
      }
      std::vector<double>().swap(update[K]);
    }
    if (!partial_cholesky(F.data(), m, s, tiny)) {
      err = "PD matrix H11 is not positive definite (no fixed vertices in a component?)";
      return -3;
    }
    double* pan = out.panel.data() + nd.panel_off;
    for (int i = 0; i < r; ++i)
      for (int c = 0; c < s; ++c) pan[static_cast<int64_t>(i) * s + c] = F[static_cast<size_t>(c) * m + s + i];
    lower_inverse(F.data(), m, s, out.dinv.data() + nd.dinv_off);
    nnz += static_cast<int64_t>(s) * (s + 1) / 2 + static_cast<int64_t>(r) * s;
    std::vector<double> U(static_cast<size_t>(r) * r);
    for (int b = 0; b < r; ++b)
      for (int a = b; a < r; ++a) U[static_cast<size_t>(b) * r + a] = F[static_cast<size_t>(s + b) * m + s + a];
    if (nd.parent >= 0) {
      update[J] = std::move(U);
    } else {                                       // child of the x2 root
      for (int b = 0; b < r; ++b) {
        const int32_t rb = R[J][b];
        if (rb < n1) continue;                     // cannot happen for a root
        for (int a = b; a < r; ++a) {
          const int32_t ra = R[J][a];
          double vv = U[static_cast<size_t>(b) * r + a];
          sigma[static_cast<size_t>(ra - n1) * n2 + (rb - n1)] += vv;
          if (ra != rb) sigma[static_cast<size_t>(rb - n1) * n2 + (ra - n1)] += vv;
        }
      }
    }
    for (int i = 0; i < s; ++i) loc[nd.c0 + i] = -1;
    for (int i = 0; i < r; ++i) loc[R[J][i]] = -1;
  }
  // Sigma_s = H22 - sum of root updates  (updates hold -H21 H11^-1 H12 parts)
  for (int32_t q = 0; q < n2; ++q) {
    const int32_t v = n1 + q;
    for (int64_t e = H.ptr[v]; e < H.ptr[v + 1]; ++e) {
      int32_t u = H.col[e];
      if (u < n1) continue;
      sigma[static_cast<size_t>(q) * n2 + (u - n1)] += H.val[e];
    }
  }
  out.sigma = std::move(sigma);
  out.factor_nnz = nnz;

  // ---- row-wise copy of all panel entries for the forward sweep -------------
  out.fwd_ptr.assign(static_cast<size_t>(N) + 1, 0);
  for (int J = 0; J < nn; ++J)
    for (int i = 0; i < D.nodes[J].r; ++i) out.fwd_ptr[R[J][i] + 1] += D.nodes[J].s;
  for (int32_t i = 0; i < N; ++i) out.fwd_ptr[i + 1] += out.fwd_ptr[i];
  out.fwd_col.resize(out.fwd_ptr[N]);
  out.fwd_val.resize(out.fwd_ptr[N]);
  std::vector<int64_t> cur(out.fwd_ptr.begin(), out.fwd_ptr.end() - 1);
  for (int J = 0; J < nn; ++J) {
    const FactorNode& nd = D.nodes[J];
    const double* pan = out.panel.data() + nd.panel_off;
    for (int i = 0; i < nd.r; ++i) {
      int64_t& c = cur[R[J][i]];
      for (int k = 0; k < nd.s; ++k) {
        out.fwd_col[c] = nd.c0 + k;
        out.fwd_val[c] = pan[static_cast<int64_t>(i) * nd.s + k];
        ++c;
      }
    }
  }
  out.nodes = std::move(D.nodes);
  (void)roots;
  return 0;
}

}  // namespace pdipc
