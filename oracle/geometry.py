"""Unsigned distances between closed collision primitives (Section 2.2).

Oracle module (test infrastructure only).

The distance between a point and a closed triangle, or between two closed
segments, is the minimum over a few smooth candidates:

* point-triangle: the plane distance if the foot point lies in the closed
  triangle, else the distance to the nearest of the three closed edges;
* edge-edge: the line-line distance if both closest-point parameters lie in
  [0, 1] (lines not parallel), else the nearest endpoint-to-segment distance.
  For parallel segments the minimum is always attained at an endpoint.

Each pair is labelled with the feature that attains the minimum (``kind`` and
the local indices of the involved points) so that derivatives can be taken of
one smooth formula.  Local point order: point-triangle (p, t0, t1, t2);
edge-edge (a0, a1, b0, b1).

Reading: the line-line candidate is skipped when the edges are numerically
parallel, i.e. |ea x eb|^2 <= 1e-12 |ea|^2 |eb|^2.
"""
from __future__ import annotations

import numpy as np

PP, PE, PT, EE = 0, 1, 2, 3
PARALLEL_EPS = 1e-12


def _dot(u, v):
    return np.sum(u * v, axis=-1)


def point_segment(p, a, b):
    """Squared distance from p to the closed segment [a, b] and the clamped t."""
    ab = b - a
    L2 = _dot(ab, ab)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(L2 > 0, _dot(p - a, ab) / np.where(L2 > 0, L2, 1.0), 0.0)
    t = np.clip(t, 0.0, 1.0)
    q = a + t[..., None] * ab
    return _dot(p - q, p - q), t


def _ps_label(t, ip, ia, ib):
    """Feature label of a point-segment candidate: PP at an end or PE inside."""
    k = t.shape[0]
    kind = np.full(k, PE)
    idx = np.tile(np.array([ip, ia, ib, -1]), (k, 1))
    at_a = t <= 0.0
    at_b = t >= 1.0
    kind[at_a | at_b] = PP
    idx[at_a] = [ip, ia, -1, -1]
    idx[at_b] = [ip, ib, -1, -1]
    return kind, idx


def point_triangle(p, a, b, c):
    """Batched point-triangle distance. Returns (d2, kind, idx[k,4])."""
    p, a, b, c = (np.atleast_2d(np.asarray(v, dtype=np.float64)) for v in (p, a, b, c))
    k = p.shape[0]
    e1, e2, ap = b - a, c - a, p - a
    m11, m12, m22 = _dot(e1, e1), _dot(e1, e2), _dot(e2, e2)
    r1, r2 = _dot(ap, e1), _dot(ap, e2)
    det = m11 * m22 - m12 * m12
    valid = det > PARALLEL_EPS * m11 * m22
    sdet = np.where(valid, det, 1.0)
    u = (m22 * r1 - m12 * r2) / sdet
    v = (m11 * r2 - m12 * r1) / sdet
    inside = valid & (u >= 0) & (v >= 0) & (u + v <= 1)
    foot = ap - u[:, None] * e1 - v[:, None] * e2
    d_in = np.where(inside, _dot(foot, foot), np.inf)
    d_ab, t_ab = point_segment(p, a, b)
    d_bc, t_bc = point_segment(p, b, c)
    d_ca, t_ca = point_segment(p, c, a)
    cand = np.stack([d_in, d_ab, d_bc, d_ca], axis=1)
    which = np.argmin(cand, axis=1)
    d2 = cand[np.arange(k), which]
    kind = np.empty(k, dtype=np.int64)
    idx = np.empty((k, 4), dtype=np.int64)
    labels = [(np.full(k, PT), np.tile([0, 1, 2, 3], (k, 1))),
              _ps_label(t_ab, 0, 1, 2), _ps_label(t_bc, 0, 2, 3), _ps_label(t_ca, 0, 3, 1)]
    for w, (kd, ix) in enumerate(labels):
        sel = which == w
        kind[sel] = kd[sel]
        idx[sel] = ix[sel]
    return d2, kind, idx


def edge_edge(a0, a1, b0, b1):
    """Batched segment-segment distance. Returns (d2, kind, idx[k,4])."""
    a0, a1, b0, b1 = (np.atleast_2d(np.asarray(v, dtype=np.float64)) for v in (a0, a1, b0, b1))
    k = a0.shape[0]
    ea, eb, w0 = a1 - a0, b1 - b0, a0 - b0
    aa, bb, ab = _dot(ea, ea), _dot(eb, eb), _dot(ea, eb)
    aw, bw = _dot(ea, w0), _dot(eb, w0)
    det = aa * bb - ab * ab
    valid = det > PARALLEL_EPS * aa * bb
    sdet = np.where(valid, det, 1.0)
    s = (ab * bw - bb * aw) / sdet
    t = (aa * bw - ab * aw) / sdet
    inside = valid & (s >= 0) & (s <= 1) & (t >= 0) & (t <= 1)
    q = w0 + s[:, None] * ea - t[:, None] * eb
    d_in = np.where(inside, _dot(q, q), np.inf)
    d0, t0 = point_segment(a0, b0, b1)
    d1, t1 = point_segment(a1, b0, b1)
    d2_, t2 = point_segment(b0, a0, a1)
    d3, t3 = point_segment(b1, a0, a1)
    cand = np.stack([d_in, d0, d1, d2_, d3], axis=1)
    which = np.argmin(cand, axis=1)
    dd = cand[np.arange(k), which]
    kind = np.empty(k, dtype=np.int64)
    idx = np.empty((k, 4), dtype=np.int64)
    labels = [(np.full(k, EE), np.tile([0, 1, 2, 3], (k, 1))),
              _ps_label(t0, 0, 2, 3), _ps_label(t1, 1, 2, 3),
              _ps_label(t2, 2, 0, 1), _ps_label(t3, 3, 0, 1)]
    for w, (kd, ix) in enumerate(labels):
        sel = which == w
        kind[sel] = kd[sel]
        idx[sel] = ix[sel]
    return dd, kind, idx


def point_triangle_distance(p, a, b, c):
    return np.sqrt(point_triangle(p, a, b, c)[0])


def edge_edge_distance(a0, a1, b0, b1):
    return np.sqrt(edge_edge(a0, a1, b0, b1)[0])
