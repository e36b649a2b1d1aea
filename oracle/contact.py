"""Constraint sets and swept candidate sets by brute force (Section 2.2).

Oracle module (test infrastructure only).

Primitives come from the proxy triangles (embedded by selection, so proxy
positions are simulation positions):
* vertices: the sorted simulation ids used by proxy triangles;
* triangles: the proxy triangle list, in the given order;
* edges: unique undirected edges (lo, hi) of the triangles, sorted
  lexicographically.

Pair families (no de-duplication across families):
* point-triangle (v, f): v a proxy vertex, f a triangle with v not in f;
* edge-edge (e, e'): e < e' in edge order, no shared vertex.

Every candidate list is the exact set of pairs whose axis-aligned boxes
overlap with margin dhat: lo_a <= hi_b + dhat and lo_b <= hi_a + dhat on all
three axes.  The constraint set keeps candidates with squared distance
strictly below dhat^2.  Both lists are sorted by (first index, second index).
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np

from . import geometry as geo


@dataclass
class Proxy:
    verts: np.ndarray   # (nv,) sim ids
    tris: np.ndarray    # (nf, 3) sim ids
    edges: np.ndarray   # (ne, 2) sim ids, lo < hi, sorted


def make_proxy(surf_tris: np.ndarray) -> Proxy:
    tris = np.asarray(surf_tris, dtype=np.int64)
    verts = np.unique(tris.reshape(-1))
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]], axis=0)
    e = np.unique(np.sort(e, axis=1), axis=0)
    return Proxy(verts=verts, tris=tris, edges=e)


def _boxes(x0, x1, prims):
    """Box of each primitive over the positions x0 and x1 (x1 may be x0)."""
    P0 = x0[prims]
    P1 = x1[prims]
    lo = np.minimum(P0.min(axis=1), P1.min(axis=1))
    hi = np.maximum(P0.max(axis=1), P1.max(axis=1))
    return lo, hi


def _overlap_pairs(lo_a, hi_a, lo_b, hi_b, margin, upper_only=False, chunk=512):
    """All (i, j) whose boxes overlap with the margin; sorted by (i, j)."""
    out_i, out_j = [], []
    nb = lo_b.shape[0]
    for s in range(0, lo_a.shape[0], chunk):
        la, ha = lo_a[s:s + chunk, None, :], hi_a[s:s + chunk, None, :]
        ok = np.all((la <= hi_b[None] + margin) & (lo_b[None] <= ha + margin), axis=2)
        if upper_only:
            ii = np.arange(s, s + ok.shape[0])[:, None]
            ok &= np.arange(nb)[None, :] > ii
        i, j = np.nonzero(ok)
        out_i.append(i + s)
        out_j.append(j)
    if not out_i:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(out_i), np.concatenate(out_j)


def candidates(x0: np.ndarray, x1: np.ndarray, prox: Proxy, dhat: float):
    """Point-triangle and edge-edge candidates over the motion x0 -> x1.

    Returns ((v_sim, f), (e, e')) index arrays, incident pairs excluded.
    """
    vlo, vhi = _boxes(x0, x1, prox.verts[:, None])
    tlo, thi = _boxes(x0, x1, prox.tris)
    elo, ehi = _boxes(x0, x1, prox.edges)
    vi, fi = _overlap_pairs(vlo, vhi, tlo, thi, dhat)
    v = prox.verts[vi]
    keep = np.all(prox.tris[fi] != v[:, None], axis=1)
    pt = np.stack([v[keep], fi[keep]], axis=1)
    ei, ej = _overlap_pairs(elo, ehi, elo, ehi, dhat, upper_only=True)
    A, B = prox.edges[ei], prox.edges[ej]
    keep = ((A[:, 0] != B[:, 0]) & (A[:, 0] != B[:, 1]) &
            (A[:, 1] != B[:, 0]) & (A[:, 1] != B[:, 1]))
    ee = np.stack([ei[keep], ej[keep]], axis=1)
    return pt.astype(np.int64), ee.astype(np.int64)


def pair_points(x: np.ndarray, prox: Proxy, pt: np.ndarray, ee: np.ndarray) -> np.ndarray:
    """(|pt| + |ee|, 4, 3) local point coordinates, point-triangle rows first."""
    Xpt = np.concatenate([x[pt[:, 0]][:, None, :], x[prox.tris[pt[:, 1]]]], axis=1) \
        if len(pt) else np.zeros((0, 4, 3))
    Xee = np.concatenate([x[prox.edges[ee[:, 0]]], x[prox.edges[ee[:, 1]]]], axis=1) \
        if len(ee) else np.zeros((0, 4, 3))
    return np.concatenate([Xpt, Xee], axis=0)


def pair_vertices(prox: Proxy, pt: np.ndarray, ee: np.ndarray) -> np.ndarray:
    """(|pt| + |ee|, 4) simulation vertex ids of each pair's local points."""
    Vpt = np.concatenate([pt[:, :1], prox.tris[pt[:, 1]]], axis=1) if len(pt) else np.zeros((0, 4), np.int64)
    Vee = np.concatenate([prox.edges[ee[:, 0]], prox.edges[ee[:, 1]]], axis=1) if len(ee) else np.zeros((0, 4), np.int64)
    return np.concatenate([Vpt, Vee], axis=0).astype(np.int64)


def pair_distances(x: np.ndarray, prox: Proxy, pt: np.ndarray, ee: np.ndarray):
    """(d2, kind, idx) for the given pairs, point-triangle rows first."""
    X4 = pair_points(x, prox, pt, ee)
    npt = len(pt)
    d2 = np.empty(X4.shape[0])
    kind = np.empty(X4.shape[0], dtype=np.int64)
    idx = np.empty((X4.shape[0], 4), dtype=np.int64)
    if npt:
        d2[:npt], kind[:npt], idx[:npt] = geo.point_triangle(X4[:npt, 0], X4[:npt, 1], X4[:npt, 2], X4[:npt, 3])
    if len(ee):
        d2[npt:], kind[npt:], idx[npt:] = geo.edge_edge(X4[npt:, 0], X4[npt:, 1], X4[npt:, 2], X4[npt:, 3])
    return d2, kind, idx


@dataclass
class ConstraintSet:
    pt: np.ndarray      # (kp, 2) [v_sim, f]
    ee: np.ndarray      # (ke, 2) [e, e']
    d2: np.ndarray      # squared distances, pt rows first
    kind: np.ndarray
    idx: np.ndarray

    @property
    def size(self):
        return len(self.pt) + len(self.ee)


def constraint_set(x: np.ndarray, prox: Proxy, dhat: float) -> ConstraintSet:
    """Active pairs: squared distance strictly below dhat^2 (Algorithm 1)."""
    pt, ee = candidates(x, x, prox, dhat)
    d2, kind, idx = pair_distances(x, prox, pt, ee)
    act = d2 < dhat * dhat
    npt = len(pt)
    return ConstraintSet(pt=pt[act[:npt]], ee=ee[act[npt:]], d2=d2[act],
                         kind=kind[act], idx=idx[act])


def min_distance(x: np.ndarray, prox: Proxy, pt=None, ee=None) -> float:
    """Smallest pair distance over the given (or all non-incident) pairs."""
    if pt is None:
        big = 1e30
        pt, ee = candidates(x, x, prox, big)
    d2, _, _ = pair_distances(x, prox, pt, ee)
    return float(np.sqrt(d2.min())) if d2.size else np.inf
