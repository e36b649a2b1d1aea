"""IPC barrier energy and its derivatives (Eq. 3, Algorithm 1).

Oracle module (test infrastructure only).

Readings:
* b(d) = -(d - dhat)^2 ln(d / dhat) for 0 < d < dhat, else 0 -- the barrier of
  Incremental Potential Contact on the unsigned distance d (the paper only
  says "logarithm-like", active below the threshold d_0 = dhat).  This is
  form 0.  Form 1 is the same function of the squared distance D = d^2 with
  threshold dhat^2: b(D) = -(D - dhat^2)^2 ln(D / dhat^2) for D < dhat^2 (the
  squared-distance variant used by IPC implementations).  Both vanish with
  their first two derivatives at the threshold and select the same pairs.
* B(x) = kappa * sum_k b(d_k(x)) (Eq. 3).
* "PositiveDefinite" (Algorithm 1) is read as: per pair, eigen-decompose the
  12 x 12 Hessian and clamp negative eigenvalues to zero.

Derivatives are taken by automatic differentiation (torch.func, CPU, float64)
of kappa * b(sqrt(D(x))), where D is the explicit squared-distance formula of
the feature that attains the minimum (see ``geometry``).  Nothing here is a
hand-derived derivative.
"""
from __future__ import annotations

import numpy as np
import torch
from torch.func import grad, hessian, vmap

from . import geometry as geo


def barrier(d, dhat, form: int = 0):
    """b for an array of distances d (numpy): b(d) (form 0) or b(d^2) with
    threshold dhat^2 (form 1)."""
    d = np.asarray(d, dtype=np.float64)
    out = np.zeros_like(d)
    act = (d > 0) & (d < dhat)
    dd = d[act]
    if form == 0:
        out[act] = -((dd - dhat) ** 2) * np.log(dd / dhat)
    else:
        D, Dh = dd * dd, dhat * dhat
        out[act] = -((D - Dh) ** 2) * np.log(D / Dh)
    return out


def _b_torch(d, dhat):
    return -((d - dhat) ** 2) * torch.log(d / dhat)


def _b_of_sqdist(D, dhat, form):
    """The barrier as a function of the squared distance D (torch)."""
    if form == 0:
        return _b_torch(torch.sqrt(D), dhat)
    return _b_torch(D, dhat * dhat)


def _sqdist(kind: int, P):
    if kind == geo.PP:
        v = P[0] - P[1]
        return torch.dot(v, v)
    if kind == geo.PE:
        e = P[2] - P[1]
        c = torch.linalg.cross(P[0] - P[1], e)
        return torch.dot(c, c) / torch.dot(e, e)
    if kind == geo.PT:
        n = torch.linalg.cross(P[2] - P[1], P[3] - P[1])
        h = torch.dot(P[0] - P[1], n)
        return h * h / torch.dot(n, n)
    if kind == geo.EE:
        n = torch.linalg.cross(P[1] - P[0], P[3] - P[2])
        h = torch.dot(P[2] - P[0], n)
        return h * h / torch.dot(n, n)
    raise ValueError(kind)


def squared_distance_by_feature(X4: np.ndarray, kind: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """D for each pair, evaluated with the labelled feature's formula."""
    out = np.empty(X4.shape[0])
    for (kd, sel), rows in _groups(kind, idx).items():
        Xt = torch.from_numpy(X4[rows].reshape(len(rows), 12))
        f = _make_sqdist_fn(kd, sel)
        out[rows] = vmap(f)(Xt).numpy()
    return out


def _make_sqdist_fn(kd, sel):
    sel = list(sel)

    def f(x12):
        return _sqdist(kd, x12.reshape(4, 3)[sel])
    return f


def _make_barrier_fn(kd, sel, dhat, kappa, form=0):
    sel = list(sel)

    def f(x12):
        D = _sqdist(kd, x12.reshape(4, 3)[sel])
        return kappa * _b_of_sqdist(D, dhat, form)
    return f


def _groups(kind, idx):
    groups: dict = {}
    for r in range(kind.shape[0]):
        sel = tuple(int(v) for v in idx[r] if v >= 0)
        groups.setdefault((int(kind[r]), sel), []).append(r)
    return {k: np.asarray(v) for k, v in groups.items()}


def pair_derivatives(X4: np.ndarray, kind: np.ndarray, idx: np.ndarray, dhat: float, kappa: float,
                     form: int = 0):
    """kappa b, its gradient (k, 12) and Hessian (k, 12, 12) for active pairs.

    X4 (k, 4, 3): the four points of each pair in local order.  All pairs
    must satisfy 0 < d < dhat.  form: 0 = b(d), 1 = b(d^2) (see above).
    """
    k = X4.shape[0]
    E = np.zeros(k)
    G = np.zeros((k, 12))
    H = np.zeros((k, 12, 12))
    for (kd, sel), rows in _groups(kind, idx).items():
        Xt = torch.from_numpy(np.ascontiguousarray(X4[rows].reshape(len(rows), 12)))
        f = _make_barrier_fn(kd, sel, dhat, kappa, form)
        E[rows] = vmap(f)(Xt).numpy()
        G[rows] = vmap(grad(f))(Xt).numpy()
        H[rows] = vmap(hessian(f))(Xt).numpy()
    return E, G, H


def project_psd(H: np.ndarray) -> np.ndarray:
    """Clamp negative eigenvalues of each symmetric block to zero."""
    if H.shape[0] == 0:
        return H.copy()
    Hs = 0.5 * (H + np.swapaxes(H, -1, -2))
    lam, Q = np.linalg.eigh(Hs)
    lam = np.maximum(lam, 0.0)
    return np.einsum("kij,kj,klj->kil", Q, lam, Q)
