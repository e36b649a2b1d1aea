"""Continuous-collision step bound (Section 2.2, "largest possible step size
that does not cause penetration").

Oracle module (test infrastructure only).

Reading (the paper names CCD without an algorithm): additive conservative
advancement with a fixed number of steps.  For a candidate pair with current
distance d_0 and per-point displacements D_j over the full step:

* subtract the mean displacement of the pair's points (only relative motion
  changes a distance);
* l = |D'_p| + max_j |D'_{t_j}| (point-triangle) or
  max(|D'_{a0}|, |D'_{a1}|) + max(|D'_{b0}|, |D'_{b1}|) (edge-edge) bounds the
  rate at which the distance can shrink per unit step;
* target gap g = eta * d_0 with eta = 0.1;
* t = 0, then N = 16 times: t <- min(1, t + max(0, d(x + t dx) - g) / l);
  l = 0 gives t = 1.

Since the distance is 1-Lipschitz in the relative motion, no pair can get
closer than g for any step up to t.  The bound is alpha_m = min(1, min_k t_k).
The result is continuous in the inputs.
"""
from __future__ import annotations

import numpy as np

from . import contact

ETA = 0.1
STEPS = 16


def motion_bound(D4: np.ndarray, n_pt: int) -> np.ndarray:
    Dc = D4 - D4.mean(axis=1, keepdims=True)
    nrm = np.linalg.norm(Dc, axis=2)
    l = np.empty(D4.shape[0])
    l[:n_pt] = nrm[:n_pt, 0] + nrm[:n_pt, 1:].max(axis=1)
    l[n_pt:] = nrm[n_pt:, :2].max(axis=1) + nrm[n_pt:, 2:].max(axis=1)
    return l


def _pair_d2(X4, n_pt):
    from . import geometry as geo
    d2 = np.empty(X4.shape[0])
    if n_pt:
        d2[:n_pt] = geo.point_triangle(X4[:n_pt, 0], X4[:n_pt, 1], X4[:n_pt, 2], X4[:n_pt, 3])[0]
    if X4.shape[0] > n_pt:
        d2[n_pt:] = geo.edge_edge(X4[n_pt:, 0], X4[n_pt:, 1], X4[n_pt:, 2], X4[n_pt:, 3])[0]
    return d2


def pair_step_bounds(x, dx, prox, pt, ee, eta=ETA, steps=STEPS):
    """t_k for each candidate pair (point-triangle rows first)."""
    X4 = contact.pair_points(x, prox, pt, ee)
    D4 = contact.pair_points(dx, prox, pt, ee)
    n_pt = len(pt)
    if X4.shape[0] == 0:
        return np.zeros(0)
    d0 = np.sqrt(_pair_d2(X4, n_pt))
    g = eta * d0
    l = motion_bound(D4, n_pt)
    t = np.zeros(X4.shape[0])
    moving = l > 0
    for _ in range(steps):
        Xt = X4 + t[:, None, None] * D4
        dt = np.sqrt(_pair_d2(Xt, n_pt))
        adv = np.where(moving, np.maximum(0.0, dt - g) / np.where(moving, l, 1.0), 1.0)
        t = np.minimum(1.0, t + adv)
    t[~moving] = 1.0
    return t


def step_bound(x, dx, prox, dhat, eta=ETA, steps=STEPS):
    """alpha_m and the swept candidate lists used to get it."""
    pt, ee = contact.candidates(x, x + dx, prox, dhat)
    t = pair_step_bounds(x, dx, prox, pt, ee, eta, steps)
    alpha_m = float(min(1.0, t.min())) if t.size else 1.0
    return alpha_m, pt, ee
