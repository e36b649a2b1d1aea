"""Algorithm 1 ("PD Solver with IPC Contact") with a plain sparse-direct
global step.

Oracle module (test infrastructure only).

Every iteration assembles H_hat = H + PositiveDefinite(Hess B) on the free DOFs
and solves Eq. (4), H_hat dx = -g_hat, with a fresh sparse LU (SuperLU via
scipy).  This is the plain definition that the paper's Schur-complement and
Woodbury steps (Eq. 6-11) reach exactly; none of those steps appear here.

Readings:
* the line search and the update use the current iterate x (the printed
  algorithm writes x_t there, which could never move past one step);
* "back-traced line search" = start at alpha_m, accept when the total energy
  does not increase (sum of per-element and per-pair differences <= 0),
  otherwise halve, at most 20 halvings, then alpha = 0 with a warning;
* barrier energies in the line search run over the swept candidate pairs, so
  pairs entering the threshold along the step are counted;
* "while not converged" = a fixed number of iterations, or, in tolerance
  mode, until max |alpha dx| <= tol;
* fixed (Dirichlet) vertices stay at their rest positions and carry no DOFs;
* an embedded proxy (Section 3.1): with a matrix W (n_s x n, rows summing to
  1) the collision primitives live on s = W x -- distances, constraint set,
  candidates, step bound and barrier energies use s, the barrier gradient is
  W^T grad_s and the projected Hessian W^T H_s W (over 3 DOFs per vertex);
  without W the proxy is a selection of simulation vertices;
* adaptive barrier stiffness (optional; the paper says only that IPC
  initialises kappa from the average stiffness and adjusts it adaptively): at
  the start of a frame, if the constraint set at x_t is not empty, kappa is the
  value that best balances the elastic and barrier gradients,
  argmin_k |g_E + k g_b|^2 = -(g_E . g_b) / (g_b . g_b) over the free DOFs
  (g_E the PD gradient, g_b the gradient of sum_k b(d_k)), clamped to
  [kappa_0, 100 kappa_0]; else kappa_0.  At each later iteration, when the
  smallest squared distance of the constraint set falls below 1e-9 l^2 (l the
  rest bounding-box diagonal) and below its value at the previous iteration,
  kappa doubles, up to 100 kappa_0.  Every frame starts again from kappa_0.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, local, contact, barrier, ccd


@dataclass
class Problem:
    X: np.ndarray
    tets: np.ndarray
    dirichlet: np.ndarray
    prox: contact.Proxy
    B: np.ndarray
    V: np.ndarray
    w: np.ndarray
    G: np.ndarray
    H: sp.csc_matrix
    free: np.ndarray
    dhat: float
    kappa: float
    barrier_form: int = 0
    kappa_adapt: bool = False
    W: sp.csr_matrix | None = None     # proxy embedding s = W x (None: selection)

    @property
    def n(self):
        return self.X.shape[0]


def setup(X, tets, dirichlet, surf_tris, youngs, poisson, dhat, kappa, barrier_form=0,
          kappa_adapt=False, W=None) -> Problem:
    """W: None (proxy triangles index simulation vertices) or (rowptr, col,
    val) of s = W x (proxy triangles index rows of W)."""
    X = np.asarray(X, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    _, B, V = fem.rest_data(X, tets)
    w = fem.weights(V, youngs, poisson)
    G = fem.gradient_operators(B)
    H = fem.assemble_H(X.shape[0], tets, G, w)
    free = fem.free_dofs(dirichlet)
    return Problem(X=X, tets=tets, dirichlet=np.asarray(dirichlet), prox=contact.make_proxy(surf_tris),
                   B=B, V=V, w=w, G=G, H=H, free=free, dhat=float(dhat), kappa=float(kappa),
                   barrier_form=int(barrier_form), kappa_adapt=bool(kappa_adapt), W=_embedding(W, X.shape[0]))


def _embedding(W, n):
    if W is None:
        return None
    rowptr, col, val = W
    return sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col), np.asarray(rowptr)),
                         shape=(len(rowptr) - 1, n))


def setup_scene(scene, barrier_form=0, kappa_adapt=False) -> Problem:
    return setup(scene.X, scene.tets, scene.dirichlet, scene.surf_tris, scene.youngs,
                 scene.poisson, scene.dhat, scene.kappa, barrier_form, kappa_adapt, getattr(scene, "W", None))


def proxy_positions(prob: Problem, x: np.ndarray) -> np.ndarray:
    """Positions of the proxy vertices: s = W x, or x itself for a selection."""
    return x if prob.W is None else prob.W @ x


def _to_sim(prob: Problem, g_s: np.ndarray, B_s: sp.spmatrix):
    """Gradient and Hessian from proxy DOFs to simulation DOFs: W^T g, W^T B W
    (with W acting on three coordinates per vertex)."""
    if prob.W is None:
        return g_s, B_s
    W3 = sp.kron(prob.W, sp.identity(3), format="csr")
    return W3.T @ g_s, (W3.T @ B_s @ W3).tocsc()


def pd_gradient(prob: Problem, F: np.ndarray, P: np.ndarray) -> np.ndarray:
    """sum_i w_i G_i^T (G_i x - p_i) over all 3n DOFs."""
    r = (F - P).reshape(-1, 9)
    ge = prob.w[:, None] * np.einsum("mki,mk->mi", prob.G, r)
    g = np.zeros(3 * prob.n)
    np.add.at(g, fem.local_dofs(prob.tets).reshape(-1), ge.reshape(-1))
    return g


def pair_dofs(prob: Problem, cs: contact.ConstraintSet) -> np.ndarray:
    V4 = contact.pair_vertices(prob.prox, cs.pt, cs.ee)
    return (3 * V4[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)


def barrier_terms(prob: Problem, x: np.ndarray, cs: contact.ConstraintSet, kappa: float | None = None):
    """(energy, gradient (3n), PSD-projected Hessian (sparse 3n x 3n), raw pieces)."""
    kappa = prob.kappa if kappa is None else kappa
    n3 = 3 * prob.n
    if cs.size == 0:
        return 0.0, np.zeros(n3), sp.csc_matrix((n3, n3)), (np.zeros(0), np.zeros((0, 12)), np.zeros((0, 12, 12)))
    s = proxy_positions(prob, x)
    X4 = contact.pair_points(s, prob.prox, cs.pt, cs.ee)
    E, Gp, Hp = barrier.pair_derivatives(X4, cs.kind, cs.idx, prob.dhat, kappa, prob.barrier_form)
    Hp = barrier.project_psd(Hp)
    dofs = pair_dofs(prob, cs)
    ns3 = 3 * s.shape[0]
    g = np.zeros(ns3)
    np.add.at(g, dofs.reshape(-1), Gp.reshape(-1))
    rows = np.repeat(dofs, 12, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, 12)).reshape(-1)
    Bm = sp.csc_matrix((Hp.reshape(-1), (rows, cols)), shape=(ns3, ns3))
    g, Bm = _to_sim(prob, g, Bm)
    return float(E.sum()), g, Bm, (E, Gp, Hp)


def total_energy_terms(prob: Problem, x, A, pt, ee, kappa: float | None = None):
    """Per-element PD energies and per-candidate barrier energies at x."""
    kappa = prob.kappa if kappa is None else kappa
    F = local.deformation_gradients(x, prob.tets, prob.B)
    Ee = local.element_energies(F, A, prob.w)
    d2, _, _ = contact.pair_distances(proxy_positions(prob, x), prob.prox, pt, ee)
    Eb = kappa * barrier.barrier(np.sqrt(d2), prob.dhat, prob.barrier_form)
    return Ee, Eb


def line_search(prob: Problem, x, dx, A, alpha_m, pt, ee, max_halvings=20, kappa: float | None = None):
    """Back-tracking from alpha_m on the energy difference; returns (alpha, halvings, ok)."""
    Ee0, Eb0 = total_energy_terms(prob, x, A, pt, ee, kappa)
    alpha = alpha_m
    for h in range(max_halvings + 1):
        Ee1, Eb1 = total_energy_terms(prob, x + alpha * dx, A, pt, ee, kappa)
        dE = np.sum(Ee1 - Ee0) + np.sum(Eb1 - Eb0)
        if dE <= 0:
            return alpha, h, True
        alpha *= 0.5
    return 0.0, max_halvings + 1, False


@dataclass
class IterRecord:
    x: np.ndarray
    R: np.ndarray
    P: np.ndarray
    cs: contact.ConstraintSet
    pair_E: np.ndarray
    pair_g: np.ndarray
    pair_H: np.ndarray
    g: np.ndarray
    dx: np.ndarray
    alpha_m: float
    alpha: float
    halvings: int
    swept_pt: np.ndarray
    swept_ee: np.ndarray
    kappa: float = 0.0


@dataclass
class FrameResult:
    x: np.ndarray
    iters: int
    alpha_m: list = field(default_factory=list)
    alpha: list = field(default_factory=list)
    n_pt: list = field(default_factory=list)
    n_ee: list = field(default_factory=list)
    n_c: list = field(default_factory=list)
    ls_failed: int = 0
    trace: list = field(default_factory=list)
    kappa: list = field(default_factory=list)


def affected_vertices(prob: Problem, cs: contact.ConstraintSet) -> np.ndarray:
    """Free simulation vertices touched by an active pair (sorted)."""
    if cs.size == 0:
        return np.zeros(0, np.int64)
    V4 = contact.pair_vertices(prob.prox, cs.pt, cs.ee)
    v = np.unique(V4.reshape(-1))
    if prob.W is not None:
        v = np.unique(prob.W[v].indices)
    return v[prob.dirichlet[v] == 0]


def balanced_kappa(prob: Problem, x: np.ndarray, A: np.ndarray, cs: contact.ConstraintSet) -> float:
    """argmin_k |g_E + k g_b|^2 over the free DOFs (g_b: the gradient of the
    unit-stiffness barrier), clamped to [kappa_0, 100 kappa_0]; kappa_0 with no
    pair."""
    if cs.size == 0:
        return prob.kappa
    F = local.deformation_gradients(x, prob.tets, prob.B)
    _, P = local.projections(F, A)
    gE = pd_gradient(prob, F, P)[prob.free]
    gb = barrier_terms(prob, x, cs, kappa=1.0)[1][prob.free]
    bb = float(gb @ gb)
    k = -float(gE @ gb) / bb if bb > 0 else prob.kappa
    return min(max(k, prob.kappa), 100.0 * prob.kappa)


def iteration(prob: Problem, x: np.ndarray, A: np.ndarray, max_halvings=20, kappa: float | None = None):
    """One pass of the Algorithm 1 loop body. Returns (x_new, IterRecord)."""
    kappa = prob.kappa if kappa is None else kappa
    F = local.deformation_gradients(x, prob.tets, prob.B)
    R, P = local.projections(F, A)
    cs = contact.constraint_set(proxy_positions(prob, x), prob.prox, prob.dhat)
    if cs.size and np.any(cs.d2 <= 0):
        raise ValueError("state is not intersection-free")
    _, gB, Bm, (pE, pg, pH) = barrier_terms(prob, x, cs, kappa)
    g = pd_gradient(prob, F, P) + gB
    f = prob.free
    K = (prob.H + Bm).tocsc()[f][:, f]
    dxf = -spla.splu(K.tocsc()).solve(g[f])
    dx = np.zeros(3 * prob.n)
    dx[f] = dxf
    dx = dx.reshape(-1, 3)
    alpha_m, spt, see = ccd.step_bound(proxy_positions(prob, x), proxy_positions(prob, dx), prob.prox, prob.dhat)
    alpha, h, ok = line_search(prob, x, dx, A, alpha_m, spt, see, max_halvings, kappa)
    rec = IterRecord(x=x.copy(), R=R, P=P, cs=cs, pair_E=pE, pair_g=pg, pair_H=pH,
                     g=g, dx=dx, alpha_m=alpha_m, alpha=alpha, halvings=h,
                     swept_pt=spt, swept_ee=see, kappa=kappa)
    return x + alpha * dx, rec, ok


def frame(prob: Problem, x_t: np.ndarray, A: np.ndarray, iters: int = 30, tol: float | None = None,
          max_iters: int = 500, trace: bool = False, max_halvings=20) -> FrameResult:
    """x_{t+1} from x_t for the actuation A (m, 3, 3)."""
    x = np.array(x_t, dtype=np.float64, copy=True)
    res = FrameResult(x=x, iters=0)
    n_it = max_iters if tol is not None else iters
    kappa = prob.kappa
    eps_d2 = 1e-9 * float(np.sum((prob.X.max(0) - prob.X.min(0)) ** 2))
    d2_prev = np.inf
    for k in range(n_it):
        if prob.kappa_adapt:
            cs = contact.constraint_set(proxy_positions(prob, x), prob.prox, prob.dhat)
            d2_min = float(cs.d2.min()) if cs.size else np.inf
            if k == 0:
                kappa = balanced_kappa(prob, x, A, cs)
            elif d2_min < eps_d2 and d2_min < d2_prev:
                kappa = min(2.0 * kappa, 100.0 * prob.kappa)
            d2_prev = d2_min
        res.kappa.append(kappa)
        x_new, rec, ok = iteration(prob, x, A, max_halvings, kappa)
        res.alpha_m.append(rec.alpha_m)
        res.alpha.append(rec.alpha)
        res.n_pt.append(len(rec.cs.pt))
        res.n_ee.append(len(rec.cs.ee))
        res.n_c.append(len(affected_vertices(prob, rec.cs)))
        res.ls_failed += 0 if ok else 1
        if trace:
            res.trace.append(rec)
        step = float(np.max(np.abs(x_new - x))) if x.size else 0.0
        x = x_new
        res.iters = k + 1
        if tol is not None and step <= tol:
            break
    res.x = x
    return res


def actuation(scene_or_R, a) -> np.ndarray:
    R = scene_or_R.act_R if hasattr(scene_or_R, "act_R") else scene_or_R
    return fem.actuation_matrices(a, R)
