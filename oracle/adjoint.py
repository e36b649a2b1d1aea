"""Adjoint of a converged frame with respect to per-tet actuation scalars.

Oracle module (test infrastructure only).

At an equilibrium x*(a) the energy gradient g(x*, a) = 0, hence
dL/da = -lambda^T dg/da with K lambda = dL/dx and K = Hess_x E_hat(x*), the
true Hessian (no positive-definite projection).  Both K and dg/da are taken
by automatic differentiation of the per-element energy written in closed form,
(w/2)(||F||^2 + ||A||^2 - 2(s1 + s2 + sign(det FA) s3)) with s the singular
values of F A (Eq. 1 minimised over the rotation), and of the barrier energy
of Eq. (3); the system is solved by a sparse LU.

A(a) = R0 diag(1 - a, 1 + a/2, 1 + a/2) R0^T (the actuation parametrisation).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch
from torch.func import hessian, jacfwd, jacrev, vmap

from . import barrier, contact, fem, local


def _elem_energy(x12, a, Bm, R0, w, sgn):
    X = x12.reshape(4, 3)
    Ds = torch.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], dim=1)
    F = Ds @ Bm
    d = torch.stack([1.0 - a, 1.0 + 0.5 * a, 1.0 + 0.5 * a])
    A = R0 @ torch.diag(d) @ R0.T
    s = torch.linalg.svdvals(F @ A)
    return 0.5 * w * (torch.sum(F * F) + torch.sum(A * A) - 2.0 * (s[0] + s[1] + sgn * s[2]))


def element_derivatives(prob, x, a, R0):
    """Per tet: K_i (12 x 12) and dg_i/da_i (12) of the PD energy."""
    T = prob.tets
    X12 = torch.from_numpy(np.ascontiguousarray(x[T].reshape(-1, 12)))
    at = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
    Bt = torch.from_numpy(np.ascontiguousarray(prob.B))
    Rt = torch.from_numpy(np.ascontiguousarray(R0))
    wt = torch.from_numpy(np.ascontiguousarray(prob.w))
    F = local.deformation_gradients(x, prob.tets, prob.B)
    A = fem.actuation_matrices(a, R0)
    sg = np.sign(np.linalg.det(F @ A))
    sg[sg == 0] = 1.0
    st = torch.from_numpy(sg)
    H = vmap(hessian(_elem_energy, argnums=0))(X12, at, Bt, Rt, wt, st)
    gx = jacrev(_elem_energy, argnums=0)
    Ga = vmap(jacfwd(gx, argnums=1))(X12, at, Bt, Rt, wt, st)
    return H.numpy(), Ga.numpy()


def energy_hessian(prob, x, a, R0):
    """Sparse true Hessian of the total energy (PD + raw barrier) over 3n DOFs."""
    n3 = 3 * prob.n
    H, _ = element_derivatives(prob, x, a, R0)
    dofs = fem.local_dofs(prob.tets)
    rows = [np.repeat(dofs, 12, axis=1).reshape(-1)]
    cols = [np.tile(dofs, (1, 12)).reshape(-1)]
    vals = [H.reshape(-1)]
    cs = contact.constraint_set(x, prob.prox, prob.dhat)
    if cs.size:
        X4 = contact.pair_points(x, prob.prox, cs.pt, cs.ee)
        _, _, Hp = barrier.pair_derivatives(X4, cs.kind, cs.idx, prob.dhat, prob.kappa, prob.barrier_form)
        V4 = contact.pair_vertices(prob.prox, cs.pt, cs.ee)
        pd = (3 * V4[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
        rows.append(np.repeat(pd, 12, axis=1).reshape(-1))
        cols.append(np.tile(pd, (1, 12)).reshape(-1))
        vals.append(Hp.reshape(-1))
    return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n3, n3))


def actuation_gradient(prob, x_star, a, R0, dLdx):
    """dL/da (m,) for a loss with gradient dLdx (n, 3) at the equilibrium x_star."""
    K = energy_hessian(prob, x_star, a, R0)
    f = prob.free
    b = np.asarray(dLdx, dtype=np.float64).reshape(-1)
    lam = np.zeros(3 * prob.n)
    lam[f] = spla.splu(K[f][:, f].tocsc()).solve(b[f])
    _, Ga = element_derivatives(prob, x_star, a, R0)
    lam_local = lam[fem.local_dofs(prob.tets)]
    return -np.einsum("mi,mi->m", Ga, lam_local)
