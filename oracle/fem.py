"""Finite-element set-up of the shape-targeting energy (Eq. 1, Eq. 2).

Oracle module (test infrastructure only).

Readings (the paper gives no material constants):
* weight ``w_i = 2 * mu * V_i`` with ``mu = E / (2 (1 + nu))`` -- the paper
  weights each element by its rest volume (Section 2.1); the factor 2 mu turns
  the dimensionless Eq. (1) into the corotational-like stiffness of the
  configured Young's modulus.  Poisson's ratio enters only through mu.
* vec(F) is row-major: entry (r, c) of F sits at 3 r + c.
* per-tet local DOFs are (x_0, x_1, x_2, x_3), three coordinates each.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def rest_data(X: np.ndarray, tets: np.ndarray):
    """Per tet: D_m = [X1-X0, X2-X0, X3-X0], B = D_m^-1, V = det(D_m)/6.

    Raises ValueError for a tet with non-positive rest volume.
    """
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(tets, dtype=np.int64)
    Dm = np.stack([X[T[:, 1]] - X[T[:, 0]], X[T[:, 2]] - X[T[:, 0]],
                   X[T[:, 3]] - X[T[:, 0]]], axis=2)          # columns are edges
    det = np.linalg.det(Dm)
    if np.any(det <= 0):
        raise ValueError(f"{int(np.sum(det <= 0))} tets with non-positive rest volume")
    B = np.linalg.inv(Dm)
    return Dm, B, det / 6.0


def weights(V: np.ndarray, youngs: float, poisson: float) -> np.ndarray:
    mu = youngs / (2.0 * (1.0 + poisson))
    return 2.0 * mu * V


def gradient_operators(B: np.ndarray) -> np.ndarray:
    """G_i (9 x 12) with vec(F_i) = G_i x_local, F = D_s B (D_s from current x).

    F[r, c] = sum_k (x_{k+1} - x_0)[r] B[k, c], so dF[r, c]/dx_a[r] equals
    B[a-1, c] for a >= 1 and -sum_k B[k, c] for a = 0.
    """
    m = B.shape[0]
    g = np.empty((m, 4, 3))
    g[:, 1:, :] = B
    g[:, 0, :] = -B.sum(axis=1)
    G = np.zeros((m, 9, 12))
    for r in range(3):
        for c in range(3):
            for a in range(4):
                G[:, 3 * r + c, 3 * a + r] = g[:, a, c]
    return G


def local_dofs(tets: np.ndarray) -> np.ndarray:
    """(m, 12) global DOF index of each local DOF: 3 * vertex + coordinate."""
    T = np.asarray(tets, dtype=np.int64)
    return (3 * T[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)


def assemble_H(n: int, tets: np.ndarray, G: np.ndarray, w: np.ndarray) -> sp.csc_matrix:
    """H = sum_i w_i G_i^T G_i over all 3n DOFs (Eq. 2), as sparse CSC."""
    Ke = w[:, None, None] * np.einsum("mki,mkj->mij", G, G)
    dofs = local_dofs(tets)
    rows = np.repeat(dofs, 12, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, 12)).reshape(-1)
    return sp.csc_matrix((Ke.reshape(-1), (rows, cols)), shape=(3 * n, 3 * n))


def actuation_matrices(a: np.ndarray, R: np.ndarray) -> np.ndarray:
    """A_i = R_i diag(1 - a_i, 1 + a_i/2, 1 + a_i/2) R_i^T (symmetric)."""
    a = np.asarray(a, dtype=np.float64)
    d = np.stack([1.0 - a, 1.0 + 0.5 * a, 1.0 + 0.5 * a], axis=1)
    return np.einsum("mij,mj,mkj->mik", R, d, R)


def actuation_derivative(R: np.ndarray) -> np.ndarray:
    """dA_i/da_i = R_i diag(-1, 1/2, 1/2) R_i^T (independent of a_i)."""
    d = np.array([-1.0, 0.5, 0.5])
    return np.einsum("mij,j,mkj->mik", R, d, R)


def free_dofs(dirichlet: np.ndarray) -> np.ndarray:
    """Sorted global DOF indices of the non-fixed vertices."""
    free_v = np.nonzero(np.asarray(dirichlet) == 0)[0]
    return (3 * free_v[:, None] + np.arange(3)[None, :]).reshape(-1)
