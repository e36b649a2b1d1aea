"""Local step of projective dynamics (Eq. 1, Section 2.1).

Oracle module (test infrastructure only).

For each element, R_i = argmin over SO(3) of ||F_i - R A_i||_F.  Because A_i
is symmetric, ||F - R A||^2 = ||F||^2 + ||A||^2 - 2 tr(R^T F A), so R_i is the
rotation nearest to M = F A: with M = U S V^T, R = U diag(1, 1, det(U V^T)) V^T.
The element energy used by the line search is (w_i / 2) ||F_i - R_i A_i||^2.
"""
from __future__ import annotations

import numpy as np


def deformation_gradients(x: np.ndarray, tets: np.ndarray, B: np.ndarray) -> np.ndarray:
    """F_i = D_s(x) B_i with D_s = [x1-x0, x2-x0, x3-x0] (columns)."""
    T = np.asarray(tets, dtype=np.int64)
    Ds = np.stack([x[T[:, 1]] - x[T[:, 0]], x[T[:, 2]] - x[T[:, 0]],
                   x[T[:, 3]] - x[T[:, 0]]], axis=2)
    return Ds @ B


def best_rotations(F: np.ndarray, A: np.ndarray) -> np.ndarray:
    """R_i in SO(3) maximising tr(R^T F_i A_i), via numpy's SVD."""
    M = F @ A
    U, _, Vt = np.linalg.svd(M)
    s = np.sign(np.linalg.det(U @ Vt))
    s[s == 0] = 1.0
    D = np.ones((F.shape[0], 3))
    D[:, 2] = s
    return (U * D[:, None, :]) @ Vt


def projections(F: np.ndarray, A: np.ndarray):
    """(R_i, P_i = R_i A_i) for every element."""
    R = best_rotations(F, A)
    return R, R @ A


def element_energies(F: np.ndarray, A: np.ndarray, w: np.ndarray) -> np.ndarray:
    """(w_i / 2) min_R ||F_i - R A_i||_F^2, evaluated directly at the minimiser."""
    _, P = projections(F, A)
    return 0.5 * w * np.sum((F - P) ** 2, axis=(1, 2))
