"""Spectral facts of the TE operator and the dense-eigenvector deflation.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

from __future__ import annotations

import numpy as np


def homogeneous_map(lam, eps):
    """Eigenvalue of A_R A from the eigenvalue lam of A for a homogeneous object.

    Section 5, eq. EigenvaluesArA: lam' = [1 + (eps_b/eps)(1 - lam)] lam (eps_b = 1).
    """
    lam = np.asarray(lam, dtype=np.complex128)
    return (1.0 + (1.0 - lam) / eps) * lam


def lossless_segment_image(eps: float) -> tuple[float, float]:
    """Image of the real segment [1, eps] under the homogeneous map for a lossless object.

    Section 5 (deflation-bound discussion): [1, eps] maps to
    [1, 1 + (1 - eps)^2 / (4 eps)].
    """
    return 1.0, 1.0 + (1.0 - eps) ** 2 / (4.0 * eps)


def segment_distance_to_origin(a: complex, b: complex) -> float:
    """Euclidean distance from 0 to the straight segment [a, b] of the complex plane."""
    d = b - a
    t = 0.0 if d == 0 else float(np.clip(-(np.conj(d) * a).real / abs(d) ** 2, 0.0, 1.0))
    return abs(a + t * d)


def essential_segment(eps: complex) -> tuple[complex, complex]:
    """Discrete image of the essential spectrum for a homogeneous object: [1, eps/eps_b]
    (Section 3, eq. EssentialSpectrum; Section 4, the dense line segments)."""
    return 1.0 + 0j, complex(eps)


def modified_gram_schmidt(W: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the columns of W by modified Gram-Schmidt (Section 4)."""
    V = np.array(W, dtype=np.complex128)
    for j in range(V.shape[1]):
        for i in range(j):
            V[:, j] -= (V[:, i].conj() @ V[:, j]) * V[:, i]
        V[:, j] /= np.linalg.norm(V[:, j])
    return V


def largest_eigvecs(M: np.ndarray, r: int):
    """The r eigenpairs of largest magnitude of the dense matrix M (all-eigenvalue solve)."""
    lam, X = np.linalg.eig(M)
    idx = np.argsort(-np.abs(lam), kind="stable")[:r]
    return lam[idx], X[:, idx]


def deflation_preconditioner(M: np.ndarray, V: np.ndarray) -> np.ndarray:
    """P^{-1} = I + V (T^{-1} - I_r) V^*, T = V^* M V (Section 4, eq. DeflatingPrecondtioner).

    V must have orthonormal columns.  Returned densely.
    """
    r = V.shape[1]
    T = V.conj().T @ M @ V
    C = np.linalg.inv(T) - np.eye(r)
    return np.eye(M.shape[0], dtype=np.complex128) + V @ C @ V.conj().T


def deflation_terms(M: np.ndarray, V: np.ndarray) -> np.ndarray:
    """C = T^{-1} - I_r with T = V^* M V: the r x r core of the deflating preconditioner."""
    T = V.conj().T @ M @ V
    return np.linalg.inv(T) - np.eye(V.shape[1])


def apply_deflation(V: np.ndarray, C: np.ndarray, x: np.ndarray) -> np.ndarray:
    """P^{-1} x = x + V (C (V^* x)) for one or more columns x."""
    return x + V @ (C @ (V.conj().T @ x))
