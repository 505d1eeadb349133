"""Principal-component basis of simulated fields (Sec. 3, PCA paragraph).

Test infrastructure (oracle): see the package docstring.

The basis is the leading left singular vectors of the matrix whose columns are
the field vectors of the training set (uncentred, no per-sample scaling),
obtained here from a full numpy SVD of that matrix.
"""
from __future__ import annotations

import numpy as np


def pca_basis(S, k):
    """S: D x M snapshot matrix; returns (U_k [D x k], singular values [k])."""
    U, s, _ = np.linalg.svd(np.asarray(S, np.complex128), full_matrices=False)
    return U[:, :k], s[:k]


def principal_angles(U1, U2):
    """Principal angles (radians) between span(U1) and span(U2)."""
    Q1, _ = np.linalg.qr(U1)
    Q2, _ = np.linalg.qr(U2)
    s = np.linalg.svd(Q1.conj().T @ Q2, compute_uv=False)
    return np.arccos(np.clip(s, -1.0, 1.0))
