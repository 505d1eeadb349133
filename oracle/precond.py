"""Diagonal preconditioners of the supplement's comparison (Table 1).

Test infrastructure (oracle): see the package docstring.

The supplement writes a preconditioned system as A' = P_L A P_R, b' = P_L b,
f' = P_R^{-1} f, and studies data-free preconditioners.  The two diagonal ones
are built here.
  * Jacobi: P_L = D(A)^{-1} (the inverse diagonal of A), P_R = I.
  * The grid-spacing preconditioner of the paper's Ref. 17.  The paper only says
    that P_L and P_R are diagonal matrices built from the grid spacing,
    including the complex PML stretching.  The reading used here is
    P_L = S^{1/2}, P_R = S^{-1/2}, with S = diag(s_x(i) s_y(j)) the diagonal
    that makes S A complex symmetric (fdfd.symmetrizer).  A' is then complex
    symmetric and has the spectrum of A.
Augmented GMRES on the preconditioned system takes V' = P_R^{-1} V, so that the
augmenting space in f is span(V) itself.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fdfd, gmres_aug


def jacobi(A):
    """(pl, pr) of the Jacobi preconditioner."""
    d = np.asarray(A.diagonal(), np.complex128)
    return 1.0 / d, np.ones_like(d)


def pml_scaling(nx: int, ny: int, omega: float, dx: float, npml: int):
    """(pl, pr) of the PML grid-spacing scaling: S^{1/2} and S^{-1/2}."""
    s = np.sqrt(fdfd.symmetrizer(nx, ny, omega, dx, npml))   # principal root, Re s > 0
    return s, 1.0 / s


def preconditioned(A, pl, pr):
    return sp.csr_matrix(sp.diags(pl) @ A @ sp.diags(pr))


def gmres_aug_precond(A, b, V, pl, pr, **kw):
    """Augmented GMRES on A' = P_L A P_R (gmres_aug); returns f = P_R f' and the
    info of the preconditioned solve (history relative to ||P_L b||)."""
    b = np.asarray(b, np.complex128)
    Vp = np.asarray(V, np.complex128).reshape(len(b), -1) / pr[:, None]
    fp, info = gmres_aug.gmres_aug(preconditioned(A, pl, pr), pl * b, Vp, **kw)
    return pr * fp, info
