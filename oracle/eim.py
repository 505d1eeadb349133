"""Effective-index approximation of the field: the CNN's second input.

Test infrastructure (oracle): see the package docstring.

The paper gives its CNN an effective-index simulation of the field next to the
permittivity (Sec. 3, data-set and CNN paragraphs, and the CNN figure).  This is
a cheap approximation that amounts to solving Maxwell's equations in one
dimension.  The paper gives no formulas.  The reading used here is the
separable (effective-index) ansatz on the FDFD grid of Eq. 1.

  * Every column ix of the permittivity is a 1D slab.  Its fundamental mode
    phi_ix is the eigenvector of the lowest eigenvalue mu_ix of the real
    symmetric operator
        T_ix = -(second difference in y) / dx^2 - omega^2 eps(ix, .),
    with zero field outside the column ends.  mu = -beta^2, where beta is the
    local propagation constant, so n_eff = beta / omega.  (The workloads'
    mode source is built from the same operator.)
  * The amplitude along x obeys the 1D FDFD equation, with the same stretched
    x-differences and periodic wrap as the 2D operator and mu in place of
    -omega^2 eps:
        (-Dxb Dxf + diag(mu)) a = j,    where j_ix = phi_ix^T b[:, ix].
  * The approximate field is F[iy, ix] = a_ix phi_ix(iy).

Normalisation of phi_ix:
  * phi_ix has unit 2-norm.
  * phi_ix is positive.  The lowest eigenvector of an unreduced tridiagonal
    matrix with negative off-diagonals has no sign change, so this fixes it.
  * The lowest eigenvalue of such a matrix is simple, so phi_ix is unique.

When F is exact: if eps(ix, iy) = e_x(ix) + e_y(iy) and the source has the form
j(x) phi(y), then F is the exact discrete solution of the 2D problem without a
y-PML (the field must have decayed at the column ends).  In that case the 2D
operator is the Kronecker sum of the x and y operators.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fdfd


def column_modes(eps, omega: float, dx: float):
    """Lowest eigenpair of T_ix for every column.

    eps has shape [ny, nx].  Returns mu with shape [nx] and phi with shape
    [ny, nx]; each column of phi has unit norm and is positive.
    """
    eps = np.asarray(eps, np.float64)
    ny, nx = eps.shape
    mu = np.empty(nx)
    phi = np.empty((ny, nx))
    off = np.full(ny - 1, -1.0 / dx ** 2)
    for ix in range(nx):
        d = 2.0 / dx ** 2 - omega ** 2 * eps[:, ix]
        w, v = sla.eigh_tridiagonal(d, off, select="i", select_range=(0, 0))
        u = v[:, 0]
        mu[ix] = w[0]
        phi[:, ix] = u * np.sign(u.sum()) / np.linalg.norm(u)
    return mu, phi


def line_operator(mu, omega: float, dx: float, npml: int) -> sp.csc_matrix:
    """The 1D operator -Dxb Dxf + diag(mu): the 2D operator's x part (stretch
    factors, periodic wrap) with the effective permittivity term."""
    nx = len(mu)
    sxi, sxh = fdfd.stretch(nx, npml, dx, omega)
    L = fdfd.diff_backward(nx, dx, sxi) @ fdfd.diff_forward(nx, dx, sxh)
    return sp.csc_matrix(-L + sp.diags(np.asarray(mu, np.float64)), dtype=np.complex128)


def eim_field(eps, b, omega: float, dx: float, npml: int) -> np.ndarray:
    """Effective-index field F (complex128, flat [ny*nx], x fastest)."""
    eps = np.asarray(eps, np.float64)
    ny, nx = eps.shape
    mu, phi = column_modes(eps, omega, dx)
    j = (phi * np.asarray(b, np.complex128).reshape(ny, nx)).sum(axis=0)
    a = spla.spsolve(line_operator(mu, omega, dx, npml), j)
    return (phi * a[None, :]).reshape(-1)


def eim_instance(inst) -> np.ndarray:
    return eim_field(inst.eps, inst.b, inst.omega, inst.dx, inst.npml)
