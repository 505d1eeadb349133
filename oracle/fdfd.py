"""FDFD operator of the 2D TM (E_z) problem, assembled as a sparse matrix.

Test infrastructure (oracle): see the package docstring.

Sec. 2, Eq. 1: [curl curl - omega^2 eps(x)/c^2] E = -i omega mu0 J, discretised
on the Yee grid, terminated by perfectly matched layers backed by periodic
boundaries.  For E = E_z(x, y) z-hat, curl curl E = -laplacian E_z, so in
stretched coordinates

    A = -(Dxb Dxf + Dyb Dyf) - omega^2 diag(eps)

with E_z on the integer nodes, forward differences living on half nodes
(i + 1/2), backward differences mapping back to integer nodes, and every
difference divided by the local complex stretch factor s = 1 - i sigma/omega
(time dependence exp(+i omega t), the convention fixed by the sign of the
right-hand side of Eq. 1).

The PML profile is not given in the paper; the reading used here is the common
polynomial grading sigma(d) = sigma_max (d/npml)^m with m = 3, ln R = -16 and
sigma_max = -(m+1) ln R / (2 L), L = npml*dx, where d is the depth into the
layer in cells, evaluated at integer and half-integer positions and clamped to
npml (the periodic link between the last and the first cell sits at depth npml).
Units: c = mu0 = eps0 = 1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

PML_GRADE = 3
PML_LNR = -16.0


def pml_depth(p: np.ndarray, n: int, npml: int) -> np.ndarray:
    """Depth (in cells) of position p (integer or half-integer) into the PML."""
    p = np.asarray(p, dtype=np.float64)
    d = np.maximum(0.0, np.maximum(npml - p, p - (n - 1 - npml)))
    return np.minimum(d, float(npml))


def stretch(n: int, npml: int, dx: float, omega: float,
            grade: int = PML_GRADE, lnR: float = PML_LNR):
    """Stretch factors (s_int, s_half): s_int[i] = s(i), s_half[i] = s(i + 1/2).

    s_half[n-1] belongs to the periodic link from node n-1 to node 0.
    """
    if npml == 0:
        return np.ones(n, dtype=np.complex128), np.ones(n, dtype=np.complex128)
    L = npml * dx
    sigma_max = -(grade + 1) * lnR / (2.0 * L)
    i = np.arange(n, dtype=np.float64)

    def s_at(p):
        sigma = sigma_max * (pml_depth(p, n, npml) / npml) ** grade
        return 1.0 - 1j * sigma / omega

    return s_at(i), s_at(i + 0.5)


def diff_forward(n: int, dx: float, s_half: np.ndarray) -> sp.csr_matrix:
    """(Df y)_i = (y_{i+1} - y_i) / (dx s(i+1/2)), periodic: y_n = y_0."""
    rows = np.arange(n)
    Dp = sp.csr_matrix((np.ones(n), (rows, (rows + 1) % n)), shape=(n, n))
    D = (Dp - sp.identity(n, format="csr")) / dx
    return sp.diags(1.0 / s_half) @ D


def diff_backward(n: int, dx: float, s_int: np.ndarray) -> sp.csr_matrix:
    """(Db g)_i = (g_{i+1/2} - g_{i-1/2}) / (dx s(i)), g_{-1/2} = g_{n-1/2}."""
    rows = np.arange(n)
    Dm = sp.csr_matrix((np.ones(n), (rows, (rows - 1) % n)), shape=(n, n))
    D = (sp.identity(n, format="csr") - Dm) / dx
    return sp.diags(1.0 / s_int) @ D


def assemble(eps: np.ndarray, omega: float, dx: float, npml: int,
             npml_y: int | None = None) -> sp.csr_matrix:
    """Sparse complex128 FDFD matrix A for permittivity eps[ny, nx] (x fastest).
    npml_y (default npml) sets the layer thickness on the y axis separately."""
    eps = np.asarray(eps, dtype=np.float64)
    ny, nx = eps.shape
    sxi, sxh = stretch(nx, npml, dx, omega)
    syi, syh = stretch(ny, npml if npml_y is None else npml_y, dx, omega)
    Lx = diff_backward(nx, dx, sxi) @ diff_forward(nx, dx, sxh)
    Ly = diff_backward(ny, dx, syi) @ diff_forward(ny, dx, syh)
    lap = sp.kron(sp.identity(ny), Lx) + sp.kron(Ly, sp.identity(nx))
    A = -lap - (omega ** 2) * sp.diags(eps.reshape(-1))
    return sp.csr_matrix(A, dtype=np.complex128)


def assemble_instance(inst) -> sp.csr_matrix:
    return assemble(inst.eps, inst.omega, inst.dx, inst.npml)


def symmetrizer(nx: int, ny: int, omega: float, dx: float, npml: int) -> np.ndarray:
    """diag(s_x(i) s_y(j)) as a flat vector: this diagonal scaling makes A
    complex symmetric (a property of the stretched-coordinate discretisation)."""
    sxi, _ = stretch(nx, npml, dx, omega)
    syi, _ = stretch(ny, npml, dx, omega)
    return (syi[:, None] * sxi[None, :]).reshape(-1)
