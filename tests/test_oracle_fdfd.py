"""Pins of the oracle's FDFD operator (Sec. 2, Eq. 1) against facts fixed by the
mathematics, not by the oracle's own formula:

* plane waves are eigenvectors of the periodic homogeneous operator with the
  discrete-Laplacian eigenvalue (4/dx^2)(sin^2(kx dx/2) + sin^2(ky dx/2));
* with a line current in a homogeneous medium the interior field is the
  outgoing discrete Green's function -omega J dx^2/(2 sin theta) e^{-i theta|n-n0|},
  theta = 2 arcsin(omega sqrt(eps) dx / 2), up to the PML reflection -- this fixes
  the sign convention (exp(+i omega t)), the dispersion and that the layer absorbs;
* diag(s_x(i) s_y(j)) A is complex symmetric (the stretched-coordinate
  discretisation's symmetriser), which pins the half-node indexing;
* the direct solve satisfies A x = b.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import direct, fdfd


@pytest.mark.parametrize("nx,ny,px,py", [(16, 12, 1, 2), (9, 7, 4, 0), (20, 20, 0, 0), (5, 11, 2, 5)])
def test_plane_wave_eigenvector(nx, ny, px, py):
    dx, omega, eps_r = 0.05, 3.3, 4.0
    A = fdfd.assemble(np.full((ny, nx), eps_r), omega, dx, 0)
    kx, ky = 2 * math.pi * px / (nx * dx), 2 * math.pi * py / (ny * dx)
    X, Y = np.meshgrid(np.arange(nx) * dx, np.arange(ny) * dx)
    f = np.exp(1j * (kx * X + ky * Y)).reshape(-1)
    lam = (4 / dx ** 2) * (math.sin(kx * dx / 2) ** 2 + math.sin(ky * dx / 2) ** 2) - omega ** 2 * eps_r
    np.testing.assert_allclose(A @ f, lam * f, atol=1e-10 * (4 / dx ** 2))


@pytest.mark.parametrize("npml,bound", [(10, 1e-3), (20, 1e-4)])
@pytest.mark.parametrize("eps_r", [2.085, 12.25])
def test_line_source_green_function(npml, bound, eps_r):
    nx, ny, dx, lam = 240, 4, 0.04, 1.55
    om = 2 * math.pi / lam
    A = fdfd.assemble(np.full((ny, nx), eps_r), om, dx, npml, npml_y=0)
    n0 = 120
    J = np.zeros((ny, nx))
    J[:, n0] = 1.0
    u = direct.sparse_solve(A, W.rhs_from_current(J, om)).reshape(ny, nx)
    th = 2 * math.asin(om * math.sqrt(eps_r) * dx / 2)
    n = np.arange(nx)
    ua = -om * dx ** 2 / (2 * math.sin(th)) * np.exp(-1j * th * np.abs(n - n0))
    interior = slice(npml + 1, nx - npml - 1)
    err = np.abs(u[:, interior] - ua[interior]).max() / abs(ua[0])
    assert err < bound
    # the field decays inside the layer (absorption, not gain)
    assert np.abs(u[0, 0]) < 0.05 * np.abs(ua[0])


def test_stretched_operator_symmetrizer():
    rng = np.random.default_rng(0)
    nx, ny, npml = 30, 22, 6
    eps = 2.085 + 10.165 * rng.random((ny, nx))
    omega, dx = 2 * math.pi / 1.3, 0.025
    A = fdfd.assemble(eps, omega, dx, npml)
    S = fdfd.symmetrizer(nx, ny, omega, dx, npml)
    SA = (A.multiply(S[:, None])).tocsr()
    diff = abs(SA - SA.T).max()
    assert diff < 1e-9 * abs(SA).max()
    # and without the scaling the PML makes A unsymmetric
    assert abs(A - A.T).max() > 1e-3 * abs(A).max()


def test_stretch_profile_properties():
    omega, dx = 4.0, 0.025
    si, sh = fdfd.stretch(50, 10, dx, omega)
    # interior nodes are unstretched, the layer has Im(s) < 0 (exp(+i w t))
    assert np.all(si[10:40] == 1.0)
    assert np.all(si[:10].imag < 0) and np.all(si[40:].imag < 0)
    assert np.all(np.abs(si[:10].imag) > np.abs(si[1:11].imag) - 1e-15)  # grows outward
    # the periodic link n-1 -> 0 sits at full depth, mirror symmetric layer
    np.testing.assert_allclose(sh[-1], si[0])
    np.testing.assert_allclose(si[:10], si[::-1][:10])
    np.testing.assert_allclose(sh[:9], sh[::-1][1:10])


def test_direct_solves_agree_and_satisfy_system():
    inst = W.small_binary()
    A = fdfd.assemble_instance(inst)
    x1 = direct.sparse_solve(A, inst.b)
    assert np.linalg.norm(A @ x1 - inst.b) / np.linalg.norm(inst.b) < 1e-12
    sub = W.Instance(inst.eps[:20, :24].copy(), inst.b[:480].copy(), 24, 20, inst.dx,
                     inst.wavelength, 4)
    As = fdfd.assemble_instance(sub)
    np.testing.assert_allclose(direct.dense_solve(As, sub.b), direct.sparse_solve(As, sub.b),
                               atol=1e-10 * np.abs(direct.dense_solve(As, sub.b)).max())
