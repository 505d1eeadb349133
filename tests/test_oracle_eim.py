"""Pins of the effective-index oracle (the CNN's second input, Sec. 3).

The anchors are exact facts, not re-typed formulas:
  * additively separable permittivity eps(ix, iy) = e_x(ix) + e_y(iy) with a
    source j(x) phi(y): the effective-index field equals the 2D FDFD solution
    of the oracle's sparse operator (Kronecker-sum structure), so a wrong sign,
    stretch, index or projection anywhere shows up as a large error;
  * a uniform column: the lowest Dirichlet eigenpair of the second difference
    is known in closed form;
  * the mode of an unreduced tridiagonal matrix with negative off-diagonals is
    positive and simple.
"""
import math

import numpy as np
import scipy.sparse.linalg as spla

import workloads as W
from oracle import eim, fdfd


def _slab_profile(ny, dx, core_um=0.4):
    e = np.full(ny, W.EPS_SIO2)
    r0, r1 = W.waveguide_rows(ny, dx, core_um)
    e[r0:r1] = W.EPS_SI
    return e


def _separable_case(ex, ey, dx, wavelength, npml, ix0):
    omega = 2 * math.pi / wavelength
    eps = ex[None, :] + ey[:, None]
    J = W.slab_mode_source(eps, ix0, dx, omega)       # J(:, ix0) = mode of that column
    b = W.rhs_from_current(J, omega)
    A = fdfd.assemble(eps, omega, dx, npml, npml_y=0)
    f = spla.spsolve(A.tocsc(), b)
    F = eim.eim_field(eps, b, omega, dx, npml)
    return F, f


def test_x_invariant_slab_is_exact():
    ny, nx, dx = 240, 96, 0.025
    ey = _slab_profile(ny, dx)
    F, f = _separable_case(np.zeros(nx), ey, dx, 1.30, 20, 30)
    assert np.linalg.norm(F - f) / np.linalg.norm(f) < 1e-9


def test_additively_separable_permittivity_is_exact():
    """A varying e_x(ix) shifts every column's mode eigenvalue, leaving its vector."""
    rng = np.random.default_rng(3)
    ny, nx, dx = 200, 80, 0.025
    ey = _slab_profile(ny, dx)
    ex = 0.6 * rng.random(nx)
    F, f = _separable_case(ex, ey, dx, 1.55, 12, 20)
    assert np.linalg.norm(F - f) / np.linalg.norm(f) < 1e-9


def test_uniform_column_closed_form():
    ny, nx, dx, lam, e0 = 50, 3, 0.04, 1.55, 3.3
    omega = 2 * math.pi / lam
    mu, phi = eim.column_modes(np.full((ny, nx), e0), omega, dx)
    mu_ref = (2 - 2 * math.cos(math.pi / (ny + 1))) / dx ** 2 - omega ** 2 * e0
    v = np.sin(math.pi * np.arange(1, ny + 1) / (ny + 1))
    v /= np.linalg.norm(v)
    np.testing.assert_allclose(mu, mu_ref, rtol=1e-12)
    np.testing.assert_allclose(phi, np.repeat(v[:, None], nx, 1), atol=1e-12)


def test_modes_positive_unit_and_lowest():
    inst = W.grating(1000, nx=96, ny=48)
    mu, phi = eim.column_modes(inst.eps, inst.omega, inst.dx)
    assert np.all(phi > 0)
    np.testing.assert_allclose(np.linalg.norm(phi, axis=0), 1.0, rtol=1e-12)
    for ix in (0, 40, 95):
        d = 2 / inst.dx ** 2 - inst.omega ** 2 * inst.eps[:, ix].astype(np.float64)
        T = np.diag(d) - (np.eye(48, k=1) + np.eye(48, k=-1)) / inst.dx ** 2
        w = np.linalg.eigvalsh(T)
        assert abs(mu[ix] - w[0]) <= 1e-9 * abs(w).max()
        assert w[1] - w[0] > 0
        np.testing.assert_allclose(T @ phi[:, ix], mu[ix] * phi[:, ix], atol=1e-8 * abs(w).max())


def test_grating_input_waveguide_resembles_the_solution():
    """Before the design region the grating is a straight waveguide: the
    effective-index field is close to the FDFD field there (reflections from
    the design region make it approximate, not exact)."""
    inst = W.grating(1000, nx=192, ny=96)
    A = fdfd.assemble_instance(inst)
    f = spla.spsolve(A.tocsc(), inst.b).reshape(inst.ny, inst.nx)
    F = eim.eim_instance(inst).reshape(inst.ny, inst.nx)
    x0, _, _, _ = W.design_box(inst.nx, inst.ny)
    sl = np.s_[:, inst.npml:x0]
    c = abs(np.vdot(F[sl], f[sl])) / (np.linalg.norm(F[sl]) * np.linalg.norm(f[sl]))
    assert c > 0.7, c          # 0.75 for this instance
