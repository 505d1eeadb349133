"""Pins of the diagonal preconditioners (supplement, Table 1 comparison)."""
import numpy as np

import workloads as W
from oracle import direct, fdfd, precond


def _tiny(seed, nx=12, ny=10, npml=3):
    rng = np.random.default_rng(seed)
    eps = (2.085 + 10.165 * rng.random((ny, nx))).astype(np.float32)
    return W.Instance(eps, W.random_complex(rng, nx * ny), nx, ny, 0.04, 1.55, npml)


def test_jacobi_is_the_inverse_diagonal():
    inst = _tiny(1)
    A = fdfd.assemble_instance(inst)
    pl, pr = precond.jacobi(A)
    Ap = precond.preconditioned(A, pl, pr)
    np.testing.assert_allclose(Ap.diagonal(), 1.0, rtol=1e-14)
    assert np.all(pr == 1.0)


def test_pml_scaling_is_a_symmetrising_similarity():
    """P_L A P_R is complex symmetric (not Hermitian) and has A's eigenvalues."""
    inst = _tiny(2)
    A = fdfd.assemble_instance(inst)
    pl, pr = precond.pml_scaling(inst.nx, inst.ny, inst.omega, inst.dx, inst.npml)
    Ap = precond.preconditioned(A, pl, pr).toarray()
    assert np.abs(Ap - Ap.T).max() <= 1e-12 * np.abs(Ap).max()
    assert np.abs(A.toarray() - A.toarray().T).max() > 1e-3 * np.abs(Ap).max()
    ea = np.sort_complex(np.linalg.eigvals(A.toarray()))
    ep = np.sort_complex(np.linalg.eigvals(Ap))
    np.testing.assert_allclose(ep, ea, rtol=1e-9, atol=1e-9 * np.abs(ea).max())


def test_preconditioned_gmres_solves_the_original_system():
    inst = _tiny(3)
    A = fdfd.assemble_instance(inst)
    xs = direct.dense_solve(A, inst.b)
    V = W.random_complex(np.random.default_rng(4), (inst.D, 2))
    for pl, pr in (precond.jacobi(A), precond.pml_scaling(inst.nx, inst.ny, inst.omega, inst.dx,
                                                            inst.npml)):
        f, info = precond.gmres_aug_precond(A, inst.b, V, pl, pr, tol=1e-12, maxit=inst.D + 5)
        assert np.linalg.norm(f - xs) / np.linalg.norm(xs) < 1e-9
