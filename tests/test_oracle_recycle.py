"""Pins of the oracle's subspace recycling (Sec. 1, recycling; supplement
Sec. 1, GCROT's kept correction directions): harmonic Ritz pairs against
dense eigendecompositions and an independent formulation, the last cycle's
search space against the Arnoldi relation, and recycled sequences against
dense LU and the brute-force augmented minimiser."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import direct, fdfd, gmres_aug, recycle


def tiny(seed, nx=6, ny=5, npml=1):
    rng = np.random.default_rng(seed)
    eps = (2.085 + 10.165 * (rng.random((ny, nx)) < 0.5)).astype(np.float32)
    return W.Instance(eps, W.random_complex(rng, nx * ny), nx, ny, 0.04, 1.55, npml)


@pytest.mark.parametrize("seed", [0, 1])
def test_full_space_gives_the_eigenpairs_nearest_zero(seed):
    """When the last cycle's Krylov space is the whole space, the harmonic
    Ritz pairs are A's eigenpairs, and the kr of smallest |theta| are those of
    the kr eigenvalues nearest zero."""
    inst = tiny(seed)
    A = fdfd.assemble_instance(inst).toarray()
    D = inst.D
    _, info = gmres_aug.gmres_aug(A, inst.b, np.zeros((D, 0)), restart=D, tol=0.0, maxit=D,
                                  record=True)
    S = recycle.last_cycle_space(np.zeros((D, 0)), info)
    assert S.shape[1] == D
    theta, Y = recycle.harmonic_ritz(A, S, 5)
    lam = np.linalg.eigvals(A)
    lam = lam[np.argsort(np.abs(lam))][:5]
    np.testing.assert_allclose(np.sort_complex(theta), np.sort_complex(lam), rtol=1e-9)
    nA = np.linalg.norm(A, 2)
    for i in range(5):
        assert np.linalg.norm(A @ Y[:, i] - theta[i] * Y[:, i]) <= 1e-9 * nA


def test_invariant_subspace_inside_the_space_is_recovered():
    """If span(S) holds eigenvectors of A, their eigenvalues are harmonic Ritz
    values and the eigenvectors are the harmonic Ritz vectors."""
    inst = tiny(2)
    A = fdfd.assemble_instance(inst).toarray()
    lam, X = np.linalg.eig(A)
    pick = [3, 11, 17]
    rng = np.random.default_rng(5)
    S = np.concatenate([X[:, pick], W.random_complex(rng, (inst.D, 5))], axis=1)
    S = S @ W.random_complex(rng, (8, 8))          # mix: only the span is given
    theta, Y = recycle.harmonic_ritz(A, S, 8)
    for i in pick:
        d = np.abs(theta - lam[i])
        q = int(np.argmin(d))
        assert d[q] <= 1e-9 * abs(lam[i])
        y, x = Y[:, q], X[:, i]
        assert abs(abs(np.vdot(x, y)) - np.linalg.norm(x) * np.linalg.norm(y)) <= 1e-8


def test_harmonic_ritz_values_are_reciprocal_ritz_values_of_the_inverse():
    """Independent formulation: with W an orthonormal basis of A S, the
    harmonic Ritz values are the reciprocals of the eigenvalues of
    W^H A^{-1} W; the selection keeps the smallest |theta| and each pair meets
    the Galerkin condition A y - theta y orthogonal to A S."""
    inst = tiny(3, nx=8, ny=6)
    A = fdfd.assemble_instance(inst).toarray()
    rng = np.random.default_rng(9)
    S = W.random_complex(rng, (inst.D, 12))
    theta, Y = recycle.harmonic_ritz(A, S, 12)
    Wq, _ = np.linalg.qr(A @ S)
    mu = np.linalg.eigvals(Wq.conj().T @ np.linalg.solve(A, Wq))
    np.testing.assert_allclose(np.sort_complex(theta), np.sort_complex(1.0 / mu), rtol=1e-8)
    assert np.all(np.diff(np.abs(theta)) >= 0)
    t4, Y4 = recycle.harmonic_ritz(A, S, 4)
    np.testing.assert_allclose(t4, theta[:4], rtol=1e-12)
    AS = A @ S
    for i in range(4):
        res = A @ Y4[:, i] - t4[i] * Y4[:, i]
        assert np.linalg.norm(AS.conj().T @ res) <= 1e-9 * np.linalg.norm(AS, 2) * np.linalg.norm(A, 2)


def test_last_cycle_space_satisfies_the_augmented_arnoldi_relation():
    """S = [V R^{-1}, Q_n] from a restarted augmented solve: A S equals
    [C, Q_{n+1}] [[I, B], [0, H]] (the matrix of eq:final_lsq) with the
    recorded C, B, H, and the columns of [C, Q_{n+1}] are orthonormal."""
    inst = tiny(4, nx=10, ny=8, npml=2)
    A = fdfd.assemble_instance(inst)
    rng = np.random.default_rng(4)
    V = W.random_complex(rng, (inst.D, 3))
    _, info = gmres_aug.gmres_aug(A, inst.b, V, restart=8, tol=1e-10, maxit=60, record=True)
    assert info["cycles"] >= 2
    S = recycle.last_cycle_space(V, info)
    k, n = 3, info["Q"].shape[1] - 1
    Wb = np.concatenate([info["C"], info["Q"]], axis=1)
    G = np.zeros((k + n + 1, k + n), np.complex128)
    G[:k, :k] = np.eye(k)
    G[:k, k:] = info["B"]
    G[k:, k:] = info["H"]
    AS = A @ S
    np.testing.assert_allclose(AS, Wb @ G, atol=1e-10 * np.abs(AS).max())
    np.testing.assert_allclose(Wb.conj().T @ Wb, np.eye(k + n + 1), atol=1e-10)


def test_recycled_sequence_converges_to_the_dense_solutions():
    """Three steps of a small design trajectory, each solved to tol with the
    previous step's 4 harmonic Ritz vectors: every solution matches dense LU,
    and the first iterates of a recycled solve are the brute-force
    minimisers over span(Y) + K_i (Eq. 3)."""
    insts = W.trajectory(7000, 700000, 3, 24, 16, 1.30, npml=3)
    As = [fdfd.assemble_instance(i) for i in insts]
    bs = [i.b for i in insts]
    out = recycle.solve_sequence(As, bs, kr=4, restart=15, tol=1e-9, maxit=4000)
    for (x, info, Vs, theta), A, b in zip(out, As, bs):
        assert info["converged"]
        xs = direct.dense_solve(A, b)
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-6
    assert out[1][2].shape[1] == 4 and out[2][2].shape[1] == 4
    assert np.all(np.diff(np.abs(out[0][3])) >= 0)
    Y = out[1][2]
    for i in (1, 3):
        xi, _ = gmres_aug.gmres_aug(As[1], bs[1], Y, tol=0.0, maxit=i)
        xb = gmres_aug.augmented_bruteforce(As[1], bs[1], Y, i)
        np.testing.assert_allclose(xi, xb, atol=1e-8 * np.abs(xb).max())
