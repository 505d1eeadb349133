"""Pins of the oracle's plain and data-driven GMRES (Eqs. 2-5, supplement).

The iterates are unique minimisers over nested spaces, so they can be checked
against brute-force least squares over explicitly built bases, against dense
LU, and against the identities the supplement derives.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import direct, fdfd, gmres, gmres_aug


def tiny(seed, nx=10, ny=8, npml=2):
    rng = np.random.default_rng(seed)
    eps = (2.085 + 10.165 * (rng.random((ny, nx)) < 0.5)).astype(np.float32)
    return W.Instance(eps, W.random_complex(rng, nx * ny), nx, ny, 0.04, 1.55, npml)


def test_unrestarted_terminates_at_dense_solution():
    inst = tiny(0)
    A = fdfd.assemble_instance(inst)
    x, info = gmres.gmres(A, inst.b, tol=1e-12)
    assert info["converged"] and info["iters"] <= inst.D
    xs = direct.dense_solve(A, inst.b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-8


@pytest.mark.parametrize("i", [1, 2, 3, 5])
def test_iterate_is_krylov_minimiser(i):
    inst = tiny(1)
    A = fdfd.assemble_instance(inst)
    x, _ = gmres.gmres(A, inst.b, tol=0.0, maxit=i)
    xb = gmres.krylov_bruteforce(A, inst.b, i)
    np.testing.assert_allclose(x, xb, atol=1e-9 * np.abs(xb).max())


def test_history_monotone_within_a_cycle_and_tolerance_met():
    inst = tiny(2, 14, 12)
    A = fdfd.assemble_instance(inst)
    x, info = gmres.gmres(A, inst.b, restart=20, tol=1e-9, maxit=5000)
    h = np.array(info["history"])
    for c in range(0, len(h), 20):
        seg = h[c:c + 20]
        assert np.all(np.diff(seg) <= 1e-14)
    assert info["converged"]
    assert np.linalg.norm(inst.b - A @ x) / np.linalg.norm(inst.b) <= 1e-9


def test_zero_rhs_and_budget():
    inst = tiny(3)
    A = fdfd.assemble_instance(inst)
    x, info = gmres.gmres(A, np.zeros(inst.D), tol=1e-8)
    assert info["converged"] and np.all(x == 0)
    x, info = gmres.gmres(A, inst.b, tol=1e-8, maxit=0)
    assert not info["converged"] and info["iters"] == 0


def test_augmented_without_vectors_is_plain_gmres():
    inst = tiny(4)
    A = fdfd.assemble_instance(inst)
    _, i0 = gmres.gmres(A, inst.b, restart=7, tol=1e-10, maxit=3000)
    _, i1 = gmres_aug.gmres_aug(A, inst.b, np.zeros((inst.D, 0)), restart=7, tol=1e-10, maxit=3000)
    assert i0["iters"] == i1["iters"]
    np.testing.assert_allclose(i0["history"][:100], i1["history"][:100], rtol=1e-8)


@pytest.mark.parametrize("i", [1, 2, 4])
def test_augmented_iterate_is_minimiser_over_augmented_space(i):
    """f_i = argmin over range(V) + K_i(P A, P b) of ||A f - b|| (Eq. 3)."""
    inst = tiny(5)
    A = fdfd.assemble_instance(inst)
    V = W.random_complex(np.random.default_rng(1), (inst.D, 3))
    x, _ = gmres_aug.gmres_aug(A, inst.b, V, tol=0.0, maxit=i)
    xb = gmres_aug.augmented_bruteforce(A, inst.b, V, i)
    np.testing.assert_allclose(x, xb, atol=1e-9 * np.abs(xb).max())


def test_augmented_depends_only_on_span():
    inst = tiny(6, 12, 10)
    A = fdfd.assemble_instance(inst)
    rng = np.random.default_rng(2)
    V = W.random_complex(rng, (inst.D, 4))
    M = W.random_complex(rng, (4, 4)) + 3 * np.eye(4)
    _, a = gmres_aug.gmres_aug(A, inst.b, V, restart=15, tol=1e-9, maxit=2000)
    _, b = gmres_aug.gmres_aug(A, inst.b, V @ M, restart=15, tol=1e-9, maxit=2000)
    Qv, _ = np.linalg.qr(V)
    _, c = gmres_aug.gmres_aug(A, inst.b, Qv, restart=15, tol=1e-9, maxit=2000)
    n = min(len(a["history"]), len(b["history"]), len(c["history"]), 200)
    np.testing.assert_allclose(a["history"][:n], b["history"][:n], rtol=1e-7)
    np.testing.assert_allclose(a["history"][:n], c["history"][:n], rtol=1e-7)


def test_solution_in_span_solved_by_projection():
    inst = tiny(7)
    A = fdfd.assemble_instance(inst)
    xs = direct.dense_solve(A, inst.b)
    rng = np.random.default_rng(3)
    a = W.random_complex(rng, inst.D)
    V = np.stack([xs + a, a, W.random_complex(rng, inst.D)], axis=1)
    x, info = gmres_aug.gmres_aug(A, inst.b, V, restart=10, tol=1e-9, maxit=50)
    assert info["converged"] and info["iters"] <= 1
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-9


def test_augmented_arnoldi_invariants():
    """C^H Q = 0, [C Q] orthonormal and A Q_i = Q_{i+1} H + C C^H A Q_i
    (supplement eq:arnoldi_matrix)."""
    inst = tiny(8, 12, 10)
    A = fdfd.assemble_instance(inst)
    V = W.random_complex(np.random.default_rng(4), (inst.D, 5))
    _, info = gmres_aug.gmres_aug(A, inst.b, V, restart=25, tol=0.0, maxit=25, record=True)
    C, Q, H, B = info["C"], info["Q"], info["H"], info["B"]
    k, m = C.shape[1], H.shape[1]
    CQ = np.concatenate([C, Q], axis=1)
    np.testing.assert_allclose(CQ.conj().T @ CQ, np.eye(k + m + 1), atol=1e-10)
    np.testing.assert_allclose(A @ Q[:, :m], Q @ H + C @ B, atol=1e-8)
    # A V R^{-1} = C (thin QR of A V)
    np.testing.assert_allclose(A @ V, C @ info["R"], atol=1e-9 * abs(A @ V).max())


def test_augmentation_cuts_first_iteration_residual():
    """A subspace close to the solution gives a large first-iteration drop
    (Sec. 3 discussion of Fig. 2)."""
    inst = tiny(9, 16, 12)
    A = fdfd.assemble_instance(inst)
    xs = direct.dense_solve(A, inst.b)
    rng = np.random.default_rng(5)
    V = np.stack([xs + 1e-5 * np.linalg.norm(xs) / math.sqrt(inst.D) * W.random_complex(rng, inst.D),
                  W.random_complex(rng, inst.D)], axis=1)
    _, ia = gmres_aug.gmres_aug(A, inst.b, V, restart=30, tol=1e-8, maxit=500)
    _, ip = gmres.gmres(A, inst.b, restart=30, tol=1e-8, maxit=500)
    assert ia["history"][0] < 1e-2 < ip["history"][0]
    assert ia["iters"] < ip["iters"]


def test_restarted_augmented_converges_to_dense_solution():
    """Many restarted cycles (restart far shorter than the iteration count,
    k > 0): the oracle must reach the tolerance, report it truthfully, and
    land on the dense LU solution (every cycle after the first starts from
    x != 0 with the right-hand side [C^H r; Q^H r] of eq:final_lsq)."""
    inst = tiny(10, 14, 12)
    A = fdfd.assemble_instance(inst)
    V = W.random_complex(np.random.default_rng(6), (inst.D, 4))
    x, info = gmres_aug.gmres_aug(A, inst.b, V, restart=6, tol=1e-10, maxit=20000)
    assert info["cycles"] >= 5 and info["iters"] > 6
    assert info["converged"]
    rr = np.linalg.norm(inst.b - A @ x) / np.linalg.norm(inst.b)
    assert rr <= 1e-10 and abs(rr - info["rel_res"]) <= 1e-12
    xs = direct.dense_solve(A, inst.b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-7


@pytest.mark.parametrize("i", [1, 2, 3])
def test_augmented_cycle_from_nonzero_start(i):
    """A cycle started from x0 != 0 minimises over x0 + range(V) + K_i(P A, P r0),
    r0 = b - A x0: it equals x0 plus the brute-force minimiser of the shifted
    system A e = r0 over explicit bases."""
    inst = tiny(11)
    A = fdfd.assemble_instance(inst)
    rng = np.random.default_rng(7)
    V = W.random_complex(rng, (inst.D, 3))
    x0 = W.random_complex(rng, inst.D)
    x, _ = gmres_aug.gmres_aug(A, inst.b, V, x0=x0, tol=0.0, maxit=i)
    xb = x0 + gmres_aug.augmented_bruteforce(A, inst.b - A @ x0, V, i)
    np.testing.assert_allclose(x, xb, atol=1e-9 * np.abs(xb).max())


@pytest.mark.parametrize("m,i", [(2, 1), (3, 2), (3, 3)])
def test_second_cycle_is_minimiser_from_first_cycle_iterate(m, i):
    """Restarted cycles: after a first cycle of m steps (iterate x1, the
    minimiser over range(V) + K_m), the next i <= m steps give x1 plus the
    minimiser over range(V) + K_i(P A, P r1) of the system A e = r1 with
    r1 = b - A x1 (brute force over explicit bases, independent code)."""
    inst = tiny(12)
    A = fdfd.assemble_instance(inst)
    V = W.random_complex(np.random.default_rng(8), (inst.D, 2))
    x1b = gmres_aug.augmented_bruteforce(A, inst.b, V, m)
    x2, info = gmres_aug.gmres_aug(A, inst.b, V, restart=m, tol=0.0, maxit=m + i)
    assert info["cycles"] == 2 and info["iters"] == m + i
    x2b = x1b + gmres_aug.augmented_bruteforce(A, inst.b - A @ x1b, V, i)
    np.testing.assert_allclose(x2, x2b, atol=1e-8 * np.abs(x2b).max())
