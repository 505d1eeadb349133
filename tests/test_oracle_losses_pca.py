"""Pins of the projection / residual losses (eq:proj_loss, eq:res_loss) and the
principal-component basis (Sec. 3)."""
import numpy as np

import workloads as W
from oracle import fdfd, losses, pca


def _tiny(seed):
    rng = np.random.default_rng(seed)
    eps = (2.085 + 10.165 * rng.random((8, 10))).astype(np.float32)
    return W.Instance(eps, W.random_complex(rng, 80), 10, 8, 0.04, 1.55, 2)


def test_proj_loss_bounds_and_special_cases():
    rng = np.random.default_rng(0)
    V = W.random_complex(rng, (60, 4))
    f_in = V @ W.random_complex(rng, 4)
    assert losses.proj_loss(V, f_in) < 1e-20
    Qv, _ = np.linalg.qr(V)
    g = W.random_complex(rng, 60)
    f_perp = g - Qv @ (Qv.conj().T @ g)
    assert abs(losses.proj_loss(V, f_perp) - 1.0) < 1e-12
    for _ in range(5):
        f = W.random_complex(rng, 60)
        l = losses.proj_loss(V, f)
        assert 0.0 <= l <= 1.0
        # closed form through an orthonormal basis of span(V)
        np.testing.assert_allclose(l, 1 - np.linalg.norm(Qv.conj().T @ f) ** 2 / np.linalg.norm(f) ** 2,
                                   rtol=1e-10)


def test_res_loss_bounds_and_closed_form():
    inst = _tiny(1)
    A = fdfd.assemble_instance(inst)
    rng = np.random.default_rng(2)
    V = W.random_complex(rng, (inst.D, 5))
    l = losses.res_loss(A, V, inst.b)
    assert 0.0 <= l <= 1.0
    C, _ = np.linalg.qr(A @ V)
    np.testing.assert_allclose(l, 1 - np.linalg.norm(C.conj().T @ inst.b) ** 2 /
                               np.linalg.norm(inst.b) ** 2, rtol=1e-10)
    # the solution in span(V) gives zero residual loss
    xs = np.linalg.solve(A.toarray(), inst.b)
    assert losses.res_loss(A, np.stack([xs, V[:, 0]], 1), inst.b) < 1e-20


def test_pca_recovers_planted_subspace():
    """Snapshots drawn from a known 6-dimensional subspace with distinct scales:
    the basis spans it and the singular values are those planted."""
    rng = np.random.default_rng(3)
    D, M, r = 400, 50, 6
    U, _ = np.linalg.qr(W.random_complex(rng, (D, r)))
    sig = np.array([50.0, 20.0, 9.0, 4.0, 2.0, 1.0])
    Wm, _ = np.linalg.qr(W.random_complex(rng, (M, r)))
    S = U @ np.diag(sig) @ Wm.conj().T
    Uk, s = pca.pca_basis(S, 4)
    np.testing.assert_allclose(s, sig[:4], rtol=1e-10)
    # arccos resolves angles down to ~sqrt(machine eps)
    assert pca.principal_angles(Uk, U[:, :4]).max() < 1e-7
    # principal angles of a space with itself are zero, of orthogonal spaces pi/2
    assert pca.principal_angles(U[:, :2], U[:, 2:4]).min() > 1.5


def test_res_loss_gradient_matches_finite_differences():
    """The conjugate gradient G of the residual loss: the real-part derivative
    is 2 Re G and the imaginary-part derivative 2 Im G (central differences on
    the loss itself, which is independent of the gradient formula)."""
    inst = _tiny(3)
    A = fdfd.assemble_instance(inst)
    rng = np.random.default_rng(4)
    V = W.random_complex(rng, (inst.D, 3))
    l0, G = losses.res_loss_grad(A, V, inst.b)
    np.testing.assert_allclose(l0, losses.res_loss(A, V, inst.b), rtol=1e-12)
    h = 1e-6
    for _ in range(8):
        i, j = rng.integers(0, inst.D), rng.integers(0, 3)
        for unit, part in ((1.0, G.real), (1j, G.imag)):
            Vp, Vm = V.copy(), V.copy()
            Vp[i, j] += h * unit
            Vm[i, j] -= h * unit
            fd = (losses.res_loss(A, Vp, inst.b) - losses.res_loss(A, Vm, inst.b)) / (2 * h)
            assert abs(fd - 2 * part[i, j]) <= 1e-6 * abs(fd) + 1e-9, (fd, 2 * part[i, j])
    # a subspace holding the solution is a minimum: zero loss and zero gradient
    xs = np.linalg.solve(A.toarray(), inst.b)
    l1, G1 = losses.res_loss_grad(A, np.stack([xs, V[:, 0]], 1), inst.b)
    assert l1 < 1e-20 and np.abs(G1).max() < 1e-8
