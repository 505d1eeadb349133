"""Data-driven (augmented) GMRES (Sec. 2, Eqs. 3-5; supplement, Sec. 1).

Test infrastructure (oracle): see the package docstring.

Given linearly independent vectors V = [v_1 .. v_N] (not necessarily
orthogonal), the i-th iterate minimises ||A f - b|| over range(V) + K_i(At, bt)
(Eq. 3) with At = P A, bt = P b, where P projects out of span(A v_1 .. A v_N)
(Eqs. 4-5).  Following the supplement:

  * thin QR  A V = C R  (C orthonormal, R upper triangular), P = I - C C^H;
  * Arnoldi on At: q_1 = bt/||bt||, each new vector is At q_i orthogonalised
    against q_1..q_i (eq:arnoldi); At q is formed as A q followed by the
    projection P; B = C^H A Q_i is kept (eq:arnoldi_matrix);
  * f_i = V R^{-1} x_i + Q_i y_i with [x_i; y_i] the least-squares solution of
    [[I, C^H A Q_i], [0, H]] [x; y] = [C^H b; Q_{i+1}^H b]  (eq:final_lsq),
    solved here with numpy.linalg.lstsq, literally, at every step.

Orthogonalisation: modified Gram-Schmidt (equal to the classical form the
supplement writes, in exact arithmetic).  The projection P is applied twice
wherever it is applied (P P = P, so the value is the same in exact
arithmetic): when a vector lies almost entirely in span(C) -- the case of a
good prediction -- a single pass cancels catastrophically and leaves O(1)
components along C in the normalised remainder.

Restarts (not covered by the paper, which runs unrestarted): C and R stay
fixed; each cycle starts from the explicitly recomputed residual r = b - A x,
which plays the role of b in the formulas above, and adds its f to x.  The
stopping rule is the one of the plain solver in oracle.gmres.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _as_matvec(A):
    return A if callable(A) else (lambda v: A @ v)


def augmentation_setup(A, V):
    """(C, R) with A V = C R (thin QR, numpy.linalg.qr)."""
    mv = _as_matvec(A)
    V = np.asarray(V, dtype=np.complex128)
    AV = np.stack([mv(V[:, c]) for c in range(V.shape[1])], axis=1) if V.shape[1] else \
        np.zeros((V.shape[0], 0), np.complex128)
    if V.shape[1] == 0:
        return AV, np.zeros((0, 0), np.complex128)
    C, R = np.linalg.qr(AV)
    return C, R


def gmres_aug(A, b, V, x0=None, restart=None, tol=1e-6, maxit=None, record=False):
    """Returns (x, info) like oracle.gmres.gmres; V is D x N (N may be 0).

    With record=True, info also holds the last cycle's C, Q, H and B for
    invariant checks."""
    mv = _as_matvec(A)
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    D = b.size
    V = np.asarray(V, dtype=np.complex128).reshape(D, -1)
    N = V.shape[1]
    maxit = D if maxit is None else int(maxit)
    m = maxit if restart is None else int(restart)
    x = np.zeros(D, np.complex128) if x0 is None else np.array(x0, np.complex128).reshape(-1)
    info = dict(iters=0, matvecs=N, history=[], true_res=[], converged=False, cycles=0)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        info.update(converged=True, rel_res=0.0)
        return np.zeros(D, np.complex128), info
    C, R = augmentation_setup(mv, V)
    while True:
        r = b - mv(x)
        info["matvecs"] += 1
        rho = np.linalg.norm(r)
        info["true_res"].append(rho / bnorm)
        if rho <= tol * bnorm:
            info["converged"] = True
            break
        if info["iters"] >= maxit:
            break
        info["cycles"] += 1
        Cr = C.conj().T @ r
        bt = r - C @ Cr
        c2 = C.conj().T @ bt
        bt = bt - C @ c2
        Cr = Cr + c2
        beta = np.linalg.norm(bt)
        Q = np.zeros((m + 1, D), np.complex128)
        H = np.zeros((m + 1, m), np.complex128)
        B = np.zeros((N, m), np.complex128)
        if beta == 0.0:
            # r lies in span(AV): the augmentation alone solves the cycle
            x = x + V @ sla.solve_triangular(R, Cr)
            continue
        Q[0] = bt / beta
        n = 0
        for j in range(m):
            Aq = mv(Q[j])
            info["matvecs"] += 1
            c1 = C.conj().T @ Aq
            w = Aq - C @ c1
            c2 = C.conj().T @ w
            w = w - C @ c2
            B[:, j] = c1 + c2
            for i in range(j + 1):
                H[i, j] = np.vdot(Q[i], w)
                w = w - H[i, j] * Q[i]
            h = np.linalg.norm(w)
            H[j + 1, j] = h
            if h > 0.0:
                Q[j + 1] = w / h
            n = j + 1
            M = np.zeros((N + n + 1, N + n), np.complex128)
            M[:N, :N] = np.eye(N)
            M[:N, N:] = B[:, :n]
            M[N:, N:] = H[:n + 1, :n]
            rhs = np.concatenate([Cr, Q[:n + 1].conj() @ r])
            sol = np.linalg.lstsq(M, rhs, rcond=None)[0]
            est = np.linalg.norm(M @ sol - rhs)
            info["iters"] += 1
            info["history"].append(est / bnorm)
            if est <= tol * bnorm or info["iters"] >= maxit or h == 0.0:
                break
        xa, y = sol[:N], sol[N:]
        x = x + (V @ sla.solve_triangular(R, xa) if N else 0.0) + Q[:n].T @ y
        if record:
            info.update(C=C, R=R, Q=Q[:n + 1].T.copy(), H=H[:n + 1, :n].copy(),
                        B=B[:, :n].copy(), r=r.copy())
    info["rel_res"] = info["true_res"][-1]
    return x, info


def augmented_bruteforce(A, b, V, i):
    """argmin over range(V) + K_i(At, bt) of ||A f - b|| from explicit bases:
    an orthonormal basis of range(V) joined with the power basis of At on bt,
    for tiny i only (x0 = 0)."""
    mv = _as_matvec(A)
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    V = np.asarray(V, dtype=np.complex128)
    AV = np.stack([mv(V[:, c]) for c in range(V.shape[1])], axis=1)
    Cq, _ = np.linalg.qr(AV)

    def P(v):
        return v - Cq @ (Cq.conj().T @ v)

    K = [P(b)]
    for _ in range(i - 1):
        K.append(P(mv(K[-1])))
    basis = np.concatenate([V, np.stack(K, axis=1)], axis=1)
    Qb, _ = np.linalg.qr(basis)
    AQ = np.stack([mv(Qb[:, c]) for c in range(Qb.shape[1])], axis=1)
    c = np.linalg.lstsq(AQ, b, rcond=None)[0]
    return Qb @ c
