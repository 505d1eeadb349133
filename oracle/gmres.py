"""Plain GMRES, restarted or not (Sec. 2, Eq. 2).

Test infrastructure (oracle): see the package docstring.

The i-th iterate is the minimiser of ||A f - b|| over x0 + K_i(A, r0)
(Eq. 2; with x0 = 0 and r0 = b it is exactly Eq. 2).  The Krylov basis is built
by Arnoldi with modified Gram-Schmidt; the small least-squares problem
min_y ||beta e1 - H y|| is handed to numpy.linalg.lstsq at every step, so the
residual history is the least-squares residual itself.  The relative residual
is r_i = ||A f_i - b|| / ||b|| (Sec. 2).

Restarts (GMRES(m)): after m Arnoldi steps the iterate is formed, the residual
b - A x is recomputed explicitly and a new cycle starts from it.

Stopping rule (shared with the GPU solver):
  * a cycle ends when its least-squares residual is <= tol*||b||, when the
    iteration budget is spent, after m steps, or on breakdown (h = 0);
  * after each cycle the true residual is recomputed; the solve has converged
    when ||b - A x|| <= tol*||b||.
"""
from __future__ import annotations

import numpy as np


def _as_matvec(A):
    return A if callable(A) else (lambda v: A @ v)


def gmres(A, b, x0=None, restart=None, tol=1e-6, maxit=None):
    """Returns (x, info); info holds iters (Arnoldi steps), matvecs, history
    (least-squares residual / ||b|| after every step), true_res (per cycle
    start and at the end), converged, cycles."""
    mv = _as_matvec(A)
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    D = b.size
    maxit = D if maxit is None else int(maxit)
    m = maxit if restart is None else int(restart)
    x = np.zeros(D, np.complex128) if x0 is None else np.array(x0, np.complex128).reshape(-1)
    info = dict(iters=0, matvecs=0, history=[], true_res=[], converged=False, cycles=0)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        info.update(converged=True, rel_res=0.0)
        return np.zeros(D, np.complex128), info
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
        Q = np.zeros((m + 1, D), np.complex128)
        H = np.zeros((m + 1, m), np.complex128)
        Q[0] = r / rho
        n = 0
        for j in range(m):
            w = mv(Q[j])
            info["matvecs"] += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(Q[i], w)
                w = w - H[i, j] * Q[i]
            h = np.linalg.norm(w)
            H[j + 1, j] = h
            if h > 0.0:
                Q[j + 1] = w / h
            n = j + 1
            e1 = np.zeros(n + 1, np.complex128)
            e1[0] = rho
            y = np.linalg.lstsq(H[:n + 1, :n], e1, rcond=None)[0]
            est = np.linalg.norm(H[:n + 1, :n] @ y - e1)
            info["iters"] += 1
            info["history"].append(est / bnorm)
            if est <= tol * bnorm or info["iters"] >= maxit or h == 0.0:
                break
        x = x + Q[:n].T @ y
    info["rel_res"] = info["true_res"][-1]
    return x, info


def krylov_bruteforce(A, b, i):
    """argmin over K_i(A, b) of ||A f - b|| from an explicit power basis
    [b, Ab, ..., A^{i-1} b] (column-orthonormalised), for tiny i only."""
    mv = _as_matvec(A)
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    K = [b]
    for _ in range(i - 1):
        K.append(mv(K[-1]))
    K = np.stack(K, axis=1)
    Qk, _ = np.linalg.qr(K)
    AQ = np.stack([mv(Qk[:, c]) for c in range(Qk.shape[1])], axis=1)
    c = np.linalg.lstsq(AQ, b, rcond=None)[0]
    return Qk @ c
