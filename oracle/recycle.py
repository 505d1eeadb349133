"""Subspace recycling along a sequence of related systems.

Test infrastructure (oracle): see the package docstring.

The paper places its method next to Krylov-subspace recycling, where
information from earlier solves of related systems (the steps of a design
optimisation) is carried into the next solve (Sec. 1), and its supplement
builds on GCROT, whose outer truncation keeps a small set of correction
directions from one cycle to the next (supplement, Sec. 1).  The reading
used here (the paper gives no formulas for it):

  * the search space of the last cycle of the solve of system s-1 is
    S = [U, Q_n]: the augmenting directions U = V R^{-1} (A U = C, so that
    A S = [C, Q_{n+1}] [[I, B], [0, H]], the matrix of eq:final_lsq) and the
    cycle's first n Arnoldi vectors;
  * S is compressed to its kr harmonic Ritz vectors of smallest magnitude:
    pairs (theta, y = S u) with A y - theta y orthogonal to A S, i.e.
    (AS)^H (AS) u = theta (AS)^H S u;
  * these kr vectors augment the solve of system s (with its own operator:
    the augmented solver forms A_s Y itself).

Harmonic Ritz values of small magnitude approximate the eigenvalues of A
nearest zero, whose eigenvectors slow a restarted Krylov method down; the
harmonic (rather than the plain) Ritz values are used because they
approximate interior eigenvalues from the outside (Morgan; Parks et al.).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import gmres_aug


def _matvec_cols(A, S):
    mv = A if callable(A) else (lambda v: A @ v)
    return np.stack([mv(S[:, c]) for c in range(S.shape[1])], axis=1)


def harmonic_ritz(A, S, kr):
    """The kr harmonic Ritz pairs of A in span(S) of smallest |theta|, from
    the generalized eigenproblem (AS)^H (AS) u = theta (AS)^H S u solved by
    scipy.linalg.eig (infinite values sort last).  Returns (theta [kr],
    Y [D, kr]) with unit-norm columns y = S u."""
    S = np.asarray(S, np.complex128)
    AS = _matvec_cols(A, S)
    G = AS.conj().T @ AS
    M = AS.conj().T @ S
    theta, U = sla.eig(G, M)
    mag = np.where(np.isfinite(theta), np.abs(theta), np.inf)
    sel = np.argsort(mag, kind="stable")[:kr]
    Y = S @ U[:, sel]
    Y = Y / np.linalg.norm(Y, axis=0, keepdims=True)
    return theta[sel], Y


def last_cycle_space(V, info):
    """S = [V R^{-1}, Q_n] from gmres_aug's record of its last cycle (the
    columns of V are the augmenting vectors, possibly none)."""
    Q = info["Q"]
    n = Q.shape[1] - 1
    parts = []
    if V is not None and np.asarray(V).shape[1] > 0:
        parts.append(sla.solve_triangular(info["R"].T, np.asarray(V, np.complex128).T,
                                          lower=True).T)
    parts.append(Q[:, :n])
    return np.concatenate(parts, axis=1)


def solve_sequence(As, bs, kr, restart, tol, maxit, V0=None):
    """Solve A_s x_s = b_s for s = 0, 1, ...: system 0 with the augmenting
    vectors V0 (or none), every later system augmented by the kr harmonic
    Ritz vectors of the previous solve's last cycle.  Returns per system
    (x, info, V used, theta of the vectors passed on)."""
    out = []
    V = V0
    for A, b in zip(As, bs):
        Vs = np.zeros((len(b), 0), np.complex128) if V is None else V
        x, info = gmres_aug.gmres_aug(A, b, Vs, restart=restart, tol=tol, maxit=maxit,
                                      record=True)
        if "Q" in info:
            theta, Y = harmonic_ritz(A, last_cycle_space(Vs, info), kr)
        else:
            theta, Y = np.zeros(0, np.complex128), Vs
        out.append((x, info, Vs, theta))
        V = Y
    return out
