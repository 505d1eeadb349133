"""Projection and residual losses of a predicted subspace (Sec. 3).

Test infrastructure (oracle): see the package docstring.

eq:proj_loss  l_proj = min over f in span(V) of ||f - f_k||^2 / ||f_k||^2
eq:res_loss   l_res  = min over f in span(V) of ||A_k f - b||^2 / ||b||^2

Both minimisations are written out as least-squares problems.
"""
from __future__ import annotations

import numpy as np


def proj_loss(V, f):
    V = np.asarray(V, np.complex128).reshape(len(f), -1)
    f = np.asarray(f, np.complex128)
    c = np.linalg.lstsq(V, f, rcond=None)[0]
    return float(np.linalg.norm(V @ c - f) ** 2 / np.linalg.norm(f) ** 2)


def res_loss(A, V, b):
    V = np.asarray(V, np.complex128).reshape(len(b), -1)
    b = np.asarray(b, np.complex128)
    AV = A @ V
    c = np.linalg.lstsq(AV, b, rcond=None)[0]
    return float(np.linalg.norm(AV @ c - b) ** 2 / np.linalg.norm(b) ** 2)


def res_loss_grad(A, V, b):
    """Residual loss and its conjugate (Wirtinger) gradient with respect to V.

    l = ||A V c - b||^2 / ||b||^2 at the least-squares c (eq:res_loss).  For a
    perturbation dV the loss changes by 2 Re tr(G^H dV); the real-part and
    imaginary-part derivatives are 2 Re G and 2 Im G.  With r = b - A V c the
    residual (orthogonal to range(A V)), only the derivative of A V c through
    A V survives: G = -A^H r c^H / ||b||^2.
    """
    V = np.asarray(V, np.complex128).reshape(len(b), -1)
    b = np.asarray(b, np.complex128)
    AV = A @ V
    c = np.linalg.lstsq(AV, b, rcond=None)[0]
    r = b - AV @ c
    bb = np.vdot(b, b).real
    G = -np.outer(A.conj().T @ r, c.conj()) / bb
    return float(np.vdot(r, r).real / bb), G
