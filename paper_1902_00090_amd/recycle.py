"""Trajectory recycling: augment the solve of design step s with what the
solves of earlier steps of the same trajectory found.

This is the recycling approach the paper sets its learned subspaces against
(Sec. 1: reuse Krylov information from the simulations of an optimisation
trajectory in its later simulations; the supplement's GCROT keeps a few
correction directions from cycle to cycle).  Two kinds of recycled vectors,
alone or together:

  * solutions: the fields of steps max(0, s - window) .. s - 1;
  * subspaces: the `ritz` harmonic Ritz vectors of smallest magnitude of
    step s - 1's last cycle (Solver.recycle), which carry the directions that
    slow the restarted iteration down from one step to the next (and, since
    step s - 1 was itself augmented by them, are refined along the
    trajectory).

Orchestration only: every solve runs in the library's batched augmented
GMRES, with the problems of one design step of all trajectories in one
lockstep batch.
"""
from __future__ import annotations

import numpy as np

from . import FdfdOp, Solver


def solve_trajectories(trajs, window=5, tol=1e-6, restart=100, maxit=30000, cgs_passes=1,
                       recycle=True, ritz=0, hist_cap=0, inner="c64", base=None):
    """trajs: T trajectories, each a list of S instances (equal S; the grids of
    one trajectory must not change).  Step s of trajectory t is augmented by
    the solutions of its steps max(0, s - window) .. s - 1 (recycle=True) and
    by the `ritz` harmonic Ritz vectors of its step s - 1 (ritz > 0); neither
    at s = 0.  recycle=False and ritz=0 run plain GMRES on the same schedule.
    base: an optional [k0, D] tensor (a predicted basis, such as the PCA
    components) that augments every step of every trajectory ahead of the
    recycled vectors.

    Returns (x, infos, hist, theta): x[t][s] complex128 device tensors,
    infos[t][s] info dicts, hist[t][s] residual histories (empty unless
    hist_cap > 0), theta[t][s] the harmonic Ritz values passed on from step s
    (empty unless ritz > 0).
    """
    import torch
    T, S = len(trajs), len(trajs[0])
    if any(len(tr) != S for tr in trajs):
        raise ValueError("all trajectories need the same number of steps")
    dt = torch.complex64 if inner == "c64" else torch.complex128
    k0 = 0 if base is None else int(base.shape[0])
    kmax = k0 + (window if recycle else 0) + int(ritz)
    solver = None
    prev = [[] for _ in range(T)]
    Y = [None] * T
    xs_all = [[None] * S for _ in range(T)]
    inf_all = [[None] * S for _ in range(T)]
    hist_all = [[np.zeros(0)] * S for _ in range(T)]
    th_all = [[np.zeros(0, np.complex128)] * S for _ in range(T)]
    for s in range(S):
        ops = [FdfdOp.from_instance(tr[s]) for tr in trajs]
        bs = [torch.tensor(tr[s].b, dtype=torch.complex128, device="cuda") for tr in trajs]
        # the solver keeps the operators it is bound to (Solver.ops), so those of
        # the previous step are released only after the new ones are bound
        if solver is None:
            solver = Solver(ops, restart=restart, kmax=kmax, inner=inner,
                            cgs_passes=cgs_passes, hist_cap=hist_cap)
        else:
            solver.bind(ops)
        U = []
        for t in range(T):
            parts = [] if base is None else [base.to(dt)]
            if recycle and s > 0:
                parts.append(torch.stack(prev[t][-window:]))
            if ritz > 0 and s > 0 and Y[t] is not None and Y[t].shape[0] > 0:
                parts.append(Y[t])
            U.append(torch.cat(parts).contiguous() if parts else None)
        solver.set_subspace(U if any(u is not None for u in U) else None)
        xs, infos, _ = solver.solve(bs, tol=tol, maxit=maxit)
        for t in range(T):
            xs_all[t][s] = xs[t]
            inf_all[t][s] = infos[t]
            if hist_cap > 0:
                hist_all[t][s] = solver.history(t)
            prev[t].append(xs[t].to(dt))
        if ritz > 0 and s + 1 < S:
            Y, theta = solver.recycle(ritz)
            for t in range(T):
                th_all[t][s] = theta[t, :Y[t].shape[0]]
    solver.close()
    return xs_all, inf_all, hist_all, th_all
