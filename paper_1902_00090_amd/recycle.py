"""Trajectory recycling: augment the solve of design step s with the fields of
earlier steps of the same trajectory.

This is the recycling approach the paper sets its learned subspaces against
(Sec. 1: reuse the subspace spanned by the simulations of an optimisation
trajectory for its later simulations).  Orchestration only: every solve runs
in the library's batched augmented GMRES, with the problems of one design step
of all trajectories in one lockstep batch.
"""
from __future__ import annotations

import numpy as np

from . import FdfdOp, Solver


def solve_trajectories(trajs, window=5, tol=1e-6, restart=100, maxit=30000, cgs_passes=1,
                       recycle=True, hist_cap=0):
    """trajs: T trajectories, each a list of S instances (equal S; the grids of
    one trajectory must not change).  Step s of trajectory t is augmented by
    the complex64 solutions of its steps max(0, s - window) .. s - 1 (none at
    s = 0); recycle=False runs plain GMRES on the same schedule.

    Returns (x, infos, hist): x[t][s] complex128 device tensors, infos[t][s]
    info dicts, hist[t][s] residual histories (empty unless hist_cap > 0).
    """
    import torch
    T, S = len(trajs), len(trajs[0])
    if any(len(tr) != S for tr in trajs):
        raise ValueError("all trajectories need the same number of steps")
    solver = None
    prev = [[] for _ in range(T)]
    xs_all = [[None] * S for _ in range(T)]
    inf_all = [[None] * S for _ in range(T)]
    hist_all = [[np.zeros(0)] * S for _ in range(T)]
    for s in range(S):
        ops = [FdfdOp.from_instance(tr[s]) for tr in trajs]
        bs = [torch.tensor(tr[s].b, dtype=torch.complex128, device="cuda") for tr in trajs]
        # the solver keeps the operators it is bound to (Solver.ops), so those of
        # the previous step are released only after the new ones are bound
        if solver is None:
            solver = Solver(ops, restart=restart, kmax=window if recycle else 0,
                            cgs_passes=cgs_passes, hist_cap=hist_cap)
        else:
            solver.bind(ops)
        if recycle and s > 0:
            solver.set_subspace([torch.stack(prev[t][-window:]).contiguous() for t in range(T)])
        else:
            solver.set_subspace(None)
        xs, infos, _ = solver.solve(bs, tol=tol, maxit=maxit)
        for t in range(T):
            xs_all[t][s] = xs[t]
            inf_all[t][s] = infos[t]
            if hist_cap > 0:
                hist_all[t][s] = solver.history(t)
            prev[t].append(xs[t].to(torch.complex64))
    solver.close()
    return xs_all, inf_all, hist_all
