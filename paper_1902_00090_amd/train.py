"""Predictor training on solver-generated data (Sec. 3; Methods).

Orchestration only: every solve, Gram matrix, target and network update runs
in the library (Solver, local_pca_targets, Cnn); torch tensors hold the data
and index the mini-batches.
"""
from __future__ import annotations

import numpy as np

from . import FdfdOp, Solver, local_pca_targets


def solve_fields(insts, tol=1e-3, restart=100, chunk=64, maxit=30000, cgs_passes=1):
    """Solve every instance with the GPU solver; returns complex64 [N, D] and the infos."""
    import torch
    out, infos = [], []
    for c0 in range(0, len(insts), chunk):
        part = insts[c0:c0 + chunk]
        ops = [FdfdOp.from_instance(i) for i in part]
        bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in part]
        s = Solver(ops, restart=restart, cgs_passes=cgs_passes)
        xs, inf, _ = s.solve(bs, tol=tol, maxit=maxit)
        out.extend(x.to(torch.complex64) for x in xs)
        infos.extend(inf)
        s.close()
    return torch.stack(out).contiguous(), infos


def trajectory_targets(fields, traj_len, window=8, k=10, rms=1.0):
    """fields: [T*S, D] complex64 ordered trajectory by trajectory (S steps
    each).  Returns the local-PCA targets [T*S, k, D] complex64, scaled so
    that the normalised field has root-mean-square `rms` per pixel (the span
    the solver uses is scale-free; the scale only sets the size of the MSE,
    which for unit-norm fields would be ~1/D and lost under the network's
    initial output)."""
    import torch
    N, D = fields.shape
    out = torch.empty((N, k, D), dtype=torch.complex64, device=fields.device)
    for t0 in range(0, N, traj_len):
        out[t0:t0 + traj_len] = local_pca_targets(fields[t0:t0 + traj_len].contiguous(), window, k)
    return out * float(rms * np.sqrt(D))


def train_cnn(net, eps, targets, steps, batch, lr=1e-3, b1=0.9, b2=0.999, seed=0, log=None,
              eim=None):
    """Adam on mini-batches drawn without replacement (reshuffled every epoch).
    eps: [N, ny, nx] float32, targets: [N, k, D] complex64, eim: [N, D]
    complex64 effective-index fields for a three-channel network (device)."""
    import torch
    N = eps.shape[0]
    rng = np.random.default_rng(seed)
    order, pos, losses = rng.permutation(N), 0, []
    for it in range(steps):
        if pos + batch > N:
            order, pos = rng.permutation(N), 0
        idx = torch.as_tensor(order[pos:pos + batch], device=eps.device)
        pos += batch
        loss = net.train_step(eps.index_select(0, idx).contiguous(),
                              targets.index_select(0, idx).contiguous(), lr, b1, b2,
                              eim=None if eim is None else eim.index_select(0, idx).contiguous())
        losses.append(loss)
        if log and (it % max(1, steps // 10) == 0 or it == steps - 1):
            log(f"  cnn step {it}: loss {loss:.4e}")
    return losses


def train_cnn_res(net, eps, ops, bs, steps, batch, lr=1e-3, b1=0.9, b2=0.999, seed=0, log=None,
                  eim=None):
    """Unsupervised training on the residual loss (Sec. 3, eq:res_loss): each
    sample is a permittivity with its operator and right-hand side, no solved
    field.  Mini-batches without replacement, reshuffled every epoch."""
    import torch
    N = eps.shape[0]
    rng = np.random.default_rng(seed)
    order, pos, losses = rng.permutation(N), 0, []
    for it in range(steps):
        if pos + batch > N:
            order, pos = rng.permutation(N), 0
        sel = order[pos:pos + batch]
        idx = torch.as_tensor(sel, device=eps.device)
        pos += batch
        loss = net.train_step_res(eps.index_select(0, idx).contiguous(), [ops[i] for i in sel],
                                  [bs[i] for i in sel], lr, b1, b2,
                                  eim=None if eim is None else eim.index_select(0, idx).contiguous())
        losses.append(loss)
        if log and (it % max(1, steps // 10) == 0 or it == steps - 1):
            log(f"  cnn step {it}: residual loss {loss:.4e}")
    return losses
