"""Benchmark: solves/s and matvecs to 1e-6 relative residual, data-driven
(PCA-augmented) vs plain GMRES, one MI355X.

Workload (one "step" = one pass of the whole hot path over one batch):
  * a synthetic design-trajectory data set of 480 x 240 grating problems
    (dx 25 nm, lambda 1.30 um, 20-cell PML), 8 trajectories x 32 steps, split
    75 / 25 at random over all steps as the paper splits its data set;
  * predictor training (outside the timed region): the training problems are
    solved by this library's GPU solver, their fields form the snapshot
    matrix, and pca_build returns the top-k (k = 20) principal components;
  * timed step: for a batch of B = 64 evaluation problems, the augmentation
    setup (A V, Cholesky QR twice) and augmented GMRES(100) in complex64 with
    FP64 true-residual restarts to ||b - A x|| / ||b|| <= 1e-6;
  * plain GMRES(100) on the same batch, timed once, for the comparison.

Prints one JSON line (stdout).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per Arnoldi-step launch of the two streaming sweeps, from two
# rocprofv3 --pmc passes (FETCH_SIZE x2.000, WRITE_SIZE x1.000 after
# calibration on a 1 GiB copy) over this workload (64 problems, k = 20); valid
# only for the kernel sources they were taken with (see profiles/).
MEASURED_TRAFFIC = {"bytes_per_launch": {"k_update_norm": 3.172e9, "k_matvec_dot": 3.189e9},
                    "sources_sha256_16": "9f9ee175871076d2"}


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("solver_kernels.h", "op.h", "common.h"):
        with open(os.path.join(ROOT, "paper_1902_00090_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def first_below(h, thr):
    idx = np.nonzero(np.asarray(h) <= thr)[0]
    return int(idx[0]) + 1 if len(idx) else None


def arnoldi_bytes(D, iters, m, k, passes=1):
    """Algorithmic HBM bytes of `iters` complex64 Arnoldi steps with restart m
    and k augmenting vectors: step j of a cycle reads the stencil input and
    eps and writes w (20 D), reads the k+j+1 basis vectors and w for the dots
    and again for the update, and writes q_{j+1}: 16 D (k+j) + 44 D; each
    further Gram-Schmidt pass adds 16 D (k+j) + 24 D."""
    full, rem = divmod(int(iters), m)
    def cyc(n):       # sum over j < n of (k + j)
        return n * k + n * (n - 1) // 2
    sj = full * cyc(m) + cyc(rem)
    return (16 * D * sj + 44 * D * iters) + (passes - 1) * (16 * D * sj + 24 * D * iters)


def cnn_flops_per_instance(net):
    """2 x multiply-adds of the 3x3 convolutions of one forward pass."""
    H, Wd, tot = net.ny, net.nx, 0
    for cin, cout, s, up, _ in net.layers():
        if up:
            H, Wd = 2 * H, 2 * Wd
        elif s == 2:
            H, Wd = H // 2, Wd // 2
        tot += 2 * 9 * cin * cout * H * Wd
    return tot


def cnn_leg(args, torch, W, data, tr_idx, train, test, Smat, ops, bs, xs, U, it_aug, plain,
            loss_mode):
    """Train the CNN on the training problems, predict k fields for every
    evaluation problem, solve the evaluation batch augmented by them; the
    effective-index field and inference are inside the timed region.
    loss_mode "proj": MSE against local-PCA targets of the training fields
    (grouped by trajectory); "res": the unsupervised residual loss."""
    from paper_1902_00090_amd import (Cnn, FdfdOp, Solver, eim_field, local_pca_targets,
                                      proj_loss_batched, res_loss_batched)
    from paper_1902_00090_amd.train import train_cnn, train_cnn_res
    k, D, B = args.cnn_k, test[0].D, len(test)
    t0 = time.time()
    targets = None
    if loss_mode == "proj":
        traj_of = np.asarray(tr_idx) // args.traj_steps
        targets = torch.empty((len(train), k, D), dtype=torch.complex64, device="cuda")
        for t in np.unique(traj_of):
            rows = np.nonzero(traj_of == t)[0]
            r0, r1 = int(rows[0]), int(rows[-1]) + 1      # sorted indices: contiguous rows
            targets[r0:r1] = local_pca_targets(Smat[r0:r1].contiguous(), args.cnn_window, k)
        targets *= float(math.sqrt(D))                     # unit RMS per pixel
    eps_tr = torch.tensor(np.stack([i.eps for i in train]), device="cuda")
    tr_ops = [FdfdOp.from_instance(i) for i in train]
    tr_bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in train]
    eim_tr = None
    if args.cnn_inputs == 3:
        eim_tr = torch.empty((len(train), D), dtype=torch.complex64, device="cuda")
        for c0 in range(0, len(train), 64):
            eim_field(tr_ops[c0:c0 + 64], tr_bs[c0:c0 + 64], out=eim_tr[c0:c0 + 64])
    net = Cnn(test[0].nx, test[0].ny, max_batch=32, k=k, seed=7, in_channels=args.cnn_inputs)
    if loss_mode == "proj":
        losses = train_cnn(net, eps_tr, targets, args.cnn_steps, 32, lr=1e-3, seed=11, eim=eim_tr)
    else:
        losses = train_cnn_res(net, eps_tr, tr_ops, tr_bs, args.cnn_steps, 32, lr=1e-3, seed=11,
                               eim=eim_tr)
    torch.cuda.synchronize()
    t_cnn_train = time.time() - t0
    del targets, eps_tr, eim_tr, tr_ops, tr_bs
    log(f"CNN ({loss_mode} loss): {args.cnn_inputs} input planes, {args.cnn_steps} Adam steps on "
        f"{len(train)} samples, {t_cnn_train:.1f}s, loss {losses[0]:.3e} -> "
        f"{np.mean(losses[-20:]):.3e}")

    eps_te = torch.tensor(np.stack([i.eps for i in test]), device="cuda")
    eim_te = None
    if args.cnn_inputs == 3:
        eim_te = torch.empty((B, D), dtype=torch.complex64, device="cuda")

    def setup():
        """Predictor inputs and inference: the per-problem setup of the CNN leg."""
        if eim_te is not None:
            eim_field(ops, bs, out=eim_te)
        net.predict(eps_te, Ucnn, eim=eim_te)

    Ucnn = torch.empty((B, k, D), dtype=torch.complex64, device="cuda")
    setup()                                            # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    net.predict(eps_te, Ucnn, eim=eim_te)
    e1.record()
    torch.cuda.synchronize()
    inf_ms = e0.elapsed_time(e1)
    t0 = time.time()
    setup()
    torch.cuda.synchronize()
    setup_ms = 1000 * (time.time() - t0)
    flops = cnn_flops_per_instance(net) * B
    xs_stack = torch.stack(xs).contiguous()
    lp_cnn = proj_loss_batched(Ucnn, xs_stack)
    lp_pca = proj_loss_batched(U.unsqueeze(0).expand(B, -1, -1).contiguous(), xs_stack)
    lp_eim = None
    if eim_te is not None:
        lp_eim = proj_loss_batched(eim_te.unsqueeze(1).contiguous(), xs_stack)
    del xs_stack
    lr_cnn = res_loss_batched(ops, bs, [Ucnn[p] for p in range(B)])
    lr_pca = res_loss_batched(ops, bs, [U] * B)

    s = Solver(ops, restart=args.restart, kmax=k, cgs_passes=args.cgs, hist_cap=args.maxit)
    xc = [torch.empty_like(b) for b in bs]
    Ul = [Ucnn[p] for p in range(B)]
    torch.cuda.synchronize()
    t0 = time.time()
    setup()
    s.set_subspace(Ul)
    _, inf, _ = s.solve(bs, tol=args.tol, maxit=args.maxit, x=xc)
    torch.cuda.synchronize()
    dt = time.time() - t0
    h = [s.history(p) for p in range(B)]
    s.close()
    net.close()
    it = np.array([i["iters"] for i in inf])
    out = {
        "solves_per_s_incl_inference": round(B / dt, 4),
        "iters_mean": float(it.mean()),
        "matvecs_mean": float(np.mean([i["matvecs"] for i in inf])),
        "all_converged": all(i["status"] == 0 for i in inf),
        "worst_rel_res_true": max(i["rel_res_true"] for i in inf),
        "rel_res_after_1_iter_mean": float(np.mean([x[0] for x in h])),
        "iters_to_0.04_mean": float(np.mean([first_below(x, 0.04) or np.nan for x in h])),
        "k": k, "input_planes": args.cnn_inputs, "training_loss": loss_mode,
        "res_loss_eval_mean": float(np.mean(lr_cnn)),
        "pca_k%d_res_loss_eval_mean" % args.k: float(np.mean(lr_pca)),
        "proj_loss_eval_mean": float(np.mean(lp_cnn)),
        "eim_field_alone_proj_loss_eval_mean": None if lp_eim is None else float(np.mean(lp_eim)),
        "pca_k%d_proj_loss_eval_mean" % args.k: float(np.mean(lp_pca)),
        "train_samples": len(train), "train_steps": args.cnn_steps, "batch": 32,
        "train_seconds": round(t_cnn_train, 1),
        "train_loss_first_last": [float(losses[0]), float(np.mean(losses[-20:]))],
        "inference_ms_batch": round(inf_ms, 3),
        "setup_ms_batch_incl_eim": round(setup_ms, 3),
        "inference_tflops": round(flops / (inf_ms * 1e-3) / 1e12, 1),
        "inference_mfma_frac_bf16": round(flops / (inf_ms * 1e-3) / 1e12 / 2500.0, 4),
        "flop_per_instance": flops // B,
    }
    log(f"CNN-augmented ({loss_mode}): {out['solves_per_s_incl_inference']:.3f} solves/s, iters mean "
        f"{it.mean():.0f}, l_proj eval {out['proj_loss_eval_mean']:.3f} "
        f"(PCA k={args.k}: {out['pca_k%d_proj_loss_eval_mean' % args.k]:.3f}), inference "
        f"{inf_ms:.2f} ms for {B} ({out['inference_tflops']} TFLOP/s)")
    return out


def cnn_kernels_only(args, torch, W):
    """Forward and training-step throughput of the predictor's kernels on
    480 x 240 grating permittivities (weights at their seeded initialisation,
    seeded random targets): the workload the MFMA-utilisation profile covers."""
    from paper_1902_00090_amd import Cnn
    insts = W.trajectory_dataset(2, 32)
    eps = torch.tensor(np.stack([i.eps for i in insts]), device="cuda")
    B, D = eps.shape[0], insts[0].D
    net = Cnn(insts[0].nx, insts[0].ny, max_batch=B, k=args.cnn_k, seed=7,
              in_channels=args.cnn_inputs)
    rng = np.random.default_rng(5)
    tgt = torch.tensor(W.random_complex(rng, (32, args.cnn_k, D)).astype(np.complex64),
                       device="cuda")
    eim = None
    if args.cnn_inputs == 3:
        eim = torch.tensor(W.random_complex(rng, (B, D)).astype(np.complex64), device="cuda")
    U = torch.empty((B, args.cnn_k, D), dtype=torch.complex64, device="cuda")
    n = args.cnn_kernels
    e32 = None if eim is None else eim[:32].contiguous()
    net.predict(eps, U, eim=eim)
    net.train_step(eps[:32].contiguous(), tgt, eim=e32)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    for _ in range(n):
        net.predict(eps, U, eim=eim)
    e[1].record()
    e1 = eps[:32].contiguous()
    e[2].record()
    for _ in range(n):
        net.train_step(e1, tgt, lr=1e-4, eim=e32)
    e[3].record()
    torch.cuda.synchronize()
    fwd_ms, tr_ms = e[0].elapsed_time(e[1]) / n, e[2].elapsed_time(e[3]) / n
    # residual-loss step: the operators and right-hand sides of the 32 images
    from paper_1902_00090_amd import FdfdOp
    ops = [FdfdOp.from_instance(i) for i in insts[:32]]
    bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in insts[:32]]
    net.train_step_res(e1, ops, bs, lr=1e-4, eim=e32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        net.train_step_res(e1, ops, bs, lr=1e-4, eim=e32)
    torch.cuda.synchronize()
    res_ms = (time.perf_counter() - t0) * 1e3 / n
    f1 = cnn_flops_per_instance(net)
    out = {"metric": "CNN predictor kernels, 480x240, 1 GPU",
           "forward_ms_batch64": round(fwd_ms, 3),
           "forward_tflops": round(f1 * B / (fwd_ms * 1e-3) / 1e12, 1),
           "train_step_ms_batch32": round(tr_ms, 3),
           "train_tflops_3x_forward": round(3 * f1 * 32 / (tr_ms * 1e-3) / 1e12, 1),
           "train_step_res_ms_batch32": round(res_ms, 3),
           "bf16_dense_peak_tflops": 2500.0, "flop_per_instance_forward": f1, "reps": n,
           "input_planes": args.cnn_inputs}
    net.close()
    print(json.dumps(out), flush=True)


def single_leg(args, torch, ops, bs, U):
    """The first evaluation problem solved alone (the single-solve
    configuration): plain and PCA-augmented GMRES(100), step groups replayed
    as HIP graphs."""
    from paper_1902_00090_amd import Solver
    out = {}
    for aug in (False, True):
        s = Solver([ops[0]], restart=args.restart, kmax=args.k if aug else 0,
                   cgs_passes=args.cgs, use_graph=True)
        if aug:
            s.set_subspace([U])
        s.solve([bs[0]], tol=args.tol, maxit=args.maxit)       # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.time()
        _, (inf,), _ = s.solve([bs[0]], tol=args.tol, maxit=args.maxit)
        torch.cuda.synchronize()
        dt = time.time() - t0
        s.close()
        out["augmented" if aug else "plain"] = {
            "seconds": round(dt, 3), "iters": inf["iters"],
            "us_per_iter": round(1e6 * dt / max(1, inf["iters"]), 1),
            "converged": inf["status"] == 0}
    log(f"single problem: {out}")
    return out


def precond_leg(args, torch, ops, bs, U):
    """The evaluation batch with the supplement's diagonal preconditioners
    (Jacobi; PML grid-spacing scaling), without and with the PCA basis."""
    from paper_1902_00090_amd import Solver
    B = len(ops)
    out = {}
    for kind in ("jacobi", "pml"):
        for aug in (False, True):
            s = Solver(ops, restart=args.restart, kmax=args.k if aug else 0, cgs_passes=args.cgs,
                       hist_cap=args.maxit, precond=kind)
            if aug:
                s.set_subspace([U] * B)
            torch.cuda.synchronize()
            t0 = time.time()
            _, inf, _ = s.solve(bs, tol=args.tol, maxit=args.maxit)
            torch.cuda.synchronize()
            dt = time.time() - t0
            h = [s.history(p) for p in range(B)]
            s.close()
            key = kind + ("+pca" if aug else "")
            out[key] = {
                "solves_per_s": round(B / dt, 4),
                "iters_mean": float(np.mean([i["iters"] for i in inf])),
                "all_converged": all(i["status"] == 0 for i in inf),
                "worst_rel_res_true": max(i["rel_res_true"] for i in inf),
                "precond_rel_res_after_1_iter_mean": float(np.mean([x[0] for x in h])),
            }
            log(f"precond {key}: {out[key]}")
    return out


def recycle_leg(args, torch, data):
    """Design steps 0..N-1 of every benchmark trajectory, one lockstep batch per
    step: augmented by the fields of the previous steps of the same trajectory,
    against plain GMRES on the same schedule."""
    from paper_1902_00090_amd.recycle import solve_trajectories
    S = args.traj_steps
    trajs = [data[t * S:t * S + args.recycle] for t in range(args.traj)]
    out = {}
    for mode in ("recycled", "plain"):
        torch.cuda.synchronize()
        t0 = time.time()
        _, inf, hist = solve_trajectories(trajs, window=args.recycle_window, tol=args.tol,
                                          restart=args.restart, maxit=args.maxit,
                                          cgs_passes=args.cgs, recycle=(mode == "recycled"),
                                          hist_cap=args.maxit)
        torch.cuda.synchronize()
        dt = time.time() - t0
        later = [(t, s) for t in range(len(trajs)) for s in range(1, args.recycle)]
        out[mode] = {
            "seconds": round(dt, 2),
            "solves_per_s": round(len(trajs) * args.recycle / dt, 4),
            "iters_mean_steps_ge_1": float(np.mean([inf[t][s]["iters"] for t, s in later])),
            "rel_res_after_1_iter_mean_steps_ge_1": float(np.mean([hist[t][s][0] for t, s in later])),
            "iters_to_0.04_mean_steps_ge_1": float(np.mean(
                [first_below(hist[t][s], 0.04) or np.nan for t, s in later])),
            "all_converged": all(i["status"] == 0 for row in inf for i in row),
        }
        log(f"trajectory {mode}: {dt:.1f}s, {out[mode]}")
    out["steps"] = args.recycle
    out["window"] = args.recycle_window
    return out


def uneven_leg(args, torch, W):
    """8 trajectories x 32 steps of uneven grids (192x96, 320x160, 480x240;
    1.30 / 1.55 um) in one lockstep batch, plain complex64 GMRES, step groups
    replayed as HIP graphs."""
    from paper_1902_00090_amd import FdfdOp, Solver
    insts = W.correlated_batch(8, 32)
    ops = [FdfdOp.from_instance(i) for i in insts]
    bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in insts]
    xs = [torch.empty_like(b) for b in bs]
    s = Solver(ops, restart=args.restart, cgs_passes=args.cgs, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.time()
    _, inf, st = s.solve(bs, tol=args.tol, maxit=args.maxit, x=xs)
    torch.cuda.synchronize()
    dt = time.time() - t0
    s.close()
    it = np.array([i["iters"] for i in inf])
    mv = sum(i["matvecs"] for i in inf)
    cells = sum(i.D for i in insts)
    alg = sum(arnoldi_bytes(p.D, i["iters"], args.restart, 0, args.cgs) + 52 * p.D * i["restarts"]
              for i, p in zip(inf, insts))
    out = {
        "problems": len(insts), "cells": cells, "solves_per_s": round(len(insts) / dt, 4),
        "seconds": round(dt, 2), "matvecs_per_s": round(mv / dt, 1),
        "cell_matvecs_per_s": round(sum(i["matvecs"] * p.D for i, p in zip(inf, insts)) / dt, 1),
        "iters_min_mean_max": [int(it.min()), float(it.mean()), int(it.max())],
        "all_converged": all(i["status"] == 0 for i in inf),
        "worst_rel_res_true": max(i["rel_res_true"] for i in inf),
        "algorithmic_GB_per_s_whole_solve": round(alg / dt / 1e9, 1),
        "hbm_frac_whole_solve": round(alg / dt / 1e9 / HBM_PEAK_GBS, 4),
    }
    log(f"uneven batch: {len(insts)} problems, {cells} cells, {dt:.1f}s, iters "
        f"{out['iters_min_mean_max']}, {out['algorithmic_GB_per_s_whole_solve']} GB/s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--k", type=int, default=20)
    ap.add_argument("--traj", type=int, default=8)
    ap.add_argument("--traj-steps", type=int, default=32)
    ap.add_argument("--restart", type=int, default=100)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--train-tol", type=float, default=1e-4)
    ap.add_argument("--maxit", type=int, default=30000)
    ap.add_argument("--cgs", type=int, default=1, help="Gram-Schmidt passes (1 or 2)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=400)
    ap.add_argument("--oracle-check", type=int, default=2)
    ap.add_argument("--no-cnn", action="store_true", help="skip the CNN-predictor leg")
    ap.add_argument("--cnn-k", type=int, default=10)
    ap.add_argument("--cnn-steps", type=int, default=400)
    ap.add_argument("--cnn-window", type=int, default=8)
    ap.add_argument("--cnn-loss", default="both", choices=("proj", "res", "both"),
                    help="CNN training loss: local-PCA targets (MSE, projection), the "
                         "unsupervised residual loss, or one leg each")
    ap.add_argument("--cnn-inputs", type=int, default=3, choices=(1, 3),
                    help="CNN input planes: 3 = permittivity + effective-index field (the "
                         "paper's input), 1 = permittivity only")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven correlated batch")
    ap.add_argument("--recycle", type=int, default=0,
                    help="also run trajectory recycling over the first N design steps of "
                         "every trajectory (augment step s by the fields of steps < s)")
    ap.add_argument("--recycle-window", type=int, default=5)
    ap.add_argument("--precond", action="store_true",
                    help="also solve the evaluation batch with the Jacobi and PML-scaling "
                         "diagonal preconditioners, plain and PCA-augmented")
    ap.add_argument("--cnn-kernels", type=int, default=0,
                    help="only time N CNN forward passes (batch 64) and N training steps "
                         "(batch 32) at 480x240, print one JSON line and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB of a plain device-to-device copy run first (for HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the problems of a batch are independent and would be split across GPUs "
              "with no communication during the solve)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1902_00090_amd import FdfdOp, Solver, pca_build

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = "cuda"
    if args.calibrate_copy > 0:
        # a copy kernel of known size: its FETCH_SIZE / WRITE_SIZE readings
        # calibrate the counters of the solver's sweeps
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_copy} MiB read + {args.calibrate_copy} MiB written")
        del src, dst

    if args.cnn_kernels > 0:
        cnn_kernels_only(args, torch, W)
        return

    # ---------------- data
    t0 = time.time()
    data = W.trajectory_dataset(args.traj, args.traj_steps)
    tr_idx, te_idx = W.split_train_test(len(data))
    train = [data[i] for i in tr_idx]
    test = [data[i] for i in te_idx][:args.batch]
    B = len(test)
    log(f"data: {len(data)} problems ({len(train)} train / {len(te_idx)} eval), "
        f"{time.time() - t0:.1f}s")

    # ---------------- predictor training: solve the training set on the GPU, PCA
    t0 = time.time()
    snaps = []
    chunk = 64
    for c0 in range(0, len(train), chunk):
        part = train[c0:c0 + chunk]
        ops = [FdfdOp.from_instance(i) for i in part]
        bs = [torch.tensor(i.b, dtype=torch.complex128, device=dev) for i in part]
        s = Solver(ops, restart=args.restart, cgs_passes=args.cgs)
        xs, infos, st = s.solve(bs, tol=args.train_tol, maxit=args.maxit)
        snaps.extend(x.to(torch.complex64) for x in xs)
        s.close()
        log(f"  train solves {c0 + len(part)}/{len(train)}: "
            f"iters max {max(i['iters'] for i in infos)}")
    Smat = torch.stack(snaps).contiguous()
    del snaps
    U, sig = pca_build(Smat, args.k)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    log(f"PCA: k={args.k} from {len(train)} solver-generated fields, {t_train:.1f}s; "
        f"sigma[0]={sig[0]:.3e} sigma[k-1]/sigma[0]={sig[-1] / sig[0]:.3f}")

    # ---------------- evaluation batch (inputs resident in HBM)
    ops = [FdfdOp.from_instance(i) for i in test]
    bs = [torch.tensor(i.b, dtype=torch.complex128, device=dev) for i in test]
    xs = [torch.empty_like(b) for b in bs]
    Ulist = [U] * B
    aug = Solver(ops, restart=args.restart, kmax=args.k, cgs_passes=args.cgs,
                 hist_cap=args.maxit)

    def step():
        aug.set_subspace(Ulist)
        return aug.solve(bs, tol=args.tol, maxit=args.maxit, x=xs)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    aug.profile(True)
    infos = None
    t0 = time.time()
    for _ in range(args.steps):
        _, infos, st = step()
    torch.cuda.synchronize()
    dt = time.time() - t0
    ks = aug.kernel_stats()
    aug.profile(False)
    ms_per_step = 1000.0 * dt / args.steps
    value = B * args.steps / dt
    conv = all(i["status"] == 0 for i in infos)
    worst = max(i["rel_res_true"] for i in infos)
    it_aug = np.array([i["iters"] for i in infos])
    mv_aug = np.array([i["matvecs"] for i in infos])
    h_aug = [aug.history(p) for p in range(B)]
    r1_aug = float(np.mean([h[0] for h in h_aug]))
    th_aug = [first_below(h, 0.04) for h in h_aug]
    log(f"augmented: {value:.3f} solves/s, {ms_per_step:.0f} ms/step, iters mean "
        f"{it_aug.mean():.0f}, all converged {conv}, worst rel res {worst:.2e}")

    # ---------------- plain GMRES on the same batch
    plain = None
    if not args.no_plain:
        ps = Solver(ops, restart=args.restart, cgs_passes=args.cgs, hist_cap=args.maxit)
        xp = [torch.empty_like(b) for b in bs]
        torch.cuda.synchronize()
        t0 = time.time()
        _, pinf, pst = ps.solve(bs, tol=args.tol, maxit=args.maxit, x=xp)
        torch.cuda.synchronize()
        dtp = time.time() - t0
        h_pl = [ps.history(p) for p in range(B)]
        it_pl = np.array([i["iters"] for i in pinf])
        plain = {
            "solves_per_s": B / dtp, "ms_per_batch": 1000 * dtp,
            "iters_mean": float(it_pl.mean()), "matvecs_mean": float(np.mean([i["matvecs"] for i in pinf])),
            "all_converged": all(i["status"] == 0 for i in pinf),
            "rel_res_after_1_iter_mean": float(np.mean([h[0] for h in h_pl])),
            "iters_to_0.04_mean": float(np.mean([first_below(h, 0.04) or np.nan for h in h_pl])),
        }
        ps.close()
        log(f"plain: {plain['solves_per_s']:.3f} solves/s, iters mean {plain['iters_mean']:.0f}")

    # ---------------- one problem alone (latency-bound), plain and augmented
    single = single_leg(args, torch, ops, bs, U)

    # ---------------- error vs the FP64 oracle (sparse LU) on a subset
    errs = []
    t_lu = []
    if args.oracle_check > 0:
        from oracle import direct, fdfd
        for p in range(min(args.oracle_check, B)):
            A = fdfd.assemble_instance(test[p])
            t0 = time.time()
            xstar = direct.sparse_solve(A, test[p].b)
            t_lu.append(time.time() - t0)
            xg = xs[p].cpu().numpy()
            errs.append(float(np.linalg.norm(xg - xstar) / np.linalg.norm(xstar)))
        log(f"error vs sparse LU on {len(errs)} problems: {errs}")

    # ---------------- CNN predictor: trained on the same solver-generated fields
    cnn = None
    if not args.no_cnn:
        modes = ("proj", "res") if args.cnn_loss == "both" else (args.cnn_loss,)
        cnn = {m: cnn_leg(args, torch, W, data, tr_idx, train, test, Smat, ops, bs, xs, U,
                          it_aug, plain, m) for m in modes}
    del Smat

    # ---------------- diagonal preconditioners (optional)
    pre = None
    if args.precond:
        pre = precond_leg(args, torch, ops, bs, U)

    # ---------------- trajectory recycling (optional)
    rec = None
    if args.recycle > 0:
        rec = recycle_leg(args, torch, data)

    # ---------------- uneven correlated batch, plain GMRES, graph replay
    uneven = None
    if not args.no_uneven:
        uneven = uneven_leg(args, torch, W)

    # ---------------- roofline of the dominant sweep
    name = max(ks, key=lambda n: ks[n][0])
    ms_k, launches_k, bytes_k = ks[name]
    achieved = bytes_k / (ms_k * 1e-3) / 1e9 if ms_k > 0 else 0.0
    kname = {"matvec_dots": "k_matvec_dot", "second_pass": "k_update_dot",
             "update_norm": "k_update_norm"}[name]
    traffic = None
    if (kname in MEASURED_TRAFFIC["bytes_per_launch"] and args.batch == 64 and args.k == 20
            and args.cgs == 1 and kernel_sources_hash() == MEASURED_TRAFFIC["sources_sha256_16"]):
        traffic = MEASURED_TRAFFIC["bytes_per_launch"][kname]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kname,
                "avg_launch_us": round(1000 * ms_k / max(1, launches_k), 2),
                "launches": int(launches_k),
                "algorithmic_bytes_per_launch": round(bytes_k / max(1, launches_k))}
    sweeps = {n: {"ms": round(v[0], 2), "launches": int(v[1]),
                  "GB_per_s": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else None}
              for n, v in ks.items()}

    # ---------------- CPU baseline: the oracle's augmented GMRES, bounded sample
    cpu = None
    if not args.no_cpu:
        from threadpoolctl import threadpool_limits
        from oracle import fdfd, gmres_aug
        inst = test[0]
        A = fdfd.assemble_instance(inst)
        V = U.cpu().numpy().T.astype(np.complex128)
        def sample(threads):
            with threadpool_limits(limits=threads):
                t0 = time.time()
                gmres_aug.gmres_aug(A, inst.b, V, restart=args.restart, tol=0.0,
                                    maxit=args.cpu_iters)
                return time.time() - t0
        tc = sample(1)
        t_iter = tc / args.cpu_iters
        # threads for the multi-threaded sample: the process's CPU share (the
        # OpenMP setting if there is one), not every core of the host
        nthr = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
        ncpu = os.cpu_count() or 1
        tc_all = sample(nthr)
        cpu = {"value": round(1.0 / (t_iter * float(it_aug.mean())), 6), "unit": "solves/s",
               "cores": 1, "kind": "oracle",
               "sample": f"oracle gmres_aug (complex128, numpy/scipy, 1 BLAS thread) on one "
                         f"evaluation problem for {args.cpu_iters} Arnoldi steps ({tc:.1f}s, "
                         f"{1000 * t_iter:.0f} ms/step incl. setup), scaled to the mean "
                         f"{it_aug.mean():.0f} steps the GPU needed per solve",
               "host_cpu_count": ncpu,
               "all_threads": {"value": round(args.cpu_iters / (tc_all * float(it_aug.mean())), 6),
                               "threads": nthr, "sample_seconds": round(tc_all, 2)},
               "sparse_lu_seconds_per_problem": (round(float(np.mean(t_lu)), 3) if t_lu
                                                 else None)}
        log(f"cpu baseline: {cpu['value']:.2e} solves/s ({tc:.1f}s sample); "
            f"{nthr} threads: {cpu['all_threads']['value']:.2e} solves/s")

    out = {
        "metric": "solves/s and matvecs to 1e-6 rel. residual: augmented vs plain GMRES, 1 GPU",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {
            "workload": f"PCA-augmented GMRES({args.restart}) on {B} evaluation problems "
                        f"(480x240 grating designs from {args.traj} synthetic design "
                        f"trajectories x {args.traj_steps} steps, 75/25 split), k={args.k}, "
                        f"tol {args.tol:g}, complex64 inner iteration with FP64 true-residual "
                        f"restarts, {args.cgs} Gram-Schmidt pass(es)",
            "batch": B, "grid": "480x240", "restart": args.restart, "k": args.k,
            "tol": args.tol, "pca_train_problems": len(train),
            "pca_train_seconds": round(t_train, 1),
        },
        "augmented": {
            "solves_per_s": round(value, 4), "iters_mean": float(it_aug.mean()),
            "matvecs_mean": float(mv_aug.mean()), "all_converged": conv,
            "worst_rel_res_true": worst,
            "rel_res_after_1_iter_mean": r1_aug,
            "iters_to_0.04_mean": float(np.mean([t or np.nan for t in th_aug])),
            "error_vs_sparse_lu": errs,
        },
        "plain": plain,
        "speedup_wallclock": round(value / plain["solves_per_s"], 3) if plain else None,
        "sweeps": sweeps,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "single_problem": single,
        "cnn_augmented": cnn,
        "uneven_batch_plain": uneven,
        "trajectory_recycling": rec,
        "diagonal_preconditioners": pre,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
