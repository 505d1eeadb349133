"""Benchmark: solves/s and matvecs to 1e-6 relative residual, data-driven
(PCA-augmented) vs plain GMRES, one MI355X.

Workload (the PCA-augmented configuration, C4):
  * predictor training, outside the timed region: 2000 fresh 480 x 240
    grating instances (dx 25 nm, lambda 1.30 um, 20-cell PML; seeds 10,000+i)
    are solved by this library's GPU solver (to a relative residual of 1e-2:
    the principal components only need the fields' dominant content); their
    fields form the snapshot matrix and pca_build returns the top k = 20
    principal components;
  * test set: 500 fresh instances of the same distribution (seeds 20,000+i),
    resident in HBM before timing;
  * one timed step = one batch of B = 25 test instances (the steps walk
    round-robin through the 500, so 20 steps cover all of them): the
    augmentation setup (A V, Cholesky QR twice) and augmented GMRES(100) in
    complex64 with FP64 true-residual restarts.  Each solve runs past
    ||b - A x|| / ||b|| = 1e-6 to the refined tolerance tol_acc (2e-7 by
    default) at which the error against the FP64 oracle is guaranteed below
    1e-5 (||x - x*|| / ||x*|| <= ||A^-1|| ||b|| / ||x*|| * rel. residual, a
    factor of about 40 on these problems, estimated on the CPU);
  * plain GMRES(100) on the same batches, and both methods again at 1e-6
    exactly, for the comparison;
  * the small binary-pixel problem (C1, 64 x 64, GMRES(50), complex128,
    tol 1e-8) and the single grating solve (C2, seed 1000, GMRES(100),
    complex64 + FP64 restarts, tol 1e-6 and tol_acc) beside their oracle
    figures.
Optional legs (flags): the CNN predictor, diagonal preconditioners,
trajectory recycling and the uneven correlated batch.

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

# HBM bytes per launch of the dominant sweep from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE, calibrated on a 1 GiB device copy) over this
# workload, as recorded in the profile summary beside the commands that took
# them; valid only for the kernel sources and batch they were taken with.
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_matvec_dot_pca_c4_480x240_b25.md")


def measured_traffic():
    import json
    try:
        with open(TRAFFIC_PROFILE) as fh:
            for line in fh:
                if line.startswith("traffic-record:"):
                    return json.loads(line.split(":", 1)[1])
    except OSError:
        pass
    return None


def _function_text(src, head):
    """The text of the function whose definition starts at `head` (its
    template line included), up to its closing brace at column 0."""
    a = src.index(head)
    a = src.rfind("template <", 0, a) if "template <" in src[max(0, a - 80):a] else a
    return src[a:src.index("\n}\n", a) + 3]


def kernel_sources_hash():
    """First 16 hex digits of the SHA-256 of the dominant sweep's own source:
    k_matvec_dot and block_dots (csrc/solver_kernels.h) and the headers they
    build on (csrc/op.h, csrc/common.h)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1902_00090_amd", "csrc")
    with open(os.path.join(csrc, "solver_kernels.h")) as fh:
        src = fh.read()
    for head in ("__device__ __forceinline__ void block_dots(",
                 "__global__ __launch_bounds__(DD_BLOCK) void k_matvec_dot("):
        h.update(_function_text(src, head).encode())
    for f in ("op.h", "common.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def first_below(h, thr):
    idx = np.nonzero(np.asarray(h) <= thr)[0]
    return int(idx[0]) + 1 if len(idx) else None


def arnoldi_bytes(D, iters, m, k, passes=1, fused=False):
    """Algorithmic HBM bytes of `iters` complex64 Arnoldi steps with restart m
    and k augmenting vectors.  One sweep per step (fused, one Gram-Schmidt
    pass): step j reads the k+j+1 basis vectors and A q_j, writes q_{j+1} and
    A q_{j+1}, and reads eps: 8 D (k+j+1) + 28 D.  Two sweeps: the stencil
    input, eps and w (20 D), the basis and w for the dots and again for the
    update, and q_{j+1}: 16 D (k+j) + 44 D; each further Gram-Schmidt pass
    adds 16 D (k+j) + 24 D."""
    full, rem = divmod(int(iters), m)
    def cyc(n):       # sum over j < n of (k + j)
        return n * k + n * (n - 1) // 2
    sj = full * cyc(m) + cyc(rem)
    if fused and passes == 1:
        return 8 * D * sj + 36 * D * iters
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


SRC_IX = 30     # the grating's mode source column (npml + 10)


def _grating_parts(seed):
    """(eps, source column of b) of one grating instance: b is zero outside
    that column, so only the column crosses the process boundary."""
    import workloads as W
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):        # one BLAS thread per worker process
        inst = W.grating(seed)
    b = inst.b.reshape(inst.ny, inst.nx)
    assert np.count_nonzero(b[:, np.arange(inst.nx) != SRC_IX]) == 0
    return inst.eps, b[:, SRC_IX].copy(), inst.name


def make_instances(seeds, workers):
    """Grating instances for the seeds, generated in a process pool (before
    the GPU is touched: the pool forks this process)."""
    import workloads as W
    seeds = list(seeds)
    if workers <= 1 or len(seeds) < 8:
        parts = [_grating_parts(s) for s in seeds]
    else:
        import multiprocessing as mp
        # close + join lets the workers exit normally (a pool's context exit
        # terminates them with SIGTERM, which profilers' signal handlers catch)
        pool = mp.get_context("fork").Pool(workers)
        try:
            parts = pool.map(_grating_parts, seeds, chunksize=16)
        finally:
            pool.close()
            pool.join()
    out = []
    for eps, col, name in parts:
        ny, nx = eps.shape
        b = np.zeros((ny, nx), np.complex128)
        b[:, SRC_IX] = col
        out.append(W.Instance(eps, b.reshape(-1), nx, ny, 0.025, 1.30, 20, name=name))
    return out


def oracle_reference(inst):
    """FP64 sparse LU solution x* of one instance and the factor that turns a
    relative residual into a bound on the relative error: ||A^-1||_2 ||b|| /
    ||x*|| (||A^-1||_2 by 30 power steps on A^-H A^-1), plus a 1-norm
    condition estimate (scipy onenormest)."""
    import scipy.sparse.linalg as spla
    from oracle import fdfd
    A = fdfd.assemble_instance(inst).tocsc()
    t0 = time.time()
    lu = spla.splu(A)
    x = lu.solve(inst.b)
    t_lu = time.time() - t0
    v = np.random.default_rng(0).standard_normal(A.shape[0]) + 0j
    s = 1.0
    for _ in range(30):
        v = lu.solve(lu.solve(v), trans="H")
        s = np.linalg.norm(v)
        v /= s
    ainv2 = math.sqrt(s)
    Ainv = spla.LinearOperator(A.shape, matvec=lu.solve,
                               rmatvec=lambda y: lu.solve(y, trans="H"), dtype=complex)
    kappa1 = float(spla.onenormest(A) * spla.onenormest(Ainv))
    return {"x": x, "lu_seconds": t_lu, "err_factor": ainv2 * np.linalg.norm(inst.b) / np.linalg.norm(x),
            "kappa_1": kappa1, "A": A}


def rel_err(x, xstar):
    return float(np.linalg.norm(x - xstar) / np.linalg.norm(xstar))


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
    """Two C4 test batches with the supplement's diagonal preconditioners
    (Jacobi; PML grid-spacing scaling), without and with the PCA basis, to
    args.tol."""
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


def recycle_leg(args, torch, W):
    """Trajectory recycling on the correlated batch (8 trajectories of uneven
    grids 192x96 / 320x160 / 480x240 and wavelengths 1.30 / 1.55 um, design
    steps 0..N-1), one lockstep batch per step: plain GMRES, augmentation by
    the fields of the previous steps, by the harmonic Ritz vectors of the
    previous step's last cycle, and by both."""
    from paper_1902_00090_amd.recycle import solve_trajectories
    S = args.traj_steps
    flat = W.correlated_batch(args.traj, S)
    trajs = [flat[t * S:t * S + args.recycle] for t in range(args.traj)]
    modes = {"plain": dict(recycle=False, ritz=0),
             "solutions": dict(recycle=True, ritz=0),
             "harmonic_ritz": dict(recycle=False, ritz=args.recycle_ritz),
             "solutions+harmonic_ritz": dict(recycle=True, ritz=args.recycle_ritz)}
    out = {}
    refs = None
    for mode, kw in modes.items():
        torch.cuda.synchronize()
        t0 = time.time()
        xs, inf, hist, _ = solve_trajectories(trajs, window=args.recycle_window, tol=args.tol,
                                              restart=args.restart, maxit=args.maxit,
                                              cgs_passes=args.cgs, hist_cap=args.maxit, **kw)
        torch.cuda.synchronize()
        dt = time.time() - t0
        later = [(t, s) for t in range(len(trajs)) for s in range(1, args.recycle)]
        allp = [(t, s) for t in range(len(trajs)) for s in range(args.recycle)]
        if refs is None:
            # errors against the oracle's sparse LU on the last step of two trajectories
            refs = {(t, args.recycle - 1): oracle_reference(trajs[t][-1]) for t in (0, 2)}
        out[mode] = {
            "seconds": round(dt, 2),
            "solves_per_s": round(len(allp) / dt, 4),
            "iters_total": int(sum(inf[t][s]["iters"] for t, s in allp)),
            "iters_mean_steps_ge_1": float(np.mean([inf[t][s]["iters"] for t, s in later])),
            "iters_to_1e-6_mean_steps_ge_1": float(np.mean(
                [first_below(hist[t][s], 1e-6) or np.nan for t, s in later])),
            "rel_res_after_1_iter_mean_steps_ge_1": float(np.mean([hist[t][s][0] for t, s in later])),
            "iters_to_0.04_mean_steps_ge_1": float(np.mean(
                [first_below(hist[t][s], 0.04) or np.nan for t, s in later])),
            "all_converged": all(i["status"] == 0 for row in inf for i in row),
            "error_vs_sparse_lu": {f"traj{t}_step{s}": rel_err(xs[t][s].cpu().numpy(), r["x"])
                                   for (t, s), r in refs.items()},
        }
        log(f"trajectory {mode}: {dt:.1f}s, {out[mode]}")
    out["steps"] = args.recycle
    out["trajectories"] = len(trajs)
    out["window"] = args.recycle_window
    out["ritz"] = args.recycle_ritz
    return out


def c4_recycle_leg(args, torch, test, U):
    """Harmonic Ritz recycling across the C4 test batches: batch s + 1 of the
    fresh instances is augmented by the harmonic Ritz vectors of batch s's
    last cycles (problem t of one batch passes its vectors to problem t of the
    next), with and without the PCA basis, against plain and PCA-only on the
    same batches (all to args.tol_acc)."""
    from paper_1902_00090_amd.recycle import solve_trajectories
    B, S = args.batch, args.c4_recycle
    trajs = [[test[s * B + t] for s in range(S)] for t in range(B)]
    modes = {"plain": dict(recycle=False, ritz=0), "pca": dict(recycle=False, ritz=0, base=U),
             "harmonic_ritz": dict(recycle=False, ritz=args.recycle_ritz),
             "pca+harmonic_ritz": dict(recycle=False, ritz=args.recycle_ritz, base=U)}
    out = {"batches": S, "batch": B, "ritz": args.recycle_ritz}
    for mode, kw in modes.items():
        torch.cuda.synchronize()
        t0 = time.time()
        _, inf, hist, _ = solve_trajectories(trajs, tol=args.tol_acc, restart=args.restart,
                                             maxit=args.maxit, cgs_passes=args.cgs,
                                             hist_cap=args.maxit, **kw)
        torch.cuda.synchronize()
        dt = time.time() - t0
        later = [(t, s) for t in range(B) for s in range(1, S)]
        out[mode] = {"seconds": round(dt, 2), "solves_per_s": round(B * S / dt, 4),
                     "iters_mean_batches_ge_1": float(np.mean([inf[t][s]["iters"] for t, s in later])),
                     "iters_to_1e-6_mean_batches_ge_1": float(np.mean(
                         [first_below(hist[t][s], 1e-6) or np.nan for t, s in later])),
                     "all_converged": all(i["status"] == 0 for row in inf for i in row)}
        log(f"C4 recycling {mode}: {out[mode]}")
    return out


def uneven_leg(args, torch, W):
    """8 trajectories x 32 steps of uneven grids (192x96, 320x160, 480x240;
    1.30 / 1.55 um) in one lockstep batch, plain complex64 GMRES to tol_acc,
    step groups replayed as HIP graphs."""
    from paper_1902_00090_amd import FdfdOp, Solver
    insts = W.correlated_batch(8, 32)
    ops = [FdfdOp.from_instance(i) for i in insts]
    bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in insts]
    xs = [torch.empty_like(b) for b in bs]
    s = Solver(ops, restart=args.restart, cgs_passes=args.cgs, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.time()
    # to tol_acc, where the error bound meets 1e-5 (as the headline)
    _, inf, st = s.solve(bs, tol=args.tol_acc, maxit=args.maxit, x=xs)
    torch.cuda.synchronize()
    dt = time.time() - t0
    s.close()
    it = np.array([i["iters"] for i in inf])
    mv = sum(i["matvecs"] for i in inf)
    cells = sum(i.D for i in insts)
    # error against the oracle's sparse LU on one problem of each grid size
    errs = {}
    for p, inst in enumerate(insts):
        key = f"{inst.nx}x{inst.ny}"
        if key not in errs:
            errs[key] = rel_err(xs[p].cpu().numpy(), oracle_reference(inst)["x"])
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
        "error_vs_sparse_lu": errs,
    }
    log(f"uneven batch: {len(insts)} problems, {cells} cells, {dt:.1f}s, iters "
        f"{out['iters_min_mean_max']}, {out['algorithmic_GB_per_s_whole_solve']} GB/s")
    return out


def _traj_parts(t, steps):
    """(eps, source column) of every step of CNN training trajectory t (seeds
    40,000 + t for the design, 400,000 + 100 t + s for the steps)."""
    import workloads as W
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        tr = W.trajectory(W.CNN_TRAJ_SEED0 + t, W.CNN_STEP_SEED0 + 100 * t, steps, 480, 240, 1.30)
    out = []
    for inst in tr:
        b = inst.b.reshape(inst.ny, inst.nx)
        out.append((inst.eps, b[:, SRC_IX].copy()))
    return out


def c5_leg(args, torch, W):
    """The CNN predictor at its stated scale: 313 design trajectories of 32
    steps (10,016 samples) solved by the library's GPU solver (each step
    augmented by the trajectory's previous solutions, to a relative residual
    of args.c5_train_tol), local-PCA targets (k = 10, window 8), 10,000 Adam
    steps at batch 32 on the permittivity alone (1 input plane), the network
    saved with its Adam state; then inference on 256 fresh gratings (seeds
    50,000 + i) and CNN-augmented GMRES against plain and PCA-augmented GMRES
    (k = 20 components of 2000 of the training fields) on the same batches."""
    import multiprocessing as mp
    from paper_1902_00090_amd import (Cnn, DDError, FdfdOp, Solver, eim_field, local_pca_targets,
                                      pca_build, proj_loss_batched)
    from paper_1902_00090_amd.train import train_cnn, train_cnn_res
    T, S, k, D = args.c5_traj, args.c5_steps, args.cnn_k, 480 * 240
    N = T * S
    omega = 2 * math.pi / 1.30
    out = {"trajectories": T, "steps_per_trajectory": S, "samples": N, "k": k,
           "window": args.cnn_window, "adam_steps": args.c5_adam, "batch": 32,
           "input_planes": args.c5_inputs, "lr": args.c5_lr, "test_instances": args.c5_test}
    net = None
    if args.c5_load:
        net = Cnn.load(args.c5_load, max_batch=32)
        out["loaded"] = args.c5_load
    else:
        t0 = time.time()
        workers = args.workers or min(16, len(os.sched_getaffinity(0)))
        pool = mp.get_context("fork").Pool(workers)
        try:
            parts = pool.starmap(_traj_parts, [(t, S) for t in range(T)], chunksize=4)
        finally:
            pool.close()
            pool.join()
        eps_h = np.stack([e for tr in parts for e, _ in tr])            # [N, ny, nx]
        cols = np.stack([c for tr in parts for _, c in tr])             # [N, ny]
        del parts
        log(f"C5 data: {N} trajectory steps generated in {time.time() - t0:.1f}s")
        eps_d = torch.tensor(eps_h, device="cuda")
        res = args.c5_loss == "res"
        t_solve = t_tgt = 0.0
        its = []
        Upca = None
        if res:
            # unsupervised: each sample's own operator and right-hand side, no solved fields
            t0 = time.time()
            all_ops = [FdfdOp(eps_h[r], omega, 0.025, 20) for r in range(N)]
            ball = torch.zeros((N, 240, 480), dtype=torch.complex128, device="cuda")
            ball[:, :, SRC_IX] = torch.tensor(cols, device="cuda")
            all_b = [ball[r].reshape(-1) for r in range(N)]
            log(f"C5 operators: {time.time() - t0:.1f}s")
        else:
            F = torch.empty((N, D), dtype=torch.complex64, device="cuda")
            bmat = torch.zeros((T, 240, 480), dtype=torch.complex128, device="cuda")
            t0 = time.time()
            solver, its = None, []
            w = args.recycle_window
            for st in range(S):
                rows = [t * S + st for t in range(T)]
                ops = [FdfdOp(eps_h[r], omega, 0.025, 20) for r in rows]
                bmat[:, :, SRC_IX] = torch.tensor(cols[rows], device="cuda")
                bs = [bmat[t].reshape(-1) for t in range(T)]
                if solver is None:
                    solver = Solver(ops, restart=args.restart, kmax=w, cgs_passes=1)
                else:
                    solver.bind(ops)
                if st > 0:
                    solver.set_subspace([F[t * S + max(0, st - w):t * S + st] for t in range(T)])
                xs, infos, _ = solver.solve(bs, tol=args.c5_train_tol, maxit=args.maxit)
                for t, x in enumerate(xs):
                    F[t * S + st] = x.to(torch.complex64)
                its.extend(i["iters"] for i in infos)
                del xs
                log(f"  C5 training solves, step {st}: mean iters {np.mean([i['iters'] for i in infos]):.0f}, "
                    f"{time.time() - t0:.0f}s")
            solver.close()
            del bmat
            t_solve = time.time() - t0
            t0 = time.time()
            targets = torch.empty((N, k, D), dtype=torch.complex64, device="cuda")
            for t in range(T):
                targets[t * S:(t + 1) * S] = local_pca_targets(F[t * S:(t + 1) * S].contiguous(),
                                                               args.cnn_window, k)
            targets.mul_(float(math.sqrt(D)))                  # unit RMS per pixel
            torch.cuda.synchronize()
            t_tgt = time.time() - t0
            log(f"C5 targets: {t_tgt:.1f}s")
            # PCA basis of 2000 of the training fields, for the comparison leg
            sel = torch.as_tensor(np.random.default_rng(3).choice(N, size=min(2000, N), replace=False),
                                  device="cuda")
            Upca, _ = pca_build(F.index_select(0, sel).contiguous(), args.k)
            del F
        eim_tr = None
        if args.c5_inputs == 3:
            t0 = time.time()
            eim_tr = torch.empty((N, D), dtype=torch.complex64, device="cuda")
            bq = torch.zeros((64, 240, 480), dtype=torch.complex128, device="cuda")
            for c0 in range(0, N, 64):
                rows = list(range(c0, min(N, c0 + 64)))
                if res:
                    ops, bl = [all_ops[r] for r in rows], [all_b[r] for r in rows]
                else:
                    ops = [FdfdOp(eps_h[r], omega, 0.025, 20) for r in rows]
                    bq.zero_()
                    bq[:len(rows), :, SRC_IX] = torch.tensor(cols[rows], device="cuda")
                    bl = [bq[j].reshape(-1) for j in range(len(rows))]
                eim_field(ops, bl, out=eim_tr[c0:c0 + len(rows)])
            torch.cuda.synchronize()
            out["eim_seconds"] = round(time.time() - t0, 1)
            log(f"C5 effective-index fields: {out['eim_seconds']}s")
        t0 = time.time()
        net = Cnn(480, 240, max_batch=32, k=k, seed=7, in_channels=args.c5_inputs)
        if res:
            losses = train_cnn_res(net, eps_d, all_ops, all_b, args.c5_adam, 32, lr=args.c5_lr,
                                   seed=11, log=log, eim=eim_tr)
        else:
            losses = train_cnn(net, eps_d, targets, args.c5_adam, 32, lr=args.c5_lr, seed=11,
                               log=log, eim=eim_tr)
            del targets
        del eim_tr
        torch.cuda.synchronize()
        t_train = time.time() - t0
        del eps_d
        if res:
            del all_ops, all_b, ball
        if args.c5_save:
            net.save(args.c5_save)
        curve = [float(np.mean(losses[i:i + 500])) for i in range(0, len(losses), 500)]
        out.update({"training_loss": args.c5_loss,
                    "train_solve_tol": None if res else args.c5_train_tol,
                    "train_solve_seconds": round(t_solve, 1),
                    "train_solve_iters_mean": float(np.mean(its)) if its else None,
                    "targets_seconds": round(t_tgt, 1), "train_seconds": round(t_train, 1),
                    "ms_per_adam_step": round(1000 * t_train / max(1, args.c5_adam), 3),
                    "loss_curve_mean_per_500_steps": curve, "saved": args.c5_save or None})
        if Upca is not None:
            out["pca_for_comparison"] = "k=%d from 2000 of the C5 training fields" % args.k
    # ---------------- evaluation on fresh instances
    test = make_instances(range(W.CNN_TEST_SEED0, W.CNN_TEST_SEED0 + args.c5_test),
                          args.workers or min(16, len(os.sched_getaffinity(0))))
    eps_te = torch.tensor(np.stack([i.eps for i in test]), device="cuda")
    Ucnn = torch.empty((len(test), k, D), dtype=torch.complex64, device="cuda")
    eim_te = None
    if net.in_channels == 3:
        eim_te = torch.empty((len(test), D), dtype=torch.complex64, device="cuda")
        for c0 in range(0, len(test), 64):
            part = test[c0:c0 + 64]
            eim_field([FdfdOp.from_instance(i) for i in part],
                      [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in part],
                      out=eim_te[c0:c0 + len(part)])
    net.predict(eps_te[:32], Ucnn[:32], eim=None if eim_te is None else eim_te[:32])   # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    net.predict(eps_te, Ucnn, eim=eim_te)
    e1.record()
    torch.cuda.synchronize()
    out["inference_ms_for_%d" % len(test)] = round(e0.elapsed_time(e1), 2)
    if args.c5_load:
        Upca = None
    EB = args.c5_eval_batch
    res = {}
    first_two = {}
    xs_plain = [None] * len(test)
    for mode in args.c5_modes.split(","):
        if mode == "pca" and Upca is None:
            continue
        kk = {"plain": 0, "cnn": k, "pca": args.k}[mode]
        inf_all, h_all, secs = [], [], 0.0
        for b0 in range(0, len(test), EB):
            part = test[b0:b0 + EB]
            ops = [FdfdOp.from_instance(i) for i in part]
            bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in part]
            sv = Solver(ops, restart=args.restart, kmax=kk, cgs_passes=args.cgs, hist_cap=args.maxit)
            torch.cuda.synchronize()
            ts = time.time()
            if mode == "cnn":
                sv.set_subspace([Ucnn[b0 + j] for j in range(len(part))])
            elif mode == "pca":
                sv.set_subspace([Upca] * len(part))
            xs, inf, _ = sv.solve(bs, tol=args.tol, maxit=args.maxit)
            torch.cuda.synchronize()
            secs += time.time() - ts
            inf_all.extend(inf)
            h_all.extend(sv.history(j) for j in range(len(part)))
            if mode == "plain":
                for j, x in enumerate(xs):
                    xs_plain[b0 + j] = x.clone()
            if b0 == 0:
                first_two[mode] = [xs[0].cpu().numpy(), xs[1].cpu().numpy()]
            sv.close()
            log(f"  C5 eval {mode}: {b0 + len(part)}/{len(test)}, {secs:.0f}s")
        res[mode] = {"solves_per_s": round(len(test) / secs, 4),
                     "seconds": round(secs, 2),
                     **batch_stats(inf_all, h_all, args.tol)}
        log(f"C5 eval {mode}: {res[mode]}")
    nz = [float(torch.linalg.vector_norm(Ucnn[p]).item()) for p in range(len(test))]
    out["predicted_fields_all_zero"] = sum(1 for v in nz if v == 0.0)
    if xs_plain[0] is not None:
        Xp = torch.stack(xs_plain).contiguous()
        for mode, V in (("cnn", Ucnn), ("pca", None if Upca is None else
                                        Upca.unsqueeze(0).expand(len(test), -1, -1).contiguous())):
            if mode in res and V is not None:
                try:
                    res[mode]["proj_loss_mean"] = float(np.mean(proj_loss_batched(V, Xp)))
                except DDError as e:            # e.g. a collapsed network's zero fields
                    res[mode]["proj_loss_mean"] = None
                    res[mode]["proj_loss_error"] = str(e)
        refs = [oracle_reference(test[p]) for p in range(2)]
        res["error_vs_sparse_lu_plain"] = [rel_err(xs_plain[p].cpu().numpy(), refs[p]["x"])
                                           for p in range(2)]
        for mode, xl in first_two.items():
            res[mode]["error_vs_sparse_lu_first_two"] = [rel_err(xl[p], refs[p]["x"])
                                                         for p in range(2)]
    out["eval"] = res
    net.close()
    return out


def train_pca(args, torch, train):
    """Solve the training instances on the GPU (plain GMRES, batches of
    args.train_batch) and build the top-k PCA basis of their fields."""
    from paper_1902_00090_amd import FdfdOp, Solver, pca_build
    t0 = time.time()
    D = train[0].D
    S = torch.empty((len(train), D), dtype=torch.complex64, device="cuda")
    its, solver = [], None
    tb = args.train_batch
    for c0 in range(0, len(train), tb):
        part = train[c0:c0 + tb]
        ops = [FdfdOp.from_instance(i) for i in part]
        bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in part]
        if solver is None or len(part) != solver.nb:
            if solver is not None:
                solver.close()
            solver = Solver(ops, restart=args.restart, cgs_passes=args.cgs)
        else:
            solver.bind(ops)
        xs, infos, _ = solver.solve(bs, tol=args.train_tol, maxit=args.maxit)
        for j, x in enumerate(xs):
            S[c0 + j] = x.to(torch.complex64)
        its.extend(i["iters"] for i in infos)
        if (c0 // tb) % 4 == 3 or c0 + tb >= len(train):
            log(f"  training solves {c0 + len(part)}/{len(train)}: mean iters {np.mean(its):.0f}, "
                f"{time.time() - t0:.0f}s")
    solver.close()
    t_solve = time.time() - t0
    U, sig = pca_build(S, args.k)
    torch.cuda.synchronize()
    t_pca = time.time() - t0 - t_solve
    del S
    log(f"PCA: k={args.k} from {len(train)} solver-generated fields (tol {args.train_tol:g}), "
        f"solves {t_solve:.1f}s + basis {t_pca:.1f}s; sigma[k-1]/sigma[0] = {sig[-1] / sig[0]:.3f}")
    return U, sig, {"problems": len(train), "snapshot_tol": args.train_tol,
                    "solve_seconds": round(t_solve, 1), "basis_seconds": round(t_pca, 2),
                    "snapshot_iters_mean": float(np.mean(its)),
                    "sigma_ratio_k": float(sig[-1] / sig[0])}


def batch_stats(infos, hists, tol_lo):
    h = hists
    return {
        "iters_mean": float(np.mean([i["iters"] for i in infos])),
        "iters_max": int(max(i["iters"] for i in infos)),
        "matvecs_mean": float(np.mean([i["matvecs"] for i in infos])),
        "all_converged": all(i["status"] == 0 for i in infos),
        "worst_rel_res_true": max(i["rel_res_true"] for i in infos),
        "iters_to_1e-6_mean": float(np.mean([first_below(x, tol_lo) or np.nan for x in h])),
        "iters_to_0.04_mean": float(np.mean([first_below(x, 0.04) or np.nan for x in h])),
        "rel_res_after_1_iter_mean": float(np.mean([x[0] for x in h])),
    }


def c1_leg(args, torch, W):
    """Small binary-pixel problem: GMRES(50) complex128 to 1e-8 on the GPU and
    in the oracle (host), iterations, time and the error against dense LU."""
    from oracle import direct, fdfd, gmres
    from paper_1902_00090_amd import FdfdOp, Solver
    inst = W.small_binary(0)
    A = fdfd.assemble_instance(inst)
    t0 = time.time()
    xo, io = gmres.gmres(A, inst.b, restart=50, tol=1e-8, maxit=20000)
    t_or = time.time() - t0
    xs = direct.dense_solve(A, inst.b)
    op = FdfdOp.from_instance(inst)
    s = Solver([op], restart=50, inner="c128", cgs_passes=2, hist_cap=20000)
    b = torch.tensor(inst.b, dtype=torch.complex128, device="cuda")
    s.solve([b], tol=1e-8, maxit=20000)                      # warm-up
    torch.cuda.synchronize()
    t0 = time.time()
    (x,), (inf,), _ = s.solve([b], tol=1e-8, maxit=20000)
    torch.cuda.synchronize()
    t_gpu = time.time() - t0
    h = s.history(0)
    s.close()
    n = min(len(h), len(io["history"]))
    dev = float(np.max(np.abs(np.log10(h[:n]) - np.log10(np.asarray(io["history"][:n])))))
    out = {"gpu": {"iters": inf["iters"], "seconds": round(t_gpu, 4),
                   "rel_res_true": inf["rel_res_true"],
                   "error_vs_dense_lu": rel_err(x.cpu().numpy(), xs)},
           "oracle": {"iters": io["iters"], "seconds": round(t_or, 3),
                      "rel_res_true": io["rel_res"], "error_vs_dense_lu": rel_err(xo, xs)},
           "history_max_log10_gap_common_steps": dev, "common_steps": n}
    log(f"C1: {out}")
    return out


def c2_leg(args, torch, W, U, ref):
    """The single grating solve (seed 1000) alone, plain and PCA-augmented
    (plain only without a basis U), step groups replayed as HIP graphs, to
    1e-6 and to tol_acc; errors against the FP64 sparse LU solution."""
    from paper_1902_00090_amd import FdfdOp, Solver
    inst = W.grating(1000)
    op = FdfdOp.from_instance(inst)
    b = torch.tensor(inst.b, dtype=torch.complex128, device="cuda")
    out = {"instance": "grating seed 1000, 480x240", "err_factor": ref["err_factor"],
           "kappa_1_estimate": ref["kappa_1"], "sparse_lu_seconds": round(ref["lu_seconds"], 2)}
    # plain and augmented with the two-sweep Arnoldi step, then both with the
    # one-sweep step (which moves each basis vector once and takes two
    # launches per step: the faster of the two for one problem alone)
    for aug, fused in ((False, False), (True, False), (False, True), (True, True)):
        if aug and U is None:
            continue
        s = Solver([op], restart=args.restart, kmax=args.k if aug else 0, cgs_passes=args.cgs,
                   use_graph=True, fused=fused)
        if aug:
            s.set_subspace([U])
        s.solve([b], tol=args.tol, maxit=args.maxit)       # warm-up (graph capture)
        res = {}
        for tol in (args.tol, args.tol_acc):
            torch.cuda.synchronize()
            t0 = time.time()
            (x,), (inf,), _ = s.solve([b], tol=tol, maxit=args.maxit)
            torch.cuda.synchronize()
            dt = time.time() - t0
            res[f"tol_{tol:g}"] = {"seconds": round(dt, 4), "iters": inf["iters"],
                                   "us_per_iter": round(1e6 * dt / max(1, inf["iters"]), 1),
                                   "converged": inf["status"] == 0,
                                   "rel_res_true": inf["rel_res_true"],
                                   "error_vs_sparse_lu": rel_err(x.cpu().numpy(), ref["x"])}
        s.close()
        out[("augmented" if aug else "plain") + ("_one_sweep" if fused else "")] = res
    log(f"C2: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=25)
    ap.add_argument("--train", type=int, default=2000, help="PCA training instances")
    ap.add_argument("--test", type=int, default=500, help="test instances")
    ap.add_argument("--train-batch", type=int, default=100)
    ap.add_argument("--k", type=int, default=20)
    ap.add_argument("--restart", type=int, default=100)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--tol-acc", type=float, default=2e-7,
                    help="refined tolerance at which the error bound meets 1e-5")
    ap.add_argument("--train-tol", type=float, default=1e-2,
                    help="relative residual of the training solves (the basis only needs "
                         "the dominant content of the fields)")
    ap.add_argument("--warmup-tol", type=float, default=1e-2)
    ap.add_argument("--maxit", type=int, default=30000)
    ap.add_argument("--cgs", type=int, default=1, help="Gram-Schmidt passes (1 or 2)")
    ap.add_argument("--fused", action="store_true",
                    help="one sweep per Arnoldi step (the slower option, for measurement)")
    ap.add_argument("--plain-batches", type=int, default=2)
    ap.add_argument("--first-cycle-batches", type=int, default=0,
                    help="batches also solved with the basis for the first cycle only")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=400)
    ap.add_argument("--oracle-check", type=int, default=4)
    ap.add_argument("--no-c1", action="store_true")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--workers", type=int, default=0, help="instance generation processes")
    ap.add_argument("--cnn", action="store_true", help="also run the CNN-predictor legs")
    ap.add_argument("--traj", type=int, default=8)
    ap.add_argument("--traj-steps", type=int, default=32)
    ap.add_argument("--cnn-k", type=int, default=10)
    ap.add_argument("--cnn-steps", type=int, default=400)
    ap.add_argument("--cnn-window", type=int, default=8)
    ap.add_argument("--cnn-loss", default="both", choices=("proj", "res", "both"))
    ap.add_argument("--cnn-inputs", type=int, default=3, choices=(1, 3))
    ap.add_argument("--uneven", action="store_true", help="also run the uneven correlated batch")
    ap.add_argument("--recycle", type=int, default=0)
    ap.add_argument("--recycle-window", type=int, default=5)
    ap.add_argument("--c4-recycle", type=int, default=0,
                    help="batches of the C4 test set solved with recycled harmonic Ritz vectors")
    ap.add_argument("--recycle-ritz", type=int, default=10,
                    help="harmonic Ritz vectors carried from step to step")
    ap.add_argument("--precond", action="store_true")
    ap.add_argument("--c5", action="store_true",
                    help="CNN predictor at scale: 313 x 32 training steps, 10,000 Adam steps, "
                         "256 fresh test instances")
    ap.add_argument("--c5-traj", type=int, default=313)
    ap.add_argument("--c5-steps", type=int, default=32)
    ap.add_argument("--c5-adam", type=int, default=10000)
    ap.add_argument("--c5-test", type=int, default=256)
    ap.add_argument("--c5-eval-batch", type=int, default=64)
    ap.add_argument("--c5-train-tol", type=float, default=1e-2)
    ap.add_argument("--c5-save", default="")
    ap.add_argument("--c5-load", default="")
    ap.add_argument("--c5-only", action="store_true", help="run only the CNN-at-scale leg")
    ap.add_argument("--c5-inputs", type=int, default=3, choices=(1, 3),
                    help="input planes: permittivity (1) or permittivity + effective-index field (3)")
    ap.add_argument("--c5-lr", type=float, default=1e-3)
    ap.add_argument("--c5-modes", default="plain,cnn,pca")
    ap.add_argument("--c5-loss", default="proj", choices=("proj", "res"),
                    help="projection-type (local-PCA targets) or residual loss (unsupervised)")
    ap.add_argument("--cnn-kernels", type=int, default=0)
    ap.add_argument("--c2-only", action="store_true",
                    help="only the single grating solve (seed 1000), plain GMRES, two-sweep and "
                         "one-sweep steps")
    ap.add_argument("--calibrate-copy", type=int, default=0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the problems of a batch are independent and would be split across GPUs "
              "with no communication during the solve)",
              file=sys.stderr)
        sys.exit(2)

    import workloads as W
    workers = args.workers or min(16, len(os.sched_getaffinity(0)))
    t0 = time.time()
    train, test = [], []
    if args.cnn_kernels <= 0 and not args.c5_only and not args.c2_only:
        train = make_instances(range(W.PCA_TRAIN_SEED0, W.PCA_TRAIN_SEED0 + args.train), workers)
        test = make_instances(range(W.PCA_TEST_SEED0, W.PCA_TEST_SEED0 + args.test), workers)
        log(f"data: {len(train)} training + {len(test)} test instances, {time.time() - t0:.1f}s "
            f"({workers} processes)")

    import torch
    from paper_1902_00090_amd import FdfdOp, Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy > 0:
        # a copy kernel of known size: its FETCH_SIZE / WRITE_SIZE readings
        # calibrate the counters of the solver's sweeps
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_copy} MiB read + {args.calibrate_copy} MiB written")
        del src, dst
    if args.cnn_kernels > 0:
        cnn_kernels_only(args, torch, W)
        return
    if args.c5_only:
        print(json.dumps({"cnn_at_scale": c5_leg(args, torch, W)}), flush=True)
        return
    if args.c2_only:
        print(json.dumps({"c2_single_grating": c2_leg(args, torch, W, None,
                                                      oracle_reference(W.grating(1000)))}),
              flush=True)
        return

    # ---------------- predictor training (untimed)
    U, sig, train_info = train_pca(args, torch, train)
    del train

    # ---------------- test set resident in HBM
    B = args.batch
    nbat = len(test) // B
    assert nbat >= 1, "need at least one full batch of test instances"
    ops = [FdfdOp.from_instance(i) for i in test[:nbat * B]]
    bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in test[:nbat * B]]
    xs = [torch.empty_like(b) for b in bs]
    # tile width from the autotuner (timed once per process, outside the timed region)
    aug = Solver(ops[:B], restart=args.restart, kmax=args.k, cgs_passes=args.cgs,
                 hist_cap=args.maxit, elems_per_thread=-1, fused=args.fused)
    Ulist = [U] * B

    def step(bi, tol):
        sl = slice(bi * B, (bi + 1) * B)
        aug.bind(ops[sl])
        aug.set_subspace(Ulist)
        return aug.solve(bs[sl], tol=tol, maxit=args.maxit, x=xs[sl])

    order = [s % nbat for s in range(args.steps)]
    # warm-up steps run the same kernels on the last batches, to a loose
    # tolerance (they are not timed and only prime the runtime)
    for w in range(args.warmup):
        step(nbat - 1 - (w % nbat), args.warmup_tol)
    torch.cuda.synchronize()
    aug.profile(True)
    infos, hists = [], []
    t_batch = {}
    t0 = time.time()
    for bi in order:
        ts = time.time()
        _, inf, _ = step(bi, args.tol_acc)
        t_batch[bi] = time.time() - ts
        infos.extend(inf)
        hists.extend(aug.history(p) for p in range(B))
    torch.cuda.synchronize()
    dt = time.time() - t0
    ks = aug.kernel_stats()
    aug.profile(False)
    ms_per_step = 1000.0 * dt / args.steps
    value = B * args.steps / dt
    astats = batch_stats(infos, hists, args.tol)
    covered = sorted(set(order))
    log(f"augmented (C4): {value:.3f} solves/s, {ms_per_step:.0f} ms/step over {args.steps} steps "
        f"({len(covered) * B} distinct test instances), iters mean {astats['iters_mean']:.0f}")

    # ---------------- the same batches at 1e-6 exactly, augmented
    x6 = {}
    t6 = {}
    for bi in range(min(args.plain_batches, nbat)):
        sl = slice(bi * B, (bi + 1) * B)
        xb = [torch.empty_like(b) for b in bs[sl]]
        aug.bind(ops[sl])
        aug.set_subspace(Ulist)
        torch.cuda.synchronize()
        ts = time.time()
        aug.solve(bs[sl], tol=args.tol, maxit=args.maxit, x=xb)
        torch.cuda.synchronize()
        t6[bi] = time.time() - ts
        x6[bi] = xb
    # ---------------- the predicted basis for the first cycle only (optional):
    # one augmented cycle, then plain GMRES from its iterate
    first_cycle = None
    if args.first_cycle_batches > 0:
        fc_t, fc_it = 0.0, []
        for bi in range(min(args.first_cycle_batches, nbat)):
            sl = slice(bi * B, (bi + 1) * B)
            xb = [torch.empty_like(b) for b in bs[sl]]
            aug.bind(ops[sl])
            torch.cuda.synchronize()
            ts = time.time()
            aug.set_subspace(Ulist)
            _, inf1, _ = aug.solve(bs[sl], tol=args.tol_acc, maxit=args.restart, x=xb)
            aug.set_subspace(None)
            _, inf2, _ = aug.solve(bs[sl], x0=xb, tol=args.tol_acc, maxit=args.maxit, x=xb)
            torch.cuda.synchronize()
            fc_t += time.time() - ts
            fc_it.extend(a["iters"] + b2["iters"] for a, b2 in zip(inf1, inf2))
        nfc = min(args.first_cycle_batches, nbat) * B
        first_cycle = {"problems": nfc, "solves_per_s": round(nfc / fc_t, 4),
                       "iters_mean": float(np.mean(fc_it)),
                       "note": "one PCA-augmented cycle, then plain GMRES from its iterate"}
        log(f"PCA basis for the first cycle only: {first_cycle}")
    tile = aug.elems_per_thread
    aug.close()

    # ---------------- plain GMRES on the same batches (tol_acc and 1e-6)
    plain = None
    # batches the timed steps covered (their augmented times are known)
    pb = [bi for bi in range(min(args.plain_batches, nbat)) if bi in t_batch]
    if pb:
        ps = Solver(ops[:B], restart=args.restart, cgs_passes=args.cgs, hist_cap=args.maxit,
                    elems_per_thread=-1)
        pinf, phist, pt, pt6, xp, xp6 = [], [], 0.0, 0.0, {}, {}
        for bi in pb:
            sl = slice(bi * B, (bi + 1) * B)
            ps.bind(ops[sl])
            for tol, store in ((args.tol_acc, xp), (args.tol, xp6)):
                xb = [torch.empty_like(b) for b in bs[sl]]
                torch.cuda.synchronize()
                ts = time.time()
                _, inf, _ = ps.solve(bs[sl], tol=tol, maxit=args.maxit, x=xb)
                torch.cuda.synchronize()
                if tol == args.tol_acc:
                    pt += time.time() - ts
                    pinf.extend(inf)
                    phist.extend(ps.history(p) for p in range(B))
                else:
                    pt6 += time.time() - ts
                store[bi] = xb
        ps.close()
        at = sum(t_batch[bi] for bi in pb)
        at6 = sum(t6[bi] for bi in pb)
        plain = {"batches": len(pb), "problems": len(pb) * B,
                 "solves_per_s": round(len(pb) * B / pt, 4),
                 "solves_per_s_to_1e-6": round(len(pb) * B / pt6, 4),
                 **batch_stats(pinf, phist, args.tol),
                 "augmented_same_batches": {"solves_per_s": round(len(pb) * B / at, 4),
                                            "solves_per_s_to_1e-6": round(len(pb) * B / at6, 4)},
                 "speedup_wallclock": round(pt / at, 3),
                 "speedup_wallclock_to_1e-6": round(pt6 / at6, 3)}
        log(f"plain on {len(pb) * B} of the test instances: {plain['solves_per_s']:.3f} solves/s "
            f"(augmented {len(pb) * B / at:.3f}); to 1e-6: {plain['solves_per_s_to_1e-6']:.3f} vs "
            f"{len(pb) * B / at6:.3f}; iters mean {plain['iters_mean']:.0f}")

    # ---------------- error against the FP64 oracle (sparse LU) on a subset
    errs = []
    if args.oracle_check > 0:
        for p in range(min(args.oracle_check, B * max(1, args.plain_batches))):
            ref = oracle_reference(test[p])
            bi, j = divmod(p, B)
            e = {"instance": p, "err_factor": round(ref["err_factor"], 2),
                 "kappa_1_estimate": ref["kappa_1"],
                 "error_bound_at_tol_acc": ref["err_factor"] * args.tol_acc,
                 "augmented_tol_acc": rel_err(xs[p].cpu().numpy(), ref["x"])}
            if bi in x6:
                e["augmented_1e-6"] = rel_err(x6[bi][j].cpu().numpy(), ref["x"])
            if plain is not None and bi in xp:
                e["plain_tol_acc"] = rel_err(xp[bi][j].cpu().numpy(), ref["x"])
                e["plain_1e-6"] = rel_err(xp6[bi][j].cpu().numpy(), ref["x"])
            errs.append(e)
            log(f"  oracle check {p}: {e}")

    c4rec = c4_recycle_leg(args, torch, test, U) if args.c4_recycle > 0 else None
    # the supplement's diagonal preconditioners on the first two C4 batches
    pre = (precond_leg(args, torch, ops[:2 * B], bs[:2 * B], U)
           if args.precond and nbat >= 2 else None)

    # ---------------- C1 and C2 beside their oracle figures
    c1 = None if args.no_c1 else c1_leg(args, torch, W)
    c2 = None
    if not args.no_c2:
        ref2 = oracle_reference(W.grating(1000))
        c2 = c2_leg(args, torch, W, U, ref2)

    # ---------------- optional legs
    cnn = rec = uneven = None
    if args.cnn:
        data = W.trajectory_dataset(args.traj, args.traj_steps)
        tr_idx, te_idx = W.split_train_test(len(data))
        ctrain = [data[i] for i in tr_idx]
        ctest = [data[i] for i in te_idx][:64]
        cops = [FdfdOp.from_instance(i) for i in ctest]
        cbs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in ctest]
        if args.cnn:
            from paper_1902_00090_amd.train import solve_fields
            Smat, _ = solve_fields(ctrain, tol=1e-4, restart=args.restart, cgs_passes=args.cgs)
            cs = Solver(cops, restart=args.restart, cgs_passes=args.cgs)
            cxs, _, _ = cs.solve(cbs, tol=args.tol, maxit=args.maxit)
            cs.close()
            modes = ("proj", "res") if args.cnn_loss == "both" else (args.cnn_loss,)
            cnn = {m: cnn_leg(args, torch, W, data, tr_idx, ctrain, ctest, Smat, cops, cbs, cxs,
                              U, None, None, m) for m in modes}
            del Smat
    if args.recycle > 0:
        rec = recycle_leg(args, torch, W)
    c5 = c5_leg(args, torch, W) if args.c5 else None
    if args.uneven:
        uneven = uneven_leg(args, torch, W)

    # ---------------- roofline of the dominant sweep
    name = max(ks, key=lambda n: ks[n][0])
    ms_k, launches_k, bytes_k = ks[name]
    achieved = bytes_k / (ms_k * 1e-3) / 1e9 if ms_k > 0 else 0.0
    kname = {"matvec_dots": "k_matvec_dot", "second_pass": "k_update_dot",
             "update_norm": "k_update_norm", "fused_sweep": "k_fused_sweep"}[name]
    traffic = None
    trec = measured_traffic()
    if (trec is not None and trec["kernel"] == kname and args.batch == trec["batch"]
            and args.k == trec["k"] and args.cgs == 1
            and kernel_sources_hash() == trec["sources_sha256_16"]):
        traffic = trec["bytes_per_launch"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_workload": None if traffic is None else
                {"run": trec["workload"],
                 "algorithmic_bytes_per_launch": trec["algorithmic_bytes_per_launch"],
                 "ratio": round(traffic / trec["algorithmic_bytes_per_launch"], 3)},
                "kernel": kname,
                "avg_launch_us": round(1000 * ms_k / max(1, launches_k), 2),
                "launches": int(launches_k),
                "algorithmic_bytes_per_launch": round(bytes_k / max(1, launches_k))}
    sweeps = {n: {"ms": round(v[0], 2), "launches": int(v[1]),
                  "GB_per_s": round(v[2] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else None,
                  "algorithmic_bytes_per_launch": round(v[2] / v[1]) if v[1] else None}
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
                ts = time.time()
                gmres_aug.gmres_aug(A, inst.b, V, restart=args.restart, tol=0.0,
                                    maxit=args.cpu_iters)
                return time.time() - ts
        tc = sample(1)
        t_iter = tc / args.cpu_iters
        nthr = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
        tc_all = sample(nthr)
        it_mean = astats["iters_mean"]
        cpu = {"value": round(1.0 / (t_iter * it_mean), 6), "unit": "solves/s",
               "cores": 1, "kind": "oracle",
               "sample": f"oracle gmres_aug (complex128, numpy/scipy, 1 BLAS thread) on one "
                         f"C4 test instance for {args.cpu_iters} Arnoldi steps ({tc:.1f}s, "
                         f"{1000 * t_iter:.0f} ms/step incl. setup), scaled to the mean "
                         f"{it_mean:.0f} steps the GPU needed per solve",
               "host_cpu_count": os.cpu_count(),
               "all_threads": {"value": round(args.cpu_iters / (tc_all * it_mean), 6),
                               "threads": nthr, "sample_seconds": round(tc_all, 2)},
               "sparse_lu_seconds_per_problem": (round(float(np.mean(
                   [c2["sparse_lu_seconds"]])), 3) if c2 else None)}
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
            "workload": f"C4: PCA-augmented GMRES({args.restart}), k={args.k} principal components "
                        f"of {train_info['problems']} solver-generated 480x240 grating fields "
                        f"(seeds 10000+i), on batches of {B} of {nbat * B} fresh test instances "
                        f"(seeds 20000+i, round-robin); complex64 inner iteration with FP64 "
                        f"true-residual restarts to {args.tol_acc:g} (past {args.tol:g}; error "
                        f"bound 1e-5), {args.cgs} Gram-Schmidt pass(es)",
            "batch": B, "grid": "480x240", "restart": args.restart, "k": args.k,
            "tol": args.tol, "tol_acc": args.tol_acc, "test_instances": nbat * B,
            "distinct_instances_timed": len(covered) * B,
            "elems_per_thread": tile,
        },
        "pca_training": train_info,
        "augmented": {"solves_per_s": round(value, 4), **astats,
                      "error_vs_sparse_lu": errs},
        "plain": plain,
        "sweeps": sweeps,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "c1_small_binary": c1,
        "c2_single_grating": c2,
        "cnn_augmented": cnn,
        "uneven_batch_plain": uneven,
        "trajectory_recycling": rec,
        "cnn_at_scale": c5,
        "c4_recycling": c4rec,
        "pca_first_cycle_only": first_cycle,
        "diagonal_preconditioners": pre,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
