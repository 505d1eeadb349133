"""Parity at the benchmark's full size and launch configuration: a PCA basis
of 20 principal components from GPU solves of 40 fresh 480 x 240 grating
instances (seeds 10,000 + i), then a lockstep batch of 8 other fresh
instances (seeds 20,000 + i) solved by complex64 GMRES(100) with one
Gram-Schmidt pass and FP64 true-residual restarts to a relative residual of
2e-7.  Sampled problems are checked by the oracle's FP64 sparse operator (true
residual) and a sparse LU solve: the error must be within 1e-5."""
import numpy as np
import pytest

import workloads as W
from oracle import direct, fdfd

pytestmark = pytest.mark.gpu


def test_full_size_batch_in_benchmark_configuration():
    import torch
    from paper_1902_00090_amd import FdfdOp, Solver, pca_build
    train = W.grating_set(10_000, 40)
    test = W.grating_set(20_000, 8)
    # basis from GPU solves of the training instances (as the benchmark builds it)
    ops = [FdfdOp.from_instance(i) for i in train]
    s = Solver(ops, restart=100, cgs_passes=1)
    xs, _, _ = s.solve([torch.tensor(i.b, device="cuda") for i in train], tol=1e-2, maxit=30000)
    U, _ = pca_build(torch.stack([x.to(torch.complex64) for x in xs]).contiguous(), 20)
    s.close()
    ops = [FdfdOp.from_instance(i) for i in test]
    bs = [torch.tensor(i.b, device="cuda") for i in test]
    aug = Solver(ops, restart=100, kmax=20, cgs_passes=1)
    aug.set_subspace([U] * len(test))
    xs, infos, st = aug.solve(bs, tol=2e-7, maxit=40000)
    assert st == 0 and all(i["status"] == 0 and i["k_used"] == 20 for i in infos)
    for p in (0, 3, 7):
        A = fdfd.assemble_instance(test[p])
        x = xs[p].cpu().numpy()
        rr = np.linalg.norm(test[p].b - A @ x) / np.linalg.norm(test[p].b)
        assert rr <= 2e-7 and abs(rr - infos[p]["rel_res_true"]) <= 1e-3 * rr, (p, rr, infos[p])
        xstar = direct.sparse_solve(A, test[p].b)
        err = np.linalg.norm(x - xstar) / np.linalg.norm(xstar)
        print(f"problem {p}: iters {infos[p]['iters']}, rel res {rr:.3e}, error {err:.3e}")
        assert err <= 1e-5
