"""Parity at the benchmark's full size and launch configuration: 480 x 240
problems in a lockstep batch (2048-element chunks), complex64 GMRES(100), one
Gram-Schmidt pass, a 20-vector PCA basis, tol 1e-6.  Sampled problems are
checked by the oracle's FP64 sparse operator (true residual) and a sparse LU
solve (error)."""
import numpy as np
import pytest

import workloads as W
from oracle import direct, fdfd

pytestmark = pytest.mark.gpu


def test_full_size_batch_in_benchmark_configuration():
    import torch
    from paper_1902_00090_amd import FdfdOp, Solver, pca_build
    data = W.trajectory_dataset(2, 16)
    tr, te = W.split_train_test(len(data))
    train, test = [data[i] for i in tr][:16], [data[i] for i in te][:8]
    # basis from GPU solves of the training steps (as the benchmark builds it)
    ops = [FdfdOp.from_instance(i) for i in train]
    s = Solver(ops, restart=100, cgs_passes=1)
    xs, _, _ = s.solve([torch.tensor(i.b, device="cuda") for i in train], tol=1e-3, maxit=30000)
    U, _ = pca_build(torch.stack([x.to(torch.complex64) for x in xs]).contiguous(), 12)
    s.close()
    ops = [FdfdOp.from_instance(i) for i in test]
    bs = [torch.tensor(i.b, device="cuda") for i in test]
    aug = Solver(ops, restart=100, kmax=12, cgs_passes=1, elems_per_thread=8)
    aug.set_subspace([U] * len(test))
    xs, infos, st = aug.solve(bs, tol=1e-6, maxit=30000)
    assert st == 0 and all(i["status"] == 0 and i["k_used"] == 12 for i in infos)
    for p in (0, 3, 7):
        A = fdfd.assemble_instance(test[p])
        x = xs[p].cpu().numpy()
        rr = np.linalg.norm(test[p].b - A @ x) / np.linalg.norm(test[p].b)
        assert rr <= 1e-6 and abs(rr - infos[p]["rel_res_true"]) <= 1e-3 * rr, (p, rr, infos[p])
        xstar = direct.sparse_solve(A, test[p].b)
        assert np.linalg.norm(x - xstar) / np.linalg.norm(xstar) < 1e-4
