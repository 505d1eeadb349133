"""What the trained network gains over the method without it: a CNN trained
(on the GPU, by the library's own kernels) on solver-generated fields of
synthetic design trajectories predicts subspaces that capture most of the
held-out fields and put augmented GMRES ahead of plain GMRES in its early
iterations (measured on this workload: projection loss 0.04; residual after 5
iterations 0.35 vs 0.45)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_trained_cnn_reduces_first_iteration_residual():
    import torch
    from paper_1902_00090_amd import Cnn, FdfdOp, Solver, proj_loss_batched
    from paper_1902_00090_amd.train import solve_fields, train_cnn, trajectory_targets
    nx, ny, T, S, k = 96, 48, 12, 16, 4
    data = W.trajectory_dataset(T, S, seed0=80_000, nx=nx, ny=ny)
    F, _ = solve_fields(data, tol=1e-5)
    tgt = trajectory_targets(F, S, window=4, k=k)
    tr, te = W.split_train_test(len(data), seed=1)
    eps = torch.tensor(np.stack([d.eps for d in data]), device="cuda")
    tr_i = torch.as_tensor(tr, device="cuda")
    net = Cnn(nx, ny, 16, k, seed=0)
    losses = train_cnn(net, eps.index_select(0, tr_i).contiguous(),
                       tgt.index_select(0, tr_i).contiguous(), steps=2000, batch=16, lr=1e-3)
    assert np.mean(losses[-20:]) < 0.5 * np.mean(losses[:5])
    # held-out steps: predicted subspace vs plain GMRES
    test = [data[i] for i in te]
    U = net.predict(eps.index_select(0, torch.as_tensor(te, device="cuda")).contiguous())
    lp = proj_loss_batched(U, F.index_select(0, torch.as_tensor(te, device="cuda")).to(torch.complex128).contiguous())
    ops = [FdfdOp.from_instance(i) for i in test]
    bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in test]
    aug = Solver(ops, restart=50, kmax=k, hist_cap=60)
    aug.set_subspace([U[i].contiguous() for i in range(len(test))])
    _, ia, _ = aug.solve(bs, tol=1e-12, maxit=60)
    plain = Solver(ops, restart=50, hist_cap=60)
    _, ip, _ = plain.solve(bs, tol=1e-12, maxit=60)
    ha = np.array([aug.history(p) for p in range(len(test))])
    hp = np.array([plain.history(p) for p in range(len(test))])
    r_aug, r_pl = ha[:, 0].mean(), hp[:, 0].mean()
    print(f"held-out: projection loss {lp.mean():.3f} (min {lp.min():.3f}); mean residual after "
          f"1/5/20/60 iterations: CNN-augmented {[round(ha[:, i].mean(), 4) for i in (0, 4, 19, 59)]}"
          f" plain {[round(hp[:, i].mean(), 4) for i in (0, 4, 19, 59)]}; final loss "
          f"{np.mean(losses[-20:]):.3e} from {np.mean(losses[:5]):.3e}")
    # the network captures most of each held-out field (projection loss, Sec. 3)
    assert lp.mean() < 0.2
    # and the augmented iteration is ahead of plain GMRES early on
    assert ha[:, 0].mean() < 0.95 * hp[:, 0].mean()
    assert ha[:, 4].mean() < 0.9 * hp[:, 4].mean()
