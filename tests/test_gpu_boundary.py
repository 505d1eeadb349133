"""The C-ABI boundary on the GPU: predictors saved and reloaded (a PCA basis,
a CNN with its Adam state) give bit-identical predictions, training resumes
exactly, the generic predict_subspace serves both kinds, and a solve can run
entirely in a workspace the caller owns."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_pca_predictor_roundtrip(tmp_path):
    import torch
    from paper_1902_00090_amd import Predictor, save_pca
    nx, ny, k = 48, 32, 5
    rng = np.random.default_rng(31)
    U = torch.tensor(W.random_complex(rng, (k, nx * ny)).astype(np.complex64), device="cuda")
    path = tmp_path / "pca.ddp"
    save_pca(path, U, nx, ny)
    p = Predictor(path, max_batch=3)
    assert (p.kind, p.nx, p.ny, p.k, p.in_channels) == ("pca", nx, ny, k, 0)
    out = p.predict(3)
    torch.cuda.synchronize()
    for i in range(3):
        assert torch.equal(torch.view_as_real(out[i]), torch.view_as_real(U))
    p.close()


def _data(nx, ny, B, k, seed):
    import torch
    rng = np.random.default_rng(seed)
    eps = torch.tensor((2.085 + 10.165 * rng.random((B, ny, nx))).astype(np.float32), device="cuda")
    tgt = torch.tensor(W.random_complex(rng, (B, k, nx * ny)).astype(np.complex64) * 0.1,
                       device="cuda")
    return eps, tgt


def test_cnn_save_load_resumes_training_exactly(tmp_path):
    """Three Adam steps, save, load: identical predictions, and one more step
    on the original and on the reloaded network gives identical parameters
    (the moments and the step count travel with the file)."""
    import torch
    from paper_1902_00090_amd import Cnn, Predictor
    nx, ny, B, k = 24, 16, 2, 3
    net = Cnn(nx, ny, B, k, seed=4)
    eps, tgt = _data(nx, ny, B, k, 9)
    for _ in range(3):
        net.train_step(eps, tgt, lr=1e-3)
    path = tmp_path / "cnn.ddp"
    net.save(path)
    net2 = Cnn.load(path, max_batch=B)
    assert (net2.nx, net2.ny, net2.k, net2.in_channels) == (nx, ny, k, 1)
    assert np.array_equal(net.get_params(), net2.get_params())
    u1, u2 = net.predict(eps), net2.predict(eps)
    assert torch.equal(torch.view_as_real(u1), torch.view_as_real(u2))
    l1 = net.train_step(eps, tgt, lr=1e-3)
    l2 = net2.train_step(eps, tgt, lr=1e-3)
    assert l1 == l2
    assert np.array_equal(net.get_params(), net2.get_params())
    # the generic predictor serves the saved network
    p = Predictor(path, max_batch=B)
    assert p.kind == "cnn"
    u3 = p.predict(B, eps=eps)
    torch.cuda.synchronize()
    net3 = Cnn.load(path, max_batch=B)
    assert torch.equal(torch.view_as_real(u3), torch.view_as_real(net3.predict(eps)))


def test_three_plane_predictor_computes_its_field_input(tmp_path):
    """A three-plane CNN behind predict_subspace computes the effective-index
    field from the operators and right-hand sides itself: the same output as
    eim_field followed by the network's forward pass."""
    import torch
    from paper_1902_00090_amd import Cnn, FdfdOp, Predictor, eim_field
    nx, ny, B, k = 48, 24, 2, 2
    insts = [W.grating(3100 + i, nx=nx, ny=ny, npml=4) for i in range(B)]
    ops = [FdfdOp.from_instance(i) for i in insts]
    bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in insts]
    eps = torch.tensor(np.stack([i.eps for i in insts]), device="cuda")
    net = Cnn(nx, ny, B, k, seed=6, in_channels=3)
    path = tmp_path / "cnn3.ddp"
    net.save(path)
    p = Predictor(path, max_batch=B)
    assert p.in_channels == 3
    u = p.predict(B, eps=eps, ops=ops, b=bs)
    F = torch.stack(eim_field(ops, bs)).contiguous()
    ref = net.predict(eps, eim=F)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(u), torch.view_as_real(ref))
    from paper_1902_00090_amd import DDError
    with pytest.raises(DDError):
        p.predict(B, eps=eps)                      # the field input needs ops and b


@pytest.mark.parametrize("k", [0, 3])
def test_solve_in_caller_workspace(k):
    """A solver built on a caller-owned workspace of the reported size
    allocates no device memory of its own and gives bit-identical results."""
    import torch
    from paper_1902_00090_amd import DDError, FdfdOp, Solver, _lib, workspace_bytes
    inst = W.grating(3200, nx=96, ny=48, npml=6)
    op = FdfdOp.from_instance(inst)
    b = torch.tensor(inst.b, dtype=torch.complex128, device="cuda")
    rng = np.random.default_rng(3)
    U = [torch.tensor(W.random_complex(rng, (k, inst.D)), dtype=torch.complex128,
                      device="cuda")] if k else None
    kw = dict(restart=30, kmax=k, inner="c128", hist_cap=4000)
    nbytes = workspace_bytes([op], **kw)
    # the one-problem query of gmres_solve agrees with the general one at its defaults
    assert _lib.lib().gmres_workspace_bytes(op.handle, k, 30, _lib.DD_C128) == \
        workspace_bytes([op], restart=30, kmax=k, inner="c128")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s1 = Solver([op], workspace=ws, **kw)
    assert s1.device_bytes == nbytes
    s2 = Solver([op], **kw)
    res = []
    for s in (s1, s2):
        if U:
            s.set_subspace(U)
        (x,), (inf,), st = s.solve([b], tol=1e-9, maxit=4000)
        torch.cuda.synchronize()
        res.append((x.cpu().numpy(), s.history(0), inf))
    assert res[0][2]["status"] == 0 and res[0][2]["iters"] == res[1][2]["iters"]
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    with pytest.raises(DDError):
        Solver([op], workspace=ws[:nbytes - 512], **kw)


def test_trained_checkpoint_serves_through_predict_subspace():
    """The network trained at scale (313 trajectories x 32 steps, 10,000 Adam
    steps, three input planes) loads through predictor_load and through
    Cnn.load; predict_subspace (which forms the effective-index planes
    itself) gives bit-identical fields to Cnn.predict with eim_field's
    planes, all finite and non-zero, on two fresh 480 x 240 gratings."""
    import os
    import torch
    from paper_1902_00090_amd import Cnn, FdfdOp, Predictor, eim_field
    path = os.path.join(os.path.dirname(__file__), "..", "paper_1902_00090_amd", "checkpoints",
                        "cnn_k10_eim_c5.ddp")
    insts = [W.grating(50_000 + i) for i in range(2)]
    ops = [FdfdOp.from_instance(i) for i in insts]
    bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in insts]
    eps = torch.tensor(np.stack([i.eps for i in insts]), device="cuda")
    pr = Predictor(path, max_batch=2)
    assert (pr.kind, pr.nx, pr.ny, pr.k, pr.in_channels) == ("cnn", 480, 240, 10, 3)
    U1 = pr.predict(2, eps=eps, ops=ops, b=bs)
    net = Cnn.load(path, max_batch=2)
    eim = torch.empty((2, insts[0].D), dtype=torch.complex64, device="cuda")
    eim_field(ops, bs, out=eim)
    U2 = net.predict(eps, eim=eim)
    torch.cuda.synchronize()
    assert torch.equal(U1, U2)
    assert torch.isfinite(torch.view_as_real(U1)).all()
    assert all(float(torch.linalg.vector_norm(U1[p, j])) > 0 for p in range(2) for j in range(10))
    pr.close()
    net.close()
