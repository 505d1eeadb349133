"""Diagonal preconditioners fused into the stencil sweep (supplement, Table 1
comparison) against the oracle: complex128 residual histories of the
preconditioned system, plain and augmented, and complex64 solves of the
480 x 240 grating to the FP64 true residual."""
import numpy as np
import pytest

import workloads as W
from oracle import direct, fdfd, precond

pytestmark = pytest.mark.gpu


def _tiny(seed, nx=20, ny=16, npml=3):
    rng = np.random.default_rng(seed)
    eps = (2.085 + 10.165 * (rng.random((ny, nx)) < 0.4)).astype(np.float32)
    return W.Instance(eps, W.random_complex(rng, nx * ny), nx, ny, 0.04, 1.55, npml)


@pytest.mark.parametrize("kind", ["jacobi", "pml"])
@pytest.mark.parametrize("k", [0, 3])
def test_preconditioned_history_matches_oracle(kind, k):
    import torch
    from gpu_util import to_dev
    from paper_1902_00090_amd import FdfdOp, Solver
    inst = _tiny(70 + k)
    A = fdfd.assemble_instance(inst)
    pl, pr = (precond.jacobi(A) if kind == "jacobi" else
              precond.pml_scaling(inst.nx, inst.ny, inst.omega, inst.dx, inst.npml))
    V = W.random_complex(np.random.default_rng(71), (k, inst.D))
    s = Solver([FdfdOp.from_instance(inst)], restart=9, kmax=max(k, 1), inner="c128",
               hist_cap=200, precond=kind)
    if k:
        s.set_subspace([to_dev(V, torch.complex128)])
    (x,), (info,), st = s.solve([to_dev(inst.b, torch.complex128)], tol=1e-30, maxit=150)
    f, io = precond.gmres_aug_precond(A, inst.b, V.T, pl, pr, restart=9, tol=1e-30, maxit=150)
    assert info["iters"] == 150
    np.testing.assert_allclose(s.history(0)[:150], io["history"][:150], rtol=1e-7, atol=1e-14)
    np.testing.assert_allclose(x.cpu().numpy(), f, rtol=1e-6,
                               atol=1e-6 * np.abs(f).max())


@pytest.mark.parametrize("kind", ["jacobi", "pml"])
def test_preconditioned_grating_c64_reaches_tol(kind):
    import torch
    from paper_1902_00090_amd import FdfdOp, Solver
    inst = W.grating(1000)
    A = fdfd.assemble_instance(inst)
    s = Solver([FdfdOp.from_instance(inst)], restart=100, cgs_passes=1, precond=kind)
    (x,), (info,), st = s.solve([torch.tensor(inst.b, device="cuda")], tol=1e-6, maxit=60000)
    x = x.cpu().numpy()
    rr = np.linalg.norm(inst.b - A @ x) / np.linalg.norm(inst.b)
    print(kind, "iterations", info["iters"], "true residual", rr)
    assert st == 0 and rr <= 1e-6 and abs(rr - info["rel_res_true"]) <= 1e-3 * rr
    xs = direct.sparse_solve(A, inst.b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-4


def test_preconditioned_graph_replay_and_uneven_batch():
    """Preconditioned solves of problems of different grids in one lockstep
    batch, with graph replay: the same iterates as direct launches and as the
    problems solved one by one."""
    import torch
    from gpu_util import to_dev
    from paper_1902_00090_amd import FdfdOp, Solver
    insts = [_tiny(80), _tiny(81, nx=36, ny=28), _tiny(82, nx=12, ny=30)]
    ops = [FdfdOp.from_instance(i) for i in insts]
    bs = [to_dev(i.b, torch.complex128) for i in insts]
    res = []
    for g in (True, False):
        s = Solver(ops, restart=15, inner="c64", precond="pml", use_graph=g, hist_cap=4000)
        xs, infos, st = s.solve(bs, tol=1e-7, maxit=4000)
        assert st == 0
        res.append(([x.cpu().numpy() for x in xs], [i["iters"] for i in infos]))
    assert res[0][1] == res[1][1]
    for a, b in zip(res[0][0], res[1][0]):
        np.testing.assert_array_equal(a, b)
    for p, inst in enumerate(insts):
        s1 = Solver([ops[p]], restart=15, inner="c64", precond="pml")
        (x1,), (i1,), _ = s1.solve([bs[p]], tol=1e-7, maxit=4000)
        A = fdfd.assemble_instance(inst)
        for x in (res[1][0][p], x1.cpu().numpy()):
            assert np.linalg.norm(inst.b - A @ x) / np.linalg.norm(inst.b) <= 1e-7
