"""The one-sweep Arnoldi step (fused update, matvec and dots; one Gram-Schmidt
pass) against the CPU oracle.

complex128: residual histories against the oracle's literal block least
squares (plain, augmented, preconditioned), a batch of uneven grids (strips of
30 columns with a ragged last strip, bands of several heights, halos across
the periodic wrap) and the solutions.
complex64: the 480 x 240 grating to 1e-6 against sparse LU, graph replay
identical to direct launches, and the fused and two-sweep paths side by side."""
import numpy as np
import pytest

import workloads as W
from oracle import direct, fdfd, gmres_aug, precond

pytestmark = pytest.mark.gpu


def _inst(seed, nx, ny, npml=3, dx=0.04):
    rng = np.random.default_rng(seed)
    eps = (2.085 + 10.165 * (rng.random((ny, nx)) < 0.4)).astype(np.float32)
    return W.Instance(eps, W.random_complex(rng, nx * ny), nx, ny, dx, 1.55, npml,
                      name=f"f{seed}_{nx}x{ny}")


def _solve(insts, Vs, restart, steps, inner="c128", fused=True, **kw):
    import torch
    from gpu_util import to_dev
    from paper_1902_00090_amd import FdfdOp, Solver
    kmax = max([1] + [0 if v is None else v.shape[1] for v in Vs])
    dt = torch.complex128 if inner == "c128" else torch.complex64
    s = Solver([FdfdOp.from_instance(i) for i in insts], restart=restart, kmax=kmax,
               inner=inner, cgs_passes=1, hist_cap=steps, fused=fused, **kw)
    if any(v is not None for v in Vs):
        s.set_subspace([None if v is None else to_dev(v.T, dt) for v in Vs])
    xs, infos, st = s.solve([to_dev(i.b, torch.complex128) for i in insts], tol=1e-30,
                            maxit=steps)
    hs = [s.history(p) for p in range(len(insts))]
    s.close()
    return [x.cpu().numpy() for x in xs], infos, hs


@pytest.mark.parametrize("k", [0, 4])
@pytest.mark.parametrize("restart", [9, 40])
@pytest.mark.parametrize("nx,ny", [(20, 16), (70, 24)])
def test_fused_history_matches_oracle(nx, ny, restart, k):
    """One problem: a single strip narrower than 30 columns (20 x 16, its halo
    columns wrapping onto its own cells) and three strips with a ragged last
    one (70 x 24); halo rows across the periodic wrap."""
    inst = _inst(400 + nx + k, nx, ny)
    A = fdfd.assemble_instance(inst)
    V = W.random_complex(np.random.default_rng(41 + k), (inst.D, k)) if k else None
    steps = 150
    (x,), (inf,), (h,) = _solve([inst], [V], restart, steps)
    xo, io = gmres_aug.gmres_aug(A, inst.b, V if k else np.zeros((inst.D, 0)), restart=restart,
                                 tol=1e-30, maxit=steps)
    assert inf["iters"] == steps
    np.testing.assert_allclose(h, io["history"][:steps], rtol=1e-7, atol=1e-14)
    np.testing.assert_allclose(x, xo, rtol=0, atol=1e-7 * np.abs(xo).max())


def test_fused_uneven_batch_matches_oracle():
    """Problems of different grids in one lockstep launch, including rows of
    500 cells (eight waves, the last one ragged) and a 1-row-thick band at the
    end."""
    insts = [_inst(500, 20, 16), _inst(501, 33, 25, npml=4), _inst(502, 500, 8, npml=2),
             _inst(503, 130, 41)]
    rng = np.random.default_rng(5)
    Vs = [W.random_complex(rng, (i.D, 3)) if p % 2 else None for p, i in enumerate(insts)]
    steps = 120
    xs, infos, hs = _solve(insts, Vs, 30, steps)
    for p, inst in enumerate(insts):
        A = fdfd.assemble_instance(inst)
        V = Vs[p] if Vs[p] is not None else np.zeros((inst.D, 0))
        xo, io = gmres_aug.gmres_aug(A, inst.b, V, restart=30, tol=1e-30, maxit=steps)
        np.testing.assert_allclose(hs[p], io["history"][:steps], rtol=1e-7, atol=1e-14,
                                   err_msg=inst.name)
        np.testing.assert_allclose(xs[p], xo, rtol=0, atol=1e-7 * np.abs(xo).max(),
                                   err_msg=inst.name)


@pytest.mark.parametrize("kind", ["jacobi", "pml"])
@pytest.mark.parametrize("k", [0, 3])
def test_fused_preconditioned_history_matches_oracle(kind, k):
    inst = _inst(600 + k, 24, 18)
    A = fdfd.assemble_instance(inst)
    pl, pr = (precond.jacobi(A) if kind == "jacobi" else
              precond.pml_scaling(inst.nx, inst.ny, inst.omega, inst.dx, inst.npml))
    V = W.random_complex(np.random.default_rng(61), (inst.D, k)) if k else None
    steps = 150
    (x,), (inf,), (h,) = _solve([inst], [V], 9, steps, precond=kind)
    f, io = precond.gmres_aug_precond(A, inst.b, V if k else np.zeros((inst.D, 0)), pl, pr,
                                      restart=9, tol=1e-30, maxit=steps)
    np.testing.assert_allclose(h, io["history"][:steps], rtol=1e-7, atol=1e-14)
    np.testing.assert_allclose(x, f, rtol=0, atol=1e-6 * np.abs(f).max())


def test_fused_c64_grating_and_graph_replay():
    """480 x 240 grating in complex64 with FP64 restarts to 1e-6: the fused
    path converges to the sparse LU solution; the two-sweep path takes about
    as many steps; graph replay of the fused steps is identical to direct
    launches."""
    import torch
    from paper_1902_00090_amd import FdfdOp, Solver
    inst = W.grating(1000)
    A = fdfd.assemble_instance(inst)
    op = FdfdOp.from_instance(inst)
    b = torch.tensor(inst.b, device="cuda")
    res = {}
    for name, kw in (("fused", dict(fused=True)), ("graph", dict(fused=True, use_graph=True)),
                     ("two-sweep", dict(fused=False))):
        s = Solver([op], restart=100, cgs_passes=1, hist_cap=20000, **kw)
        (x,), (info,), st = s.solve([b], tol=1e-6, maxit=20000)
        res[name] = (x.cpu().numpy(), info, s.history(0))
        s.close()
        print(name, info["iters"], info["rel_res_true"])
    x, info, h = res["fused"]
    assert info["status"] == 0
    rr = np.linalg.norm(inst.b - A @ x) / np.linalg.norm(inst.b)
    assert rr <= 1e-6
    xs = direct.sparse_solve(A, inst.b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-4
    assert np.array_equal(res["graph"][0], x) and np.array_equal(res["graph"][2], h)
    assert abs(info["iters"] - res["two-sweep"][1]["iters"]) <= 0.1 * info["iters"]
