"""Trajectory recycling (the approach the paper contrasts with, Sec. 1; the
supplement's GCROT keeps correction directions between cycles): later design
steps augmented by the fields of earlier ones, and by the harmonic Ritz
vectors of the previous step's last cycle, against the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import fdfd, recycle

pytestmark = pytest.mark.gpu


def test_recycled_trajectory_solves():
    from paper_1902_00090_amd.recycle import solve_trajectories
    trajs = [W.trajectory(7000 + t, 700000 + 100 * t, 6, 96, 48, 1.30) for t in range(4)]
    xr, ir, hr, _ = solve_trajectories(trajs, window=3, tol=1e-7, restart=40, hist_cap=50)
    xp, ip, hp, _ = solve_trajectories(trajs, recycle=False, tol=1e-7, restart=40, hist_cap=50)
    xh, ih, hh, th = solve_trajectories(trajs, window=3, ritz=6, tol=1e-7, restart=40,
                                        hist_cap=50)
    r1_rec = np.mean([hr[t][s][0] for t in range(4) for s in range(1, 6)])
    r1_pl = np.mean([hp[t][s][0] for t in range(4) for s in range(1, 6)])
    it_rec = sum(ir[t][s]["iters"] for t in range(4) for s in range(6))
    it_pl = sum(ip[t][s]["iters"] for t in range(4) for s in range(6))
    it_h = sum(ih[t][s]["iters"] for t in range(4) for s in range(6))
    print(f"recycled: residual after 1 iteration {r1_rec:.3e} vs plain {r1_pl:.3e}; "
          f"iterations {it_rec} (solutions), {it_h} (solutions + 6 harmonic Ritz) vs {it_pl}")
    assert all(i["status"] == 0 for row in ir + ih for i in row)
    assert all(ir[t][0]["k_used"] == 0 and ir[t][3]["k_used"] == 3 for t in range(4))
    # a short last cycle (a refinement restart) spans fewer than 6 directions
    assert all(1 <= len(th[t][s]) <= 6 and np.all(np.diff(np.abs(th[t][s])) >= 0)
               for t in range(4) for s in range(5))
    assert all(ih[t][3]["k_used"] == 3 + len(th[t][2]) for t in range(4))
    assert r1_rec < 0.5 * r1_pl
    for t in range(4):
        for s in range(6):
            b = xp[t][s].cpu().numpy()
            for x in (xr, xh):
                a = x[t][s].cpu().numpy()
                assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-4


def _span_gap(Y1, Y2):
    Q1, _ = np.linalg.qr(Y1)
    Q2, _ = np.linalg.qr(Y2)
    return np.linalg.norm(Q1 - Q2 @ (Q2.conj().T @ Q1))


def _run_sequence(trajs, kr, m, tol, maxit, fused=False):
    """GPU: the recycled sequence of each trajectory, all trajectories in one
    complex128 batch (two Gram-Schmidt passes; one on the one-sweep path).
    Per step: (x, infos, histories) and, for all but the last step, (Y,
    theta) passed on."""
    import torch
    from paper_1902_00090_amd import FdfdOp, Solver
    solver, Y, out = None, None, []
    for s in range(len(trajs[0])):
        ops = [FdfdOp.from_instance(tr[s]) for tr in trajs]
        bs = [torch.tensor(tr[s].b, dtype=torch.complex128, device="cuda") for tr in trajs]
        if solver is None:
            solver = Solver(ops, restart=m, kmax=kr, inner="c128", cgs_passes=1 if fused else 2,
                            hist_cap=maxit, fused=fused)
        else:
            solver.bind(ops)
        solver.set_subspace(Y)
        xs, infos, _ = solver.solve(bs, tol=tol, maxit=maxit)
        hist = [solver.history(t) for t in range(len(trajs))]
        rec = None
        if s + 1 < len(trajs[0]):
            Y, th = solver.recycle(kr)
            rec = ([y.cpu().numpy().T for y in Y], th)
        out.append(([x.cpu().numpy() for x in xs], infos, hist, rec))
    solver.close()
    return out


TRAJS = [(7000, 700000, 24, 16), (7004, 700100, 20, 16)]


@pytest.mark.parametrize("kr,fused", [(4, False), (7, False), (4, True)])
def test_harmonic_ritz_recycling_matches_the_oracle_c128(kr, fused):
    """Element-wise parity over short solves (two full GMRES(15) cycles per
    step, so rounding has not yet reordered the iterations): two trajectories
    of three steps on grids of two sizes in one complex128 batch.  Per step the
    residual histories match the oracle's recycled sequence (rtol 1e-7); the
    harmonic Ritz values passed on match (rtol 1e-8); the recycled vectors
    span the oracle's space (gap 1e-8) with ||A y|| = 1."""
    m, maxit = 15, 30
    trajs = [W.trajectory(b, s0, 3, nx, ny, 1.30, npml=3) for b, s0, nx, ny in TRAJS]
    gpu = _run_sequence(trajs, kr, m, 1e-14, maxit, fused)
    for t, tr in enumerate(trajs):
        As = [fdfd.assemble_instance(i) for i in tr]
        seq = recycle.solve_sequence(As, [i.b for i in tr], kr=kr, restart=m, tol=1e-14,
                                     maxit=maxit)
        for s in range(3):
            _, infos, hist, rec = gpu[s]
            _, info_o, _, th_o = seq[s]
            assert infos[t]["iters"] == info_o["iters"] == maxit
            np.testing.assert_allclose(hist[t], info_o["history"], rtol=1e-7, atol=1e-14)
            if s > 0:
                assert infos[t]["k_used"] == kr
            if rec is not None:
                y, th = rec[0][t], rec[1][t]
                assert y.shape[1] == kr
                np.testing.assert_allclose(th, th_o, rtol=1e-8)
                gap = _span_gap(y, seq[s + 1][2])
                print(f"kr {kr} traj {t} step {s}: |theta| {np.abs(th).round(2)}, span gap {gap:.1e}")
                assert gap <= 1e-8
                np.testing.assert_allclose(np.linalg.norm(As[s] @ y, axis=0), 1.0, rtol=1e-9)


def test_harmonic_ritz_recycling_converged_sequence_c128():
    """The same trajectories solved to 1e-9 at every step (hundreds of
    restarted iterations, where rounding differences grow): iteration counts
    within 2% of the oracle's, harmonic Ritz values within 2%, every solution
    within 1e-6 of dense LU."""
    from oracle import direct
    kr, m, tol = 4, 15, 1e-9
    trajs = [W.trajectory(b, s0, 3, nx, ny, 1.30, npml=3) for b, s0, nx, ny in TRAJS]
    gpu = _run_sequence(trajs, kr, m, tol, 4000)
    for t, tr in enumerate(trajs):
        As = [fdfd.assemble_instance(i) for i in tr]
        seq = recycle.solve_sequence(As, [i.b for i in tr], kr=kr, restart=m, tol=tol, maxit=4000)
        for s in range(3):
            xs, infos, _, rec = gpu[s]
            _, info_o, _, th_o = seq[s]
            print(f"traj {t} step {s}: iters {infos[t]['iters']} (oracle {info_o['iters']})")
            assert infos[t]["status"] == 0
            assert abs(infos[t]["iters"] - info_o["iters"]) <= 0.02 * info_o["iters"]
            xd = direct.dense_solve(As[s], tr[s].b)
            assert np.linalg.norm(xs[t] - xd) / np.linalg.norm(xd) <= 1e-6
            if rec is not None and infos[t]["iters"] == info_o["iters"]:
                # the last cycle follows hundreds of restarted steps whose
                # rounding differs: the pairs agree only approximately
                y, th = rec[0][t], rec[1][t]
                np.testing.assert_allclose(th, th_o[:len(th)], rtol=2e-2)
                np.testing.assert_allclose(np.linalg.norm(As[s] @ y, axis=0), 1.0, rtol=1e-9)


def test_recycle_reports_misuse():
    import torch
    from paper_1902_00090_amd import DDError, FdfdOp, Solver
    inst = W.grating(1300, nx=48, ny=32, npml=6)
    op = FdfdOp.from_instance(inst)
    b = [torch.tensor(inst.b, dtype=torch.complex128, device="cuda")]
    s = Solver([op], restart=10, kmax=4)
    with pytest.raises(DDError):
        s.recycle(4)                                   # no solve yet
    s.solve(b, tol=1e-3, maxit=200)
    Y, th = s.recycle(4)
    assert Y[0].shape == (4, inst.D)
    s.set_subspace(Y)
    with pytest.raises(DDError):
        s.recycle(4)                                   # set_subspace replaced the cycle
    with pytest.raises(ValueError):
        s.recycle(0)
    s.close()
    f = Solver([op], restart=10, kmax=4, precond="pml")
    f.solve(b, tol=1e-3, maxit=200)
    with pytest.raises(DDError):
        f.recycle(4)                                   # the preconditioned operator is not A
    f.close()


def test_recycle_edge_cases():
    """A problem already solved at the start (x0 exact: no cycle runs) keeps
    only its augmenting vectors' span; a short last cycle gives fewer vectors
    than asked for; a duplicated augmenting column is dropped and recycling
    works on the kept ones."""
    import torch
    from paper_1902_00090_amd import FdfdOp, Solver
    insts = [W.grating(1400 + i, nx=48, ny=32, npml=6) for i in range(2)]
    ops = [FdfdOp.from_instance(i) for i in insts]
    bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in insts]
    from oracle import direct, fdfd
    s = Solver(ops, restart=12, kmax=6, inner="c128", cgs_passes=2)
    # problem 1 starts from its exact solution (sparse LU): no cycle and no
    # subspace, so nothing to recycle
    x1 = torch.tensor(direct.sparse_solve(fdfd.assemble_instance(insts[1]), insts[1].b),
                      dtype=torch.complex128, device="cuda")
    _, infos, _ = s.solve(bs, x0=[torch.zeros_like(bs[0]), x1], tol=1e-9, maxit=300)
    assert infos[1]["iters"] == 0 and infos[0]["iters"] > 12
    Y, th = s.recycle(3)
    assert Y[0].shape[0] == 3 and Y[1].shape[0] == 0
    # a short cycle: 2 steps give at most 2 vectors
    s.solve(bs, tol=0.0, maxit=2)
    Y, th = s.recycle(5)
    assert Y[0].shape[0] == 2 and Y[1].shape[0] == 2
    assert np.all(np.isfinite(th[:, :2])) and np.all(th[:, 2:] == 0)
    # a duplicated column is dropped (k_used 3 of 4); recycling uses the kept 3
    rng = np.random.default_rng(1)
    v = torch.tensor(W.random_complex(rng, (3, insts[0].D)), device="cuda")
    U = torch.cat([v, v[:1]]).contiguous()
    s.set_subspace([U, U])
    _, infos, _ = s.solve(bs, tol=0.0, maxit=12)
    assert infos[0]["k_used"] == 3
    Y, th = s.recycle(6)
    assert Y[0].shape[0] == 6 and torch.isfinite(torch.view_as_real(Y[0])).all()
    A = fdfd.assemble_instance(insts[0])
    y = Y[0].cpu().numpy().T
    np.testing.assert_allclose(np.linalg.norm(A @ y, axis=0), 1.0, rtol=1e-9)
    s.close()
