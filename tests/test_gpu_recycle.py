"""Trajectory recycling (the approach the paper contrasts with, Sec. 1):
later design steps augmented by the fields of earlier ones start from a far
smaller residual and reach the same solutions."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_recycled_trajectory_solves():
    from paper_1902_00090_amd.recycle import solve_trajectories
    trajs = [W.trajectory(7000 + t, 700000 + 100 * t, 6, 96, 48, 1.30) for t in range(4)]
    xr, ir, hr = solve_trajectories(trajs, window=3, tol=1e-7, restart=40, hist_cap=50)
    xp, ip, hp = solve_trajectories(trajs, recycle=False, tol=1e-7, restart=40, hist_cap=50)
    r1_rec = np.mean([hr[t][s][0] for t in range(4) for s in range(1, 6)])
    r1_pl = np.mean([hp[t][s][0] for t in range(4) for s in range(1, 6)])
    it_rec = sum(ir[t][s]["iters"] for t in range(4) for s in range(6))
    it_pl = sum(ip[t][s]["iters"] for t in range(4) for s in range(6))
    print(f"recycled: residual after 1 iteration {r1_rec:.3e} vs plain {r1_pl:.3e}; "
          f"iterations {it_rec} vs {it_pl}")
    assert all(i["status"] == 0 for row in ir for i in row)
    assert all(ir[t][0]["k_used"] == 0 and ir[t][3]["k_used"] == 3 for t in range(4))
    assert r1_rec < 0.5 * r1_pl
    for t in range(4):
        for s in range(6):
            a, b = xr[t][s].cpu().numpy(), xp[t][s].cpu().numpy()
            assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-4
