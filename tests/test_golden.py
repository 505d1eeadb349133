"""Stored expected values under tests/golden/, written by tests/golden/make_golden.py
from the oracle alone.  The CPU test re-derives them, so an unintended change to
the oracle's arithmetic (its operator, its GMRES) shows up as a mismatch; the GPU
test compares the library's complex128 solve with the stored history."""
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    with open(os.path.join(HERE, "golden", "small_binary_gmres50.json")) as f:
        return json.load(f)


def test_oracle_reproduces_stored_small_binary_history():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_golden", os.path.join(HERE, "golden", "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    g, now = _golden(), mg.small_binary_gmres50()
    # BLAS summation order may differ between machines: rounding-level slack,
    # and 48 restarts may move the count by a step or two
    assert abs(now["iters"] - g["iters"]) <= 2
    np.testing.assert_allclose(now["history_first_400"], g["history_first_400"], rtol=1e-9)
    assert abs(now["x_norm"] - g["x_norm"]) <= 1e-8 * g["x_norm"]


@pytest.mark.gpu
def test_gpu_solve_matches_stored_small_binary_history():
    import torch
    import workloads as W
    from paper_1902_00090_amd import FdfdOp, Solver
    g = _golden()
    inst = W.small_binary(0)
    s = Solver([FdfdOp.from_instance(inst)], restart=50, inner="c128", hist_cap=20000)
    b = torch.tensor(inst.b, dtype=torch.complex128, device="cuda")
    (x,), (info,), st = s.solve([b], tol=1e-8, maxit=20000)
    assert st == 0
    assert abs(info["iters"] - g["iters"]) <= 0.01 * g["iters"], (info["iters"], g["iters"])
    h = s.history(0)
    np.testing.assert_allclose(h[:400], g["history_first_400"], rtol=1e-7)
    assert abs(float(torch.linalg.norm(x)) - g["x_norm"]) <= 1e-6 * g["x_norm"]
