"""Stencil matvec y = A x on the GPU against the oracle's assembled sparse A
(Sec. 2, Eq. 1), element by element with the componentwise rounding bound."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fdfd

pytestmark = pytest.mark.gpu

CASES = [(64, 64, 10), (37, 29, 5), (480, 240, 20), (3, 3, 0), (129, 7, 2)]


@pytest.mark.parametrize("nx,ny,npml", CASES)
@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_apply_matches_assembled(nx, ny, npml, prec):
    import torch
    from paper_1902_00090_amd import FdfdOp
    from gpu_util import to_dev
    rng = np.random.default_rng(nx * 1000 + ny)
    eps = (2.085 + 10.165 * rng.random((ny, nx))).astype(np.float32)
    omega, dx = 2 * math.pi / 1.55, 0.04
    A = fdfd.assemble(eps, omega, dx, npml)
    x = W.random_complex(rng, nx * ny)
    dt = torch.complex64 if prec == "c64" else torch.complex128
    if prec == "c64":
        x = x.astype(np.complex64).astype(np.complex128)
    op = FdfdOp(eps, omega, dx, npml)
    y = op.apply(to_dev(x, dt)).cpu().numpy().astype(np.complex128)
    yref = A @ x
    u = np.finfo(np.float32 if prec == "c64" else np.float64).eps
    # componentwise bound: each output is 5 products and 4 differences
    bound = 16 * u * (abs(A) @ np.abs(x)) + 1e-300
    assert np.all(np.abs(y - yref) <= bound), float(np.max(np.abs(y - yref) / bound))


def test_apply_grating_c64():
    import torch
    from paper_1902_00090_amd import FdfdOp
    from gpu_util import to_dev
    inst = W.grating(1000)
    A = fdfd.assemble_instance(inst)
    rng = np.random.default_rng(5)
    x = W.random_complex(rng, inst.D).astype(np.complex64).astype(np.complex128)
    op = FdfdOp.from_instance(inst)
    y = op.apply(to_dev(x, torch.complex64)).cpu().numpy().astype(np.complex128)
    bound = 16 * np.finfo(np.float32).eps * (abs(A) @ np.abs(x))
    assert np.all(np.abs(y - A @ x) <= bound)
