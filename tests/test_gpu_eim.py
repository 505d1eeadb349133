"""GPU effective-index field (the CNN's second input) against the oracle.

FP64 arithmetic on both sides.  The GPU result is rounded to complex64, so
agreement is checked element-wise to a few float32 ulps of the field's scale.
Covered: a small grating, the 480 x 240 grating of the benchmark, an uneven
batch, and the separable case where the effective-index field is the exact
2D solution."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import eim, fdfd

pytestmark = pytest.mark.gpu


def _gpu(insts):
    import torch
    from paper_1902_00090_amd import FdfdOp, eim_field
    ops = [FdfdOp.from_instance(i) for i in insts]
    bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in insts]
    return [f.cpu().numpy().astype(np.complex128) for f in eim_field(ops, bs)]


def _check(Fg, Fo):
    scale = np.abs(Fo).max()
    err = np.abs(Fg - Fo).max() / scale
    assert err < 2e-6, err


def test_small_grating_matches_oracle():
    inst = W.grating(1000, nx=96, ny=48)
    (Fg,) = _gpu([inst])
    _check(Fg, eim.eim_instance(inst))


def test_full_size_grating_and_uneven_batch():
    insts = [W.grating(1001), W.grating(1002, nx=192, ny=96, wavelength=1.55),
             W.grating(1003, nx=320, ny=160)]
    for Fg, inst in zip(_gpu(insts), insts):
        _check(Fg, eim.eim_instance(inst))


def test_separable_case_is_the_2d_solution():
    ny, nx, dx, lam, npml = 240, 96, 0.025, 1.30, 20
    ey = np.full(ny, W.EPS_SIO2)
    r0, r1 = W.waveguide_rows(ny, dx)
    ey[r0:r1] = W.EPS_SI
    # multiples of 1/64 keep every float32 sum exact, so eps stays separable
    ex = np.round(32.0 * np.sin(np.arange(nx) / 7.0) ** 2) / 64.0
    eps = (ex[None, :] + ey.astype(np.float32)[:, None].astype(np.float64)).astype(np.float32)
    assert np.array_equal(eps.astype(np.float64), ex[None, :] + ey.astype(np.float32)[:, None])
    omega = 2 * math.pi / lam
    b = W.rhs_from_current(W.slab_mode_source(eps, 30, dx, omega), omega)
    inst = W.Instance(eps, b, nx, ny, dx, lam, npml, name="separable")
    import torch
    from paper_1902_00090_amd import FdfdOp, eim_field
    op = FdfdOp(eps, omega, dx, npml, npml_y=0)
    (Fg,) = eim_field([op], [torch.tensor(b, device="cuda")])
    A = fdfd.assemble(eps, omega, dx, npml, npml_y=0)
    f = spla.spsolve(A.tocsc(), b)
    Fg = Fg.cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(Fg - f) / np.linalg.norm(f) < 1e-6


def test_odd_grids_and_pml_on_one_axis():
    """Grids that are not multiples of the launch tiles, and an operator with
    no y-PML (the effective-index field only uses the x stretching)."""
    import torch
    from paper_1902_00090_amd import FdfdOp, eim_field
    insts = [W.grating(1010, nx=97, ny=43, npml=7), W.grating(1011, nx=130, ny=61, npml=12)]
    ops = [FdfdOp.from_instance(insts[0]), FdfdOp(insts[1].eps, insts[1].omega, insts[1].dx,
                                                  insts[1].npml, npml_y=0)]
    F = eim_field(ops, [torch.tensor(i.b, device="cuda") for i in insts])
    for f, inst in zip(F, insts):
        _check(f.cpu().numpy().astype(np.complex128), eim.eim_instance(inst))
