"""eim_field_noalloc (the allocation-free variant of eim_field, for callers
that cannot allocate device memory) against eim_field through the C ABI:
identical kernels on identical inputs, so identical outputs, on two calls in
a row (the second smaller), and the size limit enforced on the host."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _problems(insts):
    import torch
    from paper_1902_00090_amd import FdfdOp
    ops = [FdfdOp.from_instance(i) for i in insts]
    bs = [torch.tensor(i.b, dtype=torch.complex128, device="cuda") for i in insts]
    return ops, bs


def test_noalloc_matches_allocating_call_twice():
    import torch
    from paper_1902_00090_amd import eim_field, eim_field_noalloc
    first = [W.grating(2300, nx=480, ny=240), W.grating(2301, nx=192, ny=96, wavelength=1.55),
             W.grating(2302, nx=320, ny=160)]
    second = [W.grating(2303, nx=96, ny=48)]
    for insts in (first, second):
        print("eim_field_noalloc:", [f"{i.nx}x{i.ny}" for i in insts], flush=True)
        ops, bs = _problems(insts)
        ref = eim_field(ops, bs)
        out = [torch.full((op.D,), complex(np.nan, np.nan), dtype=torch.complex64, device="cuda")
               for op in ops]
        eim_field_noalloc(ops, bs, out)
        torch.cuda.synchronize()
        for r, o in zip(ref, out):
            assert torch.isfinite(torch.view_as_real(o)).all()
            assert torch.equal(torch.view_as_real(o), torch.view_as_real(r))


def test_noalloc_rejects_a_batch_beyond_its_scratch():
    import torch
    from paper_1902_00090_amd import DDError, _lib, eim_field_noalloc
    inst = W.grating(2304, nx=480, ny=240)
    ops, bs = _problems([inst])
    n = 18                      # 18 x 1.86 MB > DD_EIM_NOALLOC_BYTES (32 MiB)
    out = [torch.zeros(inst.D, dtype=torch.complex64, device="cuda") for _ in range(n)]
    with pytest.raises(DDError) as ei:
        eim_field_noalloc(ops * n, bs * n, out)
    assert ei.value.status == _lib.DD_EINVAL
    assert "scratch" in _lib.lib().dd_last_error().decode()
    assert all(float(torch.abs(o).max()) == 0.0 for o in out)
