"""GPU CNN predictor (bf16 MFMA forward/backward, Adam) against the float64
oracle at identical weights.  The GPU keeps activations in bf16 (8 bits of
mantissa), so agreement is checked norm-wise at the few-percent level that
eight bf16-rounded layers allow; the oracle's own gradients are pinned by
finite differences on the CPU."""
import numpy as np
import pytest

from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu


def _bf16(a):
    """Round float32 values to bf16 (nearest even), as the GPU stores weights."""
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _setup(nx, ny, B, k, seed, in_ch=1):
    import torch
    from paper_1902_00090_amd import Cnn
    from paper_1902_00090_amd.cnn import flat_to_layers
    net = Cnn(nx, ny, B, k, seed=seed, in_channels=in_ch)
    rng = np.random.default_rng(seed)
    flat = net.get_params()
    layers = net.layers()
    params = flat_to_layers(flat.copy(), layers)
    for w, b in params:                               # non-zero biases
        b[...] = 0.05 * rng.standard_normal(b.shape)
    from paper_1902_00090_amd.cnn import layers_to_flat
    flat = layers_to_flat(params).astype(np.float32)
    net.set_params(flat)
    # the oracle sees the weights the GPU uses: bf16 for layers 2..8, FP32 for layer 1
    op = flat_to_layers(flat.astype(np.float64), layers)
    for li in range(1, 8):
        op[li][0] = _bf16(op[li][0]).astype(np.float64)
    eps = (2.085 + 10.165 * rng.random((B, ny, nx))).astype(np.float32)
    if in_ch == 1:
        return net, op, eps, torch.tensor(eps, device="cuda")
    # a seeded complex field of uneven amplitude stands in for the effective-index input
    eim = ((rng.standard_normal((B, nx * ny)) + 1j * rng.standard_normal((B, nx * ny))) *
           np.linspace(0.5, 3.0, B)[:, None]).astype(np.complex64)
    return net, op, eps, torch.tensor(eps, device="cuda"), eim, torch.tensor(eim, device="cuda")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("nx,ny,B", [(24, 16, 2), (40, 12, 3), (8, 8, 1)])
def test_forward_matches_oracle(nx, ny, B):
    k = 10
    net, op, eps, eps_d = _setup(nx, ny, B, k, seed=nx)
    U = net.predict(eps_d).cpu().numpy()
    out, cache = ocnn.forward(op, eps.astype(np.float64), k)
    # per-layer activations (NHWC on the GPU, NCHW in the oracle)
    for li in range(8):
        a_gpu = net.activation(li, B)
        z = cache[li][2]
        a_ref = np.maximum(z, 0) if li < 7 else z
        assert _rel(a_gpu.transpose(0, 3, 1, 2), a_ref) < 3e-2, li
    assert _rel(U, ocnn.channels_to_fields(out)) < 3e-2


def test_forward_full_size_sampled():
    """480 x 240 (the benchmark's grid), one image: whole-output comparison."""
    k = 10
    net, op, eps, eps_d = _setup(480, 240, 1, k, seed=7)
    U = net.predict(eps_d).cpu().numpy()
    out, _ = ocnn.forward(op, eps.astype(np.float64), k)
    assert _rel(U, ocnn.channels_to_fields(out)) < 3e-2


@pytest.mark.parametrize("nx,ny,k", [(24, 16, 10), (64, 32, 10), (40, 12, 20), (24, 16, 32),
                                     (8, 8, 10)])
def test_gradients_match_oracle(nx, ny, k):
    """Weight gradients: row chunks for the stride-1 and upsampling layers
    (one ragged chunk per row at these widths), flattened pixel stages for the
    stride-2 layers (crossing rows and images, ragged at the end).  k = 20 / 32
    give the last layer 40 / 64 real channels (padded to 64).  8 x 8 shrinks
    the stride-2 layers to 4 x 4 and 2 x 2 outputs; there a weight gradient
    sums so few products that the bf16 rounding of single activations and
    ReLU decisions shows (7% norm-wise at batch 2, 2.7% at batch 8, 1.3% at
    batch 32), so that case runs at batch 8.  Layer 1's gradient runs over
    flattened pixel ranges, crossing rows and images at every width here."""
    import torch
    from paper_1902_00090_amd.cnn import flat_to_layers
    B = 8 if nx * ny <= 64 else 2
    net, op, eps, eps_d = _setup(nx, ny, B, k, seed=3)
    rng = np.random.default_rng(11)
    tgt = (rng.standard_normal((B, k, nx * ny)) + 1j * rng.standard_normal((B, k, nx * ny))) * 0.1
    tgt = tgt.astype(np.complex64)
    loss, g = net.grad(eps_d, torch.tensor(tgt, device="cuda"))
    out, cache = ocnn.forward(op, eps.astype(np.float64), k)
    lo, dout = ocnn.mse(out, ocnn.fields_to_channels(tgt.astype(np.complex128), ny, nx))
    go = ocnn.backward(op, cache, dout, k)
    assert abs(loss - lo) < 1e-2 * lo
    gg = flat_to_layers(g.astype(np.float64), net.layers())
    for li in range(8):
        assert _rel(gg[li][0], go[li][0]) < 6e-2, ("w", li, _rel(gg[li][0], go[li][0]))
        assert _rel(gg[li][1], go[li][1]) < 6e-2, ("b", li, _rel(gg[li][1], go[li][1]))


def test_adam_step_and_training_reduces_loss():
    import torch
    from paper_1902_00090_amd.cnn import flat_to_layers
    nx, ny, B, k = 24, 16, 4, 2
    net, op, eps, eps_d = _setup(nx, ny, B, k, seed=5)
    rng = np.random.default_rng(2)
    tgt = torch.tensor(((rng.standard_normal((B, k, nx * ny)) +
                         1j * rng.standard_normal((B, k, nx * ny))) * 0.3).astype(np.complex64),
                       device="cuda")
    p0 = net.get_params().astype(np.float64)
    _, g = net.grad(eps_d, tgt)
    net.train_step(eps_d, tgt, lr=1e-3)
    p1 = net.get_params().astype(np.float64)
    # one Adam step from zero moments: p1 = p0 - lr * g / (|g| + 1e-8)
    ref = p0 - 1e-3 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p1, ref, atol=2e-7)
    losses = [net.train_step(eps_d, tgt, lr=1e-3) for _ in range(60)]
    assert losses[-1] < 0.7 * losses[0], (losses[0], losses[-1])


@pytest.mark.parametrize("nx,ny", [(24, 16), (64, 32)])
def test_three_channel_forward_and_gradients_match_oracle(nx, ny):
    """Permittivity plus effective-index field (the paper's CNN input): the
    input planes, every layer, the output and all gradients against the
    oracle at identical weights (64 x 32: two full 128-pixel row chunks per
    row in the weight gradients of layers 6-8)."""
    import torch
    from paper_1902_00090_amd.cnn import flat_to_layers
    B, k = 3, 4
    net, op, eps, eps_d, eim, eim_d = _setup(nx, ny, B, k, seed=9, in_ch=3)
    assert net.layers()[0][0] == 3
    U = net.predict(eps_d, eim=eim_d).cpu().numpy()
    out, cache = ocnn.forward(op, eps.astype(np.float64), k, eim=eim.astype(np.complex128))
    x_ref = ocnn.inputs(eps.astype(np.float64), eim.astype(np.complex128))
    np.testing.assert_allclose(net.activation(-1, B), x_ref, rtol=2e-6, atol=2e-6)
    for li in range(8):
        a_gpu = net.activation(li, B)
        z = cache[li][2]
        a_ref = np.maximum(z, 0) if li < 7 else z
        assert _rel(a_gpu.transpose(0, 3, 1, 2), a_ref) < 3e-2, li
    assert _rel(U, ocnn.channels_to_fields(out)) < 3e-2
    rng = np.random.default_rng(12)
    tgt = ((rng.standard_normal((B, k, nx * ny)) + 1j * rng.standard_normal((B, k, nx * ny)))
           * 0.1).astype(np.complex64)
    loss, g = net.grad(eps_d, torch.tensor(tgt, device="cuda"), eim=eim_d)
    lo, dout = ocnn.mse(out, ocnn.fields_to_channels(tgt.astype(np.complex128), ny, nx))
    go = ocnn.backward(op, cache, dout, k)
    assert abs(loss - lo) < 1e-2 * lo
    gg = flat_to_layers(g.astype(np.float64), net.layers())
    for li in range(8):
        assert _rel(gg[li][0], go[li][0]) < 6e-2, ("w", li, _rel(gg[li][0], go[li][0]))
        assert _rel(gg[li][1], go[li][1]) < 6e-2, ("b", li, _rel(gg[li][1], go[li][1]))


def test_full_size_three_planes_forward_and_gradients():
    """The benchmark's network at its grid: 480 x 240, permittivity plus
    effective-index field, k = 10, two images.  Every kernel runs at the
    shapes the benchmark times (LDS-staged weights, the FP32-MFMA layer 1, the
    three-dy weight gradients and the two tap groups of the upsampling
    backward); output and all gradients against the oracle."""
    import torch
    from paper_1902_00090_amd.cnn import flat_to_layers
    nx, ny, B, k = 480, 240, 2, 10
    net, op, eps, eps_d, eim, eim_d = _setup(nx, ny, B, k, seed=21, in_ch=3)
    U = net.predict(eps_d, eim=eim_d).cpu().numpy()
    out, cache = ocnn.forward(op, eps.astype(np.float64), k, eim=eim.astype(np.complex128))
    assert _rel(U, ocnn.channels_to_fields(out)) < 3e-2
    rng = np.random.default_rng(22)
    tgt = ((rng.standard_normal((B, k, nx * ny)) + 1j * rng.standard_normal((B, k, nx * ny)))
           * 0.1).astype(np.complex64)
    loss, g = net.grad(eps_d, torch.tensor(tgt, device="cuda"), eim=eim_d)
    lo, dout = ocnn.mse(out, ocnn.fields_to_channels(tgt.astype(np.complex128), ny, nx))
    go = ocnn.backward(op, cache, dout, k)
    assert abs(loss - lo) < 1e-2 * lo
    gg = flat_to_layers(g.astype(np.float64), net.layers())
    for li in range(8):
        assert _rel(gg[li][0], go[li][0]) < 6e-2, ("w", li, _rel(gg[li][0], go[li][0]))
        assert _rel(gg[li][1], go[li][1]) < 6e-2, ("b", li, _rel(gg[li][1], go[li][1]))


def test_channel_count_is_enforced():
    import torch
    from paper_1902_00090_amd import DDError
    net, op, eps, eps_d = _setup(24, 16, 1, 2, seed=1)
    with pytest.raises(ValueError):
        net.predict(eps_d, eim=torch.zeros((1, 24 * 16), dtype=torch.complex64, device="cuda"))
    net3, _, _, e3, _, f3 = _setup(24, 16, 1, 2, seed=1, in_ch=3)
    with pytest.raises(ValueError):
        net3.predict(e3)
    from paper_1902_00090_amd import _lib
    U = torch.empty((1, 2, 24 * 16), dtype=torch.complex64, device="cuda")
    import ctypes as C
    rc = _lib.lib().predict_subspace(net3._h, C.c_void_p(e3.data_ptr()), 1,
                                     C.c_void_p(U.data_ptr()), None)
    assert rc == _lib.DD_EINVAL
