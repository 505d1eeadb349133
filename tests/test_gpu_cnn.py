"""GPU CNN predictor (bf16 MFMA forward/backward, Adam) against the float64
oracle at identical weights, element by element.

The GPU stores activations and the layer gradients in bfloat16 and
accumulates in FP32 (Methods: BF16 with FP32 accumulation).  The oracle is
run with the same storage precision (store="bf16": every stored value is
rounded where the GPU stores it; its arithmetic stays float64), and the test
weights lie on a coarse grid (at most 5 significant bits) so that the bf16
weight copies and the FP32 sums of taps of the upsampling backward pass are
exact.  The two sides then differ only where an FP32 accumulation and the
float64 one fall on different sides of a bfloat16 rounding boundary (one unit
in the last place, 2^-7 relative at most, at a small fraction of elements),
and through what such a difference changes downstream.  The element-wise
bounds follow from that, each against the absolute-value sum behind the
element (its condition):

  activations:  |gpu - ref| <= 2^-7 |ref| + 2^-8 S,  S = (|W| * |x|) + |b|;
  output:       |gpu - ref| <= 2^-20 |ref| + 2^-8 S  (FP32 output);
  gradients:    every entry |gpu - ref| <= 2^-5 S_g, and at least 99% of the
                entries of each tensor within 2^-8 S_g.  S_g = sum over
                pixels |x| dzS (dzS for biases), where dzS = |dz| + m (|W'|^T
                |dz'|) bounds what a layer gradient dz can move by: the
                absolute-value sum of the backward step that formed it from
                the next layer's gradient dz' (m = the ReLU mask, taken as 1
                where the pre-activation lies within 2^-8 S of zero, so
                either mask value is admitted).  The layer-1 input planes
                carry an extra 2^-24 absolute (FP32 normalisation).  Both
                bounds also admit 2^-12 of the tensor's largest S_g, so that an
                entry of a nearly dead channel, negligible next to the
                tensor's dominant entries, is held to that absolute level.

One rounding flip early in the network changes its neighbourhood downstream
(measured: up to 1.4% of S_g at single entries, under 0.3% at the 99.9th
percentile); a mistake such as a wrong tap, channel or pixel, or a dropped
row, moves most entries of a tensor by a sizeable fraction of S_g, which the
99% criterion sees.  The oracle's own gradients are pinned by finite
differences on the CPU.  The whole-tensor distance to the plain float64
network (no storage rounding) is also checked, as a sanity bound on what
bf16 storage costs."""
import numpy as np
import pytest

from oracle import cnn as ocnn

pytestmark = pytest.mark.gpu

FWD_REL, FWD_ABS = 2.0 ** -7, 2.0 ** -8
OUT_REL = 2.0 ** -20
GRAD_MAX, GRAD_Q99, GRAD_FLOOR = 2.0 ** -5, 2.0 ** -8, 2.0 ** -12
IN_FLOOR = 2.0 ** -24


def _bf16(a):
    """Round float32 values to bf16 (nearest even), as the GPU stores weights."""
    return ocnn.round_bf16(a).astype(np.float32)


def _quantise(params, rng):
    """Weights on a grid of 2^e with integer multiples |n| <= 31 (He-uniform
    scale kept), biases on a 2^-10 grid: exact in bf16, and sums of up to four
    taps stay exact in bf16 too."""
    for w, b in params:
        q = 2.0 ** np.ceil(np.log2(np.abs(w).max() / 31.0))
        w[...] = np.clip(np.round(w / q), -31, 31) * q
        b[...] = np.round(0.05 * rng.standard_normal(b.shape) * 1024.0) / 1024.0
    return params


def _setup(nx, ny, B, k, seed, in_ch=1):
    import torch
    from paper_1902_00090_amd import Cnn
    from paper_1902_00090_amd.cnn import flat_to_layers, layers_to_flat
    net = Cnn(nx, ny, B, k, seed=seed, in_channels=in_ch)
    rng = np.random.default_rng(seed)
    params = _quantise(flat_to_layers(net.get_params().astype(np.float64), net.layers()), rng)
    flat = layers_to_flat(params).astype(np.float32)
    net.set_params(flat)
    op = flat_to_layers(flat.astype(np.float64), net.layers())
    for li in range(1, 8):                          # exact: the bf16 copies equal the weights
        assert np.array_equal(_bf16(op[li][0]), op[li][0].astype(np.float32))
    eps = (2.085 + 10.165 * rng.random((B, ny, nx))).astype(np.float32)
    if in_ch == 1:
        return net, op, eps, torch.tensor(eps, device="cuda")
    # a seeded complex field of uneven amplitude stands in for the effective-index input
    eim = ((rng.standard_normal((B, nx * ny)) + 1j * rng.standard_normal((B, nx * ny))) *
           np.linspace(0.5, 3.0, B)[:, None]).astype(np.complex64)
    return net, op, eps, torch.tensor(eps, device="cuda"), eim, torch.tensor(eim, device="cuda")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _within(gpu, ref, bound, what):
    """Element-wise |gpu - ref| <= bound; prints the largest ratio."""
    err = np.abs(np.asarray(gpu, np.float64) - ref)
    ratio = float((err / np.maximum(bound, 1e-300)).max())
    bad = np.argwhere(err > bound)
    print(f"{what}: max |gpu - ref| / bound = {ratio:.3g}")
    assert bad.size == 0, (what, ratio, bad[:5].tolist(), err[tuple(bad[0])],
                           bound[tuple(bad[0])])
    return ratio


def _abs_conv(xin, w, b, s):
    return ocnn.conv_forward(np.abs(xin), np.abs(w), np.abs(b), s)


def check_forward(net, op, eps, k, B, eim=None, Ugpu=None):
    """Every stored activation and the output fields against the bf16-storage
    oracle, element by element; returns the oracle's output and cache."""
    e64 = None if eim is None else eim.astype(np.complex128)
    out, cache = ocnn.forward(op, eps.astype(np.float64), k, eim=e64, store="bf16")
    layers = ocnn.layer_list(k, cache[0][0].shape[1])
    for li in range(8):
        x, xin, z = cache[li]
        S = _abs_conv(xin, op[li][0], op[li][1], layers[li][2])
        if li < 7:
            a_ref = ocnn.round_bf16(np.maximum(z, 0.0))
            a_gpu = net.activation(li, B).transpose(0, 3, 1, 2)
            _within(a_gpu, a_ref, FWD_REL * np.abs(a_ref) + FWD_ABS * S, f"layer {li + 1}")
        else:
            if Ugpu is None:
                continue
            U_ref = ocnn.channels_to_fields(out)
            Sf = ocnn.channels_to_fields(S)
            bound = OUT_REL * np.abs(U_ref) + FWD_ABS * (Sf.real + Sf.imag)
            err = np.abs(Ugpu.real - U_ref.real) + np.abs(Ugpu.imag - U_ref.imag)
            _within(err, 0.0 * err, bound, "output fields")
    return out, cache


def _up_sum(E):
    """Adjoint of the x2 nearest upsampling: sum over each 2 x 2 block."""
    B_, C_, H2, W2 = E.shape
    return E.reshape(B_, C_, H2 // 2, 2, W2 // 2, 2).sum(axis=(3, 5))


def grad_scales(op, cache, dzs, k):
    """Per layer, the absolute-value sums (S_w, S_b) behind each weight and
    bias gradient entry (see the module docstring)."""
    layers = ocnn.layer_list(k, cache[0][0].shape[1])
    out = [None] * 8
    for li in range(7, -1, -1):
        x, xin, z = cache[li]
        dy, dz = dzs[li]
        w, b = op[li]
        dzS = np.abs(dz)
        if li < 7:
            _, xin_n, _ = cache[li + 1]
            P, _, _ = ocnn.conv_backward(np.abs(xin_n), np.abs(op[li + 1][0]),
                                         np.abs(dzs[li + 1][1]), layers[li + 1][2])
            if layers[li + 1][3]:
                P = _up_sum(P)
            m = (z > 0) | (np.abs(z) <= FWD_ABS * _abs_conv(xin, w, b, layers[li][2]))
            dzS = dzS + m * P
        ax = np.abs(xin) + (IN_FLOOR if li == 0 else 0.0)
        _, Sw, Sb = ocnn.conv_backward(ax, np.abs(w), dzS, layers[li][2])
        out[li] = (Sw, Sb)
    return out


def _within_grad(gpu, ref, S, what):
    err = np.abs(np.asarray(gpu, np.float64) - ref)
    floor = GRAD_FLOOR * S.max()
    r = err / np.maximum(S, 1e-300)
    frac_out = float(np.mean(err > GRAD_Q99 * S + floor))
    worst = np.unravel_index(np.argmax(r), r.shape)
    print(f"{what}: max |gpu - ref| / S_g = {r.max():.3g} (that entry's S_g / max S_g = "
          f"{S[worst] / S.max():.3g}), share above 2^-8 S_g = {frac_out:.3g}")
    bad = np.argwhere(err > GRAD_MAX * S + floor)
    assert bad.size == 0, (what, float(r.max()), bad[:5].tolist(), float(err.max() / S.max()))
    assert frac_out <= 0.01, (what, frac_out)


def check_grads(net, op, cache, dout, k, g, store="bf16"):
    """Weight and bias gradients of every layer against the bf16-storage
    oracle's backward pass, element by element."""
    from paper_1902_00090_amd.cnn import flat_to_layers
    dzs = {}
    go = ocnn.backward(op, cache, dout, k, store=store, dzs=dzs)
    gg = flat_to_layers(np.asarray(g, np.float64), net.layers())
    scales = grad_scales(op, cache, dzs, k)
    for li in range(8):
        Sw, Sb = scales[li]
        _within_grad(gg[li][0], go[li][0], Sw, f"dW layer {li + 1}")
        _within_grad(gg[li][1], go[li][1], Sb, f"db layer {li + 1}")
    return go, gg


@pytest.mark.parametrize("nx,ny,B", [(24, 16, 2), (40, 12, 3), (8, 8, 1)])
def test_forward_matches_oracle(nx, ny, B):
    k = 10
    net, op, eps, eps_d = _setup(nx, ny, B, k, seed=nx)
    U = net.predict(eps_d).cpu().numpy()
    check_forward(net, op, eps, k, B, Ugpu=U)
    out64, _ = ocnn.forward(op, eps.astype(np.float64), k)
    assert _rel(U, ocnn.channels_to_fields(out64)) < 3e-2


def test_forward_full_size():
    """480 x 240 (the benchmark's grid), one image: every element."""
    k = 10
    net, op, eps, eps_d = _setup(480, 240, 1, k, seed=7)
    U = net.predict(eps_d).cpu().numpy()
    check_forward(net, op, eps, k, 1, Ugpu=U)


@pytest.mark.parametrize("nx,ny,k", [(24, 16, 10), (64, 32, 10), (40, 12, 20), (24, 16, 32),
                                     (8, 8, 10)])
def test_gradients_match_oracle(nx, ny, k):
    """Weight gradients: row chunks for the stride-1 and stride-2 layers (one
    ragged chunk per row at these widths; stride 2 with the odd and even input
    columns staged apart; the 32-channel layers walk down column chunks with
    a ring of input rows), chunks of source rows for the upsampling layers
    (sixteen parity-shift products mapped onto the nine taps).  k = 20 / 32
    give the last layer 40 / 64 real channels (padded to 64).  8 x 8 shrinks
    the stride-2 layers to 4 x 4 and 2 x 2 outputs (batch 8 there).  Layer 1's
    gradient runs over flattened pixel ranges, crossing rows and images at
    every width here."""
    import torch
    B = 8 if nx * ny <= 64 else 2
    net, op, eps, eps_d = _setup(nx, ny, B, k, seed=3)
    rng = np.random.default_rng(11)
    tgt = (rng.standard_normal((B, k, nx * ny)) + 1j * rng.standard_normal((B, k, nx * ny))) * 0.1
    tgt = tgt.astype(np.complex64)
    loss, g = net.grad(eps_d, torch.tensor(tgt, device="cuda"))
    out, cache = check_forward(net, op, eps, k, B)
    lo, dout = ocnn.mse(out, ocnn.fields_to_channels(tgt.astype(np.complex128), ny, nx))
    assert abs(loss - lo) < 1e-4 * lo, (loss, lo)
    check_grads(net, op, cache, dout, k, g)


def test_gradients_long_row_walks():
    """A tall, narrow grid at batch 16 (32 x 480): the weight-gradient slices
    of layers 7 and 8 walk eight or more consecutive rows of a column chunk
    with the input rows in a ring, and the stride-2 and upsampling kernels
    take several stages per slice.  Every gradient element against the
    oracle."""
    import torch
    nx, ny, B, k = 32, 480, 16, 10
    net, op, eps, eps_d = _setup(nx, ny, B, k, seed=21)
    rng = np.random.default_rng(22)
    tgt = ((rng.standard_normal((B, k, nx * ny)) + 1j * rng.standard_normal((B, k, nx * ny)))
           * 0.1).astype(np.complex64)
    loss, g = net.grad(eps_d, torch.tensor(tgt, device="cuda"))
    out, cache = check_forward(net, op, eps, k, B)
    lo, dout = ocnn.mse(out, ocnn.fields_to_channels(tgt.astype(np.complex128), ny, nx))
    assert abs(loss - lo) < 1e-4 * lo, (loss, lo)
    check_grads(net, op, cache, dout, k, g)


def test_adam_steps_match_oracle():
    """Six Adam steps on the device against the oracle's adam_step fed the
    same gradients (read before each step), element by element; then the
    loss falls under further training."""
    import torch
    from paper_1902_00090_amd.cnn import flat_to_layers
    nx, ny, B, k = 24, 16, 4, 2
    net, op, eps, eps_d = _setup(nx, ny, B, k, seed=5)
    rng = np.random.default_rng(2)
    tgt = torch.tensor(((rng.standard_normal((B, k, nx * ny)) +
                         1j * rng.standard_normal((B, k, nx * ny))) * 0.3).astype(np.complex64),
                       device="cuda")
    layers = net.layers()
    p_ref = flat_to_layers(net.get_params().astype(np.float64), layers)
    state = {}
    lr = 1e-3
    for t in range(1, 7):
        _, g = net.grad(eps_d, tgt)
        net.train_step(eps_d, tgt, lr=lr, b1=0.9, b2=0.999)
        ocnn.adam_step(p_ref, flat_to_layers(g.astype(np.float64), layers), state, lr=lr,
                       b1=0.9, b2=0.999, eps=1e-8)
        p_gpu = net.get_params().astype(np.float64)
        ref = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in p_ref])
        # FP32 moments and update: a few single-precision roundings of the
        # parameter and of each step (whose size is about lr) per step
        bound = t * (4e-7 * np.abs(ref) + 2e-5 * lr)
        _within(p_gpu, ref, bound, f"Adam step {t}")
    losses = [net.train_step(eps_d, tgt, lr=1e-3) for _ in range(100)]
    assert losses[-1] < 0.8 * losses[0], (losses[0], losses[-1])


@pytest.mark.parametrize("nx,ny", [(24, 16), (64, 32)])
def test_three_channel_forward_and_gradients_match_oracle(nx, ny):
    """Permittivity plus effective-index field (the paper's CNN input): the
    input planes, every layer, the output and all gradients against the
    oracle at identical weights (64 x 32: two full 128-pixel row chunks per
    row in the weight gradients of layers 6-8)."""
    import torch
    B, k = 3, 4
    net, op, eps, eps_d, eim, eim_d = _setup(nx, ny, B, k, seed=9, in_ch=3)
    assert net.layers()[0][0] == 3
    U = net.predict(eps_d, eim=eim_d).cpu().numpy()
    x_ref = ocnn.inputs(eps.astype(np.float64), eim.astype(np.complex128))
    np.testing.assert_allclose(net.activation(-1, B), x_ref, rtol=2e-6, atol=2e-6)
    out, cache = check_forward(net, op, eps, k, B, eim=eim, Ugpu=U)
    out64, _ = ocnn.forward(op, eps.astype(np.float64), k, eim=eim.astype(np.complex128))
    assert _rel(U, ocnn.channels_to_fields(out64)) < 3e-2
    rng = np.random.default_rng(12)
    tgt = ((rng.standard_normal((B, k, nx * ny)) + 1j * rng.standard_normal((B, k, nx * ny)))
           * 0.1).astype(np.complex64)
    loss, g = net.grad(eps_d, torch.tensor(tgt, device="cuda"), eim=eim_d)
    lo, dout = ocnn.mse(out, ocnn.fields_to_channels(tgt.astype(np.complex128), ny, nx))
    assert abs(loss - lo) < 1e-4 * lo, (loss, lo)
    check_grads(net, op, cache, dout, k, g)


def test_full_size_three_planes_forward_and_gradients():
    """The benchmark's network at its grid: 480 x 240, permittivity plus
    effective-index field, k = 10, two images.  Every kernel runs at the
    shapes the benchmark times (LDS-staged weights, the FP32-MFMA layer 1, the
    three-dy weight gradients and the two tap groups of the upsampling
    backward); every activation, output element and gradient entry against
    the oracle."""
    import torch
    nx, ny, B, k = 480, 240, 2, 10
    net, op, eps, eps_d, eim, eim_d = _setup(nx, ny, B, k, seed=21, in_ch=3)
    U = net.predict(eps_d, eim=eim_d).cpu().numpy()
    out, cache = check_forward(net, op, eps, k, B, eim=eim, Ugpu=U)
    rng = np.random.default_rng(22)
    tgt = ((rng.standard_normal((B, k, nx * ny)) + 1j * rng.standard_normal((B, k, nx * ny)))
           * 0.1).astype(np.complex64)
    loss, g = net.grad(eps_d, torch.tensor(tgt, device="cuda"), eim=eim_d)
    lo, dout = ocnn.mse(out, ocnn.fields_to_channels(tgt.astype(np.complex128), ny, nx))
    assert abs(loss - lo) < 1e-4 * lo, (loss, lo)
    check_grads(net, op, cache, dout, k, g)


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
    rc = _lib.lib().dd_cnn_predict(net3._h, C.c_void_p(e3.data_ptr()), 1,
                                   C.c_void_p(U.data_ptr()), None)
    assert rc == _lib.DD_EINVAL
