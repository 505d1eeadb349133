"""Pins of the float64 CNN oracle (Sec. 3 CNN paragraph; Methods: Adam)."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def test_conv_single_channel_is_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 1, 9, 13))
    w = rng.standard_normal((1, 1, 3, 3))
    b = np.array([0.3])
    out = cnn.conv_forward(x, w, b, 1)
    ref = correlate2d(x[0, 0], w[0, 0], mode="same", boundary="fill") + 0.3
    np.testing.assert_allclose(out[0, 0], ref, atol=1e-12)


def test_conv_stride2_is_subsampled_stride1():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 8, 12))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(cnn.conv_forward(x, w, b, 2),
                               cnn.conv_forward(x, w, b, 1)[:, :, ::2, ::2], atol=1e-12)


def test_conv_backward_is_adjoint():
    """<conv(x), z> - <b,sum z> = <x, dX(z)> and = <w, dW(z)> (linear in x and w)."""
    rng = np.random.default_rng(2)
    for s in (1, 2):
        x = rng.standard_normal((2, 3, 8, 10))
        w = rng.standard_normal((5, 3, 3, 3))
        b = np.zeros(5)
        y = cnn.conv_forward(x, w, b, s)
        z = rng.standard_normal(y.shape)
        dx, dw, db = cnn.conv_backward(x, w, z, s)
        np.testing.assert_allclose(np.sum(y * z), np.sum(x * dx), rtol=1e-12)
        np.testing.assert_allclose(np.sum(y * z), np.sum(w * dw), rtol=1e-12)
        np.testing.assert_allclose(db, z.sum(axis=(0, 2, 3)), rtol=1e-12)


@pytest.mark.parametrize("in_ch", [1, 3])
def test_network_gradient_matches_finite_differences(in_ch):
    rng = np.random.default_rng(3)
    k = 2
    params = cnn.init_params(k, seed=4, in_ch=in_ch)
    for p in params:                      # non-zero biases so every term is exercised
        p[1][...] = 0.05 * rng.standard_normal(p[1].shape)
    eps = 2.085 + 10.165 * rng.random((2, 8, 12))
    eim = None
    if in_ch == 3:
        eim = rng.standard_normal((2, 96)) + 1j * rng.standard_normal((2, 96))
    out, cache = cnn.forward(params, eps, k, eim=eim)
    target = rng.standard_normal(out.shape)
    loss, dout = cnn.mse(out, target)
    grads = cnn.backward(params, cache, dout, k)
    h = 1e-6
    for li in range(8):
        for which in (0, 1):
            arr = params[li][which]
            for _ in range(2):
                idx = tuple(rng.integers(0, s) for s in arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                lp, _ = cnn.mse(cnn.forward(params, eps, k, eim=eim)[0], target)
                arr[idx] = old - h
                lm, _ = cnn.mse(cnn.forward(params, eps, k, eim=eim)[0], target)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                an = grads[li][which][idx]
                # central differences with h = 1e-6 carry a rounding error of about
                # eps_mach * loss / h (1e-10 for the loss of the three-plane input)
                tol_abs = 1e-11 if in_ch == 1 else 2e-10
                assert abs(fd - an) <= 1e-6 * max(1e-8, abs(fd)) + tol_abs, (li, which, fd, an)


def test_adam_first_step_closed_form():
    """With zero moments the first bias-corrected step is lr * g / (|g| + eps)."""
    p = [[np.array([1.0, -2.0, 3.0])]]
    g = [[np.array([0.5, -4.0, 1e-3])]]
    st = {}
    cnn.adam_step(p, g, st, lr=0.1)
    np.testing.assert_allclose(p[0][0], [1.0 - 0.1 * 0.5 / (0.5 + 1e-8),
                                         -2.0 + 0.1 * 4.0 / (4.0 + 1e-8),
                                         3.0 - 0.1 * 1e-3 / (1e-3 + 1e-8)], rtol=1e-12)


def test_local_pca_targets():
    rng = np.random.default_rng(5)
    S, D, k = 9, 40, 3
    F = rng.standard_normal((S, D)) + 1j * rng.standard_normal((S, D))
    F /= np.linalg.norm(F, axis=1, keepdims=True)
    T = cnn.local_pca_targets(F, window=2, k=k)
    for s in range(S):
        lo, hi = max(0, s - 2), min(S, s + 3)
        U, _, _ = np.linalg.svd(F[lo:hi].T, full_matrices=False)
        Pf = U[:, :k] @ (U[:, :k].conj().T @ F[s])
        np.testing.assert_allclose(T[s].sum(0), Pf, atol=1e-12)      # sum of targets = projection
        G = T[s] @ T[s].conj().T                                     # targets mutually orthogonal
        np.testing.assert_allclose(G - np.diag(np.diag(G)), 0, atol=1e-12)
    # invariant under a per-step phase of the solutions
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, S))
    T2 = cnn.local_pca_targets(F * ph[:, None], window=2, k=k)
    np.testing.assert_allclose(T2, T * ph[:, None, None], atol=1e-10)
    # a window of identical fields: the target reproduces the field
    G = np.repeat(F[:1], 5, axis=0)
    np.testing.assert_allclose(cnn.local_pca_targets(G, 1, 2)[2].sum(0), F[0], atol=1e-12)


def test_channel_packing_roundtrip():
    rng = np.random.default_rng(6)
    U = rng.standard_normal((2, 3, 20)) + 1j * rng.standard_normal((2, 3, 20))
    Y = cnn.fields_to_channels(U, 4, 5)
    assert Y.shape == (2, 6, 4, 5)
    np.testing.assert_allclose(Y[:, 0], U[:, 0].real.reshape(2, 4, 5))
    np.testing.assert_allclose(Y[:, 1], U[:, 0].imag.reshape(2, 4, 5))
    np.testing.assert_allclose(cnn.channels_to_fields(Y), U)


def test_effective_index_input_planes():
    """Input planes 1 and 2 are the field's real and imaginary parts at unit
    RMS per image; a zero field gives zero planes."""
    rng = np.random.default_rng(5)
    eps = 2.085 + 10.165 * rng.random((2, 4, 6))
    F = rng.standard_normal((2, 24)) + 1j * rng.standard_normal((2, 24))
    F[1] = 0.0
    x = cnn.inputs(eps, 3.0 * F)
    assert x.shape == (2, 3, 4, 6)
    np.testing.assert_allclose(x[0, 1] ** 2 + x[0, 2] ** 2, (np.abs(F[0]) ** 2).reshape(4, 6)
                               / np.mean(np.abs(F[0]) ** 2), rtol=1e-12)
    np.testing.assert_allclose(np.mean(x[0, 1] ** 2 + x[0, 2] ** 2), 1.0, rtol=1e-12)
    assert np.all(x[1, 1:] == 0.0)
    np.testing.assert_allclose(x[:, 0], cnn.normalise(eps), rtol=0)


@pytest.mark.parametrize("b1,b2", [(0.9, 0.999), (0.5, 0.7)])
def test_adam_constant_gradient_every_step(b1, b2):
    """With a constant gradient g and zero initial moments the bias-corrected
    moments are exactly m^ = g and v^ = g^2 at every step t (the corrections
    1 - b^t cancel the geometric sums), so p_t = p_0 - t lr g / (|g| + eps).
    A wrong correction exponent (b instead of b^t) breaks this from t = 2 on."""
    g0 = np.array([0.5, -4.0, 1e-3, 2.5])
    p0 = np.array([1.0, -2.0, 3.0, 0.0])
    p = [[p0.copy()]]
    st = {}
    lr, eps = 0.01, 1e-8
    for t in range(1, 13):
        cnn.adam_step(p, [[g0.copy()]], st, lr=lr, b1=b1, b2=b2, eps=eps)
        np.testing.assert_allclose(p[0][0], p0 - t * lr * g0 / (np.abs(g0) + eps),
                                   rtol=1e-12, atol=1e-15)


def test_adam_alternating_gradient_closed_form():
    """Gradients g, -g, g, -g, ...: the first moment is a geometric sum with
    ratio -b1, m_t = (1 - b1) g sum_{i<t} (-b1)^i (-1)^(t-1) ... in closed form
    m_t = (1-b1)/(1+b1) (1 - (-b1)^t) g (-1)^(t-1), while v_t = (1 - b2^t) g^2.
    Hence the step at t is lr * (1-b1)/(1+b1) * (1 - (-b1)^t)/(1 - b1^t)
    * (-1)^(t-1) g / (|g| + eps); this separates the first and second moments
    and both bias corrections."""
    b1, b2, lr, eps = 0.9, 0.999, 0.1, 0.0
    g0 = np.array([0.3, -1.7, 4.0])
    p = [[np.zeros(3)]]
    st = {}
    ref = np.zeros(3)
    for t in range(1, 9):
        sgn = (-1.0) ** (t - 1)
        cnn.adam_step(p, [[sgn * g0]], st, lr=lr, b1=b1, b2=b2, eps=eps)
        mh = (1 - b1) / (1 + b1) * (1 - (-b1) ** t) / (1 - b1 ** t) * sgn
        ref = ref - lr * mh * g0 / np.abs(g0)
        np.testing.assert_allclose(p[0][0], ref, rtol=1e-12)


def test_round_bf16_matches_library_conversion():
    """The oracle's bfloat16 rounding equals torch's float32 -> bfloat16
    conversion (round to nearest, ties to even) on random values, exact ties,
    subnormals and values near the overflow edge."""
    import torch
    rng = np.random.default_rng(13)
    vals = [rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000)]
    # exact ties: bfloat16 values with the bit just below the kept fraction set
    base = rng.standard_normal(4000).astype(np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
    vals.append((base | np.uint32(0x8000)).view(np.float32).astype(np.float64))
    vals.append(np.array([0.0, -0.0, 1e-40, -3e-39, 3.3e38, -3.3e38, 1.0, 1.00390625]))
    x = np.concatenate(vals)
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(cnn.round_bf16(x), ref.astype(np.float64))
    np.testing.assert_array_equal(cnn.round_f32(x), x.astype(np.float32).astype(np.float64))


def test_storage_rounding_only_rounds():
    """forward/backward with bf16 storage stay within bfloat16 rounding of the
    float64 network on a small case (the arithmetic is the same), and every
    stored activation and layer gradient is a bfloat16 value."""
    rng = np.random.default_rng(14)
    k = 2
    params = cnn.init_params(k, seed=2)
    eps = 2.085 + 10.165 * rng.random((2, 24, 32))
    o64, c64 = cnn.forward(params, eps, k)
    o16, c16 = cnn.forward(params, eps, k, store="bf16")
    assert np.linalg.norm(o16 - o64) / np.linalg.norm(o64) < 3e-2
    for li in range(1, 8):
        a = c16[li][0]                      # input of layer li = stored activation of li - 1
        np.testing.assert_array_equal(a, cnn.round_bf16(a))
    tgt = rng.standard_normal(o16.shape)
    _, d16 = cnn.mse(o16, tgt)
    g16 = cnn.backward(params, c16, d16, k, store="bf16")
    _, d64 = cnn.mse(o64, tgt)
    g64 = cnn.backward(params, c64, d64, k)
    for li in range(8):
        assert np.linalg.norm(g16[li][0] - g64[li][0]) / np.linalg.norm(g64[li][0]) < 6e-2
