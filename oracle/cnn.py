"""Float64 convolutional subspace predictor: forward, backward, MSE loss, Adam.

Test infrastructure (oracle): see the package docstring.

Sec. 3 (CNN paragraph) and Methods: a convolutional network maps the
permittivity image to N complex fields v_1..v_N; complex quantities are
images with a real and an imaginary channel; training uses Adam.  The
architecture figure of the paper is not available; the layer list below is
the reading used throughout (an encoder-decoder of eight 3x3 convolutions):

    1->32, 32->64 (stride 2), 64->128 (stride 2), 128->128,
    nearest x2 upsample + 128->64, nearest x2 upsample + 64->32, 32->32,
    32->2k (linear); ReLU after every layer but the last; zero padding 1.

Input planes: (eps - 2.085) / (12.25 - 2.085), and, for the three-channel
network the paper uses (permittivity plus effective-index field, Sec. 3),
the real and imaginary parts of the effective-index field F scaled to unit
RMS per pixel (F sqrt(D) / ||F||, per image; complex inputs as two real
channels, Methods).  Output channel 2j holds Re v_j and channel 2j+1 holds
Im v_j.

Tensors are NCHW float64; weights are [out, in, 3, 3] (cross-correlation, as
every deep-learning convolution).
"""
from __future__ import annotations

import numpy as np

EPS_LO, EPS_HI = 2.085, 12.25


def layer_list(k: int = 10, in_ch: int = 1):
    """(cin, cout, stride, upsample_before, relu) per layer."""
    return [(in_ch, 32, 1, 0, 1), (32, 64, 2, 0, 1), (64, 128, 2, 0, 1), (128, 128, 1, 0, 1),
            (128, 64, 1, 1, 1), (64, 32, 1, 1, 1), (32, 32, 1, 0, 1), (32, 2 * k, 1, 0, 0)]


def normalise(eps):
    return (np.asarray(eps, np.float64) - EPS_LO) / (EPS_HI - EPS_LO)


def inputs(eps, eim=None):
    """Network input planes [B, C, H, W]: C = 1 without, 3 with the
    effective-index fields eim [B, H*W] (complex)."""
    x = normalise(eps)[:, None]
    if eim is None:
        return x
    B, H, W = x.shape[0], x.shape[2], x.shape[3]
    F = np.asarray(eim, np.complex128).reshape(B, H, W)
    nrm = np.sqrt((np.abs(F) ** 2).sum(axis=(1, 2)) / (H * W))
    G = F / np.where(nrm > 0, nrm, np.inf)[:, None, None]
    return np.concatenate([x, G.real[:, None], G.imag[:, None]], axis=1)


def init_params(k: int = 10, seed: int = 0, in_ch: int = 1):
    """He-uniform weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout, _, _, _ in layer_list(k, in_ch):
        bound = np.sqrt(6.0 / (cin * 9))
        params.append([rng.uniform(-bound, bound, (cout, cin, 3, 3)), np.zeros(cout)])
    return params


def upsample2(x):
    return x.repeat(2, axis=2).repeat(2, axis=3)


def conv_forward(x, w, b, stride):
    """out[n,o,y,x] = b[o] + sum_{c,dy,dx} w[o,c,dy,dx] xpad[n,c,y*s+dy,x*s+dx]."""
    n, c, H, W = x.shape
    Ho, Wo = (H - 1) // stride + 1, (W - 1) // stride + 1
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.broadcast_to(b[None, :, None, None], (n, w.shape[0], Ho, Wo)).copy()
    for dy in range(3):
        for dx in range(3):
            patch = xp[:, :, dy:dy + stride * (Ho - 1) + 1:stride, dx:dx + stride * (Wo - 1) + 1:stride]
            out += np.einsum("nchw,oc->nohw", patch, w[:, :, dy, dx], optimize=True)
    return out


def conv_backward(x, w, dz, stride):
    """Gradients of conv_forward w.r.t. x, w, b given dL/dout = dz."""
    n, c, H, W = x.shape
    Ho, Wo = dz.shape[2], dz.shape[3]
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for dy in range(3):
        for dx in range(3):
            sl = (slice(None), slice(None), slice(dy, dy + stride * (Ho - 1) + 1, stride),
                  slice(dx, dx + stride * (Wo - 1) + 1, stride))
            dw[:, :, dy, dx] = np.einsum("nohw,nchw->oc", dz, xp[sl], optimize=True)
            dxp[sl] += np.einsum("nohw,oc->nchw", dz, w[:, :, dy, dx], optimize=True)
    return dxp[:, :, 1:-1, 1:-1], dw, dz.sum(axis=(0, 2, 3))


def round_f32(a):
    """Nearest IEEE single-precision value, as float64."""
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def round_bf16(a):
    """Nearest bfloat16 value, as float64.  bfloat16 is the upper half of an
    IEEE single (sign, 8 exponent bits, 7 fraction bits); the value is first
    rounded to single precision, then to the nearest bfloat16, ties to the
    even fraction (adding 0x7FFF plus the lowest kept bit to the 32-bit
    pattern and truncating the lower 16 bits does exactly that)."""
    u = np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32)).view(np.uint32)
    u = u.astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


STORE = {None: (lambda a: a, lambda a: a, lambda a: a),
         "bf16": (round_f32, round_bf16, round_f32)}


def forward(params, eps, k: int = 10, eim=None, store=None):
    """eps: [B, H, W] permittivity; eim: [B, H*W] effective-index fields for a
    three-channel network.  Returns (out [B, 2k, H, W], cache).

    store: None keeps every value in float64.  "bf16" rounds the values the
    method stores between layers to their storage precision (BF16 with FP32
    accumulation): the input planes to single precision, each hidden layer's
    activation to bfloat16, the output fields to single precision.  The
    arithmetic of every layer stays float64."""
    r_in, r_act, r_out = STORE[store]
    x = r_in(inputs(eps, eim))
    cache = []
    layers = layer_list(k, x.shape[1])
    for li, ((cin, cout, s, up, relu), (w, b)) in enumerate(zip(layers, params)):
        xin = upsample2(x) if up else x
        z = conv_forward(xin, w, b, s)
        y = np.maximum(z, 0.0) if relu else z
        y = r_act(y) if li < len(layers) - 1 else r_out(y)
        cache.append((x, xin, z))
        x = y
    return x, cache


def mse(out, target):
    d = out - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(params, cache, dout, k: int = 10, store=None, dzs=None):
    """Gradients [[dw, db], ...] of the loss whose derivative w.r.t. the output is dout.

    store: as in forward; "bf16" rounds each layer's gradient with respect
    to its pre-activation (the value stored between the backward layers) to
    bfloat16.  dzs: an optional dict that receives, by layer, the pair (gradient
    with respect to the layer output, gradient with respect to its
    pre-activation)."""
    rnd = STORE[store][1]
    grads = [None] * len(params)
    dy = dout
    for li in range(len(params) - 1, -1, -1):
        cin, cout, s, up, relu = layer_list(k)[li]
        x, xin, z = cache[li]
        dz = rnd(dy * (z > 0) if relu else dy)
        if dzs is not None:
            dzs[li] = (dy, dz)
        dxin, dw, db = conv_backward(xin, params[li][0], dz, s)
        grads[li] = [dw, db]
        if up:
            B, C, H2, W2 = dxin.shape
            dxin = dxin.reshape(B, C, H2 // 2, 2, W2 // 2, 2).sum(axis=(3, 5))
        dy = dxin
    return grads


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba): state = {'t': int, 'm': [...], 'v': [...]} updated in place."""
    if not state:
        state.update(t=0, m=[[np.zeros_like(a) for a in p] for p in params],
                     v=[[np.zeros_like(a) for a in p] for p in params])
    state["t"] += 1
    t = state["t"]
    for p, g, m, v in zip(params, grads, state["m"], state["v"]):
        for i in range(len(p)):
            m[i][...] = b1 * m[i] + (1 - b1) * g[i]
            v[i][...] = b2 * v[i] + (1 - b2) * g[i] * g[i]
            mh = m[i] / (1 - b1 ** t)
            vh = v[i] / (1 - b2 ** t)
            p[i][...] = p[i] - lr * mh / (np.sqrt(vh) + eps)


def fields_to_channels(U, H, W):
    """U: [B, k, H*W] complex -> [B, 2k, H, W] real (re, im interleaved by channel)."""
    B, k, _ = U.shape
    out = np.empty((B, 2 * k, H, W))
    out[:, 0::2] = U.real.reshape(B, k, H, W)
    out[:, 1::2] = U.imag.reshape(B, k, H, W)
    return out


def channels_to_fields(Y):
    B, C, H, W = Y.shape
    return (Y[:, 0::2] + 1j * Y[:, 1::2]).reshape(B, C // 2, H * W)


def local_pca_targets(F, window: int, k: int):
    """Training targets for one trajectory (reading of the config: MSE against
    the top-k local PCA projection).  F: [S, D] complex solutions of the steps
    of one trajectory, each normalised to unit norm.  For step s, U_loc = the
    top-k left singular vectors of the solutions of steps s-window..s+window;
    target field j = u_j (u_j^H f_s).  Returns [S, k, D] complex."""
    S, D = F.shape
    out = np.zeros((S, k, D), np.complex128)
    for s in range(S):
        lo, hi = max(0, s - window), min(S, s + window + 1)
        U, _, _ = np.linalg.svd(F[lo:hi].T, full_matrices=False)
        kk = min(k, U.shape[1])
        c = U[:, :kk].conj().T @ F[s]
        out[s, :kk] = (U[:, :kk] * c[None, :]).T
    return out
