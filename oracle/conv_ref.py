"""FP64 CPU oracle of the learned 64-level propagator (the surrogate).

TEST INFRASTRUCTURE ONLY: used by the tests to check the GPU network's
forward pass and gradients; the GPU library never calls it.

The network (a reading of the unstated details): a 1D convolutional net
over the n points of a rod, channels-last tensors x[b, w, c].

    layer 1 : pre1 = conv_1(x, W1) + b1,           h1 = gelu(pre1)       (2 -> 64)
    layer l : pre_l = conv_l(h_{l-1}, W_l) + b_l,  h_l = h_{l-1} + gelu(pre_l)
              for l = 2..5                                             (64 -> 64)
    layer 6 : out = conv_6(h5, W6) + b6                                  (64 -> 1)

    conv_l(x, W)[b, w, o] = sum_{k=0..4} sum_i W[k, o, i] x[b, w + (k - 2) d_l, i],
    dilations d = (1, 2, 4, 8, 16, 1), x = 0 outside the rod (zero padding),
    gelu(z) = (z/2) (1 + tanh(c (z + 0.044715 z^3))), c = sqrt(2/pi): the
    tanh form of z Phi(z) (within 4.8e-4 of it for every z), whose GPU
    evaluation needs one exponential and one reciprocal.  The dilations give a
    receptive field of +-64 points: 64 levels of the sweep move a point's
    influence about as far (at r = 2 a fifth of the increment caused by a
    point lies more than 13 points away, which a plain kernel-5 stack of six
    layers cannot see).

Loss: mean over (b, w) of (out[b, w, 0] - t[b, w])^2.

Around the network (``features``, ``target``, ``jump``): the input of a
rod u (zero walls) is its second difference D_i = u_{i-1} - 2 u_i + u_{i+1}
scaled by its root mean square s, and the mesh ratio mapped from [0.5, 2]
to [-1, 1]; the network predicts the 64-level increment in units of 64 r s,
which is about one explicit step of length 64 tau (u_t = u_xx gives
du ~ 64 tau u_xx = 64 r D).

With ``bf16=True`` the forward and backward round to bfloat16 (round to
nearest even) at the places where the GPU stores bfloat16: the input, the
weights, every pre-activation and activation, the loss gradient, and every
activation gradient; accumulation stays in FP64 here (FP32 on the GPU).
"""
import math

import numpy as np

LAYERS = [(2, 64), (64, 64), (64, 64), (64, 64), (64, 64), (64, 1)]
DILATIONS = [1, 2, 4, 8, 16, 1]
TAPS = 5


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), via FP32."""
    a32 = np.asarray(a, dtype=np.float32)
    bits = a32.view(np.uint32).astype(np.uint64)
    rounded = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32)
    # keep NaN/Inf as they are
    out = np.where(np.isfinite(a32), out, a32)
    return out.astype(np.float64)


GELU_C = math.sqrt(2.0 / math.pi)
GELU_A = 0.044715


def gelu(z):
    """(z/2) (1 + tanh(c (z + a z^3)))."""
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + GELU_A * z ** 3)))


def gelu_grad(z):
    """d gelu / dz = (1 + tanh w)/2 + (z/2) (1 - tanh^2 w) c (1 + 3 a z^2),
    w = c (z + a z^3)."""
    t = np.tanh(GELU_C * (z + GELU_A * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * z * z)


def conv(x, w, d=1):
    """x: (B, W, Ci), w: (5, Co, Ci) -> (B, W, Co): taps at offsets (k - 2) d,
    zero padding."""
    B, Wn, Ci = x.shape
    pad = 2 * d
    xp = np.zeros((B, Wn + 2 * pad, Ci))
    xp[:, pad:pad + Wn] = x
    out = np.zeros((B, Wn, w.shape[1]))
    for k in range(TAPS):
        out += xp[:, k * d:k * d + Wn] @ w[k].T
    return out


def conv_input_grad(g, w, d=1):
    """Gradient of conv(x, w, d) w.r.t. x for output gradient g (B, W, Co)."""
    B, Wn, Co = g.shape
    pad = 2 * d
    gp = np.zeros((B, Wn + 2 * pad, Co))
    gp[:, pad:pad + Wn] = g
    out = np.zeros((B, Wn, w.shape[2]))
    # x[w'] receives W[k] g[w' - (k - 2) d]
    for k in range(TAPS):
        s = (TAPS - 1 - k) * d
        out += gp[:, s:s + Wn] @ w[k]
    return out


def conv_weight_grad(x, g, d=1):
    """Gradient of sum(conv(x, w, d) * g) w.r.t. w: (5, Co, Ci)."""
    B, Wn, Ci = x.shape
    pad = 2 * d
    xp = np.zeros((B, Wn + 2 * pad, Ci))
    xp[:, pad:pad + Wn] = x
    gw = np.zeros((TAPS, g.shape[2], Ci))
    for k in range(TAPS):
        gw[k] = np.einsum("bwo,bwi->oi", g, xp[:, k * d:k * d + Wn])
    return gw


def features(u, r):
    """u: (B, W) rod values, r: (B,) mesh ratios -> (x (B, W, 2), s (B,))."""
    u = np.asarray(u, dtype=np.float64)
    up = np.pad(u, ((0, 0), (1, 1)))
    d = up[:, :-2] - 2.0 * up[:, 1:-1] + up[:, 2:]
    s = np.sqrt(np.mean(d * d, axis=1))
    x = np.empty(u.shape + (2,))
    x[:, :, 0] = d / s[:, None]
    x[:, :, 1] = ((np.asarray(r, dtype=np.float64) - 1.25) / 0.75)[:, None]
    return x, s


def target(u, u64, r, s):
    """Normalised 64-level increment (u64 - u) / (64 r s)."""
    r = np.asarray(r, dtype=np.float64)
    return (np.asarray(u64, np.float64) - np.asarray(u, np.float64)) / (64.0 * r * s)[:, None]


def jump(u, out, r, s):
    """u + 64 r s out: the surrogate's 64-level step."""
    r = np.asarray(r, dtype=np.float64)
    return np.asarray(u, np.float64) + (64.0 * r * s)[:, None] * out


def init_params(seed):
    """He-style initialisation, seeded; the last layer starts small."""
    rng = np.random.default_rng(seed)
    params = []
    for li, (ci, co) in enumerate(LAYERS):
        std = math.sqrt(2.0 / (TAPS * ci))
        if li == len(LAYERS) - 1:
            std *= 0.1
        params.append((rng.standard_normal((TAPS, co, ci)) * std, np.zeros(co)))
    return params


def forward(params, x, bf=False):
    """Returns (out, cache).  out: (B, W) FP64."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    h = r(x)
    cache = {"inputs": [], "pre": []}
    for li, (w, b) in enumerate(params):
        w = r(w)
        cache["inputs"].append(h)
        pre = conv(h, w, DILATIONS[li]) + b
        if li == len(params) - 1:
            cache["pre"].append(pre)
            return pre[:, :, 0], cache
        act = gelu(pre)
        if li > 0:
            act = h + act
        cache["pre"].append(r(pre))
        h = r(act)
    raise AssertionError("unreachable")


def loss_and_grads(params, x, t, bf=False):
    """MSE loss and its gradients [(dW, db)] per layer."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    out, cache = forward(params, x, bf)
    m = out.size
    loss = float(np.mean((out - t) ** 2))
    g = r((2.0 / m) * (out - t))[:, :, None]          # d loss / d out
    grads = [None] * len(params)
    nl = len(params)
    g_h = None
    for li in range(nl - 1, -1, -1):
        w, b = params[li]
        w = r(w)
        x_in = cache["inputs"][li]
        if li == nl - 1:
            g_pre = g
        else:
            g_pre = r(g_h * gelu_grad(cache["pre"][li]))
        grads[li] = (conv_weight_grad(x_in, g_pre, DILATIONS[li]), g_pre.sum(axis=(0, 1)))
        if li == 0:
            break
        g_in = conv_input_grad(g_pre, w, DILATIONS[li])
        if 0 < li < nl - 1:
            g_in = g_h + g_in           # residual path of layer li
        g_h = r(g_in)
    return loss, grads
