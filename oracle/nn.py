"""FP64 CPU oracle of the learned fluence denoiser (a 3-D residual U-Net).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
baseline of bench.py, never by the library.  Plain numpy in float64, one
layer at a time, each written from its definition; nothing here is blocked,
fused or reordered for speed.

The paper itself has no learned component: the denoiser is an addition that
works on the fluence maps the paper's method produces (Fig. 1 output).  Its
frozen design:

* Input: the fluence map of one gate (per launched photon), taken to log
  space as u = (ln max(phi, EPS) - LOG_SHIFT) / LOG_SCALE, one channel.
* Network (channels c_0 < c_1 < ... < c_{L-1}, L levels, volume sides
  divisible by 2^(L-1)), channels-last arrays (D, H, W, C):
    level 0:      h = relu(conv3(u; 1 -> c0)); h = relu(conv3(h; c0 -> c0))
    level l > 0:  h = relu(down(h; c_{l-1} -> c_l)); h = relu(conv3(h; c_l -> c_l))
    bottom:       h = relu(conv3(h; c_{L-1} -> c_{L-1}))
    back up:      h = relu(up(h; c_{l+1} -> c_l) + skip_l); h = relu(conv3(h; c_l -> c_l))
    output:       out = conv3(h; c0 -> 1) + u          (global residual)
  where skip_l is the level-l encoder output, conv3 a 3x3x3 convolution with
  stride 1 and zero padding 1, down a 2x2x2 convolution with stride 2, up a
  2x2x2 transposed convolution with stride 2, all with a bias per output
  channel, and relu(x) = max(x, 0).  No normalisation layers.
* Loss: mean squared error of out against the target's u over a mask of
  voxels (the medium voxels where the target fluence is at least 1e-8 of
  its maximum); Adam (beta1 0.9, beta2 0.999, eps 1e-8) on every weight
  and bias, on the gradients averaged over the volumes of a step and
  optionally clipped to a global L2 norm (`clip_scale`).

Weight layouts (shared with the library's C interface): conv3 w[27][Cin][Cout]
with tap t = (dz+1)*9 + (dy+1)*3 + (dx+1) reading x[z+dz][y+dy][x+dx];
down w[8][Cin][Cout] with tap t = 4a + 2b + c reading x[2z+a][2y+b][2x+c];
up w[8][Cin][Cout] with tap t writing y[2z+a][2y+b][2x+c].

`precision="bf16"` makes the oracle round where the GPU path stores BF16
values: weights as used by the convolutions, every activation after its
epilogue (bias, skip, ReLU), the input u fed to the first convolution, and
the back-propagated activation gradients; the output convolution, the
global residual, weight gradients, loss and optimiser stay in full
precision.  Rounding is to nearest, ties to even.
"""
from __future__ import annotations

import numpy as np

EPS = 1e-12          # fluence floor (per launched photon, 1/mm^2)
LOG_SHIFT = -16.0    # u = (ln phi - LOG_SHIFT) / LOG_SCALE
LOG_SCALE = 4.0

TAPS3 = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
TAPS2 = [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]


# ----------------------------------------------------------------- rounding

def bf16(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    bfloat16 keeps the top 16 bits of an IEEE binary32: round the binary32
    value first, then drop 16 mantissa bits with round-to-nearest-even."""
    f = np.atleast_1d(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    out[np.isnan(f)] = np.nan
    return out.reshape(np.shape(a))


# ------------------------------------------------------------------- layers

def conv3(x, w, b):
    """y[v][o] = b[o] + sum over taps t and inputs i of x[v + t][i] w[t][i][o],
    x zero outside the volume."""
    D, H, W, Ci = x.shape
    Co = w.shape[2]
    xp = np.zeros((D + 2, H + 2, W + 2, Ci))
    xp[1:-1, 1:-1, 1:-1] = x
    y = np.empty((D, H, W, Co))
    y[...] = b
    for t, (dz, dy, dx) in enumerate(TAPS3):
        y += xp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W] @ w[t]
    return y


def conv3_backward(x, w, gy):
    """Gradients of conv3 for upstream gradient gy: the input gradient
    gx[v][i] = sum_t sum_o gy[v - t][o] w[t][i][o], the weight gradient
    gw[t][i][o] = sum_v x[v + t][i] gy[v][o], and the bias gradient."""
    D, H, W, Ci = x.shape
    xp = np.zeros((D + 2, H + 2, W + 2, Ci))
    xp[1:-1, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    g2 = gy.reshape(-1, gy.shape[-1])
    for t, (dz, dy, dx) in enumerate(TAPS3):
        sl = (slice(1 + dz, 1 + dz + D), slice(1 + dy, 1 + dy + H), slice(1 + dx, 1 + dx + W))
        gxp[sl] += gy @ w[t].T
        gw[t] = xp[sl].reshape(-1, Ci).T @ g2
    return gxp[1:-1, 1:-1, 1:-1], gw, g2.sum(axis=0)


def down(x, w, b):
    """y[v][o] = b[o] + sum_t sum_i x[2v + t][i] w[t][i][o] (stride 2, 2x2x2)."""
    y = np.empty(tuple(s // 2 for s in x.shape[:3]) + (w.shape[2],))
    y[...] = b
    for t, (a, bb, c) in enumerate(TAPS2):
        y += x[a::2, bb::2, c::2] @ w[t]
    return y


def down_backward(x, w, gy):
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    g2 = gy.reshape(-1, gy.shape[-1])
    for t, (a, bb, c) in enumerate(TAPS2):
        gx[a::2, bb::2, c::2] = gy @ w[t].T
        gw[t] = x[a::2, bb::2, c::2].reshape(-1, x.shape[-1]).T @ g2
    return gx, gw, g2.sum(axis=0)


def up(x, w, b):
    """y[2v + t][o] = b[o] + sum_i x[v][i] w[t][i][o] (transposed, stride 2)."""
    y = np.empty(tuple(2 * s for s in x.shape[:3]) + (w.shape[2],))
    for t, (a, bb, c) in enumerate(TAPS2):
        y[a::2, bb::2, c::2] = x @ w[t] + b
    return y


def up_backward(x, w, gy):
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    x2 = x.reshape(-1, x.shape[-1])
    for t, (a, bb, c) in enumerate(TAPS2):
        g = gy[a::2, bb::2, c::2]
        gx += g @ w[t].T
        gw[t] = x2.T @ g.reshape(-1, g.shape[-1])
    return gx, gw, gy.reshape(-1, gy.shape[-1]).sum(axis=0)


def relu(x):
    return np.maximum(x, 0.0)


# --------------------------------------------------------------- the network

def layers(channels) -> list:
    """(name, kind, cin, cout) of every layer, in forward order."""
    c = list(channels)
    L = len(c)
    out = [("in", "conv3", 1, c[0]), ("enc0", "conv3", c[0], c[0])]
    for l in range(1, L):
        out += [(f"down{l}", "down", c[l - 1], c[l]), (f"enc{l}", "conv3", c[l], c[l])]
    out.append(("bottom", "conv3", c[-1], c[-1]))
    for l in range(L - 2, -1, -1):
        out += [(f"up{l}", "up", c[l + 1], c[l]), (f"dec{l}", "conv3", c[l], c[l])]
    out.append(("out", "conv3", c[0], 1))
    return out


def params_from_list(channels, arrays) -> dict:
    """Name the (weight, bias) pairs of `arrays`, given in forward layer order."""
    names = [name for name, _, _, _ in layers(channels)]
    assert len(arrays) == len(names)
    return {n: (np.asarray(w, np.float64), np.asarray(b, np.float64))
            for n, (w, b) in zip(names, arrays)}


_FWD = {"conv3": conv3, "down": down, "up": up}
_BWD = {"conv3": conv3_backward, "down": down_backward, "up": up_backward}


def forward(params, u, channels, precision: str = "fp64"):
    """Network output for input u (D, H, W) and the activations backward
    needs.  See the module docstring for the graph and rounding points."""
    rnd = bf16 if precision == "bf16" else (lambda a: np.asarray(a, dtype=np.float64))
    L = len(channels)
    acts = {}
    x = rnd(u[..., None])

    def layer(name, kind, inp, skip=None, act=True):
        w, b = params[name]
        y = _FWD[kind](inp, rnd(w), b)
        if skip is not None:
            y = y + skip
        if act:
            y = rnd(relu(y))
        acts[name] = (inp, y)
        return y

    h = layer("in", "conv3", x)
    h = layer("enc0", "conv3", h)
    skips = [h]
    for l in range(1, L):
        h = layer(f"down{l}", "down", h)
        h = layer(f"enc{l}", "conv3", h)
        skips.append(h)
    h = layer("bottom", "conv3", h)
    for l in range(L - 2, -1, -1):
        h = layer(f"up{l}", "up", h, skip=skips[l])
        h = layer(f"dec{l}", "conv3", h)
    r = layer("out", "conv3", h, act=False)
    out = r[..., 0] + u
    return out, acts


def backward(params, acts, gout, channels, precision: str = "fp64", record=None):
    """Gradients of every weight and bias for the output gradient gout
    (the chain rule through the graph of `forward`, last layer first).  The
    gradient entering a layer is masked by its ReLU (where it has one) and,
    in bf16 mode, rounded as the GPU path stores it.  With a dict `record`,
    each layer's (masked, rounded) output gradient and input gradient are
    kept there under its name, so that a single layer can be checked on
    exactly the operands this chain gave it."""
    rnd = bf16 if precision == "bf16" else (lambda a: np.asarray(a, dtype=np.float64))
    L = len(channels)
    grads = {}

    def back(name, kind, g, act=True):
        inp, y = acts[name]
        gy = rnd(g * (y > 0) if act else g)
        w, _ = params[name]
        gx, gw, gb = _BWD[kind](inp, rnd(w), gy)
        grads[name] = (gw, gb)
        if record is not None:
            record[name] = (gy, gx)
        return gx

    g = back("out", "conv3", gout[..., None], act=False)
    skip_grad = {}
    for l in range(0, L - 1):
        g = back(f"dec{l}", "conv3", g)
        # s = relu(up(h) + skip): the masked gradient reaches both summands
        inp, y = acts[f"up{l}"]
        gy = rnd(g * (y > 0))
        skip_grad[l] = gy
        w, _ = params[f"up{l}"]
        g, gw, gb = up_backward(inp, rnd(w), gy)
        grads[f"up{l}"] = (gw, gb)
        if record is not None:
            record[f"up{l}"] = (gy, g)
    g = back("bottom", "conv3", g)
    for l in range(L - 1, 0, -1):
        if l < L - 1:
            g = g + skip_grad[l]
        g = back(f"enc{l}", "conv3", g)
        g = back(f"down{l}", "down", g)
    g = back("enc0", "conv3", g + skip_grad[0])
    back("in", "conv3", g)
    return grads


def to_log(phi):
    """Network input / target u of a fluence map (per launched photon)."""
    return (np.log(np.maximum(phi, EPS)) - LOG_SHIFT) / LOG_SCALE


def from_log(u):
    return np.exp(u * LOG_SCALE + LOG_SHIFT)


def loss_mask(phi_target, labels=None, rel: float = 1e-8):
    m = phi_target >= rel * phi_target.max()
    if labels is not None:
        m &= labels != 0
    return m


def loss_and_grad(out, target_u, mask):
    """Masked mean squared error and its gradient with respect to out."""
    n = int(mask.sum())
    d = np.where(mask, out - target_u, 0.0)
    return float((d * d).sum() / n), 2.0 * d / n


def clip_scale(grads, grad_scale: float = 1.0, max_norm: float = 0.0) -> float:
    """Factor applied to every gradient before Adam: grad_scale (1/B when B
    volumes' gradients were summed), shrunk so that the global L2 norm of
    all scaled gradients is at most max_norm when max_norm > 0."""
    norm = grad_scale * float(np.sqrt(sum(float(np.sum(np.square(g))) for g in grads)))
    if max_norm > 0 and norm > max_norm:
        return grad_scale * max_norm / norm
    return grad_scale


def adam(param, grad, m, v, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); returns (param, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return param - lr * mh / (np.sqrt(vh) + eps), m, v
