"""Pins of the denoiser oracle (oracle/nn.py) to things other than itself.

Library routines in float64 on the CPU (torch's conv3d, conv_transpose3d,
autograd, Adam and bfloat16 conversion) for every layer, the whole network
and the optimiser; central finite differences for the gradients; closed
forms for the bf16 rounding and for the identity an untrained network
(zero output layer) computes.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import nn as O
from paper_1711_03244_amd import workloads as W



def t_conv3(x, w, b):
    # channels-last (D,H,W,C) + w[27][ci][co] -> torch NCDHW / (co, ci, 3,3,3)
    xt = torch.as_tensor(x).permute(3, 0, 1, 2)[None]
    wt = torch.as_tensor(w).reshape(3, 3, 3, w.shape[1], w.shape[2]).permute(4, 3, 0, 1, 2)
    return F.conv3d(xt, wt, torch.as_tensor(b), padding=1)[0].permute(1, 2, 3, 0)


def t_down(x, w, b):
    xt = torch.as_tensor(x).permute(3, 0, 1, 2)[None]
    wt = torch.as_tensor(w).reshape(2, 2, 2, w.shape[1], w.shape[2]).permute(4, 3, 0, 1, 2)
    return F.conv3d(xt, wt, torch.as_tensor(b), stride=2)[0].permute(1, 2, 3, 0)


def t_up(x, w, b):
    xt = torch.as_tensor(x).permute(3, 0, 1, 2)[None]
    wt = torch.as_tensor(w).reshape(2, 2, 2, w.shape[1], w.shape[2]).permute(3, 4, 0, 1, 2)
    return F.conv_transpose3d(xt, wt, torch.as_tensor(b), stride=2)[0].permute(1, 2, 3, 0)


T_LAYER = {"conv3": t_conv3, "down": t_down, "up": t_up}
O_LAYER = {"conv3": O.conv3, "down": O.down, "up": O.up}
O_BACK = {"conv3": O.conv3_backward, "down": O.down_backward, "up": O.up_backward}
TAPS = {"conv3": 27, "down": 8, "up": 8}


def rand_layer(kind, shape, ci, co, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=tuple(shape) + (ci,))
    w = rng.normal(size=(TAPS[kind], ci, co)) / np.sqrt(TAPS[kind] * ci)
    b = rng.normal(size=co)
    return x, w, b


# ----------------------------------------------------------------- rounding

def test_bf16_rounding_closed_forms():
    one = 1.0
    assert O.bf16(one) == 1.0
    assert O.bf16(1 + 2 ** -8) == 1.0                   # tie -> even (mantissa 0)
    assert O.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6       # tie -> even (round up)
    assert O.bf16(1 + 2 ** -8 + 2 ** -12) == 1 + 2 ** -7  # above the tie
    assert O.bf16(-3.0) == -3.0
    assert O.bf16(0.0) == 0.0
    assert np.isinf(O.bf16(np.float32(3.4e38) * 1.0))  # rounds past the largest bf16
    assert np.isnan(O.bf16(np.nan))


def test_bf16_rounding_matches_library():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=10000) * 10.0 ** rng.integers(-30, 30, 10000),
                        rng.normal(size=1000)]).astype(np.float32)
    lib = torch.as_tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.bf16(x), lib)


# -------------------------------------------------------------------- layers

@pytest.mark.parametrize("kind,shape,ci,co", [
    ("conv3", (5, 4, 6), 3, 2), ("conv3", (3, 3, 3), 1, 4), ("conv3", (2, 5, 3), 4, 1),
    ("down", (4, 6, 2), 3, 5), ("down", (2, 2, 2), 1, 2),
    ("up", (2, 3, 1), 4, 3), ("up", (1, 1, 1), 2, 2)])
def test_layer_forward_matches_library(kind, shape, ci, co):
    x, w, b = rand_layer(kind, shape, ci, co, 1)
    got = O_LAYER[kind](x, w, b)
    ref = T_LAYER[kind](x, w, b).numpy()
    assert got.shape == ref.shape
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind,shape,ci,co", [
    ("conv3", (4, 3, 5), 3, 2), ("down", (4, 2, 6), 2, 3), ("up", (2, 1, 3), 3, 2)])
def test_layer_backward_matches_autograd(kind, shape, ci, co):
    x, w, b = rand_layer(kind, shape, ci, co, 2)
    y = O_LAYER[kind](x, w, b)
    gy = np.random.default_rng(3).normal(size=y.shape)
    gx, gw, gb = O_BACK[kind](x, w, gy)
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(w, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    (T_LAYER[kind](xt, wt, bt) * torch.as_tensor(gy)).sum().backward()
    assert np.allclose(gx, xt.grad.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(gw, wt.grad.numpy(), rtol=1e-12, atol=1e-12)
    assert np.allclose(gb, bt.grad.numpy(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind", ["conv3", "down", "up"])
def test_layer_backward_finite_differences(kind):
    shape = (2, 4, 2) if kind != "up" else (1, 2, 1)
    x, w, b = rand_layer(kind, shape, 2, 3, 4)
    y = O_LAYER[kind](x, w, b)
    gy = np.random.default_rng(5).normal(size=y.shape)
    gx, gw, gb = O_BACK[kind](x, w, gy)
    f = lambda xx, ww, bb: float((O_LAYER[kind](xx, ww, bb) * gy).sum())
    h = 1e-6
    rng = np.random.default_rng(6)
    for arr, g, pick in [(x, gx, 0), (w, gw, 1), (b, gb, 2)]:
        for _ in range(6):
            idx = tuple(int(rng.integers(0, s)) for s in arr.shape)
            args = [x.copy(), w.copy(), b.copy()]
            args[pick][idx] += h
            fp = f(*args)
            args[pick][idx] -= 2 * h
            fm = f(*args)
            assert g[idx] == pytest.approx((fp - fm) / (2 * h), rel=1e-6, abs=1e-8)


# ------------------------------------------------------------------- network

def t_forward(pt, u, channels):
    """The same graph, written with torch's functional layers."""
    L = len(channels)
    x = u[..., None]
    h = torch.relu(t_conv3(x, *pt["in"]))
    h = torch.relu(t_conv3(h, *pt["enc0"]))
    skips = [h]
    for l in range(1, L):
        h = torch.relu(t_down(h, *pt[f"down{l}"]))
        h = torch.relu(t_conv3(h, *pt[f"enc{l}"]))
        skips.append(h)
    h = torch.relu(t_conv3(h, *pt["bottom"]))
    for l in range(L - 2, -1, -1):
        h = torch.relu(t_up(h, *pt[f"up{l}"]) + skips[l])
        h = torch.relu(t_conv3(h, *pt[f"dec{l}"]))
    return t_conv3(h, *pt["out"])[..., 0] + u


def small_net(seed=7, channels=(3, 4, 5), side=8):
    ws = W.denoiser_weights(channels, seed=seed, zero_output=False, bias_scale=0.1)
    params = O.params_from_list(channels, ws)
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(side, side - 4 if side > 4 else side, side))
    return params, u


def test_layer_table_agrees_with_the_weight_generator():
    ch = (32, 64, 128, 256)
    a = [(k, ci, co) for _, k, ci, co in O.layers(ch)]
    b = [(k, ci, co) for k, _, ci, co in W.denoiser_layer_shapes(ch)]
    assert a == b and len(a) == 16
    n = sum(t * ci * co + co for _, t, ci, co in W.denoiser_layer_shapes(ch))
    assert 5.0e6 < n < 5.6e6


@pytest.mark.parametrize("channels", [(3, 4, 5), (2, 3), (4, 4, 4, 4)])
def test_network_forward_and_backward_match_library(channels):
    side = 2 ** (len(channels) - 1) * 2
    params, _ = small_net(channels=channels)
    u = np.random.default_rng(8).normal(size=(side, side, 2 * side))
    out, acts = O.forward(params, u, channels)
    pt = {k: (torch.tensor(w, requires_grad=True), torch.tensor(b, requires_grad=True))
          for k, (w, b) in params.items()}
    ref = t_forward(pt, torch.as_tensor(u), channels)
    assert np.allclose(out, ref.detach().numpy(), rtol=1e-11, atol=1e-11)
    target = np.random.default_rng(9).normal(size=u.shape)
    mask = np.random.default_rng(10).random(u.shape) < 0.7
    loss, gout = O.loss_and_grad(out, target, mask)
    mt = torch.as_tensor(mask)
    tl = ((ref - torch.as_tensor(target))[mt] ** 2).mean()
    assert loss == pytest.approx(float(tl.detach()), rel=1e-12)
    tl.backward()
    grads = O.backward(params, acts, gout, channels)
    for k, (w, b) in pt.items():
        assert np.allclose(grads[k][0], w.grad.numpy(), rtol=1e-9, atol=1e-12), k
        assert np.allclose(grads[k][1], b.grad.numpy(), rtol=1e-9, atol=1e-12), k


def test_network_gradient_finite_differences():
    channels = (2, 3)
    params, _ = small_net(channels=channels, seed=11)
    u = np.random.default_rng(12).normal(size=(4, 2, 4))
    target = np.random.default_rng(13).normal(size=u.shape)
    mask = np.ones(u.shape, bool)

    def loss_of(p):
        out, _ = O.forward(p, u, channels)
        return O.loss_and_grad(out, target, mask)[0]

    out, acts = O.forward(params, u, channels)
    _, gout = O.loss_and_grad(out, target, mask)
    grads = O.backward(params, acts, gout, channels)
    rng = np.random.default_rng(14)
    h = 1e-6
    for name in ["in", "enc0", "down1", "enc1", "bottom", "up0", "dec0", "out"]:
        w, b = params[name]
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in w.shape)
            pp = dict(params)
            w2 = w.copy(); w2[idx] += h; pp[name] = (w2, b)
            fp = loss_of(pp)
            w2 = w.copy(); w2[idx] -= h; pp[name] = (w2, b)
            fm = loss_of(pp)
            assert grads[name][0][idx] == pytest.approx((fp - fm) / (2 * h), rel=1e-5, abs=1e-9), name


def test_untrained_network_is_the_identity():
    channels = (4, 8)
    params = O.params_from_list(channels, W.denoiser_weights(channels, seed=3))
    u = np.random.default_rng(1).normal(size=(4, 4, 4))
    out, _ = O.forward(params, u, channels)
    assert np.array_equal(out, u)
    out16, _ = O.forward(params, u, channels, precision="bf16")
    assert np.array_equal(out16, u)   # the residual path stays in full precision


def test_bf16_mode_rounds_at_the_stated_points():
    channels = (3, 4)
    params, u = small_net(channels=channels, side=4)
    out, acts = O.forward(params, u, channels, precision="bf16")
    ref, _ = O.forward(params, u, channels)
    for name, (inp, y) in acts.items():
        assert np.array_equal(O.bf16(inp), inp), name
        if name != "out":
            assert np.array_equal(O.bf16(y), y), name
    assert np.allclose(out, ref, rtol=0.05, atol=0.05)
    assert not np.array_equal(out, ref)


def test_adam_matches_library():
    rng = np.random.default_rng(2)
    p = rng.normal(size=(3, 4))
    pt = torch.tensor(p, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step in range(1, 5):
        g = rng.normal(size=p.shape)
        p, m, v = O.adam(p, g, m, v, step, 1e-2)
        opt.zero_grad()
        pt.grad = torch.as_tensor(g).clone()
        opt.step()
        assert np.allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_log_transform_round_trip_and_floor():
    phi = np.array([0.0, 1e-13, 1e-12, 1e-5, 0.3])
    u = O.to_log(phi)
    assert u[0] == u[1] == u[2] == pytest.approx((np.log(1e-12) + 16.0) / 4.0)
    assert np.allclose(O.from_log(u[2:]), phi[2:], rtol=1e-12)
    m = O.loss_mask(np.array([1.0, 1e-9, 2e-8, 0.5]))
    assert list(m) == [True, False, True, True]


def test_gradient_clipping_matches_library():
    rng = np.random.default_rng(5)
    gs = [rng.normal(size=(3, 4)), rng.normal(size=7)]
    for scale, max_norm in [(1.0, 0.0), (0.5, 100.0), (0.25, 0.3), (1.0, 1.0)]:
        ts = [torch.tensor(g * scale, requires_grad=True) for g in gs]
        for tt in ts:
            tt.grad = tt.detach().clone()
        if max_norm > 0:
            torch.nn.utils.clip_grad_norm_(ts, max_norm)
        got = O.clip_scale(gs, scale, max_norm)
        for g, tt in zip(gs, ts):
            assert np.allclose(got * g, tt.grad.numpy(), rtol=1e-6, atol=1e-12)
