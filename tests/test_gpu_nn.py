"""Denoiser kernels and network on the GPU against the FP64 oracle.

Single layers: the oracle evaluates the layer in float64 on the same BF16
inputs and BF16-rounded weights the kernels use, so the only differences
left are the kernels' FP32 accumulation (bound: K * 2^-24 * sum |terms|,
checked as 1e-5 relative to the sum of absolute terms) and, for BF16
outputs, the final rounding (at most one BF16 unit, and only where the FP64
value sits within the FP32 error of a rounding midpoint).  Whole network:
the oracle in its bf16 mode rounds at the same points as the GPU path;
gradients are compared relative to their layer's largest value.
"""
import numpy as np
import pytest

from oracle import nn as O
from paper_1711_03244_amd import nn, workloads as W

pytestmark = pytest.mark.gpu

KIND = {"conv3": nn.MCX_NN_CONV3, "down": nn.MCX_NN_DOWN, "up": nn.MCX_NN_UP}
TAPS = {"conv3": 27, "down": 8, "up": 8}
FWD = {"conv3": O.conv3, "down": O.down, "up": O.up}
BWD = {"conv3": O.conv3_backward, "down": O.down_backward, "up": O.up_backward}


def torch():
    import torch as t
    return t


def dev_bf16(a):
    t = torch()
    return t.as_tensor(np.ascontiguousarray(a, np.float32)).to(t.bfloat16).cuda().contiguous()


def dev_f32(a):
    t = torch()
    return t.as_tensor(np.ascontiguousarray(a, np.float32)).cuda().contiguous()


def host(t):
    return t.float().cpu().numpy().astype(np.float64)


def out_shape(kind, shape):
    if kind == "conv3":
        return tuple(shape)
    if kind == "down":
        return tuple(s // 2 for s in shape)
    return tuple(2 * s for s in shape)


def layer_case(kind, shape, ci, co, seed):
    rng = np.random.default_rng(seed)
    x = O.bf16(rng.normal(size=tuple(shape) + (ci,)))
    w = (rng.normal(size=(TAPS[kind], ci, co)) / np.sqrt(TAPS[kind] * ci)).astype(np.float32)
    b = rng.normal(size=co).astype(np.float32) * 0.1
    return x, w.astype(np.float64), b.astype(np.float64)


def abs_terms(kind, x, w):
    """sum over taps and inputs of |x w| per output (FP32 error scale)."""
    return FWD[kind](np.abs(x), np.abs(w), np.zeros(w.shape[2]))


CASES = [("conv3", (6, 5, 7), 1, 32), ("conv3", (4, 6, 5), 8, 16), ("conv3", (5, 4, 6), 32, 32),
         ("conv3", (4, 4, 4), 64, 64), ("conv3", (3, 5, 4), 3, 5), ("conv3", (4, 4, 4), 32, 1),
         ("conv3", (2, 2, 2), 256, 256), ("down", (6, 4, 8), 32, 64), ("down", (4, 4, 2), 3, 7),
         ("down", (8, 8, 8), 64, 128), ("up", (3, 2, 4), 64, 32), ("up", (2, 3, 2), 5, 3),
         ("up", (4, 4, 4), 256, 128),
         # many tiles on ragged grids: weight-gradient partial sums of >= 8
         # workgroups, and a forward split over input-channel chunks
         ("conv3", (15, 13, 18), 32, 32), ("conv3", (9, 10, 11), 64, 64),
         ("conv3", (10, 9, 12), 32, 1),
         # one-channel weight gradients summed over >= 64 workgroups
         ("conv3", (20, 17, 24), 32, 1), ("conv3", (16, 20, 18), 1, 32),
         # >= 1024 tiles of 4 x 4 x 8 gathering 32 channels: the resident-weights
         # kernel (ragged in every direction; 32, 1 and 24 output channels --
         # vector, one-column and element-wise output stores)
         ("conv3", (36, 66, 62), 32, 32), ("conv3", (34, 64, 64), 32, 1),
         ("conv3", (40, 64, 60), 32, 24)]


@pytest.mark.parametrize("kind,shape,ci,co", CASES)
def test_layer_forward(kind, shape, ci, co):
    t = torch()
    x, w, b = layer_case(kind, shape, ci, co, 1)
    wq = O.bf16(w)
    oshape = out_shape(kind, shape)
    skip = O.bf16(np.random.default_rng(2).normal(size=oshape + (co,))) if kind == "up" else None
    ref = FWD[kind](x, wq, b) + (skip if skip is not None else 0.0)
    scale = abs_terms(kind, x, wq) + np.abs(b) + (np.abs(skip) if skip is not None else 0.0)
    xd, wd, bd = dev_bf16(x), dev_f32(w), dev_f32(b)
    sd = dev_bf16(skip) if skip is not None else None
    # FP32 output, no ReLU
    y32 = t.empty(oshape + (co,), dtype=t.float32, device="cuda")
    nn.mcx_nn_layer_forward(KIND[kind], shape, ci, co, xd, wd, bd, sd, relu=False, y=y32, y_f32=True)
    got = host(y32)
    assert np.all(np.abs(got - ref) <= 1e-5 * scale + 1e-30)
    # BF16 output with ReLU
    y16 = t.empty(oshape + (co,), dtype=t.bfloat16, device="cuda")
    nn.mcx_nn_layer_forward(KIND[kind], shape, ci, co, xd, wd, bd, sd, relu=True, y=y16)
    got16 = host(y16)
    want16 = O.bf16(np.maximum(ref, 0))
    diff = got16 != want16
    # a disagreement is one BF16 unit where the FP64 value lies within the
    # FP32 accumulation error of a rounding midpoint (or of the ReLU's zero)
    tol = np.abs(want16) * 2.0 ** -7 + 2e-5 * scale + 1e-38
    assert np.all(np.abs(got16 - want16)[diff] <= tol[diff])
    assert diff.mean() < 1e-3


@pytest.mark.parametrize("kind,shape,ci,co", CASES)
def test_layer_backward(kind, shape, ci, co):
    t = torch()
    x, w, _ = layer_case(kind, shape, ci, co, 3)
    wq = O.bf16(w)
    oshape = out_shape(kind, shape)
    gy = O.bf16(np.random.default_rng(4).normal(size=oshape + (co,)))
    gx_ref, gw_ref, gb_ref = BWD[kind](x, wq, gy)
    xd, wd, gyd = dev_bf16(x), dev_f32(w), dev_bf16(gy)
    gx = t.empty(tuple(shape) + (ci,), dtype=t.float32, device="cuda")
    gw = t.empty(w.shape, dtype=t.float32, device="cuda")
    gb = t.empty(co, dtype=t.float32, device="cuda")
    nn.mcx_nn_layer_backward(KIND[kind], shape, ci, co, xd, wd, gyd, gx, gw, gb)
    # error scales: sums of absolute terms
    gx_scale = BWD[kind](np.abs(x), np.abs(wq), np.abs(gy))[0]
    gw_scale = BWD[kind](np.abs(x), np.abs(wq), np.abs(gy))[1]
    gb_scale = np.abs(gy).reshape(-1, co).sum(axis=0)
    assert np.all(np.abs(host(gx) - gx_ref) <= 1e-5 * gx_scale + 1e-30)
    assert np.all(np.abs(host(gw) - gw_ref) <= 1e-5 * gw_scale + 1e-30)
    assert np.all(np.abs(host(gb) - gb_ref) <= 1e-5 * gb_scale + 1e-30)


def test_layer_rejects_bad_arguments():
    from paper_1711_03244_amd import mcx
    t = torch()
    x = t.zeros((3, 3, 3, 4), dtype=t.bfloat16, device="cuda")
    w = t.zeros((8, 4, 4), dtype=t.float32, device="cuda")
    y = t.zeros((1, 1, 1, 4), dtype=t.bfloat16, device="cuda")
    with pytest.raises(mcx.McxError) as e:
        nn.mcx_nn_layer_forward(nn.MCX_NN_DOWN, (3, 3, 3), 4, 4, x, w, y=y)
    assert e.value.status == mcx.MCX_EINVAL


# ------------------------------------------------------------------- network

def make_net(channels, shape, seed, zero_output=False):
    ws = W.denoiser_weights(channels, seed=seed, zero_output=zero_output, bias_scale=0.05)
    flat = np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in ws])
    return ws, flat


def fluence_pair(shape, seed):
    """A smooth positive 'fluence' and a noisy copy with zeros, as the
    network sees them (synthetic, for the plumbing tests)."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(*[np.arange(s) + 0.5 for s in shape], indexing="ij")
    r = np.sqrt((x - shape[2] / 2) ** 2 + (y - shape[1] / 2) ** 2 + z ** 2)
    clean = np.exp(-0.3 * r) / (1 + r * r) * 1e-2
    noisy = clean * rng.gamma(4.0, 0.25, size=shape)
    noisy[rng.random(shape) < 0.2] = 0.0
    return noisy.astype(np.float32), clean.astype(np.float32)


@pytest.mark.parametrize("channels,shape", [((8, 16, 32), (16, 12, 8)), ((4, 8), (6, 4, 8)),
                                            ((32, 64, 128, 256), (16, 16, 16))])
def test_network_forward_matches_oracle(channels, shape):
    t = torch()
    ws, flat = make_net(channels, shape, 5)
    params = O.params_from_list(channels, [(w.astype(np.float64), b.astype(np.float64)) for w, b in ws])
    noisy, _ = fluence_pair(shape, 6)
    u = O.to_log(noisy.astype(np.float64))
    # the GPU takes ln in FP32; feed the oracle the same u
    u32 = ((np.log(np.maximum(noisy, np.float32(1e-12))).astype(np.float32) + np.float32(16))
           * np.float32(0.25)).astype(np.float64)
    ref, _ = O.forward(params, u32, channels, precision="bf16")
    with nn.Denoiser(channels, shape) as d:
        d.set_params(flat)
        uo = t.empty(shape, dtype=t.float32, device="cuda")
        d.forward(dev_f32(noisy), u_out=uo)
        got = host(uo)
    assert np.allclose(u32, u, atol=3e-6)
    err = np.abs(got - ref)
    # The bf16 model is sensitive to the last FP32 bits of its sums: a sum
    # that lands next to a BF16 rounding midpoint rounds either way, and the
    # flip propagates.  The bar is the spread the oracle itself shows when
    # its pre-rounding sums move by 1e-6 (the FP32 accumulation error of
    # these sums): the GPU may differ from the oracle by no more than twice
    # that spread.
    rng = np.random.default_rng(0)
    nudged = {k: (w, b + rng.normal(size=b.shape) * 1e-6) for k, (w, b) in params.items()}
    alt, _ = O.forward(nudged, u32, channels, precision="bf16")
    spread = np.abs(alt - ref)
    print("gpu - oracle: median", np.median(err), "max", err.max(), "| oracle spread: median",
          np.median(spread), "max", spread.max(), flush=True)
    assert np.median(err) <= 2 * max(np.median(spread), 1e-6)
    assert err.max() <= 2 * max(spread.max(), 1e-5)


def test_network_gradients_match_oracle():
    t = torch()
    channels, shape = (8, 16, 32), (16, 12, 8)
    ws, flat = make_net(channels, shape, 7)
    params = O.params_from_list(channels, [(w.astype(np.float64), b.astype(np.float64)) for w, b in ws])
    noisy, clean = fluence_pair(shape, 8)
    u32 = ((np.log(np.maximum(noisy, np.float32(1e-12))).astype(np.float32) + np.float32(16))
           * np.float32(0.25)).astype(np.float64)
    t32 = ((np.log(np.maximum(clean, np.float32(1e-12))).astype(np.float32) + np.float32(16))
           * np.float32(0.25)).astype(np.float64)
    out, acts = O.forward(params, u32, channels, precision="bf16")
    mask = O.loss_mask(clean.astype(np.float64))
    loss_ref, gout = O.loss_and_grad(out, t32, mask)
    grads = O.backward(params, acts, gout, channels, precision="bf16")
    with nn.Denoiser(channels, shape) as d:
        d.set_params(flat)
        loss = d.loss_grad(dev_f32(noisy), dev_f32(clean))
        g = d.grads()
    assert loss == pytest.approx(loss_ref, rel=1e-2)
    off = 0
    for name, kind, ci, co in O.layers(channels):
        gw_ref, gb_ref = grads[name]
        n = gw_ref.size
        gw = g[off:off + n].reshape(gw_ref.shape)
        gb = g[off + n:off + n + co]
        off += n + co
        s = np.abs(gw_ref).max() + 1e-30
        rel = np.abs(gw - gw_ref).max() / s
        print(name, "max rel weight-gradient difference", rel, flush=True)
        # the chain's BF16 roundings match the oracle's bf16 mode; what is
        # left is FP32 accumulation (measured ~2e-7 of the layer's largest)
        assert rel < 1e-5, name
        assert np.abs(gb - gb_ref).max() <= 1e-5 * (np.abs(gb_ref).max() + 1e-30), name
    assert off == g.size


def test_network_64cube_every_layer_backward_on_the_chains_operands():
    """Loss and gradients of the full (32, 64, 128, 256) network on a 64^3
    volume, layer by layer: the oracle runs the whole bf16-mode forward pass,
    loss and backward chain and records each layer's operands (its BF16
    input, its masked and rounded output gradient); the GPU's layer kernels
    -- the same launches the network's backward pass makes, including the
    64^3 brick input gradient with two z-slices per wave and the 64^3 slab
    weight gradients -- then get exactly those operands.  Every input,
    weight and bias gradient must agree within 1e-5 of its sum of absolute
    terms (the FP32 accumulation bound).  (The whole network is not
    compared end to end at this size: BF16 roundings that land next to a
    midpoint flip either way and the flips propagate.)"""
    t = torch()
    channels, shape = W.DENOISER_CHANNELS, (64, 64, 64)
    ws, _ = make_net(channels, shape, 12)
    params = O.params_from_list(channels, [(w.astype(np.float64), b.astype(np.float64)) for w, b in ws])
    noisy, clean = fluence_pair(shape, 13)
    u32 = ((np.log(np.maximum(noisy, np.float32(1e-12))).astype(np.float32) + np.float32(16))
           * np.float32(0.25)).astype(np.float64)
    t32 = ((np.log(np.maximum(clean, np.float32(1e-12))).astype(np.float32) + np.float32(16))
           * np.float32(0.25)).astype(np.float64)
    out, acts = O.forward(params, u32, channels, precision="bf16")
    mask = O.loss_mask(clean.astype(np.float64))
    loss, gout = O.loss_and_grad(out, t32, mask)
    rec = {}
    grads = O.backward(params, acts, gout, channels, precision="bf16", record=rec)
    print("64^3 loss", loss, flush=True)
    for name, kind, ci, co in O.layers(channels):
        inp, _ = acts[name]
        gy, gx_ref = rec[name]
        gw_ref, gb_ref = grads[name]
        w = params[name][0]
        wq = O.bf16(w)
        ishape = inp.shape[:3]
        print(f"[gpu] layer {name} {kind} {ishape} {ci}->{co}", flush=True)
        gx = t.empty(tuple(ishape) + (ci,), dtype=t.float32, device="cuda")
        gw = t.empty(w.shape, dtype=t.float32, device="cuda")
        gb = t.empty(co, dtype=t.float32, device="cuda")
        nn.mcx_nn_layer_backward(KIND[kind], ishape, ci, co, dev_bf16(inp), dev_f32(w),
                                 dev_bf16(gy), gx, gw, gb)
        sx, sw, _ = BWD[kind](np.abs(inp), np.abs(wq), np.abs(gy))
        sb = np.abs(gy).reshape(-1, co).sum(axis=0)
        for got, ref, sc, what in [(host(gx), gx_ref, sx, "input"), (host(gw), gw_ref, sw, "weight"),
                                   (host(gb), gb_ref, sb, "bias")]:
            d = np.abs(got - ref)
            print(f"  {what} gradient: max |diff| / sum|terms| {np.max(d / (sc + 1e-30)):.2e}, "
                  f"of the layer's largest {d.max() / (np.abs(ref).max() + 1e-30):.2e}", flush=True)
            assert np.all(d <= 1e-5 * sc + 1e-30), (name, what)


def test_fused_backward_gives_the_unfused_gradients():
    """The (32, 64, 128, 256) network on a 64^3 volume: with the fused
    backward pass the 64^3 layers' input-gradient products apply the ReLU
    mask, round to BF16 and sum the bias gradient of the layer below.  The
    BF16 gradients are then the same values (the same FP32 sums, masked
    and rounded the same way), so every 3x3x3 layer's weight gradient
    (summed in a fixed order) and every bias gradient outside the folded
    layers must be the same bits.  The down and up layers' weight gradients
    are summed with FP32 atomics, in an order that changes from call to
    call (within 1e-5 of the layer's largest); a folded layer's bias
    gradient sums its values in another order (within 1e-3 of the layer's
    largest, FP32 accumulation over 64^3 voxels)."""
    t = torch()
    channels, shape = W.DENOISER_CHANNELS, (64, 64, 64)
    ws, flat = make_net(channels, shape, 21)
    noisy, clean = fluence_pair(shape, 22)
    x, y = dev_f32(noisy), dev_f32(clean)
    folded = {"in", "up0"}  # the layers below the two 64^3 32 -> 32 layers (enc0, dec0)

    def compare(g1, g0, fold):
        off, seen = 0, set()
        for name, kind, ci, co in O.layers(channels):
            n = TAPS[kind] * ci * co
            w1, w0 = g1[off:off + n], g0[off:off + n]
            if kind == "conv3":
                assert np.array_equal(w1, w0), name
            else:
                assert np.abs(w1 - w0).max() <= 1e-5 * np.abs(w0).max(), name
            b1, b0 = g1[off + n:off + n + co], g0[off + n:off + n + co]
            if fold and name in folded:
                seen.add(name)
                err = np.abs(b1 - b0).max() / (np.abs(b0).max() + 1e-30)
                print(f"  {name}: bias gradient max difference {err:.2e} of the largest", flush=True)
                assert err <= 1e-3, name
            else:
                assert np.array_equal(b1, b0), name
            off += n + co
        assert off == g0.size and seen == (folded if fold else set())

    got = {}
    with nn.Denoiser(channels, shape) as d:
        d.set_params(flat)
        for on in (False, True, False, True):
            nfold = d.set_fused_backward(on)
            print(f"[gpu] fused backward {on}: {nfold} folded layers", flush=True)
            assert nfold == (2 if on else 0)
            loss = d.loss_grad(x, y)
            g = d.grads()
            if on in got:  # the same call again
                assert loss == pytest.approx(got[on][0], rel=1e-12)
                compare(g, got[on][1], False)
            got[on] = (loss, g)
    assert got[True][0] == pytest.approx(got[False][0], rel=1e-12)
    compare(got[True][1], got[False][1], True)


def test_adam_step_matches_oracle():
    t = torch()
    channels, shape = (4, 8), (8, 8, 8)
    ws, flat = make_net(channels, shape, 9)
    noisy, clean = fluence_pair(shape, 10)
    noisy2, clean2 = fluence_pair(shape, 11)
    with nn.Denoiser(channels, shape) as d:
        d.set_params(flat)
        d.loss_grad(dev_f32(noisy), dev_f32(clean))
        g1 = d.grads().astype(np.float64)
        d.adam(1e-3)
        p1 = d.params().astype(np.float64)
        # a step on the mean gradient of two volumes, clipped to a norm below
        # the gradient's own
        d.loss_grad(dev_f32(noisy), dev_f32(clean))
        ga = d.grads().astype(np.float64)
        d.loss_grad(dev_f32(noisy2), dev_f32(clean2))
        gb = d.grads().astype(np.float64)
        d.loss_grad(dev_f32(noisy), dev_f32(clean))
        d.loss_grad(dev_f32(noisy2), dev_f32(clean2), accumulate=True)
        g2 = d.grads().astype(np.float64)
        max_norm = 0.25 * float(np.linalg.norm(0.5 * g2))
        d.adam(1e-3, grad_scale=0.5, max_norm=max_norm)
        p2 = d.params().astype(np.float64)
    assert np.allclose(g2, ga + gb, rtol=1e-5, atol=1e-7 * np.abs(g2).max())
    p = flat.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    q1, m, v = O.adam(p, g1, m, v, 1, 1e-3)
    scale = O.clip_scale([g2], 0.5, max_norm)
    assert scale == pytest.approx(0.125, rel=1e-9)
    q2, m, v = O.adam(p1, scale * g2, m, v, 2, 1e-3)
    assert np.allclose(p1, q1, rtol=1e-6, atol=1e-7)
    assert np.allclose(p2, q2, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("shape", [(3, 5, 6), (3, 8, 8)])
def test_mirror_xy_is_the_symmetry(shape):
    """Each of the eight x-y symmetries against numpy's flips and transpose
    (bit-exact: a pure permutation)."""
    rng = np.random.default_rng(31)
    a = rng.normal(size=shape).astype(np.float32)
    x = dev_f32(a)
    for op in range(8):
        if (op & 4) and shape[1] != shape[2]:
            continue
        e = a
        if op & 1:
            e = e[:, :, ::-1]
        if op & 2:
            e = e[:, ::-1, :]
        if op & 4:
            e = e.transpose(0, 2, 1)
        got = nn.mcx_nn_mirror_xy(x, op).cpu().numpy()
        torch().cuda.synchronize()
        assert np.array_equal(got, e), op


def test_untrained_network_returns_its_input():
    t = torch()
    channels, shape = (8, 16), (8, 8, 8)
    _, flat = make_net(channels, shape, 11, zero_output=True)
    noisy, _ = fluence_pair(shape, 12)
    with nn.Denoiser(channels, shape) as d:
        d.set_params(flat)
        out = host(d.forward(dev_f32(noisy)))
    keep = noisy >= 1e-12
    assert np.allclose(out[keep], noisy[keep], rtol=1e-5)
    assert np.allclose(out[~keep], 1e-12, rtol=1e-5)


def _sym_np(a, op):
    """The x-y symmetry of mcx_nn_mirror_xy on a [z][y][x] array, from its
    documented definition: out[z][y][x] = a[z][y'][x'] with (x', y') = (y, x)
    when op & 4, then x' mirrored when op & 1 and y' when op & 2."""
    nz, ny, nx = a.shape
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    sx, sy = (y, x) if op & 4 else (x, y)
    if op & 1:
        sx = nx - 1 - sx
    if op & 2:
        sy = ny - 1 - sy
    return a[:, sy, sx]


@pytest.mark.parametrize("nsym", [2, 4, 8])
def test_symmetry_averaged_inference(nsym):
    """mcx_nn_forward_sym equals the mean, in u space, of the network's
    outputs for the transformed inputs, each mapped back by the inverse
    transform (found here by search over the 8 ops); composed here from
    mcx_nn_mirror_xy and mcx_nn_forward.  nsym = 1 is the plain forward."""
    t = torch()
    channels, shape = (8, 16), (6, 8, 8)
    _, flat = make_net(channels, shape, 21)
    noisy, _ = fluence_pair(shape, 22)
    inverse = {}
    probe = np.arange(np.prod(shape), dtype=np.float64).reshape(shape)
    for op in range(8):
        inverse[op] = next(k for k in range(8) if np.array_equal(_sym_np(_sym_np(probe, op), k),
                                                                probe))
    with nn.Denoiser(channels, shape) as d:
        d.set_params(flat)
        x = dev_f32(noisy)
        acc = np.zeros(shape)
        for op in range(nsym):
            xo = x if op == 0 else nn.mcx_nn_mirror_xy(x, op)
            u = t.empty_like(x)
            d.forward(xo, u_out=u)
            t.cuda.synchronize()
            acc += _sym_np(host(u), inverse[op])
        u_sym, phi_sym = t.empty_like(x), t.empty_like(x)
        d.forward(x, phi_out=phi_sym, u_out=u_sym, symmetries=nsym)
        u1 = t.empty_like(x)
        d.forward(x, u_out=u1, symmetries=1)
        t.cuda.synchronize()
        u_plain = t.empty_like(x)
        d.forward(x, u_out=u_plain)
        t.cuda.synchronize()
    assert np.array_equal(host(u1), host(u_plain))
    want = acc / nsym
    assert np.allclose(host(u_sym), want, rtol=0, atol=1e-6 * np.abs(want).max())
    assert np.allclose(host(phi_sym), np.exp(want * 4.0 - 16.0), rtol=1e-5)


def test_checkpoint_round_trip(tmp_path):
    """save() after some training and load() into a fresh network restore
    parameters and Adam's state exactly; the forward pass is bit-identical."""
    channels, shape = (8, 16), (8, 8, 8)
    _, flat = make_net(channels, shape, 17, zero_output=True)
    noisy, clean = fluence_pair(shape, 18)
    x, y = dev_f32(noisy), dev_f32(clean)
    path = tmp_path / "denoiser.npz"
    with nn.Denoiser(channels, shape) as d:
        d.set_params(flat)
        for _ in range(5):
            d.train_step(x, y, 1e-3)
        d.save(path)
        ref_params = d.params()
        ref_m, ref_v, ref_step = nn.mcx_nn_get_adam(d.h)
        ref_out = host(d.forward(x))
    assert ref_step == 5 and np.any(ref_m != 0) and np.any(ref_v != 0)
    with nn.Denoiser(channels, shape) as e:
        e.load(path)
        m, v, step = nn.mcx_nn_get_adam(e.h)
        assert np.array_equal(e.params(), ref_params)
        assert np.array_equal(m, ref_m) and np.array_equal(v, ref_v) and step == ref_step
        assert np.array_equal(host(e.forward(x)), ref_out)
    with nn.Denoiser(channels, (8, 8, 16)) as f:
        with pytest.raises(ValueError):
            f.load(path)


def test_inference_checkpoint_computes_what_the_trained_network_does(tmp_path):
    """save_inference() keeps the weights as the BF16 values the matrix cores
    use and the biases in FP32: a network loaded from it gives a forward
    pass bit-identical to the trained FP32-master network, its weights are
    the BF16 rounding of the master weights, and the provenance survives."""
    channels, shape = (8, 16), (8, 8, 8)
    _, flat = make_net(channels, shape, 19, zero_output=False)
    noisy, clean = fluence_pair(shape, 20)
    x, y = dev_f32(noisy), dev_f32(clean)
    path = tmp_path / "denoiser_inference.npz"
    with nn.Denoiser(channels, shape) as d:
        d.set_params(flat)
        for _ in range(3):
            d.train_step(x, y, 1e-3)
        d.save_inference(path, {"history": [{"steps": 3}]})
        master = d.params()
        mask = d._weight_mask()
        ref_out = host(d.forward(x))
    with nn.Denoiser(channels, shape) as e:
        meta = e.load_inference(path)
        got = e.params()
        assert meta == {"history": [{"steps": 3}]}
        assert np.array_equal(got[~mask], master[~mask])
        want_w = (nn.bf16_bits(master[mask]).astype(np.uint32) << 16).view(np.float32)
        assert np.array_equal(got[mask], want_w)
        assert np.array_equal(host(e.forward(x)), ref_out)


def test_training_reduces_the_loss():
    t = torch()
    channels, shape = (8, 16, 32), (16, 16, 16)
    _, flat = make_net(channels, shape, 13, zero_output=True)
    pairs = [fluence_pair(shape, 100 + i) for i in range(4)]
    dev = [(dev_f32(a), dev_f32(b)) for a, b in pairs]
    with nn.Denoiser(channels, shape) as d:
        d.set_params(flat)
        first = np.mean([d.loss_grad(a, b) for a, b in dev])
        for it in range(60):
            a, b = dev[it % 4]
            d.train_step(a, b, 2e-3)
        last = np.mean([d.loss_grad(a, b) for a, b in dev])
    print("loss", first, "->", last, flush=True)
    assert last < 0.5 * first


def test_denoiser_gain_on_held_out_volumes():
    """Trained on simulator pairs, the network brings low-photon maps of
    volumes it has not seen closer to the reference than they were."""
    from paper_1711_03244_amd import denoise
    channels, side = (16, 32, 64), 32
    ds = denoise.make_dataset(range(1, 33), side, [5e4, 5e5], 1e7, say=print)
    with nn.Denoiser(channels, (side,) * 3) as d:
        d.set_params(W.denoiser_weights(channels, seed=1))
        mean_loss = lambda: np.mean([d.loss_grad(x, ds.targets[v]) for v, _, x in ds.inputs])
        before = mean_loss()
        denoise.train(d, ds, 500, lr=1e-3, log_every=100, batch=4, max_norm=0.1, say=print)
        after = mean_loss()
        ev = denoise.evaluate(d, [700001, 700002, 700003], side, 1e7, 2, [5e4, 5e5], say=print,
                              batch_seeds=[710001, 710002, 710003, 710004])
    print("mean training loss", before, "->", after, ev, flush=True)
    assert after < 0.5 * before
    # batched timing: per-volume times of a shared launch, a fitted model, a ratio per input
    b = ev["batched"]
    assert len(b["per_volume_ms"]) == 3 and all(t > 0 for _, t in b["per_volume_ms"])
    assert b["time_model"]["ms_per_photon"] > 0
    assert all(r["batched_time_ratio"] is None or r["batched_time_ratio"] > 0
               for r in ev["per_input"])
    # at the lowest input count the noise is far above the targets' (1e7
    # photons): there the network must remove a large part of it
    low = ev["per_input"][0]
    assert low["denoised_err"] < 0.7 * low["noisy_err"], low


def test_network_forward_full_size():
    """The (32, 64, 128, 256) network on a 64^3 map of the denoiser's data
    set, against the oracle's bf16 mode, with the bar derived from the
    oracle's own spread as in test_network_forward_matches_oracle."""
    from paper_1711_03244_amd import denoise
    t = torch()
    channels, shape = W.DENOISER_CHANNELS, (64, 64, 64)
    ws, flat = make_net(channels, shape, 21)
    params = O.params_from_list(channels, [(w.astype(np.float64), b.astype(np.float64)) for w, b in ws])
    maps, _ = denoise.simulate([W.denoiser_volume(3)], 100_000, [5])
    phi = maps[0]
    u32 = ((np.log(np.maximum(phi, np.float32(1e-12))).astype(np.float32) + np.float32(16))
           * np.float32(0.25)).astype(np.float64)
    with nn.Denoiser(channels, shape) as d:
        d.set_params(flat)
        uo = t.empty(shape, dtype=t.float32, device="cuda")
        d.forward(dev_f32(phi), u_out=uo)
        got = host(uo)
    ref, _ = O.forward(params, u32, channels, precision="bf16")
    rng = np.random.default_rng(0)
    nudged = {k: (w, b + rng.normal(size=b.shape) * 1e-6) for k, (w, b) in params.items()}
    alt, _ = O.forward(nudged, u32, channels, precision="bf16")
    err, spread = np.abs(got - ref), np.abs(alt - ref)
    print("64^3: gpu - oracle median", np.median(err), "max", err.max(), "| oracle spread median",
          np.median(spread), "max", spread.max(), flush=True)
    assert np.median(err) <= 2 * max(np.median(spread), 1e-6)
    assert err.max() <= 2 * max(spread.max(), 1e-5)
