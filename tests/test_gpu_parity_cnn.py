"""GPU vs oracle: the proposal network's forward pass, MSE loss, backward
pass (weight and bias gradients), Adam step, BF16 rounding and input
features, through the C-ABI.

Primary check, against the plain FP64 network (BF16 weights, the
configured parameter precision, and FP64 activations, products and sums):
whole-network outputs, losses and the proposal within 1e-2 relative (the
BF16 tolerance of the learned form), gradients within 1e-2 normwise over the
whole parameter vector on boxes of realistic size (thousands of voxels per
sum).  The matrix-core instruction multiplies BF16 operands, so activations
and output gradients are rounded to BF16 (8-bit significand) on their way
into each product; that rounding, not an error, is what separates the two
and is what these tolerances allow for.

Secondary, tight checks (the same rounding applied by the oracle to the
GPU's own layer inputs, layer by layer): the only difference left is FP32
accumulation order, 2e-6 of the largest output.  The backward pass is
pinned layer by layer the same way: the oracle differentiates the GPU's own
activations with BF16 layer inputs and output gradients as on the matrix
cores (bias gradients in full precision).  Bias gradients agree to 1e-4 of
the largest entry of each layer; weight gradients to 2e-3, since an output
gradient computed in FP32 on the GPU and in FP64 by the oracle can still
round to neighbouring BF16 values (one flip moves a sum of n products by
about 2^-8 / sqrt(n))."""
import numpy as np
import pytest

from oracle import cnn
from _util import ctx_for, dev, host, material

pytestmark = pytest.mark.gpu


def bf16_bits(a):
    """Round-to-nearest-even FP32 -> BF16 bit patterns (uint16)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_value(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def flat_params(params):
    w = np.concatenate([W.ravel() for W, _ in params])
    b = np.concatenate([bb for _, bb in params])
    return w, b


def unflat_weights(wv, bv):
    out, ow, ob = [], 0, 0
    for cin, cout in zip(cnn.CHANNELS[:-1], cnn.CHANNELS[1:]):
        n = 27 * cin * cout
        out.append((wv[ow:ow + n].reshape(27, cin, cout), bv[ob:ob + cout]))
        ow += n
        ob += cout
    return out


def setup(box, seed):
    import torch
    rng = np.random.default_rng(seed)
    params = cnn.init_params(seed)
    params = [(W, rng.standard_normal(W.shape[2]) * 0.1) for W, _ in params]
    w, b = flat_params(params)
    wbits = bf16_bits(w)
    b32 = b.astype(np.float32)
    params_q = unflat_weights(bf16_value(wbits), b32.astype(np.float64))
    nx, ny, nz = box
    x = rng.standard_normal((nz, ny, nx, 8)).astype(np.float32)
    ctx = ctx_for(3, 4, 1, material(4))
    wd = torch.from_numpy(wbits.view(np.int16)).cuda()
    bd = dev(b32)
    act = torch.zeros(ctx.nn_size(2, nx, ny, nz), dtype=torch.float32, device="cuda")
    act[: x.size] = dev(x.ravel())
    return ctx, params_q, x.astype(np.float64), wd, bd, act


def out_of(act, box):
    nx, ny, nz = box
    nvox = nx * ny * nz
    return host(act[168 * nvox:]).reshape(nz, ny, nx, 4)


BOXES = [(5, 4, 3), (7, 6, 5), (33, 20, 17), (40, 30, 29)]


@pytest.mark.parametrize("box", BOXES)
def test_forward_matches_oracle(box):
    print(f"case forward box={box}", flush=True)
    ctx, pq, x, wd, bd, act = setup(box, seed=sum(box))
    ctx.nn_forward(wd, bd, act, box)
    nx, ny, nz = box
    nvox = nx * ny * nz
    chans = cnn.CHANNELS
    offs = [0]
    for c in chans:
        offs.append(offs[-1] + c * nvox)
    layer = [host(act[offs[l]:offs[l + 1]]).astype(np.float64).reshape(nz, ny, nx, chans[l]) for l in range(7)]
    # layer by layer on the GPU's own inputs: FP32 accumulation order only
    for l, (W, b) in enumerate(pq):
        ref = cnn.conv3d(cnn.bf16_round(layer[l]), W, b)
        if l < len(pq) - 1:
            ref = np.maximum(ref, 0.0)
        assert np.abs(layer[l + 1] - ref).max() <= 2e-6 * np.abs(ref).max(), l
    # whole network against the plain FP64 network (unrounded activations)
    ref, _ = cnn.forward(pq, x)
    diff = layer[6] - ref
    assert np.sqrt(np.mean(diff ** 2)) <= 1e-2 * np.sqrt(np.mean(ref ** 2))
    assert np.abs(diff).max() <= 1e-2 * np.abs(ref).max()


@pytest.mark.parametrize("box", BOXES)
def test_loss_and_backward_match_oracle(box):
    import torch
    print(f"case backward box={box}", flush=True)
    ctx, pq, x, wd, bd, act = setup(box, seed=3 * sum(box))
    nx, ny, nz = box
    rng = np.random.default_rng(7)
    target = rng.standard_normal((nz, ny, nx, 4))
    win = (1, nx - 1, 1, ny - 1, 0, nz) if min(box) > 2 else (0, nx, 0, ny, 0, nz)
    window = (slice(win[4], win[5]), slice(win[2], win[3]), slice(win[0], win[1]))
    ctx.nn_forward(wd, bd, act, box)
    dout = torch.empty(nx * ny * nz * 4, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    out_view = act[168 * nx * ny * nz:]
    ctx.nn_mse(out_view, dev(target.astype(np.float32).ravel()), win, dout, loss, box)
    grad = torch.empty(cnn_param_count(), dtype=torch.float32, device="cuda")
    work = torch.empty(ctx.nn_size(3, nx, ny, nz), dtype=torch.float32, device="cuda")
    ctx.nn_backward(wd, act, dout, grad, work, box)
    # the oracle differentiates the GPU's own activations, layer by layer
    acts = []
    off = 0
    for c in cnn.CHANNELS:
        acts.append(host(act[off: off + c * nx * ny * nz]).astype(np.float64).reshape(nz, ny, nx, c))
        off += c * nx * ny * nz
    tq = target.astype(np.float32).astype(np.float64)
    diff = np.zeros_like(acts[6])
    diff[window] = acts[6][window] - tq[window]
    count = diff[window].size
    ref_loss = float(np.sum(diff[window] ** 2) / count)
    assert abs(host(loss)[0] - ref_loss) <= 1e-6 * ref_loss
    dy = 2.0 * diff / count
    ref_grads = [None] * 6
    for l in range(5, -1, -1):
        if l < 5:
            dy = dy * (acts[l + 1] > 0.0)
        dx, dW, db = cnn.conv3d_backward(acts[l], pq[l][0], dy, bf16_weight_grad=True)
        ref_grads[l] = (dW, db)
        dy = dx
    g = host(grad).astype(np.float64)
    gw, gb = g[:120960], g[120960:]
    got = unflat_weights(gw, gb)
    for l, ((dW, db), (rW, rb)) in enumerate(zip(got, ref_grads)):
        sw = np.abs(rW).max()
        sb = max(np.abs(rb).max(), 1e-30)
        assert np.abs(dW - rW).max() <= 2e-3 * sw, (l, np.abs(dW - rW).max() / sw)
        assert np.abs(db - rb).max() <= 1e-4 * sb, (l, np.abs(db - rb).max() / sb)
    # whole network against the plain FP64 network (unrounded activations
    # and gradients): the loss to 1e-2, and on boxes of realistic size the
    # whole gradient to 1e-2 normwise
    loss64, grads64 = cnn.loss_and_grads(pq, x, tq, window)
    assert abs(host(loss)[0] - loss64) <= 1e-2 * loss64
    if nx * ny * nz >= 10000:
        v64 = np.concatenate([np.concatenate([gw_.ravel(), gb_]) for gw_, gb_ in grads64])
        vg = np.concatenate([np.concatenate([gw_.ravel(), gb_]) for gw_, gb_ in got])
        rel = np.linalg.norm(vg - v64) / np.linalg.norm(v64)
        print(f"gradient vs FP64: {rel:.2e} normwise", flush=True)
        assert rel <= 1e-2


def cnn_param_count():
    return sum(27 * a * b + b for a, b in zip(cnn.CHANNELS[:-1], cnn.CHANNELS[1:]))


def test_backward_is_deterministic():
    import torch
    box = (40, 30, 29)
    ctx, pq, x, wd, bd, act = setup(box, seed=11)
    nx, ny, nz = box
    ctx.nn_forward(wd, bd, act, box)
    rng = np.random.default_rng(3)
    dout = dev(rng.standard_normal(nx * ny * nz * 4).astype(np.float32))
    work = torch.empty(ctx.nn_size(3, nx, ny, nz), dtype=torch.float32, device="cuda")
    g1 = torch.empty(cnn_param_count(), dtype=torch.float32, device="cuda")
    g2 = torch.empty_like(g1)
    ctx.nn_backward(wd, act, dout, g1, work, box)
    ctx.nn_backward(wd, act, dout, g2, work, box)
    assert torch.equal(g1, g2)


def test_adam_and_bf16_match_oracle():
    import torch
    n = cnn_param_count()
    rng = np.random.default_rng(5)
    p = rng.standard_normal(n).astype(np.float32)
    g = (rng.standard_normal(n) * 1e-2).astype(np.float32)
    m = (rng.standard_normal(n) * 1e-3).astype(np.float32)
    v = (rng.uniform(0, 1e-4, n)).astype(np.float32)
    ctx = ctx_for(3, 4, 1, material(4))
    pd, gd, md, vd = dev(p), dev(g), dev(m), dev(v)
    wb = torch.zeros(120960, dtype=torch.int16, device="cuda")
    ctx.nn_adam_step(1e-3, 3, gd, pd, md, vd, wb, n_bf16=120960)
    rp, rm, rv = cnn.adam_step(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                               v.astype(np.float64), 3, 1e-3)
    assert np.abs(host(md) - rm).max() <= 1e-6 * np.abs(rm).max()
    assert np.abs(host(vd) - rv).max() <= 1e-6 * np.abs(rv).max()
    assert np.abs(host(pd) - rp).max() <= 1e-6 * np.abs(rp).max()
    # the BF16 copy is the RNE rounding of the updated FP32 master, bit for bit
    assert np.array_equal(host(wb).view(np.uint16), bf16_bits(host(pd)[:120960]))
    wb2 = torch.zeros_like(wb)
    ctx.nn_to_bf16(pd, wb2)
    assert torch.equal(wb, wb2)


def test_features():
    """in8 = FP32(x) * scale (bitwise) and FP32(g / rms(g)) * scale, rms per
    component over the nodes."""
    N = 6
    ctx = ctx_for(3, N, 1, material(N))
    n = (N + 1) ** 3
    rng = np.random.default_rng(9)
    x = rng.standard_normal(4 * n)
    g = rng.standard_normal(4 * n) * np.array([1e-5, 2e-5, 3e-6, 1e-7] * n)
    g[3::4][::3] = 0.0
    sc = rng.uniform(0.5, 2e3, 12).astype(np.float32)
    got = host(ctx.nn_features(1, dev(x), dev(g), dev(sc))).reshape(n, 8)
    ref_x = x.reshape(n, 4).astype(np.float32) * sc[:4]
    assert np.array_equal(got[:, :4], ref_x)
    rms = np.sqrt((g.reshape(n, 4) ** 2).mean(axis=0))
    ref_g = (g.reshape(n, 4) / rms) * sc[4:8].astype(np.float64)
    assert np.abs(got[:, 4:] - ref_g).max() <= 1e-6 * np.abs(ref_g).max()


def test_propose_matches_oracle_and_stays_in_box():
    """Features, forward pass and projection onto [lo, hi] in one call."""
    import ctypes
    import torch
    from paper_2007_12908_amd import binding
    N = 8
    box = (N + 1,) * 3
    ctx, pq, _, wd, bd, _ = setup(box, seed=21)
    ctx = ctx_for(3, N, 1, material(N))
    n = (N + 1) ** 3
    rng = np.random.default_rng(13)
    x = rng.standard_normal(4 * n) * 1e-3
    g = rng.standard_normal(4 * n) * 1e-6
    lo = -rng.uniform(0, 2e-3, 4 * n)
    hi = rng.uniform(0, 2e-3, 4 * n)
    lo[::7] = hi[::7] = 0.0
    sc = np.array([1e3] * 4 + [1.0] * 4 + [1e3] * 4, dtype=np.float32)
    scd = dev(sc)
    net = binding.Net(ctypes.c_void_p(wd.data_ptr()), ctypes.c_void_p(bd.data_ptr()),
                      ctypes.c_void_p(scd.data_ptr()))
    s = host(ctx.nn_propose(1, net, dev(x), dev(g), dev(lo), dev(hi)))
    rms = np.sqrt((g.reshape(n, 4) ** 2).mean(axis=0))
    feat = np.empty((n, 8))
    feat[:, :4] = (x.reshape(n, 4).astype(np.float32) * sc[:4]).astype(np.float64)
    feat[:, 4:] = (g.reshape(n, 4) / rms) * sc[4:8].astype(np.float64)
    out, _ = cnn.forward(pq, feat.reshape(N + 1, N + 1, N + 1, 8))
    raw = out.reshape(n, 4) * sc[8:].astype(np.float64) * rms
    ref = np.clip(raw.ravel(), lo, hi)
    assert np.all(s >= lo) and np.all(s <= hi)
    assert np.abs(s - ref).max() <= 1e-2 * np.abs(raw).max()
    # non-finite network output (NaN bias) gives a zero step
    bnan = torch.full_like(bd, float("nan"))
    net2 = binding.Net(ctypes.c_void_p(wd.data_ptr()), ctypes.c_void_p(bnan.data_ptr()),
                       ctypes.c_void_p(scd.data_ptr()))
    s2 = host(ctx.nn_propose(1, net2, dev(x), dev(g), dev(lo), dev(hi)))
    assert np.all(s2 == np.clip(0.0, lo, hi))


def test_normalisation_calls():
    """rmtr_nn_channel_rms, rmtr_nn_target and rmtr_nn_fit_scales against
    their definitions (per-component RMS over the nodes; target = s_k /
    (scale_k rms(g_k)); scales from means over samples)."""
    import torch
    N = 6
    ctx = ctx_for(3, N, 1, material(N))
    n = (N + 1) ** 3
    rng = np.random.default_rng(17)
    samples, ref_x, ref_ratio = [], [], []
    for i in range(3):
        x = rng.standard_normal(4 * n) * np.array([1e-3, 2e-3, 5e-4, 0.3] * n)
        g = rng.standard_normal(4 * n) * np.array([1e-5, 2e-5, 3e-6, 1e-7] * n)
        s = rng.standard_normal(4 * n) * np.array([1e-4, 1e-4, 2e-4, 1e-2] * n)
        if i == 1:
            g[3::4] = 0.0                                  # a channel with rms(g) = 0
        samples.append((dev(x), dev(g), dev(s)))
        rx = np.sqrt((x.reshape(n, 4) ** 2).mean(axis=0))
        rg = np.sqrt((g.reshape(n, 4) ** 2).mean(axis=0))
        rs = np.sqrt((s.reshape(n, 4) ** 2).mean(axis=0))
        ref_x.append(rx)
        ref_ratio.append(np.where(rg > 0, rs / np.where(rg > 0, rg, 1.0), 0.0))
        got = host(ctx.nn_channel_rms(1, samples[-1][1]))
        assert np.allclose(got, rg, rtol=1e-13, atol=0)
    sc = torch.empty(12, dtype=torch.float32, device="cuda")
    ctx.nn_fit_scales(1, samples, sc)
    want = np.concatenate([1.0 / np.mean(ref_x, axis=0), np.ones(4), np.mean(ref_ratio, axis=0)])
    assert np.allclose(host(sc), want.astype(np.float32), rtol=1e-6, atol=0)
    x, g, s = samples[0]
    t = host(ctx.nn_target(1, g, s, sc)).astype(np.float64)
    rg = np.sqrt((host(g).reshape(n, 4) ** 2).mean(axis=0))
    tw = host(s).reshape(n, 4) / (host(sc)[8:].astype(np.float64) * rg)
    assert np.allclose(t.reshape(n, 4), tw, rtol=1e-6, atol=0)
    _, g1, s1 = samples[1]
    t1 = host(ctx.nn_target(1, g1, s1, sc)).reshape(n, 4)
    assert np.all(t1[:, 3] == 0.0)
