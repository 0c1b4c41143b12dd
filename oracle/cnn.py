"""Oracle: the 3D convolutional network of the learned smoother proposal.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Network (the learned-proposal form of the method): six 3x3x3 convolutions
with zero ('same') padding, channels 8 -> 32 -> 32 -> 32 -> 32 -> 32 -> 4,
ReLU after the first five.  Tensors are channels-last on a box of voxels,
shape (nz, ny, nx, C) with x fastest, matching the node-major grid layout.
Weights of layer l have shape (27, Cin, Cout) with offset index
k = (dx+1) + 3 (dy+1) + 9 (dz+1); biases (Cout,).

    y[v, co] = b[co] + sum_k sum_ci W[k, ci, co] x[v + off(k), ci]

Loss: mean squared error over the voxels of an interior window and all
output channels.  Adam (Kingma and Ba) with bias correction.

Option bf16_inputs: each layer's input is rounded to bfloat16 (nearest,
ties to even, through float32) before its convolution, and the weight and
data gradients multiply bfloat16-rounded layer inputs and output gradients
(with the bfloat16 weights), the precision of the matrix-core form; the
rounding is otherwise treated as the identity (bias gradients in full
precision, no gradient through the rounding).
"""
import numpy as np

CHANNELS = (8, 32, 32, 32, 32, 32, 4)


def offsets():
    return [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shifted(x, d):
    """out[v] = x[v + d] with zeros outside (x: (nz, ny, nx, C))."""
    dx, dy, dz = d
    out = np.zeros_like(x)
    nz, ny, nx = x.shape[:3]
    zs, ys, xs = slice(max(0, -dz), nz - max(0, dz)), slice(max(0, -dy), ny - max(0, dy)), \
        slice(max(0, -dx), nx - max(0, dx))
    zt, yt, xt = slice(max(0, dz), nz - max(0, -dz)), slice(max(0, dy), ny - max(0, -dy)), \
        slice(max(0, dx), nx - max(0, -dx))
    out[zs, ys, xs] = x[zt, yt, xt]
    return out


def conv3d(x, W, b):
    y = np.broadcast_to(b, x.shape[:3] + (W.shape[2],)).copy()
    for k, d in enumerate(offsets()):
        y += shifted(x, d) @ W[k]
    return y


def conv3d_backward(x, W, dy, bf16_weight_grad=False):
    """Gradients of sum(dy * conv3d(x, W, b)) w.r.t. x, W and b.  With
    bf16_weight_grad the weight gradient takes x and dy rounded to bfloat16
    and the data gradient dy rounded to bfloat16 (the matrix-core form); db
    uses dy unrounded."""
    dW = np.zeros_like(W)
    dx = np.zeros_like(x)
    xq = bf16_round(x) if bf16_weight_grad else x
    dyq = bf16_round(dy) if bf16_weight_grad else dy
    for k, d in enumerate(offsets()):
        xs = shifted(xq, d)
        dW[k] = xs.reshape(-1, x.shape[3]).T @ dyq.reshape(-1, dy.shape[3])
        # y[v] gets x[v + d] W: x[u] feeds y[u - d]
        dx += shifted(dyq, (-d[0], -d[1], -d[2])) @ W[k].T
    db = dy.reshape(-1, dy.shape[3]).sum(axis=0)
    return dx, dW, db


def init_params(seed, channels=CHANNELS):
    """He-normal weights from a seeded generator, zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        W = rng.standard_normal((27, cin, cout)) * np.sqrt(2.0 / (27 * cin))
        params.append((W, np.zeros(cout)))
    return params


def bf16_round(a):
    """Nearest bfloat16 (ties to even) of float32(a), as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, x, bf16_inputs=False):
    """Returns the output and the per-layer activations (inputs of each layer)."""
    acts = [x]
    h = x
    L = len(params)
    for l, (W, b) in enumerate(params):
        h = conv3d(bf16_round(h) if bf16_inputs else h, W, b)
        if l < L - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return h, acts


def loss_and_grads(params, x, target, window, bf16_inputs=False):
    """MSE over the window (slices of z, y, x) and channels; gradients."""
    out, acts = forward(params, x, bf16_inputs)
    diff = np.zeros_like(out)
    sel = (window[0], window[1], window[2], slice(None))
    diff[sel] = out[sel] - target[sel]
    count = diff[sel].size
    loss = float(np.sum(diff[sel] ** 2) / count)
    dy = 2.0 * diff / count
    grads = [None] * len(params)
    L = len(params)
    for l in range(L - 1, -1, -1):
        if l < L - 1:
            dy = dy * (acts[l + 1] > 0.0)
        W, b = params[l]
        dx, dW, db = conv3d_backward(acts[l], W, dy, bf16_inputs)
        grads[l] = (dW, db)
        dy = dx
    return loss, grads


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
