"""Learned finest-level proposal: harvesting, training and deployment.

The network (six 3x3x3 convolutions, 8 -> 32 x 5 -> 4 channels, see
include/rmtr.h) maps the state (u, c) and gradient g of the finest level to
a proposed step.  It is trained on pairs harvested from the plain method:
for a state x at the start of a V-cycle, the target is the correction the
projected Gauss-Seidel smoother computes for the trust-region subproblem
eq. (model_qp) with the Hessian at x (Sec. 3.2.1), i.e. the step the first
finest-level pre-smoothing step of Alg. 1 would take.  Training runs on the
GPU through the library's own forward, backward, loss and Adam kernels
(BF16 weights, FP32 masters and arithmetic).  Deployed, every proposal is
projected onto the step box and must pass the FP64 trust-region ratio test;
the smoother is the fallback (rmtr_solve_loadstep with use_learned).

Torch is used for device memory and copies between buffers; the
normalisation constants, features and targets are library calls.
"""
import ctypes
import time

import numpy as np
import torch

from . import binding

NW = binding.NN_WEIGHTS
NB = binding.NN_BIASES


class ProposalNet:
    """FP32 master parameters, Adam moments, BF16 weights and scales on the GPU."""

    def __init__(self, ctx, seed=0):
        self.ctx = ctx
        rng = np.random.default_rng(seed)
        parts = []
        chans = binding.NN_CHANNELS
        for cin, cout in zip(chans[:-1], chans[1:]):
            parts.append(rng.standard_normal(27 * cin * cout) * np.sqrt(2.0 / (27 * cin)))
        parts.append(np.zeros(NB))
        self.master = torch.from_numpy(np.concatenate(parts).astype(np.float32)).cuda()
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.w = torch.zeros(NW, dtype=torch.int16, device="cuda")
        self.scales = torch.ones(12, dtype=torch.float32, device="cuda")
        self.t = 0
        ctx.nn_to_bf16(self.master[:NW], self.w)

    @property
    def bias(self):
        return self.master[NW:]

    def net(self):
        """rmtr_nn view (keep this object alive while it is used)."""
        return binding.Net(ctypes.c_void_p(self.w.data_ptr()), ctypes.c_void_p(self.bias.data_ptr()),
                           ctypes.c_void_p(self.scales.data_ptr()))

    def state_dict(self):
        return {"master": self.master.cpu().numpy(), "scales": self.scales.cpu().numpy()}

    def load_state_dict(self, d):
        self.master.copy_(torch.from_numpy(np.asarray(d["master"], dtype=np.float32)))
        self.scales.copy_(torch.from_numpy(np.asarray(d["scales"], dtype=np.float32)))
        self.ctx.nn_to_bf16(self.master[:NW], self.w)


def harvest(ctx, x, p, c_lower, delta=1.0, sweeps=3, dirichlet=None):
    """(g, s) at state x of the finest level: the gradient and the projected
    Gauss-Seidel correction of the trust-region subproblem at x."""
    L = ctx.L
    g = ctx.gradient(L, x, p, dirichlet)
    lo, hi = ctx.step_box(L, x, c_lower, delta, dirichlet)
    s = torch.zeros_like(x)
    ctx.smooth(L, x, p, g, lo, hi, s, sweeps, dirichlet)
    return g, s


def harvest_run(ctx, x, p, c_lower, n_states, sweeps=3, params=None, dirichlet=None, target="pgs"):
    """States along a plain RMTR run: harvest at x, then one V-cycle, repeated.

    target "pgs": the projected Gauss-Seidel correction of the TR subproblem
    at x (what the first pre-smoothing step computes); "vcycle": the whole
    correction x_next - x that the plain V-cycle from x makes."""
    if target not in ("pgs", "vcycle"):
        raise ValueError(f"unknown target {target!r}")
    prm = params if params is not None else binding.default_params()
    prm.max_vcycles = 1
    prm.use_learned = 0
    out = []
    for _ in range(n_states):
        g, s = harvest(ctx, x, p, c_lower, prm.delta0, sweeps, dirichlet)
        x0 = x.clone()
        st = ctx.solve_loadstep(x, p, c_lower, prm, dirichlet)
        if target == "vcycle":
            s = x - x0
        out.append((x0, g, s))
        if st["code"] == binding.RMTR_OK:
            break
    return out


def fit_scales(net, samples, level=None):
    """Normalisation constants (rmtr_nn_fit_scales): x channels by their RMS
    over the samples; g enters divided by its own per-component RMS, so its
    scale is 1; output channel k is scaled by the mean ratio
    rms(s_k) / rms(g_k) of the samples (and, at run time, by rms(g_k))."""
    ctx = net.ctx
    ctx.nn_fit_scales(ctx.L if level is None else level, samples, net.scales)


def rescale_for_grid(net, h_train, h_deploy, dim):
    """Adapt the output scales of a network trained on a grid of spacing
    h_train to a grid of spacing h_deploy.  The smoother correction is about
    D^-1 g with D the diagonal of the lagged Hessian, which scales like
    h^(d-2) on displacement rows (elastic stiffness) and like h^(d-1) on
    phase-field rows (G_c / l_s and G_c l_s terms with l_s proportional to
    h), so the ratio rms(s_k) / rms(g_k) fitted at h_train is multiplied by
    (h_train / h_deploy)^(d-2) for u and (h_train / h_deploy)^(d-1) for c.
    The input scales are left alone (u and c keep their magnitudes, g enters
    divided by its own RMS).  Host-side update of the four output scales."""
    r = float(h_train) / float(h_deploy)
    sc = net.scales.detach().cpu().numpy().astype(np.float64)
    sc[8:8 + dim] *= r ** (dim - 2)
    sc[8 + dim] *= r ** (dim - 1)
    net.scales.copy_(torch.from_numpy(sc.astype(np.float32)))


class Trainer:
    """Adam on the MSE between the network output and the scaled targets,
    one whole node grid per step (every 32^3 patch of it at once)."""

    def __init__(self, net, level, lr=1e-3):
        self.net, self.ctx, self.level, self.lr = net, net.ctx, level, lr
        n = net.ctx.level_cells(level) + 1
        self.box = (n, n, n)
        self.nvox = n ** 3
        self.act = torch.zeros(self.ctx.nn_size(2, *self.box), dtype=torch.float32, device="cuda")
        self.work = torch.empty(self.ctx.nn_size(3, *self.box), dtype=torch.float32, device="cuda")
        self.dout = torch.empty(self.nvox * 4, dtype=torch.float32, device="cuda")
        self.grad = torch.empty(NW + NB, dtype=torch.float32, device="cuda")
        self.loss = torch.empty(1, dtype=torch.float64, device="cuda")
        self.window = (1, n - 1, 1, n - 1, 1, n - 1)
        self.data = []

    def add(self, samples):
        """Scaled features and targets of (x, g, s) samples (after fit_scales):
        the target of channel k is s_k / (scale_k rms(g_k)) (rmtr_nn_target)."""
        for x, g, s in samples:
            feat = self.ctx.nn_features(self.level, x, g, self.net.scales)
            tgt = self.ctx.nn_target(self.level, g, s, self.net.scales)
            self.data.append((feat, tgt))

    def forward_loss(self, i):
        feat, tgt = self.data[i]
        self.act[: feat.numel()].copy_(feat)
        self.ctx.nn_forward(self.net.w, self.net.bias, self.act, self.box)
        self.ctx.nn_mse(self.act[168 * self.nvox:], tgt, self.window, self.dout, self.loss, self.box)

    def step(self, i):
        self.forward_loss(i)
        self.ctx.nn_backward(self.net.w, self.act, self.dout, self.grad, self.work, self.box)
        self.net.t += 1
        self.ctx.nn_adam_step(self.lr, self.net.t, self.grad, self.net.master, self.net.m, self.net.v, self.net.w,
                              n_bf16=NW)

    def mean_loss(self, idx=None):
        idx = range(len(self.data)) if idx is None else idx
        tot = 0.0
        for i in idx:
            self.forward_loss(i)
            tot += float(self.loss.item())
        return tot / max(len(idx), 1)

    def train(self, steps, seed=0, time_limit=None):
        rng = np.random.default_rng(seed)
        t0 = time.perf_counter()
        done = 0
        for k in range(steps):
            self.step(int(rng.integers(len(self.data))))
            done = k + 1
            if time_limit is not None and (k & 7) == 7:
                torch.cuda.synchronize()
                if time.perf_counter() - t0 > time_limit:
                    break
        torch.cuda.synchronize()
        return done, time.perf_counter() - t0
