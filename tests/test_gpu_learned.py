"""The learned finest-level proposal inside the RMTR load step (GPU).

A proposal never weakens the method: it is projected onto the step box and
taken only if the FP64 trust-region ratio accepts it, it reaches the Cauchy
decrease of the model and it lowers the energy at least as much as the
smoother step from the same state, and the smoother runs otherwise.  So a network
whose output is not finite, or absurdly large, must leave the run bit for
bit identical to the plain one; and a trained network
is compared with the untrained one and with the plain method on a held-out
fracture network (what it gains is printed and recorded)."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import fem
from _util import material, ctx_for, dev, host

pytestmark = pytest.mark.gpu

N, L = 32, 3


def _problem(seed, n_frac):
    import torch
    mat = material(N)
    ctx = ctx_for(3, N, L, mat)
    tab = W.disc_table(n_frac, seed, 0.2, 0.8, 0.05, 0.12)
    c0, p = ctx.init_fields(L, tab, 1.0 / N, p_mode=0, p_value=1e-3)
    x = torch.zeros(4 * (N + 1) ** 3, dtype=torch.float64, device="cuda")
    x[3::4] = c0
    return ctx, mat, c0, p, x


def _certify(mat, x, p, c0):
    g = fem.Grid(3, N)
    xh, ph, ch = host(x), host(p), host(c0)
    x0 = np.zeros_like(xh)
    x0[3::4] = ch
    chi0 = fem.chi(g, x0, fem.gradient(g, x0, ph, mat), ch)
    chi = fem.chi(g, xh, fem.gradient(g, xh, ph, mat), ch)
    c = xh[3::4]
    assert np.all(c >= ch) and np.all(c <= 1.0)
    assert np.all(xh[g.default_dirichlet()] == 0.0)
    return chi / chi0


def _solve(ctx, x, p, c0, net=None, max_vcycles=200, patience=0):
    import ctypes
    import paper_2007_12908_amd as P
    prm = P.default_params(max_vcycles=max_vcycles, nn_patience=patience)
    if net is not None:
        prm.use_learned = 1
        prm.nn = ctypes.pointer(net)
    return ctx.solve_loadstep(x, p, c0, prm)


def test_nonfinite_proposals_leave_the_run_unchanged():
    import torch
    from paper_2007_12908_amd import learned
    print("case nan network", flush=True)
    ctx, mat, c0, p, x = _problem(1001, 6)
    xa = x.clone()
    sa = _solve(ctx, xa, p, c0)
    net = learned.ProposalNet(ctx, seed=1)
    net.master[learned.NW:] = float("nan")
    xb = x.clone()
    sb = _solve(ctx, xb, p, c0, net.net())
    assert torch.equal(xa, xb)
    assert sb["vcycles"] == sa["vcycles"] and sb["nn_accepted"] == 0
    assert sb["nn_proposed"] == sb["vcycles"]
    # with patience 3 the network stops proposing after three rejections
    xc = x.clone()
    sc = _solve(ctx, xc, p, c0, net.net(), patience=3)
    assert torch.equal(xa, xc) and sc["nn_proposed"] == min(3, sc["vcycles"])


def test_absurd_proposals_are_gated():
    """Outputs scaled by 1e30 land on random corners of the step box: they
    never reach the Cauchy decrease, so every one is rejected and the run is
    the plain one, bit for bit."""
    import torch
    from paper_2007_12908_amd import learned
    print("case huge network output", flush=True)
    ctx, mat, c0, p, x = _problem(1001, 6)
    xa = x.clone()
    sa = _solve(ctx, xa, p, c0)
    net = learned.ProposalNet(ctx, seed=2)
    net.scales[8:] = 1e30
    xb = x.clone()
    st = _solve(ctx, xb, p, c0, net.net())
    print({k: st[k] for k in ("code", "vcycles", "nn_proposed", "nn_accepted")}, flush=True)
    assert st["nn_proposed"] == st["vcycles"] and st["nn_accepted"] == 0
    assert torch.equal(xa, xb) and st["code"] == sa["code"] == 0
    assert _certify(mat, xb, p, c0) <= 1e-8 * (1 + 1e-6)


def test_trained_network_against_plain_and_untrained():
    """Train on states of three fracture networks, deploy on a held-out one;
    each variant runs 40 V-cycles (or to 1e-8).  Training must lower the
    loss; every result is feasible and its chi, re-evaluated by the FP64
    oracle, equals the GPU's; runs whose proposals are all refused by the
    gate are the plain run bit for bit.  What the trained network gains
    (accepted proposals, chi reached, time) is recorded, not asserted: the
    measured gain on these networks is nil (no proposal passes the gate's
    comparison with the smoother step)."""
    from paper_2007_12908_amd import learned
    print("case train and deploy", flush=True)
    samples = []
    ctxs = []
    for r in range(3):
        ctx, mat, c0, p, x = _problem(2000 + r, 4 + 2 * r)
        ctxs.append(ctx)
        samples += learned.harvest_run(ctx, x, p, c0, 8)
    ctx, mat, c0, p, x = _problem(1001, 6)
    net = learned.ProposalNet(ctx, seed=3)
    learned.fit_scales(net, samples)
    tr = learned.Trainer(net, L, lr=1e-3)
    tr.add(samples)
    loss0 = tr.mean_loss()
    done, secs = tr.train(300, seed=4)
    loss1 = tr.mean_loss()
    print(f"training: {len(samples)} samples, {done} steps, {secs:.2f} s, loss {loss0:.4f} -> {loss1:.4f}",
          flush=True)
    assert loss1 < 0.75 * loss0

    runs = {}
    untrained = learned.ProposalNet(ctx, seed=3)
    untrained.scales.copy_(net.scales)
    for name, n in (("plain", None), ("untrained", untrained), ("trained", net)):
        xr = x.clone()
        st = _solve(ctx, xr, p, c0, None if n is None else n.net(), max_vcycles=40)
        rel = _certify(mat, xr, p, c0)
        assert abs(rel - st["chi"] / st["chi0"]) <= 1e-6 * rel
        runs[name] = {k: st[k] for k in ("code", "vcycles", "nn_proposed", "nn_accepted", "seconds", "energy")}
        runs[name]["chi_rel_oracle"] = rel
    print(json.dumps(runs), flush=True)
    out = os.environ.get("RMTR_LEARNED_REPORT")
    if out:
        with open(out, "w") as f:
            json.dump({"training": {"samples": len(samples), "steps": done, "seconds": secs, "loss0": loss0,
                                    "loss1": loss1}, "runs": runs}, f, indent=1)
    for name in ("untrained", "trained"):
        if runs[name]["nn_accepted"] == 0:
            assert runs[name]["vcycles"] == runs["plain"]["vcycles"]
            assert runs[name]["energy"] == runs["plain"]["energy"]
