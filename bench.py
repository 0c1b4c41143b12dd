#!/usr/bin/env python
"""Benchmark of the RMTR hot path on one MI355X.

One step = energy, gradient and Hessian-vector product (FP64, matrix-free)
over the fine level of the workload, inputs resident in HBM.  `value` is the
fine-level dofs passed through that triple per second (GDoF/s).  The same run
reports each kernel's own rate, the mixed-precision (FP32) Hv, the roofline
of the dominant kernel (HIP events on the launch stream), the RMTR load step
to 1e-8 (plain FP64, mixed precision, and mixed precision with the learned
proposal, whose harvesting and training are timed apart), and the CPU oracle
on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDoF/s energy/grad/Hv; RMTR s/load-step plain vs mixed+learned at 1e-8"
PEAK_FP64 = 78.6      # TFLOP/s, MI355X FP64 vector (= FP64 matrix)
PEAK_HBM = 8000.0     # GB/s
KERNEL_SOURCES = ["paper_2007_12908_amd/csrc/elem_kernels.hip", "paper_2007_12908_amd/csrc/rmtr_device.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_hessvec_c2_3d_128.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """Per-launch HBM bytes of the Hv kernel from committed PMC counters, or
    None when the kernel sources changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash():
        return None
    return t.get("bytes_per_launch")


def time_calls(fn, n, torch):
    """Average duration of fn() over n calls, with HIP events on torch's
    current stream (the stream librmtr launches on)."""
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(n):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / n


def cpu_baseline(wl, x_np, p_np, v_np, budget_s=20.0):
    """The oracle, as it is, on the first z-layers of the workload grid."""
    import numpy as np
    from oracle import fem
    g = fem.Grid(3, wl.n_cells)
    mat = fem.material_from_E_nu(wl.E, wl.nu, wl.Gc, wl.ls, wl.k)
    ne = 256
    while True:
        elems = np.arange(ne)
        t0 = time.perf_counter()
        fem.energy(g, x_np, p_np, mat, elems)
        fem.gradient(g, x_np, p_np, mat, None, elems)
        H = fem.hessian(g, x_np, p_np, mat, None, elems)
        _ = H @ v_np
        dt = time.perf_counter() - t0
        if dt * 4 > budget_s or ne >= wl.n_cells ** 3:
            break
        ne *= 2
    # one element per node in the large-grid limit: 4 dofs per element
    return {"value": 4 * ne / dt / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": f"energy+gradient+Hv over the first {ne} elements of the {wl.n_cells}^3 grid "
                      f"(4 dofs per element), numpy/scipy FP64 single thread, {dt:.1f} s"}


def learned_leg(ctx, wl, P, W, torch, train_seconds, target):
    """Harvest (state, gradient) -> PGS-correction pairs from plain runs on
    other fracture networks of the same grid (10-50 discs, seeds 1000 + r),
    train the proposal network on the GPU, and return it with the training
    figures (reported apart from the load-step time)."""
    from paper_2007_12908_amd import learned
    N, L = wl.n_cells, wl.n_levels
    t0 = time.perf_counter()
    samples = []
    for r in range(3):
        nf = (10, 30, 50)[r]
        tab = W.disc_table(nf, 1000 + r, 0.2, 0.8, 0.03, 0.08)
        c0r, pr = ctx.init_fields(L, tab, band=wl.h, p_mode=0, p_value=wl.p)
        xr = torch.zeros(4 * (N + 1) ** 3, dtype=torch.float64, device="cuda")
        xr.view(-1, 4)[:, 3] = c0r
        samples += learned.harvest_run(ctx, xr, pr, c0r, 6, target=target)
    torch.cuda.synchronize()
    t_harvest = time.perf_counter() - t0
    net = learned.ProposalNet(ctx, seed=0)
    learned.fit_scales(net, samples)
    tr = learned.Trainer(net, L, lr=3e-4)
    tr.add(samples)
    del samples
    loss0 = tr.mean_loss()
    steps, t_train = tr.train(100000, seed=1, time_limit=train_seconds)
    loss1 = tr.mean_loss()
    info = {"target": target, "samples": len(tr.data), "harvest_s": t_harvest, "train_steps": steps, "train_s": t_train,
            "loss_initial": loss0, "loss_final": loss1}
    tr.data = []
    return net, info


PEAK_BF16 = 2500.0    # TFLOP/s, dense BF16 matrix cores


def cnn_leg(ctx, L, torch, reps):
    """Forward and backward pass of the proposal network over the finest node
    grid (one whole-grid training step without Adam), timed with HIP events;
    flops count the multiply-adds of the convolutions (forward 120,960 per
    voxel; backward: weight gradient of every layer plus data gradient of
    layers 2-6)."""
    from paper_2007_12908_amd import learned
    n = ctx.level_cells(L) + 1
    box = (n, n, n)
    nvox = n ** 3
    net = learned.ProposalNet(ctx, seed=0)
    gen = torch.Generator(device="cuda").manual_seed(5)
    act = torch.zeros(ctx.nn_size(2, *box), dtype=torch.float32, device="cuda")
    act[: 8 * nvox].normal_(generator=gen)
    work = torch.empty(ctx.nn_size(3, *box), dtype=torch.float32, device="cuda")
    dout = torch.empty(4 * nvox, dtype=torch.float32, device="cuda").normal_(generator=gen)
    grad = torch.empty(learned.NW + learned.NB, dtype=torch.float32, device="cuda")
    t_f = time_calls(lambda: ctx.nn_forward(net.w, net.bias, act, box), reps, torch)
    t_b = time_calls(lambda: ctx.nn_backward(net.w, act, dout, grad, work, box), reps, torch)
    mac_f = 120960 * nvox
    mac_b = (120960 + 120960 - 27 * 8 * 32) * nvox
    tf_f, tf_b = 2 * mac_f / t_f / 1e9, 2 * mac_b / t_b / 1e9
    return {"box": n, "forward_ms": t_f, "backward_ms": t_b, "forward_TFLOP/s": tf_f, "backward_TFLOP/s": tf_b,
            "forward_frac_bf16": tf_f / PEAK_BF16, "backward_frac_bf16": tf_b / PEAK_BF16}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2_3d_128")
    ap.add_argument("--no-loadstep", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--train-seconds", type=float, default=60.0)
    ap.add_argument("--learned-target", choices=("pgs", "vcycle"), default="pgs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kernels-only", action="store_true",
                    help="time only the kernel triple (for profiler runs)")
    ap.add_argument("--cnn-only", action="store_true",
                    help="time only the network's forward and backward passes (for profiler runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    import paper_2007_12908_amd as P
    from paper_2007_12908_amd import binding

    wl = W.WORKLOADS[args.workload]
    assert wl.dim == 3
    N, L = wl.n_cells, wl.n_levels
    ctx = P.Context(3, N, L, wl.lam, wl.mu, wl.Gc, wl.ls, wl.k)
    c0, p = ctx.init_fields(L, wl.fractures(), band=wl.h, p_mode=0, p_value=wl.p)
    n_nodes = (N + 1) ** 3
    n_dofs = 4 * n_nodes
    rng = np.random.default_rng(1234)
    x_np = np.zeros(n_dofs)
    x_np.reshape(-1, 4)[:, :3] = rng.standard_normal((n_nodes, 3)) * 1e-4
    c0_np = c0.cpu().numpy()
    x_np.reshape(-1, 4)[:, 3] = c0_np
    ijk = np.stack(np.unravel_index(np.arange(n_nodes), (N + 1,) * 3, order="F"), axis=1)
    bnd = np.any((ijk == 0) | (ijk == N), axis=1)
    x_np.reshape(-1, 4)[bnd, :3] = 0.0
    v_np = rng.standard_normal(n_dofs)
    x = torch.from_numpy(x_np).cuda()
    v = torch.from_numpy(v_np).cuda()
    x32, p32, v32 = x.float(), p.float(), v.float()
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty_like(x)
    hv = torch.empty_like(x)
    hv32 = torch.empty_like(x32)

    if args.cnn_only:
        log(json.dumps({"cnn": cnn_leg(ctx, L, torch, max(args.steps, 5))}))
        return

    def step():
        ctx.energy(L, x, p, out=E)
        ctx.gradient(L, x, p, out=g)
        ctx.hessvec(L, x, p, v, out=hv)

    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float64, device="cuda")   # 2 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) / args.steps * 1e3

    reps = max(args.steps, 5)
    t_e = time_calls(lambda: ctx.energy(L, x, p, out=E), reps, torch)
    t_g = time_calls(lambda: ctx.gradient(L, x, p, out=g), reps, torch)
    t_h = time_calls(lambda: ctx.hessvec(L, x, p, v, out=hv), reps, torch)
    t_h32 = time_calls(lambda: ctx.hessvec(L, x32, p32, v32, out=hv32), reps, torch)
    if args.kernels_only:
        log(json.dumps({"ms": {"energy": t_e, "gradient": t_g, "hessvec": t_h, "hessvec_fp32": t_h32}}))
        return

    ne = N ** 3
    fl = {k: binding.element_flops(3, kk) for k, kk in (("energy", 0), ("gradient", 2), ("hessvec", 3))}
    per = {
        "energy": {"ms": t_e, "GDoF/s": n_dofs / t_e / 1e6, "TFLOP/s": fl["energy"] * ne / t_e / 1e9},
        "gradient": {"ms": t_g, "GDoF/s": n_dofs / t_g / 1e6, "TFLOP/s": fl["gradient"] * ne / t_g / 1e9},
        "hessvec": {"ms": t_h, "GDoF/s": n_dofs / t_h / 1e6, "TFLOP/s": fl["hessvec"] * ne / t_h / 1e9},
        "hessvec_fp32": {"ms": t_h32, "GDoF/s": n_dofs / t_h32 / 1e6,
                         "TFLOP/s": fl["hessvec"] * ne / t_h32 / 1e9},
    }
    # dominant kernel of the step: the slowest of the three FP64 kernels
    dom = max(("energy", "gradient", "hessvec"), key=lambda k: per[k]["ms"])
    achieved = per[dom]["TFLOP/s"]
    traffic = measured_traffic() if dom == "hessvec" else None
    roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": PEAK_FP64, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64, "traffic": traffic,
            "flops_per_element": fl[dom], "elements": ne,
            "hbm_GB/s_algorithmic": {"energy": 40 * n_nodes / t_e / 1e6, "gradient": 72 * n_nodes / t_g / 1e6,
                                     "hessvec": 104 * n_nodes / t_h / 1e6,
                                     "hessvec_fp32": 52 * n_nodes / t_h32 / 1e6}}

    cnn = None if args.no_learned else cnn_leg(ctx, L, torch, 10)

    rmtr = None
    if not args.no_loadstep:
        import ctypes
        rmtr = {}
        legs = [("plain_fp64", 0, None), ("mixed_fp32", 1, None)]
        net = None
        if not args.no_learned:
            net, rmtr["training"] = learned_leg(ctx, wl, P, W, torch, args.train_seconds, args.learned_target)
            log("training", rmtr["training"])
            legs.append(("mixed_learned", 1, net))
        for name, prec, nn in legs:
            xs = torch.zeros_like(x)
            xs.view(-1, 4)[:, 3] = c0
            prm = P.default_params(precision=prec, **wl.solver)
            if nn is not None:
                nnv = nn.net()
                prm.use_learned = 1
                prm.nn = ctypes.pointer(nnv)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = ctx.solve_loadstep(xs, p, c0, prm)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rmtr[name] = {"s_per_loadstep": dt, "vcycles": st["vcycles"], "chi_rel": st["chi"] / st["chi0"],
                          "tr_accepted": st["tr_accepted"], "tr_rejected": st["tr_rejected"],
                          "nn_proposed": st["nn_proposed"], "nn_accepted": st["nn_accepted"],
                          "energy": st["energy"], "converged": st["code"] == 0}
            log(name, rmtr[name])

    cpu = None if args.no_cpu else cpu_baseline(wl, x_np, p.cpu().numpy(), v_np)

    out = {
        "metric": METRIC,
        "value": n_dofs / (ms_step / 1e3) / 1e9,
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: 3D Q1 {N}^3 cells, {wl.n_frac} penny fractures, "
                               f"{L} levels, p={wl.p} uniform", "n_cells": N, "n_dofs": n_dofs,
                   "step": "energy + gradient + Hv (FP64) on the finest level"},
        "kernels": per,
        "roofline": roof,
        "cnn": cnn,
        "rmtr": rmtr,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
