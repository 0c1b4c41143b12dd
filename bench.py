#!/usr/bin/env python
"""Benchmark of the RMTR hot path on one MI355X.

One step = energy, gradient and Hessian-vector product (FP64, matrix-free)
over the fine level of the workload, inputs resident in HBM.  `value` is the
fine-level dofs passed through that triple per second (GDoF/s).  The same run
reports each kernel's own rate, the mixed-precision (FP32) Hv, the roofline
of the dominant kernel (HIP events on the launch stream) on the 256^3
workload, whose working set is larger than the Infinity Cache, the RMTR load
step to 1e-8 (plain FP64, mixed precision, and mixed precision with the
learned proposal, whose harvesting and training are timed apart), and the
CPU oracle on a bounded sample at one core and at the host's cores.
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
PEAK_FP32 = 157.3     # TFLOP/s, MI355X FP32 vector
PEAK_HBM = 8000.0     # GB/s
KERNEL_SOURCES = ["paper_2007_12908_amd/csrc/elem_kernels.hip", "paper_2007_12908_amd/csrc/rmtr_device.h"]
ROOFLINE_WORKLOAD = "c3_3d_256"   # x alone (543 MB) is twice the 256 MB Infinity Cache
TRAFFIC_FILE = os.path.join(ROOT, "profiles", f"traffic_hessvec_{ROOFLINE_WORKLOAD}.json")

# Algorithmic work of the 3D element kernels, per fine node (bytes that must
# cross HBM once: x 32, p 8, v 32, and the output) and per element (flops of
# a sum-factorised evaluation: interpolation of the nodal fields to the 8
# Gauss points, the pointwise density terms, the adjoint back to the nodes).
# The flop figures are the hot-path scope estimates, not the executed
# instruction count (which includes recomputed subexpressions).
ALGO = {
    "energy": {"bytes_per_node": 40, "flops_per_element": 700, "peak": PEAK_FP64},
    "gradient": {"bytes_per_node": 72, "flops_per_element": 1300, "peak": PEAK_FP64},
    "hessvec": {"bytes_per_node": 104, "flops_per_element": 1800, "peak": PEAK_FP64},
    "hessvec_fp32": {"bytes_per_node": 52, "flops_per_element": 1800, "peak": PEAK_FP32},
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """Per-launch HBM bytes of the Hv kernel at the roofline workload from
    committed PMC counters, or None when the kernel sources changed since
    they were taken."""
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


_CPU = {}


def _cpu_init(shm_names, shapes, n_cells, mat_args):
    from multiprocessing import shared_memory
    import numpy as np
    from oracle import fem
    arrs = []
    for name, n in zip(shm_names, shapes):
        sh = shared_memory.SharedMemory(name=name)
        arrs.append((sh, np.ndarray((n,), dtype=np.float64, buffer=sh.buf)))
    _CPU["arrs"] = arrs
    _CPU["grid"] = fem.Grid(3, n_cells)
    _CPU["mat"] = fem.material_from_E_nu(*mat_args)


def _cpu_chunk(elems):
    """The oracle's energy, gradient and assembled Hessian times v over a
    chunk of elements (one process, one thread)."""
    from oracle import fem
    (_, x), (_, p), (_, v) = _CPU["arrs"]
    g, mat = _CPU["grid"], _CPU["mat"]
    fem.energy(g, x, p, mat, elems)
    fem.gradient(g, x, p, mat, None, elems)
    H = fem.hessian(g, x, p, mat, None, elems)
    H @ v
    return len(elems)


def cpu_baseline(wl, x_np, p_np, v_np, budget_s=12.0):
    """The oracle, as it is, timed on the host: energy, gradient and Hv over
    the first elements of the workload grid, in one process (one core) and in
    as many single-threaded processes as the host offers (at most 16), each
    over its own chunk of elements.  The 1-core sample is grown until it
    takes about budget_s; the parallel sample is that size times the process
    count."""
    import multiprocessing as mp
    from multiprocessing import shared_memory
    import numpy as np
    os.environ["OMP_NUM_THREADS"] = "1"
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    shms = []
    for a in (x_np, p_np, v_np):
        sh = shared_memory.SharedMemory(create=True, size=a.nbytes)
        np.ndarray(a.shape, dtype=np.float64, buffer=sh.buf)[:] = a
        shms.append(sh)
    try:
        args = ([sh.name for sh in shms], [a.size for a in (x_np, p_np, v_np)], wl.n_cells,
                (wl.E, wl.nu, wl.Gc, wl.ls, wl.k))
        ctxmp = mp.get_context("spawn")
        ne_max = wl.n_cells ** 3
        with ctxmp.Pool(cores, initializer=_cpu_init, initargs=args) as pool:
            pool.map(_cpu_chunk, [np.arange(64)] * cores)          # imports and warm-up
            ne = 1024
            while True:
                t0 = time.perf_counter()
                pool.apply(_cpu_chunk, (np.arange(ne),))
                t1 = time.perf_counter() - t0
                if t1 * 2 > budget_s or 2 * ne > ne_max // cores:
                    break
                ne *= 2
            chunk = ne
            work = [np.arange(i * chunk, (i + 1) * chunk) for i in range(cores)]
            t0 = time.perf_counter()
            pool.map(_cpu_chunk, work, chunksize=1)
            tp = time.perf_counter() - t0
    finally:
        for sh in shms:
            sh.close()
            sh.unlink()
    # one element per node in the large-grid limit: 4 dofs per element
    one = 4 * ne / t1 / 1e9
    par = 4 * chunk * cores / tp / 1e9
    return {"value": par, "unit": "GDoF/s", "cores": cores, "kind": "oracle",
            "value_1core": one,
            "sample": f"energy + gradient + assembled-Hessian Hv (numpy/scipy FP64, one thread per process) over "
                      f"the first {chunk * cores} elements of the {wl.n_cells}^3 grid in {cores} processes of "
                      f"{chunk} elements ({tp:.1f} s); one process over {ne} elements: {t1:.1f} s; "
                      f"4 dofs per element"}


def kernel_leg(ctx, wl, c0, p, reps, torch):
    """Energy, gradient and Hv (FP64 and FP32) on the finest level of a
    workload, each timed with HIP events over `reps` launches on the launch
    stream, with its algorithmic HBM rate and arithmetic rate."""
    import numpy as np
    N, L = wl.n_cells, wl.n_levels
    n_nodes = (N + 1) ** 3
    n_dofs = 4 * n_nodes
    ne = N ** 3
    gen = torch.Generator(device="cuda").manual_seed(1234)
    x = torch.empty(n_dofs, dtype=torch.float64, device="cuda").normal_(0.0, 1e-4, generator=gen)
    xv = x.view(-1, 4)
    xv[:, 3] = c0
    idx = torch.arange(n_nodes, device="cuda")
    i, j, k = idx % (N + 1), (idx // (N + 1)) % (N + 1), idx // ((N + 1) ** 2)
    bnd = (i == 0) | (i == N) | (j == 0) | (j == N) | (k == 0) | (k == N)
    xv[bnd, :3] = 0.0
    v = torch.empty(n_dofs, dtype=torch.float64, device="cuda").normal_(generator=gen)
    x32, p32, v32 = x.float(), p.float(), v.float()
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    g, hv, hv32 = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x32)
    calls = {
        "energy": lambda: ctx.energy(L, x, p, out=E),
        "gradient": lambda: ctx.gradient(L, x, p, out=g),
        "hessvec": lambda: ctx.hessvec(L, x, p, v, out=hv),
        "hessvec_fp32": lambda: ctx.hessvec(L, x32, p32, v32, out=hv32),
    }
    out = {}
    for name, fn in calls.items():
        for _ in range(5):     # warm-up: clocks and caches settle
            fn()
        ms = time_calls(fn, reps, torch)
        a = ALGO[name]
        gbs = a["bytes_per_node"] * n_nodes / ms / 1e6
        tfs = a["flops_per_element"] * ne / ms / 1e9
        out[name] = {"ms": ms, "GDoF/s": n_dofs / ms / 1e6, "GB/s": gbs, "hbm_frac": gbs / PEAK_HBM,
                     "TFLOP/s": tfs, "alu_frac": tfs / a["peak"],
                     "bound": "alu" if a["flops_per_element"] / a["bytes_per_node"] > a["peak"] * 1e3 / PEAK_HBM
                     else "hbm"}
    del x, v, x32, p32, v32, g, hv, hv32
    return out


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


def loadstep_legs(ctx, wl, x_shape_like, p, c0, P, torch, net):
    """Plain FP64, mixed FP32 and (with a network) mixed + learned load steps
    from u = 0, c = c0, each timed from the call to its return."""
    import ctypes
    legs = [("plain_fp64", 0, None), ("mixed_fp32", 1, None)]
    if net is not None:
        legs.append(("mixed_learned", 1, net))
    out = {}
    for name, prec, nn in legs:
        xs = torch.zeros_like(x_shape_like)
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
        out[name] = {"s_per_loadstep": dt, "vcycles": st["vcycles"], "chi_rel": st["chi"] / st["chi0"],
                     "tr_accepted": st["tr_accepted"], "tr_rejected": st["tr_rejected"],
                     "nn_proposed": st["nn_proposed"], "nn_accepted": st["nn_accepted"],
                     "energy": st["energy"], "converged": st["code"] == 0}
        log(name, out[name])
        del xs
    return out


def learned_c5_leg(args, P, W, torch):
    """The learned form as configured for the 256^3 deployment: harvest and
    train on 128^3 runs with 10-50 fractures, deploy on the 256^3 network of
    100 fractures (its solver setting), against plain FP64 and mixed FP32."""
    from paper_2007_12908_amd import learned
    wt = W.WORKLOADS["c2_3d_128"]
    tctx = P.Context(3, wt.n_cells, wt.n_levels, wt.lam, wt.mu, wt.Gc, wt.ls, wt.k)
    net, info = learned_leg(tctx, wt, P, W, torch, args.train_seconds, args.learned_target)
    log("training", info)
    wl = W.WORKLOADS["c3_3d_256"]
    learned.rescale_for_grid(net, wt.h, wl.h, 3)
    ctx = P.Context(3, wl.n_cells, wl.n_levels, wl.lam, wl.mu, wl.Gc, wl.ls, wl.k)
    c0, p = ctx.init_fields(wl.n_levels, wl.fractures(), band=wl.h, p_mode=0, p_value=wl.p)
    x = torch.zeros(4 * (wl.n_cells + 1) ** 3, dtype=torch.float64, device="cuda")
    runs = loadstep_legs(ctx, wl, x, p, c0, P, torch, net)
    return {"train_workload": wt.name, "deploy_workload": wl.name, "training": info, **runs}


def ramp_leg(args, P, W, torch):
    """Load-step sequence on the 256^3 network: p ramped linearly from p to
    2p over `--ramp` steps, each step starting from the previous solution
    with c_lower <- c (irreversibility), in the precision of
    `--ramp-precision`."""
    wl = W.WORKLOADS["c3_3d_256"]
    ctx = P.Context(3, wl.n_cells, wl.n_levels, wl.lam, wl.mu, wl.Gc, wl.ls, wl.k)
    c0, p0 = ctx.init_fields(wl.n_levels, wl.fractures(), band=wl.h, p_mode=0, p_value=wl.p)
    x = torch.zeros(4 * (wl.n_cells + 1) ** 3, dtype=torch.float64, device="cuda")
    x.view(-1, 4)[:, 3] = c0
    cl = c0.clone()
    steps = []
    n = args.ramp
    for t in range(n):
        f = 1.0 + t / max(n - 1, 1)
        p = p0 * f
        prm = P.default_params(precision=args.ramp_precision, **wl.solver)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.solve_loadstep(x, p, cl, prm)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cl = x.view(-1, 4)[:, 3].clone()
        rec = {"p": wl.p * f, "s": dt, "vcycles": st["vcycles"], "chi_rel": st["chi"] / st["chi0"],
               "energy": st["energy"], "converged": st["code"] == 0, "c_sum": float(cl.sum())}
        log("load step", t + 1, rec)
        steps.append(rec)
    return {"workload": wl.name, "precision": "fp32" if args.ramp_precision else "fp64", "steps": steps,
            "total_s": sum(r["s"] for r in steps)}


def loadstep_leg(args, P, W, torch):
    """One load step of any workload (2D or 3D) from u = 0, c = c0, with the
    strain split of `--split` (the workloads' model is 1), the precision of
    `--ramp-precision` and solver settings from `--solver` (JSON; default:
    the workload's own)."""
    wl = W.WORKLOADS[args.loadstep]
    N, L, d = wl.n_cells, wl.n_levels, wl.dim
    ctx = P.Context(d, N, L, wl.lam, wl.mu, wl.Gc, wl.ls, wl.k, split=args.split)
    if wl.extra.get("p_lo") is not None:
        c0, p = ctx.init_fields(L, wl.fractures(), band=wl.h, p_mode=1, p_band=4.0 * wl.ls)
    else:
        c0, p = ctx.init_fields(L, wl.fractures(), band=wl.h, p_mode=0, p_value=wl.p)
    x = torch.zeros((d + 1) * (N + 1) ** d, dtype=torch.float64, device="cuda")
    x.view(-1, d + 1)[:, d] = c0
    settings = dict(wl.solver) if args.solver is None else json.loads(args.solver)
    prm = P.default_params(precision=args.ramp_precision, max_vcycles=args.max_vcycles, **settings)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ctx.solve_loadstep(x, p, c0, prm)
    torch.cuda.synchronize()
    return {"workload": wl.name, "split": args.split, "precision": args.ramp_precision, "settings": settings,
            "s": time.perf_counter() - t0, "vcycles": st["vcycles"], "chi_rel": st["chi"] / st["chi0"],
            "tr_accepted": st["tr_accepted"], "tr_rejected": st["tr_rejected"], "delta": st["delta"],
            "converged": st["code"] == 0}


def roofline_of(kernels, wl, traffic):
    """Roofline of the dominant (slowest) FP64 kernel of a kernel leg."""
    dom = max(("energy", "gradient", "hessvec"), key=lambda k: kernels[k]["ms"])
    k = kernels[dom]
    a = ALGO[dom]
    alu = k["bound"] == "alu"
    # the FP64 gradient and Hv on a 3D level are two launches: the element
    # kernel on non-overlapping tiles, then the sums of the tile-border nodes;
    # the time is that of both
    launches = {"energy": ["k_energy_q3", "k_reduce_partials"], "gradient": ["k_elem_q3<0>", "k_ring_sum"],
                "hessvec": ["k_elem_q3<1>", "k_ring_sum"]}[dom]
    return {"kernel": dom, "launches": launches, "workload": wl.name, "bound": k["bound"],
            "achieved": k["TFLOP/s"] if alu else k["GB/s"], "peak": a["peak"] if alu else PEAK_HBM,
            "unit": "TFLOP/s" if alu else "GB/s", "frac": k["alu_frac"] if alu else k["hbm_frac"],
            "traffic": traffic if dom == "hessvec" else None,
            "flops_per_element": a["flops_per_element"], "elements": wl.n_cells ** 3,
            "bytes_per_node": a["bytes_per_node"], "nodes": (wl.n_cells + 1) ** 3,
            "hbm_frac": k["hbm_frac"], "ms": k["ms"]}


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
    ap.add_argument("--no-roofline-leg", action="store_true",
                    help="skip the kernel leg on the roofline workload")
    ap.add_argument("--kernels-only", action="store_true",
                    help="time only the kernel triple (for profiler runs)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="time only the kernels on the roofline workload (for profiler runs)")
    ap.add_argument("--cnn-only", action="store_true",
                    help="time only the network's forward and backward passes (for profiler runs)")
    ap.add_argument("--split", type=int, default=1, choices=(0, 1, 2),
                    help="strain split of --roofline-only and --loadstep: 0 unsplit (the paper's energy), "
                         "1 volumetric-deviatoric (the workloads' model), 2 spectral")
    ap.add_argument("--learned-c5", action="store_true",
                    help="train on 128^3 runs, deploy on the 256^3 network: plain, mixed and mixed + learned "
                         "load steps (several minutes; not part of the default run)")
    ap.add_argument("--ramp", type=int, default=0,
                    help="run this many load steps on the 256^3 network with p ramped from p to 2p "
                         "(several minutes; not part of the default run)")
    ap.add_argument("--ramp-precision", type=int, default=1, choices=(0, 1),
                    help="precision of --ramp and --loadstep: 0 FP64, 1 mixed")
    ap.add_argument("--loadstep", default=None, help="run one load step of this workload (any split) and exit")
    ap.add_argument("--max-vcycles", type=int, default=200)
    ap.add_argument("--solver", default=None, help="solver settings of --loadstep as JSON (default: the workload's)")
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

    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float64, device="cuda")   # 2 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def roofline_leg():
        rw = W.WORKLOADS[ROOFLINE_WORKLOAD]
        rctx = P.Context(3, rw.n_cells, rw.n_levels, rw.lam, rw.mu, rw.Gc, rw.ls, rw.k,
                         split=args.split if args.roofline_only else 1)
        rc0, rp = rctx.init_fields(rw.n_levels, rw.fractures(), band=rw.h, p_mode=0, p_value=rw.p)
        ker = kernel_leg(rctx, rw, rc0, rp, max(args.steps // 2, 5), torch)
        del rctx, rc0, rp
        torch.cuda.synchronize()
        return rw, ker

    if args.roofline_only:
        rw, ker = roofline_leg()
        log(json.dumps({"workload": rw.name, "split": args.split, "kernels": ker}))
        return

    if args.ramp:
        print(json.dumps({"ramp": ramp_leg(args, P, W, torch)}), flush=True)
        return

    if args.loadstep:
        print(json.dumps({"loadstep": loadstep_leg(args, P, W, torch)}), flush=True)
        return

    if args.learned_c5:
        print(json.dumps({"learned_c5": learned_c5_leg(args, P, W, torch)}), flush=True)
        return

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
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty_like(x)
    hv = torch.empty_like(x)

    if args.cnn_only:
        log(json.dumps({"cnn": cnn_leg(ctx, L, torch, max(args.steps, 5))}))
        return

    def step():
        ctx.energy(L, x, p, out=E)
        ctx.gradient(L, x, p, out=g)
        ctx.hessvec(L, x, p, v, out=hv)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) / args.steps * 1e3

    per = kernel_leg(ctx, wl, c0, p, max(args.steps, 5), torch)
    if args.kernels_only:
        log(json.dumps({"ms": {k: v_["ms"] for k, v_ in per.items()}}))
        return

    # the roofline is taken where the working set does not fit the
    # Infinity Cache (the benchmark workload's x does)
    if args.no_roofline_leg:
        rw, rker = wl, per
    else:
        rw, rker = roofline_leg()
    roof = roofline_of(rker, rw, measured_traffic() if rw.name == ROOFLINE_WORKLOAD else None)
    log("roofline", json.dumps(roof))

    cnn = None if args.no_learned else cnn_leg(ctx, L, torch, 10)

    rmtr = None
    if not args.no_loadstep:
        rmtr = {}
        net = None
        if not args.no_learned:
            net, rmtr["training"] = learned_leg(ctx, wl, P, W, torch, args.train_seconds, args.learned_target)
            log("training", rmtr["training"])
        rmtr.update(loadstep_legs(ctx, wl, x, p, c0, P, torch, net))

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
                   "step": "energy + gradient + Hv (FP64) on the finest level",
                   "roofline_workload": f"{rw.name}: 3D Q1 {rw.n_cells}^3 cells, {rw.n_frac} penny fractures"},
        "kernels": per,
        "kernels_roofline_workload": rker,
        "roofline": roof,
        "cnn": cnn,
        "rmtr": rmtr,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
