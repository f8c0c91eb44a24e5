#!/usr/bin/env python
"""Throughput of one mODIL iteration on one MI355X.

A step is one full iteration of the method on one batch of synthetic input:
multigrid prolongation of every level, residuals / data terms and the FP64
loss, the exact adjoint, restriction to every level and Adam on every level.

    python bench.py [--steps K] [--warmup W] [--workload ns3d128] [--optimizer adam|lbfgs]

Prints one JSON line: fine-grid cell-iterations per second (fine cells x
steps / seconds, inputs resident in HBM), the per-kernel-class durations from
HIP events recorded on the library's stream during the timed steps, the
roofline of the dominant kernel (algorithmic bytes / its average launch
duration against 8 TB/s), and the CPU oracle timed on a bounded sample.
With --optimizer lbfgs a step is one L-BFGS iteration instead (direction from
the stored pairs, line search with one or more loss-and-gradient
evaluations, new pair); the CPU baseline is not run in that mode.
"""
import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
CLASSES = ("fine", "horner", "restrict", "adam", "reduce", "lbfgs_dots", "lbfgs_update")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="ns3d128")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="budget of the oracle CPU-baseline sample (0 disables it)")
    ap.add_argument("--copy-probe-mib", type=int, default=1024,
                    help="size of the plain device copy timed as the measured HBM peak "
                         "(and used to scale the traffic counters); 0 skips it")
    ap.add_argument("--optimizer", choices=("adam", "lbfgs", "autograd"), default="adam",
                    help="adam: the library's fused iteration; lbfgs: L-BFGS on the device; autograd: "
                         "the loss as a torch.autograd.Function (adjoint kernels in backward) with "
                         "torch.optim.Adam")
    ap.add_argument("--loop", choices=("run", "step"), default="run",
                    help="Adam iterations through modil_run (all K in one call) or one modil_step per call")
    ap.add_argument("--history", type=int, default=50, help="L-BFGS pairs")
    return ap.parse_args()


MEAS_BYTES = 12  # one measurement: int32 cell index and its value in double


def alg_bytes(ctx, spec, fused, adam=True, tiled=False, n_meas=0):
    """Algorithmic bytes of one launch of each kernel class and of one iteration.

    One iteration reads and writes every parameter of every level, and Adam's
    two moments of it, once: 6 * b * S, plus the measurements it must read
    (cell index and value, B_data).  Intermediates (the prolonged coarse
    levels w_l, the gradients g_l), halo re-reads and caching are not counted:
    they are the implementation's traffic, which rocprofv3 counters measure.

    Fused channel-flow path: the finest-level kernel owns the finest level's
    share, 6 * b * F * N + B_data (theta, m, v of level 0 read and written and
    the measurements; plus the fixed body fraction when chi is given); the
    restriction class owns the coarse levels' 6 * b * F * S_l (it applies Adam
    to them) and the Horner class none.  The iteration's figure is
    6 * b * S + B_data.  Generic path (no Adam in the fine kernel): the fine
    kernel reads the prolonged field and writes the finest gradient; Adam is
    one sweep, or (2-D tiled engine) Adam of level 0 sits in the fine kernel
    and that of the coarse levels in the restriction, as in the fused path.
    """
    b = 4 if spec.dtype == "f32" else 8
    lay = ctx.lay
    L = spec.n_levels
    size = [int(lay.level_stride[l]) * spec.batch for l in range(L)]
    S = int(lay.total)
    chi = spec.batch * spec.fine_cells * b if spec.chi_fixed else 0
    data = MEAS_BYTES * n_meas
    if fused and not adam:  # loss and gradient only (L-BFGS evaluations)
        fine = 2 * size[0] * b + chi + data
        horner = sum(size[l + 1] * b for l in range(L - 1))
        restrict = sum(size[l + 1] * b for l in range(L - 1))
        adam = 0
    elif fused:
        fine = 6 * size[0] * b + chi + data
        horner = 0
        restrict = sum(6 * size[l + 1] * b for l in range(L - 1))
        adam = 0
    elif tiled and adam:
        fine = 8 * size[0] * b + chi
        horner = sum((2 * size[l] + size[l + 1]) * b for l in range(L - 1))
        restrict = sum((size[l] + 7 * size[l + 1]) * b for l in range(L - 1))
        adam = 0
    else:
        fine = 2 * size[0] * b + chi
        horner = sum((2 * size[l] + size[l + 1]) * b for l in range(L - 1))
        restrict = sum((size[l] + size[l + 1]) * b for l in range(L - 1))
        adam = 7 * S * b if adam else 0
    return {"fine": fine, "horner": horner, "restrict": restrict, "adam": adam,
            "reduce": 0, "lbfgs_dots": 0, "lbfgs_update": 0, "iteration": 6 * S * b + data}


def lbfgs_vector_bytes(n, b, infos, pairs0):
    """Algorithmic bytes of the L-BFGS vector kernels over the timed iterations.

    Per iteration with k stored pairs: the direction reads 2k + 1 vectors and
    writes d; every line-search evaluation forms the trial point (2 reads,
    1 write) and the dot product g . d (2 reads); the new pair reads d, g_new,
    g and writes s, y; the accepted point is copied (1 read, 1 write); the dot
    products with the new gradient and the new y read 2k + 3 + 2 vectors.
    """
    dots = update = 0
    k = pairs0
    for info in infos:
        ev = info["evals"]
        update += (2 * k + 2 + 3 * ev + 5 + 2) * n * b
        dots += (2 * ev + 2 * k + 5) * n * b
        k = info["pairs"]
    return dots, update


def measured_traffic(workload, kernel_class):
    """HBM bytes per launch from the committed counter summary, or None.

    profiles/traffic_<workload>.json holds FETCH_SIZE and WRITE_SIZE of the
    dominant kernel, scaled by what the same counters read for a plain device
    copy of known size, together with the SHA-256 of that kernel's source
    files (listed in the record) at the time; a changed source makes the
    figure stale (None).
    """
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_class") != kernel_class or not rec.get("sources"):
        return None
    h = hashlib.sha256()
    csrc = os.path.join(here, "paper_2303_04679_amd", "csrc")
    for name in rec["sources"]:
        f = os.path.join(csrc, name)
        if not os.path.exists(f):
            return None
        h.update(open(f, "rb").read())
    if h.hexdigest() != rec.get("source_sha256"):
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_baseline(workload, theta_levels, seconds):
    """The FP64 oracle (loss, autodiff gradient, Adam) on the same workload,
    on one host core: the process is pinned to the first core of its affinity
    set and torch to one thread for the duration (both restored after)."""
    import torch
    from oracle import adam as oadam
    from oracle import operators as ops
    affinity = sorted(os.sched_getaffinity(0))
    threads = torch.get_num_threads()
    os.sched_setaffinity(0, {affinity[0]})
    torch.set_num_threads(1)
    try:
        return _oracle_baseline(workload, theta_levels, seconds, ops, oadam, affinity)
    finally:
        torch.set_num_threads(threads)
        os.sched_setaffinity(0, affinity)


def _oracle_baseline(workload, theta_levels, seconds, ops, oadam, affinity):
    import torch
    spec = workload.spec
    op = "ns3d_fixed" if spec.chi_fixed else spec.op
    ospec = ops.Spec(op, spec.dims, spec.lengths, spec.n_levels,
                     params={"re": spec.re, "diam": spec.diam, "lam": spec.lam,
                             "chi_shift": spec.chi_shift, "tau_coef": spec.tau_coef,
                             "u_ref": spec.u_ref},
                     weights={"pde": spec.w_pde, "reg": spec.w_reg, "bc": spec.w_bc},
                     meas=[(f, t, idx, vals, w) for inst, f, t, idx, vals, w in workload.meas if inst == 0],
                     chi=workload.chi if spec.chi_fixed else None, centering=spec.centering)
    state = [[(x, x * 0.0, x * 0.0) for x in row] for row in theta_levels]
    t0 = time.perf_counter()
    it = 0
    while True:
        cur = [[s[0] for s in row] for row in state]
        _, grads = ops.loss_and_grad(ospec, cur)
        it += 1
        state = [[oadam.adam_step(s[0], s[1], s[2], g, workload.lr, 0.9, 0.999, 1e-8, it)
                  for s, g in zip(row, grow)] for row, grow in zip(state, grads)]
        el = time.perf_counter() - t0
        if el >= seconds or it >= 50:
            break
    return {"value": spec.fine_cells * spec.batch * it / el, "unit": "cell-iter/s",
            "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{it} full iterations (loss, autodiff gradient, Adam) of {workload.name} "
                      f"in FP64 on one host core, {el:.1f} s",
            "nproc": os.cpu_count(), "affinity_cpus": len(affinity), "cpu_model": cpu_model()}


def copy_probe(device, mib, reps=5):
    """A plain device-to-device copy of `mib` MiB timed with HIP events: the
    HBM bandwidth a streaming kernel reaches on this GPU (read + write bytes
    per second), the measured counterpart of the vendor peak."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=device)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"bytes": 2 * n * 4, "avg_ms": ms, "gbs": 2 * n * 4 / (ms * 1e-3) / 1e9}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the mODIL iteration runs on one GPU only; "
              "multi-GPU domain decomposition is not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2303_04679_amd import configs
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    wl = configs.WORKLOADS[args.workload]()
    spec = wl.spec
    print(f"[bench] workload {wl.name} dims {tuple(spec.dims)} L={spec.n_levels} {spec.dtype}",
          file=sys.stderr, flush=True)
    ctx, theta = configs.build(wl)
    if args.optimizer == "lbfgs":
        return main_lbfgs(args, wl, ctx, theta)
    if args.optimizer == "autograd":
        return main_autograd(args, wl, ctx, theta)
    a, b = theta, ctx.new_pack()
    m, v = ctx.new_pack(), ctx.new_pack()
    terms = torch.empty((spec.batch, 5), dtype=torch.float64, device=ctx.device)
    step = 0

    def run(n):
        nonlocal a, b, step
        if args.loop == "run":  # n iterations in one library call
            out = ctx.run(a, b, m, v, step + 1, n, lr=wl.lr, terms=terms)
            if out is b:
                a, b = b, a
            step += n
            return
        for _ in range(n):  # one library call per iteration
            step += 1
            ctx.step(a, b, m, v, step, lr=wl.lr, terms=terms)
            a, b = b, a

    run(args.warmup)
    torch.cuda.synchronize()
    ctx.check()
    # plain timed region
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    run(args.steps)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ctx.check()
    print(f"[bench] {args.steps} steps in {ms:.3f} ms", file=sys.stderr, flush=True)
    # per-kernel-class durations (HIP events on the library stream)
    ctx.profile(True)
    for k in range(len(CLASSES)):
        ctx.profile_read(k)
    e0.record(ctx.stream)
    run(args.steps)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    ms_prof = e0.elapsed_time(e1)
    kern = {}
    for k, name in enumerate(CLASSES):
        tot, cnt = ctx.profile_read(k)
        kern[name] = {"total_ms": tot, "launches": cnt, "avg_ms": tot / max(cnt, 1)}
    ctx.profile(False)
    fused = ctx.fused_active()
    n_meas = sum(len(m[3]) for m in wl.meas)
    ab = alg_bytes(ctx, spec, fused, tiled=ctx.tiled_active(), n_meas=n_meas)
    dom = max(CLASSES, key=lambda n: kern[n]["total_ms"])
    avg_s = kern[dom]["avg_ms"] * 1e-3
    achieved = ab[dom] / avg_s / 1e9 if avg_s > 0 else 0.0
    ms_step = ms / args.steps
    value = spec.fine_cells * spec.batch * args.steps / (ms * 1e-3)
    it_gbs = ab["iteration"] / (ms_step * 1e-3) / 1e9
    copy = copy_probe(ctx.device, args.copy_probe_mib) if args.copy_probe_mib else None
    cpu = None
    if args.cpu_seconds > 0:
        print("[bench] oracle CPU baseline ...", file=sys.stderr, flush=True)
        lv = [[x.detach().cpu().double().numpy() for x in row] for row in ctx.level_views(theta, 0)]
        cpu = oracle_baseline(wl, lv, args.cpu_seconds)
    out = {
        "metric": "fine-grid cell-iters/s",
        "value": value,
        "unit": "cell-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": spec.dtype,
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": "x".join(str(d) for d in spec.dims),
                   "levels": spec.n_levels, "fields": len(spec.fields), "params": int(ctx.lay.total),
                   "batch": spec.batch, "optimizer": "adam", "loss_reduction": "f64",
                   "loop": "modil_run" if args.loop == "run" else "modil_step"},
        "iteration_bytes_algorithmic": ab["iteration"],
        "hbm_gbs_algorithmic": it_gbs,
        "iteration_roofline_frac": it_gbs / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "bytes_per_launch": ab[dom], "avg_launch_ms": kern[dom]["avg_ms"],
                     "traffic": measured_traffic(wl.name, dom)},
        "hbm_copy_probe": None if copy is None else dict(copy, frac_of_peak=copy["gbs"] / HBM_PEAK_GBS),
        "kernels": kern,
        "fused_fine_kernel": fused,
        "ms_per_step_profiled": ms_prof / args.steps,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main_lbfgs(args, wl, ctx, theta):
    """One step = one L-BFGS iteration (see lbfgs_vector_bytes for its vector work)."""
    import torch

    from paper_2303_04679_amd.modil import LBFGS
    spec = wl.spec
    lb = LBFGS(ctx, history=args.history)
    th = theta.clone()
    for _ in range(args.warmup):
        lb.step(th)
    torch.cuda.synchronize()
    pairs0 = lb.step(th)["pairs"]
    ctx.profile(True)
    for k in range(len(CLASSES)):
        ctx.profile_read(k)
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(lb.step(th))
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    kern = {}
    for k, name in enumerate(CLASSES):
        tot, cnt = ctx.profile_read(k)
        kern[name] = {"total_ms": tot, "launches": cnt, "avg_ms": tot / max(cnt, 1)}
    ctx.profile(False)
    ctx.check()
    b = 4 if spec.dtype == "f32" else 8
    fused = ctx.fused_active()
    ab = alg_bytes(ctx, spec, fused, adam=False)
    evals = sum(i["evals"] for i in infos)
    dots, upd = lbfgs_vector_bytes(int(ctx.lay.total), b, infos, pairs0)
    total_bytes = {n: ab[n] * kern[n]["launches"] for n in ("fine", "horner", "restrict", "reduce")}
    total_bytes.update({"adam": 0, "lbfgs_dots": dots, "lbfgs_update": upd})
    dom = max(CLASSES, key=lambda n: kern[n]["total_ms"])
    launches = max(kern[dom]["launches"], 1)
    achieved = total_bytes[dom] / (kern[dom]["total_ms"] * 1e-3) / 1e9 if kern[dom]["total_ms"] else 0.0
    ms_it = secs * 1e3 / args.steps
    out = {
        "metric": "fine-grid cell-iters/s",
        "value": spec.fine_cells * spec.batch * args.steps / secs,
        "unit": "cell-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_it,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": spec.dtype,
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": "x".join(str(d) for d in spec.dims),
                   "levels": spec.n_levels, "fields": len(spec.fields), "params": int(ctx.lay.total),
                   "batch": spec.batch, "optimizer": f"lbfgs(m={args.history})", "loss_reduction": "f64"},
        "evaluations_per_step": evals / args.steps,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "bytes_per_launch": total_bytes[dom] / launches,
                     "avg_launch_ms": kern[dom]["avg_ms"], "traffic": None},
        "kernels": kern,
        "fused_fine_kernel": fused,
        "final_loss": infos[-1]["loss"],
        "cpu_baseline": None,
    }
    lb.close()
    print(json.dumps(out), flush=True)


def main_autograd(args, wl, ctx, theta):
    """One step = loss forward (loss kernels), backward (the adjoint kernels,
    prolonged field recomputed) and torch.optim.Adam over the pack: the
    unfused differentiation pattern, timed apart from the fused iteration."""
    import torch

    from paper_2303_04679_amd.autograd import modil_loss
    spec = wl.spec
    th = torch.nn.Parameter(theta.clone())
    opt = torch.optim.Adam([th], lr=wl.lr)

    def run(n):
        for _ in range(n):
            opt.zero_grad(set_to_none=False)
            loss = modil_loss(th, ctx)
            loss.backward()
            opt.step()
        return loss

    run(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    loss = run(args.steps)
    e1.record()
    torch.cuda.synchronize()
    ctx.check()
    ms = e0.elapsed_time(e1)
    b = 4 if spec.dtype == "f32" else 8
    S = int(ctx.lay.total)
    out = {
        "metric": "fine-grid cell-iters/s",
        "value": spec.fine_cells * spec.batch * args.steps / (ms * 1e-3),
        "unit": "cell-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": spec.dtype,
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": "x".join(str(d) for d in spec.dims),
                   "levels": spec.n_levels, "fields": len(spec.fields), "params": S,
                   "batch": spec.batch, "optimizer": "autograd.Function + torch.optim.Adam",
                   "loss_reduction": "f64"},
        "unfused_bytes_per_step": 9 * b * S,
        "final_loss": float(loss),
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
