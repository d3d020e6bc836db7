"""DISC throughput on one MI355X: voxel-iterations/s of whole registrations.

A step is one full DISC registration of the 256 x 256 x 96 head-and-neck
phantom pair (patch 11^3, sigma 2, 3-level pyramid x 100 iterations):
set-up (global shift, pyramid, static patch moments) plus every iteration
and level switch, with the inputs already resident in HBM. The value counts
the voxel-iterations of all levels (sum_l N_l K_l) per second of step time.

Besides the JSON line on stdout, the run reports per-kernel HIP-event timing
of the same timed steps (roofline of the dominant kernel against the 8 TB/s
HBM peak) and the FP64 CPU oracle timed on a bounded sample of the same
workload (cpu_baseline). Progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per voxel of each kernel launch (reads + writes of
# its inputs and outputs once; gathers and halos counted once).
BYTES_PER_VOXEL = {
    "warp": 20.0,      # r 12 + CT 4 + m 4
    "correct": 12.0,   # m 4 + ys 4 + f 4
    "force_xy": 32.0,  # m 4 + f 4 + r 12 + xy-filtered r~ 12
    "smooth_z": 32.0,  # xy-filtered r~ 12 + r 12, and the next warp: CT 4 + m 4
    "upsample": 13.5,  # fine r 12 + coarse r 12/8, per fine voxel
}
ALGORITHMIC_MIN_BYTES = 32.0  # read CT, CBCT, r; write r (whole iteration)

WORKLOADS = {
    "hn256x256x96": dict(case="hn256x256x96"),
    "hn512x512x160": dict(case="hn512x512x160"),
    "ellipsoid48": dict(case="ellipsoid48"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel, workload):
    """HBM bytes per finest-level launch of `kernel` from the committed
    FETCH_SIZE / WRITE_SIZE summary, or None when there is none for this
    kernel and workload, or the kernel's sources have changed since the
    counters were taken (sha256 recorded with the summary)."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_b = re.search(r"^traffic_bytes_per_launch:\s*(\d+)", text, re.M)
    m_h = re.search(r"^traffic_source_sha256:\s*([0-9a-f]{64})", text, re.M)
    if not (m_b and m_h):
        return None
    h = hashlib.sha256()
    for rel in ("smooth.hip", "device.h"):
        with open(os.path.join(ROOT, "paper_1204_6295_amd", "csrc", rel), "rb") as fh:
            h.update(fh.read())
    return int(m_b.group(1)) if h.hexdigest() == m_h.group(1) else None


def _ms_per_call(fn, reps, warm=2):
    import torch

    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1000.0 / reps


def finest_level_rate(reg, ct, cb, cfg, reps=5):
    """Wall time of the finest level's iterations alone (the coarse levels
    and the set-up run first, untimed); median of reps runs."""
    import torch

    times = []
    for _ in range(reps):
        reg.set_volumes(ct, cb)
        if cfg["levels"] > 1:
            reg.iterate(sum(cfg["iters"][:-1]))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reg.iterate(cfg["iters"][-1])
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t = sorted(times)[len(times) // 2]
    n = float(cfg["shape"][0] * cfg["shape"][1] * cfg["shape"][2])
    return {"ms": round(t * 1000.0, 3), "iterations": cfg["iters"][-1],
            "voxel_iterations_per_s": round(n * cfg["iters"][-1] / t, 1),
            "ms_per_iteration": round(t * 1000.0 / cfg["iters"][-1], 4)}


def backward_rate(disc, ct, cb, r, cfg, plain_ms_per_it, reps=10):
    """Differentiable DISC at the workload size: SSD loss alone and loss +
    hand-written gradient (patch moments recomputed), against one plain
    finest-level iteration on the same GPU."""
    patch = cfg["patch"]
    ys = disc.static_stats(cb, patch)
    ms_loss = _ms_per_call(lambda: disc.ssd_loss(ct, ys, r, patch), reps)
    ms_grad = _ms_per_call(lambda: disc.ssd_grad(ct, ys, r, patch, want_loss=True), reps)
    n = float(ct.numel())
    return {"ms_loss": round(ms_loss, 4), "ms_loss_and_grad": round(ms_grad, 4),
            "voxels_per_s_loss_and_grad": round(n / (ms_grad * 1e-3), 1),
            "vs_plain_iteration": round(ms_grad / plain_ms_per_it, 3)}


def gd_vs_demons(disc, ct, cb, r_true, cfg, steps=200):
    """Differentiable DISC used as a registration: `steps` gradient-descent
    steps on the SSD loss, r <- r - eta G_sigma * dL/dr (the gradient smoothed
    by the same Gaussian that regularises the demons field), against `steps`
    demons iterations, both at the finest level from r = 0. eta is fixed from
    the first smoothed gradient so that the largest first update is half a
    voxel, the bound each demons force obeys. Reported: wall time of each loop
    and the loss and mean field error (vs the known deformation, inside the
    body) each reaches."""
    import torch

    patch, sigma = cfg["patch"], cfg["sigma"]
    s, _ = disc.shift(ct, cb)
    ys = disc.static_stats(s, patch)
    body = ct > -500

    def field_error(r):
        return ((r - r_true) ** 2).sum(0).sqrt()[body].mean().item()

    r = torch.zeros((3,) + tuple(ct.shape), dtype=torch.float32, device=ct.device)
    loss0 = disc.ssd_loss(ct, ys, r, patch).item()
    eta = 0.5 / disc.smooth(disc.ssd_grad(ct, ys, r, patch), sigma).abs().max()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = r - eta * disc.smooth(disc.ssd_grad(ct, ys, r, patch), sigma)
    torch.cuda.synchronize()
    ms_gd = (time.perf_counter() - t0) * 1000.0
    loss_gd = disc.ssd_loss(ct, ys, r, patch).item()
    err_gd = field_error(r)
    reg = disc.Registration(patch=patch, sigma=sigma, levels=1, iters=(steps,))
    reg.set_volumes(ct, cb)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reg.run()
    torch.cuda.synchronize()
    ms_dm = (time.perf_counter() - t0) * 1000.0
    rd = reg.field()
    loss_dm = disc.ssd_loss(ct, ys, rd, patch).item()
    err_dm = field_error(rd)
    reg.close()
    return {"steps": steps, "eta": float(eta),
            "loss_at_r0": loss0,
            "gradient_descent": {"ms": round(ms_gd, 3), "loss": loss_gd, "loss_ratio": round(loss_gd / loss0, 5),
                                 "mean_field_error_body_vox": round(err_gd, 4)},
            "demons": {"ms": round(ms_dm, 3), "loss": loss_dm, "loss_ratio": round(loss_dm / loss0, 5),
                       "mean_field_error_body_vox": round(err_dm, 4)},
            "mean_field_error_body_vox_at_r0": round(field_error(torch.zeros_like(r)), 4)}


def variant_rates(disc, ct, cb, cfg, plain_ms, reps=3):
    """The same registration with the method's variants on: both terms of
    Eq. 1, the Eq. 7-10 mask and fill, and the Sec. 2.3 stopping rule
    (iterations actually run per level reported), each against the plain
    path on the same GPU."""
    import torch

    base = dict(patch=cfg["patch"], sigma=cfg["sigma"], levels=cfg["levels"], iters=cfg["iters"])
    out = {}
    for name, kw in (("double_force", dict(force_mode=1)), ("mask_fill", dict(mask_mode=1)),
                     ("stopping_rule", dict(stop_eps=1e-4, stop_lag=10))):
        reg = disc.Registration(**base, **kw)

        def run():
            reg.set_volumes(ct, cb)
            reg.run()

        ms = _ms_per_call(run, reps=reps, warm=1)
        row = {"ms_per_registration": round(ms, 3), "vs_plain": round(ms / plain_ms, 3)}
        if name == "stopping_rule":
            row["iterations_run"] = [reg.stats(lv)[0] for lv in range(cfg["levels"])]
        out[name] = row
        reg.close()
        torch.cuda.synchronize()
    return out


def batched_rate(disc, n_pairs=16, iters=100):
    """Batched DISC: n uneven head-and-neck pairs (sizes drawn from
    128^2x64, 192^2x80, 256^2x96, 384^2x128), patch 11^3, sigma 2, one level,
    `iters` iterations: sequential single-volume registrations against one
    batch (eager launches, and the captured graph), tiles autotuned."""
    import torch

    from synth.phantom import make_batch

    cases = make_batch(n_pairs, device="cuda")
    cts = [torch.from_numpy(c.ct).cuda() for c in cases]
    cbs = [torch.from_numpy(c.cbct).cuda() for c in cases]
    shapes = [tuple(c.ct.shape) for c in cases]
    vox = float(sum(int(np.prod(s)) for s in shapes))
    kw = dict(patch=(11, 11, 11), sigma=2.0)
    regs = [disc.Registration(levels=1, iters=(iters,), **kw) for _ in cases]

    def seq():
        for reg, ct, cb in zip(regs, cts, cbs):
            reg.set_volumes(ct, cb)
            reg.run()

    ms_seq = _ms_per_call(seq, reps=1, warm=1)
    b = disc.Batch(shapes, iters=iters, **kw)
    tiles, ms_tune, _ = disc.autotune(b, cts, cbs, cache_path=None, iters=3)

    def run(graph):
        def f():
            b.set_volumes(cts, cbs)
            b.run(use_graph=graph)
        return f

    ms_eager = _ms_per_call(run(False), reps=1, warm=1)
    ms_graph = _ms_per_call(run(True), reps=2, warm=1)
    # batched result against the single-volume path, first pair (same
    # kernels and arithmetic; only launch knobs differ)
    fe = (b.field(0) - regs[0].field()).abs().max().item()
    if not fe <= 0.05:
        raise RuntimeError("batched pair 0 differs from the single-volume path by %.3g voxel" % fe)
    small = small_batch_rate(disc, iters=iters)
    return {"pairs": n_pairs, "shapes_zyx": [list(s) for s in shapes], "voxels": vox, "iterations": iters,
            "small_volumes": small,
            "ms_sequential": round(ms_seq, 3), "ms_batched_eager": round(ms_eager, 3),
            "ms_batched_graph": round(ms_graph, 3),
            "voxel_iterations_per_s_graph": round(vox * iters / (ms_graph * 1e-3), 1),
            "speedup_graph_vs_sequential": round(ms_seq / ms_graph, 3),
            "tiles": tiles, "autotune_ms_per_iteration": round(ms_tune, 4),
            "pair0_field_max_diff_vs_single": fe}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def small_batch_rate(disc, n_pairs=16, shape=(32, 64, 64), iters=100):
    """Where batching pays: n small pairs (131,072 voxels each, patch 11^3,
    sigma 2, one level), whose single-volume iterations are bound by launch
    latency, as sequential registrations against one batch (eager launches
    and the captured HIP graph)."""
    import torch

    from synth.phantom import make_hn_pair

    cases = [make_hn_pair(shape, pair=200 + i, device="cuda") for i in range(n_pairs)]
    cts = [torch.from_numpy(c.ct).cuda() for c in cases]
    cbs = [torch.from_numpy(c.cbct).cuda() for c in cases]
    kw = dict(patch=(11, 11, 11), sigma=2.0)
    regs = [disc.Registration(levels=1, iters=(iters,), **kw) for _ in cases]

    def seq():
        for reg, ct, cb in zip(regs, cts, cbs):
            reg.set_volumes(ct, cb)
            reg.run()

    ms_seq = _ms_per_call(seq, reps=2, warm=1)
    b = disc.Batch([shape] * n_pairs, iters=iters, **kw)

    def run(graph):
        def f():
            b.set_volumes(cts, cbs)
            b.run(use_graph=graph)
        return f

    ms_eager = _ms_per_call(run(False), reps=2, warm=1)
    ms_graph = _ms_per_call(run(True), reps=3, warm=1)
    fe = (b.field(0) - regs[0].field()).abs().max().item()
    if not fe <= 0.05:
        raise RuntimeError("small batch pair 0 differs from the single-volume path by %.3g voxel" % fe)
    vox = float(n_pairs * shape[0] * shape[1] * shape[2])
    return {"pairs": n_pairs, "shape_zyx": list(shape), "iterations": iters, "ms_sequential": round(ms_seq, 3),
            "ms_batched_eager": round(ms_eager, 3), "ms_batched_graph": round(ms_graph, 3),
            "voxel_iterations_per_s_graph": round(vox * iters / (ms_graph * 1e-3), 1),
            "speedup_graph_vs_sequential": round(ms_seq / ms_graph, 3),
            "speedup_graph_vs_eager": round(ms_eager / ms_graph, 3),
            "pair0_field_max_diff_vs_single": fe}


def cpu_baseline(case, params, budget_s=10.0, max_iters=10):
    """FP64 oracle on the finest level of the same pair, from r = 0: as many
    iterations as fit in about budget_s on all host threads, then one
    iteration on one thread. Static patch moments are computed beforehand and
    not timed (the GPU computes them once per registration)."""
    import numpy as np

    import oracle

    ct = case.ct.astype(np.float64)
    _, s = oracle.global_shift(ct, case.cbct.astype(np.float64))
    p = oracle.make_params(patch=params["patch"], sigma=params["sigma"], levels=1,
                           iters=(1,))
    mu_s, var_s = oracle.patch_moments(s, params["patch"])
    all_threads = oracle.threads()

    def timed(threads, limit):
        oracle.set_threads(threads)
        r = np.zeros((3,) + ct.shape)
        n = 0
        t0 = time.perf_counter()
        while True:
            r, _, _, _ = oracle.iterate(ct, s, r, p, n=1, mu_s=mu_s, var_s=var_s)
            n += 1
            el = time.perf_counter() - t0
            log("  oracle, %d thread(s), iteration %d: %.1f s" % (threads, n, el))
            if n >= limit or el * (n + 1) / n > budget_s:
                return n, el

    n, el = timed(all_threads, max_iters)
    n1, el1 = timed(1, 1)
    oracle.set_threads(all_threads)
    desc = "finest-level iteration(s) of the %dx%dx%d pair from r = 0, patch %s, sigma %g" % (
        ct.shape[2], ct.shape[1], ct.shape[0], "x".join(map(str, params["patch"])), params["sigma"])
    return {
        "value": float(ct.size) * n / el,
        "unit": "voxel-iterations/s",
        "cores": all_threads,
        "kind": "oracle",
        "sample": "%d %s on %d threads (%.1f s)" % (n, desc, all_threads, el),
        "one_thread": {"value": float(ct.size) * n1 / el1, "unit": "voxel-iterations/s", "cores": 1,
                       "sample": "%d %s on 1 thread (%.1f s)" % (n1, desc, el1)},
        "cpu_model": _cpu_model(),
        "host_threads_visible": os.cpu_count(),
    }


def workload_summary(disc, name, steps=3):
    """Another workload of the same registration: whole-registration time,
    the finest level alone (median of 5) and per-kernel averages at the
    finest level with their algorithmic GB/s."""
    import torch

    from synth.phantom import CONFIGS, make_case

    cfg = CONFIGS[name]
    case = make_case(name, device="cuda")
    ct = torch.from_numpy(case.ct).cuda()
    cb = torch.from_numpy(case.cbct).cuda()
    params = dict(patch=cfg["patch"], sigma=cfg["sigma"], levels=cfg["levels"], iters=cfg["iters"])
    reg = disc.Registration(**params)

    def step():
        reg.set_volumes(ct, cb)
        reg.run()

    ms = _ms_per_call(step, reps=steps, warm=1)
    fin = finest_level_rate(reg, ct, cb, cfg)
    reg.timing_enable(4 * sum(cfg["iters"]) + 16)
    step()
    torch.cuda.synchronize()
    kern = {}
    for kname in disc.KERNELS:
        n, kms, vox = reg.timing_read(kname, cfg["levels"] - 1)
        if n:
            kern[kname] = {"launches": n, "avg_us": round(1000.0 * kms / n, 2),
                           "gbs": round(BYTES_PER_VOXEL[kname] * vox / (kms * 1e-3) / 1e9, 1)}
    reg.timing_enable(0)
    reg.close()
    n_fin = float(np.prod(cfg["shape"]))
    return {
        "shape_zyx": list(cfg["shape"]), "patch": list(cfg["patch"]), "sigma": cfg["sigma"],
        "levels": cfg["levels"], "iters_per_level": list(cfg["iters"]),
        "ms_per_registration": round(ms, 3), "finest_level": fin,
        "finest_level_kernels": kern,
        "effective_hbm_frac_at_32B": round(ALGORITHMIC_MIN_BYTES * fin["voxel_iterations_per_s"]
                                           / (HBM_PEAK_GBS * 1e9), 4),
        "finest_voxels": n_fin,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="hn256x256x96", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the finest-level, differentiable and batched measurements")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel events in the timed steps")
    ap.add_argument("--dump-inputs", metavar="DIR",
                    help="write the workload's CT and CBCT as raw float32 files (for the native driver) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: DISC here runs on a single MI355X "
              "(no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("RANK", "0")) != 0:
        return

    import torch

    import paper_1204_6295_amd as disc
    from synth.phantom import CONFIGS, make_case

    dev = torch.device("cuda:0")
    cname = WORKLOADS[args.workload]["case"]
    cfg = CONFIGS[cname]
    log("generating %s phantom pair %s" % (args.workload, cfg["shape"]))
    case = make_case(cname, device="cuda")
    if args.dump_inputs:
        os.makedirs(args.dump_inputs, exist_ok=True)
        case.ct.tofile(os.path.join(args.dump_inputs, "ct.f32"))
        case.cbct.tofile(os.path.join(args.dump_inputs, "cbct.f32"))
        log("wrote %s/{ct,cbct}.f32, shape (nz, ny, nx) = %s" % (args.dump_inputs, cfg["shape"]))
        return
    ct = torch.from_numpy(case.ct).to(dev)
    cb = torch.from_numpy(case.cbct).to(dev)
    params = dict(patch=cfg["patch"], sigma=cfg["sigma"], levels=cfg["levels"], iters=cfg["iters"])
    reg = disc.Registration(**params)

    def step():
        reg.set_volumes(ct, cb)
        reg.run()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warmup done")

    # timed steps: no instrumentation, the value is the plain throughput
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1000.0 / args.steps
    log("timed %d steps: %.3f ms/step" % (args.steps, ms_per_step))

    # the same steps again with a HIP event pair around every kernel launch,
    # recorded on the launch stream: per-kernel averages for the roofline
    launches_per_step = 4 * sum(cfg["iters"]) + (cfg["levels"] - 1)
    if not args.no_timing:
        reg.timing_enable(launches_per_step * args.steps + 16)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()

    # voxel-iterations per step over all levels
    dims = [tuple(cfg["shape"])]
    for _ in range(cfg["levels"] - 1):
        nz, ny, nx = dims[0]
        dims.insert(0, ((nz + 1) // 2, (ny + 1) // 2, (nx + 1) // 2))
    vox_it = sum(float(d[0] * d[1] * d[2]) * k for d, k in zip(dims, cfg["iters"]))
    value = vox_it * args.steps / wall

    roofline = None
    kernels = {}
    if not args.no_timing:
        for name in disc.KERNELS:
            n, ms, vox = reg.timing_read(name)
            if n:
                kernels[name] = dict(launches=n, total_ms=ms, avg_us=1000.0 * ms / n,
                                     gbs=BYTES_PER_VOXEL[name] * vox / (ms * 1e-3) / 1e9)
        # dominant kernel by total time; its roofline per finest-level launch
        dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
        n, ms, vox = reg.timing_read(dom, cfg["levels"] - 1)
        avg_s = ms / n * 1e-3
        achieved = BYTES_PER_VOXEL[dom] * (vox / n) / avg_s / 1e9
        traffic = measured_traffic(dom, args.workload)
        # the whole finest-level iteration (every kernel of one iteration)
        it_us = 0.0
        for name in ("correct", "force_xy", "smooth_z"):
            nk, msk, _ = reg.timing_read(name, cfg["levels"] - 1)
            it_us += 1000.0 * msk / nk if nk else 0.0
        design_b = BYTES_PER_VOXEL["correct"] + BYTES_PER_VOXEL["force_xy"] + BYTES_PER_VOXEL["smooth_z"]
        roofline = {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_gbs": round(traffic / avg_s / 1e9, 1) if traffic else None,
            "kernel": dom, "level": "finest", "avg_launch_us": round(avg_s * 1e6, 2), "launches": n,
            "bytes_per_voxel": BYTES_PER_VOXEL[dom], "voxels_per_launch": vox / n,
            "iteration": {
                "us": round(it_us, 2), "design_bytes_per_voxel": design_b,
                "design_frac": round(design_b * (vox / n) / (it_us * 1e-6) / (HBM_PEAK_GBS * 1e9), 4),
                "effective_frac_at_32B": round(ALGORITHMIC_MIN_BYTES * (vox / n) / (it_us * 1e-6)
                                               / (HBM_PEAK_GBS * 1e9), 4),
            },
        }
        for name, kk in kernels.items():
            log("  %-9s launches %5d  avg %8.2f us  %7.1f GB/s  share %.1f%%" % (
                name, kk["launches"], kk["avg_us"], kk["gbs"],
                100.0 * kk["total_ms"] / sum(q["total_ms"] for q in kernels.values())))
        for lv in range(cfg["levels"]):
            parts = []
            for name in disc.KERNELS:
                n, ms, vox = reg.timing_read(name, lv)
                if n:
                    parts.append("%s %.1f us" % (name, 1000.0 * ms / n))
            log("  level %d %s: %s" % (lv, "x".join(map(str, dims[lv][::-1])), ", ".join(parts)))

    out = {
        "metric": "DISC voxel-iterations/s (whole registration, all pyramid levels)",
        "value": round(value, 1),
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "shape_zyx": list(cfg["shape"]),
            "patch": list(cfg["patch"]),
            "sigma": cfg["sigma"],
            "levels": cfg["levels"],
            "iters_per_level": list(cfg["iters"]),
            "voxel_iterations_per_step": vox_it,
            "effective_hbm_frac_at_32B": round(ALGORITHMIC_MIN_BYTES * value / (HBM_PEAK_GBS * 1e9), 4),
            "kernels": {k: {q: round(v, 3) for q, v in kk.items()} for k, kk in kernels.items()},
        },
    }
    if roofline is not None:
        out["roofline"] = roofline
    if not args.no_extras:
        reg.timing_enable(0)  # no event pairs in the remaining measurements
        fin = finest_level_rate(reg, ct, cb, cfg)
        log("finest level alone: %.3f ms for %d iterations, %.3g voxel-it/s" % (
            fin["ms"], fin["iterations"], fin["voxel_iterations_per_s"]))
        out["finest_level"] = fin
        r_mid = torch.from_numpy(0.6 * case.r_true).float().contiguous().to(dev)
        bwd = backward_rate(disc, ct, cb, r_mid, cfg, fin["ms_per_iteration"])
        log("differentiable: loss %.3f ms, loss + gradient %.3f ms (%.2fx a plain iteration)" % (
            bwd["ms_loss"], bwd["ms_loss_and_grad"], bwd["vs_plain_iteration"]))
        gd = gd_vs_demons(disc, ct, cb, torch.from_numpy(case.r_true).float().to(dev), cfg)
        log("gradient descent vs demons, %d steps: GD %.1f ms, loss x%.4f, field err %.3f vox; "
            "demons %.1f ms, loss x%.4f, field err %.3f vox (r = 0: %.3f vox)" % (
                gd["steps"], gd["gradient_descent"]["ms"], gd["gradient_descent"]["loss_ratio"],
                gd["gradient_descent"]["mean_field_error_body_vox"], gd["demons"]["ms"],
                gd["demons"]["loss_ratio"], gd["demons"]["mean_field_error_body_vox"],
                gd["mean_field_error_body_vox_at_r0"]))
        bwd["gd_vs_demons"] = gd
        out["backward"] = bwd
        var = variant_rates(disc, ct, cb, cfg, ms_per_step)
        log("variants: " + ", ".join("%s %.2f ms (%.2fx)" % (k, v["ms_per_registration"], v["vs_plain"])
                                       for k, v in var.items()))
        out["variants"] = var
        log("batched: generating 16 uneven pairs")
        bat = batched_rate(disc)
        log("batched: sequential %.1f ms, batch eager %.1f ms, batch graph %.1f ms (%.2fx), tiles %s" % (
            bat["ms_sequential"], bat["ms_batched_eager"], bat["ms_batched_graph"],
            bat["speedup_graph_vs_sequential"], bat["tiles"]))
        sm = bat["small_volumes"]
        log("batched small volumes (16 x 64x64x32): sequential %.2f ms, batch eager %.2f ms, graph %.2f ms "
            "(%.2fx vs sequential, %.2fx vs eager)" % (sm["ms_sequential"], sm["ms_batched_eager"],
                                                       sm["ms_batched_graph"], sm["speedup_graph_vs_sequential"],
                                                       sm["speedup_graph_vs_eager"]))
        out["batched"] = bat
        others = {}
        for wname in ("ellipsoid48", "hn512x512x160"):
            if wname == args.workload:
                continue
            log("workload %s" % wname)
            others[wname] = workload_summary(disc, wname)
            fl = others[wname]["finest_level"]
            log("  %.3f ms per registration; finest level %.4f ms per iteration, %.3g voxel-it/s; kernels %s" % (
                others[wname]["ms_per_registration"], fl["ms_per_iteration"], fl["voxel_iterations_per_s"],
                others[wname]["finest_level_kernels"]))
        out["workloads"] = others
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(case, params)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
