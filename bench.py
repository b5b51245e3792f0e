#!/usr/bin/env python3
"""Benchmark of the BSI hot path on one MI355X.

A step is one pass of the hot path over one batch of synthetic input: forward BSI
(control grid -> field, Eq. 1) followed by the adjoint (dfield -> control-grid
gradient) on a 512 x 512 x 256 volume at spacing 5 (grid 106 x 106 x 55 x 3,
N(0, 3) box-filtered; dfield N(0, 1)), with every input resident in HBM before
the timed region.  value = voxels / (time per step) in GVoxel/s.

Printed as ONE JSON line on stdout (logs go to stderr), with:
  roofline      the dominant kernel's algorithmic bytes / its mean duration
                (HIP events on the launch stream) against 8 TB/s, and the HBM
                traffic measured by rocprofv3 counters when the committed
                measurement matches the current kernel sources;
  cpu_baseline  the FP64 oracle (forward + adjoint) on the first 128 z-planes of
                the same volume, and its adjoint at 256^3, on the host's cores
                (medians of 3 runs);
  extras        forward at spacings 3 and 8, the adjoint alone at 256^3
                (MALL flushed between repetitions), the 32-volume batched
                graph launch against per-volume launches, and one SSD
                registration iteration at 256 x 256 x 160, fused (one pass,
                no field in memory) and unfused (forward, SSD, adjoint), and
                scalar B-spline upsampling to 512 x 512 x 256 (factor 4), the
                forward in the paper's lerp form (ablation), and forward +
                adjoint for a grid with real spacing and an origin offset.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GVoxel/s BSI fwd+adjoint (fp32), % HBM peak; batched vs per-volume, 1 GPU"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = {
    "fwd_kernel": ["paper_2004_05962_amd/csrc/bsi_device.h", "paper_2004_05962_amd/csrc/forward.hip"],
    "adj_pass1_kernel": ["paper_2004_05962_amd/csrc/bsi_device.h", "paper_2004_05962_amd/csrc/adjoint_device.h",
                         "paper_2004_05962_amd/csrc/adjoint.hip"],
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_only(text):
    """Source text without comments and whitespace: edits to comments keep the hash."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return "".join(text.split())


def source_hash(kernel):
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, rel)) as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None when
    they were taken on other sources or another workload."""
    try:
        with open(TRAFFIC_FILE) as f:
            data = json.load(f)
        rec = data[kernel]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("src_hash") != source_hash(kernel) or rec.get("workload") != workload:
        return None
    return rec.get("hbm_bytes_per_launch")


def median(xs):
    return float(np.median(np.asarray(xs, np.float64)))


def time_events(torch, fn, reps, flush=None):
    """Durations (ms) of fn() between HIP events on the current stream."""
    out = []
    for _ in range(reps):
        if flush is not None:
            flush()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b))
    return out


def cpu_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(grid_np, dfield_np, dims, spacing, cfg3, planes=128, planes_1t=16, reps=3):
    """FP64 oracle on the host's cores: forward (triple sum, OpenMP over z) and
    adjoint (per-control-point gather, OpenMP over control points) on the first
    `planes` z-planes of the benchmark volume, the median of `reps` runs each;
    the adjoint alone on the 256^3 workload (median of `reps`); and the forward
    on `planes_1t` planes with one thread."""
    import oracle
    d = spacing[2]

    def sub(p):
        return (dims[0], dims[1], p), grid_np[:-(-p // d) + 3], dfield_np[:p]

    def timed(fn, *args):
        t0 = time.perf_counter()
        fn(*args)
        return time.perf_counter() - t0

    sub_dims, g, y = sub(planes)
    t_fwd = median([timed(oracle.forward, g, sub_dims, spacing) for _ in range(reps)])
    t_adj = median([timed(oracle.adjoint_gather, y, sub_dims, spacing) for _ in range(reps)])
    c3_dims, c3_sp = cfg3["dims"], cfg3["spacing"]
    t_c3 = median([timed(oracle.adjoint_gather, cfg3["dfield"], c3_dims, c3_sp) for _ in range(reps)])
    threads = oracle.num_threads()
    dims1, g1, _ = sub(planes_1t)
    oracle.set_num_threads(1)
    t_1t = timed(oracle.forward, g1, dims1, spacing)
    oracle.set_num_threads(threads)
    vox = dims[0] * dims[1] * planes
    vox1 = dims[0] * dims[1] * planes_1t
    vox3 = c3_dims[0] * c3_dims[1] * c3_dims[2]
    model, affinity = cpu_info()
    return {"value": vox / (t_fwd + t_adj) / 1e9, "unit": "GVoxel/s", "cores": threads, "kind": "oracle",
            "sample": f"first {planes} of {dims[2]} z-planes ({vox / 1e6:.1f} M voxels): forward {t_fwd:.2f} s "
                      f"(triple sum) + adjoint {t_adj:.2f} s (per-point gather), FP64, {threads} OpenMP threads, "
                      f"median of {reps}",
            "forward_gvoxel_s": vox / t_fwd / 1e9, "adjoint_gvoxel_s": vox / t_adj / 1e9,
            "adjoint_256cubed_d5_gvoxel_s": vox3 / t_c3 / 1e9,
            "forward_1_thread_gvoxel_s": vox1 / t_1t / 1e9, "cpu_model": model, "affinity_cpus": affinity}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--quick", action="store_true", help="main step only: no extras, no CPU baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--with-registration", action="store_true",
                    help="with --quick: also time the registration iteration, fused and unfused")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 3 plain device-to-device copies of 805,306,368 bytes (the known-size "
                         "reference that rocprofv3 FETCH_SIZE / WRITE_SIZE are scaled by)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path here runs on a single MI355X; "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch
    import paper_2004_05962_amd as bsi
    import workloads

    torch.cuda.set_device(0)
    log("setup: 512x512x256 spacing 5")
    case = workloads.cfg2(5)
    dims, spacing = case["dims"], case["spacing"]
    V = dims[0] * dims[1] * dims[2]
    gx, gy, gz = bsi.bsi_grid_dims(dims, spacing)
    G = gx * gy * gz
    dfield_np = workloads.random_field(dims, 1.0, seed=1102)
    grid = torch.from_numpy(case["grid"]).cuda()
    dfield = torch.from_numpy(dfield_np).cuda()
    field = torch.empty(bsi.field_shape(dims), device="cuda")
    grad = torch.empty(bsi.grid_shape(dims, spacing), device="cuda")
    ws = torch.empty(bsi.bsi_adjoint_workspace_size(dims, spacing), dtype=torch.uint8, device="cuda")

    def step():
        bsi.bsi_forward(grid, dims, spacing, field)
        bsi.bsi_adjoint_partials(dfield, dims, spacing, ws)
        bsi.bsi_adjoint_reduce(ws, dims, spacing, grad)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # events on the current stream, which is the stream every call above launches on
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in ev:
        e[0].record()
        bsi.bsi_forward(grid, dims, spacing, field)
        e[1].record()
        bsi.bsi_adjoint_partials(dfield, dims, spacing, ws)
        e[2].record()
        bsi.bsi_adjoint_reduce(ws, dims, spacing, grad)
        e[3].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    p1_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    p2_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in ev]))
    adj_ms = p1_ms + p2_ms
    ms_per_step = wall * 1e3 / args.steps
    value = V / (ms_per_step * 1e-3) / 1e9

    # algorithmic bytes: forward reads the grid and writes the field; the adjoint
    # reads dfield (pass 1) and writes the gradient (pass 2); the partials in
    # between are scratch and not counted
    fwd_bytes = 12 * V + 12 * G
    adj_bytes = 12 * V + 12 * G
    p1_bytes = 12 * V
    workload = "512x512x256 d5"
    if fwd_ms >= p1_ms:
        kern, ms, nbytes = "fwd_kernel", fwd_ms, fwd_bytes
    else:
        kern, ms, nbytes = "adj_pass1_kernel", p1_ms, p1_bytes
    achieved = nbytes / (ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kern, workload),
                "kernel": kern, "algorithmic_bytes": nbytes, "mean_ms": round(ms, 4)}
    other = {"forward_ms": round(fwd_ms, 4), "adjoint_ms": round(adj_ms, 4),
             "adjoint_pass1_ms": round(p1_ms, 4), "adjoint_pass2_ms": round(p2_ms, 4),
             "forward_hbm_frac": round(fwd_bytes / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "adjoint_hbm_frac": round(adj_bytes / (adj_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "forward_gvoxel_s": round(V / (fwd_ms * 1e-3) / 1e9, 2),
             "adjoint_gvoxel_s": round(V / (adj_ms * 1e-3) / 1e9, 2)}
    log("main:", json.dumps(other))

    # ceilings measured live on this GPU with plain torch kernels of the same size:
    # a fill (write-only) and a copy, each on 805,306,368 bytes
    nb = 12 * V
    a_buf = torch.empty(nb // 4, device="cuda")
    b_buf = torch.empty_like(a_buf)
    a_buf.fill_(1.0)
    fill_gbs = nb / median(time_events(torch, lambda: a_buf.fill_(2.0), 10)) / 1e6
    copy_gbs = 2 * nb / median(time_events(torch, lambda: b_buf.copy_(a_buf), 10)) / 1e6
    del a_buf, b_buf
    fwd_gbs = fwd_bytes / (fwd_ms * 1e-3) / 1e9
    p1_gbs = p1_bytes / (p1_ms * 1e-3) / 1e9
    ceilings = {"fill_gbs": round(fill_gbs, 1), "copy_gbs": round(copy_gbs, 1),
                "forward_frac_of_fill": round(fwd_gbs / fill_gbs, 4),
                "adjoint_pass1_frac_of_copy": round(p1_gbs / copy_gbs, 4)}
    log("ceilings:", json.dumps(ceilings))

    if args.copy_calibration:
        src = torch.ones(805306368 // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    extras = {}
    if not args.quick:
        extras = run_extras(torch, bsi, workloads)
    elif args.with_registration:
        extras = registration_iterations(torch, bsi, workloads)
    cpu = None
    if not args.quick and not args.no_cpu and rank == 0:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(case["grid"], dfield_np, dims, spacing, workloads.cfg3())

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "GVoxel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "BSI forward + adjoint, 512x512x256 voxels, spacing 5, grid 106x106x55x3",
                   "global_batch": 1, "voxels": V, "spacing": list(spacing), "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "breakdown": other, "ceilings": ceilings, "extras": extras,
    }
    print(json.dumps(out), flush=True)


def run_extras(torch, bsi, workloads):
    ex = {}
    # Evict the 256 MB MALL between repetitions by READING 1 GiB: a write-based
    # flush would leave dirty lines whose write-back lands inside the next
    # measured kernel.
    flush_buf = torch.ones(1 << 28, dtype=torch.float32, device="cuda")

    def flush():
        flush_buf.sum()

    # forward at the other clinical spacings
    for d in (3, 8):
        c = workloads.cfg2(d)
        dims, sp = c["dims"], c["spacing"]
        V = dims[0] * dims[1] * dims[2]
        gx, gy, gz = bsi.bsi_grid_dims(dims, sp)
        g = torch.from_numpy(c["grid"]).cuda()
        f = torch.empty(bsi.field_shape(dims), device="cuda")
        for _ in range(3):
            bsi.bsi_forward(g, dims, sp, f)
        ms = median(time_events(torch, lambda: bsi.bsi_forward(g, dims, sp, f), 20))
        nb = 12 * V + 12 * gx * gy * gz
        ex[f"forward_512x512x256_d{d}"] = {"ms": round(ms, 4), "gvoxel_s": round(V / ms / 1e6, 2),
                                           "hbm_frac": round(nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"forward d{d}:", ex[f"forward_512x512x256_d{d}"])
        del g, f

    # adjoint alone at 256^3 (its dfield fits the MALL: flush between repetitions)
    c = workloads.cfg3()
    dims, sp = c["dims"], c["spacing"]
    V = dims[0] * dims[1] * dims[2]
    gx, gy, gz = bsi.bsi_grid_dims(dims, sp)
    y = torch.from_numpy(c["dfield"]).cuda()
    out = torch.empty(bsi.grid_shape(dims, sp), device="cuda")
    ws = torch.empty(bsi.bsi_adjoint_workspace_size(dims, sp), dtype=torch.uint8, device="cuda")
    for _ in range(3):
        bsi.bsi_adjoint(y, dims, sp, out, ws)
    ms = median(time_events(torch, lambda: bsi.bsi_adjoint(y, dims, sp, out, ws), 20, flush=flush))
    nb = 12 * V + 12 * gx * gy * gz
    ex["adjoint_256cubed_d5"] = {"ms": round(ms, 4), "gvoxel_s": round(V / ms / 1e6, 2),
                                 "hbm_frac": round(nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    log("adjoint 256^3:", ex["adjoint_256cubed_d5"])
    del y, out, ws

    # batched: 32 uneven volumes, forward + adjoint, one graph vs per-volume launches
    dims_l, sp_l = workloads.cfg5_geometry()
    grids, dfields, fields, grads = [], [], [], []
    for i, (d, s) in enumerate(zip(dims_l, sp_l)):
        g, y = workloads.cfg5_volume(tuple(d), tuple(s), i)
        grids.append(torch.from_numpy(g).cuda())
        dfields.append(torch.from_numpy(y).cuda())
        fields.append(torch.empty(bsi.field_shape(d), device="cuda"))
        grads.append(torch.empty(bsi.grid_shape(d, s), device="cuda"))
    vox = int(sum(int(np.prod(d)) for d in dims_l))
    plan = bsi.BatchPlan(dims_l, sp_l)
    plan.bind(grids, fields, dfields, grads)
    chosen, nsched = plan.tune()
    # the legacy null stream cannot be captured: capture on a side stream, replay on the current one
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    plan.capture(side)
    torch.cuda.current_stream().wait_stream(side)
    for _ in range(3):
        plan.launch()
        plan.run_separate()
    t_graph = median(time_events(torch, plan.launch, 20))
    t_sep = median(time_events(torch, plan.run_separate, 20))
    ex["batched_32_volumes"] = {"voxels": vox, "graph_ms": round(t_graph, 4), "separate_ms": round(t_sep, 4),
                                "speedup": round(t_sep / t_graph, 3), "graph_gvoxel_s": round(vox / t_graph / 1e6, 2),
                                "schedule": chosen, "schedules": nsched, "schedule_knobs": plan.describe()}
    log("batched:", ex["batched_32_volumes"])
    plan.close()
    del grids, dfields, fields, grads

    # the paper's lerp form of the forward (ablation): 63 lerps (a subtraction and
    # an FMA each, 3 flops) per component and voxel, against about 22 FMA for the
    # sum-factorised kernel
    field_l = torch.empty(256, 512, 512, 3, device="cuda")
    c2 = workloads.cfg2(5)
    grid_l = torch.from_numpy(c2["grid"]).cuda()
    fn = lambda: bsi.bsi_forward_lerp(grid_l, c2["dims"], c2["spacing"], field_l)
    fn()
    ms = median(time_events(torch, fn, 10))
    Vl = 512 * 512 * 256
    flops = Vl * 63 * 3 * 3
    ex["forward_lerp_form_512x512x256_d5"] = {
        "ms": round(ms, 4), "gvoxel_s": round(Vl / ms / 1e6, 2),
        "tflops": round(flops / ms / 1e9, 2), "frac_fp32_vector_peak": round(flops / ms / 1e9 / 157.3, 4)}
    log("forward lerp form:", ex["forward_lerp_form_512x512x256_d5"])
    del field_l, grid_l

    # real spacing and an origin offset: forward and the separable adjoint on
    # 512 x 512 x 256 with spacing (5.3, 4.7, 5.1), origin (-2.5, -0.25, -4.0)
    dims_g, sp_g, org_g = (512, 512, 256), (5.3, 4.7, 5.1), (-2.5, -0.25, -4.0)
    gg = torch.randn(bsi.general_grid_shape(dims_g, sp_g, org_g), device="cuda")
    fg = torch.empty(256, 512, 512, 3, device="cuda")
    grad_g = torch.empty_like(gg)
    ws_g = torch.empty(bsi.bsi_adjoint_general_workspace_size(dims_g, sp_g, org_g), dtype=torch.uint8, device="cuda")
    f_fwd = lambda: bsi.bsi_forward_general(gg, dims_g, sp_g, org_g, fg)
    f_adj = lambda: bsi.bsi_adjoint_general(fg, dims_g, sp_g, org_g, grad_g, ws_g)
    f_fwd()
    f_adj()
    t_f = median(time_events(torch, f_fwd, 10))
    t_a = median(time_events(torch, f_adj, 10))
    Vg, Gg = 512 * 512 * 256, gg.numel() // 3
    ex["general_spacing_512x512x256"] = {
        "spacing": list(sp_g), "origin": list(org_g), "forward_ms": round(t_f, 4), "adjoint_ms": round(t_a, 4),
        "forward_hbm_frac": round((12 * Vg + 12 * Gg) / t_f / 1e6 / HBM_PEAK_GBS, 4),
        "adjoint_hbm_frac": round((12 * Vg + 12 * Gg) / t_a / 1e6 / HBM_PEAK_GBS, 4)}
    log("general spacing:", ex["general_spacing_512x512x256"])
    del gg, fg, grad_g, ws_g

    # scalar B-spline upsampling: a 131 x 131 x 67 coarse volume (control points)
    # to 512 x 512 x 256 voxels, factor 4 on every axis
    dims_s, sp_s = (512, 512, 256), (4, 4, 4)
    gx, gy, gz = bsi.bsi_grid_dims(dims_s, sp_s)
    coarse = torch.randn(gz, gy, gx, device="cuda")
    image = torch.empty(256, 512, 512, device="cuda")
    fn = lambda: bsi.bsi_forward_scalar(coarse, dims_s, sp_s, image)
    fn()
    ms = median(time_events(torch, fn, 20))
    Vs = 512 * 512 * 256
    ex["scalar_upsample_512x512x256_x4"] = {"ms": round(ms, 4), "gvoxel_s": round(Vs / ms / 1e6, 2),
                                            "hbm_frac": round((4 * Vs + 4 * gx * gy * gz) / ms / 1e6 / HBM_PEAK_GBS, 4)}
    log("scalar upsampling:", ex["scalar_upsample_512x512x256_x4"])
    del coarse, image

    ex.update(registration_iterations(torch, bsi, workloads))
    return ex


def registration_iterations(torch, bsi, workloads):
    """One SSD registration iteration at 256 x 256 x 160, fused and unfused
    (the moving image is made on the GPU)."""
    ex = {}
    c = workloads.cfg4()
    dims, sp = c["dims"], c["spacing"]
    fixed = torch.from_numpy(c["fixed"]).cuda()
    Ttrue = bsi.forward(torch.from_numpy(c["grid_true"]).cuda(), dims, sp)
    moving = torch.empty_like(fixed)
    bsi.bsi_warp(Ttrue, fixed, dims, moving)
    V = dims[0] * dims[1] * dims[2]
    for fused in (True, False):
        reg = bsi.SSDRegistration(fixed, moving, sp, max_steps=64, fused=fused)
        reg.auto_eta()
        reg.run(3)
        ms = median(time_events(torch, reg.step, 20))
        key = "registration_iteration_256x256x160_d5_" + ("fused" if fused else "unfused")
        ex[key] = {"ms": round(ms, 4), "gvoxel_s": round(V / ms / 1e6, 2), "loss_first": float(reg.losses[0]),
                   "loss_last": float(reg.losses[reg.step_index - 1])}
        log("registration:", key, ex[key])
        del reg
    return ex


if __name__ == "__main__":
    main()
