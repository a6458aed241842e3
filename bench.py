#!/usr/bin/env python3
"""Throughput benchmark of the GPSS renderer on one MI355X.

Headline workload (default "mixed"): union-SDF mean of 16 seeded spheres and boxes in
[-1, 1]^3, squared-exponential kernel with a 128^3 value-noise variance grid in
[1e-4, 1e-2], lengthscale 0.03, per-primitive albedo, point light plus environment,
pinhole 1024x1024, 256 spp, max depth 64.  One step renders the whole image (268.4 M
paths) with the scene already resident on the GPU.

Prints one JSON line: Mpaths/s of the headline, the roofline entry of its render kernel
(algorithmic FP32 FLOPs per launch / the launch time measured with HIP events on the render
stream), the image MSE against the FP64 oracle on sampled pixels, secondary rows (the sphere
lengthscale sweep and the paper's variants, each with its roofline), the path-replay adjoint
and the batched render (median of 10 timed calls after 3 warm-ups, each with a roofline
entry), and the FP64 CPU oracle timed on a bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpaths/s forward + adjoint at fixed image MSE vs oracle; % FP32 VALU peak"
FP32_PEAK_TFLOPS = 157.3      # MI355X vector FP32 (packed); non-packed FMA issue gives 78.6

WORKLOADS = {
    "sphere": "unit-sphere SDF mean, SE kernel variance 0.0025, lengthscales 0.005/0.02/0.1/0.5, "
              "albedo 0.8, point light + environment, pinhole 512x512, 64 spp, max depth 32",
    "plane": "planar GPSS m(x)=z, variance 0.01, lengthscale 0.05, |z|<0.4, albedo 0.9, "
             "directional light 30 deg, ortho 64x64 at 45 deg, 16 spp, max depth 8",
    "mixed": "union SDF of 16 seeded spheres/boxes, 128^3 value-noise variance grid in "
             "[1e-4,1e-2], lengthscale 0.03, 1024x1024, 256 spp, max depth 64, 80^3 majorant grid",
    "cond": "unit-sphere SDF prior conditioned on 32 noisy point observations (Fibonacci directions, "
            "radii jittered +-0.08, value 0, noise 0.05 x variance), variance 0.0025, lengthscale 0.25, "
            "pinhole 512x512, 64 spp, max depth 32",
}


# HBM traffic of the render kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by
# the same counters on a plain copy (see --summarize-traffic); valid only while the kernel
# sources hash to the recorded value.
def traffic_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"sched_render_kernel_{workload}_traffic.md")


KERNEL_SOURCES = ["gpss_sched.hpp", "gpss_persistent.hip", "gpss_trace.hpp", "gpss_device.hpp", "gpss_waves.hpp",
                  "gpss_accum.hpp"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2603_00280_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload: str):
    """Bytes of HBM traffic per render launch recorded for the current kernel, else None."""
    try:
        lines = open(traffic_file(workload)).read().splitlines()
    except OSError:
        return None
    kv = {}
    for ln in lines:
        if ln.startswith("    ") and ":" in ln:
            k, v = ln.strip().split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return json.loads(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def summarize_traffic(workload, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, commands):
    """Write the workload's traffic file from four rocprofv3 --pmc runs (FETCH_SIZE and
    WRITE_SIZE of the bench render and of the plain-copy calibration), each a directory of
    counter CSVs."""
    import csv
    import glob

    def per_dispatch(d, counter, kernel):
        vals = []
        for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == counter and kernel in r["Kernel_Name"]:
                    vals.append((int(r["Dispatch_Id"]), float(r["Counter_Value"])))
        return [v for _, v in sorted(vals)]

    kern = "sched_render_kernel<false, 0>"
    fetch = per_dispatch(fetch_dir, "FETCH_SIZE", kern)
    write = per_dispatch(write_dir, "WRITE_SIZE", kern)
    cf = per_dispatch(copy_fetch_dir, "FETCH_SIZE", "copy")
    cw = per_dispatch(copy_write_dir, "WRITE_SIZE", "copy")
    f_fac = copy_bytes / 1024.0 / cf[-1]
    w_fac = copy_bytes / 1024.0 / cw[-1]
    traffic = [1024.0 * (a * f_fac + b * w_fac) for a, b in zip(fetch, write)]
    path = traffic_file(workload)
    with open(path, "w") as f:
        f.write(f"# HBM traffic of sched_render_kernel on the {workload} workload\n\n")
        f.write("Counters per dispatch of the forward render kernel (its timed launches in bench\n"
                "order), in KiB, from separate rocprofv3 runs:\n\n")
        for c in commands:
            f.write(f"    {c}\n")
        f.write("\nA plain device copy of known size calibrates each counter (known bytes / counter\n"
                "bytes); traffic = FETCH_SIZE x fetch factor + WRITE_SIZE x write factor.\n\n")
        f.write(f"    source_sha256: {kernel_source_hash()}\n")
        f.write(f"    fetch_kib_per_launch: {json.dumps(fetch)}\n")
        f.write(f"    write_kib_per_launch: {json.dumps(write)}\n")
        f.write(f"    copy_bytes: {copy_bytes}\n")
        f.write(f"    copy_fetch_kib: {cf[-1]}\n")
        f.write(f"    copy_write_kib: {cw[-1]}\n")
        f.write(f"    fetch_factor: {f_fac:.4f}\n")
        f.write(f"    write_factor: {w_fac:.4f}\n")
        f.write(f"    traffic_bytes_per_launch: {json.dumps([round(t) for t in traffic])}\n")
    print(open(path).read())


def _csv_rows(d, pattern):
    import csv
    import glob
    out = []
    for f in sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True)):
        out += list(csv.DictReader(open(f)))
    return out


def summarize_trace(workload, kt_dir, bench_json, commands):
    """Write profiles/sched_render_kernel_<workload>.md from a rocprofv3 --kernel-trace --stats
    run of bench.py: the per-kernel summary of the whole run, and the headline render's launches
    (the dispatches of the default render kernel longer than half its longest) against the
    launch time bench.py measured with HIP events in the same run."""
    stats = _csv_rows(kt_dir, "*kernel_stats.csv")
    trace = _csv_rows(kt_dir, "*kernel_trace.csv")
    res = json.loads([ln for ln in open(bench_json).read().splitlines() if ln.startswith("{")][-1])
    kern = "sched_render_kernel<false, 0>"
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in trace if kern in r["Kernel_Name"]]
    top = max(durs)
    head = [d for d in durs if d > 0.5 * top]
    path = os.path.join(ROOT, "profiles", f"sched_render_kernel_{workload}.md")
    with open(path, "w") as f:
        f.write(f"# sched_render_kernel<false, 0> on the {workload} workload: kernel trace of the default bench run\n\n")
        f.write("Command (repo root):\n\n")
        for c in commands:
            f.write(f"    {c}\n")
        f.write(f"\nWorkload: {res['config']['workload']}.\n\n")
        f.write(f"Headline render launches (warm-up and timed, {len(head)} dispatches of `{kern}` longer than "
                f"half the longest):\n\n")
        f.write("    " + ", ".join(f"{d:.2f}" for d in head) + " ms\n")
        f.write(f"    kernel-trace average: {sum(head) / len(head):.2f} ms\n")
        f.write(f"    bench.py HIP-event average over its timed launches (same run): "
                f"{res['roofline']['avg_launch_ms']:.2f} ms (clear, render, finalize)\n")
        f.write(f"    value: {res['value']:.1f} {res['unit']}, roofline frac {100 * res['roofline']['frac']:.2f} % "
                f"of {res['roofline']['peak']} {res['roofline']['unit']}\n\n")
        f.write("Whole run, kernels by total time:\n\n")
        f.write("| Kernel | Calls | Total (ms) | Average (ms) | Max (ms) | % |\n|---|--:|--:|--:|--:|--:|\n")
        for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:14]:
            name = r["Name"].split("(")[0].replace("void ", "")
            f.write(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                    f"{float(r['AverageNs']) / 1e6:.3f} | {float(r['MaxNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |\n")
    print(open(path).read())


def summarize_counters(workload, dirs, kt_dir, commands):
    """Write profiles/sched_render_kernel_<workload>_counters.md from rocprofv3 --pmc runs of
    bench.py (SQ counters, any split over the runs) and the kernel trace of the default run
    (for launch times): the headline render (the longest dispatch of the default render
    kernel), the adjoint's forward render (the other dispatches of that kernel, median), the
    adjoint and the batch kernel (medians)."""
    import statistics
    per = {}
    for d in dirs:
        for r in _csv_rows(d, "*counter_collection.csv"):
            key = (d, int(r["Dispatch_Id"]))
            e = per.setdefault(key, {"kernel": r["Kernel_Name"]})
            e[r["Counter_Name"]] = float(r["Counter_Value"])
    groups = {"headline render": [], "adjoint's forward render": [], "adjoint": [], "batch": []}
    for d in dirs:
        mine = sorted(((k[1], v) for k, v in per.items() if k[0] == d), key=lambda kv: kv[0])
        fwd = [(i, v) for i, v in mine if "sched_render_kernel<false, 0>" in v["kernel"]]
        adj = [i for i, v in mine if "sched_adjoint_kernel" in v["kernel"]]
        bat = [i for i, v in mine if "batch_kernel" in v["kernel"]]
        if fwd:
            groups["headline render"].append(max((v for _, v in fwd), key=lambda v: v.get("SQ_INSTS_VALU", 0.0)))
        if adj:
            # bench.py times the adjoint's forward render right after the adjoint, before the batch
            hi = min(bat) if bat else float("inf")
            groups["adjoint's forward render"] += [v for i, v in fwd if max(adj) < i < hi]
        groups["adjoint"] += [v for i, v in mine if i in adj]
        groups["batch"] += [v for i, v in mine if i in bat]
    trace = _csv_rows(kt_dir, "*kernel_trace.csv")

    def durs(pat):
        return sorted((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in trace if pat in r["Kernel_Name"])
    fwd_d = durs("sched_render_kernel<false, 0>")
    times = {"headline render": fwd_d[-1] if fwd_d else None, "adjoint's forward render": None,
             "adjoint": None, "batch": None}
    # the adjoint's forward render: the default render kernel's dispatches between the last
    # adjoint dispatch and the first batch dispatch of the traced run
    order = sorted(trace, key=lambda r: int(r["Dispatch_Id"]))
    ai = [int(r["Dispatch_Id"]) for r in order if "sched_adjoint_kernel" in r["Kernel_Name"]]
    bi = [int(r["Dispatch_Id"]) for r in order if "batch_kernel" in r["Kernel_Name"]]
    if ai:
        hi = min(bi) if bi else float("inf")
        fd = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in order
              if "sched_render_kernel<false, 0>" in r["Kernel_Name"] and max(ai) < int(r["Dispatch_Id"]) < hi]
        times["adjoint's forward render"] = statistics.median(fd) if fd else None
    adj_d, bat_d = durs("sched_adjoint_kernel"), durs("batch_kernel")
    times["adjoint"] = statistics.median(adj_d) if adj_d else None
    times["batch"] = statistics.median(bat_d) if bat_d else None

    def med(vs, c):
        xs = [v[c] for v in vs if c in v]
        return statistics.median(xs) if xs else float("nan")
    path = os.path.join(ROOT, "profiles", f"sched_render_kernel_{workload}_counters.md")
    with open(path, "w") as f:
        f.write(f"# Scheduled tracer kernels on the {workload} workload, the adjoint and the batch: SQ counters\n\n")
        f.write("Commands (repo root; counter passes within the per-block limits, and the kernel trace of the\n"
                "default bench run for launch times):\n\n")
        for c in commands:
            f.write(f"    {c}\n")
        f.write("\nPer dispatch (medians over a group's dispatches).  The FP32 FLOP instruction counter counts\n"
                "per wave instruction (FMA as 2); times 64 lanes it gives the issued FP32 rate, masked lanes\n"
                "included.  Lane utilization = SQ_THREAD_CYCLES_VALU / (64 x SQ_ACTIVE_INST_VALU).  VALU busy =\n"
                "VALU wave instructions x 4 cycles / (1024 SIMDs x 2.4 GHz x launch time).\n\n")
        f.write("| Kernel (group) | Launch (ms) | VALU instr. | lane util. | VALU busy | FP32 FLOP instr. x 64 "
                "(TFLOP/s) | FP64 FLOP instr. | SALU instr. | LDS instr. | vector loads | scalar loads | "
                "waits / wave cycles | waves |\n")
        f.write("|---|--:|--:|--:|--:|--:|--:|--:|--:|--:|--:|--:|--:|\n")
        for g, vs in groups.items():
            if not vs:
                continue
            valu = med(vs, "SQ_INSTS_VALU")
            lu = med(vs, "SQ_THREAD_CYCLES_VALU") / (64.0 * med(vs, "SQ_ACTIVE_INST_VALU"))
            t = times[g]
            fp32 = med(vs, "SQ_INSTS_VALU_FLOPS_FP32") * 64.0
            busy = f"{100 * valu * 4 / (1024 * 2.4e9 * t / 1e3):.0f} %" if t else "-"
            rate = f"{fp32 / (t / 1e3) / 1e12:.2f}" if t else "-"
            f.write(f"| {g} | {t:.2f} | {valu:.3g} | {100 * lu:.1f} % | {busy} | {rate} | "
                    f"{med(vs, 'SQ_INSTS_VALU_FLOPS_FP64'):.3g} | {med(vs, 'SQ_INSTS_SALU'):.3g} | "
                    f"{med(vs, 'SQ_INSTS_LDS'):.3g} | {med(vs, 'SQ_INSTS_VMEM_RD'):.3g} | "
                    f"{med(vs, 'SQ_INSTS_SMEM'):.3g} | "
                    f"{med(vs, 'SQ_WAIT_INST_ANY') / med(vs, 'SQ_WAVE_CYCLES'):.2f} | {med(vs, 'SQ_WAVES'):.0f} |\n"
                    if t else
                    f"| {g} | - | {valu:.3g} | {100 * lu:.1f} % | - | - | {med(vs, 'SQ_INSTS_VALU_FLOPS_FP64'):.3g} | "
                    f"{med(vs, 'SQ_INSTS_SALU'):.3g} | {med(vs, 'SQ_INSTS_LDS'):.3g} | {med(vs, 'SQ_INSTS_VMEM_RD'):.3g} | "
                    f"{med(vs, 'SQ_INSTS_SMEM'):.3g} | "
                    f"{med(vs, 'SQ_WAIT_INST_ANY') / med(vs, 'SQ_WAVE_CYCLES'):.2f} | {med(vs, 'SQ_WAVES'):.0f} |\n")
    print(open(path).read())


def copy_calibration(nbytes: int):
    """One plain device-to-device copy of nbytes (the calibration kernel of the traffic runs)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes}), flush=True)


TRACERS = {"auto": "persistent scheduled waves", "persistent": "persistent scheduled waves",
           "wavefront": "wavefront", "mega": "one thread per path"}


def make_scenes(name):
    from gpss_inputs import scenes as sc
    if name == "sphere":
        return [sc.sphere_scene(l) for l in sc.SPHERE_LENGTHSCALES]
    if name == "plane":
        return [sc.plane_scene()]
    if name == "mixed":
        return [sc.mixed_scene()]
    if name == "cond":
        return [sc.cond_sphere_scene()]
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(scenes, spp: int):
    """FP64 oracle on a bounded sample: every pixel of every scene at `spp` samples, with
    one OpenMP thread per core available to this process (capped by OMP_NUM_THREADS)."""
    from oracle.oracle import OracleScene
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count() or 1
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        cores = min(cores, int(os.environ["OMP_NUM_THREADS"]))
    n = 0
    t0 = time.perf_counter()
    for s in scenes:
        OracleScene(s).render(0, spp, nthreads=cores)
        n += s.n_pixels * spp
    dt = time.perf_counter() - t0
    # one core on a smaller sample of the same scenes (one sample per pixel of each)
    n1 = 0
    t1 = time.perf_counter()
    for s in scenes:
        OracleScene(s).render(0, 1, nthreads=1)
        n1 += s.n_pixels
    dt1 = time.perf_counter() - t1
    return {"value": n / dt / 1e6, "unit": "Mpaths/s", "cores": cores, "kind": "oracle",
            "sample": f"all pixels of each scene at {spp} spp ({n} paths, {dt:.1f} s)",
            "single_core_mpaths_s": n1 / dt1 / 1e6,
            "single_core_sample": f"all pixels of each scene at 1 spp ({n1} paths, {dt1:.1f} s)",
            "cpu": cpu_model()}


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def image_mse(torch, scene, img, npix: int = 256, factor: int = 4, seed: int = 11):
    """MSE of the timed image (samples [0, spp)) against the FP64 oracle's image of the same
    scene at factor x spp (samples [spp, (1 + factor) spp), independent of the timed ones) on
    npix pixels sampled at random.  Every GPU form (persistent, wavefront, one thread per path,
    batch, no-alloc) gives the same image, hence the same MSE."""
    import numpy as np
    from oracle.oracle import OracleScene
    rng = np.random.default_rng(seed)
    px = np.sort(rng.choice(scene.n_pixels, size=min(npix, scene.n_pixels), replace=False))
    ref = OracleScene(scene).render_pixels(px, scene.spp, (1 + factor) * scene.spp)
    g = img.reshape(-1)[torch.as_tensor(px, device=img.device)].double().cpu().numpy()
    d2 = (g - ref["mean"]) ** 2
    return {"reference": f"FP64 oracle, samples [spp, {1 + factor} spp) of {px.size} random pixels",
            "mse": float(d2.mean()), "mse_stderr": float(d2.std(ddof=1) / np.sqrt(d2.size)),
            "pixels": int(px.size)}


def median_ms(torch, fn, reps: int = 10, warmup: int = 3, stream=None):
    """Median of `reps` calls of fn timed with HIP events on the stream it runs on (torch's
    current stream by default), after `warmup` untimed calls."""
    stream = stream or torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    ms.sort()
    return 0.5 * (ms[(reps - 1) // 2] + ms[reps // 2]), ms


def roofline(flops: float, ms: float, traffic=None) -> dict:
    rate = flops / (ms / 1e3) / 1e12
    return {"bound": "alu", "achieved": rate, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": rate / FP32_PEAK_TFLOPS, "traffic": traffic, "flops_per_launch": flops}


def forward_flops(gpss, flops, torch, scene, g) -> float:
    """Algorithmic FLOPs of one full render of `scene` from the event counts of the same paths."""
    _, cnt = g.render_paths(counters=True)
    torch.cuda.synchronize()
    return flops.flops_from_counters(scene, gpss.counters_dict(cnt))


def row_measurement(torch, gpss, label: str, scenes):
    """Mpaths/s of one secondary row (median of 10 passes over its scenes after 3 warm-ups) and
    the roofline entry of its render kernel (algorithmic FLOPs / pass time on the render stream)."""
    from paper_2603_00280_amd import flops
    gs = [gpss.GpssScene(s) for s in scenes]
    imgs = [torch.empty(s.height, s.width, dtype=torch.float32, device="cuda") for s in scenes]
    fl = sum(forward_flops(gpss, flops, torch, s, g) for s, g in zip(scenes, gs))

    def one_pass():
        for g, im in zip(gs, imgs):
            g.render(out=im)
    ms, _ = median_ms(torch, one_pass)
    n = sum(s.n_paths for s in scenes)
    out = {"workload": label, "value": n / (ms / 1e3) / 1e6, "unit": "Mpaths/s", "ms_per_pass": ms,
           "roofline": roofline(fl, ms)}
    del gs, imgs
    return out


def adjoint_measurement(torch, gpss):
    """Path-replay adjoint of the L2 image loss on the offset-sphere workload (256^2, 16 spp,
    depth 16, 64^3 mean-offset grid) at theta0 against the target image, beside the forward
    render of the same scene; median of 10 after 3 warm-ups each.  A path counts once although
    it is traced (primal pass) and replayed.  The roofline's algorithmic work counts the
    forward arithmetic of every path twice (primal and replay) and leaves out the gradient
    terms, a lower bound of the adjoint's work."""
    from gpss_inputs import scenes as sc
    from paper_2603_00280_amd import flops
    s0, st = sc.offset_sphere_scene(False), sc.offset_sphere_scene(True)
    target = gpss.GpssScene(st).render()
    g = gpss.GpssScene(s0)
    img = g.render()
    dl = (2.0 * (img - target) / img.numel()).contiguous()
    fwd_fl = forward_flops(gpss, flops, torch, s0, g)
    adj_ms, _ = median_ms(torch, lambda: g.render_adjoint(dl))
    fwd_ms, _ = median_ms(torch, lambda: g.render(out=img))
    return {"workload": "offset sphere: 64^3 mean-offset grid, 256x256, 16 spp, max depth 16, "
                        "L2 loss against the seeded target",
            "adjoint_mpaths_s": s0.n_paths / (adj_ms / 1e3) / 1e6,
            "forward_mpaths_s": s0.n_paths / (fwd_ms / 1e3) / 1e6,
            "adjoint_ms": adj_ms, "forward_ms": fwd_ms, "adjoint_over_forward": adj_ms / fwd_ms,
            "loss": float(((img - target) ** 2).mean()),
            "roofline": roofline(2.0 * fwd_fl, adj_ms),
            "memory": "no per-path buffer: the replay runs in the lane that traced the path"}


def batch_measurement(torch, gpss, tune: bool):
    """64 sphere scenes of uneven resolution, spp and lengthscale: one persistent
    hipGraph-captured launch (tile and grid from the autotuner unless tune is False) against
    64 sequential plain launches (same images); median of 10 after 3 warm-ups each."""
    from gpss_inputs import scenes as sc
    from paper_2603_00280_amd import flops
    scenes = sc.batch_scenes()
    gs = [gpss.GpssScene(s) for s in scenes]
    outs = [torch.empty(g.shape, dtype=torch.float32, device="cuda") for g in gs]
    plain = [torch.empty(g.shape, dtype=torch.float32, device="cuda") for g in gs]
    npaths = sum(s.n_paths for s in scenes)
    fl = sum(forward_flops(gpss, flops, torch, s, g) for s, g in zip(scenes, gs))
    tuned = None
    if tune:
        tuned = gpss.gpss_batch_autotune([g.handle for g in gs], [o.data_ptr() for o in outs])
    batch_ms, _ = median_ms(torch, lambda: gpss.render_batch(gs, outs))

    def seq():
        for g, o in zip(gs, plain):
            g.render(out=o)
    plain_ms, _ = median_ms(torch, seq)
    torch.cuda.synchronize()
    same = all(bool(torch.equal(a, b)) for a, b in zip(outs, plain))
    return {"workload": "64 sphere scenes, resolution {64..512}^2, spp {4,16,64}, lengthscale "
                        "log-uniform [0.005, 0.5], max depth 32", "paths": npaths,
            "batch_mpaths_s": npaths / (batch_ms / 1e3) / 1e6,
            "plain_sequential_mpaths_s": npaths / (plain_ms / 1e3) / 1e6,
            "batch_ms": batch_ms, "plain_ms": plain_ms, "images_identical": same, "tuning": tuned,
            "roofline": roofline(fl, batch_ms)}


def secondary_rows():
    """Workloads measured beside the headline: the sphere lengthscale sweep and the rows built
    beyond the plain method, each at the sphere workload's launch (512^2, 64 spp, depth 32)."""
    from gpss_inputs import scenes as sc
    return {
        "sphere_sweep": ("sphere: " + WORKLOADS["sphere"], lambda: [sc.sphere_scene(l) for l in sc.SPHERE_LENGTHSCALES]),
        "anisotropic": ("sphere, alpha 0.8 across the normal and 0.01 along it (l_n = sqrt(2) sigma / 0.01)",
                        lambda: [sc.aniso_sphere_scene(0.01)]),
        "ggx": ("sphere, variance 1e-4, GGX macrofacet with alpha 0.1 / 0.5 / 1.0",
                lambda: [sc.ggx_sphere_scene(a) for a in sc.GGX_ALPHAS]),
        "fresnel": ("sphere l = 0.1 as three colour channels, gold conductor IOR per channel",
                    lambda: sc.fresnel_rgb_scenes(sc.sphere_scene(0.1), "gold")),
        "conditioned": ("cond: " + WORKLOADS["cond"], lambda: [sc.cond_sphere_scene()]),
    }


CPU_SPP = {"mixed": 24, "sphere": 48, "plane": 4096, "cond": 16}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="mixed", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-spp", type=int, default=0,
                    help="spp of the oracle CPU sample (default: about 10-20 s of the workload on 16 cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel", default="auto", choices=["auto", "persistent", "mega", "wavefront"],
                    help="tracer form timed for the headline value")
    ap.add_argument("--compare", action="store_true",
                    help="also time one step of the other tracer forms")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint measurement on the offset-sphere workload")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-render measurement on the 64-scene workload")
    ap.add_argument("--no-mse", action="store_true",
                    help="skip the image MSE against the oracle on sampled pixels")
    ap.add_argument("--no-rows", "--no-next", "--no-cond", dest="no_rows", action="store_true",
                    help="skip the secondary rows (sphere sweep, anisotropic, GGX, Fresnel, conditioned)")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the batch with the cached or default tiles instead of running the autotuner")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run one plain device copy of BYTES (traffic calibration) and exit")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write the traffic profile from four rocprofv3 --pmc output directories and exit")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("KERNEL_TRACE_DIR", "BENCH_JSON"),
                    help="write the kernel-trace profile of a rocprofv3 --kernel-trace --stats bench run and exit")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="write the SQ-counter profile from rocprofv3 --pmc output directories; the last "
                         "directory is the kernel trace of the default run (launch times); then exit")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--commands", nargs="*", default=[], help="commands recorded in a profile summary")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(args.workload, *args.summarize_traffic, args.copy_bytes, args.commands)
        return
    if args.summarize_trace:
        summarize_trace(args.workload, *args.summarize_trace, args.commands)
        return
    if args.summarize_counters:
        summarize_counters(args.workload, args.summarize_counters[:-1], args.summarize_counters[-1], args.commands)
        return
    if args.calibrate_copy:
        copy_calibration(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the renderer's paths would shard across GPUs by sample range; only one GPU is implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_00280_amd import flops, gpss

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    scenes = make_scenes(args.workload)
    gs = [gpss.GpssScene(s, kernel=args.kernel) for s in scenes]
    imgs = [torch.empty(s.height, s.width, dtype=torch.float32, device=dev) for s in scenes]
    stream = torch.cuda.current_stream()
    print(f"[bench] workload {args.workload}: {len(scenes)} scene(s), "
          f"{sum(s.n_paths for s in scenes) / 1e6:.1f} M paths per step", file=sys.stderr, flush=True)

    # algorithmic work per launch from the event counts (deterministic: same paths)
    work = []
    for s, g in zip(scenes, gs):
        _, cnt = g.render_paths(counters=True)
        torch.cuda.synchronize()
        c = gpss.counters_dict(cnt)
        work.append((flops.flops_from_counters(s, c), c))
    print("[bench] counters", [w[1] for w in work], file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        for g, im in zip(gs, imgs):
            g.render(out=im)
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    evs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for g, im in zip(gs, imgs):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            g.render(out=im)
            e1.record(stream)
            evs.append((e0, e1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    paths = args.steps * sum(s.n_paths for s in scenes)
    launch_ms = [a.elapsed_time(b) for a, b in evs]
    per_scene_ms = [sum(launch_ms[i::len(scenes)]) / args.steps for i in range(len(scenes))]
    traffic = None
    if args.kernel in ("auto", "persistent"):
        rec = recorded_traffic(args.workload)
        if rec:
            traffic = sum(rec) / len(rec)
    rl = roofline(sum(w[0] for w in work), sum(per_scene_ms), traffic)
    rl["avg_launch_ms"] = sum(launch_ms) / len(launch_ms)
    rl["flops_per_launch"] = [w[0] for w in work]
    result = {
        "metric": METRIC,
        "value": paths / wall / 1e6,
        "unit": "Mpaths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload + ": " + WORKLOADS[args.workload],
                   "paths_per_step": sum(s.n_paths for s in scenes),
                   "tracer": TRACERS[args.kernel]},
        "roofline": rl,
        "per_scene_mpaths_s": [s.n_paths / (ms / 1e3) / 1e6 for s, ms in zip(scenes, per_scene_ms)],
        "counters": [w[1] for w in work],
    }
    if not args.no_mse:
        print("[bench] image MSE against the oracle", file=sys.stderr, flush=True)
        result["image_mse"] = [image_mse(torch, s, im) for s, im in zip(scenes, imgs)]
    if args.compare:
        result["compare"] = {}
        for other in ("persistent", "wavefront", "mega"):
            if TRACERS[other] == TRACERS[args.kernel]:
                continue
            for g in gs:
                g.set_kernel(other)
            for g, im in zip(gs, imgs):   # warm-up (wavefront buffers are allocated here)
                g.render(out=im)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for g, im in zip(gs, imgs):
                g.render(out=im)
            torch.cuda.synchronize()
            result["compare"][TRACERS[other]] = sum(s.n_paths for s in scenes) / (time.perf_counter() - t0) / 1e6
    del gs, imgs
    if not args.no_rows:
        result["rows"] = {}
        for name, (label, make) in secondary_rows().items():
            if name == "sphere_sweep" and args.workload == "sphere":
                continue
            print(f"[bench] {name}", file=sys.stderr, flush=True)
            result["rows"][name] = row_measurement(torch, gpss, label, make())
    if not args.no_adjoint:
        print("[bench] adjoint", file=sys.stderr, flush=True)
        result["adjoint"] = adjoint_measurement(torch, gpss)
    if not args.no_batch:
        print("[bench] batch", file=sys.stderr, flush=True)
        result["batch"] = batch_measurement(torch, gpss, not args.no_tune)
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the CPU", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(scenes, args.cpu_spp or CPU_SPP[args.workload])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
