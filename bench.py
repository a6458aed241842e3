#!/usr/bin/env python3
"""Throughput benchmark of the GPSS forward renderer on one MI355X.

Workload (default "sphere"): the single-object sphere of the lengthscale sweep -- unit
sphere SDF mean, squared-exponential kernel variance 0.0025, lengthscales
{0.005, 0.02, 0.1, 0.5}, albedo 0.8, point light plus constant environment, pinhole
512x512, 64 spp, max depth 32.  One step renders all four lengthscales (4 x 16.78 M
paths) with the scenes already resident on the GPU.

Prints one JSON line: Mpaths/s, the roofline entry of the dominant kernel (algorithmic
FP32 FLOPs per launch / the launch time measured with HIP events on the render stream),
and the FP64 CPU oracle timed on a bounded sample of the same workload.
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
             "[1e-4,1e-2], lengthscale 0.03, 1024x1024, 256 spp, max depth 64",
    "cond": "unit-sphere SDF prior conditioned on 32 noisy point observations (Fibonacci directions, "
            "radii jittered +-0.08, value 0, noise 0.05 x variance), variance 0.0025, lengthscale 0.25, "
            "pinhole 512x512, 64 spp, max depth 32",
}


# HBM traffic of the render kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by
# the same counters on a plain copy (see --summarize-traffic); valid only while the kernel
# sources hash to the recorded value.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sched_render_kernel_sphere_traffic.md")
KERNEL_SOURCES = ["gpss_sched.hpp", "gpss_persistent.hip", "gpss_trace.hpp", "gpss_device.hpp", "gpss_waves.hpp"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2603_00280_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recorded_traffic():
    """Bytes of HBM traffic per render launch recorded for the current kernel, else None."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
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


def summarize_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, commands):
    """Write TRAFFIC_FILE from four rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE of the
    bench render and of the plain-copy calibration), each a directory of counter CSVs."""
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
    with open(TRAFFIC_FILE, "w") as f:
        f.write("# HBM traffic of sched_render_kernel on the sphere sweep\n\n")
        f.write("Counters per dispatch of the forward render kernel (launches of the sphere sweep in\n"
                "bench order: warm-up and timed renders of the four lengthscales), in KiB, from\n"
                "separate rocprofv3 runs:\n\n")
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
    print(open(TRAFFIC_FILE).read())


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


def image_mse(torch, gs, scenes, imgs, factor: int = 16):
    """MSE of each timed image (samples [0, spp)) against an independent reference of the same
    scene at factor x spp (samples [spp, (1 + factor) spp)).  The GPU matches the oracle path by
    path, so the reference stands in for a high-spp oracle image; every form (persistent,
    wavefront, one thread per path, batch) gives the same image and hence the same MSE."""
    out = []
    for g, s, im in zip(gs, scenes, imgs):
        ref = g.render(s.spp, (1 + factor) * s.spp)
        torch.cuda.synchronize()
        out.append(float(((im - ref) ** 2).mean()))
    return {"reference": f"same scene, samples [spp, {1 + factor} spp)", "per_scene": out}


def next_row_scenes():
    """Workloads of the rows built beyond the plain method, each at the sphere workload's
    launch (512^2, 64 spp, depth 32)."""
    from gpss_inputs import scenes as sc
    return {
        "anisotropic": ("sphere, alpha 0.8 across the normal and 0.01 along it (l_n = sqrt(2) sigma / 0.01)",
                        [sc.aniso_sphere_scene(0.01)]),
        "ggx": ("sphere, variance 1e-4, GGX macrofacet with alpha 0.1 / 0.5 / 1.0",
                [sc.ggx_sphere_scene(a) for a in sc.GGX_ALPHAS]),
        "fresnel": ("sphere l = 0.1 as three colour channels, gold conductor IOR per channel",
                    sc.fresnel_rgb_scenes(sc.sphere_scene(0.1), "gold")),
        "conditioned": ("cond: " + WORKLOADS["cond"], [sc.cond_sphere_scene()]),
    }


def row_measurement(torch, gpss, label: str, scenes, steps: int = 2):
    """Mpaths/s of one row's workload and the roofline entry of its render kernel (algorithmic
    FLOPs / launch time on the render stream, summed over the row's scenes)."""
    from paper_2603_00280_amd import flops
    gs = [gpss.GpssScene(s) for s in scenes]
    imgs = [torch.empty(s.height, s.width, dtype=torch.float32, device="cuda") for s in scenes]
    fl = 0.0
    for s, g in zip(scenes, gs):
        _, cnt = g.render_paths(counters=True)
        torch.cuda.synchronize()
        fl += flops.flops_from_counters(s, gpss.counters_dict(cnt))
    for g, im in zip(gs, imgs):
        g.render(out=im)
    stream = torch.cuda.current_stream()
    evs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for g, im in zip(gs, imgs):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            g.render(out=im)
            e1.record(stream)
            evs.append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = sum(a.elapsed_time(b) for a, b in evs) / steps
    rate = fl / (ms / 1e3) / 1e12
    n = sum(s.n_paths for s in scenes)
    return {"workload": label, "value": steps * n / wall / 1e6, "unit": "Mpaths/s", "ms_per_pass": ms,
            "roofline": {"bound": "alu", "achieved": rate, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": rate / FP32_PEAK_TFLOPS, "traffic": None, "flops_per_pass": fl}}


def adjoint_measurement(torch, gpss):
    """Path-replay adjoint of the L2 image loss on the offset-sphere workload (256^2, 16 spp,
    depth 16, 64^3 mean-offset grid) at theta0 against the target image; a path counts once
    although it is traced and replayed."""
    from gpss_inputs import scenes as sc
    s0, st = sc.offset_sphere_scene(False), sc.offset_sphere_scene(True)
    target = gpss.GpssScene(st).render()
    g = gpss.GpssScene(s0)
    img = g.render()
    dl = (2.0 * (img - target) / img.numel()).contiguous()
    g.render_adjoint(dl)      # warm-up
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    res = {}
    for name, fn in (("forward", lambda: g.render(out=img)), ("adjoint", lambda: g.render_adjoint(dl))):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1)
    return {"workload": "offset sphere: 64^3 mean-offset grid, 256x256, 16 spp, max depth 16, "
                        "L2 loss against the seeded target",
            "adjoint_mpaths_s": s0.n_paths / (res["adjoint"] / 1e3) / 1e6,
            "forward_mpaths_s": s0.n_paths / (res["forward"] / 1e3) / 1e6,
            "adjoint_ms": res["adjoint"], "forward_ms": res["forward"],
            "loss": float(((img - target) ** 2).mean())}


def batch_measurement(torch, gpss, tune: bool):
    """64 sphere scenes of uneven resolution, spp and lengthscale: one persistent
    hipGraph-captured launch against 64 sequential plain launches (same images)."""
    from gpss_inputs import scenes as sc
    scenes = sc.batch_scenes()
    gs = [gpss.GpssScene(s) for s in scenes]
    outs = [torch.empty(g.shape, dtype=torch.float32, device="cuda") for g in gs]
    plain = [torch.empty(g.shape, dtype=torch.float32, device="cuda") for g in gs]
    npaths = sum(s.n_paths for s in scenes)
    tuned = None
    if tune:
        tuned = gpss.gpss_batch_autotune([g.handle for g in gs], [o.data_ptr() for o in outs])
    gpss.render_batch(gs, outs)             # plan + graph capture
    for g, o in zip(gs, plain):
        g.render(out=o)                      # warm-up of the single-scene path
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gpss.render_batch(gs, outs)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    for g, o in zip(gs, plain):
        g.render(out=o)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    same = all(bool(torch.equal(a, b)) for a, b in zip(outs, plain))
    return {"workload": "64 sphere scenes, resolution {64..512}^2, spp {4,16,64}, lengthscale "
                        "log-uniform [0.005, 0.5], max depth 32", "paths": npaths,
            "batch_mpaths_s": npaths / t_batch / 1e6, "plain_sequential_mpaths_s": npaths / t_plain / 1e6,
            "batch_ms": t_batch * 1e3, "plain_ms": t_plain * 1e3, "images_identical": same,
            "tuning": tuned}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-spp", type=int, default=48, help="spp of the oracle CPU sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel", default="auto", choices=["auto", "persistent", "mega", "wavefront"],
                    help="tracer form timed for the headline value")
    ap.add_argument("--compare", action="store_true",
                    help="also time one step of the other tracer form")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint measurement on the offset-sphere workload")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-render measurement on the 64-scene workload")
    ap.add_argument("--no-mse", action="store_true",
                    help="skip the image MSE against a 16x-spp reference of each scene")
    ap.add_argument("--no-cond", "--no-next", dest="no_next", action="store_true",
                    help="skip the measurements of the anisotropic, GGX, Fresnel and conditioned rows")
    ap.add_argument("--tune", action="store_true",
                    help="run the batch autotuner first (its choice is cached on disk)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run one plain device copy of BYTES (traffic calibration) and exit")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="write the traffic profile from four rocprofv3 --pmc output directories and exit")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--commands", nargs="*", default=[], help="commands recorded in the traffic profile")
    args = ap.parse_args()
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic, args.copy_bytes, args.commands)
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
    # roofline of the render kernel: algorithmic FLOPs of each launch / its duration
    flop_rate = sum(w[0] for w in work) / (sum(per_scene_ms) / 1e3)
    traffic = None
    if args.workload == "sphere" and args.kernel in ("auto", "persistent"):
        rec = recorded_traffic()
        if rec:
            traffic = sum(rec) / len(rec)
    avg_launch_ms = sum(launch_ms) / len(launch_ms)
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
        "roofline": {"bound": "alu", "achieved": flop_rate / 1e12, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": flop_rate / 1e12 / FP32_PEAK_TFLOPS, "traffic": traffic,
                     "avg_launch_ms": avg_launch_ms,
                     "flops_per_launch": [w[0] for w in work]},
        "per_scene_mpaths_s": [s.n_paths / (ms / 1e3) / 1e6 for s, ms in zip(scenes, per_scene_ms)],
    }
    if not args.no_mse:
        result["image_mse"] = image_mse(torch, gs, scenes, imgs)
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
    if not args.no_adjoint:
        print("[bench] adjoint", file=sys.stderr, flush=True)
        result["adjoint"] = adjoint_measurement(torch, gpss)
    if not args.no_next and args.workload == "sphere":
        result["next_rows"] = {}
        for name, (label, row_scenes) in next_row_scenes().items():
            print(f"[bench] {name}", file=sys.stderr, flush=True)
            result["next_rows"][name] = row_measurement(torch, gpss, label, row_scenes)
            del row_scenes
    if not args.no_batch:
        print("[bench] batch", file=sys.stderr, flush=True)
        result["batch"] = batch_measurement(torch, gpss, args.tune)
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on the CPU", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(scenes, args.cpu_spp)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
