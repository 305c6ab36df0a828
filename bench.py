"""Benchmark of the line radiative-transfer ray march on one MI355X.

A step is one full-size forward render: 512 x 512 pixels x 64 channels x 512
samples per ray through a 256 x 128 (r, z/r) disk (seeded parametric disk
with three density gaps), inputs resident in HBM.  Prints one JSON line with
ray-samples/s, the roofline of the dominant kernel (the forward march), the
forward rate over eight seeded disks of the family, the forward+adjoint rate
at 256 x 256 x 48 x 256 and at full size, the served stream (latency and
capacity against one request at a time), and the FP64 oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X unit counts and clock: 256 CUs, each issuing 128 FP32 VALU lanes per
# clock (4 SIMDs x 32 lanes: the published 157.3 TFLOP/s FP32 vector rate is
# 256 x 128 x 2 FLOP x 2.4 GHz, reached by unpacked v_fma_f32), i.e. 7.86e13
# lane-instructions per second; a transcendental (exp2, log2, rcp, rsq,
# sqrt) runs at a quarter of that rate, i.e. takes 4 issue slots.
LANE_SLOTS_PER_S = 256 * 128 * 2.4e9
TRANS_SLOTS = 4
# Algorithmic work of one ray-sample in the channel loop: d = a - v b (FMA),
# x = K 2^-d^2 = 2^(log2 K - d^2) (FMA + exp2), att = 2^-x, 1 - att,
# Tr (1 - att), I += . S (FMA), Tr *= att  ->  11 FLOP (FMA = 2,
# transcendental = 1) in 6 VALU + 2 TRANS.  On an optically thin sample
# (line-centre depth below the series threshold) 1 - 2^-x comes from its
# cubic series instead of the second exp2: d (FMA), x (FMA + exp2), series
# (2 FMA + mul), t = Tr (1 - att), I += t S (FMA), Tr -= t  ->  14 FLOP in
# 8 VALU + 1 TRANS.  The census of each render gives the thin share.
LOOP_FLOP, LOOP_VALU, LOOP_TRANS = 11, 6, 2
THIN_FLOP, THIN_VALU, THIN_TRANS = 14, 8, 1
# Channel-independent shading of one pixel-sample, shared by the channels of
# a lane: position, grid fetch and bilinear interpolation, density, CO mask,
# partition function, populations, source function, width, projected
# velocity, log2 of the line-centre depth.
SHADE_FLOP, SHADE_VALU, SHADE_TRANS = 151, 100, 15
# The 3-D march's shading of one pixel-sample (spherical coordinates, radial
# refinement, two atan2, trilinear fetch of six fields, physics, projected
# velocity), counted in the compiled sample loop of march3_fwd<24, 4>: 307
# VALU + 16 transcendental = 371 issue slots, shared by a lane's channels.
SHADE3_SLOTS = 307 + 4 * 16


# HBM traffic of one forward launch on the full-size render of each disk,
# from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch)
# of `bench.py --copy-probe`, each scaled by what the same counter reads for
# a 1 GiB device-to-device copy (FETCH_SIZE 524 303 KiB -> x2.0000,
# WRITE_SIZE 1 048 576 KiB -> x1.0000).  Valid only for the kernel sources it
# was taken on: the hash of those files is checked at run time.
FWD_TRAFFIC = {"sources": ("paper_2509_03623_amd/csrc/rt_forward.hip", "paper_2509_03623_amd/csrc/rt_kernels.h",
                           "paper_2509_03623_amd/csrc/rt_launch.h"),
               "sha256": "6ea039cd02742bf7d552e6ef90fd250c8277a33ca373562feed8ec088c478f49",
               "fetch_scale": 1048576 / 524302.5, "write_scale": 1.0,
               # seed -> (FETCH_SIZE KiB, WRITE_SIZE KiB), mean of three launches each
               "disks": {2000: (1196.8, 65536.0), 2001: (1184.7, 65536.0), 2002: (1343.3, 65536.0), 2003: (1291.7, 65536.0), 2004: (1150.5, 65536.0), 2005: (1193.9, 65536.0), 2006: (1309.5, 65536.0), 2007: (1454.9, 65536.0)}}


def measured_traffic(seed: int):
    """HBM bytes per forward launch of disk `seed`, or None if the kernel has
    changed since the counters were taken (or none were taken for it)."""
    import hashlib
    if seed not in FWD_TRAFFIC["disks"]:
        return None
    h = hashlib.sha256()
    for f in FWD_TRAFFIC["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != FWD_TRAFFIC["sha256"]:
        return None
    fetch_kib, write_kib = FWD_TRAFFIC["disks"][seed]
    return 1024.0 * (fetch_kib * FWD_TRAFFIC["fetch_scale"] + write_kib * FWD_TRAFFIC["write_scale"])


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic(nch: int, cb: int, thin: float = 0.0, emit: float = 1.0, shaded: float = 1.0):
    """(FLOP per ray-sample, issue slots per ray-sample) of the march: the
    shading of the share `shaded` of the pixel-samples inside the grid's
    edge taper (shared by the cb channels that use it; the others stop
    after locating the sample, not counted) and the channel loop on the
    share `emit` with any opacity, `thin` of those on the series form.  A
    sample with K = 0 changes no channel: the march skips its channel loop
    wherever no ray of the wave has opacity at that sample, so only the
    samples with opacity are counted as loop work (a lower bound on what the
    lanes execute)."""
    flop = emit * ((1.0 - thin) * LOOP_FLOP + thin * THIN_FLOP) + shaded * SHADE_FLOP / cb
    slots = (emit * ((1.0 - thin) * (LOOP_VALU + TRANS_SLOTS * LOOP_TRANS) +
                     thin * (THIN_VALU + TRANS_SLOTS * THIN_TRANS)) +
             shaded * (SHADE_VALU + TRANS_SLOTS * SHADE_TRANS) / cb)
    return flop, slots


def time_forward(rt, sc, cube, steps, warmup):
    """Wall-clock and HIP-event (launch stream) milliseconds per forward
    render of scene sc: `warmup` untimed steps, then `steps` timed with
    Python's collector held off."""
    import torch
    for _ in range(warmup):
        rt.render(sc, out=cube)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    gc.collect()
    gc.disable()
    try:
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            rt.render(sc, out=cube)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        gc.enable()
    return wall * 1e3 / steps, e0.elapsed_time(e1) / steps


def micro_rates(L):
    """Issue rates of the march's instruction classes on this GPU
    (rt_microbench, register-only kernels on every CU)."""
    import ctypes as C
    lib = L.lib()
    lib.rt_microbench.argtypes = [C.c_int32, C.c_int64, C.POINTER(C.c_double)]
    lib.rt_microbench.restype = C.c_int32
    kinds = {"fma_lane_ops_per_s": (0, 20000), "exp2_lane_ops_per_s": (1, 5000), "rcp_lane_ops_per_s": (2, 5000),
             "log2_lane_ops_per_s": (3, 5000), "exp_fma_lane_ops_per_s": (6, 5000),
             "loop_thick_ray_samples_per_s": (4, 2000), "loop_thin_ray_samples_per_s": (5, 2000)}
    out = {}
    for name, (k, iters) in kinds.items():
        v = C.c_double()
        if lib.rt_microbench(k, iters, C.byref(v)) == 0:
            out[name] = v.value
    return out


def auto_shape(nch: int, npix: int, nsamp: int):
    """The library's automatic (channel block, ray split) of the forward
    march (same rule as its host code)."""
    cb = next((c for c in (8, 16, 24, 32, 48, 64) if c >= nch), 64)
    waves = lambda c, ns: ((npix * ns + 63) // 64) * ((nch + c - 1) // c)
    if cb == 64 and waves(64, 1) < 4096:
        cb = 32
    max_split = 1 if cb >= 64 else (4 if cb >= 48 else 8)
    ns = 1
    while ns < max_split and waves(cb, ns) < 4096 and nsamp >= 32 * ns:
        ns *= 2
    return cb, ns


def auto_shape3(nch: int, npix: int, nsamp: int):
    """The library's automatic (channel block, ray split) of the 3-D march."""
    cb = next((c for c in (8, 16, 24, 32, 48, 64) if c >= nch), 64)
    waves = lambda ns: ((npix * ns + 63) // 64) * ((nch + cb - 1) // cb)
    ns = 2 if nsamp >= 128 else 1
    while ns < 8 and waves(2 * ns) <= 1024 and nsamp >= 128 * ns:
        ns *= 2
    return cb, ns


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(prob, live, seconds, nthreads, seed):
    """(ray-samples/s, pixels, crossing pixels, seconds) of the FP64 oracle on
    seeded random pixels of the workload for about `seconds`."""
    import numpy as np
    import oracle
    nx, ny = prob.camera.nx, prob.camera.ny
    rng = np.random.Generator(np.random.PCG64(seed))
    per_pix = prob.nch * prob.nsamp
    n = 16 if nthreads == 1 else 256
    t_used = 0.0
    done = done_live = 0
    while t_used < seconds:
        px = rng.integers(0, nx, n)
        py = rng.integers(0, ny, n)
        t0 = time.perf_counter()
        oracle.render_pixels(prob, px, py, nthreads=nthreads)
        dt = time.perf_counter() - t0
        t_used += dt
        done += n
        done_live += int(live[py, px].sum())
        n = int(min(max(n * 2, 8), max(8, n * (seconds - t_used) / max(dt, 1e-3))))
        if t_used >= seconds or n < 8:
            break
    return done_live * per_pix / t_used, done, done_live, t_used


def cpu_baseline(prob, live, seconds=12.0, disk=None):
    """FP64 oracle on seeded pixels of the same workload, on all host cores
    and on one; live: [ny, nx] mask of the rays that cross the grid (the
    others have no samples and are not counted)."""
    ncores = os.cpu_count() or 1
    v, done, done_live, t_used = _oracle_rate(prob, live, seconds, ncores, 99)
    v1, done1, live1, t1 = _oracle_rate(prob, live, max(2.0, seconds / 2), 1, 98)
    per_pix = prob.nch * prob.nsamp
    return dict(value=v, unit="ray-samples/s", cores=ncores, kind="oracle",
                sample=f"{done} seeded random pixels ({done_live} crossing the grid) of the 512x512x64ch "
                       f"x512-sample disk {disk} ({done_live * per_pix:.3g} ray-samples, {t_used:.1f} s, FP64 scalar "
                       f"C, OpenMP)",
                value_1core=v1,
                sample_1core=f"{done1} seeded random pixels ({live1} crossing) on one thread, {t1:.1f} s",
                cpu_model=cpu_model())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--seed", type=int, default=2000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--one-disk", action="store_true",
                    help="time only disk --seed instead of the median over the eight seeded disks")
    ap.add_argument("--no-mlp", action="store_true", help="skip the neural CO layer leg")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3-D spherical-grid leg")
    ap.add_argument("--no-beam", action="store_true", help="skip the beam-convolution leg")
    ap.add_argument("--only", choices=("render3d", "beam", "adjoint", "mlp"), default=None,
                    help="run one leg alone and print its JSON (for profiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 1 GiB device to device three times (a kernel of known traffic, to scale "
                         "hardware byte counters)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson request trace (200 req/s) for the serving leg; 0 = skip")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the renderer is a single-GPU build (rays are independent, "
              "so more GPUs would each render their own pixel tiles); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_2509_03623_amd as rt
    from paper_2509_03623_amd import _lib as L

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        src = torch.ones(1 << 28, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only == "render3d":
        print(json.dumps({"render3d": bench_render3d(rt, dev, args)}), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps({"fwd_adjoint": bench_adjoint(rt, synth, dev, args)}), flush=True)
        return
    if args.only == "mlp":
        print(json.dumps({"neural": bench_mlp(rt, synth, dev, args)}), flush=True)
        return
    if args.only == "beam":
        prob = synth.config2(args.seed)
        sc = rt.scene_from_problem(prob, device=dev)
        cube = rt.render(sc)
        print(json.dumps({"beam": bench_beam(rt, cube, args)}), flush=True)
        return
    # the full-size render of each of the eight seeded disks of the family,
    # each timed alike; the headline is the median rate
    seeds = [args.seed] if args.one_disk else list(range(2000, 2008))
    per_seed = {}
    scenes = {}
    cube = None
    for sd in seeds:
        prob_sd = synth.config2(sd)
        sc_sd = rt.scene_from_problem(prob_sd, device=dev)
        if cube is None:
            cube = torch.empty(sc_sd.nch, sc_sd.ny, sc_sd.nx, device=dev)
        cen = sc_sd.census()
        wall_ms, kern_ms_sd = time_forward(rt, sc_sd, cube, args.steps, args.warmup)
        rs_sd = sc_sd.ray_samples
        # samples with opacity; those without count as thin in the census
        n_all, n_em = cen["pixel_samples"], cen["emitting_pixel_samples"]
        n_thin_em = cen["thin_pixel_samples"] - (n_all - n_em)
        per_seed[sd] = dict(ray_samples_per_s=rs_sd / (wall_ms * 1e-3), ms_per_step=wall_ms, kernel_ms=kern_ms_sd,
                            ray_samples=rs_sd, live_fraction=cen["rays"] / (sc_sd.nx * sc_sd.ny),
                            emitting_fraction=n_em / max(n_all, 1),
                            shaded_fraction=cen["shaded_pixel_samples"] / max(n_all, 1),
                            emitting_ray_samples_per_s=n_em * sc_sd.nch / (wall_ms * 1e-3),
                            thin_fraction=n_thin_em / max(n_em, 1),
                            incl_deg=prob_sd.camera.incl_deg)
        scenes[sd] = (prob_sd, sc_sd)
        log(f"disk {sd}: {wall_ms:.3f} ms/step (kernel {kern_ms_sd:.3f} ms), "
            f"{per_seed[sd]['ray_samples_per_s']:.3e} ray-samples/s "
            f"({per_seed[sd]['emitting_fraction']:.3f} of them with opacity: "
            f"{per_seed[sd]['emitting_ray_samples_per_s']:.3e}/s)")
    rates = np.array([per_seed[sd]["ray_samples_per_s"] for sd in seeds])
    value = float(np.median(rates))
    # the disk at the median (the lower of the two middle ones) carries the roofline
    med = seeds[int(np.argsort(rates)[(len(seeds) - 1) // 2])]
    prob, sc = scenes[med]
    ms_per_step = float(np.median([per_seed[sd]["ms_per_step"] for sd in seeds]))
    kern_ms = per_seed[med]["kernel_ms"]
    rs = per_seed[med]["ray_samples"]
    thin = per_seed[med]["thin_fraction"]
    emit = per_seed[med]["emitting_fraction"]
    shaded = per_seed[med]["shaded_fraction"]
    cb, split = auto_shape(sc.nch, sc.nx * sc.ny, sc.nsamp)
    cb = rt.get_option(L.RT_OPT_CHANNEL_BLOCK) or cb
    split = rt.get_option(L.RT_OPT_RAY_SPLIT) or split
    # 64-channel blocks on one lane per pixel run on a group of lanes per
    # pixel (uniform channels; 4 lanes unless set)
    group = rt.get_option(L.RT_OPT_FWD_GROUP) or 4
    kname = f"march_fwd_group<{group}>" if cb == 64 and split == 1 and group > 1 else "march_fwd"
    flop, slots = algorithmic(sc.nch, cb, thin, emit, shaded)
    achieved = flop * rs / (kern_ms * 1e-3) / 1e12
    peak = flop / slots * LANE_SLOTS_PER_S / 1e12
    out = {
        "metric": "ray-samples/s fwd & fwd+adjoint at 512^2x64ch; p50/p99 served latency",
        "value": value,
        "unit": "ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "forward render 512x512 px x 64 ch x 512 samples/ray, 256x128 (r,z/r) grid, "
                               f"median over the seeded disks {seeds[0]}-{seeds[-1]} (3 gaps each; "
                               f"roofline on disk {med}, incl {prob.camera.incl_deg:.1f} deg)",
                   "global_batch": 1, "ray_samples": rs, "live_fraction": per_seed[med]["live_fraction"],
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": measured_traffic(med),
                     "kernel": kname, "kernel_ms": kern_ms, "disk": med,
                     "emitting_fraction": emit, "thin_fraction_of_emitting": thin, "shaded_fraction": shaded,
                     "flop_per_ray_sample": flop, "issue_slots_per_ray_sample": slots,
                     "hbm_bytes_algorithmic": 4 * sc.nch * sc.nx * sc.ny + 4 * (3 * sc.nr * sc.nz + 2 * sc.nr)},
        "disks": {str(sd): v for sd, v in per_seed.items()},
    }
    log(f"forward median {ms_per_step:.3f} ms/step, {value:.3e} ray-samples/s")
    log("instruction-class issue rates")
    mr = micro_rates(L)
    if "loop_thick_ray_samples_per_s" in mr and "loop_thin_ray_samples_per_s" in mr:
        # the march's measured mix: the channel loop at its measured rates
        # (thin share on the series form) plus the shading's issue slots
        sh = shaded * (SHADE_VALU + TRANS_SLOTS * SHADE_TRANS) / cb / LANE_SLOTS_PER_S
        t_rs = emit * ((1.0 - thin) / mr["loop_thick_ray_samples_per_s"] +
                       thin / mr["loop_thin_ray_samples_per_s"]) + sh
        mr["mix_roof_ray_samples_per_s"] = 1.0 / t_rs
        out["roofline"]["frac_of_measured_mix"] = (rs / (kern_ms * 1e-3)) * t_rs
    out["micro"] = mr
    if not args.no_mlp:
        log("neural CO layer")
        out["neural"] = bench_mlp(rt, synth, dev, args)
    if not args.no_beam:
        log("beam convolution of the full-size cube")
        out["beam"] = bench_beam(rt, cube, args)
    if not args.no_3d:
        log("3-D spherical grid 512x96x256 (channel and image-size sweeps)")
        out["render3d"] = bench_render3d(rt, dev, args)
    if not args.no_adjoint:
        log("forward + adjoint")
        try:
            out["fwd_adjoint"] = bench_adjoint(rt, synth, dev, args)
        except rt.RtError as e:
            out["fwd_adjoint"] = {"error": str(e)}
        out["derived_fields"] = bench_derived(rt, synth, dev, args)
        log("neural-temperature fitting step")
        out["neural_t_fit"] = bench_fit(rt, synth, dev, args)
        log("ensemble-sampler iteration (60 walkers)")
        out["walkers"] = bench_walkers(rt, synth, dev, args)
    if args.serve_seconds > 0:
        log(f"served stream ({args.serve_seconds:g} s trace, then the serial replay and the saturated runs)")
        out["served"], out["serial"], out["saturated"] = bench_serving(rt, synth, dev, args.serve_seconds)
        out["served_vs_serial_throughput"] = (out["saturated"]["served_ray_samples_per_s"] /
                                              out["saturated"]["serial_ray_samples_per_s"])
    if not args.no_cpu:
        log("oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(prob, sc.live_mask(), args.cpu_seconds, disk=med)
    print(json.dumps(out), flush=True)


def bench_render3d(rt, dev, args):
    """Forward march over a seeded non-axisymmetric disk on the 512 x 96 x 256
    spherical grid of the paper's runtime benchmark, 512 samples per ray:
    256^2 pixels at 20, 64 and 128 channels, and 20 channels at 128^2, 256^2
    and 512^2 pixels.  The node packing (six planes -> interleaved records,
    once per snapshot) is timed on its own.  Ray-samples count the samples of
    the rays that cross the bounding sphere (live_fraction of them; the
    others do no work); alu_frac credits the full shading of the samples
    inside the grid's fade and the channel loop of those with opacity only
    (the march skips the rest), from the census."""
    import numpy as np
    import torch
    from synth import disk3d as S3
    grid = S3.Grid3Spec(512, 96, 256)
    base = S3.make_problem3(grid, seed=65, nx=256, ny=256, nch=20, dv=0.25, nsamp=512, incl=40.0, pa=30.0)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=dev)
    planes = [t(a) for a in (base.ln_nh2, base.temp_k, base.x_co, base.v_r_kms, base.v_theta_kms, base.v_phi_kms)]
    sc0 = rt.scene3d_from_problem(base, device=dev)
    nodes = sc0.nodes
    steps = max(5, args.steps // 2)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        rt.pack_fields3d(sc0.grid, *planes, out=nodes)
    e1.record()
    torch.cuda.synchronize()
    pack_ms = e0.elapsed_time(e1) / steps
    out = {"grid": "512x96x256", "nsamp": 512, "pack_ms": pack_ms,
           "pack_gb_per_s": (24 + 32) * nodes.numel() / 8 / (pack_ms * 1e-3) / 1e9}
    legs = [("256x256x20ch", 256, 20), ("256x256x64ch", 256, 64), ("256x256x128ch", 256, 128),
            ("128x128x20ch", 128, 20), ("512x512x20ch", 512, 20)]
    for name, npx, nch in legs:
        sc = sc0.replace(nx=npx, ny=npx, v_kms=synth_channels(nch, 0.25))
        cube = torch.empty(nch, npx, npx, device=dev)
        for _ in range(2):
            rt.render3d(sc, out=cube)
        torch.cuda.synchronize()
        # no collector pause inside the short timed loop (one such pause, 1.2 ms
        # on the host, left the GPU idle and added 0.24 ms to a 5-call average)
        gc.collect()
        gc.disable()
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            rt.render3d(sc, out=cube)
        e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        gc.enable()
        kern = e0.elapsed_time(e1) / steps * 1e-3
        cen = sc.census()
        n_all, n_em, n_in = cen["pixel_samples"], cen["emitting_pixel_samples"], cen["shaded_pixel_samples"]
        live = cen["rays"] / (npx * npx)
        # samples without opacity count as thin in the census
        thin = (cen["thin_pixel_samples"] - (n_all - n_em)) / max(n_em, 1)
        cb, ns = auto_shape3(nch, npx * npx, 512)
        nchb = -(-nch // cb)
        loop = ((1.0 - thin) * (LOOP_VALU + TRANS_SLOTS * LOOP_TRANS) +
                thin * (THIN_VALU + TRANS_SLOTS * THIN_TRANS))
        # the channel loop of the samples with opacity and the full shading of
        # those inside the grid's fade, per channel block (the rest skipped)
        slots = nchb * (n_em * cb * loop + n_in * SHADE3_SLOTS)
        hbm = 24 * grid.nr * grid.nt * grid.nphi + 4 * nch * npx * npx
        out[name] = {"ms": wall * 1e3, "kernel_ms": kern * 1e3, "ray_samples_per_s": sc.ray_samples / wall,
                     "live_fraction": live, "emitting_fraction": n_em / max(n_all, 1),
                     "shaded_fraction": n_in / max(n_all, 1), "thin_fraction_of_emitting": thin,
                     "channel_block": cb, "ray_split": ns,
                     "alu_frac": slots / LANE_SLOTS_PER_S / kern, "hbm_frac": hbm / kern / 8e12}
        log(f"3-D {name}: {wall * 1e3:.3f} ms, {sc.ray_samples / wall:.3e} ray-samples/s")
    if not args.no_cpu:
        import oracle
        rng = np.random.Generator(np.random.PCG64(98))
        n = 2000
        px, py = rng.integers(0, 256, n).astype(np.int32), rng.integers(0, 256, n).astype(np.int32)
        nlive = int(sc0.live_mask()[py, px].sum())
        ncores = os.cpu_count() or 1
        t0 = time.perf_counter()
        oracle.render3_pixels(base, px, py, nthreads=ncores)
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"ray_samples_per_s": nlive * 20 * 512 / dt, "cores": ncores,
                             "sample": f"{n} seeded random pixels ({nlive} crossing the grid) of 256x256x20ch, "
                                       "FP64 scalar C, OpenMP"}
    return out


def bench_beam(rt, cube, args, beam=(6.0, 4.0, 30.0)):
    """The full-size cube (512^2 x 64) convolved with a 6 x 4 px beam at
    30 deg: (2R+1)^2 FMAs per output (R = 8), against the FP32 issue rate."""
    import math
    import torch
    out = torch.empty_like(cube)
    steps = max(5, args.steps // 2)
    for _ in range(2):
        rt.beam_convolve(cube, *beam, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    gc.collect()
    gc.disable()
    e0.record()
    for _ in range(steps):
        rt.beam_convolve(cube, *beam, out=out)
    e1.record()
    torch.cuda.synchronize()
    gc.enable()
    ms = e0.elapsed_time(e1) / steps
    R = math.ceil(3.0 * beam[0] / (2.0 * math.sqrt(2.0 * math.log(2.0))))
    fma = (2 * R + 1) ** 2 * cube.numel()
    return {"ms": ms, "beam_px": list(beam), "radius": R, "outputs_per_s": cube.numel() / (ms * 1e-3),
            "tflop_per_s": 2 * fma / (ms * 1e-3) / 1e12, "alu_frac": fma / LANE_SLOTS_PER_S / (ms * 1e-3),
            "hbm_gb_per_s": 8 * cube.numel() / (ms * 1e-3) / 1e9}


def synth_channels(nch, dv):
    import numpy as np
    return (np.arange(nch, dtype=np.float64) - (nch - 1) / 2.0) * dv


def bench_adjoint(rt, synth, dev, args):
    """Forward + adjoint of an L2 loss, on the 256 x 256 x 48 x 256 gradient
    case and the full-size 512 x 512 x 64 x 512 render: fused (one call: the
    reverse march forms dL/dI from its own forward sweep) and separate
    (forward render, loss in torch, adjoint)."""
    import torch
    out = {}
    want = ("ln_nh2", "temp_k", "z_lo_au", "z_up_au")
    for name, prob in (("256x256x48ch_256s", synth.config3()), ("512x512x64ch_512s", synth.config2(args.seed))):
        sc = rt.scene_from_problem(prob, device=dev)
        tgt = rt.render(sc.replace(z_up_au=sc.z_up_au * 1.05))
        steps = max(3, args.steps // 2)
        cube = torch.empty_like(tgt)

        def separate():
            c = rt.render(sc)
            dl = 2.0 * (c - tgt)
            return rt.render_adjoint(sc, dl, want=want)

        def fused():
            return rt.render_l2_adjoint(sc, tgt, want=want, cube_out=cube)

        res = {}
        for leg, step in (("fused", fused), ("separate", separate)):
            for _ in range(max(1, args.warmup // 2)):
                step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                step()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            res[leg] = {"ray_samples_per_s": sc.ray_samples / dt, "ms_per_step": dt * 1e3}
        out[name] = dict(res, steps=steps, grads="ln n_H2, T, z_lo, z_up")
    return out


def bench_derived(rt, synth, dev, args):
    """Fields derived from a temperature grid (hydrostatic density, column,
    CO surfaces, v_phi with the pressure term) on the 256 x 128 grid: forward
    and adjoint alone, and the temperature-fitting step at 256 x 256 x 48 x
    256 -- derive, fused render + L2 + adjoint, adjoint of the derivation --
    giving dL/dT through the derived fields and directly."""
    import numpy as np
    import torch
    prob = synth.config3()
    gs = prob.grid
    grid = (gs.nr, gs.nz, gs.r_min_au, gs.r_max_au, gs.zr_max)
    p = synth.disk.DiskParams()
    phys = rt.DiskPhysics(p.mstar_msun, p.mgas_msun, p.rc_au, p.gamma, synth.disk.MU_GAS, p.t_freeze_k, p.n_dissoc)
    T = torch.tensor(prob.temp_k, device=dev)
    sc = rt.scene_from_problem(prob, device=dev)
    d0 = rt.derive_fields(grid, T, phys)
    tgt = rt.render(sc.replace(**{k: d0[k] for k in ("ln_nh2", "vphi_kms", "z_lo_au")},
                               z_up_au=d0["z_up_au"] * 1.05))
    cube = torch.empty_like(tgt)
    want = ("ln_nh2", "temp_k", "vphi_kms", "z_lo_au", "z_up_au")

    def fit_step():
        d = rt.derive_fields(grid, T, phys)
        _, loss, g = rt.render_l2_adjoint(sc.replace(**d), tgt, want=want, cube_out=cube)
        return rt.derive_fields_adjoint(grid, T, phys, g, add_to=g["temp_k"])

    cot = {k: torch.ones_like(v) for k, v in d0.items()}
    legs = (("forward", lambda: rt.derive_fields(grid, T, phys)),
            ("adjoint", lambda: rt.derive_fields_adjoint(grid, T, phys, cot)),
            ("fit_step_256x256x48ch_256s", fit_step))
    out = {"grid": f"{gs.nr}x{gs.nz}"}
    for name, f in legs:
        steps = 50 if name != legs[-1][0] else max(3, args.steps // 2)
        for _ in range(3):
            f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            f()
        torch.cuda.synchronize()
        out[name + "_ms"] = (time.perf_counter() - t0) / steps * 1e3
    return out


def bench_fit(rt, synth, dev, args):
    """The neural-temperature fitting step of Methods, "Neural Temperature
    Recovery", at 256 x 256 px x 256 samples on a 115-channel cube (0.04 km/s),
    a random batch of 50 slices per step, chi^2 with sigma = 1.5 % of peak:
    network -> T, derived fields, fused render + L2 + adjoint on the batch,
    derived-field and network adjoints, Adam.  The target is the same disk's
    parametric temperature pushed through the derived fields."""
    import numpy as np
    import torch
    prob = synth.config3(nch=115, dv=0.04)
    gs = prob.grid
    grid = (gs.nr, gs.nz, gs.r_min_au, gs.r_max_au, gs.zr_max)
    p = synth.disk.DiskParams()
    phys = rt.DiskPhysics(p.mstar_msun, p.mgas_msun, p.rc_au, p.gamma, synth.disk.MU_GAS, p.t_freeze_k, p.n_dissoc)
    sc = rt.scene_from_problem(prob, device=dev)
    T_true = torch.tensor(prob.temp_k, device=dev)
    target = rt.render(sc.replace(temp_k=T_true, **rt.derive_fields(grid, T_true, phys)))
    sigma = 0.015 * float(target.abs().max())
    w = torch.tensor(synth.mlp.make_neural_t_weights(6), device=dev)
    opt = rt.Adam(w)
    rng = np.random.Generator(np.random.PCG64(7))
    batch = 50
    steps = max(5, args.steps // 2)
    chans = [np.sort(rng.choice(sc.nch, size=batch, replace=False)) for _ in range(steps + 2)]
    for t in range(2):
        rt.fit_step(sc, grid, phys, opt, target, chans[t], sigma, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chi2 = []
    for t in range(steps):
        c2, _ = rt.fit_step(sc, grid, phys, opt, target, chans[t + 2], sigma, rt.poly_lr(t, 30000))
        chi2.append(c2)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    rs = int(sc.live_mask().sum()) * batch * sc.nsamp
    return {"workload": "256x256 px, 115 ch (0.04 km/s), 256 samples, batch 50, 256x128 grid",
            "ms_per_step": dt * 1e3, "ray_samples_per_s": rs / dt, "steps": steps,
            "chi2_first": float(chi2[0].item()) / sigma ** 2, "chi2_last": float(chi2[-1].item()) / sigma ** 2}


def bench_walkers(rt, synth, dev, args, nwalk=60, iters=3):
    """One iteration of an ensemble sampler's likelihood evaluations (Methods,
    "MCMC inference": 60 walkers): per walker a two-layer parametric
    temperature and stellar mass perturbed around the truth, the derived fields
    on the device, and the render of 128 x 128 px x 32 ch x 256 samples with
    L = sum (cube - observed)^2 -- served as loss-only requests (batched into
    the persistent launch) against one at a time (render, then the loss);
    and the same with the model cube convolved with a beam before the loss."""
    import numpy as np
    import torch
    prob = synth.config2(2000, nx=128, ny=128, nch=32, nsamp=256)
    gs = prob.grid
    grid = (gs.nr, gs.nz, gs.r_min_au, gs.r_max_au, gs.zr_max)
    sc0 = rt.scene_from_problem(prob, device=dev)
    p = synth.disk.DiskParams()
    truth = np.array([30.0, 60.0, -0.5, 100.0, 70.0, 2.0, p.mstar_msun])

    def fields(th):
        T = rt.parametric_temperature(grid, *th[:6], device=dev)
        phys = rt.DiskPhysics(th[6], p.mgas_msun, p.rc_au, p.gamma, synth.disk.MU_GAS, p.t_freeze_k, p.n_dissoc)
        return dict(temp_k=T, **rt.derive_fields(grid, T, phys))

    observed = rt.render(sc0.replace(**fields(truth)))
    rng = np.random.Generator(np.random.PCG64(21))
    walkers = [truth * (1.0 + 0.05 * rng.standard_normal(truth.shape)) for _ in range(nwalk)]
    cubes = [torch.empty_like(observed) for _ in range(nwalk)]
    out = {"walkers": nwalk, "workload": "128x128 px x 32 ch x 256 samples per walker, 256x128 grid"}
    rs = sc0.ray_samples * nwalk
    with rt.Server(max_slots=nwalk, streams=4) as sv:
        def served():
            scs = [sc0.replace(**fields(th)) for th in walkers]
            torch.cuda.synchronize()
            ts = [sv.submit(sc, c, target=observed, loss_only=True) for sc, c in zip(scs, cubes)]
            return [sv.wait(t)["loss"] for t in ts]

        def serial():
            losses = []
            for th, c in zip(walkers, cubes):
                rt.render(sc0.replace(**fields(th)), out=c)
                losses.append(float(((c.double() - observed.double()) ** 2).sum()))
            return losses

        beam = (4.0, 3.0, 30.0)
        observed_b = rt.beam_convolve(observed, *beam)
        tmp = torch.empty_like(observed)

        def served_beam():
            scs = [sc0.replace(**fields(th)) for th in walkers]
            torch.cuda.synchronize()
            ts = [sv.submit(sc, c, target=observed_b, loss_only=True, beam=beam) for sc, c in zip(scs, cubes)]
            return [sv.wait(t)["loss"] for t in ts]

        def serial_beam():
            losses = []
            for th, c in zip(walkers, cubes):
                rt.render(sc0.replace(**fields(th)), out=tmp)
                rt.beam_convolve(tmp, *beam, out=c)
                losses.append(float(((c.double() - observed_b.double()) ** 2).sum()))
            return losses

        for name, f in (("served", served), ("serial", serial), ("served_beam", served_beam),
                        ("serial_beam", serial_beam)):
            f()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(iters):
                losses = f()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / iters
            out[name] = {"ms_per_iteration": dt * 1e3, "walkers_per_s": nwalk / dt, "ray_samples_per_s": rs / dt}
        out["best_walker_loss_over_truth_scale"] = float(min(losses) / float((observed.double() ** 2).sum()))
    out["served_vs_serial"] = out["served"]["walkers_per_s"] / out["serial"]["walkers_per_s"]
    out["beam"] = "4 x 3 px at 30 deg (model and observed cubes convolved; *_beam legs)"
    return out


def bench_mlp(rt, synth, dev, args):
    """Neural CO layer at 256 x 256 x 32 x 256: the network evaluated at every
    pixel-sample on the matrix cores, then the march; forward and
    forward + adjoint to the network weights, BF16 and FP32 paths."""
    import torch
    prob = synth.config4()
    out = {}
    for name, prec in (("bf16", rt.RT_MLP_BF16), ("fp32", rt.RT_MLP_FP32)):
        sc = rt.scene_from_problem(prob, device=dev, mlp_precision=prec)
        cube = torch.empty(sc.nch, sc.ny, sc.nx, device=dev)
        dl = torch.ones_like(cube)
        steps = max(3, args.steps // 4)
        res = {}
        for leg in ("forward", "forward_adjoint"):
            def step():
                if leg == "forward":
                    rt.render(sc, out=cube)
                else:
                    # one pass: the adjoint's own forward writes the cube
                    rt.render_adjoint(sc, dl, want=("temp_k", "mlp_w"), cube_out=cube)
            step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                step()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            res[leg] = {"ms": dt * 1e3, "ray_samples_per_s": sc.ray_samples / dt,
                        "network_evals_per_s": sc.nx * sc.ny * sc.nsamp / dt}
        out[name] = res
    return out


def bench_serving(rt, synth, dev, seconds, rate=200.0, seed=5, pool=16, saturated=600):
    """Served stream of the full-size disk family: each request one of `pool`
    pre-generated seeded disks with pixels in {64..512}^2, channels in
    {16..128}, 128-512 samples, 25% with forward+adjoint gradients of an L2
    loss.

    Open loop: Poisson arrivals at `rate` req/s for `seconds`, served by the
    continuous-batching server, then replayed one request at a time (FIFO) on
    the same arrival times: latency p50/p99 and ray-samples per second of
    makespan.  Saturated: the first `saturated` requests of the trace all
    submitted at once, served vs one at a time: the capacity of each."""
    import numpy as np
    import torch
    trace = synth.make_trace(rate_hz=rate, duration_s=seconds, seed=seed)
    bases = [rt.scene_from_problem(synth.config2(3000 + i, nx=64, ny=64, nch=16, nsamp=128), device=dev)
             for i in range(pool)]
    keys = ("ln_nh2", "temp_k", "z_lo_au", "z_up_au")
    targets, reqs = {}, []
    for r in trace:
        b = bases[r["disk_seed"] % pool]
        nch = r["nch"]
        v = (np.arange(nch) - (nch - 1) / 2.0) * 0.1
        sc = b.replace(nx=r["nx"], ny=r["ny"], v_kms=v, nsamp=r["nsamp"])
        key = (nch, r["ny"], r["nx"])
        if r["grad"] and key not in targets:
            targets[key] = torch.zeros(key, device=dev)
        # every gradient request writes gradients of its own
        g = {k: torch.empty_like(getattr(b, k)) for k in keys} if r["grad"] else None
        reqs.append((sc, key, g))
    torch.cuda.synchronize()

    def submit(sv, i):
        sc, key, g = reqs[i]
        cube = torch.empty(key, device=dev)
        if g is not None:
            return sv.submit(sc, cube, target=targets[key], grads=g)
        return sv.submit(sc, cube)

    def serial_one(i):
        # one request at a time with the library's direct calls: a render, or
        # the fused forward + L2 loss + adjoint (the single-request path the
        # server also takes for requests that fill the device)
        sc, key, g = reqs[i]
        if g is not None:
            rt.render_l2_adjoint(sc, targets[key], want=keys)
        else:
            rt.render(sc)
        torch.cuda.synchronize()

    def served_run(order, arrivals):
        # buffers the previous run left in torch's cache go back to the device,
        # so the server's own allocations meet the memory its budget assumes
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        with rt.Server(hbm_budget_bytes=96 << 30, max_slots=64, streams=4) as sv:
            first = submit(sv, order[0])
            sv.wait(first)
            sv.release(first)
            t0 = time.perf_counter()
            tickets, done, live = [], {}, []
            last = [t0]

            def reap():
                # finished requests hand their output cube back to torch's
                # cache as the trace goes, so a long trace holds only the
                # requests in flight
                still = []
                for t in live:
                    x = sv.poll(t)
                    if x["state"] in ("done", "canceled", "failed"):
                        done[t] = x
                        sv.release(t)
                    else:
                        still.append(t)
                live[:] = still

            for i, ta in zip(order, arrivals):
                while time.perf_counter() - t0 < ta:
                    time.sleep(2e-4)
                t = submit(sv, i)
                tickets.append(t)
                live.append(t)
                now = time.perf_counter()
                if now - last[0] > 2e-3:
                    reap()
                    last[0] = now
            for t in live:
                done[t] = sv.wait(t, timeout_s=300)
                sv.release(t)
        infos = [done[t] for t in tickets]
        for t, x in zip(tickets, infos):
            if x["state"] != "done":
                log(f"request {t} ended {x['state']} (status {x['status']})")
        t_sub = np.array([x["t_submit_ns"] for x in infos], dtype=np.float64)
        t_done = np.array([x["t_done_ns"] for x in infos], dtype=np.float64)
        return (t_done - t_sub) * 1e-6, (t_done.max() - t_sub.min()) * 1e-9, sum(x["state"] != "done" for x in infos)

    def serial_run(order, arrivals):
        lat = []
        t0 = time.perf_counter()
        for i, ta in zip(order, arrivals):
            now = time.perf_counter() - t0
            if now < ta:
                time.sleep(ta - now)
            serial_one(i)
            lat.append((time.perf_counter() - t0 - ta) * 1e3)
        return np.array(lat), time.perf_counter() - t0 - arrivals[0]

    for i in range(min(len(reqs), 32)):      # warm-up of the direct path
        serial_one(i)
    order = list(range(len(trace)))
    arrivals = [r["t_arrive"] - trace[0]["t_arrive"] for r in trace]
    total_rs = sum(sc.ray_samples for sc, _, _ in reqs)
    ngrad = sum(1 for r in trace if r["grad"])
    log(f"served run of {len(trace)} requests")
    lat, span, failed = served_run(order, arrivals)
    log(f"served: makespan {span:.2f} s; serial replay")
    served = {"ray_samples_per_s": total_rs / span, "p50_ms": float(np.percentile(lat, 50)),
              "p99_ms": float(np.percentile(lat, 99)), "requests": len(trace), "grad_requests": ngrad,
              "makespan_s": span, "failed": int(failed),
              "trace": f"Poisson {rate:g} req/s for {seconds:g} s, seed {seed}"}
    lat_s, span_s = serial_run(order, arrivals)
    log(f"serial: makespan {span_s:.2f} s; saturated runs")
    serial = {"ray_samples_per_s": total_rs / span_s, "p50_ms": float(np.percentile(lat_s, 50)),
              "p99_ms": float(np.percentile(lat_s, 99)), "makespan_s": span_s}
    # saturated: every request of the head of the trace at time 0
    head = order[:min(saturated, len(order))]
    rs_head = sum(reqs[i][0].ray_samples for i in head)
    zeros = [0.0] * len(head)
    lat_h, span_h, failed_h = served_run(head, zeros)
    _, span_hs = serial_run(head, zeros)
    sat = {"requests": len(head), "grad_requests": sum(1 for i in head if trace[i]["grad"]),
           "served_ray_samples_per_s": rs_head / span_h, "serial_ray_samples_per_s": rs_head / span_hs,
           "served_makespan_s": span_h, "serial_makespan_s": span_hs, "served_p99_ms": float(np.percentile(lat_h, 99)),
           "failed": int(failed_h)}
    return served, serial, sat


if __name__ == "__main__":
    main()
