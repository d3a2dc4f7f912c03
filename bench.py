"""Benchmark: spectral ray samples per second of the plain form on the
church-nave workload (512 x 512 pixels, 64 samples per pixel, 81 wavelengths
380-780 nm, depth 8, FP32 geometry and shading with FP64 accumulation), one
MI355X.  A step is one full render.

Prints one JSON line with the throughput, a roofline entry for the dominant
kernel (per-kernel durations from HIP events the library records on the
launch stream during the timed steps) and the FP64 CPU oracle timed on a
bounded pixel sample of the same workload.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Plain VALU issue rate of FP32 arithmetic without packed math:
# 256 CUs x 64 lanes x 2.4 GHz x 2 (FMA) = 78.6 TFLOP/s.
ALU_PEAK_TFLOPS = 78.6
FLOPS_PER_NODE = 48     # two slab box tests (6 sub, 6 mul, 12 min/max each)
FLOPS_PER_TRI = 50      # Moeller-Trumbore: edges, two cross products, four dots, reciprocal


def kernel_models(stats, nb, npix, nl):
    """Algorithmic work of each kernel class (see the design doc for the model)."""
    Ng, Nc, Ns, F = stats["paths"], stats["closest_segments"], stats["shadow_segments"], stats["forks"]
    m = {
        "generate": ("hbm", Ng * (44 + 4 * nb)),
        "trace": ("alu", stats["nodes_visited"]["closest"] * FLOPS_PER_NODE
                  + stats["tris_tested"]["closest"] * FLOPS_PER_TRI),
        "shade": ("hbm", Nc * (84 + 8 * nb) + Ns * (24 + 4 * nb) + F * (40 + 4 * nb)),
        "shadow": ("alu", stats["nodes_visited"]["shadow"] * FLOPS_PER_NODE
                   + stats["tris_tested"]["shadow"] * FLOPS_PER_TRI),
        "shadow_accum": ("hbm", Ns * (16 + 4 * nb)),
        "shade_glass": ("alu", 0),
        "finalize": ("hbm", npix * nl * 12 + npix * 24),
    }
    return m


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary (FETCH_SIZE and WRITE_SIZE scaled by the copy-kernel factors),
    or None when the kernel source has changed since it was measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "nave512_pmc_traffic.json")
    src = os.path.join(ROOT, "paper_1912_05494_amd", "csrc", "wavefront.hip")
    try:
        meta = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if meta.get("kernel_source_sha256") != sha or kernel not in meta.get("kernels", {}):
        return None
    return meta["kernels"][kernel]["bytes_per_launch"]


def profile_once():
    """One render of the workload, then a 256 MiB device-to-device copy whose
    FETCH_SIZE / WRITE_SIZE calibrate the traffic counters."""
    import torch
    from paper_1912_05494_amd import sdm, synth
    ctx = sdm.Context(0)
    gs = sdm.Scene(ctx, synth.nave_scene(seed=1))
    spec, xyz, stats = sdm.render(ctx, gs, synth.nave_settings())
    torch.cuda.synchronize()
    a = torch.ones(64 * 2 ** 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"closest": stats["closest_segments"], "shadow": stats["shadow_segments"],
                      "copy_bytes": a.numel() * 4}), flush=True)
    ctx.close()


def cpu_baseline(scene, settings, budget_s=12.0, max_pixels=4096):
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(threads, 16))
    W, H = settings.camera.W, settings.camera.H
    step = max(1, (W * H) // max_pixels)
    pixels = np.arange(0, W * H, step, dtype=np.int32)[:max_pixels]
    os_ = oracle.OracleScene(scene)
    done, t0 = 0, time.perf_counter()
    while done < len(pixels):
        batch = pixels[done:done + 256]
        oracle.render_pixels(os_, settings, batch, n_threads=threads)
        done += len(batch)
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    nl = len(settings.lambda_nm)
    value = done * settings.spp * nl / dt
    cpu = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": value, "unit": "spectral ray samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} pixels (every {step}th of {W}x{H}), all {settings.spp} spp x {nl} "
                      f"wavelengths, FP64, {dt:.1f} s on {threads} threads of {cpu}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--bands", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-once", action="store_true",
                    help="one render plus a 256 MiB calibration copy (for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.profile_once:
        profile_once()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the spectral and pixel sub-domains are work items of a single device)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1912_05494_amd import sdm, synth

    if not os.path.exists(sdm.LIB_PATH):
        from paper_1912_05494_amd.build import build
        build()
    scene = synth.nave_scene(seed=1)
    st = synth.nave_settings(W=512, H=512, spp=64, max_depth=8, n_bands=args.bands)
    W, H, nl = st.camera.W, st.camera.H, len(st.lambda_nm)
    ctx = sdm.Context(0)
    gs = sdm.Scene(ctx, scene)
    dev = torch.device("cuda", 0)
    spec = torch.empty((H, W, nl), dtype=torch.float32, device=dev)
    xyz = torch.empty((H, W, 3), dtype=torch.float64, device=dev)
    params, keep = sdm.make_params(st, precision=args.precision, timing=True)
    for _ in range(args.warmup):
        sdm.render_into(ctx, gs, params, spec, xyz)
    torch.cuda.synchronize()
    kms = {k: 0.0 for k in sdm.KERNELS}
    kl = {k: 0 for k in sdm.KERNELS}
    t0 = time.perf_counter()
    for i in range(args.steps):
        s = sdm.render_into(ctx, gs, params, spec, xyz)
        for k in sdm.KERNELS:
            kms[k] += s["kernel_ms"][k]
            kl[k] += s["kernel_launches"][k]
        print(f"step {i}: {s['ms_render']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    samples = W * H * st.spp * nl
    value = samples * args.steps / dt
    nb = -(-nl // args.bands)
    models = kernel_models(s, nb, W * H, nl)
    kernels = {}
    for k in sdm.KERNELS:
        if kl[k] == 0:
            continue
        avg_ms = kms[k] / kl[k]
        bound, work = models[k]
        per_launch = work / (kl[k] / args.steps)
        if bound == "hbm":
            ach, peak, unit = per_launch / (avg_ms * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            ach, peak, unit = per_launch / (avg_ms * 1e-3) / 1e12, ALU_PEAK_TFLOPS, "TFLOP/s"
        kernels[k] = {"ms_per_step": kms[k] / args.steps, "launches_per_step": kl[k] // args.steps,
                      "avg_launch_ms": avg_ms, "bound": bound, "achieved": ach, "peak": peak,
                      "unit": unit, "frac": ach / peak}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    kd = kernels[dom]
    out = {
        "metric": "spectral ray samples/sec (plain form)",
        "value": value,
        "unit": "spectral ray samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"procedural church nave, {scene.nt} triangles (24 glass panes), "
                               f"{W}x{H}, {st.spp} spp, {nl} wavelengths 380-780 nm, depth "
                               f"{st.max_depth}, {args.bands} spectral band(s)",
                   "W": W, "H": H, "spp": st.spp, "n_lambda": nl, "max_depth": st.max_depth,
                   "triangles": scene.nt, "bands": args.bands, "accumulation": "f64"},
        "roofline": {"kernel": dom, "bound": kd["bound"], "achieved": kd["achieved"], "peak": kd["peak"],
                     "unit": kd["unit"], "frac": kd["frac"], "traffic": measured_traffic(dom)},
        "kernels": kernels,
        "segments_per_s": (s["closest_segments"] + s["shadow_segments"]) * args.steps / dt,
        "distinct_rays_per_step": {"closest": s["closest_segments"], "shadow": s["shadow_segments"],
                                   "forks": s["forks"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, st)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
