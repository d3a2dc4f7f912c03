"""Benchmark: spectral ray samples per second of the plain form on the
church-nave workload (512 x 512 pixels, 64 samples per pixel, 81 wavelengths
380-780 nm, depth 8, FP32 geometry and shading with FP64 accumulation), one
MI355X.  A step is one full render.

Prints one JSON line with the throughput, a roofline entry for the dominant
kernel (per-kernel durations from HIP events the library records on the
stream each pass runs on during the timed steps: the caller's, or for the
shadow walk and accumulation the library's second stream, where they run
beside the next bounce's closest-hit pass), the FP64 CPU oracle timed on a
bounded pixel sample of the same workload, and (surrogate_form) the same
nave with its panes bubbly: the plain form (exact walks) against the trained
surrogate, with both forms' colour differences from a converged reference
(the run of --form bubbly, summarised; --no-surrogate skips it).
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

# chunk size and pixel tile of the workload as chosen by sdm_autotune on MI355X
# (bench.py --autotune repeats the choice): all 2^24 primary paths of the
# 512x512x64 image in one chunk, 16x16 tiles; the timed runs and the counter
# runs use the same
CHUNK_PATHS = 1 << 24
TILE = 16
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0
# Published FP32 vector rate of MI355X (157.3 TFLOP/s: 256 CUs x 2.4 GHz x
# 256 flop per clock, which counts packed FP32 issue).  This build keeps
# packed FP32 instructions out of the device code, so the rate its kernels
# can reach is half: 256 x 64 lanes x 2.4 GHz x 2 (FMA) = 78.6 TFLOP/s.
FP32_PEAK_TFLOPS = 157.3
FP32_UNPACKED_TFLOPS = 78.6
# Algorithmic work of a traversal step: a ray-box slab test is 16 flop (6
# plane distances, 6 min/max, 2 comparisons against the interval, 2 for the
# entry/exit), so a wide node (four boxes) is 64; a ray-triangle test is 30.
FLOPS_PER_NODE = 64
FLOPS_PER_TRI = 30
# bytes a traversal reads for a node / triangle that is not cached
NODE_BYTES, TRI_BYTES, CAND_BYTES = 128, 48, 48


def kernel_models(stats, nb, npix, nl, sun_grid=False, launches=8):
    """Algorithmic work of each kernel class per render: (bound, work) with
    work in flop for "alu"/"mfma" kernels and bytes for "hbm" ones, plus the
    bytes every kernel must move (for the whole-render HBM figure).  Weights
    are stored as a scalar per path or shadow record plus nb per-wavelength
    factors only for paths and records whose wavelengths differ (glass,
    coloured albedo):
      generate      44 B per path written (origin, direction, pixel, sample,
                    depth/band/job word, skip, scalar factor)
      trace         64 flop per wide node visited, 30 per triangle tested;
                    moves 24 B of ray read and 16 B of hit written per ray
      shade         per closest segment 56 B read (ray 36, hit 16, factor 4)
                    and 44 B written for the continuing path, 28 B per shadow
                    record; 8 nb B per spectral path (read + write), 4 nb B
                    per spectral record
      shade_glass   per glass vertex 60 B read (queue entry 4, ray 36, hit
                    16, factor 4), 44 + 4 nb B written (the continuing path
                    and its factors); 4 nb B read where the factors already
                    differed on arrival; a fork writes a second path and row,
                    44 + 4 nb B
      shadow        a memory and latency walk: 20 B of record read (origin,
                    skip, aux) and 4 B written per shadow ray, plus the 48-B
                    grid candidates it examines (or the 128-B nodes and 48-B
                    triangles of a BVH walk)
      shadow_accum  16 B per record plus 4 nb B per spectral record, plus the
                    FP64 accumulator's read-modify-write: 16 B per entry a
                    launch adds to, at least min(records x nb, launches x
                    pixels x wavelengths) entries (a pixel's records are
                    summed before they are added)
      shade_bubbly  per bubbly vertex 60 B read, 44 + 4 nb B written, 4 nb B
                    read (factors or the network's reflectance ratios)
      finalize      12 nl + 24 B per pixel
    The network: 2 x 9216 flop per (vertex, wavelength)."""
    Ng, Nc, Ns, F = stats["paths"], stats["closest_segments"], stats["shadow_segments"], stats["forks"]
    Nsp, Nsr = stats.get("spectral_paths", 0), stats.get("spectral_records", 0)
    gv = stats.get("glass_vertices", {"all": 0, "spectral": 0})
    Nb = stats.get("bubbly_vertices", 0)
    nodes_s, tris_s = stats["nodes_visited"]["shadow"], stats["tris_tested"]["shadow"]
    walk_bytes = (nodes_s * CAND_BYTES if sun_grid else nodes_s * NODE_BYTES + tris_s * TRI_BYTES)
    acc_rmw = 16 * min(Ns * nb, launches * npix * nl)
    trace_bytes = Nc * (24 + 16)
    m = {
        "generate": ("hbm", Ng * 44),
        "trace": ("alu", stats["nodes_visited"]["closest"] * FLOPS_PER_NODE
                  + stats["tris_tested"]["closest"] * FLOPS_PER_TRI),
        "shade": ("hbm", Nc * (56 + 44) + Ns * 28 + Nsp * 8 * nb + Nsr * 4 * nb),
        "shadow": ("hbm", Ns * 24 + walk_bytes),
        "shadow_accum": ("hbm", Ns * 16 + Nsr * 4 * nb + acc_rmw),
        "shade_glass": ("hbm", gv["all"] * (60 + 44 + 4 * nb) + gv["spectral"] * 4 * nb + F * (44 + 4 * nb)),
        "finalize": ("hbm", npix * nl * 12 + npix * 24),
        # network on the matrix cores: 2 x 9216 multiply-adds per (vertex, wavelength) tuple,
        # nb wavelengths plus the reference one per bubbly vertex
        "bubbly_eval": ("mfma", stats.get("bubbly_vertices", 0) * (nb + 1) * 2 * 9216),
        "shade_bubbly": ("hbm", Nb * (60 + 44 + 8 * nb)),
    }
    moved = {k: (w if bound == "hbm" else 0) for k, (bound, w) in m.items()}
    moved["trace"] = trace_bytes
    return m, moved


def source_digest():
    """sha256 over the library's sources (every file of csrc/, by name): the
    kernels and the structures the host builds for them."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1912_05494_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".cpp", ".hpp")):
            h.update(name.encode())
            h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of kernel class `kernel` from the committed
    rocprofv3 --pmc summary (FETCH_SIZE and WRITE_SIZE scaled by the
    copy-kernel factors), or None when the sources have changed since it was
    measured."""
    path = os.path.join(ROOT, "profiles", "nave512_pmc_traffic.json")
    try:
        meta = json.load(open(path))
        sha = source_digest()
    except (OSError, ValueError):
        return None
    if meta.get("source_sha256") != sha or kernel not in meta.get("kernels", {}):
        return None
    return meta["kernels"][kernel]["bytes_per_launch"]


def profile_once():
    """One render of the workload, then a 256 MiB device-to-device copy whose
    FETCH_SIZE / WRITE_SIZE calibrate the traffic counters, then two tiny
    kernels (a fill and an add on 1 KiB)."""
    import torch
    from paper_1912_05494_amd import sdm, synth
    ctx = sdm.Context(0)
    gs = sdm.Scene(ctx, synth.nave_scene(seed=1))
    spec, xyz, stats = sdm.render(ctx, gs, synth.nave_settings(), chunk_paths=CHUNK_PATHS, tile=(TILE, TILE))
    torch.cuda.synchronize()
    a = torch.ones(64 * 2 ** 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    # a tiny kernel after the copy: its counters show whether write-backs of
    # the copy's dirty cache lines land in the next dispatch's window
    c = torch.zeros(256, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    c.add_(1.0)
    torch.cuda.synchronize()
    print(json.dumps({"closest": stats["closest_segments"], "shadow": stats["shadow_segments"],
                      "copy_bytes": a.numel() * 4}), flush=True)
    ctx.close()


def cpu_baseline(scene, settings, pixels_n=1024, pixels_1=48, reps=3):
    """The oracle on the host's cores: the same workload on a bounded pixel
    sample (every k-th pixel, all spp and wavelengths), best of `reps` runs,
    at all threads (up to 16) and at one thread."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(threads, 16))
    W, H = settings.camera.W, settings.camera.H
    nl = len(settings.lambda_nm)
    os_ = oracle.OracleScene(scene)

    def best(n_pix, n_threads):
        step = max(1, (W * H) // n_pix)
        pixels = np.arange(0, W * H, step, dtype=np.int32)[:n_pix]
        dts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.render_pixels(os_, settings, pixels, n_threads=n_threads)
            dts.append(time.perf_counter() - t0)
        return len(pixels) * settings.spp * nl / min(dts), min(dts), step

    value, dt, step = best(pixels_n, threads)
    value1, dt1, step1 = best(pixels_1, 1)
    cpu = platform.processor() or "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": value, "unit": "spectral ray samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{pixels_n} pixels (every {step}th of {W}x{H}), all {settings.spp} spp x {nl} "
                      f"wavelengths, FP64, best of {reps} runs ({dt:.1f} s) on {threads} threads of {cpu}",
            "value_1_thread": value1,
            "sample_1_thread": f"{pixels_1} pixels (every {step1}th), best of {reps} runs ({dt1:.1f} s) on 1 thread",
            "parallel_speedup": value / value1}


def cpu_table1(threads=(1, 2, 4, 8, 16), bands=(1, 2, 4, 8), W=48, H=36, spp=4, reps=1, scene=None,
               settings=None):
    """The shape of the paper's Table 1 (speedup against threads x spectral
    sub-domains) replayed with the oracle on the host's cores: one image of
    the church nave (W x H, spp, 81 wavelengths, depth 8) rendered with
    OpenMP over (pixel tile x band) items at each thread count and band
    count; speedups are against 1 thread and 1 band (best of `reps`).  The
    images of every cell are identical (the decomposition does not change
    the result), which is checked."""
    import oracle
    from paper_1912_05494_amd import synth
    sc = scene if scene is not None else synth.nave_scene(seed=1)
    st = settings if settings is not None else synth.nave_settings(W=W, H=H, spp=spp)
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = [t for t in threads if t <= max(1, avail)]
    osc = oracle.OracleScene(sc)
    times, ref = {}, None
    for nb in bands:
        for t in threads:
            best = 1e30
            for _ in range(reps):
                t0 = time.perf_counter()
                img, _ = oracle.render(osc, st, n_threads=t, n_bands=nb)
                best = min(best, time.perf_counter() - t0)
            if ref is None:
                ref = img
            elif not np.array_equal(img, ref):
                raise AssertionError(f"image differs at {t} threads, {nb} bands")
            times[(nb, t)] = best
            print(f"table1: {nb} band(s), {t} thread(s): {best:.2f} s", file=sys.stderr, flush=True)
    base = times[(bands[0], threads[0])]
    return {"speedup": {str(nb): {str(t): base / times[(nb, t)] for t in threads} for nb in bands},
            "seconds": {str(nb): {str(t): times[(nb, t)] for t in threads} for nb in bands},
            "workload": f"church nave {st.camera.W}x{st.camera.H}, {st.spp} spp, {len(st.lambda_nm)} wavelengths, "
                        f"depth {st.max_depth}, FP64 oracle, OpenMP over (16x16 tile x band) items",
            "host_threads": avail}


def copy_bandwidth(nbytes=2 << 30, reps=5):
    """GB/s of a device-to-device copy of nbytes (read + write counted) in
    this session: the HBM rate a streaming kernel can reach."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    return 2 * nbytes / best / 1e9


def bubbly_bench(args, emit=True):
    """Bubbly panes on the nave: MC tables of the slab (GPU), network training
    (matrix cores), validation and error table, then four forms of the render:
    exact walks (the plain form for bubbly panes), surrogate, fallback, and
    the bubble-free analytic slab.  Reports each form's rate and its
    CIEDE2000 against a converged exact reference and against the exact form
    at the same spp, per pixel and on block means."""
    import torch
    from paper_1912_05494_amd import color, sdm, surrogate, synth

    scene = synth.nave_scene(seed=1, bubbly=True, rho_min=args.bubbly_rho_min)
    scene_free = synth.nave_scene(seed=1, bubbly=True, rho_min=args.bubbly_rho_min, bubble_free=True)
    st = synth.nave_settings(W=512, H=512, spp=args.bubbly_spp, max_depth=8)
    W, H, nl = st.camera.W, st.camera.H, len(st.lambda_nm)
    ctx = sdm.Context(0)
    gs = sdm.Scene(ctx, scene)
    gs_free = sdm.Scene(ctx, scene_free)
    dev = torch.device("cuda", 0)
    panes = [m for m in scene.materials if m.type == synth.GLASS_BUBBLY]
    n_panes = len(panes)

    def tuples_for(n, seed, own=0.0):
        return surrogate.scene_tuples(scene.materials, scene.tab_lambda, n, st.lambda_nm, seed=seed, own=own)

    def mc(tup, nk, nph, seed):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y = surrogate.mc_targets(ctx, tup, nk, nph, seed, dev)
        torch.cuda.synchronize()
        return y, time.perf_counter() - t0

    tup, pane, nk = tuples_for(args.bubbly_train, seed=101, own=0.5)
    target, t_mc = mc(tup, nk, 64, 7)
    print(f"MC tables: {len(tup)} tuples x 64 photons in {t_mc:.2f} s", file=sys.stderr, flush=True)
    net = sdm.MLP(ctx, n_panes, surrogate.init_params(n_panes, seed=0))
    tt = torch.from_numpy(tup).to(dev)
    tp = torch.from_numpy(pane).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    curve = surrogate.train_stepped(net, tt, tp, target, args.bubbly_steps)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print(f"training: {args.bubbly_steps} steps in {t_train:.2f} s, loss {curve[0]:.4g} -> "
          f"{curve[-50:].mean():.4g}", file=sys.stderr, flush=True)
    vt, vp, vnk = tuples_for(args.bubbly_val, seed=202)
    vtarget, _ = mc(vt, vnk, args.bubbly_val_photons, 9)
    vout = net.infer(torch.from_numpy(vt).to(dev), torch.from_numpy(vp).to(dev))
    verr = (vout - vtarget).cpu().numpy()
    vy = vtarget.cpu().numpy()
    validation = {"rms_R": float(np.sqrt(np.mean(verr[:, 0] ** 2))),
                  "rms_T": float(np.sqrt(np.mean(verr[:, 1] ** 2))),
                  "rms_w": float(np.sqrt(np.mean(verr[:, 2] ** 2))),
                  "mean_R_error": float(np.mean(verr[:, 0])), "mean_T_error": float(np.mean(verr[:, 1])),
                  # binomial standard error of the validation targets themselves
                  "mc_se_R": float(np.sqrt(np.mean(vy[:, 0] * (1 - vy[:, 0]))) / np.sqrt(args.bubbly_val_photons)),
                  "tuples": args.bubbly_val, "photons": args.bubbly_val_photons}
    table = net.error_table(torch.from_numpy(vt).to(dev), torch.from_numpy(vp).to(dev), vtarget,
                            dims=(8, 3, 4)).cpu().numpy()

    def run(gs_, btdf, st_, timed):
        params, keep = sdm.make_params(st_, timing=timed, btdf=btdf)
        spec = torch.empty((H, W, nl), dtype=torch.float32, device=dev)
        xyz = torch.empty((H, W, 3), dtype=torch.float64, device=dev)
        s_ = sdm.render_into(ctx, gs_, params, spec, xyz)
        if not timed:
            return xyz.cpu().numpy(), None, s_
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s_ = sdm.render_into(ctx, gs_, params, spec, xyz)
        torch.cuda.synchronize()
        return xyz.cpu().numpy(), (time.perf_counter() - t0) / args.steps, s_

    forms, images = {}, {}
    cases = (("exact", gs, {"mode": "exact"}), ("surrogate", gs, {"mode": "surrogate", "mlp": net}),
             ("fallback", gs, {"mode": "fallback", "mlp": net, "err_table": table, "bound": args.bubbly_bound}),
             ("bubble_free", gs_free, None))
    for form, gs_, btdf in cases:
        images[form], dt, s_ = run(gs_, btdf, st, True)
        forms[form] = {"value": W * H * st.spp * nl / dt, "ms_per_step": dt * 1e3,
                       "bubbly_vertices": s_["bubbly_vertices"],
                       "kernel_ms": {k: v for k, v in s_["kernel_ms"].items() if v > 0}}
        print(f"{form}: {dt * 1e3:.1f} ms", file=sys.stderr, flush=True)
    # converged reference: the exact form at args.bubbly_ref seeds x 256 spp
    ref = None
    for s in range(args.bubbly_ref):
        x, _, _ = run(gs, {"mode": "exact"}, synth.nave_settings(W=512, H=512, spp=256, max_depth=8, seed=100 + s),
                      False)
        ref = x if ref is None else ref + x
    ref /= args.bubbly_ref
    # sampling noise: the exact form against itself at another seed
    st2 = synth.nave_settings(W=512, H=512, spp=args.bubbly_spp, max_depth=8, seed=1)
    other, _, _ = run(gs, {"mode": "exact"}, st2, False)

    def blocks(x, b=16):
        return x.reshape(H // b, b, W // b, b, 3).mean((1, 3))

    def de(a, b):
        return float(np.mean(color.image_delta_e(a, b, st.cmf, st.lambda_nm)))

    de_pixel = {f: de(ref, images[f]) for f in forms}
    de_pixel["exact_vs_exact_other_seed"] = de(images["exact"], other)
    de_vs_exact = {f: de(images["exact"], images[f]) for f in ("surrogate", "fallback", "bubble_free")}
    # on 16 x 16 pixel block means sampling noise is 16x lower
    de_blocks = {f: de(blocks(ref), blocks(images[f])) for f in forms}
    de_blocks["exact_vs_exact_other_seed"] = de(blocks(images["exact"]), blocks(other))
    de_blocks_vs_exact = {f: de(blocks(images["exact"]), blocks(images[f]))
                          for f in ("surrogate", "fallback", "bubble_free")}
    for f in forms:
        forms[f]["mean_Y_over_reference"] = float(images[f][..., 1].mean() / ref[..., 1].mean())
    out = {
        "metric": "spectral ray samples/sec (bubbly panes, surrogate form at mean block dE2000 < 1 against "
                  "the exact walk)",
        "value": forms["surrogate"]["value"],
        "unit": "spectral ray samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": forms["surrogate"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"procedural church nave with {n_panes} bubbly panes (density "
                               f"{args.bubbly_rho_min:g}-34 per mm^3, "
                               f"radii 10-200 um), {W}x{H}, {st.spp} spp, {nl} wavelengths, depth 8",
                   "surrogate": f"12-64-64-64-3 trained {args.bubbly_steps} Adam steps of 8192 (lr 2e-3, 5e-4, "
                                f"1e-4) on {args.bubbly_train} MC tuples (64 photons, half at the panes' "
                                f"own densities)",
                   "error_table": f"8x3x4 cells per pane from {args.bubbly_val} tuples x "
                                  f"{args.bubbly_val_photons} photons, bound {args.bubbly_bound}"},
        "forms": forms,
        "validation": validation,
        "reference": f"exact form, {args.bubbly_ref} seeds x 256 spp",
        "mean_delta_e2000_vs_reference": de_pixel,
        "mean_delta_e2000_vs_reference_16x16_blocks": de_blocks,
        "mean_delta_e2000_vs_exact": de_vs_exact,
        "mean_delta_e2000_vs_exact_16x16_blocks": de_blocks_vs_exact,
        "flagged_cells": float((table > args.bubbly_bound).mean()),
        "mc_tuple_photons_per_s": len(tup) * 64 / t_mc,
        "train_samples_per_s": args.bubbly_steps * 8192 / t_train,
    }
    net.close()
    ctx.close()
    if emit:
        print(json.dumps(out), flush=True)
    return out


def large_bench(args):
    """The large configuration: the ~1 M-triangle nave with 200 bubbly panes of
    40 glass types at 1920 x 1080, 81 wavelengths, 256 spp, depth 12.  The
    network is trained on MC tables of the 40 pane types, its error table
    built from 10^4 tuples x 65,536 photons; the fallback form (surrogate,
    exact walk where a cell's error exceeds the bound) is timed against the
    plain form (exact walks) on the same GPU, with the surrogate form beside
    them, and compared by CIEDE2000 on 16 x 16 pixel block means."""
    import torch
    from paper_1912_05494_amd import color, sdm, surrogate, synth

    scene = synth.large_scene()
    st = synth.large_settings(spp=args.large_spp)
    W, H, nl = st.camera.W, st.camera.H, len(st.lambda_nm)
    dev = torch.device("cuda", 0)
    ctx = sdm.Context(0)
    t0 = time.perf_counter()
    gs = sdm.Scene(ctx, scene)
    t_scene = time.perf_counter() - t0
    n_types = 1 + max(m.pane_id for m in scene.materials if m.type == synth.GLASS_BUBBLY)
    print(f"scene: {len(scene.idx)} triangles, built in {t_scene:.2f} s", file=sys.stderr, flush=True)
    tup, pane, nk = surrogate.scene_tuples(scene.materials, scene.tab_lambda, args.bubbly_train, st.lambda_nm,
                                           seed=101, own=0.5)
    target = surrogate.mc_targets(ctx, tup, nk, 64, 7, dev)
    net = sdm.MLP(ctx, n_types, surrogate.init_params(n_types, seed=0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    surrogate.train_stepped(net, torch.from_numpy(tup).to(dev), torch.from_numpy(pane).to(dev), target,
                            args.bubbly_steps)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    vt, vp, vnk = surrogate.scene_tuples(scene.materials, scene.tab_lambda, args.bubbly_val, st.lambda_nm, seed=202)
    vtarget = surrogate.mc_targets(ctx, vt, vnk, args.bubbly_val_photons, 9, dev)
    table = net.error_table(torch.from_numpy(vt).to(dev), torch.from_numpy(vp).to(dev), vtarget,
                            dims=(8, 3, 4)).cpu().numpy()
    print(f"training: {args.bubbly_steps} steps in {t_train:.2f} s", file=sys.stderr, flush=True)
    spec = torch.empty((H, W, nl), dtype=torch.float32, device=dev)
    xyz = torch.empty((H, W, 3), dtype=torch.float64, device=dev)

    def run(btdf, st_, steps):
        params, keep = sdm.make_params(st_, timing=steps > 0, btdf=btdf)
        s_ = sdm.render_into(ctx, gs, params, spec, xyz)
        dt = None
        if steps > 0:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                s_ = sdm.render_into(ctx, gs, params, spec, xyz)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
        return xyz.cpu().numpy(), dt, s_

    forms, images = {}, {}
    for form, btdf in (("exact", {"mode": "exact"}),
                       ("fallback", {"mode": "fallback", "mlp": net, "err_table": table, "bound": args.bubbly_bound}),
                       ("surrogate", {"mode": "surrogate", "mlp": net})):
        images[form], dt, s_ = run(btdf, st, args.large_steps)
        forms[form] = {"value": W * H * st.spp * nl / dt, "ms_per_step": dt * 1e3,
                       "bubbly_vertices": s_["bubbly_vertices"],
                       "kernel_ms": {k: v for k, v in s_["kernel_ms"].items() if v > 0}}
        print(f"{form}: {dt * 1e3:.1f} ms", file=sys.stderr, flush=True)
    other, _, _ = run({"mode": "exact"}, synth.large_settings(spp=args.large_spp, seed=1), 0)

    def blocks(x, b=20):
        return x.reshape(H // b, b, W // b, b, 3).mean((1, 3))

    def de(a, b):
        return float(np.mean(color.image_delta_e(a, b, st.cmf, st.lambda_nm)))

    de_blocks = {f: de(blocks(images["exact"]), blocks(images[f])) for f in ("fallback", "surrogate")}
    de_blocks["exact_vs_exact_other_seed"] = de(blocks(images["exact"]), blocks(other))
    out = {
        "metric": "spectral ray samples/sec (large nave, fallback form at error bound "
                  f"{args.bubbly_bound:g} against the plain form)",
        "value": forms["fallback"]["value"],
        "unit": "spectral ray samples/s",
        "n_gpus": 1, "steps": args.large_steps, "warmup": 1,
        "ms_per_step": forms["fallback"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"procedural church nave, {len(scene.idx)} triangles, 200 bubbly panes of 200 "
                               f"triangles ({n_types} glass types, densities 0-34 per mm^3), {W}x{H}, {st.spp} spp, "
                               f"{nl} wavelengths, depth {st.max_depth}",
                   "surrogate": f"12-64-64-64-3 trained {args.bubbly_steps} Adam steps of 8192 on "
                                f"{args.bubbly_train} MC tuples (64 photons)",
                   "error_table": f"8x3x4 cells per pane type from {args.bubbly_val} tuples x "
                                  f"{args.bubbly_val_photons} photons, bound {args.bubbly_bound}"},
        "forms": forms,
        "fallback_speed_vs_plain": forms["fallback"]["value"] / forms["exact"]["value"],
        "mean_delta_e2000_vs_exact_20x20_blocks": de_blocks,
        "flagged_cells": float((table > args.bubbly_bound).mean()),
        "scene_build_s": t_scene,
    }
    print(json.dumps(out), flush=True)
    net.close()
    ctx.close()


def maps_bench(args):
    """Distribution maps: the benchmark nave with every pane's optical
    constants and thickness taken from its own stained-glass map (6 x 16
    texels, six tile glasses and a yellow edging) against the same nave with
    per-pane glass, both at 512 x 512, 64 spp, 81 wavelengths, depth 8."""
    import torch
    from paper_1912_05494_amd import sdm, synth

    ctx = sdm.Context(0)
    st = synth.nave_settings()
    W, H, nl = st.camera.W, st.camera.H, len(st.lambda_nm)
    dev = torch.device("cuda", 0)
    spec = torch.empty((H, W, nl), dtype=torch.float32, device=dev)
    xyz = torch.empty((H, W, 3), dtype=torch.float64, device=dev)
    forms = {}
    for form, scene in (("per_pane_glass", synth.nave_scene()), ("distribution_maps", synth.nave_scene(dist_maps=True))):
        gs = sdm.Scene(ctx, scene)
        params, keep = sdm.make_params(st, timing=True)
        for _ in range(args.warmup):
            s_ = sdm.render_into(ctx, gs, params, spec, xyz)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s_ = sdm.render_into(ctx, gs, params, spec, xyz)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        forms[form] = {"value": W * H * st.spp * nl / dt, "ms_per_step": dt * 1e3,
                       "kernel_ms": {k: v for k, v in s_["kernel_ms"].items() if v > 0}}
        print(f"{form}: {dt * 1e3:.2f} ms", file=sys.stderr, flush=True)
        gs.close()
    out = {
        "metric": "spectral ray samples/sec (nave with stained-glass distribution maps)",
        "value": forms["distribution_maps"]["value"], "unit": "spectral ray samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": forms["distribution_maps"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "procedural church nave, 24 panes each with a 6x16-texel map of 7 glasses and "
                               "per-texel thickness, 512x512, 64 spp, 81 wavelengths, depth 8"},
        "forms": forms,
        "maps_speed_vs_per_pane_glass": forms["distribution_maps"]["value"] / forms["per_pane_glass"]["value"],
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def subdomains_bench(args):
    """Geometric sub-domains (Sec. 5): the benchmark nave (512 x 512, 64 spp)
    and the large nave (1920 x 1080, --subdomain-large-spp spp, depth 12)
    rendered whole and cut into grids of cells; per cut the render time, the
    closest-hit pass time, the rays handed across interfaces and the cells'
    triangle references.  The images are identical to the uncut ones (the
    sub-domain tests check it)."""
    import torch
    from paper_1912_05494_amd import sdm, synth

    ctx = sdm.Context(0)
    dev = torch.device("cuda", 0)
    cases = [("nave", synth.nave_scene(), synth.nave_settings(), [(1, 1, 1), (4, 1, 1), (8, 2, 2), (16, 4, 4)]),
             ("large", synth.large_scene(bubbly=False), synth.large_settings(spp=args.subdomain_large_spp),
              [(1, 1, 1), (8, 2, 2), (16, 4, 4), (32, 8, 8)])]
    results = {}
    for name, scene, st, cuts in cases:
        W, H, nl = st.camera.W, st.camera.H, len(st.lambda_nm)
        spec = torch.empty((H, W, nl), dtype=torch.float32, device=dev)
        xyz = torch.empty((H, W, 3), dtype=torch.float64, device=dev)
        rows = []
        for cut, handoff in [(c, m) for c in cuts for m in (("queue", "march") if c != (1, 1, 1) else ("queue",))]:
            gs = sdm.Scene(ctx, scene, subdomains=cut, handoff=handoff)
            params, keep = sdm.make_params(st, timing=True)
            s_ = sdm.render_into(ctx, gs, params, spec, xyz)
            steps = args.steps if name == "nave" else 1
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                s_ = sdm.render_into(ctx, gs, params, spec, xyz)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            cells, refs, nodes = gs.subdomains()
            rows.append({"cells": list(cells), "handoff": handoff, "ms_per_step": dt * 1e3, "value": W * H * st.spp * nl / dt,
                         "trace_ms": s_["kernel_ms"]["trace"], "interface_rays": s_["interface_rays"],
                         "closest_segments": s_["closest_segments"], "tri_refs": refs, "nodes": nodes,
                         "nodes_visited": s_["nodes_visited"]["closest"],
                         "tris_tested": s_["tris_tested"]["closest"]})
            print(f"{name} {cut} {handoff}: {dt * 1e3:.2f} ms, trace {s_['kernel_ms']['trace']:.2f} ms, "
                  f"{s_['interface_rays']} interface rays", file=sys.stderr, flush=True)
            gs.close()
        results[name] = {"workload": f"{len(scene.idx)} triangles, {W}x{H}, {st.spp} spp, {nl} wavelengths, "
                                     f"depth {st.max_depth}", "cuts": rows}
    best = min(results["large"]["cuts"][1:], key=lambda r: r["ms_per_step"])
    out = {"metric": "spectral ray samples/sec (large nave, geometric sub-domains)", "value": best["value"],
           "unit": "spectral ray samples/s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": best["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic", "config": {"workload": results["large"]["workload"],
                                                         "cells": best["cells"], "handoff": best["handoff"]},
           "results": results}
    print(json.dumps(out), flush=True)
    ctx.close()


def photons_bench(args):
    """Caustic photon map (photon mapping, Sec. 3.2): the bubbly nave (24
    panes, exact walks) at 512 x 512, 64 spp, 81 wavelengths, depth 8, with
    0 and 2^20 .. 2^24 sun photons, radius --photon-radius; per count the
    render time, the photon pass and gather times and the photons stored."""
    import torch
    from paper_1912_05494_amd import sdm, synth

    ctx = sdm.Context(0)
    st = synth.nave_settings()
    W, H, nl = st.camera.W, st.camera.H, len(st.lambda_nm)
    dev = torch.device("cuda", 0)
    spec = torch.empty((H, W, nl), dtype=torch.float32, device=dev)
    xyz = torch.empty((H, W, 3), dtype=torch.float64, device=dev)
    gs = sdm.Scene(ctx, synth.nave_scene(seed=1, bubbly=True))
    rows = []
    for n in (0, 1 << 20, 1 << 22, 1 << 24):
        params, keep = sdm.make_params(st, timing=True, btdf={"mode": "exact"}, photons=n,
                                       photon_radius=args.photon_radius)
        for _ in range(args.warmup):
            s_ = sdm.render_into(ctx, gs, params, spec, xyz)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s_ = sdm.render_into(ctx, gs, params, spec, xyz)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        km = s_["kernel_ms"]
        rows.append({"photons": n, "ms_per_step": dt * 1e3, "value": W * H * st.spp * nl / dt,
                     "photons_stored": s_["photons_stored"], "photon_ms": km["photon"], "caustic_ms": km["caustic"],
                     "photons_per_s": n / (km["photon"] * 1e-3) if n and km["photon"] > 0 else None,
                     "kernel_ms": {k: v for k, v in km.items() if v > 0}})
        print(f"{n} photons: {dt * 1e3:.2f} ms, stored {s_['photons_stored']}, photon pass {km['photon']:.2f} ms, "
              f"gather {km['caustic']:.2f} ms", file=sys.stderr, flush=True)
    gs.close()
    main_row = rows[2]
    out = {
        "metric": "spectral ray samples/sec (bubbly nave with the caustic photon map, 2^22 photons)",
        "value": main_row["value"], "unit": "spectral ray samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": main_row["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "procedural church nave, 24 bubbly panes (exact walks), 512x512, 64 spp, "
                               f"81 wavelengths, depth 8, photon radius {args.photon_radius} m"},
        "counts": rows,
        "map_cost_vs_no_map": main_row["ms_per_step"] / rows[0]["ms_per_step"],
    }
    print(json.dumps(out), flush=True)
    ctx.close()


# useful multiply-adds of one training sample, x2 for flops: forward
# 12x64 + 64x64 + 64x64 + 64x3, the input gradients of the four layers and
# the weight gradients the same again (the padded tile entries not counted)
TRAIN_FLOP_PER_SAMPLE = 3 * 2 * (12 * 64 + 64 * 64 + 64 * 64 + 64 * 3)


def train_bench(args):
    """Surrogate training on the matrix cores: Adam steps of the 12-64-64-64-3
    network with 24 pane embeddings, batches of 8192 and 65536 drawn from
    2^20 synthetic tuples (cos U(0, 1], the 81-wavelength grid, thickness
    U(2, 5) mm, density U(0, 34)) with uniform targets; the step time does
    not depend on the values.  Per step: the gradient pass and the fused
    sum / Adam / repack pass."""
    import torch
    from paper_1912_05494_amd import sdm, surrogate, synth

    ctx = sdm.Context(0)
    dev = torch.device("cuda", 0)
    n_panes = 24
    tup, pane = surrogate.random_tuples(1 << 20, n_panes, synth.LAMBDA_81, seed=4)
    t, pn = torch.from_numpy(tup).to(dev), torch.from_numpy(pane).to(dev)
    target = torch.rand((len(tup), 3), dtype=torch.float32, device=dev, generator=torch.Generator(dev).manual_seed(5))
    net = sdm.MLP(ctx, n_panes, surrogate.init_params(n_panes, seed=0))
    rows = {}
    for batch, steps in ((8192, 20 * args.steps), (65536, 5 * args.steps)):
        net.train(t, pn, target, steps=max(args.warmup, 1) * 10, batch=batch, lr=1e-3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net.train(t, pn, target, steps=steps, batch=batch, lr=1e-3)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        sps = batch / dt
        rows[batch] = {"us_per_step": dt * 1e6, "samples_per_s": sps,
                       "tflops": sps * TRAIN_FLOP_PER_SAMPLE / 1e12,
                       "frac_bf16_peak": sps * TRAIN_FLOP_PER_SAMPLE / 2.5e15}
        print(f"batch {batch}: {dt * 1e6:.1f} us per step, {sps / 1e6:.1f} M samples/s", file=sys.stderr, flush=True)
    net.close()
    ctx.close()
    r = rows[8192]
    out = {"metric": "surrogate training samples/sec (batch 8192)", "value": r["samples_per_s"],
           "unit": "samples/s", "n_gpus": 1, "steps": 20 * args.steps, "warmup": args.warmup,
           "ms_per_step": r["us_per_step"] / 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "Adam steps of the 12-64-64-64-3 surrogate, 24 pane embeddings, batch 8192 "
                                  "(and 65536) from 2^20 synthetic tuples"},
           "roofline": {"bound": "mfma", "achieved": r["tflops"], "peak": 2500.0, "unit": "TFLOP/s",
                        "frac": r["frac_bf16_peak"], "traffic": None,
                        "work_model": f"{TRAIN_FLOP_PER_SAMPLE} flop per sample (forward, input and weight "
                                      "gradients)"},
           "batches": rows}
    print(json.dumps(out), flush=True)


def batch_bench(args):
    """The uneven 32-job batch (square sides 128-1024, 10k-200k triangles,
    8-81 wavelengths, 16-128 spp; scene seed 2 + job) through the batch
    scheduler (jobs that fill the device alone, the others in shared
    wavefronts), against the same jobs rendered one after the other; then
    the same for 64 small jobs (sides 32-256)."""
    import torch
    from paper_1912_05494_amd import sdm, synth

    t0 = time.perf_counter()
    jobs = synth.batch_jobs(n_jobs=args.batch_jobs, seed=2, scale=args.batch_scale)
    ctx = sdm.Context(0)
    scenes = [sdm.Scene(ctx, sc) for sc, _ in jobs]
    print(f"{len(jobs)} scenes built in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    samples = sum(st.camera.W * st.camera.H * st.spp * len(st.lambda_nm) for _, st in jobs)
    tris = sum(sc.nt for sc, _ in jobs)
    batch = [(g, st) for g, (_, st) in zip(scenes, jobs)]
    sdm.render_batch(ctx, batch, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, stats = sdm.render_batch(ctx, batch, graph=True)
        print(f"batch step {i}: {stats['ms_render']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # the same jobs one after the other
    t0 = time.perf_counter()
    for g, st in batch:
        sdm.render(ctx, g, st, graph=True)
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t0
    # a batch of small jobs (sides 32-256, 2k-12.5k triangles), most of which
    # share wavefronts
    small = synth.batch_jobs(n_jobs=64, seed=3, scale=0.25)
    sscenes = [sdm.Scene(ctx, sc) for sc, _ in small]
    sbatch = [(g, st) for g, (_, st) in zip(sscenes, small)]
    ssamples = sum(st.camera.W * st.camera.H * st.spp * len(st.lambda_nm) for _, st in small)
    sdm.render_batch(ctx, sbatch, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sdm.render_batch(ctx, sbatch, graph=True)
    torch.cuda.synchronize()
    dts = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for g, st in sbatch:
        sdm.render(ctx, g, st, graph=True)
    torch.cuda.synchronize()
    dts_seq = time.perf_counter() - t0
    print(f"small-job batch: {dts * 1e3:.1f} ms, one by one {dts_seq * 1e3:.1f} ms", file=sys.stderr, flush=True)
    out = {
        "metric": "spectral ray samples/sec (32-job batch)",
        "value": samples / dt,
        "unit": "spectral ray samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(jobs)} procedural naves, {tris} triangles in all, square sides "
                               f"128-1024 x {args.batch_scale}, 8-81 wavelengths, 16-128 spp, depth 8, "
                               "one wavefront with graph replay",
                   "spectral_samples_per_step": samples},
        "sequential_single_renders": {"value": samples / dt_seq, "ms": dt_seq * 1e3},
        "batch_speedup_over_sequential": dt_seq / dt,
        "small_jobs": {"jobs": len(small), "spectral_samples": ssamples, "value": ssamples / dts, "ms": dts * 1e3,
                       "sequential_ms": dts_seq * 1e3, "speedup_over_sequential": dts_seq / dts,
                       "workload": "64 procedural naves, square sides 32-256, 2k-12.5k triangles, 8-81 "
                                   "wavelengths, 16-128 spp, depth 8"},
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--bands", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the bubbly nave's plain-against-surrogate comparison in the default line")
    ap.add_argument("--no-band-split", action="store_true", help="skip the 4- and 16-band timings")
    ap.add_argument("--profile-once", action="store_true",
                    help="one render plus a 256 MiB calibration copy (for rocprofv3 --pmc)")
    ap.add_argument("--form", default="plain",
                    choices=["plain", "bubbly", "batch", "table1", "large", "maps", "subdomains", "photons", "train"],
                    help="plain: the clear-glass nave (default); bubbly: bubbly panes in four forms; "
                         "batch: the uneven 32-job batch in one wavefront; table1: the oracle's speedup "
                         "against threads x bands on the host (no GPU); large: the 1 M-triangle nave "
                         "with 200 bubbly panes at 1920x1080, fallback against exact; maps: the nave with "
                         "stained-glass distribution maps against per-pane glass; subdomains: geometric "
                         "sub-domain cuts of the nave and the large nave; photons: the bubbly nave with "
                         "the caustic photon map at 2^20 to 2^24 photons; train: surrogate training steps")
    ap.add_argument("--photon-radius", type=float, default=0.1, help="gather radius of --form photons (m)")
    ap.add_argument("--batch-jobs", type=int, default=32)
    ap.add_argument("--batch-scale", type=float, default=1.0)
    ap.add_argument("--autotune", action="store_true",
                    help="choose chunk size and tile with sdm_autotune before timing")
    ap.add_argument("--bubbly-spp", type=int, default=64)
    ap.add_argument("--large-spp", type=int, default=256)
    ap.add_argument("--subdomain-large-spp", type=int, default=64)
    ap.add_argument("--large-steps", type=int, default=1, help="timed renders per form of --form large")
    ap.add_argument("--bubbly-train", type=int, default=10_000_000)
    ap.add_argument("--bubbly-steps", type=int, default=30000)
    ap.add_argument("--bubbly-val", type=int, default=10000, help="validation tuples")
    ap.add_argument("--bubbly-ref", type=int, default=16, help="256-spp exact renders in the reference")
    ap.add_argument("--bubbly-val-photons", type=int, default=65536)
    # the validation tables carry MC noise of ~2e-3 per tuple (16384 photons),
    # so a bound below ~1e-2 flags nearly every cell
    ap.add_argument("--bubbly-bound", type=float, default=1e-3)
    ap.add_argument("--bubbly-rho-min", type=float, default=0.0,
                    help="least bubble density of a pane (per mm^3; densities are uniform up to 34)")
    args = ap.parse_args()
    if args.profile_once:
        profile_once()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the spectral and pixel sub-domains are work items of a single device)",
              file=sys.stderr)
        sys.exit(2)

    if args.form == "table1":
        # the oracle's speedup against threads x spectral sub-domains (CPU only)
        out = {"metric": "oracle speedup against threads x spectral sub-domains (shape of the paper's Table 1)",
               "cpu_baseline": cpu_table1()}
        print(json.dumps(out), flush=True)
        return
    if args.form == "large":
        return large_bench(args)
    if args.form == "maps":
        return maps_bench(args)
    if args.form == "subdomains":
        return subdomains_bench(args)
    if args.form == "photons":
        return photons_bench(args)
    if args.form == "train":
        return train_bench(args)
    if args.form == "bubbly":
        bubbly_bench(args)
        return
    if args.form == "batch":
        batch_bench(args)
        return

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
    chunk, tile = CHUNK_PATHS, (TILE, TILE)
    tuned = None
    if args.autotune:
        # chunk size and pixel tile for this scene and shape (untimed)
        tuned = sdm.autotune(ctx, gs, st, precision=args.precision)
        chunk, tile = tuned["chunk_paths"], tuned["tile"]
        print(f"autotune: {tuned}", file=sys.stderr, flush=True)
    params, keep = sdm.make_params(st, precision=args.precision, timing=True, chunk_paths=chunk, tile=tile)
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
    info = gs.info()
    models, moved = kernel_models(s, nb, W * H, nl, sun_grid=info["grid_cells"] > 0,
                                  launches=kl["shadow_accum"] // args.steps)
    kernels = {}
    for k in sdm.KERNELS:
        if kl[k] == 0:
            continue
        avg_ms = kms[k] / kl[k]
        bound, work = models[k]
        per_launch = work / (kl[k] / args.steps)
        if bound == "hbm":
            ach, peak, unit = per_launch / (avg_ms * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s"
        elif bound == "mfma":
            ach, peak, unit = per_launch / (avg_ms * 1e-3) / 1e12, MFMA_BF16_PEAK_TFLOPS, "TFLOP/s"
        else:
            ach, peak, unit = per_launch / (avg_ms * 1e-3) / 1e12, FP32_PEAK_TFLOPS, "TFLOP/s"
        kernels[k] = {"ms_per_step": kms[k] / args.steps, "launches_per_step": kl[k] // args.steps,
                      "avg_launch_ms": avg_ms, "bound": bound, "achieved": ach, "peak": peak,
                      "unit": unit, "frac": ach / peak}
        traffic = measured_traffic(k)
        if traffic is not None:
            kernels[k]["counter_GBps"] = traffic / (avg_ms * 1e-3) / 1e9
    # the same render replayed as a graph per chunk (no per-kernel events)
    gparams, gkeep = sdm.make_params(st, precision=args.precision, graph=True, chunk_paths=chunk, tile=tile)
    sdm.render_into(ctx, gs, gparams, spec, xyz)
    torch.cuda.synchronize()
    tg = time.perf_counter()
    for _ in range(max(1, args.steps // 2)):
        sdm.render_into(ctx, gs, gparams, spec, xyz)
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - tg) / max(1, args.steps // 2) * 1e3
    # the same render split into 4 and 16 spectral sub-domains (bands)
    band_split = {str(args.bands): dt / args.steps * 1e3}
    if args.bands == 1 and not args.no_band_split:
        for nbands in (4, 16):
            stb = synth.nave_settings(W=512, H=512, spp=64, max_depth=8, n_bands=nbands)
            bp, bkeep = sdm.make_params(stb, precision=args.precision, chunk_paths=chunk, tile=tile)
            sdm.render_into(ctx, gs, bp, spec, xyz)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            for _ in range(3):
                sdm.render_into(ctx, gs, bp, spec, xyz)
            torch.cuda.synchronize()
            band_split[str(nbands)] = (time.perf_counter() - tb) / 3 * 1e3
            print(f"{nbands} bands: {band_split[str(nbands)]:.1f} ms", file=sys.stderr, flush=True)
    # whole-render HBM rate: algorithmic bytes, and the counters' bytes where
    # the committed rocprofv3 summary matches these sources
    ms_step = dt / args.steps * 1e3
    alg_bytes = sum(moved.values())
    ctr = {k: measured_traffic(k) for k in sdm.KERNELS}
    ctr_bytes = (sum(v * (kl[k] // args.steps) for k, v in ctr.items() if v is not None)
                 if any(v is not None for v in ctr.values()) else None)
    copy_gbps = copy_bandwidth()
    hbm = {"ms_per_step": ms_step,
           "algorithmic_bytes": alg_bytes, "algorithmic_GBps": alg_bytes / (ms_step * 1e-3) / 1e9,
           "algorithmic_frac": alg_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "counter_bytes": ctr_bytes,
           "counter_GBps": None if ctr_bytes is None else ctr_bytes / (ms_step * 1e-3) / 1e9,
           "counter_frac": None if ctr_bytes is None else ctr_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "copy_kernel_GBps": copy_gbps, "copy_kernel_frac": copy_gbps / HBM_PEAK_GBS, "peak_GBps": HBM_PEAK_GBS}
    # The shadow walk, accumulation and caustic gather of a bounce run on the
    # library's second stream beside the next bounce's closest-hit pass: their
    # event spans include the time their blocks wait for wave slots, so the
    # dominant kernel is taken among the passes of the caller's stream.
    side = ("shadow", "shadow_accum", "caustic")
    for k in side:
        if k in kernels:
            kernels[k]["stream"] = ("second stream, beside the next bounce's closest-hit pass (the span includes "
                                    "waiting for wave slots; SDM_SERIAL=1 times it alone)")
    dom = max((k for k in kernels if k not in side), key=lambda k: kernels[k]["ms_per_step"])
    kd = kernels[dom]
    roof = {"kernel": dom, "bound": kd["bound"], "achieved": kd["achieved"], "peak": kd["peak"],
            "unit": kd["unit"], "frac": kd["frac"], "traffic": measured_traffic(dom)}
    if kd["bound"] == "alu":
        roof["peak_note"] = ("published FP32 vector rate; the kernels are built without packed FP32 "
                             f"instructions, whose rate is {FP32_UNPACKED_TFLOPS} TFLOP/s")
        roof["frac_of_unpacked_rate"] = kd["achieved"] / FP32_UNPACKED_TFLOPS
        roof["work_model"] = f"{FLOPS_PER_NODE} flop per wide node visited, {FLOPS_PER_TRI} per triangle tested"
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
        "roofline": roof,
        "hbm": hbm,
        "kernels": kernels,
        "band_split_ms": band_split,
        "accel": {"bvh_nodes": info["n_nodes"], "bvh_depth": info["depth"], "stack_bound": info["stack"],
                  "sun_grid_cells": info["grid_cells"], "sun_grid_candidates": info["grid_candidates"]},
        "segments_per_s": (s["closest_segments"] + s["shadow_segments"]) * args.steps / dt,
        "distinct_rays_per_step": {"closest": s["closest_segments"], "shadow": s["shadow_segments"],
                                   "forks": s["forks"], "glass_vertices": s["glass_vertices"]["all"],
                                   "spectral_paths": s["spectral_paths"], "spectral_records": s["spectral_records"]},
        "traversal_per_ray": {k: {"nodes": s["nodes_visited"][k] / max(1, s[seg]),
                                  "tris": s["tris_tested"][k] / max(1, s[seg])}
                              for k, seg in (("closest", "closest_segments"), ("shadow", "shadow_segments"))},
        "graph_replay": {"ms_per_step": graph_ms, "value": samples / (graph_ms * 1e-3)},
        "chunk_paths": chunk, "tile": list(tile), "autotune": tuned,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, st)
    ctx.close()
    if not args.no_surrogate:
        # the other half of the metric: the same nave with its panes bubbly,
        # plain form (exact walks) against the trained surrogate at a mean
        # block dE2000 < 1 (the whole run of --form bubbly, summarised)
        b = bubbly_bench(args, emit=False)
        f = b["forms"]
        out["surrogate_form"] = {
            "metric": b["metric"], "workload": b["config"]["workload"], "surrogate": b["config"]["surrogate"],
            "plain_value": f["exact"]["value"], "plain_ms": f["exact"]["ms_per_step"],
            "surrogate_value": f["surrogate"]["value"], "surrogate_ms": f["surrogate"]["ms_per_step"],
            "surrogate_vs_plain": f["surrogate"]["value"] / f["exact"]["value"],
            "fallback_value": f["fallback"]["value"], "bubble_free_value": f["bubble_free"]["value"],
            "reference": b["reference"],
            "block_de2000_vs_reference": b["mean_delta_e2000_vs_reference_16x16_blocks"],
            "pixel_de2000_vs_reference": b["mean_delta_e2000_vs_reference"],
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
