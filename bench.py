"""Benchmark: combined ray query vs triangle-only vs distance-field-only on the
GI-shaped workload (188k-triangle room, 128^3 exact grid, one cosine diffuse
ray per pixel of a 1920x1080 rasterized G-buffer, tmax 0.5).

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  `value` is the combined query's rays/s (Mrays/s) at the
smallest threshold of the sweep {0, 0.5, 1, 2, 4, inf} voxels whose artefact
rate against triangle-only tracing is no worse than that of distance-field-only
tracing at twice the grid resolution (the paper's setup gives the DF-only path
the finer grid, Section 3).  A step is one trace of all rays; inputs are
resident in device memory before timing starts.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TAUS = (0.0, 0.5, 1.0, 2.0, 4.0, math.inf)
TMAX = 0.5
HBM_PEAK_GBS = 8000.0
# Vector ALU issue rate of one MI355X: 256 compute units x 4 SIMDs x 16 lanes
# x 2.4 GHz, one unpacked FP32 (or integer) lane operation per lane and clock
# (a wave64 instruction issues over 4 clocks); an FMA counts as one operation.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
N_SIMD, CLOCK_HZ = 256 * 4, 2.4e9

# Algorithmic work per unit of the path (the traversal and march themselves):
# bytes moved and VALU lane operations per four-wide BVH node visited (four
# boxes of 24 B + four child references; four slab tests), per triangle tested
# (48 B; the watertight test), per distance-field fetch (8 FP32 corners; the
# trilinear value and the step), plus 24 B of ray in and 16 B of hit out.
BYTES_RAY, BYTES_NODE, BYTES_TRI, BYTES_FETCH = 40.0, 128.0, 48.0, 32.0
OPS_NODE, OPS_TRI, OPS_FETCH = 48.0, 35.0, 30.0

# The paper's own measurements (Fig. 1 and Fig. 2; AMD Radeon RX 6800 XT,
# DX12/DXR research renderer, resolution and ray counts not stated): context,
# not targets, and not comparable per ray.
PAPER = {
    "hardware": "AMD Radeon RX 6800 XT (hardware ray tracing), DX12/DXR; resolution and ray count not stated",
    "gi10_frame_ms": {"hwrt_only": 5.66, "combined": 4.55, "df_only": 3.58, "source": "Fig. 1"},
    "ao_tracing_ms": [
        {"scene": "Bistro, AO distance 100", "hwrt_only": 8.33, "combined": 3.16, "df_only": 1.35, "source": "Fig. 2"},
        {"scene": "simpler scene, AO distance 10", "hwrt_only": 2.73, "combined": 1.86, "df_only": 1.13,
         "source": "Fig. 2"},
        {"scene": "simpler scene, AO distance 10", "hwrt_only": 1.72, "combined": 1.64, "df_only": 1.14,
         "source": "Fig. 2"}],
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# Untimed load before every timed section: after the host work between
# sections (a fraction of a second with the GPU idle) the first launches run
# up to 10% slower until the GPU's clock has settled under load, which takes
# some tens of ms (0.33 ms per launch of the threshold-0 query after 3 warm
# launches, 0.300 ms after 30 ms or more of them).
SETTLE_MS = 50.0


def settle(fn, warmup):
    """`warmup` untimed calls of fn(), then about SETTLE_MS more of them,
    issued back to back with one wait at the end (frequent waits between
    launches left the following launches slower for a few ms)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    one = max(time.perf_counter() - t0, 1e-5)
    for _ in range(min(int(SETTLE_MS * 1e-3 / one), 5000)):
        fn()
    torch.cuda.synchronize()


def time_launches(fn, stream, reps, warmup):
    """Average duration of fn() (one kernel launch) over `reps` launches,
    bracketed by HIP events on the stream the kernel runs on, after `warmup`
    untimed launches and SETTLE_MS of untimed load."""
    import torch
    settle(fn, warmup)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / reps


def source_sha256():
    """Hash of the kernel sources' code: whole-line // comments and blank
    lines are left out, so editing a comment keeps a traffic record valid."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2305_07253_amd", "csrc", "*"))):
        if f.endswith((".hpp", ".hip", ".cpp")):
            for line in open(f, encoding="utf-8"):
                code = line.strip()
                if code and not code.startswith("//"):
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def measured_counters(tau):
    """Counters per launch of the GI query at this threshold from the
    committed rocprofv3 summary (profiles/counters_gi1080p.json), if they were
    taken on the current kernel source; else None."""
    f = os.path.join(ROOT, "profiles", "counters_gi1080p.json")
    if not os.path.exists(f):
        return None
    rec = json.load(open(f))
    if rec.get("source_sha256") != source_sha256():
        return None
    key = "inf" if math.isinf(tau) else repr(float(tau))
    return rec.get("thresholds", {}).get(key)


def work_model(c):
    """Algorithmic bytes and VALU lane operations per ray from mean counts
    (four-wide nodes, triangles, distance-field fetches)."""
    b = BYTES_RAY + BYTES_NODE * c[0] + BYTES_TRI * c[1] + BYTES_FETCH * c[2]
    ops = OPS_NODE * c[0] + OPS_TRI * c[1] + OPS_FETCH * c[2]
    return b, ops


def roofline(c, n, ms, tau):
    """Roofline of one query launch: the VALU roof (the kernels issue-bound
    under divergence, which the counters show) with the HBM figures beside it;
    `traffic` and the issue model come from the committed counters when they
    match the source."""
    b, ops = work_model(c)
    sec = ms * 1e-3
    alu = ops * n / sec / 1e12
    gbs = b * n / sec / 1e9
    prof = measured_counters(tau)
    r = {"bound": "alu", "achieved": alu, "peak": VALU_PEAK_TOPS, "unit": "TOP/s (VALU lane operations)",
         "frac": alu / VALU_PEAK_TOPS, "traffic": None if prof is None else prof["read_bytes"] + prof["write_bytes"],
         "ops_per_ray": ops, "bytes_per_ray": b, "nodes_per_ray": float(c[0]), "tris_per_ray": float(c[1]),
         "df_fetches_per_ray": float(c[2]),
         "hbm": {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}}
    if prof is not None:
        issue_s = prof["valu_insts"] * 4.0 / N_SIMD / CLOCK_HZ
        r["issue"] = {"valu_insts_per_launch": prof["valu_insts"], "valu_issue_us": issue_s * 1e6,
                      "valu_issue_frac_of_launch": issue_s / (prof["kernel_us"] * 1e-6),
                      "lane_utilisation": prof["lane_utilisation"], "l2_hit": prof["l2_hit"],
                      "kernel": prof["kernel"], "profile_kernel_us": prof["kernel_us"]}
    return r


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def artefacts(t, prim, o, d, t_ref, prim_ref, o_ref, h):
    """Artefact rate against the triangle reference: hit/miss differs, or the
    hit points are more than one voxel apart; plus |dp|/h statistics over rays
    that hit in both."""
    hit, hit_ref = prim != -1, prim_ref != -1
    both = hit & hit_ref
    p = o[both] + t[both, None] * d[both]
    q = o_ref[both] + t_ref[both, None] * d[both]
    dp = np.linalg.norm(p - q, axis=1) / h
    bad = (hit != hit_ref).sum() + (dp > 1.0).sum()
    return dict(rate=float(bad / len(t)), mean_dp_over_h=float(dp.mean()) if len(dp) else 0.0,
                p99_dp_over_h=float(np.percentile(dp, 99)) if len(dp) else 0.0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed launches before the timed region (200 at threshold 0 are about 60 ms of load, "
                         "enough for the GPU's clock to settle)")
    ap.add_argument("--reps", type=int, default=10, help="launches per sweep point")
    ap.add_argument("--cpu-sample", type=int, default=4096, help="rays for the CPU oracle baseline (0: skip)")
    ap.add_argument("--tau", type=float, default=None,
                    help="fix the threshold (voxels) instead of selecting it at the fixed artefact rate")
    ap.add_argument("--profile", action="store_true",
                    help="profiling driver: a 256 MiB copy probe, then --steps launches of the combined, "
                         "triangle-only and DF-only kernels; no sweep, no JSON line")
    ap.add_argument("--config", default="gi", choices=["gi", "diff", "precision", "batch", "shadow", "ao"],
                    help="gi: the headline combined-query benchmark (one JSON line with value); the others print "
                         "their own JSON line for the differentiation, precision, batching and shadow workloads")
    ap.add_argument("--adam-steps", type=int, default=200)
    ap.add_argument("--lr-scale", type=float, default=0.002, help="Adam learning rate in voxels (diff config)")
    ap.add_argument("--loss", default="dfhit", choices=["both", "dfhit"],
                    help="diff config: MSE over rays where both hit, or over every DF hit with triangle misses "
                         "targeting tmax (pulls false DF hits out)")
    ap.add_argument("--oracle-sample", type=int, default=2048, help="precision config: rays checked by the oracle")
    ap.add_argument("--max-error", type=float, default=0.03,
                    help="batch config: per-scene cap on the fraction of rays that differ from triangles-only")
    ap.add_argument("--scenes", type=int, default=64, help="batch config: number of scenes")
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="gi config: skip the GPU timings of the shadow, refit, precision and batch workloads")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the ray query shards by rays with no exchange step; "
              "a multi-GPU job is one independent process per GPU on its share of the rays", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2305_07253_amd as hyb
    from paper_2305_07253_amd import workloads as W

    hyb.lib()
    if args.config != "gi":
        return run_extra(args)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    t0 = time.time()
    scene = W.gi_scene(2)
    g128, g256 = W.room_grid(128), W.room_grid(256)
    h128, h256 = float(g128[3]), float(g256[3])
    gb = W.gbuffer(scene, args.width, args.height)
    rays = W.gbuffer_rays(gb, 21)
    rays_df128 = W.rebias(rays, gb, h128)
    rays_df256 = W.rebias(rays, gb, h256)
    n = rays.n
    log("workload: %d triangles, %d rays (%.1fs)" % (scene.n_tris, n, time.time() - t0))

    t0 = time.time()
    bvh = hyb.build_bvh(scene.verts, scene.tris)
    t_bvh = time.time() - t0
    t0 = time.time()
    sdf128 = hyb.build_sdf(bvh, 128, g128)
    torch.cuda.synchronize()
    t_sdf128 = time.time() - t0
    sdf256 = hyb.build_sdf(bvh, 256, g256)
    log("bvh %d nodes depth %d (%.2fs); sdf128 L=%.4f (%.2fs); sdf256 L=%.4f" % (
        bvh.n_nodes, bvh.depth, t_bvh, sdf128.lipschitz, t_sdf128, sdf256.lipschitz))

    R = torch.from_numpy(rays.soa()).to(dev)
    R128 = torch.from_numpy(rays_df128.soa()).to(dev)
    R256 = torch.from_numpy(rays_df256.soa()).to(dev)
    out = hyb.alloc_hits(n)
    o_np, d_np = rays.o.astype(np.float64), rays.d.astype(np.float64)

    if args.profile:
        # counters do not depend on the clock: each phase runs its warm-up and
        # steps only, so a counter run has the same dispatches every time
        global SETTLE_MS
        SETTLE_MS = 0.0
        tau = 0.0 if args.tau is None else args.tau
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev)  # 256 MiB copy probe
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        srays, stmax = W.shadow_rays(gb.p, gb.n, 22)
        RS, TS = torch.from_numpy(srays.soa()).to(dev), torch.from_numpy(stmax).to(dev)
        s16 = hyb.build_sdf(bvh, 128, g128, fmt=hyb.SDF_F16)
        s8 = hyb.build_sdf(bvh, 128, g128, fmt=hyb.SDF_I8_BRICK)
        for name, fn in (("combined", lambda: hyb.trace(bvh, sdf128, R, TMAX, tau, out=out)),
                         ("bvh_only", lambda: hyb.trace_bvh(bvh, R, TMAX, out=out)),
                         ("df_only", lambda: hyb.trace_df(sdf128, R128, TMAX, out=out)),
                         ("combined_f16", lambda: hyb.trace(bvh, s16, R, TMAX, tau, out=out)),
                         ("combined_i8", lambda: hyb.trace(bvh, s8, R, TMAX, tau, out=out)),
                         ("shadow", lambda: hyb.trace_shadow(bvh, sdf128, RS, 10.0, 1.0, 1.0, tmax_ray=TS, out=out)),
                         ("shadow_bvh", lambda: hyb.trace_bvh(bvh, RS, 10.0, tmax_ray=TS, out=out))):
            ms = time_launches(fn, stream, args.steps, args.warmup)
            log("%s: %.4f ms per launch (%d rays)" % (name, ms, n))
        torch.cuda.synchronize()
        return

    # triangle-only reference and timing
    ms_bvh = time_launches(lambda: hyb.trace_bvh(bvh, R, TMAX, out=out), stream, args.reps, 2)
    ref_t, ref_p = out[0].cpu().numpy().astype(np.float64), out[1].cpu().numpy()

    sweep = []
    for tau in TAUS:
        ms = time_launches(lambda: hyb.trace(bvh, sdf128, R, TMAX, tau, out=out), stream, args.reps, 2)
        t, p = out[0].cpu().numpy().astype(np.float64), out[1].cpu().numpy()
        a = artefacts(t, p, o_np, d_np, ref_t, ref_p, o_np, h128)
        sweep.append(dict(tau=tau if math.isfinite(tau) else "inf", ms=ms, mrays_s=n / ms / 1e3, **a))
        log("tau=%s: %.3f ms %.1f Mrays/s artefacts %.4f" % (tau, ms, n / ms / 1e3, a["rate"]))

    df_only = {}
    for name, sdf, Rb, rb, hh in (("df128", sdf128, R128, rays_df128, h128), ("df256", sdf256, R256, rays_df256, h256)):
        ms = time_launches(lambda: hyb.trace_df(sdf, Rb, TMAX, out=out), stream, args.reps, 2)
        t, p = out[0].cpu().numpy().astype(np.float64), out[1].cpu().numpy()
        a = artefacts(t, p, rb.o.astype(np.float64), d_np, ref_t, ref_p, o_np, h128)
        df_only[name] = dict(ms=ms, mrays_s=n / ms / 1e3, **a)
        log("%s only: %.3f ms %.1f Mrays/s artefacts %.4f" % (name, ms, n / ms / 1e3, a["rate"]))

    target = df_only["df256"]["rate"]
    chosen = next((s for s in sweep if s["rate"] <= target), sweep[-1])
    if args.tau is not None:
        chosen = next((s for s in sweep if s["tau"] == (args.tau if math.isfinite(args.tau) else "inf")), chosen)
    tau = math.inf if chosen["tau"] == "inf" else chosen["tau"]

    # work counters at the chosen threshold -> algorithmic bytes per ray
    def counts(t):
        (_, _, _, _), cnt = hyb.trace_counters(bvh, sdf128, R, TMAX, t, hyb.MODE_COMBINED)
        cnt_np = cnt.cpu().numpy()
        return cnt.double().mean(dim=0).cpu().numpy(), {
            name: {"mean": float(cnt_np[:, k].mean()), "p50": float(np.percentile(cnt_np[:, k], 50)),
                   "p99": float(np.percentile(cnt_np[:, k], 99)), "max": int(cnt_np[:, k].max())}
            for k, name in enumerate(("bvh_nodes", "triangles", "df_fetches"))}

    c, work = counts(tau)

    # timed region: K steps of the combined query at the chosen threshold,
    # right after the warm-up
    for _ in range(args.warmup):
        hyb.trace(bvh, sdf128, R, TMAX, tau, out=out)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.time()
    start.record(stream)
    for _ in range(args.steps):
        hyb.trace(bvh, sdf128, R, TMAX, tau, out=out)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - wall0
    ms_step = start.elapsed_time(stop) / args.steps
    value = n / ms_step / 1e3  # Mrays/s
    # the median of K single launches, each bracketed by its own events, after
    # the timed region (run between the warm-up and the timed region, these
    # event-bracketed launches left the next few ms of back-to-back launches
    # up to 10% slower); the timed launches are the K before the last K
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in evs:
        e0.record(stream)
        hyb.trace(bvh, sdf128, R, TMAX, tau, out=out)
        e1.record(stream)
    torch.cuda.synchronize()
    ms_median = float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))

    # the combined query that runs both techniques on every ray (threshold 1
    # voxel): its own time, work, roofline and error
    s1 = next(s for s in sweep if s["tau"] == 1.0)
    c1, work1 = counts(1.0)
    ms1 = time_launches(lambda: hyb.trace(bvh, sdf128, R, TMAX, 1.0, out=out), stream, args.steps, args.warmup)
    combined_tau1 = {"threshold": 1.0, "ms": ms1, "mrays_s": n / ms1 / 1e3, "speedup_vs_bvh_only": ms_bvh / ms1,
                     "artefact_rate": s1["rate"], "mean_dp_over_h": s1["mean_dp_over_h"],
                     "roofline": roofline(c1, n, ms1, 1.0), "work_per_ray": work1}
    log("tau=1: %.3f ms, ALU frac %.3f, HBM frac %.3f" % (ms1, combined_tau1["roofline"]["frac"],
                                                          combined_tau1["roofline"]["hbm"]["frac"]))
    extras = run_extras(args, torch, hyb, W, dev, stream, scene, gb, bvh, g128) if args.extras else None

    cpu = None
    if args.cpu_sample > 0:
        import oracle
        oracle.build()
        log("oracle grid 128^3 (setup, untimed)")
        og = oracle.sdf_grid(scene, g128, 128)
        # grow a fixed-stride sample until it holds about 15 s of oracle work
        m = args.cpu_sample
        while True:
            idx = np.linspace(0, n - 1, m).astype(np.int64)
            sub = rays.subset(idx)
            t0 = time.time()
            oracle.query(scene.verts, scene.tris, og, g128, sub.soa(), TMAX, tau)
            el = time.time() - t0
            if el >= 10.0 or m >= n:
                break
            m = int(min(n, max(2 * m, m * 15.0 / max(el, 1e-3))))
        cpu = dict(value=sub.n / el / 1e6, unit="Mrays/s", cores=oracle.threads(), kind="oracle", cpu_model=cpu_model(),
                   sample="%d of the %d rays at a fixed stride over the tile-ordered G-buffer rays (%.1f s), "
                          "combined query at threshold %s in FP64: %s" % (
                              sub.n, n, el, chosen["tau"],
                              "distance field only (the triangle segment is empty at threshold 0), cell-by-cell "
                              "walk with exact per-cell roots" if tau == 0 else
                              "brute force over all %d triangles on the triangle segment, cell-by-cell walk with "
                              "exact per-cell roots on the distance-field segment" % scene.n_tris))
        log("cpu oracle: %.4f Mrays/s (%.1fs, %d threads)" % (cpu["value"], el, cpu["cores"]))

    line = {
        "metric": "Mrays/s for combined vs BVH-only vs DF-only at fixed t-error; HBM GB/s % of peak",
        "value": value,
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_launch_median": ms_median,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "GI-shaped: %d-triangle room, 128^3 FP32 exact SDF, %dx%d G-buffer cosine "
                               "diffuse rays (%d), tmax 0.5, threshold %s voxels" % (
                                   scene.n_tris, args.width, args.height, n, chosen["tau"]),
                   "rays": n, "triangles": scene.n_tris, "grid": 128, "tmax": TMAX, "threshold": chosen["tau"]},
        "roofline": roofline(c, n, ms_step, tau),
        "cpu_baseline": cpu,
        "combined_tau1": combined_tau1,
        "bvh_only": {"ms": ms_bvh, "mrays_s": n / ms_bvh / 1e3},
        "df_only": df_only,
        "sweep": sweep,
        "target_artefact_rate": target,
        "speedup_vs_bvh_only": ms_bvh / ms_step,
        "work_per_ray": work,
        "timed_wall_s": wall,
        "extras": extras,
        "paper": PAPER,
    }
    print(json.dumps(line), flush=True)


def run_extras(args, torch, hyb, W, dev, stream, scene, gb, bvh, g128):
    """GPU timings of the other workloads (no oracle): shadow rays and the
    refit step on the GI scene, the 256^3 precision workload in three storage
    formats, and the 64-scene batch in one graph launch."""
    t0 = time.time()
    ex = {}
    sdf = hyb.build_sdf(bvh, 128, g128)
    h = float(g128[3])
    # shadow rays to an area light: thresholds (1, 1) against exact any-hit triangles
    srays, stmax = W.shadow_rays(gb.p, gb.n, 22)
    RS, TS = torch.from_numpy(srays.soa()).to(dev), torch.from_numpy(stmax).to(dev)
    out = hyb.alloc_hits(srays.n)
    ms_ref = time_launches(lambda: hyb.trace_shadow(bvh, sdf, RS, 10.0, math.inf, math.inf, tmax_ray=TS, out=out),
                           stream, args.reps, 2)
    ref = out[1].cpu().numpy() != -1
    ms_s = time_launches(lambda: hyb.trace_shadow(bvh, sdf, RS, 10.0, 1.0, 1.0, tmax_ray=TS, out=out), stream,
                         args.reps, 2)
    occ = out[1].cpu().numpy() != -1
    ex["shadow"] = {"workload": "%d shadow rays from the GI G-buffer to a 0.3 x 0.3 area light, any hit" % srays.n,
                    "thresholds": [1.0, 1.0], "ms": ms_s, "mrays_s": srays.n / ms_s / 1e3,
                    "triangles_anyhit_ms": ms_ref, "speedup": ms_ref / ms_s,
                    "occlusion_mismatch": float((occ != ref).mean())}
    log("extras: shadow %.3f ms vs %.3f ms (%.1fs)" % (ms_s, ms_ref, time.time() - t0))

    # refit: forward, backward and one Adam step on a learnable 128^3 grid
    from paper_2305_07253_amd.autograd import df_hit
    gbr = W.gbuffer(scene, 1024, 1024)
    rr = W.rebias(W.gbuffer_rays(gbr, 41), gbr, h)
    RR = torch.from_numpy(rr.soa()).to(dev)
    target = hyb.trace_bvh(bvh, torch.from_numpy(W.gbuffer_rays(gbr, 41).soa()).to(dev), TMAX)[0]
    goal = torch.where(torch.isfinite(target), target, torch.full_like(target, TMAX))
    theta = hyb.sdf_read(sdf).reshape(-1).contiguous().clone().requires_grad_(True)
    handle = hyb.sdf_from_grid(theta.detach().clone(), g128)
    opt = torch.optim.Adam([theta], lr=0.002 * h)

    def adam_step():
        opt.zero_grad()
        t = df_hit(theta, g128, RR, TMAX, sdf=handle)
        use = torch.isfinite(t)
        d = torch.where(use, t - goal, torch.zeros_like(t))
        ((d * d).sum() / use.sum().clamp(min=1)).backward()
        opt.step()

    # the GPU settles on the forward query, which leaves the grid alone; the
    # optimiser then takes a fixed number of steps, so the timed steps and
    # kernels always see the same grid
    o2 = hyb.alloc_hits(rr.n)
    settle(lambda: hyb.trace_df(handle, RR, TMAX, out=o2), 0)
    for _ in range(5):
        adam_step()
    torch.cuda.synchronize()
    t1 = time.time()
    for _ in range(20):
        adam_step()
    torch.cuda.synchronize()
    step_ms = (time.time() - t1) * 1e3 / 20
    ms_fwd = time_launches(lambda: hyb.trace_df(handle, RR, TMAX, out=o2), stream, args.reps, 2)
    grad = torch.zeros(128 ** 3, device=dev)
    ones = torch.ones(rr.n, device=dev)
    ms_bwd = time_launches(lambda: hyb.df_backward(handle, RR, TMAX, o2[0], ones, grad), stream, args.reps, 2)
    ex["refit"] = {"workload": "128^3 FP32 learnable grid, %d G-buffer rays from p + h n, loss MSE vs triangle hits"
                   % rr.n, "ms_per_adam_step": step_ms, "forward_kernel_ms": ms_fwd, "backward_kernel_ms": ms_bwd}
    log("extras: refit step %.3f ms, fwd %.3f, bwd %.3f (%.1fs)" % (step_ms, ms_fwd, ms_bwd, time.time() - t0))
    del theta, handle, opt, grad

    # precision workload: 1.88M triangles, 256^3, 8.3M rays, three formats
    ps = W.precision_scene(3)
    g256 = W.room_grid(256)
    prays = W.gbuffer_rays(W.gbuffer(ps, 1920, 1080), 31, spp=4)
    pbvh = hyb.build_bvh(ps.verts, ps.tris)
    f32 = hyb.build_sdf(pbvh, 256, g256)
    vals = hyb.sdf_read(f32).reshape(-1).contiguous()
    grids = {"f32": f32, "f16": hyb.sdf_from_grid(vals, g256, fmt=hyb.SDF_F16),
             "i8": hyb.sdf_from_grid(vals, g256, fmt=hyb.SDF_I8_BRICK)}
    del vals
    PR = torch.from_numpy(prays.soa()).to(dev)
    po = hyb.alloc_hits(prays.n)
    prec = {"workload": "%d triangles, 256^3 grid, %d rays (4 per pixel at 1080p), tmax 0.5" % (ps.n_tris, prays.n)}
    for tau in (0.0, 1.0):
        for name, g in grids.items():
            ms = time_launches(lambda: hyb.trace(pbvh, g, PR, TMAX, tau, out=po), stream, args.reps, 2)
            prec["%s_tau%g_ms" % (name, tau)] = ms
    prec["bvh_only_ms"] = time_launches(lambda: hyb.trace_bvh(pbvh, PR, TMAX, out=po), stream, args.reps, 2)
    ex["precision"] = prec
    log("extras: precision %s (%.1fs)" % (prec, time.time() - t0))
    del grids, f32, pbvh, PR, po

    # 64 scenes of uneven size in one persistent graph launch, autotuned
    items, n_rays = [], 0
    for sp in W.batch_specs(4, 64):
        bs = W.batch_scene(sp)
        bb = hyb.build_bvh(bs.verts, bs.tris)
        brays = W.gbuffer_rays(W.gbuffer(bs, sp.width, sp.height), sp.seed)
        items.append(dict(bvh=bb, sdf=hyb.build_sdf(bb, sp.n_grid, W.room_grid(sp.n_grid)),
                          rays=torch.from_numpy(brays.soa()).to(dev), tmax=TMAX, threshold=1.0))
        n_rays += brays.n
    batch = hyb.Batch(items)
    err, _ = batch.tune(max_error_rate=0.03, reps=3)
    taus = [batch.threshold(k) for k in range(len(items))]
    ms_graph = time_launches(lambda: batch.launch(), stream, args.reps, 2)

    def per_scene():
        for k, it in enumerate(items):
            hyb.trace(it["bvh"], it["sdf"], it["rays"], TMAX, taus[k], out=batch.outs[k])

    ms_loop = time_launches(per_scene, stream, args.reps, 2)
    ex["batch"] = {"workload": "64 scenes (log-uniform 1k-500k triangles, %d rays in all), one graph launch, "
                   "thresholds tuned per scene under a 3%% error cap" % n_rays, "ms_graph": ms_graph,
                   "mrays_s": n_rays / ms_graph / 1e3, "ms_per_scene_launches": ms_loop,
                   "speedup_vs_per_scene_launches": ms_loop / ms_graph, "error_rate_max": float(np.max(err)),
                   "config": batch.config}
    log("extras: batch %.3f ms vs %.3f ms per scene (%.1fs)" % (ms_graph, ms_loop, time.time() - t0))
    ex["seconds"] = time.time() - t0
    return ex


def run_extra(args):
    import torch
    import paper_2305_07253_amd as hyb
    from paper_2305_07253_amd import workloads as W
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.config == "diff":
        line = bench_diff(args, torch, hyb, W, dev, stream)
    elif args.config == "precision":
        line = bench_precision(args, torch, hyb, W, dev, stream)
    elif args.config == "batch":
        line = bench_batch(args, torch, hyb, W, dev, stream)
    elif args.config == "shadow":
        line = bench_shadow(args, torch, hyb, W, dev, stream)
    elif args.config == "ao":
        line = bench_ao(args, torch, hyb, W, dev, stream)
    else:
        raise SystemExit("config %s not implemented" % args.config)
    print(json.dumps(line), flush=True)


def bench_precision(args, torch, hyb, W, dev, stream):
    """2M-triangle scene, 256^3 grid stored FP32 / FP16 / int8 + block scales,
    4 rays per pixel at 1080p; rays/s per format and each format's t error
    against the FP64 oracle on the exact grid (a fixed-stride ray sample)."""
    import oracle
    oracle.build()
    t0 = time.time()
    scene = W.precision_scene(3)
    g4 = W.room_grid(256)
    h = float(g4[3])
    gb = W.gbuffer(scene, args.width, args.height)
    rays = W.gbuffer_rays(gb, 31, spp=4)
    log("precision workload: %d triangles, %d rays (%.1fs)" % (scene.n_tris, rays.n, time.time() - t0))
    t0 = time.time()
    bvh = hyb.build_bvh(scene.verts, scene.tris)
    t_bvh = time.time() - t0
    t0 = time.time()
    f32 = hyb.build_sdf(bvh, 256, g4)
    torch.cuda.synchronize()
    t_sdf = time.time() - t0
    vals = hyb.sdf_read(f32).reshape(-1).contiguous()
    grids = {"f32": f32, "f16": hyb.sdf_from_grid(vals, g4, fmt=hyb.SDF_F16),
             "i8": hyb.sdf_from_grid(vals, g4, fmt=hyb.SDF_I8_BRICK)}
    log("bvh %.1fs (%d nodes, depth %d), sdf 256^3 %.2fs" % (t_bvh, bvh.n_nodes, bvh.depth, t_sdf))
    R = torch.from_numpy(rays.soa()).to(dev)
    out = hyb.alloc_hits(rays.n)
    idx = np.linspace(0, rays.n - 1, args.oracle_sample).astype(np.int64)
    sub = rays.subset(idx)
    t0 = time.time()
    og, n_nodes = oracle.sdf_grid_sparse(scene, g4, 256, sub.o, sub.d, TMAX, progress=log)
    log("oracle: exact samples at %d nodes (%.1fs)" % (n_nodes, time.time() - t0))
    refs = {tau: oracle.query(scene.verts, scene.tris, og, g4, sub.soa(), TMAX, tau) for tau in (0.0, 1.0)}
    for ref in refs.values():
        assert np.all(np.isfinite(ref[0]) | (ref[1] == -1)), "oracle read a node outside the sampled cells"
    # the oracle above kept the GPU idle for a minute or more: bring it back to
    # its working clocks before timing (a second of launches; nothing but GPU
    # work and the checks of its results runs between here and the last timing)
    t0 = time.time()
    while time.time() - t0 < 1.0:
        hyb.trace(bvh, grids["f32"], R, TMAX, 0.0, out=out)
        torch.cuda.synchronize()
    res = {}
    for tau in (0.0, 1.0):
        ref = refs[tau]
        for name, sdf in grids.items():
            ms = time_launches(lambda: hyb.trace(bvh, sdf, R, TMAX, tau, out=out), stream, 20, 3)
            t = out[0].cpu().numpy()[idx].astype(np.float64)
            prim = out[1].cpu().numpy()[idx]
            same = (prim == ref[1]) | ((prim >= 0) & (ref[1] >= 0))
            both = np.isfinite(t) & np.isfinite(ref[0])
            rel = np.abs(t - ref[0])[both] / np.maximum(ref[0][both], 0.05)
            res["%s_tau%s" % (name, tau)] = dict(
                ms=ms, mrays_s=rays.n / ms / 1e3, class_agreement=float(same.mean()),
                hit_agreement=float((np.isfinite(t) == np.isfinite(ref[0])).mean()),
                rel_t_err_mean=float(rel.mean()), rel_t_err_p99=float(np.percentile(rel, 99)),
                rel_t_err_max=float(rel.max()), abs_t_err_over_h_p99=float(np.percentile(rel * np.maximum(
                    ref[0][both], 0.05) / h, 99)))
            log("%s tau=%s: %.3f ms (%.0f Mrays/s), class agreement %.5f, rel t err mean %.2e p99 %.2e" % (
                name, tau, ms, rays.n / ms / 1e3, same.mean(), rel.mean(), np.percentile(rel, 99)))
    return {"config": "precision", "workload": "%d-triangle room, 256^3 grid (h=1/251), %d rays (4 per pixel, "
            "1920x1080 G-buffer), tmax 0.5" % (scene.n_tris, rays.n), "oracle_sample": int(len(idx)),
            # the bricked copies the kernels read at n = 256: FP32 and F16 in
            # two-cell bricks of 32 slots (128^3 bricks; F16 takes them past
            # n = 205), I8 in one-cell bricks of 8 codes + the block scale
            # (255^3 cells of 12 B); I8 also keeps its 32^3 block scales
            "kernel_store_bytes": {"f32": 4 * 32 * 128 ** 3, "f16": 2 * 32 * 128 ** 3, "i8": 12 * 255 ** 3},
            "i8_scale_table_bytes": 4 * 32 ** 3,
            "linear_fp32_bytes": 4 * 256 ** 3,
            "results": res}


def bench_diff(args, torch, hyb, W, dev, stream):
    """Refit the DF against triangle hits: forward DF-only hit t from p + h n on
    [0, 0.5], loss = MSE against triangle-only t from the same origins over rays
    where both hit, backward by implicit differentiation, Adam on the samples."""
    from paper_2305_07253_amd.autograd import df_hit
    scene = W.gi_scene(2)
    g4 = W.room_grid(128)
    h = float(g4[3])
    gb = W.gbuffer(scene, 1024, 1024)
    rays = W.rebias(W.gbuffer_rays(gb, 41), gb, h)
    held = W.rebias(W.gbuffer_rays(gb, 42), gb, h)
    bvh = hyb.build_bvh(scene.verts, scene.tris)
    theta0 = hyb.sdf_read(hyb.build_sdf(bvh, 128, g4)).reshape(-1).contiguous()
    R = torch.from_numpy(rays.soa()).to(dev)
    Rh = torch.from_numpy(held.soa()).to(dev)
    target = hyb.trace_bvh(bvh, R, TMAX)[0]
    target_h = hyb.trace_bvh(bvh, Rh, TMAX)[0]

    def artefact_rate(theta, Rx, tref):
        t = hyb.trace_df(hyb.sdf_from_grid(theta.detach().contiguous(), g4), Rx, TMAX)[0]
        hit, hit_ref = torch.isfinite(t), torch.isfinite(tref)
        both = hit & hit_ref
        bad = (hit != hit_ref).sum() + ((t - tref).abs()[both] > h).sum()
        return float(bad) / t.numel(), float(((t - tref).abs()[both] / h).mean())

    goal = torch.where(torch.isfinite(target), target, torch.full_like(target, TMAX))

    def loss_of(theta, grid=None):
        t = df_hit(theta, g4, R, TMAX, sdf=grid)
        if args.loss == "both":
            use = torch.isfinite(t) & torch.isfinite(target)
            d = torch.where(use, t - target, torch.zeros_like(t))
        else:
            use = torch.isfinite(t)
            d = torch.where(use, t - goal, torch.zeros_like(t))
        return (d * d).sum() / use.sum().clamp(min=1)

    before = artefact_rate(theta0, Rh, target_h)

    def run(theta, steps, grid, losses):
        """Adam steps; wall clock per step (forward, backward, Adam, loss read
        back) from step 10 on: the first steps also load torch's and Adam's
        kernels.  grid: the handle the forward updates in place, or None for
        a new grid per step."""
        opt = torch.optim.Adam([theta], lr=args.lr_scale * h)
        skip = min(10, steps // 2)
        t0 = time.time()
        for it in range(steps):
            if it == skip:
                torch.cuda.synchronize()
                t0 = time.time()
            opt.zero_grad()
            loss = loss_of(theta, grid)
            loss.backward()
            opt.step()
            losses.append(float(loss.detach()))
            if it % 50 == 0:
                log("adam step %d loss %.3e" % (it, losses[-1]))
        torch.cuda.synchronize()
        return (time.time() - t0) * 1e3 / max(steps - skip, 1), steps - skip

    # a new grid per step, on a copy (for comparison only)
    ms_new_grid, _ = run(theta0.clone().requires_grad_(True), 40, None, [])
    theta = theta0.clone().requires_grad_(True)
    losses = []
    step_ms, timed = run(theta, args.adam_steps, hyb.sdf_from_grid(theta0.clone(), g4), losses)
    after = artefact_rate(theta, Rh, target_h)
    # kernel times of one forward and one backward on the final grid
    sdf = hyb.sdf_from_grid(theta.detach().contiguous(), g4)
    out = hyb.alloc_hits(rays.n)
    ms_fwd = time_launches(lambda: hyb.trace_df(sdf, R, TMAX, out=out), stream, 20, 2)
    grad = torch.zeros(128 ** 3, device=dev)
    ones = torch.ones(rays.n, device=dev)
    ms_bwd = time_launches(lambda: hyb.df_backward(sdf, R, TMAX, out[0], ones, grad), stream, 20, 2)
    x = theta.detach().contiguous()
    torch.cuda.synchronize()
    t1 = time.time()
    for _ in range(20):
        hyb.sdf_from_grid(x, g4)
    torch.cuda.synchronize()
    ms_upload = (time.time() - t1) * 1e3 / 20
    torch.cuda.synchronize()
    t1 = time.time()
    for _ in range(20):
        hyb.sdf_update(sdf, x)
    torch.cuda.synchronize()
    ms_update = (time.time() - t1) * 1e3 / 20
    log("refit: loss %.3e -> %.3e; artefacts %.4f -> %.4f; step %.2f ms" % (losses[0], losses[-1], before[0],
                                                                            after[0], step_ms))
    return {"config": "differentiation", "workload": "GI scene (%d triangles), 128^3 FP32 learnable grid, "
            "1024x1024 G-buffer diffuse rays from p + h n, tmax 0.5, loss MSE vs triangle hits (%s)" % (
                scene.n_tris, args.loss),
            "rays": rays.n, "adam_steps": args.adam_steps, "lr": args.lr_scale * h, "loss": args.loss,
            "lipschitz_after": sdf.lipschitz,
            "loss_first": losses[0] if losses else None, "loss_last": losses[-1] if losses else None,
            "heldout_artefact_rate_before": before[0], "heldout_artefact_rate_after": after[0],
            "heldout_mean_dt_over_h_before": before[1], "heldout_mean_dt_over_h_after": after[1],
            "ms_per_adam_step": step_ms, "adam_steps_timed": timed,
            "ms_per_adam_step_new_grid_each_step": ms_new_grid, "forward_kernel_ms": ms_fwd,
            "backward_kernel_ms": ms_bwd, "sdf_from_grid_ms": ms_upload, "sdf_update_ms": ms_update,
            "forward_mrays_s": rays.n / ms_fwd / 1e3, "backward_mrays_s": rays.n / ms_bwd / 1e3}


def bench_batch(args, torch, hyb, W, dev, stream):
    """Many scenes of uneven size: one persistent graph launch against one
    launch per scene, both at the autotuned thresholds."""
    specs = W.batch_specs(4, args.scenes)
    items, meta = [], []
    t0 = time.time()
    for k, sp in enumerate(specs):
        scene = W.batch_scene(sp)
        bvh = hyb.build_bvh(scene.verts, scene.tris)
        sdf = hyb.build_sdf(bvh, sp.n_grid, W.room_grid(sp.n_grid))
        rays = W.gbuffer_rays(W.gbuffer(scene, sp.width, sp.height), sp.seed)
        items.append(dict(bvh=bvh, sdf=sdf, rays=torch.from_numpy(rays.soa()).to(dev), tmax=TMAX, threshold=1.0))
        meta.append(dict(tris=scene.n_tris, rays=rays.n, grid=sp.n_grid))
        log("scene %d/%d: %d triangles, %d rays, grid %d^3 (%.0fs)" % (k + 1, len(specs), scene.n_tris, rays.n,
                                                                       sp.n_grid, time.time() - t0))
    torch.cuda.synchronize()
    n_rays = sum(m["rays"] for m in meta)
    n_tris = sum(m["tris"] for m in meta)

    batch = hyb.Batch(items)
    default_cfg = batch.config
    ms_default = time_launches(lambda: batch.launch(), stream, args.reps, 2)
    log("batch, default config %s, threshold 1: %.3f ms (%.0f Mrays/s)" % (default_cfg, ms_default,
                                                                           n_rays / ms_default / 1e3))
    t0 = time.time()
    err, tuned_ms = batch.tune(max_error_rate=args.max_error, reps=3)
    tune_s = time.time() - t0
    cfg = batch.config
    taus = [batch.threshold(k) for k in range(len(items))]
    log("tuned in %.1fs: config %s, %.3f ms; thresholds %s" % (tune_s, cfg, tuned_ms, taus))

    def per_scene():
        for k, it in enumerate(items):
            hyb.trace(it["bvh"], it["sdf"], it["rays"], TMAX, taus[k], out=batch.outs[k])

    ms_loop = time_launches(per_scene, stream, args.reps, 2)
    # the same launches captured in one graph (no host gaps between them)
    ms_loop_graph = None
    try:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            per_scene()
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            per_scene()
        torch.cuda.synchronize()
        ms_loop_graph = time_launches(g.replay, stream, args.reps, 2)
    except Exception as e:  # reported, not fatal: the persistent batch is the measured path
        log("per-scene graph capture failed: %s" % e)
    ms_eager = time_launches(lambda: batch.launch(graph=False), stream, args.reps, 2)
    for _ in range(args.warmup):
        batch.launch()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.time()
    start.record(stream)
    for _ in range(args.steps):
        batch.launch()
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - wall0
    ms_graph = start.elapsed_time(stop) / args.steps
    log("graph %.3f ms, eager %.3f ms, %d per-scene launches %.3f ms (captured: %s ms)" % (
        ms_graph, ms_eager, len(items), ms_loop, ms_loop_graph))

    # algorithmic bytes and lane operations at the tuned thresholds (same
    # accounting as the GI line)
    total_bytes, total_ops = 0.0, 0.0
    for k, it in enumerate(items):
        _, cnt = hyb.trace_counters(it["bvh"], it["sdf"], it["rays"], TMAX, taus[k], hyb.MODE_COMBINED)
        c = cnt.double().sum(dim=0).cpu().numpy()
        total_bytes += BYTES_RAY * meta[k]["rays"] + BYTES_NODE * c[0] + BYTES_TRI * c[1] + BYTES_FETCH * c[2]
        total_ops += OPS_NODE * c[0] + OPS_TRI * c[1] + OPS_FETCH * c[2]
    achieved = total_bytes / (ms_graph * 1e-3) / 1e9
    alu = total_ops / (ms_graph * 1e-3) / 1e12
    hist = {}
    for t in taus:
        key = "inf" if math.isinf(t) else t
        hist[key] = hist.get(key, 0) + 1
    return {
        "config": "batch",
        "workload": "%d seeded scenes, %d triangles in all (%d to %d, log-uniform), grids 32^3 to 128^3, %d "
                    "G-buffer diffuse rays in all (%d to %d per scene, log-uniform), tmax 0.5" % (
                        len(items), n_tris, min(m["tris"] for m in meta), max(m["tris"] for m in meta), n_rays,
                        min(m["rays"] for m in meta), max(m["rays"] for m in meta)),
        "metric": "Mrays/s, whole batch in one graph launch", "value": n_rays / ms_graph / 1e3, "unit": "Mrays/s",
        "ms_graph": ms_graph, "ms_eager": ms_eager, "ms_per_scene_launches": ms_loop,
        "speedup_vs_per_scene_launches": ms_loop / ms_graph, "ms_per_scene_launches_in_one_graph": ms_loop_graph,
        "ms_default_config_tau1": ms_default, "default_config": default_cfg,
        "tuned_config": cfg, "tune_seconds": tune_s, "max_error_rate": args.max_error,
        "threshold_histogram": hist, "error_rate_max": float(np.max(err)), "error_rate_mean": float(np.mean(err)),
        "roofline": {"bound": "alu", "achieved": alu, "peak": VALU_PEAK_TOPS, "unit": "TOP/s (VALU lane operations)",
                     "frac": alu / VALU_PEAK_TOPS, "ops_per_ray": total_ops / n_rays,
                     "bytes_per_ray": total_bytes / n_rays,
                     "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": achieved / HBM_PEAK_GBS}},
        "steps": args.steps, "timed_wall_s": wall,
        "scenes": [{"triangles": m["tris"], "rays": m["rays"], "grid": m["grid"],
                    "threshold": None if math.isinf(taus[k]) else taus[k], "error_rate": float(err[k])}
                   for k, m in enumerate(meta)],
    }


def bench_shadow(args, torch, hyb, W, dev, stream):
    """The shadow-ray query on the GI-shaped scene: one ray per G-buffer pixel
    to a uniform sample of the area light, thresholds swept at both ends,
    against the exact any-hit triangle query (both thresholds +inf)."""
    t0 = time.time()
    scene = W.gi_scene(2)
    gb = W.gbuffer(scene, args.width, args.height)
    srays, stmax = W.shadow_rays(gb.p, gb.n, 22)
    n = srays.n
    bvh = hyb.build_bvh(scene.verts, scene.tris)
    g4 = W.room_grid(128)
    sdf = hyb.build_sdf(bvh, 128, g4)
    R, TS = torch.from_numpy(srays.soa()).to(dev), torch.from_numpy(stmax).to(dev)
    out = hyb.alloc_hits(n)
    log("shadow workload: %d triangles, %d rays (%.1fs)" % (scene.n_tris, n, time.time() - t0))
    big = 10.0  # every ray ends at its light sample (per-ray tmax)

    def run(ts, te):
        return lambda: hyb.trace_shadow(bvh, sdf, R, big, ts, te, tmax_ray=TS, out=out)

    ms_ref = time_launches(run(math.inf, math.inf), stream, args.reps, 2)
    ref = out[1].cpu().numpy() != -1
    res = []
    for ts, te in ((0.0, 0.0), (0.5, 0.5), (1.0, 1.0), (2.0, 2.0), (4.0, 4.0), (1.0, 4.0)):
        ms = time_launches(run(ts, te), stream, args.reps, 2)
        occ = out[1].cpu().numpy() != -1
        res.append(dict(threshold_start=ts, threshold_end=te, ms=ms, mrays_s=n / ms / 1e3,
                        occlusion_mismatch=float((occ != ref).mean()), false_occlusion=float((occ & ~ref).mean()),
                        missed_occlusion=float((~occ & ref).mean()), df_occluded=float((out[1] == -2).float().mean())))
        log("shadow (%s, %s): %.3f ms, mismatch %.4f" % (ts, te, ms, res[-1]["occlusion_mismatch"]))
    ms_closest = time_launches(lambda: hyb.trace_bvh(bvh, R, big, tmax_ray=TS, out=out), stream, args.reps, 2)
    return {"config": "shadow",
            "workload": "GI-shaped scene (%d triangles), 128^3 exact grid, %d shadow rays from the G-buffer points "
                        "to uniform samples of a 0.3 x 0.3 area light, any hit" % (scene.n_tris, n),
            "metric": "Mrays/s of the shadow query; occlusion mismatch against the exact any-hit triangle query",
            "triangles_anyhit": {"ms": ms_ref, "mrays_s": n / ms_ref / 1e3},
            "triangles_closest_hit": {"ms": ms_closest, "mrays_s": n / ms_closest / 1e3},
            "sweep": res, "occluded_fraction": float(ref.mean())}



def bench_ao(args, torch, hyb, W, dev, stream):
    """Occlusion (AO) rays of several lengths on the GI-shaped scene: first hit
    on [0, t_ao] from the G-buffer points, triangles only against the combined
    query at thresholds 0.5, 1, 2 voxels and the DF-only baseline (from p + h n),
    each with its artefact rate against the triangles-only hits."""
    scene = W.gi_scene(2)
    g4 = W.room_grid(128)
    h = float(g4[3])
    gb = W.gbuffer(scene, args.width, args.height)
    rays = W.gbuffer_rays(gb, 51)
    rb = W.rebias(rays, gb, h)
    bvh = hyb.build_bvh(scene.verts, scene.tris)
    sdf = hyb.build_sdf(bvh, 128, g4)
    R, RB = torch.from_numpy(rays.soa()).to(dev), torch.from_numpy(rb.soa()).to(dev)
    n = rays.n
    out = hyb.alloc_hits(n)
    o_np, d_np, ob_np = rays.o.astype(np.float64), rays.d.astype(np.float64), rb.o.astype(np.float64)
    res = []
    for t_ao in (0.05, 0.1, 0.25, 0.5, 1.0, 2.0):
        ms_bvh = time_launches(lambda: hyb.trace_bvh(bvh, R, t_ao, out=out), stream, args.reps, 2)
        ref_t, ref_p = out[0].cpu().numpy().astype(np.float64), out[1].cpu().numpy()
        row = dict(t_ao=t_ao, t_ao_voxels=t_ao / h, triangles_ms=ms_bvh, occluded=float((ref_p != -1).mean()))
        for tau in (0.5, 1.0, 2.0):
            ms = time_launches(lambda: hyb.trace(bvh, sdf, R, t_ao, tau, out=out), stream, args.reps, 2)
            a = artefacts(out[0].cpu().numpy().astype(np.float64), out[1].cpu().numpy(), o_np, d_np, ref_t, ref_p,
                          o_np, h)
            row["tau%g" % tau] = dict(ms=ms, speedup=ms_bvh / ms, artefacts=a["rate"])
        ms = time_launches(lambda: hyb.trace_df(sdf, RB, t_ao, out=out), stream, args.reps, 2)
        a = artefacts(out[0].cpu().numpy().astype(np.float64), out[1].cpu().numpy(), ob_np, d_np, ref_t, ref_p,
                      o_np, h)
        row["df_only"] = dict(ms=ms, speedup=ms_bvh / ms, artefacts=a["rate"])
        log("t_ao %.2f: triangles %.3f ms; tau 1 %.3f ms (x%.2f, artefacts %.4f); DF only %.3f ms (artefacts %.4f)" % (
            t_ao, ms_bvh, row["tau1"]["ms"], row["tau1"]["speedup"], row["tau1"]["artefacts"], ms, a["rate"]))
        res.append(row)
    return {"config": "ao", "workload": "GI-shaped scene (%d triangles), 128^3 exact grid, %d cosine AO rays from the "
            "G-buffer points, first hit on [0, t_ao]" % (scene.n_tris, n),
            "metric": "tracing time per AO distance: triangles only vs combined vs DF only", "sweep": res}


if __name__ == "__main__":
    main()
