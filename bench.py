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
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TAUS = (0.0, 0.5, 1.0, 2.0, 4.0, math.inf)
TMAX = 0.5
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def time_launches(fn, stream, reps, warmup):
    """Average duration of fn() (one kernel launch) over `reps` launches,
    bracketed by HIP events on the stream the kernel runs on."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / reps


def source_sha256():
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2305_07253_amd", "csrc", "*"))):
        if f.endswith((".hpp", ".hip", ".cpp")):
            h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(tau):
    """HBM bytes per launch of the combined kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source at
    this threshold; else None."""
    f = os.path.join(ROOT, "profiles", "traffic_gi1080p.json")
    if not os.path.exists(f):
        return None
    rec = json.load(open(f))
    if rec.get("source_sha256") != source_sha256() or rec.get("threshold") != tau:
        return None
    return rec["read_bytes"] + rec["write_bytes"]


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
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=10, help="launches per sweep point")
    ap.add_argument("--cpu-sample", type=int, default=4096, help="rays for the CPU oracle baseline (0: skip)")
    ap.add_argument("--tau", type=float, default=None,
                    help="fix the threshold (voxels) instead of selecting it at the fixed artefact rate")
    ap.add_argument("--profile", action="store_true",
                    help="profiling driver: a 256 MiB copy probe, then --steps launches of the combined, "
                         "triangle-only and DF-only kernels; no sweep, no JSON line")
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the ray query shards by rays with no exchange step; "
              "multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2305_07253_amd as hyb
    from paper_2305_07253_amd import workloads as W

    hyb.lib()
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
    (_, _, _, _), cnt = hyb.trace_counters(bvh, sdf128, R, TMAX, tau, hyb.MODE_COMBINED)
    c = cnt.double().mean(dim=0).cpu().numpy()
    bytes_per_ray = 24 + 16 + 64 * c[0] + 48 * c[1] + 32 * c[2]

    # timed region: K steps of the combined query at the chosen threshold
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
    achieved = bytes_per_ray * n / (ms_step * 1e-3) / 1e9

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
        cpu = dict(value=sub.n / el / 1e6, unit="Mrays/s", cores=oracle.threads(), kind="oracle",
                   sample="%d of the %d rays at a fixed stride over the tile-ordered G-buffer rays (%.1f s), "
                          "combined query at threshold %s, brute force over all %d triangles, FP64" % (
                              sub.n, n, el, chosen["tau"], scene.n_tris))
        log("cpu oracle: %.4f Mrays/s (%.1fs, %d threads)" % (cpu["value"], el, cpu["cores"]))

    line = {
        "metric": "Mrays/s for combined vs BVH-only vs DF-only at fixed t-error; HBM GB/s % of peak",
        "value": value,
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "GI-shaped: %d-triangle room, 128^3 FP32 exact SDF, %dx%d G-buffer cosine "
                               "diffuse rays (%d), tmax 0.5, threshold %s voxels" % (
                                   scene.n_tris, args.width, args.height, n, chosen["tau"]),
                   "rays": n, "triangles": scene.n_tris, "grid": 128, "tmax": TMAX, "threshold": chosen["tau"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(tau),
                     "bytes_per_ray": bytes_per_ray, "nodes_per_ray": c[0], "tris_per_ray": c[1],
                     "df_fetches_per_ray": c[2]},
        "cpu_baseline": cpu,
        "bvh_only": {"ms": ms_bvh, "mrays_s": n / ms_bvh / 1e3},
        "df_only": df_only,
        "sweep": sweep,
        "target_artefact_rate": target,
        "speedup_vs_bvh_only": ms_bvh / ms_step,
        "timed_wall_s": wall,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
