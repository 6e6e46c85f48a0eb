#!/usr/bin/env python3
"""Candidate poses scored per second (render + explanation cost) on one MI355X.

Workload (default): the 3-DoF search with the RGB term -- 5 objects of
2k-8k triangles, 640x480 RGB-D, a 20 x 20 grid at 3 cm x 16 yaws = 6,400
candidate poses per object, 32,000 renders per scene; delta = 10 mm,
tau_c = 20.  One step is the plain path for one scene: every candidate of
every object rendered and scored (J_r, J_o with occluder marking and the
CIEDE2000 gate) and the best pose of each object reduced on the device and
returned to the host.  The scene, meshes and poses are resident in HBM
before the timed region.

Prints one JSON line.  With --gpus above 1 it exits: the library scores
poses on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12      # one VALU op per lane per clock: 39.3 T lane-ops/s


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def tile_areas(w):
    """Per pose: (raster tile area, J_o region area) in pixels, by the same
    projected-AABB rule the set-up kernel applies (host re-statement for the
    work accounting only)."""
    W, H, fx, fy, cx, cy = w.scene.K
    out = []
    for o in w.objects:
        m = w.meshes[o.mesh]
        lo = m.xyz.min(0).astype(np.float64)
        hi = m.xyz.max(0).astype(np.float64)
        P = o.poses.reshape(-1, 3, 4).astype(np.float64)
        res = []
        for pad in (0.0, w.delta_mm + 0.5):
            C = np.array([[x, y, z] for z in (lo[2] - pad, hi[2] + pad) for y in (lo[1] - pad, hi[1] + pad)
                          for x in (lo[0] - pad, hi[0] + pad)])
            X = np.einsum("pij,cj->pci", P[:, :, :3], C) + P[:, None, :, 3]
            u = fx * X[..., 0] / X[..., 2] + cx
            v = fy * X[..., 1] / X[..., 2] + cy
            i0 = np.clip(np.floor(u.min(1)) - 1, 0, W - 1)
            i1 = np.clip(np.ceil(u.max(1)) + 1, 0, W - 1)
            j0 = np.clip(np.floor(v.min(1)) - 1, 0, H - 1)
            j1 = np.clip(np.ceil(v.max(1)) + 1, 0, H - 1)
            res.append((i1 - i0 + 1) * (j1 - j0 + 1))
        out.append(np.stack(res, 1))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2,
                    help="1-3: plain path on that scene; 4: batched vs plain on the uneven many-scene workload")
    ap.add_argument("--batched-scenes", type=int, default=64, help="scenes of the batched workload")
    ap.add_argument("--batched-steps", type=int, default=3, help="timed passes of the batched leg of a plain run")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched leg of a plain run")
    ap.add_argument("--batched-small", type=int, default=32,
                    help="the batched leg also scores the first N candidates of each object (0: not)")
    ap.add_argument("--batched-small-only", action="store_true",
                    help="config 4: only the small searches (the first --batched-small candidates of each object)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (default ~/.cache/perch)")
    ap.add_argument("--tuning", default=None,
                    help="launch tuning of the plain path as JSON, e.g. '{\"key_bands\": 1}' (results never change)")
    ap.add_argument("--rates", default="20,50,100", help="config 5: arrival rates, scenes/s")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="config 5: arrival window per rate")
    ap.add_argument("--served-rate", type=float, default=150.0,
                    help="arrival rate (scenes/s) of the served leg of a plain run, above the plain path's capacity")
    ap.add_argument("--served-seconds", type=float, default=8.0, help="arrival window of the served leg")
    ap.add_argument("--served-capacity-rate", type=float, default=200.0,
                    help="a second arrival rate of the served leg that saturates both forms (0: none), so that "
                         "their poses/s are capacities")
    ap.add_argument("--no-served", action="store_true", help="skip the served leg of a plain run")
    ap.add_argument("--served-small", type=int, default=64,
                    help="the served leg also serves requests of the first N candidates of each object (0: not)")
    ap.add_argument("--served-small-rate", type=float, default=800.0,
                    help="arrival rate of the small requests, scenes/s (above both forms' capacity)")
    ap.add_argument("--scene-cache-gb", type=float, default=0.0,
                    help="config 5: scene cache of both forms, GB (0: every arrival prepares its scene)")
    ap.add_argument("--served-small-cached-rate", type=float, default=3000.0,
                    help="arrival rate of the small requests with resident (cached) scenes, scenes/s (0: not)")
    ap.add_argument("--prep-workers", type=int, default=2, help="preparation threads of the server")
    ap.add_argument("--hold-ms", type=float, default=8.0,
                    help="while a batch runs, how long a lone ready request waits for another to join it")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--volume", choices=["aabb", "cyl", "label"], default=None,
                    help="V(O) of the plain run (default: the workload's)")
    ap.add_argument("--jo", choices=["exact", "nn"], default=None,
                    help="J_o of the plain run: the exact Eq. 3 test or nearest-neighbour marking")
    ap.add_argument("--search", choices=["table", "hash", "knn2"], default="table",
                    help="J_r neighbour search of the plain run: the scene table, the voxel hash, or the paper's "
                         "kNN II scan")
    ap.add_argument("--poses-per-object", type=int, default=0,
                    help="score only the first N candidates of each object (0 = all)")
    ap.add_argument("--no-refine", action="store_true", help="skip the ICP refine-and-rescore leg of a plain run")
    ap.add_argument("--pipeline6d", action="store_true",
                    help="add the 6-DoF leg: proposals, scoring, ICP of the best, rescoring (cfg3 scene)")
    ap.add_argument("--icp-method", choices=("plane", "point", "both"), default="plane",
                    help="refinement of the 6-DoF leg: plane-to-plane GICP (the paper's), point-to-point ICP, or both")
    ap.add_argument("--refine-steps", type=int, default=2, help="timed passes of the refine leg")
    ap.add_argument("--no-msg", action="store_true", help="skip the Monotone Scene Generation tree leg")
    ap.add_argument("--knn-sample", type=int, default=0,
                    help="add the search comparison leg: this many poses per object scored with the neighbour "
                         "table, the paper's kNN II scan and its kNN I distance array (0 = skip)")
    ap.add_argument("--msg-beam", type=int, default=4, help="states kept per level by the tree leg's search")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="poses per object the CPU oracle scores for the baseline (0 = every candidate)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--reduce-profile", default=None, metavar="DIR",
                    help="only reduce rocprofv3 CSV output under DIR (subfolders trace, FETCH_SIZE, WRITE_SIZE, sq, "
                         "copy_FETCH_SIZE, copy_WRITE_SIZE) to the per-launch counter record of the last --steps "
                         "dispatches of each scoring kernel, written to --profile-out")
    ap.add_argument("--profile-out", default=os.path.join(ROOT, "profiles", "score_kernel_cfg2_counters.json"))
    ap.add_argument("--trace-gaps", default=None, metavar="DIR",
                    help="only read a rocprofv3 kernel + marker trace of a --config 4 run under DIR and print, per "
                         "pass of the plain loop and per graph launch, the GPU's busy share and idle gaps")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.trace_gaps:
        trace_gaps(args.trace_gaps)
        return
    if args.reduce_profile:
        reduce_profile(args.reduce_profile, args.steps, args.profile_out, args.config, args.seed,
                       variant=counter_variant(args.volume, args.jo, args.search))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the library scores poses on one GPU only; run with --gpus 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    import paper_2008_00326_amd as pk
    from paper_2008_00326_amd.workloads import make_config

    if not os.path.exists(pk.library_path()):
        from paper_2008_00326_amd import build as _b
        _b.build()

    if args.config == 5:
        rates = [float(x) for x in args.rates.split(",")]
        r = served_vs_plain(rates, args.serve_seconds, args.seed, prep_workers=args.prep_workers,
                            hold_s=args.hold_ms / 1e3, poses_per_object=args.poses_per_object,
                            scene_cache_gb=args.scene_cache_gb)
        top = r["rates"][str(rates[0])]
        line = {"metric": "candidate poses scored/sec (render+cost), p50/p99 scene latency, vs plain",
                "value": top["served"]["poses_per_s"], "unit": "poses/s", "n_gpus": 1, "steps": len(rates),
                "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "f64/i64 geometry, i32 counts, f32 colour", "data": "synthetic",
                "config": {"workload": r["workload"], "config": 5, "seed": args.seed, "path": "served",
                           "rate_of_value": rates[0], "parallelism": "single GPU"},
                "served": r, "kernel_source_sha": kernel_source_sha()}
        print(json.dumps(line), flush=True)
        return

    if args.config == 4:
        ctx = pk.Context(0)
        r = batched_vs_plain(ctx, args.seed, args.steps, args.warmup, args.batched_scenes, args.tune_cache,
                             args.batched_small, full=not args.batched_small_only or args.batched_small <= 0)
        ctx.close()
        line = {"metric": "candidate poses scored/sec (render+cost), p50/p99 scene latency, vs plain",
                "value": r["batched_poses_per_s"], "unit": "poses/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": r["batched_ms_per_step"], "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "f64/i64 geometry, i32 counts, f32 colour",
                "data": "synthetic", "config": {"workload": r["workload"], "config": 4, "seed": args.seed,
                                                "path": "batched (one graph launch)", "parallelism": "single GPU"},
                "batched": r, "kernel_source_sha": kernel_source_sha()}
        print(json.dumps(line), flush=True)
        return

    _log(f"[bench] generating config {args.config} seed {args.seed}")
    w = make_config(args.config, args.seed)
    if args.volume:
        w.volume = args.volume
    if args.jo:
        w.jo = args.jo
    w.search = args.search
    if args.poses_per_object > 0:
        for o in w.objects:
            o.poses = np.ascontiguousarray(o.poses[:args.poses_per_object])
    dev = torch.device("cuda:0")
    ctx = pk.Context(0)
    if args.tuning:
        ctx.set_tuning(json.loads(args.tuning))
    stream = torch.cuda.current_stream(dev)

    t0 = time.perf_counter()
    sid, mids = pk.load_workload(ctx, w)
    torch.cuda.synchronize()
    scene_ms = (time.perf_counter() - t0) * 1e3
    poses = [torch.from_numpy(o.poses).to(dev) for o in w.objects]
    obj_mesh = [mids[o.mesh] for o in w.objects]
    obj_label = [o.label for o in w.objects]
    n_poses = sum(p.shape[0] for p in poses)

    # per-pose L, Q and footprint class for the work accounting (untimed)
    LQ = []
    for p, mid, lab in zip(poses, obj_mesh, obj_label):
        jr, jo, nr, nq = ctx.score_poses(sid, mid, p, label=lab, stream=stream)
        cls = ctx.last_classes(p.shape[0], stream=stream)
        LQ.append((nr.cpu().numpy().astype(np.float64), nq.cpu().numpy().astype(np.float64), cls))
    torch.cuda.synchronize()

    def step():
        return ctx.best_poses(sid, obj_mesh, obj_label, poses, stream=stream)

    _log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    _log(f"[bench] timing {args.steps} steps")
    ctx.profile(True)
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        best_idx, best_cost = step()
        lat.append((time.perf_counter() - a) * 1e3)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = ctx.profile_read()
    ctx.profile(False)
    ms_per_step = elapsed * 1e3 / args.steps
    value = n_poses * args.steps / elapsed

    # dominant kernel and its roofline
    score_slots = ["score_lds_small", "score_lds_large", "score_lds_tile", "score_device"]
    dom = max(score_slots, key=lambda k: prof[k][0])
    dom_ms, dom_launches = prof[dom]
    areas = tile_areas(w)
    W, H = w.scene.K[0], w.scene.K[1]
    info = ctx.scene_info(sid)
    caps = (info["tile_cap_small"], info["tile_cap_large"])
    cls_idx = score_slots.index(dom)
    ops = 0.0
    byts = 0.0
    c_q = 600.0 + (300.0 if w.use_rgb else 0.0)
    c_o = 300.0
    b_pix = 5.0 if w.use_rgb else 2.0
    class_poses = [0, 0, 0, 0]
    for o, (L, Q, cls), ar in zip(w.objects, LQ, areas):
        m = w.meshes[o.mesh]
        tile = ar[:, 0]
        for c in range(4):
            class_poses[c] += int((cls == c).sum())
        sel = cls == cls_idx
        ops += float(np.sum(60.0 * m.n_tris + 10.0 * tile[sel] + c_q * L[sel] + c_o * Q[sel]))
        if sel.any():
            byts += float(np.sum(48.0 + 8.0 + ar[sel, 1] * b_pix)) + m.n_verts * 20.0 + m.n_tris * 16.0
    # per launch = totals over the timed steps / launches
    ops_per_launch = ops * args.steps / max(dom_launches, 1)
    bytes_per_launch = byts * args.steps / max(dom_launches, 1)
    avg_s = dom_ms / max(dom_launches, 1) / 1e3
    achieved_tops = ops_per_launch / avg_s / 1e12 if avg_s > 0 else 0.0
    hbm_gbs = bytes_per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    # counters apply only to the workload they were taken on
    wvar = counter_variant(w.volume, w.jo, w.search)
    mc = measured_counters(dom, args.config, wvar)

    result = {
        "metric": "candidate poses scored/sec (render+cost), p50/p99 scene latency, vs plain",
        "value": round(value, 1),
        "unit": "poses/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64/i64 geometry, i32 counts, f32 colour",
        "data": "synthetic",
        "config": {"workload": w.name, "config": args.config, "seed": args.seed, "objects": len(w.objects),
                   "poses_per_step": n_poses, "image": [int(W), int(H)], "triangles": [m.n_tris for m in w.meshes],
                   "delta_mm": w.delta_mm, "tau_c": w.tau_c if w.use_rgb else None, "path": "plain",
                   "volume": w.volume, "jo": w.jo, "search": w.search,
                   "parallelism": "single GPU"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3),
                       "set_scene_and_meshes": round(scene_ms, 3)},
        "scene": {"device_MB": round(info["device_bytes"] / 2**20, 1), "table_entries": info["table_entries"],
                  "window": [info["window_x"], info["window_y"]], "tile_caps": list(caps)},
        "roofline": {"bound": "alu", "kernel": dom, "achieved": round(achieved_tops, 4), "peak": round(ALU_PEAK_TOPS, 2),
                     "unit": "TOP/s", "frac": round(achieved_tops / ALU_PEAK_TOPS, 5),
                     "traffic": measured_traffic(dom, args.config, wvar), "algorithmic_bytes_per_launch": round(bytes_per_launch, 1),
                     "avg_launch_ms": round(dom_ms / max(dom_launches, 1), 4), "launches": dom_launches,
                     "hbm_achieved_GBs": round(hbm_gbs, 2), "hbm_frac": round(hbm_gbs / HBM_PEAK_GBS, 6),
                     "valu_issue_frac": (round(mc["valu_frac_of_39.3T"], 4)
                                         if mc and mc.get("valu_frac_of_39.3T") is not None else None)},
        "kernels_ms": {k: round(v[0] / max(args.steps, 1), 4) for k, v in prof.items() if v[1]},
        "tuning": ctx.tuning(),
        "poses_per_class": class_poses,
        "kernel_source_sha": kernel_source_sha(),
    }

    # the served leg first: run after the many-scene leg, its scene preparations took three times as long
    # (12.5 against 3.9 ms at the median) and every launch then held a single request
    if not args.no_served:
        rates = [args.served_rate] + ([args.served_capacity_rate] if args.served_capacity_rate > 0 else [])
        r = served_vs_plain(rates, args.served_seconds, args.seed, drain_s=4.0,
                            prep_workers=args.prep_workers, hold_s=args.hold_ms / 1e3)
        top = r["rates"][str(args.served_rate)]
        result["served"] = {"workload": r["workload"], "rate_scenes_per_s": args.served_rate,
                            "seconds": args.served_seconds,
                            "served_poses_per_s": top["served"]["poses_per_s"],
                            "plain_poses_per_s": top["plain"]["poses_per_s"], "vs_plain": top["vs_plain"],
                            "latency_ms": {"served": top["served"]["latency_ms"], "plain": top["plain"]["latency_ms"]},
                            "offered_poses_per_s": top["offered_poses_per_s"],
                            "kernel_bound_poses_per_s": r.get("kernel_bound_poses_per_s"),
                            "detail": top}
        if args.served_capacity_rate > 0:
            cap = r["rates"][str(args.served_capacity_rate)]
            result["served"]["capacity"] = {
                "rate_scenes_per_s": args.served_capacity_rate, "offered_poses_per_s": cap["offered_poses_per_s"],
                "served_poses_per_s": cap["served"]["poses_per_s"], "plain_poses_per_s": cap["plain"]["poses_per_s"],
                "vs_plain": cap["vs_plain"], "mean_scenes_per_launch": cap["served"].get("mean_scenes_per_launch"),
                "mismatches_vs_alone": cap["served"]["mismatches_vs_alone"] + cap["plain"]["mismatches_vs_alone"]}
        if args.served_small > 0 and args.served_small_rate > 0:
            rs = served_vs_plain([args.served_small_rate], args.served_seconds, args.seed, drain_s=4.0,
                                 prep_workers=args.prep_workers, hold_s=args.hold_ms / 1e3,
                                 poses_per_object=args.served_small)
            sm = rs["rates"][str(args.served_small_rate)]
            result["served"]["small"] = {
                "workload": rs["workload"], "rate_scenes_per_s": args.served_small_rate,
                "offered_poses_per_s": sm["offered_poses_per_s"], "served_poses_per_s": sm["served"]["poses_per_s"],
                "plain_poses_per_s": sm["plain"]["poses_per_s"], "vs_plain": sm["vs_plain"],
                "served_scenes_per_s": round(sm["served"]["answered"] / max(sm["served"].get("span_s", 0), 1e-9), 1),
                "plain_scenes_per_s": round(sm["plain"]["answered"] / max(sm["plain"].get("span_s", 0), 1e-9), 1),
                "mean_scenes_per_launch": sm["served"].get("mean_scenes_per_launch"),
                "preparation_p50_ms": sm["served"].get("preparation_p50_ms"),
                "kernel_bound_poses_per_s": rs.get("kernel_bound_poses_per_s"),
                "mismatches_vs_alone": sm["served"]["mismatches_vs_alone"] + sm["plain"]["mismatches_vs_alone"]}
            if args.served_small_cached_rate > 0:
                rc = served_vs_plain([args.served_small_cached_rate], args.served_seconds, args.seed, drain_s=4.0,
                                     prep_workers=args.prep_workers, hold_s=args.hold_ms / 1e3,
                                     poses_per_object=args.served_small, scene_cache_gb=4.0)
                sc = rc["rates"][str(args.served_small_cached_rate)]
                result["served"]["small"]["scene_cache"] = {
                    "workload": rc["workload"], "rate_scenes_per_s": args.served_small_cached_rate,
                    "served_poses_per_s": sc["served"]["poses_per_s"], "plain_poses_per_s": sc["plain"]["poses_per_s"],
                    "vs_plain": sc["vs_plain"],
                    "served_scenes_per_s": round(sc["served"]["answered"] / max(sc["served"]["span_s"], 1e-9), 1),
                    "plain_scenes_per_s": round(sc["plain"]["answered"] / max(sc["plain"]["span_s"], 1e-9), 1),
                    "mean_scenes_per_launch": sc["served"].get("mean_scenes_per_launch"),
                    "scene_cache_misses": [sc["served"].get("scene_cache_misses"), sc["plain"].get("scene_cache_misses")],
                    "mismatches_vs_alone": sc["served"]["mismatches_vs_alone"] + sc["plain"]["mismatches_vs_alone"]}
    if not args.no_refine:
        result["refine"] = refine_leg(ctx, w, mids, args.refine_steps, 0 if args.no_cpu_baseline else 16)
    if args.knn_sample > 0:
        result["knn"] = knn_leg(ctx, w, mids, args.knn_sample)
    if not args.no_msg:
        result["msg"] = msg_leg(ctx, w, mids, args.msg_beam, 0 if args.no_cpu_baseline else 4)
    if args.pipeline6d:
        methods = ("plane", "point") if args.icp_method == "both" else (args.icp_method,)
        legs = {m: pipeline6d_leg(ctx, args.seed, method=m) for m in methods}
        result["pipeline6d"] = legs[methods[0]] if len(methods) == 1 else legs
    if not args.no_batched:
        ctx.drop_scene(sid)
        ctx.set_tuning(None)
        result["batched"] = batched_vs_plain(ctx, args.seed, args.batched_steps, 1, args.batched_scenes,
                                             args.tune_cache, args.batched_small)
    ctx.close()
    # the CPU oracle last: its worker threads share the host with the server's threads
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    print(json.dumps(result), flush=True)


def refine_leg(ctx, w, mids, steps, cpu_sample):
    """ICP refinement (point-to-point, 3-DoF, rho 20 mm, at most 10 updates,
    source stride 2) of every candidate against its object's labelled pixels,
    then every refined pose rendered and scored again, as the segmented
    pipeline of the paper does before selecting poses.  Returns poses/s of
    the refinement and of refinement plus rescoring, the costs before and
    after, and the CPU oracle's refinement rate on a small sample.  The same
    candidates are also refined by plane-to-plane GICP (6-DoF) and timed."""
    import torch
    s = w.scene
    _log("[bench] refine: ICP + rescore")
    sid = ctx.set_scene(s.K, s.depth, s.rgb if w.use_rgb else None, s.labels, delta_mm=w.delta_mm, tau_c=w.tau_c,
                        use_rgb=w.use_rgb, mark_occluders=w.mark_occluders, volume="label")
    prm = dict(rho_mm=20.0, iterations=10, stride=2, dof=3)
    meshes = [mids[o.mesh] for o in w.objects]
    labels = [o.label for o in w.objects]
    polys = [torch.from_numpy(o.poses).cuda() for o in w.objects]
    outs = [torch.empty_like(p) for p in polys]
    n = sum(p.shape[0] for p in polys)
    stats = []

    def refine():
        stats.clear()
        for mid, lab, p, out in zip(meshes, labels, polys, outs):
            stats.append(ctx.refine_poses(sid, mid, p, label=lab, out=out, **prm)[1:])

    refine()
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        refine()
    torch.cuda.synchronize()
    t_ref = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        bi_after, bc_after = ctx.best_poses(sid, meshes, labels, outs)
    t_score = (time.perf_counter() - t0) / steps
    prof = ctx.profile_read()
    ctx.profile(False)
    bi_before, bc_before = ctx.best_poses(sid, meshes, labels, polys)
    j0, j1 = [], []
    for mid, lab, p, out in zip(meshes, labels, polys, outs):
        a = ctx.score_poses(sid, mid, p, label=lab)
        b = ctx.score_poses(sid, mid, out, label=lab)
        j0.append((a[0] + a[1]).cpu().numpy())
        j1.append((b[0] + b[1]).cpu().numpy())
    j0, j1 = np.concatenate(j0), np.concatenate(j1)
    it = np.concatenate([x[0].cpu().numpy() for x in stats])
    mt = np.concatenate([x[1].cpu().numpy() for x in stats])
    out = {"workload": f"{w.name}, label volumes, every candidate refined", "icp": dict(prm, min_points=16),
           "poses": n, "refine_poses_per_s": round(n / t_ref, 1), "refine_ms": round(t_ref * 1e3, 3),
           "rescore_ms": round(t_score * 1e3, 3), "refine_and_rescore_poses_per_s": round(n / (t_ref + t_score), 1),
           "icp_kernel_ms": round(prof["icp"][0] / max(prof["icp"][1], 1) * len(polys), 3),
           "mean_updates": round(float(it.mean()), 2), "mean_matches_last": round(float(mt.mean()), 1),
           "mean_J_before": round(float(j0.mean()), 1), "mean_J_after": round(float(j1.mean()), 1),
           "fraction_J_lower": round(float(np.mean(j1 < j0)), 4),
           "best_J_before": [int(x) for x in bc_before], "best_J_after": [int(x) for x in bc_after]}
    # the same candidates through plane-to-plane GICP (6-DoF, the paper's refinement of its 6-DoF pipeline)
    gprm = dict(prm, dof=6, method="plane")
    gstats = [ctx.refine_poses(sid, mid, p, label=lab, out=o, **gprm)[1:]
              for mid, lab, p, o in zip(meshes, labels, polys, outs)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        gstats = [ctx.refine_poses(sid, mid, p, label=lab, out=o, **gprm)[1:]
                  for mid, lab, p, o in zip(meshes, labels, polys, outs)]
    torch.cuda.synchronize()
    t_g = (time.perf_counter() - t0) / steps
    jg = np.concatenate([sum(ctx.score_poses(sid, mid, o, label=lab)[:2]).cpu().numpy()
                         for mid, lab, o in zip(meshes, labels, outs)])
    out["gicp"] = {"icp": dict(gprm, min_points=16), "refine_poses_per_s": round(n / t_g, 1),
                   "refine_ms": round(t_g * 1e3, 3),
                   "mean_updates": round(float(np.concatenate([x[0].cpu().numpy() for x in gstats]).mean()), 2),
                   "mean_J_after": round(float(jg.mean()), 1), "fraction_J_lower": round(float(np.mean(jg < j0)), 4)}
    if cpu_sample:
        import oracle
        rng = np.random.default_rng(7)
        per = max(1, cpu_sample // len(w.objects))
        threads = oracle.threads()           # every thread the oracle's OpenMP runtime uses
        flags = (oracle.MARK_OCCLUDERS if w.mark_occluders else 0) | oracle.VOL_LABEL
        k = 0
        t0 = time.perf_counter()
        for o in w.objects:
            sel = np.sort(rng.choice(o.poses.shape[0], per, replace=False))
            oracle.icp(w.meshes[o.mesh], s, o.poses[sel], delta_mm=w.delta_mm, flags=flags,
                       label=o.label, threads=threads, **prm)
            k += len(sel)
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"poses_per_s": round(k / dt, 3), "cores": threads,
                             "sample": f"{k} poses ({per} per object, seeded uniform), brute-force matches, {dt:.1f} s"}
    ctx.drop_scene(sid)
    return out


def knn_leg(ctx, w, mids, per_object):
    """The paper's two neighbour searches against the scene's table on a
    sample of the same workload (the first `per_object` candidates of each
    object): kNN II, each rendered point scanning the whole observed cloud,
    and kNN I, every rendered-observed distance of a pose in one array (one
    pose at a time).  Same outputs by construction, checked here; reports
    poses/s of each and kNN I's array size per pose."""
    import torch
    s = w.scene
    _log(f"[bench] search comparison: {per_object} poses per object")
    polys = [torch.from_numpy(np.ascontiguousarray(o.poses[:per_object])).cuda() for o in w.objects]
    n = sum(p.shape[0] for p in polys)
    out = {"workload": f"{w.name}, first {per_object} candidates per object", "poses": n}
    ref = None
    for search in ("table", "knn2", "knn1"):
        sid = ctx.set_scene(s.K, s.depth, s.rgb if w.use_rgb else None, s.labels, delta_mm=w.delta_mm,
                            tau_c=w.tau_c, use_rgb=w.use_rgb, mark_occluders=w.mark_occluders, volume=w.volume,
                            jo=w.jo, search=search)
        for o, p in zip(w.objects, polys):                          # warm-up
            ctx.score_poses(sid, mids[o.mesh], p[:1], label=o.label)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        res = [ctx.score_poses(sid, mids[o.mesh], p, label=o.label) for o, p in zip(w.objects, polys)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = ctx.profile_read()
        ctx.profile(False)
        got = [np.concatenate([r[k].cpu().numpy() for r in res]) for k in range(4)]
        if ref is None:
            ref = got
        leg = {"poses_per_s": round(n / dt, 2), "ms": round(dt * 1e3, 3),
               "identical_to_table": all(np.array_equal(a, b) for a, b in zip(got, ref))}
        if search == "knn1":
            n_obs = int((s.depth > 0).sum())
            arr = got[2].astype(np.float64) * n_obs * 4
            leg.update({"observed_points": n_obs, "mean_L": round(float(got[2].mean()), 1),
                        "array_bytes_mean": round(float(arr.mean())), "array_bytes_max": round(float(arr.max())),
                        "kernel_ms": round(prof["knn1"][0] + prof["render"][0], 3)})
        out[search] = leg
        ctx.drop_scene(sid)
    return out


def msg_leg(ctx, w, mids, beam, cpu_sample):
    """The Monotone Scene Generation tree (the sequential variant 2.0-B) on
    the same scene and candidates: a beam search of width `beam` over all
    objects, every successor of every kept state scored on the GPU.  Reports
    successors scored per second, the tree kernel's time, the goal's cost and
    placement order, and each object's pose against the one the flat search
    (every object scored alone, 2.0-C) picks; the CPU oracle's edge rate on a
    small sample."""
    import torch
    s = w.scene
    _log(f"[bench] tree: beam {beam}")
    sid = ctx.set_scene(s.K, s.depth, s.rgb if w.use_rgb else None, s.labels, delta_mm=w.delta_mm, tau_c=w.tau_c,
                        use_rgb=w.use_rgb, mark_occluders=w.mark_occluders, volume="label")
    objs = [(mids[o.mesh], o.label, torch.from_numpy(o.poses).cuda()) for o in w.objects]
    ctx.msg_search(sid, objs, beam=beam)                       # warm-up
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    goal, scored = ctx.msg_search(sid, objs, beam=beam)
    dt = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    flat_idx, flat_cost = ctx.best_poses(sid, [m for m, _, _ in objs], [lab for _, lab, _ in objs],
                                         [p for _, _, p in objs])
    out = {"workload": f"{w.name}, label volumes, beam search over the tree", "beam": beam,
           "successors_scored": int(scored), "search_ms": round(dt * 1e3, 3),
           "successors_per_s": round(scored / dt, 1),
           "msg_kernel_ms": round(prof["msg"][0], 3), "msg_launches": prof["msg"][1]}
    if goal is not None:
        cost, seq = goal
        pick = dict(seq)
        out.update({"goal_cost": int(cost), "order": [int(o) for o, _ in seq],
                    "same_pose_as_flat": [bool(pick[o] == int(flat_idx[o])) for o in range(len(w.objects))],
                    "flat_sum_cost": int(sum(int(c) for c in flat_cost))})
    if cpu_sample:
        import oracle
        threads = oracle.threads()           # every thread the oracle's OpenMP runtime uses
        o = w.objects[-1]
        flags = (oracle.USE_RGB if w.use_rgb else 0) | (oracle.MARK_OCCLUDERS if w.mark_occluders else 0) | \
            oracle.VOL_LABEL
        state = [(w.meshes[q.mesh], q.label, q.gt_pose) for q in w.objects[:2]]
        rng = np.random.default_rng(8)
        sel = np.sort(rng.choice(o.poses.shape[0], cpu_sample, replace=False))
        t0 = time.perf_counter()
        oracle.msg_expand(s, state, w.meshes[o.mesh], o.poses[sel], label=o.label, delta_mm=w.delta_mm,
                          tau_c=w.tau_c, flags=flags, threads=threads)
        dt = time.perf_counter() - t0
        out["cpu_oracle"] = {"successors_per_s": round(len(sel) / dt, 3), "cores": threads,
                             "sample": f"{len(sel)} successors of a two-object state (seeded uniform), "
                                       f"brute force, {dt:.1f} s"}
    ctx.drop_scene(sid)
    return out


def _pose_errors(a, b):
    A = np.asarray(a, np.float64).reshape(3, 4)
    B = np.asarray(b, np.float64).reshape(3, 4)
    dR = A[:, :3] @ B[:, :3].T
    ang = float(np.degrees(np.arccos(np.clip((np.trace(dR) - 1) / 2, -1, 1))))
    return float(np.linalg.norm(A[:, 3] - B[:, 3])), ang


def pipeline6d_leg(ctx, seed, viewpoints=256, inplane=12, z_step=10.0, max_depths=12, top=128, method="plane"):
    """The 6-DoF pipeline of the paper (Sec. V-C) on the cfg3 scene with its
    labels standing in for the segmentation: per object, rotation x
    translation proposals (Sec. V-B), every proposal rendered and scored with
    label volumes, the `top` cheapest refined against the object's labelled
    pixels (plane-to-plane GICP, or 6-DoF point-to-point ICP with method
    "point"), rendered and scored again, and the cheapest
    kept.  Reports the time of each stage, poses/s over the whole pipeline
    and the final pose's distance to the generating pose (rotation error is
    only meaningful for shapes without symmetry), with the cost of the final
    pose beside that of the generating pose."""
    import torch
    from paper_2008_00326_amd.workloads import make_config
    w = make_config(3, seed)
    s = w.scene
    _log(f"[bench] 6-DoF pipeline: proposals, scoring, {'GICP' if method == 'plane' else 'ICP'}, rescoring")
    sid = ctx.set_scene(s.K, s.depth, s.rgb, s.labels, delta_mm=w.delta_mm, tau_c=w.tau_c, use_rgb=True,
                        volume="label")
    mids = [ctx.load_mesh(m.xyz, m.tri, m.rgb) for m in w.meshes]
    icp = dict(rho_mm=20.0, iterations=15, stride=2, dof=6, method=method)
    streams = [torch.cuda.Stream() for _ in range(4)]

    def run():
        t = {}
        torch.cuda.synchronize()
        a = time.perf_counter()
        props = [ctx.propose_poses(sid, mids[o.mesh], o.label, viewpoints=viewpoints, inplane=inplane,
                                   z_step_mm=z_step, max_depths=max_depths) for o in w.objects]
        torch.cuda.synchronize()
        t["propose"] = time.perf_counter() - a
        a = time.perf_counter()
        # every object's proposals in one launch sequence (per-pose costs back)
        items = ctx.score_batch([{"scene": sid, "mesh": mids[o.mesh], "label": o.label, "poses": p}
                                 for o, p in zip(w.objects, props)])
        costs = [it["jr"] + it["jo"] for it in items]
        torch.cuda.synchronize()
        t["score"] = time.perf_counter() - a
        a = time.perf_counter()
        best = [torch.topk(c, min(top, c.numel()), largest=False).indices for c in costs]
        cand = [p[b].contiguous() for p, b in zip(props, best)]
        # one launch per object holds only `top` poses (a work-group each), so
        # the objects' refinements go to separate streams and run side by side
        refined = []
        for k, (o, c) in enumerate(zip(w.objects, cand)):
            sk = streams[k % len(streams)]
            sk.wait_stream(torch.cuda.current_stream())
            refined.append(ctx.refine_poses(sid, mids[o.mesh], c, label=o.label, stream=sk, **icp)[0])
        torch.cuda.synchronize()
        t["refine"] = time.perf_counter() - a
        a = time.perf_counter()
        final = []
        for o, c, r in zip(w.objects, cand, refined):
            both = torch.cat([c, r])
            jr, jo, _, _ = ctx.score_poses(sid, mids[o.mesh], both, label=o.label, counts=False)
            k = int(torch.argmin(jr + jo))
            final.append((both[k].cpu().numpy(), int((jr + jo)[k]), k >= c.shape[0]))
        t["rescore"] = time.perf_counter() - a
        return t, sum(p.shape[0] for p in props), final

    run()                                             # warm-up
    t, n_props, final = run()
    errs = [_pose_errors(f[0], o.gt_pose) for f, o in zip(final, w.objects)]
    j_gt = []
    for o in w.objects:
        g = torch.from_numpy(np.ascontiguousarray(o.gt_pose[None])).cuda()
        jr, jo, _, _ = ctx.score_poses(sid, mids[o.mesh], g, label=o.label, counts=False)
        j_gt.append(int((jr + jo)[0]))
    total = sum(t.values())
    out = {"workload": f"cfg3 6-DoF scene (640x480, {len(w.objects)} objects, 20k-triangle meshes), labels as masks",
           "proposals": {"viewpoints": viewpoints, "inplane": inplane, "z_step_mm": z_step, "max_depths": max_depths,
                         "total": n_props}, "icp": dict(icp, top=top),
           "ms": {k: round(v * 1e3, 3) for k, v in t.items()}, "total_ms": round(total * 1e3, 3),
           "poses_per_s": round((n_props + 2 * top * len(w.objects)) / total, 1),
           "final_from_icp": int(sum(f[2] for f in final)),
           "translation_error_mm": [round(e[0], 1) for e in errs],
           "rotation_error_deg": [round(e[1], 1) for e in errs],
           "median_translation_error_mm": round(float(np.median([e[0] for e in errs])), 1),
           "J_final": [f[1] for f in final], "J_true_pose": j_gt}
    ctx.drop_scene(sid)
    for m in mids:
        ctx.unload_mesh(m)
    return out


def batched_vs_plain(ctx, seed, steps, warmup, n_scenes=64, tune_cache=None, small=0, full=True):
    """The uneven many-scene workload (640x480 RGB-D scenes with 1-10 objects,
    200-8000 candidates per object, meshes of 500-50k triangles, 3-DoF and
    6-DoF mixed) scored two ways on identical inputs: the plain path, one
    best_poses launch sequence per scene, and the batched path, every scene
    in one graph-captured persistent launch with autotuned work spreading.
    Returns poses/s of both, their ratio, the per-object agreement and the
    tuning used.  With small > 0 the same resident scenes are scored again
    with only the first `small` candidates of each object (a small search
    per scene, as when refining around a few proposals), returned under
    "small": there one scene's launch leaves most compute units idle.
    full=False measures the small searches alone and returns their result."""
    import torch
    from paper_2008_00326_amd.workloads import scenes

    _log(f"[bench] batched: generating {n_scenes} scenes")
    lib = scenes.mesh_library(seed)
    ws = scenes.config4(seed, n_scenes=n_scenes, library=lib)
    mids = [ctx.load_mesh(m.xyz, m.tri, m.rgb) for m in lib]
    scene_ids, polys = [], []
    for w in ws:
        scene_ids.append(ctx.set_scene(w.scene.K, w.scene.depth, w.scene.rgb, delta_mm=w.delta_mm, tau_c=w.tau_c))
        polys.append([torch.from_numpy(o.poses).cuda() for o in w.objects])
    tris = np.mean([lib[o.mesh].n_tris for w in ws for o in w.objects])

    def workload(cut):
        per_scene, items = [], []
        for w, sid, ps in zip(ws, scene_ids, polys):
            ps = [p[:cut] if cut else p for p in ps]
            per_scene.append((sid, [mids[o.mesh] for o in w.objects], [o.label for o in w.objects], ps))
            items += [{"scene": sid, "mesh": mids[o.mesh], "label": o.label, "poses": p}
                      for o, p in zip(w.objects, ps)]
        return per_scene, items

    r = {}
    if full:
        per_scene, items = workload(0)
        r = _plain_and_batched(ctx, per_scene, items, tris, steps, warmup, tune_cache)
        r = dict({"workload": f"cfg4-batched-uneven ({n_scenes} scenes, {len(items)} objects, seed {seed})"}, **r)
    if small > 0:
        per_scene, items = workload(small)
        _log(f"[bench] batched: the same scenes, first {small} candidates of each object")
        r["small"] = dict({"workload": f"cfg4-batched-uneven, first {small} candidates of each object "
                                       f"({n_scenes} scenes, {len(items)} objects, seed {seed})"},
                          **_plain_and_batched(ctx, per_scene, items, tris, max(steps, 10), warmup, tune_cache))
    for sid in scene_ids:
        ctx.drop_scene(sid)
    for m in mids:
        ctx.unload_mesh(m)
    return r if full else r["small"]


def _plain_and_batched(ctx, per_scene, items, tris, steps, warmup, tune_cache):
    """Time resident scenes' items the plain way (one blocking best_poses per
    scene) and as one graph-captured batch, after autotuning the batch on
    every fourth scene's items; the plain loop's GPU busy fraction bounds
    what removing host gaps could gain."""
    import torch
    from paper_2008_00326_amd import autotune

    n_poses = sum(it["poses"].shape[0] for it in items)
    stream = torch.cuda.current_stream()
    sample = [it for it in items if any(it["scene"] == per_scene[k][0] for k in range(0, len(per_scene), 4))]
    bucket = autotune.shape_bucket(640 * 480, tris, n_poses / len(items), True)
    _log(f"[bench] batched: autotuning on {sum(i['poses'].shape[0] for i in sample)} poses ({bucket})")
    tuned = autotune.autotune(ctx, sample, bucket, cache_path=tune_cache or autotune.DEFAULT_CACHE, stream=stream)

    def plain():
        out = []
        for sid, ms, ls, ps in per_scene:
            bi, bc = ctx.best_poses(sid, ms, ls, ps, stream=stream)
            out += list(zip(bi.tolist(), bc.tolist()))
        return out

    _log(f"[bench] batched: plain path, {len(per_scene)} scenes, {n_poses} poses")
    for _ in range(warmup):
        ref = plain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ref = plain()
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / steps
    # the plain loop's GPU busy time (every kernel bracketed by HIP events on
    # the launch stream; nothing overlaps in this loop): wall / busy bounds
    # what any batching or overlap of the same kernels can gain
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain()
    torch.cuda.synchronize()
    traced_s = time.perf_counter() - t0
    busy_ms = sum(v[0] for v in ctx.profile_read().values())
    ctx.profile(False)

    b = ctx.batch(max_items=len(items), max_poses=n_poses, max_image_pixels=640 * 480)
    b.set(items)
    for _ in range(warmup):
        b.launch(stream)
        b.wait()
    _log("[bench] batched: graph launches")
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.launch(stream)
        bi, bc = b.wait()
    torch.cuda.synchronize()
    batched_s = (time.perf_counter() - t0) / steps
    prof = ctx.profile_read()
    ctx.profile(False)
    got = list(zip(bi.tolist(), bc.tolist()))
    # the same items in one direct (not captured) launch, every kernel timed
    ctx.profile(True)
    ctx.score_batch(items, stream=stream)
    torch.cuda.synchronize()
    direct = ctx.profile_read()
    ctx.profile(False)
    b.close()
    return {"poses_per_step": n_poses, "scenes": len(per_scene), "objects": len(items),
            "plain_poses_per_s": round(n_poses / plain_s, 1), "plain_ms_per_step": round(plain_s * 1e3, 3),
            "batched_poses_per_s": round(n_poses / batched_s, 1), "batched_ms_per_step": round(batched_s * 1e3, 3),
            "vs_plain": round(plain_s / batched_s, 3), "identical_best_poses": got == ref,
            "plain_gpu_busy_frac": round(busy_ms / 1e3 / traced_s, 4), "plain_gpu_busy_ms": round(busy_ms, 3),
            "vs_plain_bound": round(traced_s / max(busy_ms / 1e3, 1e-9), 3),
            "tuning": tuned["tuning"], "tuning_key": tuned["key"], "tuning_cached": tuned["cached"],
            "tuning_default_ms": tuned.get("default_ms"), "tuning_best_ms": tuned.get("ms"),
            "tuning_fastest_ms": tuned.get("fastest_ms"),
            "kernels_ms": {k: round(v[0] / max(steps, 1), 4) for k, v in prof.items() if v[1]},
            "direct_launch_kernels_ms": {k: round(v[0], 4) for k, v in direct.items() if v[1]}}


_POOLS = {}


def _served_pool(seed, pool_size):
    """The served workload's seeded scene pool, generated once per process."""
    from paper_2008_00326_amd.workloads import make_config
    if (seed, pool_size) not in _POOLS:
        _log(f"[bench] served: generating a pool of {pool_size} scenes")
        _POOLS[(seed, pool_size)] = [make_config(3, seed + k) for k in range(pool_size)]
    return _POOLS[(seed, pool_size)]


def served_vs_plain(rates, seconds, seed, pool_size=8, drain_s=10.0, budget_gb=32.0, prep_workers=2, hold_s=0.0,
                    poses_per_object=0, scene_cache_gb=0.0):
    """Poisson arrivals of 6-DoF scenes (8 objects of ~20k triangles, 8,192
    candidates, 640x480 RGB-D; a seeded pool of generated scenes, each arrival
    a new upload of one of them) served two ways on identical schedules: the
    continuous-batching server and the plain loop (one scene at a time,
    prepared and scored alone).  Arrivals run for `seconds`; what is not
    answered `drain_s` later counts as unfinished, with its waiting time as a
    lower bound of its latency.  poses_per_object > 0 keeps only the first
    candidates of each object (small searches).  scene_cache_gb > 0 gives
    both forms a scene cache of that size, so a scene of the pool is prepared
    once and later arrivals of it skip preparation."""
    import dataclasses
    import threading
    import torch
    import paper_2008_00326_amd as pk
    from paper_2008_00326_amd import serve

    pool = _served_pool(seed, pool_size)
    if poses_per_object > 0:
        pool = [dataclasses.replace(w, objects=[dataclasses.replace(o, poses=np.ascontiguousarray(
            o.poses[:poses_per_object])) for o in w.objects]) for w in pool]
    ctx = pk.Context(0)
    # reference answers, each scene scored alone; the GPU busy time of
    # preparing and scoring a scene (every kernel timed by HIP events) bounds
    # the throughput any serving schedule can reach
    ref = []
    busy_ms = 0.0
    for w in pool:
        ctx.profile(True)
        sid, mids = pk.load_workload(ctx, w)
        polys = [torch.from_numpy(o.poses).cuda() for o in w.objects]
        bi, bc = ctx.best_poses(sid, [mids[o.mesh] for o in w.objects], [o.label for o in w.objects], polys)
        busy_ms += sum(v[0] for v in ctx.profile_read().values())
        ctx.profile(False)
        ref.append([(int(a), int(b)) for a, b in zip(bi, bc)])
        ctx.drop_scene(sid)
        for m in mids:
            ctx.unload_mesh(m)
    cut = f", first {poses_per_object} candidates of each object" if poses_per_object > 0 else ""
    cut += ", scenes cached" if scene_cache_gb > 0 else ""
    out = {"workload": f"cfg5-served (Poisson arrivals of 6-DoF 640x480 scenes{cut}, pool of {pool_size}, "
                       f"seed {seed})",
           "seconds": seconds, "drain_s": drain_s, "rates": {},
           "gpu_busy_ms_per_scene": round(busy_ms / pool_size, 3),
           "kernel_bound_poses_per_s": round(float(np.mean([w.n_poses for w in pool])) / (busy_ms / pool_size) * 1e3,
                                             1)}
    rng = np.random.default_rng(5000 + seed)
    for rate in rates:
        n = int(rng.poisson(rate * seconds))
        offsets = np.sort(rng.uniform(0.0, seconds, n))
        picks = rng.integers(0, pool_size, n)
        res = {}
        for mode in ("served", "plain"):
            _log(f"[bench] served: {rate}/s, {n} arrivals, {mode}")
            reqs = [serve.Request(k, pool[int(picks[k])], pool[int(picks[k])].n_poses) for k in range(n)]
            t0 = time.perf_counter() + 0.2
            for r, off in zip(reqs, offsets):
                r.arrival = t0 + float(off)
            horizon = t0 + seconds + drain_s
            if mode == "served":
                ex = serve.GpuExecutor(ctx, slots=2, max_items=256, max_poses=65536,
                                       scene_cache_bytes=int(scene_cache_gb * 2**30))
                srv = serve.Server(ex, budget_bytes=int(budget_gb * 2**30), max_items=256, max_poses=65536,
                                   prep_workers=prep_workers, hold_s=hold_s)

                def producer():
                    for r in reqs:
                        d = r.arrival - time.perf_counter()
                        if d > 0:
                            time.sleep(d)
                        srv.submit(r)
                    d = horizon - time.perf_counter()
                    if d > 0:
                        time.sleep(d)
                    srv.cancel_pending()
                    srv.close()

                th = threading.Thread(target=producer, daemon=True)
                th.start()
                done = srv.run()
                th.join()
                def stage(a, b):
                    v = [(getattr(r, b) - getattr(r, a)) * 1e3 for r in reqs
                         if getattr(r, a) is not None and getattr(r, b) is not None]
                    return ({"p50": round(float(np.percentile(v, 50)), 3), "p99": round(float(np.percentile(v, 99)), 3)}
                            if v else None)

                def p50(attr):
                    v = [getattr(r, attr) * 1e3 for r in reqs if getattr(r, attr) is not None]
                    return round(float(np.percentile(v, 50)), 3) if v else None

                extra = {"prep_workers": prep_workers,
                         "preparation_p50_ms": {"set_scene": p50("scene_s"), "pose_upload": p50("upload_s")},
                         "stage_ms": {"admission": stage("arrival", "admitted"), "preparation": stage("admitted", "ready"),
                                      "ready_to_launch": stage("ready", "launched"),
                                      "launch_to_answer": stage("launched", "done")},
                         "launches": len(srv.batches),
                         "mean_scenes_per_launch": round(float(np.mean([b[1] for b in srv.batches])), 2)
                         if srv.batches else 0.0, "peak_admitted_MB": round(srv.peak_bytes / 2**20, 1),
                         "mesh_cache_hits": ex.meshes.hits, "mesh_cache_misses": ex.meshes.misses}
                if ex.scenes is not None:
                    extra["scene_cache_hits"], extra["scene_cache_misses"] = ex.scenes.hits, ex.scenes.misses
                ex.close()
            else:
                cache = serve.SceneCache(ctx, int(scene_cache_gb * 2**30)) if scene_cache_gb > 0 else None
                done = serve.plain_loop(ctx, reqs, stop_at=horizon, scenes=cache)
                extra = {}
                if cache is not None:
                    extra = {"scene_cache_hits": cache.hits, "scene_cache_misses": cache.misses}
                    cache.clear()
            ok = [r for r in done if r.error is None and r.result is not None]
            mismatch = sum(1 for r in ok if r.result != ref[int(picks[r.rid])])
            end = max([r.done for r in ok], default=t0)
            poses = sum(r.n_poses for r in ok)
            lat = serve.latency_stats(reqs, horizon=horizon)
            res[mode] = dict({"poses_per_s": round(poses / max(end - t0, 1e-9), 1), "answered": len(ok),
                              "span_s": round(end - t0, 3),
                              "errors": sum(1 for r in done if r.error), "latency_ms": lat,
                              "mismatches_vs_alone": mismatch}, **extra)
        res["vs_plain"] = round(res["served"]["poses_per_s"] / max(res["plain"]["poses_per_s"], 1e-9), 3)
        res["offered_poses_per_s"] = round(rate * float(np.mean([w.n_poses for w in pool])), 1)
        out["rates"][str(rate)] = res
    ctx.close()
    return out


def calibrate_copy():
    """A plain device-to-device copy of exactly 1 GiB, five times: the
    reference that scales FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    n = 1 << 30
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": 5}), flush=True)


KERNEL_SLOTS = {  # (threads, tile in device memory, keys in device memory) -> profiler slot
    ("256", "false", "false"): "score_lds_small", ("512", "false", "false"): "score_lds_small",
    ("1024", "false", "false"): "score_lds_large", ("1024", "false", "true"): "score_lds_tile",
    ("256", "true", "true"): "score_device"}


def _slot_of(name):
    import re
    m = re.search(r"score_kernel<\s*(\d+)\s*,\s*(\w+)\s*,\s*(\w+)\s*,", name)
    if m:
        return KERNEL_SLOTS.get(m.groups())
    m = re.search(r"(\w+)_kernel\b", name)
    return m.group(1) if m else None


def _csv_rows(folder, suffix):
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(folder, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as f:
            rows += list(csv.DictReader(f))
    if not rows:
        raise SystemExit(f"no *{suffix} under {folder}")
    return rows


def _last_dispatches(rows, steps):
    """Per profiler slot, the dispatch ids of its last `steps` dispatches
    (the timed step launches: bench.py's accounting and warm-up launches of
    the same kernels come first)."""
    by_slot = {}
    for r in rows:
        slot = _slot_of(r["Kernel_Name"])
        if slot:
            by_slot.setdefault(slot, set()).add(int(r["Dispatch_Id"]))
    return {slot: sorted(ids)[-steps:] for slot, ids in by_slot.items()}


def _counter_per_dispatch(folder, counter):
    """{dispatch id: summed value of `counter`} from a --pmc run."""
    out, names = {}, {}
    for r in _csv_rows(folder, "counter_collection.csv"):
        if r["Counter_Name"] != counter:
            continue
        d = int(r["Dispatch_Id"])
        out[d] = out.get(d, 0.0) + float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    return out, names


def reduce_profile(root, steps, out_path, cfg, seed, variant=None):
    """Counter record of the scoring kernels from rocprofv3 runs of one
    command: durations from the kernel trace and every counter from the
    same dispatches (the last `steps` of each kernel, i.e. the timed step
    launches), bytes scaled by a plain 1 GiB copy's readings."""
    trace = _csv_rows(os.path.join(root, "trace"), "kernel_trace.csv")
    sel = _last_dispatches(trace, steps)
    dur = {int(r["Dispatch_Id"]): (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in trace}
    cal = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        vals, _ = _counter_per_dispatch(os.path.join(root, f"copy_{c}"), c)
        per = max(vals.values())                  # KiB of the 1 GiB copy
        cal[c] = {"copy_kib_per_dispatch": per, "expected_kib": 1048576.0, "scale": 1048576.0 / per}
    # every counter of every --pmc run folder (all but the trace and the copies)
    counters = {}
    for folder in sorted(os.listdir(root)):
        if folder == "trace" or folder.startswith("copy_") or not os.path.isdir(os.path.join(root, folder)):
            continue
        names = sorted({r["Counter_Name"] for r in _csv_rows(os.path.join(root, folder), "counter_collection.csv")})
        for c in names:
            vals, kn = _counter_per_dispatch(os.path.join(root, folder), c)
            if vals:
                counters[c] = (vals, kn)
    kernels = {}
    for slot, ids in sel.items():
        ms = [dur[d] for d in ids]
        rec = {"dispatches": ids, "avg_ms": float(np.mean(ms)), "min_ms": float(np.min(ms)), "max_ms": float(np.max(ms))}
        for c, (vals, kn) in counters.items():
            cid = _last_dispatches([{"Kernel_Name": kn[d], "Dispatch_Id": d} for d in vals], steps).get(slot)
            if not cid:
                continue
            v = float(np.mean([vals[d] for d in cid]))
            if c in cal:
                rec[f"{c.lower()}_bytes_per_launch"] = v * 1024.0 * cal[c]["scale"]
            else:
                rec[f"{c.lower()}_per_launch"] = v
            rec.setdefault("counter_dispatches", {})[c] = cid
        if "sq_insts_valu_per_launch" in rec:
            lane_ops = rec["sq_insts_valu_per_launch"] * 64 / (rec["avg_ms"] / 1e3)
            rec["valu_lane_ops_per_s"] = lane_ops
            frac = lane_ops / (ALU_PEAK_TOPS * 1e12)
            # above 1 the counter holds instructions that issue faster than one
            # wave64 per 4 clocks; no fraction is reported then
            rec["valu_frac_of_39.3T"] = frac if frac <= 1.0 else None
        kernels[slot] = rec
    out = {"kernel_source_sha": kernel_source_sha(), "config": cfg, "seed": seed,
           "variant": variant or counter_variant(None, None, None), "steps": steps,
           "selection": "the last `steps` dispatches of each kernel in each run (the timed step launches)",
           "calibration": cal, "kernels": kernels}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: {"avg_ms": round(v["avg_ms"], 4),
                          "traffic_GB": round((v.get("fetch_size_bytes_per_launch", 0)
                                               + v.get("write_size_bytes_per_launch", 0)) / 1e9, 4)}
                      for k, v in kernels.items()}), flush=True)


def trace_gaps(root):
    """GPU idle time of the many-scene run from its rocprofv3 trace: the
    roctx ranges of the library's entry points delimit each pass of the plain
    loop (one perch_best_poses per scene) and each graph launch; within each,
    the union of kernel intervals is the busy time and what lies between
    kernels the idle gaps."""
    marks = _csv_rows(root, "marker_api_trace.csv")
    kern = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in _csv_rows(root, "kernel_trace.csv"))
    best = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in marks
                  if r["Function"] == "perch_best_poses")
    graph = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in marks
                   if r["Function"] == "perch_batch_launch")
    n_scenes = sum(1 for r in marks if r["Function"] == "perch_set_scene")

    def window(t0, t1):
        busy, gaps, cur = 0, [], None
        for a, b in kern:
            if b <= t0 or a >= t1:
                continue
            a, b = max(a, t0), min(b, t1)
            if cur is None:
                cur = [a, b]
            elif a > cur[1]:
                busy += cur[1] - cur[0]
                gaps.append(a - cur[1])
                cur = [a, b]
            else:
                cur[1] = max(cur[1], b)
        if cur is not None:
            busy += cur[1] - cur[0]
        return busy, gaps

    out = {"scenes": n_scenes, "plain_passes": [], "graph_launches": []}
    for k in range(len(best) // max(n_scenes, 1)):
        seg = best[k * n_scenes:(k + 1) * n_scenes]
        t0, t1 = seg[0][0], max(b for a, b in kern if a < seg[-1][1])
        busy, gaps = window(t0, t1)
        out["plain_passes"].append({"wall_ms": round((t1 - t0) / 1e6, 3), "busy_frac": round(busy / (t1 - t0), 5),
                                    "gaps": len(gaps), "gaps_ms": round(sum(gaps) / 1e6, 3),
                                    "largest_gap_ms": round(max(gaps, default=0) / 1e6, 4)})
    for n, (a, _) in enumerate(graph):
        # up to the next call into the library
        nxt = min((int(r["Start_Timestamp"]) for r in marks if int(r["Start_Timestamp"]) > a), default=1 << 62)
        ends = [e for s_, e in kern if a <= s_ < nxt]
        if not ends:
            continue
        t1 = max(ends)
        busy, gaps = window(a, t1)
        out["graph_launches"].append({"wall_ms": round((t1 - a) / 1e6, 3), "busy_frac": round(busy / (t1 - a), 5),
                                      "gaps": len(gaps), "gaps_ms": round(sum(gaps) / 1e6, 3)})
    print(json.dumps(out), flush=True)


def kernel_source_sha():
    """Hash of the scoring kernels' source (the kernel file and the device
    helpers it includes), which the committed counter record must match."""
    import hashlib
    h = hashlib.sha256()
    for name in ("perch_kernels.hip", "perch_device.h"):
        h.update(open(os.path.join(ROOT, "paper_2008_00326_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def counter_variant(volume, jo, search):
    """The scene options a counter record was taken with (None: the default)."""
    return {"volume": volume or "aabb", "jo": jo or "exact", "search": search or "table"}


def measured_counters(kernel_slot, cfg=2, variant=None):
    """The committed counter record of the kernel (HBM bytes per launch from
    FETCH_SIZE / WRITE_SIZE scaled by a plain copy, executed VALU
    instructions) when it was taken on this workload (configuration and
    scene options) with this kernel source, else None."""
    path = os.path.join(ROOT, "profiles", "score_kernel_cfg2_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    if rec.get("config") != cfg or rec.get("variant") != (variant or counter_variant(None, None, None)):
        return None
    return rec.get("kernels", {}).get(kernel_slot)


def measured_traffic(kernel_slot, cfg=2, variant=None):
    k = measured_counters(kernel_slot, cfg, variant)
    if not k or k.get("fetch_size_bytes_per_launch") is None or k.get("write_size_bytes_per_launch") is None:
        return None
    return round(k["fetch_size_bytes_per_launch"] + k["write_size_bytes_per_launch"], 1)


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or the platform's."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(w, sample):
    """The CPU oracle, as it stands, on the same workload: its windowed exact
    search (pinned equal to brute force) over every candidate of every object
    when `sample` is 0, else over `sample` seeded poses per object, on every
    thread its OpenMP runtime uses."""
    import oracle
    threads = oracle.threads()
    rng = np.random.default_rng(12345)
    flags = (oracle.USE_RGB if w.use_rgb else 0) | (oracle.MARK_OCCLUDERS if w.mark_occluders else 0)
    flags |= {"aabb": oracle.VOL_AABB, "cyl": oracle.VOL_CYL, "label": oracle.VOL_LABEL}[w.volume]
    flags |= oracle.JO_NN if w.jo == "nn" else 0
    n = 0
    t0 = time.perf_counter()
    for o in w.objects:
        sel = (np.arange(o.poses.shape[0]) if sample <= 0 else
               np.sort(rng.choice(o.poses.shape[0], min(sample, o.poses.shape[0]), replace=False)))
        m = w.meshes[o.mesh]
        oracle.score(m, w.scene, o.poses[sel], delta_mm=w.delta_mm, tau_c=w.tau_c, flags=flags, stride=w.stride,
                     label=o.label, search="window")
        n += len(sel)
    dt = time.perf_counter() - t0
    what = "every candidate" if sample <= 0 else f"{sample} seeded candidates per object"
    return {"value": round(n / dt, 3), "unit": "poses/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"{n} poses ({what}) of the same workload, the oracle's windowed exact search "
                      f"(equal to brute force, Eq. 3 / Eq. 4), {dt:.1f} s"}


if __name__ == "__main__":
    main()
