#!/usr/bin/env python3
"""Relocalisation throughput on one MI355X.

Workload (640x480): a seeded synthetic room, five random depth-15 trees,
reservoirs of 1024 entries adapted from 50 posed frames, at most 10 modes per
leaf; relocalisation with 1024 hypotheses, eta = 500 pixels per round, ten
halving rounds and the final inlier refit.  One benchmark step relocalises a
batch of 64 such frames (16 distinct query frames x 4 request seeds) through
the batched path, replayed from a HIP graph.  The plain path (one frame per
synchronous call) is timed beside it for latency and reloc/s.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import collections
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "relocalisations/s at 640x480, batched/served vs plain; p50/p99 latency"
MI355X_VALU_OPS = 256 * 4 * 16 * 2.4e9        # VALU lane-ops/s (one op per lane per clock per SIMD)
MI355X_HBM = 8.0e12

# Algorithmic unit of hypothesis generation: one generation iteration of a
# slot, up to and including the first one that passes every check (or all
# I_max when none does), priced at two Philox4x32-10 blocks, about 150 integer
# lane-ops.  The checks that follow the draws are not counted: about nine in
# ten iterations stop at the colour check of the first pair.
HYP_ITER_OPS = 150
# Traversal: the compulsory HBM bytes of a pixel are its depth and colour
# read once (8 B) and its leaf index per tree written (2 B each); the bytes a
# node test gathers (16 B node + 4 B probe word) come from the caches and are
# reported beside it, not as an HBM fraction.
NODE_TEST_BYTES = 20
TRAVERSE_PIXEL_IN = 8
# FP64 flops of Eq. 5 scoring: per mode evaluation d = y - mu (3), Sigma^-1 d
# (9 mul + 6 add), d . (Sigma^-1 d) (3 mul + 2 add) and the running minimum (1);
# per (hypothesis, pixel) the rigid transform (9 mul + 9 add) and the square
# root with its accumulation (2).
SCORE_MODE_FLOPS = 24
SCORE_PAIR_FLOPS = 20
MI355X_FP64 = 78.6e12
# FP64 flops per pixel of one Levenberg-Marquardt pass besides its mode
# evaluations: the transform (18), the residual's A r (15), A J (90), the
# gradient (42) and the normal matrix's upper triangle (147), the root and
# the weight (3), and the energy sum (1).
LM_PIXEL_FLOPS = 316


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """SHA-256 of the device sources (kernels, their launchers and shared
    device code); the host runtime (rl_runtime.hip) is left out, since it
    changes no kernel."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1810_12163_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))):
        if os.path.basename(f) == "rl_runtime.hip":
            continue
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_values(name: str) -> dict:
    """Figures of a committed counter summary under profiles/ (traffic bytes
    per launch from FETCH_SIZE and WRITE_SIZE scaled by a copy kernel's
    readings, VALU busy, L2 hit rate), or {} when the summary was taken on
    other kernel sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return {}
    taken_on, vals = None, {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if line.startswith("# device sources sha256"):
                taken_on = parts[-1]
            elif len(parts) >= 2 and parts[0] in ("traffic_bytes_per_launch", "valu_busy", "l2_hit_rate"):
                vals[parts[0]] = float(parts[1])
    return vals if taken_on == kernel_source_hash() else {}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def percentile(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--queries", type=int, default=16)
    ap.add_argument("--adapt-frames", type=int, default=50)
    ap.add_argument("--plain", type=int, default=32, help="plain relocalisations timed for latency")
    ap.add_argument("--cpu-frames", type=int, default=160,
                    help="oracle relocalisations on all host threads, about 10-20 s of host work (0 = skip)")
    ap.add_argument("--cpu-frames-1t", type=int, default=4,
                    help="oracle relocalisations on one thread, beside the threaded figure")
    ap.add_argument("--c1-queries", type=int, default=200,
                    help="plain relocalisations of the 160x120 one-tree workload (0 = skip)")
    ap.add_argument("--c3-queries", type=int, default=300,
                    help="frames through the three-stage cascade of 640x480 relocalisers, 30%% of them "
                         "far from every adaptation pose (0 = skip)")
    ap.add_argument("--c3-calibration", type=int, default=60,
                    help="queries of the disjoint set that calibrates the cascade's fallback thresholds")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--timer", default="hyp_search", choices=["traverse", "hyp_search", "ransac"])
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="measured seconds per arrival rate of the served leg (0 = skip it)")
    ap.add_argument("--serve-rates", default="200,500,1000")
    ap.add_argument("--saturation-rates", default="4000,8000,16000,32000",
                    help="offered rates of the served leg driven towards its throughput ceiling")
    ap.add_argument("--saturation-seconds", type=float, default=3.0)
    ap.add_argument("--serve-rooms", type=int, default=16)
    ap.add_argument("--serve-leaves-per-frame", type=int, default=256,
                    help="mode update schedule of the served rooms: 0 exact, K leaves per adapted frame")
    ap.add_argument("--no-robustness", action="store_true",
                    help="skip the missing-depth and depth-noise sweeps (Default RANSAC settings)")
    ap.add_argument("--robustness-queries", type=int, default=16)
    ap.add_argument("--render-procs", type=int, default=16,
                    help="worker processes rendering the inputs before the GPU is used (1 = in this process)")
    ap.add_argument("--cascade-frames", type=int, default=64,
                    help="frames relocalised by the paper's Fast -> Intermediate -> Slow cascade (0 = skip)")
    ap.add_argument("--lm-steps", type=int, default=5,
                    help="steps of the batch with LM refinement (0 = skip that leg)")
    ap.add_argument("--schedule", default="auto",
                    help="launch schedule 'ipt,fast_waves[,lds_levels[,score_window]]' (e.g. 4,1,8,0), or 'auto' to "
                         "time every one first")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device-to-device copy of this size (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}, WORLD_SIZE {world}): "
              "the relocaliser shards by room across GPUs with no collectives; only the one-GPU "
              "share is measured here.", file=sys.stderr)
        sys.exit(2)

    from rlsynth import scene, workloads

    # every CPU-side input is generated before the GPU runtime is initialised
    t_setup = time.time()
    log(f"[bench] rendering {args.adapt_frames} adaptation frames and {args.queries} queries (640x480)")
    # the standard 640x480 workload, rendered in worker processes.  Workers
    # are started only here, before this process touches the GPU (a profiler
    # that initialises the GPU first needs --render-procs 1).
    procs = max(1, min(args.render_procs, os.cpu_count() or 1))
    w = workloads.c2_corrupted(0, n_adapt=args.adapt_frames, n_queries=args.queries, processes=procs)
    robust_inputs = robustness_inputs(args, procs) if not args.no_robustness else None
    c1_inputs = workloads.c1(0, n_queries=8) if args.c1_queries > 0 else None
    c3_inputs = None
    if args.c3_queries > 0:
        c3_inputs = workloads.queries_for(w.room, [f.pose for f in w.adapt], args.c3_queries, room_id=0,
                                          novel_fraction=0.3, start=1000, processes=procs)
        # a disjoint calibration set for the cascade's fallback thresholds
        c3_calib = workloads.queries_for(w.room, [f.pose for f in w.adapt], args.c3_calibration, room_id=0,
                                         novel_fraction=0.3, start=3000, processes=procs)
        c3_inputs = (c3_inputs, c3_calib)
    serve_inputs = None
    if args.serve_seconds > 0:
        serve_inputs = workloads.serving_setup(n_rooms=args.serve_rooms, n_adapt=20, n_cameras=32,
                                               frames_per_camera=4, processes=procs, query_rooms=8,
                                               queries_per_room=8)
    log(f"[bench] inputs ready ({time.time() - t_setup:.1f} s)")

    import torch

    import paper_1810_12163_amd as rl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe_mib > 0:
        # a copy of known size: the hardware byte counters of this dispatch give
        # the scale between counted and moved bytes
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)          # one elementwise kernel: reads and writes the size
        torch.cuda.synchronize()
        log(f"[bench] copy probe: 3 copies of {args.copy_probe_mib} MiB")
        del src, dst
    p = w.params
    room = rl.Room(p, w.nodes, 640, 480, device=dev)
    for i, f in enumerate(w.adapt):
        room.adapt(torch.from_numpy(f.depth).to(dev), torch.from_numpy(f.rgb).to(dev), f.K, f.pose)
    room.update_modes()
    torch.cuda.synchronize()
    log(f"[bench] room adapted and clustered ({time.time() - t_setup:.1f} s)")
    qd = [torch.from_numpy(q.depth).to(dev) for q in w.queries]
    qc = [torch.from_numpy(q.rgb).to(dev) for q in w.queries]
    B = args.batch
    frames = [(i % len(w.queries), i // len(w.queries)) for i in range(B)]   # (query, seed)

    # ---- launch schedule (result-invariant) -------------------------------
    from paper_1810_12163_amd import autotune
    fixed = None if args.schedule == "auto" else tuple(int(v) for v in args.schedule.split(","))
    tuning = {}
    if fixed:
        room.set_schedule(*fixed)
    elif args.plain > 0:
        best, t = autotune.tune_room(room, qd[0], qc[0], w.queries[0].K, reps=5)
        tuning["plain"] = {",".join(str(x) for x in k): float(np.median(v)) for k, v in t.items()}
        log(f"[bench] plain schedule {best} (median ms {tuning['plain']})")

    # ---- plain path: one frame per synchronous call -----------------------
    lat = []
    for k in range((3 + args.plain) if args.plain > 0 else 0):
        qi = k % len(w.queries)
        t0 = time.perf_counter()
        room.relocalise(qd[qi], qc[qi], w.queries[qi].K, request_seed=k)
        dt = time.perf_counter() - t0
        if k >= 3:
            lat.append(dt)
    plain = None
    if lat:
        plain = dict(relocs_per_s=len(lat) / sum(lat), p50_ms=percentile(lat, 50) * 1e3,
                     p99_ms=percentile(lat, 99) * 1e3, mean_ms=float(np.mean(lat)) * 1e3, frames=len(lat))
        log(f"[bench] plain: {plain['relocs_per_s']:.1f} reloc/s, p50 {plain['p50_ms']:.2f} ms, "
            f"p99 {plain['p99_ms']:.2f} ms")

    # algorithmic work of one batch, from the plain path on the same (frame, seed) pairs
    iters = 0
    node_tests = 0
    mode_evals = 0
    pairs = 0
    Imax = p["max_candidate_generation_iterations"]
    eta = p["ransac_inliers_per_iteration"]
    plain_res = []
    for (qi, s) in frames:
        r = room.relocalise(qd[qi], qc[qi], w.queries[qi].K, request_seed=s)
        plain_res.append(r)
        hy = room.buffer_np(rl.BUF_HYPS, rl.HYP_DTYPE)[:p["max_pose_candidates"]]
        it = np.where(hy["valid"] != 0, hy["iter"] + 1, Imax)
        iters += int(it.sum())
        node_tests += int(np.count_nonzero(w.queries[qi].depth > 0)) * p["n_trees"] * p["depth"]
        # scoring work as defined: survivors entering each round x that round's pixels x |M(u)|
        if r["rounds"] > 0:
            I = room.buffer_np(rl.BUF_ILIST, np.int32)[:r["rounds"] * eta].reshape(r["rounds"], eta)
            nm = room.buffer_np(rl.BUF_NM, np.uint8).astype(np.int64)
            n = r["n_valid"]
            for rr in range(r["rounds"]):
                mode_evals += n * int(nm[I[rr]].sum())
                pairs += n * eta
                cull = p["max_pose_candidates_after_cull"]
                n = cull if (rr == 0 and cull < n) else ((n + 1) // 2 if n > p["max_relocalisations_to_output"] else n)

    # ---- batched path ----------------------------------------------------
    rounds = rl.rounds_for(p["max_pose_candidates"], p["max_pose_candidates_after_cull"],
                           p["max_relocalisations_to_output"])
    batch = rl.Batch(B, 640, 480, p["max_pose_candidates"], p["ransac_inliers_per_iteration"], rounds,
                     p["n_trees"], p["n_trees"] * p["max_cluster_count"], device=dev)
    reqs = [(room, qd[qi], qc[qi], w.queries[qi].K, s) for (qi, s) in frames]
    if fixed:
        batch.set_schedule(*fixed)
    else:
        best, t = autotune.tune_batch(batch, reqs, reps=5, use_graph=not args.no_graph)
        tuning["batched"] = {",".join(str(x) for x in k): float(np.median(v)) for k, v in t.items()}
        log(f"[bench] batched schedule {best} (median ms {tuning['batched']})")
    timer = {"traverse": rl.TIMER_TRAVERSE, "hyp_search": rl.TIMER_HYP_SEARCH, "ransac": rl.TIMER_RANSAC}[args.timer]
    use_graph = not args.no_graph
    for _ in range(args.warmup):
        res = batch.relocalise(reqs, use_graph=use_graph)
    torch.cuda.synchronize()
    # the timed steps: each batch queued on the batch's stream as soon as the
    # previous one is queued (no host wait between steps), results into one
    # device buffer; the last step's results are checked below
    import ctypes
    dres = torch.empty(B * ctypes.sizeof(rl.Result), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batch.relocalise_async(reqs, dres, use_graph=use_graph)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = B * args.steps / elapsed
    res = rl.Batch.decode(dres.cpu().numpy(), B)
    log(f"[bench] batched: {value:.1f} reloc/s ({elapsed / args.steps * 1e3:.2f} ms per {B}-frame step)")
    # step latency of the synchronous call (one batch at a time)
    step_ms = []
    for _ in range(args.steps):
        s0 = time.perf_counter()
        batch.relocalise(reqs, use_graph=use_graph)
        step_ms.append((time.perf_counter() - s0) * 1e3)

    # kernel timing: the same steps with direct launches, HIP events recorded by
    # the library around each timed stage on the stream it launches it on
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    ev1.record()               # torch creates the underlying hipEvent on first record
    torch.cuda.synchronize()
    stage_ms = {}
    for name, t in (("hyp_search", rl.TIMER_HYP_SEARCH), ("traverse", rl.TIMER_TRAVERSE), ("ransac", rl.TIMER_RANSAC)):
        batch.set_timer(t, ev0, ev1)
        ms = []
        for _ in range(args.steps):
            batch.relocalise(reqs, use_graph=False)
            ms.append(ev0.elapsed_time(ev1))
        batch.set_timer(rl.TIMER_NONE)
        stage_ms[name] = float(np.mean(ms))
        log(f"[bench] {name}: {stage_ms[name]:.3f} ms per launch ({B} frames)")

    same = all(np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"]
               for a, b in zip(res, plain_res))
    errs = [scene.pose_error(r["pose"].astype(np.float64), w.queries[qi].pose) for r, (qi, _) in zip(res, frames)]
    ok = [e[0] <= 0.05 and e[1] <= 5.0 for e in errs]

    lm = lm_leg(args, rl, room, batch, reqs, frames, w, qd, qc, use_graph) if args.lm_steps > 0 else None
    cascade = cascade_leg(args, rl, w, dev, c3_inputs[0] if c3_inputs else w.queries) if args.cascade_frames > 0 else None
    robustness = robustness_leg(args, rl, dev, robust_inputs) if robust_inputs is not None else None

    # ---- rooflines -------------------------------------------------------------
    def roof_search(ms):
        k = ms * 1e-3
        ops = iters * HYP_ITER_OPS
        prof = profile_values("k_hyp_search_640x480_batch64_counters.txt") if B == 64 else {}
        traffic = prof.get("traffic_bytes_per_launch")
        return dict(kernel="k_hyp_search", bound="alu", achieved=ops / k / 1e12, peak=MI355X_VALU_OPS / 1e12,
                    unit="TOP/s (VALU lane-ops)", frac=ops / k / MI355X_VALU_OPS, traffic=traffic,
                    launch_ms=ms, work=f"{iters} generation iterations (each slot up to its accepted one) x "
                                       f"{HYP_ITER_OPS} lane-ops (two Philox blocks)",
                    valu_busy=prof.get("valu_busy"), l2_hit_rate=prof.get("l2_hit_rate"),
                    traffic_unit="HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    traffic_GBps=(traffic / k / 1e9) if traffic else None)

    def roof_traverse(ms):
        k = ms * 1e-3
        hbm = B * 640 * 480 * (TRAVERSE_PIXEL_IN + 2 * p["n_trees"])
        prof = profile_values("k_traverse_640x480_batch64_counters.txt") if B == 64 else {}
        traffic = prof.get("traffic_bytes_per_launch")
        return dict(kernel="k_pack+k_traverse", bound="hbm", achieved=hbm / k / 1e9, peak=MI355X_HBM / 1e9,
                    unit="GB/s", frac=hbm / k / MI355X_HBM, traffic=traffic, launch_ms=ms,
                    touched_GBps=node_tests * NODE_TEST_BYTES / k / 1e9, valu_busy=prof.get("valu_busy"),
                    l2_hit_rate=prof.get("l2_hit_rate"),
                    work=f"{B} frames x 307200 px x {TRAVERSE_PIXEL_IN + 2 * p['n_trees']} B compulsory "
                         f"(depth and colour in, one 2-byte leaf per tree out); touched: {node_tests} node "
                         f"tests x {NODE_TEST_BYTES} B gathered, served by the caches")

    def roof_scoring(ms):
        k = ms * 1e-3
        fl = mode_evals * SCORE_MODE_FLOPS + pairs * SCORE_PAIR_FLOPS
        return dict(kernel="k_score+k_select+k_score_all+k_select_all", bound="alu", achieved=fl / k / 1e12,
                    peak=MI355X_FP64 / 1e12, unit="TFLOP/s (FP64)", frac=fl / k / MI355X_FP64, traffic=None,
                    launch_ms=ms, work=f"{mode_evals} mode evaluations x {SCORE_MODE_FLOPS} + {pairs} "
                                       f"(hypothesis, pixel) pairs x {SCORE_PAIR_FLOPS} FP64 flops")

    rooflines = {"hyp_search": roof_search(stage_ms["hyp_search"]), "traverse": roof_traverse(stage_ms["traverse"]),
                 "ransac": roof_scoring(stage_ms["ransac"])}
    roof = rooflines[args.timer]

    # ---- CPU baseline: the oracle on a bounded sample ----------------------
    cpu = None
    if args.cpu_frames > 0:
        cpu = cpu_leg(args, rl, room, w, p)

    c1 = c1_leg(args, rl, dev, c1_inputs) if c1_inputs is not None else None
    c3 = c3_leg(args, rl, dev, w, c3_inputs) if c3_inputs is not None else None
    served = serve_leg(args, rl, dev, serve_inputs) if serve_inputs is not None else None

    out = {
        "metric": METRIC, "value": value, "unit": "relocalisations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "640x480 synthetic room; 5 random trees of depth 15; reservoirs 1024; "
                               "<=10 modes/leaf; 50 adaptation frames; 1024 hypotheses of up to 6000 "
                               "generation iterations; eta 500; halving while more than one survives "
                               "(rounds run and valid hypotheses per frame under 'batched'); inlier refit",
                   "form": "batched" + (" (hipGraph replay)" if use_graph else ""), "batch": B,
                   "distinct_frames": len(w.queries),
                   "schedule": {"plain": list(room.schedule), "batched": list(batch.schedule),
                                "tuned": not fixed}},
        "schedule_tuning_ms": tuning or None,
        "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_kernel": {k: v for k, v in roof.items() if k not in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "rooflines_other": {n: r for n, r in rooflines.items() if r is not roof},
        "cpu_baseline": cpu,
        "plain": plain,
        "plain_c1": c1,
        "batched": dict(relocs_per_s=value, step_p50_ms=percentile(step_ms, 50),
                        step_p99_ms=percentile(step_ms, 99), identical_to_plain=bool(same),
                        mean_n_valid=float(np.mean([r["n_valid"] for r in res])),
                        mean_rounds_run=float(np.mean([r["rounds"] for r in res])),
                        rounds_run_counts={str(k): v for k, v in
                                           sorted(collections.Counter(r["rounds"] for r in res).items())}),
        "cascade_c3": c3,
        "served": served,
        "lm": lm,
        "cascade": cascade,
        "robustness": robustness,
        "accuracy": dict(frac_within_5cm_5deg=float(np.mean(ok)),
                         median_cm=float(np.median([e[0] for e in errs]) * 100),
                         median_deg=float(np.median([e[1] for e in errs]))),
        "paper_context": "Fast relocaliser 25.1 ms/frame on a GTX 1080 Ti (Table 3)",
    }
    print(json.dumps(out), flush=True)


def cpu_leg(args, rl, room, w, p):
    """The oracle (traversal, hypotheses, RANSAC and refit of 640x480 query
    frames, modes taken from the GPU room) on the host: on every host thread
    (its OpenMP loops over pixels and hypotheses), and on one thread."""
    import oracle
    nm = room.buffer_np(rl.BUF_NMODES, np.uint8).copy()
    modes = room.buffer_np(rl.BUF_MODES, np.float32).copy()
    T, D, M = p["n_trees"], p["depth"], p["max_cluster_count"]

    def run(n, threads):
        used = oracle.lib().oracle_set_threads(threads)
        t0 = time.perf_counter()
        for k in range(n):
            q = w.queries[k % len(w.queries)]
            leaves = oracle.traverse(q.depth, q.rgb, None, w.nodes, T, D, p["ref_width"])
            oracle.estimate_pose(q.depth, q.rgb, q.K, leaves, nm, modes, T, D, M, p, k, trace=False)
        return time.perf_counter() - t0, used

    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    ct, used = run(args.cpu_frames, threads)
    c1t, _ = run(args.cpu_frames_1t, 1) if args.cpu_frames_1t > 0 else (None, 1)
    oracle.lib().oracle_set_threads(threads)
    model = cpu_model()
    cpu = dict(value=args.cpu_frames / ct, unit="relocalisations/s", cores=used, kind="oracle",
               cpu_model=model, host_threads=os.cpu_count(),
               sample=f"{args.cpu_frames} relocalisations of 640x480 query frames (traversal, hypotheses, "
                      f"RANSAC, refit; modes taken from the room) on {used} threads of {model}, {ct:.1f} s",
               single_thread=(dict(value=args.cpu_frames_1t / c1t, frames=args.cpu_frames_1t, seconds=c1t)
                              if c1t else None))
    log(f"[bench] oracle: {cpu['value']:.3f} reloc/s on {used} threads over {ct:.1f} s"
        + (f"; 1 thread {args.cpu_frames_1t / c1t:.3f} reloc/s" if c1t else ""))
    return cpu


def c1_leg(args, rl, dev, w1):
    """The small plain workload: 160x120 frames, one depth-8 tree, reservoirs
    of 64, 64 hypotheses, eta 100; one synchronous relocalisation at a time."""
    import torch

    from rlsynth import scene
    room = rl.Room(w1.params, w1.nodes, 160, 120, device=dev)
    for f in w1.adapt:
        room.adapt(torch.from_numpy(f.depth).to(dev), torch.from_numpy(f.rgb).to(dev), f.K, f.pose)
    room.update_modes()
    qd = [torch.from_numpy(q.depth).to(dev) for q in w1.queries]
    qc = [torch.from_numpy(q.rgb).to(dev) for q in w1.queries]
    torch.cuda.synchronize()
    lat, errs = [], []
    for k in range(5 + args.c1_queries):
        qi = k % len(w1.queries)
        t0 = time.perf_counter()
        r = room.relocalise(qd[qi], qc[qi], w1.queries[qi].K, request_seed=k)
        dt = time.perf_counter() - t0
        if k >= 5:
            lat.append(dt)
            errs.append(scene.pose_error(r["pose"].astype(np.float64), w1.queries[qi].pose)
                        if r["status"] == "ok" else (np.inf, np.inf))
    room.close()
    out = dict(relocs_per_s=len(lat) / sum(lat), p50_ms=percentile(lat, 50) * 1e3, p99_ms=percentile(lat, 99) * 1e3,
               mean_ms=float(np.mean(lat)) * 1e3, frames=len(lat),
               frac_within_5cm_5deg=float(np.mean([e[0] <= 0.05 and e[1] <= 5.0 for e in errs])))
    log(f"[bench] c1 plain (160x120): {out['relocs_per_s']:.1f} reloc/s, p50 {out['p50_ms']:.3f} ms, "
        f"p99 {out['p99_ms']:.3f} ms")
    return out


# fallback thresholds of the three-stage cascade on the plane score of a
# stage's pose (metres): the paper's 5 cm after the first stage, 7.5 cm after
# the second.  The winner's mean Eq. 5 energy does not separate right from
# wrong poses on these rooms (its median is higher for correct poses), so the
# fallback uses the model-based score as the paper's cascade does.
C3_THRESHOLDS = (0.05, 0.075)


def c3_leg(args, rl, dev, w, inputs):
    """The three-stage cascade of 640x480 relocalisers on the shared forest:
    (a) the 2x decimated 320x240 frame with 256 hypotheses, (b) the full frame
    with 1024 hypotheses and the inlier refit, (c) 4096 hypotheses culled to
    16, re-ranked by the plane score (mean distance of the back-projected depth
    to the nearest surface).  A stage falls back when the plane score of its
    pose exceeds its threshold: the paper's 5 cm (stage a) and 7.5 cm (stage
    b), and thresholds calibrated on a disjoint set of queries (the 95th
    percentile of each stage's score over the frames it relocalises within
    5 cm / 5 deg).  30% of the queries lie >= 50 cm or >= 50 deg from every
    adaptation pose.  Frames one at a time: latency, stage reached, accuracy."""
    import torch

    from paper_1810_12163_amd.cascade import Cascade, c3_stages, calibrate_thresholds
    from rlsynth import presets, scene
    queries, calib = inputs
    room = rl.Room(dict(w.params, **{k: presets.preset("c3c")[k] for k in
                                     ("max_pose_candidates", "max_pose_candidates_after_cull",
                                      "max_relocalisations_to_output", "final_refine")}),
                   w.nodes, 640, 480, device=dev)
    for f in w.adapt:
        room.adapt(torch.from_numpy(f.depth).to(dev), torch.from_numpy(f.rgb).to(dev), f.K, f.pose)
    room.update_modes()
    cas = Cascade(room, c3_stages(C3_THRESHOLDS), scene.surface_records(w.room), model="plane",
                  fallback="model")
    adapt_poses = [f.pose for f in w.adapt]
    for k in range(3):                                   # graph capture of each stage's shape
        q = queries[k]
        cas.relocalise(torch.from_numpy(q.depth).to(dev), torch.from_numpy(q.rgb).to(dev), q.K, request_seed=5000 + k)
    torch.cuda.synchronize()
    frames = [(torch.from_numpy(q.depth).to(dev), torch.from_numpy(q.rgb).to(dev), q) for q in queries]
    novel = np.array([all(scene.pose_error(q.pose, a)[0] >= 0.5 or scene.pose_error(q.pose, a)[1] >= 50.0
                          for a in adapt_poses) for q in queries])

    def run(thresholds):
        ms, stages, errs, energies = [], [], [], []
        for k, (d, c, q) in enumerate(frames):
            torch.cuda.synchronize()
            out = cas.relocalise(d, c, q.K, request_seed=k)
            ms.append(out["ms"])
            stages.append(out["stage"])
            e = scene.pose_error(out["pose"].astype(np.float64), q.pose) if out["status"] == "ok" else (np.inf, np.inf)
            errs.append(e)
            energies.append(out.get("mean_energy", np.inf))
        ok = np.array([e[0] <= 0.05 and e[1] <= 5.0 for e in errs])
        first = np.array(energies)
        return dict(frames=len(ms), mean_ms=float(np.mean(ms)), p50_ms=percentile(ms, 50), p99_ms=percentile(ms, 99),
                    relocs_per_s=len(ms) / (sum(ms) * 1e-3),
                    stage_counts={s.name: stages.count(s.name) for s in cas.stages},
                    frac_within_5cm_5deg=float(np.mean(ok)),
                    frac_within_5cm_5deg_near=float(np.mean(ok[~novel])) if np.any(~novel) else None,
                    frac_within_5cm_5deg_novel=float(np.mean(ok[novel])) if np.any(novel) else None,
                    novel_fraction=float(np.mean(novel)), thresholds_m=[float(t) for t in thresholds],
                    mean_energy_median_correct=float(np.median(first[ok])) if np.any(ok) else None,
                    mean_energy_median_wrong=float(np.median(first[~ok])) if np.any(~ok) else None,
                    median_cm=float(np.median([e[0] for e in errs]) * 100))

    res = run(C3_THRESHOLDS)
    log(f"[bench] c3 cascade: {res['mean_ms']:.2f} ms per frame (p50 {res['p50_ms']:.2f}, p99 {res['p99_ms']:.2f}), "
        f"stages {res['stage_counts']}, within 5cm/5deg {res['frac_within_5cm_5deg']:.3f} "
        f"(near {res['frac_within_5cm_5deg_near']}, novel {res['frac_within_5cm_5deg_novel']}); returned pose's "
        f"mean energy, median: correct {res['mean_energy_median_correct']} / wrong {res['mean_energy_median_wrong']}")
    if calib:
        cal = [(torch.from_numpy(q.depth).to(dev), torch.from_numpy(q.rgb).to(dev), q.K, 20000 + k, q.pose)
               for k, q in enumerate(calib)]

        def correct(pose, truth):
            e = scene.pose_error(pose.astype(np.float64), truth)
            return e[0] <= 0.05 and e[1] <= 5.0

        th = calibrate_thresholds(cas, cal, correct, q=95.0)
        rc = run(th)
        rc["calibration_frames"] = len(cal)
        res["calibrated"] = rc
        log(f"[bench] c3 cascade, thresholds calibrated on {len(cal)} disjoint queries "
            f"({', '.join(f'{t * 100:.1f} cm' for t in th)}): {rc['mean_ms']:.2f} ms per frame, stages "
            f"{rc['stage_counts']}, within 5cm/5deg {rc['frac_within_5cm_5deg']:.3f} "
            f"(near {rc['frac_within_5cm_5deg_near']}, novel {rc['frac_within_5cm_5deg_novel']})")
    room.close()
    return res


def lm_leg(args, rl, room, batch, reqs, frames, w, qd, qc, use_graph):
    """The same batch with Levenberg-Marquardt refinement in se(3) in every
    round after the first (the paper's pose update), through the batched
    path: throughput, the RANSAC stage's FP64 rate, equality with the plain
    path and accuracy."""
    import torch

    from rlsynth import scene
    p = w.params
    eta = p["ransac_inliers_per_iteration"]
    iters = p["lm_iterations"]
    plain = []
    flops = 0
    for (qi, s) in frames:
        r = room.relocalise(qd[qi], qc[qi], w.queries[qi].K, request_seed=s, pose_update=1)
        plain.append(r)
        if r["rounds"] == 0:
            continue
        I = room.buffer_np(rl.BUF_ILIST, np.int32)[:r["rounds"] * eta]
        nm = room.buffer_np(rl.BUF_NM, np.uint8).astype(np.int64)
        per_px = nm[I] * SCORE_MODE_FLOPS
        n, first = r["n_valid"], True
        for rr in range(r["rounds"]):
            if rr == 0:
                flops += n * int(per_px[:eta].sum() + eta * SCORE_PAIR_FLOPS)
            else:
                flops += n * (iters + 1) * int(per_px[:(rr + 1) * eta].sum() + (rr + 1) * eta * LM_PIXEL_FLOPS)
            cull = p["max_pose_candidates_after_cull"]
            n = cull if (first and cull < n) else ((n + 1) // 2 if n > p["max_relocalisations_to_output"] else n)
            first = False
    lreqs = [q + (0, 1) for q in reqs]            # n_hypotheses: the room's; pose_update: on
    for _ in range(args.warmup):
        res = batch.relocalise(lreqs, use_graph=use_graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.lm_steps):
        res = batch.relocalise(lreqs, use_graph=use_graph)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    ev1.record()
    torch.cuda.synchronize()
    batch.set_timer(rl.TIMER_RANSAC, ev0, ev1)
    ms = []
    for _ in range(args.lm_steps):
        batch.relocalise(lreqs, use_graph=False)
        ms.append(ev0.elapsed_time(ev1))
    batch.set_timer(rl.TIMER_NONE)
    rms = float(np.mean(ms))
    same = all(np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"] for a, b in zip(res, plain))
    errs = [scene.pose_error(r["pose"].astype(np.float64), w.queries[qi].pose) for r, (qi, _) in zip(res, frames)]
    B = len(reqs)
    out = dict(relocs_per_s=B * args.lm_steps / el, ms_per_step=el / args.lm_steps * 1e3, lm_iterations=iters,
               identical_to_plain=bool(same),
               frac_within_5cm_5deg=float(np.mean([e[0] <= 0.05 and e[1] <= 5.0 for e in errs])),
               median_cm=float(np.median([e[0] for e in errs]) * 100),
               roofline=dict(kernel="k_score+k_lm+k_select (RANSAC stage)", bound="alu",
                             achieved=flops / (rms * 1e-3) / 1e12, peak=MI355X_FP64 / 1e12, unit="TFLOP/s (FP64)",
                             frac=flops / (rms * 1e-3) / MI355X_FP64, launch_ms=rms,
                             work=f"{flops} FP64 flops (first-round scoring; LM passes x pixels x "
                                  f"(|M(u)| x {SCORE_MODE_FLOPS} + {LM_PIXEL_FLOPS}))"))
    log(f"[bench] LM: {out['relocs_per_s']:.1f} reloc/s ({out['ms_per_step']:.2f} ms per {B}-frame step), "
        f"RANSAC stage {rms:.3f} ms, {out['roofline']['achieved']:.2f} TFLOP/s FP64, "
        f"within 5cm/5deg {out['frac_within_5cm_5deg']:.3f}, identical to plain {same}")
    return out


def cascade_leg(args, rl, w, dev, queries):
    """The paper's cascade (Sec. 3.2.5): Fast -> Intermediate -> Slow with
    Table 8's RANSAC settings on one shared forest built with Table 8's Forest
    row for those relocalisers (M_max 50, reservoirs of 2048, tau_c 0.2,
    minimum cluster size 5), falling back when the depth-raycast score
    (Eq. 6-7) of a stage's pose exceeds 5 cm, then 7.5 cm; the slow stage
    ranks its 16 outputs by that score (Eq. 8).  Frames one at a time (the
    cascade queries: 30% of them far from every adaptation pose): latency per
    frame, stage reached, accuracy."""
    import torch

    from paper_1810_12163_amd.cascade import Cascade, paper_stages
    from rlsynth import presets, scene
    fast = presets.preset("fast")
    p = dict(w.params, max_pose_candidates=2048, max_pose_candidates_after_cull=64,
             **{k: fast[k] for k in ("clusterer_sigma", "clusterer_tau", "max_cluster_count", "min_cluster_size",
                                     "reservoir_capacity")})
    room = rl.Room(p, w.nodes, 640, 480, device=dev)
    for f in w.adapt:
        room.adapt(torch.from_numpy(f.depth).to(dev), torch.from_numpy(f.rgb).to(dev), f.K, f.pose)
    room.update_modes()
    cas = Cascade(room, paper_stages(), scene.surface_records(w.room), min_depth=scene.DEPTH_MIN,
                  max_depth=scene.DEPTH_MAX)
    qs = [queries[k % len(queries)] for k in range(args.cascade_frames)]
    dev_q = [(torch.from_numpy(q.depth).to(dev), torch.from_numpy(q.rgb).to(dev)) for q in qs]
    for k in range(2):                                   # graph capture of each stage's shape
        cas.relocalise(*dev_q[k], qs[k].K, request_seed=1000 + k)
    torch.cuda.synchronize()
    ms, stages, errs = [], [], []
    for k, q in enumerate(qs):
        out = cas.relocalise(*dev_q[k], q.K, request_seed=k)
        ms.append(out["ms"])
        stages.append(out["stage"])
        errs.append(scene.pose_error(out["pose"].astype(np.float64), q.pose) if out["status"] == "ok"
                    else (np.inf, np.inf))
    room.close()
    res = dict(frames=len(ms), mean_ms=float(np.mean(ms)), p50_ms=percentile(ms, 50), p99_ms=percentile(ms, 99),
               stage_counts={s.name: stages.count(s.name) for s in cas.stages},
               frac_within_5cm_5deg=float(np.mean([e[0] <= 0.05 and e[1] <= 5.0 for e in errs])),
               median_cm=float(np.median([e[0] for e in errs]) * 100),
               thresholds_m=[s.threshold for s in cas.stages[:-1]],
               forest_row=dict(max_cluster_count=p["max_cluster_count"], reservoir_capacity=p["reservoir_capacity"],
                               clusterer_tau=p["clusterer_tau"], min_cluster_size=p["min_cluster_size"]))
    log(f"[bench] cascade: {res['mean_ms']:.2f} ms per frame (p50 {res['p50_ms']:.2f}), stages {res['stage_counts']}, "
        f"within 5cm/5deg {res['frac_within_5cm_5deg']:.3f}")
    return res


ROBUSTNESS_LEVELS = [("missing", p) for p in (0.1, 0.3, 0.5, 0.7, 0.9, 0.95)] + \
                    [("noise", s) for s in (0.0, 0.025, 0.05, 0.075, 0.1)] + [("novel", 1.0)]


def robustness_inputs(args, procs):
    """Frames of every sweep level, rendered before the GPU is used (each pose
    raycast once, every level's sensor noise drawn from the frame's seed)."""
    from rlsynth import workloads
    sensor = [(k, v) for k, v in ROBUSTNESS_LEVELS if k != "novel"]
    kws = [dict(dropout=v) if k == "missing" else dict(depth_rel_sigma=v) for k, v in sensor]
    ws = workloads.c2_sweep(kws, 0, n_adapt=50, n_queries=args.robustness_queries, processes=procs)
    out = [(k, v, w) for (k, v), w in zip(sensor, ws)]
    for k, v in ROBUSTNESS_LEVELS:
        if k == "novel":
            out.append((k, v, workloads.c2_sweep([{}], 0, n_adapt=50, n_queries=args.robustness_queries,
                                                 processes=procs, novel_fraction=v)[0]))
    log(f"[bench] robustness inputs rendered ({len(out)} levels)")
    return out


def robustness_leg(args, rl, dev, inputs):
    """The paper's robustness protocols on the 640x480 workload: every
    adaptation and query frame re-rendered with a fraction p of the depth
    pixels zeroed (r <= p, r ~ U[0,1]), or with depth-dependent noise
    d + n d, n ~ N(0, sigma^2); relocalised with the Default relocaliser's
    RANSAC settings (1024 hypotheses, cull to 64, eta 512, LM with the
    covariance, one output).  Also queries all drawn >= 50 cm or >= 50 deg
    from every adaptation pose.  Fraction of queries within 5 cm / 5 deg."""
    import torch

    from rlsynth import scene
    out = {}
    for kind, v, w in inputs:
        t0 = time.time()
        room = rl.Room(dict(w.params, max_pose_candidates_after_cull=64, ransac_inliers_per_iteration=512),
                       w.nodes, 640, 480, device=dev)
        for f in w.adapt:
            room.adapt(torch.from_numpy(f.depth).to(dev), torch.from_numpy(f.rgb).to(dev), f.K, f.pose)
        room.update_modes()
        errs = []
        for k, q in enumerate(w.queries):
            r = room.relocalise(torch.from_numpy(q.depth).to(dev), torch.from_numpy(q.rgb).to(dev), q.K,
                                request_seed=k, pose_update=1, final_refine=0)
            errs.append(scene.pose_error(r["pose"].astype(np.float64), q.pose) if r["status"] == "ok"
                        else (np.inf, np.inf))
        room.close()
        key = f"{kind}_{v:g}"
        out[key] = dict(frac_within_5cm_5deg=float(np.mean([e[0] <= 0.05 and e[1] <= 5.0 for e in errs])),
                        median_cm=float(np.median([e[0] for e in errs]) * 100), queries=len(errs))
        log(f"[bench] robustness {key}: within 5cm/5deg {out[key]['frac_within_5cm_5deg']:.3f}, "
            f"median {out[key]['median_cm']:.1f} cm ({time.time() - t0:.1f} s)")
    return out


def serve_leg(args, rl, dev, inputs):
    """Open-loop Poisson arrivals from 32 cameras over 16 resident rooms; 75%
    relocalise / 25% adapt; resolutions 160x120, 320x240, 640x480 with 256,
    512, 1024 hypotheses.  Frames arrive in host memory and are copied into
    the server's frame slots; rooms, batch contexts and frame slots are
    charged against one device-memory budget.  Continuous batching, two
    batches in flight.  The configured rates run for --serve-seconds each;
    higher rates then drive the server towards its throughput ceiling."""
    import torch

    from paper_1810_12163_amd import serve
    from rlsynth import presets, scene, workloads

    t0 = time.time()
    specs, cams = inputs
    p = presets.preset("c5")
    room_bytes = sum(rl.room_state_bytes(p, 640, 480))
    ctx_bytes = serve.batch_workspace_bytes(64, 640, 480, 1024, 500, 10, 5, 50)
    slots = 128
    budget = len(specs) * room_bytes + 2 * ctx_bytes + slots * serve.FramePool.slot_bytes(640, 480)
    server = serve.Server(max_batch=64, max_width=640, max_height=480, max_hypotheses=1024, max_eta=500,
                          max_rounds=10, n_trees=5, max_modes_per_pixel=50, contexts=2, memory_budget=budget,
                          frame_slots=slots, device=dev)
    rooms = []
    for sp in specs:
        room = server.create_room(p, sp["nodes"])
        assert room is not None, "the budget holds every room"
        for f in sp["adapt"]:
            room.adapt(torch.from_numpy(f.depth).to(dev), torch.from_numpy(f.rgb).to(dev), f.K, f.pose)
        room.update_modes()
        room.set_mode_schedule(args.serve_leaves_per_frame)
        rooms.append(room)
    torch.cuda.synchronize()
    # camera frames in pinned host memory; device copies for the mixed-batch leg
    camh = [[serve.pack_host_frame(f.depth, f.rgb) + (f,) for f in c["frames"]] for c in cams]
    camf = [[(torch.from_numpy(f.depth).to(dev), torch.from_numpy(f.rgb).to(dev), f) for f in c["frames"]]
            for c in cams]
    extra = server.create_room(p, specs[0]["nodes"])
    log(f"[bench] serving: {len(rooms)} rooms resident ({len(rooms) * room_bytes / 2**30:.1f} GiB), budget "
        f"{budget / 2**30:.2f} GiB ({slots} frame slots, {len(server.ctx)} contexts); a 17th room "
        f"{'refused' if extra is None else 'ADMITTED'}; setup {time.time() - t0:.1f} s")
    out = {"memory_budget_GiB": budget / 2**30, "frame_slots": slots, "contexts": len(server.ctx),
           "room_GiB": room_bytes / 2**30, "extra_room_refused": extra is None}
    # a steady mixed batch: 64 frames over 8 rooms, resolutions and hypothesis
    # counts drawn with the cameras' frames, and 16 adaptation frames applied
    # after every batch's relocalisations
    rng = np.random.default_rng(64)
    near = [c for c in range(len(cams)) if cams[c]["room"] < 8]
    picks = [(c, int(rng.integers(len(camf[c])))) for c in rng.choice(near, size=64)]
    breqs = [(rooms[cams[c]["room"]], camf[c][k][0], camf[c][k][1], camf[c][k][2].K, i,
              workloads.HYPOTHESES[camf[c][k][2].w]) for i, (c, k) in enumerate(picks)]
    adapts = [(rooms[cams[c]["room"]], camf[c][k][0], camf[c][k][1], camf[c][k][2]) for (c, k) in picks[:16]]
    mb = rl.Batch(64, 640, 480, 1024, 500, 10, 5, 50, device=dev)
    from paper_1810_12163_amd import autotune
    if args.schedule == "auto":
        mb_sched, _ = autotune.tune_batch(mb, breqs, reps=3)
    else:
        mb_sched = tuple(int(v) for v in args.schedule.split(","))
        mb.set_schedule(*mb_sched)
    for _ in range(2):
        mb.relocalise(breqs)
    torch.cuda.synchronize()
    steps = max(3, args.steps)
    t1 = time.perf_counter()
    for _ in range(steps):
        mb.relocalise(breqs)
    torch.cuda.synchronize()
    el_r = time.perf_counter() - t1
    # the 16 adaptations inside the batch, after its relocalisations
    areqs = breqs + [rl.AdaptRequest(room, d, rgb, f.K, f.pose) for room, d, rgb, f in adapts]
    mba = rl.Batch(80, 640, 480, 1024, 500, 10, 5, 50, device=dev)
    mba.set_schedule(*mb_sched)
    for _ in range(2):
        mba.relocalise(areqs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        mba.relocalise(areqs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    # the same adaptations as separate calls on the rooms' streams
    t1 = time.perf_counter()
    for _ in range(steps):
        mb.relocalise(breqs)
        for room, d, rgb, f in adapts:
            room.adapt(d, rgb, f.K, f.pose)
    torch.cuda.synchronize()
    el_sep = time.perf_counter() - t1
    mb.close()
    mba.close()
    mix = collections.Counter(camf[c][k][2].w for c, k in picks)
    out["mixed_batch"] = dict(relocs_per_s=64 * steps / el_r, ms_per_batch=el_r / steps * 1e3,
                              relocs_per_s_with_adapt=64 * steps / el, ms_per_step_with_adapt=el / steps * 1e3,
                              ms_per_step_with_separate_adapt_calls=el_sep / steps * 1e3,
                              rooms=8, widths={str(k): v for k, v in sorted(mix.items())}, adapts_per_step=16,
                              schedule=list(mb_sched))
    mbo = out["mixed_batch"]
    log(f"[bench] mixed batch (8 rooms, {dict(mix)} by width, schedule {mb_sched}): {mbo['relocs_per_s']:.1f} reloc/s "
        f"({mbo['ms_per_batch']:.2f} ms per 64-frame batch); with 16 adaptations in the batch "
        f"{mbo['relocs_per_s_with_adapt']:.1f} reloc/s ({mbo['ms_per_step_with_adapt']:.2f} ms; as separate calls "
        f"{mbo['ms_per_step_with_separate_adapt_calls']:.2f} ms)")
    # the headline workload over distinct frames: 64 different 640x480 queries,
    # 8 per room over 8 rooms, 1024 hypotheses each
    hq = [(r, f) for r in range(8) for f in specs[r]["queries"]]
    hreqs = [(rooms[r], torch.from_numpy(f.depth).to(dev), torch.from_numpy(f.rgb).to(dev), f.K, i, 1024)
             for i, (r, f) in enumerate(hq)]
    hb = rl.Batch(64, 640, 480, 1024, 500, 10, 5, 50, device=dev)
    hb.set_schedule(*mb_sched)
    res = hb.relocalise(hreqs)
    hb.relocalise(hreqs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        hb.relocalise(hreqs)
    torch.cuda.synchronize()
    el_h = time.perf_counter() - t1
    hb.close()
    herr = [scene.pose_error(x["pose"].astype(np.float64), f.pose) if x["status"] == "ok" else (np.inf, np.inf)
            for x, (_, f) in zip(res, hq)]
    out["distinct_640x480"] = dict(relocs_per_s=64 * steps / el_h, ms_per_batch=el_h / steps * 1e3, rooms=8,
                                   distinct_frames=len(hq),
                                   frac_within_5cm_5deg=float(np.mean([e[0] < 0.05 and e[1] < 5.0 for e in herr])))
    hdo = out["distinct_640x480"]
    log(f"[bench] 64 distinct 640x480 frames over 8 rooms: {hdo['relocs_per_s']:.1f} reloc/s "
        f"({hdo['ms_per_batch']:.2f} ms per batch), within 5cm/5deg {hdo['frac_within_5cm_5deg']:.3f}")
    del camf, hreqs
    warm = 2.0
    rates = [(float(v), args.serve_seconds) for v in args.serve_rates.split(",") if v] + \
            [(float(v), args.saturation_seconds) for v in args.saturation_rates.split(",") if v]
    for rate, seconds in rates:
        server.reset_stats()
        arr = serve.poisson_arrivals(rate, warm + seconds, seed=int(rate))
        rng = np.random.default_rng(int(rate) + 1)
        reqs = []
        for i in range(len(arr)):
            c = int(rng.integers(len(cams)))
            buf, hw, f = camh[c][int(rng.integers(len(camh[c])))]
            kind = "adapt" if rng.uniform() < 0.25 else "relocalise"
            reqs.append(serve.Request(rid=i, kind=kind, room=rooms[cams[c]["room"]], host_frame=buf, frame_hw=hw,
                                      K=f.K, pose=f.pose if kind == "adapt" else None,
                                      n_hypotheses=workloads.HYPOTHESES[f.w]))
        st = serve.run_open_loop(server, reqs, arr, warmup_s=warm)
        st["measured_s"] = seconds
        out[f"{int(rate)}/s"] = st
        log(f"[bench] served {int(rate)}/s over {seconds:g} s: {st['relocs_per_s']:.1f} reloc/s, p50 "
            f"{st['p50_ms']:.2f} ms, p99 {st['p99_ms']:.2f} ms, mean batch {st['mean_batch']:.1f}, waited for a "
            f"frame slot {st['deferred']}, refused {st['refused']}")
    server.close()
    sat = [out[f"{int(r)}/s"] for r, _ in rates]
    out["ceiling_relocs_per_s"] = max(x["relocs_per_s"] for x in sat)
    return out


if __name__ == "__main__":
    main()
