"""Benchmark of the TPC track-finding hot path on one MI355X.

Workload: the batched uneven set, 512 independent single-sector instances
(half pp-like with 20-200 tracks, half Pb-Pb-like with 50-800, log-uniform,
shuffled; ~10.9M float32 clusters, seed 40040000), all inputs resident in
HBM.  One step = the whole hot path over the batch:
  grid -> neighbours -> cleaning/starts -> tracklets -> selection of every
  instance (tpc_track_batch, one launch sequence over all instances, one HIP
  graph replay) -> calibrated refit of the found tracks -> adjoint.
value = clusters of the batch / step time (clusters/s).

Also reported (same JSON line): per-kernel durations from HIP events over a
second timed region (eager launches, same step) and the roofline of the
dominant kernel; tracking alone in each launch form (batched staged and
batched persistent, per-sector in a graph and eager) with equal outputs;
the grid-to-starts stages against the HBM peak; the oracle timed on the
host on one core and on all cores (cpu_baseline) with the paper's
GPU-equivalent cores; and as extras the central event, the continuous
read-out slice and the refit+adjoint throughput on 1M tracks (tracks/s).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak as published (packed FMA: 4 flops per lane and cycle);
# the float work here is unpacked and uncontracted, for which the issue
# ceiling is 256 CUs x 64 lanes x 2.4 GHz = 39.3 T operations/s (reported
# beside it, labelled)
ALU_PEAK_TFLOPS = 157.3
ALU_ISSUE_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic float operations per call, counted from the formulas
# (division and square root count as one operation each)
FLOPS_PROPAGATE = 179
FLOPS_UPDATE = 130
FLOPS_CHI2 = 20
# grid build to chain starts: read row, y, z (9 B) and write the grid
# (12 B); neighbours read y, z (8 B) and write two links (8 B); cleaning
# reads the links (8 B) and writes the clean ones (8 B); bin starts ~4 B
SEEDING_BYTES_PER_CLUSTER = 57


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--refit-tracks", type=int, default=1_000_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing")
    ap.add_argument("--no-refit-bench", action="store_true")
    ap.add_argument("--no-central-bench", action="store_true",
                    help="skip the central event (events in flight, attachment, merging)")
    ap.add_argument("--no-slice-bench", action="store_true",
                    help="skip the continuous read-out slice (100 collisions)")
    ap.add_argument("--no-attach-bench", action="store_true",
                    help="skip the track-based cluster attachment of the central event")
    ap.add_argument("--no-merge-bench", action="store_true",
                    help="skip the sector-track merging of the central event")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the "
                         "reference size for scaling the HBM byte counters) and exit")
    ap.add_argument("--seeding-probe", action="store_true",
                    help="only build the grid and find the chain starts of the 512-instance "
                         "set three times (eager launches; the workload of the HBM byte "
                         "counters of those stages) and exit")
    ap.add_argument("--tracking-probe", choices=("central", "batched", "slice"),
                    help="only track the central event, the 512-instance set or the "
                         "continuous read-out slice three times (eager staged launches; the "
                         "workload of the counter profiles of the tracking kernels) and exit")
    ap.add_argument("--step-probe", nargs="?", const="batched", choices=("batched", "central"),
                    help="only run the step on the batched set (default) or the central event "
                         "(tracking with eager staged launches, refit and adjoint of the found "
                         "tracks) --steps times after one warm-up, with the automatic launch "
                         "shapes, and exit (the workload of the profiles of the step's kernels)")
    ap.add_argument("--refit-probe", action="store_true",
                    help="only run the refit and adjoint of the 1M-track refit set three times "
                         "and exit")
    ap.add_argument("--probe-mode", default="staged", choices=("staged", "persistent"),
                    help="launch form of --tracking-probe")
    ap.add_argument("--batches-in-flight", type=int, default=3,
                    help="batched set: independent batches (same recipe, seeds 40040000 + k) "
                         "whose steps overlap in the timed region, each on its own stream with "
                         "its own buffers and context; step i runs on batch i mod depth")
    ap.add_argument("--inflight", default="3",
                    help="central event: events in flight in its timed step loop (each on its own stream "
                         "with its own buffers; with four hardware queues per process more "
                         "than three streams serialise), or 'auto' (times 1-3 first and "
                         "takes the fastest; after those trials the timed region has run "
                         "2.5x slower in most runs, so a fixed depth is the default)")
    ap.add_argument("--occupancy", default="auto",
                    help="clusters per grid bin, or 'auto' (autotuned per workload before "
                         "the timed region; the tracks do not depend on it)")
    return ap.parse_args()


def pick_layout(args, api, ctx, e, stream, mode="staged"):
    """Autotune (or set) the bin occupancy of an event; returns the record
    for the JSON line."""
    if args.occupancy == "auto":
        best, times = api.autotune(ctx, e, mode=mode, stream=stream)
        tried = ", ".join(f"{k}: {v:.3f} ms" for k, v in times.items())
        log(f"[bench] autotuned occupancy {best} ({tried})")
        return {"occupancy": best, "tried_ms": {str(k): round(v, 4) for k, v in times.items()}}
    api.relayout(e, float(args.occupancy))
    return {"occupancy": float(args.occupancy)}


def pick_shapes(args, api, ctx, e, stream, modes):
    """Tune the launch shapes of the context for each tracking form (the
    tracks are checked equal for every shape tried); returns the record for
    the JSON line.  The staged form's shapes last: they are the ones in
    force for the timed step."""
    rec = {}
    if args.occupancy != "auto":
        return rec
    for mode in modes:
        shapes, times = api.autotune_shapes(ctx, e, mode=mode, stream=stream)
        tried = ", ".join(f"{f}={v}: {ms:.3f} ms" for (f, v), ms in times.items())
        log(f"[bench] launch shapes ({mode}): {tried}")
        rec[mode] = {"tried_ms": {f"{f}={v}": round(ms, 4) for (f, v), ms in times.items()}}
    rec["chosen"] = api.get_tuning(ctx)
    return rec


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library "
              "runs on a single MI355X and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1905_05515_amd import api

    if (args.copy_probe or args.seeding_probe or args.tracking_probe or args.step_probe or
            args.refit_probe):
        assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.refit_probe:
        rs = synth.make_config5()
        prm = synth.default_params()
        dev = "cuda"
        h = api.TrackHits(torch.as_tensor(rs.trk_off).to(dev), torch.as_tensor(rs.row).to(dev),
                          torch.as_tensor(rs.y).to(dev), torch.as_tensor(rs.z).to(dev))
        rx = torch.as_tensor(rs.row_x).to(dev)
        th = torch.as_tensor(rs.theta_eval).to(dev)
        g = torch.ones(rs.n_tracks, dtype=torch.float32, device=dev)
        ctx = api.Context(0)
        out, adj = None, {}
        for _ in range(3):
            out = api.refit(ctx, h, rx, prm, th, out=out)
            api.refit_adjoint(ctx, h, rx, prm, th, out, g, out=adj)
        torch.cuda.synchronize()
        log(f"[bench] refit and adjoint of {rs.n_tracks} tracks ({rs.n_hits} hits), 3 times")
        return
    if args.step_probe:
        ev = synth.make_config4() if args.step_probe == "batched" else synth.make_config2()
        prm = synth.default_params()
        occ = 0.125 if args.occupancy == "auto" else float(args.occupancy)
        e = api.make_event(ev.row, ev.y, ev.z, ev.sector_offsets, ev.sector_range, ev.row_x,
                           prm, occupancy=occ, sector_side=ev.sector_side)
        ctx = api.Context(0)
        th = torch.as_tensor(synth_theta()).cuda()
        g = torch.ones(e.track_capacity, dtype=torch.float32, device="cuda")
        hits = api.found_track_hits(e, copies=True)
        fwd, adj = None, {}
        for _ in range(args.steps + 1):
            api.track_batch(ctx, e, mode="staged", use_graph=False)
            fwd = api.refit(ctx, hits, e.t["row_x"], prm, th, out=fwd)
            api.refit_adjoint(ctx, hits, e.t["row_x"], prm, th, fwd, g, out=adj)
        torch.cuda.synchronize()
        log(f"[bench] {args.step_probe} step of {ev.n_clusters} clusters, occupancy {occ}, "
            f"{args.steps + 1} times")
        return
    if args.tracking_probe:
        make = {"central": synth.make_config2, "batched": synth.make_config4,
                "slice": synth.make_config3}[args.tracking_probe]
        ev = make()
        occ = 0.125 if args.occupancy == "auto" else float(args.occupancy)
        e = api.make_event(ev.row, ev.y, ev.z, ev.sector_offsets, ev.sector_range, ev.row_x,
                           synth.default_params(), occupancy=occ, sector_side=ev.sector_side)
        ctx = api.Context(0)
        for _ in range(3):
            api.track_batch(ctx, e, mode=args.probe_mode, use_graph=False)
        torch.cuda.synchronize()
        log(f"[bench] tracked {ev.n_clusters} clusters ({args.tracking_probe}, "
            f"{args.probe_mode}), occupancy {occ}, 3 times")
        return
    if args.copy_probe:
        n = 1 << 28
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {4 * n} bytes 3 times")
        return
    if args.seeding_probe:
        ev = synth.make_config4()
        occ = 0.125 if args.occupancy == "auto" else float(args.occupancy)
        e = api.make_event(ev.row, ev.y, ev.z, ev.sector_offsets, ev.sector_range, ev.row_x,
                           synth.default_params(), occupancy=occ, sector_side=ev.sector_side)
        ctx = api.Context(0)
        for _ in range(3):
            api.build_grid(ctx, e)
            api.find_neighbours(ctx, e)
        torch.cuda.synchronize()
        log(f"[bench] grid and starts of {ev.n_clusters} clusters, occupancy {occ}, 3 times")
        return
    dev = torch.device("cuda:0")
    prm = synth.default_params()
    t0 = time.time()
    ev = synth.make_config4()
    log(f"[bench] batched set: {ev.n_sectors} instances, {ev.n_clusters} clusters, generated "
        f"in {time.time() - t0:.1f}s")
    # the oracle first: its worker processes fork before the GPU is touched
    cpu = None if args.no_cpu else cpu_baseline(args, ev, prm)
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = api.Context(0)
    stream = torch.cuda.Stream()      # default priority; graphs need a non-default stream
    e = api.make_event(ev.row, ev.y, ev.z, ev.sector_offsets, ev.sector_range, ev.row_x, prm,
                       sector_side=ev.sector_side)
    tuned = pick_layout(args, api, ctx, e, stream)
    tuned["launch_shapes"] = pick_shapes(args, api, ctx, e, stream, ("persistent", "staged"))
    th = torch.as_tensor(synth_theta()).to(dev)
    gchi2 = torch.ones(e.track_capacity, dtype=torch.float32, device=dev)
    hits = api.found_track_hits(e, copies=True)
    S = dict(fwd=None, adj={})

    def step(mode="staged", graph=True):
        """One pass of the hot path over the batch: tracking of every
        instance (one launch sequence over all of them, HIP graph), then the
        calibrated refit of the found tracks and its adjoint."""
        with torch.cuda.stream(stream):
            api.track_batch(ctx, e, mode=mode, use_graph=graph, stream=stream)
            S["fwd"] = api.refit(ctx, hits, e.t["row_x"], prm, th, stream=stream, out=S["fwd"])
            api.refit_adjoint(ctx, hits, e.t["row_x"], prm, th, S["fwd"], gchi2, stream=stream,
                              out=S["adj"])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # one batch at a time: K steps between two events on the step's stream
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(args.steps):
        step()
    b.record(stream)
    torch.cuda.synchronize()
    ms_one = a.elapsed_time(b) / args.steps

    # Batches in flight, as an online farm keeps several time frames in
    # flight: lane k owns batch k (the same recipe with its own seed), its
    # buffers, a context (whose cached graph is that batch's, with the tuned
    # layout and shapes) and a stream; step i runs on lane i % depth, a
    # lane's steps follow each other on its stream and the lanes overlap on
    # the GPU.  Every step does the whole work of its batch.
    depth = max(1, args.batches_in_flight)
    lanes = [dict(ctx=ctx, e=e, ev=ev, stream=stream, hits=hits, S=S)]
    for k in range(1, depth):
        ev_k = synth.make_config4(seed=synth.CONFIG_SEEDS[4] + k)
        e_k = api.make_event(ev_k.row, ev_k.y, ev_k.z, ev_k.sector_offsets, ev_k.sector_range,
                             ev_k.row_x, prm, occupancy=tuned["occupancy"],
                             sector_side=ev_k.sector_side)
        ctx_k = api.Context(0)
        api.set_tuning(ctx_k, **api.get_tuning(ctx))
        lanes.append(dict(ctx=ctx_k, e=e_k, ev=ev_k, stream=torch.cuda.Stream(),
                          hits=api.found_track_hits(e_k, copies=True),
                          S=dict(fwd=None, adj={})))

    def lane_step(L):
        with torch.cuda.stream(L["stream"]):
            api.track_batch(L["ctx"], L["e"], mode="staged", use_graph=True, stream=L["stream"])
            L["S"]["fwd"] = api.refit(L["ctx"], L["hits"], L["e"].t["row_x"], prm, th,
                                      stream=L["stream"], out=L["S"]["fwd"])
            api.refit_adjoint(L["ctx"], L["hits"], L["e"].t["row_x"], prm, th, L["S"]["fwd"],
                              gchi2, stream=L["stream"], out=L["S"]["adj"])

    for L in lanes[1:]:
        for _ in range(max(args.warmup, 1)):
            lane_step(L)
    torch.cuda.synchronize()
    # timed region: K steps over the lanes, between two events that bracket
    # all of them, device-synchronised on both sides
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    ru0 = host_cpu_seconds()
    w0 = time.perf_counter()
    a.record(stream)
    for L in lanes[1:]:
        L["stream"].wait_event(a)
    clusters = 0
    for i in range(args.steps):
        L = lanes[i % depth]
        lane_step(L)
        clusters += L["ev"].n_clusters
    for L in lanes[1:]:
        done = torch.cuda.Event()
        done.record(L["stream"])
        stream.wait_event(done)
    b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    host_cpu = host_cpu_seconds() - ru0
    gpu_ms = a.elapsed_time(b)
    ms_per_step = gpu_ms / args.steps
    value = clusters / (gpu_ms * 1e-3)
    st = api.get_status(e, stream)
    log(f"[bench] step {ms_per_step:.3f} ms with {depth} batches in flight ({value:.3e} "
        f"clusters/s; wall {1e3 * wall / args.steps:.3f} ms, host CPU "
        f"{1e3 * host_cpu / args.steps:.3f} ms per step; one at a time {ms_one:.3f} ms), "
        f"tracks {st['n_tracks']}")

    # the same step with eager launches and HIP events around every kernel
    with torch.cuda.stream(stream):
        step(graph=False)
        torch.cuda.synchronize()
        api.timing_enable(ctx, True)
        for _ in range(args.steps):
            step(graph=False)
        torch.cuda.synchronize()
        kt = api.timing_report(ctx)
        api.timing_enable(ctx, False)
    kernels = {k: {"launches": n, "avg_ms": ms / n, "ms_per_step": ms / args.steps}
               for k, (n, ms) in kt.items()}
    eager_ms = sum(v["ms_per_step"] for v in kernels.values())
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        log(f"[bench]   {k:28s} {v['avg_ms'] * 1e3:9.1f} us x {v['launches'] // args.steps}")
    n_cl = ev.n_clusters
    n_hits_trk = int(st["n_track_hits"])
    roof = roofline(dom, kernels[dom]["avg_ms"], st, n_cl, n_hits_trk)
    roof["traffic"] = counter_traffic(dom.split("<")[0], "batched_set")
    roof["source_sha256"] = source_hash(dom.split("<")[0])

    forms = forms_bench(args, api, ctx, e, ev, stream)
    extra = {"launch_forms": forms}
    if cpu is not None:
        # GPU time per pass over the oracle's batch: the in-flight time per
        # step scaled to that batch's clusters
        cpu["gpu_equivalent_cores"] = gpu_equivalent_cores(
            cpu, forms, gpu_ms * n_cl / clusters, host_cpu, args.steps)
    extra["grid_to_starts"] = seeding_roofline(api, ctx, e, stream, max(2, args.steps // 4),
                                               n_cl, "batched_set")
    log(f"[bench] grid..starts {extra['grid_to_starts']['ms'] * 1e3:.1f} us, "
        f"{extra['grid_to_starts']['frac'] * 100:.1f}% of HBM peak at "
        f"{SEEDING_BYTES_PER_CLUSTER} B/cluster")
    if not args.no_central_bench:
        extra["central_event"] = central_bench(args, api, synth, prm, dev, tuned,
                                               [L["stream"] for L in lanes])
    if not args.no_slice_bench:
        extra["continuous_readout"] = slice_bench(args, api, synth, ctx, stream, prm)
    if not args.no_refit_bench:
        extra["refit_adjoint"] = refit_bench(args, api, synth, ctx, stream, prm, dev)

    line = {
        "metric": ("TPC clusters/s tracked on 1 MI355X (batched vs per-sector); "
                   "refit+adjoint tracks/s"),
        "value": value,
        "unit": "clusters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "batched uneven set: 512 independent single-sector instances, half "
                        "pp-like (20-200 tracks), half Pb-Pb-like (50-800 tracks), log-uniform, "
                        "shuffled, 5% noise, float32 SoA clusters (seed 40040000); step = grid, "
                        "neighbours, cleaning, starts, tracklets, selection of every instance "
                        "(one launch sequence over all instances, HIP graph) + calibrated refit "
                        "and adjoint of the found tracks; batches of the same recipe (seeds "
                        "40040000 + k) in flight on their own streams",
            "clusters": n_cl,
            "batches_in_flight": depth,
            "clusters_per_batch": [L["ev"].n_clusters for L in lanes],
            "ms_per_step_one_at_a_time": ms_one,
            "clusters_per_s_one_at_a_time": n_cl / (ms_one * 1e-3),
            "instances": ev.n_sectors,
            "tracks_found": int(st["n_tracks"]),
            "track_hits": n_hits_trk,
            "launch_form": "batched: staged stages over all instances, HIP graph",
            "wall_ms_per_step": 1e3 * wall / args.steps,
            "host_cpu_ms_per_step": 1e3 * host_cpu / args.steps,
            "grid_layout": tuned,
            "parallelism": "single GPU",
        },
        "roofline": roof,
        "kernels": {k: {"avg_us": round(v["avg_ms"] * 1e3, 2),
                        "launches_per_step": v["launches"] // args.steps}
                    for k, v in kernels.items()},
        "eager_kernel_ms_per_step": eager_ms,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line), flush=True)


def host_cpu_seconds():
    """User + system CPU time of this process and its finished children."""
    import resource
    a = resource.getrusage(resource.RUSAGE_SELF)
    return a.ru_utime + a.ru_stime


def forms_bench(args, api, ctx, e, ev, stream):
    """Tracking alone (grid to selection) of the batch in each launch form:
    batched staged (one launch per stage over all instances) and batched
    persistent (one work-queue launch), both HIP graphs, against the
    per-sector form (one launch sequence per instance) captured in a graph
    and eager.  Outputs are checked equal."""
    import torch
    ref = None
    res = {}
    steps = max(2, args.steps // 4)
    forms = (("staged", True), ("persistent", True), ("per_sector", True), ("per_sector", False))
    for mode, graph in forms:
        name = f"{mode}_{'graph' if graph else 'eager'}"
        n = steps if mode != "per_sector" or graph else 2
        with torch.cuda.stream(stream):
            api.track_batch(ctx, e, mode=mode, use_graph=graph, stream=stream)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            ru0 = host_cpu_seconds()
            a.record(stream)
            for _ in range(n):
                api.track_batch(ctx, e, mode=mode, use_graph=graph, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            host = (host_cpu_seconds() - ru0) / n
        ms = a.elapsed_time(b) / n
        r = api.results(e, stream)
        key = (r["trk_off"].tobytes(), r["trk_hits"].tobytes(), r["t_par"].tobytes())
        ref = key if ref is None else ref
        res[name] = {"ms": ms, "clusters_per_s": ev.n_clusters / (ms * 1e-3),
                     "host_cpu_ms": 1e3 * host, "equal_output": bool(key == ref),
                     "tracks": int(r["status"]["n_tracks"])}
        log(f"[bench]   {name:18s} {ms:8.3f} ms  {ev.n_clusters / (ms * 1e-3):.3e} clusters/s "
            f"equal={key == ref}")
    # per-kernel times of the staged form (eager launches, HIP events)
    with torch.cuda.stream(stream):
        api.timing_enable(ctx, True)
        for _ in range(steps):
            api.track_batch(ctx, e, mode="staged", use_graph=False, stream=stream)
        torch.cuda.synchronize()
        kt = api.timing_report(ctx)
        api.timing_enable(ctx, False)
    res["staged_kernels_us"] = {k: round(ms / steps * 1e3, 1) for k, (n, ms) in
                                sorted(kt.items(), key=lambda kv: -kv[1][1])}
    return res


def gpu_equivalent_cores(cpu, forms, ms_step, host_cpu_s, steps):
    """The paper's figure of merit: CPU cores one GPU replaces, counted as
    (oracle time on one core - host CPU time the GPU run consumed) / GPU
    wall time, for the whole step and for tracking alone."""
    t1 = cpu["seconds_one_core"]
    whole = (t1["tracking"] + t1["refit"] + t1["adjoint"] - host_cpu_s / steps) / (ms_step * 1e-3)
    tf = forms["staged_graph"]
    trk = (t1["tracking"] - tf["host_cpu_ms"] * 1e-3) / (tf["ms"] * 1e-3)
    return {"whole_step": whole, "tracking": trk,
            "method": "(oracle seconds on one core - host CPU seconds of the GPU run, from "
                      "getrusage) / GPU seconds, per pass over the batch"}


def central_bench(args, api, synth, prm, dev, tuned_batch, streams=()):
    """The central Pb-Pb-like event (36 sectors, ~1.3M clusters): the step
    with events in flight, per-kernel times, cluster attachment and
    sector-track merging of its tracks.  `streams`: idle streams to give the
    lanes (the batched set's, which sit on distinct hardware queues; new
    streams beyond the process's four queues can share one, and lanes that
    share a queue run one after the other)."""
    import torch
    t0 = time.time()
    ev = synth.make_config2()
    log(f"[bench] central event: {ev.n_clusters} clusters, generated in {time.time() - t0:.1f}s")
    ctx = api.Context(0)
    streams = list(streams)
    stream = streams[0] if streams else torch.cuda.Stream()
    e = api.make_event(ev.row, ev.y, ev.z, ev.sector_offsets, ev.sector_range, ev.row_x, prm,
                       sector_side=ev.sector_side)
    tuned = pick_layout(args, api, ctx, e, stream)
    tuned["launch_shapes"] = pick_shapes(args, api, ctx, e, stream, ("persistent", "staged"))
    th = torch.as_tensor(synth_theta()).to(dev)
    gchi2 = torch.ones(e.track_capacity, dtype=torch.float32, device=dev)
    # Events in flight: lane k owns an event's buffers, a context (whose
    # cached graph is that event's) and a stream; step i runs on lane
    # i % depth.  A lane's steps follow each other on its stream, so no
    # buffer is shared between steps in flight; lanes overlap on the GPU (one
    # central event keeps only a fraction of the chip busy).
    lanes = [dict(ctx=ctx, e=e, stream=stream, hits=api.found_track_hits(e, copies=True),
                  fwd=None, adj={})]

    def lane(k):
        while len(lanes) <= k:
            e_k = api.make_event(ev.row, ev.y, ev.z, ev.sector_offsets, ev.sector_range,
                                 ev.row_x, prm, sector_side=ev.sector_side)
            api.relayout(e_k, tuned["occupancy"])
            s_k = streams[len(lanes)] if len(lanes) < len(streams) else torch.cuda.Stream()
            lanes.append(dict(ctx=api.Context(0), e=e_k, stream=s_k,
                              hits=api.found_track_hits(e_k, copies=True), fwd=None, adj={}))
        return lanes[k]

    def step(L, graph=True):
        with torch.cuda.stream(L["stream"]):
            api.track_batch(L["ctx"], L["e"], mode="staged", use_graph=graph,
                            stream=L["stream"])
            L["fwd"] = api.refit(L["ctx"], L["hits"], L["e"].t["row_x"], prm, th,
                                 stream=L["stream"], out=L["fwd"])
            api.refit_adjoint(L["ctx"], L["hits"], L["e"].t["row_x"], prm, th, L["fwd"], gchi2,
                              stream=L["stream"], out=L["adj"])

    def run(depth, n_steps):
        """n_steps steps over `depth` lanes; GPU ms between two events that
        bracket all of them, and host wall seconds."""
        ls = [lane(k) for k in range(depth)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(ls[0]["stream"])
        for L in ls[1:]:
            L["stream"].wait_event(a)
        for i in range(n_steps):
            step(ls[i % depth])
        for L in ls[1:]:
            done = torch.cuda.Event()
            done.record(L["stream"])
            ls[0]["stream"].wait_event(done)
        b.record(ls[0]["stream"])
        torch.cuda.synchronize()
        return a.elapsed_time(b), time.perf_counter() - t0

    for _ in range(args.warmup):
        step(lanes[0])
    torch.cuda.synchronize()
    # one event at a time: the latency of a step
    lat_ms = run(1, args.steps)[0] / args.steps
    if args.inflight == "auto":
        tried = {}
        for d in (1, 2, 3):
            run(d, 2 * d)                               # warm-up (graph capture per lane)
            tried[d] = run(d, max(args.steps // 2, 2 * d))[0] / max(args.steps // 2, 2 * d)
        depth = min(tried, key=tried.get)
        log(f"[bench] events in flight: {depth} "
            f"({', '.join(f'{d}: {v:.3f} ms' for d, v in tried.items())})")
    else:
        depth = int(args.inflight)
        tried = None
        run(depth, 2 * depth)
    # timed region 1: graph replay of the tracking + refit + adjoint
    gpu_ms, wall = run(depth, args.steps)
    # every lane produced the same tracks
    same = True
    ref = None
    for L in lanes[:depth]:
        r = api.results(L["e"], L["stream"])
        key = (r["trk_off"].tobytes(), r["trk_hits"].tobytes())
        ref = key if ref is None else ref
        same &= key == ref
    st = api.get_status(e, stream)
    ms_per_step = gpu_ms / args.steps
    log(f"[bench] step {ms_per_step:.3f} ms with {depth} in flight (wall "
        f"{1e3 * wall / args.steps:.3f} ms; one at a time {lat_ms:.3f} ms), "
        f"tracks {st['n_tracks']}, starts {st['n_starts']}, lanes equal {same}")

    def step_eager():
        step(lanes[0], graph=False)

    # timed region 2: the same step with eager launches and per-kernel events
    with torch.cuda.stream(stream):
        step_eager()
        torch.cuda.synchronize()
        api.timing_enable(ctx, True)
        for _ in range(args.steps):
            step_eager()
        torch.cuda.synchronize()
        kt = api.timing_report(ctx)
        api.timing_enable(ctx, False)
    kernels = {k: {"launches": n, "avg_ms": ms / n, "ms_per_step": ms / args.steps}
               for k, (n, ms) in kt.items()}
    eager_ms = sum(v["ms_per_step"] for v in kernels.values())
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        log(f"[bench]   {k:28s} {v['avg_ms'] * 1e3:9.1f} us x {v['launches'] // args.steps}")

    n_cl = ev.n_clusters
    n_hits_trk = int(st["n_track_hits"])
    roof = roofline(dom, kernels[dom]["avg_ms"], st, n_cl, n_hits_trk)
    roof["traffic"] = counter_traffic(dom.split("<")[0], "central_event")
    roof["source_sha256"] = source_hash(dom.split("<")[0])
    res = {"workload": "central Pb-Pb-like event: 36 sectors, 8000 primaries + 10% secondaries "
                       "+ 5% noise (seed 2002); step = tracking (graph) + refit + adjoint",
           "clusters": n_cl, "tracks_found": int(st["n_tracks"]),
           "ms_per_step": ms_per_step, "clusters_per_s": n_cl / (ms_per_step * 1e-3),
           "events_in_flight": depth,
           "events_in_flight_tried_ms": ({str(k): round(v, 4) for k, v in tried.items()}
                                         if tried else None),
           "ms_per_step_one_at_a_time": lat_ms, "lanes_equal_output": bool(same),
           "grid_layout": tuned, "roofline": roof,
           "kernels_us": {k: round(v["avg_ms"] * 1e3, 2) for k, v in kernels.items()},
           "eager_kernel_ms_per_step": eager_ms}
    if not args.no_attach_bench:
        res["cluster_attachment"] = attach_bench(args, api, ctx, e, ev, stream)
    if not args.no_merge_bench:
        res["sector_merging"] = merge_bench(args, api, ctx, e, ev, stream)
    res["compression"] = compress_bench(args, api, ctx, e, ev, stream)
    return res


def compress_bench(args, api, ctx, e, ev, stream):
    """Cluster compression of the tracked central event (integer format,
    residuals to tracks, rANS): time per event, per-kernel times, blob size
    against the float32 SoA input (row, y, z, charge: 13 bytes per
    cluster)."""
    import torch
    steps = max(args.steps // 2, 2)
    charge = torch.as_tensor(ev.charge).cuda()
    state = {}
    with torch.cuda.stream(stream):
        api.track_batch(ctx, e, mode="staged", use_graph=False, stream=stream)
        api.compress_clusters(ctx, e, charge, stream=stream, state=state)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            blob, size = api.compress_clusters(ctx, e, charge, stream=stream, state=state)
        b.record(stream)
        torch.cuda.synchronize()
        api.timing_enable(ctx, True)
        api.compress_clusters(ctx, e, charge, stream=stream, state=state)
        torch.cuda.synchronize()
        kt = api.timing_report(ctx)
        api.timing_enable(ctx, False)
    ms = a.elapsed_time(b) / steps
    n = int(size.item())
    res = {"workload": "clusters of the tracked central event: y, z at 2^-5 cm, charge with 5 "
                       "significant bits, residuals to tracks, rANS in 4096-symbol chunks",
           "ms": ms, "clusters_per_s": ev.n_clusters / (ms * 1e-3), "bytes": n,
           "bytes_per_cluster": n / ev.n_clusters,
           "factor_vs_float_soa": 13.0 * ev.n_clusters / n,
           "kernels_us": {k: round(ms_ / c * 1e3, 1) for k, (c, ms_) in kt.items()}}
    log(f"[bench] compression {ms:.3f} ms: {n} bytes, {n / ev.n_clusters:.3f} B/cluster, "
        f"factor {res['factor_vs_float_soa']:.2f} against 13 B/cluster")
    return res


def roofline(name, avg_ms, st, n_cl, n_trk_hits):
    """Algorithmic traffic (bytes) or operations per launch of a kernel."""
    sec = avg_ms * 1e-3
    base = name.split("<")[0]
    bytes_per_cluster = {
        # row bucket counts: row (1 B)
        "k_grid_rows": 1,
        # row partition: read row, y, z (9 B), write id, y, z (12 B)
        "k_grid_rows_scatter": 21,
        # per-row bin sort: read y, z (8 B), write slot and bin (8 B)
        "k_grid_bins": 16,
        # final place: read slot, bin, id, y, z (20 B), write y, z, id, gsr (16 B)
        "k_grid_place": 36,
        # reads y, z, gsr (12 B) writes up0, down0 (8 B)
        "k_neighbours": 20,
        # reads up0, down0, idg (12 B), writes up, down (8 B)
        "k_clean": 20,
    }
    if base in bytes_per_cluster:
        b = bytes_per_cluster[base] * n_cl
        gbs = b / sec / 1e9
        return {"kernel": name, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                "units_per_launch": n_cl, "unit_name": "cluster",
                "algorithmic_bytes_per_unit": bytes_per_cluster[base]}
    if base == "k_tracklets":
        fl = FLOPS_PROPAGATE * st["n_propagations"] + FLOPS_UPDATE * st["n_updates"]
        tf = fl / sec / 1e12
        return {"kernel": name, "bound": "alu", "achieved": tf, "peak": ALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": tf / ALU_PEAK_TFLOPS, "traffic": None,
                "issue_ceiling_tops": ALU_ISSUE_PEAK_TOPS,
                "frac_of_issue_ceiling": tf / ALU_ISSUE_PEAK_TOPS,
                "flops_per_launch": fl, "propagations": st["n_propagations"],
                "updates": st["n_updates"], "candidates": st["n_candidates"]}
    if base in ("k_refit_fwd", "k_refit_adj"):
        per_hit = 4 + 9 + (80 if name == "k_refit_fwd" else 88)
        b = per_hit * n_trk_hits
        gbs = b / sec / 1e9
        return {"kernel": name, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                "units_per_launch": n_trk_hits, "unit_name": "track hit",
                "algorithmic_bytes_per_unit": per_hit}
    return {"kernel": name, "bound": "unknown", "achieved": None, "peak": None, "unit": None,
            "frac": None, "traffic": None}


# sources a kernel is built from (a counter summary applies while they are
# unchanged)
KERNEL_SOURCES = {
    "k_tracklets": ["tracklets.hip", "tracklet_dev.hpp", "tpc_internal.hpp"],
    "k_refit_fwd": ["refit.hip", "tpc_internal.hpp"],
    "k_refit_adj": ["refit.hip", "tpc_internal.hpp"],
    # every kernel that tpc_build_grid and tpc_find_neighbours launch
    "grid_to_starts": ["grid.hip", "grid_dev.hpp", "neighbours.hip", "seed_dev.hpp",
                       "block_dev.hpp", "util.hip", "tpc_internal.hpp"],
}


def source_hash(kernel=None):
    """SHA-256 over the sources of `kernel` (all kernel sources when it has
    no entry) and the header."""
    import glob
    import hashlib
    csrc = os.path.join(ROOT, "paper_1905_05515_amd", "csrc")
    if kernel in KERNEL_SOURCES:
        files = [os.path.join(csrc, f) for f in KERNEL_SOURCES[kernel]]
    else:
        files = sorted(glob.glob(os.path.join(csrc, "*.hip")) +
                       glob.glob(os.path.join(csrc, "*.hpp")))
    h = hashlib.sha256()
    for f in files + [os.path.join(ROOT, "include", "tpc.h")]:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE and WRITE_SIZE, each scaled by the
    factor a plain copy of known size reads), or None when there is none or
    the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_hash(kernel):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def attach_bench(args, api, ctx, e, ev, stream):
    """Track-based cluster attachment (1.5 cm tubes) of the central event's
    found tracks: time per event, per-kernel times, the tube kernel against
    the ALU ceiling (transport operations counted from the tracks' row
    spans), and the attachment figures with truth-label fake rates."""
    import numpy as np
    import torch
    steps = max(args.steps, 2)
    with torch.cuda.stream(stream):
        api.track_batch(ctx, e, mode="staged", use_graph=False, stream=stream)
        api.attach_clusters(ctx, e, stream=stream)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            track, state = api.attach_clusters(ctx, e, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        api.timing_enable(ctx, True)
        for _ in range(steps):
            api.attach_clusters(ctx, e, stream=stream)
        torch.cuda.synchronize()
        kt = api.timing_report(ctx)
        api.timing_enable(ctx, False)
    per = {k: ms_ / n for k, (n, ms_) in kt.items()}
    r = api.results(e, stream)
    track = track.cpu().numpy()
    state = state.cpu().numpy()
    off, hits, tt = r["trk_off"], r["trk_hits"], r["trk_tracklet"]
    nt = len(off) - 1
    last_row = ev.row[hits[off[1:] - 1]].astype(np.int64) if nt else np.zeros(0, np.int64)
    rows = int(np.sum(np.maximum(last_row - r["t_rin"][tt], 0))) if nt else 0
    tube_ms = per.get("k_attach_tube", ms)
    fl = FLOPS_PROPAGATE * rows
    maj = np.array([np.bincount(np.maximum(ev.label[hits[off[k]:off[k + 1]]], 0)).argmax()
                    for k in range(nt)], np.int64)
    att, adj = (state & 1) != 0, (state & 2) != 0
    fake = lambda m: float(np.mean(ev.label[m] != maj[track[m]])) if m.any() else None
    res = {"workload": "tubes of 1.5 cm around the found tracks of the central event, "
                       "protection above 0.05 GeV",
           "ms": ms, "clusters_per_s": ev.n_clusters / (ms * 1e-3), "tracks": nt,
           "kernels_us": {k: round(v * 1e3, 1) for k, v in per.items()},
           "roofline_tube": {"kernel": "k_attach_tube", "bound": "alu",
                             "achieved": fl / (tube_ms * 1e-3) / 1e12, "peak": ALU_PEAK_TFLOPS,
                             "unit": "TFLOP/s",
                             "frac": fl / (tube_ms * 1e-3) / 1e12 / ALU_PEAK_TFLOPS,
                             "flops_per_launch": fl, "row_transports": rows},
           "attached": int(att.sum()), "adjacent": int(adj.sum()),
           "protected": int(((state & 4) != 0).sum()), "removed": int(((state & 8) != 0).sum()),
           "fake_attached": fake(att), "fake_adjacent": fake(adj)}
    log(f"[bench] attachment {ms:.3f} ms ({nt} tracks): attached {res['attached']} "
        f"(fake {res['fake_attached']}), adjacent {res['adjacent']} (fake "
        f"{res['fake_adjacent']}), removed {res['removed']}")
    return res


# float operations of one candidate pair in k_merge_best: the transport's
# parameter part (dx, k, sin, two cosines, chord slope, chord, series of the
# arc, y and z: 33) and the windowed distance (5 x 4)
FLOPS_MERGE_PAIR = 53


def merge_bench(args, api, ctx, e, ev, stream):
    """Sector-track merging of the central event's found tracks: time per
    event, per-kernel times, the pair kernel against the ALU ceiling
    (candidate pairs counted from the tracks' sectors), links and their
    truth-label purity."""
    import numpy as np
    import torch
    steps = max(args.steps, 2)
    with torch.cuda.stream(stream):
        api.track_batch(ctx, e, mode="staged", use_graph=False, stream=stream)
        api.merge_sector_tracks(ctx, e, stream=stream)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            up, dn, grp = api.merge_sector_tracks(ctx, e, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        api.timing_enable(ctx, True)
        for _ in range(steps):
            api.merge_sector_tracks(ctx, e, stream=stream)
        torch.cuda.synchronize()
        kt = api.timing_report(ctx)
        api.timing_enable(ctx, False)
    per = {k: ms_ / n for k, (n, ms_) in kt.items()}
    r = api.results(e, stream)
    off, hits = r["trk_off"], r["trk_hits"]
    nt = len(off) - 1
    links = (up, dn, grp)             # device tensors for the full-track fit
    up = up[:nt].cpu().numpy()
    grp = grp[:nt].cpu().numpy()
    sec = np.searchsorted(ev.sector_offsets, hits[off[:-1]], side="right") - 1
    # candidate pairs the pair kernel evaluates: the tracks of each neighbour
    # sector whose tan(lambda) lies within the window of the track's
    tl = r["t_par"][r["trk_tracklet"], 3].astype(np.float32)
    iw3 = np.float32(1.0) / np.float32(api.MERGE_WINDOWS[3])
    side, idx = sec // 18, sec % 18
    srt = {s_: np.sort(tl[sec == s_]) for s_ in range(len(ev.sector_offsets) - 1)}
    pairs = 0
    for nb in ((side * 18 + (idx + 1) % 18), (side * 18 + (idx + 17) % 18)):
        for s_ in np.unique(nb):
            m = nb == s_
            c = srt[s_]
            lo = np.searchsorted(c, tl[m] - np.float32(1.0) / iw3, side="right")
            hi = np.searchsorted(c, tl[m] + np.float32(1.0) / iw3, side="left")
            pairs += int(np.sum(hi - lo))
    best_ms = per.get("k_merge_best", ms)
    fl = FLOPS_MERGE_PAIR * pairs
    maj = np.array([np.bincount(np.maximum(ev.label[hits[off[k]:off[k + 1]]], 0)).argmax()
                    for k in range(nt)], np.int64)
    k = np.nonzero(up >= 0)[0]
    res = {"workload": "sector-track merging of the found tracks of the central event "
                       "(18 sectors per side, windows 3 cm, 2 cm, 0.1, 0.02, 2 c/GeV)",
           "ms": ms, "tracks_per_s": nt / (ms * 1e-3), "tracks": nt,
           "kernels_us": {k_: round(v * 1e3, 1) for k_, v in per.items()},
           "roofline_pairs": {"kernel": "k_merge_best", "bound": "alu",
                              "achieved": fl / (best_ms * 1e-3) / 1e12,
                              "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": fl / (best_ms * 1e-3) / 1e12 / ALU_PEAK_TFLOPS,
                              "flops_per_launch": fl,
                              "candidate_pairs_in_tan_lambda_windows": pairs},
           "links": int(len(k)), "groups": int(len(np.unique(grp))),
           "link_purity": float(np.mean(maj[k] == maj[up[k]])) if len(k) else None}
    log(f"[bench] merging {ms:.3f} ms ({nt} tracks, {pairs} pairs): {res['links']} links, "
        f"purity {res['link_purity']}, {res['groups']} groups")
    res["full_track_fit"] = fullfit_bench(api, ctx, e, stream, steps, nt, links)
    return res


def fullfit_bench(api, ctx, e, stream, steps, n_tracks, links):
    """Full-track fit of the merged tracks (three passes, out-in-out):
    time per call, per-kernel time, merged tracks and their chi2 / ndf."""
    import torch
    with torch.cuda.stream(stream):
        api.fit_merged_tracks(ctx, e, links, stream=stream)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            f = api.fit_merged_tracks(ctx, e, links, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    nt = min(n_tracks, e.track_capacity)
    st = f["status"][:nt]
    ok = st == 0
    nh = f["n_hits"][:nt][ok].double()
    chi2 = f["chi2"][:nt][ok].double()
    res = {"ms": ms, "merged_tracks": int((st >= 0).sum()), "fitted": int(ok.sum()),
           "multi_sector": int((ok & (f["n_members"][:nt] > 1)).sum()),
           "hits_fitted": int(nh.sum()), "passes": 3,
           "chi2_per_ndf": float(chi2.sum() / (2 * nh - 5).sum()) if int(ok.sum()) else None}
    log(f"[bench]   full-track fit {ms:.3f} ms: {res['fitted']} merged tracks "
        f"({res['multi_sector']} over sectors), chi2/ndf {res['chi2_per_ndf']}")
    return res


def seeding_roofline(api, ctx, e, stream, steps, n_clusters, workload=None):
    """Grid build to chain starts alone (tpc_build_grid + tpc_find_neighbours,
    eager launches, HIP events) against the HBM peak."""
    import torch
    with torch.cuda.stream(stream):
        api.build_grid(ctx, e, stream)
        api.find_neighbours(ctx, e, stream)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            api.build_grid(ctx, e, stream)
            api.find_neighbours(ctx, e, stream)
        b.record(stream)
        torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    by = SEEDING_BYTES_PER_CLUSTER * n_clusters
    return {"bound": "hbm", "kernels": "tpc_build_grid + tpc_find_neighbours (grid, neighbours, "
                                       "cleaning, starts), eager launches",
            "achieved": by / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "ms": ms,
            "algorithmic_bytes_per_cluster": SEEDING_BYTES_PER_CLUSTER,
            "traffic": counter_traffic("grid_to_starts", workload) if workload else None}


def slice_bench(args, api, synth, ctx, stream, prm):
    """The continuous read-out slice: 100 collisions at 50 kHz, time turned
    into z with the drift velocity, loopers up to three turns."""
    import torch
    t0 = time.time()
    ev = synth.make_config3()
    log(f"[bench] continuous read-out slice: {ev.n_clusters} clusters, generated in "
        f"{time.time() - t0:.1f}s")
    e = api.make_event(ev.row, ev.y, ev.z, ev.sector_offsets, ev.sector_range, ev.row_x, prm,
                       sector_side=ev.sector_side)
    res = {"grid_layout": pick_layout(args, api, ctx, e, stream)}
    steps = max(2, args.steps // 4)
    with torch.cuda.stream(stream):
        api.track_batch(ctx, e, mode="staged", use_graph=True, stream=stream)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            api.track_batch(ctx, e, mode="staged", use_graph=True, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        api.timing_enable(ctx, True)
        api.track_batch(ctx, e, mode="staged", use_graph=False, stream=stream)
        torch.cuda.synchronize()
        kt = api.timing_report(ctx)
        api.timing_enable(ctx, False)
    st = api.get_status(e, stream)
    # before the seeding probe, which runs the grid and neighbour calls again
    # and so resets the event's track count
    res["track_t0"] = slice_t0(api, ctx, e, ev, stream, steps, int(st["n_tracks"]))
    res["track_merging"] = slice_merge(api, ctx, e, stream, steps, int(st["n_tracks"]))
    res.update({
        "workload": "100 collisions, Poisson arrivals at 50 kHz, multiplicity U(5%, 100%) of the "
                    "central event, pT >= 0.05 GeV, loopers inside the drift volume up to 3 "
                    "turns, z* = z - vd t "
                    "(seed 3003)",
        "clusters": ev.n_clusters, "ms": ms, "clusters_per_s": ev.n_clusters / (ms * 1e-3),
        "launch_form": "staged, HIP graph", "starts": int(st["n_starts"]),
        "tracks": int(st["n_tracks"]), "overflow": int(st["overflow"]),
        "kernels_us": {k: round(ms_ / n * 1e3, 1) for k, (n, ms_) in
                       sorted(kt.items(), key=lambda kv: -kv[1][1])},
        "roofline_grid_to_starts": seeding_roofline(api, ctx, e, stream, steps, ev.n_clusters),
    })
    log(f"[bench]   slice {ms:.3f} ms  {ev.n_clusters / (ms * 1e-3):.3e} clusters/s, tracks "
        f"{st['n_tracks']}; grid..starts {res['roofline_grid_to_starts']['ms'] * 1e3:.0f} us, "
        f"{res['roofline_grid_to_starts']['frac'] * 100:.1f}% of HBM peak")
    del e
    torch.cuda.empty_cache()
    return res


def slice_merge(api, ctx, e, stream, steps, n_tracks):
    """Sector-track merging of every found track of the slice (buckets
    sorted by tan(lambda), windowed candidate ranges)."""
    import torch
    with torch.cuda.stream(stream):
        api.merge_sector_tracks(ctx, e, stream=stream)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            up, dn, grp = api.merge_sector_tracks(ctx, e, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        api.timing_enable(ctx, True)
        api.merge_sector_tracks(ctx, e, stream=stream)
        torch.cuda.synchronize()
        kt = api.timing_report(ctx)
        api.timing_enable(ctx, False)
    ms = a.elapsed_time(b) / steps
    nt = min(n_tracks, e.track_capacity)
    links = int((up[:nt] >= 0).sum().item())
    res = {"ms": ms, "tracks": nt, "tracks_per_s": nt / (ms * 1e-3), "links": links,
           "kernels_us": {k: round(ms_ / n * 1e3, 1) for k, (n, ms_) in kt.items()}}
    log(f"[bench]   slice merging {ms:.3f} ms for {nt} tracks, {links} links")
    res["full_track_fit"] = fullfit_bench(api, ctx, e, stream, steps, nt, (up, dn, grp))
    return res


T0_BYTES_PER_TRACK = 4 + 4 + 4 + 20 + 4 + 13


def slice_t0(api, ctx, e, ev, stream, steps, n_tracks):
    """Interaction time of every found track of the slice: time per call and
    the resolution on primaries above 0.3 GeV/c (truth: the generating track
    of the track's first hit)."""
    import numpy as np
    import torch
    from synth.events import VD_CM_PER_US
    with torch.cuda.stream(stream):
        api.track_t0(ctx, e, VD_CM_PER_US, stream=stream)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            z0, y0, t0, ok = api.track_t0(ctx, e, VD_CM_PER_US, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        api.timing_enable(ctx, True)
        for _ in range(steps):
            api.track_t0(ctx, e, VD_CM_PER_US, stream=stream)
        torch.cuda.synchronize()
        kt = api.timing_report(ctx)
        api.timing_enable(ctx, False)
    ms = a.elapsed_time(b) / steps
    n_k, ms_k = kt.get("k_track_t0", (1, ms))
    k_ms = ms_k / max(n_k, 1)
    nt = min(n_tracks, e.track_capacity)
    off = e.t["trk_off"][:nt + 1].cpu().numpy()
    hits = e.t["trk_hits"]
    idx = np.clip(off[:-1], 0, hits.numel() - 1)
    first = hits[torch.as_tensor(idx, device=hits.device).long()]
    lab = ev.label[first.cpu().numpy()]
    t0, ok = t0[:nt].cpu().numpy(), ok[:nt].cpu().numpy().astype(bool)
    T = ev.tracks
    li = np.maximum(lab, 0)
    prim = (lab >= 0) & (T["vx"][li] == 0) & (T["vy"][li] == 0) & (np.abs(T["qpt"][li]) < 1 / 0.3)
    sel = ok & prim
    d = np.abs(t0[sel] - T["t_us"][li][sel])
    # algorithmic bytes per track: off, first hit, tracklet index, state (20),
    # innermost row; z0, y0, t0 and ok written
    gbs = T0_BYTES_PER_TRACK * nt / (k_ms * 1e-3) / 1e9
    res = {"ms": ms, "tracks_per_s": nt / (ms * 1e-3), "tracks": nt,
           "roofline": {"kernel": "k_track_t0", "bound": "hbm", "achieved": gbs,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                        "kernel_ms": k_ms, "bytes_per_track": T0_BYTES_PER_TRACK},
           "ok_fraction": float(ok.mean()) if nt else None,
           "primaries_above_0.3_GeV": int(sel.sum()),
           "abs_dt_us_median": float(np.median(d)) if len(d) else None,
           "abs_dt_us_q90": float(np.quantile(d, 0.9)) if len(d) else None}
    log(f"[bench]   slice t0 {ms * 1e3:.1f} us for {nt} tracks; primaries |dt| median "
        f"{res['abs_dt_us_median']} us, q90 {res['abs_dt_us_q90']} us")
    return res


def refit_bench(args, api, synth, ctx, stream, prm, dev):
    import torch
    t0 = time.time()
    rs = synth.make_config5(n_tracks=args.refit_tracks)
    log(f"[bench] refit set: {rs.n_tracks} tracks, {rs.n_hits} hits, generated in "
        f"{time.time() - t0:.1f}s")
    h = api.TrackHits(torch.as_tensor(rs.trk_off).to(dev), torch.as_tensor(rs.row).to(dev),
                      torch.as_tensor(rs.y).to(dev), torch.as_tensor(rs.z).to(dev))
    rx = torch.as_tensor(rs.row_x).to(dev)
    th = torch.as_tensor(rs.theta_eval).to(dev)
    g = torch.ones(rs.n_tracks, dtype=torch.float32, device=dev)
    steps = max(3, args.steps // 4)
    adj = {}
    with torch.cuda.stream(stream):
        out = api.refit(ctx, h, rx, prm, th, stream=stream)
        api.refit_adjoint(ctx, h, rx, prm, th, out, g, stream=stream, out=adj)
        torch.cuda.synchronize()
        api.timing_enable(ctx, True)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            out = api.refit(ctx, h, rx, prm, th, stream=stream, out=out)
            api.refit_adjoint(ctx, h, rx, prm, th, out, g, stream=stream, out=adj)
        b.record(stream)
        torch.cuda.synchronize()
        kt = api.timing_report(ctx)
        api.timing_enable(ctx, False)
    ms = a.elapsed_time(b) / steps
    kern = {k: round(ms_ / n * 1e3, 1) for k, (n, ms_) in kt.items()}
    nh = rs.n_hits
    fwd_ms = kt["k_refit_fwd"][1] / kt["k_refit_fwd"][0]
    adj_ms = kt["k_refit_adj"][1] / kt["k_refit_adj"][0]
    fwd_b = nh * (9 + 80)
    adj_b = nh * (9 + 80 + 8)
    log(f"[bench] refit+adjoint {ms:.3f} ms per pass, {rs.n_tracks / (ms * 1e-3):.3e} tracks/s")
    calib = calibration_bench(api, ctx, stream, prm, rs, h, rx, th, steps)
    return {
        "calibration": calib,
        "workload": "1M truth track segments of 40-152 consecutive-row hits (seed 5005), "
                    "calibrated refit (16 parameters) + adjoint, float32",
        "tracks": rs.n_tracks, "hits": nh,
        "tracks_per_s": rs.n_tracks / (ms * 1e-3),
        "ms_per_pass": ms,
        "kernels_us": kern,
        "roofline_fwd": {"bound": "hbm", "achieved": fwd_b / (fwd_ms * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": fwd_b / (fwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_hit": 89},
        "roofline_adj": {"bound": "hbm", "achieved": adj_b / (adj_ms * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": adj_b / (adj_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "algorithmic_bytes_per_hit": 97},
    }


def calibration_bench(api, ctx, stream, prm, rs, h, rx, th, steps):
    """Global calibration on the refit set: one evaluation of the objective
    and its gradient (refit, beam-axis term, seeded adjoint, the value read
    back to the host), then a whole damped-Newton calibration from the
    evaluation point to convergence."""
    import numpy as np
    import torch
    st = {}
    with torch.cuda.stream(stream):
        api.calibration_objective(ctx, h, rx, prm, th, None, stream=stream, state=st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            api.calibration_objective(ctx, h, rx, prm, th, None, stream=stream, state=st)
        torch.cuda.synchronize()
        ms_eval = (time.perf_counter() - t0) / steps * 1e3
        free = np.array(api.CALIB_FREE)
        th_true = rs.theta_true.astype(np.float64)
        th0 = th_true.copy()
        th0[free] = rs.theta_eval.astype(np.float64)[free]
        t0 = time.perf_counter()
        res = api.calibrate(ctx, h, rx, prm, th0, stream=stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    left = np.abs(res["theta"][free] - th_true[free]) / np.abs(th0[free] - th_true[free])
    log(f"[bench] calibration: objective+gradient {ms_eval:.3f} ms, fit {wall:.2f} s in "
        f"{len(res['history'])} iterations, offset left {np.round(left, 3).tolist()}")
    return {
        "free_parameters": [int(k) for k in free],
        "ms_per_objective_and_gradient": ms_eval,
        "fit_seconds": wall,
        "iterations": len(res["history"]),
        "offset_left_fraction": [float(x) for x in left],
    }


# the batch the forked oracle workers read (set before the pool forks)
_ORACLE_EVENT = None


def _oracle_instance(k):
    """Worker: the oracle's tracking of instance k of the batch, alone."""
    import numpy as np

    import oracle
    from paper_1905_05515_amd.layout import grid_layout
    ev, prm, occ = _ORACLE_EVENT
    b0, b1 = int(ev.sector_offsets[k]), int(ev.sector_offsets[k + 1])
    off = np.array([0, b1 - b0], np.int64)
    tab, nb = grid_layout(off, ev.sector_range[k:k + 1], occupancy=occ,
                          sides=ev.sector_side[k:k + 1])
    t0 = time.perf_counter()
    r = oracle.track_event(ev.row[b0:b1], ev.y[b0:b1], ev.z[b0:b1], tab, nb, ev.row_x, prm)
    return time.perf_counter() - t0, r["tracks"]["trk_off"].shape[0] - 1


def cpu_baseline(args, ev, prm, occupancy=0.25):
    """The oracle (plain single-threaded C) on the host over the same batch:
    tracking of every instance on one core, the same on all host cores with
    one instance per task (the paper's sector-parallel CPU tracking), the
    float refit of the found tracks, and the float64 reverse-mode gradient
    timed on a sample of them and scaled to all.  Runs before the GPU is
    used, so the worker processes fork from a process without device
    state."""
    import multiprocessing as mp

    import numpy as np

    import oracle
    from paper_1905_05515_amd.layout import grid_layout
    global _ORACLE_EVENT
    tab, nb = grid_layout(ev.sector_offsets, ev.sector_range, occupancy=occupancy,
                          sides=ev.sector_side)
    t0 = time.perf_counter()
    res = oracle.track_event(ev.row, ev.y, ev.z, tab, nb, ev.row_x, prm)
    t_track = time.perf_counter() - t0
    trk = res["tracks"]
    off, ids = trk["trk_off"], trk["trk_hits"]
    n_trk = off.shape[0] - 1
    sec = np.searchsorted(ev.sector_offsets, ids[off[:-1]], side="right") - 1
    side = np.where(ev.sector_side[sec] < 0, -1, 1).astype(np.int8)
    th = synth_theta()
    t0 = time.perf_counter()
    oracle.refit(off, ev.row[ids], ev.y[ids], ev.z[ids], ev.row_x, prm, th, side=side)
    t_refit = time.perf_counter() - t0
    k = min(4000, n_trk)
    so = off[:k + 1]
    sel = ids[:so[-1]]
    t0 = time.perf_counter()
    oracle.refit_adjoint64(so, ev.row[sel], ev.y[sel], ev.z[sel], ev.row_x, prm,
                           th.astype(np.float64), np.ones(k), side=side[:k])
    t_adj = (time.perf_counter() - t0) * n_trk / max(k, 1)
    # all host cores, one instance per task, largest first
    cores = min(16, len(os.sched_getaffinity(0)))
    _ORACLE_EVENT = (ev, prm, occupancy)
    order = np.argsort(-np.diff(ev.sector_offsets), kind="stable").tolist()
    with mp.get_context("fork").Pool(cores) as pool:
        pool.map(_oracle_instance, order[-cores:])          # start-up of the workers
        t0 = time.perf_counter()
        per = pool.map(_oracle_instance, order, chunksize=1)
        t_par = time.perf_counter() - t0
    _ORACLE_EVENT = None
    same = sum(n for _, n in per) == n_trk
    log(f"[bench] oracle: tracking {t_track:.2f}s on one core, {t_par:.2f}s on {cores} "
        f"(tracks equal {same}), refit {t_refit:.2f}s, reverse-mode gradient {t_adj:.1f}s "
        f"(from {k} tracks)")
    total = t_track + t_refit + t_adj
    return {"value": ev.n_clusters / t_track, "unit": "clusters/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole batch ({ev.n_clusters} clusters, {ev.n_sectors} instances) "
                      f"tracked on one core; value = tracking (grid to selection) only",
            "whole_step_clusters_per_s": ev.n_clusters / total,
            "whole_step_sample": f"tracking + float refit of the {n_trk} found tracks + "
                                 f"float64 reverse-mode gradient timed on {k} of them and "
                                 f"scaled to all",
            "multi_core": {"cores": cores, "clusters_per_s": ev.n_clusters / t_par,
                           "seconds": t_par, "same_track_count": bool(same),
                           "form": "one instance per task over a process pool, largest first"},
            "seconds_one_core": {"tracking": t_track, "refit": t_refit, "adjoint": t_adj}}


def synth_theta():
    import numpy as np
    import synth
    return np.asarray(synth.make_config5(n_tracks=1).theta_eval, np.float32)


if __name__ == "__main__":
    main()
