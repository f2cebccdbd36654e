#!/usr/bin/env python
"""Throughput of the pixelated-LArTPC charge path on one MI355X.

A step is one pass of the whole path (recombination, drift, rasterisation, charge cells, induction, per-pixel sum,
electronics, FP64 charge report) over one module-scale event: 20,000 segments from 40 tracks in a 140 x 140-pixel
tile, 3000 ticks, 45 x 45 x 1950 response table (seeded synthetic input, see paper_2212_09807_amd.workloads).
Inputs are resident in device memory before the timed region; each step is one lts_simulate call followed by a
stream synchronisation (plain per-event launches), so the per-step wall times give the event latency.

Printed: one JSON line with segments/s and events/s, per-event latency percentiles, the induction kernel's roofline
position (its duration measured with HIP events on the launch stream during the timed steps, its multiply-adds
counted exactly by the library), and the FP64 CPU oracle timed on a bounded sample of the same event.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz; one FP32 FMA (2 flops) per lane per clock without packed-FP32
# instructions (which this build does not emit).
PEAK_FP32_FMA_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
# The published 157.3 TFLOP/s FP32 vector figure counts packed FP32 (two FMAs per lane per clock); reported beside
# the non-packed peak so the fraction against either is visible.
PEAK_FP32_PACKED_TFLOPS = 157.3
PEAK_FP32_MFMA_TFLOPS = 157.3       # dense FP32 matrix-core rate
HBM_PEAK_GBS = 8000.0


INDUCE_KERNEL = {"sorted": "k_induce_sorted", "atomic": "k_induce_atomic", "summed": "k_induce_summed"}


def kernel_source_digest():
    """SHA-256 over the device sources (kernels.hip, device.hpp): identifies the kernel build a profile was taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "device.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2212_09807_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel):
    """Memory traffic per launch of `kernel` (bytes read + written beyond L2, from rocprofv3 FETCH_SIZE / WRITE_SIZE
    counters scaled by a plain copy's readings), taken from the committed profile summaries; None unless a summary
    was recorded on the current kernel sources."""
    import glob
    digest = kernel_source_digest()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(f):
            if line.startswith("traffic-record:"):
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                if kv.get("kernel") == kernel and kv.get("source") == digest:
                    return float(kv["read_bytes"]) + float(kv["write_bytes"])
    return None


def cpu_baseline(w, budget_s=15.0):
    """The oracle as it stands, on the first S segments of the same event (all pixels they reach, full window,
    electronics); S grows until the run takes about budget_s."""
    import oracle
    from paper_2212_09807_amd import workloads as W
    oracle.build(force=False)
    table = W.response_table(w.table, w.readout, w.physics.v_drift)
    full = w.events[0]
    S, dt = 8, 0.0
    while True:
        sub = full.subset(list(range(S)))
        t0 = time.perf_counter()
        pix = oracle.active_pixels(w.physics, w.readout, w.table, sub)
        wave, _ = oracle.waveforms(w.physics, w.readout, table, sub, pix)
        oracle.electronics(w.electronics, w.readout, w.event_ids[0], pix, wave)
        dt = time.perf_counter() - t0
        if dt >= budget_s / 3 or S >= full.n:
            break
        S = min(full.n, int(S * max(2.0, budget_s / max(dt, 1e-3) * 0.5)))
    cores = oracle.num_threads()
    # one thread, on a sample 1/cores the size (about the same wall time)
    S1 = max(1, S // max(cores, 1))
    sub = full.subset(list(range(S1)))
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        pix1 = oracle.active_pixels(w.physics, w.readout, w.table, sub)
        wave, _ = oracle.waveforms(w.physics, w.readout, table, sub, pix1)
        oracle.electronics(w.electronics, w.readout, w.event_ids[0], pix1, wave)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(cores)
    return {"value": S / dt, "unit": "segments/s", "cores": cores, "kind": "oracle",
            "sample": f"first {S} of {full.n} segments of the module-scale event, all {len(pix)} pixels they reach, "
                      f"3000 ticks, induction + electronics, FP64, {dt:.1f} s",
            "single_thread": {"value": S1 / dt1, "unit": "segments/s",
                              "sample": f"first {S1} segments, {len(pix1)} pixels, {dt1:.1f} s"}}


def batched_vs_plain(ltsim, W, n_events, mode, cfg=3):
    """The first n_events of the batched-spill workload (cfg 3), or n_events single-track events (cfg 1): one
    lts_simulate_batch call vs one lts_simulate per event, same results; events/s of each (one untimed pass of each
    first)."""
    import numpy as np
    import torch
    w = W.make_workload(cfg, n_events=n_events)
    ctx = ltsim.Context.from_workload(w, reduce_mode=mode)
    allsegs = W.Segments.concat(w.events)
    offs = np.r_[0, np.cumsum([e.n for e in w.events])]
    dsegs = ltsim.to_device(allsegs)
    singles = [ltsim.to_device(e) for e in w.events]
    outs = [ctx._alloc(ctx.plan(d)["pixels"], ctx.plan(d)["packets"], 1, False) for d in singles]
    cap = sum(int(o.pixel_id.numel()) for o in outs)
    bout = ctx._alloc(cap, cap * w.electronics.max_packets // 4, n_events, True)
    res = {}
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.simulate_batch(dsegs, offs, w.event_ids, out=bout)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        t0 = time.perf_counter()
        for d, o, i in zip(singles, outs, w.event_ids):
            ctx.simulate(d, event_id=i, out=o)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        print(f"[bench] batched pass {rep}: batch {tb:.3f} s, plain {tp:.3f} s", file=sys.stderr, flush=True)
    # the same plain calls and batch with each call's launch sequence replayed as a HIP graph
    ctx.set_graph(True)
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for d, o, i in zip(singles, outs, w.event_ids):
            ctx.simulate(d, event_id=i, out=o)
        torch.cuda.synchronize()
        tpg = time.perf_counter() - t0
        t0 = time.perf_counter()
        ctx.simulate_batch(dsegs, offs, w.event_ids, out=bout)
        torch.cuda.synchronize()
        tbg = time.perf_counter() - t0
    ctx.set_graph(False)
    res = {"workload": "batched spill (log-normal event sizes)" if cfg == 3 else "single-track events, 200 segments",
           "events": n_events, "segments": int(allsegs.n), "batched_events_per_s": n_events / tb,
           "plain_events_per_s": n_events / tp, "batched_segments_per_s": allsegs.n / tb,
           "plain_segments_per_s": allsegs.n / tp, "gain": tp / tb,
           "graph": {"plain_events_per_s": n_events / tpg, "batched_events_per_s": n_events / tbg,
                     "updates_instantiations": list(ctx.graph_stats())}}
    return res


PEAK_FP64_FMA_TFLOPS = PEAK_FP32_FMA_TFLOPS     # gfx950: FP64 vector FMA at the non-packed FP32 rate


def light_leg(ltsim, W, reps=10):
    """The light path (Sec. 4.2-4.3) on the synthetic spill photocurrents: per-event time of one lts_light_simulate
    (HIP events on its stream, inputs resident), detector-ticks per second, and the FP64 rate of the scintillation
    convolution's useful multiply-adds over the whole call (a lower bound of that kernel's own rate)."""
    import torch
    lp, ipe, r, amp = W.light_workload()
    sim = ltsim.LightSim(lp, r, amp)
    x = torch.from_numpy(ipe).cuda()

    def timed(s):
        out = s.simulate(x, 1)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for i in range(reps):
            s.simulate(x, 1 + i, out=out)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ms = timed(sim)
    gsim = ltsim.LightSim(lp, r, amp)
    gsim.set_graph(True)
    ms_graph = timed(gsim)
    gsim.close()
    K = int(lp.trunc * lp.tau_s / lp.tick) + 1
    T = lp.n_ticks
    fma = lp.n_det * (min(K, T) * (min(K, T) + 1) // 2 + max(T - K, 0) * K)
    sim.close()
    ach = 2.0 * fma / (ms / 1e3) / 1e12
    return {"workload": f"light spill: {lp.n_det} detectors x {T} ticks of {lp.tick} ns, {K}-tap scintillation kernel, "
                        f"{len(r)}-tap response, {len(amp)} noise sinusoids, 4 interactions",
            "ms_per_event": ms, "ms_per_event_graph": ms_graph, "detector_ticks_per_s": lp.n_det * T / (ms / 1e3),
            "roofline": {"kernel": "k_light_scint (whole light call timed)", "bound": "alu", "achieved": ach,
                         "peak": PEAK_FP64_FMA_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP64_FMA_TFLOPS,
                         "flops_per_launch": 2.0 * fma, "dtype": "f64"}}


def large_spill_leg(ltsim, W, modes):
    """The large spill (35 tiles of 140 x 140 pixels, 2,000,000 segments plus halo replicas, 5000 ticks, full noise):
    one plain lts_simulate per tile, device-resident segments, wall time of the whole spill per reduce mode."""
    import torch
    w = W.make_workload(5)
    n_orig = 2_000_000
    n_all = sum(e.n for e in w.events)
    dsegs = [ltsim.to_device(e) for e in w.events]
    out = {"workload": f"large spill: {len(w.events)} tiles of {w.readout.n_x}x{w.readout.n_y} pixels, {n_orig} "
                       f"segments ({n_all} with halo replicas), {w.readout.n_ticks} ticks, 45x45x1950 table, "
                       f"noise 900/650/500 e-, one plain call per tile"}
    for name in modes:
        mode, shift, rt = MODES[name]
        ctx = ltsim.Context.from_workload(w, reduce_mode=mode)
        ctx.set_lane_exchange(shift)
        ctx.set_ticks_per_thread(rt)
        big = max(range(len(dsegs)), key=lambda i: w.events[i].n)
        ctx.simulate(dsegs[big], event_id=w.event_ids[big])            # warm-up: allocations, table upload
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for d, i in zip(dsegs, w.event_ids):
            ctx.simulate(d, event_id=i)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(f"[bench] large spill {name}: {el:.2f} s", file=sys.stderr, flush=True)
        out[name] = {"seconds": el, "segments_per_s": n_orig / el}
        ctx.close()
    return out


def materialised_leg(ltsim, W, steps=3):
    """The paper's data flow on the module-scale event: every (segment, pixel) pair's current written out as its own
    n_ticks waveform (lts_stage_induce), then summed per pixel (lts_stage_reduce); wall time per event against the
    fused per-pair path, and the bytes of the materialised tensor."""
    import torch
    w = W.make_workload(2)
    d = ltsim.to_device(w.events[0])
    ctx = ltsim.Context.from_workload(w)
    eid = w.event_ids[0]
    sg, px, cur = ctx.stage_induce(d, event_id=eid)
    ctx.stage_reduce(px, cur)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        del sg, px, cur                                # one materialised tensor at a time
        sg, px, cur = ctx.stage_induce(d, event_id=eid)
        pid, red = ctx.stage_reduce(px, cur)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    fused = ctx.simulate(d, event_id=eid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fused = ctx.simulate(d, event_id=eid)
    torch.cuda.synchronize()
    fe = (time.perf_counter() - t0) / steps
    n_pairs = int(px.numel())
    out = {"workload": "module-scale event, materialised (segment, pixel, tick) currents then per-pixel sum",
           "pairs": n_pairs, "tensor_bytes": 4 * n_pairs * w.readout.n_ticks,
           "ms_per_event": el * 1e3, "fused_ms_per_event": fe * 1e3,
           "note": "materialised = stage_induce + stage_reduce (no electronics); fused = whole lts_simulate"}
    del sg, px, cur, pid, red, fused
    ctx.close()
    torch.cuda.empty_cache()
    return out


def served(ltsim, W, rate_hz, n_events, mode, lanes=2):
    """Poisson arrivals at rate_hz of the batched-spill event mix through the library's request loop."""
    import numpy as np
    w = W.make_workload(4, n_events=n_events)
    arr = W.poisson_arrivals(rate_hz, n_events)
    ctx = ltsim.Context.from_workload(w, reduce_mode=mode)
    srv = ltsim.Server(ctx, n_lanes=lanes, max_batch_events=64)
    try:
        t0 = time.perf_counter()
        tickets = []
        for seg, eid, ta in zip(w.events, w.event_ids, arr):
            dt = t0 + ta - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            tickets.append(srv.submit(seg, eid))
        res = [srv.wait(t) for t in tickets]
        t1 = time.perf_counter()
        for t in tickets:
            srv.release(t)
    finally:
        srv.stop()
    lat = np.array([r["t_done"] - r["t_submit"] for r in res])
    nseg = sum(e.n for e in w.events)
    return {"rate_hz": rate_hz, "events": n_events, "events_per_s": n_events / (t1 - t0),
            "segments_per_s": nseg / (t1 - t0), "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                                                               "p99": float(np.percentile(lat, 99) * 1e3)},
            "mean_batch_events": float(np.mean([r["batch_events"] for r in res])), "lanes": lanes}


def served_burst(ltsim, W, n_events, mode, lanes=2):
    """n_events single-track events (200 segments each) submitted to the request loop at once, host segments in:
    completed events/s and latency, against the same events as plain calls (device-resident segments, one
    lts_simulate and synchronisation each)."""
    import numpy as np
    import torch
    w = W.make_workload(1, n_events=n_events)
    ctx = ltsim.Context.from_workload(w, reduce_mode=mode)
    singles = [ltsim.to_device(e) for e in w.events]
    for d, i in zip(singles[:4], w.event_ids):                      # warm-up
        ctx.simulate(d, event_id=i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d, i in zip(singles, w.event_ids):
        ctx.simulate(d, event_id=i)
        torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    srv = ltsim.Server(ctx, n_lanes=lanes, max_batch_events=64)
    try:
        for _ in range(2):                                            # the second burst is timed
            t0 = time.perf_counter()
            tickets = [srv.submit(seg, eid) for seg, eid in zip(w.events, w.event_ids)]
            res = [srv.wait(t) for t in tickets]
            t1 = time.perf_counter()
            for t in tickets:
                srv.release(t)
    finally:
        srv.stop()
    lat = np.array([r["t_done"] - r["t_submit"] for r in res])
    return {"workload": "single-track events, 200 segments, submitted at once", "events": n_events,
            "events_per_s": n_events / (t1 - t0), "plain_events_per_s": n_events / t_plain,
            "gain": t_plain / (t1 - t0), "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                                                         "p99": float(np.percentile(lat, 99) * 1e3)},
            "mean_batch_events": float(np.mean([r["batch_events"] for r in res])), "lanes": lanes}


# name: (reduce mode, lane exchange, ticks per thread)
MODES = {"sorted": (0, 0, 0), "atomic": (1, 0, 0), "summed": (2, 0, 0), "sorted-shift": (0, 1, 0),
         "sorted-noprefetch": (0, 0, 8), "sorted-mfma": (0, 0, 0)}


def time_mode(ltsim, w, segs, name, steps):
    """Whole path in another variant (reduce mode, and for the per-pair kernels whether lanes exchange table
    windows) on the same device-resident event: segments/s and its induction roofline."""
    import torch
    mode, shift, rt = MODES[name]
    ctx = ltsim.Context.from_workload(w, reduce_mode=mode)
    ctx.set_lane_exchange(shift)
    ctx.set_ticks_per_thread(rt)
    ctx.set_matrix_cores(name.endswith("-mfma"))
    need = ctx.plan(segs)
    out = ctx._alloc(need["pixels"], need["packets"], 1, False)
    ctx.simulate(segs, event_id=w.event_ids[0], out=out)
    torch.cuda.synchronize()
    stats = ctx.work_stats()
    ctx.set_timing(True)
    ctx.get_timing()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.simulate(segs, event_id=w.event_ids[0], out=out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tm = ctx.get_timing()
    ind_ms = tm["induce"][0] / max(tm["induce"][1], 1)
    ach = 2.0 * stats["fma"] / (ind_ms / 1e3) / 1e12
    mfma = name.endswith("-mfma")
    peak = PEAK_FP32_MFMA_TFLOPS if mfma else PEAK_FP32_FMA_TFLOPS
    return {"value": segs.n * steps / el, "unit": "segments/s", "ms_per_step": el / steps * 1e3,
            "stage_ms": {k: v[0] / max(v[1], 1) for k, v in tm.items()},
            "roofline": {"bound": "mfma" if mfma else "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                         "frac": ach / peak, "traffic": None, "flops_per_launch": 2.0 * stats["fma"],
                         "launch_ms": ind_ms}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", choices=("sorted", "atomic", "summed"), default="sorted")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--batched", type=int, default=8, help="also compare a batch of N spill events with N plain calls")
    ap.add_argument("--served", type=float, nargs=2, default=(2.0, 16), metavar=("RATE_HZ", "N"),
                    help="also serve N spill events arriving as a Poisson process at RATE_HZ")
    ap.add_argument("--slices", type=int, default=1)
    ap.add_argument("--no-light", action="store_true", help="skip the light-path leg")
    ap.add_argument("--served-sweep", default="", metavar="RATES",
                    help="comma-separated arrival rates (events/s) to serve 16 spill events each at, to find saturation")
    ap.add_argument("--materialised", action="store_true",
                    help="also time the paper's data flow: per-pair currents written out, then summed per pixel")
    ap.add_argument("--large-spill", default="", help="comma-separated modes to time on the 2M-segment large spill "
                                                      "(minutes of GPU time; off by default)")
    ap.add_argument("--also", default=None,
                    help="comma-separated other reduce modes to time on the same event (default: summed; none with --quick)")
    ap.add_argument("--quick", action="store_true", help="only the headline path (no batch or serving, and no other "
                                                         "modes unless --also names them)")
    args = ap.parse_args()
    if args.quick:
        args.batched, args.served, args.no_light = 0, None, True
    if args.also is None:
        args.also = "" if args.quick else "summed"
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (events shard across GPUs "
              f"with no exchange, so a multi-GPU run is one such process per GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2212_09807_amd import ltsim, workloads as W

    w = W.make_workload(2)
    segs_h = w.events[0]
    mode = {"sorted": 0, "atomic": 1, "summed": 2}[args.mode]
    ctx = ltsim.Context.from_workload(w, reduce_mode=mode)
    ctx.set_induce_slices(args.slices)
    segs = ltsim.to_device(segs_h)
    need = ctx.plan(segs)
    out = ctx._alloc(need["pixels"], need["packets"], 1, False)
    print(f"[bench] event: {segs_h.n} segments, {need['pairs']} pairs, {need['pixels']} active pixels, "
          f"{need['cells']} cells", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        ctx.simulate(segs, event_id=w.event_ids[0], out=out)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    stats = ctx.work_stats()
    ctx.set_timing(True)
    ctx.get_timing()
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        ctx.simulate(segs, event_id=w.event_ids[0], out=out)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        print(f"[bench] step {i + 1}/{args.steps}: {lat[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    timing = ctx.get_timing()
    ctx.set_timing(False)

    ind_ms, ind_calls = timing["induce"]
    ind_s = ind_ms / 1e3 / max(ind_calls, 1)
    achieved = 2.0 * stats["fma"] / ind_s / 1e12
    n_seg = segs_h.n
    line = {
        "metric": "segments/s",
        "value": n_seg * args.steps / elapsed,
        "unit": "segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "module-scale event: 20000 segments (30 muon-like + 10 proton-like tracks), "
                               "140x140 pixels, 3000 ticks, 45x45x1950 response table, plain per-event path",
                   "segments_per_event": n_seg, "pairs": int(stats["pairs"]), "active_pixels": need["pixels"],
                   "reduce": args.mode},
        "events_per_s": args.steps / elapsed,
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
        "stage_ms": {k: (v[0] / max(v[1], 1)) for k, v in timing.items()},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_FMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_FMA_TFLOPS,
                     "peak_basis": "FP32 FMA without packed-FP32 instructions (not emitted by this build)",
                     "frac_of_packed_fp32_peak": achieved / PEAK_FP32_PACKED_TFLOPS,
                     "traffic": profiled_traffic(INDUCE_KERNEL[args.mode]),
                     "traffic_unit": "bytes per launch beyond L2 (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel_source": kernel_source_digest(),
                     "kernel": INDUCE_KERNEL[args.mode],
                     "flops_per_launch": 2.0 * stats["fma"], "launch_ms": ind_s * 1e3},
    }
    line["config"]["induce_slices"] = args.slices if args.mode == "sorted" else 1
    for other in [m for m in args.also.split(",") if m and m != args.mode]:
        line.setdefault("modes", {})[other] = time_mode(ltsim, w, segs, other, args.steps)
    if args.batched:
        line["batched"] = batched_vs_plain(ltsim, W, args.batched, mode)
        line["batched_small"] = batched_vs_plain(ltsim, W, 64, mode, cfg=1)
    if not args.no_light:
        line["light"] = light_leg(ltsim, W)
    if args.materialised:
        line["materialised"] = materialised_leg(ltsim, W)
    if args.large_spill:
        line["large_spill"] = large_spill_leg(ltsim, W, [m for m in args.large_spill.split(",") if m])
    if args.served:
        line["served"] = served(ltsim, W, args.served[0], int(args.served[1]), mode)
        line["served_small"] = served_burst(ltsim, W, 64, mode)
    if args.served_sweep:
        line["served_sweep"] = [served(ltsim, W, float(r), 16, mode) for r in args.served_sweep.split(",") if r]
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
