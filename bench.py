#!/usr/bin/env python
"""Throughput of the pixelated-LArTPC charge path on one MI355X.

Headline (default): the large spill on one GPU: 2,000,000 energy-deposit segments (30 neutrino-like vertices and 200
cosmic muons, seeded synthetic input, see paper_2212_09807_amd.workloads) over 35 module tiles of 140 x 140 pixels
(2,256,481 segments with the halo replicas of tile edges), 5000 ticks, 45 x 45 x 1950 response table, full front-end
noise (reset 900, discriminator 650, uncorrelated 500 electrons).  A step is one pass of the whole path
(recombination, drift, rasterisation, charge cells, induction, per-pixel sum, electronics, FP64 charge report) over
the whole spill: one lts_simulate_batch call with the 35 tiles as events, then a stream synchronisation.  Inputs are
resident in device memory before the timed region.  The headline reduce mode is the exact sum-then-convolve form
(LTS_REDUCE_SUMMED); the per-pair form and the module-scale event are timed as further legs.

Printed: one JSON line with segments/s (original segments, halo replicas not counted), the induction kernel's
roofline position (its launch duration measured with HIP events on the launch stream during the timed steps, its
multiply-adds counted exactly by the library), the other legs (per-pair path on the spill, reduce modes on the
module-scale event, batching and serving on the spill event mix, the light path) and the FP64 CPU oracle timed on a
bounded sample of one tile, with the per-output error of the headline run on a sample of pixels.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks.  FP32 vector 157.3 TFLOP/s counts packed FP32 (two FMAs per lane per clock); this build
# emits no packed-FP32 instructions, so its vector ALU ceiling is 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz x 2 flop =
# 78.6 TFLOP/s, reported beside the published figure.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
PEAK_FP64_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0

INDUCE_KERNEL = {"sorted": "k_induce_sorted", "atomic": "k_induce_atomic", "summed": "k_induce_summed4"}
MODE_ID = {"sorted": 0, "atomic": 1, "summed": 2}
SPILL_SEGMENTS = 2_000_000


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_digest():
    """SHA-256 over the device sources (kernels.hip, device.hpp): identifies the kernel build a profile was taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "device.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2212_09807_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel, workload):
    """HBM traffic per launch of `kernel` on `workload` (bytes read + written, from rocprofv3 FETCH_SIZE / WRITE_SIZE
    scaled by a plain copy's readings), taken from the committed profile summaries; None unless a summary was
    recorded on the current kernel sources."""
    import glob
    digest = kernel_source_digest()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(f):
            if line.startswith("traffic-record:"):
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                if kv.get("kernel") == kernel and kv.get("source") == digest and kv.get("workload") == workload:
                    return float(kv["read_bytes"]) + float(kv["write_bytes"])
    return None


def roofline(kernel, workload, fma, launch_ms, extra=None):
    ach = 2.0 * fma / (launch_ms / 1e3) / 1e12
    r = {"bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP32_TFLOPS,
         "traffic": profiled_traffic(kernel, workload), "kernel": kernel, "flops_per_launch": 2.0 * fma,
         "launch_ms": launch_ms, "frac_of_nonpacked_fp32_peak": ach / PEAK_FP32_NONPACKED_TFLOPS,
         "nonpacked_fp32_peak": PEAK_FP32_NONPACKED_TFLOPS, "kernel_source": kernel_source_digest(),
         "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"}
    if extra:
        r.update(extra)
    return r


def stage_ms(timing):
    return {k: v[0] / max(v[1], 1) for k, v in timing.items() if v[1]}


# ----------------------------------------------------------------------------------------------- the large spill

def spill_inputs(ltsim, W):
    """The large spill as one batch: device segments of the 35 tiles concatenated, offsets and event ids."""
    import numpy as np
    w = W.make_workload(5)
    allsegs = W.Segments.concat(w.events)
    offs = np.r_[0, np.cumsum([e.n for e in w.events])].astype(np.int64)
    return w, ltsim.to_device(allsegs), offs


def spill_batch_out(ctx, w, ltsim, tile_segs):
    """Output buffers for the whole spill as one batch, sized from each tile's plan."""
    pix = 0
    for d in tile_segs:
        pix += ctx.plan(d)["pixels"]
    return ctx._alloc(pix, pix * w.electronics.max_packets // 4 + 4096, len(w.events), True)


def headline(ltsim, W, args):
    import numpy as np
    import torch
    w, dsegs, offs = spill_inputs(ltsim, W)
    n_all = int(offs[-1])
    ctx = ltsim.Context.from_workload(w, reduce_mode=MODE_ID[args.mode])
    tiles = [ltsim.to_device(e) for e in w.events]
    out = spill_batch_out(ctx, w, ltsim, tiles)
    del tiles
    log(f"spill: {len(w.events)} tiles, {n_all} segments with halo replicas, capacity {out.pixel_id.numel()} pixels")
    for i in range(args.warmup):
        ctx.simulate_batch(dsegs, offs, w.event_ids, out=out)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    ctx.set_timing(True)
    ctx.get_timing()
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        t0 = time.perf_counter()
        ctx.simulate_batch(dsegs, offs, w.event_ids, out=out)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        log(f"step {i + 1}/{args.steps}: {lat[-1] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    timing = ctx.get_timing()
    ctx.set_timing(False)
    stats = ctx.work_stats()                                   # exact multiply-adds of the last (timed) call
    st = stage_ms(timing)
    # host copies of everything but the currents (those stay on the device; the accuracy leg reads sampled rows)
    cnt = out.counts.cpu().numpy()
    n_pix, n_pk = int(cnt[0]), int(cnt[1])
    h = {"counts": cnt, "pixel_id": out.pixel_id[:n_pix].cpu().numpy(), "report": out.report.cpu().numpy(),
         "event_pixel_offsets": out.event_pixel_offsets.cpu().numpy(),
         "event_packet_offsets": out.event_packet_offsets.cpu().numpy(),
         "pkt_pixel": out.pkt_pixel[:n_pk].cpu().numpy(), "pkt_tick": out.pkt_tick[:n_pk].cpu().numpy(),
         "pkt_adc": out.pkt_adc[:n_pk].cpu().numpy().view(np.uint16), "current_dev": out.current}
    line = {
        "metric": "segments/s",
        "value": SPILL_SEGMENTS * args.steps / elapsed,
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
        "config": {"workload": f"large spill: {SPILL_SEGMENTS} segments (30 neutrino-like vertices + 200 cosmic muons) "
                               f"over {len(w.events)} tiles of {w.readout.n_x}x{w.readout.n_y} pixels, "
                               f"{w.readout.n_ticks} ticks, 45x45x1950 response table, noise 900/650/500 e-, "
                               f"one lts_simulate_batch per spill, {args.mode} induction",
                   "segments_with_halo": n_all, "tiles": len(w.events), "active_pixels": int(h["counts"][0]),
                   "packets": int(h["counts"][1]), "pairs": int(stats["pairs"]), "reduce": args.mode},
        "events_per_s": args.steps / elapsed,
        "tiles_per_s": len(w.events) * args.steps / elapsed,
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3)},
        "stage_ms": st,
        "roofline": roofline(INDUCE_KERNEL[args.mode], "large_spill", stats["fma"], st["induce_kernel"],
                             {"fma_issued_per_launch": stats["fma_issued"] or None,
                              "useful_fraction_of_issued": stats["fma"] / stats["fma_issued"] if stats["fma_issued"]
                              else None, "records": stats["records"]}),
    }
    # the report's conservation check at full size: collected = induced in window + clipped + off-grid (per tile)
    rep = h["report"]
    line["charge_conservation_max_rel"] = float(np.max(np.abs(rep[:, 2] + rep[:, 3] + rep[:, 4] - rep[:, 1]) /
                                                      np.maximum(rep[:, 1], 1.0)))
    ctx.close()
    return line, (w, h)


def spill_tiles_leg(ltsim, W, mode_name):
    """The spill as 35 plain calls (one lts_simulate per tile) in the given reduce mode: one pass after a warm-up
    on the largest tile; wall time, segments/s and the induction kernel's roofline."""
    import torch
    w = W.make_workload(5)
    tiles = [ltsim.to_device(e) for e in w.events]
    ctx = ltsim.Context.from_workload(w, reduce_mode=MODE_ID[mode_name])
    big = max(range(len(tiles)), key=lambda i: w.events[i].n)
    ctx.simulate(tiles[big], event_id=w.event_ids[big])
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ctx.get_timing()
    fma = 0.0
    t0 = time.perf_counter()
    for d, i in zip(tiles, w.event_ids):
        ctx.simulate(d, event_id=i)
        if mode_name != "summed":
            fma += ctx.work_stats()["fma"]                    # synchronises; per-pair passes are seconds per tile
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tm = ctx.get_timing()
    if mode_name == "summed":                                 # untimed recount (the summed pass is short)
        for d, i in zip(tiles, w.event_ids):
            ctx.simulate(d, event_id=i)
            fma += ctx.work_stats()["fma"]
    st = stage_ms(tm)
    kern_ms = tm["induce_kernel"][0]
    ctx.close()
    log(f"spill as tile calls, {mode_name}: {el:.2f} s")
    return {"workload": "large spill, one lts_simulate per tile", "seconds": el, "segments_per_s": SPILL_SEGMENTS / el,
            "induce_kernel_ms_total": kern_ms,
            "roofline": roofline(INDUCE_KERNEL[mode_name], "large_spill", fma, kern_ms,
                                 {"launch_ms": kern_ms / len(tiles), "flops_per_launch": 2.0 * fma / len(tiles),
                                  "launches": len(tiles)})}


# ----------------------------------------------------------------------------------------------- module event

def module_leg(ltsim, W, modes, steps):
    """The module-scale event (20,000 segments, 140 x 140 pixels, 3000 ticks) in each reduce mode: segments/s and
    the induction kernel's roofline (sorted vs atomic per-pixel reduction, and the summed form)."""
    import torch
    w = W.make_workload(2)
    segs = ltsim.to_device(w.events[0])
    res = {"workload": "module-scale event: 20000 segments (30 muon-like + 10 proton-like tracks), 140x140 pixels, "
                       "3000 ticks, 45x45x1950 table, plain per-event calls"}
    for name in modes:
        ctx = ltsim.Context.from_workload(w, reduce_mode=MODE_ID[name])
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
        st = stage_ms(ctx.get_timing())
        res[name] = {"segments_per_s": segs.n * steps / el, "ms_per_event": el / steps * 1e3, "stage_ms": st,
                     "roofline": roofline(INDUCE_KERNEL[name], "module_event", stats["fma"], st["induce_kernel"])}
        log(f"module event {name}: {el / steps * 1e3:.1f} ms")
        ctx.close()
    return res


# ----------------------------------------------------------------------------------------------- batching

def tuning_leg(ltsim, W, cfg=3):
    """The project autotuner on the batched-spill geometry (size classes of 500 to 32,000 segments per event, three
    seeded events each): the chosen work-split table, applied by the library per call in the tuned batching and
    serving legs."""
    from paper_2212_09807_amd import autotune as AT
    w = W.make_workload(cfg, n_events=1)
    t0 = time.perf_counter()
    res = AT.autotune(w)
    names = {0: "sorted", 1: "atomic", 2: "summed"}
    table = [{"from_segments_per_event": e[0], "reduce": names[e[1]], "slices": e[2], "ticks_per_thread": e[3],
              "lane_exchange": e[4]} for e in res["table"]]
    log(f"autotune: {table} in {time.perf_counter() - t0:.1f} s")
    return res["table"], {"table": table, "sweep_s": time.perf_counter() - t0,
                          "classes": [{"segments_per_event": c["segments_per_event"],
                                       "ms": {f"{names[r['choice']['reduce_mode']]}/s{r['choice']['slices']}"
                                              f"/t{r['choice']['ticks_per_thread']}": r["ms"] for r in c["all"]}}
                                      for c in res["classes"]]}


def _context(ltsim, w, mode_name, table):
    if mode_name == "tuned":
        ctx = ltsim.Context.from_workload(w)
        ctx.set_tuning(table)
        return ctx
    return ltsim.Context.from_workload(w, reduce_mode=MODE_ID[mode_name])


def batched_vs_plain(ltsim, W, n_events, mode_name, cfg=3, table=None):
    """The first n_events of the batched-spill workload (cfg 3: log-normal sizes, median 8000 segments), or n_events
    single-track events (cfg 1): one lts_simulate_batch call vs one lts_simulate per event.  The batch results are
    checked bit-identical to the plain calls' (same accuracy).  Untimed warm-up: one batch call, and a plain call of
    the largest event."""
    import numpy as np
    import torch
    w = W.make_workload(cfg, n_events=n_events)
    ctx = _context(ltsim, w, mode_name, table)
    allsegs = W.Segments.concat(w.events)
    offs = np.r_[0, np.cumsum([e.n for e in w.events])]
    dsegs = ltsim.to_device(allsegs)
    singles = [ltsim.to_device(e) for e in w.events]
    outs = []
    for d in singles:
        need = ctx.plan(d)
        outs.append(ctx._alloc(need["pixels"], need["packets"], 1, False))
    cap = sum(int(o.pixel_id.numel()) for o in outs)
    bout = ctx._alloc(cap, cap * w.electronics.max_packets // 4 + 4096, n_events, True)
    big = max(range(n_events), key=lambda i: w.events[i].n)
    ctx.simulate_batch(dsegs, offs, w.event_ids, out=bout)
    ctx.simulate(singles[big], event_id=w.event_ids[big], out=outs[big])
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
    b = bout.host()
    po = b["event_pixel_offsets"]
    same = True
    for e, o in enumerate(outs):
        s = o.host()
        same &= bool(np.array_equal(b["pixel_id"][po[e]:po[e + 1]], s["pixel_id"]) and
                     np.array_equal(b["current"][po[e]:po[e + 1]], s["current"]))
    log(f"batched {mode_name} ({'spill mix' if cfg == 3 else 'single tracks'}): batch {tb:.3f} s, plain {tp:.3f} s")
    res = {"workload": "batched spill (log-normal event sizes)" if cfg == 3 else "single-track events, 200 segments",
           "mode": mode_name, "events": n_events, "segments": int(allsegs.n), "batched_events_per_s": n_events / tb,
           "plain_events_per_s": n_events / tp, "batched_segments_per_s": allsegs.n / tb,
           "plain_segments_per_s": allsegs.n / tp, "gain": tp / tb, "identical_to_plain": same}
    ctx.close()
    return res


# ----------------------------------------------------------------------------------------------- serving

def served(ltsim, W, rate_hz, n_events, mode_name, lanes=2, table=None):
    """Poisson arrivals at rate_hz of the batched-spill event mix through the library's request loop (host segments
    in, continuous batching over `lanes` lanes): completed events/s and submit-to-done latency."""
    import numpy as np
    w = W.make_workload(4, n_events=n_events)
    arr = W.poisson_arrivals(rate_hz, n_events)
    ctx = _context(ltsim, w, mode_name, table)
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
    ctx.close()
    lat = np.array([r["t_done"] - r["t_submit"] for r in res])
    nseg = sum(e.n for e in w.events)
    log(f"served {mode_name} at {rate_hz} Hz: {n_events / (t1 - t0):.2f} events/s")
    return {"mode": mode_name, "rate_hz": rate_hz, "events": n_events, "events_per_s": n_events / (t1 - t0),
            "segments_per_s": nseg / (t1 - t0), "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                                                               "p99": float(np.percentile(lat, 99) * 1e3)},
            "mean_batch_events": float(np.mean([r["batch_events"] for r in res])), "lanes": lanes,
            "all_ok": all(r["status"] == 0 for r in res)}


def served_burst(ltsim, W, n_events, mode_name, lanes=2):
    """n_events single-track events (200 segments each) submitted to the request loop at once, host segments in:
    completed events/s and latency, against the same events as plain calls (device-resident segments, one
    lts_simulate and synchronisation each)."""
    import numpy as np
    import torch
    w = W.make_workload(1, n_events=n_events)
    ctx = ltsim.Context.from_workload(w, reduce_mode=MODE_ID[mode_name])
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
    ctx.close()
    lat = np.array([r["t_done"] - r["t_submit"] for r in res])
    return {"workload": "single-track events, 200 segments, submitted at once", "mode": mode_name,
            "events": n_events, "events_per_s": n_events / (t1 - t0), "plain_events_per_s": n_events / t_plain,
            "gain": t_plain / (t1 - t0), "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                                                         "p99": float(np.percentile(lat, 99) * 1e3)},
            "mean_batch_events": float(np.mean([r["batch_events"] for r in res])), "lanes": lanes}


# ----------------------------------------------------------------------------------------------- light path

def light_leg(ltsim, W, reps=10):
    """The light path (Sec. 4.2-4.3) on the synthetic spill photocurrents: per-event time of one lts_light_simulate
    (HIP events on its stream, inputs resident) and detector-ticks per second."""
    import torch
    lp, ipe, r, amp = W.light_workload()
    sim = ltsim.LightSim(lp, r, amp)
    x = torch.from_numpy(ipe).cuda()
    out = sim.simulate(x, 1)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for i in range(reps):
        sim.simulate(x, 1 + i, out=out)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    sim.close()
    K = int(lp.trunc * lp.tau_s / lp.tick) + 1
    T = lp.n_ticks
    fma = lp.n_det * (min(K, T) * (min(K, T) + 1) // 2 + max(T - K, 0) * K)
    ach = 2.0 * fma / (ms / 1e3) / 1e12
    return {"workload": f"light spill: {lp.n_det} detectors x {T} ticks of {lp.tick} ns, {K}-tap scintillation kernel",
            "ms_per_event": ms, "detector_ticks_per_s": lp.n_det * T / (ms / 1e3),
            "scint_fp64_tflops_whole_call": ach, "frac_of_fp64_peak": ach / PEAK_FP64_TFLOPS}


# ----------------------------------------------------------------------------------------------- oracle leg

def cpu_baseline_leg(w, h, budget_s, n_err_pixels):
    """The FP64 oracle (test infrastructure, as it stands) on the machine's host cores.

    Timing: the first S segments of the spill's median tile, all pixels they reach, the 5000-tick window with full
    noise (induction + electronics), S grown until the run takes about budget_s / 3 or more; scaled to segments/s.
    Accuracy of the headline run: on n_err_pixels pixels of three tiles (the largest-current ones and a seeded random
    set), the oracle recomputes every segment's induction and the front end; per-pixel relative L2 error of the
    currents and packet agreement (tick and ADC code bit-exact except decisions the oracle flags within the FP32
    error margin)."""
    import numpy as np
    import torch
    import oracle
    from paper_2212_09807_amd import workloads as W
    oracle.build(force=False)
    table = W.response_table(w.table, w.readout, w.physics.v_drift)
    order = sorted(range(len(w.events)), key=lambda i: w.events[i].n)
    tile = order[len(order) // 2]
    full = w.events[tile]
    S, dt = 8, 0.0
    while True:
        sub = full.subset(list(range(S)))
        t0 = time.perf_counter()
        pix = oracle.active_pixels(w.physics, w.readout, w.table, sub)
        wave, _ = oracle.waveforms(w.physics, w.readout, table, sub, pix)
        oracle.electronics(w.electronics, w.readout, w.event_ids[tile], pix, wave)
        dt = time.perf_counter() - t0
        if dt >= budget_s / 3 or S >= full.n:
            break
        S = min(full.n, int(S * max(2.0, budget_s / max(dt, 1e-3) * 0.5)))
    cores = oracle.num_threads()
    rate = S / dt
    base = {"value": rate, "unit": "segments/s", "cores": cores, "kind": "oracle",
            "sample": f"first {S} of {full.n} segments of tile {tile} (median size) of the large spill, all "
                      f"{len(pix)} pixels they reach, {w.readout.n_ticks} ticks, full noise, induction + "
                      f"electronics, FP64, {dt:.1f} s; the whole spill would take ~{SPILL_SEGMENTS / rate / 3600:.1f} h "
                      f"at this rate (extrapolated by segment count)"}
    # accuracy of the headline run on sampled pixels
    rng = np.random.default_rng(2212)
    po = h["event_pixel_offsets"]
    ko = h["event_packet_offsets"]
    errs, n_cmp, n_flag, n_bad, n_pk = [], 0, 0, 0, 0
    t0 = time.perf_counter()
    for t in (order[-1], order[len(order) // 2], order[len(order) // 4]):
        pid = h["pixel_id"][po[t]:po[t + 1]]
        if len(pid) == 0:
            continue
        cur = h["current_dev"][int(po[t]):int(po[t + 1])]
        k = max(1, n_err_pixels // 3)
        tot = cur.abs().sum(dim=1).cpu().numpy()
        pick = np.unique(np.r_[np.argsort(tot)[-(k // 2):], rng.choice(len(pid), min(len(pid), k - k // 2),
                                                                        replace=False)])
        o_wave, _ = oracle.waveforms(w.physics, w.readout, table, w.events[t], pid[pick])
        g = cur[torch.from_numpy(pick).to(cur.device)].cpu().numpy().astype(np.float64)
        errs.append(np.sqrt(((g - o_wave) ** 2).sum(1)) / np.maximum(np.sqrt((o_wave ** 2).sum(1)), 10.0))
        pk, _, uf = oracle.electronics(w.electronics, w.readout, w.event_ids[t], pid[pick], o_wave, 2e-6, 0.1,
                                       with_uncertain=True)
        gp, gt, ga = (h[x][ko[t]:ko[t + 1]] for x in ("pkt_pixel", "pkt_tick", "pkt_adc"))
        for q, p in enumerate(pid[pick]):
            ot, oa, of = pk[q]
            sel = gp == p
            st_, sa_ = gt[sel].astype(np.int64), ga[sel].astype(np.int64)
            n_pk += len(ot)
            # packets agree in tick and code; a code may differ only within the FP32 margin of an LSB boundary
            # (oracle flag bit 0), and the timelines may part only at or after a threshold decision the oracle
            # found within the FP32 margin (tick >= uf): such packets are the flagged ones
            k = 0
            while k < min(len(ot), len(st_)) and ot[k] == st_[k] and (oa[k] == sa_[k] or (of[k] & 1)):
                k += 1
            same = int(np.sum(oa[:k] == sa_[:k]))
            n_cmp += same
            n_flag += k - same
            if k < len(ot) or k < len(st_):
                t_part = min(ot[k] if k < len(ot) else 1 << 40, st_[k] if k < len(st_) else 1 << 40)
                if t_part >= uf[q]:
                    n_flag += len(ot) - k
                else:
                    n_bad += len(ot) - k
    e = np.concatenate(errs) if errs else np.zeros(1)
    acc = {"pixels": int(len(e)), "e_p": {"p50": float(np.percentile(e, 50)), "p99": float(np.percentile(e, 99)),
                                          "max": float(e.max())}, "e_p_bar": 1e-4,
           "packets": n_pk, "packets_identical": n_cmp, "packets_flagged": n_flag, "packets_differing": n_bad,
           "flagged_fraction": n_flag / max(n_pk, 1),
           "sample": "largest-current and random pixels of the largest, median and lower-quartile tiles of the "
                     f"headline run, oracle recomputed in {time.perf_counter() - t0:.1f} s"}
    return base, acc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", choices=("sorted", "atomic", "summed"), default="summed",
                    help="reduce mode of the headline spill (default: the exact sum-then-convolve form)")
    ap.add_argument("--spill-tiles", default="sorted,summed",
                    help="reduce modes to time on the spill as one plain call per tile (one pass each)")
    ap.add_argument("--module", default="sorted,atomic,summed", help="reduce modes timed on the module-scale event")
    ap.add_argument("--module-steps", type=int, default=3)
    ap.add_argument("--batched", type=int, default=64, help="batched-spill events (cfg3) per batching leg")
    ap.add_argument("--batched-modes", default="summed,sorted,tuned",
                    help="reduce modes of the batching legs; tuned = the autotuner's table applied per call")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner sweep (and the tuned legs)")
    ap.add_argument("--served-rates", default="50,200,2000", help="Poisson arrival rates (events/s) of the summed "
                                                                  "path's serving leg (64 spill-mix events each)")
    ap.add_argument("--served-sorted-rate", type=float, default=50.0,
                    help="arrival rate of the per-pair path's serving leg (32 events); 0 = skip")
    ap.add_argument("--no-light", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--err-pixels", type=int, default=96)
    ap.add_argument("--quick", action="store_true", help="only the headline")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer 5 times (the plain-copy reference that scales rocprofv3 "
                         "FETCH_SIZE / WRITE_SIZE readings to bytes) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 18                  # float32 elements
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": 4 * n, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (events and spill tiles shard "
              f"across GPUs with no exchange but the tile-edge halo, so a multi-GPU run is one such process per GPU)",
              file=sys.stderr)
        sys.exit(2)
    if args.quick:
        args.spill_tiles = args.module = args.batched_modes = args.served_rates = ""
        args.no_tune = True
        args.served_sorted_rate, args.no_light, args.no_cpu_baseline = 0.0, True, True

    import torch
    from paper_2212_09807_amd import ltsim, workloads as W

    line, (w5, h5) = headline(ltsim, W, args)
    torch.cuda.empty_cache()
    errors = {}

    def leg(name, fn, *a, **kw):
        """A secondary leg: its failure is recorded in the line (and logged), never the end of the run."""
        try:
            return fn(*a, **kw)
        except Exception as exc:                      # noqa: BLE001 -- reported, the headline stands
            log(f"{name} failed: {type(exc).__name__}: {exc}")
            errors[name] = f"{type(exc).__name__}: {exc}"
            return None
        finally:
            torch.cuda.synchronize()
            torch.cuda.empty_cache()

    for m in [x for x in args.spill_tiles.split(",") if x]:
        line.setdefault("spill_tile_calls", {})[m] = leg(f"spill_tiles_{m}", spill_tiles_leg, ltsim, W, m)
    mods = [x for x in args.module.split(",") if x]
    if mods:
        line["module_event"] = leg("module_event", module_leg, ltsim, W, mods, args.module_steps)
    table = None
    bmodes = [x for x in args.batched_modes.split(",") if x]
    if args.no_tune:
        bmodes = [m for m in bmodes if m != "tuned"]
    elif "tuned" in bmodes or args.served_rates:
        tuned = leg("tuning", tuning_leg, ltsim, W)
        if tuned is not None:
            table, line["tuning"] = tuned
        else:
            bmodes = [m for m in bmodes if m != "tuned"]
    for m in bmodes:
        line.setdefault("batched", {})[m] = leg(f"batched_{m}", batched_vs_plain, ltsim, W, args.batched, m,
                                                 table=table)
        if m != "tuned":
            line.setdefault("batched_small", {})[m] = leg(f"batched_small_{m}", batched_vs_plain, ltsim, W, 64, m,
                                                          cfg=1)
    rates = [float(r) for r in args.served_rates.split(",") if r]
    if rates:
        line["served"] = [leg(f"served_{r}", served, ltsim, W, r, 64, "summed") for r in rates]
        if table is not None:
            line["served"].append(leg("served_tuned", served, ltsim, W, rates[-1], 64, "tuned", table=table))
        line["served_small"] = leg("served_small", served_burst, ltsim, W, 64, "summed")
    if args.served_sorted_rate > 0:
        line.setdefault("served", []).append(leg("served_sorted", served, ltsim, W, args.served_sorted_rate, 32,
                                                 "sorted"))
    if not args.no_light:
        line["light"] = leg("light", light_leg, ltsim, W)
    if not args.no_cpu_baseline:
        cb = leg("cpu_baseline", cpu_baseline_leg, w5, h5, args.cpu_budget, args.err_pixels)
        line["cpu_baseline"], line["accuracy"] = cb if cb is not None else (None, None)
    if errors:
        line["leg_errors"] = errors
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
