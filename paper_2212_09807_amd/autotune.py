"""Project autotuner of the induction stage's work split, per event-size class.

The knobs are the library's work-split settings (lts_set_tuning applies one table entry per call, chosen by the
call's mean segments per event, in lts_simulate, lts_simulate_batch and every batch of a server):

* reduce mode, which fixes the unit of work: per-pair pixel-major with Kahan sums (one workgroup per active pixel,
  its pairs in segment order), per-pair segment-major with FP32 atomics (one workgroup per segment, its pairs in
  pixel order), or sum-then-convolve (one wavefront per (active pixel, 512-tick tile) unit over the pixel's column
  pieces);
* tick tile (ticks per thread: 0 = automatic, 1, 2, 4, 8): the per-pair kernels' output ticks per thread; in the
  summed mode 0 runs the 256-tick LDS-staged wavefront kernel, 8 the 512-tick register one, and 1, 2 or 4 the
  pixel-per-workgroup kernel over the pieces;
* induce slices (sorted mode: workgroups per pixel, one table slice each) and lane exchange (table windows shared
  across lanes).

For every size class a few seeded events of that size (the module-event generator, the content of the batched-spill
mix) run as one batch per candidate, timed with the library's stage events after an untimed warm-up; the fastest
candidate whose currents agree with the deterministic sorted reference to 1e-5 (per-pixel relative L2) wins the
class.  Results are cached in a JSON file keyed by the readout and table shape.
"""
from __future__ import annotations

import json
import os
from dataclasses import asdict, dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import ltsim
from . import workloads as W


@dataclass(frozen=True)
class Choice:
    reduce_mode: int = ltsim.LTS_REDUCE_SORTED
    slices: int = 1
    ticks_per_thread: int = 0
    lane_exchange: int = 0

    def apply(self, ctx: "ltsim.Context"):
        ctx.set_reduce_mode(self.reduce_mode)
        ctx.set_induce_slices(self.slices)
        ctx.set_ticks_per_thread(self.ticks_per_thread)
        ctx.set_lane_exchange(self.lane_exchange)


S, A, M = ltsim.LTS_REDUCE_SORTED, ltsim.LTS_REDUCE_ATOMIC, ltsim.LTS_REDUCE_SUMMED
DEFAULT_CANDIDATES = (Choice(S, 1, 0), Choice(S, 1, 4), Choice(S, 8, 0), Choice(A, 1, 0), Choice(M, 1, 0),
                      Choice(M, 1, 8), Choice(M, 1, 4))
DEFAULT_SIZES = (500, 2000, 8000, 32000)
ACCEPT_REL_L2 = 1e-4


def shape_key(w) -> str:
    ro, tb = w.readout, w.table
    return f"{ro.n_x}x{ro.n_y}x{ro.n_ticks}_t{tb.t_r}x{tb.b_x}x{tb.b_y}"


def class_events(w, n_segments: int, n_events: int, seed: int = 0) -> List:
    """n_events seeded events of about n_segments segments with the workload's geometry: module-event content for
    the 140 x 140-pixel readout, single straight tracks for the 70 x 70 one."""
    rng = np.random.default_rng([2212, 9807, 77, n_segments, seed])
    if w.readout.n_x == W.TILE_PIXELS_MODULE0:
        return [W._cfg1_event(rng) for _ in range(n_events)]
    return [W._cfg2_event(rng, n_segments) for _ in range(n_events)]


def _time_batch(ctx, dsegs, offs, ids, out):
    import torch
    ctx.simulate_batch(dsegs, offs, ids, out=out)              # warm-up: this choice's allocations
    torch.cuda.synchronize()
    ctx.get_timing()
    ctx.set_timing(True)
    ctx.simulate_batch(dsegs, offs, ids, out=out)
    torch.cuda.synchronize()
    t = ctx.get_timing()
    ctx.set_timing(False)
    ms = sum(v[0] for k, v in t.items() if k != "induce_kernel")
    h = out.host()
    return ms, h


def autotune(w, sizes: Sequence[int] = DEFAULT_SIZES, candidates: Sequence[Choice] = DEFAULT_CANDIDATES,
             events_per_class: int = 3, cache: Optional[str] = None, verbose: bool = False) -> Dict:
    """Time every candidate on every size class; returns {"key", "table": [[min_segments, mode, slices, rt,
    exchange], ...], "classes": per-class timings}.  The table's first entry applies below its size too."""
    key = shape_key(w) + "_" + "-".join(str(s) for s in sizes) + f"_{events_per_class}"
    if cache and os.path.exists(cache):
        db = json.load(open(cache))
        if key in db:
            return db[key]
    ctx = ltsim.Context.from_workload(w)
    classes, table = [], []
    for n in sizes:
        evs = class_events(w, n, events_per_class)
        allsegs = W.Segments.concat(evs)
        offs = np.r_[0, np.cumsum([e.n for e in evs])]
        ids = list(range(1000 * n, 1000 * n + len(evs)))
        dsegs = ltsim.to_device(allsegs)
        Choice().apply(ctx)
        cap = sum(ctx.plan(ltsim.to_device(e))["pixels"] for e in evs)
        out = ctx._alloc(cap, cap * w.electronics.max_packets, len(evs), True)
        _, ref = _time_batch(ctx, dsegs, offs, ids, out)
        rows = []
        for c in candidates:
            c.apply(ctx)
            ms, h = _time_batch(ctx, dsegs, offs, ids, out)
            if not np.array_equal(h["pixel_id"], ref["pixel_id"]):
                err = np.inf
            else:
                g, o = h["current"].astype(np.float64), ref["current"].astype(np.float64)
                e = np.sqrt(((g - o) ** 2).sum(1)) / np.maximum(np.sqrt((o ** 2).sum(1)), 10.0)
                err = float(e.max()) if e.size else 0.0
            rows.append({"choice": asdict(c), "ms": ms, "max_rel_l2_vs_sorted": err})
            if verbose:
                print(f"[autotune] {n} segments/event {asdict(c)}: {ms:.2f} ms, err {err:.1e}", flush=True)
        best = min((r for r in rows if r["max_rel_l2_vs_sorted"] <= ACCEPT_REL_L2), key=lambda r: r["ms"])
        b = best["choice"]
        # a class's entry starts at the geometric midpoint between its size and the previous class's
        lo = 0 if not table else int(np.sqrt(float(sizes[len(table) - 1]) * n))
        table.append([lo, b["reduce_mode"], b["slices"], b["ticks_per_thread"], b["lane_exchange"]])
        classes.append({"segments_per_event": int(n), "events": len(evs), "best": best, "all": rows})
    ctx.close()
    res = {"key": key, "table": table, "classes": classes}
    if cache:
        db = json.load(open(cache)) if os.path.exists(cache) else {}
        db[key] = res
        json.dump(db, open(cache, "w"), indent=1)
    return res
