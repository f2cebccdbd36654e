"""Full-size parity through the C ABI: every active pixel and every packet of the module-scale event (20,000
segments, 3000 ticks), of one large-spill tile (13,639 segments with its halo replicas, 5000 ticks, reset /
discriminator / sample noise 900 / 650 / 500 e-) and of the largest of the first eight events of the batched-spill
mix (46,448 segments), against the FP64 oracle computed at test time (minutes on the host cores; progress is
printed), in the launch configurations the benchmark times.  Also: batch = single and served = alone, bit for bit,
on those eight spill-mix events.

Bars: per-pixel e_p = ||I_gpu - I_orc||_2 / max(||I_orc||_2, 10 e-) <= 1e-4 on every pixel; packet ticks and ADC
codes identical, except that a pixel's GPU timeline may part from the oracle's at a threshold decision the oracle
finds within the FP32 error margin, and an ADC code may differ where the oracle's sample lies within that margin of
an LSB boundary; such flagged packets (every oracle packet from a parting on, and the differing codes) < 0.1 % of all
packets; the FP64 charge report within the FP32 accumulation error.
"""
import time

import numpy as np
import pytest

from paper_2212_09807_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_WAVE = 1e-4
FLAG_BAR = 1e-3
EPS_REL, EPS_ABS = 2e-6, 0.1
_ORACLE = {}


@pytest.fixture(scope="module")
def lt():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_2212_09807_amd import ltsim
    ltsim.lib()
    return ltsim


def _workload(name):
    if name == "module":
        return W.make_workload(2), 0
    if name == "spill-tile":
        return W.make_workload(5), 8                # 13,639 segments, cosmic muons and halo replicas
    w = W.make_workload(3, n_events=8)
    return w, int(np.argmax([e.n for e in w.events]))


def oracle_event(orc, name, say, chunk=1024):
    """All active pixels of the event through the oracle (waveforms in pixel chunks, then the front end), cached
    for the other tests of the module."""
    if name in _ORACLE:
        return _ORACLE[name]
    w, ev = _workload(name)
    segs = w.events[ev]
    table = W.response_table(w.table, w.readout, w.physics.v_drift)
    t0 = time.perf_counter()
    pix = orc.active_pixels(w.physics, w.readout, w.table, segs)
    waves, clips = [], []
    sums = None
    for k in range(0, len(pix), chunk):
        if k == 0:
            wv, cl, sums = orc.waveforms(w.physics, w.readout, table, segs, pix[k:k + chunk], with_sums=True)
        else:
            wv, cl = orc.waveforms(w.physics, w.readout, table, segs, pix[k:k + chunk])
        waves.append(wv)
        clips.append(cl)
        say(f"[oracle {name}] {min(k + chunk, len(pix))}/{len(pix)} pixels, {time.perf_counter() - t0:.0f} s")
    wave = np.concatenate(waves) if waves else np.zeros((0, w.readout.n_ticks))
    pk, st, uf = orc.electronics(w.electronics, w.readout, w.event_ids[ev], pix, wave, EPS_REL, EPS_ABS,
                                 with_uncertain=True)
    rep = {"q_after_quench": sums[0], "q_collected": sums[1], "q_induced": float(wave.sum()),
           "q_clipped": float(np.concatenate(clips).sum()), "q_offgrid": sums[2]}
    say(f"[oracle {name}] {segs.n} segments, {len(pix)} pixels done in {time.perf_counter() - t0:.0f} s")
    _ORACLE[name] = (w, ev, pix, wave, pk, st, uf, rep)
    return _ORACLE[name]


def _packets_by_pixel(h):
    out = {}
    for p, t, a, f in zip(h["pkt_pixel"], h["pkt_tick"], h["pkt_adc"], h["pkt_flags"]):
        out.setdefault(int(p), []).append((int(t), int(a)))
    return out


def compare_timelines(ot, oa, of, uf, gt, ga):
    """One pixel's packets: the oracle's (ticks ot, codes oa, flags of, first uncertain threshold decision at tick uf)
    against the GPU's (gt, ga).  Packets must agree in tick and ADC code; a code may differ only where the oracle
    flags its sample within the FP32 margin of an LSB boundary (of & 1), and the timelines may part only at or after
    a threshold decision the oracle found within the FP32 margin (tick >= uf).  Returns (identical packets, oracle
    packets that differ legitimately: codes at an LSB boundary and every packet from a parting on, ok)."""
    n, m = len(ot), len(gt)
    k = 0
    while k < min(n, m) and ot[k] == gt[k] and (oa[k] == ga[k] or (of[k] & 1)):
        k += 1
    ident = int(np.sum(oa[:k] == ga[:k]))
    flagged = k - ident
    if k == n and k == m:
        return ident, flagged, True
    t_part = min(ot[k] if k < n else np.iinfo(np.int64).max, gt[k] if k < m else np.iinfo(np.int64).max)
    return ident, flagged + (n - k), bool(t_part >= uf)


def compare_all(orc, h, w, ev, pix, wave, pk, uf, rep):
    """Every pixel and packet of one event; returns the statistics printed by the tests."""
    gpix = h["pixel_id"]
    assert np.all(np.diff(gpix) > 0)
    pos = np.searchsorted(gpix, pix)
    assert np.all(pos < len(gpix)) and np.array_equal(gpix[pos], pix), "oracle pixels missing on the GPU"
    extra = np.setdiff1d(np.arange(len(gpix)), pos)
    assert np.all(h["current"][extra] == 0.0), "pixels only the GPU lists carry current"
    g = h["current"][pos].astype(np.float64)
    e = np.sqrt(((g - wave) ** 2).sum(1)) / np.maximum(np.sqrt((wave ** 2).sum(1)), 10.0)
    # pixels only the GPU lists (table reach meets a charge box, zero current) still see noise: their packets too
    ex_pix = gpix[extra]
    ex_pk, _, ex_uf = orc.electronics(w.electronics, w.readout, w.event_ids[ev], ex_pix,
                                      np.zeros((len(ex_pix), w.readout.n_ticks)), EPS_REL, EPS_ABS,
                                      with_uncertain=True)
    gb = _packets_by_pixel(h)
    total = identical = flagged = at_risk = 0
    bad = []
    for plist, pks, ufs in ((pix, pk, uf), (ex_pix, ex_pk, ex_uf)):
        for q, p in enumerate(plist):
            ot, oa, of = pks[q]
            gl = gb.get(int(p), [])
            gt = np.array([x[0] for x in gl], np.int64)
            ga = np.array([x[1] for x in gl], np.int64)
            total += len(ot)
            at_risk += int((ot >= ufs[q]).sum() + ((of[ot < ufs[q]] & 1) != 0).sum())
            ident, flg, ok = compare_timelines(ot, oa, of, int(ufs[q]), gt, ga)
            identical += ident
            flagged += flg
            if not ok:
                bad.append((int(p), ot.tolist()[:8], oa.tolist()[:8], gt.tolist()[:8], ga.tolist()[:8], int(ufs[q])))
    n_gpu_pk = len(h["pkt_tick"])
    r = h["report"][0]
    scale = rep["q_collected"]
    stats = {"pixels": len(pix), "gpu_only_pixels": len(ex_pix), "e_p_p50": float(np.percentile(e, 50)),
             "e_p_p99": float(np.percentile(e, 99)), "e_p_max": float(e.max()), "packets": total,
             "gpu_packets": n_gpu_pk, "identical": identical, "flagged": flagged, "flagged_fraction": flagged / max(total, 1),
             "within_margin": at_risk,
             "mismatches": len(bad), "report_rel": [abs(r[0] / rep["q_after_quench"] - 1), abs(r[1] / scale - 1),
                                                    abs(r[2] - rep["q_induced"]) / scale,
                                                    abs(r[3] - rep["q_clipped"]) / scale,
                                                    abs(r[4] - rep["q_offgrid"]) / scale]}
    assert not bad, bad[:5]
    assert e.max() <= TOL_WAVE, (e.max(), pix[np.argmax(e)])
    assert stats["flagged_fraction"] < FLAG_BAR, stats
    assert r[0] == pytest.approx(rep["q_after_quench"], rel=2e-6)
    assert r[1] == pytest.approx(rep["q_collected"], rel=2e-6)
    assert r[2] == pytest.approx(rep["q_induced"], abs=1e-5 * scale)
    assert r[3] == pytest.approx(rep["q_clipped"], abs=1e-5 * scale)
    assert r[4] == pytest.approx(rep["q_offgrid"], abs=1e-5 * scale)
    return stats


@pytest.mark.parametrize("name,mode", [("module", 2), ("module", 0), ("spill-tile", 2), ("spill-tile", 0),
                                       ("spill-mix-largest", 2), ("spill-mix-largest", 0)])
def test_every_pixel_and_packet(lt, orc, capsys, name, mode):
    def say(msg):
        with capsys.disabled():
            print(msg, flush=True)
    w, ev, pix, wave, pk, st, uf, rep = oracle_event(orc, name, say)
    ctx = lt.Context.from_workload(w, reduce_mode=mode)
    h = ctx.simulate(lt.to_device(w.events[ev]), event_id=w.event_ids[ev]).host()
    ctx.close()
    s = compare_all(orc, h, w, ev, pix, wave, pk, uf, rep)
    say(f"[full {name} mode={mode}] pixels {s['pixels']} (+{s['gpu_only_pixels']} GPU-only, zero current), "
        f"e_p p50 {s['e_p_p50']:.2e} p99 {s['e_p_p99']:.2e} max {s['e_p_max']:.2e}; packets {s['packets']} "
        f"identical {s['identical']} flagged {s['flagged']} ({100 * s['flagged_fraction']:.3f} %; "
        f"{s['within_margin']} within the FP32 margin); "
        f"report rel {['%.1e' % x for x in s['report_rel']]}")


_SINGLES = {}


def _spill_mix_singles(lt, mode):
    if mode not in _SINGLES:
        w = W.make_workload(3, n_events=8)
        ctx = lt.Context.from_workload(w, reduce_mode=mode)
        _SINGLES[mode] = (w, [ctx.simulate(lt.to_device(s), event_id=i).host() for s, i in zip(w.events, w.event_ids)])
        ctx.close()
    return _SINGLES[mode]


@pytest.mark.parametrize("mode", [2, 0])
def test_spill_mix_batch_equals_single(lt, mode):
    """The first eight events of the batched-spill mix (500 to 46,448 segments) in one lts_simulate_batch call give
    each event's single-call pixels, currents, packets, counts and report bit for bit."""
    w, singles = _spill_mix_singles(lt, mode)
    ctx = lt.Context.from_workload(w, reduce_mode=mode)
    offs = np.r_[0, np.cumsum([s.n for s in w.events])]
    cap = sum(int(s["counts"][0]) for s in singles)
    out = ctx._alloc(cap, cap * w.electronics.max_packets // 4 + 4096, len(w.events), True)
    b = ctx.simulate_batch(lt.to_device(W.Segments.concat(w.events)), offs, w.event_ids, out=out).host()
    ctx.close()
    po, ko = b["event_pixel_offsets"], b["event_packet_offsets"]
    for e, s in enumerate(singles):
        for k in ("pixel_id", "current"):
            assert np.array_equal(b[k][po[e]:po[e + 1]], s[k]), (e, k)
        for k in ("pkt_pixel", "pkt_tick", "pkt_adc", "pkt_flags"):
            assert np.array_equal(b[k][ko[e]:ko[e + 1]], s[k]), (e, k)
        np.testing.assert_allclose(b["report"][e], s["report"][0], rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("mode", [2, 0])
def test_spill_mix_served_equals_alone(lt, mode):
    """The same eight spill-mix events through the request loop (host segments in, continuous batching over two
    lanes, several events per batch) give each event's single-call results bit for bit, counts included."""
    w, singles = _spill_mix_singles(lt, mode)
    ctx = lt.Context.from_workload(w, reduce_mode=mode)
    srv = lt.Server(ctx, n_lanes=2, max_batch_events=4, return_currents=True)
    try:
        tickets = [srv.submit(s, i) for s, i in zip(w.events, w.event_ids)]
        got = [srv.wait(t, 300.0) for t in tickets]
        for t in tickets:
            srv.release(t)
    finally:
        srv.stop()
        ctx.close()
    assert max(g["batch_events"] for g in got) > 1
    for e, (a, g) in enumerate(zip(singles, got)):
        assert g["status"] == 0
        for k in ("pixel_id", "current", "pkt_pixel", "pkt_tick", "pkt_adc", "pkt_flags", "counts"):
            assert np.array_equal(a[k], g[k]), (e, k)
        np.testing.assert_allclose(a["report"][0], g["report"], rtol=1e-12, atol=1e-9)
