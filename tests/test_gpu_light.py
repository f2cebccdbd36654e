"""Light path (Sec. 4.2, 4.3) on the device vs the FP64 oracle, through the C ABI (needs an MI355X).

Bars: the scintillated means agree to 1e-12 (FP64 on both sides); photoelectron counts are identical except where
the oracle flags a uniform within 1e-12 of a cumulative Poisson value (none expected) and, in the normal regime,
agree to 1e-12; waveforms per detector to 1e-4 relative L2 (FP32 response and noise); trigger ticks identical
before any decision the oracle flags as within FP32 reach of the threshold.
"""
import dataclasses

import numpy as np
import pytest

from paper_2212_09807_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible MI355X"
    return t


@pytest.fixture(scope="module")
def lt(torch):
    from paper_2212_09807_amd import ltsim
    ltsim.lib()
    return ltsim


@pytest.fixture(scope="module")
def OL(orc):
    import oracle.light as light
    return light


def check(lt, OL, torch, lp, ipe, r, amp, event_id):
    ref = OL.simulate(lp, event_id, ipe, r, amp)
    sim = lt.LightSim(lp, r, amp)
    out = sim.simulate(torch.from_numpy(np.ascontiguousarray(ipe, np.float32)).cuda(), event_id, keep_mu=True,
                       keep_pe=True)
    torch.cuda.synchronize()
    mu, pe, V = out["mu"].cpu().numpy(), out["pe"].cpu().numpy(), out["V"].cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(mu, ref["mu"], rtol=1e-12, atol=1e-300)
    near = ref["near"] != 0
    normal = ref["mu"] > lp.normal_above
    poisson = ~normal & ~near
    assert np.array_equal(pe[poisson], ref["n"][poisson])
    np.testing.assert_allclose(pe[normal], ref["n"][normal], rtol=1e-12)
    bad_det = np.unique(np.nonzero(near)[0])
    e = np.sqrt(((V - ref["V"]) ** 2).sum(1)) / np.maximum(np.sqrt((ref["V"] ** 2).sum(1)), 1.0)
    keep = np.setdiff1d(np.arange(lp.n_det), bad_det)
    assert e[keep].max() <= 1e-4, e.max()
    cnt, trig = out["trig_count"].cpu().numpy(), out["trig"].cpu().numpy()
    for g, (tr, u) in enumerate(zip(ref["triggers"], ref["trigger_uncertain_from"])):
        if any(lp.group * g <= d < lp.group * (g + 1) for d in bad_det):
            continue
        got = trig[g, :cnt[g]]
        assert got[got < u].tolist() == tr[tr < u].tolist(), (g, got, tr, u)
        assert np.all(trig[g, cnt[g]:] == -1)
    sim.close()
    return ref, e, cnt


def test_light_spill_parity(lt, OL, torch):
    lp, ipe, r, amp = W.light_workload()
    ref, e, cnt = check(lt, OL, torch, lp, ipe, r, amp, 7)
    print(f"light spill: {lp.n_det} detectors x {lp.n_ticks} ticks, normal-regime ticks "
          f"{int((ref['mu'] > lp.normal_above).sum())}, max V error {e.max():.2e}, triggers {cnt.tolist()}")
    assert cnt.sum() > 0


def test_light_ragged_and_degenerate_shapes(lt, OL, torch):
    """A window shorter than the scintillation kernel and not a multiple of 8 ticks, no noise, single-detector groups,
    no trigger slots; then one with a trigger cap."""
    rng = np.random.default_rng(3)
    lp = dataclasses.replace(W.Light(), n_det=5, n_ticks=1003, group=1, max_trig=0)
    ipe = np.zeros((5, 1003), np.float32)
    ipe[:, rng.integers(0, 1003, 40)] = rng.uniform(0, 400, 40).astype(np.float32)
    check(lt, OL, torch, lp, ipe, W.light_response(n_resp=77), np.zeros(0, np.float32), 99)
    lp2 = dataclasses.replace(lp, max_trig=2, trig_threshold=20.0, trig_deadtime=50)
    check(lt, OL, torch, lp2, ipe, W.light_response(n_resp=77), W.light_noise_amplitudes(n_freq=300, sigma=1.0), 100)


def test_light_invalid_parameters(lt, torch):
    lp = W.Light()
    r, a = W.light_response(), W.light_noise_amplitudes()
    for bad in (dataclasses.replace(lp, group=7), dataclasses.replace(lp, tau_s=0.0),
                dataclasses.replace(lp, trig_deadtime=0)):
        with pytest.raises(lt.LtsimError):
            lt.LightSim(bad, r, a)
    with pytest.raises(lt.LtsimError):
        lt.LightSim(dataclasses.replace(lp, n_ticks=64), r, a)            # n_freq >= n_ticks / 2


def test_light_graph_replay_equals_eager(lt, torch):
    """The HIP-graph replay of the light kernels gives the eager results bit for bit, replay after replay with
    eager calls and host synchronisation between them, for several event ids, and again after the output buffers
    change (a new capture)."""
    lp, ipe, r, amp = W.light_workload(n_events=2, light=dataclasses.replace(W.Light(), n_det=16, n_ticks=8192))
    x = torch.from_numpy(np.ascontiguousarray(ipe, np.float32)).cuda()
    eager = lt.LightSim(lp, r, amp)
    graph = lt.LightSim(lp, r, amp)
    graph.set_graph(True)
    out = None
    for rep, ev in enumerate([5, 6, 5, 9, 6]):
        a = eager.simulate(x, ev, keep_pe=True)
        out = graph.simulate(x, ev, keep_pe=True, out=out)
        torch.cuda.synchronize()
        for k in ("V", "pe", "trig", "trig_count"):
            assert torch.equal(a[k], out[k]), (rep, ev, k)
    # back to back without host synchronisation: each launch's result is copied in stream order before the next
    # call re-parameterises a graph instance, and every copy must hold its own event's result
    evs = [11, 12, 13, 14, 15]
    copies = []
    for ev in evs:
        out = graph.simulate(x, ev, keep_pe=True, out=out)
        copies.append((out["V"].clone(), out["trig"].clone()))
    torch.cuda.synchronize()
    for ev, (v, t) in zip(evs, copies):
        a = eager.simulate(x, ev, keep_pe=True)
        torch.cuda.synchronize()
        assert torch.equal(a["V"], v) and torch.equal(a["trig"], t), ev
    b = graph.simulate(x, 7, keep_pe=True)                 # new buffers: captured again
    c = eager.simulate(x, 7, keep_pe=True)
    torch.cuda.synchronize()
    assert torch.equal(b["V"], c["V"]) and torch.equal(b["trig"], c["trig"])
    assert not torch.equal(b["V"], out["V"])                # a different event draws differently
