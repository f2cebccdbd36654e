"""Pins of where the three front-end noise sources enter the oracle's electronics (Sec. 3.4; CPU only).

The paper names reset noise (the pedestal after each reset), discriminator noise (on the threshold comparison) and
uncorrelated noise (on the digitised sample).  Each test switches on one source, drives many pixels (independent
streams) with a constant current so every noiseless quantity is known in closed form, and checks the packets
against (a) the analytic distribution the placement implies (chi-square), and (b) draws computed outside the
oracle: rocRAND's Philox4x32-10 engine (an independent implementation of the generator, built on the host) at the
counters of the documented layout (pixel, tick, event low word, event high word << 4 | stream), turned into normals
by Box-Muller.  A draw keyed at the wrong tick or stream, noise left in the integrated charge, or a reset applied at
the wrong tick fails one of them.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from paper_2212_09807_amd import workloads as W

STREAM_DISC, STREAM_RESET, STREAM_SAMPLE = 0, 1, 2
TICK_INITIAL = 0xFFFFFFFF
SEED = 0x2212098070000005
EVENT = 0x1_0000_0007          # a high word too, so the stream field carries event bits
NPIX = 4000


@pytest.fixture(scope="module")
def rocrand_blocks(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc or the rocRAND headers are not installed")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_blocks")
    src = os.path.join(os.path.dirname(__file__), "rocrand_philox_blocks.cpp")
    subprocess.run([hipcc, "-O1", src, "-o", exe], check=True, capture_output=True, timeout=300)

    def blocks(pixel, tick, stream):
        pixel = np.asarray(pixel, np.uint64).ravel()
        tick = np.broadcast_to(np.asarray(tick, np.uint64), pixel.shape).ravel()
        c2 = EVENT & 0xFFFFFFFF
        c3 = ((EVENT >> 32) << 4) | stream
        k0, k1 = SEED & 0xFFFFFFFF, SEED >> 32
        lines = "\n".join(f"{p:x} {t:x} {c2:x} {c3:x} {k0:x} {k1:x}" for p, t in zip(pixel.tolist(), tick.tolist()))
        out = subprocess.run([exe], input=lines + "\n", check=True, capture_output=True, text=True,
                             timeout=300).stdout.split()
        return np.array([int(x, 16) for x in out], np.float64).reshape(-1, 4)

    return blocks


def normals(words):
    """Box-Muller on the first two words, u = (x + 1/2) 2^-32 (the documented transform), in FP64."""
    u0 = (words[:, 0] + 0.5) * 2.0 ** -32
    u1 = (words[:, 1] + 0.5) * 2.0 ** -32
    return np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)


def run(orc, el, current, n_ticks):
    ro = W.Readout(n_ticks=n_ticks)
    pix = np.arange(NPIX, dtype=np.int32)
    wave = np.broadcast_to(np.asarray(current, float)[None, :], (NPIX, n_ticks)).copy()
    pk, st = orc.electronics(el, ro, EVENT, pix, wave)
    return pk, st


def electronics(**kw):
    base = dict(threshold=5000.0, hold_ticks=16, min_spacing=11, q_lsb=1000.0, pedestal=0, adc_bits=8,
                sigma_reset=0.0, sigma_disc=0.0, sigma_unc=0.0, max_packets=64, seed=SEED, reset_period=0)
    base.update(kw)
    return W.Electronics(**base)


def chi2_pvalue(observed, expected_prob, min_expected=5.0):
    """Chi-square goodness of fit of integer counts to probabilities, adjacent bins merged to >= min_expected."""
    n = observed.sum()
    obs, exp, o_acc, e_acc = [], [], 0.0, 0.0
    for o, p in zip(observed, expected_prob):
        o_acc += o
        e_acc += n * p
        if e_acc >= min_expected:
            obs.append(o_acc)
            exp.append(e_acc)
            o_acc = e_acc = 0.0
    if e_acc > 0 and exp:
        obs[-1] += o_acc
        exp[-1] += e_acc
    obs, exp = np.array(obs), np.array(exp)
    chi2 = ((obs - exp) ** 2 / exp).sum()
    return stats.chi2.sf(chi2, len(obs) - 1)


def test_uncorrelated_noise_is_added_to_the_sample_only(orc, rocrand_blocks):
    """sigma_unc alone: with c = 250 e-/tick from tick 0 and threshold 5000 the crossings (ticks 19, 55, ...) and the
    samples (35, 71, ...) are noiseless, Q_s = 36 c = 9000 e- at every sample; the code is floor((Q_s + s g) / LSB)
    with g keyed at the sample tick."""
    c, T, sig = 250.0, 400, 500.0
    el = electronics(sigma_unc=sig)
    pk, _ = run(orc, el, np.full(T, c), T)
    exp_ticks = np.arange(35, T, 36)
    codes, ticks, pids = [], [], []
    for p, (t, a, f) in enumerate(pk):
        assert np.array_equal(t, exp_ticks), "the noiseless crossing / sample times moved"
        codes.append(a)
        ticks.append(t)
        pids.append(np.full(len(t), p))
    codes, ticks, pids = np.concatenate(codes), np.concatenate(ticks), np.concatenate(pids)
    # (a) distribution of the codes: Q_s + N(0, sig^2), floor over LSB
    k = np.arange(0, 20)
    prob = stats.norm.cdf(((k + 1) * 1000.0 - 9000.0) / sig) - stats.norm.cdf((k * 1000.0 - 9000.0) / sig)
    assert chi2_pvalue(np.bincount(codes, minlength=20)[:20], prob) > 1e-4
    # (b) every code from the draw at (pixel, sample tick, SAMPLE)
    g = normals(rocrand_blocks(pids, ticks, STREAM_SAMPLE))
    x = (9000.0 + sig * g) / 1000.0
    clear = np.abs(x - np.round(x)) > 1e-9
    assert np.array_equal(codes[clear], np.floor(x[clear]).astype(int))
    # the same check keyed at the crossing tick (or on the discriminator stream) does not hold: the pin discriminates
    g_cross = normals(rocrand_blocks(pids[:2000], ticks[:2000] - 16, STREAM_SAMPLE))
    assert np.mean(np.floor((9000.0 + sig * g_cross) / 1000.0) == codes[:2000]) < 0.6
    g_disc = normals(rocrand_blocks(pids[:2000], ticks[:2000], STREAM_DISC))
    assert np.mean(np.floor((9000.0 + sig * g_disc) / 1000.0) == codes[:2000]) < 0.6


def test_discriminator_noise_enters_the_comparison_only(orc, rocrand_blocks):
    """sigma_disc alone, c = 100 e-/tick from tick 0: a crossing at tick n happens with probability
    p_n = Phi((Q_n - thr) / s), Q_n = (n + 1) c, independently per tick, so the first crossing has the distribution
    prod_{m<n} (1 - p_m) p_n; the integrated charge keeps no discriminator draw, so every code is
    floor(Q_s / LSB) exactly, Q_s = (n_s - n_start + 1) c."""
    c, T, sig, thr, lsb, h = 100.0, 600, 650.0, 5000.0, 7.0, 16
    el = electronics(sigma_disc=sig, q_lsb=lsb, adc_bits=16)
    pk, _ = run(orc, el, np.full(T, c), T)
    first = np.array([t[0] - h for t, _, _ in pk])
    # (a) every code equals the noiseless integral since the previous sample
    for t, a, f in pk:
        start = np.r_[0, t[:-1] + 1]
        assert np.array_equal(a, np.floor((t - start + 1) * c / lsb).astype(int))
    # (b) first-crossing distribution: independent draws per compared tick
    n = np.arange(0, 120)
    p = stats.norm.cdf(((n + 1) * c - thr) / sig)
    surv = np.r_[1.0, np.cumprod(1.0 - p)[:-1]]
    prob = surv * p
    assert first.max() < 120
    obs = np.bincount(first, minlength=120)[:120]
    assert chi2_pvalue(obs, prob) > 1e-4
    # one draw reused for every tick would give P(first = n) = p_n - p_{n-1}; the data reject it
    alt = np.diff(np.r_[0.0, p])
    assert chi2_pvalue(obs, alt) < 1e-8
    # (c) the first crossing recomputed from the draws at (pixel, tick, DISC) for every compared tick
    ticks = np.arange(0, 120)
    g = normals(rocrand_blocks(np.repeat(np.arange(NPIX), len(ticks)), np.tile(ticks, NPIX), STREAM_DISC))
    m = (ticks[None, :] + 1) * c + sig * g.reshape(NPIX, len(ticks)) - thr
    exp_first = np.argmax(m >= 0.0, axis=1)
    clear = np.all(np.abs(m) > 1e-9, axis=1)
    assert np.array_equal(first[clear], exp_first[clear])


def test_reset_noise_is_the_pedestal_from_the_tick_after_each_sample(orc, rocrand_blocks):
    """sigma_reset alone, c = 300 e-/tick from tick 0, LSB = 1 e-: the integrator starts at P_0 (drawn once, tick
    field 0xFFFFFFFF) and restarts at P_k (drawn at the sample tick) from the tick after each sample, so a packet at
    n_s after a restart at n_start has code floor(P + (n_s - n_start + 1) c) and floor(P) = code - (n_s - n_start + 1) c
    is the floor of an N(0, s^2) pedestal: mean 0 (charge of the sample tick counted twice would shift it by c)."""
    c, T, sig, thr, h = 300.0, 300, 900.0, 5000.0, 16
    el = electronics(sigma_reset=sig, q_lsb=1.0, adc_bits=16)
    pk, _ = run(orc, el, np.full(T, c), T)
    ped0, ped1, prev_tick, first_cross = [], [], [], []
    for t, a, f in pk:
        assert len(t) >= 2
        ped0.append(a[0] - (t[0] + 1) * c)
        ped1.append(a[1] - (t[1] - t[0]) * c)
        prev_tick.append(t[0])
        first_cross.append(t[0] - h)
    ped0, ped1 = np.array(ped0), np.array(ped1)
    for ped in (ped0, ped1):
        # (a) floor(P) distribution of an N(0, s^2) pedestal, in 300 e- bins
        edges = np.arange(-6000.0, 6001.0, 300.0)
        obs = np.histogram(ped, bins=edges)[0]
        prob = np.diff(stats.norm.cdf(edges / sig))
        assert chi2_pvalue(obs, prob) > 1e-4
        assert abs(ped.mean() + 0.5) < 4.0 * sig / math.sqrt(NPIX)
    # (b) the pedestals from the draws: tick field 0xFFFFFFFF before the first sample, the sample tick afterwards
    g0 = normals(rocrand_blocks(np.arange(NPIX), TICK_INITIAL, STREAM_RESET))
    g1 = normals(rocrand_blocks(np.arange(NPIX), np.array(prev_tick), STREAM_RESET))
    for ped, g in ((ped0, g0), (ped1, g1)):
        x = sig * g
        clear = np.abs(x - np.round(x)) > 1e-9
        assert np.array_equal(ped[clear], np.floor(x[clear]))
    # (c) the first crossing is where P_0 + (n + 1) c reaches the threshold
    n = np.arange(T)
    exp_cross = np.argmax(sig * g0[:, None] + (n[None, :] + 1) * c >= thr, axis=1)
    assert np.array_equal(np.array(first_cross), exp_cross)
