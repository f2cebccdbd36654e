"""FP64 oracle of the light simulation on given photocurrents (arXiv 2212.09807, Sec. 4.2 and 4.3).

TEST INFRASTRUCTURE ONLY (imported by tests/, the smoke check and the benchmark's CPU leg).  The scintillation
convolution, the photoelectron statistics and the noise phases are C functions of ``oracle.c``; the electronics
response (a convolution, ``numpy.convolve``), the random-phase noise (a real inverse FFT, ``numpy.fft.irfft``) and the
trigger scan are written here in NumPy, step by step as the paper states them:

  1. mu[d, t] = sum_{k=0}^{5 tau_s / dt} I_pe[d, t - k] f_scint(k dt) dt   (truncated direct convolution)
  2. n[d, t] ~ Poisson(mu) by inverse transform sampling, or mu + sqrt(mu) g above 30 p.e.
  3. V[d, t] = noise[d, t] + G sum_k n[d, t - k] r[k],  noise[d, t] = sum_f A_f cos(2 pi f t / T + phi_{d,f})
  4. triggers: per group of detectors, the first tick where the group sum of V reaches the threshold, then again
     after the dead time.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lib as _orc_lib, _ptr

_FP = C.POINTER(C.c_float)


class _LightParams(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("tick", "tau_p", "tau_s", "f_prompt", "trunc", "gain", "normal_above")] + [
        ("n_det", C.c_int32), ("n_ticks", C.c_int32), ("seed", C.c_uint64)]


def _params(light):
    return _LightParams(light.tick, light.tau_p, light.tau_s, light.f_prompt, light.trunc, light.gain,
                        light.normal_above, light.n_det, light.n_ticks, light.seed)


_READY = False


def _lib():
    global _READY
    L = _orc_lib()
    if not _READY:
        L.orc_light_taps.argtypes = [C.POINTER(_LightParams)]
        L.orc_light_taps.restype = C.c_int32
        L.orc_light_scint.argtypes = [C.POINTER(_LightParams), _FP, C.POINTER(C.c_double)]
        L.orc_light_scint.restype = None
        L.orc_light_fluct.argtypes = [C.POINTER(_LightParams), C.c_uint64, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.orc_light_fluct.restype = None
        L.orc_light_noise_phases.argtypes = [C.POINTER(_LightParams), C.c_uint64, C.c_int32, C.POINTER(C.c_double)]
        L.orc_light_noise_phases.restype = None
        _READY = True
    return L


def taps(light) -> int:
    return int(_lib().orc_light_taps(C.byref(_params(light))))


def scint(light, ipe) -> np.ndarray:
    """Step 1: expected photoelectrons per tick after scintillation, [n_det, n_ticks] FP64."""
    ipe = np.ascontiguousarray(ipe, dtype=np.float32).reshape(light.n_det, light.n_ticks)
    mu = np.zeros((light.n_det, light.n_ticks))
    _lib().orc_light_scint(C.byref(_params(light)), ipe.ctypes.data_as(_FP), _ptr(mu))
    return mu


def fluct(light, event_id, mu):
    """Step 2: photoelectron counts (FP64; integers below the normal threshold) and the near-decision flags."""
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    n = np.zeros_like(mu)
    near = np.zeros(mu.shape, np.int32)
    _lib().orc_light_fluct(C.byref(_params(light)), event_id, _ptr(mu), _ptr(n), _ptr(near, C.c_int32))
    return n, near


def noise(light, event_id, amp) -> np.ndarray:
    """Random-phase sinusoids: noise[d, t] = sum_{f=1}^{F} A_f cos(2 pi f t / T + phi_{d,f}), via a real inverse FFT
    (numpy's irfft of X_f = (T / 2) A_f exp(i phi) returns exactly that sum for f < T / 2)."""
    amp = np.asarray(amp, dtype=np.float64)
    F, T = len(amp), light.n_ticks
    assert F < T // 2
    phi = np.zeros((light.n_det, F))
    _lib().orc_light_noise_phases(C.byref(_params(light)), event_id, F, _ptr(phi))
    X = np.zeros((light.n_det, T // 2 + 1), np.complex128)
    X[:, 1:F + 1] = (T / 2.0) * amp[None, :] * np.exp(1j * phi)
    return np.fft.irfft(X, n=T, axis=1)


def noise_phases(light, event_id, n_freq) -> np.ndarray:
    phi = np.zeros((light.n_det, n_freq))
    _lib().orc_light_noise_phases(C.byref(_params(light)), event_id, n_freq, _ptr(phi))
    return phi


def response(light, n, resp) -> np.ndarray:
    """Step 3 without noise: G * sum_{k} n[d, t - k] r[k], causal, cut to the window."""
    r = np.asarray(resp, dtype=np.float64)
    T = light.n_ticks
    return np.stack([light.gain * np.convolve(n[d], r)[:T] for d in range(light.n_det)])


def triggers(light, V, eps_abs=1e-3, eps_rel=1e-5, with_uncertain=False):
    """Step 4: per group of `group` consecutive detectors, ticks where the summed waveform reaches the threshold,
    scanning in time and skipping `trig_deadtime` ticks after each trigger; at most `max_trig` per group.  With
    with_uncertain, also per group the first tick whose decision compared a sum within eps_abs + eps_rel * |sum| of
    the threshold (an FP32 evaluation of the sum may decide it the other way; n_ticks if none)."""
    out, unc = [], []
    for g in range(light.n_det // light.group):
        s = V[g * light.group:(g + 1) * light.group].sum(axis=0)
        trig, t, u = [], 0, light.n_ticks
        while t < light.n_ticks and len(trig) < light.max_trig:
            if u == light.n_ticks and abs(s[t] - light.trig_threshold) < eps_abs + eps_rel * abs(s[t]):
                u = t
            if s[t] >= light.trig_threshold:
                trig.append(t)
                t += light.trig_deadtime
            else:
                t += 1
        out.append(np.array(trig, np.int64))
        unc.append(u)
    return (out, np.array(unc, np.int64)) if with_uncertain else out


def simulate(light, event_id, ipe, resp, amp):
    """The whole light path for one event."""
    mu = scint(light, ipe)
    n, near = fluct(light, event_id, mu)
    V = response(light, n, resp) + (noise(light, event_id, amp) if len(amp) else 0.0)
    trig, unc = triggers(light, V, with_uncertain=True)
    return {"mu": mu, "n": n, "near": near, "V": V, "triggers": trig, "trigger_uncertain_from": unc}
