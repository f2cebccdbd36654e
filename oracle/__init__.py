"""FP64 CPU oracle of the pixelated-LArTPC charge path (arXiv 2212.09807, Sec. 3).

TEST INFRASTRUCTURE ONLY: this package may be imported by ``tests/``, by ``__graft_entry__.smoke()`` and by the
CPU-baseline leg of ``bench.py``, and by nothing else.  It shares no code with the HIP library
(``paper_2212_09807_amd``); both consume the same seeded inputs from ``paper_2212_09807_amd.workloads``.

The arithmetic lives in ``oracle.c`` (plain C, IEEE double, OpenMP over independent pixels or segments).
This module only marshals arguments.  ``brute.py`` is a second, independent implementation (direct NumPy
loops) used to cross-check the C oracle on tiny inputs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

STREAM_DISC, STREAM_RESET, STREAM_SAMPLE, STREAM_MC = 0, 1, 2, 3
TICK_INITIAL = 0xFFFFFFFF


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (IEEE double, no FP contraction, OpenMP)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter",
                               SRC_PATH, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Physics(C.Structure):
    _fields_ = [("recomb_model", C.c_int32)] + [(n, C.c_double) for n in (
        "e_field", "lar_density", "w_ion", "birks_ab", "birks_kb", "box_alpha", "box_beta", "v_drift", "lifetime",
        "d_long", "d_tran", "z_anode", "sample_step", "n_sigma")] + [("mc_draws", C.c_int32), ("per_point", C.c_int32)]


class _MCKey(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("event_id", C.c_uint64)]


class _Readout(C.Structure):
    _fields_ = [("pitch", C.c_double), ("n_x", C.c_int32), ("n_y", C.c_int32), ("x0", C.c_double),
                ("y0", C.c_double), ("n_sub", C.c_int32), ("tick", C.c_double), ("n_ticks", C.c_int32),
                ("t_begin", C.c_double)]


class _Electronics(C.Structure):
    _fields_ = [("threshold", C.c_double), ("hold_ticks", C.c_int32), ("min_spacing", C.c_int32),
                ("q_lsb", C.c_double), ("pedestal", C.c_int32), ("adc_bits", C.c_int32),
                ("sigma_reset", C.c_double), ("sigma_disc", C.c_double), ("sigma_unc", C.c_double),
                ("max_packets", C.c_int32), ("seed", C.c_uint64), ("reset_period", C.c_int32)]


_FP = C.POINTER(C.c_float)


class _Segments(C.Structure):
    _fields_ = [(n, _FP) for n in ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1", "energy", "dedx")] + [
        ("n", C.c_int64)]


def _fill(struct_type, obj):
    s = struct_type()
    for name, _ in struct_type._fields_:
        setattr(s, name, getattr(obj, name))
    return s


def _ptr(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


class _SegHolder:
    """Keeps the float32 arrays alive while the C struct points at them."""

    def __init__(self, segs):
        self.arrs = [np.ascontiguousarray(c, dtype=np.float32) for c in segs.columns()]
        self.dedx = None if segs.dedx is None else np.ascontiguousarray(segs.dedx, dtype=np.float32)
        self.s = _Segments(*[a.ctypes.data_as(_FP) for a in self.arrs],
                           self.dedx.ctypes.data_as(_FP) if self.dedx is not None else None, segs.n)


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_quench_drift.argtypes = [C.POINTER(_Physics), C.POINTER(_Segments), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.orc_bin_masses.argtypes = [C.c_double] * 5 + [C.c_int64, C.c_int64, C.POINTER(C.c_double)]
        L.orc_bin_masses.restype = None
        L.orc_segment_cells.argtypes = [C.POINTER(_Physics), C.POINTER(_Readout), C.POINTER(_Segments), C.c_int64,
                                        C.POINTER(_MCKey), C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.orc_active_pixels.argtypes = [C.POINTER(_Physics), C.POINTER(_Readout), C.c_int32, C.c_int32, C.c_int32,
                                        C.POINTER(_Segments), C.POINTER(C.c_int32), C.c_int64]
        L.orc_active_pixels.restype = C.c_int64
        L.orc_waveforms.argtypes = [C.POINTER(_Physics), C.POINTER(_Readout), _FP, C.c_int32, C.c_int32, C.c_int32,
                                    C.POINTER(_Segments), C.POINTER(C.c_int32), C.c_int64, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(_MCKey)]
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_philox4x32_10.restype = None
        L.orc_noise_normal.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32]
        L.orc_noise_normal.restype = C.c_double
        L.orc_electronics.argtypes = [C.POINTER(_Electronics), C.POINTER(_Readout), C.c_uint64, C.c_int64,
                                      C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_double, C.c_double,
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
        L.orc_num_threads.restype = C.c_int
        L.orc_mc_clear_near_edges.restype = None
        L.orc_mc_near_edges.argtypes = [C.POINTER(C.c_int32), C.c_int64]
        L.orc_mc_near_edges.restype = C.c_int64
        _LIB = L
    return _LIB


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of later oracle calls (for timing only)."""
    L = lib()
    L.orc_set_num_threads.argtypes = [C.c_int]
    L.orc_set_num_threads.restype = None
    L.orc_set_num_threads(int(n))


# --------------------------------------------------------------------------------------------
# Steps
# --------------------------------------------------------------------------------------------

QD_FIELDS = ("length", "dedx", "recomb", "q0", "q_r", "t_drift", "q_a", "sigma_t", "sigma_time")


def quench_drift(physics, segs):
    h = _SegHolder(segs)
    out = np.zeros((segs.n, 9))
    npts = np.zeros(segs.n, np.int32)
    flags = np.zeros(segs.n, np.int32)
    lib().orc_quench_drift(C.byref(_fill(_Physics, physics)), C.byref(h.s), _ptr(out), _ptr(npts, C.c_int32),
                           _ptr(flags, C.c_int32))
    d = {k: out[:, i] for i, k in enumerate(QD_FIELDS)}
    d["n_points"] = npts
    d["flags"] = flags
    return d


def bin_masses(mean, sigma, n_sigma, origin, width, k0, nk):
    out = np.zeros(nk)
    lib().orc_bin_masses(mean, sigma, n_sigma, origin, width, k0, nk, _ptr(out))
    return out


def _key(mc_key):
    return None if mc_key is None else C.byref(_MCKey(int(mc_key[0]), int(mc_key[1])))


def segment_cells(physics, readout, segs, i, mc_key=None):
    """(box, cells): box = (a0, na, u0, nu, v0, nv); cells[a, u, v] in FP64.  mc_key = (seed, event_id) selects the
    Monte Carlo draws when physics.mc_draws > 0."""
    h = _SegHolder(segs)
    box = np.zeros(6, np.int64)
    P, R = _fill(_Physics, physics), _fill(_Readout, readout)
    rc = lib().orc_segment_cells(C.byref(P), C.byref(R), C.byref(h.s), i, _key(mc_key), _ptr(box, C.c_int64), None)
    if rc:
        raise ValueError(f"orc_segment_cells rc={rc}")
    cells = np.zeros(int(box[1] * box[3] * box[5]))
    rc = lib().orc_segment_cells(C.byref(P), C.byref(R), C.byref(h.s), i, _key(mc_key), _ptr(box, C.c_int64),
                                 _ptr(cells))
    if rc:
        raise ValueError(f"orc_segment_cells rc={rc}")
    return tuple(int(b) for b in box), cells.reshape(int(box[1]), int(box[3]), int(box[5]))


def active_pixels(physics, readout, table_shape, segs):
    h = _SegHolder(segs)
    P, R = _fill(_Physics, physics), _fill(_Readout, readout)
    n = lib().orc_active_pixels(C.byref(P), C.byref(R), table_shape.t_r, table_shape.b_x, table_shape.b_y,
                                C.byref(h.s), None, 0)
    out = np.zeros(max(n, 1), np.int32)
    lib().orc_active_pixels(C.byref(P), C.byref(R), table_shape.t_r, table_shape.b_x, table_shape.b_y, C.byref(h.s),
                            _ptr(out, C.c_int32), n)
    return out[:n]


def waveforms(physics, readout, table, segs, pixels, with_sums=False, mc_key=None):
    """FP64 waveforms [len(pixels), n_ticks], per-pixel clipped charge, and (if with_sums) the segment sums
    (sum Q_R, sum Q_a, off-grid charge).  mc_key = (seed, event_id) is required when physics.mc_draws > 0."""
    table = np.ascontiguousarray(table, dtype=np.float32)
    T, bx, by = table.shape
    pixels = np.ascontiguousarray(pixels, dtype=np.int32)
    h = _SegHolder(segs)
    wave = np.zeros((len(pixels), readout.n_ticks))
    clipped = np.zeros(len(pixels))
    sums = np.zeros(3)
    rc = lib().orc_waveforms(C.byref(_fill(_Physics, physics)), C.byref(_fill(_Readout, readout)),
                             table.ctypes.data_as(_FP), T, bx, by, C.byref(h.s), _ptr(pixels, C.c_int32),
                             len(pixels), _ptr(wave), _ptr(clipped), _ptr(sums) if with_sums else None,
                             _key(mc_key))
    if rc:
        raise ValueError(f"orc_waveforms rc={rc}")
    return (wave, clipped, sums) if with_sums else (wave, clipped)


def mc_clear_near_edges():
    lib().orc_mc_clear_near_edges()


def mc_near_edges():
    """(u, v) bins of the Monte Carlo draws recorded since the last clear that landed within 1e-5 of a bin or tick
    edge (an FP32 evaluation may put them in the neighbouring cell)."""
    n = int(lib().orc_mc_near_edges(None, 0))
    out = np.zeros((max(n, 1), 2), np.int32)
    n2 = int(lib().orc_mc_near_edges(_ptr(out, C.c_int32), n))
    return out[:min(n, n2, 65536)]


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return o


def noise_normal(seed, pixel, tick, event_id, stream):
    return float(lib().orc_noise_normal(seed, pixel, tick, event_id, stream))


def electronics(el, readout, event_id, pixels, wave, eps_rel=0.0, eps_abs=0.0, with_uncertain=False):
    """Packets per pixel: list of (tick, adc, flag) arrays; plus stats (dropped, over cap, flagged decisions) and,
    if asked, per pixel the first tick whose threshold decision lay within eps (2**31-1 if none)."""
    pixels = np.ascontiguousarray(pixels, dtype=np.int32)
    wave = np.ascontiguousarray(wave, dtype=np.float64)
    n = len(pixels)
    mp = el.max_packets
    tick = np.zeros(n * mp, np.int32)
    adc = np.zeros(n * mp, np.int32)
    flag = np.zeros(n * mp, np.int32)
    cnt = np.zeros(n, np.int32)
    stats = np.zeros(3, np.int64)
    ufrom = np.zeros(n, np.int32)
    lib().orc_electronics(C.byref(_fill(_Electronics, el)), C.byref(_fill(_Readout, readout)), event_id, n,
                          _ptr(pixels, C.c_int32), _ptr(wave), eps_rel, eps_abs, _ptr(tick, C.c_int32),
                          _ptr(adc, C.c_int32), _ptr(flag, C.c_int32), _ptr(cnt, C.c_int32), _ptr(stats, C.c_int64),
                          _ptr(ufrom, C.c_int32))
    out = []
    for q in range(n):
        s = slice(q * mp, q * mp + cnt[q])
        out.append((tick[s].copy(), adc[s].copy(), flag[s].copy()))
    return (out, stats, ufrom) if with_uncertain else (out, stats)


def simulate(workload, event_index=0, pixels=None, table=None, eps_rel=0.0, eps_abs=0.0, with_packets=True):
    """Whole event through the oracle: active pixels (or the given subset), waveforms, packets, report."""
    from paper_2212_09807_amd.workloads import response_table
    segs = workload.events[event_index]
    if table is None:
        table = response_table(workload.table, workload.readout, workload.physics.v_drift)
    full = pixels is None
    if full:
        pixels = active_pixels(workload.physics, workload.readout, workload.table, segs)
    key = (workload.electronics.seed, workload.event_ids[event_index])
    mc_clear_near_edges()
    out = waveforms(workload.physics, workload.readout, table, segs, pixels, with_sums=full, mc_key=key)
    wave, clipped, sums = out if full else (out[0], out[1], None)
    res = {"pixels": np.asarray(pixels, np.int32), "wave": wave, "clipped": clipped, "mc_near_edges": mc_near_edges()}
    if full:
        res["report"] = {"q_after_quench": sums[0], "q_collected": sums[1], "q_induced": float(wave.sum()),
                         "q_clipped": float(clipped.sum()), "q_offgrid": sums[2]}
    if with_packets:
        pk, st, uf = electronics(workload.electronics, workload.readout, workload.event_ids[event_index], pixels,
                                 wave, eps_rel, eps_abs, with_uncertain=True)
        res["packets"] = pk
        res["electronics_stats"] = st
        res["uncertain_from"] = uf
    return res
