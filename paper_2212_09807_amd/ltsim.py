"""Thin Python binding of libltsim (include/ltsim.h): argument marshalling only.

Every step of the simulation runs in the library's gfx950 kernels; this module converts parameter dataclasses to
the C structs, passes torch device pointers and the current HIP stream, and allocates output tensors of the sizes
the library reports.  PyTorch provides device memory and streams only.  If the shared library has not been built
the import of any entry point raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libltsim.so")

LTS_REDUCE_SORTED, LTS_REDUCE_ATOMIC, LTS_REDUCE_SUMMED = 0, 1, 2
STATUS = {0: "LTS_OK", 1: "LTS_ERR_INVALID_ARG", 2: "LTS_ERR_CAPACITY", 3: "LTS_ERR_OOM", 4: "LTS_ERR_DEVICE",
          5: "LTS_ERR_NOT_READY", 6: "LTS_ERR_CANCELLED", 7: "LTS_ERR_STATE"}
REPORT_FIELDS = ("q_after_quench", "q_collected", "q_induced", "q_clipped", "q_offgrid")


class LtsimError(RuntimeError):
    def __init__(self, status, msg=""):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class lts_physics(C.Structure):
    _fields_ = [("recomb_model", C.c_int32)] + [(n, C.c_double) for n in (
        "e_field", "lar_density", "w_ion", "birks_ab", "birks_kb", "box_alpha", "box_beta", "v_drift", "lifetime",
        "d_long", "d_tran", "z_anode", "sample_step", "n_sigma")] + [("mc_draws", C.c_int32), ("per_point", C.c_int32)]


class lts_readout(C.Structure):
    _fields_ = [("pitch", C.c_double), ("n_x", C.c_int32), ("n_y", C.c_int32), ("x0", C.c_double),
                ("y0", C.c_double), ("n_sub", C.c_int32), ("tick", C.c_double), ("n_ticks", C.c_int32),
                ("t_begin", C.c_double)]


class lts_electronics(C.Structure):
    _fields_ = [("threshold", C.c_double), ("hold_ticks", C.c_int32), ("min_spacing", C.c_int32),
                ("q_lsb", C.c_double), ("pedestal", C.c_int32), ("adc_bits", C.c_int32),
                ("sigma_reset", C.c_double), ("sigma_disc", C.c_double), ("sigma_unc", C.c_double),
                ("max_packets", C.c_int32), ("seed", C.c_uint64), ("reset_period", C.c_int32)]


class lts_segments(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("x0", "y0", "z0", "t0", "x1", "y1", "z1", "t1", "energy", "dedx")] + [
        ("n", C.c_int64)]


class lts_outputs(C.Structure):
    _fields_ = [("pixel_id", C.c_void_p), ("current", C.c_void_p), ("cap_pixels", C.c_int64),
                ("pkt_pixel", C.c_void_p), ("pkt_tick", C.c_void_p), ("pkt_adc", C.c_void_p),
                ("pkt_flags", C.c_void_p), ("cap_packets", C.c_int64), ("counts", C.c_void_p),
                ("report", C.c_void_p), ("event_pixel_offsets", C.c_void_p), ("event_packet_offsets", C.c_void_p)]


class lts_tuning(C.Structure):
    _fields_ = [("min_segments_per_event", C.c_int64), ("reduce_mode", C.c_int32), ("induce_slices", C.c_int32),
                ("ticks_per_thread", C.c_int32), ("lane_exchange", C.c_int32)]


class lts_server_cfg(C.Structure):
    _fields_ = [("n_lanes", C.c_int32), ("max_batch_events", C.c_int32), ("max_batch_segments", C.c_int64),
                ("mem_budget_bytes", C.c_int64), ("return_currents", C.c_int32)]


class lts_result_view(C.Structure):
    _fields_ = [("event_id", C.c_uint64), ("status", C.c_int32), ("n_pixels", C.c_int64), ("n_packets", C.c_int64),
                ("pixel_id", C.c_void_p), ("current", C.c_void_p), ("pkt_pixel", C.c_void_p),
                ("pkt_tick", C.c_void_p), ("pkt_adc", C.c_void_p), ("pkt_flags", C.c_void_p),
                ("report", C.c_double * 5), ("counts", C.c_int64 * 4), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double), ("batch_events", C.c_int32)]


STAGES = ("quench_drift", "rasterize", "cells", "induce", "electronics", "induce_kernel")

EXPORTS = ("lts_server_start", "lts_server_submit", "lts_server_poll", "lts_server_wait", "lts_server_release",
           "lts_server_stop", "lts_set_timing", "lts_get_timing", "lts_work_stats", "lts_context_create", "lts_context_destroy",
           "lts_set_response", "lts_set_reduce_mode", "lts_set_tuning", "lts_set_induce_slices", "lts_set_ticks_per_thread", "lts_set_lane_exchange", "lts_set_matrix_cores", "lts_set_graph", "lts_graph_stats", "lts_set_channel_mask",
           "lts_plan", "lts_simulate", "lts_simulate_batch", "lts_stage_quench_drift", "lts_debug_cells",
           "lts_stage_electronics", "lts_stage_electronics_noalloc", "lts_stage_philox", "lts_debug_fail_host_alloc", "lts_stage_rasterize", "lts_stage_induce", "lts_stage_reduce", "lts_status_str", "lts_last_error", "lts_version",
           "lts_light_create", "lts_light_destroy", "lts_light_simulate", "lts_light_set_graph", "lts_light_last_error")


class lts_light_params(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("tick", "tau_p", "tau_s", "f_prompt", "trunc", "gain", "normal_above")] + [
        ("n_det", C.c_int32), ("n_ticks", C.c_int32), ("group", C.c_int32), ("trig_threshold", C.c_double),
        ("trig_deadtime", C.c_int32), ("max_trig", C.c_int32), ("seed", C.c_uint64)]

_LIB = None


def lib():
    """Load libltsim.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise LtsimError(4, f"{LIB_PATH} not built: run __graft_entry__.build() or "
                                "python paper_2212_09807_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.lts_context_create.argtypes = [C.c_int, C.POINTER(lts_physics), C.POINTER(lts_readout),
                                         C.POINTER(lts_electronics), C.POINTER(P)]
        L.lts_context_destroy.argtypes = [P]
        L.lts_context_destroy.restype = None
        L.lts_set_response.argtypes = [P, P, C.c_int32, C.c_int32, C.c_int32]
        L.lts_set_reduce_mode.argtypes = [P, C.c_int32]
        L.lts_set_tuning.argtypes = [P, C.POINTER(lts_tuning), C.c_int32]
        L.lts_set_induce_slices.argtypes = [P, C.c_int32]
        L.lts_set_ticks_per_thread.argtypes = [P, C.c_int32]
        L.lts_set_lane_exchange.argtypes = [P, C.c_int32]
        L.lts_set_matrix_cores.argtypes = [P, C.c_int32]
        L.lts_set_graph.argtypes = [P, C.c_int32]
        L.lts_graph_stats.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.lts_set_channel_mask.argtypes = [P, P, C.c_int64]
        L.lts_plan.argtypes = [P, C.POINTER(lts_segments), C.POINTER(C.c_int64), P]
        L.lts_simulate.argtypes = [P, C.c_uint64, C.POINTER(lts_segments), C.POINTER(lts_outputs), P]
        L.lts_simulate_batch.argtypes = [P, C.c_int32, P, P, C.POINTER(lts_segments), C.POINTER(lts_outputs), P]
        L.lts_stage_quench_drift.argtypes = [P, C.POINTER(lts_segments), P, P, P]
        L.lts_debug_cells.argtypes = [P, C.c_int64, C.POINTER(C.c_int64), P, C.c_int64]
        L.lts_stage_electronics.argtypes = [P, C.c_uint64, P, P, C.c_int64, C.POINTER(lts_outputs), P]
        L.lts_stage_electronics_noalloc.argtypes = [P, C.c_uint64, P, P, C.c_int64, C.POINTER(lts_outputs), P]
        L.lts_stage_philox.argtypes = [P, C.c_uint32, C.c_uint32, P, C.c_int64, P]
        L.lts_stage_rasterize.argtypes = [P, C.POINTER(lts_segments), P, P, C.c_int64, C.POINTER(C.c_int64), P]
        L.lts_stage_induce.argtypes = [P, C.c_uint64, C.POINTER(lts_segments), P, P, P, C.c_int64,
                                       C.POINTER(C.c_int64), P]
        L.lts_stage_reduce.argtypes = [P, P, P, C.c_int64, P, P, C.c_int64, C.POINTER(C.c_int64), P]
        L.lts_work_stats.argtypes = [P, C.POINTER(C.c_double)]
        L.lts_debug_fail_host_alloc.argtypes = [C.c_int64]
        L.lts_server_start.argtypes = [P, C.POINTER(lts_server_cfg), C.POINTER(P)]
        L.lts_server_submit.argtypes = [P, C.c_uint64, C.POINTER(lts_segments), C.POINTER(C.c_uint64)]
        L.lts_server_poll.argtypes = [P, C.c_uint64, C.POINTER(lts_result_view)]
        L.lts_server_wait.argtypes = [P, C.c_uint64, C.POINTER(lts_result_view), C.c_double]
        L.lts_server_release.argtypes = [P, C.c_uint64]
        L.lts_server_stop.argtypes = [P]
        L.lts_set_timing.argtypes = [P, C.c_int32]
        L.lts_get_timing.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        for f in ("lts_status_str", "lts_last_error", "lts_version"):
            getattr(L, f).restype = C.c_char_p
        L.lts_status_str.argtypes = [C.c_int]
        L.lts_last_error.argtypes = [P]
        L.lts_light_create.argtypes = [C.c_int, C.POINTER(lts_light_params), P, C.c_int32, P, C.c_int32, C.POINTER(P)]
        L.lts_light_destroy.argtypes = [P]
        L.lts_light_destroy.restype = None
        L.lts_light_simulate.argtypes = [P, C.c_uint64, P, P, P, P, P, P, P]
        L.lts_light_last_error.argtypes = [P]
        L.lts_light_set_graph.argtypes = [P, C.c_int32]
        L.lts_light_last_error.restype = C.c_char_p
        _LIB = L
    return _LIB


def _fill(struct_type, obj):
    s = struct_type()
    for name, _ in struct_type._fields_:
        setattr(s, name, getattr(obj, name))
    return s


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclass
class DeviceSegments:
    """Segment columns as torch float32 tensors on the GPU (keeps them alive while the struct points at them)."""
    cols: list
    dedx: object
    n: int

    def struct(self):
        ptrs = [c.data_ptr() for c in self.cols]
        return lts_segments(*ptrs, self.dedx.data_ptr() if self.dedx is not None else None, self.n)


def to_device(segs, device="cuda") -> DeviceSegments:
    import torch
    cols = [torch.from_numpy(np.ascontiguousarray(c, dtype=np.float32)).to(device) for c in segs.columns()]
    dedx = None if segs.dedx is None else torch.from_numpy(np.ascontiguousarray(segs.dedx, np.float32)).to(device)
    return DeviceSegments(cols, dedx, segs.n)


@dataclass
class Result:
    pixel_id: object          # int32 [n_pixels] (torch, device)
    current: object           # float32 [n_pixels, n_ticks]
    pkt_pixel: object
    pkt_tick: object
    pkt_adc: object           # int16 storage of uint16 codes
    pkt_flags: object
    counts: object            # int64 [4]
    report: object            # float64 [n_events, 5]
    event_pixel_offsets: object = None
    event_packet_offsets: object = None

    def host(self):
        """Copy to numpy (synchronises)."""
        cnt = self.counts.cpu().numpy()
        n_pix, n_pk = int(cnt[0]), int(cnt[1])
        d = {"pixel_id": self.pixel_id[:n_pix].cpu().numpy(), "current": self.current[:n_pix].cpu().numpy(),
             "pkt_pixel": self.pkt_pixel[:n_pk].cpu().numpy(), "pkt_tick": self.pkt_tick[:n_pk].cpu().numpy(),
             "pkt_adc": self.pkt_adc[:n_pk].cpu().numpy().view(np.uint16),
             "pkt_flags": self.pkt_flags[:n_pk].cpu().numpy(), "counts": cnt,
             "report": self.report.cpu().numpy()}
        if self.event_pixel_offsets is not None:
            d["event_pixel_offsets"] = self.event_pixel_offsets.cpu().numpy()
            d["event_packet_offsets"] = self.event_packet_offsets.cpu().numpy()
        return d


class Context:
    """One lts_context on a device, with its response table installed."""

    def __init__(self, physics, readout, electronics, table: np.ndarray, device: int = 0,
                 reduce_mode: int = LTS_REDUCE_SORTED):
        L = lib()
        self.physics, self.readout, self.electronics = physics, readout, electronics
        self._h = C.c_void_p()
        self._ph, self._ro, self._el = (_fill(lts_physics, physics), _fill(lts_readout, readout),
                                        _fill(lts_electronics, electronics))
        st = L.lts_context_create(device, C.byref(self._ph), C.byref(self._ro), C.byref(self._el), C.byref(self._h))
        if st:
            raise LtsimError(st, "lts_context_create")
        self.device = device
        table = np.ascontiguousarray(table, dtype=np.float32)
        self._check(L.lts_set_response(self._h, table.ctypes.data_as(C.c_void_p), *table.shape))
        self.set_reduce_mode(reduce_mode)

    @classmethod
    def from_workload(cls, w, table=None, **kw):
        from .workloads import response_table
        if table is None:
            table = response_table(w.table, w.readout, w.physics.v_drift)
        return cls(w.physics, w.readout, w.electronics, table, **kw)

    def _check(self, st):
        if st:
            raise LtsimError(st, lib().lts_last_error(self._h).decode())

    def set_timing(self, enabled: bool):
        self._check(lib().lts_set_timing(self._h, int(bool(enabled))))

    def get_timing(self):
        """{stage: (total ms, calls)} since the previous call (waits for the recorded events)."""
        ms = (C.c_double * len(STAGES))()
        calls = (C.c_int64 * len(STAGES))()
        self._check(lib().lts_get_timing(self._h, ms, calls))
        return {k: (ms[i], calls[i]) for i, k in enumerate(STAGES)}

    def work_stats(self):
        """Algorithmic work of the last call: pairs, induction multiply-adds, cells in reach, cells, multiply-adds the
        summed kernel issues (zeros included), summed records."""
        out = (C.c_double * 6)()
        self._check(lib().lts_work_stats(self._h, out))
        return {"pairs": out[0], "fma": out[1], "cells_in_reach": out[2], "cells": out[3], "fma_issued": out[4],
                "records": out[5]}

    def set_induce_slices(self, slices: int):
        self._check(lib().lts_set_induce_slices(self._h, slices))

    def set_channel_mask(self, disabled=None):
        """Disable pixels (bool / uint8 array of n_x * n_y, True = disabled); None enables all."""
        if disabled is None:
            self._check(lib().lts_set_channel_mask(self._h, None, 0))
            return
        m = np.ascontiguousarray(disabled, dtype=np.uint8)
        self._check(lib().lts_set_channel_mask(self._h, m.ctypes.data_as(C.c_void_p), m.size))

    def set_ticks_per_thread(self, rt: int):
        self._check(lib().lts_set_ticks_per_thread(self._h, rt))

    def set_lane_exchange(self, on: bool):
        self._check(lib().lts_set_lane_exchange(self._h, int(bool(on))))

    def set_matrix_cores(self, on: bool):
        self._check(lib().lts_set_matrix_cores(self._h, int(bool(on))))

    def set_reduce_mode(self, mode: int):
        self._check(lib().lts_set_reduce_mode(self._h, mode))

    def set_tuning(self, table):
        """Install a work-split table: a list of (min_segments_per_event, reduce_mode, slices, ticks_per_thread,
        lane_exchange) in ascending order (lts_set_tuning); None or [] removes it."""
        table = list(table or [])
        arr = (lts_tuning * max(len(table), 1))(*[lts_tuning(*map(int, e)) for e in table])
        self._check(lib().lts_set_tuning(self._h, arr if table else None, len(table)))

    def set_graph(self, on: bool):
        """Replay each call's launch sequence after the sizing read-back as one HIP graph (lts_set_graph)."""
        self._check(lib().lts_set_graph(self._h, int(bool(on))))

    def graph_stats(self):
        """(in-place updates, instantiations) of the context's executable graph."""
        u, i = C.c_int64(0), C.c_int64(0)
        self._check(lib().lts_graph_stats(self._h, C.byref(u), C.byref(i)))
        return int(u.value), int(i.value)

    def close(self):
        if self._h:
            lib().lts_context_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ pipeline
    def plan(self, segs: DeviceSegments, stream=None):
        need = (C.c_int64 * 4)()
        s = segs.struct()
        self._check(lib().lts_plan(self._h, C.byref(s), need, _stream(stream)))
        return {"pairs": need[0], "pixels": need[1], "cells": need[2], "packets": need[3]}

    def _alloc(self, n_pixels, n_packets, n_events, batch):
        import torch
        dev = torch.device("cuda", self.device)
        nt = self.readout.n_ticks
        r = Result(torch.empty(max(n_pixels, 1), dtype=torch.int32, device=dev),
                   torch.empty((max(n_pixels, 1), nt), dtype=torch.float32, device=dev),
                   torch.empty(max(n_packets, 1), dtype=torch.int32, device=dev),
                   torch.empty(max(n_packets, 1), dtype=torch.int32, device=dev),
                   torch.empty(max(n_packets, 1), dtype=torch.int16, device=dev),
                   torch.empty(max(n_packets, 1), dtype=torch.uint8, device=dev),
                   torch.zeros(4, dtype=torch.int64, device=dev),
                   torch.zeros((n_events, 5), dtype=torch.float64, device=dev))
        if batch:
            r.event_pixel_offsets = torch.zeros(n_events + 1, dtype=torch.int64, device=dev)
            r.event_packet_offsets = torch.zeros(n_events + 1, dtype=torch.int64, device=dev)
        return r

    @staticmethod
    def _out_struct(r: Result):
        return lts_outputs(r.pixel_id.data_ptr(), r.current.data_ptr(), r.pixel_id.numel(), r.pkt_pixel.data_ptr(),
                           r.pkt_tick.data_ptr(), r.pkt_adc.data_ptr(), r.pkt_flags.data_ptr(), r.pkt_pixel.numel(),
                           r.counts.data_ptr(), r.report.data_ptr(),
                           r.event_pixel_offsets.data_ptr() if r.event_pixel_offsets is not None else None,
                           r.event_packet_offsets.data_ptr() if r.event_packet_offsets is not None else None)

    def simulate(self, segs: DeviceSegments, event_id: int = 0, stream=None, out: Optional[Result] = None) -> Result:
        if out is None:
            need = self.plan(segs, stream)
            out = self._alloc(need["pixels"], need["packets"], 1, False)
        s = segs.struct()
        o = self._out_struct(out)
        self._check(lib().lts_simulate(self._h, event_id, C.byref(s), C.byref(o), _stream(stream)))
        return out

    def simulate_batch(self, segs: DeviceSegments, seg_offsets: Sequence[int], event_ids: Sequence[int],
                       stream=None, out: Optional[Result] = None, cap_pixels=None, cap_packets=None) -> Result:
        n_ev = len(event_ids)
        offs = np.ascontiguousarray(seg_offsets, dtype=np.int64)
        ids = np.ascontiguousarray(event_ids, dtype=np.uint64)
        assert offs.shape == (n_ev + 1,)
        if out is None:
            cp = cap_pixels if cap_pixels is not None else n_ev * self.readout.n_x * self.readout.n_y
            out = self._alloc(cp, cap_packets if cap_packets is not None else cp * self.electronics.max_packets,
                              n_ev, True)
        s = segs.struct()
        o = self._out_struct(out)
        self._check(lib().lts_simulate_batch(self._h, n_ev, ids.ctypes.data_as(C.c_void_p),
                                             offs.ctypes.data_as(C.c_void_p), C.byref(s), C.byref(o), _stream(stream)))
        return out

    # ------------------------------------------------------------------ stages
    def stage_quench_drift(self, segs: DeviceSegments, stream=None):
        import torch
        dev = torch.device("cuda", self.device)
        f = torch.empty((segs.n, 6), dtype=torch.float32, device=dev)
        i = torch.empty((segs.n, 2), dtype=torch.int32, device=dev)
        s = segs.struct()
        self._check(lib().lts_stage_quench_drift(self._h, C.byref(s), _ptr(f), _ptr(i), _stream(stream)))
        return f, i

    def debug_cells(self, segment: int):
        box = (C.c_int64 * 6)()
        self._check(lib().lts_debug_cells(self._h, segment, box, None, 0))
        b = tuple(int(x) for x in box)
        cells = np.zeros(b[1] * b[3] * b[5], np.float32)
        self._check(lib().lts_debug_cells(self._h, segment, box, cells.ctypes.data_as(C.c_void_p), cells.size))
        return b, cells.reshape(b[1], b[3], b[5])

    def stage_electronics(self, event_id: int, pixel_ids, current, stream=None) -> Result:
        n = int(pixel_ids.numel())
        out = self._alloc(n, n * self.electronics.max_packets, 1, False)
        o = self._out_struct(out)
        self._check(lib().lts_stage_electronics(self._h, event_id, _ptr(pixel_ids), _ptr(current), n, C.byref(o),
                                                _stream(stream)))
        return out

    def stage_electronics_noalloc(self, event_id: int, pixel_ids, current, out: Result, stream=None) -> Result:
        """lts_stage_electronics_noalloc into caller-allocated outputs (`out`, e.g. from an earlier call): the library
        allocates nothing during the call."""
        n = int(pixel_ids.numel())
        o = self._out_struct(out)
        self._check(lib().lts_stage_electronics_noalloc(self._h, event_id, _ptr(pixel_ids), _ptr(current), n,
                                                        C.byref(o), _stream(stream)))
        return out

    def stage_rasterize(self, segs: DeviceSegments, stream=None):
        """(segment, pixel) pairs, pixel-major and ascending in segment: int32 tensors (pair_segment, pair_pixel)."""
        import torch
        dev = torch.device("cuda", self.device)
        cap = self.plan(segs, stream)["pairs"]
        seg = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        pix = torch.empty_like(seg)
        n = C.c_int64(0)
        s = segs.struct()
        self._check(lib().lts_stage_rasterize(self._h, C.byref(s), _ptr(seg), _ptr(pix), cap, C.byref(n),
                                              _stream(stream)))
        return seg[:n.value], pix[:n.value]

    def stage_induce(self, segs: DeviceSegments, event_id: int = 0, stream=None):
        """Materialised per-pair currents: (pair_segment, pair_pixel, current [n_pairs, n_ticks] float32)."""
        import torch
        dev = torch.device("cuda", self.device)
        cap = self.plan(segs, stream)["pairs"]
        seg = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        pix = torch.empty_like(seg)
        cur = torch.empty((max(cap, 1), self.readout.n_ticks), dtype=torch.float32, device=dev)
        n = C.c_int64(0)
        s = segs.struct()
        self._check(lib().lts_stage_induce(self._h, event_id, C.byref(s), _ptr(seg), _ptr(pix), _ptr(cur), cap,
                                           C.byref(n), _stream(stream)))
        return seg[:n.value], pix[:n.value], cur[:n.value]

    def stage_reduce(self, pair_pixel, pair_current, stream=None):
        """Per-pixel sums of pair waveforms grouped by pixel: (pixel_id int32 [k], current float32 [k, n_ticks])."""
        import torch
        dev = torch.device("cuda", self.device)
        n_pairs = int(pair_pixel.numel())
        assert pair_current.shape == (n_pairs, self.readout.n_ticks) and pair_current.is_contiguous()
        n = C.c_int64(0)
        st = lib().lts_stage_reduce(self._h, _ptr(pair_pixel), _ptr(pair_current), n_pairs, None, None, 0,
                                    C.byref(n), _stream(stream))       # sizing pass: the number of pixels
        if st != 2:
            self._check(st)
        cap = n.value
        pid = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        cur = torch.empty((max(cap, 1), self.readout.n_ticks), dtype=torch.float32, device=dev)
        self._check(lib().lts_stage_reduce(self._h, _ptr(pair_pixel), _ptr(pair_current), n_pairs, _ptr(pid),
                                           _ptr(cur), cap, C.byref(n), _stream(stream)))
        return pid[:n.value], cur[:n.value]


def philox(ctr, k0: int, k1: int, stream=None):
    """Raw Philox4x32-10 blocks on the GPU: ctr int32 tensor [n, 4] (bit pattern of uint32) -> int32 [n, 4]."""
    import torch
    out = torch.empty_like(ctr)
    st = lib().lts_stage_philox(_ptr(ctr), k0, k1, _ptr(out), ctr.shape[0], _stream(stream))
    if st:
        raise LtsimError(st, "lts_stage_philox")
    return out


def fail_host_alloc(after: int):
    """Test hook (lts_debug_fail_host_alloc): the library's `after`-th next host allocation point fails once; -1 off."""
    st = lib().lts_debug_fail_host_alloc(after)
    if st:
        raise LtsimError(st, "lts_debug_fail_host_alloc")


def _arr(ptr, n, dtype):
    if n == 0 or not ptr:
        return np.zeros(0, dtype)
    return np.frombuffer(C.string_at(ptr, n * np.dtype(dtype).itemsize), dtype=dtype).copy()


class Server:
    """Continuous-batching request loop of the library (lts_server_*): submit host events, poll / wait results."""

    def __init__(self, ctx: Context, n_lanes=2, max_batch_events=64, max_batch_segments=4_000_000,
                 mem_budget_bytes=32 << 30, return_currents=False):
        self.ctx = ctx
        self._h = C.c_void_p()
        cfg = lts_server_cfg(n_lanes, max_batch_events, max_batch_segments, mem_budget_bytes, int(return_currents))
        ctx._check(lib().lts_server_start(ctx._h, C.byref(cfg), C.byref(self._h)))
        self.n_ticks = ctx.readout.n_ticks

    def submit(self, segs, event_id: int) -> int:
        cols = [np.ascontiguousarray(c, dtype=np.float32) for c in segs.columns()]
        dedx = None if segs.dedx is None else np.ascontiguousarray(segs.dedx, dtype=np.float32)
        st = lts_segments(*[c.ctypes.data for c in cols], dedx.ctypes.data if dedx is not None else None, segs.n)
        t = C.c_uint64()
        rc = lib().lts_server_submit(self._h, event_id, C.byref(st), C.byref(t))
        if rc:
            raise LtsimError(rc, "lts_server_submit")
        return t.value

    def _result(self, v):
        d = {"event_id": v.event_id, "status": v.status, "pixel_id": _arr(v.pixel_id, v.n_pixels, np.int32),
             "pkt_pixel": _arr(v.pkt_pixel, v.n_packets, np.int32), "pkt_tick": _arr(v.pkt_tick, v.n_packets, np.int32),
             "pkt_adc": _arr(v.pkt_adc, v.n_packets, np.uint16), "pkt_flags": _arr(v.pkt_flags, v.n_packets, np.uint8),
             "report": np.array(v.report[:]), "counts": np.array(v.counts[:]), "t_submit": v.t_submit,
             "t_start": v.t_start, "t_done": v.t_done, "batch_events": v.batch_events}
        if v.current:
            d["current"] = _arr(v.current, v.n_pixels * self.n_ticks, np.float32).reshape(v.n_pixels, self.n_ticks)
        return d

    def poll(self, ticket: int):
        v = lts_result_view()
        rc = lib().lts_server_poll(self._h, ticket, C.byref(v))
        if rc == 5:
            return None
        if rc:
            raise LtsimError(rc, "lts_server_poll")
        return self._result(v)

    def wait(self, ticket: int, timeout: float = -1.0):
        v = lts_result_view()
        rc = lib().lts_server_wait(self._h, ticket, C.byref(v), timeout)
        if rc:
            raise LtsimError(rc, "lts_server_wait")
        return self._result(v)

    def release(self, ticket: int):
        rc = lib().lts_server_release(self._h, ticket)
        if rc:
            raise LtsimError(rc, "lts_server_release")

    def stop(self):
        if self._h:
            lib().lts_server_stop(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


class LightSim:
    """Light path on given photocurrents (lts_light_*): scintillation, photoelectron statistics, response with
    noise and group triggers, all on the device."""

    def __init__(self, light, resp, noise_amp, device: int = 0):
        L = lib()
        self._p = _fill(lts_light_params, light)
        self.light = light
        r = np.ascontiguousarray(resp, dtype=np.float32)
        a = np.ascontiguousarray(noise_amp, dtype=np.float32)
        self._h = C.c_void_p()
        st = L.lts_light_create(device, C.byref(self._p), r.ctypes.data, len(r), a.ctypes.data, len(a),
                                C.byref(self._h))
        if st:
            raise LtsimError(st, "lts_light_create")
        self.device = device

    def set_graph(self, on: bool):
        """Replay the light kernels through a HIP graph (pass the same `out` buffers each call to reuse it)."""
        st = lib().lts_light_set_graph(self._h, int(bool(on)))
        if st:
            raise LtsimError(st, lib().lts_light_last_error(self._h).decode())

    def simulate(self, ipe, event_id: int, keep_mu: bool = False, keep_pe: bool = False, stream=None, out=None):
        """ipe: device float32 tensor [n_det, n_ticks].  Returns device tensors V (and mu, pe if asked), trigger ticks
        [n_groups, max_trig] and counts [n_groups].  `out`, a result of an earlier call with the same keep flags,
        is written in place."""
        import torch
        lp = self.light
        shape = (lp.n_det, lp.n_ticks)
        if tuple(ipe.shape) != shape or ipe.dtype != torch.float32 or not ipe.is_cuda or not ipe.is_contiguous():
            raise LtsimError(1, f"photocurrent must be a contiguous float32 device tensor of shape {shape}")
        dev = ipe.device
        ng = lp.n_det // lp.group
        if out is not None:
            V, mu, pe, trig, cnt = out["V"], out.get("mu"), out.get("pe"), out["_trig"], out["trig_count"]
            if (mu is not None) != keep_mu or (pe is not None) != keep_pe:
                raise LtsimError(1, "out was made with other keep_mu / keep_pe flags")
        else:
            V = torch.empty(shape, dtype=torch.float32, device=dev)
            mu = torch.empty(shape, dtype=torch.float64, device=dev) if keep_mu else None
            pe = torch.empty(shape, dtype=torch.float64, device=dev) if keep_pe else None
            trig = torch.empty((ng, max(lp.max_trig, 1)), dtype=torch.int32, device=dev)
            cnt = torch.empty(ng, dtype=torch.int32, device=dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev).cuda_stream
        st = lib().lts_light_simulate(self._h, event_id, ipe.data_ptr(), mu.data_ptr() if keep_mu else None,
                                      pe.data_ptr() if keep_pe else None, V.data_ptr(), trig.data_ptr(),
                                      cnt.data_ptr(), s)
        if st:
            raise LtsimError(st, lib().lts_light_last_error(self._h).decode())
        res = {"V": V, "trig": trig[:, :lp.max_trig], "_trig": trig, "trig_count": cnt}
        if keep_mu:
            res["mu"] = mu
        if keep_pe:
            res["pe"] = pe
        return res

    def close(self):
        if self._h:
            lib().lts_light_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
