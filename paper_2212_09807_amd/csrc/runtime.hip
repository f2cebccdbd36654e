// runtime.hip -- C ABI of libltsim (see include/ltsim.h): contexts, the device-resident field-response table, the
// scratch pool and the stage sequence of one event or a batch of events.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ltsim.h"
#include "device.hpp"
#include "launch.hpp"

using namespace ltsim;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct lts_context {
    int device = 0;
    lts_physics ph{};
    lts_readout ro{};
    lts_electronics el{};
    int32_t reduce_mode = LTS_REDUCE_SORTED;
    DevParams P{};
    bool has_table = false;
    DevBuf Rpad, prefix;
    // scratch pool
    DevBuf si, cell_off, pix_cnt, cursor, pix_slot, slot_gp, slot_off, pairs_u, pairs, cells, pk_tick, pk_adc,
        pk_flag, pk_off, hdr, scan_tmp, ev_off, ev_ids, report_tmp, counts_tmp;
    DevHeader *hdr_host = nullptr;   // pinned
    int64_t last_n_seg = -1;
    std::string err;
    lts_status sticky = LTS_OK;
};

namespace {

lts_status fail(lts_context *c, lts_status s, const std::string &msg) {
    if (c) {
        c->err = msg;
        if (s == LTS_ERR_DEVICE) c->sticky = LTS_ERR_DEVICE;
    }
    return s;
}

#define HIP_TRY(ctx, call)                                                                                    \
    do {                                                                                                      \
        hipError_t e_ = (call);                                                                               \
        if (e_ != hipSuccess)                                                                                 \
            return fail((ctx), e_ == hipErrorOutOfMemory ? LTS_ERR_OOM : LTS_ERR_DEVICE,                        \
                        std::string(#call) + ": " + hipGetErrorString(e_));                                   \
    } while (0)

lts_status ensure(lts_context *c, DevBuf &b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.bytes >= bytes) return LTS_OK;
    if (b.p) {
        HIP_TRY(c, hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = std::max(bytes, b.bytes + b.bytes / 2);
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        e = hipMalloc(&b.p, bytes);
        want = bytes;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(c, LTS_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    b.bytes = want;
    return LTS_OK;
}

void free_buf(DevBuf &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

bool finite_all(std::initializer_list<double> v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

void split(double v, float &hi, float &lo) {
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

lts_status validate_and_derive(lts_context *c) {
    const lts_physics &ph = c->ph;
    const lts_readout &ro = c->ro;
    const lts_electronics &el = c->el;
    if (!finite_all({ph.e_field, ph.lar_density, ph.w_ion, ph.birks_ab, ph.birks_kb, ph.box_alpha, ph.box_beta,
                     ph.v_drift, ph.lifetime, ph.d_long, ph.d_tran, ph.z_anode, ph.sample_step, ph.n_sigma, ro.pitch,
                     ro.x0, ro.y0, ro.tick, ro.t_begin, el.threshold, el.q_lsb, el.sigma_reset, el.sigma_disc,
                     el.sigma_unc}))
        return fail(c, LTS_ERR_INVALID_ARG, "non-finite parameter");
    if (ph.recomb_model != 0 && ph.recomb_model != 1) return fail(c, LTS_ERR_INVALID_ARG, "recomb_model must be 0 or 1");
    if (!(ph.e_field > 0 && ph.lar_density > 0 && ph.w_ion > 0))
        return fail(c, LTS_ERR_INVALID_ARG, "e_field, lar_density and w_ion must be > 0");
    if (!(ph.v_drift > 0)) return fail(c, LTS_ERR_INVALID_ARG, "v_drift must be > 0");
    if (!(ph.lifetime > 0)) return fail(c, LTS_ERR_INVALID_ARG, "lifetime must be > 0");
    if (!(ph.d_long >= 0 && ph.d_tran >= 0)) return fail(c, LTS_ERR_INVALID_ARG, "diffusion coefficients must be >= 0");
    if (!(ph.sample_step > 0)) return fail(c, LTS_ERR_INVALID_ARG, "sample_step must be > 0");
    if (!(ph.n_sigma >= 1 && ph.n_sigma <= 10)) return fail(c, LTS_ERR_INVALID_ARG, "n_sigma must be in [1, 10]");
    if (!(ro.pitch > 0 && ro.tick > 0)) return fail(c, LTS_ERR_INVALID_ARG, "pitch and tick must be > 0");
    if (ro.n_sub < 2 || (ro.n_sub & 1) || ro.n_sub > 64) return fail(c, LTS_ERR_INVALID_ARG, "n_sub must be even in [2, 64]");
    if (ro.n_x < 1 || ro.n_y < 1 || (int64_t)ro.n_x * ro.n_y > (1 << 22))
        return fail(c, LTS_ERR_INVALID_ARG, "pixel grid must be 1..4M pixels");
    // the sorted reduction keeps a Kahan pair (2 floats) per tick of the window in LDS: <= 64000 bytes
    if (ro.n_ticks < 1 || ro.n_ticks > 8000) return fail(c, LTS_ERR_INVALID_ARG, "n_ticks must be in [1, 8000]");
    if (el.adc_bits < 1 || el.adc_bits > 16) return fail(c, LTS_ERR_INVALID_ARG, "adc_bits must be in [1, 16]");
    if (el.max_packets < 1 || el.max_packets > 65536) return fail(c, LTS_ERR_INVALID_ARG, "max_packets must be in [1, 65536]");
    if (!(el.q_lsb > 0)) return fail(c, LTS_ERR_INVALID_ARG, "q_lsb must be > 0");
    if (el.hold_ticks < 0 || el.min_spacing < 0) return fail(c, LTS_ERR_INVALID_ARG, "hold / spacing must be >= 0");
    if (!(el.sigma_reset >= 0 && el.sigma_disc >= 0 && el.sigma_unc >= 0))
        return fail(c, LTS_ERR_INVALID_ARG, "noise sigmas must be >= 0");
    DevParams &P = c->P;
    const double eps = ph.e_field * ph.lar_density;
    P.recomb_model = ph.recomb_model;
    P.birks_ab = (float)ph.birks_ab;
    P.birks_kb_eps = (float)(ph.birks_kb / eps);
    P.box_alpha = (float)ph.box_alpha;
    P.box_beta_eps = (float)(ph.box_beta / eps);
    P.inv_w_ion = (float)(1.0 / ph.w_ion);
    split(1.0 / ph.v_drift, P.inv_vd_hi, P.inv_vd_lo);
    P.inv_lifetime = (float)(1.0 / ph.lifetime);
    P.two_dl = (float)(2.0 * ph.d_long);
    P.two_dt = (float)(2.0 * ph.d_tran);
    split(ph.z_anode, P.za_hi, P.za_lo);
    P.step = (float)ph.sample_step;
    P.nsig = (float)ph.n_sigma;
    P.inv_norm = (float)(1.0 / std::erf(ph.n_sigma / std::sqrt(2.0)));
    split(ro.pitch / ro.n_sub, P.b_hi, P.b_lo);
    split(ro.x0, P.x0_hi, P.x0_lo);
    split(ro.y0, P.y0_hi, P.y0_lo);
    split(ro.tick, P.tick_hi, P.tick_lo);
    split(ro.t_begin, P.tb_hi, P.tb_lo);
    P.nx = ro.n_x;
    P.ny = ro.n_y;
    P.nsub = ro.n_sub;
    P.nticks = ro.n_ticks;
    P.npx = ro.n_x * ro.n_y;
    P.thr = (float)el.threshold;
    P.q_lsb = (float)el.q_lsb;
    P.sig_reset = (float)el.sigma_reset;
    P.sig_disc = (float)el.sigma_disc;
    P.sig_unc = (float)el.sigma_unc;
    P.hold = el.hold_ticks;
    P.spacing = el.min_spacing;
    P.pedestal = el.pedestal;
    P.adc_max = (1 << el.adc_bits) - 1;
    P.max_packets = el.max_packets;
    P.key0 = (uint32_t)(el.seed & 0xffffffffu);
    P.key1 = (uint32_t)(el.seed >> 32);
    P.eps_rel = 2e-6f;
    P.eps_abs = 0.05f;
    return LTS_OK;
}

template <typename T>
T *as(DevBuf &b) { return (T *)b.p; }

hipStream_t to_stream(void *s) { return (hipStream_t)s; }

lts_status check_segments(lts_context *c, const lts_segments *s) {
    if (!s) return fail(c, LTS_ERR_INVALID_ARG, "segments is NULL");
    if (s->n < 0 || s->n > (int64_t)INT32_MAX) return fail(c, LTS_ERR_INVALID_ARG, "segment count out of range");
    if (s->n > 0 && !(s->x0 && s->y0 && s->z0 && s->t0 && s->x1 && s->y1 && s->z1 && s->t1 && s->energy))
        return fail(c, LTS_ERR_INVALID_ARG, "segment column pointer is NULL");
    return LTS_OK;
}

SegArrays seg_arrays(const lts_segments *s) {
    return SegArrays{s->x0, s->y0, s->z0, s->t0, s->x1, s->y1, s->z1, s->t1, s->energy, s->dedx};
}

// Sizing half of the pipeline: quench / drift / rasterisation counts and scans; synchronises the stream and
// returns the header on the host.
lts_status run_sizing(lts_context *c, int32_t n_ev, const uint64_t *event_ids, const int64_t *seg_offsets,
                      const lts_segments *segs, double *report, hipStream_t st, Work &w, DevHeader &h) {
    lts_status r;
    const int64_t n_seg = segs->n;
    const int64_t n_gp = (int64_t)n_ev * c->P.npx;
    if (n_gp + 1 >= (1ll << 24)) return fail(c, LTS_ERR_INVALID_ARG, "events x pixels exceeds 2^24 - 1");
    if (seg_offsets[0] != 0 || seg_offsets[n_ev] != n_seg)
        return fail(c, LTS_ERR_INVALID_ARG, "seg_offsets must start at 0 and end at segs->n");
    for (int32_t e = 0; e < n_ev; ++e)
        if (seg_offsets[e + 1] < seg_offsets[e]) return fail(c, LTS_ERR_INVALID_ARG, "seg_offsets must be non-decreasing");
    const int64_t scan_n = std::max<int64_t>(n_gp + 1, n_seg + 1);
    if ((r = ensure(c, c->si, sizeof(SegInfo) * (size_t)std::max<int64_t>(n_seg, 1)))) return r;
    if ((r = ensure(c, c->cell_off, sizeof(int64_t) * (size_t)(n_seg + 1)))) return r;
    if ((r = ensure(c, c->pix_cnt, sizeof(uint64_t) * (size_t)(n_gp + 1)))) return r;
    if ((r = ensure(c, c->cursor, sizeof(int32_t) * (size_t)n_gp))) return r;
    if ((r = ensure(c, c->pix_slot, sizeof(int32_t) * (size_t)n_gp))) return r;
    if ((r = ensure(c, c->hdr, sizeof(DevHeader)))) return r;
    if ((r = ensure(c, c->ev_off, sizeof(int64_t) * (size_t)(n_ev + 1)))) return r;
    if ((r = ensure(c, c->ev_ids, sizeof(uint64_t) * (size_t)n_ev))) return r;
    if ((r = ensure(c, c->scan_tmp, sizeof(int64_t) * (size_t)scan_tmp_needed(scan_n)))) return r;
    HIP_TRY(c, hipMemcpyAsync(c->ev_off.p, seg_offsets, sizeof(int64_t) * (size_t)(n_ev + 1), hipMemcpyHostToDevice, st));
    HIP_TRY(c, hipMemcpyAsync(c->ev_ids.p, event_ids, sizeof(uint64_t) * (size_t)n_ev, hipMemcpyHostToDevice, st));
    HIP_TRY(c, hipMemsetAsync(c->pix_cnt.p, 0, sizeof(uint64_t) * (size_t)(n_gp + 1), st));
    HIP_TRY(c, hipMemsetAsync(c->cursor.p, 0, sizeof(int32_t) * (size_t)n_gp, st));
    HIP_TRY(c, hipMemsetAsync(c->hdr.p, 0, sizeof(DevHeader), st));
    HIP_TRY(c, hipMemsetAsync(as<int64_t>(c->cell_off) + n_seg, 0, sizeof(int64_t), st));
    HIP_TRY(c, hipMemsetAsync(report, 0, sizeof(double) * 5 * (size_t)n_ev, st));
    w = Work{};
    w.n_seg = n_seg;
    w.n_ev = n_ev;
    w.seg_ev_off = as<int64_t>(c->ev_off);
    w.event_ids = as<uint64_t>(c->ev_ids);
    w.si = as<SegInfo>(c->si);
    w.cell_off = as<int64_t>(c->cell_off);
    w.pix_cnt = as<uint64_t>(c->pix_cnt);
    w.cursor = as<int32_t>(c->cursor);
    w.pix_slot = as<int32_t>(c->pix_slot);
    w.hdr = as<DevHeader>(c->hdr);
    w.report = report;
    w.scan_tmp = c->scan_tmp.p;
    SegArrays S = seg_arrays(segs);
    launch_quench_drift(c->P, S, w, st);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipMemcpyAsync(c->hdr_host, c->hdr.p, sizeof(DevHeader), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    h = *c->hdr_host;
    if (h.status & ST_INVALID)
        return fail(c, LTS_ERR_INVALID_ARG, "invalid segment (non-finite value, negative energy, or zero length without dE/dx)");
    if (h.status & ST_TOO_LONG)
        return fail(c, LTS_ERR_INVALID_ARG, "a segment's charge box exceeds 256 ticks or 256 sub-pixel bins; split long segments");
    c->last_n_seg = n_seg;
    return LTS_OK;
}

lts_status run_pipeline(lts_context *c, int32_t n_ev, const uint64_t *event_ids, const int64_t *seg_offsets,
                        const lts_segments *segs, const lts_outputs *out, hipStream_t st) {
    if (c->sticky) return fail(c, c->sticky, "context is in a failed state: " + c->err);
    if (!c->has_table) return fail(c, LTS_ERR_STATE, "no response table: call lts_set_response first");
    lts_status r;
    if ((r = check_segments(c, segs))) return r;
    if (!out || !out->counts || !out->report || !out->pixel_id || !out->current)
        return fail(c, LTS_ERR_INVALID_ARG, "outputs: pixel_id, current, counts and report are required");
    if (n_ev < 1 || !event_ids || !seg_offsets) return fail(c, LTS_ERR_INVALID_ARG, "bad event list");
    HIP_TRY(c, hipSetDevice(c->device));
    Work w;
    DevHeader h;
    if ((r = run_sizing(c, n_ev, event_ids, seg_offsets, segs, out->report, st, w, h))) return r;
    const int64_t n_slots = h.n_slots, n_pairs = h.n_pairs, n_cells = h.n_cells;
    const int64_t mp = c->P.max_packets;
    if (n_slots > out->cap_pixels) {
        int64_t need[4] = {n_slots, n_slots * mp, 0, 0};
        HIP_TRY(c, hipMemcpy(out->counts, need, sizeof(need), hipMemcpyHostToDevice));
        return fail(c, LTS_ERR_CAPACITY, "cap_pixels " + std::to_string(out->cap_pixels) + " < " + std::to_string(n_slots));
    }
    if ((r = ensure(c, c->slot_gp, sizeof(int32_t) * (size_t)std::max<int64_t>(n_slots, 1)))) return r;
    if ((r = ensure(c, c->slot_off, sizeof(int64_t) * (size_t)(n_slots + 1)))) return r;
    if ((r = ensure(c, c->pairs_u, sizeof(int32_t) * (size_t)std::max<int64_t>(n_pairs, 1)))) return r;
    if ((r = ensure(c, c->pairs, sizeof(int32_t) * (size_t)std::max<int64_t>(n_pairs, 1)))) return r;
    if ((r = ensure(c, c->cells, sizeof(float) * (size_t)std::max<int64_t>(n_cells, 1)))) return r;
    if ((r = ensure(c, c->pk_tick, sizeof(int32_t) * (size_t)(n_slots * mp)))) return r;
    if ((r = ensure(c, c->pk_adc, sizeof(uint16_t) * (size_t)(n_slots * mp)))) return r;
    if ((r = ensure(c, c->pk_flag, sizeof(uint8_t) * (size_t)(n_slots * mp)))) return r;
    if ((r = ensure(c, c->pk_off, sizeof(int64_t) * (size_t)(n_slots + 1)))) return r;
    if ((r = ensure(c, c->scan_tmp, sizeof(int64_t) * (size_t)scan_tmp_needed(n_slots + 1)))) return r;
    w.slot_gp = as<int32_t>(c->slot_gp);
    w.slot_off = as<int64_t>(c->slot_off);
    w.pairs_unsorted = as<int32_t>(c->pairs_u);
    w.pairs = as<int32_t>(c->pairs);
    w.cells = as<float>(c->cells);
    w.pk_tick = as<int32_t>(c->pk_tick);
    w.pk_adc = as<uint16_t>(c->pk_adc);
    w.pk_flag = as<uint8_t>(c->pk_flag);
    w.pk_off = as<int64_t>(c->pk_off);
    w.scan_tmp = c->scan_tmp.p;
    HIP_TRY(c, hipMemsetAsync(w.pk_off, 0, sizeof(int64_t) * (size_t)(n_slots + 1), st));
    const DevParams &P = c->P;
    launch_slots(P, w, out->pixel_id, out->event_pixel_offsets, st);
    launch_fill_pairs(P, w, st);
    if (c->reduce_mode == LTS_REDUCE_SORTED) launch_sort_pairs(w, n_slots, st);
    launch_cells(P, w, st);
    Table T{as<float>(c->Rpad), as<double>(c->prefix)};
    if (c->reduce_mode == LTS_REDUCE_ATOMIC)
        HIP_TRY(c, hipMemsetAsync(out->current, 0, sizeof(float) * (size_t)n_slots * P.nticks, st));
    if (c->reduce_mode == LTS_REDUCE_ATOMIC) {
        // the atomic variant walks segments, not pairs: reuse the pixel-major pair arrays only for slots
    }
    launch_induce(P, w, T, out->current, c->reduce_mode, n_slots, st);
    launch_electronics(P, out->current, w.slot_gp, w.event_ids, n_slots, w, st);
    launch_compact_packets(P, w, n_slots, out->pkt_pixel, out->pkt_tick, out->pkt_adc, out->pkt_flags, out->cap_packets,
                           out->event_pixel_offsets, out->event_packet_offsets, out->counts, st);
    HIP_TRY(c, hipGetLastError());
    if (out->cap_packets < n_slots * mp) {
        int64_t cnt[4];
        HIP_TRY(c, hipMemcpyAsync(cnt, out->counts, sizeof(cnt), hipMemcpyDeviceToHost, st));
        HIP_TRY(c, hipStreamSynchronize(st));
        if (cnt[1] > out->cap_packets)
            return fail(c, LTS_ERR_CAPACITY, "cap_packets " + std::to_string(out->cap_packets) + " < " + std::to_string(cnt[1]));
    }
    return LTS_OK;
}

}  // namespace

extern "C" {

const char *lts_version(void) { return "ltsim 0.1 (gfx950)"; }

const char *lts_status_str(lts_status s) {
    switch (s) {
        case LTS_OK: return "ok";
        case LTS_ERR_INVALID_ARG: return "invalid argument";
        case LTS_ERR_CAPACITY: return "output capacity too small";
        case LTS_ERR_OOM: return "device out of memory";
        case LTS_ERR_DEVICE: return "device error";
        case LTS_ERR_NOT_READY: return "not ready";
        case LTS_ERR_CANCELLED: return "cancelled";
        case LTS_ERR_STATE: return "invalid state";
    }
    return "unknown status";
}

const char *lts_last_error(const lts_context *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

lts_status lts_context_create(int device, const lts_physics *physics, const lts_readout *readout,
                              const lts_electronics *electronics, lts_context **out) {
    if (!out || !physics || !readout || !electronics) return LTS_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return LTS_ERR_DEVICE;
    }
    lts_context *c = new (std::nothrow) lts_context();
    if (!c) return LTS_ERR_OOM;
    c->device = device;
    c->ph = *physics;
    c->ro = *readout;
    c->el = *electronics;
    lts_status r = validate_and_derive(c);
    if (r == LTS_OK && hipSetDevice(device) != hipSuccess) r = LTS_ERR_DEVICE;
    if (r == LTS_OK && hipHostMalloc((void **)&c->hdr_host, sizeof(DevHeader), hipHostMallocDefault) != hipSuccess)
        r = LTS_ERR_OOM;
    if (r != LTS_OK) {
        delete c;
        return r;
    }
    *out = c;
    return LTS_OK;
}

void lts_context_destroy(lts_context *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    DevBuf *bufs[] = {&c->Rpad, &c->prefix, &c->si, &c->cell_off, &c->pix_cnt, &c->cursor, &c->pix_slot, &c->slot_gp,
                      &c->slot_off, &c->pairs_u, &c->pairs, &c->cells, &c->pk_tick, &c->pk_adc, &c->pk_flag,
                      &c->pk_off, &c->hdr, &c->scan_tmp, &c->ev_off, &c->ev_ids, &c->report_tmp, &c->counts_tmp};
    for (DevBuf *b : bufs) free_buf(*b);
    if (c->hdr_host) (void)hipHostFree(c->hdr_host);
    delete c;
}

lts_status lts_set_reduce_mode(lts_context *c, int32_t mode) {
    if (!c) return LTS_ERR_INVALID_ARG;
    if (mode != LTS_REDUCE_SORTED && mode != LTS_REDUCE_ATOMIC) return fail(c, LTS_ERR_INVALID_ARG, "unknown reduce mode");
    c->reduce_mode = mode;
    return LTS_OK;
}

lts_status lts_set_response(lts_context *c, const float *R, int32_t t_r, int32_t b_x, int32_t b_y) {
    if (!c) return LTS_ERR_INVALID_ARG;
    if (!R || t_r < 1 || t_r > 8192 || b_x < 1 || b_x > 256 || b_y < 1 || b_y > 256)
        return fail(c, LTS_ERR_INVALID_ARG, "response table shape must be 1..8192 x 1..256 x 1..256");
    const size_t ncol = (size_t)b_x * b_y;
    const int32_t col_len = kPad + t_r + kPad;
    std::vector<float> pad(ncol * (size_t)col_len, 0.0f);
    std::vector<double> pre(ncol * (size_t)(t_r + 1), 0.0);
    for (int32_t i = 0; i < b_x; ++i)
        for (int32_t j = 0; j < b_y; ++j) {
            const size_t col = (size_t)i * b_y + j;
            double run = 0.0;
            pre[col * (t_r + 1)] = 0.0;
            for (int32_t k = 0; k < t_r; ++k) {
                const float v = R[((size_t)k * b_x + i) * b_y + j];
                if (!std::isfinite(v)) return fail(c, LTS_ERR_INVALID_ARG, "non-finite response table entry");
                pad[col * col_len + kPad + k] = v;
                run += (double)v;
                pre[col * (t_r + 1) + k + 1] = run;
            }
        }
    HIP_TRY(c, hipSetDevice(c->device));
    lts_status r;
    if ((r = ensure(c, c->Rpad, sizeof(float) * pad.size()))) return r;
    if ((r = ensure(c, c->prefix, sizeof(double) * pre.size()))) return r;
    HIP_TRY(c, hipMemcpy(c->Rpad.p, pad.data(), sizeof(float) * pad.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->prefix.p, pre.data(), sizeof(double) * pre.size(), hipMemcpyHostToDevice));
    c->P.t_r = t_r;
    c->P.bx = b_x;
    c->P.by = b_y;
    c->P.col_len = col_len;
    c->has_table = true;
    return LTS_OK;
}

lts_status lts_plan(lts_context *c, const lts_segments *segs, int64_t need[4], void *stream) {
    if (!c || !need) return LTS_ERR_INVALID_ARG;
    if (c->sticky) return fail(c, c->sticky, "context is in a failed state: " + c->err);
    if (!c->has_table) return fail(c, LTS_ERR_STATE, "no response table: call lts_set_response first");
    lts_status r;
    if ((r = check_segments(c, segs))) return r;
    HIP_TRY(c, hipSetDevice(c->device));
    if ((r = ensure(c, c->report_tmp, sizeof(double) * 5))) return r;
    const uint64_t eid = 0;
    const int64_t off[2] = {0, segs->n};
    Work w;
    DevHeader h;
    if ((r = run_sizing(c, 1, &eid, off, segs, as<double>(c->report_tmp), to_stream(stream), w, h))) return r;
    need[0] = h.n_pairs;
    need[1] = h.n_slots;
    need[2] = h.n_cells;
    need[3] = h.n_slots * c->P.max_packets;
    return LTS_OK;
}

lts_status lts_simulate(lts_context *c, uint64_t event_id, const lts_segments *segs, const lts_outputs *out,
                        void *stream) {
    if (!c) return LTS_ERR_INVALID_ARG;
    if (!segs) return fail(c, LTS_ERR_INVALID_ARG, "segments is NULL");
    const int64_t off[2] = {0, segs->n};
    return run_pipeline(c, 1, &event_id, off, segs, out, to_stream(stream));
}

lts_status lts_simulate_batch(lts_context *c, int32_t n_events, const uint64_t *event_ids, const int64_t *seg_offsets,
                              const lts_segments *segs, const lts_outputs *out, void *stream) {
    if (!c) return LTS_ERR_INVALID_ARG;
    if (out && (!out->event_pixel_offsets || !out->event_packet_offsets))
        return fail(c, LTS_ERR_INVALID_ARG, "batch outputs need event_pixel_offsets and event_packet_offsets");
    return run_pipeline(c, n_events, event_ids, seg_offsets, segs, out, to_stream(stream));
}

lts_status lts_stage_quench_drift(lts_context *c, const lts_segments *segs, float *out_f, int32_t *out_i, void *stream) {
    if (!c) return LTS_ERR_INVALID_ARG;
    lts_status r;
    if ((r = check_segments(c, segs))) return r;
    if (!out_f || !out_i) return fail(c, LTS_ERR_INVALID_ARG, "NULL output");
    HIP_TRY(c, hipSetDevice(c->device));
    launch_stage_quench_drift(c->P, seg_arrays(segs), segs->n, out_f, out_i, to_stream(stream));
    HIP_TRY(c, hipGetLastError());
    return LTS_OK;
}

lts_status lts_debug_cells(lts_context *c, int64_t segment, int64_t box[6], float *cells_host, int64_t cap) {
    if (!c || !box) return LTS_ERR_INVALID_ARG;
    if (segment < 0 || segment >= c->last_n_seg) return fail(c, LTS_ERR_STATE, "segment not in the last simulated call");
    HIP_TRY(c, hipSetDevice(c->device));
    SegInfo g;
    HIP_TRY(c, hipDeviceSynchronize());
    HIP_TRY(c, hipMemcpy(&g, as<SegInfo>(c->si) + segment, sizeof(SegInfo), hipMemcpyDeviceToHost));
    box[0] = g.a0; box[1] = g.na; box[2] = g.u0; box[3] = g.nu; box[4] = g.v0; box[5] = g.nv;
    const int64_t size = (int64_t)g.na * g.nu * g.nv;
    if (!cells_host || cap < size) return LTS_OK;
    std::vector<float> tmp((size_t)g.nu * g.nv * g.na_pad);
    HIP_TRY(c, hipMemcpy(tmp.data(), as<float>(c->cells) + g.cell_off, sizeof(float) * tmp.size(), hipMemcpyDeviceToHost));
    for (int32_t a = 0; a < g.na; ++a)
        for (int32_t u = 0; u < g.nu; ++u)
            for (int32_t v = 0; v < g.nv; ++v)
                cells_host[((int64_t)a * g.nu + u) * g.nv + v] = tmp[((size_t)u * g.nv + v) * g.na_pad + a];
    return LTS_OK;
}

lts_status lts_stage_electronics(lts_context *c, uint64_t event_id, const int32_t *pixel_ids, const float *current,
                                 int64_t n_pix, const lts_outputs *out, void *stream) {
    if (!c) return LTS_ERR_INVALID_ARG;
    if (!pixel_ids || !current || n_pix < 0 || !out || !out->counts)
        return fail(c, LTS_ERR_INVALID_ARG, "bad electronics stage arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = to_stream(stream);
    lts_status r;
    const int64_t mp = c->P.max_packets;
    if ((r = ensure(c, c->pk_tick, sizeof(int32_t) * (size_t)(n_pix * mp)))) return r;
    if ((r = ensure(c, c->pk_adc, sizeof(uint16_t) * (size_t)(n_pix * mp)))) return r;
    if ((r = ensure(c, c->pk_flag, sizeof(uint8_t) * (size_t)(n_pix * mp)))) return r;
    if ((r = ensure(c, c->pk_off, sizeof(int64_t) * (size_t)(n_pix + 1)))) return r;
    if ((r = ensure(c, c->hdr, sizeof(DevHeader)))) return r;
    if ((r = ensure(c, c->ev_ids, sizeof(uint64_t)))) return r;
    if ((r = ensure(c, c->report_tmp, sizeof(double) * 5))) return r;
    if ((r = ensure(c, c->scan_tmp, sizeof(int64_t) * (size_t)scan_tmp_needed(n_pix + 1)))) return r;
    HIP_TRY(c, hipMemcpyAsync(c->ev_ids.p, &event_id, sizeof(uint64_t), hipMemcpyHostToDevice, st));
    HIP_TRY(c, hipMemsetAsync(c->hdr.p, 0, sizeof(DevHeader), st));
    HIP_TRY(c, hipMemsetAsync(c->pk_off.p, 0, sizeof(int64_t) * (size_t)(n_pix + 1), st));
    double *rep = out->report ? out->report : as<double>(c->report_tmp);
    HIP_TRY(c, hipMemsetAsync(rep, 0, sizeof(double) * 5, st));
    Work w;
    w.n_ev = 1;
    w.pk_tick = as<int32_t>(c->pk_tick);
    w.pk_adc = as<uint16_t>(c->pk_adc);
    w.pk_flag = as<uint8_t>(c->pk_flag);
    w.pk_off = as<int64_t>(c->pk_off);
    w.hdr = as<DevHeader>(c->hdr);
    w.report = rep;
    w.scan_tmp = c->scan_tmp.p;
    w.slot_gp = const_cast<int32_t *>(pixel_ids);
    launch_electronics(c->P, current, pixel_ids, as<uint64_t>(c->ev_ids), n_pix, w, st);
    launch_compact_packets(c->P, w, n_pix, out->pkt_pixel, out->pkt_tick, out->pkt_adc, out->pkt_flags, out->cap_packets,
                           nullptr, nullptr, out->counts, st);
    HIP_TRY(c, hipGetLastError());
    return LTS_OK;
}

lts_status lts_stage_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out, int64_t n, void *stream) {
    if (!ctr || !out || n < 0) return LTS_ERR_INVALID_ARG;
    launch_philox(ctr, k0, k1, out, n, to_stream(stream));
    return hipGetLastError() == hipSuccess ? LTS_OK : LTS_ERR_DEVICE;
}

}  // extern "C"
