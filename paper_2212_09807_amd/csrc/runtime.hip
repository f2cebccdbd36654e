// runtime.hip -- C ABI of libltsim (see include/ltsim.h): contexts, the device-resident field-response table, the
// scratch pool and the stage sequence of one event or a batch of events.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ltsim.h"
#include "admission.hpp"
#include "api.hpp"
#include "device.hpp"
#include "launch.hpp"

using namespace ltsim;

std::atomic<int64_t> ltsim::g_host_alloc_fail{-1};

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
    int32_t induce_slices = 1;       // sorted variant: table slices (one per XCD); 1 = unsliced kernel
    int32_t ticks_per_thread = 0;    // induction tick tile per thread (0 = chosen from the table length)
    int32_t lane_exchange = 0;       // 8-tick tiles share table windows across lanes (1) or load their own (0)
    int32_t matrix_cores = 0;        // sorted per-pair induction on the FP32 matrix cores (1) or the vector ALUs (0)
    std::vector<lts_tuning> tuning;  // autotuned work split per event-size class (empty = the settings above)
    // HIP-graph replay of the launch sequence after the sizing read-back (per-pair and atomic modes)
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;  // capture stream (captures never run on the caller's stream)
    // summed mode: the charge cells run on a side stream beside the column lists (which need only the boxes)
    hipStream_t side_stream = nullptr;
    hipEvent_t side_fork = nullptr, side_join = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t gdone = nullptr;        // recorded behind every graph launch
    bool glaunched = false;
    int64_t graph_updates = 0, graph_instantiations = 0;
    DevBuf part;                     // per-slice partial waveforms of the sliced sorted variant
    DevBuf mask;                     // disabled-channel mask (npx bytes) when set
    bool has_mask = false;
    DevBuf col_seg_off, col_cursor, col_seg, col_tmp, piece_off, s_off, piece, pdesc, S, list_off, list, rec;
    DevBuf mlist_off, m_off, mrec, Sm;          // the mirror-merged records of the summed induction
    DevBuf segc;                                // compact segment fields for the column passes
    DevParams P{};
    bool has_table = false;
    DevBuf Rpad, prefix;
    std::vector<float> table_host;   // kept to build server lanes
    int32_t t_r = 0, b_x = 0, b_y = 0;
    // scratch pool
    DevBuf si, cell_off, pix_cnt, cursor, pix_slot, slot_gp, slot_off, pairs_u, pairs, cells, pk_tick, pk_adc,
        pk_flag, pk_off, hdr, scan_tmp, ev_off, ev_ids, report_tmp, counts_tmp, red_head, red_start, order;
    DevHeader *hdr_host = nullptr;   // pinned
    int64_t last_n_seg = -1;
    int64_t last_n_slots = 0;
    int32_t last_mode = -1;
    int32_t last_rt = 0;                        // the last summed call's kernel choice (ticks per thread, exchange)
    bool last_shift = false;
    // optional stage timing: HIP events recorded on the caller's stream around each stage group
    bool timing = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending_ev;
    std::vector<hipEvent_t> free_ev;
    double stage_ms[LTS_N_STAGES] = {0};
    int64_t stage_calls[LTS_N_STAGES] = {0};
    // stream order of the calls on this context: every call that uses the scratch pool waits for the previous one
    // (an event recorded on the previous call's stream), so calls on different streams never share scratch in flight
    hipEvent_t call_done = nullptr;
    bool call_recorded = false;
    // request-loop lanes only: asked, once the sizes of a call are known, whether the call may grow the context's
    // pool to `total` bytes (`growth` of them not yet allocated); it also sizes the lane's outputs.  LTS_OK runs the
    // call, kNotAdmitted abandons it before any further allocation.
    std::function<lts_status(const DevHeader &, int64_t total, int64_t growth)> admit;
    DevBuf ev_cnt;                   // [2 per event] samples dropped past the window, packets over max_packets
    void *noalloc_scratch = nullptr; // this device's copy of the static scratch array (lts_stage_electronics_noalloc)
    std::string err;
    lts_status sticky = LTS_OK;
};

namespace {

lts_status fail(lts_context *c, lts_status s, const std::string &msg) {
    if (c) {
        if (s == LTS_ERR_DEVICE) c->sticky = LTS_ERR_DEVICE;
        c->err = msg;
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
    // buffers grow to exactly the size asked for (the request loop's admission accounts for them byte for byte)
    const hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(c, LTS_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    b.bytes = bytes;
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
    if (ph.mc_draws < 0 || ph.mc_draws > 65535) return fail(c, LTS_ERR_INVALID_ARG, "mc_draws must be in [0, 65535]");
    if (ph.per_point != 0 && ph.per_point != 1) return fail(c, LTS_ERR_INVALID_ARG, "per_point must be 0 or 1");
    if (ph.per_point && ph.mc_draws > 0)
        return fail(c, LTS_ERR_INVALID_ARG, "per-point drift is not combined with Monte Carlo diffusion");
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
    if (el.reset_period < 0) return fail(c, LTS_ERR_INVALID_ARG, "reset_period must be >= 0");
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
    P.mc_draws = ph.mc_draws;
    P.per_point = ph.per_point;
    P.cell_pad = kAC;                              // set per call by the sizing pass
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
    // a hold or spacing beyond 2^20 ticks acts as one of 2^20 (every later sample falls past the last tick, and the
    // "no sample yet" sentinel of -2^28 stays below tick 0); the clamp keeps the tick arithmetic inside int32
    P.hold = std::min(el.hold_ticks, 1 << 20);
    P.spacing = std::min(el.min_spacing, 1 << 20);
    P.pedestal = el.pedestal;
    P.adc_max = (1 << el.adc_bits) - 1;
    P.max_packets = el.max_packets;
    P.reset_period = el.reset_period;
    P.key0 = (uint32_t)(el.seed & 0xffffffffu);
    P.key1 = (uint32_t)(el.seed >> 32);
    P.eps_rel = 2e-6f;
    P.eps_abs = 0.05f;
    return LTS_OK;
}

template <typename T>
T *as(DevBuf &b) { return (T *)b.p; }

// A call's refusal by the request loop's admission: a status the pipeline returns for nothing else (only the
// server's poll uses it, for unfinished tickets); the lanes turn it into a smaller batch or LTS_ERR_OOM.
constexpr lts_status kNotAdmitted = LTS_ERR_NOT_READY;

std::vector<DevBuf *> pool_buffers(lts_context *c) {
    return {&c->ev_cnt, &c->mask, &c->col_seg_off, &c->col_cursor, &c->col_seg, &c->col_tmp, &c->piece_off,
            &c->s_off, &c->piece, &c->pdesc, &c->S, &c->list_off, &c->list, &c->rec, &c->mlist_off, &c->m_off,
            &c->mrec, &c->Sm, &c->segc, &c->part, &c->Rpad, &c->prefix, &c->si, &c->cell_off, &c->pix_cnt, &c->cursor,
            &c->pix_slot, &c->slot_gp, &c->slot_off, &c->pairs_u, &c->pairs, &c->cells, &c->pk_tick, &c->pk_adc,
            &c->pk_flag, &c->pk_off, &c->hdr, &c->scan_tmp, &c->ev_off, &c->ev_ids, &c->report_tmp, &c->counts_tmp,
            &c->red_head, &c->red_start, &c->order};
}

// Frees the context's per-call scratch (everything in the pool but the response table and the channel mask, which
// persist across calls); every buffer is grown again to the exact size the next call needs.  The caller makes sure
// no queued work still uses them.
void release_scratch(lts_context *c) {
    for (DevBuf *b : pool_buffers(c))
        if (b != &c->Rpad && b != &c->prefix && b != &c->mask) free_buf(*b);
}

// One buffer and the bytes a call needs in it.
struct Need {
    DevBuf *b;
    size_t bytes;
};

// Grows the listed buffers to their needs, first asking the admission hook (if any) whether the pool may grow.
lts_status grow(lts_context *c, const DevHeader &h, const std::vector<Need> &needs) {
    if (c->admit) {
        int64_t total = 0, growth = 0;
        for (DevBuf *b : pool_buffers(c)) total += (int64_t)b->bytes;
        for (const Need &n : needs) {
            const size_t want = std::max<size_t>(n.bytes, 16);
            if (want > n.b->bytes) growth += (int64_t)(want - n.b->bytes);
        }
        const lts_status r = c->admit(h, total + growth, growth);
        if (r) return r;
    }
    lts_status r;
    for (const Need &n : needs)
        if ((r = ensure(c, *n.b, n.bytes))) return r;
    return LTS_OK;
}

// Orders a call that uses the context's scratch after the previous such call, whatever streams they use: the
// constructor makes `st` wait for the previous call's completion event, the destructor records it on `st`.
struct CallOrder {
    lts_context *c;
    hipStream_t st;
    lts_status status = LTS_OK;
    CallOrder(lts_context *c_, hipStream_t st_) : c(c_), st(st_) {
        if (!c->call_done && hipEventCreateWithFlags(&c->call_done, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            c->call_done = nullptr;
            status = fail(c, LTS_ERR_DEVICE, "hipEventCreateWithFlags failed");
            return;
        }
        if (c->call_recorded && hipStreamWaitEvent(st, c->call_done, 0) != hipSuccess) {
            (void)hipGetLastError();
            status = fail(c, LTS_ERR_DEVICE, "hipStreamWaitEvent failed");
        }
    }
    ~CallOrder() {
        if (!c->call_done) return;
        if (hipEventRecord(c->call_done, st) == hipSuccess) c->call_recorded = true;
        else (void)hipGetLastError();
    }
};

hipEvent_t take_event(lts_context *c) {
    if (!c->free_ev.empty()) {
        hipEvent_t e = c->free_ev.back();
        c->free_ev.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Brackets a stage group with events on the stream when timing is enabled.
struct StageTimer {
    lts_context *c;
    hipStream_t st;
    int stage;
    hipEvent_t a = nullptr;
    StageTimer(lts_context *c_, hipStream_t st_, int stage_) : c(c_), st(st_), stage(stage_) {
        if (c->timing && (a = take_event(c))) (void)hipEventRecord(a, st);
    }
    ~StageTimer() {
        if (!a) return;
        hipEvent_t b = take_event(c);
        if (!b) { c->free_ev.push_back(a); return; }
        (void)hipEventRecord(b, st);
        c->pending_ev.push_back({stage, {a, b}});
    }
};

hipStream_t to_stream(void *s) { return (hipStream_t)s; }

// Device-resident scratch of lts_stage_electronics_noalloc, for callers that cannot allocate (graph capture, tight
// serving loops).  Each device holds its own copy from module load to process end.  In host code `scratch` only
// names the symbol: its device address comes from hipGetSymbolAddress, taken once per device (with that device
// current) at context creation and kept in g_scratch_dev; only that address is ever passed to kernels.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// The calling thread's current device must be `device`.
lts_status scratch_address(lts_context *c, int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return LTS_OK;       // the no-alloc entry point then reports STATE
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(c, LTS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_dev[device] = p;
    }
    *out = g_scratch_dev[device];
    return LTS_OK;
}

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
// padded: charge-cell rows in whole 8-tick blocks (the per-pair kernels read them in blocks); the summed mode reads
// each row's ticks only, unpadded.
lts_status run_sizing(lts_context *c, int32_t n_ev, const uint64_t *event_ids, const int64_t *seg_offsets,
                      const lts_segments *segs, double *report, hipStream_t st, Work &w, DevHeader &h, bool padded) {
    lts_status r;
    c->P.cell_pad = padded ? kAC : 1;
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
    if ((r = ensure(c, c->ev_cnt, sizeof(int64_t) * 2 * (size_t)n_ev))) return r;
    HIP_TRY(c, hipMemsetAsync(c->ev_cnt.p, 0, sizeof(int64_t) * 2 * (size_t)n_ev, st));
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
    w.ev_cnt = as<int64_t>(c->ev_cnt);
    w.scan_tmp = c->scan_tmp.p;
    w.disabled = c->has_mask ? as<uint8_t>(c->mask) : nullptr;
    SegArrays S = seg_arrays(segs);
    {
        StageTimer t(c, st, LTS_STAGE_QUENCH_DRIFT);
        launch_quench_drift(c->P, S, w, st);
    }
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

// Sum-then-convolve induction (exact by linearity): columns summed over segments, then the sorted induction kernel
// over per-pixel lists of column pieces.
// Absolute sub-pixel column grid of the summed induction: per event the columns some in-grid pixel can reach.
SumWork summed_grid(const DevParams &P, int32_t n_ev) {
    SumWork sw;
    const int32_t half = P.nsub / 2;
    sw.UL = half - P.bx;
    sw.VL = half - P.by;
    sw.CU = (P.nx - 1) * P.nsub + 2 * P.bx;
    sw.CV = (P.ny - 1) * P.nsub + 2 * P.by;
    sw.n_cols = (int64_t)n_ev * sw.CU * sw.CV;
    return sw;
}

// Buffers of the summed induction whose sizes the sizing pass already fixes (column lists, offsets, pixel lists).
void summed_needs(lts_context *c, const DevHeader &h, int64_t n_slots, int32_t n_ev, int64_t n_seg,
                  std::vector<Need> &needs) {
    const SumWork sw = summed_grid(c->P, n_ev);
    const int64_t nc1 = sw.n_cols + 1;
    needs.push_back({&c->segc, sizeof(SumSeg) * (size_t)std::max<int64_t>(n_seg, 1)});
    needs.push_back({&c->col_seg_off, sizeof(int64_t) * (size_t)nc1});
    needs.push_back({&c->col_cursor, sizeof(int32_t) * (size_t)sw.n_cols});
    needs.push_back({&c->col_seg, sizeof(uint64_t) * (size_t)std::max<int64_t>(h.n_colseg, 1)});
    needs.push_back({&c->col_tmp, sizeof(uint64_t) * (size_t)std::max<int64_t>(h.n_colseg, 1)});
    needs.push_back({&c->piece_off, sizeof(int64_t) * (size_t)nc1});
    needs.push_back({&c->s_off, sizeof(int64_t) * (size_t)nc1});
    needs.push_back({&c->list_off, sizeof(int64_t) * (size_t)(n_slots + 1)});
    needs.push_back({&c->mlist_off, sizeof(int64_t) * (size_t)(n_slots + 1)});
    needs.push_back({&c->m_off, sizeof(int64_t) * (size_t)(n_slots + 1)});
    needs.push_back({&c->scan_tmp, sizeof(int64_t) * (size_t)scan_tmp_needed(std::max(nc1, n_slots + 1))});
}

// The buffers of summed_needs are grown by the caller.
// cells_ready (may be null): recorded behind the charge cells on another stream; awaited before the column sums.
lts_status run_summed(lts_context *c, const Work &w, const DevHeader &h, int64_t n_slots, float *wave, hipStream_t st,
                      hipEvent_t cells_ready) {
    const DevParams &P = c->P;
    lts_status r;
    SumWork sw = summed_grid(P, w.n_ev);
    const int64_t nc1 = sw.n_cols + 1;
    if (sw.n_cols > (int64_t)INT32_MAX)
        return fail(c, LTS_ERR_INVALID_ARG, "summed induction: events x sub-pixel columns exceeds 2^31 - 1");
    sw.segc = as<SumSeg>(c->segc);
    sw.col_seg_off = as<int64_t>(c->col_seg_off);
    sw.col_cursor = as<int32_t>(c->col_cursor);
    sw.col_seg = as<uint64_t>(c->col_seg);
    sw.col_tmp = as<uint64_t>(c->col_tmp);
    sw.active = as<int32_t>(c->col_cursor);         // the fill's cursors are free once the lists are filled
    sw.n_active = &w.hdr->work[3];
    sw.piece_off = as<int64_t>(c->piece_off);
    sw.s_off = as<int64_t>(c->s_off);
    sw.list_off = as<int64_t>(c->list_off);
    sw.mlist_off = as<int64_t>(c->mlist_off);
    sw.m_off = as<int64_t>(c->m_off);
    sw.align_res = summed_align_res(P, c->ticks_per_thread, c->lane_exchange != 0);
    sw.piece_lists = !((c->ticks_per_thread == 0 || c->ticks_per_thread == 8) && c->lane_exchange == 0);
    void *tmp = c->scan_tmp.p;
    HIP_TRY(c, hipMemsetAsync(sw.col_seg_off, 0, sizeof(int64_t) * (size_t)nc1, st));
    HIP_TRY(c, hipMemsetAsync(sw.col_cursor, 0, sizeof(int32_t) * (size_t)sw.n_cols, st));
    HIP_TRY(c, hipMemsetAsync(sw.piece_off + sw.n_cols, 0, sizeof(int64_t), st));
    HIP_TRY(c, hipMemsetAsync(sw.s_off + sw.n_cols, 0, sizeof(int64_t), st));
    HIP_TRY(c, hipMemsetAsync(sw.list_off + n_slots, 0, sizeof(int64_t), st));
    HIP_TRY(c, hipMemsetAsync(sw.mlist_off + n_slots, 0, sizeof(int64_t), st));
    HIP_TRY(c, hipMemsetAsync(sw.m_off + n_slots, 0, sizeof(int64_t), st));
    launch_sum_ranges(P, w, sw, st);
    scan_exclusive_i64(sw.col_seg_off, nc1, nullptr, tmp, st);
    launch_sum_fill(P, w, sw, st);
    scan_exclusive_i64(sw.piece_off, nc1, nullptr, tmp, st);
    scan_exclusive_i64(sw.s_off, nc1, nullptr, tmp, st);
    // exact sizes of the piece records and the summed charges (a column's merged tick intervals are only known
    // after its segments are sorted)
    int64_t tot[3] = {0, 0, 0};
    HIP_TRY(c, hipMemcpyAsync(&tot[1], sw.piece_off + sw.n_cols, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipMemcpyAsync(&tot[2], sw.s_off + sw.n_cols, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (tot[2] / kAC >= (int64_t)UINT32_MAX)          // piece records hold the charge offset in units of kAC floats
        return fail(c, LTS_ERR_CAPACITY, "summed induction: too many summed charge values for one call");
    if ((r = grow(c, h, {{&c->pdesc, sizeof(PieceRef) * (size_t)std::max<int64_t>(tot[1], 1)},
                         {&c->S, sizeof(float) * (size_t)(tot[2] + kCellSlack)}})))
        return r;
    if (sw.piece_lists) {
        if ((r = grow(c, h, {{&c->piece, sizeof(SegInfo) * (size_t)std::max<int64_t>(tot[1], 1)}}))) return r;
        sw.piece = as<SegInfo>(c->piece);
    }
    sw.pdesc = as<PieceRef>(c->pdesc);
    sw.S = as<float>(c->S);
    if (cells_ready) HIP_TRY(c, hipStreamWaitEvent(st, cells_ready, 0));
    launch_sum_pieces(P, w, sw, st);
    launch_sum_lists_count(P, w, sw, n_slots, st);
    scan_exclusive_i64(sw.list_off, n_slots + 1, nullptr, tmp, st);
    HIP_TRY(c, hipMemcpyAsync(&tot[0], sw.list_off + n_slots, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if ((r = grow(c, h, {{&c->rec, sizeof(PieceRef) * (size_t)std::max<int64_t>(tot[0], 1)}}))) return r;
    if (sw.piece_lists) {
        if ((r = grow(c, h, {{&c->list, sizeof(int32_t) * (size_t)std::max<int64_t>(tot[0], 1)}}))) return r;
        sw.list = as<int32_t>(c->list);
    }
    sw.rec = as<PieceRef>(c->rec);
    launch_sum_lists_fill(P, w, sw, n_slots, tot[0], st);
    // mirror merge: sizes of the merged records and charges, then the records
    sw.nS8 = (uint32_t)(tot[2] / kAC);
    launch_sum_merge(sw, n_slots, false, st);
    scan_exclusive_i64(sw.mlist_off, n_slots + 1, nullptr, tmp, st);
    scan_exclusive_i64(sw.m_off, n_slots + 1, nullptr, tmp, st);
    int64_t mt[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(&mt[0], sw.mlist_off + n_slots, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipMemcpyAsync(&mt[1], sw.m_off + n_slots, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (tot[2] / kAC + mt[1] / kAC >= (int64_t)UINT32_MAX)
        return fail(c, LTS_ERR_CAPACITY, "summed induction: too many summed charge values for one call");
    if ((r = grow(c, h, {{&c->mrec, sizeof(PieceRef) * (size_t)std::max<int64_t>(mt[0], 1)},
                         {&c->Sm, sizeof(float) * (size_t)(mt[1] + kCellSlack)}})))
        return r;
    sw.mrec = as<PieceRef>(c->mrec);
    sw.Sm = as<float>(c->Sm);
    launch_sum_merge(sw, n_slots, true, st);
    Table T{as<float>(c->Rpad), as<double>(c->prefix)};
    const int32_t *order = launch_summed_order(w, sw, n_slots, c->ticks_per_thread, c->lane_exchange != 0, st);
    StageTimer tk(c, st, LTS_STAGE_INDUCE_KERNEL);
    launch_induce_summed(P, w, sw, T, wave, n_slots, c->ticks_per_thread, c->lane_exchange != 0, order, st);
    return LTS_OK;
}

// Captures the launch sequence `launch` on the context's capture stream, brings the context's executable graph up
// to date (an update when the node structure is unchanged, else a new instantiation) and launches it on `st`.  The
// executable graph is only changed after its previous launch has finished.  Stage timing is not recorded here.
template <class Launch>
lts_status run_graph(lts_context *c, hipStream_t st, Launch &launch) {
    if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    if (!c->gdone) HIP_TRY(c, hipEventCreateWithFlags(&c->gdone, hipEventDisableTiming));
    if (c->glaunched) HIP_TRY(c, hipEventSynchronize(c->gdone));
    const bool timing = c->timing;
    c->timing = false;
    HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    const lts_status r = launch(c->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
    c->timing = timing;
    if (r) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (ec != hipSuccess || !g) return fail(c, LTS_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
    bool ok = false;
    if (c->gexec) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        ok = hipGraphExecUpdate(c->gexec, g, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
        (void)hipGetLastError();                        // a refused update is not an error of this call
        if (ok) {
            ++c->graph_updates;
        } else {
            (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
        }
    }
    if (!ok) {
        const hipError_t ei = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            c->gexec = nullptr;
            (void)hipGraphDestroy(g);
            return fail(c, LTS_ERR_DEVICE, std::string("graph instantiation: ") + hipGetErrorString(ei));
        }
        ++c->graph_instantiations;
    }
    (void)hipGraphDestroy(g);
    HIP_TRY(c, hipGraphLaunch(c->gexec, st));
    HIP_TRY(c, hipEventRecord(c->gdone, st));
    c->glaunched = true;
    return LTS_OK;
}

// For the duration of one call: the tuning table's entry for the call's mean event size replaces the context's
// work-split settings (restored afterwards).
struct TunedKnobs {
    lts_context *c;
    int32_t mode, slices, rt, shift;
    TunedKnobs(lts_context *c_, int64_t n_seg, int32_t n_ev)
        : c(c_), mode(c_->reduce_mode), slices(c_->induce_slices), rt(c_->ticks_per_thread), shift(c_->lane_exchange) {
        if (c->tuning.empty() || n_ev < 1) return;
        const int64_t mean = n_seg / n_ev;
        const lts_tuning *t = &c->tuning[0];
        for (const lts_tuning &e : c->tuning)
            if (e.min_segments_per_event <= mean) t = &e;
        c->reduce_mode = t->reduce_mode;
        c->induce_slices = t->induce_slices;
        c->ticks_per_thread = t->ticks_per_thread;
        c->lane_exchange = t->lane_exchange;
    }
    ~TunedKnobs() {
        c->reduce_mode = mode;
        c->induce_slices = slices;
        c->ticks_per_thread = rt;
        c->lane_exchange = shift;
    }
};

lts_status run_pipeline(lts_context *c, int32_t n_ev, const uint64_t *event_ids, const int64_t *seg_offsets,
                        const lts_segments *segs, const lts_outputs *out, hipStream_t st) {
    if (c->sticky) return fail(c, c->sticky, "context is in a failed state: " + c->err);
    TunedKnobs tuned(c, segs ? segs->n : 0, n_ev);
    if (!c->has_table) return fail(c, LTS_ERR_STATE, "no response table: call lts_set_response first");
    lts_status r;
    if ((r = check_segments(c, segs))) return r;
    if (!out || !out->counts || !out->report || !out->pixel_id || !out->current)
        return fail(c, LTS_ERR_INVALID_ARG, "outputs: pixel_id, current, counts and report are required");
    if (n_ev < 1 || !event_ids || !seg_offsets) return fail(c, LTS_ERR_INVALID_ARG, "bad event list");
    HIP_TRY(c, hipSetDevice(c->device));
    CallOrder order_(c, st);
    if (order_.status) return order_.status;
    Work w;
    DevHeader h;
    if ((r = run_sizing(c, n_ev, event_ids, seg_offsets, segs, out->report, st, w, h,
                        c->reduce_mode != LTS_REDUCE_SUMMED)))
        return r;
    const int64_t n_slots = h.n_slots, n_pairs = h.n_pairs, n_cells = h.n_cells;
    c->last_n_slots = n_slots;
    c->last_mode = c->reduce_mode;
    c->last_rt = c->ticks_per_thread;
    c->last_shift = c->lane_exchange != 0;
    const int64_t mp = c->P.max_packets;
    const bool summed = c->reduce_mode == LTS_REDUCE_SUMMED;
    const int64_t pair_cap = summed ? 1 : std::max<int64_t>(n_pairs, 1);   // the summed induction has no pair lists
    std::vector<Need> needs = {
        {&c->slot_gp, sizeof(int32_t) * (size_t)std::max<int64_t>(n_slots, 1)},
        {&c->slot_off, sizeof(int64_t) * (size_t)(n_slots + 1)},
        {&c->pairs_u, sizeof(int32_t) * (size_t)pair_cap},
        {&c->pairs, sizeof(int32_t) * (size_t)pair_cap},
        {&c->cells, sizeof(float) * (size_t)(n_cells + kCellSlack)},
        {&c->pk_tick, sizeof(int32_t) * (size_t)(n_slots * mp)},
        {&c->pk_adc, sizeof(uint16_t) * (size_t)(n_slots * mp)},
        {&c->pk_flag, sizeof(uint8_t) * (size_t)(n_slots * mp)},
        {&c->pk_off, sizeof(int64_t) * (size_t)(n_slots + 1)},
        {&c->scan_tmp, sizeof(int64_t) * (size_t)scan_tmp_needed(n_slots + 1)},
        {&c->order, sizeof(int32_t) * (size_t)(2 * n_slots + 2 * kOrderBuckets)}};
    if (c->reduce_mode == LTS_REDUCE_SUMMED) summed_needs(c, h, n_slots, n_ev, w.n_seg, needs);
    if (c->reduce_mode == LTS_REDUCE_SORTED && c->induce_slices > 1 && n_slots > 0) {
        const int64_t row_bytes = (int64_t)c->induce_slices * c->P.nticks * (int64_t)sizeof(float);
        const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n_slots, (1ll << 30) / row_bytes));
        needs.push_back({&c->part, (size_t)(row_bytes * chunk)});
    }
    // the admission hook (request-loop lanes) sizes the outputs: the capacity check comes after it
    if ((r = grow(c, h, needs))) return r;
    if (n_slots > out->cap_pixels) {
        int64_t need[4] = {n_slots, n_slots * mp, 0, 0};
        HIP_TRY(c, hipMemcpy(out->counts, need, sizeof(need), hipMemcpyHostToDevice));
        return fail(c, LTS_ERR_CAPACITY, "cap_pixels " + std::to_string(out->cap_pixels) + " < " + std::to_string(n_slots));
    }
    w.order = as<int32_t>(c->order);
    w.slot_gp = as<int32_t>(c->slot_gp);
    w.slot_off = as<int64_t>(c->slot_off);
    w.pairs_unsorted = summed ? nullptr : as<int32_t>(c->pairs_u);
    w.pairs = summed ? nullptr : as<int32_t>(c->pairs);
    w.cells = as<float>(c->cells);
    w.pk_tick = as<int32_t>(c->pk_tick);
    w.pk_adc = as<uint16_t>(c->pk_adc);
    w.pk_flag = as<uint8_t>(c->pk_flag);
    w.pk_off = as<int64_t>(c->pk_off);
    w.scan_tmp = c->scan_tmp.p;
    const DevParams &P = c->P;
    Table T{as<float>(c->Rpad), as<double>(c->prefix)};
    // The sequence from here to the packets has no host synchronisation in the per-pair and atomic modes, so it can
    // be captured and replayed as one HIP graph (zero fills are kernels, not memset nodes).
    const bool graph = c->use_graph && c->reduce_mode != LTS_REDUCE_SUMMED;
    auto launch_all = [&](hipStream_t s) -> lts_status {
        launch_zero(w.pk_off, (int64_t)sizeof(int64_t) * (n_slots + 1), s);
        {
            StageTimer t(c, s, LTS_STAGE_RASTERIZE);
            launch_slots(P, w, out->pixel_id, out->event_pixel_offsets, s);
            launch_fill_pairs(P, w, s);
            if (c->reduce_mode == LTS_REDUCE_SORTED) launch_sort_pairs(w, n_slots, s);
        }
        // summed mode: the cells on the side stream, beside the column lists (forked after everything queued so far,
        // joined before the column sums and before anything this call leaves behind)
        hipEvent_t cells_ready = nullptr;
        if (summed && !graph) {
            if (!c->side_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking));
            if (!c->side_fork) HIP_TRY(c, hipEventCreateWithFlags(&c->side_fork, hipEventDisableTiming));
            if (!c->side_join) HIP_TRY(c, hipEventCreateWithFlags(&c->side_join, hipEventDisableTiming));
            HIP_TRY(c, hipEventRecord(c->side_fork, s));
            HIP_TRY(c, hipStreamWaitEvent(c->side_stream, c->side_fork, 0));
            {
                StageTimer t(c, c->side_stream, LTS_STAGE_CELLS);
                launch_cells(P, w, c->side_stream);
            }
            HIP_TRY(c, hipEventRecord(c->side_join, c->side_stream));
            cells_ready = c->side_join;
        } else {
            StageTimer t(c, s, LTS_STAGE_CELLS);
            launch_cells(P, w, s);
        }
        if (c->reduce_mode == LTS_REDUCE_ATOMIC)
            launch_zero(out->current, (int64_t)sizeof(float) * n_slots * P.nticks, s);
        if (c->reduce_mode == LTS_REDUCE_SUMMED) {
            lts_status r2;
            {
                StageTimer t(c, s, LTS_STAGE_INDUCE);
                r2 = run_summed(c, w, h, n_slots, out->current, s, cells_ready);
            }
            if (cells_ready) HIP_TRY(c, hipStreamWaitEvent(s, cells_ready, 0));   // also on an early return
            if (r2) return r2;
        } else if (c->reduce_mode == LTS_REDUCE_SORTED && c->induce_slices > 1 && n_slots > 0) {
            // slices of at most 1 GiB of partial waveforms at a time
            const int64_t row_bytes = (int64_t)c->induce_slices * P.nticks * (int64_t)sizeof(float);
            const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n_slots, (1ll << 30) / row_bytes));
            StageTimer t(c, s, LTS_STAGE_INDUCE);
            launch_induce_slices(P, w, T, out->current, n_slots, c->induce_slices, as<float>(c->part), chunk,
                                 c->ticks_per_thread, s);
        } else if (c->reduce_mode == LTS_REDUCE_SORTED && c->matrix_cores) {
            StageTimer t(c, s, LTS_STAGE_INDUCE);
            StageTimer tk(c, s, LTS_STAGE_INDUCE_KERNEL);
            launch_induce_mfma(P, w, T, out->current, n_slots, s);
        } else {
            StageTimer t(c, s, LTS_STAGE_INDUCE);
            StageTimer tk(c, s, LTS_STAGE_INDUCE_KERNEL);
            launch_induce(P, w, T, out->current, c->reduce_mode, n_slots, c->ticks_per_thread, c->lane_exchange != 0,
                          s);
        }
        {
            StageTimer t(c, s, LTS_STAGE_ELECTRONICS);
            launch_electronics(P, out->current, w.slot_gp, w.event_ids, n_slots, w, s);
            launch_compact_packets(P, w, n_slots, out->pkt_pixel, out->pkt_tick, out->pkt_adc, out->pkt_flags,
                                   out->cap_packets, out->event_pixel_offsets, out->event_packet_offsets, out->counts,
                                   s);
        }
        return LTS_OK;
    };
    if (!graph) {
        if ((r = launch_all(st))) return r;
    } else {
        if ((r = run_graph(c, st, launch_all))) return r;
    }
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
    LTS_API_BEGIN
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
    if (r == LTS_OK) r = scratch_address(c, device, &c->noalloc_scratch);
    if (r == LTS_OK && hipHostMalloc((void **)&c->hdr_host, sizeof(DevHeader), hipHostMallocDefault) != hipSuccess)
        r = LTS_ERR_OOM;
    if (r != LTS_OK) {
        delete c;
        return r;
    }
    *out = c;
    return LTS_OK;
    LTS_API_END(nullptr)
}

void lts_context_destroy(lts_context *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->glaunched) (void)hipEventSynchronize(c->gdone);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->gdone) (void)hipEventDestroy(c->gdone);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->side_stream) {
        (void)hipStreamSynchronize(c->side_stream);
        (void)hipStreamDestroy(c->side_stream);
    }
    if (c->side_fork) (void)hipEventDestroy(c->side_fork);
    if (c->side_join) (void)hipEventDestroy(c->side_join);
    for (auto &pe : c->pending_ev) {
        (void)hipEventDestroy(pe.second.first);
        (void)hipEventDestroy(pe.second.second);
    }
    for (hipEvent_t e : c->free_ev) (void)hipEventDestroy(e);
    if (c->call_done) {
        (void)hipEventSynchronize(c->call_done);
        (void)hipEventDestroy(c->call_done);
    }
    for (DevBuf *b : pool_buffers(c)) free_buf(*b);
    if (c->hdr_host) (void)hipHostFree(c->hdr_host);
    delete c;
}

lts_status lts_set_timing(lts_context *c, int32_t enabled) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    c->timing = enabled != 0;
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_get_timing(lts_context *c, double ms[LTS_N_STAGES], int64_t calls[LTS_N_STAGES]) {
    LTS_API_BEGIN
    if (!c || !ms) return LTS_ERR_INVALID_ARG;
    HIP_TRY(c, hipSetDevice(c->device));
    for (auto &pe : c->pending_ev) {
        float t = 0.0f;
        HIP_TRY(c, hipEventSynchronize(pe.second.second));
        HIP_TRY(c, hipEventElapsedTime(&t, pe.second.first, pe.second.second));
        c->stage_ms[pe.first] += t;
        c->stage_calls[pe.first] += 1;
        c->free_ev.push_back(pe.second.first);
        c->free_ev.push_back(pe.second.second);
    }
    c->pending_ev.clear();
    for (int i = 0; i < LTS_N_STAGES; ++i) {
        ms[i] = c->stage_ms[i];
        if (calls) calls[i] = c->stage_calls[i];
        c->stage_ms[i] = 0.0;
        c->stage_calls[i] = 0;
    }
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_set_induce_slices(lts_context *c, int32_t slices) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (slices < 1 || slices > 64) return fail(c, LTS_ERR_INVALID_ARG, "slices must be in [1, 64]");
    c->induce_slices = slices;
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_set_ticks_per_thread(lts_context *c, int32_t rt) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (rt != 0 && rt != 1 && rt != 2 && rt != 4 && rt != 8)
        return fail(c, LTS_ERR_INVALID_ARG, "ticks per thread must be 0 (auto), 1, 2, 4 or 8");
    c->ticks_per_thread = rt;
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_set_lane_exchange(lts_context *c, int32_t on) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (on != 0 && on != 1) return fail(c, LTS_ERR_INVALID_ARG, "lane exchange must be 0 or 1");
    c->lane_exchange = on;
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_set_matrix_cores(lts_context *c, int32_t on) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (on != 0 && on != 1) return fail(c, LTS_ERR_INVALID_ARG, "matrix cores must be 0 or 1");
    c->matrix_cores = on;
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_set_graph(lts_context *c, int32_t on) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (on != 0 && on != 1) return fail(c, LTS_ERR_INVALID_ARG, "graph must be 0 or 1");
    c->use_graph = on != 0;
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_graph_stats(lts_context *c, int64_t *updates, int64_t *instantiations) {
    LTS_API_BEGIN
    if (!c || !updates || !instantiations) return LTS_ERR_INVALID_ARG;
    *updates = c->graph_updates;
    *instantiations = c->graph_instantiations;
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_set_channel_mask(lts_context *c, const uint8_t *mask, int64_t n) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (!mask || n == 0) {
        c->has_mask = false;
        return LTS_OK;
    }
    if (n != (int64_t)c->P.npx) return fail(c, LTS_ERR_INVALID_ARG, "channel mask must have n_x * n_y entries");
    HIP_TRY(c, hipSetDevice(c->device));
    lts_status r;
    if ((r = ensure(c, c->mask, (size_t)n))) return r;
    HIP_TRY(c, hipMemcpy(c->mask.p, mask, (size_t)n, hipMemcpyHostToDevice));
    c->has_mask = true;
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_set_tuning(lts_context *c, const lts_tuning *entries, int32_t n) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (!entries || n <= 0) {
        c->tuning.clear();
        return LTS_OK;
    }
    std::vector<lts_tuning> t(entries, entries + n);
    for (int32_t i = 0; i < n; ++i) {
        const lts_tuning &e = t[i];
        if (i > 0 && e.min_segments_per_event <= t[i - 1].min_segments_per_event)
            return fail(c, LTS_ERR_INVALID_ARG, "tuning entries must be in ascending min_segments_per_event");
        if (e.reduce_mode != LTS_REDUCE_SORTED && e.reduce_mode != LTS_REDUCE_ATOMIC && e.reduce_mode != LTS_REDUCE_SUMMED)
            return fail(c, LTS_ERR_INVALID_ARG, "tuning entry: unknown reduce mode");
        if (e.induce_slices < 1 || e.induce_slices > 64)
            return fail(c, LTS_ERR_INVALID_ARG, "tuning entry: slices must be in [1, 64]");
        const int32_t rt = e.ticks_per_thread;
        if (rt != 0 && rt != 1 && rt != 2 && rt != 4 && rt != 8)
            return fail(c, LTS_ERR_INVALID_ARG, "tuning entry: ticks per thread must be 0, 1, 2, 4 or 8");
        if (e.lane_exchange != 0 && e.lane_exchange != 1)
            return fail(c, LTS_ERR_INVALID_ARG, "tuning entry: lane exchange must be 0 or 1");
    }
    c->tuning.swap(t);
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_set_reduce_mode(lts_context *c, int32_t mode) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (mode != LTS_REDUCE_SORTED && mode != LTS_REDUCE_ATOMIC && mode != LTS_REDUCE_SUMMED)
        return fail(c, LTS_ERR_INVALID_ARG, "unknown reduce mode");
    c->reduce_mode = mode;
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_set_response(lts_context *c, const float *R, int32_t t_r, int32_t b_x, int32_t b_y) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (!R || t_r < 1 || t_r > 8192 || b_x < 1 || b_x > 256 || b_y < 1 || b_y > 256)
        return fail(c, LTS_ERR_INVALID_ARG, "response table shape must be 1..8192 x 1..256 x 1..256");
    const size_t ncol = (size_t)b_x * b_y;
    const int32_t col_len = kPad + (t_r + 7) / 8 * 8 + kPad;      // a multiple of 8: columns start 32-byte aligned
    host_alloc_point();
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
    c->table_host.assign(R, R + (size_t)t_r * b_x * b_y);
    c->t_r = t_r;
    c->b_x = b_x;
    c->b_y = b_y;
    c->P.t_r = t_r;
    c->P.bx = b_x;
    c->P.by = b_y;
    c->P.col_len = col_len;
    c->has_table = true;
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_plan(lts_context *c, const lts_segments *segs, int64_t need[4], void *stream) {
    LTS_API_BEGIN
    if (!c || !need) return LTS_ERR_INVALID_ARG;
    if (c->sticky) return fail(c, c->sticky, "context is in a failed state: " + c->err);
    if (!c->has_table) return fail(c, LTS_ERR_STATE, "no response table: call lts_set_response first");
    lts_status r;
    if ((r = check_segments(c, segs))) return r;
    HIP_TRY(c, hipSetDevice(c->device));
    CallOrder order_(c, to_stream(stream));
    if (order_.status) return order_.status;
    if ((r = ensure(c, c->report_tmp, sizeof(double) * 5))) return r;
    const uint64_t eid = 0;
    const int64_t off[2] = {0, segs->n};
    Work w;
    DevHeader h;
    if ((r = run_sizing(c, 1, &eid, off, segs, as<double>(c->report_tmp), to_stream(stream), w, h,
                        c->reduce_mode != LTS_REDUCE_SUMMED)))
        return r;
    need[0] = h.n_pairs;
    need[1] = h.n_slots;
    need[2] = h.n_cells;
    need[3] = h.n_slots * c->P.max_packets;
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_simulate(lts_context *c, uint64_t event_id, const lts_segments *segs, const lts_outputs *out,
                        void *stream) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (!segs) return fail(c, LTS_ERR_INVALID_ARG, "segments is NULL");
    const int64_t off[2] = {0, segs->n};
    return run_pipeline(c, 1, &event_id, off, segs, out, to_stream(stream));
    LTS_API_END(c)
}

lts_status lts_simulate_batch(lts_context *c, int32_t n_events, const uint64_t *event_ids, const int64_t *seg_offsets,
                              const lts_segments *segs, const lts_outputs *out, void *stream) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (out && (!out->event_pixel_offsets || !out->event_packet_offsets))
        return fail(c, LTS_ERR_INVALID_ARG, "batch outputs need event_pixel_offsets and event_packet_offsets");
    return run_pipeline(c, n_events, event_ids, seg_offsets, segs, out, to_stream(stream));
    LTS_API_END(c)
}

lts_status lts_stage_quench_drift(lts_context *c, const lts_segments *segs, float *out_f, int32_t *out_i, void *stream) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    lts_status r;
    if ((r = check_segments(c, segs))) return r;
    if (!out_f || !out_i) return fail(c, LTS_ERR_INVALID_ARG, "NULL output");
    HIP_TRY(c, hipSetDevice(c->device));
    launch_stage_quench_drift(c->P, seg_arrays(segs), segs->n, out_f, out_i, to_stream(stream));
    HIP_TRY(c, hipGetLastError());
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_debug_cells(lts_context *c, int64_t segment, int64_t box[6], float *cells_host, int64_t cap) {
    LTS_API_BEGIN
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
    LTS_API_END(c)
}

lts_status lts_stage_electronics(lts_context *c, uint64_t event_id, const int32_t *pixel_ids, const float *current,
                                 int64_t n_pix, const lts_outputs *out, void *stream) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (!pixel_ids || !current || n_pix < 0 || !out || !out->counts)
        return fail(c, LTS_ERR_INVALID_ARG, "bad electronics stage arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = to_stream(stream);
    CallOrder order_(c, st);
    if (order_.status) return order_.status;
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
    w.disabled = c->has_mask ? as<uint8_t>(c->mask) : nullptr;
    launch_electronics(c->P, current, pixel_ids, as<uint64_t>(c->ev_ids), n_pix, w, st);
    launch_compact_packets(c->P, w, n_pix, out->pkt_pixel, out->pkt_tick, out->pkt_adc, out->pkt_flags, out->cap_packets,
                           nullptr, nullptr, out->counts, st);
    HIP_TRY(c, hipGetLastError());
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_stage_electronics_noalloc(lts_context *c, uint64_t event_id, const int32_t *pixel_ids,
                                         const float *current, int64_t n_pix, const lts_outputs *out, void *stream) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (!pixel_ids || !current || n_pix < 0 || !out || !out->counts)
        return fail(c, LTS_ERR_INVALID_ARG, "bad electronics stage arguments");
    if (!c->noalloc_scratch) return fail(c, LTS_ERR_STATE, "no static scratch on this device");
    // layout of the static scratch: header, event id, report, packet offsets, scan partials, per-slot packets
    const int64_t mp = c->P.max_packets;
    auto up = [](int64_t b) { return (b + 255) / 256 * 256; };
    const int64_t o_hdr = 0, o_ev = up(sizeof(DevHeader)), o_rep = o_ev + 256, o_off = o_rep + 256;
    const int64_t o_scan = o_off + up(8 * (n_pix + 1));
    const int64_t o_tick = o_scan + up(8 * scan_tmp_needed(n_pix + 1));
    const int64_t o_adc = o_tick + up(4 * n_pix * mp);
    const int64_t o_flag = o_adc + up(2 * n_pix * mp);
    const int64_t need = o_flag + up(n_pix * mp);
    if (n_pix > (int64_t)kNoAllocScratchBytes || need > (int64_t)kNoAllocScratchBytes)
        return fail(c, LTS_ERR_INVALID_ARG,
                    "lts_stage_electronics_noalloc: " + std::to_string(n_pix) + " pixels x " + std::to_string(mp) +
                        " packets need " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                        std::to_string(kNoAllocScratchBytes));
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = to_stream(stream);
    unsigned char *base = (unsigned char *)c->noalloc_scratch;
    Work w;
    w.n_ev = 1;
    w.hdr = (DevHeader *)(base + o_hdr);
    w.report = out->report ? out->report : (double *)(base + o_rep);
    w.pk_off = (int64_t *)(base + o_off);
    w.scan_tmp = base + o_scan;
    w.pk_tick = (int32_t *)(base + o_tick);
    w.pk_adc = (uint16_t *)(base + o_adc);
    w.pk_flag = (uint8_t *)(base + o_flag);
    w.slot_gp = const_cast<int32_t *>(pixel_ids);
    w.disabled = c->has_mask ? as<uint8_t>(c->mask) : nullptr;
    // the scratch keeps the previous call's contents: clear what is accumulated (by kernels, not memset nodes, so a
    // caller may capture the call into a graph)
    launch_zero(w.hdr, sizeof(DevHeader), st);
    launch_zero(w.report, sizeof(double) * 5, st);
    launch_zero(w.pk_off, 8 * (n_pix + 1), st);
    launch_store_u64((uint64_t *)(base + o_ev), event_id, st);
    launch_electronics(c->P, current, pixel_ids, (const uint64_t *)(base + o_ev), n_pix, w, st);
    launch_compact_packets(c->P, w, n_pix, out->pkt_pixel, out->pkt_tick, out->pkt_adc, out->pkt_flags, out->cap_packets,
                           nullptr, nullptr, out->counts, st);
    HIP_TRY(c, hipGetLastError());
    return LTS_OK;
    LTS_API_END(c)
}

// Front half of the pipeline for the pair-level hooks: sizing, slots, pixel-major pairs in ascending segment order,
// and (with_cells) the charge cells.  Returns the header; the pair count is h.n_pairs.
static lts_status stage_front(lts_context *c, uint64_t event_id, const lts_segments *segs, bool with_cells,
                              hipStream_t st, Work &w, DevHeader &h) {
    if (c->sticky) return fail(c, c->sticky, "context is in a failed state: " + c->err);
    if (!c->has_table) return fail(c, LTS_ERR_STATE, "no response table: call lts_set_response first");
    lts_status r;
    if ((r = check_segments(c, segs))) return r;
    HIP_TRY(c, hipSetDevice(c->device));
    if ((r = ensure(c, c->report_tmp, sizeof(double) * 5))) return r;
    const int64_t off[2] = {0, segs->n};
    if ((r = run_sizing(c, 1, &event_id, off, segs, as<double>(c->report_tmp), st, w, h, true))) return r;
    // lts_debug_cells and lts_work_stats describe the last call that computed charge cells
    if (!with_cells) c->last_n_seg = -1;
    c->last_mode = LTS_REDUCE_SORTED;
    c->last_n_slots = h.n_slots;
    const int64_t n_slots = h.n_slots, n_pairs = h.n_pairs;
    if ((r = ensure(c, c->slot_gp, sizeof(int32_t) * (size_t)std::max<int64_t>(n_slots, 1)))) return r;
    if ((r = ensure(c, c->slot_off, sizeof(int64_t) * (size_t)(n_slots + 1)))) return r;
    if ((r = ensure(c, c->pairs_u, sizeof(int32_t) * (size_t)std::max<int64_t>(n_pairs, 1)))) return r;
    if ((r = ensure(c, c->pairs, sizeof(int32_t) * (size_t)std::max<int64_t>(n_pairs, 1)))) return r;
    if (with_cells && (r = ensure(c, c->cells, sizeof(float) * (size_t)(h.n_cells + kCellSlack)))) return r;
    w.slot_gp = as<int32_t>(c->slot_gp);
    w.slot_off = as<int64_t>(c->slot_off);
    w.pairs_unsorted = as<int32_t>(c->pairs_u);
    w.pairs = as<int32_t>(c->pairs);
    w.cells = with_cells ? as<float>(c->cells) : nullptr;
    launch_slots(c->P, w, nullptr, nullptr, st);
    launch_fill_pairs(c->P, w, st);
    launch_sort_pairs(w, n_slots, st);
    if (with_cells) launch_cells(c->P, w, st);
    HIP_TRY(c, hipGetLastError());
    return LTS_OK;
}

static lts_status stage_pairs(lts_context *c, uint64_t event_id, const lts_segments *segs, int32_t *pair_segment,
                              int32_t *pair_pixel, float *pair_current, int64_t cap_pairs, int64_t *n_pairs_out,
                              void *stream) {
    if (!c) return LTS_ERR_INVALID_ARG;
    if (!n_pairs_out || cap_pairs < 0) return fail(c, LTS_ERR_INVALID_ARG, "n_pairs_out is NULL or cap_pairs < 0");
    hipStream_t st = to_stream(stream);
    HIP_TRY(c, hipSetDevice(c->device));
    CallOrder order_(c, st);
    if (order_.status) return order_.status;
    Work w;
    DevHeader h;
    lts_status r;
    if ((r = stage_front(c, event_id, segs, pair_current != nullptr, st, w, h))) return r;
    *n_pairs_out = h.n_pairs;
    if (h.n_pairs > cap_pairs)
        return fail(c, LTS_ERR_CAPACITY, "cap_pairs " + std::to_string(cap_pairs) + " < " + std::to_string(h.n_pairs));
    if (pair_segment || pair_pixel) launch_pair_list(c->P, w, h.n_slots, pair_segment, pair_pixel, st);
    if (pair_current) {
        Table T{as<float>(c->Rpad), as<double>(c->prefix)};
        launch_induce_pairs(c->P, w, T, h.n_slots, pair_current, st);
    }
    HIP_TRY(c, hipGetLastError());
    return LTS_OK;
}

lts_status lts_stage_rasterize(lts_context *c, const lts_segments *segs, int32_t *pair_segment, int32_t *pair_pixel,
                               int64_t cap_pairs, int64_t *n_pairs_out, void *stream) {
    LTS_API_BEGIN
    if (c && (!pair_segment || !pair_pixel)) return fail(c, LTS_ERR_INVALID_ARG, "NULL pair output");
    return stage_pairs(c, 0, segs, pair_segment, pair_pixel, nullptr, cap_pairs, n_pairs_out, stream);
    LTS_API_END(c)
}

lts_status lts_stage_induce(lts_context *c, uint64_t event_id, const lts_segments *segs, int32_t *pair_segment,
                            int32_t *pair_pixel, float *pair_current, int64_t cap_pairs, int64_t *n_pairs_out,
                            void *stream) {
    LTS_API_BEGIN
    if (c && !pair_current) return fail(c, LTS_ERR_INVALID_ARG, "NULL pair_current");
    return stage_pairs(c, event_id, segs, pair_segment, pair_pixel, pair_current, cap_pairs, n_pairs_out, stream);
    LTS_API_END(c)
}

lts_status lts_stage_reduce(lts_context *c, const int32_t *pair_pixel, const float *pair_current, int64_t n_pairs,
                            int32_t *pixel_id, float *current, int64_t cap_pixels, int64_t *n_pixels_out,
                            void *stream) {
    LTS_API_BEGIN
    if (!c) return LTS_ERR_INVALID_ARG;
    if (!n_pixels_out || n_pairs < 0 || cap_pixels < 0 || (n_pairs > 0 && (!pair_pixel || !pair_current)) ||
        (cap_pixels > 0 && (!pixel_id || !current)))
        return fail(c, LTS_ERR_INVALID_ARG, "bad reduce stage arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = to_stream(stream);
    CallOrder order_(c, st);
    if (order_.status) return order_.status;
    *n_pixels_out = 0;
    if (n_pairs == 0) return LTS_OK;
    lts_status r;
    if ((r = ensure(c, c->red_head, sizeof(int64_t) * (size_t)(n_pairs + 1)))) return r;
    if ((r = ensure(c, c->red_start, sizeof(int64_t) * (size_t)(n_pairs + 1)))) return r;
    if ((r = ensure(c, c->hdr, sizeof(DevHeader)))) return r;
    if ((r = ensure(c, c->scan_tmp, sizeof(int64_t) * (size_t)scan_tmp_needed(n_pairs + 1)))) return r;
    int64_t *head = as<int64_t>(c->red_head), *start = as<int64_t>(c->red_start);
    HIP_TRY(c, hipMemsetAsync(c->hdr.p, 0, sizeof(DevHeader), st));
    launch_run_heads(pair_pixel, n_pairs, head, as<DevHeader>(c->hdr), st);
    scan_exclusive_i64(head, n_pairs + 1, nullptr, c->scan_tmp.p, st);
    launch_run_starts(pair_pixel, n_pairs, head, start, pixel_id, cap_pixels, st);
    HIP_TRY(c, hipGetLastError());
    int64_t n_runs = 0;
    HIP_TRY(c, hipMemcpyAsync(&n_runs, head + n_pairs, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipMemcpyAsync(c->hdr_host, c->hdr.p, sizeof(DevHeader), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    if (c->hdr_host->status & ST_INVALID)
        return fail(c, LTS_ERR_INVALID_ARG, "pairs are not grouped by ascending pixel id");
    *n_pixels_out = n_runs;
    if (n_runs > cap_pixels)
        return fail(c, LTS_ERR_CAPACITY, "cap_pixels " + std::to_string(cap_pixels) + " < " + std::to_string(n_runs));
    launch_reduce_runs(pair_current, start, n_runs, c->P.nticks, current, st);
    HIP_TRY(c, hipGetLastError());
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_work_stats(lts_context *c, double out[6]) {
    LTS_API_BEGIN
    if (!c || !out) return LTS_ERR_INVALID_ARG;
    if (c->last_n_seg < 0) return fail(c, LTS_ERR_STATE, "no pipeline call yet");
    HIP_TRY(c, hipSetDevice(c->device));
    lts_status r;
    if ((r = ensure(c, c->counts_tmp, 4 * sizeof(unsigned long long)))) return r;
    HIP_TRY(c, hipDeviceSynchronize());
    HIP_TRY(c, hipMemset(c->counts_tmp.p, 0, 4 * sizeof(unsigned long long)));
    if (c->last_mode == LTS_REDUCE_SUMMED) {
        launch_work_stats_summed(c->P, c->last_n_slots, as<int64_t>(c->list_off), as<PieceRef>(c->rec),
                                 as<float>(c->S), as<int64_t>(c->mlist_off), as<PieceRef>(c->mrec),
                                 summed_tile256(c->last_rt, c->last_shift), as<unsigned long long>(c->counts_tmp),
                                 nullptr);
        HIP_TRY(c, hipGetLastError());
        unsigned long long hs[4];
        HIP_TRY(c, hipMemcpy(hs, c->counts_tmp.p, sizeof(hs), hipMemcpyDeviceToHost));
        HIP_TRY(c, hipMemset(c->counts_tmp.p, 0, 4 * sizeof(unsigned long long)));
        launch_work_stats(c->P, as<SegInfo>(c->si), c->last_n_seg, as<unsigned long long>(c->counts_tmp), nullptr);
        HIP_TRY(c, hipGetLastError());
        unsigned long long hp[4];
        HIP_TRY(c, hipMemcpy(hp, c->counts_tmp.p, sizeof(hp), hipMemcpyDeviceToHost));
        out[0] = (double)hp[0];
        out[1] = (double)hs[1];
        out[2] = (double)hs[2];
        out[3] = (double)hp[3];
        out[4] = (double)hs[3];
        out[5] = (double)hs[0];
        return LTS_OK;
    }
    launch_work_stats(c->P, as<SegInfo>(c->si), c->last_n_seg, as<unsigned long long>(c->counts_tmp), nullptr);
    HIP_TRY(c, hipGetLastError());
    unsigned long long h[4];
    HIP_TRY(c, hipMemcpy(h, c->counts_tmp.p, sizeof(h), hipMemcpyDeviceToHost));
    for (int i = 0; i < 4; ++i) out[i] = (double)h[i];
    out[4] = 0.0;
    out[5] = (double)h[0];
    return LTS_OK;
    LTS_API_END(c)
}

lts_status lts_debug_fail_host_alloc(int64_t after) {
    if (after < -1) return LTS_ERR_INVALID_ARG;
    g_host_alloc_fail.store(after);
    return LTS_OK;
}

lts_status lts_stage_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out, int64_t n, void *stream) {
    LTS_API_BEGIN
    if (!ctr || !out || n < 0) return LTS_ERR_INVALID_ARG;
    launch_philox(ctr, k0, k1, out, n, to_stream(stream));
    return hipGetLastError() == hipSuccess ? LTS_OK : LTS_ERR_DEVICE;
    LTS_API_END(nullptr)
}

}  // extern "C"

// ================================================================================================= server
namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket = 0, event_id = 0;
    int64_t n = 0;
    std::vector<float> cols;        // 10 columns of n floats (dedx column filled with NaN when absent)
    double t_submit = 0.0;
};

struct Finished {
    lts_result_view v{};
    std::vector<int32_t> pixel_id, pkt_pixel, pkt_tick;
    std::vector<float> current;
    std::vector<uint16_t> pkt_adc;
    std::vector<uint8_t> pkt_flags;
};

struct PinnedBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

bool ensure_pinned(PinnedBuf &b, size_t bytes) {
    if (b.bytes >= bytes) return true;
    if (b.p) (void)hipHostFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    size_t want = std::max(bytes, b.bytes * 3 / 2);
    if (hipHostMalloc(&b.p, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    b.bytes = want;
    return true;
}

}  // namespace

struct lts_server;

struct Lane {
    lts_server *srv = nullptr;
    lts_context *ctx = nullptr;
    hipStream_t stream = nullptr;
    std::thread th;
    DevBuf seg, pix, cur, pkp, pkt, pka, pkf, counts, report, evpix, evpkt;
    int64_t cap_pixels = 0, cap_packets = 0;
    PinnedBuf stage, hcounts, hevpix, hevpkt, hreport;
};

struct lts_server {
    lts_server_cfg cfg{};
    int device = 0;
    int32_t n_ticks = 0;
    std::vector<std::unique_ptr<Lane>> lanes;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, Finished *> done;
    std::unordered_map<uint64_t, int> state;   // 0 queued, 1 running, 2 finished, 3 cancelled
    uint64_t next_ticket = 1;
    bool stopping = false;
    int64_t mem_reserve = int64_t(1) << 30;     // device memory left free by admission decisions
};

namespace {

void lane_run_batch(Lane *L, std::vector<Request *> &batch) {
    lts_server *S = L->srv;
    lts_context *c = L->ctx;
    const int32_t ne = (int32_t)batch.size();
    const double t_start = now_s();
    int64_t nseg = 0;
    for (Request *r : batch) nseg += r->n;
    std::vector<int64_t> offs(ne + 1, 0);
    std::vector<uint64_t> ids(ne);
    for (int32_t e = 0; e < ne; ++e) {
        offs[e + 1] = offs[e] + batch[e]->n;
        ids[e] = batch[e]->event_id;
    }
    host_alloc_point();
    lts_status st = LTS_OK;
    const size_t colb = sizeof(float) * (size_t)std::max<int64_t>(nseg, 1);
    if (!ensure_pinned(L->stage, 10 * colb)) st = LTS_ERR_OOM;
    if (st == LTS_OK) st = ensure(c, L->seg, 10 * colb);
    if (st == LTS_OK) {
        float *h = (float *)L->stage.p;
        for (int k = 0; k < 10; ++k)
            for (int32_t e = 0; e < ne; ++e)
                if (batch[e]->n)
                    std::memcpy(h + (size_t)k * nseg + offs[e], batch[e]->cols.data() + (size_t)k * batch[e]->n,
                                sizeof(float) * (size_t)batch[e]->n);
        if (hipMemcpyAsync(L->seg.p, L->stage.p, 10 * colb, hipMemcpyHostToDevice, L->stream) != hipSuccess)
            st = LTS_ERR_DEVICE;
    }
    float *d = (float *)L->seg.p;
    // memory-based admission: size the tentative batch (the first k events) on the device; run it if the lane's
    // footprint after growing to the exact sizes fits its share of the budget and the device's free memory, else
    // halve it; a single event that does not fit fails alone with LTS_ERR_OOM
    const int64_t mp = c->P.max_packets;
    const int64_t share = S->cfg.mem_budget_bytes / S->cfg.n_lanes;
    DevBuf *outs[] = {&L->pix, &L->cur, &L->pkp, &L->pkt, &L->pka, &L->pkf, &L->counts, &L->report, &L->evpix,
                      &L->evpkt};
    lts_outputs o{};
    auto set_outputs = [&](int64_t cap_px) {
        o = lts_outputs{(int32_t *)L->pix.p, (float *)L->cur.p, cap_px, (int32_t *)L->pkp.p, (int32_t *)L->pkt.p,
                        (uint16_t *)L->pka.p, (uint8_t *)L->pkf.p, cap_px * mp, (int64_t *)L->counts.p,
                        (double *)L->report.p, (int64_t *)L->evpix.p, (int64_t *)L->evpkt.p};
    };
    // the sizing pass already writes the per-event report: counts, report and event offsets are sized for the
    // whole tentative batch up front, the large outputs (non-null placeholders until then) by the admission hook
    const size_t small[] = {16, 16, 16, 16, 16, 16, sizeof(int64_t) * 4, sizeof(double) * 5 * (size_t)ne,
                            sizeof(int64_t) * (size_t)(ne + 1), sizeof(int64_t) * (size_t)(ne + 1)};
    for (int i = 0; i < 10 && st == LTS_OK; ++i) st = ensure(c, *outs[i], small[i]);
    set_outputs(0);
    int32_t ran = 0;
    if (st == LTS_OK) {
        ran = admission_loop(
            ne,
            [&](int32_t k) -> Admit {
                lts_segments segs{d, d + nseg, d + 2 * nseg, d + 3 * nseg, d + 4 * nseg, d + 5 * nseg, d + 6 * nseg,
                                  d + 7 * nseg, d + 8 * nseg, d + 9 * nseg, offs[k]};
                Admit decision = Admit::Run;
                c->admit = [&](const DevHeader &h, int64_t total, int64_t growth) -> lts_status {
                    const int64_t px = std::max<int64_t>(h.n_slots, 1), pk = std::max<int64_t>(h.n_slots * mp, 1);
                    const size_t want[] = {sizeof(int32_t) * (size_t)px, sizeof(float) * (size_t)px * S->n_ticks,
                                           sizeof(int32_t) * (size_t)pk, sizeof(int32_t) * (size_t)pk,
                                           sizeof(uint16_t) * (size_t)pk, sizeof(uint8_t) * (size_t)pk,
                                           sizeof(int64_t) * 4, sizeof(double) * 5 * (size_t)k,
                                           sizeof(int64_t) * (size_t)(k + 1), sizeof(int64_t) * (size_t)(k + 1)};
                    int64_t out_total = (int64_t)L->seg.bytes, out_growth = 0;
                    for (int i = 0; i < 10; ++i) {
                        out_total += (int64_t)std::max(outs[i]->bytes, want[i]);
                        if (want[i] > outs[i]->bytes) out_growth += (int64_t)(want[i] - outs[i]->bytes);
                    }
                    size_t free_b = 0, total_b = 0;
                    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
                        (void)hipGetLastError();
                        free_b = 0;
                    }
                    decision = admit_decision(k, total + out_total, growth + out_growth, share, (int64_t)free_b,
                                              S->mem_reserve);
                    if (decision != Admit::Run) return kNotAdmitted;
                    lts_status r2 = LTS_OK;
                    for (int i = 0; i < 10 && r2 == LTS_OK; ++i) r2 = ensure(c, *outs[i], want[i]);
                    if (r2) return r2;
                    set_outputs(h.n_slots);
                    return LTS_OK;
                };
                struct Unhook {                                   // the hook captures this frame: never outlive it
                    lts_context *c;
                    ~Unhook() { c->admit = nullptr; }
                } unhook{c};
                st = run_pipeline(c, k, ids.data(), offs.data(), &segs, &o, L->stream);
                if (st == kNotAdmitted) {
                    st = LTS_OK;
                    return decision;
                }
                return Admit::Run;                                // ran (or failed with its own status)
            },
            [&]() -> bool {                                       // the lane's pooled scratch, before refusing
                if (hipStreamSynchronize(L->stream) != hipSuccess) {
                    (void)hipGetLastError();
                    st = LTS_ERR_DEVICE;
                    return false;
                }
                release_scratch(c);
                for (int i = 0; i < 10; ++i) free_buf(*outs[i]);
                for (int i = 0; i < 10 && st == LTS_OK; ++i) st = ensure(c, *outs[i], small[i]);
                set_outputs(0);
                return st == LTS_OK;
            });
    }
    // events the batch no longer holds go back to the front of the queue, in order; a rejected head event (it alone
    // exceeds the lane's share) finishes with LTS_ERR_OOM
    const bool rejected = st == LTS_OK && ran == 0;
    const size_t keep = st != LTS_OK ? (size_t)ne : rejected ? 1 : (size_t)ran;
    if (keep < (size_t)ne) {
        std::lock_guard<std::mutex> lk(S->mu);
        for (size_t e = keep; e < (size_t)ne; ++e) S->state[batch[e]->ticket] = 0;
        requeue_tail(S->queue, batch, keep);
        S->cv_work.notify_all();
    }
    if (rejected) st = LTS_ERR_OOM;
    const int32_t nr = (int32_t)batch.size();
    // results back to host
    std::vector<std::unique_ptr<Finished>> fin(nr);
    int64_t cnt[4] = {0, 0, 0, 0};
    std::vector<int64_t> evpix(nr + 1, 0), evpkt(nr + 1, 0);
    std::vector<double> rep(5 * (size_t)nr, 0.0);
    std::vector<int64_t> evc(2 * (size_t)nr, 0);
    if (st == LTS_OK) {
        if (hipMemcpyAsync(cnt, L->counts.p, sizeof(cnt), hipMemcpyDeviceToHost, L->stream) != hipSuccess ||
            hipMemcpyAsync(evc.data(), c->ev_cnt.p, sizeof(int64_t) * 2 * nr, hipMemcpyDeviceToHost, L->stream) != hipSuccess ||
            hipMemcpyAsync(evpix.data(), L->evpix.p, sizeof(int64_t) * (nr + 1), hipMemcpyDeviceToHost, L->stream) != hipSuccess ||
            hipMemcpyAsync(evpkt.data(), L->evpkt.p, sizeof(int64_t) * (nr + 1), hipMemcpyDeviceToHost, L->stream) != hipSuccess ||
            hipMemcpyAsync(rep.data(), L->report.p, sizeof(double) * 5 * nr, hipMemcpyDeviceToHost, L->stream) != hipSuccess ||
            hipStreamSynchronize(L->stream) != hipSuccess)
            st = LTS_ERR_DEVICE;
    }
    // the whole batch's pixels and packets in one copy per array, then cut per event on the host
    const int64_t np_all = st == LTS_OK ? evpix[nr] : 0, nk_all = st == LTS_OK ? evpkt[nr] : 0;
    std::vector<int32_t> h_pix(np_all), h_pkp(nk_all), h_pkt(nk_all);
    std::vector<uint16_t> h_pka(nk_all);
    std::vector<uint8_t> h_pkf(nk_all);
    std::vector<float> h_cur(S->cfg.return_currents ? (size_t)np_all * S->n_ticks : 0);
    if (st == LTS_OK) {
        bool ok = true;
        auto get = [&](void *dst, const void *src, size_t bytes) {
            if (ok && bytes) ok = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, L->stream) == hipSuccess;
        };
        get(h_pix.data(), L->pix.p, sizeof(int32_t) * (size_t)np_all);
        get(h_pkp.data(), L->pkp.p, sizeof(int32_t) * (size_t)nk_all);
        get(h_pkt.data(), L->pkt.p, sizeof(int32_t) * (size_t)nk_all);
        get(h_pka.data(), L->pka.p, sizeof(uint16_t) * (size_t)nk_all);
        get(h_pkf.data(), L->pkf.p, sizeof(uint8_t) * (size_t)nk_all);
        get(h_cur.data(), L->cur.p, sizeof(float) * h_cur.size());
        if (!ok || hipStreamSynchronize(L->stream) != hipSuccess) st = LTS_ERR_DEVICE;
    }
    for (int32_t e = 0; e < nr; ++e) {
        fin[e].reset(new Finished());
        Finished *f = fin[e].get();
        f->v.event_id = batch[e]->event_id;
        f->v.t_submit = batch[e]->t_submit;
        f->v.t_start = t_start;
        f->v.batch_events = nr;
        if (st == LTS_OK) {
            const int64_t p0 = evpix[e], p1 = evpix[e + 1], k0 = evpkt[e], k1 = evpkt[e + 1];
            f->pixel_id.resize(p1 - p0);
            f->pkt_pixel.resize(k1 - k0);
            f->pkt_tick.resize(k1 - k0);
            f->pkt_adc.resize(k1 - k0);
            f->pkt_flags.resize(k1 - k0);
            std::copy(h_pix.begin() + p0, h_pix.begin() + p1, f->pixel_id.begin());
            std::copy(h_pkp.begin() + k0, h_pkp.begin() + k1, f->pkt_pixel.begin());
            std::copy(h_pkt.begin() + k0, h_pkt.begin() + k1, f->pkt_tick.begin());
            std::copy(h_pka.begin() + k0, h_pka.begin() + k1, f->pkt_adc.begin());
            std::copy(h_pkf.begin() + k0, h_pkf.begin() + k1, f->pkt_flags.begin());
            if (S->cfg.return_currents)
                f->current.assign(h_cur.begin() + (size_t)p0 * S->n_ticks, h_cur.begin() + (size_t)p1 * S->n_ticks);
            f->v.n_pixels = p1 - p0;
            f->v.n_packets = k1 - k0;
            for (int k = 0; k < 5; ++k) f->v.report[k] = rep[5 * (size_t)e + k];
            f->v.counts[0] = p1 - p0;
            f->v.counts[1] = k1 - k0;
            f->v.counts[2] = evc[2 * (size_t)e];         // this event's own dropped samples and overflow packets
            f->v.counts[3] = evc[2 * (size_t)e + 1];
        }
        f->v.status = st;
        f->v.pixel_id = f->pixel_id.data();
        f->v.current = S->cfg.return_currents ? f->current.data() : nullptr;
        f->v.pkt_pixel = f->pkt_pixel.data();
        f->v.pkt_tick = f->pkt_tick.data();
        f->v.pkt_adc = f->pkt_adc.data();
        f->v.pkt_flags = f->pkt_flags.data();
    }
    const double t_done = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    for (int32_t e = 0; e < nr; ++e) {
        fin[e]->v.t_done = t_done;
        const uint64_t t = batch[e]->ticket;
        auto it = S->state.find(t);
        bool kept = false;
        if (it != S->state.end()) {
            try {
                S->done[t] = fin[e].get();
                it->second = 2;
                kept = true;
            } catch (...) {
                it->second = 3;                          // no room for the result: the ticket reads as cancelled
            }
        }
        if (kept) (void)fin[e].release();
        delete batch[e];
    }
    batch.clear();
    S->cv_done.notify_all();
}

// A batch whose host-side work threw before its results were published: every ticket of it finishes with `st`
// (or reads as cancelled if even that cannot be recorded).  Never throws.
void lane_fail_batch(Lane *L, std::vector<Request *> &batch, lts_status st) noexcept {
    lts_server *S = L->srv;
    const double t = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    for (Request *r : batch) {
        auto it = S->state.find(r->ticket);
        if (it != S->state.end()) {
            Finished *f = new (std::nothrow) Finished();
            bool kept = false;
            if (f) {
                f->v.event_id = r->event_id;
                f->v.status = st;
                f->v.t_submit = r->t_submit;
                f->v.t_start = f->v.t_done = t;
                f->v.batch_events = (int32_t)batch.size();
                try {
                    S->done[r->ticket] = f;
                    it->second = 2;
                    kept = true;
                } catch (...) {
                }
            }
            if (!kept) {
                delete f;
                it->second = 3;
            }
        }
        delete r;
    }
    batch.clear();
    S->cv_done.notify_all();
}

void lane_loop(Lane *L) {
    lts_server *S = L->srv;
    (void)hipSetDevice(S->device);
    for (;;) {
        std::vector<Request *> batch;
        try {
            batch.reserve((size_t)S->cfg.max_batch_events);
        } catch (...) {
            std::this_thread::sleep_for(std::chrono::milliseconds(10));   // host memory is short: try again
            continue;
        }
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stopping || !S->queue.empty(); });
            if (S->stopping) return;
            int64_t segs = 0;
            while (!S->queue.empty() && (int32_t)batch.size() < S->cfg.max_batch_events) {
                Request *r = S->queue.front();
                if (!batch.empty() && segs + r->n > S->cfg.max_batch_segments) break;
                S->queue.pop_front();
                S->state[r->ticket] = 1;
                batch.push_back(r);
                segs += r->n;
            }
        }
        try {
            lane_run_batch(L, batch);
        } catch (const std::bad_alloc &) {
            lane_fail_batch(L, batch, LTS_ERR_OOM);
        } catch (...) {
            lane_fail_batch(L, batch, LTS_ERR_DEVICE);
        }
    }
}

}  // namespace

extern "C" {

lts_status lts_server_start(lts_context *ctx, const lts_server_cfg *cfg, lts_server **out) {
    LTS_API_BEGIN
    if (!ctx || !out) return LTS_ERR_INVALID_ARG;
    *out = nullptr;
    if (!ctx->has_table) return fail(ctx, LTS_ERR_STATE, "no response table: call lts_set_response first");
    size_t free_b = 0, total_b = 0;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipMemGetInfo(&free_b, &total_b));
    lts_server *S = new (std::nothrow) lts_server();
    if (!S) return LTS_ERR_OOM;
    if (cfg) S->cfg = *cfg;
    if (S->cfg.n_lanes <= 0) S->cfg.n_lanes = 2;
    if (S->cfg.max_batch_events <= 0) S->cfg.max_batch_events = 64;
    if (S->cfg.max_batch_segments <= 0) S->cfg.max_batch_segments = 4000000;
    if (S->cfg.mem_budget_bytes <= 0) S->cfg.mem_budget_bytes = (int64_t)(total_b / 2);   // half of the device
    S->device = ctx->device;
    S->n_ticks = ctx->ro.n_ticks;
    auto undo = [&] {                                  // destroys the lanes made so far (no thread started yet)
        for (auto &l : S->lanes) {
            if (l->ctx) lts_context_destroy(l->ctx);
            if (l->stream) (void)hipStreamDestroy(l->stream);
        }
        delete S;
    };
    try {
        S->lanes.reserve((size_t)S->cfg.n_lanes);
        for (int i = 0; i < S->cfg.n_lanes; ++i) {
            S->lanes.emplace_back(new Lane());
            Lane *L = S->lanes.back().get();
            L->srv = S;
            lts_status r = lts_context_create(ctx->device, &ctx->ph, &ctx->ro, &ctx->el, &L->ctx);
            if (r == LTS_OK) r = lts_set_response(L->ctx, ctx->table_host.data(), ctx->t_r, ctx->b_x, ctx->b_y);
            if (r == LTS_OK) r = lts_set_reduce_mode(L->ctx, ctx->reduce_mode);
            if (r == LTS_OK) r = lts_set_induce_slices(L->ctx, ctx->induce_slices);
            if (r == LTS_OK) r = lts_set_ticks_per_thread(L->ctx, ctx->ticks_per_thread);
            if (r == LTS_OK) r = lts_set_lane_exchange(L->ctx, ctx->lane_exchange);
            if (r == LTS_OK) r = lts_set_matrix_cores(L->ctx, ctx->matrix_cores);
            if (r == LTS_OK)
                r = lts_set_tuning(L->ctx, ctx->tuning.empty() ? nullptr : ctx->tuning.data(), (int32_t)ctx->tuning.size());
            if (r == LTS_OK && hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) != hipSuccess) {
                L->stream = nullptr;
                r = LTS_ERR_DEVICE;
            }
            if (r != LTS_OK) {
                undo();
                return fail(ctx, r, "server lane creation failed");
            }
        }
    } catch (...) {
        undo();
        throw;
    }
    try {
        for (auto &L : S->lanes) L->th = std::thread(lane_loop, L.get());
    } catch (...) {                                     // a lane thread could not start: undo the started ones
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stopping = true;
            S->cv_work.notify_all();
        }
        for (auto &L : S->lanes) {
            if (L->th.joinable()) L->th.join();
            lts_context_destroy(L->ctx);
            (void)hipStreamDestroy(L->stream);
        }
        delete S;
        return fail(ctx, LTS_ERR_DEVICE, "server lane thread could not be started");
    }
    *out = S;
    return LTS_OK;
    LTS_API_END(ctx)
}

lts_status lts_server_submit(lts_server *S, uint64_t event_id, const lts_segments *h, uint64_t *ticket) {
    LTS_API_BEGIN
    if (!S || !h || !ticket || h->n < 0) return LTS_ERR_INVALID_ARG;
    if (h->n > 0 && !(h->x0 && h->y0 && h->z0 && h->t0 && h->x1 && h->y1 && h->z1 && h->t1 && h->energy))
        return LTS_ERR_INVALID_ARG;
    host_alloc_point();
    std::unique_ptr<Request> held(new Request());     // freed if anything below throws
    Request *r = held.get();
    r->event_id = event_id;
    r->n = h->n;
    r->t_submit = now_s();
    r->cols.resize(10 * (size_t)h->n);
    const float *src[10] = {h->x0, h->y0, h->z0, h->t0, h->x1, h->y1, h->z1, h->t1, h->energy, h->dedx};
    for (int k = 0; k < 10; ++k) {
        float *dst = r->cols.data() + (size_t)k * h->n;
        if (src[k]) std::memcpy(dst, src[k], sizeof(float) * (size_t)h->n);
        else std::fill(dst, dst + h->n, NAN);
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) return LTS_ERR_STATE;
    r->ticket = S->next_ticket++;
    S->state[r->ticket] = 0;
    try {
        S->queue.push_back(r);
    } catch (...) {
        S->state.erase(r->ticket);
        throw;
    }
    held.release();
    *ticket = r->ticket;
    S->cv_work.notify_one();
    return LTS_OK;
    LTS_API_END(nullptr)
}

static lts_status server_view(lts_server *S, uint64_t t, lts_result_view *out) {
    auto it = S->state.find(t);
    if (it == S->state.end()) return LTS_ERR_INVALID_ARG;
    if (it->second == 3) return LTS_ERR_CANCELLED;
    if (it->second != 2) return LTS_ERR_NOT_READY;
    Finished *f = S->done[t];
    if (out) *out = f->v;
    return (lts_status)f->v.status;
}

lts_status lts_server_poll(lts_server *S, uint64_t t, lts_result_view *out) {
    LTS_API_BEGIN
    if (!S) return LTS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    return server_view(S, t, out);
    LTS_API_END(nullptr)
}

lts_status lts_server_wait(lts_server *S, uint64_t t, lts_result_view *out, double timeout_s) {
    LTS_API_BEGIN
    if (!S) return LTS_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto ready = [&] {
        auto it = S->state.find(t);
        return it == S->state.end() || it->second >= 2;
    };
    if (timeout_s < 0) S->cv_done.wait(lk, ready);
    else S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    return server_view(S, t, out);
    LTS_API_END(nullptr)
}

lts_status lts_server_release(lts_server *S, uint64_t t) {
    LTS_API_BEGIN
    if (!S) return LTS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->state.find(t);
    if (it == S->state.end()) return LTS_ERR_INVALID_ARG;
    if (it->second < 2) return LTS_ERR_NOT_READY;
    auto d = S->done.find(t);
    if (d != S->done.end()) {
        delete d->second;
        S->done.erase(d);
    }
    S->state.erase(it);
    return LTS_OK;
    LTS_API_END(nullptr)
}

lts_status lts_server_stop(lts_server *S) {
    LTS_API_BEGIN
    if (!S) return LTS_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
        for (Request *r : S->queue) {
            S->state[r->ticket] = 3;
            delete r;
        }
        S->queue.clear();
        S->cv_work.notify_all();
        S->cv_done.notify_all();
    }
    for (auto &L : S->lanes)
        if (L->th.joinable()) L->th.join();
    for (auto &L : S->lanes) {
        (void)hipSetDevice(S->device);
        (void)hipStreamSynchronize(L->stream);
        DevBuf *bufs[] = {&L->seg, &L->pix, &L->cur, &L->pkp, &L->pkt, &L->pka, &L->pkf, &L->counts, &L->report,
                          &L->evpix, &L->evpkt};
        for (DevBuf *b : bufs) free_buf(*b);
        PinnedBuf *pins[] = {&L->stage, &L->hcounts, &L->hevpix, &L->hevpkt, &L->hreport};
        for (PinnedBuf *p : pins)
            if (p->p) (void)hipHostFree(p->p);
        (void)hipStreamDestroy(L->stream);
        lts_context_destroy(L->ctx);
    }
    for (auto &kv : S->done) delete kv.second;
    delete S;
    return LTS_OK;
    LTS_API_END(nullptr)
}

}  // extern "C"
