/*
 * ltsim.h -- C ABI of the MI355X (gfx950) pixelated-LArTPC charge-simulation library (libltsim.so).
 *
 * The calls follow the statement of the problem in arXiv 2212.09807: a table of energy-deposit segments
 * S_i = (r_s, r_e, E), r 4-dimensional (x, y, z, t) (Sec. 2), together with detector and response parameters
 * (Sec. 3.1 recombination, Sec. 3.2 drift, Sec. 3.3.1 pixel field-response table, Sec. 3.4 front end), goes
 * in; per-pixel induced currents (Sec. 3.3.2, eq. (current), summed over segments as in Sec. 3.4) and the
 * digitised ADC counts with their timestamps per pixel (Sec. 3.4, last paragraph) come out.
 *
 * Conventions
 *   - Units: cm, microseconds, MeV, electrons, kV/cm.  The anode plane is z = z_anode; charge drifts along -z.
 *   - Pixel ids are tile-local: id = iy * n_x + ix, pixel (ix, iy) covering [x0 + ix*pitch, x0 + (ix+1)*pitch)
 *     x [y0 + iy*pitch, ...).  Tick n covers [t_begin + n*tick, t_begin + (n+1)*tick).
 *   - Currents are electrons per tick, FP32.  Charge reports are FP64.
 *   - All pointers inside lts_segments / lts_outputs are DEVICE pointers (HIP global memory on the
 *     context's device) unless a field says otherwise.  The caller owns them; the library never frees them.
 *   - Stream arguments are hipStream_t values passed as void* (NULL = the null stream).  Entry points that
 *     take a stream enqueue their work on it and return; results are valid after the stream is synchronised.
 *     lts_simulate / lts_simulate_batch additionally synchronise that stream once (after sizing) to size
 *     scratch and check output capacities, so a capacity error is returned synchronously (LTS_REDUCE_SUMMED
 *     synchronises three times more, to size the summed columns, the pixels' piece lists and the merged records;
 *     it also runs the charge cells on a stream of the context's own, forked from the call's stream and joined back
 *     to it before anything the call leaves behind, so the call's stream still orders all of its work).  Calls on
 *     one context that use its scratch pool (lts_plan, lts_simulate, lts_simulate_batch, lts_stage_rasterize, lts_stage_induce,
 *     lts_stage_reduce, lts_stage_electronics) are ordered on the device whatever streams they are given: each one
 *     first makes its stream wait for the previous one's completion (a HIP event), so work of consecutive calls on
 *     different streams never overlaps in the shared scratch.
 *   - No call throws across the ABI.  Every call returns an lts_status; on failure lts_last_error() gives a
 *     message.  A failed device call makes the context's status sticky (LTS_ERR_DEVICE).  A failed host-memory
 *     allocation inside a call returns LTS_ERR_OOM and leaves the context usable; any other internal C++
 *     exception returns LTS_ERR_DEVICE without making it sticky.
 *   - A context is not thread-safe: serialise calls on one context.  The server API is thread-safe.
 */
#ifndef LTSIM_H
#define LTSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lts_status {
    LTS_OK = 0,
    LTS_ERR_INVALID_ARG = 1,   /* bad parameter, table shape, NaN/Inf, zero-length segment without dE/dx ... */
    LTS_ERR_CAPACITY = 2,      /* an output buffer is too small; required sizes are written to counts[] */
    LTS_ERR_OOM = 3,           /* device allocation failed */
    LTS_ERR_DEVICE = 4,        /* a HIP call failed (sticky for the context) */
    LTS_ERR_NOT_READY = 5,     /* server: the ticket has not finished */
    LTS_ERR_CANCELLED = 6,     /* server: the ticket was dropped (server stopped or request failed) */
    LTS_ERR_STATE = 7          /* call not valid in the current state (e.g. no response table set) */
} lts_status;

/* Charge-transport constants (Sec. 3.1, Sec. 3.2, Sec. 3.3.2). */
typedef struct lts_physics {
    int32_t recomb_model;      /* 0 = Birks, eq. (birks) (default); 1 = modified Box, eq. (box) */
    double e_field;            /* kV/cm */
    double lar_density;        /* g/cm^3; epsilon = e_field * lar_density */
    double w_ion;              /* MeV per ionisation electron: Q_0 = E / w_ion */
    double birks_ab, birks_kb; /* A_b, k_b */
    double box_alpha, box_beta;/* alpha, beta */
    double v_drift;            /* cm/us, eq. (drift) */
    double lifetime;           /* us, eq. (lifetime) */
    double d_long, d_tran;     /* cm^2/us, sigma = sqrt(2 D t_drift) */
    double z_anode;            /* cm */
    double sample_step;        /* cm; N = max(1, ceil(L / sample_step)) points per segment, eq. (rho) */
    double n_sigma;            /* diffusion truncation in sigmas (>= 1) */
    int32_t mc_draws;          /* diffusion estimator of eq. (rho): 0 = expectation over the Gaussian perturbations
                                  (deterministic); M in [1, 65535] = the paper's Monte Carlo form, M perturbations per
                                  sample point drawn from Philox4x32-10 (key = electronics seed, counter = (segment
                                  index within the event, point * M + draw, event id low word, (event id high word << 4)
                                  | 3 + try)), each normal truncated to n_sigma by re-drawing; every moved copy puts
                                  Q_a / (N M) into the cell that holds it */
    int32_t per_point;         /* 0 = lifetime (eq. (lifetime)) and diffusion widths at the segment midpoint (default);
                                  1 = at every sample point's own drift time: charge Q_R / N * exp(-t_mu / tau), widths
                                  sqrt(2 D t_mu); then Q_a is the sum of the points' charges.  Not with mc_draws > 0 */
} lts_physics;

/* Pixel plane and time sampling. */
typedef struct lts_readout {
    double pitch;              /* cm */
    int32_t n_x, n_y;          /* pixels */
    double x0, y0;             /* cm, lower edge of pixel (0, 0) */
    int32_t n_sub;             /* sub-pixel bins per pitch (even) = field-table granularity */
    double tick;               /* us */
    int32_t n_ticks;           /* readout window length (<= 8000) */
    double t_begin;            /* us, lower edge of tick 0 */
} lts_readout;

/* LArPix-like front end (Sec. 3.4). */
typedef struct lts_electronics {
    double threshold;          /* electrons; a sample is triggered when integral + discriminator noise >= threshold */
    int32_t hold_ticks;        /* ticks from the threshold crossing to digitisation (1.6 us = 16); >= 0, values
                                  above 2^20 act as 2^20 (every later sample falls past the last tick) */
    int32_t min_spacing;       /* minimum ticks between consecutive samples (11); >= 0, above 2^20 acts as 2^20 */
    double q_lsb;              /* electrons per ADC count */
    int32_t pedestal;          /* ADC counts added before clamping */
    int32_t adc_bits;          /* ADC resolution (<= 16) */
    double sigma_reset;        /* electrons: pedestal drawn at start and after each reset */
    double sigma_disc;         /* electrons: per-tick noise on the discriminator comparison */
    double sigma_unc;          /* electrons: per-sample uncorrelated noise */
    int32_t max_packets;       /* per pixel (further samples are counted as overflow) */
    uint64_t seed;             /* Philox4x32-10 key (low word, high word) */
    int32_t reset_period;      /* periodic reset every reset_period ticks (0 = off): at ticks k * reset_period, k >= 1,
                                  before that tick's charge, a pixel with no pending sample restarts from reset noise */
} lts_electronics;

/* Segment table, structure of arrays, FP32, device pointers; n rows.  dedx may be NULL; it is read only
 * for zero-length segments (and must then be finite). */
typedef struct lts_segments {
    const float *x0, *y0, *z0, *t0;   /* start point r_s (cm, cm, cm, us) */
    const float *x1, *y1, *z1, *t1;   /* end point r_e */
    const float *energy;              /* deposited energy E, MeV */
    const float *dedx;                /* MeV/cm, optional */
    int64_t n;
} lts_segments;

/* Outputs (caller-owned device buffers).
 *   pixel_id[cap_pixels]           ascending tile-local ids of the active pixels (those whose table reach meets
 *                                  some segment's charge cloud; their waveform may be all zero)
 *   current[cap_pixels * n_ticks]  row-major [pixel slot][tick], electrons per tick
 *   pkt_*[cap_packets]             packets ordered by (pixel slot, tick): pixel id, tick index of the
 *                                  digitisation, ADC code, flags (bit0: ADC value within the FP32 error margin of
 *                                  an LSB boundary; bit1: an earlier threshold decision of this pixel lay within
 *                                  the FP32 error margin; bit2: ADC clamped)
 *   counts[4]                      written: active pixels, packets, samples dropped past the window, packets over
 *                                  max_packets.  On LTS_ERR_CAPACITY they hold the required sizes instead.
 *   report[5 per event]            FP64: sum Q_R (after recombination), sum Q_a (after lifetime), sum of current
 *                                  over pixels and ticks in the window, signed induction that fell outside the
 *                                  tick window, charge whose cells lie outside the pixel grid.
 *   event_pixel_offsets, event_packet_offsets  [n_events + 1] (batch only; may be NULL for one event):
 *                                  slot / packet ranges of each event in the arrays above.
 */
typedef struct lts_outputs {
    int32_t *pixel_id;
    float *current;
    int64_t cap_pixels;
    int32_t *pkt_pixel;
    int32_t *pkt_tick;
    uint16_t *pkt_adc;
    uint8_t *pkt_flags;
    int64_t cap_packets;
    int64_t *counts;
    double *report;
    int64_t *event_pixel_offsets;
    int64_t *event_packet_offsets;
} lts_outputs;

typedef struct lts_context lts_context;

/* Reduction variant for the per-pixel sum over segments (Sec. 3.4):
 *   LTS_REDUCE_SORTED: pairs sorted pixel-major, one workgroup per pixel, Kahan-compensated FP32 accumulation in a
 *                      fixed segment order (deterministic, batch-invariant; default);
 *   LTS_REDUCE_ATOMIC: segment-major, per-pair currents added with FP32 atomics (order-dependent rounding);
 *   LTS_REDUCE_SUMMED: sum-then-convolve: eq. (current) is linear in the charge, so each sub-pixel column's charge
 *                      is first summed over all segments (fixed order, Kahan) and each pixel then convolves the summed
 *                      columns in its reach once; the same result without per-pair currents, with fewer
 *                      multiply-adds where clouds of neighbouring segments overlap (deterministic).  Per pixel, the
 *                      column pieces seen through the same mirror-folded table column that overlap in time (up to
 *                      248 ticks together) are summed first and convolved once. */
enum { LTS_REDUCE_SORTED = 0, LTS_REDUCE_ATOMIC = 1, LTS_REDUCE_SUMMED = 2 };

/* Create a context on HIP device `device` with copies of the parameter sets.  Validates them
 * (LTS_ERR_INVALID_ARG: non-positive v_drift / lifetime / pitch / tick / sample_step, negative diffusion,
 * odd n_sub, n_sigma < 1, n_ticks outside [1, 8000], adc_bits outside [1, 16], ...). */
lts_status lts_context_create(int device, const lts_physics *physics, const lts_readout *readout,
                              const lts_electronics *electronics, lts_context **out);
void lts_context_destroy(lts_context *ctx);

/* Install the pixel field-response table (Sec. 3.3.1): host array R[t_r][b_x][b_y] (FP32, C order), entry
 * [k][i][j] = electrons induced in tick k on a pad by one electron whose lateral offset from the pad centre is
 * the centre of sub-pixel bin (i, j) of the quadrant (bin width pitch / n_sub); entry t_r-1 is the tick of
 * arrival.  The table is copied to device memory (the caller keeps ownership of R_host).  Requires
 * 1 <= t_r <= 8192 and 1 <= b_x, b_y <= 256. */
lts_status lts_set_response(lts_context *ctx, const float *R_host, int32_t t_r, int32_t b_x, int32_t b_y);

lts_status lts_set_reduce_mode(lts_context *ctx, int32_t mode);

/* Disabled channels (Sec. 6: part of the pixels of a tile can be switched off): host mask of n_x * n_y bytes
 * indexed by tile-local pixel id, non-zero = disabled.  Disabled pixels keep their currents but produce no packets.
 * mask = NULL (or n = 0) enables every pixel.  Copied; applies to every later event on the context. */
lts_status lts_set_channel_mask(lts_context *ctx, const uint8_t *mask, int64_t n);

/* Sorted variant only: split each pixel's induction over `slices` workgroups by the mirror-folded x-bin index of
 * the table (e.g. 8, one slice per XCD, so each XCD's L2 holds only its part of the table); the slices'
 * waveforms are added in a fixed order.  1 (default) = one workgroup per pixel. */
lts_status lts_set_induce_slices(lts_context *ctx, int32_t slices);

/* Induction tick tile: each of the 256 threads of a workgroup computes `rt` consecutive ticks of a pair's window
 * (1, 2, 4 or 8; 0 = the smallest that covers the table length plus a typical charge extent, and for 8 ticks the
 * loop that loads the next cell-tick block's window while computing the current one; an explicit 8 selects the
 * loop without that prefetch).  All choices give the same sums in the same order.  In LTS_REDUCE_SUMMED: 0 = one
 * wavefront per (pixel, 256-tick tile) with the table window staged in LDS (default), 8 = one wavefront per
 * (pixel, 512-tick tile) with register-resident table windows, 1, 2, 4 = the per-pair workgroup kernel over the
 * summed pieces; these agree to FP32 summation order. */
lts_status lts_set_ticks_per_thread(lts_context *ctx, int32_t rt);

/* Per-pair induction with 8-tick tiles: 1 = lanes share each table window by shifting it one lane per cell-tick
 * block (one coalesced load per column and lane); 0 (default, faster on gfx950) = every lane loads its own 15-value
 * window per block.
 * Both give the same sums in the same order.  A tuning option (Sec. 3.3.2 sets no kernel design). */
lts_status lts_set_lane_exchange(lts_context *ctx, int32_t on);

/* Sorted per-pair induction (Sec. 3.3.2, eq. (current)) on the FP32 matrix cores: 1 = per pair, the product of
 * its cell-tick x column charges with its columns' table rows on 32x32x2 MFMA instructions, then sums along the
 * product's anti-diagonals (one per output tick); 0 (default, faster on gfx950) = the vector-ALU loop.  Same pair
 * order and Kahan accumulation; the products are summed in a different order, so results agree to FP32 rounding,
 * not bit for bit.  Used only when the reduce mode is LTS_REDUCE_SORTED and induce slices are 1; ignored
 * otherwise. */
lts_status lts_set_matrix_cores(lts_context *ctx, int32_t on);

/* HIP-graph replay of each call's launch sequence (Sec. 3.4 pipeline; a launch-overhead option for batched and
 * small events): 1 = after the sizing read-back that every call makes, the rest of the call (rasterisation,
 * cells, induction, reduction, electronics, packets) is captured on a capture stream owned by the context and
 * launched as one graph on the call's stream; the context keeps one executable graph and updates it in place when
 * the next call has the same launch structure (else instantiates a new one), only after the previous launch has
 * finished.  Results are identical to 0 (default: direct launches).  Ignored in LTS_REDUCE_SUMMED mode, which reads
 * sizes back in the middle of the call; the server's lanes always launch directly.  Stage timing (lts_set_timing)
 * records nothing for graph-launched calls. */
lts_status lts_set_graph(lts_context *ctx, int32_t on);
/* Number of in-place updates and of instantiations of the context's executable graph so far (host pointers). */
lts_status lts_graph_stats(lts_context *ctx, int64_t *updates, int64_t *instantiations);

/* Work-split table chosen by an autotuner (the package's autotune module sweeps it): entry k applies to calls whose
 * mean segments per event is at least min_segments_per_event of entry k and below that of entry k+1 (entries in
 * ascending order; calls below the first entry use it too).  For the duration of such a call (lts_simulate,
 * lts_simulate_batch, and every batch of a server started from this context) the entry's reduce mode, induce
 * slices, ticks per thread and lane exchange replace the context's own settings.  n = 0 (or entries = NULL) removes
 * the table.  Copied; LTS_ERR_INVALID_ARG for an unsorted table or invalid knob values. */
typedef struct lts_tuning {
    int64_t min_segments_per_event;
    int32_t reduce_mode, induce_slices, ticks_per_thread, lane_exchange;
} lts_tuning;
lts_status lts_set_tuning(lts_context *ctx, const lts_tuning *entries, int32_t n);

/* Sizing pass (synchronous on `stream`): need[4] = (segment-pixel pairs, active pixels, charge cells,
 * packet upper bound = active pixels * max_packets).  Host pointer need. */
lts_status lts_plan(lts_context *ctx, const lts_segments *segs, int64_t need[4], void *stream);

/* Simulate one event (Sec. 3: recombination -> drift -> rasterisation -> induction -> per-pixel sum ->
 * electronics, plus the FP64 charge report).  event_id keys the noise streams, so results do not depend on
 * batch placement.  Capacity errors return LTS_ERR_CAPACITY with the needs in out->counts (device). */
lts_status lts_simulate(lts_context *ctx, uint64_t event_id, const lts_segments *segs, const lts_outputs *out,
                        void *stream);

/* Simulate n_events independent events whose segments are concatenated in `segs` (event e owns rows
 * [seg_offsets[e], seg_offsets[e+1]), host array of n_events + 1 entries) in one set of launches.  event_ids is a
 * host array.  Outputs are concatenated event-major; out->event_pixel_offsets / event_packet_offsets must be
 * provided; report holds 5 doubles per event. */
lts_status lts_simulate_batch(lts_context *ctx, int32_t n_events, const uint64_t *event_ids,
                              const int64_t *seg_offsets, const lts_segments *segs, const lts_outputs *out,
                              void *stream);

/* ---- stage entry points (test hooks; same kernels as the pipeline) ---------------------------------- */

/* Steps of Sec. 3.1-3.2 per segment.  out_f[n * 6] (device): Q_R, Q_a, t_drift (us), sigma_T (cm),
 * sigma_t (us), dE/dx; out_i[n * 2] (device): number of sample points N, flags (bit0 Box clamp, bit1 invalid). */
lts_status lts_stage_quench_drift(lts_context *ctx, const lts_segments *segs, float *out_f, int32_t *out_i,
                                  void *stream);

/* Charge cells of the segments of the last lts_simulate call on this context (synchronous, host outputs):
 * box[6] = (a0, na, u0, nu, v0, nv) in absolute tick / sub-pixel-bin indices, cells[na][nu][nv] if cap >= size. */
lts_status lts_debug_cells(lts_context *ctx, int64_t segment, int64_t box[6], float *cells_host, int64_t cap);

/* Rasterisation alone (Sec. 3.3.2: the pixels a segment's charge reaches; Sec. 3.3.1: a pixel reaches the table's
 * extent of sub-pixel bins around its centre).  Writes the (segment, pixel) pairs of the call, pixel-major with
 * ascending segment index within a pixel: pair_segment[k] = row of segs, pair_pixel[k] = tile-local pixel id
 * (both device, cap_pairs entries).  *n_pairs_out (host) receives the pair count; LTS_ERR_CAPACITY if it exceeds
 * cap_pairs (nothing is written then).  Synchronises the stream once (sizing). */
lts_status lts_stage_rasterize(lts_context *ctx, const lts_segments *segs, int32_t *pair_segment,
                               int32_t *pair_pixel, int64_t cap_pairs, int64_t *n_pairs_out, void *stream);

/* Induction per pair, materialised (Sec. 3.3.2, eq. (current), the per-(segment, pixel, tick) waveforms of the
 * paper's design, Sec. 3.4): pair k of the list lts_stage_rasterize returns gets row k of pair_current
 * (device, cap_pairs * n_ticks floats), its current over the whole window (zero outside the pair's reach in time).
 * pair_segment / pair_pixel (device, may be NULL) receive the pair list.  event_id keys the Monte Carlo draws.
 * Capacity and synchronisation as lts_stage_rasterize.  Memory: 4 * n_ticks bytes per pair. */
lts_status lts_stage_induce(lts_context *ctx, uint64_t event_id, const lts_segments *segs, int32_t *pair_segment,
                            int32_t *pair_pixel, float *pair_current, int64_t cap_pairs, int64_t *n_pairs_out,
                            void *stream);

/* Per-pixel sum of materialised pair waveforms (Sec. 3.4: the current on a pixel is the sum over the segments
 * reaching it).  pair_pixel[n_pairs] (device) must be grouped by ascending pixel id (as lts_stage_rasterize
 * returns it; LTS_ERR_INVALID_ARG otherwise); pair_current[n_pairs * n_ticks] (device).  Writes one row per
 * distinct pixel: pixel_id[k] and current[k * n_ticks ...] (device, cap_pixels rows), each the FP32 Kahan sum of
 * its pairs in stored order.  *n_pixels_out (host) receives the row count; LTS_ERR_CAPACITY if above cap_pixels.
 * Synchronises the stream once. */
lts_status lts_stage_reduce(lts_context *ctx, const int32_t *pair_pixel, const float *pair_current, int64_t n_pairs,
                            int32_t *pixel_id, float *current, int64_t cap_pixels, int64_t *n_pixels_out,
                            void *stream);

/* Front end alone on given currents: n_pix pixels with tile-local ids pixel_ids[] (device), currents
 * current[n_pix * n_ticks] (device).  Packets as in lts_outputs (counts and packet arrays). */
lts_status lts_stage_electronics(lts_context *ctx, uint64_t event_id, const int32_t *pixel_ids, const float *current,
                                 int64_t n_pix, const lts_outputs *out, void *stream);

/* The front end of lts_stage_electronics for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and results, but the staging it
 * needs (per-pixel packet slots, offsets, scan partials, counters, the event id and, when out->report is NULL, the
 * report) lives in a static device array of 32 MiB that each GPU holds from library load to process end, and the
 * call enqueues kernels only (no allocation, no memset or host copy), so it may be captured into a graph.  Limit:
 * about 16 * n_pix + 7 * n_pix * max_packets bytes must fit in 32 MiB (e.g. 35,000 pixels at 128 packets);
 * larger inputs return LTS_ERR_INVALID_ARG with the sizes in lts_last_error.  Every call on a device shares that
 * device's array, so calls that overlap on one GPU (other streams, other contexts or threads) race: serialise
 * them.  Arguments, outputs and stream semantics as lts_stage_electronics. */
lts_status lts_stage_electronics_noalloc(lts_context *ctx, uint64_t event_id, const int32_t *pixel_ids,
                                         const float *current, int64_t n_pix, const lts_outputs *out, void *stream);

/* Algorithmic work of the last lts_simulate / lts_simulate_batch / lts_plan call on this context (synchronous):
 * out[0] (segment, pixel) pairs; out[1] products c[a,u,v] * R[k,i,j] of eq. (current) that land in the tick
 * window, summed over pairs (the multiply-adds of the induction; in LTS_REDUCE_SUMMED the products of summed
 * column charges, summed over pixels, counting only ticks that hold charge); out[2] charge cells in reach summed over
 * pairs (summed columns' ticks with charge in reach summed over pixels in LTS_REDUCE_SUMMED); out[3] charge cells of all segments; out[4] (LTS_REDUCE_SUMMED
 * only, else 0) the products the summed induction kernel computes, zeros included (every 256- or 512-tick tile,
 * as the kernel choice sets, that a merged record's window meets, all its lanes, charge ticks rounded up to 8):
 * out[1] / out[4] is the useful fraction of its multiply-adds; out[5] the (pixel, merged record) records the
 * kernel walks in LTS_REDUCE_SUMMED, else the pairs. */
lts_status lts_work_stats(lts_context *ctx, double out[6]);

/* Test hook for the error paths: after `after` further host-allocation points inside the library have passed
 * (0 = the next one), one of them fails as if host memory were exhausted, once; -1 disarms.  The points are the
 * host-side copies of lts_set_response, lts_server_submit, a server lane's batch set-up and lts_light_create.  The
 * failing call returns LTS_ERR_OOM (a failing server batch gives its tickets that status) and the object stays
 * usable.  Process-wide; LTS_ERR_INVALID_ARG for after < -1. */
lts_status lts_debug_fail_host_alloc(int64_t after);

/* Raw Philox4x32-10 blocks: ctr[n*4] (device) with key (k0, k1) -> out[n*4] (device). */
lts_status lts_stage_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out, int64_t n, void *stream);

/* ---- serving ----------------------------------------------------------------------------------------------
 * A request loop with continuous batching: submitted events (segments in HOST memory, copied at submit) wait in a
 * queue; each of n_lanes worker lanes (own HIP stream, own scratch pool and device buffers, the response table of
 * the parent context) repeatedly takes the waiting events at the queue's head (at most max_batch_events events and
 * max_batch_segments segments) and runs them as one batch (lts_simulate_batch), so events that arrive while other
 * batches are on the GPU are admitted as soon as a lane frees up, and the lanes' work overlaps on the device.
 * Admission by device memory: a lane sizes its tentative batch on the device and runs it only if its footprint
 * (scratch pool, segments and outputs, grown to the batch's exact sizes) stays within mem_budget_bytes / n_lanes and
 * the growth fits the device's free memory (hipMemGetInfo) less 1 GiB; otherwise it halves the batch (the events cut
 * off go back to the queue front, in order).  A single event that does not fit is sized once more after the lane
 * frees its pooled scratch (buffers that earlier, larger batches grew), and finishes with LTS_ERR_OOM only if it
 * still does not fit.
 * Results are copied back to host memory owned by the server until lts_server_release.  Thread-safe. */
typedef struct lts_server lts_server;

typedef struct lts_server_cfg {
    int32_t n_lanes;              /* concurrent batches in flight (>= 1; default 2 if 0) */
    int32_t max_batch_events;     /* events per batch (default 64 if 0) */
    int64_t max_batch_segments;   /* segments per batch (default 4,000,000 if 0) */
    int64_t mem_budget_bytes;     /* device-memory budget for all lanes (default if 0: half the device's memory) */
    int32_t return_currents;      /* copy per-pixel currents back (otherwise only pixel ids, packets, report) */
} lts_server_cfg;

typedef struct lts_result_view {  /* host memory owned by the server, valid until lts_server_release */
    uint64_t event_id;
    int32_t status;               /* lts_status of the event's batch */
    int64_t n_pixels, n_packets;
    const int32_t *pixel_id;      /* [n_pixels] */
    const float *current;         /* [n_pixels * n_ticks] or NULL if return_currents == 0 */
    const int32_t *pkt_pixel, *pkt_tick;
    const uint16_t *pkt_adc;
    const uint8_t *pkt_flags;
    double report[5];
    int64_t counts[4];            /* this event's pixels, packets, samples dropped past the window, packets over
                                     max_packets (the same as the event alone) */
    double t_submit, t_start, t_done;   /* seconds on a monotonic clock: submission, batch launch, completion */
    int32_t batch_events;         /* events in the batch that carried this one */
} lts_result_view;

/* Start a server for the parameters and response table of ctx (the server creates its own lane contexts; ctx
 * stays usable and must outlive nothing of the server). */
lts_status lts_server_start(lts_context *ctx, const lts_server_cfg *cfg, lts_server **out);
/* Copy an event's host segment table and queue it; *ticket identifies it. */
lts_status lts_server_submit(lts_server *srv, uint64_t event_id, const lts_segments *host_segs, uint64_t *ticket);
/* LTS_ERR_NOT_READY until the ticket's batch has finished; then LTS_OK (or the batch's error) and a view. */
lts_status lts_server_poll(lts_server *srv, uint64_t ticket, lts_result_view *out);
/* Like poll, but blocks up to timeout_s seconds (< 0: forever). */
lts_status lts_server_wait(lts_server *srv, uint64_t ticket, lts_result_view *out, double timeout_s);
/* Free a finished ticket's host results. */
lts_status lts_server_release(lts_server *srv, uint64_t ticket);
/* Cancel queued tickets (their poll returns LTS_ERR_CANCELLED), finish in-flight batches, free everything. */
lts_status lts_server_stop(lts_server *srv);

/* ---- stage timing --------------------------------------------------------------------------------------
 * When enabled, the library records HIP events on the caller's stream around each stage group of every
 * pipeline call.  lts_get_timing waits for the recorded events, returns the summed elapsed milliseconds and the
 * number of timed calls per stage since the previous lts_get_timing, and resets them (in LTS_REDUCE_SUMMED the
 * charge-cell stage is timed on the context's own stream, where it runs beside the start of LTS_STAGE_INDUCE).
 * Host arrays of LTS_N_STAGES entries; calls may be NULL. */
enum {
    LTS_STAGE_QUENCH_DRIFT = 0,   /* recombination, drift, charge boxes, pair counts, scans (Sec. 3.1-3.2) */
    LTS_STAGE_RASTERIZE = 1,      /* active-pixel compaction, pair lists, per-pixel ordering */
    LTS_STAGE_CELLS = 2,          /* diffused charge cells per segment (Sec. 3.3.2, eq. (rho)) */
    LTS_STAGE_INDUCE = 3,         /* induced current and per-pixel sum (Sec. 3.3.2 eq. (current), Sec. 3.4) */
    LTS_STAGE_ELECTRONICS = 4,    /* front end, packets and the FP64 current sum (Sec. 3.4) */
    LTS_STAGE_INDUCE_KERNEL = 5,  /* inside LTS_STAGE_INDUCE: the induction kernel itself (with the per-pair kernels'
                                     work-order sort; without the summed mode's column sums and piece lists) */
    LTS_N_STAGES = 6
};
lts_status lts_set_timing(lts_context *ctx, int32_t enabled);
lts_status lts_get_timing(lts_context *ctx, double ms[LTS_N_STAGES], int64_t calls[LTS_N_STAGES]);

/* ---- light path (Sec. 4) --------------------------------------------------------------------------------
 * On given photocurrents (expected photoelectrons emitted per light tick per detector, the output of the visibility
 * look-up of Sec. 4.1, which is the caller's): scintillation time profile, photoelectron statistics, electronics
 * response with noise, and group triggers.  An lts_light object holds the response kernel, the noise spectrum and
 * its device buffers (sized at creation); it is not thread-safe. */
typedef struct lts_light_params {
    double tick;               /* ns per light tick */
    double tau_p, tau_s;       /* ns: prompt and slow scintillation decay times (Sec. 4.2) */
    double f_prompt;           /* prompt fraction f_p of the two-exponential profile (Sec. 4.2) */
    double trunc;              /* the scintillation kernel is truncated after trunc * tau_s (5 in Sec. 4.2) */
    double gain;               /* G: ADC counts per photoelectron (Sec. 4.3) */
    double normal_above;       /* mean p.e. per tick above which a normal draw replaces Poisson (30 in Sec. 4.2) */
    int32_t n_det, n_ticks;    /* detectors; ticks of the window (<= 1 << 19) */
    int32_t group;             /* consecutive detectors summed for triggering (divides n_det) */
    double trig_threshold;     /* ADC counts on a group's summed waveform */
    int32_t trig_deadtime;     /* ticks after a trigger before the group can trigger again (>= 1) */
    int32_t max_trig;          /* triggers kept per group */
    uint64_t seed;             /* Philox key of the photoelectron draws and the noise phases */
} lts_light_params;
typedef struct lts_light lts_light;

/* Create a light simulator on `device`.  resp: unit-normalised impulse response sampled at the light tick (n_resp
 * values, host, copied); noise_amp: amplitudes A_f of the noise sinusoids f = 1 .. n_freq cycles per window (host,
 * copied; n_freq < n_ticks / 2).  INVALID_ARG for inconsistent parameters, OOM / DEVICE on allocation failures. */
lts_status lts_light_create(int device, const lts_light_params *p, const float *resp, int32_t n_resp,
                            const float *noise_amp, int32_t n_freq, lts_light **out);
void lts_light_destroy(lts_light *L);

/* One event, stream-ordered on `stream` (a hipStream_t; NULL = default), all pointers device memory:
 *   ipe   [n_det][n_ticks] FP32 photocurrent (expected p.e. emitted per tick), read only;
 *   mu    [n_det][n_ticks] FP64 expected p.e. per tick after the truncated scintillation convolution (Sec. 4.2:
 *         mu[t] = sum_{k=0}^{trunc tau_s / tick} ipe[t-k] f_scint(k tick) tick) or NULL;
 *   pe    [n_det][n_ticks] FP64 photoelectrons per tick: Poisson by inverse transform sampling (mean <= normal_above)
 *         or mu + sqrt(mu) g, Philox counter (detector, tick, event low word, event high word << 4 | 12), or NULL;
 *   V     [n_det][n_ticks] FP32 waveform: G sum_k pe[t-k] resp[k] + sum_f A_f cos(2 pi f t / n_ticks + phi_f),
 *         phi_f = 2 pi u, u from Philox counter (detector, f, event low word, event high word << 4 | 13);
 *   trig  [n_det / group][max_trig] INT32 trigger ticks (-1 after the last), trig_count [n_det / group] INT32:
 *         per group, scanning in time, each tick where the group's summed V reaches trig_threshold, then none for
 *         trig_deadtime ticks (Sec. 4.3); may be NULL together.
 * The event id keys the draws, so results do not depend on call order. */
lts_status lts_light_simulate(lts_light *L, uint64_t event_id, const float *ipe, double *mu, double *pe, float *V,
                              int32_t *trig, int32_t *trig_count, void *stream);

/* Replay lts_light_simulate through a HIP graph (1) or launch its kernels one by one (0, default).  The graph is
 * captured on the first call and again whenever the caller's buffers change; later calls only set the event id in
 * the graph's two random-number kernels and launch it on `stream`.  Results are the same either way.  No memory
 * is allocated or set by the captured sequence. */
lts_status lts_light_set_graph(lts_light *L, int32_t on);
const char *lts_light_last_error(const lts_light *L);

const char *lts_status_str(lts_status s);
const char *lts_last_error(const lts_context *ctx);
const char *lts_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LTSIM_H */
