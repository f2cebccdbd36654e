// launch.hpp -- host-side launchers of the gfx950 kernels (internal interface between runtime.hip and kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace ltsim {

struct SegArrays {
    const float *x0, *y0, *z0, *t0, *x1, *y1, *z1, *t1, *energy, *dedx;
};

// Device buffers of one pipeline invocation (owned by the context's scratch pool).
struct Work {
    int64_t n_seg = 0;
    int32_t n_ev = 0;
    const int64_t *seg_ev_off = nullptr;     // [n_ev + 1] segment ranges of the events
    const uint64_t *event_ids = nullptr;     // [n_ev]
    SegInfo *si = nullptr;                   // [n_seg]
    int64_t *cell_off = nullptr;             // [n_seg + 1] counts, then exclusive offsets
    uint64_t *pix_cnt = nullptr;             // [n_ev * npx + 1] packed (pairs | active << 40), then offsets
    int32_t *cursor = nullptr;               // [n_ev * npx]
    int32_t *pix_slot = nullptr;             // [n_ev * npx]
    int32_t *slot_gp = nullptr;              // [cap_slots] global pixel index e * npx + p
    int64_t *slot_off = nullptr;             // [cap_slots + 1] pair ranges per slot
    int32_t *pairs_unsorted = nullptr;       // [cap_pairs]
    int32_t *pairs = nullptr;                // [cap_pairs] segment ids, pixel-major, ascending per pixel
    float *cells = nullptr;                  // [cap_cells]
    int32_t *pk_tick = nullptr;              // [cap_slots * max_packets]
    uint16_t *pk_adc = nullptr;
    uint8_t *pk_flag = nullptr;
    int64_t *pk_off = nullptr;               // [cap_slots + 1] counts, then exclusive offsets
    DevHeader *hdr = nullptr;
    double *report = nullptr;                // [5 * n_ev]
    int64_t *ev_cnt = nullptr;               // [2 * n_ev] per event: samples dropped past the window, packets over
                                             // max_packets (or null)
    const uint8_t *disabled = nullptr;       // [npx] disabled-channel mask or null
    void *scan_tmp = nullptr;                // scan partials
    int64_t scan_tmp_elems = 0;
    int32_t *order = nullptr;                // [2 * cap_slots + 2 * kOrderBuckets] per-pair induction work order
};
constexpr int kOrderBuckets = 512;            // log-scale work buckets of the largest-first pixel order

struct Table {
    const float *Rpad = nullptr;             // [bx * by][col_len], zero-padded columns
    const double *prefix = nullptr;          // [bx * by][t_r + 1] FP64 prefix sums of each column
};

// Device buffers of the summed (sum-then-convolve) induction: per event an absolute grid of sub-pixel columns
// u in [UL, UL + CU) x v in [VL, VL + CV), UL = nsub/2 - bx (the columns some in-grid pixel can reach).
// One column piece as seen from one active pixel: what the summed induction loop needs, in one 16-byte record
// (no dependent loads): the piece's first tick and length, its summed charge at S + 8 * cell8 (at
// Sm + 8 * (cell8 - nS8) for a merged record, cell8 >= nS8), and the folded table column that the pixel sees it
// through.
struct alignas(16) PieceRef {
    int32_t a0, na;
    uint32_t cell8;
    int32_t bin;
};

// The fields of a segment that the column passes read for every (segment, column) entry, 32 bytes (the full record is
// 176): a spill's array stays in the last-level cache.
struct alignas(16) SumSeg {
    int32_t a0, na, u0, v0, nv, na_pad;
    int64_t cell_off;
};
static_assert(sizeof(SumSeg) == 32, "SumSeg layout");

struct SumWork {
    int32_t CU = 0, CV = 0, UL = 0, VL = 0;
    int64_t n_cols = 0;                      // n_ev * CU * CV
    SumSeg *segc = nullptr;                  // [n_seg] written by the count pass
    int64_t *col_seg_off = nullptr;          // [n_cols + 1] segments per column, then offsets
    int32_t *col_cursor = nullptr;           // [n_cols]
    uint64_t *col_tmp = nullptr;             // [n_col_seg] per column: keys (first tick << 32 | segment index)
    uint64_t *col_seg = nullptr;             // [n_col_seg] the same keys, ascending per column
    int32_t *active = nullptr;               // [n_cols] columns with pieces (any order), n_active of them
    uint32_t *n_active = nullptr;
    int64_t *piece_off = nullptr;            // [n_cols + 1] pieces per column, then offsets
    int64_t *s_off = nullptr;                // [n_cols + 1] summed-cell floats per column, then offsets
    SegInfo *piece = nullptr;                // [n_pieces] one 1 x 1 x L box per column piece
    PieceRef *pdesc = nullptr;               // [n_pieces] the same pieces as compact records (bin not set)
    float *S = nullptr;                      // [n_s] summed charge per column piece (padded to kAC)
    int64_t *list_off = nullptr;             // [n_slots + 1] pieces in reach per active pixel, then offsets
    int32_t *list = nullptr;                 // [n_list] piece ids per active pixel, by folded column, then first tick
    PieceRef *rec = nullptr;                 // [n_list] the same pieces as records
    int64_t *mlist_off = nullptr;            // [n_slots + 1] records per active pixel after the mirror merge, offsets
    int64_t *m_off = nullptr;                // [n_slots + 1] merged charge floats per active pixel, then offsets
    PieceRef *mrec = nullptr;                // [n_mlist] the merged records
    float *Sm = nullptr;                     // [n_m] charges of the merged records (padded to kAC)
    uint32_t nS8 = 0;                        // S floats / kAC: cell8 at or above it points into Sm
    int32_t align_res = 0;                   // first tick of every column interval, mod 8 (set by the kernel choice)
    bool piece_lists = true;                 // write `piece` and `list` (read only by the lane-exchange kernel and the
                                             // per-pair kernels over the pieces)
};
// The summed induction kernel a tuning choice runs: the 256-tick LDS-staged one (automatic), the 512-tick register
// one (8 ticks per thread), or the per-pair kernels over the pieces; and the interval alignment each one wants.
bool summed_tile256(int32_t rt, bool shift);
int32_t summed_align_res(const DevParams &P, int32_t rt, bool shift);
constexpr int32_t kPieceTicks = kPieceMax;   // ticks per column piece (a multiple of kAC, <= kNaMax)
static_assert(kPieceTicks % kAC == 0 && kPieceTicks <= kNaMax, "piece length");

void launch_sum_ranges(const DevParams &P, const Work &w, const SumWork &sw, hipStream_t st);   // counts
void launch_sum_fill(const DevParams &P, const Work &w, const SumWork &sw, hipStream_t st);     // lists, pieces
void launch_sum_pieces(const DevParams &P, const Work &w, const SumWork &sw, hipStream_t st);   // piece records, S
void launch_sum_lists_count(const DevParams &P, const Work &w, const SumWork &sw, int64_t n_slots, hipStream_t st);
void launch_sum_lists_fill(const DevParams &P, const Work &w, const SumWork &sw, int64_t n_slots, int64_t n_list,
                           hipStream_t st);                                                    // + records
void launch_sum_merge(const SumWork &sw, int64_t n_slots, bool fill, hipStream_t st);          // mirror merge
// largest-first pixel order of the summed induction (null when the chosen kernel takes pixels in slot order)
const int32_t *launch_summed_order(const Work &w, const SumWork &sw, int64_t n_slots, int32_t rt, bool shift,
                                   hipStream_t st);
void launch_induce_summed(const DevParams &P, const Work &w, const SumWork &sw, const Table &T, float *wave,
                          int64_t n_slots, int32_t rt, bool shift, const int32_t *order, hipStream_t st);

int64_t scan_tmp_needed(int64_t n);
void scan_exclusive_i64(int64_t *data, int64_t n, int64_t *total_dst, void *tmp, hipStream_t st);
void scan_exclusive_u64(uint64_t *data, int64_t n, void *tmp, hipStream_t st);

void launch_quench_drift(const DevParams &P, const SegArrays &S, const Work &w, hipStream_t st);
void launch_slots(const DevParams &P, const Work &w, int32_t *pixel_id_out, int64_t *ev_pix_off, hipStream_t st);
void launch_zero(void *p, int64_t bytes, hipStream_t st);   // bytes: a multiple of 4
void launch_store_u64(uint64_t *p, uint64_t v, hipStream_t st); // one value written by a kernel (capture-safe)
void launch_fill_pairs(const DevParams &P, const Work &w, hipStream_t st);
void launch_sort_pairs(const Work &w, int64_t n_slots_host, hipStream_t st);
void launch_cells(const DevParams &P, const Work &w, hipStream_t st);
void launch_induce(const DevParams &P, const Work &w, const Table &T, float *wave, int mode, int64_t n_slots_host,
                   int32_t rt, bool shift, hipStream_t st);
void launch_induce_mfma(const DevParams &P, const Work &w, const Table &T, float *wave, int64_t n_slots,
                        hipStream_t st);
void launch_induce_slices(const DevParams &P, const Work &w, const Table &T, float *wave, int64_t n_slots, int32_t NS,
                          float *part, int64_t chunk, int32_t rt, hipStream_t st);
void launch_pair_list(const DevParams &P, const Work &w, int64_t n_slots, int32_t *pair_seg, int32_t *pair_pix,
                      hipStream_t st);
void launch_induce_pairs(const DevParams &P, const Work &w, const Table &T, int64_t n_slots, float *out,
                         hipStream_t st);
void launch_run_heads(const int32_t *pix, int64_t n, int64_t *head, DevHeader *H, hipStream_t st);
void launch_run_starts(const int32_t *pix, int64_t n, const int64_t *idx, int64_t *start, int32_t *pixel_out,
                       int64_t cap, hipStream_t st);
void launch_reduce_runs(const float *pair_current, const int64_t *start, int64_t n_runs, int32_t NT, float *current,
                        hipStream_t st);
void launch_electronics(const DevParams &P, const float *wave, const int32_t *slot_gp, const uint64_t *event_ids,
                        int64_t n_slots, const Work &w, hipStream_t st);
void launch_compact_packets(const DevParams &P, const Work &w, int64_t n_slots, int32_t *pkt_pixel, int32_t *pkt_tick,
                            uint16_t *pkt_adc, uint8_t *pkt_flags, int64_t cap_packets, const int64_t *ev_pix_off,
                            int64_t *ev_pkt_off, int64_t *counts, hipStream_t st);
void launch_stage_quench_drift(const DevParams &P, const SegArrays &S, int64_t n, float *out_f, int32_t *out_i,
                               hipStream_t st);
void launch_work_stats(const DevParams &P, const SegInfo *si, int64_t n_seg, unsigned long long *acc, hipStream_t st);
void launch_work_stats_summed(const DevParams &P, int64_t n_slots, const int64_t *list_off, const PieceRef *rec,
                              const float *S, const int64_t *mlist_off, const PieceRef *mrec, bool tile256,
                              unsigned long long *acc, hipStream_t st);
void launch_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out, int64_t n, hipStream_t st);

}  // namespace ltsim
